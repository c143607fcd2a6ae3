"""Pins of the oracle's coefficient tables and stencil selection against the paper and exact
rational arithmetic (no GPU).

Table 2 rows are re-derived from first principles: row m is the unique finite-difference flux
reconstruction that is exact for every polynomial h of degree < w on its w-point support when the
point values f_j are the cell averages of h (eq:flux, section "Higher-order spatial
reconstructions"). Table 3 is checked against the printed patterns and the selection rule stated
in the text (no reconstruction crosses a cut sub-stencil; the two tie-breaks).
"""
from fractions import Fraction as Fr
import itertools

import numpy as np
import pytest

from conftest import read_golden


def _rational_rows(name):
    return [[Fr(t) for t in row] for row in read_golden(name)]


def _cell_average_monomial(l, d):
    """(1/dx) * integral over cell l (centred at l, width 1) of x^d, exactly."""
    a, b = Fr(2 * l - 1, 2), Fr(2 * l + 1, 2)
    return (b ** (d + 1) - a ** (d + 1)) / (d + 1)


def _solve(A, b):
    n = len(A)
    M = [row[:] + [b[i]] for i, row in enumerate(A)]
    for col in range(n):
        piv = next(r for r in range(col, n) if M[r][col] != 0)
        M[col], M[piv] = M[piv], M[col]
        for r in range(n):
            if r != col and M[r][col] != 0:
                f = M[r][col] / M[col][col]
                M[r] = [x - f * y for x, y in zip(M[r], M[col])]
    return [M[i][n] / M[i][i] for i in range(n)]


def reconstruction_row(support):
    """Coefficients (offsets -3..3) of the reconstruction at x = 1/2 from cell averages on
    `support` (cell offsets relative to i), exact for degree < len(support)."""
    w = len(support)
    A = [[_cell_average_monomial(l, d) for l in support] for d in range(w)]
    b = [Fr(1, 2) ** d for d in range(w)]
    sol = _solve(A, b)
    row = [Fr(0)] * 7
    for l, a in zip(support, sol):
        row[l + 3] = a
    return row


def test_table2_doubles_are_the_printed_rationals(orc):
    t2, _ = orc.tables()
    gold = _rational_rows("table2.txt")
    assert len(gold) == 13
    for m in range(13):
        for l in range(7):
            assert t2[m, l] == float(gold[m][l]), (m, l)


def test_table2_rows_are_exact_reconstructions_on_their_support():
    gold = _rational_rows("table2.txt")
    orders = []
    for m, row in enumerate(gold):
        support = [l - 3 for l in range(7) if row[l] != 0]
        assert support == list(range(support[0], support[-1] + 1)), "support must be contiguous"
        assert 0 in support, "every candidate contains the upwind cell i"
        assert reconstruction_row(support) == row, f"row {m}"
        assert sum(row) == 1
        orders.append(len(support))
    # order of accuracy listed in the text: 7, 6, 6, 5, 5, 5, 4, 4, 4, 4, 3, 3, 3
    assert orders == [7, 6, 6, 5, 5, 5, 4, 4, 4, 4, 3, 3, 3]


def test_table2_row0_is_the_linear_seventh_order_upwind_scheme():
    gold = _rational_rows("table2.txt")
    assert [x * 420 for x in gold[0]] == [-3, 25, -101, 319, 214, -38, 4]


def test_three_point_candidates_are_table2_rows_10_to_12():
    # eq:3_rd: the 3rd-order candidates on S0 = {i-2..i}, S1 = {i-1..i+1}, S2 = {i..i+2}
    gold = _rational_rows("table2.txt")
    assert reconstruction_row([-2, -1, 0]) == gold[12]
    assert reconstruction_row([-1, 0, 1]) == gold[11]
    assert reconstruction_row([0, 1, 2]) == gold[10]
    assert gold[12][1:4] == [Fr(2, 6), Fr(-7, 6), Fr(11, 6)]


def test_table1_is_the_teno5_weight_mix_of_the_three_point_candidates(orc):
    """Table 1 row for (delta0, delta1, delta2) = sum_k omega_k q_k with omega from eq:TENO_W."""
    d = [Fr(1, 10), Fr(6, 10), Fr(3, 10)]  # eq:opt
    q = [reconstruction_row([-2, -1, 0]), reconstruction_row([-1, 0, 1]), reconstruction_row([0, 1, 2])]
    gold = read_golden("table1.txt")
    _, t1 = orc.tables()
    for r, row in enumerate(gold):
        delta = [int(v) for v in row[:3]]
        coeff = [Fr(v) for v in row[3:]]
        dsum = sum(dk * dl for dk, dl in zip(d, delta))
        mix = [sum(d[k] * delta[k] / dsum * q[k][l] for k in range(3)) for l in range(7)]
        assert mix[0] == 0 and mix[6] == 0
        assert mix[1:6] == coeff, f"Table 1 row {r}"
        for l in range(5):
            assert t1[r, l] == float(coeff[l])


def test_teno5_weights_equal_table1_lut(orc):
    """The oracle's TENO5 reconstruction (eq:TENO_W on eq:3_rd) equals Table 1 to a few ulp."""
    rng = np.random.default_rng(3)
    cfg = orc.Config(orc.ADV1D, 16, scheme=orc.TENO5)
    for delta in itertools.product([0, 1], repeat=3):
        if delta == (0, 0, 0):
            continue
        code = (delta[0] << 2) | (delta[1] << 1) | delta[2]
        for _ in range(20):
            w7 = rng.uniform(-1, 1, 7)
            a = orc.recon(cfg, code, w7)
            b = orc.table1_apply(*delta, w7[1:6])
            assert abs(a - b) <= 8 * np.finfo(float).eps * np.abs(w7).max() * 4, (delta, a, b)


def _pattern_match(pat, bits):
    return all(p == "*" or int(p) == b for p, b in zip(pat, bits))


def test_table3_is_the_printed_table_and_a_partition(orc):
    gold = read_golden("table3.txt")
    for p in range(32):
        bits = [(p >> (4 - q)) & 1 for q in range(5)]
        hits = [row[1] for row in gold if _pattern_match(row[0], bits)]
        assert len(hits) == 1, (bits, hits)
        expect = -1 if hits[0] == "none" else int(hits[0])
        assert orc.select7(p) == expect, bits


def _run_rule(bits):
    """Selection rule stated in the text: use the widest stencil made of consecutive smooth
    three-point sub-stencils A={i-3..i-1}, B={i-2..i}, C={i-1..i+1}, D={i..i+2}, E={i+1..i+3}
    that contains the upwind cell and crosses no cut sub-stencil; prefer interpolation
    (stencils through C) over extrapolation."""
    a, b, c, d, e = bits
    if c:
        lo = "C"
        if b:
            lo = "B"
            if a:
                lo = "A"
        hi = "C"
        if d:
            hi = "D"
            if e:
                hi = "E"
        return lo, hi
    if d:
        return "D", ("E" if e else "D")
    if b:
        return ("A" if a else "B"), "B"
    return None


_SUB = {"A": (-3, -1), "B": (-2, 0), "C": (-1, 1), "D": (0, 2), "E": (1, 3)}


def test_table3_equals_the_run_rule_and_never_crosses_a_cut_substencil(orc):
    gold = _rational_rows("table2.txt")
    for p in range(32):
        bits = [(p >> (4 - q)) & 1 for q in range(5)]
        m = orc.select7(p)
        run = _run_rule(bits)
        if run is None:
            assert m == -1
            continue
        lo, hi = _SUB[run[0]][0], _SUB[run[1]][1]
        support = [l - 3 for l in range(7) if gold[m][l] != 0]
        assert (support[0], support[-1]) == (lo, hi), (bits, m, support)
        for name, smooth in zip("ABCDE", bits):
            s0, s1 = _SUB[name]
            if not smooth:
                # the chosen stencil may not contain a cut sub-stencil entirely
                assert not (support[0] <= s0 and s1 <= support[-1]), (bits, name)


def test_table3_tie_breaks_stated_in_the_text(orc):
    assert orc.select7(0b11011) == 6   # (1,1,0,1,1): f6 (interpolation), not f9
    assert orc.select7(0b11010) == 10  # (1,1,0,1,0): f10, not f9
    assert orc.select7(0b11111) == 0
    for p in (0b00000, 0b00001, 0b10000, 0b10001):
        assert orc.select7(p) == -1    # (*,0,0,0,*): no stencil exists
