"""Pins of the oracle's scheme options (no GPU): the constants C and q of eq:TENO1, and the
reconstruction per conserved component instead of in characteristic variables (Remark 3).

C and q enter only through gamma_k = (C + tau5/(beta_k + eps))^q. Data whose smoothness measures are
known by hand give chi in closed form: for f = (0, 0, 0, 0, 1) (upwind order i-2..i+2), beta_0 =
beta_1 = 0 and beta_2 = 1/4 + 13/12 = 4/3, so tau5 = 4/3, and with eps = 4/3
    r_0 = r_1 = C + 1,  r_2 = C + 1/2,  chi_2 = (C + 1/2)^q / (2 (C + 1)^q + (C + 1/2)^q);
the mirror image (1, 0, 0, 0, 0) swaps stencils 0 and 2.
"""
import math

import numpy as np
import pytest

from paper_1808_00037_amd import workloads as W


def _chi_closed(C, q):
    g_smooth, g_cut = (C + 1.0) ** q, (C + 0.5) ** q
    s = 2 * g_smooth + g_cut
    return g_smooth / s, g_cut / s


@pytest.mark.parametrize("C", [0.5, 1.0, 2.0, 7.0])
@pytest.mark.parametrize("q", [1, 2, 3, 5, 6, 8])
def test_chi_closed_form_in_C_and_q(orc, C, q):
    smooth, cut = _chi_closed(C, q)
    for f5, k_cut in (([0, 0, 0, 0, 1], 2), ([1, 0, 0, 0, 0], 0)):
        d, chi = orc.flags5(f5, 4.0 / 3.0, ct=1e-5, C=C, q=q)
        want = [smooth, smooth, smooth]
        want[k_cut] = cut
        assert np.allclose(chi, want, rtol=1e-14, atol=0), (C, q, chi, want)
        # a cut-off just above / below the closed-form chi cuts / keeps that stencil
        for ct, expect in ((cut * (1 + 1e-9), 0), (cut * (1 - 1e-9), 1)):
            if ct < 1.0 / 3.0:
                d, _ = orc.flags5(f5, 4.0 / 3.0, ct=ct, C=C, q=q)
                assert d[k_cut] == expect and d[1] == 1, (C, q, ct, d)


def test_paper_constants_are_the_default(orc):
    rng = np.random.default_rng(5)
    for _ in range(50):
        f5 = rng.standard_normal(5)
        d0, c0 = orc.flags5(f5, 1e-6)
        d1, c1 = orc.flags5(f5, 1e-6, C=1.0, q=6)
        assert np.array_equal(d0, d1) and np.array_equal(c0, c1)


def test_larger_q_separates_smooth_from_cut_more_sharply(orc):
    # gamma_k grows like r_k^q: the ratio of the cut stencil's chi to a smooth one's is
    # ((C + 1/2) / (C + 1))^q, decreasing geometrically in q
    prev = None
    for q in range(1, 13):
        _, chi = orc.flags5([0, 0, 0, 0, 1], 4.0 / 3.0, q=q)
        ratio = chi[2] / chi[0]
        assert abs(ratio - 0.75 ** q) <= 1e-14 * 0.75 ** q
        if prev is not None:
            assert ratio < prev
        prev = ratio


@pytest.mark.parametrize("sys", [0, 3])
def test_componentwise_equals_characteristic_for_scalar_laws(orc, sys):
    pr = W.advection(2, 150) if sys == 0 else W.burgers(150, shift=0.1)
    a = orc.Config(sys, 150, x0=pr.x0, x1=pr.x1)
    b = orc.Config(sys, 150, x0=pr.x0, x1=pr.x1, characteristic=0)
    assert np.array_equal(orc.rhs(a, pr.U0), orc.rhs(b, pr.U0))


def test_componentwise_lax_friedrichs_constant_is_the_largest_wave_speed(orc):
    pr = W.euler2d(7, n=40, ny=36)
    rho, mx, my, E = pr.U0
    u, v = mx / rho, my / rho
    p = 0.4 * (E - 0.5 * rho * (u * u + v * v))
    c = np.sqrt(1.4 * p / rho)
    cfg = orc.Config(orc.EULER2D, 40, 36, characteristic=0)
    alpha, _ = orc.wave_speeds(cfg, pr.U0)
    assert np.allclose(alpha[:4], np.max(np.abs(u) + c), rtol=1e-15, atol=0)
    assert np.allclose(alpha[4:], np.max(np.abs(v) + c), rtol=1e-15, atol=0)


def _order(errs):
    return [math.log2(errs[k] / errs[k + 1]) for k in range(len(errs) - 1)]


def test_componentwise_euler_rhs_converges_to_minus_flux_divergence(orc):
    """Smooth 2D Euler state: without the characteristic projection the operator still converges to
    -(dF/dx + dG/dy) at seventh order (all stencils kept)."""
    errs = []
    for n in (16, 32, 64):
        x = W.cell_centres(0.0, 1.0, n)
        X, Y = np.meshgrid(x, x)

        def prim(X, Y):
            s = np.sin(2 * np.pi * X) * np.cos(2 * np.pi * Y)
            return 1 + 0.2 * s, 0.3 + 0.1 * np.cos(2 * np.pi * X), -0.2 + 0.1 * np.sin(2 * np.pi * Y), 1 + 0.1 * s

        def FG(Xc, Yc, direction):
            rho, u, v, p = prim(Xc, Yc)
            E = p / 0.4 + 0.5 * rho * (u * u + v * v)
            if direction == 0:
                return np.array([rho * u, rho * u * u + p, rho * u * v, u * (E + p)])
            return np.array([rho * v, rho * u * v, rho * v * v + p, v * (E + p)])

        h = 1e-30
        dF = np.imag(FG(X + 1j * h, Y, 0)) / h
        dG = np.imag(FG(X, Y + 1j * h, 1)) / h
        cfg = orc.Config(orc.EULER2D, n, n, characteristic=0)
        out = orc.rhs(cfg, W.conserved_2d(*prim(X, Y)))
        errs.append(np.abs(out + dF + dG).max())
    o = _order(errs)
    assert errs[-1] < 1e-6 and min(o) > 5.0, (errs, o)


def test_componentwise_is_conservative_and_keeps_a_free_stream(orc):
    pr = W.euler2d(8, n=48, ny=40)
    cfg = orc.Config(orc.EULER2D, 48, 40, characteristic=0)
    d = orc.rhs(cfg, pr.U0)
    scale = np.abs(d).max()
    assert np.all(np.abs(d.sum(axis=(1, 2))) <= 48 * 40 * 1e-15 * scale)
    U = np.empty((4, 12, 13))
    U[:] = np.array([0.7, 0.3, -0.2, 2.1])[:, None, None]
    assert np.all(orc.rhs(orc.Config(orc.EULER2D, 13, 12, characteristic=0), U) == 0.0)


def test_componentwise_selection_never_crosses_a_contact(orc):
    """A contact discontinuity (density jump at constant velocity and pressure) on a smooth
    background jumps in every conserved component: no selected stencil of any component, on either
    side, contains cells on both sides of it. (The energy jumps by rho u^2 / 2 only, so |u| is kept
    at 0.3 or more: the jump h of every split component then has h^2 far above eps = dx^3, the regime
    in which the cut-off separates a jump from smooth variation.)"""
    t2, _ = orc.tables()
    support = {m: [l - 3 for l in range(7) if t2[m, l] != 0.0] for m in range(13)}
    n = 128
    x = W.cell_centres(0.0, 1.0, n)
    rng = np.random.default_rng(9)
    bad = 0
    for trial in range(40):
        J = int(rng.integers(10, n - 10))
        u0, p0 = rng.choice([-1.0, 1.0]) * rng.uniform(0.3, 0.5), rng.uniform(0.5, 1.5)
        rho = 1.0 + 0.1 * np.sin(2 * np.pi * (x + rng.uniform())) + (np.arange(n) >= J) * rng.uniform(0.5, 1.5)
        U = np.stack([rho, rho * u0, p0 / 0.4 + 0.5 * rho * u0 * u0])[:, None, :]
        cfg = orc.Config(orc.EULER1D, n, bc_x=orc.OUTFLOW, characteristic=0)
        _, ex = orc.rhs(cfg, U, want_faces=True)
        masks = ex["masks_x"][0]
        for f in range(J - 5, J + 6):
            i = f - 1
            for s in range(3):
                mp, mm = int((masks[f] >> (8 * s)) & 0xF), int((masks[f] >> (8 * s + 4)) & 0xF)
                for cells in ([i + l for l in support[mp]], [i + 1 - l for l in support[mm]]):
                    if min(cells) <= J - 1 and max(cells) >= J:
                        bad += 1
    assert bad == 0
