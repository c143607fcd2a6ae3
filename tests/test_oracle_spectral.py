"""Approximate dispersion relation (section "Approximate dispersion relation analysis") computed
with the oracle: pinned to the Fourier symbol of the seventh-order linear scheme (Table 2, row 0)
when every stencil is kept, to consistency Phi(phi) -> phi at small phi, and to the paper's claim
that the nonlinear scheme recovers the linear one on well-resolved modes while cutting stencils
near the grid cut-off."""
import math
from fractions import Fraction as Fr

import numpy as np
import pytest


def oracle_adr(orc, n, eps=None, scheme=0):
    """Modes 1 .. N/2 of the N-cell grid on [0, 2 pi): Phi = i dx r_hat / u_hat, the Fourier
    coefficients taken by numpy's FFT (cell centres shift every coefficient by the same phase,
    which cancels in the ratio). Returns phi, Phi and the number of cut masks per mode."""
    dx = 2.0 * math.pi / n
    x = (np.arange(n) + 0.5) * dx
    cfg = orc.Config(orc.ADV1D, n, 1, 0.0, 2.0 * math.pi, scheme=scheme, eps=eps)
    out, cut = [], []
    for k in range(1, n // 2 + 1):
        u = np.cos(k * x)
        r, ex = orc.rhs(cfg, u[None, None, :], want_faces=True)
        out.append(1j * dx * np.fft.fft(r[0, 0])[k] / np.fft.fft(u)[k])
        cut.append(int(np.count_nonzero(ex["masks_x"])))
    return 2.0 * math.pi * np.arange(1, n // 2 + 1) / n, np.array(out), np.array(cut)


def _linear_symbol(phi):
    from conftest import read_golden
    a = [float(Fr(t)) for t in read_golden("table2.txt")[0]]
    s = sum(a[l + 3] * np.exp(1j * l * phi) for l in range(-3, 4))
    return -1j * (1.0 - np.exp(-1j * phi)) * s


def test_all_stencils_kept_gives_the_linear_symbol(orc):
    phi, Phi, cut = oracle_adr(orc, 128, eps=1e30)
    assert not cut.any()
    assert np.abs(Phi - _linear_symbol(phi)).max() < 1e-12


def test_consistency_at_small_wavenumbers(orc):
    phi, Phi, _ = oracle_adr(orc, 256)
    small = phi < 0.3
    assert np.all(np.abs(Phi[small] - phi[small]) < 1e-5 * phi[small])
    assert np.all(Phi.imag <= 1e-12)                   # never anti-dissipative


def test_nonlinear_scheme_recovers_the_linear_one_on_resolved_modes(orc):
    phi, Phi, cut = oracle_adr(orc, 256)
    lin = _linear_symbol(phi)
    resolved = phi < 1.0
    assert not cut[resolved].any()
    assert np.abs(Phi[resolved] - lin[resolved]).max() < 1e-12
    # near the grid cut-off the smoothness indicators cut stencils and the symbol departs
    assert cut[phi > 2.5].any()
