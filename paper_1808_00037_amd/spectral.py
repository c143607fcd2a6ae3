"""Approximate dispersion relation of the semi-discrete operator (section "Approximate dispersion
relation analysis"), evaluated with the GPU operator through the C ABI.

For each resolved mode n = 1 .. N/2 of a periodic grid of N cells on [0, 2 pi) (reduced wavenumber
phi = 2 pi n / N), the linear-advection operator (a = 1) is applied to u_j = cos(n x_j) and its
result r is projected onto the mode: Phi(phi) = i dx r_hat / u_hat, with the discrete Fourier
coefficients r_hat, u_hat of mode n. The exact derivative gives Phi = phi; Re(Phi) measures
dispersion and Im(Phi) dissipation (negative: dissipative). For a linear scheme this is its exact
Fourier symbol; for the nonlinear scheme it is the symbol of the stencils it selects on each mode
(the paper does not spell out its procedure; unit amplitude on [0, 2 pi) is this implementation's
reading).
"""
import math

import numpy as np
import torch

from . import teno as T


def modes(n):
    """Cell centres of the N-cell grid on [0, 2 pi) and the resolved mode numbers 1 .. N/2."""
    x = (np.arange(n) + 0.5) * (2.0 * math.pi / n)
    return x, np.arange(1, n // 2 + 1)


def project(x, r, k):
    """Phi = i dx r_hat / u_hat for u = cos(k x) and operator output r."""
    n = len(x)
    dx = 2.0 * math.pi / n
    e = np.exp(-1j * k * x)
    u_hat = np.sum(np.cos(k * x) * e)
    r_hat = np.sum(r * e)
    return 1j * dx * r_hat / u_hat


def adr(n=256, scheme=T.TENO7X, eps=None):
    """(phi, Phi) for the modes 1 .. N/2, the operator evaluated on the GPU."""
    x, ks = modes(n)
    sv = T.Solver(T.ADV1D, n, 1, 0.0, 2.0 * math.pi, 0.0, 1.0, T.PERIODIC, T.PERIODIC, scheme=scheme, eps=eps)
    out = np.zeros(len(ks), dtype=complex)
    for i, k in enumerate(ks):
        U = torch.from_numpy(np.cos(k * x)[None, None, :].copy()).cuda()
        r = sv.rhs(U).cpu().numpy()[0, 0]
        out[i] = project(x, r, k)
    sv.poll()
    return 2.0 * math.pi * ks / n, out
