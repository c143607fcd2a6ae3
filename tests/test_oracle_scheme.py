"""Pins of the oracle's operator against what the paper and mathematics fix (no GPU):
smoothness indicators vs their integral definition, closed-form flag cases, polynomial exactness,
the Fourier solution of the linear scheme, convergence orders, conservation, free stream, mirror
and transpose symmetry, 2D->1D reduction, the Roe property and eigen-decomposition, the
no-crossing property on brute-forced steps, and the shock-tube regression.
"""
from fractions import Fraction as Fr
import math

import numpy as np
import pytest

from paper_1808_00037_amd import workloads as W

EPS64 = np.finfo(float).eps


# ----------------------------------------------------------------------------- smoothness flags
def _beta_k(f5, k):
    """beta_k for the stencil S_k of the five upwind values (a,b,c,d,e) at i-2..i+2, evaluated over
    the target cell i, from the integral definition."""
    # the quadratic through cell averages on S_k, expanded about cell i (offset o of S_k's centre)
    vals = [f5[k + j] for j in range(3)]          # S_0: i-2..i, S_1: i-1..i+1, S_2: i..i+2
    o = k - 1                                      # S_k centre offset relative to cell i
    b, c, d = vals
    c2 = (b - 2 * c + d) / 2
    c1 = (d - b) / 2
    # p(x) = c0 + c1 (x - o) + c2 (x - o)^2 ;  over x in [-1/2, 1/2]:
    # p' = c1 + 2 c2 (x - o), p'' = 2 c2
    # int (c1 - 2 c2 o + 2 c2 x)^2 = (c1 - 2 c2 o)^2 + (4 c2^2)/12
    lin = c1 - 2 * c2 * o
    return lin * lin + Fr(1, 3) * c2 * c2 + 4 * c2 * c2


def test_beta_equals_integral_definition(orc):
    rng = np.random.default_rng(11)
    for _ in range(200):
        ints = rng.integers(-50, 50, size=5)
        f5 = [Fr(int(v), 16) for v in ints]
        _, _, beta = orc.flags5([float(v) for v in f5], 1e-6, want_beta=True)
        for k in range(3):
            exact = _beta_k(f5, k)
            assert abs(beta[k] - float(exact)) <= 8 * EPS64 * max(1.0, float(exact)), (f5, k)


def test_flags_linear_and_constant_data_keep_every_stencil(orc):
    for f5 in ([0, 0, 0, 0, 0], [1, 2, 3, 4, 5], [0.3, 0.1, -0.1, -0.3, -0.5]):
        d, chi = orc.flags5(f5, 1e-12)
        assert list(d) == [1, 1, 1]
        assert np.allclose(chi, 1.0 / 3.0, rtol=0, atol=1e-12)


@pytest.mark.parametrize("f5,expect", [
    ([0, 0, 0, 1, 1], [1, 0, 0]),   # jump between i and i+1: only S0 = {i-2..i} is smooth
    ([1, 1, 0, 0, 0], [0, 0, 1]),   # jump between i-1 and i: only S2 is smooth
    ([0, 0, 1, 1, 1], [0, 0, 1]),   # jump between i-1 and i
    ([0, 1, 1, 1, 1], [0, 1, 1]),   # jump between i-2 and i-1: S1, S2 smooth
    ([1, 1, 1, 1, 0], [1, 1, 0]),   # jump between i+1 and i+2: S0, S1 smooth
])
def test_flags_isolated_step(orc, f5, expect):
    d, chi = orc.flags5(f5, (1 / 200) ** 3)
    assert list(d) == expect
    assert abs(chi.sum() - 1.0) < 1e-14


def test_smooth_data_keeps_every_stencil(orc):
    """Remark 2: on smooth data with eps = dx^3, no stencil is cut (the two-mode advection wave,
    N >= 100)."""
    for seed in range(6):
        for n in (100, 200):
            pr = W.advection(seed, n)
            cfg = orc.Config(orc.ADV1D, n, x0=-1.0, x1=1.0)
            _, ex = orc.rhs(cfg, pr.U0, want_faces=True)
            assert np.all(ex["masks_x"] == 0), (seed, n)
            assert np.all(ex["flags_x"] == 0x3F)


# ------------------------------------------------------------------------------- accuracy pins
def test_polynomial_exactness_degree_7(orc):
    """With every stencil kept, point values of a degree-7 polynomial give dU/dt = -p'(x) exactly
    (Table 2 row 0 is exact for the cell-average primitive of degree <= 6; the degree-7 error is the
    same constant at both faces and cancels)."""
    rng = np.random.default_rng(5)
    n = 64
    cfg = orc.Config(orc.ADV1D, n, x0=0.0, x1=1.0, bc_x=orc.OUTFLOW)
    x = W.cell_centres(0.0, 1.0, n)
    for _ in range(5):
        c = rng.uniform(-1, 1, 8)
        z = x - 0.5
        p = sum(c[k] * z ** k for k in range(8))
        dp = sum(k * c[k] * z ** (k - 1) for k in range(1, 8))
        out, ex = orc.rhs(cfg, p[None, None, :], want_faces=True)
        inner = slice(8, n - 8)
        assert np.all(ex["masks_x"][0, 8:n - 7] == 0)
        err = np.abs(out[0, 0, inner] + dp[inner]).max()
        assert err < 2e-11, err


def fourier_prediction(pr, nsteps, coeffs):
    """Exact discrete solution of the linear scheme (row 0 on the '+' side, a = 1) under SSP-RK3:
    each Fourier mode e^{ikx} is multiplied per step by G(z) = 1 + z + z^2/2 + z^3/6 with
    z = dt * lambda(k), lambda(k) = -(1/dx) (sum_l a_l e^{ikl dx}) (1 - e^{-ik dx})."""
    dx, dt = pr.dx, pr.dt
    x = W.cell_centres(pr.x0, pr.x1, pr.nx)
    phi = pr.meta["phi"]

    def mode(k):
        A = sum(coeffs[l + 3] * np.exp(1j * k * l * dx) for l in range(-3, 4))
        lam = -(1.0 / dx) * A * (1.0 - np.exp(-1j * k * dx))
        z = dt * lam
        return (1 + z + z * z / 2 + z ** 3 / 6) ** nsteps

    return (np.imag(mode(math.pi) * np.exp(1j * math.pi * x))
            + 0.3 * np.imag(mode(3 * math.pi) * np.exp(1j * (3 * math.pi * x + phi))))


@pytest.mark.parametrize("n", [100, 200])
def test_advection_matches_fourier_closed_form(orc, n):
    from conftest import read_golden
    row0 = [float(Fr(t)) for t in read_golden("table2.txt")[0]]
    pr = W.advection(7, n)
    cfg = orc.Config(orc.ADV1D, n, x0=-1.0, x1=1.0)
    U = orc.run(cfg, pr.U0, pr.nsteps, dt=pr.dt)
    pred = fourier_prediction(pr, pr.nsteps, row0)
    assert np.abs(U[0, 0] - pred).max() < 1e-12
    exact = W.advection_exact(pr, pr.nsteps * pr.dt)
    l1 = np.abs(U[0, 0] - exact).mean()
    assert 1e-8 < l1 < 1e-4


def _order(e):
    return [math.log2(e[k] / e[k + 1]) for k in range(len(e) - 1)]


def test_rhs_convergence_order_teno7x_and_teno5(orc):
    errs7, errs5 = [], []
    for n in (50, 100, 200):
        pr = W.advection(2, n)
        x = W.cell_centres(-1.0, 1.0, n)
        phi = pr.meta["phi"]
        exact = -(math.pi * np.cos(math.pi * x) + 0.9 * math.pi * np.cos(3 * math.pi * x + phi))
        c7 = orc.Config(orc.ADV1D, n, x0=-1.0, x1=1.0)
        c5 = orc.Config(orc.ADV1D, n, x0=-1.0, x1=1.0, scheme=orc.TENO5, eps=(2.0 / n) ** 3)
        errs7.append(np.abs(orc.rhs(c7, pr.U0)[0, 0] - exact).max())
        errs5.append(np.abs(orc.rhs(c5, pr.U0)[0, 0] - exact).max())
    o7, o5 = _order(errs7), _order(errs5)
    assert min(o7) > 6.5, o7
    assert 4.5 < min(o5) and max(o5) < 5.6, o5


def test_trajectory_order_seven_with_refined_time_step(orc):
    """Two-mode advection wave to t = 2 with dt = 0.2 dx (dx/0.04)^(4/3), so that the RK3 error
    falls like dx^7 and the spatial order shows."""
    errs = []
    for n in (50, 100, 200):
        pr = W.advection(4, n)
        dx = pr.dx
        dt0 = 0.2 * dx * (dx / 0.04) ** (4.0 / 3.0)
        nsteps = int(math.ceil(2.0 / dt0))
        dt = 2.0 / nsteps
        cfg = orc.Config(orc.ADV1D, n, x0=-1.0, x1=1.0)
        U = orc.run(cfg, pr.U0, nsteps, dt=dt)
        errs.append(np.abs(U[0, 0] - W.advection_exact(pr, 2.0)).mean())
    o = _order(errs)
    assert min(o) > 6.3, (errs, o)


# ---------------------------------------------------------------------------- structural pins
def _euler2d_state(seed, nx, ny):
    rng = np.random.default_rng(seed)
    rho = 1.0 + 0.3 * rng.random((ny, nx))
    u = 0.5 * rng.standard_normal((ny, nx))
    v = 0.5 * rng.standard_normal((ny, nx))
    p = 1.0 + 0.3 * rng.random((ny, nx))
    return W.conserved_2d(rho, u, v, p)


def test_conservation_periodic(orc):
    U = _euler2d_state(1, 24, 20)
    cfg = orc.Config(orc.EULER2D, 24, 20)
    out = orc.rhs(cfg, U)
    scale = np.abs(out).max()
    assert np.abs(out.sum(axis=(1, 2))).max() < 1e-12 * scale * out[0].size
    U1 = orc.run(cfg, U, 5, cfl=0.5)
    tot0, tot1 = U.sum(axis=(1, 2)), U1.sum(axis=(1, 2))
    assert np.abs(tot1 - tot0).max() < 1e-12 * np.abs(tot0).max()


@pytest.mark.parametrize("sys", [1, 2])
@pytest.mark.parametrize("bc", [0, 1])
def test_free_stream_is_exactly_preserved(orc, sys, bc):
    if sys == 2:
        cfg = orc.Config(orc.EULER2D, 12, 10, bc_x=bc, bc_y=bc)
        U = W.conserved_2d(np.full((10, 12), 0.7), np.full((10, 12), 0.3), np.full((10, 12), -0.2),
                           np.full((10, 12), 1.1))
    else:
        cfg = orc.Config(orc.EULER1D, 20, bc_x=bc)
        U = W.conserved_1d(np.full(20, 0.7), np.full(20, 0.3), np.full(20, 1.1))
    assert np.all(orc.rhs(cfg, U) == 0.0)


def test_mirror_symmetry_euler1d(orc):
    """Reflecting x -> -x and u -> -u reflects the operator (tests the mirrored '-' side)."""
    rng = np.random.default_rng(9)
    n = 64
    rho = 1 + 0.5 * (np.arange(n) > 30) + 0.1 * rng.random(n)
    u = 0.3 * rng.standard_normal(n)
    p = 1 + 0.8 * (np.arange(n) < 20) + 0.1 * rng.random(n)
    U = W.conserved_1d(rho, u, p)
    Um = U[:, :, ::-1].copy()
    Um[1] *= -1
    cfg = orc.Config(orc.EULER1D, n, bc_x=orc.PERIODIC)
    a = orc.rhs(cfg, U)
    b = orc.rhs(cfg, Um)
    b = b[:, :, ::-1].copy()
    b[1] *= -1
    assert np.abs(a - b).max() <= 1e-12 * np.abs(a).max()


def test_transpose_commutes(orc):
    """Swapping x <-> y (and u <-> v) commutes with the operator up to the summation order of the
    momentum components inside the projection L U."""
    U = _euler2d_state(4, 16, 16)
    UT = np.stack([U[0].T, U[2].T, U[1].T, U[3].T])
    cfg = orc.Config(orc.EULER2D, 16, 16)
    a = orc.rhs(cfg, U)
    b = orc.rhs(cfg, UT)
    bT = np.stack([b[0].T, b[2].T, b[1].T, b[3].T])
    assert np.abs(a - bT).max() <= 64 * EPS64 * np.abs(a).max()


def test_y_uniform_2d_state_reduces_to_1d(orc):
    rng = np.random.default_rng(2)
    n, ny = 48, 6
    rho = 1 + 0.4 * (np.arange(n) > 20) + 0.05 * rng.random(n)
    u = 0.2 * rng.standard_normal(n)
    p = 1 + 0.05 * rng.random(n)
    U1 = W.conserved_1d(rho, u, p)
    U2 = W.conserved_2d(np.tile(rho, (ny, 1)), np.tile(u, (ny, 1)), np.zeros((ny, n)), np.tile(p, (ny, 1)))
    c1 = orc.Config(orc.EULER1D, n, bc_x=orc.OUTFLOW)
    c2 = orc.Config(orc.EULER2D, n, ny, bc_x=orc.OUTFLOW, y1=ny / n)
    r1 = orc.rhs(c1, U1)
    r2 = orc.rhs(c2, U2)
    assert np.all(r2[2] == 0.0)                       # no transverse momentum change
    for j in range(ny):
        for a, b in ((0, 0), (1, 1), (2, 3)):
            assert np.abs(r2[b, j] - r1[a, 0]).max() <= 1e-12 * np.abs(r1[a]).max()


def _euler_flux_x(U, g=1.4):
    rho, mx, my, E = U
    u, v = mx / rho, my / rho
    p = (g - 1) * (E - 0.5 * rho * (u * u + v * v))
    return np.array([mx, mx * u + p, my * u, u * (E + p)])


def _jacobian(fun, U):
    J = np.zeros((4, 4))
    for k in range(4):
        d = np.zeros(4, dtype=complex)
        d[k] = 1e-30j
        J[:, k] = np.imag(fun(U.astype(complex) + d)) / 1e-30
    return J


def test_roe_average_and_eigenvectors(orc):
    """L R = I; L A(U~) R = diag(u-c, u, u, u+c); and the Roe property
    A(U~)(U_R - U_L) = F(U_R) - F(U_L) with A the exact Euler flux Jacobian."""
    g = 1.4
    rng = np.random.default_rng(8)
    cfg = orc.Config(orc.EULER2D, 4, 4)
    for _ in range(20):
        prim = [(rng.uniform(0.2, 2), rng.normal(0, 1), rng.normal(0, 1), rng.uniform(0.2, 2)) for _ in range(2)]
        UL, UR = [W.conserved_2d(*[np.array(v) for v in pr]) for pr in prim]
        UL, UR = UL.reshape(4), UR.reshape(4)
        Lm, Rm = orc.eigen(cfg, 0, UL, UR)
        assert np.abs(Lm @ Rm - np.eye(4)).max() < 1e-12
        u, v = Rm[1, 1], Rm[2, 1]
        H = 0.5 * (Rm[3, 0] + Rm[3, 3])
        c = 0.5 * (Rm[1, 3] - Rm[1, 0])
        E = (H + 0.5 * (g - 1) * (u * u + v * v)) / g
        Uroe = np.array([1.0, u, v, E])
        A = _jacobian(_euler_flux_x, Uroe)
        assert np.abs(A @ (UR - UL) - (_euler_flux_x(UR) - _euler_flux_x(UL))).max() < 1e-11
        lam = np.diag([u - c, u, u, u + c])
        assert np.abs(Lm @ A @ Rm - lam).max() < 1e-11 * (1 + abs(u) + c)
        assert abs(c * c - (g - 1) * (H - 0.5 * (u * u + v * v))) < 1e-12
        # physical flux of the oracle equals the textbook flux
        assert np.abs(orc.phys_flux(cfg, 0, UL) - _euler_flux_x(UL)).max() < 1e-14 * np.abs(UL).max()


def test_euler_rhs_converges_to_minus_flux_divergence(orc):
    """Smooth 2D state: dU/dt -> -(dF/dx + dG/dy) at high order (pins the fluxes, the EOS and the
    characteristic round trip)."""
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
        U = W.conserved_2d(*prim(X, Y))
        cfg = orc.Config(orc.EULER2D, n, n)
        out = orc.rhs(cfg, U)
        errs.append(np.abs(out + dF + dG).max())
    o = _order(errs)
    assert errs[-1] < 1e-6 and min(o) > 5.0, (errs, o)


# ------------------------------------------------------------------------ no-crossing, brute force
def _support(t2, m):
    return [l - 3 for l in range(7) if t2[m, l] != 0.0]


@pytest.mark.parametrize("n", [32, 256])
@pytest.mark.parametrize("speed", [1.0, -1.0])
def test_no_selected_stencil_crosses_an_isolated_step(orc, n, speed):
    """A smooth O(1) background plus one jump of height 1: no selected reconstruction contains
    cells on both sides of the jump (section "Higher-order spatial reconstructions": reconstructions
    crossing discontinuities are avoided). a = +1 exercises the '+' side, a = -1 the mirrored side."""
    t2, _ = orc.tables()
    rng = np.random.default_rng(n)
    cfg = orc.Config(orc.ADV1D, n, adv_speed=speed)
    x = W.cell_centres(0.0, 1.0, n)
    bad = 0
    for trial in range(120):
        J = int(rng.integers(8, n - 8))            # jump between cells J-1 and J
        g = 0.5 * np.sin(2 * np.pi * (x + rng.uniform())) * rng.uniform(0.2, 1.0)
        u = g + (np.arange(n) >= J) * rng.choice([-1.0, 1.0])
        _, ex = orc.rhs(cfg, u[None, None, :], want_faces=True)
        masks = ex["masks_x"][0]
        for f in range(J - 5, J + 6):
            i = f - 1
            if speed > 0:
                m = int(masks[f] & 0xF)
                cells = [i + l for l in _support(t2, m)]
            else:
                m = int((masks[f] >> 4) & 0xF)
                cells = [i + 1 - l for l in _support(t2, m)]
            if min(cells) <= J - 1 and max(cells) >= J:
                bad += 1
    assert bad == 0


def test_selection_invariants_on_a_shocked_euler_state(orc):
    pr = W.euler2d(3, n=48)
    cfg = orc.Config(orc.EULER2D, 48, 48)
    _, ex = orc.rhs(cfg, pr.U0, want_faces=True)
    for key in ("masks_x", "masks_y"):
        m = ex[key].astype(np.int64)
        for s in range(4):
            for side in range(2):
                code = (m >> (8 * s + 4 * side)) & 0xF
                assert code.max() <= 12
    for key in ("flags_x", "flags_y"):
        f = ex[key].astype(np.int64)
        for s in range(4):
            for side in range(2):
                central = (f >> (6 * s + 3 * side)) & 0x7
                assert np.all(central != 0)
    for key in ("chi_x", "chi_y"):
        chi = ex[key].reshape(-1, 4, 2, 3)
        assert np.abs(chi.sum(axis=-1) - 1.0).max() < 1e-14
    assert (ex["masks_x"] != 0).any()                 # the quadrant interfaces do cut stencils


def test_sod_shock_tube_positive_and_non_oscillatory(orc):
    pr = W.shock_tube("sod", 200)
    cfg = orc.Config(orc.EULER1D, 200, bc_x=orc.OUTFLOW)
    U = pr.U0.copy()
    t, steps = 0.0, 0
    while t < 0.2 - 1e-14:
        a, den = orc.wave_speeds(cfg, U)
        dt = min(0.6 / den, 0.2 - t)
        U = orc.run(cfg, U, 1, dt=dt)
        t += dt
        steps += 1
    rho = U[0, 0]
    assert rho.min() > 0.125 - 2e-3 and rho.max() < 1.0 + 2e-3
    tv = np.abs(np.diff(rho)).sum()
    assert tv < 0.875 * 1.02, tv


def test_window_evaluation_matches_the_full_domain(orc):
    """The sampled full-size parity check evaluates one cell on a 17 x 17 window (outflow padding)
    with the domain's Lax-Friedrichs constants: the cell depends only on cells within five along
    its row and column, so the window reproduces the full periodic operator."""
    pr = W.euler2d(4, n=256)
    cfg = orc.Config(orc.EULER2D, 256, 256, 0.0, 1.0, 0.0, 1.0)
    full = orc.rhs(cfg, pr.U0)
    alpha, _ = orc.wave_speeds(cfg, pr.U0)
    hw, w = 8, 17
    wcfg = orc.Config(orc.EULER2D, w, w, 0.0, w * pr.dx, 0.0, w * pr.dy, orc.OUTFLOW, orc.OUTFLOW)
    rng = np.random.default_rng(5)
    pts = [tuple(p) for p in rng.integers(0, 256, size=(150, 2))] + [(0, 0), (255, 255), (127, 128), (128, 0)]
    for (j, i) in pts:
        rows = np.arange(j - hw, j + hw + 1) % 256
        cols = np.arange(i - hw, i + hw + 1) % 256
        Uw = np.ascontiguousarray(pr.U0[:, rows][:, :, cols])
        o = orc.rhs(wcfg, Uw, alpha=alpha)[:, hw, hw]
        assert np.array_equal(o, full[:, j, i]), (j, i, o - full[:, j, i])
