"""Oracle pins for the inviscid Burgers equation (section "One-dimensional inviscid Burgers
equation"): u_t + (u^2/2)_x = 0 on [0, 2), periodic, u0 = 1/2 + sin(pi x), global Lax-Friedrichs
splitting with alpha = max |u|.

Pins: the semi-discrete operator against the exact -u u_x with its order of accuracy; the smooth
solution at t = 0.5/pi against the characteristic solution; the Rankine-Hugoniot speed of a shock;
boundedness and conservation after the shock forms (t = 1.5/pi).
"""
import math

import numpy as np
import pytest

from oracle import oracle as O
from paper_1808_00037_amd import workloads as W


def _cfg(pr, **kw):
    return O.Config(O.BURGERS1D, pr.nx, 1, pr.x0, pr.x1, 0.0, 1.0, pr.bc_x, pr.bc_x, **kw)


def test_rhs_is_minus_u_ux_to_seventh_order():
    errs = []
    for n in (40, 80, 160):
        pr = W.burgers(n, shift=0.3)
        x = W.cell_centres(0.0, 2.0, n)
        u = W.burgers_wave(x, 0.3)
        exact = -u * np.pi * np.cos(np.pi * (x - 0.3))
        r = O.rhs(_cfg(pr), pr.U0)[0, 0]
        errs.append(np.abs(r - exact).max())
    orders = [math.log2(errs[k] / errs[k + 1]) for k in range(2)]
    assert min(orders) > 6.5, (errs, orders)
    assert errs[-1] < 1e-9


def test_smooth_solution_matches_characteristics():
    """Before the shock (t = 0.5/pi) the RK3 trajectory converges to u = u0(x - u t). With dt
    refined like dx^(7/3) the error falls by about 2^7 per halving once asymptotic (N >= 160), and
    no stencil is ever cut: the linear seventh-order scheme is recovered."""
    errs = []
    for n in (160, 320):
        pr = W.burgers(n)
        t_end = 0.5 / math.pi
        dt0 = 0.2 * pr.dx / 1.5 * (pr.dx / (2.0 / 40)) ** (4.0 / 3.0)
        nsteps = int(math.ceil(t_end / dt0))
        dt = t_end / nsteps
        U, rec = O.run(_cfg(pr), pr.U0, nsteps, dt=dt, record=True)
        assert not np.any(rec["masks"]), n
        errs.append(np.abs(U[0, 0] - W.burgers_exact(pr, t_end)).max())
    assert errs[1] < 1e-9, errs
    assert math.log2(errs[0] / errs[1]) > 6.8, errs


def test_shock_moves_at_the_rankine_hugoniot_speed():
    """Riemann data u = 1 | 0 (outflow): a shock of speed (1 + 0)/2; the discrete profile's
    mid-crossing follows x0 + t/2 to within a cell."""
    n = 400
    pr = W.burgers(n)
    pr.bc_x = O.OUTFLOW
    x = W.cell_centres(0.0, 2.0, n)
    U = np.where(x < 0.5, 1.0, 0.0)[None, None, :]
    cfg = _cfg(pr)
    dt = 0.4 * pr.dx
    nsteps = int(round(1.0 / dt))
    U = O.run(cfg, U, nsteps, dt=dt)[0, 0]
    t = nsteps * dt
    k = int(np.argmax(U < 0.5))
    xs = x[k - 1] + (U[k - 1] - 0.5) / (U[k - 1] - U[k]) * pr.dx
    assert abs(xs - (0.5 + 0.5 * t)) < pr.dx, (xs, 0.5 + 0.5 * t)
    # the shock stays sharp: the transition from 0.95 to 0.05 takes a few cells
    width = np.sum((U > 0.05) & (U < 0.95))
    assert width <= 4, width


def test_after_the_shock_forms_solution_stays_bounded_and_conservative():
    n = 160
    pr = W.burgers(n)
    t_end = 1.5 / math.pi
    dt = 0.4 * pr.dx / 1.5
    nsteps = int(math.ceil(t_end / dt))
    dt = t_end / nsteps
    U = O.run(_cfg(pr), pr.U0, nsteps, dt=dt)[0, 0]
    assert abs(U.sum() - pr.U0.sum()) < 1e-12 * n
    # the exact solution stays within the initial range [-1/2, 3/2]; allow a small overshoot
    assert U.min() > -0.5 - 1e-3 and U.max() < 1.5 + 1e-3, (U.min(), U.max())
