"""The paper's one-dimensional Euler problems (section "One dimensional Euler equations": Sod and
Lax shock tubes, the Shu-Osher and Titarev-Toro shock/entropy-wave interactions), its Burgers case and
its linear-advection data u1, u2, u3, run on the GPU to the paper's end times with its CFL number
(the step that would pass the end time is cut to land on it), against the oracle run step for step.

The paper's reference solutions are figures only, so these runs are pinned by oracle parity over the
whole trajectory, positivity, and conservation while no wave has reached an outflow boundary.
"""
import math

import numpy as np
import pytest
import torch

from oracle import oracle as O
from paper_1808_00037_amd import workloads as W

from gpu_common import oracle_cfg, solver_for

pytestmark = pytest.mark.gpu


def _steps_to(pr, t_end):
    """Step count reaching about t_end with the CFL rule (the oracle's dt of the first step)."""
    _, rec = O.run(oracle_cfg(pr), pr.U0, 1, cfl=pr.cfl, record=True)
    return max(1, int(round(t_end / rec["dt"][0])))


def _run_to(pr, t_end):
    """The oracle and the GPU advanced to exactly t_end with the CFL rule: whole steps while they end
    before t_end, then one step of the remaining time. Returns (oracle state, GPU state, steps)."""
    cfg = oracle_cfg(pr)
    n = 2 * _steps_to(pr, t_end) + 10
    _, rec = O.run(cfg, pr.U0, n, cfl=pr.cfl, record=True)
    t, m = 0.0, 0
    while t + rec["dt"][m] < t_end:
        t += rec["dt"][m]
        m += 1
    assert m < n - 1
    # the end time must not sit within rounding of a step boundary (the two sides' dt agree to ~1e-14)
    assert min(t_end - t, t + rec["dt"][m] - t_end) > 1e-9 * t_end
    Uo = O.run(cfg, pr.U0, m, cfl=pr.cfl) if m else pr.U0.copy()
    Uo = O.run(cfg, Uo, 1, dt=t_end - t)
    sv = solver_for(pr)
    U = torch.from_numpy(pr.U0.copy()).cuda()
    sv.set_time(0.0, t_end)
    sv.run(U, m + 5, graph=True)
    sv.poll()
    assert sv.time() == t_end
    return Uo, U.cpu().numpy(), m + 1


def _euler_flux(U):
    rho, m, E = U
    u = m / rho
    p = 0.4 * (E - 0.5 * rho * u * u)
    return np.array([m, m * u + p, u * (E + p)])


@pytest.mark.parametrize("kind", ["sod", "lax", "shu_osher", "titarev_toro"])
def test_shock_tube_runs(kind):
    pr = W.shock_tube(kind, n=400 if kind == "titarev_toro" else 200)
    t_end = pr.meta["t_end"]
    Uo, Ug, nsteps = _run_to(pr, t_end)
    print("[case]", kind, nsteps, "steps to t =", t_end, flush=True)
    err = np.abs(Ug - Uo).max() / np.abs(Uo).max()
    assert err < 1e-10, err
    rho, m, E = Ug[0, 0], Ug[1, 0], Ug[2, 0]
    p = 0.4 * (E - 0.5 * m * m / rho)
    assert rho.min() > 0 and p.min() > 0
    if kind in ("sod", "lax"):
        # no wave reaches either boundary before the end time: the boundary cells keep their states
        # up to the schemes' small tails (Lax's rarefaction head comes within a few cells of the left
        # boundary by t = 0.14), so the totals change by the boundary fluxes, sum(U) dx grows by
        # T (F(U_left) - F(U_right)), up to T times the boundary fluxes' drift
        drift = np.abs(Ug[:, 0, [0, -1]] - pr.U0[:, 0, [0, -1]]).max() / np.abs(pr.U0[:, 0, [0, -1]]).max()
        print("[case]", kind, "boundary drift", drift, flush=True)
        assert drift < (1e-12 if kind == "sod" else 1e-8), drift     # (measured 4e-15 and 1.1e-9)
        flux_in = t_end * (_euler_flux(pr.U0[:, 0, 0]) - _euler_flux(pr.U0[:, 0, -1]))
        dflux = t_end * (np.abs(_euler_flux(Ug[:, 0, 0]) - _euler_flux(pr.U0[:, 0, 0])) +
                         np.abs(_euler_flux(Ug[:, 0, -1]) - _euler_flux(pr.U0[:, 0, -1])))
        change = (Ug.sum(axis=(1, 2)) - pr.U0.sum(axis=(1, 2))) * pr.dx
        scale = np.maximum(np.abs(pr.U0).sum(axis=(1, 2)) * pr.dx, np.abs(flux_in))
        assert np.all(np.abs(change - flux_in) <= 1e-11 * scale + dflux), (change, flux_in, dflux)


def test_burgers_to_after_the_shock():
    pr = W.burgers(160, cfl=0.6)
    Uo, Ug, _ = _run_to(pr, 1.5 / math.pi)
    assert np.abs(Ug - Uo).max() < 1e-10
    assert abs(Ug.sum() - pr.U0.sum()) < 1e-12 * pr.nx


@pytest.mark.parametrize("kind", ["u1", "u2", "u3"])
def test_paper_advection_one_period(kind):
    """One period at N = 200, CFL 0.2: the GPU equals the oracle; the smooth data come back to within
    the RK3-limited error, the four-wave data stay within 1 % of their range (no oscillations)."""
    pr = W.paper_advection(kind, 200)
    print("[case] advection", kind, pr.nsteps, "steps", flush=True)
    Uo = O.run(oracle_cfg(pr), pr.U0, pr.nsteps, dt=pr.dt)
    sv = solver_for(pr)
    U = torch.from_numpy(pr.U0.copy()).cuda()
    sv.run(U, pr.nsteps, dt=pr.dt, graph=True)
    sv.poll()
    Ug = U.cpu().numpy()[0, 0]
    assert np.abs(Ug - Uo[0, 0]).max() < 1e-12
    err = np.abs(Ug - pr.U0[0, 0])          # after whole periods the exact solution is the data
    if kind == "u1":
        assert err.max() < 1e-4, err.max()
    elif kind == "u2":
        assert err.max() < 5e-6, err.max()
    else:
        assert -0.01 < Ug.min() and Ug.max() < 1.01, (Ug.min(), Ug.max())


def test_sod_on_fine_grids_approaches_the_exact_solution():
    # the GPU at N = 1024, 2048, 4096 against the exact Riemann solution at t = 0.2: the L1 error of
    # the density falls at about first order (discontinuities), and is small
    from test_oracle_exact_riemann import CASES, exact
    wl, wr = CASES["sod"]
    errs = []
    for n in (1024, 2048, 4096):
        pr = W.shock_tube("sod", n=n)
        sv = solver_for(pr)
        U = torch.from_numpy(pr.U0.copy()).cuda()
        sv.set_time(0.0, 0.2)
        sv.run(U, int(0.2 * 3.0 * n / pr.cfl) + 10, graph=True)     # (|u| + c < 3 on these data)
        sv.poll()
        assert sv.time() == 0.2
        x = (np.arange(n) + 0.5) / n
        ref = exact(wl, wr, (x - 0.5) / 0.2)
        errs.append(np.mean(np.abs(U.cpu().numpy()[0, 0] - ref[0])))
    print("[case] sod L1(rho)", errs, flush=True)
    # (measured 5.2e-4, 2.9e-4, 1.7e-4)
    assert errs[1] < 0.8 * errs[0] and errs[2] < 0.8 * errs[1] and errs[2] < 2e-4, errs
