"""2D Euler on the GPU against an exact solution: the isentropic vortex translating with a uniform
stream on a periodic domain, run to exactly t = 1 (the last step cut by the end time). The GPU
equals the oracle at N = 64 and converges to the exact solution at order 7 (with the time step
refined so that SSP-RK3's error falls faster than the spatial one) as N grows."""
import numpy as np
import pytest
import torch

from oracle import oracle as O
from paper_1808_00037_amd import workloads as W

from gpu_common import oracle_cfg, solver_for

pytestmark = pytest.mark.gpu


def _gpu_to(pr, t_end):
    sv = solver_for(pr)
    U = torch.from_numpy(pr.U0.copy()).cuda()
    sv.set_time(0.0, t_end)
    # (dt = cfl / ((|u| + c)/dx + (|v| + c)/dy) >= cfl dx / 6 on these data; steps beyond t_end
    # stand still)
    sv.run(U, int(t_end * 6.0 * pr.nx / (pr.x1 - pr.x0) / pr.cfl) + 10, graph=True)
    sv.poll()
    assert sv.time() == t_end
    return U.cpu().numpy()


def _errors(refine_dt):
    errs = []
    for n in (128, 256, 512):
        # [0, 20]^2, so that the periodic data are smooth to rounding; refine_dt: CFL 0.5 (128/n)^(4/3),
        # so that dt ~ dx^(7/3) and SSP-RK3's dt^3 error falls like dx^7
        pr = W.vortex(n, cfl=0.5 * (128.0 / n) ** (4.0 / 3.0) if refine_dt else 0.5, length=20.0)
        U = _gpu_to(pr, 1.0)
        x = W.cell_centres(0.0, 20.0, n)
        X, Y = np.meshgrid(x, x)
        rho = W.vortex_exact_primitive(X, Y, 1.0, length=20.0)[0]
        errs.append(np.mean(np.abs(U[0] - rho)))
    orders = np.log2(np.array(errs[:-1]) / np.array(errs[1:]))
    print("[case] vortex refine_dt", refine_dt, "L1(rho)", errs, "orders", orders, flush=True)
    return errs, orders


def test_vortex_converges_to_the_exact_solution():
    # at CFL 0.5 the spatial error dominates at first, then SSP-RK3's third order takes over
    errs, orders = _errors(False)
    assert orders[0] > 5.0 and orders[1] > 2.8, (errs, orders)
    # with the time step refined the high spatial order shows at every refinement
    errs, orders = _errors(True)
    assert np.all(orders > 6.3), (errs, orders)      # (measured 6.73, 6.93)


def test_vortex_equals_the_oracle():
    pr = W.vortex(64)
    cfg = oracle_cfg(pr)
    _, rec = O.run(cfg, pr.U0, 80, cfl=pr.cfl, record=True)
    t, m = 0.0, 0
    while t + rec["dt"][m] < 1.0:
        t += rec["dt"][m]
        m += 1
    Uo = O.run(cfg, O.run(cfg, pr.U0, m, cfl=pr.cfl), 1, dt=1.0 - t)
    Ug = _gpu_to(pr, 1.0)
    err = np.abs(Ug - Uo).max() / np.abs(Uo).max()
    assert err < 1e-11, err
