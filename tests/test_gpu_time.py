"""Runs to an end time: the step that would pass t_end is cut to land on it, later steps leave the
state unchanged, and the result equals the oracle advanced by the same steps."""
import math

import numpy as np
import pytest
import torch

from oracle import oracle as O
from paper_1808_00037_amd import teno as T
from paper_1808_00037_amd import workloads as W

from gpu_common import oracle_cfg, solver_for

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("graph", [False, True], ids=["eager", "graph"])
def test_fixed_dt_run_stops_at_end_time(graph):
    pr = W.advection(4, 200)
    dt = pr.dt
    t_end = 6.85 * dt
    sv = solver_for(pr)
    U = torch.from_numpy(pr.U0.copy()).cuda()
    sv.set_time(0.0, t_end)
    sv.run(U, 10, dt=dt, graph=graph)
    sv.poll()
    assert sv.time() == t_end
    # the oracle: six full steps, then the remainder (time summed in the same order)
    t6 = 0.0
    for _ in range(6):
        t6 += dt
    cfg = oracle_cfg(pr)
    Uo = O.run(cfg, pr.U0, 6, dt=dt)
    Uo = O.run(cfg, Uo, 1, dt=t_end - t6)
    err = np.abs(U.cpu().numpy() - Uo).max() / np.abs(Uo).max()
    assert err < 1e-12, err
    # further steps stand still, bit for bit
    V = U.clone()
    sv.run(U, 3, dt=dt, graph=graph)
    sv.poll()
    assert torch.equal(U, V)
    assert sv.last_dt() == 0.0
    # removing the limit lets the run continue
    sv.set_time(sv.time())
    sv.run(U, 1, dt=dt, graph=graph)
    sv.poll()
    assert not torch.equal(U, V)
    assert sv.time() == t_end + dt


@pytest.mark.parametrize("name", ["sod", "euler2d"])
def test_cfl_run_stops_at_end_time(name):
    if name == "sod":
        pr = W.shock_tube("sod", n=200)
    else:
        pr = W.euler2d(13, n=48, ny=40)
    cfg = oracle_cfg(pr)
    n = 12
    _, rec = O.run(cfg, pr.U0, n, cfl=pr.cfl, record=True)
    times = np.cumsum(rec["dt"])
    m = 8                                    # end inside step m + 1
    t_end = times[m - 1] + 0.37 * rec["dt"][m]
    tm = 0.0
    for k in range(m):
        tm += rec["dt"][k]
    Uo = O.run(cfg, pr.U0, m, cfl=pr.cfl)
    Uo = O.run(cfg, Uo, 1, dt=t_end - tm)
    sv = solver_for(pr)
    U = torch.from_numpy(pr.U0.copy()).cuda()
    sv.set_time(0.0, t_end)
    sv.run(U, n, graph=True)
    sv.poll()
    assert sv.time() == t_end
    err = np.abs(U.cpu().numpy() - Uo).max() / np.abs(Uo).max()
    assert err < 1e-10, err


def test_recorded_run_with_end_time_replays_bitwise():
    pr = W.euler2d(14, n=40, ny=32)
    sv = solver_for(pr)
    U = torch.from_numpy(pr.U0.copy()).cuda()
    sv.run(U.clone(), 3, graph=False)
    t3 = sv.time()
    sv.set_time(0.0, 0.5 * t3)
    rec = sv.run_record(U, 6, 2)
    sv.poll()
    dts = rec["alpha_dt"][:, 24].cpu().numpy()
    assert (dts[:2] > 0).all() and (dts[3:] == 0).all()
    assert sv.time() == 0.5 * t3
    V = torch.from_numpy(pr.U0.copy()).cuda()
    sv.run_replay(V, rec)
    sv.poll()
    assert torch.equal(U, V)
    assert sv.time() == 0.5 * t3            # replays leave the time alone


def test_set_time_rejects_bad_arguments():
    pr = W.advection(1, 50)
    sv = solver_for(pr)
    with pytest.raises(T.TenoError):
        sv.set_time(math.nan, 1.0)
    with pytest.raises(T.TenoError):
        sv.set_time(0.0, math.nan)
    assert sv.time() == 0.0
