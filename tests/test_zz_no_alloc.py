"""teno_step_noalloc, the entry point for callers that cannot allocate device memory, against
teno_step (the same SSP-RK3 step through a context): two calls in a row, the second on a smaller
problem (the shared fixed scratch keeps the first call's contents), bitwise equal states, the same
dt and status; a problem beyond the fixed scratch is refused before anything runs."""
import ctypes

import numpy as np
import pytest
import torch

from paper_1808_00037_amd import teno as T
from paper_1808_00037_amd import workloads as W

from gpu_common import solver_for

pytestmark = pytest.mark.gpu


def _reference_step(pr, **opts):
    sv = solver_for(pr, **opts)
    U = torch.from_numpy(pr.U0.copy()).cuda()
    sv.step(U)
    sv.poll()
    return sv, U, sv.last_dt()


def _noalloc_step(sv, pr, dt=0.0):
    U = torch.from_numpy(pr.U0.copy()).cuda()
    status = torch.full((1,), 99, dtype=torch.int32, device="cuda")
    dt_out = torch.zeros(1, dtype=torch.float64, device="cuda")
    code = T.lib().teno_step_noalloc(ctypes.byref(sv.grid), ctypes.byref(sv.opts), T._ptr(U), float(dt),
                                    T._stream(), T._ptr(status), T._ptr(dt_out))
    assert code == 0, code
    torch.cuda.synchronize()
    return U, int(status.item()), float(dt_out.item())


def test_noalloc_step_equals_the_context_step_twice_in_a_row():
    for pr in (W.euler2d(71, n=300, ny=200), W.euler2d(72, n=100, ny=60)):     # the second is smaller
        print("[case] no-allocation step", pr.nx, pr.ny, flush=True)
        sv, Uref, dt_ref = _reference_step(pr)
        U, st, dt = _noalloc_step(sv, pr)
        assert st == 0
        assert dt == dt_ref
        assert torch.equal(U, Uref)


def test_noalloc_step_one_dimensional_and_options():
    for pr, opts in ((W.euler1d(73, n=4096), {}), (W.euler1d(74, n=500), dict(scheme=T.TENO5, eps=1e-6)),
                     (W.euler2d(75, n=64, ny=48), dict(characteristic=0, q=4))):
        print("[case] no-allocation step", pr.name, pr.nx, pr.ny, opts, flush=True)
        sv, Uref, dt_ref = _reference_step(pr, **opts)
        U, st, dt = _noalloc_step(sv, pr)
        assert st == 0 and dt == dt_ref
        assert torch.equal(U, Uref)
        # a fixed dt is taken as given
        sv2, Uref2, _ = _reference_step(pr, **opts)
        U2 = torch.from_numpy(pr.U0.copy()).cuda()
        sv2.step(U2, 1e-5)
        sv2.poll()
        U3, st3, dt3 = _noalloc_step(sv, pr, dt=1e-5)
        assert st3 == 0 and dt3 == 1e-5 and torch.equal(U3, U2)


def test_noalloc_step_reports_a_device_failure():
    pr = W.euler1d(76, n=128)
    U0 = pr.U0.copy()
    U0[2, 0, 40] = -1.0                      # negative energy: negative pressure
    pr.U0 = U0
    sv = solver_for(pr)
    U, st, _ = _noalloc_step(sv, pr)
    assert st in (-4, -5)
    # the next call starts from a cleared scratch
    ok = W.euler1d(77, n=128)
    U, st, _ = _noalloc_step(solver_for(ok), ok)
    assert st == 0


def test_noalloc_step_refuses_problems_beyond_its_scratch():
    pr = W.euler2d(78, n=600, ny=400)        # 240k cells: more than the fixed scratch holds
    sv = solver_for(pr)
    U = torch.from_numpy(pr.U0.copy()).cuda()
    before = U.clone()
    code = T.lib().teno_step_noalloc(ctypes.byref(sv.grid), ctypes.byref(sv.opts), T._ptr(U), 0.0, T._stream(),
                                    None, None)
    assert code == -7
    torch.cuda.synchronize()
    assert torch.equal(U, before)
    assert T.lib().teno_step_noalloc(None, ctypes.byref(sv.opts), T._ptr(U), 0.0, None, None, None) == -1
    with pytest.raises(T.TenoError):
        T.step_noalloc(sv.grid, sv.opts, U)
