"""GPU frozen-selection adjoint vs the oracle and vs central finite differences, through the C ABI.

Oracle side: complex-step directional derivatives of its own frozen operator / trajectory (the
selection, Lax-Friedrichs constants and dt recorded by the oracle itself). GPU side: the reverse-mode
kernels fed the oracle's recording as frozen inputs. Checks: element-wise J^T lam on small grids
(the oracle assembles J column by column), dot-product identities <lam, J d> = <J^T lam, d> on larger
grids and trajectories, the GPU's own record/replay being bitwise reproducible, and central finite
differences of the GPU's frozen trajectory map.
"""
import numpy as np
import pytest
import torch

from oracle import oracle as O
from paper_1808_00037_amd import teno as T
from paper_1808_00037_amd import workloads as W

from gpu_common import oracle_cfg, solver_for, trajectory_census

pytestmark = pytest.mark.gpu


def _case(name):
    if name == "adv":
        pr = W.advection(3, 40)
        U = pr.U0.copy()
        U[0, 0, 18:] += 0.8
        return pr, U
    if name == "bu":
        pr = W.burgers(48, shift=0.2)
        U = pr.U0.copy()
        U[0, 0, 30:] -= 0.7          # a step: some stencils cut
        return pr, U
    if name == "e1o":
        pr = W.euler1d(4, n=30)
        pr.x1 = 1.0
        return pr, pr.U0
    if name == "e1p":
        pr = W.euler1d(5, n=24)
        pr.bc_x = O.PERIODIC
        return pr, pr.U0
    if name == "e2p":
        pr = W.euler2d(6, n=12, ny=10)
        return pr, pr.U0
    if name == "e2o":
        pr = W.euler2d(7, n=10, ny=9)
        pr.bc_x = pr.bc_y = O.OUTFLOW
        return pr, pr.U0
    raise ValueError(name)


def _frozen_inputs(pr, U):
    cfg = oracle_cfg(pr)
    _, ex = O.rhs(cfg, U, want_faces=True)
    masks = ex["masks_x"].reshape(-1)
    if pr.sys == O.EULER2D:
        masks = np.concatenate([masks, ex["masks_y"].reshape(-1)])
    return cfg, ex, masks


@pytest.mark.parametrize("name", ["adv", "bu", "e1o", "e1p", "e2p", "e2o"])
def test_rhs_vjp_elementwise(name):
    pr, U = _case(name)
    print("[case] rhs_vjp", name, flush=True)
    cfg, ex, masks = _frozen_inputs(pr, U)
    my = ex.get("masks_y")
    rng = np.random.default_rng(1)
    lam = rng.standard_normal(U.shape)
    n = U.size
    # oracle: (J^T lam)_i = lam . (J e_i), columns by complex step
    g_orc = np.zeros(n)
    for i in range(n):
        e = np.zeros(n)
        e[i] = 1.0
        g_orc[i] = np.sum(lam * O.rhs_frozen_jvp(cfg, U, e.reshape(U.shape), ex["alpha"], ex["masks_x"], my))
    sv = solver_for(pr)
    g = sv.rhs_vjp(torch.from_numpy(np.ascontiguousarray(U)).cuda(),
                   torch.from_numpy(masks.view(np.int32)).cuda(), torch.from_numpy(ex["alpha"]).cuda(),
                   torch.from_numpy(lam).cuda()).cpu().numpy().reshape(-1)
    sv.poll()
    err = np.abs(g - g_orc).max() / np.abs(g_orc).max()
    assert err < 1e-12, err


def test_rhs_vjp_dot_product_2d():
    pr = W.euler2d(8, n=70, ny=52)
    cfg, ex, masks = _frozen_inputs(pr, pr.U0)
    sv = solver_for(pr)
    rng = np.random.default_rng(2)
    Ug = torch.from_numpy(pr.U0).cuda()
    mg = torch.from_numpy(masks.view(np.int32)).cuda()
    ag = torch.from_numpy(ex["alpha"]).cuda()
    for _ in range(3):
        lam = rng.standard_normal(pr.U0.shape)
        d = W.random_directions(int(rng.integers(1 << 30)), pr.U0, 1)[0]
        jd = O.rhs_frozen_jvp(cfg, pr.U0, d, ex["alpha"], ex["masks_x"], ex["masks_y"])
        g = sv.rhs_vjp(Ug, mg, ag, torch.from_numpy(lam).cuda()).cpu().numpy()
        a, b = np.sum(lam * jd), np.sum(g * d)
        scale = np.sum(np.abs(lam * jd))
        assert abs(a - b) <= 1e-12 * scale, (a, b)
    sv.poll()


def _gpu_recording_from_oracle(rec):
    n = len(rec["dt"])
    ad = np.concatenate([rec["alpha"].reshape(n, 24), rec["dt"][:, None]], axis=1)
    return (torch.from_numpy(np.ascontiguousarray(rec["masks"]).view(np.int32)).cuda(),
            torch.from_numpy(np.ascontiguousarray(ad)).cuda())


@pytest.mark.parametrize("sys", ["e1", "e2"])
def test_trajectory_vjp_dot_product(sys):
    if sys == "e1":
        pr = W.euler1d(9, n=200)
        nsteps, ck = 8, 3
    else:
        pr = W.euler2d(9, n=40, ny=32)
        nsteps, ck = 6, 4
    cfg = oracle_cfg(pr)
    _, rec = O.run(cfg, pr.U0, nsteps, cfl=pr.cfl, record=True)
    masks, ad = _gpu_recording_from_oracle(rec)
    sv = solver_for(pr)
    # checkpoints of the frozen map, computed on the GPU
    nck = (nsteps + ck - 1) // ck
    ckpt = torch.empty((nck,) + pr.U0.shape, dtype=torch.float64, device="cuda")
    U = torch.from_numpy(pr.U0.copy()).cuda()
    nf = sv.nfaces
    for c in range(nck):
        ckpt[c] = U
        n = min(ck, nsteps - c * ck)
        T.lib().teno_run_replay(sv._h, T._ptr(U), n, T._ptr(masks[c * ck:]), T._ptr(ad[c * ck:]))
    rng = np.random.default_rng(3)
    lamT = rng.standard_normal(pr.U0.shape)
    lam = torch.from_numpy(lamT.copy()).cuda()
    code = T.lib().teno_run_vjp(sv._h, T._ptr(ckpt), T._ptr(masks), T._ptr(ad), nsteps, ck, T._ptr(lam))
    assert code == 0
    sv.poll()
    g = lam.cpu().numpy()
    for k in range(3):
        d = W.random_directions(100 + k, pr.U0, 1)[0]
        jd = O.run_frozen_jvp(cfg, pr.U0, d, rec)
        a, b = np.sum(lamT * jd), np.sum(g * d)
        assert abs(a - b) <= 1e-11 * np.sum(np.abs(lamT * jd)), (a, b)


def test_record_replay_bitwise_and_masks_match_oracle():
    pr = W.euler2d(10, n=48, ny=40)
    sv = solver_for(pr)
    U = torch.from_numpy(pr.U0.copy()).cuda()
    rec = sv.run_record(U, 5, 2)
    U2 = torch.from_numpy(pr.U0.copy()).cuda()
    sv.run_replay(U2, rec)
    sv.poll()
    assert torch.equal(U, U2)
    # the recorded selection equals the oracle's own on the same trajectory, word by word; a word may
    # differ only where a cut-off decision it depends on lies within rounding of C_T
    _, _, dts, rep = trajectory_census(pr, oracle_cfg(pr), pr.U0, 5, rec["masks"].cpu().numpy())
    print("[census]", rep, flush=True)
    assert rep["unexplained"] == 0 and rep["downstream"] == 0, rep
    assert np.allclose(rec["alpha_dt"].cpu().numpy()[:, 24], dts, rtol=1e-13)


def test_trajectory_gradient_matches_central_differences():
    """Frozen map U0 -> U(T) of the GPU itself: <grad J, d> vs (J(U0 + h d) - J(U0 - h d)) / 2h."""
    pr = W.euler2d(11, n=64, ny=64)
    sv = solver_for(pr)
    target = torch.from_numpy(W.density_target(3, 64)).cuda()
    area = pr.dx * pr.dy
    U0 = torch.from_numpy(pr.U0.copy()).cuda()
    nsteps, ck = 12, 5
    U = U0.clone()
    rec = sv.run_record(U, nsteps, ck)

    def loss(Ufin):
        return torch.sqrt(torch.sum((Ufin[0] - target) ** 2) * area)

    J = loss(U)
    lam = torch.zeros_like(U)
    lam[0] = (U[0] - target) * area / J
    sv.run_vjp(rec, lam)
    for k in range(4):
        d = torch.from_numpy(W.random_directions(200 + k, pr.U0, 1)[0]).cuda()
        h = 1e-6 * U0.abs().max() / d.abs().max()
        Up = U0 + h * d
        Um = U0 - h * d
        sv.run_replay(Up, rec)
        sv.run_replay(Um, rec)
        fd = (loss(Up) - loss(Um)) / (2 * h)
        an = torch.sum(lam * d)
        rel = abs(float(fd - an)) / abs(float(an))
        assert rel < 1e-6, (float(fd), float(an))
    sv.poll()


@pytest.mark.parametrize("sys,nsteps", [("e2", 7), ("e2", 8), ("e1", 9)])
def test_stored_stages_equal_checkpointed(sys, nsteps):
    """A recording that keeps every stage input (CKPT_STAGES) against checkpoints every 3 steps:
    the same forward state and masks, and the same gradient bit for bit (the frozen replay of a
    checkpointed segment reproduces the stored stage inputs exactly, and the reverse steps are the
    same launches). Odd and even step counts cover both buffers the running adjoint ends in."""
    if sys == "e2":
        pr = W.euler2d(31, n=72, ny=60)
    else:
        pr = W.euler1d(32, n=150)
    print(f"[case] stored stages {sys} {nsteps} steps", flush=True)
    sv = solver_for(pr)
    U0 = torch.from_numpy(pr.U0.copy()).cuda()
    Ua, Ub = U0.clone(), U0.clone()
    ra = sv.run_record(Ua, nsteps, 3)
    rb = sv.run_record(Ub, nsteps, T.CKPT_STAGES)
    sv.poll()
    assert torch.equal(Ua, Ub)
    assert torch.equal(ra["masks"], rb["masks"]) and torch.equal(ra["alpha_dt"], rb["alpha_dt"])
    assert rb["ckpt"].shape[0] == 3 * nsteps and torch.equal(rb["ckpt"][0], U0)
    lam0 = torch.from_numpy(W.random_directions(33, pr.U0, 1)[0]).cuda()
    la, lb = lam0.clone(), lam0.clone()
    sv.run_vjp(ra, la)
    sv.run_vjp(rb, lb)
    sv.poll()
    assert torch.equal(la, lb)
    assert float(la.abs().max()) > 0


def test_autograd_functions():
    pr = W.euler2d(12, n=40, ny=30)
    sv = solver_for(pr)
    U0 = torch.from_numpy(pr.U0.copy()).cuda().requires_grad_(True)
    Ut = T.trajectory(U0, sv, 4, ckpt_every=2)
    loss = (Ut[0] ** 2).sum()
    loss.backward()
    assert U0.grad is not None and torch.isfinite(U0.grad).all()
    # every stage input kept: the same gradient bit for bit
    U0s = torch.from_numpy(pr.U0.copy()).cuda().requires_grad_(True)
    Uts = T.trajectory(U0s, sv, 4, ckpt_every=T.CKPT_STAGES)
    assert torch.equal(Uts.detach(), Ut.detach())
    (Uts[0] ** 2).sum().backward()
    assert torch.equal(U0s.grad, U0.grad)
    U1 = torch.from_numpy(pr.U0.copy()).cuda().requires_grad_(True)
    r = T.rhs(U1, sv)
    w = torch.randn_like(r)
    (r * w).sum().backward()
    assert torch.isfinite(U1.grad).all()
    sv.poll()


def test_adjoint_rejects_single_precision():
    pr = W.euler1d(1, n=64)
    sv = solver_for(pr, dtype=torch.float32)
    U = torch.from_numpy(pr.U0.astype(np.float32)).cuda()
    m = sv.masks_buffer()
    a = torch.zeros(8, dtype=torch.float64, device="cuda")
    with pytest.raises(T.TenoError):
        sv.rhs_vjp(U, m, a, U.clone())


@pytest.mark.parametrize("shape", [(56, 1), (57, 1), (113, 1), (56, 57), (57, 56), (113, 30), (30, 113)])
@pytest.mark.parametrize("bc", [O.PERIODIC, O.OUTFLOW], ids=["periodic", "outflow"])
def test_rhs_vjp_dot_product_sizes(shape, bc):
    # a backward wave owns 56 cells: lines one short of, at and past multiples of that, 1D and 2D,
    # against the oracle's forward derivative: <lam, J d> = <J^T lam, d>
    nx, ny = shape
    pr = W.euler1d(nx, n=nx) if ny == 1 else W.euler2d(nx + ny, n=nx, ny=ny)
    pr.bc_x = pr.bc_y = bc
    cfg, ex, masks = _frozen_inputs(pr, pr.U0)
    sv = solver_for(pr)
    rng = np.random.default_rng(nx * 1000 + ny)
    Ug = torch.from_numpy(pr.U0).cuda()
    mg = torch.from_numpy(masks.view(np.int32)).cuda()
    ag = torch.from_numpy(ex["alpha"]).cuda()
    for _ in range(2):
        lam = rng.standard_normal(pr.U0.shape)
        d = W.random_directions(int(rng.integers(1 << 30)), pr.U0, 1)[0]
        jd = O.rhs_frozen_jvp(cfg, pr.U0, d, ex["alpha"], ex["masks_x"], ex.get("masks_y"))
        g = sv.rhs_vjp(Ug, mg, ag, torch.from_numpy(lam).cuda()).cpu().numpy()
        a, b = np.sum(lam * jd), np.sum(g * d)
        scale = np.sum(np.abs(lam * jd))
        assert abs(a - b) <= 1e-12 * scale, (a, b)
    sv.poll()
