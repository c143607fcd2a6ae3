"""Batched runs of many uneven Euler instances (1D and 2D mixed) through the C ABI.

The graph-captured form (mode 0: static work-list launches over all instances, autotuned tile
shapes) and the one-launch-per-instance form (mode 1) must give bitwise identical states, each equal
bitwise to the instance run alone with the single-problem solver, and the oracle agrees with an
instance after a few steps.
"""
import numpy as np
import pytest
import torch

from oracle import oracle as O
from paper_1808_00037_amd import teno as T
from paper_1808_00037_amd import workloads as W

from gpu_common import oracle_cfg, solver_for

pytestmark = pytest.mark.gpu


def _problems():
    # 2D sizes with short ragged last segments (64, 70, 130 along x; 130, 200 along y) are packed
    # several lines to a wave, over several tail tiles with a partial last one; one instance has
    # outflow boundaries, where the packed pieces meet the boundary condition
    probs = [W.euler1d(1, n=300), W.euler1d(2, n=1000), W.euler1d(3, n=61), W.euler1d(4, n=4096),
             W.euler2d(5, n=40), W.euler2d(6, n=64, ny=48), W.euler2d(7, n=33, ny=50), W.euler2d(8, n=130, ny=90),
             W.euler2d(9, n=70, ny=200), W.euler2d(10, n=64, ny=130)]
    probs[2].bc_x = O.PERIODIC
    probs[9].bc_x = probs[9].bc_y = O.OUTFLOW
    return probs


def test_batch_modes_are_bitwise_equal_and_match_single_runs():
    probs = _problems()
    b = T.Batch(probs)
    buf0 = b.pack([torch.from_numpy(p.U0) for p in probs])
    nsteps = 3
    a = buf0.clone()
    b.run(a, nsteps, mode=0)
    b.poll()
    c = buf0.clone()
    b.run(c, nsteps, mode=1)
    b.poll()
    assert torch.equal(a, c)
    for k, p in enumerate(probs):
        sv = solver_for(p)
        U = torch.from_numpy(p.U0.copy()).cuda()
        sv.run(U, nsteps, graph=False)
        sv.poll()
        assert torch.equal(b.unpack(a, k), U), k
    # one instance against the oracle
    p = probs[5]
    Uo = O.run(oracle_cfg(p), p.U0, nsteps, cfl=p.cfl)
    err = np.abs(b.unpack(a, 5).cpu().numpy() - Uo).max() / np.abs(Uo).max()
    assert err < 1e-11, err
    # a second graph replay continues from the new state
    b.run(a, 2, mode=0)
    b.run(c, 2, mode=1)
    b.poll()
    assert torch.equal(a, c)


def test_every_launch_shape_gives_the_same_states():
    probs = _problems()
    b = T.Batch(probs)
    buf0 = b.pack([torch.from_numpy(p.U0) for p in probs])
    ref = buf0.clone()
    b.run(ref, 3, mode=1)
    b.poll()
    for xt in (4, 8):
        for yt in (4, 8):
            for packed in (0, 1):
                b.set_shape(xt, yt, packed)
                a = buf0.clone()
                b.run(a, 3, mode=0)
                b.poll()
                assert torch.equal(a, ref), (xt, yt, packed)
    with pytest.raises(T.TenoError):
        b.set_shape(6, 4, 0)
    with pytest.raises(T.TenoError):
        b.set_shape(4, 4, 2)
    b.close()


def test_batch_rejects_scalar_systems():
    with pytest.raises(T.TenoError):
        T.Batch([W.advection(1, 64)])


def test_single_precision_batch():
    # FP32 instances: both modes bitwise equal to each other and to the FP32 single-problem solver,
    # and within single-precision rounding of the FP64 oracle after a few steps
    probs = _problems()
    b = T.Batch(probs, dtype=torch.float32)
    buf0 = b.pack([torch.from_numpy(p.U0) for p in probs])
    a = buf0.clone()
    b.run(a, 3, mode=0)
    c = buf0.clone()
    b.run(c, 3, mode=1)
    b.poll()
    assert torch.equal(a, c)
    for k, p in enumerate(probs):
        sv = solver_for(p, dtype=torch.float32)
        U = torch.from_numpy(p.U0.astype(np.float32)).cuda()
        sv.run(U, 3, graph=False)
        sv.poll()
        assert torch.equal(b.unpack(a, k), U), k
    p = probs[7]
    Uo = O.run(oracle_cfg(p), p.U0, 3, cfl=p.cfl)
    err = np.abs(b.unpack(a, 7).double().cpu().numpy() - Uo).max() / np.abs(Uo).max()
    assert err < 1e-4, err


@pytest.mark.parametrize("opts", [dict(scheme=T.TENO5), dict(alpha_mode=1), dict(eps=1e-6), dict(ct=1e-4),
                                  dict(C=2.0, q=4), dict(characteristic=0)],
                         ids=["teno5", "scalar_alpha", "constant_eps", "ct_1e-4", "C2_q4", "componentwise"])
def test_batch_options_match_single_runs(opts):
    # every scheme option reaches the batched kernels as it reaches the single-problem solver
    probs = _problems()
    b = T.Batch(probs, **opts)
    buf0 = b.pack([torch.from_numpy(p.U0) for p in probs])
    a = buf0.clone()
    b.run(a, 3, mode=0)
    c = buf0.clone()
    b.run(c, 3, mode=1)
    b.poll()
    assert torch.equal(a, c)
    for k, p in enumerate(probs):
        sv = solver_for(p, **opts)
        U = torch.from_numpy(p.U0.copy()).cuda()
        sv.run(U, 3, graph=False)
        sv.poll()
        assert torch.equal(b.unpack(a, k), U), k


def test_batch_of_tiny_and_single_instances():
    # instances smaller than the stencil (down to one cell), and a batch of one
    for probs in ([W.euler1d(1, n=1), W.euler1d(2, n=2), W.euler2d(3, n=1, ny=1), W.euler2d(4, n=2, ny=3),
                   W.euler2d(5, n=7, ny=5), W.euler2d(6, n=3, ny=26)],
                  [W.euler2d(7, n=90, ny=70)]):
        b = T.Batch(probs)
        buf0 = b.pack([torch.from_numpy(p.U0) for p in probs])
        a = buf0.clone()
        b.run(a, 2, mode=0)
        c = buf0.clone()
        b.run(c, 2, mode=1)
        b.poll()
        assert torch.equal(a, c)
        for k, p in enumerate(probs):
            sv = solver_for(p)
            U = torch.from_numpy(p.U0.copy()).cuda()
            sv.run(U, 2, graph=False)
            sv.poll()
            assert torch.equal(b.unpack(a, k), U), (len(probs), k)
