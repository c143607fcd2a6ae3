"""Pins of the oracle's frozen-selection derivatives (no GPU).

With every selected stencil, alpha and dt held at their recorded values, the operator and the RK3
trajectory are smooth maps of the state. The oracle differentiates them by the complex step; these
tests pin that against central finite differences (an independent route) and against linearity.
"""
import numpy as np

from paper_1808_00037_amd import workloads as W


def _rel(a, b):
    return np.abs(a - b).max() / max(np.abs(b).max(), 1e-300)


def test_rhs_jvp_matches_central_differences_euler2d(orc):
    pr = W.euler2d(5, n=20)
    cfg = orc.Config(orc.EULER2D, 20, 20)
    _, ex = orc.rhs(cfg, pr.U0, want_faces=True)
    d = W.random_directions(1, pr.U0, 1)[0]
    jd = orc.rhs_frozen_jvp(cfg, pr.U0, d, ex["alpha"], ex["masks_x"], ex["masks_y"])
    h = 1e-6 * np.abs(pr.U0).max() / np.abs(d).max()
    fp = orc.rhs_frozen(cfg, pr.U0 + h * d, ex["alpha"], ex["masks_x"], ex["masks_y"])
    fm = orc.rhs_frozen(cfg, pr.U0 - h * d, ex["alpha"], ex["masks_x"], ex["masks_y"])
    assert _rel(jd, (fp - fm) / (2 * h)) < 1e-6


def test_rhs_jvp_of_linear_advection_is_the_operator_itself(orc):
    """f = a u and frozen selection: the operator is linear, so J d = L_frozen(d)."""
    pr = W.advection(1, 64)
    cfg = orc.Config(orc.ADV1D, 64, x0=-1.0, x1=1.0)
    u = pr.U0.copy()
    u[0, 0, 30:] += 1.0                      # a step, so that some stencils are cut
    _, ex = orc.rhs(cfg, u, want_faces=True)
    assert (ex["masks_x"] != 0).any()
    d = np.random.default_rng(0).standard_normal(u.shape)
    jd = orc.rhs_frozen_jvp(cfg, u, d, ex["alpha"], ex["masks_x"])
    assert _rel(jd, orc.rhs_frozen(cfg, d, ex["alpha"], ex["masks_x"])) < 1e-13


def test_frozen_replay_reproduces_the_recorded_trajectory_bitwise(orc):
    pr = W.euler1d(3, n=128)
    cfg = orc.Config(orc.EULER1D, 128, x0=0.0, x1=10.0, bc_x=orc.OUTFLOW)
    U1, rec = orc.run(cfg, pr.U0, 6, cfl=0.5, record=True)
    U2 = orc.run_frozen(cfg, pr.U0, rec)
    assert np.array_equal(U1, U2)


def test_trajectory_jvp_matches_central_differences(orc):
    pr = W.euler2d(2, n=16)
    cfg = orc.Config(orc.EULER2D, 16, 16)
    _, rec = orc.run(cfg, pr.U0, 3, cfl=0.5, record=True)
    d = W.random_directions(4, pr.U0, 1)[0]
    jd = orc.run_frozen_jvp(cfg, pr.U0, d, rec)
    h = 1e-6 * np.abs(pr.U0).max() / np.abs(d).max()
    fp = orc.run_frozen(cfg, pr.U0 + h * d, rec)
    fm = orc.run_frozen(cfg, pr.U0 - h * d, rec)
    assert _rel(jd, (fp - fm) / (2 * h)) < 1e-6
