"""Host-side checks of the paper's test data as generated here (no GPU): the linear-advection
profiles u1, u2, u3 and the Titarev-Toro initial state, against their printed definitions and the
reading taken for u3 (pieces moved 1 to the left so that each lies in [-1, 1) around its centre),
plus the oracle's own run of the four-wave data: bounded, conservative, back near the data after
one period."""

import numpy as np

from oracle import oracle as O
from paper_1808_00037_amd import workloads as W

from gpu_common import oracle_cfg


def test_u1_u2_are_the_printed_functions():
    p1, p2 = W.paper_advection("u1", 200), W.paper_advection("u2", 200)
    x1 = W.cell_centres(0.0, 1.0, 200)
    x2 = W.cell_centres(0.0, 2.0, 200)
    assert np.array_equal(p1.U0[0, 0], np.exp(-300.0 * (x1 - 0.5) ** 2))
    assert np.allclose(p2.U0[0, 0], np.sin(np.pi * x2) ** 3, rtol=0, atol=1e-15)
    # one period at CFL 0.2: 5 N steps of dt = 0.2 dx
    assert p1.nsteps == 1000 and abs(p1.nsteps * p1.dt - 1.0) < 1e-12
    assert p2.nsteps == 1000 and abs(p2.nsteps * p2.dt - 2.0) < 1e-12


def test_u3_pieces_sit_around_their_centres():
    x = np.linspace(-1.0, 1.0, 200001)[:-1]
    u = W._u3(x)
    # zero outside the four pieces
    inside = ((x >= -0.8) & (x <= -0.6)) | ((x >= -0.4) & (x <= -0.2)) | ((x >= 0.0) & (x <= 0.2)) | \
             ((x >= 0.4) & (x <= 0.6))
    assert np.all(u[~inside] == 0.0)
    # Gaussian triple around z = -0.7, square, triangle peaking at 0.1, ellipse triple around 0.5
    assert abs(x[np.argmax(np.where((x > -0.8) & (x < -0.6), u, 0))] + 0.7) < 1e-4
    assert np.all(u[(x >= -0.4) & (x <= -0.2)] == 1.0)
    tri = (x >= 0.0) & (x <= 0.2)
    assert np.allclose(u[tri], 1.0 - np.abs(10.0 * (x[tri] - 0.1)))
    assert abs(x[np.argmax(np.where((x > 0.4) & (x < 0.6), u, 0))] - 0.5) < 1e-4
    # the triple averages stay below the single profile's peak of 1
    assert u.max() == 1.0


def test_titarev_toro_state():
    pr = W.shock_tube("titarev_toro", n=400)
    x = W.cell_centres(0.0, 10.0, 400)
    rho, m, E = pr.U0[:, 0, :]
    left = x <= 0.5
    assert np.allclose(rho[left], 1.515695) and np.allclose(m[left] / rho[left], 0.523346)
    assert np.allclose(rho[~left], 1.0 + 0.1 * np.sin(20.0 * np.pi * x[~left]))
    p = 0.4 * (E - 0.5 * m * m / rho)
    assert np.allclose(p[left], 1.805) and np.allclose(p[~left], 1.0)
    assert pr.bc_x == W.OUTFLOW and pr.meta["t_end"] == 5.0


def test_oracle_four_wave_period():
    pr = W.paper_advection("u3", 200)
    U = O.run(oracle_cfg(pr), pr.U0, pr.nsteps, dt=pr.dt)
    assert -0.01 < U.min() and U.max() < 1.01
    assert abs(U.sum() - pr.U0.sum()) < 1e-12 * pr.nx
    assert np.abs(U - pr.U0).mean() < 0.03
