"""The oracle's drivers for large 2D states against the oracle itself (CPU).

rhs_strips evaluates the operator on row strips with five halo rows and the whole state's
Lax-Friedrichs constants; step_stages takes one SSP-RK3 step stage by stage. Both must be bitwise
equal to the plain whole-domain calls (rhs, run), for both boundary conditions along y, any strip
height and any number of threads, so that the full-size GPU comparisons rest on the oracle proper.
"""
import numpy as np
import pytest

from oracle import oracle as O
from paper_1808_00037_amd import workloads as W


def _cfg(pr, bc):
    return O.Config(O.EULER2D, pr.nx, pr.ny, pr.x0, pr.x1, pr.y0, pr.y1, bc, bc)


@pytest.mark.parametrize("bc", [O.PERIODIC, O.OUTFLOW], ids=["periodic", "outflow"])
@pytest.mark.parametrize("rows,threads", [(7, 1), (16, 4), (64, 3)])
def test_rhs_strips_equal_the_whole_domain(bc, rows, threads):
    pr = W.euler2d(41, n=60, ny=53)
    cfg = _cfg(pr, bc)
    d, ex = O.rhs(cfg, pr.U0, want_faces=True)
    got = {k: [] for k in ("masks_x", "flags_x", "chi_x", "masks_y", "flags_y", "chi_y")}
    spans = []

    def on_faces(j0, j1, f):
        spans.append((j0, j1))
        for k in got:
            got[k].append(f[k])

    ds = O.rhs_strips(cfg, pr.U0, ex["alpha"], strip_rows=rows, threads=threads, on_faces=on_faces)
    assert np.array_equal(ds, d)
    assert spans == sorted(spans) and spans[0][0] == 0 and spans[-1][1] == pr.ny
    for k, parts in got.items():
        assert np.array_equal(np.concatenate(parts), ex[k]), k
    assert np.array_equal(O.rhs_strips(cfg, pr.U0, ex["alpha"], strip_rows=rows, threads=threads), d)


@pytest.mark.parametrize("bc", [O.PERIODIC, O.OUTFLOW], ids=["periodic", "outflow"])
def test_step_stages_equal_run(bc):
    pr = W.euler2d(42, n=48, ny=44)
    cfg = _cfg(pr, bc)
    Uo, rec = O.run(cfg, pr.U0, 1, cfl=pr.cfl, record=True)
    masks = []
    U1, info = O.step_stages(cfg, pr.U0, cfl=pr.cfl,
                             on_faces=lambda s, j0, j1, f: masks.append(np.concatenate(
                                 [f["masks_x"].ravel(), f["masks_y"].ravel()])))
    assert np.array_equal(U1, Uo)
    assert info["dt"] == rec["dt"][0]
    assert np.array_equal(info["alpha"], rec["alpha"][0])
    assert np.array_equal(np.stack(masks), rec["masks"][0])
    U2, info2 = O.step_stages(cfg, pr.U0, cfl=pr.cfl, strip_rows=9, threads=3)
    assert np.array_equal(U2, Uo)
    assert np.array_equal(info2["alpha"], info["alpha"])
