"""Host-side bounds and coverage check of the batched sweeps' tiles (no GPU).

tests/tail_bounds.cpp is compiled for the host with hipcc against the library's own headers: it
calls the index maps the kernels use (tile_segment, pack_map, pack_piece, pack_line, tail_geom,
bc_index) and the item counts the batch uses (teno_worklist.hpp), and replays every item of a 2D
instance's sweep for 120,000 shapes (line lengths 1..500, 15 line counts, 4- and 8-segment tiles,
both directions, packed or not, both boundary conditions). Every staged access must be in bounds,
every needed lane's stencil inside its own piece of a packed wave, and every cell produced exactly
once. (Planting an off-by-one in the divisor, the piece width or the main items' segment count makes
it report violations.)
"""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")


def test_packed_tails_and_tiles_stay_in_bounds(tmp_path):
    if not os.path.exists(HIPCC) and not shutil.which("hipcc"):
        pytest.skip("hipcc is not available")
    exe = str(tmp_path / "tail_bounds")
    subprocess.run([HIPCC, "-x", "hip", "--offload-arch=gfx950", "--cuda-host-only", "-O2", "-std=c++17",
                    "-I", os.path.join(ROOT, "include"), "-I", os.path.join(ROOT, "paper_1808_00037_amd", "csrc"),
                    os.path.join(ROOT, "tests", "tail_bounds.cpp"), "-o", exe],
                   check=True, capture_output=True, text=True)
    out = subprocess.run([exe], capture_output=True, text=True, timeout=300)
    print(out.stdout[-2000:])
    assert out.returncode == 0, out.stdout[-2000:]
    assert "shapes 120000 violations 0" in out.stdout
