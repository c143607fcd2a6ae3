// teno_worklist.hpp -- item counts of the batched sweeps' static work lists: host code shared by the
// batch library (teno_batch.hip) and the host-side bounds check of the test-suite, so that the check
// runs the same arithmetic as the library.
//
// A 2D instance of nx x ny cells takes, per sweep direction, main items (tiles of ns segments: x,
// consecutive segments of the row-major segment list; y, ns adjacent columns at one segment position)
// and, when its ragged last segments are packed, tail items (the last segments of ns x P lines each).
// A 1D instance takes x main items only.
#pragma once
#include "teno_device.hpp"

namespace teno {

__host__ __device__ inline int nseg_of(int len) { return (len + SEG_CELLS - 1) / SEG_CELLS; }

// Whether the ragged last segments of a 2D instance's lines (line length len, nlines lines) are packed
// several lines to a wave: at least two pieces fit and there are lines to share a wave.
__host__ __device__ inline bool packable(int len, int nlines) { return nlines > 1 && tail_geom(len).P >= 2; }

// Segments per line that the main items cover (the last one is a tail item's when packed).
__host__ __device__ inline int main_nseg(int len, bool packed) { return nseg_of(len) - (packed ? 1 : 0); }

inline long long x_main_items(int nx, int ny, int ns, bool packed)
{
    const long long segs = (long long)main_nseg(nx, packed) * ny;
    return (segs + ns - 1) / ns;
}
inline long long x_tail_items(int nx, int ny, int ns)
{
    const int per = ns * tail_geom(nx).P;          // lines per tail item
    return (ny + per - 1) / per;
}
inline long long y_main_items(int nx, int ny, int ns, bool packed)
{
    return (long long)((nx + ns - 1) / ns) * main_nseg(ny, packed);
}
inline long long y_tail_items(int nx, int ny, int ns)
{
    const int per = ns * tail_geom(ny).P;          // columns per tail item
    return (nx + per - 1) / per;
}

}  // namespace teno
