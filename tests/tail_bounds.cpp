// Host-side bounds and coverage check of the batched sweeps' tiles (compiled and run by
// tests/test_tail_bounds.py; no GPU). It calls the library's own index maps (tile_segment, pack_map,
// pack_piece, pack_line, tail_geom, bc_index, bc_index_near from teno_device.hpp) and item counts
// (teno_worklist.hpp) and replays, for every item of a 2D instance's sweep, what each thread stages
// and what each lane computes and stores, exactly as the kernels index them. It checks that every
// staged global access is in bounds, every record position inside the block's LDS record, every
// needed lane's stencil inside its own piece, and that every cell of the instance is produced
// exactly once over the main and tail items. Prints the number of shapes checked and of violations.
#include <cstdio>
#include <vector>

#include "teno_device.hpp"
#include "teno_worklist.hpp"

using namespace teno;

static long long violations = 0;
static void fail(const char *what, int len, int nlines, int ns, int dir, int packed, int bc, int a, int b)
{
    if (violations < 20)
        std::printf("violation: %s (len %d lines %d ns %d dir %d packed %d bc %d: %d %d)\n", what, len, nlines, ns, dir,
                    packed, bc, a, b);
    ++violations;
}

// One sweep direction of an instance whose lines have len cells (nlines lines), tiles of ns
// segments, tail packing as the batch decides it (packed = 1 asks for it), boundary condition bc.
static void check(int len, int nlines, int ns, int dir, int packed, int bc)
{
    const bool pk = packed && packable(len, nlines);
    std::vector<int> produced((size_t)len * nlines, 0);
    const bool near = len >= SEG_LOAD;
    auto src = [&](int i) { return near ? bc_index_near(i, len, bc) : bc_index(i, len, bc); };
    const int nx = dir == 0 ? len : nlines, ny = dir == 0 ? nlines : len;
    // main items: the plain tiles over main_nseg segments per line
    const long long nmain = dir == 0 ? x_main_items(nx, ny, ns, pk) : y_main_items(nx, ny, ns, pk);
    const int nseg = main_nseg(len, pk);
    for (long long t = 0; t < nmain; ++t) {
        for (int s = 0; s < ns; ++s) {
            int line, c0;
            tile_segment(dir, ns, (int)t, s, nseg, nlines, line, c0);
            if (line < 0) continue;
            if (c0 >= len) fail("segment starts past the line", len, nlines, ns, dir, packed, bc, c0, line);
            for (int q = 0; q < SEG_LOAD; ++q) {             // staged cells c0-5 .. c0+66
                const int g = src(c0 - SEG_HALO + q);
                if (g < 0 || g >= len) fail("main staging out of the line", len, nlines, ns, dir, packed, bc, q, g);
            }
            for (int k = 1; k <= SEG_CELLS; ++k) {           // lanes 1..61 own cells c0 .. c0+60
                const int c = c0 - 1 + k;
                if (c < len) produced[(size_t)line * len + c] += 1;
            }
        }
    }
    // tail items: the ragged last segments of ns x P lines each
    if (pk) {
        const long long ntail = dir == 0 ? x_tail_items(nx, ny, ns) : y_tail_items(nx, ny, ns);
        for (long long t = 0; t < ntail; ++t) {
            const PackMap m = pack_map(len, (int)t, ns);
            if (m.c0 != (nseg_of(len) - 1) * SEG_CELLS || m.nt != len - m.c0 || m.P * m.W > PACK_SPAN + 1)
                fail("tail geometry", len, nlines, ns, dir, packed, bc, m.c0, m.P);
            for (int s = 0; s < ns; ++s) {
                const int line0 = m.l0 + s;
                if (line0 >= nlines) continue;               // (the slot is skipped as a whole)
                const int rec_base = s * seg_stride<EULER2D>();
                for (int q = 0; q < SEG_LOAD; ++q) {         // staging of record position q
                    const int i = pack_piece(m, q), ql = q - i * m.W;
                    if (i != q / m.W) fail("piece of a staged position", len, nlines, ns, dir, packed, bc, q, i);
                    int line = pack_line(m, i, s, ns, nlines);
                    if (line < 0) line = line0;
                    const int g = src(m.c0 - SEG_HALO + ql);
                    if (line < 0 || line >= nlines || g < 0 || g >= len)
                        fail("tail staging out of the instance", len, nlines, ns, dir, packed, bc, line, g);
                    // (tail tiles keep one record per segment slot: rec_size of the PACK kernels)
                    const int rec_sz = ns == 4 ? rec_size<EULER2D, 0, 4, true>() : rec_size<EULER2D, 0, 8, true>();
                    if (rec_base + q + (Rec<EULER2D>::NREC - 1) * SEG_LOAD >= rec_sz)
                        fail("record position past the block's record", len, nlines, ns, dir, packed, bc, s, q);
                }
                for (int k = 0; k < WAVE; ++k) {             // compute lane k
                    const int i = pack_piece(m, k), kl = k - i * m.W;
                    if (i != k / m.W) fail("piece of a lane", len, nlines, ns, dir, packed, bc, k, i);
                    const int line = pack_line(m, i, s, ns, nlines);
                    const bool needed = line >= 0 && kl <= m.nt + 2;
                    // a needed lane reads positions k .. k+7: all inside its own piece
                    if (needed && (k + 7 >= (i + 1) * m.W || k + 7 >= SEG_LOAD))
                        fail("stencil leaves its piece", len, nlines, ns, dir, packed, bc, k, kl);
                    const bool cell_ok = line >= 0 && kl >= 1 && kl <= 61 && m.c0 - 1 + kl < len;
                    if (cell_ok) {
                        if (dir == 0) produced[(size_t)line * len + m.c0 - 1 + kl] += 1;
                        // the cell's faces (lanes kl, kl+1) and their neighbour flags (kl-1 .. kl+2)
                        if (!(kl + 2 <= m.nt + 2)) fail("cell needs an idle lane", len, nlines, ns, dir, packed, bc, k, kl);
                    }
                }
                if (dir == 1) {
                    // y-sweeps store through the record: entry kk of the slot holds lane kk + 1's cell
                    for (int kk = 0; kk < WAVE; ++kk) {
                        const int i = pack_piece(m, kk + 1), kl = kk + 1 - i * m.W;
                        const int line = pack_line(m, i, s, ns, nlines);
                        if (line < 0 || kl < 1 || kl > m.nt) continue;
                        produced[(size_t)line * len + m.c0 + kl - 1] += 1;
                    }
                }
            }
        }
    }
    for (int l = 0; l < nlines; ++l)
        for (int c = 0; c < len; ++c)
            if (produced[(size_t)l * len + c] != 1)
                fail("cell not produced exactly once", len, nlines, ns, dir, packed, bc, l, c);
}

int main()
{
    // M: (k M) >> 16 == k / W for every width a tail can have and every k < 72
    for (int W = PACK_GAP + 1; W <= PACK_GAP + SEG_CELLS; ++W) {
        const int M = 65536 / W + 1;
        for (int k = 0; k < SEG_LOAD; ++k)
            if (((k * M) >> 16) != k / W) fail("multiply-shift division", W, 0, 0, 0, 0, 0, k, M);
    }
    long long shapes = 0;
    const int lines[] = {1, 2, 3, 4, 5, 7, 8, 9, 15, 16, 17, 24, 33, 64, 100};
    for (int len = 1; len <= 500; ++len)
        for (int nl : lines)
            for (int ns : {4, 8})
                for (int dir = 0; dir < 2; ++dir)
                    for (int packed = 0; packed < 2; ++packed)
                        for (int bc = 0; bc < 2; ++bc) {
                            check(len, nl, ns, dir, packed, bc);
                            ++shapes;
                        }
    std::printf("shapes %lld violations %lld\n", shapes, violations);
    return violations ? 1 : 0;
}
