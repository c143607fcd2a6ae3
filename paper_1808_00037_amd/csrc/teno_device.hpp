// teno_device.hpp -- gfx950 device code of the TENO7X semi-discrete operator.
//
// Method: F. Zhang, J. Liu, H. Zhang, C. Xu, "An extending strategy based on TENO framework for
// hyperbolic conservation laws" (arXiv:1808.00037); equations by their labels in the paper.
//
// Work decomposition (one kernel per sweep direction):
//   * A wave (64 lanes) owns one line segment: lane k owns face f = c0 - 1 + k of the line
//     (face f = left face of cell f). All 64 faces get their smoothness flags; lanes 1..62 then
//     have both neighbour faces in the same wave and finish the reconstruction; lanes 1..61 own
//     cells c0 .. c0+60 and apply the conservative difference. Consecutive segments start 61 cells
//     apart, so every face and cell is finished by exactly the lanes that can finish it.
//   * Segment cells are staged in LDS (conserved variables plus velocity, pressure and
//     1/sqrt(rho), computed once per cell); every lane then reads its eight stencil cells from LDS.
//     In x-sweeps each wave stages its own segment (a coalesced run of a row, wave-uniform index
//     arithmetic) and the stage operands of its cells arrive by background direct-to-LDS copies;
//     y-sweeps stage 8 adjacent columns with the same rows so that a global load of one row reads
//     8 consecutive doubles, and write their results back through LDS row by row. LDS holds each
//     segment contiguously, so lanes read consecutive LDS words.
//   * Tiles are renumbered per XCD so that neighbouring tiles share an L2.
//   * The neighbour flags of eq:vec come from lanes k-1 and k+1 through cross-lane shuffles; no
//     flag array is stored (the paper's whole-domain flag pass lives in registers).
//   * Characteristic fields are streamed one at a time: project eight points, cut-off flags on
//     both split sides, exchange, select, reconstruct, accumulate R[:,s] * (v+ + v-).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>


namespace teno {

// Multiply-adds are fused only within one expression, as written (no fusion across statements): the
// rounding of every result then follows the source alone, whatever kernel variant inlines the code,
// so that all launch shapes of a sweep give bitwise equal results.
#pragma clang fp contract(on)

enum : int { ADV1D = 0, EULER1D = 1, EULER2D = 2, BURGERS1D = 3 };
enum : int { MODE_RHS = 0, MODE_STAGE = 1, MODE_FACES = 2 };
enum : unsigned { ERR_NONFINITE = 1u, ERR_NONPHYSICAL = 2u, ERR_SELECTION = 4u };

constexpr int WAVE = 64;
constexpr int BLOCK = 256;
constexpr int SEG_CELLS = 61;   // cells finished per segment
constexpr int SEG_HALO = 5;     // first staged cell is c0 - 5
constexpr int SEG_LOAD = 72;    // staged cells per segment (faces c0-1..c0+62 read c0-5..c0+65)

// Packed ragged segments. The last segment of a line holds nt = len - c0 cells (c0 its first cell).
// When nt is short, one wave can take that segment of P lines at once: piece i of the wave stages
// cells c0-5 .. c0+nt+4 of its line at record positions [i W, (i+1) W), W = nt + 10, and lane
// i W + kl then computes face c0-1+kl of that line (kl = 0 .. nt+2 are the faces the piece's cells
// and their neighbour vectors need; the other lanes of the piece straddle two lines and are idle).
// The last piece's lanes must stay below 64: P W <= 71.
constexpr int PACK_GAP = 10;
constexpr int PACK_SPAN = 71;
struct TailGeom {
    int c0, nt, W, P;
};
__host__ __device__ inline TailGeom tail_geom(int len)
{
    TailGeom g;
    const int nseg = (len + SEG_CELLS - 1) / SEG_CELLS;
    g.c0 = (nseg - 1) * SEG_CELLS;
    g.nt = len - g.c0;
    g.W = g.nt + PACK_GAP;
    g.P = PACK_SPAN / g.W;
    return g;
}
// Segment s of a sweep's tile `tile` (nseg_tile segments per tile): its line (-1: none) and first
// cell. x-sweeps: consecutive segments of the row-major list of nseg segments per line; y-sweeps:
// nseg_tile adjacent lines at one segment position. (Index maps shared by the kernels and the host.)
__host__ __device__ inline void tile_segment(int dir, int nseg_tile, int tile, int s, int nseg, int nlines, int &line,
                                             int &c0)
{
    if (dir == 0) {
        const int id = tile * nseg_tile + s;
        line = id / nseg;
        c0 = (id % nseg) * SEG_CELLS;
    } else {
        const int ntile = (nlines + nseg_tile - 1) / nseg_tile;
        line = (tile % ntile) * nseg_tile + s;
        c0 = (tile / ntile) * SEG_CELLS;
    }
    if (line >= nlines) line = -1;
}

// A tail tile: the ragged last segments of nseg_tile x P lines starting at line l0; M makes
// (k M) >> 16 the exact quotient k / W for 0 <= k < 72 (checked on the host for every W).
struct PackMap {
    int c0, nt, W, P, M, l0;
};
__host__ __device__ inline PackMap pack_map(int len, int tile, int nseg_tile)
{
    const TailGeom g = tail_geom(len);
    PackMap m;
    m.c0 = g.c0;
    m.nt = g.nt;
    m.W = g.W;
    m.P = g.P;
    m.M = 65536 / g.W + 1;
    m.l0 = tile * nseg_tile * g.P;
    return m;
}
// The piece that lane (or staged position) k < 72 of a segment slot belongs to.
__host__ __device__ inline int pack_piece(const PackMap &m, int k) { return (k * m.M) >> 16; }
// The line of piece i of segment slot s, or -1 past the tile's pieces or the instance's lines.
__host__ __device__ inline int pack_line(const PackMap &m, int i, int s, int nseg_tile, int nlines)
{
    const int line = m.l0 + i * nseg_tile + s;
    return (i < m.P && line < nlines) ? line : -1;
}

#ifndef TENO_NSEG_X
#define TENO_NSEG_X 4
#endif
constexpr int NSEG_X = TENO_NSEG_X;  // segments per block, x-sweeps
#ifndef TENO_X_WAVE_LOCAL
#define TENO_X_WAVE_LOCAL 1         // x-sweeps order their staging per wave (0: a block barrier)
#endif
#ifndef TENO_NSEG_Y
#define TENO_NSEG_Y 8
#endif
constexpr int NSEG_Y = TENO_NSEG_Y;  // columns per block, y-sweeps
constexpr int NCOPY = 64;       // spread copies of the wave-speed maxima (atomic contention)
constexpr int NWORD = 16;       // words per copy: 0-3 x fields, 4-7 y fields, 8 CFL denominator

// Device control block of one context (zeroed at creation).
struct Ctrl {
    unsigned long long part[4][NCOPY][NWORD];  // [ring][copy][word] maxima of non-negative doubles
    double alpha[8];                           // Lax-Friedrichs constants of the current stage
    double den;                                // CFL denominator of the current stage's state
    double dt;                                 // dt of the current step
    double t;                                  // simulated time, advanced by every step
    double t_end;                              // end time of the runs (used when end_on)
    unsigned err;
    unsigned end_on;                           // steps are cut at t_end, and stand still there
    unsigned steps;                            // steps begun since the counters were reset
    unsigned err_at;                           // 1 + index of the step a failure was first seen in (0: none)
};

// ------------------------------------------------------------------------------------------------
// System traits: number of conserved variables, staged record layout.
// Adjoint Euler records hold (rho, m_n, [m_t], E, u_n, [u_t], p, 1/sqrt(rho), H), n the sweep direction;
// the conserved variables come first, so record index v is local conserved variable v.
// ------------------------------------------------------------------------------------------------
template <int SYS> struct Sys;
template <> struct Sys<ADV1D> { static constexpr int NV = 1, NREC = 1; };
template <> struct Sys<BURGERS1D> { static constexpr int NV = 1, NREC = 1; };
template <> struct Sys<EULER1D> {
    static constexpr int NV = 3, NREC = 7, E = 2, UN = 3, UT = -1, P = 4, RS = 5, H = 6;
};
template <> struct Sys<EULER2D> {
    static constexpr int NV = 4, NREC = 9, E = 3, UN = 4, UT = 5, P = 6, RS = 7, H = 8;
};

// Staged per-cell record of the forward sweeps: the conserved variables in local order, then u_n,
// [u_t], p and 1/sqrt(rho) (sqrt(rho) = rho / sqrt(rho) and H sqrt(rho) = (E + p) / sqrt(rho) are
// recovered in the Roe average, which keeps the record one value shorter than with H).
template <int SYS> struct Rec;
template <> struct Rec<ADV1D> { static constexpr int NREC = 1; };
template <> struct Rec<BURGERS1D> { static constexpr int NREC = 1; };
template <> struct Rec<EULER1D> { static constexpr int NREC = 6, E = 2, UN = 3, UT = -1, P = 4, RS = 5; };
template <> struct Rec<EULER2D> { static constexpr int NREC = 8, E = 3, UN = 4, UT = 5, P = 6, RS = 7; };

// Global variable index of local (normal/tangential) component v in direction DIR.
template <int SYS, int DIR> __device__ __forceinline__ constexpr int gvar(int v)
{
    return (SYS == EULER2D && DIR == 1 && (v == 1 || v == 2)) ? 3 - v : v;
}

__host__ __device__ inline int bc_index(int i, int n, int bc)
{
    if (bc == 0) {
        i %= n;
        return i < 0 ? i + n : i;
    }
    return i < 0 ? 0 : (i >= n ? n - 1 : i);
}

// Copy 64 consecutive elements of a row, starting at cell c >= 0 (cells past the row end read as 0),
// straight from global memory into LDS at dst with the direct-to-LDS buffer load: no registers are
// involved and the wave goes on at once; the copy completes under vmcnt. Each lane moves one dword
// (so the copy is exact for any 4-byte alignment of dst and of the row), 256 bytes per instruction.
// The buffer descriptor spans exactly the row, so offsets past its end return zeros instead of
// touching other memory.
template <typename T>
__device__ __forceinline__ void lds_dma_row(const T *row, int nx, int c, T *dst, int lane)
{
    const __amdgpu_buffer_rsrc_t rs =
        __builtin_amdgcn_make_buffer_rsrc((void *)row, (short)0, nx * (int)sizeof(T), 0x00020000);
    constexpr int CHUNK = WAVE * 4;                        // bytes per instruction
#pragma unroll
    for (int b = 0; b < WAVE * (int)sizeof(T); b += CHUNK)
        __builtin_amdgcn_raw_ptr_buffer_load_lds(rs, (__attribute__((address_space(3))) void *)((char *)dst + b), 4,
                                                 c * (int)sizeof(T) + b + 4 * lane, 0, 0, 0);
}

// Workgroup barrier for LDS only: the wave's LDS operations complete (lgkmcnt 0), then s_barrier.
// Unlike __syncthreads() it does not wait for outstanding vector-memory operations, so background
// copies into a wave's own LDS area stay in flight. The empty asm statements keep the compiler from
// moving memory accesses across it.
__device__ __forceinline__ void lds_barrier()
{
    asm volatile("" ::: "memory");
    __builtin_amdgcn_s_waitcnt(0xC07F);
    __builtin_amdgcn_s_barrier();
    asm volatile("" ::: "memory");
}

// Ordering of a wave's own LDS stores before its later LDS loads of other lanes' elements: the
// wave's LDS operations complete (lgkmcnt 0) and the compiler may not move accesses across.
__device__ __forceinline__ void wave_lds_fence()
{
    asm volatile("" ::: "memory");
    __builtin_amdgcn_s_waitcnt(0xC07F);
    asm volatile("" ::: "memory");
}

// Lane number within the wave, recomputed where it is used (two ALU instructions) rather than kept
// in a register from the start of the kernel as threadIdx.x would be. Volatile, so the compiler
// neither merges nor hoists it.
__device__ __forceinline__ int lane_id_now()
{
    int lo, id;
    asm volatile("v_mbcnt_lo_u32_b32 %0, -1, 0" : "=v"(lo));
    asm volatile("v_mbcnt_hi_u32_b32 %0, -1, %1" : "=v"(id) : "v"(lo));
    return id;
}

// A wave-uniform double moved into scalar registers.
__device__ __forceinline__ double uniform_f64(double x)
{
    const long long b = __double_as_longlong(x);
    const int lo = __builtin_amdgcn_readfirstlane((int)b), hi = __builtin_amdgcn_readfirstlane((int)(b >> 32));
    return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
}

// Wait for every outstanding vector-memory operation of the wave (vmcnt 0), including the
// direct-to-LDS copies; lgkmcnt and expcnt are left alone.
__device__ __forceinline__ void wait_vmem() { __builtin_amdgcn_s_waitcnt(0x0F70); }

// bc_index for -n <= i < 2n (one wrap at most, no division).
__host__ __device__ inline int bc_index_near(int i, int n, int bc)
{
    if (bc == 0) return i < 0 ? i + n : (i >= n ? i - n : i);
    return i < 0 ? 0 : (i >= n ? n - 1 : i);
}

// ------------------------------------------------------------------------------------------------
// Reconstruction coefficients. Rows 0..12: Table 2 (a_{m,l}, l = i-3..i+3). Rows 13..19: Table 1
// (TENO5 single polynomials, l = i-2..i+2 placed in columns 1..5). Exact rationals; each entry is
// the correctly rounded quotient in the working precision.
// ------------------------------------------------------------------------------------------------
struct Rat { int n, d; };
constexpr int NCOEF_ROWS = 20;
__device__ constexpr Rat COEF[NCOEF_ROWS][7] = {
    {{-1, 140}, {5, 84}, {-101, 420}, {319, 420}, {107, 210}, {-19, 210}, {1, 105}},
    {{0, 1}, {1, 60}, {-2, 15}, {37, 60}, {37, 60}, {-2, 15}, {1, 60}},
    {{-1, 60}, {7, 60}, {-23, 60}, {19, 20}, {11, 30}, {-1, 30}, {0, 1}},
    {{0, 1}, {0, 1}, {-1, 20}, {9, 20}, {47, 60}, {-13, 60}, {1, 30}},
    {{0, 1}, {1, 30}, {-13, 60}, {47, 60}, {9, 20}, {-1, 20}, {0, 1}},
    {{-1, 20}, {17, 60}, {-43, 60}, {77, 60}, {1, 5}, {0, 1}, {0, 1}},
    {{0, 1}, {0, 1}, {0, 1}, {1, 4}, {13, 12}, {-5, 12}, {1, 12}},
    {{0, 1}, {0, 1}, {-1, 12}, {7, 12}, {7, 12}, {-1, 12}, {0, 1}},
    {{0, 1}, {1, 12}, {-5, 12}, {13, 12}, {1, 4}, {0, 1}, {0, 1}},
    {{-1, 4}, {13, 12}, {-23, 12}, {25, 12}, {0, 1}, {0, 1}, {0, 1}},
    {{0, 1}, {0, 1}, {0, 1}, {1, 3}, {5, 6}, {-1, 6}, {0, 1}},
    {{0, 1}, {0, 1}, {-1, 6}, {5, 6}, {1, 3}, {0, 1}, {0, 1}},
    {{0, 1}, {1, 3}, {-7, 6}, {11, 6}, {0, 1}, {0, 1}, {0, 1}},
    // Table 1, rows for (delta0,delta1,delta2) = 111, 011, 110, 001, 010, 100, 101
    {{0, 1}, {1, 30}, {-13, 60}, {47, 60}, {9, 20}, {-1, 20}, {0, 1}},
    {{0, 1}, {0, 1}, {-1, 9}, {2, 3}, {1, 2}, {-1, 18}, {0, 1}},
    {{0, 1}, {1, 21}, {-13, 42}, {41, 42}, {2, 7}, {0, 1}, {0, 1}},
    {{0, 1}, {0, 1}, {0, 1}, {1, 3}, {5, 6}, {-1, 6}, {0, 1}},
    {{0, 1}, {0, 1}, {-1, 6}, {5, 6}, {1, 3}, {0, 1}, {0, 1}},
    {{0, 1}, {1, 3}, {-7, 6}, {11, 6}, {0, 1}, {0, 1}, {0, 1}},
    {{0, 1}, {1, 12}, {-7, 24}, {17, 24}, {5, 8}, {-1, 8}, {0, 1}},
};
// TENO5 code (delta0<<2 | delta1<<1 | delta2) -> row of the table above. Code 0 cannot occur
// (at least one chi_k >= 1/3 > C_T); it maps to the full stencil and is reported as an error.
__device__ constexpr int TENO5_ROW[8] = {13, 16, 17, 14, 18, 19, 15, 13};

// TENO5_ROW for a per-lane code without a memory lookup: the table packed into one 64-bit word.
constexpr unsigned long long pack_teno5_rows()
{
    unsigned long long w = 0;
    for (int k = 0; k < 8; ++k) w |= (unsigned long long)TENO5_ROW[k] << (8 * k);
    return w;
}
__device__ __forceinline__ int teno5_row(int code)
{
    constexpr unsigned long long W = pack_teno5_rows();
    return (int)((W >> (8 * (code & 7))) & 0xffull);
}

// Row R of the coefficient table applied to seven upwind-ordered values, with the constants folded
// at compile time (each the correctly rounded quotient in T) and the zero taps dropped; the sum
// runs left to right like the table-driven path.
template <typename T, int R, int L>
__device__ __forceinline__ void recon_tap(T &h, bool &first, T w)
{
    if constexpr (COEF[R][L].n != 0) {
        constexpr T c = T(COEF[R][L].n) / T(COEF[R][L].d);
        if (first) {
            h = c * w;
            first = false;
        } else {
            h += c * w;
        }
    }
}

template <typename T, int R>
__device__ __forceinline__ T recon_const(T w0, T w1, T w2, T w3, T w4, T w5, T w6)
{
    T h = T(0);
    bool first = true;
    recon_tap<T, R, 0>(h, first, w0);
    recon_tap<T, R, 1>(h, first, w1);
    recon_tap<T, R, 2>(h, first, w2);
    recon_tap<T, R, 3>(h, first, w3);
    recon_tap<T, R, 4>(h, first, w4);
    recon_tap<T, R, 5>(h, first, w5);
    recon_tap<T, R, 6>(h, first, w6);
    return h;
}

// Table 3 as printed: neighbour vector (a,b,c,d,e) = (delta_{i-1,0}, delta_{i,0}, delta_{i,1},
// delta_{i,2}, delta_{i+1,2}) -> Table 2 row; '*' matches 0 or 1; (*,0,0,0,*) has no stencil.
struct Pattern { const char *p; int m; };
constexpr Pattern TABLE3[13] = {
    {"11111", 0}, {"01111", 1}, {"11110", 2}, {"*0111", 3}, {"01110", 4}, {"1110*", 5},
    {"**011", 6}, {"*0110", 7}, {"0110*", 8}, {"1100*", 9}, {"**010", 10}, {"*010*", 11},
    {"0100*", 12}};

constexpr bool pattern_matches(const char *p, int idx)
{
    for (int q = 0; q < 5; ++q) {
        int bit = (idx >> (4 - q)) & 1;
        if (p[q] != '*' && (p[q] - '0') != bit) return false;
    }
    return true;
}

// 32 entries x 4 bits: entry idx = 16a+8b+4c+2d+e, value m, 15 = no stencil.
constexpr unsigned long long table3_lut_half(int half)
{
    unsigned long long w = 0;
    for (int j = 0; j < 16; ++j) {
        int idx = half * 16 + j, m = 15;
        for (int r = 0; r < 13; ++r)
            if (pattern_matches(TABLE3[r].p, idx)) m = TABLE3[r].m;
        w |= (unsigned long long)m << (4 * j);
    }
    return w;
}
constexpr unsigned long long LUT_LO = table3_lut_half(0);
constexpr unsigned long long LUT_HI = table3_lut_half(1);

__device__ __forceinline__ int table3(unsigned idx)
{
    unsigned long long w = (idx & 16u) ? LUT_HI : LUT_LO;
    return (int)((w >> (4u * (idx & 15u))) & 15ull);
}

// The same table indexed in reversed bit order, r = a + 2b + 4c + 8d + 16e, which is how the
// kernels assemble the neighbour vector (the three flags of a face are stored as delta_0 | delta_1 << 1
// | delta_2 << 2, so b, c, d land in order with one shift).
constexpr int reverse5(int x)
{
    int r = 0;
    for (int i = 0; i < 5; ++i)
        if ((x >> i) & 1) r |= 1 << (4 - i);
    return r;
}
constexpr unsigned long long table3_rev_half(int half)
{
    unsigned long long w = 0;
    for (int j = 0; j < 16; ++j) {
        const int idx = reverse5(half * 16 + j);
        const unsigned long long hw = (idx & 16) ? table3_lut_half(1) : table3_lut_half(0);
        w |= ((hw >> (4 * (idx & 15))) & 15ull) << (4 * j);
    }
    return w;
}
constexpr unsigned long long LUT_REV_LO = table3_rev_half(0);
constexpr unsigned long long LUT_REV_HI = table3_rev_half(1);

__device__ __forceinline__ int table3_rev(unsigned r)
{
    unsigned long long w = (r & 16u) ? LUT_REV_HI : LUT_REV_LO;
    return (int)((w >> (4u * (r & 15u))) & 15ull);
}

// ------------------------------------------------------------------------------------------------
// Five-point cut-off of one split side (eq:smooth_expl, eq:tau5, eq:TENO1 with C = 1, q = 6,
// eq:norm, eq:seclect). (a..e) = values at i-2..i+2 in upwind order.
//
// smooth5() computes B_k = 4 beta_k and 4 tau5 = |B_0 - B_2|. The cut-off and the shortcut below
// depend on the measures only through tau5 / (beta_k + eps), so the kernels carry the measures four
// times larger together with eps4 = 4 eps (a power of two: the same ratios).
// Exact shortcut: with r_k = 1 + tau5/(beta_k + eps) >= 1, the smallest chi_k is at least
// 1 / (1 + 2 (r_max/r_min)^6); if tau5 <= K (min_k beta_k + eps) then r_max/r_min <= 1 + K and
// chi_min >= 1 / (1 + 2 (1 + K)^6). K is chosen on the host from C_T (smooth_shortcut_k) with a
// margin that covers rounding, so every delta_k = 1 on that branch (C_T = 1e-5: K = 5.0, chi_min
// >= 1/93313). The test is evaluated as 4 tau5 <= K min_k B_k + K eps4, with K eps4 from the host.
// cutoff3() evaluates the definition: delta_k = 0 iff gamma_k / sum(gamma) < C_T, computed as
// gamma_k < C_T * sum(gamma) with gamma_k = (1 + tau (D_j D_l) / (D0 D1 D2))^6, D_k = B_k + eps4:
// one reciprocal per side instead of six divisions; equal to the definition up to rounding, so a
// flag can differ from a straight evaluation only when chi_k lies within rounding of C_T.
// ------------------------------------------------------------------------------------------------
template <typename T> struct Smooth { T b0, b1, b2, tau; };

template <typename T>
__device__ __forceinline__ Smooth<T> smooth5(T a, T b, T c, T d, T e)
{
    // eq:smooth_expl regrouped: 4 beta_k = q_k^2 + (13/3) u_k^2 with the second differences u_k and
    // the one-sided first differences q_k, all from the central differences x = c - b, y = c - d:
    //   u0 = a - 2b + c = (a - b) + x,  u1 = b - 2c + d = -(x + y),  u2 = c - 2d + e = (e - d) + y,
    //   q0 = a - 4b + 3c = u0 + 2x,     q1 = b - d = y - x,          q2 = 3c - 4d + e = u2 + 2y
    // (u1 enters squared, so its sign is dropped)
    const T x = c - b, y = c - d;
    const T u0 = (a - b) + x;
    const T u1 = x + y;
    const T u2 = (e - d) + y;
    const T q0 = fma(T(2), x, u0);
    const T q1 = y - x;
    const T q2 = fma(T(2), y, u2);
    constexpr T K = T(13.0 / 3.0);
    Smooth<T> r;
    r.b0 = fma(K * u0, u0, q0 * q0);
    r.b1 = fma(K * u1, u1, q1 * q1);
    r.b2 = fma(K * u2, u2, q2 * q2);
    r.tau = fabs(r.b0 - r.b2);
    return r;
}

template <typename T>
__device__ __forceinline__ bool all_smooth(const Smooth<T> &m, T k, T keps4)
{
    T bmin = fmin(m.b0, fmin(m.b1, m.b2));
    return m.tau <= fma(k, bmin, keps4);
}

// Largest K of the shortcut for cut-off ct and the constants C, q of eq:TENO1: with
// tau5 <= K (beta_min + eps) every r_k lies in [C, C + K], so chi_min >= 1 / (1 + 2 (1 + K/C)^q), which
// must stay >= ct with room for rounding; K is taken 1% below the bound and capped at 5 C
// (C = 1, q = 6, ct = 1e-5: K = 5).
inline double smooth_shortcut_k(double ct, double C, int q)
{
    double kmax = C * (pow((1.0 / ct - 1.0) * 0.5, 1.0 / q) - 1.0);
    double k = 0.99 * kmax;
    return k < 0.0 ? 0.0 : (k > 5.0 * C ? 5.0 * C : k);
}

// Reciprocal from the hardware estimate and two Newton steps (argument normal and positive).
__device__ __forceinline__ double recip(double x)
{
    double r = __builtin_amdgcn_rcp(x);
    double e = fma(-x, r, 1.0);
    r = fma(r, e, r);
    e = fma(-x, r, 1.0);
    return fma(r, e, r);
}
__device__ __forceinline__ float recip(float x) { return 1.0f / x; }

// Square root and reciprocal square root of a normal positive double: the hardware estimate
// y ~ 1/sqrt(x), then coupled Newton steps on g ~ sqrt(x) and h ~ 1/(2 sqrt(x)) (each step squares
// the relative error), ending with a residual correction of g. Within about an ulp of the correctly
// rounded values; non-positive or non-finite x give NaN or infinities.
__device__ __forceinline__ void sqrt_rsqrt(double x, double &s, double &rs)
{
    const double y = __builtin_amdgcn_rsq(x);
    double g = x * y, h = 0.5 * y;
    double r = fma(-h, g, 0.5);
    g = fma(g, r, g);
    h = fma(h, r, h);
    r = fma(-h, g, 0.5);
    g = fma(g, r, g);
    h = fma(h, r, h);
    const double d = fma(-g, g, x);
    s = fma(d, h, g);
    rs = 2.0 * h;
}
__device__ __forceinline__ void sqrt_rsqrt(float x, float &s, float &rs)
{
    s = sqrtf(x);
    rs = 1.0f / s;
}
template <typename T> __device__ __forceinline__ T fast_sqrt(T x)
{
    T s, rs;
    sqrt_rsqrt(x, s, rs);
    return s;
}

// r^q for the exponent q of eq:TENO1. QC = 6: the paper's q = 6 fixed at compile time, ((r r) r)^2;
// QC = 0: q taken at run time, q - 1 products (for q = 6 the same products in the same order).
template <int QC, typename T> __device__ __forceinline__ T pow_q(T r, int q)
{
    if constexpr (QC == 6) {
        T g = r * r * r;
        return g * g;
    } else {
        if (q == 6) return pow_q<6>(r, 6);
        T g = r;
        for (int j = 1; j < q; ++j) g *= r;
        return g;
    }
}

// gamma_k = (C + tau5 / (beta_k + eps))^q of the three substencils, up to one common positive factor
// (the cut-off and chi only use their ratios).
template <int QC>
__device__ __forceinline__ void gamma3(const Smooth<double> &m, double eps4, double C, int q, double g[3])
{
    double D0 = m.b0 + eps4, D1 = m.b1 + eps4, D2 = m.b2 + eps4;
    double D01 = D0 * D1;
    double tinv = m.tau * recip(D01 * D2);
    double r0 = C + tinv * (D1 * D2);
    double r1 = C + tinv * (D0 * D2);
    double r2 = C + tinv * D01;
    g[0] = pow_q<QC>(r0, q);
    g[1] = pow_q<QC>(r1, q);
    g[2] = pow_q<QC>(r2, q);
}

// Single precision: gamma_k / gamma_max keeps every term in [0, 1] (no overflow of r^q).
template <int QC>
__device__ __forceinline__ void gamma3(const Smooth<float> &m, float eps4, float C, int q, float g[3])
{
    float r0 = C + m.tau / (m.b0 + eps4), r1 = C + m.tau / (m.b1 + eps4), r2 = C + m.tau / (m.b2 + eps4);
    float rm = fmaxf(r0, fmaxf(r1, r2));
    g[0] = pow_q<QC>(r0 / rm, q);
    g[1] = pow_q<QC>(r1 / rm, q);
    g[2] = pow_q<QC>(r2 / rm, q);
}

template <int QC, typename T>
__device__ __forceinline__ unsigned cutoff3(const Smooth<T> &m, T eps4, T ct, T C, int q)
{
    T g[3];
    gamma3<QC>(m, eps4, C, q, g);
    T thr = ct * ((g[0] + g[1]) + g[2]);
    return (g[0] < thr ? 0u : 1u) | (g[1] < thr ? 0u : 2u) | (g[2] < thr ? 0u : 4u);
}

// chi_k of eq:norm from the same gamma_k.
template <typename T>
__device__ __forceinline__ void chi3(const Smooth<T> &m, T eps4, T C, int q, T chi[3])
{
    T g[3];
    gamma3<0>(m, eps4, C, q, g);
    const T s = (g[0] + g[1]) + g[2];
    chi[0] = g[0] / s;
    chi[1] = g[1] / s;
    chi[2] = g[2] / s;
}

// Roe-averaged quantities of one face and the rows/columns of its eigenvector matrices.
template <typename T> struct Roe {
    T un = T(0), ut = T(0), cs = T(1), ic = T(1), H = T(0), q2 = T(0), b1 = T(0), b2 = T(0);
};

// Left eigenvector (row s of L) and right eigenvector (column s of R) of the flux Jacobian at the
// Roe state, in local variable order (rho, m_n, [m_t], E). Fields: u_n - c, u_n (entropy),
// [u_n (shear)], u_n + c. With b1 = (gamma-1)/c^2 and b2 = b1 |u|^2 / 2, L R = I.
// LS scales the row by LS (a power of two, so the scaled row is exactly LS times the plain one);
// the sweeps take LS = 1/2, the half of the flux splitting, folded into each row's own constants.
// Scalar systems: L = LS, R = 1.
// characteristic = false: the reconstruction runs per conserved component; field s is the conserved
// variable s (global order), which is local component `comp` of the sweep: L = LS e_comp, R = e_comp.
template <typename T, int NV, int LSINV = 1>
__device__ __forceinline__ void char_basis(const Roe<T> &r, int s, T L[NV], T R[NV], bool characteristic = true,
                                           int comp = 0)
{
    static_assert(LSINV == 1 || LSINV == 2, "row scale 1 or 1/2");
    constexpr T LS = T(1) / T(LSINV);
    if constexpr (NV == 1) {
        L[0] = LS;
        R[0] = T(1);
    } else if (!characteristic) {
#pragma unroll
        for (int v = 0; v < NV; ++v) {
            L[v] = v == comp ? LS : T(0);
            R[v] = v == comp ? T(1) : T(0);
        }
    } else {
        const T h = T(0.5) * LS;
        // map the 1D fields (0, 1, 2) onto the 2D ones (0, 1, 3)
        const int s4 = (NV == 3 && s == 2) ? 3 : s;
        T l0, l1, l2 = T(0), l3, r0, r1, r2 = T(0), r3;
        switch (s4) {
        case 0:
            l0 = h * (r.b2 + r.un * r.ic); l1 = -h * (r.b1 * r.un + r.ic); l2 = -h * r.b1 * r.ut; l3 = h * r.b1;
            r0 = T(1); r1 = r.un - r.cs; r2 = r.ut; r3 = r.H - r.un * r.cs;
            break;
        case 1: {
            const T t = LS * r.b1;
            l0 = fma(-LS, r.b2, LS); l1 = t * r.un; l2 = t * r.ut; l3 = -t;
            r0 = T(1); r1 = r.un; r2 = r.ut; r3 = T(0.5) * r.q2;
            break;
        }
        case 2:
            l0 = -LS * r.ut; l1 = T(0); l2 = LS; l3 = T(0);
            r0 = T(0); r1 = T(0); r2 = T(1); r3 = r.ut;
            break;
        default:
            l0 = h * (r.b2 - r.un * r.ic); l1 = -h * (r.b1 * r.un - r.ic); l2 = -h * r.b1 * r.ut; l3 = h * r.b1;
            r0 = T(1); r1 = r.un + r.cs; r2 = r.ut; r3 = r.H + r.un * r.cs;
            break;
        }
        if constexpr (NV == 3) {
            L[0] = l0; L[1] = l1; L[2] = l3;
            R[0] = r0; R[1] = r1; R[2] = r3;
        } else {
            L[0] = l0; L[1] = l1; L[2] = l2; L[3] = l3;
            R[0] = r0; R[1] = r1; R[2] = r2; R[3] = r3;
        }
    }
}

// Neighbour exchange along the wave with the data-parallel-primitive whole-wave shifts (one ALU move
// per 32-bit word, no LDS traffic): shfl_up1 gives lane k the value of lane k-1 (wave_shr:1),
// shfl_dn1 the value of lane k+1 (wave_shl:1); the end lane keeps its own value.
template <int CTRL> __device__ __forceinline__ unsigned dpp_word(unsigned v)
{
    return (unsigned)__builtin_amdgcn_update_dpp((int)v, (int)v, CTRL, 0xf, 0xf, false);
}
template <int CTRL> __device__ __forceinline__ double dpp_shift(double v)
{
    const unsigned long long b = (unsigned long long)__double_as_longlong(v);
    const unsigned lo = dpp_word<CTRL>((unsigned)b), hi = dpp_word<CTRL>((unsigned)(b >> 32));
    return __longlong_as_double((long long)(((unsigned long long)hi << 32) | lo));
}
template <int CTRL> __device__ __forceinline__ float dpp_shift(float v)
{
    return __uint_as_float(dpp_word<CTRL>(__float_as_uint(v)));
}
template <int CTRL> __device__ __forceinline__ unsigned dpp_shift(unsigned v) { return dpp_word<CTRL>(v); }
template <typename T> __device__ __forceinline__ T shfl_up1(T v) { return dpp_shift<0x138>(v); }
template <typename T> __device__ __forceinline__ T shfl_dn1(T v) { return dpp_shift<0x130>(v); }
// Same moves for a double where lanes without a source may read 0 (bound_ctrl): one instruction per
// word, no copy of the old value.
template <int CTRL> __device__ __forceinline__ double dpp_shift_z(double v)
{
    const unsigned long long b = (unsigned long long)__double_as_longlong(v);
    const unsigned lo = (unsigned)__builtin_amdgcn_update_dpp(0, (int)(unsigned)b, CTRL, 0xf, 0xf, true);
    const unsigned hi = (unsigned)__builtin_amdgcn_update_dpp(0, (int)(unsigned)(b >> 32), CTRL, 0xf, 0xf, true);
    return __longlong_as_double((long long)(((unsigned long long)hi << 32) | lo));
}
template <int CTRL> __device__ __forceinline__ float dpp_shift_z(float v)
{
    return __uint_as_float((unsigned)__builtin_amdgcn_update_dpp(0, (int)__float_as_uint(v), CTRL, 0xf, 0xf, true));
}
template <typename T> __device__ __forceinline__ T shfl_dn1_z(T v) { return dpp_shift_z<0x130>(v); }

// ------------------------------------------------------------------------------------------------
// Sweep kernel arguments.
// ------------------------------------------------------------------------------------------------
template <typename T> struct SweepArgs {
    const T *U;                 // stage input state [nv][ny][nx]
    const T *U0;                // MODE_STAGE: RK base state
    const T *addend;            // nullable: dU of the other direction, added per cell
    T *out;                     // MODE_RHS: dU/dt; MODE_STAGE: next stage state
    T *Fout;                    // MODE_FACES: face fluxes
    T *chi_out;                 // MODE_FACES, nullable: chi of eq:norm, 24 per face (this direction's section)
    uint32_t *masks_out;        // nullable: face mask words (this direction's section)
    uint32_t *flags_out;        // nullable: face flag words (this direction's section)
    const uint32_t *masks_in;   // FROZEN kernels: mask words (this direction's section)
    const double *alpha;        // 8 Lax-Friedrichs constants (device)
    const double *dt;           // MODE_STAGE: step size (device)
    unsigned long long *part;   // MODE_STAGE: [NCOPY][NWORD] maxima of the produced state
    unsigned *err;
    int nx, ny;                 // grid
    int len, nlines;            // cells per line along the sweep, number of lines
    int nseg;                   // segments per line
    int ntiles;                 // tiles of the sweep (one block each)
    int bc;                     // boundary condition along the sweep
    int bc_other;               // (unused by the sweep itself)
    int mode, stage, scheme, alpha_mode;
    T inv_h, ct, gamma, adv;
    T eps4;                     // 4 eps: the eps of the measures as smooth5() scales them
    T smooth_k;                 // all-smooth shortcut factor for ct (smooth_shortcut_k)
    T keps4;                    // smooth_k * eps4
    T gm1;                      // gamma - 1
    T inv_dx, inv_dy;           // for the CFL denominator of the produced state
    T C;                        // C of eq:TENO1
    int q;                      // q of eq:TENO1
    int characteristic;         // 0: reconstruction per conserved component
};

// Wave speeds of one cell for the GLF constants and the CFL rule.
// w[0..3]: |lambda| of the x fields, w[4..7]: y fields, w[8]: (|u|+c)/dx [+ (|v|+c)/dy].
template <typename T, int SYS>
__device__ __forceinline__ bool cell_speeds(const T *u, T gamma, T adv, T inv_dx, T inv_dy, int alpha_mode,
                                            double w[9])
{
    for (int k = 0; k < 9; ++k) w[k] = 0.0;
    if constexpr (SYS == ADV1D) {
        double a = fabs((double)adv);
        w[0] = a;
        w[8] = a * (double)inv_dx;
        return isfinite(u[0]);
    } else if constexpr (SYS == BURGERS1D) {
        double a = fabs((double)u[0]);
        w[0] = a;
        w[8] = a * (double)inv_dx;
        return isfinite(u[0]);
    } else {
        constexpr int NV = Sys<SYS>::NV;
        T rho = u[0], mx = u[1], my = NV == 4 ? u[2] : T(0), E = u[NV - 1];
        T ir = rho > T(0) ? recip(rho) : T(1) / rho;
        T vx = mx * ir, vy = my * ir;
        T p = (gamma - T(1)) * (E - T(0.5) * rho * (vx * vx + vy * vy));
        bool ok = rho > T(0) && p > T(0) && isfinite(E);
        T cs = sqrt(gamma * p * ir);
        double c = (double)cs, ux = (double)vx, uy = (double)vy;
        if (alpha_mode) {
            w[0] = w[1] = w[2] = fabs(ux) + c;      // (one-dimensional Euler has three fields)
            if (NV == 4) {
                w[3] = w[0];
                w[4] = w[5] = w[6] = w[7] = fabs(uy) + c;
            }
        } else if (NV == 3) {
            w[0] = fabs(ux - c); w[1] = fabs(ux); w[2] = fabs(ux + c);
        } else {
            w[0] = fabs(ux - c); w[1] = fabs(ux); w[2] = fabs(ux); w[3] = fabs(ux + c);
            w[4] = fabs(uy - c); w[5] = fabs(uy); w[6] = fabs(uy); w[7] = fabs(uy + c);
        }
        w[8] = (fabs(ux) + c) * (double)inv_dx;
        if (NV == 4) w[8] = w[8] + (fabs(uy) + c) * (double)inv_dy;
        return ok;
    }
}

// Velocity components and sound speed of one cell (scalar systems: the characteristic speed in
// sx, 0 elsewhere). Returns false for a non-physical or non-finite state.
template <typename T, int SYS>
__device__ __forceinline__ bool cell_primitive_speeds(const T *u, T gamma, T gm1, T adv, double &sx, double &sy,
                                                      double &sc)
{
    if constexpr (SYS == ADV1D) {
        sx = (double)adv; sy = 0.0; sc = 0.0;
        return isfinite(u[0]);
    } else if constexpr (SYS == BURGERS1D) {
        sx = (double)u[0]; sy = 0.0; sc = 0.0;
        return isfinite(u[0]);
    } else {
        constexpr int NV = Sys<SYS>::NV;
        T rho = u[0], mx = u[1], my = NV == 4 ? u[2] : T(0), E = u[NV - 1];
        T ir = recip(rho);
        T vx = mx * ir, vy = my * ir;
        T p = gm1 * (E - T(0.5) * rho * (vx * vx + vy * vy));
        bool ok = rho > T(0) && p > T(0) && isfinite(E);
        sc = (double)fast_sqrt(gamma * p * ir);
        sx = (double)vx;
        sy = (double)vy;
        return ok;
    }
}

// The physicality test of cell_primitive_speeds alone (rho > 0, p > 0, finite energy; scalar systems:
// a finite value), the same arithmetic.
template <typename T, int SYS>
__device__ __forceinline__ bool cell_physical(const T *u, T gm1)
{
    if constexpr (SYS == ADV1D || SYS == BURGERS1D) {
        return isfinite(u[0]);
    } else {
        constexpr int NV = Sys<SYS>::NV;
        T rho = u[0], mx = u[1], my = NV == 4 ? u[2] : T(0), E = u[NV - 1];
        T ir = recip(rho);
        T vx = mx * ir, vy = my * ir;
        T p = gm1 * (E - T(0.5) * rho * (vx * vx + vy * vy));
        return rho > T(0) && p > T(0) && isfinite(E);
    }
}

// The words of the wave-speed record a system with NV conserved variables produces (the second
// acoustic-free x/y field repeats the first), and their indices packed 4 bits per used slot.
template <int NV> struct SpeedWords {
    static constexpr bool use(int q)
    {
        return q == 0 || q == 8 || (q == 1 && NV != 1) || (q == 2 && NV == 3) ||
               ((q == 3 || q == 4 || q == 5 || q == 7) && NV == 4);
    }
    static constexpr int count()
    {
        int n = 0;
        for (int q = 0; q < 9; ++q) n += use(q) ? 1 : 0;
        return n;
    }
    static constexpr unsigned pack()
    {
        unsigned p = 0;
        int u = 0;
        for (int q = 0; q < 9; ++q)
            if (use(q)) p |= (unsigned)q << (4 * u++);
        return p;
    }
};

// Word q of the wave-speed record (same layout as cell_speeds): 0-3 |lambda| of the x fields,
// 4-7 of the y fields, 8 the CFL denominator.
template <int SYS>
__device__ __forceinline__ double speed_word(int q, double ux, double uy, double c, double inv_dx, double inv_dy,
                                             int alpha_mode)
{
    constexpr int NV = Sys<SYS>::NV;
    if (SYS == ADV1D || SYS == BURGERS1D) return q == 0 ? fabs(ux) : (q == 8 ? fabs(ux) * inv_dx : 0.0);
    if (q == 8) {
        double w = (fabs(ux) + c) * inv_dx;
        if (NV == 4) w = w + (fabs(uy) + c) * inv_dy;
        return w;
    }
    const double un = q < 4 ? ux : uy;
    if (alpha_mode) return fabs(un) + c;
    const int f = q & 3;
    if (NV == 3) return f == 0 ? fabs(un - c) : (f == 1 ? fabs(un) : (f == 2 ? fabs(un + c) : 0.0));
    return f == 0 ? fabs(un - c) : (f == 3 ? fabs(un + c) : fabs(un));
}

__device__ __forceinline__ double wave_max(double v)
{
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v = fmax(v, __shfl_xor(v, o, WAVE));
    return v;
}

// Maximum of an unsigned word over the wave (returned in every lane): running maxima inside each
// 16-lane row by row shifts of 1, 2, 4, 8, then across rows by the row-15 and row-31 broadcasts,
// which leave the wave's maximum in lane 63. Lanes without a source read 0, the identity.
__device__ __forceinline__ unsigned wave_max_u32(unsigned v)
{
    v = max(v, (unsigned)__builtin_amdgcn_update_dpp(0, (int)v, 0x111, 0xf, 0xf, false));   // row_shr:1
    v = max(v, (unsigned)__builtin_amdgcn_update_dpp(0, (int)v, 0x112, 0xf, 0xf, false));   // row_shr:2
    v = max(v, (unsigned)__builtin_amdgcn_update_dpp(0, (int)v, 0x114, 0xf, 0xf, false));   // row_shr:4
    v = max(v, (unsigned)__builtin_amdgcn_update_dpp(0, (int)v, 0x118, 0xf, 0xf, false));   // row_shr:8
    v = max(v, (unsigned)__builtin_amdgcn_update_dpp(0, (int)v, 0x142, 0xa, 0xf, false));   // row_bcast:15
    v = max(v, (unsigned)__builtin_amdgcn_update_dpp(0, (int)v, 0x143, 0xc, 0xf, false));   // row_bcast:31
    return (unsigned)__builtin_amdgcn_readlane((int)v, 63);
}

// Maximum over the wave of a finite non-negative double. Such doubles order like their bit
// patterns, so the maximum is taken on the high words, then on the low words of the lanes that
// hold the maximal high word: exact, and without floating-point compares.
__device__ __forceinline__ double wave_max_nonneg(double x)
{
    const unsigned long long b = (unsigned long long)__double_as_longlong(x);
    const unsigned hi = (unsigned)(b >> 32), lo = (unsigned)b;
    const unsigned mh = wave_max_u32(hi);
    const unsigned ml = wave_max_u32(hi == mh ? lo : 0u);
    return __longlong_as_double((long long)(((unsigned long long)mh << 32) | ml));
}

// Block-wide maxima of nine per-lane values -> one atomicMax per word into one spread copy.
__device__ __forceinline__ void block_max_atomic(double w[9], unsigned long long *copy, double *lds9)
{
    const int lane = threadIdx.x & (WAVE - 1), wid = threadIdx.x / WAVE;
#pragma unroll
    for (int k = 0; k < 9; ++k) w[k] = wave_max(w[k]);
    if (lane == 0)
        for (int k = 0; k < 9; ++k) lds9[wid * 9 + k] = w[k];
    __syncthreads();
    if (threadIdx.x < 9) {
        double m = 0.0;
        for (int q = 0; q < BLOCK / WAVE; ++q) m = fmax(m, lds9[q * 9 + threadIdx.x]);
        atomicMax(copy + threadIdx.x, (unsigned long long)__double_as_longlong(m));
    }
}

// ------------------------------------------------------------------------------------------------
// The sweep kernel.
//   DIR: 0 = x (lines are rows), 1 = y (lines are columns).
//   FROZEN: the selection is read from masks_in instead of being measured.
// ------------------------------------------------------------------------------------------------
// Register budget of the sweep kernels: the minimum number of waves per SIMD the compiler must fit.
// Measured on MI355X (2D Euler, FP64, 4096^2): 4 for x- and y-sweeps; frozen-selection 1D Euler
// sweeps keep 3 (4 makes them spill).
#ifndef TENO_MIN_WAVES_X
#define TENO_MIN_WAVES_X 4
#endif
#ifndef TENO_MIN_WAVES_Y
#define TENO_MIN_WAVES_Y 4
#endif

// LDS record stride of one staged segment (odd: the y staging stores spread over the banks).
template <int SYS> constexpr int seg_stride() { return Rec<SYS>::NREC * SEG_LOAD + 1; }

// LDS pointer type, and the record field of the projection's i-th stencil operand (the conserved
// variables, then u_n and p).
template <typename T> using lds_cptr = __attribute__((address_space(3))) const T *;
template <int SYS> constexpr int proj_field(int i)
{
    if constexpr (SYS == EULER1D || SYS == EULER2D)
        return i < Sys<SYS>::NV ? i : (i == Sys<SYS>::NV ? Rec<SYS>::UN : Rec<SYS>::P);
    else
        return 0;
}

// x-sweeps (other than packed tails) keep one field-major record for the whole tile, [NREC][stride]:
// the tile's segments, when they lie on one line, overlap at positions 61 s (their cells are staged
// once), else sit at positions 72 s. Other sweeps keep one record per segment, [NSEG][NREC][72] + 1.
template <int NSEG> constexpr int xrec_stride() { return NSEG * SEG_LOAD + 1; }
template <int SYS, int DIR, int NSEG, bool PACK> constexpr int rec_size()
{
    return (DIR == 0 && !PACK && Rec<SYS>::NREC * xrec_stride<NSEG>() > NSEG * seg_stride<SYS>())
               ? Rec<SYS>::NREC * xrec_stride<NSEG>()
               : NSEG * seg_stride<SYS>();
}

// Fill the block's coefficient table (rows of Tables 2 and 1, correctly rounded in T).
// The coefficient rows in the working precision, 8 per row (the eighth 0), divided at compile time
// (correctly rounded, as a run-time division would be); each block copies them into its LDS.
template <typename T> struct CoefTable { T v[NCOEF_ROWS * 8]; };
template <typename T> constexpr CoefTable<T> make_coef_table()
{
    CoefTable<T> t{};
    for (int r = 0; r < NCOEF_ROWS; ++r)
        for (int l = 0; l < 8; ++l) t.v[r * 8 + l] = l < 7 ? T(COEF[r][l].n) / T(COEF[r][l].d) : T(0);
    return t;
}
__device__ constexpr CoefTable<double> COEF_TAB_F64 = make_coef_table<double>();
__device__ constexpr CoefTable<float> COEF_TAB_F32 = make_coef_table<float>();
template <typename T> __device__ __forceinline__ const T *coef_table();
template <> __device__ __forceinline__ const double *coef_table<double>() { return COEF_TAB_F64.v; }
template <> __device__ __forceinline__ const float *coef_table<float>() { return COEF_TAB_F32.v; }

template <typename T> __device__ __forceinline__ void fill_coef(T *coef)
{
    const T *tab = coef_table<T>();
    for (int q = threadIdx.x; q < NCOEF_ROWS * 8; q += BLOCK) coef[q] = tab[q];
}

// One tile of a sweep: NSEG line segments staged together in LDS. `tile` enumerates the tiles of
// the sweep (x: NSEG consecutive segments of the row-major segment list; y: NSEG adjacent columns
// at one segment position). rec/ext: the block's LDS; coef: the coefficient rows (LDS or global);
// MODE_STAGE puts the wave-speed maxima of the produced cells into a.part, the block's spread copy.
// ext (x-sweeps with an RK stage or a y-part): LDS for the epilogue operands of the owned cells,
// [NSEG][2][NV][WAVE] (U^n, then the y-part of dU/dt), loaded with the tile.
template <typename T, int SYS, int DIR, bool FROZEN, int NSEG, int MODE, bool PACK = false>
__device__ __forceinline__ void sweep_tile(const SweepArgs<T> &a, int tile, T *rec, T *ext, const T *coef)
{
    static_assert(!PACK || (SYS == EULER2D && !FROZEN && MODE != MODE_FACES),
                  "packed ragged segments: 2D Euler sweeps without recorded selections");
    constexpr int NV = Sys<SYS>::NV;
    constexpr int SEG_STRIDE = seg_stride<SYS>();
    constexpr bool EULER = SYS == EULER1D || SYS == EULER2D;
    constexpr bool XREC = DIR == 0 && !PACK;                 // field-major tile record (x-sweeps)
    constexpr int FSTR = XREC ? xrec_stride<NSEG>() : SEG_LOAD;   // record stride between fields

    const int tid = threadIdx.x, lane = tid & (WAVE - 1), wid = tid / WAVE;
    const size_t ncell = (size_t)a.nx * a.ny;

    // segment s of this block -> (line, c0); line < 0 marks an empty slot
    auto seg_of = [&](int s, int &line, int &c0) { tile_segment(DIR, NSEG, tile, s, a.nseg, a.nlines, line, c0); };

    // packed ragged segments (PACK): the tile's lines start at pm.l0; piece i of segment s is line
    // pm.l0 + i NSEG + s; lane k belongs to piece pack_piece(pm, k)
    PackMap pm{0, 0, 1, 1, 0, 0};
    if constexpr (PACK) pm = pack_map(a.len, tile, NSEG);

    // Lax-Friedrichs constants of this direction and the stage's dt, read before any background copy
    // is issued (vector-memory completions are waited for in order) and kept in scalar registers
    double alv[4];
#pragma unroll
    for (int v = 0; v < 4; ++v) alv[v] = v < NV ? uniform_f64(a.alpha[4 * DIR + v]) : 0.0;
    const double dtv = MODE == MODE_STAGE ? uniform_f64(*a.dt) : 0.0;

    // ---- stage cells into LDS ----
    // x-sweeps: a tile whose segments lie on one line is staged by the whole block in one run of
    // (NSEG-1) 61 + 72 cells (one pass for 4 segments: the 11-cell overlaps of neighbouring segments
    // are loaded and converted once); otherwise each wave stages its own segments. y-sweeps: the
    // block stages its NSEG adjacent columns row by row, so that one global load reads NSEG
    // consecutive doubles of a row. A staged run spans cells c0-5 .. c0+66 with c0 < len (x tiles:
    // up to the last segment's), so for len >= SEG_LOAD one wrap suffices.
    unsigned bad = 0;
    const bool near = a.len >= SEG_LOAD;
    // packed x tails: a wave stages exactly the segment it computes, so the only block-wide ordering
    // needed is that of the caller's coefficient table and maxima slots; it is taken here, before any
    // load is in flight, and each wave then starts as soon as its own staging is done
    constexpr bool WAVE_LOCAL = DIR == 0 && PACK && TENO_X_WAVE_LOCAL;
    if constexpr (WAVE_LOCAL) lds_barrier();
    // record position of cell q of segment s (the field-major x record: 61 s + q when the tile lies
    // on one line, else 72 s + q); block-uniform
    int segoff = SEG_STRIDE;
    bool xcontig = false;
    if constexpr (XREC) {
        const int id0 = tile * NSEG;
        xcontig = id0 % a.nseg + NSEG <= a.nseg && id0 / a.nseg < a.nlines;
        segoff = xcontig ? SEG_CELLS : SEG_LOAD;
    }
    // a cell's conserved variables (sweep-local order: rho, m_n, [m_t], E), then its record entry
    auto load_cell = [&](size_t off, T u[NV]) {
        u[0] = a.U[off];
        if constexpr (EULER) {
            u[1] = a.U[(size_t)gvar<SYS, DIR>(1) * ncell + off];
            if constexpr (NV == 4) u[2] = a.U[(size_t)gvar<SYS, DIR>(2) * ncell + off];
            u[NV - 1] = a.U[(size_t)(NV - 1) * ncell + off];
        }
    };
    auto put_cell = [&](int pos, const T u[NV]) {
        T *r = rec + pos;
        if constexpr (!EULER) {
            r[0] = u[0];
        } else {
            using S = Rec<SYS>;
            const T rho = u[0], mn = u[1], mt = NV == 4 ? u[2] : T(0), E = u[NV - 1];
            T sq, rs;
            sqrt_rsqrt(rho, sq, rs);
            T ir = rs * rs;               // (rho <= 0 or NaN: rs is NaN, reported below and at the faces)
            T un = mn * ir, ut = mt * ir;
            T p = a.gm1 * (E - T(0.5) * rho * (un * un + ut * ut));
            if (!(rho > T(0) && p > T(0))) bad |= (isfinite(rho) && isfinite(p)) ? ERR_NONPHYSICAL : ERR_NONFINITE;
            r[0] = rho;
            r[FSTR * 1] = mn;
            if constexpr (NV == 4) r[FSTR * 2] = mt;
            r[FSTR * S::E] = E;
            r[FSTR * S::UN] = un;
            if constexpr (NV == 4) r[FSTR * S::UT] = ut;
            r[FSTR * S::P] = p;
            r[FSTR * S::RS] = rs;
        }
    };
    auto stage_cell = [&](int pos, size_t off) {
        T u[NV];
        load_cell(off, u);
        put_cell(pos, u);
    };
    // epilogue operands of the owned cells (lanes 1..61), staged with the tile so that their
    // latency overlaps the staging instead of the end of the face computation
    constexpr bool HAS_EXT = DIR == 0 && MODE != MODE_FACES && !PACK;
    if constexpr (PACK && DIR == 0) {
        for (int s = __builtin_amdgcn_readfirstlane(wid); s < NSEG; s += BLOCK / WAVE) {
            const int line0 = pm.l0 + s;                 // piece 0: the wave has no line if absent
            if (line0 >= a.nlines) continue;             // wave-uniform
            constexpr int IT = (SEG_LOAD + WAVE - 1) / WAVE;        // loads first, then conversions
            T uc[IT][NV];
#pragma unroll
            for (int it = 0; it < IT; ++it) {
                const int q = lane + it * WAVE;
                if (q < SEG_LOAD) {
                    const int i = pack_piece(pm, q), ql = q - i * pm.W;
                    int line = pack_line(pm, i, s, NSEG, a.nlines);
                    if (line < 0) line = line0;                 // idle positions: any valid cell
                    const int g = near ? bc_index_near(pm.c0 - SEG_HALO + ql, a.len, a.bc)
                                       : bc_index(pm.c0 - SEG_HALO + ql, a.len, a.bc);
                    load_cell((size_t)line * a.nx + g, uc[it]);
                }
            }
#pragma unroll
            for (int it = 0; it < IT; ++it)
                if (lane + it * WAVE < SEG_LOAD) put_cell(s * SEG_STRIDE + lane + it * WAVE, uc[it]);
        }
    } else if constexpr (PACK) {
        constexpr int NCELL = NSEG * SEG_LOAD, IT = (NCELL + BLOCK - 1) / BLOCK;   // loads first
        T uc[IT][NV];
        int pos[IT];
#pragma unroll
        for (int it = 0; it < IT; ++it) {
            const int idx = tid + it * BLOCK;
            pos[it] = -1;
            if (idx < NCELL) {
                const int s = idx % NSEG, q = idx / NSEG;
                const int line0 = pm.l0 + s;
                if (line0 < a.nlines) {
                    const int i = pack_piece(pm, q), ql = q - i * pm.W;
                    int line = pack_line(pm, i, s, NSEG, a.nlines);
                    if (line < 0) line = line0;
                    const int g = near ? bc_index_near(pm.c0 - SEG_HALO + ql, a.len, a.bc)
                                       : bc_index(pm.c0 - SEG_HALO + ql, a.len, a.bc);
                    pos[it] = s * SEG_STRIDE + q;
                    load_cell((size_t)g * a.nx + line, uc[it]);
                }
            }
        }
#pragma unroll
        for (int it = 0; it < IT; ++it)
            if (pos[it] >= 0) put_cell(pos[it], uc[it]);
    } else if constexpr (DIR == 0) {
        if (xcontig) {
            constexpr int NCELL = (NSEG - 1) * SEG_CELLS + SEG_LOAD;
            const int id0 = tile * NSEG;
            const int c00 = (id0 % a.nseg) * SEG_CELLS;
            const size_t lbase = (size_t)(id0 / a.nseg) * a.nx;
            for (int q = tid; q < NCELL; q += BLOCK) {
                const int g = near ? bc_index_near(c00 - SEG_HALO + q, a.len, a.bc)
                                   : bc_index(c00 - SEG_HALO + q, a.len, a.bc);
                stage_cell(q, lbase + g);
            }
        } else {
            for (int s = __builtin_amdgcn_readfirstlane(wid); s < NSEG; s += BLOCK / WAVE) {
                int line, c0;
                seg_of(s, line, c0);
                if (line < 0) continue;         // wave-uniform
                const size_t lbase = (size_t)line * a.nx;
                constexpr int IT = (SEG_LOAD + WAVE - 1) / WAVE;    // loads first, then conversions
                T uc[IT][NV];
#pragma unroll
                for (int it = 0; it < IT; ++it) {
                    const int q = lane + it * WAVE;
                    if (q < SEG_LOAD) {
                        const int g = near ? bc_index_near(c0 - SEG_HALO + q, a.len, a.bc)
                                           : bc_index(c0 - SEG_HALO + q, a.len, a.bc);
                        load_cell(lbase + g, uc[it]);
                    }
                }
#pragma unroll
                for (int it = 0; it < IT; ++it)
                    if (lane + it * WAVE < SEG_LOAD) put_cell(s * SEG_LOAD + lane + it * WAVE, uc[it]);
            }
        }
        for (int s = __builtin_amdgcn_readfirstlane(wid); s < NSEG; s += BLOCK / WAVE) {
            int line, c0;
            seg_of(s, line, c0);
            if (line < 0) continue;             // wave-uniform
            const size_t lbase = (size_t)line * a.nx;
            if constexpr (HAS_EXT) {
                // the owned cells' U^n and y-part (lanes 1..61 read cells c0 .. c0+60): copied into
                // LDS in the background (issued after the record loads, which are waited for in
                // order); waited for just before the epilogue
                // (slot element kk holds cell c0-1+kk; the copy fills elements 1..64, the last one
                // landing on the next slot's unused element 0, or on the array's padding)
                T *e = ext + (size_t)s * 2 * NV * WAVE + 1;
#pragma unroll
                for (int v = 0; v < NV; ++v) {
                    const size_t fo = (size_t)gvar<SYS, DIR>(v) * ncell + lbase;
                    if (MODE == MODE_STAGE && a.U0 != a.U) lds_dma_row(a.U0 + fo, a.nx, c0, e + v * WAVE, lane);
                    if (a.addend) lds_dma_row(a.addend + fo, a.nx, c0, e + (NV + v) * WAVE, lane);
                }
            }
        }
    } else {
        static_assert(DIR == 0 || (NSEG & (NSEG - 1)) == 0, "y-tiles hold a power-of-two number of columns");
        const int ntile = (a.nlines + NSEG - 1) / NSEG;
        const int line0 = (tile % ntile) * NSEG, c0 = (tile / ntile) * SEG_CELLS;
        // a thread's cells (up to IT of them) are all loaded before any is converted, so that the
        // loads' latencies overlap
        constexpr int NCELL = NSEG * SEG_LOAD, IT = (NCELL + BLOCK - 1) / BLOCK;
        T uc[IT][NV];
        int pos[IT];
#pragma unroll
        for (int it = 0; it < IT; ++it) {
            const int idx = tid + it * BLOCK;
            pos[it] = -1;
            if (idx < NCELL) {
                const int s = idx % NSEG, q = idx / NSEG;
                const int line = line0 + s;
                if (line < a.nlines) {
                    const int g = near ? bc_index_near(c0 - SEG_HALO + q, a.len, a.bc)
                                       : bc_index(c0 - SEG_HALO + q, a.len, a.bc);
                    pos[it] = s * SEG_STRIDE + q;
                    load_cell((size_t)g * a.nx + line, uc[it]);
                }
            }
        }
#pragma unroll
        for (int it = 0; it < IT; ++it)
            if (pos[it] >= 0) put_cell(pos[it], uc[it]);
    }
    if constexpr (WAVE_LOCAL)
        wave_lds_fence();
    else
        lds_barrier();

    // y-sweeps producing dU/dt leave their results in the segment's own LDS record and store the
    // tile row by row at the end (a lane's cells run down a column: direct stores would be strided)
    constexpr bool STAGE_OUT = DIR == 1 && MODE == MODE_RHS;
    constexpr int OUTW = PACK ? WAVE : SEG_CELLS;   // staged output per variable
    static_assert(NV * OUTW <= SEG_STRIDE, "staged output must fit in a segment record");

    // the segment loop is wave-uniform: keep its indices in scalar registers
    for (int s = __builtin_amdgcn_readfirstlane(wid); s < NSEG; s += BLOCK / WAVE) {
        int line, c0;
        if constexpr (PACK) {
            line = pm.l0 + s;
            c0 = pm.c0;
            if (line >= a.nlines) continue;     // wave-uniform
        } else {
            seg_of(s, line, c0);
            if (line < 0) continue;             // wave-uniform
        }
        const T *R0 = rec + s * segoff;
        const int k = lane_id_now();
        // this lane's line and position in it (packed: its piece's line and the lane within the piece)
        int kl = k;
        bool needed = true;                     // the lane's face or its flags are used
        if constexpr (PACK) {
            const int i = pack_piece(pm, k);
            kl = k - i * pm.W;
            needed = pack_line(pm, i, s, NSEG, a.nlines) >= 0 && kl <= pm.nt + 2;
        }
        const int f = c0 - 1 + kl;              // this lane's face
        bool face_ok = needed && kl >= 1 && kl <= 62 && f <= a.len;
        bool cell_ok = needed && kl >= 1 && kl <= 61 && f < a.len;
        // face index in this direction's face arrays
        auto face_index = [&](int ff) {
            return DIR == 0 ? (size_t)line * (a.len + 1) + ff : (size_t)ff * a.nx + line;
        };
        uint32_t mword_in = 0;
        if constexpr (FROZEN) mword_in = face_ok ? a.masks_in[face_index(f)] : 0u;

        T Fh[NV];
#pragma unroll
        for (int v = 0; v < NV; ++v) Fh[v] = T(0);
        uint32_t mword = 0, fword = 0;

        // Roe-averaged state of the face (cells i = q k+3 and i+1 = q k+4, Remark 3)
        Roe<T> roe;
        if constexpr (EULER) {
            using S = Rec<SYS>;
            const T gm1 = a.gm1;
            const T rsL = R0[FSTR * S::RS + k + 3], rsR = R0[FSTR * S::RS + k + 4];
            const T sL = R0[k + 3] * rsL, sR = R0[k + 4] * rsR;          // sqrt(rho)
            T isum = recip(sL + sR);
            roe.un = (sL * R0[FSTR * S::UN + k + 3] + sR * R0[FSTR * S::UN + k + 4]) * isum;
            roe.ut = T(0);
            if constexpr (NV == 4)
                roe.ut = (sL * R0[FSTR * S::UT + k + 3] + sR * R0[FSTR * S::UT + k + 4]) * isum;
            // sqrt(rho) H = (E + p) / sqrt(rho)
            roe.H = ((R0[FSTR * S::E + k + 3] + R0[FSTR * S::P + k + 3]) * rsL +
                     (R0[FSTR * S::E + k + 4] + R0[FSTR * S::P + k + 4]) * rsR) * isum;
            roe.q2 = roe.un * roe.un + roe.ut * roe.ut;
            T c2 = gm1 * (roe.H - T(0.5) * roe.q2);
            if (face_ok && !(c2 > T(0))) bad |= isfinite(c2) ? ERR_NONPHYSICAL : ERR_NONFINITE;
            sqrt_rsqrt(c2, roe.cs, roe.ic);
            roe.b1 = gm1 * roe.ic * roe.ic;
            roe.b2 = T(0.5) * roe.b1 * roe.q2;
        }

        // LDS addresses of this lane's stencil in the record fields the projection reads (the
        // conserved variables, u_n, p), made opaque so that they stay in registers across the field
        // loop: the fields lie farther apart than the paired reads' offsets reach, and addresses
        // rebuilt from the lane's base would cost an add per paired read
        constexpr int NPF = EULER ? NV + 2 : 1;
        lds_cptr<T> Fp[NPF];
#pragma unroll
        for (int i = 0; i < NPF; ++i) {
            Fp[i] = (lds_cptr<T>)(R0 + FSTR * proj_field<SYS>(i) + k);
            asm volatile("" : "+v"(Fp[i]));
        }

        // Characteristic fields one at a time (kept as a loop: only one field's split values are
        // live, which keeps the wave's register budget low enough for several waves per SIMD).
#pragma unroll 1
        for (int sf = 0; sf < NV; ++sf) {
            asm volatile("" ::: "memory");      // keep the stencil reads inside the field loop
            const T al = (T)(sf == 0 ? alv[0] : sf == 1 ? alv[1] : sf == 2 ? alv[2] : alv[3]);
            T Ls[NV], Rs[NV];
            {
                // computed here for this field only: the face state passes through an empty asm
                // statement that may change it, so the compiler can neither hoist all fields' rows out
                // of the loop (registers held across it) nor needs copies to keep them in place
                asm volatile("" : "+v"(roe.un), "+v"(roe.ut), "+v"(roe.cs), "+v"(roe.ic), "+v"(roe.H), "+v"(roe.q2),
                                  "+v"(roe.b1), "+v"(roe.b2));
                // (L/2: the 1/2 of the splitting)
                char_basis<T, NV, 2>(roe, sf, Ls, Rs, a.characteristic != 0, gvar<SYS, DIR>(sf));
            }
            T vp[8], vm[8];
            if (NV == 4 && sf == 2 && a.characteristic) {
                // shear field: L_2 = (-u_t, 0, 1, 0), so L_2 U = m_t - u_t rho and L_2 F = u_n L_2 U
#pragma unroll
                for (int j = 0; j < 8; ++j) {
                    T lu = Fp[2][j] * Ls[2] + Ls[0] * Fp[0][j];
                    T lf = Fp[NV][j] * lu;                    // u_n
                    vp[j] = lf + al * lu;
                    vm[j] = lf - al * lu;
                }
            } else {
#pragma unroll
                for (int j = 0; j < 8; ++j) {
                    T lu, lf;
                    if constexpr (!EULER) {
                        T u = Fp[0][j];
                        lu = T(0.5) * u;
                        lf = SYS == ADV1D ? a.adv * lu : lu * u * T(0.5);
                    } else {
                        T un = Fp[NV][j], p = Fp[NV + 1][j];
                        lu = Ls[0] * Fp[0][j];
#pragma unroll
                        for (int v = 1; v < NV; ++v) lu += Ls[v] * Fp[v][j];
                        // L_s F = u_n (L_s U) + p (L_s[n] + u_n L_s[E]): F = u_n U + p (0, 1, 0, u_n)
                        lf = un * lu + p * (Ls[1] + un * Ls[NV - 1]);
                    }
                    vp[j] = lf + al * lu;
                    vm[j] = lf - al * lu;
                }
            }

            int mp = 0, mm = 0;
            if constexpr (FROZEN) {
                mp = (int)((mword_in >> (8 * sf)) & 15u);
                mm = (int)((mword_in >> (8 * sf + 4)) & 15u);
                if (a.scheme == 1) { mp = teno5_row(mp); mm = teno5_row(mm); }
            } else {
                Smooth<T> sp = smooth5(vp[1], vp[2], vp[3], vp[4], vp[5]);
                Smooth<T> sm = smooth5(vm[6], vm[5], vm[4], vm[3], vm[2]);
                if constexpr (MODE == MODE_FACES) {
                    if (a.chi_out && face_ok) {
                        T cp[3], cm[3];
                        chi3(sp, a.eps4, a.C, a.q, cp);
                        chi3(sm, a.eps4, a.C, a.q, cm);
                        T *o = a.chi_out + face_index(f) * 24 + 6 * sf;
#pragma unroll
                        for (int j = 0; j < 3; ++j) {
                            o[j] = cp[j];
                            o[3 + j] = cm[j];
                        }
                    }
                }
                // (lanes of a packed wave that no piece needs count as smooth: their stencils straddle
                // two lines)
                // (both sides evaluated, without a branch between them)
                const bool easy = ((int)all_smooth(sp, a.smooth_k, a.keps4) & (int)all_smooth(sm, a.smooth_k, a.keps4)) | !needed;
                if (__all(easy)) {
                    // every flag of every face of the wave is 1: the full stencil on both sides
                    fword |= 63u << (6 * sf);
                    if (a.scheme == 0) {
                        mword |= 0u;
                    } else {
                        mword |= (uint32_t)(7 | (7 << 4)) << (8 * sf);
                        mp = mm = TENO5_ROW[7];
                    }
                } else {
                    // both sides of the lanes off the shortcut in one branch, the paper's exponent
                    // as a constant (any other q at run time)
                    unsigned dp = 7u, dm = 7u;
                    if (!easy) {
                        if (a.q == 6) {
                            dp = cutoff3<6>(sp, a.eps4, a.ct, a.C, 6);
                            dm = cutoff3<6>(sm, a.eps4, a.ct, a.C, 6);
                        } else {
                            dp = cutoff3<0>(sp, a.eps4, a.ct, a.C, a.q);
                            dm = cutoff3<0>(sm, a.eps4, a.ct, a.C, a.q);
                        }
                    }
                    unsigned bits = dp | (dm << 3);
                    fword |= bits << (6 * sf);
                    if (a.scheme == 0) {
                        unsigned left = shfl_up1(bits), right = shfl_dn1(bits);
                        // Delta+ = (d+_{i-1,0}, d+_{i,0}, d+_{i,1}, d+_{i,2}, d+_{i+1,2}) and the mirrored
                        // Delta- = (d-_{i+1,0}, d-_{i,0}, d-_{i,1}, d-_{i,2}, d-_{i-1,2}), bit-reversed
                        unsigned ip = (left & 1u) | (dp << 1) | (((right >> 2) & 1u) << 4);
                        unsigned im = ((right >> 3) & 1u) | (dm << 1) | (((left >> 5) & 1u) << 4);
                        mp = table3_rev(ip);
                        mm = table3_rev(im);
                        if (face_ok && (mp == 15 || mm == 15)) bad |= ERR_SELECTION;
                        mp = (mp == 15 || !needed) ? 0 : mp;
                        mm = (mm == 15 || !needed) ? 0 : mm;
                        mword |= (uint32_t)(mp | (mm << 4)) << (8 * sf);
                    } else {
                        int cp = (int)(((dp & 1u) << 2) | (dp & 2u) | ((dp >> 2) & 1u));
                        int cm = (int)(((dm & 1u) << 2) | (dm & 2u) | ((dm >> 2) & 1u));
                        if (face_ok && (cp == 0 || cm == 0)) bad |= ERR_SELECTION;
                        mword |= (uint32_t)(cp | (cm << 4)) << (8 * sf);
                        mp = teno5_row(cp);
                        mm = teno5_row(cm);
                    }
                }
            }
            T hp, hm;
            if (__all(mp == 0 && mm == 0)) {
                // Table 2 row 0 (the seventh-order linear scheme) as compile-time constants
                hp = recon_const<T, 0>(vp[0], vp[1], vp[2], vp[3], vp[4], vp[5], vp[6]);
                hm = recon_const<T, 0>(vm[7], vm[6], vm[5], vm[4], vm[3], vm[2], vm[1]);
            } else {
                const T *cp_ = coef + mp * 8;
                const T *cm_ = coef + mm * 8;
                hp = cp_[0] * vp[0];
                hm = cm_[0] * vm[7];
#pragma unroll
                for (int l = 1; l < 7; ++l) {
                    hp += cp_[l] * vp[l];
                    hm += cm_[l] * vm[7 - l];
                }
            }
            T w = hp + hm;
#pragma unroll
            for (int v = 0; v < NV; ++v) Fh[v] += Rs[v] * w;
        }

        // ---- epilogue ----
        // lane-dependent predicates recomputed from an opaque copy of the lane id (keeping them
        // live across the field loop costs registers the loop needs)
        int fe;                                 // this lane's face again
        int eline = line;                       // and its line
        {
            int kk = lane_id_now();
            asm volatile("" ::: "memory");      // orders the record reads before the epilogue
            bool pv = true;
            if constexpr (PACK) {
                const int i = pack_piece(pm, kk);
                eline = pack_line(pm, i, s, NSEG, a.nlines);
                pv = eline >= 0;
                kk -= i * pm.W;
            }
            fe = c0 - 1 + kk;
            face_ok = pv && kk >= 1 && kk <= 62 && fe <= a.len;
            cell_ok = pv && kk >= 1 && kk <= 61 && fe < a.len;
        }
        if constexpr (MODE == MODE_FACES) {
            if (face_ok) {
#pragma unroll
                for (int v = 0; v < NV; ++v) {
                    int gv = gvar<SYS, DIR>(v);
                    size_t o = DIR == 0 ? ((size_t)gv * a.ny + line) * (a.len + 1) + fe
                                        : ((size_t)gv * (a.len + 1) + fe) * a.nx + line;
                    a.Fout[o] = Fh[v];
                }
                if (a.flags_out) a.flags_out[face_index(fe)] = fword;
            }
        }
        if (a.masks_out && face_ok) a.masks_out[face_index(fe)] = mword;
        if constexpr (MODE != MODE_FACES) {
            if constexpr (HAS_EXT) wait_vmem();  // the background copies of the epilogue operands
            T Fr[NV];
#pragma unroll
            for (int v = 0; v < NV; ++v) Fr[v] = shfl_dn1_z(Fh[v]);   // (lane 63, never a cell: 0)
            // primitive speeds of the produced cell (stage mode); lanes without a cell contribute 0
            double sx = 0.0, sy = 0.0, sc = 0.0;
            if (cell_ok) {
                size_t off = DIR == 0 ? (size_t)eline * a.nx + fe : (size_t)fe * a.nx + eline;
                const T *e = ext + (size_t)s * 2 * NV * WAVE + k;
                T unew[NV];
                // every field's operands are read before any of the arithmetic, so that the reads
                // overlap instead of waiting field by field
                T dv[NV];
#pragma unroll
                for (int v = 0; v < NV; ++v) dv[v] = -(Fr[v] - Fh[v]) * a.inv_h;
                if (a.addend) {
                    T yv[NV];
#pragma unroll
                    for (int v = 0; v < NV; ++v)
                        yv[v] = HAS_EXT ? e[(NV + v) * WAVE] : a.addend[(size_t)gvar<SYS, DIR>(v) * ncell + off];
#pragma unroll
                    for (int v = 0; v < NV; ++v) dv[v] = dv[v] + yv[v];
                }
                if constexpr (STAGE_OUT) {
#pragma unroll
                    for (int v = 0; v < NV; ++v) rec[s * SEG_STRIDE + v * OUTW + k - 1] = dv[v];   // own record, no longer read
                } else if constexpr (MODE == MODE_RHS) {
#pragma unroll
                    for (int v = 0; v < NV; ++v) a.out[(size_t)gvar<SYS, DIR>(v) * ncell + off] = dv[v];
                } else {
                    // SSP-RK3 stage, Shu-Osher form: U' = c0 U^n + c1 (U^(k) + dt L) with (c0, c1) =
                    // (0, 1), (3/4, 1/4), (1/3, 2/3); at the first stage U^(k) is U^n
                    // (a step of dt = 0, at a run's end time, leaves the state exactly as it is)
                    const bool still = dtv == 0.0;
                    const T c0 = (a.stage == 0 || still) ? T(0) : a.stage == 1 ? T(0.75) : T(1.0 / 3.0);
                    const T c1 = (a.stage == 0 || still) ? T(1) : a.stage == 1 ? T(0.25) : T(2.0 / 3.0);
                    T ukv[NV], u0v[NV];
#pragma unroll
                    for (int v = 0; v < NV; ++v) ukv[v] = R0[FSTR * v + k + 4];   // staged record: conserved variable v first
                    // U^n: the staged stage input itself at the first stage, else its copy
#pragma unroll
                    for (int v = 0; v < NV; ++v)
                        u0v[v] = HAS_EXT ? (a.U0 == a.U ? ukv[v] : e[v * WAVE]) : a.U0[(size_t)gvar<SYS, DIR>(v) * ncell + off];
                    const T dt = (T)dtv;
#pragma unroll
                    for (int v = 0; v < NV; ++v) {
                        const T t = fma(dt, dv[v], ukv[v]);
                        const T un = fma(c0, u0v[v], c1 * t);
                        a.out[(size_t)gvar<SYS, DIR>(v) * ncell + off] = un;
                        unew[gvar<SYS, DIR>(v)] = un;
                    }
                }
                if constexpr (MODE == MODE_STAGE && FROZEN) {
                    // a replay takes its constants and dt from the recording: no maxima, only the
                    // produced state's check
                    if (!cell_physical<T, SYS>(unew, a.gm1)) bad |= ERR_NONPHYSICAL;
                } else if constexpr (MODE == MODE_STAGE) {
                    if (!cell_primitive_speeds<T, SYS>(unew, a.gamma, a.gm1, a.adv, sx, sy, sc)) {
                        bad |= ERR_NONPHYSICAL;       // reported; keep the maxima finite
                        sx = sy = sc = 0.0;
                    }
                }
            }
            if constexpr (MODE == MODE_STAGE && !FROZEN) {
                // this segment's maxima into the wave's LDS slots (the wave owns them: no race)
                constexpr int NU = SpeedWords<NV>::count();
                constexpr int WSTRIDE = WAVE + 1;          // per word, padded against bank conflicts
                constexpr int SWROOM = XREC ? 2 * NV * WAVE - 1 : SEG_STRIDE;
                if constexpr (sizeof(T) == 8 && NU * WSTRIDE <= SWROOM) {
                    // Through the segment's own record, which is no longer read: every lane stores its
                    // words, then lane 8u+j takes the maximum of values j, j+8, .., j+56 of word slot u
                    // and three row shifts bring the slot's maximum to lane 8u+7. Exact (a maximum of
                    // doubles), and far fewer instructions than a whole-wave reduction per word.
                    // (x-stage: the segment's epilogue-operand slot instead, past its element 0, which
                    // the previous segment's copy may still be writing; the tile record is shared)
                    T *sw = XREC ? ext + (size_t)s * 2 * NV * WAVE + 1 : rec + s * SEG_STRIDE;
                    asm volatile("" ::: "memory");     // after the epilogue's reads
                    {
                        int u = 0;
#pragma unroll
                        for (int q = 0; q < 9; ++q) {
                            if (!SpeedWords<NV>::use(q)) continue;
                            // (lanes without a cell have zero speeds, so all their words are 0)
                            sw[u * WSTRIDE + k] = speed_word<SYS>(q, sx, sy, sc, (double)a.inv_dx, (double)a.inv_dy,
                                                                  a.alpha_mode);
                            ++u;
                        }
                    }
                    wave_lds_fence();
                    const int u = k >> 3, j = k & 7;
                    double m = 0.0;
                    if (u < NU) {
#pragma unroll
                        for (int i = 0; i < 8; ++i) m = fmax(m, (double)sw[u * WSTRIDE + j + 8 * i]);
                    }
                    m = fmax(m, dpp_shift_z<0x111>(m));  // row_shr:1 (lanes without a source: 0)
                    m = fmax(m, dpp_shift_z<0x112>(m));  // row_shr:2
                    m = fmax(m, dpp_shift_z<0x114>(m));  // row_shr:4
                    if (j == 7 && u < NU) {
                        const int q = (int)((SpeedWords<NV>::pack() >> (4 * u)) & 15u);   // word of slot u
                        // each wave puts its maxima straight into the block's spread copy (a.part): no
                        // LDS slots and no barrier at the block's end (a maximum of non-negative doubles
                        // is the maximum of their bit patterns)
                        const unsigned long long mb = (unsigned long long)__double_as_longlong(m);
                        atomicMax(a.part + q, mb);
                        if (NV == 4 && (q == 1 || q == 5)) atomicMax(a.part + q + 1, mb);
                    }
                } else {
                    // the words reduced side by side so that their cross-lane steps interleave
                    unsigned hi[9], lo[9], mh[9], ml[9];
#pragma unroll
                    for (int q = 0; q < 9; ++q) {
                        if (!SpeedWords<NV>::use(q)) continue;
                        const double val = speed_word<SYS>(q, sx, sy, sc, (double)a.inv_dx, (double)a.inv_dy,
                                                           a.alpha_mode);
                        const unsigned long long b = (unsigned long long)__double_as_longlong(val);
                        hi[q] = (unsigned)(b >> 32);
                        lo[q] = (unsigned)b;
                    }
#pragma unroll
                    for (int q = 0; q < 9; ++q)
                        if (SpeedWords<NV>::use(q)) mh[q] = wave_max_u32(hi[q]);
#pragma unroll
                    for (int q = 0; q < 9; ++q)
                        if (SpeedWords<NV>::use(q)) ml[q] = wave_max_u32(hi[q] == mh[q] ? lo[q] : 0u);
#pragma unroll
                    for (int q = 0; q < 9; ++q) {
                        if (!SpeedWords<NV>::use(q)) continue;
                        const double m = __longlong_as_double((long long)(((unsigned long long)mh[q] << 32) | ml[q]));
                        if (k == 0) {
                            const unsigned long long mb = (unsigned long long)__double_as_longlong(m);
                            atomicMax(a.part + q, mb);
                            if (NV == 4 && (q == 1 || q == 5)) atomicMax(a.part + q + 1, mb);
                        }
                    }
                }
            }
        }
    }
    if constexpr (STAGE_OUT && PACK) {
        __syncthreads();
        for (int idx = tid; idx < NV * WAVE * NSEG; idx += BLOCK) {
            const int sg = idx % NSEG, kk = (idx / NSEG) % WAVE, v = idx / (NSEG * WAVE);
            const int i = pack_piece(pm, kk + 1), kl = kk + 1 - i * pm.W;   // lane kk + 1
            const int line = pack_line(pm, i, sg, NSEG, a.nlines);
            if (line < 0 || kl < 1 || kl > pm.nt) continue;
            a.out[(size_t)gvar<SYS, DIR>(v) * ncell + (size_t)(pm.c0 + kl - 1) * a.nx + line] =
                rec[sg * SEG_STRIDE + v * WAVE + kk];
        }
    } else if constexpr (STAGE_OUT) {
        // thread t stores column t mod NSEG of the tile, entries (v, c) = t / NSEG, t / NSEG + BLOCK /
        // NSEG, .. of the flattened [NV][SEG_CELLS] results, the pair advanced without divisions
        static_assert(BLOCK % NSEG == 0, "a fixed column per thread");
        constexpr int STEP = BLOCK / NSEG, DV = STEP / SEG_CELLS, DC = STEP % SEG_CELLS;
        __syncthreads();
        const int sg = tid % NSEG;
        int line, c0;
        seg_of(sg, line, c0);
        if (line >= 0) {
            const T *src = rec + sg * SEG_STRIDE;
            int v = 0, c = tid / NSEG;              // (tid / NSEG < SEG_CELLS for NSEG >= 8; else wrap)
            if (c >= SEG_CELLS) {
                c -= SEG_CELLS;
                ++v;
            }
            for (int it = tid / NSEG; it < NV * SEG_CELLS; it += STEP) {
                if (c0 + c < a.len)
                    a.out[(size_t)gvar<SYS, DIR>(v) * ncell + (size_t)(c0 + c) * a.nx + line] = src[v * SEG_CELLS + c];
                v += DV;
                c += DC;
                if (c >= SEG_CELLS) {
                    c -= SEG_CELLS;
                    ++v;
                }
            }
        }
    }
    if (bad) atomicOr(a.err, bad);
}

// Workgroups of a launch are handed to the 8 XCDs round-robin (block b to XCD b mod 8), and each
// XCD has its own L2. Renumber so that every XCD walks a contiguous range of tiles in order:
// neighbouring tiles, which share cache lines and halo cells, then meet in the same L2. A bijection
// of [0, n) for any n.
constexpr int NXCD = 8;
__device__ __forceinline__ int xcd_tile(int b, int n)
{
    const int q = n / NXCD, r = n % NXCD, x = b % NXCD;
    return x * q + min(x, r) + b / NXCD;
}

// LDS of the epilogue operands (x-sweeps that add a y-part or apply an RK stage): one 64-element
// slot per segment and field, plus one element of padding for the last slot's copy overrun.
template <typename T, int SYS, int DIR, int NSEG, int MODE> constexpr int ext_size()
{
    return (DIR == 0 && MODE != MODE_FACES) ? NSEG * 2 * Sys<SYS>::NV * WAVE + 2 : 1;
}

// Minimum waves per SIMD of a sweep kernel's register budget.
template <int SYS, int DIR, bool FROZEN, int MODE> constexpr int sweep_min_waves()
{
    return (SYS == EULER1D && FROZEN) ? 3 : (DIR == 0 ? TENO_MIN_WAVES_X : TENO_MIN_WAVES_Y);
}

// x-sweep stage kernels read the coefficient rows (needed only where a face cuts a stencil) from the
// global table instead of copying it into LDS first (with the maxima posted per wave, 2.5 % faster on
// the 4096^2 benchmark state).
template <int DIR, int MODE> constexpr bool coef_global() { return DIR == 0 && MODE == MODE_STAGE; }

// One tile per block (measured faster on MI355X than persistent blocks looping over tiles: freshly
// scheduled blocks overlap their staging with the compute of resident ones).
// REC = false: no selection masks or flags are written (the pointers are known null at compile
// time, so the mask words are not assembled at all).
template <typename T, int SYS, int DIR, bool FROZEN, int MODE, bool REC = true>
__global__ void __launch_bounds__(BLOCK, (sweep_min_waves<SYS, DIR, FROZEN, MODE>()))
    sweep_kernel(SweepArgs<T> a)
{
    if constexpr (!REC) {
        a.masks_out = nullptr;
        a.flags_out = nullptr;
    }
    constexpr int NSEG = DIR == 0 ? NSEG_X : NSEG_Y;
    constexpr bool CG = coef_global<DIR, MODE>();
    __shared__ T rec[rec_size<SYS, DIR, NSEG, false>()];
    __shared__ __align__(16) T ext[ext_size<T, SYS, DIR, NSEG, MODE>()];
    __shared__ T coef_lds[CG ? 1 : NCOEF_ROWS * 8];
    if constexpr (!CG) fill_coef(coef_lds);                 // (ordered by the tile's first barrier)
    const T *coef = CG ? coef_table<T>() : coef_lds;
    if constexpr (MODE == MODE_STAGE) a.part += (size_t)(blockIdx.x % NCOPY) * NWORD;   // the block's copy
    sweep_tile<T, SYS, DIR, FROZEN, NSEG, MODE>(a, xcd_tile(blockIdx.x, gridDim.x), rec, ext, coef);
}

// ------------------------------------------------------------------------------------------------
// Wave-speed maxima of a state (the first stage of a run and the stand-alone operator).
// ------------------------------------------------------------------------------------------------
template <typename T, int SYS>
__global__ void __launch_bounds__(BLOCK) wavespeed_kernel(const T *U, size_t ncell, T gamma, T adv, T inv_dx,
                                                          T inv_dy, int alpha_mode, unsigned long long *part,
                                                          unsigned *err)
{
    __shared__ double red[BLOCK / WAVE * 9];
    constexpr int NV = Sys<SYS>::NV;
    double wmax[9];
    for (int k = 0; k < 9; ++k) wmax[k] = 0.0;
    unsigned bad = 0;
    for (size_t i = (size_t)blockIdx.x * BLOCK + threadIdx.x; i < ncell; i += (size_t)gridDim.x * BLOCK) {
        T u[4];
#pragma unroll
        for (int v = 0; v < NV; ++v) u[v] = U[(size_t)v * ncell + i];
        double w[9];
        if (!cell_speeds<T, SYS>(u, gamma, adv, inv_dx, inv_dy, alpha_mode, w)) bad |= ERR_NONPHYSICAL;
#pragma unroll
        for (int k = 0; k < 9; ++k) wmax[k] = fmax(wmax[k], w[k]);
    }
    block_max_atomic(wmax, part + (size_t)(blockIdx.x % NCOPY) * NWORD, red);
    if (bad) atomicOr(err, bad);
}

// Reduce the spread maxima of one ring slot into alpha/den (and dt at the first stage of a step),
// then clear the slot for its next accumulation. One block of 64 threads.
//   frozen (nullable): replay the 8 constants (+ dt when stage == 0) from a recorded buffer.
//   record (nullable): write the 8 constants (+ dt when stage == 0) to a recording buffer.
// Recording layout per step: [stage0 alpha 8][stage1 alpha 8][stage2 alpha 8][dt].
static __global__ void prep_kernel(Ctrl *ctrl, int ring, int stage, double dt_fixed, double cfl, const double *frozen,
                            double *record)
{
    __shared__ double vals[NWORD];
    const int t = threadIdx.x;
    if (t < 9) {
        unsigned long long m = 0;
        for (int c = 0; c < NCOPY; ++c) {
            unsigned long long v = ctrl->part[ring][c][t];
            m = v > m ? v : m;
        }
        vals[t] = __longlong_as_double((long long)m);
    }
    __syncthreads();
    for (int q = t; q < NCOPY * NWORD; q += blockDim.x) (&ctrl->part[ring][0][0])[q] = 0ull;
    if (t < 8) {
        double al = frozen ? frozen[8 * stage + t] : vals[t];
        ctrl->alpha[t] = al;
        if (record) record[8 * stage + t] = al;
    }
    if (t == 8) {
        ctrl->den = vals[8];
        // a failure raised since the last preparation belongs to the step in progress (before the
        // first step: to the first step)
        if (ctrl->err && !ctrl->err_at) ctrl->err_at = stage == 0 ? (ctrl->steps ? ctrl->steps : 1u) : ctrl->steps;
        if (stage == 0) ctrl->steps += 1;
        if (stage == 0) {
            double dt = dt_fixed > 0.0 ? dt_fixed : cfl / vals[8];
            double tn = ctrl->t + dt;
            bool at_end = false;
            if (frozen) {
                dt = frozen[24];
                tn = ctrl->t;               // replays of recorded steps leave the time alone
                at_end = dt == 0.0;         // (a recorded step at an end time)
            } else if (ctrl->end_on) {
                // the step that would pass t_end lands on it exactly; later steps have dt = 0
                const double rest = ctrl->t_end - ctrl->t;
                if (!(dt < rest)) {
                    dt = rest > 0.0 ? rest : 0.0;
                    tn = ctrl->t_end;
                    at_end = true;
                }
            }
            if (!(dt > 0.0 || (at_end && dt == 0.0)) || !isfinite(dt)) {
                atomicOr(&ctrl->err, ERR_NONFINITE);
                if (!ctrl->err_at) ctrl->err_at = ctrl->steps;
            }
            ctrl->dt = dt;
            ctrl->t = tn;
            if (record) record[24] = dt;
        }
    }
}

static __global__ void clear_ring_kernel(Ctrl *ctrl, int ring)
{
    for (int q = threadIdx.x; q < NCOPY * NWORD; q += blockDim.x) (&ctrl->part[ring][0][0])[q] = 0ull;
}

// Simulated time and end time of the runs that follow.
static __global__ void set_time_kernel(Ctrl *ctrl, double t0, double t_end, unsigned on)
{
    if (threadIdx.x == 0) {
        ctrl->t = t0;
        ctrl->t_end = t_end;
        ctrl->end_on = on;
    }
}

// Start counting steps and attributing failures to them from here (the error word is kept).
static __global__ void reset_counters_kernel(Ctrl *ctrl)
{
    if (threadIdx.x == 0) {
        ctrl->steps = 0;
        ctrl->err_at = 0;
    }
}

// Copy the eight constants of the current stage out (parity/debug form).
static __global__ void copy_alpha_kernel(const Ctrl *ctrl, double *dst)
{
    if (threadIdx.x < 8) dst[threadIdx.x] = ctrl->alpha[threadIdx.x];
}

}  // namespace teno
