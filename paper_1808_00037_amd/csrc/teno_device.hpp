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
//   * The block stages its segments' cells (conserved variables plus per-cell velocity, pressure,
//     sqrt(rho) and enthalpy, computed once per cell) in LDS; every lane then reads its eight
//     stencil cells from LDS. x-sweeps stage 4 consecutive segments of a row (coalesced);
//     y-sweeps stage 8 adjacent columns with the same rows so that a global load of one row reads
//     8 consecutive doubles; LDS holds each column contiguously, so lanes running along y read
//     consecutive LDS words.
//   * The neighbour flags of eq:vec come from lanes k-1 and k+1 through cross-lane shuffles; no
//     flag array is stored (the paper's whole-domain flag pass lives in registers).
//   * Characteristic fields are streamed one at a time: project eight points, cut-off flags on
//     both split sides, exchange, select, reconstruct, accumulate R[:,s] * (v+ + v-).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace teno {

enum : int { ADV1D = 0, EULER1D = 1, EULER2D = 2, BURGERS1D = 3 };
enum : int { MODE_RHS = 0, MODE_STAGE = 1, MODE_FACES = 2 };
enum : unsigned { ERR_NONFINITE = 1u, ERR_NONPHYSICAL = 2u, ERR_SELECTION = 4u };

constexpr int WAVE = 64;
constexpr int BLOCK = 256;
constexpr int SEG_CELLS = 61;   // cells finished per segment
constexpr int SEG_HALO = 5;     // first staged cell is c0 - 5
constexpr int SEG_LOAD = 72;    // staged cells per segment (faces c0-1..c0+62 read c0-5..c0+65)
constexpr int NSEG_X = 4;       // segments per block, x-sweeps (one per wave)
constexpr int NSEG_Y = 8;       // columns per block, y-sweeps (two per wave)
constexpr int NCOPY = 64;       // spread copies of the wave-speed maxima (atomic contention)
constexpr int NWORD = 16;       // words per copy: 0-3 x fields, 4-7 y fields, 8 CFL denominator

// Device control block of one context (zeroed at creation).
struct Ctrl {
    unsigned long long part[4][NCOPY][NWORD];  // [ring][copy][word] maxima of non-negative doubles
    double alpha[8];                           // Lax-Friedrichs constants of the current stage
    double den;                                // CFL denominator of the current stage's state
    double dt;                                 // dt of the current step
    unsigned err;
    unsigned pad_;
};

// ------------------------------------------------------------------------------------------------
// System traits: number of conserved variables, staged record layout.
// Euler records hold (rho, m_n, [m_t], E, u_n, [u_t], p, sqrt(rho), H), with n the sweep direction;
// the conserved variables come first, so record index v is local conserved variable v.
// ------------------------------------------------------------------------------------------------
template <int SYS> struct Sys;
template <> struct Sys<ADV1D> { static constexpr int NV = 1, NREC = 1; };
template <> struct Sys<BURGERS1D> { static constexpr int NV = 1, NREC = 1; };
template <> struct Sys<EULER1D> {
    static constexpr int NV = 3, NREC = 7, E = 2, UN = 3, UT = -1, P = 4, S = 5, H = 6;
};
template <> struct Sys<EULER2D> {
    static constexpr int NV = 4, NREC = 9, E = 3, UN = 4, UT = 5, P = 6, S = 7, H = 8;
};

// Global variable index of local (normal/tangential) component v in direction DIR.
template <int SYS, int DIR> __device__ __forceinline__ constexpr int gvar(int v)
{
    return (SYS == EULER2D && DIR == 1 && (v == 1 || v == 2)) ? 3 - v : v;
}

__device__ __forceinline__ int bc_index(int i, int n, int bc)
{
    if (bc == 0) {
        i %= n;
        return i < 0 ? i + n : i;
    }
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

// ------------------------------------------------------------------------------------------------
// Five-point cut-off of one split side (eq:smooth_expl, eq:tau5, eq:TENO1 with C = 1, q = 6,
// eq:norm, eq:seclect). Returns bit k = delta_k. (a..e) = values at i-2..i+2 in upwind order.
// delta_k = 0 iff gamma_k / sum(gamma) < C_T, evaluated as gamma_k < C_T * sum(gamma) with
// gamma_k = (1 + tau (D_j D_l) / (D0 D1 D2))^6, D_k = beta_k + eps: one division per side instead
// of six; equal to the definition up to rounding (so flags can differ only when chi_k lies within
// rounding of C_T).
// ------------------------------------------------------------------------------------------------
__device__ __forceinline__ unsigned cutoff3(double a, double b, double c, double d, double e,
                                            double eps, double ct)
{
    double t0 = a - 4.0 * b + 3.0 * c, t1 = a - 2.0 * b + c;
    double t2 = b - d, t3 = b - 2.0 * c + d;
    double t4 = 3.0 * c - 4.0 * d + e, t5 = c - 2.0 * d + e;
    double b0 = 0.25 * t0 * t0 + (13.0 / 12.0) * t1 * t1;
    double b1 = 0.25 * t2 * t2 + (13.0 / 12.0) * t3 * t3;
    double b2 = 0.25 * t4 * t4 + (13.0 / 12.0) * t5 * t5;
    double tau = fabs(b0 - b2);
    double D0 = b0 + eps, D1 = b1 + eps, D2 = b2 + eps;
    double D01 = D0 * D1;
    double inv = 1.0 / (D01 * D2);
    double tinv = tau * inv;
    double r0 = 1.0 + tinv * (D1 * D2);
    double r1 = 1.0 + tinv * (D0 * D2);
    double r2 = 1.0 + tinv * D01;
    double g0 = r0 * r0 * r0, g1 = r1 * r1 * r1, g2 = r2 * r2 * r2;
    g0 *= g0;
    g1 *= g1;
    g2 *= g2;
    double thr = ct * ((g0 + g1) + g2);
    return (g0 < thr ? 0u : 1u) | (g1 < thr ? 0u : 2u) | (g2 < thr ? 0u : 4u);
}

// Single precision: gamma_k / gamma_max keeps every term in [0, 1] (no overflow of r^6).
__device__ __forceinline__ unsigned cutoff3(float a, float b, float c, float d, float e, float eps, float ct)
{
    float t0 = a - 4.0f * b + 3.0f * c, t1 = a - 2.0f * b + c;
    float t2 = b - d, t3 = b - 2.0f * c + d;
    float t4 = 3.0f * c - 4.0f * d + e, t5 = c - 2.0f * d + e;
    float b0 = 0.25f * t0 * t0 + (13.0f / 12.0f) * t1 * t1;
    float b1 = 0.25f * t2 * t2 + (13.0f / 12.0f) * t3 * t3;
    float b2 = 0.25f * t4 * t4 + (13.0f / 12.0f) * t5 * t5;
    float tau = fabsf(b0 - b2);
    float r0 = 1.0f + tau / (b0 + eps), r1 = 1.0f + tau / (b1 + eps), r2 = 1.0f + tau / (b2 + eps);
    float rm = fmaxf(r0, fmaxf(r1, r2));
    float q0 = r0 / rm, q1 = r1 / rm, q2 = r2 / rm;
    float g0 = q0 * q0 * q0, g1 = q1 * q1 * q1, g2 = q2 * q2 * q2;
    g0 *= g0;
    g1 *= g1;
    g2 *= g2;
    float thr = ct * ((g0 + g1) + g2);
    return (g0 < thr ? 0u : 1u) | (g1 < thr ? 0u : 2u) | (g2 < thr ? 0u : 4u);
}

template <typename T> __device__ __forceinline__ T shfl_up1(T v) { return __shfl_up(v, 1, WAVE); }
template <typename T> __device__ __forceinline__ T shfl_dn1(T v) { return __shfl_down(v, 1, WAVE); }

// ------------------------------------------------------------------------------------------------
// Sweep kernel arguments.
// ------------------------------------------------------------------------------------------------
template <typename T> struct SweepArgs {
    const T *U;                 // stage input state [nv][ny][nx]
    const T *U0;                // MODE_STAGE: RK base state
    const T *addend;            // nullable: dU of the other direction, added per cell
    T *out;                     // MODE_RHS: dU/dt; MODE_STAGE: next stage state
    T *Fout;                    // MODE_FACES: face fluxes
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
    int bc;                     // boundary condition along the sweep
    int bc_other;               // (unused by the sweep itself)
    int mode, stage, scheme, alpha_mode;
    T inv_h, eps, ct, gamma, adv;
    T inv_dx, inv_dy;           // for the CFL denominator of the produced state
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
        T ir = T(1) / rho;
        T vx = mx * ir, vy = my * ir;
        T p = (gamma - T(1)) * (E - T(0.5) * rho * (vx * vx + vy * vy));
        bool ok = rho > T(0) && p > T(0) && isfinite(E);
        T cs = sqrt(gamma * p * ir);
        double c = (double)cs, ux = (double)vx, uy = (double)vy;
        if (alpha_mode) {
            w[0] = w[1] = w[2] = w[3] = fabs(ux) + c;
            if (NV == 4) w[4] = w[5] = w[6] = w[7] = fabs(uy) + c;
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

__device__ __forceinline__ double wave_max(double v)
{
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v = fmax(v, __shfl_xor(v, o, WAVE));
    return v;
}

// Block-wide maxima of nine per-lane values -> one atomicMax per word into a spread copy.
__device__ __forceinline__ void block_max_atomic(double w[9], unsigned long long *part, double *lds9)
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
        unsigned long long *dst = part + (size_t)(blockIdx.x % NCOPY) * NWORD + threadIdx.x;
        atomicMax(dst, (unsigned long long)__double_as_longlong(m));
    }
}

// ------------------------------------------------------------------------------------------------
// The sweep kernel.
//   DIR: 0 = x (lines are rows), 1 = y (lines are columns).
//   FROZEN: the selection is read from masks_in instead of being measured.
// ------------------------------------------------------------------------------------------------
template <typename T, int SYS, int DIR, bool FROZEN>
__global__ void __launch_bounds__(BLOCK) sweep_kernel(SweepArgs<T> a)
{
    constexpr int NV = Sys<SYS>::NV;
    constexpr int NREC = Sys<SYS>::NREC;
    constexpr int NSEG = DIR == 0 ? NSEG_X : NSEG_Y;
    constexpr int SEG_STRIDE = NREC * SEG_LOAD + 1;   // odd stride: y staging stores spread banks
    constexpr bool EULER = SYS == EULER1D || SYS == EULER2D;

    __shared__ T rec[NSEG * SEG_STRIDE];
    __shared__ T coef[NCOEF_ROWS * 8];
    __shared__ double red[BLOCK / WAVE * 9];

    const int tid = threadIdx.x, lane = tid & (WAVE - 1), wid = tid / WAVE;
    const size_t ncell = (size_t)a.nx * a.ny;

    for (int q = tid; q < NCOEF_ROWS * 8; q += BLOCK) {
        int r = q / 8, l = q % 8;
        coef[q] = l < 7 ? T(COEF[r][l].n) / T(COEF[r][l].d) : T(0);
    }

    // segment s of this block -> (line, c0); line < 0 marks an empty slot
    auto seg_of = [&](int s, int &line, int &c0) {
        if (DIR == 0) {
            int id = blockIdx.x * NSEG + s;
            line = id / a.nseg;
            c0 = (id % a.nseg) * SEG_CELLS;
            if (line >= a.nlines) line = -1;
        } else {
            int ntile = (a.nlines + NSEG - 1) / NSEG;
            int pos = blockIdx.x / ntile;
            line = (blockIdx.x % ntile) * NSEG + s;
            c0 = pos * SEG_CELLS;
            if (line >= a.nlines) line = -1;
        }
    };

    // ---- stage cells into LDS (coalesced along x in both sweeps) ----
    unsigned bad = 0;
    for (int idx = tid; idx < NSEG * SEG_LOAD; idx += BLOCK) {
        int s, q;
        if (DIR == 0) { s = idx / SEG_LOAD; q = idx % SEG_LOAD; }
        else          { s = idx % NSEG;     q = idx / NSEG; }
        int line, c0;
        seg_of(s, line, c0);
        if (line < 0) continue;
        int g = bc_index(c0 - SEG_HALO + q, a.len, a.bc);
        size_t off = DIR == 0 ? (size_t)line * a.nx + g : (size_t)g * a.nx + line;
        T *r = rec + s * SEG_STRIDE + q;
        if constexpr (!EULER) {
            r[0] = a.U[off];
        } else {
            using S = Sys<SYS>;
            T rho = a.U[off];
            T mn = a.U[(size_t)gvar<SYS, DIR>(1) * ncell + off];
            T mt = NV == 4 ? a.U[(size_t)gvar<SYS, DIR>(2) * ncell + off] : T(0);
            T E = a.U[(size_t)(NV - 1) * ncell + off];
            T ir = T(1) / rho;
            T un = mn * ir, ut = mt * ir;
            T p = (a.gamma - T(1)) * (E - T(0.5) * rho * (un * un + ut * ut));
            if (!(rho > T(0) && p > T(0))) bad |= (isfinite(rho) && isfinite(p)) ? ERR_NONPHYSICAL : ERR_NONFINITE;
            r[0] = rho;
            r[SEG_LOAD * 1] = mn;
            if constexpr (NV == 4) r[SEG_LOAD * 2] = mt;
            r[SEG_LOAD * S::E] = E;
            r[SEG_LOAD * S::UN] = un;
            if constexpr (NV == 4) r[SEG_LOAD * S::UT] = ut;
            r[SEG_LOAD * S::P] = p;
            r[SEG_LOAD * S::S] = sqrt(rho);
            r[SEG_LOAD * S::H] = (E + p) * ir;
        }
    }
    __syncthreads();

    const double *alpha = a.alpha + 4 * DIR;
    double dtv = a.mode == MODE_STAGE ? *a.dt : 0.0;
    double wmax[9];
    for (int k = 0; k < 9; ++k) wmax[k] = 0.0;

    for (int s = wid; s < NSEG; s += BLOCK / WAVE) {
        int line, c0;
        seg_of(s, line, c0);
        if (line < 0) continue;                 // wave-uniform
        const T *R0 = rec + s * SEG_STRIDE;
        const int k = lane;
        const int f = c0 - 1 + k;               // this lane's face
        const bool face_ok = k >= 1 && k <= 62 && f <= a.len;
        const bool cell_ok = k >= 1 && k <= 61 && f < a.len;
        size_t fidx = 0;                        // face index in this direction's face arrays
        if (face_ok) fidx = DIR == 0 ? (size_t)line * (a.len + 1) + f : (size_t)f * a.nx + line;
        uint32_t mword_in = 0;
        if constexpr (FROZEN) mword_in = face_ok ? a.masks_in[fidx] : 0u;

        T Fh[NV];
#pragma unroll
        for (int v = 0; v < NV; ++v) Fh[v] = T(0);
        uint32_t mword = 0, fword = 0;

        // characteristic basis at the face (Roe average of cells i = q k+3 and i+1 = q k+4)
        T Lm[NV][NV], Rm[NV][NV];
        if constexpr (!EULER) {
            Lm[0][0] = T(1);
            Rm[0][0] = T(1);
        } else {
            using S = Sys<SYS>;
            const T gm1 = a.gamma - T(1);
            T sL = R0[SEG_LOAD * S::S + k + 3], sR = R0[SEG_LOAD * S::S + k + 4];
            T isum = T(1) / (sL + sR);
            T un = (sL * R0[SEG_LOAD * S::UN + k + 3] + sR * R0[SEG_LOAD * S::UN + k + 4]) * isum;
            T ut = T(0);
            if constexpr (NV == 4) ut = (sL * R0[SEG_LOAD * S::UT + k + 3] + sR * R0[SEG_LOAD * S::UT + k + 4]) * isum;
            T H = (sL * R0[SEG_LOAD * S::H + k + 3] + sR * R0[SEG_LOAD * S::H + k + 4]) * isum;
            T q2 = un * un + ut * ut;
            T c2 = gm1 * (H - T(0.5) * q2);
            if (face_ok && !(c2 > T(0))) bad |= isfinite(c2) ? ERR_NONPHYSICAL : ERR_NONFINITE;
            T cs = sqrt(c2);
            T ic = T(1) / cs;
            T b1 = gm1 * ic * ic;
            T b2 = T(0.5) * b1 * q2;
            T hb1 = T(0.5) * b1;
            if constexpr (NV == 3) {
                Lm[0][0] = T(0.5) * (b2 + un * ic); Lm[0][1] = -T(0.5) * (b1 * un + ic); Lm[0][2] = hb1;
                Lm[1][0] = T(1) - b2;               Lm[1][1] = b1 * un;                  Lm[1][2] = -b1;
                Lm[2][0] = T(0.5) * (b2 - un * ic); Lm[2][1] = -T(0.5) * (b1 * un - ic); Lm[2][2] = hb1;
                Rm[0][0] = T(1);          Rm[0][1] = T(1);            Rm[0][2] = T(1);
                Rm[1][0] = un - cs;       Rm[1][1] = un;              Rm[1][2] = un + cs;
                Rm[2][0] = H - un * cs;   Rm[2][1] = T(0.5) * q2;     Rm[2][2] = H + un * cs;
            } else {
                Lm[0][0] = T(0.5) * (b2 + un * ic); Lm[0][1] = -T(0.5) * (b1 * un + ic);
                Lm[0][2] = -hb1 * ut;               Lm[0][3] = hb1;
                Lm[1][0] = T(1) - b2; Lm[1][1] = b1 * un; Lm[1][2] = b1 * ut; Lm[1][3] = -b1;
                Lm[2][0] = -ut; Lm[2][1] = T(0); Lm[2][2] = T(1); Lm[2][3] = T(0);
                Lm[3][0] = T(0.5) * (b2 - un * ic); Lm[3][1] = -T(0.5) * (b1 * un - ic);
                Lm[3][2] = -hb1 * ut;               Lm[3][3] = hb1;
                Rm[0][0] = T(1);        Rm[0][1] = T(1);        Rm[0][2] = T(0); Rm[0][3] = T(1);
                Rm[1][0] = un - cs;     Rm[1][1] = un;          Rm[1][2] = T(0); Rm[1][3] = un + cs;
                Rm[2][0] = ut;          Rm[2][1] = ut;          Rm[2][2] = T(1); Rm[2][3] = ut;
                Rm[3][0] = H - un * cs; Rm[3][1] = T(0.5) * q2; Rm[3][2] = ut;   Rm[3][3] = H + un * cs;
            }
        }

#pragma unroll
        for (int sf = 0; sf < NV; ++sf) {
            const T al = (T)alpha[sf];
            T vp[8], vm[8];
#pragma unroll
            for (int j = 0; j < 8; ++j) {
                const int q = k + j;
                T lu, lf;
                if constexpr (!EULER) {
                    T u = R0[q];
                    lu = u;
                    lf = SYS == ADV1D ? a.adv * u : T(0.5) * u * u;
                } else {
                    using S = Sys<SYS>;
                    T un = R0[SEG_LOAD * S::UN + q], p = R0[SEG_LOAD * S::P + q];
                    lu = Lm[sf][0] * R0[q];
#pragma unroll
                    for (int v = 1; v < NV; ++v) lu += Lm[sf][v] * R0[SEG_LOAD * v + q];
                    // L_s F = u_n (L_s U) + p (L_s[n] + u_n L_s[E]): F = u_n U + p (0, 1, 0, u_n)
                    lf = un * lu + p * (Lm[sf][1] + un * Lm[sf][NV - 1]);
                }
                vp[j] = T(0.5) * (lf + al * lu);
                vm[j] = T(0.5) * (lf - al * lu);
            }

            int mp, mm;
            if constexpr (FROZEN) {
                mp = (int)((mword_in >> (8 * sf)) & 15u);
                mm = (int)((mword_in >> (8 * sf + 4)) & 15u);
                if (a.scheme == 1) { mp = TENO5_ROW[mp & 7]; mm = TENO5_ROW[mm & 7]; }
            } else {
                unsigned dp = cutoff3(vp[1], vp[2], vp[3], vp[4], vp[5], a.eps, a.ct);
                unsigned dm = cutoff3(vm[6], vm[5], vm[4], vm[3], vm[2], a.eps, a.ct);
                unsigned bits = dp | (dm << 3);
                fword |= bits << (6 * sf);
                if (a.scheme == 0) {
                    unsigned left = shfl_up1(bits), right = shfl_dn1(bits);
                    // Delta+ = (d+_{i-1,0}, d+_{i,0}, d+_{i,1}, d+_{i,2}, d+_{i+1,2})
                    unsigned ip = ((left & 1u) << 4) | ((dp & 1u) << 3) | ((dp & 2u) << 1) | ((dp & 4u) >> 1)
                                | ((right >> 2) & 1u);
                    // Delta- (mirror) = (d-_{i+1,0}, d-_{i,0}, d-_{i,1}, d-_{i,2}, d-_{i-1,2})
                    unsigned im = (((right >> 3) & 1u) << 4) | ((dm & 1u) << 3) | ((dm & 2u) << 1)
                                | ((dm & 4u) >> 1) | ((left >> 5) & 1u);
                    mp = table3(ip);
                    mm = table3(im);
                    if (face_ok && (mp == 15 || mm == 15)) bad |= ERR_SELECTION;
                    mp = mp == 15 ? 0 : mp;
                    mm = mm == 15 ? 0 : mm;
                    mword |= (uint32_t)(mp | (mm << 4)) << (8 * sf);
                } else {
                    int cp = (int)(((dp & 1u) << 2) | (dp & 2u) | ((dp >> 2) & 1u));
                    int cm = (int)(((dm & 1u) << 2) | (dm & 2u) | ((dm >> 2) & 1u));
                    if (face_ok && (cp == 0 || cm == 0)) bad |= ERR_SELECTION;
                    mword |= (uint32_t)(cp | (cm << 4)) << (8 * sf);
                    mp = TENO5_ROW[cp];
                    mm = TENO5_ROW[cm];
                }
            }
            const T *cp_ = coef + mp * 8;
            const T *cm_ = coef + mm * 8;
            T hp = cp_[0] * vp[0];
            T hm = cm_[0] * vm[7];
#pragma unroll
            for (int l = 1; l < 7; ++l) {
                hp += cp_[l] * vp[l];
                hm += cm_[l] * vm[7 - l];
            }
            T w = hp + hm;
#pragma unroll
            for (int v = 0; v < NV; ++v) Fh[v] += Rm[v][sf] * w;
        }

        // ---- epilogue ----
        if (a.mode == MODE_FACES) {
            if (face_ok) {
#pragma unroll
                for (int v = 0; v < NV; ++v) {
                    int gv = gvar<SYS, DIR>(v);
                    size_t o = DIR == 0 ? ((size_t)gv * a.ny + line) * (a.len + 1) + f
                                        : ((size_t)gv * (a.len + 1) + f) * a.nx + line;
                    a.Fout[o] = Fh[v];
                }
                if (a.flags_out) a.flags_out[fidx] = fword;
            }
        }
        if (a.masks_out && face_ok) a.masks_out[fidx] = mword;
        if (a.mode != MODE_FACES) {
            T Fr[NV];
#pragma unroll
            for (int v = 0; v < NV; ++v) Fr[v] = shfl_dn1(Fh[v]);
            if (cell_ok) {
                size_t off = DIR == 0 ? (size_t)line * a.nx + f : (size_t)f * a.nx + line;
                T unew[NV];
#pragma unroll
                for (int v = 0; v < NV; ++v) {
                    const size_t go = (size_t)gvar<SYS, DIR>(v) * ncell + off;
                    T d = -(Fr[v] - Fh[v]) * a.inv_h;
                    if (a.addend) d = d + a.addend[go];
                    if (a.mode == MODE_RHS) {
                        a.out[go] = d;
                    } else {
                        // SSP-RK3 stage, Shu-Osher form
                        T uk = R0[SEG_LOAD * v + k + 4];   // staged record: conserved variable v first
                        T u0 = a.U0[go];
                        T dt = (T)dtv;
                        T un;
                        if (a.stage == 0) un = u0 + dt * d;
                        else if (a.stage == 1) un = T(0.75) * u0 + T(0.25) * (uk + dt * d);
                        else un = T(1.0 / 3.0) * u0 + T(2.0 / 3.0) * (uk + dt * d);
                        a.out[go] = un;
                        unew[gvar<SYS, DIR>(v)] = un;
                    }
                }
                if (a.mode == MODE_STAGE) {
                    double w9[9];
                    bool ok = cell_speeds<T, SYS>(unew, a.gamma, a.adv, a.inv_dx, a.inv_dy, a.alpha_mode, w9);
                    if (!ok) bad |= ERR_NONPHYSICAL;
#pragma unroll
                    for (int q = 0; q < 9; ++q) wmax[q] = fmax(wmax[q], w9[q]);
                }
            }
        }
    }
    if (a.mode == MODE_STAGE) block_max_atomic(wmax, a.part, red);
    if (bad) atomicOr(a.err, bad);
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
    block_max_atomic(wmax, part, red);
    if (bad) atomicOr(err, bad);
}

// Reduce the spread maxima of one ring slot into alpha/den (and dt at the first stage of a step),
// then clear the slot for its next accumulation. One block of 64 threads.
//   frozen (nullable): replay the 8 constants (+ dt when stage == 0) from a recorded buffer.
//   record (nullable): write the 8 constants (+ dt when stage == 0) to a recording buffer.
// Recording layout per step: [stage0 alpha 8][stage1 alpha 8][stage2 alpha 8][dt].
__global__ void prep_kernel(Ctrl *ctrl, int ring, int stage, double dt_fixed, double cfl, const double *frozen,
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
        if (stage == 0) {
            double dt = dt_fixed > 0.0 ? dt_fixed : cfl / vals[8];
            if (frozen) dt = frozen[24];
            if (!(dt > 0.0) || !isfinite(dt)) atomicOr(&ctrl->err, ERR_NONFINITE);
            ctrl->dt = dt;
            if (record) record[24] = dt;
        }
    }
}

__global__ void clear_ring_kernel(Ctrl *ctrl, int ring)
{
    for (int q = threadIdx.x; q < NCOPY * NWORD; q += blockDim.x) (&ctrl->part[ring][0][0])[q] = 0ull;
}

// Copy the eight constants of the current stage out (parity/debug form).
__global__ void copy_alpha_kernel(const Ctrl *ctrl, double *dst)
{
    if (threadIdx.x < 8) dst[threadIdx.x] = ctrl->alpha[threadIdx.x];
}

}  // namespace teno
