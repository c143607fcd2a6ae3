// teno_adjoint.hpp -- gfx950 reverse-mode (vector-Jacobian) kernels of the frozen-selection operator
// and of the SSP-RK3 stages (double precision).
//
// With the stencil codes m+/m- of every face and field and the Lax-Friedrichs constants alpha held
// fixed, the numerical flux of a face is a smooth function of its eight stencil states:
//     Fhat = sum_s R_s (L_s . Y_s),   Y_s = sum_k ( cF_{s,k} F(U_k) + cU_{s,k} U_k ),
//     cF_{s,k} = (a+_{s,k} + a-_{s,k}) / 2,   cU_{s,k} = alpha_s (a+_{s,k} - a-_{s,k}) / 2,
// where a+ / a- are the selected Table 2 rows placed on the eight cells (the right-biased row
// mirrored), and L_s / R_s the Roe-averaged eigenvectors (Remark 3). Its reverse mode given the
// flux adjoint Fbar is
//     wbar_s = R_s . Fbar,   Lbar_s = wbar_s Y_s,   Rbar_{:,s} = Fbar (L_s . Y_s),
//     Ubar_k += L^T (cU_{:,k} o wbar) + A(U_k)^T L^T (cF_{:,k} o wbar),
// followed by the chain through the Roe average into the two cells of the face.
//
// Work decomposition: a wave owns 56 consecutive cells of a line and computes every face that
// touches them (faces c0-3 .. c0+59, one per lane); contributions are accumulated in LDS in eight
// passes (pass j: lane k adds to cell k+j, so no two lanes of a pass share a cell), which makes the
// result deterministic without global atomics. Periodic lines need at least 8 cells.
#pragma once
#include "teno_device.hpp"

namespace teno {

constexpr int ADJ_CELLS = 56;   // cells owned per segment
constexpr int ADJ_HALO = 7;     // first staged cell is c0 - 7
constexpr int ADJ_NSEG = 4;     // segments per block (one per wave)

struct VjpArgs {
    const double *U;            // state at which the operator is linearised
    const double *lam;          // adjoint of dU/dt
    double *grad;               // output (rk < 0)
    const uint32_t *masks;      // this direction's face mask words
    const double *alpha;        // 8 Lax-Friedrichs constants (device)
    int nx, ny, len, nlines, nseg, bc;
    int accumulate;             // rk < 0: 0 grad = result, 1 grad += result
    int scheme;
    double inv_h, gamma, adv;
    // rk = 0, 1, 2: the product G = (the other direction's part gy, if any) + this direction's is
    // not stored; the adjoint of SSP-RK3 stage rk is applied to it in place (rk_stage_adjoint), with
    // lam (above, the stencil input) the adjoint of the stage output
    int rk;
    const double *gy;           // the y-direction part of G (2D), else null
    double *lam_step;           // rk = 0, 1: the running adjoint of the step's input, updated in place
    double *lam_next;           // rk = 2: the running adjoint of the step's input, started here
    double *mu_next;            // rk = 2, 1: the adjoint of the stage input
    const double *dt;           // the step's dt (device)
};

// Adjoint of one SSP-RK3 stage (Shu-Osher form) at one element. g = J^T m is the operator's
// vector-Jacobian product at the stage input, m the adjoint of the stage output, l the running
// adjoint of the step's input U^n:
//   k = 2 (U^{n+1} = U^n/3 + 2/3 (U2 + dt L(U2))): m is the adjoint of U^{n+1}; mu <- 2/3 (m + dt g),
//          l <- m/3
//   k = 1 (U2 = 3/4 U^n + 1/4 (U1 + dt L(U1))):    l += 3/4 m, mu <- 1/4 (m + dt g)
//   k = 0 (U1 = U^n + dt L(U^n)):                   l += m + dt g
struct StageAdj { double l, mu; };
__device__ __forceinline__ StageAdj rk_stage_adjoint(int k, double m, double l, double g, double dt)
{
    StageAdj r;
    if (k == 2) {
        r.mu = (2.0 / 3.0) * (m + dt * g);
        r.l = (1.0 / 3.0) * m;
    } else if (k == 1) {
        r.l = l + 0.75 * m;
        r.mu = 0.25 * (m + dt * g);
    } else {
        r.l = l + (m + dt * g);
        r.mu = 0.0;
    }
    return r;
}

// Flux Jacobian transpose (local order rho, m_n, [m_t], E) applied to g, added to out.
template <int SYS>
__device__ __forceinline__ void flux_jac_t(double rho, double un, double ut, double H, double gm1, double adv,
                                           const double *u, const double *g, double *out)
{
    if constexpr (SYS == ADV1D) {
        out[0] += adv * g[0];
    } else if constexpr (SYS == BURGERS1D) {
        out[0] += u[0] * g[0];
    } else {
        constexpr int NV = Sys<SYS>::NV;
        const double pr = 0.5 * gm1 * (un * un + ut * ut);   // dp/drho
        const double pn = -gm1 * un;                         // dp/dm_n
        const double pt = -gm1 * ut;                         // dp/dm_t
        const double gE = g[NV - 1];
        out[0] += g[1] * (pr - un * un) + gE * un * (pr - H);
        out[1] += g[0] + g[1] * (2.0 * un + pn) + gE * (H + un * pn);
        out[NV - 1] += g[1] * gm1 + gE * un * (1.0 + gm1);
        if constexpr (NV == 4) {
            out[0] += -g[2] * un * ut;
            out[1] += g[2] * ut;
            out[2] += g[1] * pt + g[2] * un + gE * un * pt;
        }
    }
}

template <int SYS, int DIR>
__global__ void __launch_bounds__(BLOCK) vjp_kernel(VjpArgs a)
{
    constexpr int NV = Sys<SYS>::NV;
    constexpr int NREC = Sys<SYS>::NREC;
    constexpr bool EULER = SYS == EULER1D || SYS == EULER2D;
    constexpr int FIELDS = NREC + 2 * NV;                   // record, lam, accumulator
    constexpr int STRIDE = FIELDS * SEG_LOAD + 1;
    constexpr int LAM = NREC, ACC = NREC + NV;

    __shared__ double rec[ADJ_NSEG * STRIDE];
    __shared__ double coef[NCOEF_ROWS * 8];

    const int tid = threadIdx.x, lane = tid & (WAVE - 1), wid = tid / WAVE;
    const size_t ncell = (size_t)a.nx * a.ny;
    const bool periodic = a.bc == 0;

    fill_coef(coef);

    // tiles renumbered per XCD (neighbouring tiles share cache lines of the staged rows in one L2)
    const int tile = xcd_tile(blockIdx.x, gridDim.x);
    auto seg_of = [&](int s, int &line, int &c0) {
        if (DIR == 0) {
            int id = tile * ADJ_NSEG + s;
            line = id / a.nseg;
            c0 = (id % a.nseg) * ADJ_CELLS;
        } else {
            int ntile = (a.nlines + ADJ_NSEG - 1) / ADJ_NSEG;
            line = (tile % ntile) * ADJ_NSEG + s;
            c0 = (tile / ntile) * ADJ_CELLS;
        }
        if (line >= a.nlines) line = -1;
    };

    // ---- stage the state record, lambda and a zeroed accumulator ----
    // a thread's cells (up to IT of them) are all loaded before any is converted, so that the loads'
    // latencies overlap
    constexpr int NCELL = ADJ_NSEG * SEG_LOAD, IT = (NCELL + BLOCK - 1) / BLOCK;
    double uc[IT][NV], lc[IT][NV];
    int pos[IT];
#pragma unroll
    for (int it = 0; it < IT; ++it) {
        const int idx = tid + it * BLOCK;
        pos[it] = -1;
        if (idx >= NCELL) continue;
        int s, q;
        if (DIR == 0) { s = idx / SEG_LOAD; q = idx % SEG_LOAD; }
        else          { s = idx % ADJ_NSEG; q = idx / ADJ_NSEG; }
        int line, c0;
        seg_of(s, line, c0);
        if (line < 0) continue;
        const int c = c0 - ADJ_HALO + q;
        const int g = bc_index(c, a.len, a.bc);
        const bool real = periodic || (c >= 0 && c < a.len);
        const size_t off = DIR == 0 ? (size_t)line * a.nx + g : (size_t)g * a.nx + line;
        pos[it] = s * STRIDE + q;
#pragma unroll
        for (int v = 0; v < NV; ++v) {
            const size_t fo = (size_t)gvar<SYS, DIR>(v) * ncell + off;
            uc[it][v] = a.U[fo];
            lc[it][v] = real ? a.lam[fo] : 0.0;
        }
    }
#pragma unroll
    for (int it = 0; it < IT; ++it) {
        if (pos[it] < 0) continue;
        double *r = rec + pos[it];
        if constexpr (!EULER) {
            r[0] = uc[it][0];
        } else {
            using S = Sys<SYS>;
            const double rho = uc[it][0], mn = uc[it][1], mt = NV == 4 ? uc[it][2] : 0.0, E = uc[it][NV - 1];
            double sq, rs;
            sqrt_rsqrt(rho, sq, rs);
            double ir = rs * rs;          // (the recorded forward states are physical)
            double un = mn * ir, ut = mt * ir;
            double p = (a.gamma - 1.0) * (E - 0.5 * rho * (un * un + ut * ut));
            r[0] = rho;
            r[SEG_LOAD * 1] = mn;
            if constexpr (NV == 4) r[SEG_LOAD * 2] = mt;
            r[SEG_LOAD * S::E] = E;
            r[SEG_LOAD * S::UN] = un;
            if constexpr (NV == 4) r[SEG_LOAD * S::UT] = ut;
            r[SEG_LOAD * S::P] = p;
            r[SEG_LOAD * S::RS] = rs;                            // 1/sqrt(rho)
            r[SEG_LOAD * S::H] = (E + p) * ir;
        }
#pragma unroll
        for (int v = 0; v < NV; ++v) {
            r[SEG_LOAD * (LAM + v)] = lc[it][v];
            r[SEG_LOAD * (ACC + v)] = 0.0;
        }
    }
    __syncthreads();

    // Lax-Friedrichs constants in scalar registers (a vector load inside the stencil loop would wait
    // on every outstanding memory operation of the wave)
    double alpha[4];
#pragma unroll
    for (int v = 0; v < 4; ++v) alpha[v] = v < NV ? uniform_f64(a.alpha[4 * DIR + v]) : 0.0;
    const double gm1 = a.gamma - 1.0;

    for (int s = wid; s < ADJ_NSEG; s += BLOCK / WAVE) {
        int line, c0;
        seg_of(s, line, c0);
        if (line < 0) continue;
        double *R0 = rec + s * STRIDE;
        const int k = lane;
        const int f = c0 - 3 + k;                               // this lane's face
        const bool face_ok = k <= 62 && (periodic || (f >= 0 && f <= a.len));
        uint32_t mword = 0;
        if (face_ok) {
            int fc = periodic ? bc_index(f, a.len, 0) : f;      // face len of a periodic line = face 0
            size_t fidx = DIR == 0 ? (size_t)line * (a.len + 1) + fc : (size_t)fc * a.nx + line;
            mword = a.masks[fidx];
        }
        // flux adjoint: dU_i/dt = -(Fhat_{i+1/2} - Fhat_{i-1/2}) / h  =>  Fbar_f = (lam_f - lam_{f-1}) / h
        double Fb[NV];
#pragma unroll
        for (int v = 0; v < NV; ++v)
            Fb[v] = face_ok ? (R0[SEG_LOAD * (LAM + v) + k + 4] - R0[SEG_LOAD * (LAM + v) + k + 3]) * a.inv_h : 0.0;

        Roe<double> roe;
        double W = 1.0, iW = 1.0;
        if constexpr (EULER) {
            using S = Sys<SYS>;
            // sqrt(rho) = rho / sqrt(rho) from the staged reciprocal square root
            double sL = R0[k + 3] * R0[SEG_LOAD * S::RS + k + 3], sR = R0[k + 4] * R0[SEG_LOAD * S::RS + k + 4];
            W = sL + sR;
            iW = recip(W);
            roe.un = (sL * R0[SEG_LOAD * S::UN + k + 3] + sR * R0[SEG_LOAD * S::UN + k + 4]) * iW;
            if constexpr (NV == 4) roe.ut = (sL * R0[SEG_LOAD * S::UT + k + 3] + sR * R0[SEG_LOAD * S::UT + k + 4]) * iW;
            roe.H = (sL * R0[SEG_LOAD * S::H + k + 3] + sR * R0[SEG_LOAD * S::H + k + 4]) * iW;
            roe.q2 = roe.un * roe.un + roe.ut * roe.ut;
            double c2 = gm1 * (roe.H - 0.5 * roe.q2);
            sqrt_rsqrt(c2 > 0.0 ? c2 : 1.0, roe.cs, roe.ic);
            roe.b1 = gm1 * roe.ic * roe.ic;
            roe.b2 = 0.5 * roe.b1 * roe.q2;
        }
        double L[NV][NV], Rm[NV][NV];
#pragma unroll
        for (int sf = 0; sf < NV; ++sf) {
            double Ls[NV], Rs[NV];
            char_basis<double, NV>(roe, sf, Ls, Rs);
#pragma unroll
            for (int v = 0; v < NV; ++v) {
                L[sf][v] = Ls[v];
                Rm[v][sf] = Rs[v];
            }
        }
        double wb[NV];
#pragma unroll
        for (int sf = 0; sf < NV; ++sf) {
            double t = 0.0;
#pragma unroll
            for (int v = 0; v < NV; ++v) t += Rm[v][sf] * Fb[v];
            wb[sf] = t;
        }
        int mp[NV], mm[NV];
#pragma unroll
        for (int sf = 0; sf < NV; ++sf) {
            int cp = (int)((mword >> (8 * sf)) & 15u), cm = (int)((mword >> (8 * sf + 4)) & 15u);
            if (a.scheme == 1) { cp = TENO5_ROW[cp & 7]; cm = TENO5_ROW[cm & 7]; }
            mp[sf] = cp > 12 && a.scheme == 0 ? 0 : cp;
            mm[sf] = cm > 12 && a.scheme == 0 ? 0 : cm;
        }

        double Y[NV][NV];
#pragma unroll
        for (int sf = 0; sf < NV; ++sf)
#pragma unroll
            for (int v = 0; v < NV; ++v) Y[sf][v] = 0.0;

        // stencil cells k8 = 0..7 <-> cells i-3..i+4 (staged index q = k + k8)
#pragma unroll 1
        for (int k8 = 0; k8 < 8; ++k8) {
            asm volatile("" ::: "memory");
            const int q = k + k8;
            double u[NV], F[NV];
#pragma unroll
            for (int v = 0; v < NV; ++v) u[v] = R0[SEG_LOAD * v + q];
            double un = 0.0, ut = 0.0, p = 0.0, H = 0.0;
            if constexpr (!EULER) {
                F[0] = SYS == ADV1D ? a.adv * u[0] : 0.5 * u[0] * u[0];
            } else {
                using S = Sys<SYS>;
                un = R0[SEG_LOAD * S::UN + q];
                if constexpr (NV == 4) ut = R0[SEG_LOAD * S::UT + q];
                p = R0[SEG_LOAD * S::P + q];
                H = R0[SEG_LOAD * S::H + q];
                F[0] = u[1];
                F[1] = u[1] * un + p;
                if constexpr (NV == 4) F[2] = u[2] * un;
                F[NV - 1] = un * (u[NV - 1] + p);
            }
            double gU[NV], gF[NV];
#pragma unroll
            for (int v = 0; v < NV; ++v) { gU[v] = 0.0; gF[v] = 0.0; }
#pragma unroll
            for (int sf = 0; sf < NV; ++sf) {
                double ap = k8 <= 6 ? coef[mp[sf] * 8 + k8] : 0.0;
                double am = k8 >= 1 ? coef[mm[sf] * 8 + 7 - k8] : 0.0;
                double cF = 0.5 * (ap + am), cU = 0.5 * alpha[sf] * (ap - am);
                double tU = cU * wb[sf], tF = cF * wb[sf];
#pragma unroll
                for (int v = 0; v < NV; ++v) {
                    Y[sf][v] += cF * F[v] + cU * u[v];
                    gU[v] += tU * L[sf][v];
                    gF[v] += tF * L[sf][v];
                }
            }
            flux_jac_t<SYS>(u[0], un, ut, H, gm1, a.adv, u, gF, gU);
            if (face_ok) {
#pragma unroll
                for (int v = 0; v < NV; ++v) atomicAdd(&R0[SEG_LOAD * (ACC + v) + q], gU[v]);
            }
        }

        // ---- back through the Roe average into the face's two cells ----
        if constexpr (EULER) {
            using S = Sys<SYS>;
            const double h = 0.5;
            double Lb[4][4], Rb[4][4];       // in the two-dimensional layout (rho, n, t, E)
#pragma unroll
            for (int i = 0; i < 4; ++i)
#pragma unroll
                for (int j = 0; j < 4; ++j) { Lb[i][j] = 0.0; Rb[i][j] = 0.0; }
#pragma unroll
            for (int sf = 0; sf < NV; ++sf) {
                double w = 0.0;
#pragma unroll
                for (int v = 0; v < NV; ++v) w += L[sf][v] * Y[sf][v];
                const int s4 = (NV == 3 && sf == 2) ? 3 : sf;
#pragma unroll
                for (int v = 0; v < NV; ++v) {
                    const int v4 = (NV == 3 && v == 2) ? 3 : v;
                    Lb[s4][v4] = wb[sf] * Y[sf][v];
                    Rb[v4][s4] = Fb[v] * w;
                }
            }
            const double un = roe.un, ut = roe.ut, cs = roe.cs, ic = roe.ic, b1 = roe.b1, q2 = roe.q2;
            double unb = 0.0, utb = 0.0, Hb = 0.0, csb = 0.0, icb = 0.0, b1b = 0.0, b2b = 0.0, q2b = 0.0;
            // L rows: 0 = (h(b2+un ic), -h(b1 un + ic), -h b1 ut, h b1); 1 = (1-b2, b1 un, b1 ut, -b1);
            //         2 = (-ut, 0, 1, 0); 3 = (h(b2-un ic), -h(b1 un - ic), -h b1 ut, h b1)
            b2b += h * Lb[0][0] - Lb[1][0] + h * Lb[3][0];
            double X = h * (Lb[0][0] - Lb[3][0]);
            unb += X * ic;
            icb += X * un;
            b1b += -h * un * (Lb[0][1] + Lb[3][1]) - h * ut * (Lb[0][2] + Lb[3][2]) + h * (Lb[0][3] + Lb[3][3])
                 + un * Lb[1][1] + ut * Lb[1][2] - Lb[1][3];
            unb += -h * b1 * (Lb[0][1] + Lb[3][1]) + b1 * Lb[1][1];
            icb += -h * Lb[0][1] + h * Lb[3][1];
            utb += -h * b1 * (Lb[0][2] + Lb[3][2]) + b1 * Lb[1][2] - Lb[2][0];
            // R columns: 0 = (1, un-cs, ut, H-un cs); 1 = (1, un, ut, q2/2); 2 = (0, 0, 1, ut);
            //            3 = (1, un+cs, ut, H+un cs)
            unb += Rb[1][0] + Rb[1][1] + Rb[1][3] - cs * Rb[3][0] + cs * Rb[3][3];
            csb += -Rb[1][0] + Rb[1][3] - un * Rb[3][0] + un * Rb[3][3];
            utb += Rb[2][0] + Rb[2][1] + Rb[2][3] + Rb[3][2];
            Hb += Rb[3][0] + Rb[3][3];
            q2b += h * Rb[3][1];
            // b2 = b1 q2 / 2, b1 = gm1 ic^2, ic = 1/cs, cs = sqrt(c2), c2 = gm1 (H - q2/2), q2 = un^2 + ut^2
            b1b += h * q2 * b2b;
            q2b += h * b1 * b2b;
            icb += 2.0 * gm1 * ic * b1b;
            csb += -ic * ic * icb;
            double c2b = h * ic * csb;
            Hb += gm1 * c2b;
            q2b += -h * gm1 * c2b;
            unb += 2.0 * un * q2b;
            utb += 2.0 * ut * q2b;
            if constexpr (NV == 3) utb = 0.0;
            // Roe averages of (u_n, u_t, H) weighted by sqrt(rho) of cells i (q k+3) and i+1 (q k+4)
#pragma unroll
            for (int side = 0; side < 2; ++side) {
                const int q = k + 3 + side;
                const double rho = R0[q], rsq = R0[SEG_LOAD * S::RS + q], sq = rho * rsq;
                const double uc = R0[SEG_LOAD * S::UN + q];
                const double vc = NV == 4 ? R0[SEG_LOAD * S::UT + q] : 0.0;
                const double Hc = R0[SEG_LOAD * S::H + q];
                double sb = (unb * (uc - un) + utb * (vc - ut) + Hb * (Hc - roe.H)) * iW;
                double ucb = unb * sq * iW, vcb = utb * sq * iW, Hcb = Hb * sq * iW;
                const double ir = rsq * rsq;
                double g[NV];
#pragma unroll
                for (int v = 0; v < NV; ++v) g[v] = 0.0;
                // sqrt(rho)
                g[0] += sb * 0.5 * rsq;
                // u = m_n / rho, v = m_t / rho
                g[1] += ucb * ir;
                g[0] += -ucb * uc * ir;
                if constexpr (NV == 4) {
                    g[2] += vcb * ir;
                    g[0] += -vcb * vc * ir;
                }
                // H = (E + p) / rho
                g[NV - 1] += Hcb * ir;
                double pb = Hcb * ir;
                g[0] += -Hcb * Hc * ir;
                // p = gm1 (E - (m_n^2 + m_t^2) / (2 rho))
                g[NV - 1] += gm1 * pb;
                g[1] += -gm1 * uc * pb;
                if constexpr (NV == 4) g[2] += -gm1 * vc * pb;
                g[0] += 0.5 * gm1 * (uc * uc + vc * vc) * pb;
                if (face_ok) {
#pragma unroll
                    for (int v = 0; v < NV; ++v) atomicAdd(&R0[SEG_LOAD * (ACC + v) + q], g[v]);
                }
            }
        }

        // ---- owned cells: sum (outflow: fold the ghost copies into the boundary cells) and store ----
        asm volatile("" ::: "memory");
        __builtin_amdgcn_wave_barrier();
        const int c = c0 + k;
        if (k < ADJ_CELLS && c < a.len) {
            double tot[NV];
#pragma unroll
            for (int v = 0; v < NV; ++v) tot[v] = R0[SEG_LOAD * (ACC + v) + k + ADJ_HALO];
            if (!periodic) {
                if (c == 0) {
                    for (int qq = 0; qq < ADJ_HALO; ++qq)        // cells -7 .. -1
#pragma unroll
                        for (int v = 0; v < NV; ++v) tot[v] += R0[SEG_LOAD * (ACC + v) + qq];
                }
                if (c == a.len - 1) {
                    for (int qq = k + ADJ_HALO + 1; qq < SEG_LOAD; ++qq)   // cells len .. c0+64
#pragma unroll
                        for (int v = 0; v < NV; ++v) tot[v] += R0[SEG_LOAD * (ACC + v) + qq];
                }
            }
            size_t off = DIR == 0 ? (size_t)line * a.nx + c : (size_t)c * a.nx + line;
            if (a.rk < 0) {
#pragma unroll
                for (int v = 0; v < NV; ++v) {
                    size_t go = (size_t)gvar<SYS, DIR>(v) * ncell + off;
                    a.grad[go] = a.accumulate ? a.grad[go] + tot[v] : tot[v];
                }
            } else {
                // the stage adjoint on the finished product: m is the staged stencil input of this
                // (owned, so real) cell; every field's operands are read before any store
                const double dtv = *a.dt;
                double gv[NV], lv[NV];
#pragma unroll
                for (int v = 0; v < NV; ++v) {
                    size_t go = (size_t)gvar<SYS, DIR>(v) * ncell + off;
                    gv[v] = a.gy ? a.gy[go] + tot[v] : tot[v];
                    lv[v] = a.rk == 2 ? 0.0 : a.lam_step[go];
                }
#pragma unroll
                for (int v = 0; v < NV; ++v) {
                    size_t go = (size_t)gvar<SYS, DIR>(v) * ncell + off;
                    const double m = R0[SEG_LOAD * (LAM + v) + k + ADJ_HALO];
                    const StageAdj r = rk_stage_adjoint(a.rk, m, lv[v], gv[v], dtv);
                    if (a.rk == 2) {
                        a.lam_next[go] = r.l;
                        a.mu_next[go] = r.mu;
                    } else {
                        a.lam_step[go] = r.l;
                        if (a.rk == 1) a.mu_next[go] = r.mu;
                    }
                }
            }
        }
    }
}

}  // namespace teno
