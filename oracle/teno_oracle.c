/*
 * teno_oracle.c -- plain CPU reference (the "oracle") of the TENO7X semi-discrete operator and its
 * SSP-RK3 time stepping, in double precision.
 *
 * TEST INFRASTRUCTURE. Only the test-suite, the package's smoke check and the CPU-baseline leg of
 * the benchmark may load this library. It shares no code, header, table or helper with the GPU
 * library, and the GPU library never calls it.
 *
 * Method: F. Zhang, J. Liu, H. Zhang, C. Xu, "An extending strategy based on TENO framework for
 * hyperbolic conservation laws" (arXiv:1808.00037). Equations are named by their labels in the
 * paper's source.
 *
 * The oracle follows the paper's order of work: first the five-point TENO smoothness measurement
 * and cut-off of every face of the domain (eq:smooth_expl, eq:tau5, eq:TENO1, eq:norm, eq:seclect;
 * section "The stencil-selection procedure": the smoothness of the whole domain is computed before
 * any reconstruction), then per face the neighbour vector (eq:vec), the stencil from Table 3 and the
 * reconstruction with Table 2, then the conservative difference (eq:app). Systems are handled
 * characteristic-wise with Roe-averaged eigenvectors and global Lax-Friedrichs splitting (Remark 3,
 * section "One dimensional Euler equations"). Readings where the paper is silent are listed in the
 * design notes of the repository; the ones that shape code are repeated at the point of use.
 *
 * Build: gcc -O2 -ffp-contract=off -std=c11 -fPIC -shared (no fast-math: evaluation order is the
 * written one).
 */
#include <complex.h>
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define ORC_ADV1D 0
#define ORC_EULER1D 1
#define ORC_EULER2D 2
#define ORC_BURGERS1D 3

#define ORC_TENO7X 0
#define ORC_TENO5 1

#define ORC_BC_PERIODIC 0
#define ORC_BC_OUTFLOW 1

#define ORC_E_ARG (-1)
#define ORC_E_NONFINITE (-4)
#define ORC_E_NONPHYSICAL (-5)
#define ORC_E_ALLOC (-7)

#define ORC_G 4 /* ghost cells: face i+1/2 reads i-3..i+4 and the flags of its neighbour faces */

/* The constants C and q of eq:TENO1 are configuration (the paper's values: C = 1, q = 6). */

typedef struct {
    int32_t sys;        /* ORC_ADV1D, ORC_EULER1D, ORC_EULER2D, ORC_BURGERS1D */
    int32_t nx, ny;     /* ny = 1 for one-dimensional systems */
    int32_t bc_x, bc_y; /* ORC_BC_PERIODIC or ORC_BC_OUTFLOW */
    int32_t scheme;     /* ORC_TENO7X or ORC_TENO5 */
    int32_t alpha_mode; /* 0: one alpha per characteristic field, 1: one scalar max(|u_n|+c) */
    int32_t pad_;
    double dx, dy;
    double gamma;       /* ratio of specific heats */
    double ct;          /* cut-off C_T of eq:seclect */
    double eps_x, eps_y;/* epsilon of eq:TENO1 for x- and y-faces */
    double adv_speed;   /* a in u_t + a u_x = 0 */
    double C;           /* C of eq:TENO1 (the paper: 1) */
    int32_t q;          /* q of eq:TENO1 (the paper: 6), q >= 1 */
    int32_t characteristic; /* 1: reconstruct in characteristic variables (Remark 3); 0: per conserved
                               component (L = R = I, one Lax-Friedrichs constant max(|u_n| + c)) */
} orc_cfg;

static int orc_nvar(const orc_cfg *c)
{
    switch (c->sys) {
    case ORC_EULER1D: return 3;
    case ORC_EULER2D: return 4;
    default: return 1;
    }
}

static size_t orc_nfaces(const orc_cfg *c)
{
    size_t n = (size_t)c->ny * (c->nx + 1);
    if (c->sys == ORC_EULER2D) n += (size_t)(c->ny + 1) * c->nx;
    return n;
}

static int orc_bc_index(int i, int n, int bc)
{
    if (bc == ORC_BC_PERIODIC) return ((i % n) + n) % n;
    return i < 0 ? 0 : (i >= n ? n - 1 : i);
}

/* ---------------------------------------------------------------------------------------------
 * Table 2: coefficients a_{m,l}, l = i-3..i+3, of the thirteen candidate reconstructions of the
 * presented method, as printed (numerator, denominator). Each double is the correctly rounded
 * quotient of two exactly representable integers.
 * ------------------------------------------------------------------------------------------- */
static const int ORC_T2_RAT[13][7][2] = {
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
};

/* Table 1: the seven single five-point polynomials equivalent to the TENO5 weights, rows selected
 * by (delta0, delta1, delta2), coefficients for l = i-2..i+2. Used only to cross-check eq:TENO_W. */
static const int ORC_T1_RAT[7][5][2] = {
    {{1, 30}, {-13, 60}, {47, 60}, {9, 20}, {-1, 20}},
    {{0, 1}, {-1, 9}, {2, 3}, {1, 2}, {-1, 18}},
    {{1, 21}, {-13, 42}, {41, 42}, {2, 7}, {0, 1}},
    {{0, 1}, {0, 1}, {1, 3}, {5, 6}, {-1, 6}},
    {{0, 1}, {-1, 6}, {5, 6}, {1, 3}, {0, 1}},
    {{1, 3}, {-7, 6}, {11, 6}, {0, 1}, {0, 1}},
    {{1, 12}, {-7, 24}, {17, 24}, {5, 8}, {-1, 8}},
};
static const char *ORC_T1_FLAGS[7] = {"111", "011", "110", "001", "010", "100", "101"};

static double ORC_TABLE2[13][7];
static double ORC_TABLE1[7][5];

/* Table 3: neighbour vector Delta_i = (delta_{i-1,0}, delta_{i,0}, delta_{i,1}, delta_{i,2},
 * delta_{i+1,2}) -> stencil m, '*' = either value. The pattern (*,0,0,0,*) has no stencil. */
static const struct { const char *pat; int m; } ORC_T3[13] = {
    {"11111", 0}, {"01111", 1}, {"11110", 2}, {"*0111", 3}, {"01110", 4}, {"1110*", 5},
    {"**011", 6}, {"*0110", 7}, {"0110*", 8}, {"1100*", 9}, {"**010", 10}, {"*010*", 11},
    {"0100*", 12},
};

static void orc_init_tables(void)
{
    static int done = 0;
    if (done) return;
    for (int m = 0; m < 13; ++m)
        for (int l = 0; l < 7; ++l)
            ORC_TABLE2[m][l] = (double)ORC_T2_RAT[m][l][0] / (double)ORC_T2_RAT[m][l][1];
    for (int m = 0; m < 7; ++m)
        for (int l = 0; l < 5; ++l)
            ORC_TABLE1[m][l] = (double)ORC_T1_RAT[m][l][0] / (double)ORC_T1_RAT[m][l][1];
    done = 1;
}

/* Stencil index for a neighbour vector given as five 0/1 values; -1 when Table 3 has none. */
static int orc_table3(const int d[5])
{
    int found = -1, nmatch = 0;
    for (int r = 0; r < 13; ++r) {
        int ok = 1;
        for (int q = 0; q < 5; ++q) {
            char ch = ORC_T3[r].pat[q];
            if (ch != '*' && (ch - '0') != d[q]) { ok = 0; break; }
        }
        if (ok) { found = ORC_T3[r].m; ++nmatch; }
    }
    return nmatch == 1 ? found : -1;
}

/* Five-point TENO smoothness measurement and cut-off for one side of one face.
 * (a,b,c,d,e) = values at i-2..i+2 in upwind order.
 *   beta_k: eq:smooth_expl; tau5 = |beta0 - beta2| (eq:tau5);
 *   gamma_k = (C + tau5/(beta_k + eps))^q (eq:TENO1); chi_k = gamma_k / sum gamma (eq:norm);
 *   delta_k = 0 if chi_k < C_T else 1 (eq:seclect; equality keeps the stencil). */
static void orc_beta5(double a, double b, double c, double d, double e, double beta[3])
{
    beta[0] = 0.25 * (a - 4.0 * b + 3.0 * c) * (a - 4.0 * b + 3.0 * c)
            + (13.0 / 12.0) * (a - 2.0 * b + c) * (a - 2.0 * b + c);
    beta[1] = 0.25 * (b - d) * (b - d)
            + (13.0 / 12.0) * (b - 2.0 * c + d) * (b - 2.0 * c + d);
    beta[2] = 0.25 * (3.0 * c - 4.0 * d + e) * (3.0 * c - 4.0 * d + e)
            + (13.0 / 12.0) * (c - 2.0 * d + e) * (c - 2.0 * d + e);
}

static void orc_flags5(double a, double b, double c, double d, double e, double eps, double ct,
                       double C, int q, int delta[3], double chi[3])
{
    double beta[3];
    orc_beta5(a, b, c, d, e, beta);
    double tau = fabs(beta[0] - beta[2]);
    double g[3], sum = 0.0;
    for (int k = 0; k < 3; ++k) {
        double r = C + tau / (beta[k] + eps);
        double p = 1.0;
        for (int j = 0; j < q; ++j) p *= r;
        g[k] = p;
        sum += g[k];
    }
    for (int k = 0; k < 3; ++k) {
        chi[k] = g[k] / sum;
        delta[k] = chi[k] < ct ? 0 : 1;
    }
}

/* ---- generic per-face arithmetic: real and complex instantiations ---- */
#define REAL double
#define FN(x) x##_r
#define SQRT(x) sqrt(x)
#include "oracle_face.inc"
#undef REAL
#undef FN
#undef SQRT

#define REAL double complex
#define FN(x) x##_c
#define SQRT(x) csqrt(x)
#include "oracle_face.inc"
#undef REAL
#undef FN
#undef SQRT

/* Primitive check of one cell; also returns |u_n| + c etc. for the wave speeds. */
static int orc_cell_speeds(const orc_cfg *c, const double *U, size_t stride, double *ux, double *uy, double *cs)
{
    const double gm1 = c->gamma - 1.0;
    *uy = 0.0;
    *cs = 0.0;
    if (c->sys == ORC_ADV1D) { *ux = c->adv_speed; return isfinite(U[0]) ? 0 : ORC_E_NONFINITE; }
    if (c->sys == ORC_BURGERS1D) { *ux = U[0]; return isfinite(U[0]) ? 0 : ORC_E_NONFINITE; }
    double rho = U[0], mx = U[stride];
    double my = c->sys == ORC_EULER2D ? U[2 * stride] : 0.0;
    double E = U[(c->sys == ORC_EULER2D ? 3 : 2) * stride];
    if (!isfinite(rho) || !isfinite(mx) || !isfinite(my) || !isfinite(E)) return ORC_E_NONFINITE;
    if (!(rho > 0.0)) return ORC_E_NONPHYSICAL;
    double u = mx / rho, v = my / rho;
    double p = gm1 * (E - 0.5 * rho * (u * u + v * v));
    if (!(p > 0.0)) return ORC_E_NONPHYSICAL;
    *ux = u;
    *uy = v;
    *cs = sqrt(c->gamma * p / rho);
    return 0;
}

/* Global Lax-Friedrichs constants and the CFL denominator of one state.
 * alpha[0..3]: x-direction fields, alpha[4..7]: y-direction fields (unused entries 0).
 * Per field: alpha_s = max over interior cells of |lambda_s|, with lambda = (u_n - c, u_n, [u_n],
 * u_n + c) (reading of "global Lax-Friedrichs"); alpha_mode 1: max(|u_n| + c) for every field.
 * *cfl_den = max_j ( (|u_j|+c_j)/dx [+ (|v_j|+c_j)/dy] ); dt = CFL / *cfl_den. */
int orc_wave_speeds(const orc_cfg *c, const double *U, double *alpha, double *cfl_den)
{
    const int nv = orc_nvar(c);
    const size_t n = (size_t)c->nx * c->ny;
    for (int k = 0; k < 8; ++k) alpha[k] = 0.0;
    double den = 0.0;
    for (size_t q = 0; q < n; ++q) {
        double ux, uy, cs;
        int st = orc_cell_speeds(c, U + q, n, &ux, &uy, &cs);
        if (st) return st;
        double lx[4], ly[4];
        int nf = nv;
        if (c->sys == ORC_EULER1D) { lx[0] = ux - cs; lx[1] = ux; lx[2] = ux + cs; }
        else if (c->sys == ORC_EULER2D) {
            lx[0] = ux - cs; lx[1] = ux; lx[2] = ux; lx[3] = ux + cs;
            ly[0] = uy - cs; ly[1] = uy; ly[2] = uy; ly[3] = uy + cs;
        } else lx[0] = ux;
        /* per conserved component, every component needs the largest wave speed */
        const int scalar = c->alpha_mode || !c->characteristic;
        for (int s = 0; s < nf; ++s) {
            double ax = scalar ? fabs(ux) + cs : fabs(lx[s]);
            if (ax > alpha[s]) alpha[s] = ax;
            if (c->sys == ORC_EULER2D) {
                double ay = scalar ? fabs(uy) + cs : fabs(ly[s]);
                if (ay > alpha[4 + s]) alpha[4 + s] = ay;
            }
        }
        double s = (fabs(ux) + cs) / c->dx;
        if (c->sys == ORC_EULER2D) s = s + (fabs(uy) + cs) / c->dy;
        if (s > den) den = s;
    }
    *cfl_den = den;
    return 0;
}

/* Smoothness flags of every face (including one extra face beyond each end of every line) and the
 * selection codes derived from them.
 * flags word of a face: bits 6s+k = delta^+_k, bits 6s+3+k = delta^-_k of characteristic field s.
 * mask word of a face: bits 8s..8s+3 = code of the '+' side, 8s+4..8s+7 = code of the '-' side.
 * chi (nullable): 24 doubles per face, [s][side][k].
 * The '-' side is the mirror image about the face (reading: the paper describes only the
 * left-biased side): its five-point values are taken at i+3, i+2, i+1, i, i-1 and its neighbour
 * vector is (delta^-_{i+1,0}, delta^-_{i,0}, delta^-_{i,1}, delta^-_{i,2}, delta^-_{i-1,2}). */
static int orc_select_all(const orc_cfg *c, const double *U, const double *alpha8,
                          uint32_t *masks_x, uint32_t *masks_y, uint32_t *flags_x, uint32_t *flags_y,
                          double *chi_x, double *chi_y)
{
    const int nv = orc_nvar(c), nx = c->nx, ny = c->ny;
    const int two_d = c->sys == ORC_EULER2D;
    const int gy = two_d ? ORC_G : 0;
    size_t psize = (size_t)nv * (nx + 2 * ORC_G) * (ny + 2 * gy);
    double *P = (double *)malloc(psize * sizeof(double));
    int maxlen = nx > ny ? nx : ny;
    uint32_t *fl = (uint32_t *)malloc((size_t)(maxlen + 3) * sizeof(uint32_t));
    double *chl = (double *)malloc((size_t)(maxlen + 3) * 24 * sizeof(double));
    if (!P || !fl || !chl) { free(P); free(fl); free(chl); return ORC_E_ALLOC; }
    pad_r(c, U, P);
    int status = 0;
    for (int dir = 0; dir < (two_d ? 2 : 1) && status == 0; ++dir) {
        const int nlines = dir == 0 ? ny : nx, len = dir == 0 ? nx : ny;
        const double *alpha = alpha8 + 4 * dir;
        const double eps = dir == 0 ? c->eps_x : c->eps_y;
        for (int ln = 0; ln < nlines && status == 0; ++ln) {
            /* pass 1: smoothness flags of faces -1..len+1 (every face of the line) */
            for (int f = -1; f <= len + 1; ++f) {
                double Us[8][4], L[4][4], R[4][4], c2, v[2][4][8];
                /* the flags read cells i-2..i+3 (k = 1..6); the two unused end slots hold copies
                   of their neighbours so that no state outside the padded array is read */
                {
                    const int px = nx + 2 * ORC_G, py = ny + 2 * gy;
                    for (int k = 0; k < 8; ++k) {
                        int kk = k < 1 ? 1 : (k > 6 ? 6 : k);
                        int off = f - 4 + kk, ip, jp;
                        if (dir == 0) { ip = off + ORC_G; jp = ln + gy; }
                        else          { ip = ln + ORC_G; jp = off + gy; }
                        for (int var = 0; var < nv; ++var) Us[k][var] = P[((size_t)var * py + jp) * px + ip];
                    }
                }
                face_basis_r(c, dir, Us[3], Us[4], L, R, &c2);
                if (!(c2 > 0.0)) { status = isfinite(c2) ? ORC_E_NONPHYSICAL : ORC_E_NONFINITE; break; }
                project_r(c, dir, nv, Us, L, alpha, v);
                uint32_t word = 0;
                for (int s = 0; s < nv; ++s) {
                    int dp[3], dm[3];
                    double xp[3], xm[3];
                    orc_flags5(v[0][s][1], v[0][s][2], v[0][s][3], v[0][s][4], v[0][s][5],
                               eps, c->ct, c->C, c->q, dp, xp);
                    orc_flags5(v[1][s][6], v[1][s][5], v[1][s][4], v[1][s][3], v[1][s][2],
                               eps, c->ct, c->C, c->q, dm, xm);
                    for (int k = 0; k < 3; ++k) {
                        word |= (uint32_t)dp[k] << (6 * s + k);
                        word |= (uint32_t)dm[k] << (6 * s + 3 + k);
                        chl[(size_t)(f + 1) * 24 + s * 6 + k] = xp[k];
                        chl[(size_t)(f + 1) * 24 + s * 6 + 3 + k] = xm[k];
                    }
                }
                fl[f + 1] = word;
            }
            if (status) break;
            /* pass 2: neighbour vectors and Table 3 (TENO7X) or the own three flags (TENO5) */
            for (int f = 0; f <= len; ++f) {
                uint32_t wl = fl[f], w0 = fl[f + 1], wr = fl[f + 2];
                uint32_t mword = 0;
                for (int s = 0; s < nv; ++s) {
#define DB(w, side, k) ((int)(((w) >> (6 * s + 3 * (side) + (k))) & 1u))
                    int cp, cm;
                    if (c->scheme == ORC_TENO7X) {
                        int Dp[5] = {DB(wl, 0, 0), DB(w0, 0, 0), DB(w0, 0, 1), DB(w0, 0, 2), DB(wr, 0, 2)};
                        int Dm[5] = {DB(wr, 1, 0), DB(w0, 1, 0), DB(w0, 1, 1), DB(w0, 1, 2), DB(wl, 1, 2)};
                        cp = orc_table3(Dp);
                        cm = orc_table3(Dm);
                    } else {
                        cp = (DB(w0, 0, 0) << 2) | (DB(w0, 0, 1) << 1) | DB(w0, 0, 2);
                        cm = (DB(w0, 1, 0) << 2) | (DB(w0, 1, 1) << 1) | DB(w0, 1, 2);
                        if (cp == 0) cp = -1;
                        if (cm == 0) cm = -1;
                    }
#undef DB
                    /* no admissible stencil: only reachable when chi is not a number */
                    if (cp < 0 || cm < 0) { status = ORC_E_NONFINITE; break; }
                    mword |= (uint32_t)cp << (8 * s);
                    mword |= (uint32_t)cm << (8 * s + 4);
                }
                if (status) break;
                size_t fi = dir == 0 ? (size_t)ln * (nx + 1) + f : (size_t)f * nx + ln;
                uint32_t *mo = dir == 0 ? masks_x : masks_y;
                uint32_t *fo = dir == 0 ? flags_x : flags_y;
                double *co = dir == 0 ? chi_x : chi_y;
                mo[fi] = mword;
                if (fo) fo[fi] = w0;
                if (co) memcpy(co + fi * 24, chl + (size_t)(f + 1) * 24, 24 * sizeof(double));
            }
        }
    }
    free(P);
    free(fl);
    free(chl);
    return status;
}

/* ============================== exported API (called through ctypes) ============================== */

void orc_tables(double *t2 /* [13][7] */, double *t1 /* [7][5] */)
{
    orc_init_tables();
    memcpy(t2, ORC_TABLE2, sizeof ORC_TABLE2);
    memcpy(t1, ORC_TABLE1, sizeof ORC_TABLE1);
}

/* Table 3 for one vector (a,b,c,d,e) packed as 16a+8b+4c+2d+e; -1 = no stencil. */
int orc_select7(int pattern)
{
    int d[5];
    for (int q = 0; q < 5; ++q) d[q] = (pattern >> (4 - q)) & 1;
    return orc_table3(d);
}

/* Flags of one five-point stencil (upwind order), for tests. */
void orc_flags5_api(const double *f5, double eps, double ct, double C, int32_t q, int32_t *delta, double *chi,
                    double *beta)
{
    int d[3];
    orc_flags5(f5[0], f5[1], f5[2], f5[3], f5[4], eps, ct, C, q, d, chi);
    orc_beta5(f5[0], f5[1], f5[2], f5[3], f5[4], beta);
    for (int k = 0; k < 3; ++k) delta[k] = d[k];
}

/* One side's reconstruction from seven upwind-ordered values and a selection code. */
double orc_recon_api(const orc_cfg *c, int code, const double *w7)
{
    orc_init_tables();
    return recon_side_r(c, code, w7);
}

/* Table 1 row for flags (d0,d1,d2) applied to five values; -1 row index if (0,0,0). */
double orc_table1_api(int d0, int d1, int d2, const double *f5)
{
    orc_init_tables();
    char key[4] = {(char)('0' + d0), (char)('0' + d1), (char)('0' + d2), 0};
    for (int m = 0; m < 7; ++m)
        if (strcmp(key, ORC_T1_FLAGS[m]) == 0) {
            double acc = 0.0;
            for (int l = 0; l < 5; ++l) acc += ORC_TABLE1[m][l] * f5[l];
            return acc;
        }
    return NAN;
}

/* Roe state and eigenvectors at a face between two states (for tests): L, R as [4][4]. */
int orc_eigen_api(const orc_cfg *c, int dir, const double *UL, const double *UR, double *L, double *R)
{
    double Lm[4][4], Rm[4][4], c2;
    face_eigen_r(c, dir, UL, UR, Lm, Rm, &c2);
    memcpy(L, Lm, sizeof Lm);
    memcpy(R, Rm, sizeof Rm);
    return c2 > 0.0 ? 0 : ORC_E_NONPHYSICAL;
}

void orc_phys_flux_api(const orc_cfg *c, int dir, const double *U, double *F)
{
    phys_flux_r(c, dir, U, F);
}

size_t orc_nfaces_api(const orc_cfg *c) { return orc_nfaces(c); }

/* The full operator dU/dt = L(U): wave speeds (unless alpha_in is given), flags of the whole
 * domain, selection, reconstruction and the conservative difference.
 * All output pointers except dUdt are nullable. alpha_out/alpha_in: [8] (x fields, y fields). */
int orc_rhs(const orc_cfg *c, const double *U, const double *alpha_in, double *dUdt,
            uint32_t *masks_x, uint32_t *masks_y, uint32_t *flags_x, uint32_t *flags_y,
            double *chi_x, double *chi_y, double *Fx, double *Fy, double *alpha_out)
{
    orc_init_tables();
    if (!c || !U || !dUdt || c->nx < 1 || c->ny < 1) return ORC_E_ARG;
    if (c->sys != ORC_EULER2D && c->ny != 1) return ORC_E_ARG;
    if (c->q < 1 || !(c->C > 0.0)) return ORC_E_ARG;
    double alpha[8], den;
    int st = orc_wave_speeds(c, U, alpha, &den);
    if (st) return st;
    if (alpha_in) memcpy(alpha, alpha_in, sizeof alpha);
    if (alpha_out) memcpy(alpha_out, alpha, sizeof alpha);
    const size_t nfx = (size_t)c->ny * (c->nx + 1), nfy = (size_t)(c->ny + 1) * c->nx;
    uint32_t *mx = masks_x ? masks_x : (uint32_t *)malloc(nfx * sizeof(uint32_t));
    uint32_t *my = masks_y ? masks_y : (uint32_t *)malloc(nfy * sizeof(uint32_t));
    if (!mx || !my) return ORC_E_ALLOC;
    st = orc_select_all(c, U, alpha, mx, my, flags_x, flags_y, chi_x, chi_y);
    if (st == 0) st = rhs_frozen_r(c, U, alpha, alpha + 4, mx, my, dUdt, Fx, Fy);
    if (!masks_x) free(mx);
    if (!masks_y) free(my);
    return st;
}

/* The operator with the selection codes and alphas given (frozen). */
int orc_rhs_frozen(const orc_cfg *c, const double *U, const double *alpha8, const uint32_t *masks_x,
                   const uint32_t *masks_y, double *dUdt)
{
    orc_init_tables();
    return rhs_frozen_r(c, U, alpha8, alpha8 + 4, masks_x, masks_y, dUdt, NULL, NULL);
}

/* Directional derivative (J d) of the frozen operator at U, by the complex step
 * L(U + i h d) = L(U) + i h J d + O(h^2): J d = Im(L(U + i h d)) / h, exact up to rounding. */
int orc_rhs_frozen_jvp(const orc_cfg *c, const double *U, const double *d, const double *alpha8,
                       const uint32_t *masks_x, const uint32_t *masks_y, double h, double *Jd)
{
    orc_init_tables();
    const size_t n = (size_t)orc_nvar(c) * c->nx * c->ny;
    double complex *Uc = (double complex *)malloc(n * sizeof(double complex));
    double complex *Rc = (double complex *)malloc(n * sizeof(double complex));
    if (!Uc || !Rc) { free(Uc); free(Rc); return ORC_E_ALLOC; }
    for (size_t q = 0; q < n; ++q) Uc[q] = U[q] + I * (h * d[q]);
    int st = rhs_frozen_c(c, Uc, alpha8, alpha8 + 4, masks_x, masks_y, Rc, NULL, NULL);
    for (size_t q = 0; q < n; ++q) Jd[q] = cimag(Rc[q]) / h;
    free(Uc);
    free(Rc);
    return st;
}

/* One stage of the Shu-Osher SSP-RK3 step (Gottlieb, Shu & Tadmor 2001; the paper omits the
 * formula), over n values: Us holds the stage input U^(k) and receives the stage output,
 *   stage 0: U1 = U0 + dt L(U0);  stage 1: U2 = 3/4 U0 + 1/4 (U1 + dt L(U1));
 *   stage 2: U3 = 1/3 U0 + 2/3 (U2 + dt L(U2)),
 * with dU = L(U^(k)) given. */
void orc_rk3_combine(int stage, size_t n, const double *U0, double *Us, const double *dU, double dt)
{
    for (size_t q = 0; q < n; ++q) {
        if (stage == 0)      Us[q] = U0[q] + dt * dU[q];
        else if (stage == 1) Us[q] = 0.75 * U0[q] + 0.25 * (Us[q] + dt * dU[q]);
        else                 Us[q] = (1.0 / 3.0) * U0[q] + (2.0 / 3.0) * (Us[q] + dt * dU[q]);
    }
}

/* SSP-RK3 trajectory. dt_fixed > 0: that step size; else dt = cfl / max_j(...) from U^n.
 * Recording (all nullable): masks [nsteps][3][nfaces], alpha [nsteps][3][8], dt [nsteps].
 * Each stage's alpha and selection come from that stage's own input state. */
int orc_run(const orc_cfg *c, double *U, int nsteps, double dt_fixed, double cfl,
            uint32_t *rec_masks, double *rec_alpha, double *rec_dt)
{
    orc_init_tables();
    const int nv = orc_nvar(c);
    const size_t n = (size_t)nv * c->nx * c->ny;
    const size_t nf = orc_nfaces(c), nfx = (size_t)c->ny * (c->nx + 1);
    double *U0 = (double *)malloc(n * sizeof(double));
    double *Us = (double *)malloc(n * sizeof(double));
    double *dU = (double *)malloc(n * sizeof(double));
    uint32_t *m = (uint32_t *)malloc(nf * sizeof(uint32_t));
    if (!U0 || !Us || !dU || !m) { free(U0); free(Us); free(dU); free(m); return ORC_E_ALLOC; }
    int st = 0;
    for (int step = 0; step < nsteps && st == 0; ++step) {
        double dt = dt_fixed;
        if (!(dt > 0.0)) {
            double a8[8], den;
            st = orc_wave_speeds(c, U, a8, &den);
            if (st) break;
            dt = cfl / den;
        }
        if (rec_dt) rec_dt[step] = dt;
        memcpy(U0, U, n * sizeof(double));
        memcpy(Us, U, n * sizeof(double));
        for (int stage = 0; stage < 3 && st == 0; ++stage) {
            double a8[8];
            st = orc_rhs(c, Us, NULL, dU, m, m + nfx, NULL, NULL, NULL, NULL, NULL, NULL, a8);
            if (st) break;
            if (rec_masks) memcpy(rec_masks + ((size_t)step * 3 + stage) * nf, m, nf * sizeof(uint32_t));
            if (rec_alpha) memcpy(rec_alpha + ((size_t)step * 3 + stage) * 8, a8, sizeof a8);
            orc_rk3_combine(stage, n, U0, Us, dU, dt);
        }
        if (st == 0) memcpy(U, Us, n * sizeof(double));
    }
    free(U0);
    free(Us);
    free(dU);
    free(m);
    return st;
}

/* The trajectory with every stage's selection, alpha and every step's dt given (frozen). */
int orc_run_frozen(const orc_cfg *c, double *U, int nsteps, const uint32_t *rec_masks,
                   const double *rec_alpha, const double *rec_dt)
{
    orc_init_tables();
    const size_t nf = orc_nfaces(c);
    int st = 0;
    for (int step = 0; step < nsteps && st == 0; ++step)
        st = rk3_frozen_r(c, U, rec_dt[step], rec_alpha + (size_t)step * 24, rec_masks + (size_t)step * 3 * nf);
    return st;
}

/* Directional derivative of the frozen trajectory map U0 -> U_n by the complex step. */
int orc_run_frozen_jvp(const orc_cfg *c, const double *U, const double *d, int nsteps,
                       const uint32_t *rec_masks, const double *rec_alpha, const double *rec_dt,
                       double h, double *Jd)
{
    orc_init_tables();
    const size_t n = (size_t)orc_nvar(c) * c->nx * c->ny;
    const size_t nf = orc_nfaces(c);
    double complex *Uc = (double complex *)malloc(n * sizeof(double complex));
    if (!Uc) return ORC_E_ALLOC;
    for (size_t q = 0; q < n; ++q) Uc[q] = U[q] + I * (h * d[q]);
    int st = 0;
    for (int step = 0; step < nsteps && st == 0; ++step)
        st = rk3_frozen_c(c, Uc, rec_dt[step], rec_alpha + (size_t)step * 24, rec_masks + (size_t)step * 3 * nf);
    for (size_t q = 0; q < n; ++q) Jd[q] = cimag(Uc[q]) / h;
    free(Uc);
    return st;
}
