// teno_adjoint.hip -- host side of the frozen-selection adjoint ABI (include/teno.h).
//
// Recording run: the forward steps of teno_run, plus a checkpoint copy of the state every
// ckpt_every steps (or, with TENO_CKPT_STAGES, the three stage inputs of every step), every stage's
// mask words and every stage's Lax-Friedrichs constants and step dt (written by the
// stage-preparation kernel on the device).
// Reverse sweep: per checkpoint segment, in reverse: replay the segment forward with the recorded
// selection/constants/dt while keeping the three stage inputs of every step (or read them from the
// recording when it stored every stage input), then apply the adjoint of every stage in reverse: G = J^T mu by the vector-Jacobian kernels (y into a buffer, then x),
// with the stage adjoint applied to G in the x kernel's epilogue (G itself is never stored).
#include <hip/hip_runtime.h>

#include <cstring>

#include "teno.h"
#include "teno_adjoint.hpp"
#include "teno_device.hpp"
#include "teno_internal.hpp"

using namespace teno;

#define HIP_TRY(expr)                                   \
    do {                                                \
        hipError_t e_ = (expr);                         \
        if (e_ != hipSuccess) return TENO_E_HIP;        \
    } while (0)

// Plain product (rk < 0): grad = / += J^T lam. Fused (rk = 0, 1, 2, see VjpArgs): the adjoint of RK stage
// rk applied to G = gy + this direction's product.
struct StageIO {
    int rk = -1;
    const double *gy = nullptr;
    double *lam_step = nullptr, *lam_next = nullptr, *mu_next = nullptr;
    const double *dt = nullptr;
};

template <int SYS, int DIR>
static void launch_vjp_t(teno_ctx *c, const double *U, const double *lam, double *grad, const uint32_t *masks,
                         const double *alpha, int accumulate, const StageIO &io = StageIO())
{
    VjpArgs a;
    std::memset(&a, 0, sizeof a);
    a.U = U;
    a.lam = lam;
    a.grad = grad;
    a.masks = masks;
    a.alpha = alpha;
    a.nx = c->grid.nx;
    a.ny = c->grid.ny;
    a.len = DIR == 0 ? c->grid.nx : c->grid.ny;
    a.nlines = DIR == 0 ? c->grid.ny : c->grid.nx;
    a.nseg = (a.len + ADJ_CELLS - 1) / ADJ_CELLS;
    a.bc = DIR == 0 ? c->grid.bc_x : c->grid.bc_y;
    a.accumulate = accumulate;
    a.scheme = c->opts.scheme;
    a.inv_h = 1.0 / (DIR == 0 ? c->dx : c->dy);
    a.gamma = c->opts.gamma;
    a.adv = c->opts.adv_speed;
    a.rk = io.rk;
    a.gy = io.gy;
    a.lam_step = io.lam_step;
    a.lam_next = io.lam_next;
    a.mu_next = io.mu_next;
    a.dt = io.dt;
    unsigned nblocks;
    if (DIR == 0) {
        nblocks = (unsigned)(((size_t)a.nseg * a.nlines + ADJ_NSEG - 1) / ADJ_NSEG);
    } else {
        nblocks = (unsigned)((size_t)((a.nlines + ADJ_NSEG - 1) / ADJ_NSEG) * a.nseg);
    }
    hipLaunchKernelGGL((vjp_kernel<SYS, DIR>), dim3(nblocks), dim3(BLOCK), 0, c->stream, a);
}

// grad = J(U)^T lam for the frozen operator (both directions).
static void enqueue_rhs_vjp(teno_ctx *c, const double *U, const uint32_t *masks, const double *alpha,
                            const double *lam, double *grad)
{
    switch (c->grid.sys) {
    case TENO_ADV1D: launch_vjp_t<ADV1D, 0>(c, U, lam, grad, masks, alpha, 0); break;
    case TENO_BURGERS1D: launch_vjp_t<BURGERS1D, 0>(c, U, lam, grad, masks, alpha, 0); break;
    case TENO_EULER1D: launch_vjp_t<EULER1D, 0>(c, U, lam, grad, masks, alpha, 0); break;
    default:
        launch_vjp_t<EULER2D, 1>(c, U, lam, grad, masks + c->nfx, alpha, 0);
        launch_vjp_t<EULER2D, 0>(c, U, lam, grad, masks, alpha, 1);
        break;
    }
}

// The adjoint of one RK stage: G = J(U)^T m (the y part into Gy first for 2D), then the stage adjoint
// in the x kernel's epilogue (io.gy set here).
static void enqueue_stage_vjp(teno_ctx *c, const double *U, const uint32_t *masks, const double *alpha,
                              const double *m, double *Gy, StageIO io)
{
    switch (c->grid.sys) {
    case TENO_ADV1D: launch_vjp_t<ADV1D, 0>(c, U, m, nullptr, masks, alpha, 0, io); break;
    case TENO_BURGERS1D: launch_vjp_t<BURGERS1D, 0>(c, U, m, nullptr, masks, alpha, 0, io); break;
    case TENO_EULER1D: launch_vjp_t<EULER1D, 0>(c, U, m, nullptr, masks, alpha, 0, io); break;
    default:
        launch_vjp_t<EULER2D, 1>(c, U, m, Gy, masks + c->nfx, alpha, 0);
        io.gy = Gy;
        launch_vjp_t<EULER2D, 0>(c, U, m, nullptr, masks, alpha, 0, io);
        break;
    }
}

static bool adjoint_supported(const teno_ctx *c)
{
    if (c->grid.dtype != TENO_F64 || !c->opts.characteristic) return false;
    if (c->grid.bc_x == TENO_BC_PERIODIC && c->grid.nx < 8) return false;
    if (c->grid.sys == TENO_EULER2D && c->grid.bc_y == TENO_BC_PERIODIC && c->grid.ny < 8) return false;
    return true;
}

// Reverse-sweep scratch: with checkpoints (ckpt_every >= 1) the 3 * ckpt_every stage states of one
// segment and the running state X, then (both modes) the y part Gy, two buffers of mu and a second
// buffer of lam.
static size_t adj_scratch_states(int ckpt_every)
{
    return ckpt_every == TENO_CKPT_STAGES ? 4 : (size_t)3 * (size_t)ckpt_every + 5;
}

static teno_status ensure_adj_scratch(teno_ctx *c, int ckpt_every)
{
    size_t need = adj_scratch_states(ckpt_every) * c->nelem * sizeof(double);
    if (c->adj_scratch && c->adj_scratch_bytes >= need) return TENO_OK;
    if (c->adj_scratch) HIP_TRY(hipFree(c->adj_scratch));
    c->adj_scratch = nullptr;
    c->adj_scratch_bytes = 0;
    HIP_TRY(hipMalloc(&c->adj_scratch, need));
    c->adj_scratch_bytes = need;
    return TENO_OK;
}

// The adjoint of one recorded step whose three stage inputs start at s0 (stride ne): stage 2 (m = lam)
// starts the next lam buffer and mu in muA, stage 1 (m = muA) writes muB, stage 0 (m = muB) finishes
// lam. The running adjoint alternates between lamv[0] and lamv[1] (stage 2 reads it as its stencil
// input while writing the next one; stages 1 and 0 update it in place, reading only their own cells).
struct RevBufs {
    double *Gy, *muA, *muB;
    double *lamv[2];
    int cur;
};

static void enqueue_reverse_step(teno_ctx *c, const double *s0, const double *ad, const uint32_t *mj, RevBufs &b)
{
    const size_t ne = c->nelem, nf = c->nfx + c->nfy;
    double *lnew = b.lamv[b.cur ^ 1];
    for (int k = 2; k >= 0; --k) {
        StageIO io;
        io.rk = k;
        io.dt = ad + 24;
        io.lam_next = lnew;
        io.lam_step = lnew;
        io.mu_next = k == 2 ? b.muA : k == 1 ? b.muB : nullptr;
        const double *m = k == 2 ? b.lamv[b.cur] : k == 1 ? b.muA : b.muB;
        enqueue_stage_vjp(c, s0 + (size_t)k * ne, mj + (size_t)k * nf, ad + 8 * k, m, b.Gy, io);
    }
    b.cur ^= 1;
}

extern "C" {

teno_status teno_rhs_vjp(teno_ctx *c, const void *U, const uint32_t *masks, const double *alpha_dev, const void *lam,
                         void *grad)
{
    if (!c || !U || !masks || !alpha_dev || !lam || !grad || lam == grad) return TENO_E_ARG;
    if (!adjoint_supported(c)) return TENO_E_UNSUPPORTED;
    enqueue_rhs_vjp(c, (const double *)U, masks, alpha_dev, (const double *)lam, (double *)grad);
    return hipGetLastError() == hipSuccess ? TENO_OK : TENO_E_HIP;
}

teno_status teno_run_record(teno_ctx *c, void *U, int32_t nsteps, double dt_fixed, int32_t ckpt_every, void *ckpt_dev,
                            uint32_t *masks_dev, double *alpha_dt_dev)
{
    if (!c || !U || nsteps < 0 || !ckpt_dev || !alpha_dt_dev) return TENO_E_ARG;
    if (ckpt_every < 1 && ckpt_every != TENO_CKPT_STAGES) return TENO_E_ARG;
    teno_status st = teno_ensure_scratch(c);
    if (st) return st;
    const size_t nf = c->nfx + c->nfy;
    const size_t bytes = c->nelem * c->esize;
    teno_launch_clear(c, 0);
    teno_launch_wavespeed(c, U, 0);
    for (int n = 0; n < nsteps; ++n) {
        uint32_t *mrec = masks_dev ? masks_dev + (size_t)n * 3 * nf : nullptr;
        if (ckpt_every == TENO_CKPT_STAGES) {
            // the step's input, then its two intermediate stages written in place by the step
            char *s0 = (char *)ckpt_dev + (size_t)3 * n * bytes;
            HIP_TRY(hipMemcpyAsync(s0, U, bytes, hipMemcpyDeviceToDevice, c->stream));
            void *states[3] = {s0, s0 + bytes, s0 + 2 * bytes};
            teno_enqueue_step(c, U, dt_fixed, nullptr, alpha_dt_dev + (size_t)n * 25, mrec, nullptr, states);
            continue;
        }
        if (n % ckpt_every == 0)
            HIP_TRY(hipMemcpyAsync((char *)ckpt_dev + (size_t)(n / ckpt_every) * bytes, U, bytes,
                                   hipMemcpyDeviceToDevice, c->stream));
        teno_enqueue_step(c, U, dt_fixed, nullptr, alpha_dt_dev + (size_t)n * 25, mrec, nullptr, nullptr);
    }
    return hipGetLastError() == hipSuccess ? TENO_OK : TENO_E_HIP;
}

teno_status teno_run_replay(teno_ctx *c, void *U, int32_t nsteps, const uint32_t *masks_dev, const double *alpha_dt_dev)
{
    if (!c || !U || nsteps < 0 || !masks_dev || !alpha_dt_dev) return TENO_E_ARG;
    teno_status st = teno_ensure_scratch(c);
    if (st) return st;
    const size_t nf = c->nfx + c->nfy;
    for (int n = 0; n < nsteps; ++n)
        teno_enqueue_step(c, U, 0.0, alpha_dt_dev + (size_t)n * 25, nullptr, nullptr, masks_dev + (size_t)n * 3 * nf,
                          nullptr);
    return hipGetLastError() == hipSuccess ? TENO_OK : TENO_E_HIP;
}

teno_status teno_run_vjp(teno_ctx *c, const void *ckpt_dev, const uint32_t *masks_dev, const double *alpha_dt_dev,
                         int32_t nsteps, int32_t ckpt_every, void *lam_io)
{
    if (!c || !ckpt_dev || !masks_dev || !alpha_dt_dev || !lam_io || nsteps < 0) return TENO_E_ARG;
    if (ckpt_every < 1 && ckpt_every != TENO_CKPT_STAGES) return TENO_E_ARG;
    if (!adjoint_supported(c)) return TENO_E_UNSUPPORTED;
    teno_status st = teno_ensure_scratch(c);
    if (st) return st;
    st = ensure_adj_scratch(c, ckpt_every);
    if (st) return st;
    const size_t nf = c->nfx + c->nfy;
    const size_t ne = c->nelem, bytes = ne * sizeof(double);
    const bool stages = ckpt_every == TENO_CKPT_STAGES;
    double *seg = (double *)c->adj_scratch;                 // 3 * ckpt_every states (checkpoint mode)
    double *X = seg + (stages ? 0 : (size_t)3 * ckpt_every * ne);
    RevBufs b;
    b.Gy = stages ? seg : X + ne;
    b.muA = b.Gy + ne;
    b.muB = b.muA + ne;
    b.lamv[0] = (double *)lam_io;
    b.lamv[1] = b.muB + ne;
    b.cur = 0;
    if (stages) {
        // every stage input was stored by the recording run: nothing is recomputed
        for (int j = nsteps - 1; j >= 0; --j)
            enqueue_reverse_step(c, (const double *)ckpt_dev + (size_t)3 * j * ne, alpha_dt_dev + (size_t)j * 25,
                                 masks_dev + (size_t)j * 3 * nf, b);
    } else {
        const int nseg = (nsteps + ckpt_every - 1) / ckpt_every;
        for (int sgi = nseg - 1; sgi >= 0; --sgi) {
            const int j0 = sgi * ckpt_every;
            const int j1 = j0 + ckpt_every < nsteps ? j0 + ckpt_every : nsteps;
            HIP_TRY(hipMemcpyAsync(X, (const char *)ckpt_dev + (size_t)sgi * bytes, bytes, hipMemcpyDeviceToDevice,
                                   c->stream));
            // frozen replay of the segment, keeping every stage input
            for (int j = j0; j < j1; ++j) {
                double *s0 = seg + (size_t)3 * (j - j0) * ne;
                HIP_TRY(hipMemcpyAsync(s0, X, bytes, hipMemcpyDeviceToDevice, c->stream));
                void *states[3] = {s0, s0 + ne, s0 + 2 * ne};
                teno_enqueue_step(c, X, 0.0, alpha_dt_dev + (size_t)j * 25, nullptr, nullptr,
                                  masks_dev + (size_t)j * 3 * nf, states);
            }
            for (int j = j1 - 1; j >= j0; --j)
                enqueue_reverse_step(c, seg + (size_t)3 * (j - j0) * ne, alpha_dt_dev + (size_t)j * 25,
                                     masks_dev + (size_t)j * 3 * nf, b);
        }
    }
    if (b.cur != 0)
        HIP_TRY(hipMemcpyAsync(lam_io, b.lamv[1], bytes, hipMemcpyDeviceToDevice, c->stream));
    return hipGetLastError() == hipSuccess ? TENO_OK : TENO_E_HIP;
}

}  // extern "C"
