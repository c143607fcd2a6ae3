// teno_lib.hip -- host side of the C ABI declared in include/teno.h (gfx950).
//
// A context owns: the grid and options, the caller's stream, a device control block (spread
// wave-speed maxima, the current Lax-Friedrichs constants and dt, the sticky error word) and three
// state-sized scratch buffers for the SSP-RK3 stages. All launches are asynchronous on the stream;
// no step needs a host round trip (dt is computed and consumed on the device), so a whole step
// can be captured into a HIP graph and replayed.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <mutex>
#include <new>
#include <vector>

#include "teno.h"
#include "teno_device.hpp"
#include "teno_internal.hpp"

using namespace teno;

// ------------------------------------------------------------------------------------------------
// helpers
// ------------------------------------------------------------------------------------------------
#define HIP_TRY(expr)                                   \
    do {                                                \
        hipError_t e_ = (expr);                         \
        if (e_ != hipSuccess) return TENO_E_HIP;        \
    } while (0)

static int nvar_of(int sys) { return sys == TENO_EULER1D ? 3 : sys == TENO_EULER2D ? 4 : 1; }

static teno_status err_to_status(unsigned e)
{
    if (e & ERR_NONFINITE) return TENO_E_NONFINITE;
    if (e & ERR_NONPHYSICAL) return TENO_E_NONPHYSICAL;
    if (e & ERR_SELECTION) return TENO_E_NONFINITE;
    return TENO_OK;
}

bool teno_validate(const teno_grid *g, const teno_opts *o)
{
    if (!g || !o) return false;
    if (g->sys < 0 || g->sys > 3) return false;
    if (g->nx < 1 || g->ny < 1 || g->nx > (1 << 20) || g->ny > (1 << 20)) return false;
    if (g->sys != TENO_EULER2D && g->ny != 1) return false;
    if ((double)nvar_of(g->sys) * g->nx * g->ny >= 2147483647.0) return false;
    if (g->bc_x < 0 || g->bc_x > 1 || g->bc_y < 0 || g->bc_y > 1) return false;
    if (g->dtype != TENO_F64 && g->dtype != TENO_F32) return false;
    if (!(g->x1 > g->x0) || !(g->y1 > g->y0)) return false;
    return teno_validate_opts(o);
}

bool teno_validate_opts(const teno_opts *o)
{
    if (!o) return false;
    if (o->scheme < 0 || o->scheme > 1 || o->alpha_mode < 0 || o->alpha_mode > 1) return false;
    if (o->eps_mode < 0 || o->eps_mode > 1) return false;
    if (!(o->gamma > 1.0) || !(o->ct > 0.0 && o->ct < 1.0 / 3.0) || !(o->cfl > 0.0)) return false;
    if (o->eps_mode == 1 && !(o->eps > 0.0)) return false;
    if (o->q < 1 || o->q > 12 || !(o->C > 0.0) || !std::isfinite(o->C)) return false;
    if (o->characteristic < 0 || o->characteristic > 1) return false;
    return true;
}

void teno_fill_derived(teno_ctx *c)
{
    const teno_grid &g = c->grid;
    c->nv = nvar_of(g.sys);
    c->dx = (g.x1 - g.x0) / g.nx;
    c->dy = (g.y1 - g.y0) / g.ny;
    if (c->opts.eps_mode == 1) {
        c->eps_x = c->eps_y = c->opts.eps;
    } else if (c->opts.scheme == TENO_SCHEME_TENO5) {
        c->eps_x = c->eps_y = 1e-40;
    } else {
        c->eps_x = c->dx * c->dx * c->dx;
        c->eps_y = c->dy * c->dy * c->dy;
    }
    c->ncell = (size_t)g.nx * g.ny;
    c->nelem = (size_t)c->nv * c->ncell;
    c->nfx = (size_t)g.ny * (g.nx + 1);
    c->nfy = g.sys == TENO_EULER2D ? (size_t)(g.ny + 1) * g.nx : 0;
    c->esize = g.dtype == TENO_F64 ? 8 : 4;
}

// ------------------------------------------------------------------------------------------------
// Fixed scratch of teno_step_noalloc: the control block, then the stage states. Each device holds its
// own copy; host code reaches it only through the device address hipGetSymbolAddress returns for
// that device (the array's name is a host-side stand-in).
// ------------------------------------------------------------------------------------------------
static __device__ __align__(256) unsigned char scratch[TENO_NOALLOC_SCRATCH_BYTES];

constexpr int NOALLOC_MAX_DEVICES = 64;
static std::mutex noalloc_mutex;
static void *noalloc_ptr[NOALLOC_MAX_DEVICES];

// Device address of this device's scratch (looked up once per device, with that device current).
static teno_status noalloc_scratch(void **out)
{
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= NOALLOC_MAX_DEVICES) return TENO_E_HIP;
    std::lock_guard<std::mutex> lock(noalloc_mutex);
    if (!noalloc_ptr[dev]) {
        void *p = nullptr;
        if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) != hipSuccess || !p) {
            (void)hipGetLastError();
            return TENO_E_HIP;
        }
        noalloc_ptr[dev] = p;
    }
    *out = noalloc_ptr[dev];
    return TENO_OK;
}

// Zero a control block with a kernel (stream-ordered, and a plain kernel node under graph capture).
static __global__ void zero_ctrl_kernel(Ctrl *ctrl)
{
    unsigned *w = (unsigned *)ctrl;
    for (size_t q = threadIdx.x; q < sizeof(Ctrl) / sizeof(unsigned); q += blockDim.x) w[q] = 0u;
}

// The step's outcome for the caller: status as teno_poll reports it, and dt.
static __global__ void noalloc_report_kernel(const Ctrl *ctrl, int32_t *status_dev, double *dt_dev)
{
    if (threadIdx.x == 0) {
        const unsigned e = ctrl->err;
        if (status_dev)
            *status_dev = (e & ERR_NONFINITE) ? TENO_E_NONFINITE
                        : (e & ERR_NONPHYSICAL) ? TENO_E_NONPHYSICAL
                        : (e & ERR_SELECTION) ? TENO_E_NONFINITE : TENO_OK;
        if (dt_dev) *dt_dev = ctrl->dt;
    }
}

// ------------------------------------------------------------------------------------------------
// launch helpers
// ------------------------------------------------------------------------------------------------

// Event pair for the next instrumented launch of a kernel kind (null when timing is off or the
// stream is being captured).
static std::pair<hipEvent_t, hipEvent_t> *teno_timing_slot(teno_ctx *c, int kind)
{
    if (!c->timing) return nullptr;
    hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
    if (hipStreamIsCapturing(c->stream, &cs) != hipSuccess || cs != hipStreamCaptureStatusNone) return nullptr;
    if (c->events_used == c->events.size()) {
        hipEvent_t a, b;
        if (hipEventCreate(&a) != hipSuccess) return nullptr;
        if (hipEventCreate(&b) != hipSuccess) { (void)hipEventDestroy(a); return nullptr; }
        c->events.push_back({kind, {a, b}});
    }
    auto &slot = c->events[c->events_used++];
    slot.first = kind;
    return &slot.second;
}

template <typename T, int SYS, int DIR, bool FROZEN>
static void launch_sweep_t(teno_ctx *c, const SweepReq &r)
{
    SweepArgs<T> a;
    std::memset(&a, 0, sizeof a);
    a.U = (const T *)r.U;
    a.U0 = (const T *)r.U0;
    a.addend = (const T *)r.addend;
    a.out = (T *)r.out;
    a.Fout = (T *)r.Fout;
    a.chi_out = (T *)r.chi_out;
    a.masks_out = r.masks_out;
    a.flags_out = r.flags_out;
    a.masks_in = r.masks_in;
    a.alpha = r.alpha ? r.alpha : c->ctrl_d->alpha;
    a.dt = &c->ctrl_d->dt;
    a.part = r.part;
    a.err = &c->ctrl_d->err;
    a.nx = c->grid.nx;
    a.ny = c->grid.ny;
    a.len = DIR == 0 ? c->grid.nx : c->grid.ny;
    a.nlines = DIR == 0 ? c->grid.ny : c->grid.nx;
    a.nseg = (a.len + SEG_CELLS - 1) / SEG_CELLS;
    a.bc = DIR == 0 ? c->grid.bc_x : c->grid.bc_y;
    a.mode = r.mode;
    a.stage = r.stage;
    a.scheme = c->opts.scheme;
    a.alpha_mode = teno_alpha_mode(c->opts);
    a.C = (T)c->opts.C;
    a.q = c->opts.q;
    a.characteristic = c->opts.characteristic;
    a.inv_h = (T)(1.0 / (DIR == 0 ? c->dx : c->dy));
    const double eps = DIR == 0 ? c->eps_x : c->eps_y, sk = smooth_shortcut_k(c->opts.ct, c->opts.C, c->opts.q);
    a.ct = (T)c->opts.ct;
    a.eps4 = (T)(4.0 * eps);
    a.smooth_k = (T)sk;
    a.keps4 = (T)(sk * (4.0 * eps));
    a.gamma = (T)c->opts.gamma;
    a.gm1 = (T)(c->opts.gamma - 1.0);
    a.adv = (T)c->opts.adv_speed;
    a.inv_dx = (T)(1.0 / c->dx);
    a.inv_dy = (T)(1.0 / c->dy);
    size_t ntiles;
    if (DIR == 0) {
        size_t nseg_total = (size_t)a.nseg * a.nlines;
        ntiles = (nseg_total + NSEG_X - 1) / NSEG_X;
    } else {
        ntiles = (size_t)((a.nlines + NSEG_Y - 1) / NSEG_Y) * a.nseg;
    }
    a.ntiles = (int)ntiles;
    std::pair<hipEvent_t, hipEvent_t> *ev = teno_timing_slot(c, DIR);
    if (ev) (void)hipEventRecord(ev->first, c->stream);
    const dim3 grid((unsigned)ntiles);
    // measured selections that nobody records take the variant without mask output
    const bool rec = FROZEN || a.masks_out || a.flags_out;
    if (r.mode == MODE_RHS && rec)
        hipLaunchKernelGGL((sweep_kernel<T, SYS, DIR, FROZEN, MODE_RHS>), grid, dim3(BLOCK), 0, c->stream, a);
    else if (r.mode == MODE_RHS)
        hipLaunchKernelGGL((sweep_kernel<T, SYS, DIR, false, MODE_RHS, false>), grid, dim3(BLOCK), 0, c->stream, a);
    else if (DIR == 0 && r.mode == MODE_STAGE && rec)
        hipLaunchKernelGGL((sweep_kernel<T, SYS, 0, FROZEN, MODE_STAGE>), grid, dim3(BLOCK), 0, c->stream, a);
    else if (DIR == 0 && r.mode == MODE_STAGE)
        hipLaunchKernelGGL((sweep_kernel<T, SYS, 0, false, MODE_STAGE, false>), grid, dim3(BLOCK), 0, c->stream, a);
    else
        hipLaunchKernelGGL((sweep_kernel<T, SYS, DIR, FROZEN, MODE_FACES>), grid, dim3(BLOCK), 0, c->stream, a);
    if (ev) (void)hipEventRecord(ev->second, c->stream);
}

template <typename T>
static void launch_sweep_sys(teno_ctx *c, const SweepReq &r)
{
    switch (c->grid.sys) {
    case TENO_ADV1D:
        r.frozen ? launch_sweep_t<T, ADV1D, 0, true>(c, r) : launch_sweep_t<T, ADV1D, 0, false>(c, r);
        break;
    case TENO_BURGERS1D:
        r.frozen ? launch_sweep_t<T, BURGERS1D, 0, true>(c, r) : launch_sweep_t<T, BURGERS1D, 0, false>(c, r);
        break;
    case TENO_EULER1D:
        r.frozen ? launch_sweep_t<T, EULER1D, 0, true>(c, r) : launch_sweep_t<T, EULER1D, 0, false>(c, r);
        break;
    default:
        if (r.dir == 0)
            r.frozen ? launch_sweep_t<T, EULER2D, 0, true>(c, r) : launch_sweep_t<T, EULER2D, 0, false>(c, r);
        else
            r.frozen ? launch_sweep_t<T, EULER2D, 1, true>(c, r) : launch_sweep_t<T, EULER2D, 1, false>(c, r);
        break;
    }
}

void teno_launch_sweep(teno_ctx *c, const SweepReq &r)
{
    if (c->grid.dtype == TENO_F64) launch_sweep_sys<double>(c, r);
    else launch_sweep_sys<float>(c, r);
}

template <typename T>
static void launch_wavespeed_t(teno_ctx *c, const void *U, int ring)
{
    size_t nb = (c->ncell + BLOCK - 1) / BLOCK;
    unsigned grid = (unsigned)(nb < 1024 ? (nb ? nb : 1) : 1024);
    unsigned long long *part = &c->ctrl_d->part[ring][0][0];
    const T g = (T)c->opts.gamma, adv = (T)c->opts.adv_speed, ix = (T)(1.0 / c->dx), iy = (T)(1.0 / c->dy);
    const T *u = (const T *)U;
    switch (c->grid.sys) {
    case TENO_ADV1D:
        hipLaunchKernelGGL((wavespeed_kernel<T, ADV1D>), dim3(grid), dim3(BLOCK), 0, c->stream, u, c->ncell, g, adv,
                           ix, iy, teno_alpha_mode(c->opts), part, &c->ctrl_d->err);
        break;
    case TENO_BURGERS1D:
        hipLaunchKernelGGL((wavespeed_kernel<T, BURGERS1D>), dim3(grid), dim3(BLOCK), 0, c->stream, u, c->ncell, g,
                           adv, ix, iy, teno_alpha_mode(c->opts), part, &c->ctrl_d->err);
        break;
    case TENO_EULER1D:
        hipLaunchKernelGGL((wavespeed_kernel<T, EULER1D>), dim3(grid), dim3(BLOCK), 0, c->stream, u, c->ncell, g,
                           adv, ix, iy, teno_alpha_mode(c->opts), part, &c->ctrl_d->err);
        break;
    default:
        hipLaunchKernelGGL((wavespeed_kernel<T, EULER2D>), dim3(grid), dim3(BLOCK), 0, c->stream, u, c->ncell, g,
                           adv, ix, iy, teno_alpha_mode(c->opts), part, &c->ctrl_d->err);
        break;
    }
}

void teno_launch_wavespeed(teno_ctx *c, const void *U, int ring)
{
    if (c->grid.dtype == TENO_F64) launch_wavespeed_t<double>(c, U, ring);
    else launch_wavespeed_t<float>(c, U, ring);
}

void teno_launch_prep(teno_ctx *c, int ring, int stage, double dt_fixed, const double *frozen, double *record)
{
    hipLaunchKernelGGL(prep_kernel, dim3(1), dim3(64), 0, c->stream, c->ctrl_d, ring, stage, dt_fixed, c->opts.cfl,
                       frozen, record);
}

void teno_launch_clear(teno_ctx *c, int ring)
{
    hipLaunchKernelGGL(clear_ring_kernel, dim3(1), dim3(256), 0, c->stream, c->ctrl_d, ring);
}

// Constants of the operator at U (ring 3 is reserved for stand-alone evaluations).
static void alpha_of(teno_ctx *c, const void *U)
{
    teno_launch_clear(c, 3);
    teno_launch_wavespeed(c, U, 3);
    teno_launch_prep(c, 3, -1, 0.0, nullptr, nullptr);
}

// The operator with the selection measured (masks_in == null) or frozen, into dUdt.
static void rhs_core(teno_ctx *c, const void *U, void *dUdt, uint32_t *masks_out, const uint32_t *masks_in,
                     const double *alpha)
{
    const bool two_d = c->grid.sys == TENO_EULER2D;
    SweepReq r;
    std::memset(&r, 0, sizeof r);
    r.mode = MODE_RHS;
    r.frozen = masks_in != nullptr;
    r.U = U;
    r.alpha = alpha;
    if (two_d) {
        r.dir = 1;
        r.out = dUdt;
        r.masks_out = masks_out ? masks_out + c->nfx : nullptr;
        r.masks_in = masks_in ? masks_in + c->nfx : nullptr;
        teno_launch_sweep(c, r);
    }
    r.dir = 0;
    r.out = dUdt;
    r.addend = two_d ? dUdt : nullptr;
    r.masks_out = masks_out;
    r.masks_in = masks_in;
    teno_launch_sweep(c, r);
}

// One SSP-RK3 step: stage k reads ring k (constants of its input) and accumulates the maxima of
// its output into ring (k+1) % 3. The caller has filled ring 0 for U.
// frozen_ad / record_ad: per-step alpha/dt replay or recording buffers (25 doubles).
// masks_rec: per-step 3*nfaces mask words to record; masks_in: per-step frozen masks.
void teno_enqueue_step(teno_ctx *c, void *U, double dt_fixed, const double *frozen_ad, double *record_ad,
                       uint32_t *masks_rec, const uint32_t *masks_in, void **stage_states)
{
    const bool two_d = c->grid.sys == TENO_EULER2D;
    const size_t nf = c->nfx + c->nfy;
    void *in[3] = {U, c->S1, c->S2};
    void *outp[3] = {c->S1, c->S2, U};
    if (stage_states) {
        in[1] = stage_states[1];
        in[2] = stage_states[2];
        outp[0] = stage_states[1];
        outp[1] = stage_states[2];
    }
    for (int k = 0; k < 3; ++k) {
        teno_launch_prep(c, k, k, dt_fixed, frozen_ad, record_ad);
        SweepReq r;
        std::memset(&r, 0, sizeof r);
        r.stage = k;
        r.frozen = masks_in != nullptr;
        r.U = in[k];
        uint32_t *mrec = masks_rec ? masks_rec + (size_t)k * nf : nullptr;
        const uint32_t *min_ = masks_in ? masks_in + (size_t)k * nf : nullptr;
        if (two_d) {
            r.dir = 1;
            r.mode = MODE_RHS;
            r.out = c->dUy;
            r.masks_out = mrec ? mrec + c->nfx : nullptr;
            r.masks_in = min_ ? min_ + c->nfx : nullptr;
            teno_launch_sweep(c, r);
        }
        r.dir = 0;
        r.mode = MODE_STAGE;
        r.U0 = U;
        r.addend = two_d ? c->dUy : nullptr;
        r.out = outp[k];
        r.masks_out = mrec;
        r.masks_in = min_;
        r.part = &c->ctrl_d->part[(k + 1) % 3][0][0];
        teno_launch_sweep(c, r);
    }
}

teno_status teno_ensure_scratch(teno_ctx *c)
{
    if (c->S1) return TENO_OK;
    const size_t bytes = c->nelem * c->esize;
    void *s1 = nullptr, *s2 = nullptr, *dy = nullptr;
    bool ok = hipMalloc(&s1, bytes) == hipSuccess && hipMalloc(&s2, bytes) == hipSuccess &&
              (c->grid.sys != TENO_EULER2D || hipMalloc(&dy, bytes) == hipSuccess);
    if (!ok) {
        // all or nothing: a later call must not find a partial set
        (void)hipFree(s1);
        (void)hipFree(s2);
        (void)hipFree(dy);
        (void)hipGetLastError();
        return TENO_E_HIP;
    }
    c->S1 = s1;
    c->S2 = s2;
    c->dUy = dy;
    return TENO_OK;
}

// ------------------------------------------------------------------------------------------------
// C ABI
// ------------------------------------------------------------------------------------------------
extern "C" {

void teno_default_opts(teno_opts *o)
{
    if (!o) return;
    std::memset(o, 0, sizeof *o);
    o->scheme = TENO_SCHEME_TENO7X;
    o->alpha_mode = 0;
    o->eps_mode = 0;
    o->gamma = 1.4;
    o->ct = 1e-5;
    o->eps = 0.0;
    o->cfl = 0.5;
    o->adv_speed = 1.0;
    o->C = 1.0;
    o->q = 6;
    o->characteristic = 1;
    o->reserved = 0;
}

const char *teno_status_str(teno_status s)
{
    switch (s) {
    case TENO_OK: return "ok";
    case TENO_E_ARG: return "invalid argument";
    case TENO_E_UNSUPPORTED: return "unsupported";
    case TENO_E_HIP: return "HIP runtime error";
    case TENO_E_NONFINITE: return "non-finite value";
    case TENO_E_NONPHYSICAL: return "non-physical state";
    case TENO_E_STATE: return "invalid context state";
    case TENO_E_CAPACITY: return "problem exceeds the fixed scratch of the no-allocation entry point";
    }
    return "unknown status";
}

teno_status teno_create(const teno_grid *grid, const teno_opts *opts, void *stream, teno_ctx **out)
{
    if (!out) return TENO_E_ARG;
    *out = nullptr;
    if (!teno_validate(grid, opts)) return TENO_E_ARG;
    teno_ctx *c = new (std::nothrow) teno_ctx();
    if (!c) return TENO_E_HIP;
    c->grid = *grid;
    c->opts = *opts;
    c->stream = (hipStream_t)stream;
    teno_fill_derived(c);
    {
        int dev = 0, cu = 0;
        if (hipGetDevice(&dev) == hipSuccess &&
            hipDeviceGetAttribute(&cu, hipDeviceAttributeMultiprocessorCount, dev) == hipSuccess && cu > 0)
            c->num_cu = cu;
    }
    if (hipMalloc(&c->ctrl_d, sizeof(Ctrl)) != hipSuccess) {
        delete c;
        return TENO_E_HIP;
    }
    if (hipMemsetAsync(c->ctrl_d, 0, sizeof(Ctrl), c->stream) != hipSuccess ||
        hipStreamSynchronize(c->stream) != hipSuccess) {
        hipFree(c->ctrl_d);
        delete c;
        return TENO_E_HIP;
    }
    *out = c;
    return TENO_OK;
}

teno_status teno_destroy(teno_ctx *c)
{
    if (!c) return TENO_E_ARG;
    hipStreamSynchronize(c->stream);
    if (c->graph_exec) hipGraphExecDestroy(c->graph_exec);
    if (c->graph) hipGraphDestroy(c->graph);
    hipFree(c->S1);
    hipFree(c->S2);
    hipFree(c->dUy);
    hipFree(c->adj_scratch);
    hipFree(c->ctrl_d);
    if (c->cap_stream) hipStreamDestroy(c->cap_stream);
    for (auto &e : c->events) {
        (void)hipEventDestroy(e.second.first);
        (void)hipEventDestroy(e.second.second);
    }
    delete c;
    return TENO_OK;
}

size_t teno_workspace_bytes(const teno_grid *grid, const teno_opts *opts, int32_t ckpt_every)
{
    if (!teno_validate(grid, opts) || (ckpt_every < 0 && ckpt_every != TENO_CKPT_STAGES)) return 0;
    teno_ctx c;
    c.grid = *grid;
    c.opts = *opts;
    teno_fill_derived(&c);
    const size_t state = c.nelem * c.esize;
    size_t bytes = sizeof(Ctrl) + 2 * state + (grid->sys == TENO_EULER2D ? state : 0);
    if (ckpt_every > 0) bytes += ((size_t)3 * (size_t)ckpt_every + 5) * c.nelem * sizeof(double);
    if (ckpt_every == TENO_CKPT_STAGES) bytes += (size_t)4 * c.nelem * sizeof(double);
    return bytes;
}

size_t teno_state_elems(const teno_ctx *c) { return c ? c->nelem : 0; }
size_t teno_nfaces(const teno_ctx *c) { return c ? c->nfx + c->nfy : 0; }

teno_status teno_set_stream(teno_ctx *c, void *stream)
{
    if (!c) return TENO_E_ARG;
    if (c->graph_exec) {
        hipGraphExecDestroy(c->graph_exec);
        c->graph_exec = nullptr;
    }
    if (c->graph) {
        hipGraphDestroy(c->graph);
        c->graph = nullptr;
    }
    c->stream = (hipStream_t)stream;
    return TENO_OK;
}

teno_status teno_rhs(teno_ctx *c, const void *U, void *dUdt, uint32_t *masks_out)
{
    if (!c || !U || !dUdt || U == dUdt) return TENO_E_ARG;
    alpha_of(c, U);
    rhs_core(c, U, dUdt, masks_out, nullptr, nullptr);
    return hipGetLastError() == hipSuccess ? TENO_OK : TENO_E_HIP;
}

teno_status teno_rhs_frozen(teno_ctx *c, const void *U, const uint32_t *masks, const double *alpha_dev, void *dUdt)
{
    if (!c || !U || !dUdt || !masks || !alpha_dev || U == dUdt) return TENO_E_ARG;
    rhs_core(c, U, dUdt, nullptr, masks, alpha_dev);
    return hipGetLastError() == hipSuccess ? TENO_OK : TENO_E_HIP;
}

teno_status teno_face_fluxes(teno_ctx *c, const void *U, void *Fx, void *Fy, uint32_t *masks, uint32_t *flags,
                             void *chi, double *alpha_dev)
{
    if (!c || !U || !Fx) return TENO_E_ARG;
    const bool two_d = c->grid.sys == TENO_EULER2D;
    if (two_d && !Fy) return TENO_E_ARG;
    alpha_of(c, U);
    SweepReq r;
    std::memset(&r, 0, sizeof r);
    r.mode = MODE_FACES;
    r.U = U;
    r.dir = 0;
    r.Fout = Fx;
    r.chi_out = chi;
    r.masks_out = masks;
    r.flags_out = flags;
    teno_launch_sweep(c, r);
    if (two_d) {
        r.dir = 1;
        r.Fout = Fy;
        r.chi_out = chi ? (char *)chi + c->nfx * 24 * c->esize : nullptr;
        r.masks_out = masks ? masks + c->nfx : nullptr;
        r.flags_out = flags ? flags + c->nfx : nullptr;
        teno_launch_sweep(c, r);
    }
    if (alpha_dev) hipLaunchKernelGGL(copy_alpha_kernel, dim3(1), dim3(64), 0, c->stream, c->ctrl_d, alpha_dev);
    return hipGetLastError() == hipSuccess ? TENO_OK : TENO_E_HIP;
}

teno_status teno_step(teno_ctx *c, void *U, double dt_fixed)
{
    if (!c || !U) return TENO_E_ARG;
    teno_status st = teno_ensure_scratch(c);
    if (st) return st;
    teno_launch_clear(c, 0);
    teno_launch_wavespeed(c, U, 0);
    teno_enqueue_step(c, U, dt_fixed, nullptr, nullptr, nullptr, nullptr, nullptr);
    return hipGetLastError() == hipSuccess ? TENO_OK : TENO_E_HIP;
}

// Make sure the one-step graph for (U, dt_fixed) exists.
static teno_status ensure_step_graph(teno_ctx *c, void *U, double dt_fixed)
{
    if (!c->graph_exec || c->graph_U != U || c->graph_dt != dt_fixed) {
        if (c->graph_exec) hipGraphExecDestroy(c->graph_exec);
        if (c->graph) hipGraphDestroy(c->graph);
        c->graph_exec = nullptr;
        c->graph = nullptr;
        // capture on the context's private stream (the legacy null stream cannot be captured);
        // the graph is then launched on the caller's stream
        if (!c->cap_stream) HIP_TRY(hipStreamCreateWithFlags(&c->cap_stream, hipStreamNonBlocking));
        hipStream_t user = c->stream;
        c->stream = c->cap_stream;
        hipError_t e1 = hipStreamBeginCapture(c->stream, hipStreamCaptureModeThreadLocal);
        if (e1 == hipSuccess) {
            teno_enqueue_step(c, U, dt_fixed, nullptr, nullptr, nullptr, nullptr, nullptr);
            e1 = hipStreamEndCapture(c->stream, &c->graph);
        }
        c->stream = user;
        HIP_TRY(e1);
        HIP_TRY(hipGraphInstantiate(&c->graph_exec, c->graph, nullptr, nullptr, 0));
        c->graph_U = U;
        c->graph_dt = dt_fixed;
    }
    return TENO_OK;
}

// Synchronise, read the error word and the failing step; clear both on a failure.
static teno_status read_failure(teno_ctx *c, unsigned *err_at)
{
    HIP_TRY(hipStreamSynchronize(c->stream));
    unsigned w[2] = {0, 0};
    HIP_TRY(hipMemcpy(&w[0], &c->ctrl_d->err, sizeof(unsigned), hipMemcpyDeviceToHost));
    HIP_TRY(hipMemcpy(&w[1], &c->ctrl_d->err_at, sizeof(unsigned), hipMemcpyDeviceToHost));
    unsigned steps = 0;
    HIP_TRY(hipMemcpy(&steps, &c->ctrl_d->steps, sizeof(unsigned), hipMemcpyDeviceToHost));
    if (w[0]) {
        // raised by the last stage of the last step and not yet seen by a stage preparation
        *err_at = w[1] ? w[1] : (steps ? steps : 1u);
        const unsigned z[2] = {0, 0};
        HIP_TRY(hipMemcpy(&c->ctrl_d->err, &z[0], sizeof(unsigned), hipMemcpyHostToDevice));
        HIP_TRY(hipMemcpy(&c->ctrl_d->err_at, &z[1], sizeof(unsigned), hipMemcpyHostToDevice));
    }
    return err_to_status(w[0]);
}

teno_status teno_step_noalloc(const teno_grid *grid, const teno_opts *opts, void *U, double dt_fixed, void *stream,
                              int32_t *status_dev, double *dt_dev)
{
    if (!U || !teno_validate(grid, opts)) return TENO_E_ARG;
    teno_ctx c;                                  // host-side description only: no allocation
    c.grid = *grid;
    c.opts = *opts;
    c.stream = (hipStream_t)stream;
    teno_fill_derived(&c);
    const size_t ctrl_bytes = (sizeof(Ctrl) + 255) / 256 * 256;
    const size_t state = (c.nelem * c.esize + 255) / 256 * 256;
    const int nstates = grid->sys == TENO_EULER2D ? 3 : 2;
    if (ctrl_bytes + nstates * state > (size_t)TENO_NOALLOC_SCRATCH_BYTES) return TENO_E_CAPACITY;
    void *base = nullptr;
    teno_status st = noalloc_scratch(&base);
    if (st) return st;
    char *p = (char *)base;
    c.ctrl_d = (Ctrl *)p;
    c.S1 = p + ctrl_bytes;
    c.S2 = p + ctrl_bytes + state;
    c.dUy = grid->sys == TENO_EULER2D ? p + ctrl_bytes + 2 * state : nullptr;
    // the previous call's contents: every ring slot, the constants, dt and the error word start at zero
    hipLaunchKernelGGL(zero_ctrl_kernel, dim3(1), dim3(256), 0, c.stream, c.ctrl_d);
    teno_launch_wavespeed(&c, U, 0);
    teno_enqueue_step(&c, U, dt_fixed, nullptr, nullptr, nullptr, nullptr, nullptr);
    if (status_dev || dt_dev)
        hipLaunchKernelGGL(noalloc_report_kernel, dim3(1), dim3(64), 0, c.stream, c.ctrl_d, status_dev, dt_dev);
    c.S1 = c.S2 = c.dUy = nullptr;               // not the context's to free
    c.ctrl_d = nullptr;
    return hipGetLastError() == hipSuccess ? TENO_OK : TENO_E_HIP;
}

teno_status teno_run(teno_ctx *c, void *U, int32_t nsteps, double dt_fixed, int32_t use_graph, int32_t check_every,
                     int32_t *steps_done_host)
{
    if (!c || !U || nsteps < 0) return TENO_E_ARG;
    if (steps_done_host) *steps_done_host = 0;
    teno_status st = teno_ensure_scratch(c);
    if (st) return st;
    if (use_graph) {
        st = ensure_step_graph(c, U, dt_fixed);
        if (st) return st;
    }
    if (check_every > 0) hipLaunchKernelGGL(reset_counters_kernel, dim3(1), dim3(64), 0, c->stream, c->ctrl_d);
    teno_launch_clear(c, 0);
    teno_launch_wavespeed(c, U, 0);
    const int chunk = check_every > 0 ? check_every : (nsteps > 0 ? nsteps : 1);
    for (int n0 = 0; n0 < nsteps; n0 += chunk) {
        const int n1 = n0 + chunk < nsteps ? n0 + chunk : nsteps;
        for (int n = n0; n < n1; ++n) {
            if (use_graph) HIP_TRY(hipGraphLaunch(c->graph_exec, c->stream));
            else teno_enqueue_step(c, U, dt_fixed, nullptr, nullptr, nullptr, nullptr, nullptr);
        }
        if (hipGetLastError() != hipSuccess) return TENO_E_HIP;
        if (check_every > 0) {
            unsigned at = 0;
            st = read_failure(c, &at);
            if (st) {
                if (steps_done_host) *steps_done_host = (int32_t)at - 1;
                return st;
            }
        }
    }
    if (steps_done_host) *steps_done_host = nsteps;
    return TENO_OK;
}

teno_status teno_poll(teno_ctx *c)
{
    if (!c) return TENO_E_ARG;
    HIP_TRY(hipStreamSynchronize(c->stream));
    unsigned e = 0;
    HIP_TRY(hipMemcpy(&e, &c->ctrl_d->err, sizeof e, hipMemcpyDeviceToHost));
    if (e) {
        unsigned z = 0;
        HIP_TRY(hipMemcpy(&c->ctrl_d->err, &z, sizeof z, hipMemcpyHostToDevice));
        HIP_TRY(hipMemcpy(&c->ctrl_d->err_at, &z, sizeof z, hipMemcpyHostToDevice));
    }
    return err_to_status(e);
}

teno_status teno_set_timing(teno_ctx *c, int32_t enable)
{
    if (!c) return TENO_E_ARG;
    c->timing = enable != 0;
    c->events_used = 0;
    return TENO_OK;
}

teno_status teno_read_timing(teno_ctx *c, double *ms, int32_t *count)
{
    if (!c || !ms || !count) return TENO_E_ARG;
    HIP_TRY(hipStreamSynchronize(c->stream));
    ms[0] = ms[1] = 0.0;
    count[0] = count[1] = 0;
    for (size_t q = 0; q < c->events_used; ++q) {
        float t = 0.f;
        HIP_TRY(hipEventElapsedTime(&t, c->events[q].second.first, c->events[q].second.second));
        int k = c->events[q].first;
        ms[k] += t;
        count[k] += 1;
    }
    return TENO_OK;
}

teno_status teno_last_alpha(teno_ctx *c, double *alpha_dev)
{
    if (!c || !alpha_dev) return TENO_E_ARG;
    hipLaunchKernelGGL(copy_alpha_kernel, dim3(1), dim3(64), 0, c->stream, c->ctrl_d, alpha_dev);
    return hipGetLastError() == hipSuccess ? TENO_OK : TENO_E_HIP;
}

teno_status teno_last_dt(teno_ctx *c, double *dt_host)
{
    if (!c || !dt_host) return TENO_E_ARG;
    HIP_TRY(hipStreamSynchronize(c->stream));
    HIP_TRY(hipMemcpy(dt_host, &c->ctrl_d->dt, sizeof(double), hipMemcpyDeviceToHost));
    return TENO_OK;
}

teno_status teno_set_time(teno_ctx *c, double t0, double t_end)
{
    if (!c || !std::isfinite(t0) || std::isnan(t_end)) return TENO_E_ARG;
    const unsigned on = t_end > t0 ? 1u : 0u;
    hipLaunchKernelGGL(set_time_kernel, dim3(1), dim3(64), 0, c->stream, c->ctrl_d, t0, on ? t_end : 0.0, on);
    return hipGetLastError() == hipSuccess ? TENO_OK : TENO_E_HIP;
}

teno_status teno_get_time(teno_ctx *c, double *t_host)
{
    if (!c || !t_host) return TENO_E_ARG;
    HIP_TRY(hipStreamSynchronize(c->stream));
    HIP_TRY(hipMemcpy(t_host, &c->ctrl_d->t, sizeof(double), hipMemcpyDeviceToHost));
    return TENO_OK;
}

}  // extern "C"
