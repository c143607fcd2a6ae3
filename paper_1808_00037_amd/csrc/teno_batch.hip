// teno_batch.hip -- many independent Euler problems (1D and 2D, uneven sizes) advanced together.
//
// All instances live in one packed state buffer (and packed RK-stage scratch). Each sweep of a
// stage is one launch per system over a static work list of (instance, tile) items, one item per
// block, with the single-problem kernels' tile code and register budget; the list is instance-major
// and blocks are renumbered per XCD, so blocks running together on one XCD share an instance's rows
// in L2. Every instance keeps its own Lax-Friedrichs constants, CFL dt and spread wave-speed
// maxima. The short ragged last segments of 2D instances' lines can be left to tail launches whose
// waves take one such segment of several lines each (a 64-cell line would otherwise fill a second
// wave with 3 cells). Mode 0 captures the whole nsteps run (per step: 3 x [stage prep, y-sweep of
// the 2D instances, x-sweep + stage update of the 2D and of the 1D instances]) in one HIP graph and
// launches it once; mode 1 launches the plain tiles once per instance per kernel on the stream. A
// face or cell is computed by the same code whatever tile or launch holds it, its multiply-adds are
// fused as the source writes them, and the maxima are exact, so both modes and every launch shape
// give bitwise identical states.
//
// Launch shapes (segments per x-tile, columns per y-tile, tail packing on or off) are picked by a
// small autotuner at the first mode-0 run: each candidate advances a scratch copy of the batch by
// three timed steps (after a warm-up step) and the one with the fastest step is kept for the batch.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstring>
#include <new>
#include <vector>

#include "teno.h"
#include "teno_device.hpp"
#include "teno_internal.hpp"
#include "teno_worklist.hpp"

using namespace teno;

#define HIP_TRY(expr)                                   \
    do {                                                \
        hipError_t e_ = (expr);                         \
        if (e_ != hipSuccess) return TENO_E_HIP;        \
    } while (0)

namespace {

constexpr int NCOPY_B = 16;         // spread copies of the maxima per instance
constexpr int WS_CHUNK = 8192;      // cells per wave-speed work item

struct BatchInst {
    int sys, nx, ny, bc_x, bc_y;
    int pack_x, pack_y;             // ragged last segments packed (2D instances with short tails)
    int pad_;
    long long off;                  // element offset of the instance in the packed buffers
    double inv_dx, inv_dy;
    double eps4_x, eps4_y;          // 4 eps per direction (the measures' scale in smooth5)
    double keps4_x, keps4_y;        // shortcut factor times eps4
};

struct InstCtrl {
    unsigned long long part[3][NCOPY_B][NWORD];
    double alpha[8];
    double den, dt;
};

struct Item {
    int inst, tile;
};

template <typename T> struct BatchSweep {
    const BatchInst *inst;
    InstCtrl *ictrl;
    const Item *items;
    int begin, end;                 // item range of this launch
    const T *U;                     // stage input (packed)
    const T *U0;                    // RK base state (packed)
    const T *addend;                // y-part of dU/dt (packed, 2D instances only)
    T *out;                         // dU/dt (y) or the next stage (x)
    unsigned *err;
    int mode, stage, ring_next, scheme, alpha_mode;
    int packed;                     // the item lists leave packable ragged segments to the tail items
    T ct, gamma;
    T gm1;                          // gamma - 1, formed in double as the single-problem solver does
    T smooth_k;                     // all-smooth shortcut factor for ct
    T C;                            // C and q of eq:TENO1
    int q;
    int characteristic;             // 0: reconstruction per conserved component
};

int tiles_x(const teno_grid &g, int nseg_x) { return (int)x_main_items(g.nx, g.ny, nseg_x, false); }

}  // namespace

// per-item arguments of the plain sweep code
template <typename T, int SYS, int DIR>
__device__ __forceinline__ SweepArgs<T> item_args(const BatchSweep<T> &b, const BatchInst &I, int k)
{
    SweepArgs<T> a;
    a.U = b.U + I.off;
    a.U0 = b.U0 ? b.U0 + I.off : nullptr;
    a.addend = (b.addend && SYS == EULER2D) ? b.addend + I.off : nullptr;
    a.out = b.out + I.off;
    a.Fout = nullptr;
    a.chi_out = nullptr;
    a.masks_out = nullptr;
    a.flags_out = nullptr;
    a.masks_in = nullptr;
    a.alpha = b.ictrl[k].alpha;
    a.dt = &b.ictrl[k].dt;
    a.part = nullptr;
    a.err = b.err;
    a.nx = I.nx;
    a.ny = I.ny;
    a.len = DIR == 0 ? I.nx : I.ny;
    a.nlines = DIR == 0 ? I.ny : I.nx;
    a.nseg = main_nseg(a.len, b.packed && (DIR == 0 ? I.pack_x : I.pack_y));   // (packed: the last is a tail item's)
    a.bc = DIR == 0 ? I.bc_x : I.bc_y;
    a.bc_other = 0;
    a.mode = b.mode;
    a.stage = b.stage;
    a.scheme = b.scheme;
    a.alpha_mode = b.alpha_mode;
    a.inv_h = (T)(DIR == 0 ? I.inv_dx : I.inv_dy);
    a.ct = b.ct;
    a.eps4 = (T)(DIR == 0 ? I.eps4_x : I.eps4_y);
    a.smooth_k = b.smooth_k;
    a.keps4 = (T)(DIR == 0 ? I.keps4_x : I.keps4_y);
    a.gamma = b.gamma;
    a.gm1 = b.gm1;
    a.adv = T(1);
    a.inv_dx = (T)I.inv_dx;
    a.inv_dy = (T)I.inv_dy;
    a.C = b.C;
    a.q = b.q;
    a.characteristic = b.characteristic;
    return a;
}

// One (instance, tile) item per block. y-sweeps produce the y-part of dU/dt (MODE_RHS); x-sweeps
// apply the RK stage (MODE_STAGE) and put the block's wave-speed maxima into one spread copy of the
// instance's next ring slot. The grid is exactly the item range [begin, end).
// PACK: tail items, each the ragged last segments of NSEG x P lines of one instance (P per wave).
template <typename T, int SYS, int DIR, int NSEG, bool PACK>
__global__ void __launch_bounds__(BLOCK, (sweep_min_waves<SYS, DIR, false, DIR == 0 ? MODE_STAGE : MODE_RHS>()))
    batch_sweep_kernel(BatchSweep<T> b)
{
    constexpr int MODE = DIR == 0 ? MODE_STAGE : MODE_RHS;
    // (the coefficient rows stay in LDS here: the mixture's small instances cut many stencils, and
    // reading the rows from global memory measured 2 % slower on the 512-instance batch)
    constexpr bool CG = false;
    __shared__ T rec[rec_size<SYS, DIR, NSEG, PACK>()];
    __shared__ __align__(16) T ext[ext_size<T, SYS, DIR, NSEG, MODE>()];
    __shared__ T coef_lds[CG ? 1 : NCOEF_ROWS * 8];
    const Item item = b.items[b.begin + xcd_tile(blockIdx.x, gridDim.x)];
    const BatchInst I = b.inst[item.inst];
    SweepArgs<T> a = item_args<T, SYS, DIR>(b, I, item.inst);
    // the x-sweep's wave-speed maxima go to one spread copy of the instance's next ring slot
    if constexpr (MODE == MODE_STAGE) a.part = &b.ictrl[item.inst].part[b.ring_next][blockIdx.x % NCOPY_B][0];
    if constexpr (!CG) fill_coef(coef_lds);                 // (ordered by the tile's first barrier)
    const T *coef = CG ? coef_table<T>() : coef_lds;
    sweep_tile<T, SYS, DIR, false, NSEG, MODE, PACK>(a, item.tile, rec, ext, coef);
}

// Wave-speed maxima of every instance of a packed state (items: (instance, chunk of WS_CHUNK cells)).
template <typename T>
__global__ void __launch_bounds__(BLOCK) batch_wavespeed_kernel(const T *U, const BatchInst *inst, InstCtrl *ictrl,
                                                                const Item *items, int begin, int end, T gamma,
                                                                int alpha_mode, int ring, unsigned *err)
{
    __shared__ double red[BLOCK / WAVE * 9];
    for (int it = begin + (int)blockIdx.x; it < end; it += (int)gridDim.x) {
        const Item item = items[it];
        const BatchInst I = inst[item.inst];
        const size_t ncell = (size_t)I.nx * I.ny;
        const size_t c0 = (size_t)item.tile * WS_CHUNK;
        const size_t c1 = c0 + WS_CHUNK < ncell ? c0 + WS_CHUNK : ncell;
        double wmax[9];
        for (int k = 0; k < 9; ++k) wmax[k] = 0.0;
        unsigned bad = 0;
        for (size_t i = c0 + threadIdx.x; i < c1; i += BLOCK) {
            T u[4];
            const int nv = I.sys == EULER2D ? 4 : 3;
            for (int v = 0; v < nv; ++v) u[v] = U[I.off + (size_t)v * ncell + i];
            double w[9];
            bool ok = I.sys == EULER2D
                          ? cell_speeds<T, EULER2D>(u, gamma, T(1), (T)I.inv_dx, (T)I.inv_dy, alpha_mode, w)
                          : cell_speeds<T, EULER1D>(u, gamma, T(1), (T)I.inv_dx, (T)I.inv_dy, alpha_mode, w);
            if (!ok) bad |= ERR_NONPHYSICAL;
            for (int k = 0; k < 9; ++k) wmax[k] = fmax(wmax[k], w[k]);
        }
        block_max_atomic(wmax, &ictrl[item.inst].part[ring][item.tile % NCOPY_B][0], red);
        if (bad) atomicOr(err, bad);
        __syncthreads();
    }
}

// Per-instance stage preparation (the batched form of prep_kernel): reduce the spread maxima of
// one ring slot into alpha/den (and dt at stage 0), then clear the slot. One block per instance.
__global__ void batch_prep_kernel(InstCtrl *ictrl, int first, int count, int ring, int stage, double cfl,
                                  unsigned *err)
{
    for (int k = first + (int)blockIdx.x; k < first + count; k += (int)gridDim.x) {
        __shared__ double vals[NWORD];
        InstCtrl &C = ictrl[k];
        const int t = threadIdx.x;
        if (t < 9) {
            unsigned long long m = 0;
            for (int c = 0; c < NCOPY_B; ++c) {
                unsigned long long v = C.part[ring][c][t];
                m = v > m ? v : m;
            }
            vals[t] = __longlong_as_double((long long)m);
        }
        __syncthreads();
        for (int q = t; q < NCOPY_B * NWORD; q += blockDim.x) (&C.part[ring][0][0])[q] = 0ull;
        if (t < 8) C.alpha[t] = vals[t];
        if (t == 8) {
            C.den = vals[8];
            if (stage == 0) {
                double dt = cfl / vals[8];
                if (!(dt > 0.0) || !isfinite(dt)) atomicOr(err, ERR_NONFINITE);
                C.dt = dt;
            }
        }
        __syncthreads();
    }
}

__global__ void batch_clear_kernel(InstCtrl *ictrl, int n, int ring)
{
    for (int k = blockIdx.x; k < n; k += gridDim.x)
        for (int q = threadIdx.x; q < NCOPY_B * NWORD; q += blockDim.x) (&ictrl[k].part[ring][0][0])[q] = 0ull;
}

struct teno_batch {
    int n = 0;
    teno_opts opts;
    hipStream_t stream = nullptr;
    int dtype = TENO_F64;
    size_t esize = 8, total = 0;
    std::vector<teno_grid> grids;
    std::vector<BatchInst> inst;
    BatchInst *inst_d = nullptr;
    InstCtrl *ictrl_d = nullptr;
    unsigned *err_d = nullptr;
    void *S1 = nullptr, *S2 = nullptr, *dUy = nullptr;
    // work lists, one per tile-shape variant v (0: 4 segments, 1: 8 segments per tile) and layout p
    // (0: plain, every segment a main item; 1: packable ragged segments as tail items). The x-list
    // holds the 2D instances' main items [0, x2m_end), their tail items [x2m_end, x2_end), then the
    // 1D instances' items; the y-list the main items [0, ym_end), then the tail items.
    Item *items_x_d[2][2] = {{nullptr, nullptr}, {nullptr, nullptr}};
    Item *items_y_d[2][2] = {{nullptr, nullptr}, {nullptr, nullptr}};
    std::vector<int> xb[2], xe[2], yb[2], ye[2];      // per-instance item ranges of the plain lists
    int x2m_end[2][2] = {}, x2_end[2][2] = {}, x_total[2][2] = {}, ym_end[2][2] = {}, y_total[2][2] = {};
    Item *items_w_d = nullptr;
    std::vector<int> begin_w;
    // tuned launch shape
    bool tuned = false;
    int vx = 0, vy = 1, pk = 1;
    // captured run (a second stream for the parallel branches)
    hipStream_t cap_stream = nullptr, cap_stream2 = nullptr;
    hipEvent_t ev_fork[2][3] = {}, ev_join[2][3] = {};     // [y phase, x phase][stage]
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    void *graph_U = nullptr;
    int graph_steps = -1;
};

namespace {

template <typename T>
BatchSweep<T> base_args(const teno_batch *b)
{
    BatchSweep<T> a;
    std::memset(&a, 0, sizeof a);
    a.inst = b->inst_d;
    a.ictrl = b->ictrl_d;
    a.err = b->err_d;
    a.scheme = b->opts.scheme;
    a.alpha_mode = teno_alpha_mode(b->opts);
    a.ct = (T)b->opts.ct;
    a.smooth_k = (T)smooth_shortcut_k(b->opts.ct, b->opts.C, b->opts.q);
    a.C = (T)b->opts.C;
    a.q = b->opts.q;
    a.characteristic = b->opts.characteristic;
    a.gamma = (T)b->opts.gamma;
    a.gm1 = (T)(b->opts.gamma - 1.0);
    return a;
}

template <typename T, int SYS, int DIR, bool PACK = false>
void launch_batch_sweep(hipStream_t s, int variant, const BatchSweep<T> &a)
{
    const int grid = a.end - a.begin;
    if (grid <= 0) return;
    if (variant == 0)
        hipLaunchKernelGGL((batch_sweep_kernel<T, SYS, DIR, 4, PACK>), dim3(grid), dim3(BLOCK), 0, s, a);
    else
        hipLaunchKernelGGL((batch_sweep_kernel<T, SYS, DIR, 8, PACK>), dim3(grid), dim3(BLOCK), 0, s, a);
}

// Item ranges of one launch group in the lists of layout p: y main and tail items, 2D x main and
// tail items, 1D x-items.
struct Ranges {
    int p;
    int y0, y1, yt0, yt1, x2a, x2b, x2ta, x2tb, x1a, x1b;
};

Ranges all_ranges(const teno_batch *b, int vx, int vy, int p)
{
    return {p,
            0, b->ym_end[vy][p], b->ym_end[vy][p], b->y_total[vy][p],
            0, b->x2m_end[vx][p], b->x2m_end[vx][p], b->x2_end[vx][p],
            b->x2_end[vx][p], b->x_total[vx][p]};
}

// one instance's items in the plain lists
Ranges instance_ranges(const teno_batch *b, int k, int vx, int vy)
{
    Ranges r{0, b->yb[vy][k], b->ye[vy][k], 0, 0, 0, 0, 0, 0, 0, 0};
    if (b->inst[k].sys == EULER2D) {
        r.x2a = b->xb[vx][k];
        r.x2b = b->xe[vx][k];
    } else {
        r.x1a = b->xb[vx][k];
        r.x1b = b->xe[vx][k];
    }
    return r;
}

// Enqueue one SSP-RK3 step of the instances [first, first + count) whose items are r. With a second
// stream s2 (graph capture), the launches that share no data with the main ones run on a parallel
// branch beside them and join before the next phase: the y tail items beside the y main items, and
// the x tail items and the 1D instances' x-sweep beside the 2D x main items.
template <typename T>
void enqueue_step(teno_batch *b, hipStream_t s, T *U, int first, int count, const Ranges &r, int vx, int vy,
                  hipStream_t s2 = nullptr)
{
    T *in[3] = {U, (T *)b->S1, (T *)b->S2};
    T *outp[3] = {(T *)b->S1, (T *)b->S2, U};
    for (int k = 0; k < 3; ++k) {
        hipLaunchKernelGGL(batch_prep_kernel, dim3(count < 1024 ? count : 1024), dim3(64), 0, s, b->ictrl_d, first,
                           count, k, k, b->opts.cfl, b->err_d);
        BatchSweep<T> a = base_args<T>(b);
        a.packed = r.p;
        a.stage = k;
        a.U = in[k];
        a.items = b->items_y_d[vy][r.p];
        a.mode = MODE_RHS;
        a.out = (T *)b->dUy;
        // y-sweeps
        const bool fork_y = s2 != nullptr && r.yt1 > r.yt0;
        BatchSweep<T> at = a;
        at.begin = r.yt0;
        at.end = r.yt1;
        if (fork_y) {
            (void)hipEventRecord(b->ev_fork[0][k], s);
            (void)hipStreamWaitEvent(s2, b->ev_fork[0][k], 0);
            launch_batch_sweep<T, EULER2D, 1, true>(s2, vy, at);
            (void)hipEventRecord(b->ev_join[0][k], s2);
        }
        a.begin = r.y0;
        a.end = r.y1;
        launch_batch_sweep<T, EULER2D, 1>(s, vy, a);
        if (fork_y)
            (void)hipStreamWaitEvent(s, b->ev_join[0][k], 0);
        else
            launch_batch_sweep<T, EULER2D, 1, true>(s, vy, at);
        // x-sweeps with the stage update
        a.items = b->items_x_d[vx][r.p];
        a.mode = MODE_STAGE;
        a.U0 = U;
        a.addend = (T *)b->dUy;
        a.out = outp[k];
        a.ring_next = (k + 1) % 3;
        BatchSweep<T> a1 = a;
        a1.begin = r.x1a;
        a1.end = r.x1b;
        at = a;
        at.begin = r.x2ta;
        at.end = r.x2tb;
        const bool fork_x = s2 != nullptr && (r.x1b > r.x1a || r.x2tb > r.x2ta);
        if (fork_x) {
            (void)hipEventRecord(b->ev_fork[1][k], s);
            (void)hipStreamWaitEvent(s2, b->ev_fork[1][k], 0);
            launch_batch_sweep<T, EULER2D, 0, true>(s2, vx, at);
            launch_batch_sweep<T, EULER1D, 0>(s2, vx, a1);
            (void)hipEventRecord(b->ev_join[1][k], s2);
        }
        a.begin = r.x2a;
        a.end = r.x2b;
        launch_batch_sweep<T, EULER2D, 0>(s, vx, a);
        if (fork_x) {
            (void)hipStreamWaitEvent(s, b->ev_join[1][k], 0);
        } else {
            launch_batch_sweep<T, EULER2D, 0, true>(s, vx, at);
            launch_batch_sweep<T, EULER1D, 0>(s, vx, a1);
        }
    }
}

template <typename T>
void enqueue_init(teno_batch *b, hipStream_t s, const T *U, int first, int last)
{
    hipLaunchKernelGGL(batch_clear_kernel, dim3(256), dim3(256), 0, s, b->ictrl_d, b->n, 0);
    int beg = b->begin_w[first], end = b->begin_w[last];
    int grid = end - beg < 4096 ? end - beg : 4096;
    if (grid > 0)
        hipLaunchKernelGGL((batch_wavespeed_kernel<T>), dim3(grid), dim3(BLOCK), 0, s, U, b->inst_d, b->ictrl_d,
                           b->items_w_d, beg, end, (T)b->opts.gamma, teno_alpha_mode(b->opts), 0, b->err_d);
}

template <typename T>
teno_status run_t(teno_batch *b, T *U, int nsteps, int mode)
{
    if (mode == 1) {
        // one launch per instance per kernel, plain stream launches
        enqueue_init<T>(b, b->stream, U, 0, b->n);
        for (int n = 0; n < nsteps; ++n)
            for (int k = 0; k < b->n; ++k)
                enqueue_step<T>(b, b->stream, U, k, 1, instance_ranges(b, k, 0, 1), 0, 1);
        return hipGetLastError() == hipSuccess ? TENO_OK : TENO_E_HIP;
    }
    if (!b->tuned) {
        // autotune on a scratch copy of the batch: candidates (x-tile, y-tile, packing); the scratch
        // copy and the events are released on every path out of this block (hipFree waits for the
        // device, so no launch still reads the copy)
        struct TuneScratch {
            T *tmp = nullptr;
            hipEvent_t e0 = nullptr, e1 = nullptr;
            ~TuneScratch()
            {
                if (e0) (void)hipEventDestroy(e0);
                if (e1) (void)hipEventDestroy(e1);
                if (tmp) (void)hipFree(tmp);
            }
        } ts;
        HIP_TRY(hipMalloc(&ts.tmp, b->total * sizeof(T)));
        T *tmp = ts.tmp;
        HIP_TRY(hipMemcpyAsync(tmp, U, b->total * sizeof(T), hipMemcpyDeviceToDevice, b->stream));
        HIP_TRY(hipEventCreate(&ts.e0));
        HIP_TRY(hipEventCreate(&ts.e1));
        hipEvent_t e0 = ts.e0, e1 = ts.e1;
        float best = 1e30f;
        int bvx = 0, bvy = 1, bp = 0;
        for (int p = 0; p < 2; ++p)
            for (int vx = 0; vx < 2; ++vx)
                for (int vy = 0; vy < 2; ++vy) {
                    const Ranges r = all_ranges(b, vx, vy, p);
                    enqueue_init<T>(b, b->stream, tmp, 0, b->n);
                    enqueue_step<T>(b, b->stream, tmp, 0, b->n, r, vx, vy);    // warm-up
                    // the fastest of three timed steps (one step of the mixture takes about 12 ms;
                    // single timings of shapes a few per cent apart can come out in either order)
                    float fastest = 1e30f;
                    for (int rep = 0; rep < 3; ++rep) {
                        HIP_TRY(hipEventRecord(e0, b->stream));
                        enqueue_step<T>(b, b->stream, tmp, 0, b->n, r, vx, vy);
                        HIP_TRY(hipEventRecord(e1, b->stream));
                        HIP_TRY(hipEventSynchronize(e1));
                        float ms = 0.f;
                        HIP_TRY(hipEventElapsedTime(&ms, e0, e1));
                        fastest = std::min(fastest, ms);
                    }
                    if (fastest < best) { best = fastest; bvx = vx; bvy = vy; bp = p; }
                }
        b->vx = bvx;
        b->vy = bvy;
        b->pk = bp;
        b->tuned = true;
        unsigned z = 0;     // the tuning run's state is discarded, and so is its status
        HIP_TRY(hipMemcpy(b->err_d, &z, sizeof z, hipMemcpyHostToDevice));
    }
    if (!b->exec || b->graph_U != (void *)U || b->graph_steps != nsteps) {
        if (b->exec) (void)hipGraphExecDestroy(b->exec);
        if (b->graph) (void)hipGraphDestroy(b->graph);
        b->exec = nullptr;
        b->graph = nullptr;
        if (!b->cap_stream) HIP_TRY(hipStreamCreateWithFlags(&b->cap_stream, hipStreamNonBlocking));
        if (!b->cap_stream2) HIP_TRY(hipStreamCreateWithFlags(&b->cap_stream2, hipStreamNonBlocking));
        for (int k = 0; k < 3; ++k) {
            for (int ph = 0; ph < 2; ++ph) {
                if (!b->ev_fork[ph][k]) HIP_TRY(hipEventCreateWithFlags(&b->ev_fork[ph][k], hipEventDisableTiming));
                if (!b->ev_join[ph][k]) HIP_TRY(hipEventCreateWithFlags(&b->ev_join[ph][k], hipEventDisableTiming));
            }
        }
        HIP_TRY(hipStreamBeginCapture(b->cap_stream, hipStreamCaptureModeThreadLocal));
        enqueue_init<T>(b, b->cap_stream, U, 0, b->n);
        const Ranges r = all_ranges(b, b->vx, b->vy, b->pk);
        for (int n = 0; n < nsteps; ++n)
            enqueue_step<T>(b, b->cap_stream, U, 0, b->n, r, b->vx, b->vy, b->cap_stream2);
        HIP_TRY(hipStreamEndCapture(b->cap_stream, &b->graph));
        HIP_TRY(hipGraphInstantiate(&b->exec, b->graph, nullptr, nullptr, 0));
        b->graph_U = U;
        b->graph_steps = nsteps;
    }
    HIP_TRY(hipGraphLaunch(b->exec, b->stream));
    return TENO_OK;
}

}  // namespace

extern "C" {

teno_status teno_batch_create(const teno_grid *grids, int32_t n, const teno_opts *opts, void *stream, teno_batch **out)
{
    if (!out || !grids || !opts || n < 1) return TENO_E_ARG;
    *out = nullptr;
    const int dtype = grids[0].dtype;
    for (int k = 0; k < n; ++k) {
        const teno_grid &g = grids[k];
        if (g.sys != TENO_EULER1D && g.sys != TENO_EULER2D) return TENO_E_UNSUPPORTED;
        if (g.dtype != dtype || g.dtype < 0 || g.dtype > 1) return TENO_E_ARG;
        if (g.nx < 1 || g.ny < 1 || g.nx > (1 << 20) || g.ny > (1 << 20)) return TENO_E_ARG;
        if ((g.sys == TENO_EULER2D ? 4.0 : 3.0) * g.nx * g.ny >= 2147483647.0) return TENO_E_ARG;
        if (g.sys == TENO_EULER1D && g.ny != 1) return TENO_E_ARG;
        if (g.bc_x < 0 || g.bc_x > 1 || g.bc_y < 0 || g.bc_y > 1) return TENO_E_ARG;
        if (!(g.x1 > g.x0) || !(g.y1 > g.y0)) return TENO_E_ARG;
    }
    if (!teno_validate_opts(opts)) return TENO_E_ARG;

    teno_batch *b = new (std::nothrow) teno_batch();
    if (!b) return TENO_E_HIP;
    b->n = n;
    b->opts = *opts;
    b->stream = (hipStream_t)stream;
    b->dtype = dtype;
    b->esize = dtype == TENO_F64 ? 8 : 4;
    b->grids.assign(grids, grids + n);
    size_t off = 0;
    for (int k = 0; k < n; ++k) {
        const teno_grid &g = grids[k];
        BatchInst I;
        std::memset(&I, 0, sizeof I);
        I.sys = g.sys;
        I.nx = g.nx;
        I.ny = g.ny;
        I.bc_x = g.bc_x;
        I.bc_y = g.bc_y;
        I.pack_x = g.sys == TENO_EULER2D && packable(g.nx, g.ny);
        I.pack_y = g.sys == TENO_EULER2D && packable(g.ny, g.nx);
        I.off = (long long)off;
        double dx = (g.x1 - g.x0) / g.nx, dy = (g.y1 - g.y0) / g.ny;
        I.inv_dx = 1.0 / dx;
        I.inv_dy = 1.0 / dy;
        double eps_x, eps_y;
        if (opts->eps_mode == 1) eps_x = eps_y = opts->eps;
        else if (opts->scheme == TENO_SCHEME_TENO5) eps_x = eps_y = 1e-40;
        else { eps_x = dx * dx * dx; eps_y = dy * dy * dy; }
        const double sk = smooth_shortcut_k(opts->ct, opts->C, opts->q);
        I.eps4_x = 4.0 * eps_x;
        I.eps4_y = 4.0 * eps_y;
        I.keps4_x = sk * I.eps4_x;
        I.keps4_y = sk * I.eps4_y;
        b->inst.push_back(I);
        size_t ne = (size_t)(g.sys == TENO_EULER2D ? 4 : 3) * g.nx * g.ny;
        off += (ne + 63) / 64 * 64;                       // 512-byte aligned instances (FP64)
    }
    b->total = off;
    teno_status st = TENO_OK;
    // work lists: x-items of the 2D instances, then of the 1D ones; y-items of the 2D instances.
    // Item counts are launch grid sizes: they must stay below 2^31.
    {
        double nx_items = 0.0, ny_items = 0.0;
        for (int k = 0; k < n; ++k) {
            nx_items += (double)tiles_x(grids[k], 4);
            if (grids[k].sys == TENO_EULER2D) ny_items += (double)((grids[k].nx + 3) / 4) * nseg_of(grids[k].ny);
        }
        // (the packed lists hold at most one more item per instance)
        if (nx_items + n >= 2147483647.0 || ny_items + n >= 2147483647.0) {
            delete b;
            return TENO_E_ARG;
        }
    }
    // work lists (see teno_batch): per tile shape v and layout p, x-items of the 2D instances (main,
    // then tail), then of the 1D ones; y-items of the 2D instances (main, then tail)
    std::vector<Item> it;
    for (int v = 0; v < 2; ++v) {
        const int ns = v == 0 ? 4 : 8;
        b->xb[v].assign(n, 0);
        b->xe[v].assign(n, 0);
        b->yb[v].assign(n, 0);
        b->ye[v].assign(n, 0);
        for (int p = 0; p < 2; ++p) {
            it.clear();
            for (int k = 0; k < n; ++k) {                       // 2D main items
                if (grids[k].sys != TENO_EULER2D) continue;
                const bool pk = p == 1 && b->inst[k].pack_x;
                const int t = (int)x_main_items(grids[k].nx, grids[k].ny, ns, pk);
                if (p == 0) b->xb[v][k] = (int)it.size();
                for (int q = 0; q < t; ++q) it.push_back({k, q});
                if (p == 0) b->xe[v][k] = (int)it.size();
            }
            b->x2m_end[v][p] = (int)it.size();
            for (int k = 0; k < n && p == 1; ++k) {             // 2D tail items
                if (grids[k].sys != TENO_EULER2D || !b->inst[k].pack_x) continue;
                const int t = (int)x_tail_items(grids[k].nx, grids[k].ny, ns);
                for (int q = 0; q < t; ++q) it.push_back({k, q});
            }
            b->x2_end[v][p] = (int)it.size();
            for (int k = 0; k < n; ++k) {                       // 1D items
                if (grids[k].sys == TENO_EULER2D) continue;
                const int t = tiles_x(grids[k], ns);
                if (p == 0) b->xb[v][k] = (int)it.size();
                for (int q = 0; q < t; ++q) it.push_back({k, q});
                if (p == 0) b->xe[v][k] = (int)it.size();
            }
            b->x_total[v][p] = (int)it.size();
            if (hipMalloc(&b->items_x_d[v][p], (it.size() + 1) * sizeof(Item)) != hipSuccess ||
                (it.size() &&
                 hipMemcpy(b->items_x_d[v][p], it.data(), it.size() * sizeof(Item), hipMemcpyHostToDevice) != hipSuccess))
                st = TENO_E_HIP;
            it.clear();
            for (int k = 0; k < n; ++k) {                       // y main items
                if (p == 0) b->yb[v][k] = (int)it.size();
                if (grids[k].sys == TENO_EULER2D) {
                    const bool pk = p == 1 && b->inst[k].pack_y;
                    const int t = (int)y_main_items(grids[k].nx, grids[k].ny, ns, pk);
                    for (int q = 0; q < t; ++q) it.push_back({k, q});
                }
                if (p == 0) b->ye[v][k] = (int)it.size();
            }
            b->ym_end[v][p] = (int)it.size();
            for (int k = 0; k < n && p == 1; ++k) {             // y tail items
                if (grids[k].sys != TENO_EULER2D || !b->inst[k].pack_y) continue;
                const int t = (int)y_tail_items(grids[k].nx, grids[k].ny, ns);
                for (int q = 0; q < t; ++q) it.push_back({k, q});
            }
            b->y_total[v][p] = (int)it.size();
            if (hipMalloc(&b->items_y_d[v][p], (it.size() + 1) * sizeof(Item)) != hipSuccess ||
                (it.size() &&
                 hipMemcpy(b->items_y_d[v][p], it.data(), it.size() * sizeof(Item), hipMemcpyHostToDevice) != hipSuccess))
                st = TENO_E_HIP;
        }
    }
    it.clear();
    b->begin_w.assign(1, 0);
    for (int k = 0; k < n; ++k) {
        size_t nc = (size_t)grids[k].nx * grids[k].ny;
        int t = (int)((nc + WS_CHUNK - 1) / WS_CHUNK);
        for (int q = 0; q < t; ++q) it.push_back({k, q});
        b->begin_w.push_back((int)it.size());
    }
    if (hipMalloc(&b->items_w_d, it.size() * sizeof(Item)) != hipSuccess ||
        hipMemcpy(b->items_w_d, it.data(), it.size() * sizeof(Item), hipMemcpyHostToDevice) != hipSuccess)
        st = TENO_E_HIP;
    if (hipMalloc(&b->inst_d, n * sizeof(BatchInst)) != hipSuccess ||
        hipMemcpy(b->inst_d, b->inst.data(), n * sizeof(BatchInst), hipMemcpyHostToDevice) != hipSuccess)
        st = TENO_E_HIP;
    if (hipMalloc(&b->ictrl_d, n * sizeof(InstCtrl)) != hipSuccess ||
        hipMemset(b->ictrl_d, 0, n * sizeof(InstCtrl)) != hipSuccess)
        st = TENO_E_HIP;
    if (hipMalloc(&b->err_d, sizeof(unsigned)) != hipSuccess || hipMemset(b->err_d, 0, sizeof(unsigned)) != hipSuccess)
        st = TENO_E_HIP;
    if (hipMalloc(&b->S1, b->total * b->esize) != hipSuccess || hipMalloc(&b->S2, b->total * b->esize) != hipSuccess ||
        hipMalloc(&b->dUy, b->total * b->esize) != hipSuccess)
        st = TENO_E_HIP;
    if (st != TENO_OK) {
        teno_batch_destroy(b);
        return st;
    }
    *out = b;
    return TENO_OK;
}

teno_status teno_batch_destroy(teno_batch *b)
{
    if (!b) return TENO_E_ARG;
    (void)hipStreamSynchronize(b->stream);
    if (b->exec) (void)hipGraphExecDestroy(b->exec);
    if (b->graph) (void)hipGraphDestroy(b->graph);
    if (b->cap_stream) (void)hipStreamDestroy(b->cap_stream);
    if (b->cap_stream2) (void)hipStreamDestroy(b->cap_stream2);
    for (int k = 0; k < 3; ++k) {
        for (int ph = 0; ph < 2; ++ph) {
            if (b->ev_fork[ph][k]) (void)hipEventDestroy(b->ev_fork[ph][k]);
            if (b->ev_join[ph][k]) (void)hipEventDestroy(b->ev_join[ph][k]);
        }
    }
    for (int v = 0; v < 2; ++v)
        for (int p = 0; p < 2; ++p) {
            (void)hipFree(b->items_x_d[v][p]);
            (void)hipFree(b->items_y_d[v][p]);
        }
    (void)hipFree(b->items_w_d);
    (void)hipFree(b->inst_d);
    (void)hipFree(b->ictrl_d);
    (void)hipFree(b->err_d);
    (void)hipFree(b->S1);
    (void)hipFree(b->S2);
    (void)hipFree(b->dUy);
    delete b;
    return TENO_OK;
}

teno_status teno_batch_set_shape(teno_batch *b, int32_t x_tile, int32_t y_tile, int32_t packed)
{
    if (!b || (x_tile != 4 && x_tile != 8) || (y_tile != 4 && y_tile != 8) || (packed != 0 && packed != 1))
        return TENO_E_ARG;
    b->vx = x_tile == 4 ? 0 : 1;
    b->vy = y_tile == 4 ? 0 : 1;
    b->pk = packed;
    b->tuned = true;
    b->graph_steps = -1;            // recapture at the next mode-0 run
    return TENO_OK;
}

size_t teno_batch_total_elems(const teno_batch *b) { return b ? b->total : 0; }

size_t teno_batch_offset(const teno_batch *b, int32_t k)
{
    if (!b || k < 0 || k >= b->n) return (size_t)-1;
    return (size_t)b->inst[k].off;
}

teno_status teno_batch_run(teno_batch *b, void *U_dev, int32_t nsteps, int32_t mode)
{
    if (!b || !U_dev || nsteps < 0 || mode < 0 || mode > 1) return TENO_E_ARG;
    if (b->dtype == TENO_F64) return run_t<double>(b, (double *)U_dev, nsteps, mode);
    return run_t<float>(b, (float *)U_dev, nsteps, mode);
}

teno_status teno_batch_poll(teno_batch *b)
{
    if (!b) return TENO_E_ARG;
    HIP_TRY(hipStreamSynchronize(b->stream));
    unsigned e = 0;
    HIP_TRY(hipMemcpy(&e, b->err_d, sizeof e, hipMemcpyDeviceToHost));
    if (e) {
        unsigned z = 0;
        HIP_TRY(hipMemcpy(b->err_d, &z, sizeof z, hipMemcpyHostToDevice));
    }
    if (e & ERR_NONFINITE) return TENO_E_NONFINITE;
    if (e & ERR_NONPHYSICAL) return TENO_E_NONPHYSICAL;
    if (e & ERR_SELECTION) return TENO_E_NONFINITE;
    return TENO_OK;
}

}  // extern "C"
