/*
 * teno.h -- C ABI of the MI355X (gfx950) library for the TENO7X semi-discrete operator.
 *
 * Method: F. Zhang, J. Liu, H. Zhang, C. Xu, "An extending strategy based on TENO framework for
 * hyperbolic conservation laws" (arXiv:1808.00037). Equations are named by their labels in the
 * paper's source (eq:app, eq:smooth_expl, eq:TENO1, eq:norm, eq:seclect, eq:vec; Tables 1-3).
 *
 * Conventions shared by every entry point
 *  - Pointers named U, dUdt, lam, grad, F*, masks*, flags*, *_dev are DEVICE pointers owned by the
 *    caller. The library never frees caller memory.
 *  - States are structure-of-arrays [nvar][ny][nx], contiguous, element type given by the grid's
 *    dtype (double for TENO_F64, float for TENO_F32). nvar = 1 (scalar), 3 (1D Euler),
 *    4 (2D Euler: rho, rho u, rho v, E). ny = 1 for one-dimensional systems.
 *  - Faces: face f of a line is the left face of cell f (f = 0..len). x-face arrays are
 *    [..][ny][nx+1], y-face arrays [..][ny+1][nx]. Face-word arrays (masks, flags) hold the x-faces
 *    first, then (2D) the y-faces: teno_nfaces() words in total.
 *  - Mask word of a face: bits 8s..8s+3 = stencil code of the left-biased ('+') reconstruction of
 *    characteristic field s, bits 8s+4..8s+7 = code of the right-biased ('-') one. TENO7X codes are
 *    the candidate index m of Table 2 (0..12); TENO5 codes are (delta0<<2)|(delta1<<1)|delta2.
 *  - Flag word of a face: bits 6s+k = cut-off flag delta_k of the '+' side, bits 6s+3+k of the
 *    '-' side (eq:seclect), k = 0..2, field s.
 *  - All work is enqueued on the context's HIP stream and returns immediately. Argument errors are
 *    returned synchronously; device-side failures (non-finite or non-physical states, impossible
 *    selection patterns) set a sticky error word that teno_poll() reads (and clears).
 *  - A context is not thread-safe; use one context per host thread or stream.
 */
#ifndef TENO_H
#define TENO_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    TENO_OK = 0,
    TENO_E_ARG = -1,          /* invalid argument (null pointer, size, enum value) */
    TENO_E_UNSUPPORTED = -2,  /* valid request the library does not implement */
    TENO_E_HIP = -3,          /* a HIP runtime call failed */
    TENO_E_NONFINITE = -4,    /* a NaN/Inf reached a smoothness measure or state */
    TENO_E_NONPHYSICAL = -5,  /* density, pressure or Roe sound speed squared <= 0 */
    TENO_E_STATE = -6,        /* call not valid in the context's current state */
    TENO_E_CAPACITY = -7      /* the problem needs more than the fixed scratch of teno_step_noalloc */
} teno_status;

typedef enum { TENO_ADV1D = 0, TENO_EULER1D = 1, TENO_EULER2D = 2, TENO_BURGERS1D = 3 } teno_system;
typedef enum { TENO_SCHEME_TENO7X = 0, TENO_SCHEME_TENO5 = 1 } teno_scheme;
typedef enum { TENO_BC_PERIODIC = 0, TENO_BC_OUTFLOW = 1 } teno_bc;
typedef enum { TENO_F64 = 0, TENO_F32 = 1 } teno_dtype;

/* Uniform grid of cell centres x_i = x0 + (i + 1/2) dx, dx = (x1 - x0)/nx (point values, eq:flux). */
typedef struct {
    int32_t sys;      /* teno_system */
    int32_t nx, ny;   /* cells; ny = 1 for 1D systems; 1 <= nx, ny <= 2^20, nvar*nx*ny < 2^31 */
    int32_t bc_x, bc_y; /* teno_bc; outflow = zero-gradient copy of the boundary cell */
    int32_t dtype;    /* teno_dtype */
    double x0, x1, y0, y1;
} teno_grid;

typedef struct {
    int32_t scheme;     /* teno_scheme; TENO7X is the paper's presented method */
    int32_t alpha_mode; /* 0: Lax-Friedrichs constant per characteristic field, max_j |lambda_s(U_j)|;
                           1: one constant max_j(|u_n| + c) for all fields */
    int32_t eps_mode;   /* 0: eps = dx^3 per direction for TENO7X (section "The parameter epsilon"),
                           1e-40 for TENO5 (eq:TENO1); 1: the constant `eps` below */
    int32_t q;          /* exponent q of eq:TENO1, 1..12 (the paper: 6) */
    double gamma;       /* ratio of specific heats (1.4) */
    double ct;          /* cut-off C_T of eq:seclect, 0 < C_T < 1/3 (the paper: 1e-5) */
    double eps;         /* used when eps_mode = 1 */
    double cfl;         /* CFL number of the time-step rule */
    double adv_speed;   /* a of u_t + a u_x = 0 (TENO_ADV1D) */
    double C;           /* constant C of eq:TENO1, > 0 (the paper: 1) */
    int32_t characteristic; /* 1: reconstruct in characteristic variables (Remark 3; the paper);
                               0: per conserved component (no projection), with the one
                               Lax-Friedrichs constant max_j(|u_n| + c) for every component */
    int32_t reserved;   /* 0 */
} teno_opts;

typedef struct teno_ctx teno_ctx;

/* Fill *o with the paper's parameters: TENO7X, per-field alpha, eps = dx^3, C = 1, q = 6
 * (eq:TENO1), characteristic-wise reconstruction, gamma = 1.4, C_T = 1e-5, CFL 0.5, a = 1. */
void teno_default_opts(teno_opts *o);

/* Human-readable name of a status code (static string). */
const char *teno_status_str(teno_status s);

/* Measurement support (not part of the method): the current device's FP64 vector FMA rate in
 * TFLOP/s (an FMA counted as 2 flops), from a register-resident FMA loop of `iters` steps per chain
 * run over every compute unit on `stream` and timed with HIP events. Blocking; allocates and frees
 * a small output buffer. Errors: TENO_E_ARG (null tflops, iters outside 1..2^24), TENO_E_HIP. */
teno_status teno_probe_fp64_fma(void *stream, int32_t iters, double *tflops);

/* Device memory, in bytes, that a context for (grid, opts) allocates by itself at most: the control
 * block (at teno_create), the SSP-RK3 stage scratch (two states, plus the y-part of dU/dt for 2D
 * Euler; at the first step), and, when ckpt_every > 0, the scratch of a reverse sweep
 * teno_run_vjp(.., ckpt_every, ..) ((3 ckpt_every + 5) double states; 4 states for
 * ckpt_every = TENO_CKPT_STAGES). Caller-owned buffers (states, masks, checkpoints) are not
 * included. Returns 0 for an invalid grid or opts, or a negative ckpt_every other than
 * TENO_CKPT_STAGES. */
size_t teno_workspace_bytes(const teno_grid *grid, const teno_opts *opts, int32_t ckpt_every);

/* Create a context for one problem on the current HIP device; `stream` is a hipStream_t (NULL =
 * the null stream). Allocates the context's control block now and its RK3 scratch at the first
 * step (teno_workspace_bytes). Errors: TENO_E_ARG for an invalid grid/opts,
 * TENO_E_HIP if an allocation fails. */
teno_status teno_create(const teno_grid *grid, const teno_opts *opts, void *stream, teno_ctx **out);

/* Release the context and its scratch (never caller memory). Synchronises its stream. */
teno_status teno_destroy(teno_ctx *ctx);

/* Elements of one state (nvar*nx*ny) and face words (x-faces + y-faces). */
size_t teno_state_elems(const teno_ctx *ctx);
size_t teno_nfaces(const teno_ctx *ctx);

/* Replace the context's stream (hipStream_t). */
teno_status teno_set_stream(teno_ctx *ctx, void *stream);

/* The semi-discrete operator dU/dt = L(U) (eq:app): per face, the five-point TENO smoothness
 * measure and cut-off of every characteristic field and both split sides (eq:smooth_expl,
 * eq:tau5, eq:TENO1, eq:norm, eq:seclect), the neighbour vector of eq:vec mapped by Table 3
 * (TENO7X) to a Table 2 reconstruction, Roe-averaged characteristic projection with global
 * Lax-Friedrichs splitting (Remark 3), and the conservative difference, in x then (2D) y.
 * The Lax-Friedrichs constants come from U itself. U and dUdt must not overlap.
 * masks_out (nullable): teno_nfaces() mask words. */
teno_status teno_rhs(teno_ctx *ctx, const void *U, void *dUdt, uint32_t *masks_out);

/* Parity/debug form of teno_rhs: the numerical face fluxes Fx [nvar][ny][nx+1] and (2D)
 * Fy [nvar][ny+1][nx], mask and flag words (each nullable except Fx), the normalised smoothness
 * measures chi_k of eq:norm (chi, nullable: 24 values of the state's element type per face, in
 * face-word order, value 6s + 3 side + k for field s, side 0 = '+' / 1 = '-', k = 0..2; every face's
 * chi is evaluated, also where all stencils are provably kept), and the eight Lax-Friedrichs
 * constants used (alpha_dev, nullable: [0..3] x-fields, [4..7] y-fields, double). */
teno_status teno_face_fluxes(teno_ctx *ctx, const void *U, void *Fx, void *Fy, uint32_t *masks,
                             uint32_t *flags, void *chi, double *alpha_dev);

/* The operator with the selection (masks, teno_nfaces() words) and the eight Lax-Friedrichs
 * constants (alpha_dev, double) held fixed instead of computed from U. */
teno_status teno_rhs_frozen(teno_ctx *ctx, const void *U, const uint32_t *masks, const double *alpha_dev,
                            void *dUdt);

/* One SSP-RK3 step in Shu-Osher form (the paper cites Gottlieb, Shu & Tadmor 2001 and omits the
 * formula): U1 = U + dt L(U); U2 = 3/4 U + 1/4 (U1 + dt L(U1)); U <- 1/3 U + 2/3 (U2 + dt L(U2)).
 * dt_fixed > 0 sets dt; otherwise dt = cfl / max_j((|u|+c)/dx [+ (|v|+c)/dy]) from U on the
 * device (no host synchronisation). U is updated in place. */
teno_status teno_step(teno_ctx *ctx, void *U, double dt_fixed);

/* For callers that cannot allocate device memory (code under HIP graph capture, tight serving
 * loops, harnesses that forbid allocation): one SSP-RK3 step exactly as teno_step takes it, without a
 * context and without allocating anything. The control block and the stage scratch live in one fixed
 * device array of TENO_NOALLOC_SCRATCH_BYTES per GPU, part of the library's code object, held until
 * the process ends. A problem needing more (control block, two stage states, plus the y-part of dU/dt
 * for 2D Euler: about 96 bytes per cell for 2D Euler in double precision, i.e. up to about 174k cells)
 * is refused with TENO_E_CAPACITY before anything is enqueued; TENO_E_ARG for an invalid grid, opts
 * or pointer. U (device, [nvar][ny][nx], caller-owned) is advanced in place on `stream`
 * (hipStream_t). dt_fixed > 0 sets dt, else the CFL rule. status_dev (nullable, device int32)
 * receives TENO_OK or the device failure of this step (as teno_poll would report it); dt_dev
 * (nullable, device double) the step's dt. Every call on a GPU shares that GPU's scratch and starts
 * by clearing it, so calls that overlap on one GPU (several streams or threads) race and must be
 * ordered by the caller. Enqueues only; TENO_E_HIP if the scratch cannot be located. */
#define TENO_NOALLOC_SCRATCH_BYTES (16u << 20)
teno_status teno_step_noalloc(const teno_grid *grid, const teno_opts *opts, void *U, double dt_fixed,
                              void *stream, int32_t *status_dev, double *dt_dev);

/* nsteps calls of teno_step. use_graph = 1 captures one step into a HIP graph on first use and
 * replays it (identical results; fewer launches).
 * check_every <= 0: everything is enqueued without synchronisation; device failures are left to
 * teno_poll. check_every = k > 0: after every k steps (and after the last) the stream is
 * synchronised and the device error word read; on a failure no further step is enqueued, the error
 * word is cleared and TENO_E_NONPHYSICAL / TENO_E_NONFINITE returned. steps_done_host (nullable)
 * receives the number of steps that completed without a failure: nsteps on success, else the index
 * of the first step in which one was detected (U then holds the state after the last enqueued
 * step). Each step's failures are attributed to it by the device as they are raised, so the index
 * does not depend on k. */
teno_status teno_run(teno_ctx *ctx, void *U, int32_t nsteps, double dt_fixed, int32_t use_graph,
                     int32_t check_every, int32_t *steps_done_host);

/* Synchronise the stream and return (then clear) the sticky device error status. */
teno_status teno_poll(teno_ctx *ctx);

/* dt of the most recent step (synchronises). */
teno_status teno_last_dt(teno_ctx *ctx, double *dt_host);

/* Simulated time. Every step (teno_step, teno_run, teno_run_record; also the steps of a replayed
 * graph) advances the context's time t by its dt on the device; a new context starts at t = 0.
 * Replays of recorded steps (teno_run_replay, the recomputation inside teno_run_vjp) leave t alone.
 * teno_set_time sets t = t0 and, when t_end > t0, an end time: a step whose dt (from the CFL rule
 * or dt_fixed) would pass t_end is cut to end exactly there, and steps taken at t = t_end have
 * dt = 0 and leave the state unchanged bit for bit, so a run of more steps than needed stops at
 * t_end. t_end <= t0 removes the limit. Stream-ordered; TENO_E_ARG for a non-finite t0 or a NaN
 * t_end. (The paper runs its problems to fixed end times.) */
teno_status teno_set_time(teno_ctx *ctx, double t0, double t_end);

/* The simulated time t after the work enqueued so far (synchronises the stream). */
teno_status teno_get_time(teno_ctx *ctx, double *t_host);

/* Copy (stream-ordered, no synchronisation) the eight Lax-Friedrichs constants of the most recent
 * operator evaluation or stage to alpha_dev (device, 8 doubles: x fields then y fields). */
teno_status teno_last_alpha(teno_ctx *ctx, double *alpha_dev);

/* ------------------------------------------------------------------------------ measurement ----
 * Per-kernel timing with HIP events recorded on the context's stream around every sweep launch
 * (eager launches only; graph replays are not instrumented). kind 0 = x-sweep (with the RK stage
 * update when stepping), kind 1 = y-sweep. */
teno_status teno_set_timing(teno_ctx *ctx, int32_t enable);
/* Synchronise, then return for each kind the summed duration in ms and the launch count since
 * timing was enabled (arrays of 2). */
teno_status teno_read_timing(teno_ctx *ctx, double *ms, int32_t *count);

/* ---------------------------------------------------------------- frozen-selection adjoint ----
 * These entry points differentiate the operator and the RK3 trajectory with every stencil
 * selection, every Lax-Friedrichs constant and every dt held at the values of a recorded forward
 * run (the selection is piecewise constant in U, so this is the derivative almost everywhere).
 * Only TENO_F64 contexts with characteristic-wise reconstruction support them (TENO_E_UNSUPPORTED
 * otherwise). */

/* Vector-Jacobian product of the frozen operator at U: grad = (dL/dU)^T lam. Overwrites grad.
 * Periodic directions need at least 8 cells (TENO_E_UNSUPPORTED otherwise). */
teno_status teno_rhs_vjp(teno_ctx *ctx, const void *U, const uint32_t *masks, const double *alpha_dev,
                         const void *lam, void *grad);

/* Value of ckpt_every for teno_run_record / teno_run_vjp that stores every stage input of every
 * step (3 nsteps states in ckpt_dev: for step j, U^n, U1, U2 at states 3j, 3j+1, 3j+2), so that the
 * reverse sweep recomputes nothing; memory for speed (2D Euler 1024^2, 400 steps: 40 GB). */
#define TENO_CKPT_STAGES (-1)

/* Forward run of nsteps steps that records what the adjoint needs: ckpt_dev holds
 * ceil(nsteps/ckpt_every) states (the state before steps 0, ckpt_every, 2*ckpt_every, ...),
 * masks_dev (nullable) nsteps*3*teno_nfaces() mask words, alpha_dt_dev nsteps*(3*8+1) doubles
 * (per step: the three stages' eight constants, then dt). U is advanced in place. ckpt_every must be
 * >= 1 or TENO_CKPT_STAGES (ckpt_dev then holds 3*nsteps states); otherwise TENO_E_ARG. */
teno_status teno_run_record(teno_ctx *ctx, void *U, int32_t nsteps, double dt_fixed, int32_t ckpt_every,
                            void *ckpt_dev, uint32_t *masks_dev, double *alpha_dt_dev);

/* The frozen forward map from the state U over nsteps recorded steps (same masks/alpha/dt). */
teno_status teno_run_replay(teno_ctx *ctx, void *U, int32_t nsteps, const uint32_t *masks_dev,
                            const double *alpha_dt_dev);

/* Reverse sweep: given lam = dJ/dU(T) in lam_io, overwrite it with dJ/dU(0). Recomputes each
 * checkpoint segment forward (frozen) and applies the adjoint of every RK stage in reverse.
 * With ckpt_every = TENO_CKPT_STAGES (a recording that stored every stage input) nothing is
 * recomputed. Needs masks_dev (recorded). Scratch: 3*ckpt_every+5 double states (4 with
 * TENO_CKPT_STAGES), allocated on first use (the stage states of one segment and the running
 * state, then the y part of J^T mu, two mu and one lam). */
teno_status teno_run_vjp(teno_ctx *ctx, const void *ckpt_dev, const uint32_t *masks_dev,
                         const double *alpha_dt_dev, int32_t nsteps, int32_t ckpt_every, void *lam_io);

/* -------------------------------------------------------------------------------- batching ----
 * Many independent problems (1D and 2D Euler mixed, uneven sizes, same dtype and options)
 * advanced together. The batch owns a packed state buffer; instance k's state lives at element
 * offset teno_batch_offset(b, k) with the usual [nvar][ny][nx] layout. */
typedef struct teno_batch teno_batch;

teno_status teno_batch_create(const teno_grid *grids, int32_t n, const teno_opts *opts, void *stream,
                              teno_batch **out);
teno_status teno_batch_destroy(teno_batch *b);
size_t teno_batch_total_elems(const teno_batch *b);
size_t teno_batch_offset(const teno_batch *b, int32_t k);

/* Advance every instance by nsteps SSP-RK3 steps (each instance with its own CFL dt).
 * mode 0: all instances per kernel in static work-list launches (one (instance, tile) item per
 * block), the whole run captured once in a HIP graph and replayed; mode 1: one launch per
 * instance per kernel (reference form).
 * U_dev: the packed state of teno_batch_total_elems() elements. Both modes give bitwise equal
 * results. Unless teno_batch_set_shape() fixed it, the first mode-0 run picks the launch shape:
 * it advances a temporary copy of the state (allocated and freed inside the call, synchronising
 * the stream) by a warm-up and three timed steps per candidate shape and keeps the fastest. */
teno_status teno_batch_run(teno_batch *b, void *U_dev, int32_t nsteps, int32_t mode);

/* Fix mode 0's launch shape instead of letting the first mode-0 run pick it by timing:
 * x_tile segments per x-sweep block and y_tile columns per y-sweep block (4 or 8 each), and
 * packed = 1 to give the short ragged last segments of 2D instances' lines to tail launches that
 * take several lines per wave (0: every segment in the main launches). The result does not depend
 * on the shape. Host-only; TENO_E_ARG for other values or a null batch. Discards a captured graph. */
teno_status teno_batch_set_shape(teno_batch *b, int32_t x_tile, int32_t y_tile, int32_t packed);

/* Synchronise and return (then clear) the batch's sticky device error status. */
teno_status teno_batch_poll(teno_batch *b);

#ifdef __cplusplus
}
#endif
#endif /* TENO_H */
