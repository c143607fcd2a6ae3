"""Python binding of the gfx950 TENO7X library (include/teno.h) through ctypes.

Argument marshalling only: every step of the operator, the time stepper, the adjoint and the
batched runs executes in the HIP kernels of libteno.so. torch provides device memory and the
current stream. There is no CPU fallback: without the built library every call fails.

States are torch tensors on the GPU, shape [nvar, ny, nx], contiguous, float64 (or float32 for
single-precision contexts); conserved variables (rho, rho u, [rho v], E).
"""
import ctypes
import os

import torch

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libteno.so")

ADV1D, EULER1D, EULER2D, BURGERS1D = 0, 1, 2, 3
TENO7X, TENO5 = 0, 1
PERIODIC, OUTFLOW = 0, 1
F64, F32 = 0, 1
NVAR = {ADV1D: 1, EULER1D: 3, EULER2D: 4, BURGERS1D: 1}

STATUS = {0: "ok", -1: "invalid argument", -2: "unsupported", -3: "HIP runtime error",
          -4: "non-finite value", -5: "non-physical state", -6: "invalid context state",
          -7: "problem exceeds the fixed scratch of the no-allocation entry point"}
NOALLOC_SCRATCH_BYTES = 16 << 20
CKPT_STAGES = -1          # ckpt_every that stores every stage input (TENO_CKPT_STAGES)


class TenoError(RuntimeError):
    def __init__(self, code, where):
        super().__init__(f"{where}: {STATUS.get(code, code)} ({code})")
        self.code = code


class Grid(ctypes.Structure):
    _fields_ = [("sys", ctypes.c_int32), ("nx", ctypes.c_int32), ("ny", ctypes.c_int32),
                ("bc_x", ctypes.c_int32), ("bc_y", ctypes.c_int32), ("dtype", ctypes.c_int32),
                ("x0", ctypes.c_double), ("x1", ctypes.c_double), ("y0", ctypes.c_double),
                ("y1", ctypes.c_double)]


class Opts(ctypes.Structure):
    _fields_ = [("scheme", ctypes.c_int32), ("alpha_mode", ctypes.c_int32), ("eps_mode", ctypes.c_int32),
                ("q", ctypes.c_int32), ("gamma", ctypes.c_double), ("ct", ctypes.c_double),
                ("eps", ctypes.c_double), ("cfl", ctypes.c_double), ("adv_speed", ctypes.c_double),
                ("C", ctypes.c_double), ("characteristic", ctypes.c_int32), ("reserved", ctypes.c_int32)]


_lib = None

# exported symbol -> (restype, argtypes)
_P = ctypes.c_void_p
_SIGS = {
    "teno_default_opts": (None, [_P]),
    "teno_status_str": (ctypes.c_char_p, [ctypes.c_int]),
    "teno_create": (ctypes.c_int, [_P, _P, _P, _P]),
    "teno_destroy": (ctypes.c_int, [_P]),
    "teno_state_elems": (ctypes.c_size_t, [_P]),
    "teno_nfaces": (ctypes.c_size_t, [_P]),
    "teno_set_stream": (ctypes.c_int, [_P, _P]),
    "teno_rhs": (ctypes.c_int, [_P, _P, _P, _P]),
    "teno_face_fluxes": (ctypes.c_int, [_P, _P, _P, _P, _P, _P, _P, _P]),
    "teno_workspace_bytes": (ctypes.c_size_t, [_P, _P, ctypes.c_int32]),
    "teno_rhs_frozen": (ctypes.c_int, [_P, _P, _P, _P, _P]),
    "teno_step": (ctypes.c_int, [_P, _P, ctypes.c_double]),
    "teno_step_noalloc": (ctypes.c_int, [_P, _P, _P, ctypes.c_double, _P, _P, _P]),
    "teno_run": (ctypes.c_int, [_P, _P, ctypes.c_int32, ctypes.c_double, ctypes.c_int32, ctypes.c_int32,
                                ctypes.POINTER(ctypes.c_int32)]),
    "teno_poll": (ctypes.c_int, [_P]),
    "teno_last_dt": (ctypes.c_int, [_P, _P]),
    "teno_set_time": (ctypes.c_int, [_P, ctypes.c_double, ctypes.c_double]),
    "teno_get_time": (ctypes.c_int, [_P, _P]),
    "teno_last_alpha": (ctypes.c_int, [_P, _P]),
    "teno_set_timing": (ctypes.c_int, [_P, ctypes.c_int32]),
    "teno_read_timing": (ctypes.c_int, [_P, _P, _P]),
    "teno_rhs_vjp": (ctypes.c_int, [_P, _P, _P, _P, _P, _P]),
    "teno_run_record": (ctypes.c_int, [_P, _P, ctypes.c_int32, ctypes.c_double, ctypes.c_int32, _P, _P, _P]),
    "teno_run_replay": (ctypes.c_int, [_P, _P, ctypes.c_int32, _P, _P]),
    "teno_run_vjp": (ctypes.c_int, [_P, _P, _P, _P, ctypes.c_int32, ctypes.c_int32, _P]),
    "teno_batch_create": (ctypes.c_int, [_P, ctypes.c_int32, _P, _P, _P]),
    "teno_batch_destroy": (ctypes.c_int, [_P]),
    "teno_batch_total_elems": (ctypes.c_size_t, [_P]),
    "teno_batch_offset": (ctypes.c_size_t, [_P, ctypes.c_int32]),
    "teno_batch_run": (ctypes.c_int, [_P, _P, ctypes.c_int32, ctypes.c_int32]),
    "teno_batch_poll": (ctypes.c_int, [_P]),
    "teno_batch_set_shape": (ctypes.c_int, [_P, ctypes.c_int32, ctypes.c_int32, ctypes.c_int32]),
    "teno_probe_fp64_fma": (ctypes.c_int, [_P, ctypes.c_int32, ctypes.POINTER(ctypes.c_double)]),
}


def lib():
    """Load libteno.so (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: build it with paper_1808_00037_amd/build.py")
        L = ctypes.CDLL(LIB_PATH)
        for name, (res, args) in _SIGS.items():
            fn = getattr(L, name)
            fn.restype = res
            fn.argtypes = args
        _lib = L
    return _lib


def _check(code, where):
    if code != 0:
        raise TenoError(code, where)


def _ptr(t):
    return None if t is None else ctypes.c_void_p(t.data_ptr())


def _stream():
    return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)


_WORD_TYPES = (torch.int32,) + ((torch.uint32,) if hasattr(torch, "uint32") else ())


def _buf(t, dtypes, numel, what):
    """A device buffer the library writes or reads by pointer: contiguous, on the GPU, of one of
    dtypes and with at least numel elements (the C ABI cannot check sizes)."""
    if not (isinstance(t, torch.Tensor) and t.is_cuda and t.is_contiguous() and t.dtype in dtypes
            and t.numel() >= numel):
        names = "/".join(str(d).replace("torch.", "") for d in dtypes)
        raise ValueError(f"{what} must be a contiguous {names} CUDA tensor of at least {numel} elements")
    return t


def default_opts():
    o = Opts()
    lib().teno_default_opts(ctypes.byref(o))
    return o


def make_opts(scheme=TENO7X, alpha_mode=0, eps=None, gamma=1.4, ct=1e-5, cfl=0.5, adv_speed=1.0, C=1.0, q=6,
              characteristic=1):
    """teno_opts from the paper's defaults with the given changes (eps None: dx^3 / 1e-40 by scheme)."""
    o = default_opts()
    o.scheme, o.alpha_mode, o.gamma, o.ct, o.cfl, o.adv_speed = scheme, alpha_mode, gamma, ct, cfl, adv_speed
    o.C, o.q, o.characteristic = float(C), int(q), int(characteristic)
    if eps is not None:
        o.eps_mode, o.eps = 1, float(eps)
    return o


def workspace_bytes(sys, nx, ny=1, dtype=torch.float64, ckpt_every=0, **opts):
    """Device bytes a context allocates by itself (teno_workspace_bytes); 0 for invalid arguments."""
    g = Grid(sys, nx, ny, PERIODIC, PERIODIC, F64 if dtype == torch.float64 else F32, 0.0, 1.0, 0.0, 1.0)
    o = make_opts(**opts)
    return lib().teno_workspace_bytes(ctypes.byref(g), ctypes.byref(o), int(ckpt_every))


def step_noalloc(grid, opts, U, dt=0.0, status=None, dt_out=None):
    """teno_step_noalloc: one SSP-RK3 step of U in place on the current stream, without a context and
    without any device allocation (fixed scratch of NOALLOC_SCRATCH_BYTES per GPU). grid/opts: Grid
    and Opts structures (e.g. a Solver's .grid and .opts). status (int32, 1 element) and dt_out
    (float64, 1 element): optional device outputs."""
    dt_type = torch.float64 if grid.dtype == F64 else torch.float32
    nv = NVAR[grid.sys]
    if not (isinstance(U, torch.Tensor) and U.is_cuda and U.is_contiguous() and U.dtype == dt_type
            and tuple(U.shape) == (nv, grid.ny, grid.nx)):
        raise ValueError(f"state must be a contiguous {dt_type} CUDA tensor of shape {(nv, grid.ny, grid.nx)}")
    if status is not None:
        _buf(status, (torch.int32,), 1, "status")
    if dt_out is not None:
        _buf(dt_out, (torch.float64,), 1, "dt_out")
    _check(lib().teno_step_noalloc(ctypes.byref(grid), ctypes.byref(opts), _ptr(U), float(dt), _stream(),
                                   _ptr(status), _ptr(dt_out)), "teno_step_noalloc")
    return U


class Solver:
    """One problem instance on the current GPU: grid, boundary conditions and scheme options."""

    def __init__(self, sys, nx, ny=1, x0=0.0, x1=1.0, y0=0.0, y1=1.0, bc_x=PERIODIC, bc_y=PERIODIC,
                 dtype=torch.float64, scheme=TENO7X, alpha_mode=0, eps=None, gamma=1.4, ct=1e-5,
                 cfl=0.5, adv_speed=1.0, C=1.0, q=6, characteristic=1):
        self.sys, self.nx, self.ny = sys, nx, ny
        self.dtype = dtype
        self.nvar = NVAR[sys]
        g = Grid(sys, nx, ny, bc_x, bc_y, F64 if dtype == torch.float64 else F32, x0, x1, y0, y1)
        o = make_opts(scheme=scheme, alpha_mode=alpha_mode, eps=eps, gamma=gamma, ct=ct, cfl=cfl,
                      adv_speed=adv_speed, C=C, q=q, characteristic=characteristic)
        self.grid, self.opts = g, o
        self._stream_val = torch.cuda.current_stream().cuda_stream
        h = ctypes.c_void_p()
        _check(lib().teno_create(ctypes.byref(g), ctypes.byref(o), _stream(), ctypes.byref(h)), "teno_create")
        self._h = h
        self.nfaces = lib().teno_nfaces(h)
        self.nfaces_x = ny * (nx + 1)

    @classmethod
    def for_problem(cls, pr, dtype=torch.float64, **kw):
        """Build from a workloads.Problem."""
        return cls(pr.sys, pr.nx, pr.ny, pr.x0, pr.x1, pr.y0, pr.y1, pr.bc_x, pr.bc_y, dtype=dtype,
                   cfl=pr.cfl, gamma=pr.gamma, **kw)

    @property
    def shape(self):
        return (self.nvar, self.ny, self.nx)

    def close(self):
        if getattr(self, "_h", None):
            lib().teno_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _sync_stream(self):
        s = torch.cuda.current_stream().cuda_stream
        if s != self._stream_val:
            _check(lib().teno_set_stream(self._h, ctypes.c_void_p(s)), "teno_set_stream")
            self._stream_val = s

    def _state(self, U):
        if not (U.is_cuda and U.dtype == self.dtype and U.is_contiguous() and tuple(U.shape) == self.shape):
            raise ValueError(f"state must be a contiguous {self.dtype} CUDA tensor of shape {self.shape}")
        return U

    def empty_state(self):
        return torch.empty(self.shape, dtype=self.dtype, device="cuda")

    def masks_buffer(self):
        return torch.empty(self.nfaces, dtype=torch.int32, device="cuda")

    def rhs(self, U, out=None, masks=None):
        self._sync_stream()
        U = self._state(U)
        out = self.empty_state() if out is None else self._state(out)
        if masks is not None:
            _buf(masks, _WORD_TYPES, self.nfaces, "masks")
        _check(lib().teno_rhs(self._h, _ptr(U), _ptr(out), _ptr(masks)), "teno_rhs")
        return out

    def face_fluxes(self, U, chi=False):
        """Face fluxes, mask and flag words and the Lax-Friedrichs constants of one evaluation; with
        chi, also chi of eq:norm ([nfaces, 24]: field s, side, k at 6 s + 3 side + k)."""
        self._sync_stream()
        U = self._state(U)
        nv, nx, ny = self.nvar, self.nx, self.ny
        Fx = torch.empty((nv, ny, nx + 1), dtype=self.dtype, device="cuda")
        Fy = torch.empty((nv, ny + 1, nx), dtype=self.dtype, device="cuda") if self.sys == EULER2D else None
        masks = torch.empty(self.nfaces, dtype=torch.int32, device="cuda")
        flags = torch.empty(self.nfaces, dtype=torch.int32, device="cuda")
        chis = torch.empty((self.nfaces, 24), dtype=self.dtype, device="cuda") if chi else None
        alpha = torch.zeros(8, dtype=torch.float64, device="cuda")
        _check(lib().teno_face_fluxes(self._h, _ptr(U), _ptr(Fx), _ptr(Fy), _ptr(masks), _ptr(flags), _ptr(chis),
                                      _ptr(alpha)), "teno_face_fluxes")
        out = dict(Fx=Fx, masks=masks, flags=flags, alpha=alpha)
        if Fy is not None:
            out["Fy"] = Fy
        if chis is not None:
            out["chi"] = chis
        return out

    def rhs_frozen(self, U, masks, alpha, out=None):
        self._sync_stream()
        U = self._state(U)
        out = self.empty_state() if out is None else self._state(out)
        _buf(masks, _WORD_TYPES, self.nfaces, "masks")
        _buf(alpha, (torch.float64,), 8, "alpha")
        _check(lib().teno_rhs_frozen(self._h, _ptr(U), _ptr(masks), _ptr(alpha), _ptr(out)), "teno_rhs_frozen")
        return out

    def step(self, U, dt=0.0):
        self._sync_stream()
        _check(lib().teno_step(self._h, _ptr(self._state(U)), float(dt)), "teno_step")
        return U

    def run(self, U, nsteps, dt=0.0, graph=True, check_every=0):
        """nsteps SSP-RK3 steps in place. check_every > 0: the device status is read every
        check_every steps; a failure raises TenoError with .steps_done, the number of steps that
        completed before the one it was detected in."""
        self._sync_stream()
        done = ctypes.c_int32(0)
        code = lib().teno_run(self._h, _ptr(self._state(U)), int(nsteps), float(dt), 1 if graph else 0,
                              int(check_every), ctypes.byref(done))
        if code != 0:
            err = TenoError(code, "teno_run")
            err.steps_done = done.value
            raise err
        return U

    def poll(self):
        _check(lib().teno_poll(self._h), "device status")

    def last_dt(self):
        v = ctypes.c_double()
        _check(lib().teno_last_dt(self._h, ctypes.byref(v)), "teno_last_dt")
        return v.value

    def set_time(self, t0=0.0, t_end=0.0):
        """Set the simulated time to t0 and, when t_end > t0, stop the runs that follow at t_end
        (the step that would pass it is cut; later steps leave the state unchanged)."""
        self._sync_stream()
        _check(lib().teno_set_time(self._h, float(t0), float(t_end)), "teno_set_time")

    def time(self):
        v = ctypes.c_double()
        _check(lib().teno_get_time(self._h, ctypes.byref(v)), "teno_get_time")
        return v.value

    def last_alpha(self):
        """The eight Lax-Friedrichs constants of the most recent evaluation (device tensor)."""
        out = torch.empty(8, dtype=torch.float64, device="cuda")
        _check(lib().teno_last_alpha(self._h, _ptr(out)), "teno_last_alpha")
        return out

    def set_timing(self, enable=True):
        _check(lib().teno_set_timing(self._h, 1 if enable else 0), "teno_set_timing")

    def read_timing(self):
        """{kind: (total ms, launches)} for kind 'x' (x-sweep [+ RK stage]) and 'y' (y-sweep)."""
        ms = (ctypes.c_double * 2)()
        cnt = (ctypes.c_int32 * 2)()
        _check(lib().teno_read_timing(self._h, ms, cnt), "teno_read_timing")
        return {"x": (ms[0], cnt[0]), "y": (ms[1], cnt[1])}

    # ------------------------------------------------------------------ frozen-selection adjoint
    def rhs_vjp(self, U, masks, alpha, lam, out=None):
        self._sync_stream()
        out = self.empty_state() if out is None else self._state(out)
        _buf(masks, _WORD_TYPES, self.nfaces, "masks")
        _buf(alpha, (torch.float64,), 8, "alpha")
        _check(lib().teno_rhs_vjp(self._h, _ptr(self._state(U)), _ptr(masks), _ptr(alpha), _ptr(self._state(lam)),
                                  _ptr(out)), "teno_rhs_vjp")
        return out

    def run_record(self, U, nsteps, ckpt_every, dt=0.0, record_masks=True):
        """Advance U in place; returns the recording (checkpoints, masks, alpha/dt). ckpt_every =
        CKPT_STAGES keeps every stage input (3 nsteps states) so that the backward pass recomputes
        nothing."""
        self._sync_stream()
        if ckpt_every != CKPT_STAGES and ckpt_every < 1:
            raise ValueError("ckpt_every must be >= 1 or CKPT_STAGES")
        nck = max(3 * nsteps, 1) if ckpt_every == CKPT_STAGES else nsteps // ckpt_every + 1
        ckpt = torch.empty((nck,) + self.shape, dtype=self.dtype, device="cuda")
        masks = torch.empty((nsteps, 3, self.nfaces), dtype=torch.int32, device="cuda") if record_masks else None
        ad = torch.empty((nsteps, 25), dtype=torch.float64, device="cuda")
        _check(lib().teno_run_record(self._h, _ptr(self._state(U)), int(nsteps), float(dt), int(ckpt_every),
                                     _ptr(ckpt), _ptr(masks), _ptr(ad)), "teno_run_record")
        return dict(ckpt=ckpt, masks=masks, alpha_dt=ad, nsteps=nsteps, ckpt_every=ckpt_every)

    def run_replay(self, U, rec, nsteps=None):
        self._sync_stream()
        n = rec["nsteps"] if nsteps is None else nsteps
        if not 0 <= n <= rec["nsteps"]:
            raise ValueError("nsteps exceeds the recording")
        _buf(rec["masks"], _WORD_TYPES, n * 3 * self.nfaces, "recorded masks")
        _buf(rec["alpha_dt"], (torch.float64,), n * 25, "recorded alpha/dt")
        _check(lib().teno_run_replay(self._h, _ptr(self._state(U)), int(n), _ptr(rec["masks"]), _ptr(rec["alpha_dt"])),
               "teno_run_replay")
        return U

    def run_vjp(self, rec, lam):
        """lam: dJ/dU(T) (overwritten in place with dJ/dU(0))."""
        self._sync_stream()
        n, ck = int(rec["nsteps"]), int(rec["ckpt_every"])
        if rec["masks"] is None:
            raise ValueError("the backward pass needs a recording with masks")
        nck = 3 * n if ck == CKPT_STAGES else -(-n // ck)
        _buf(rec["ckpt"], (self.dtype,), nck * self.nvar * self.nx * self.ny, "checkpoints")
        _buf(rec["masks"], _WORD_TYPES, n * 3 * self.nfaces, "recorded masks")
        _buf(rec["alpha_dt"], (torch.float64,), n * 25, "recorded alpha/dt")
        _check(lib().teno_run_vjp(self._h, _ptr(rec["ckpt"]), _ptr(rec["masks"]), _ptr(rec["alpha_dt"]),
                                  int(rec["nsteps"]), int(rec["ckpt_every"]), _ptr(self._state(lam))), "teno_run_vjp")
        return lam


class TenoRHS(torch.autograd.Function):
    """dU/dt = L(U) with a backward pass through the frozen-selection adjoint (the stencil
    selection and Lax-Friedrichs constants of the forward evaluation held fixed)."""

    @staticmethod
    def forward(ctx, U, solver):
        masks = solver.masks_buffer()
        out = solver.rhs(U.detach().contiguous(), masks=masks)
        ctx.solver, ctx.masks, ctx.alpha = solver, masks, solver.last_alpha()
        ctx.save_for_backward(U)
        return out

    @staticmethod
    def backward(ctx, gout):
        (U,) = ctx.saved_tensors
        g = ctx.solver.rhs_vjp(U.detach().contiguous(), ctx.masks, ctx.alpha, gout.contiguous())
        return g, None


class TenoTrajectory(torch.autograd.Function):
    """U(T) after nsteps SSP-RK3 steps from U0, differentiable through the frozen-selection adjoint
    with checkpoints every ckpt_every steps (the backward pass recomputes one segment at a time), or
    with every stage input kept (ckpt_every = CKPT_STAGES: nothing recomputed)."""

    @staticmethod
    def forward(ctx, U0, solver, nsteps, ckpt_every, dt=0.0):
        U = U0.detach().clone().contiguous()
        rec = solver.run_record(U, nsteps, ckpt_every, dt=dt)
        ctx.solver, ctx.rec = solver, rec
        return U

    @staticmethod
    def backward(ctx, gout):
        lam = gout.detach().clone().contiguous()
        ctx.solver.run_vjp(ctx.rec, lam)
        return lam, None, None, None, None


def rhs(U, solver):
    return TenoRHS.apply(U, solver)


def trajectory(U0, solver, nsteps, ckpt_every=20, dt=0.0):
    return TenoTrajectory.apply(U0, solver, nsteps, ckpt_every, dt)


def probe_fp64_fma(iters=4096):
    """Measured FP64 vector FMA rate of the current device, TFLOP/s (an FMA counted as 2 flops)."""
    out = ctypes.c_double(0.0)
    _check(lib().teno_probe_fp64_fma(_stream(), int(iters), ctypes.byref(out)), "teno_probe_fp64_fma")
    return out.value


class Batch:
    """Many independent Euler problems advanced together (one packed state buffer)."""

    def __init__(self, problems, dtype=torch.float64, cfl=0.5, gamma=1.4, scheme=TENO7X, alpha_mode=0, eps=None,
                 ct=1e-5, C=1.0, q=6, characteristic=1):
        n = len(problems)
        grids = (Grid * n)()
        for k, pr in enumerate(problems):
            grids[k] = Grid(pr.sys, pr.nx, pr.ny, pr.bc_x, pr.bc_y, F64 if dtype == torch.float64 else F32,
                            pr.x0, pr.x1, pr.y0, pr.y1)
        o = make_opts(scheme=scheme, alpha_mode=alpha_mode, eps=eps, gamma=gamma, ct=ct, cfl=cfl, C=C, q=q,
                      characteristic=characteristic)
        self.dtype = dtype
        self.problems = problems
        self._stream_val = torch.cuda.current_stream().cuda_stream
        h = ctypes.c_void_p()
        _check(lib().teno_batch_create(grids, n, ctypes.byref(o), _stream(), ctypes.byref(h)), "teno_batch_create")
        self._h = h
        self.total = lib().teno_batch_total_elems(h)
        self.offsets = [lib().teno_batch_offset(h, k) for k in range(n)]

    def pack(self, states):
        buf = torch.empty(self.total, dtype=self.dtype, device="cuda")
        for off, U in zip(self.offsets, states):
            buf[off:off + U.numel()] = U.reshape(-1).to(device="cuda", dtype=self.dtype)
        return buf

    def unpack(self, buf, k):
        pr = self.problems[k]
        nv = NVAR[pr.sys]
        off = self.offsets[k]
        return buf[off:off + nv * pr.ny * pr.nx].view(nv, pr.ny, pr.nx)

    def run(self, buf, nsteps, mode=0):
        if torch.cuda.current_stream().cuda_stream != self._stream_val:
            raise RuntimeError("a Batch runs on the stream it was created on")
        _buf(buf, (self.dtype,), self.total, "the packed batch state")
        _check(lib().teno_batch_run(self._h, _ptr(buf), int(nsteps), int(mode)), "teno_batch_run")
        return buf

    def set_shape(self, x_tile, y_tile, packed):
        """Fix mode 0's launch shape (4 or 8 segments per x-tile and columns per y-tile; packed
        ragged last segments or not) instead of the timing-based choice of the first run."""
        _check(lib().teno_batch_set_shape(self._h, int(x_tile), int(y_tile), int(packed)), "teno_batch_set_shape")

    def poll(self):
        _check(lib().teno_batch_poll(self._h), "batch device status")

    def close(self):
        if getattr(self, "_h", None):
            lib().teno_batch_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
