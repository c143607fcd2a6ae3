"""ctypes front end of the CPU oracle (test infrastructure only).

Only the test-suite, the package smoke check and the CPU-baseline leg of the benchmark import this
module. It knows nothing of the GPU package and the GPU package knows nothing of it.

States are numpy float64 arrays shaped [nvar, ny, nx] (ny = 1 for one-dimensional systems).
Face arrays: x-faces [.., ny, nx+1] and y-faces [.., ny+1, nx]; face f is the left face of cell f.
"""
import ctypes
import os
import threading
from concurrent.futures import ThreadPoolExecutor
from dataclasses import dataclass, replace

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
_LIB_PATH = os.path.join(HERE, "libteno_oracle.so")

ADV1D, EULER1D, EULER2D, BURGERS1D = 0, 1, 2, 3
TENO7X, TENO5 = 0, 1
PERIODIC, OUTFLOW = 0, 1
NVAR = {ADV1D: 1, EULER1D: 3, EULER2D: 4, BURGERS1D: 1}

E_ARG, E_NONFINITE, E_NONPHYSICAL, E_ALLOC = -1, -4, -5, -7


class OracleError(RuntimeError):
    def __init__(self, code, where):
        super().__init__(f"oracle {where} failed with status {code}")
        self.code = code


class _Cfg(ctypes.Structure):
    _fields_ = [("sys", ctypes.c_int32), ("nx", ctypes.c_int32), ("ny", ctypes.c_int32),
                ("bc_x", ctypes.c_int32), ("bc_y", ctypes.c_int32), ("scheme", ctypes.c_int32),
                ("alpha_mode", ctypes.c_int32), ("pad_", ctypes.c_int32),
                ("dx", ctypes.c_double), ("dy", ctypes.c_double), ("gamma", ctypes.c_double),
                ("ct", ctypes.c_double), ("eps_x", ctypes.c_double), ("eps_y", ctypes.c_double),
                ("adv_speed", ctypes.c_double), ("C", ctypes.c_double), ("q", ctypes.c_int32),
                ("characteristic", ctypes.c_int32)]


@dataclass
class Config:
    """Problem and scheme parameters of one operator instance."""
    sys: int
    nx: int
    ny: int = 1
    x0: float = 0.0
    x1: float = 1.0
    y0: float = 0.0
    y1: float = 1.0
    bc_x: int = PERIODIC
    bc_y: int = PERIODIC
    scheme: int = TENO7X
    alpha_mode: int = 0
    gamma: float = 1.4
    ct: float = 1e-5
    eps: float = None       # None: dx^3 per direction for TENO7X, 1e-40 for TENO5
    adv_speed: float = 1.0
    C: float = 1.0          # C and q of eq:TENO1 (the paper's values)
    q: int = 6
    characteristic: int = 1     # 0: reconstruct per conserved component (L = R = I)
    dx_: float = None       # cell widths given exactly (windows and strips cut from a larger grid)
    dy_: float = None

    @property
    def dx(self):
        return self.dx_ if self.dx_ is not None else (self.x1 - self.x0) / self.nx

    @property
    def dy(self):
        return self.dy_ if self.dy_ is not None else (self.y1 - self.y0) / self.ny

    @property
    def nvar(self):
        return NVAR[self.sys]

    @property
    def shape(self):
        return (self.nvar, self.ny, self.nx)

    def c(self):
        if self.eps is not None:
            ex = ey = float(self.eps)
        elif self.scheme == TENO5:
            ex = ey = 1e-40
        else:
            ex, ey = self.dx ** 3, self.dy ** 3
        return _Cfg(self.sys, self.nx, self.ny, self.bc_x, self.bc_y, self.scheme, self.alpha_mode, 0,
                    self.dx, self.dy, self.gamma, self.ct, ex, ey, self.adv_speed, self.C, self.q,
                    self.characteristic)

    @property
    def nfaces_x(self):
        return self.ny * (self.nx + 1)

    @property
    def nfaces_y(self):
        return (self.ny + 1) * self.nx if self.sys == EULER2D else 0

    @property
    def nfaces(self):
        return self.nfaces_x + self.nfaces_y


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB_PATH):
            from . import build_oracle
            build_oracle.build()
        L = ctypes.CDLL(_LIB_PATH)
        P = ctypes.c_void_p
        C = ctypes.POINTER(_Cfg)
        L.orc_tables.argtypes = [P, P]
        L.orc_select7.argtypes = [ctypes.c_int]
        L.orc_select7.restype = ctypes.c_int
        L.orc_flags5_api.argtypes = [P, ctypes.c_double, ctypes.c_double, ctypes.c_double, ctypes.c_int32, P, P, P]
        L.orc_recon_api.argtypes = [C, ctypes.c_int, P]
        L.orc_recon_api.restype = ctypes.c_double
        L.orc_table1_api.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_int, P]
        L.orc_table1_api.restype = ctypes.c_double
        L.orc_eigen_api.argtypes = [C, ctypes.c_int, P, P, P, P]
        L.orc_phys_flux_api.argtypes = [C, ctypes.c_int, P, P]
        L.orc_wave_speeds.argtypes = [C, P, P, P]
        L.orc_rhs.argtypes = [C, P, P, P, P, P, P, P, P, P, P, P, P]
        L.orc_rhs_frozen.argtypes = [C, P, P, P, P, P]
        L.orc_rhs_frozen_jvp.argtypes = [C, P, P, P, P, P, ctypes.c_double, P]
        L.orc_run.argtypes = [C, P, ctypes.c_int, ctypes.c_double, ctypes.c_double, P, P, P]
        L.orc_run_frozen.argtypes = [C, P, ctypes.c_int, P, P, P]
        L.orc_run_frozen_jvp.argtypes = [C, P, P, ctypes.c_int, P, P, P, ctypes.c_double, P]
        L.orc_rk3_combine.argtypes = [ctypes.c_int, ctypes.c_size_t, P, P, P, ctypes.c_double]
        _lib = L
    return _lib


def _p(a):
    return None if a is None else a.ctypes.data_as(ctypes.c_void_p)


def _f64(a, shape=None):
    a = np.ascontiguousarray(a, dtype=np.float64)
    if shape is not None:
        a = a.reshape(shape)
    return a


def _check(st, where):
    if st != 0:
        raise OracleError(st, where)


def tables():
    """(Table 2 as [13,7], Table 1 as [7,5]) in double precision."""
    t2 = np.zeros((13, 7))
    t1 = np.zeros((7, 5))
    lib().orc_tables(_p(t2), _p(t1))
    return t2, t1


def select7(pattern):
    """Table 3 lookup for the neighbour vector packed as 16a+8b+4c+2d+e; -1 means none."""
    return lib().orc_select7(int(pattern))


def flags5(f5, eps, ct=1e-5, want_beta=False, C=1.0, q=6):
    """Cut-off flags (delta0..2) and chi of one five-point stencil given in upwind order."""
    f5 = _f64(f5)
    d = np.zeros(3, dtype=np.int32)
    chi = np.zeros(3)
    beta = np.zeros(3)
    lib().orc_flags5_api(_p(f5), float(eps), float(ct), float(C), int(q), _p(d), _p(chi), _p(beta))
    if want_beta:
        return d, chi, beta
    return d, chi


def recon(cfg, code, w7):
    w7 = _f64(w7)
    cc = cfg.c()
    return lib().orc_recon_api(ctypes.byref(cc), int(code), _p(w7))


def table1_apply(d0, d1, d2, f5):
    f5 = _f64(f5)
    return lib().orc_table1_api(int(d0), int(d1), int(d2), _p(f5))


def eigen(cfg, direction, UL, UR):
    UL = _f64(np.pad(np.asarray(UL, dtype=np.float64), (0, 4 - len(UL))))
    UR = _f64(np.pad(np.asarray(UR, dtype=np.float64), (0, 4 - len(UR))))
    Lm = np.zeros((4, 4))
    Rm = np.zeros((4, 4))
    cc = cfg.c()
    st = lib().orc_eigen_api(ctypes.byref(cc), int(direction), _p(UL), _p(UR), _p(Lm), _p(Rm))
    _check(st, "eigen")
    n = cfg.nvar
    return Lm[:n, :n].copy(), Rm[:n, :n].copy()


def phys_flux(cfg, direction, U):
    U = _f64(np.pad(np.asarray(U, dtype=np.float64), (0, 4 - len(U))))
    F = np.zeros(4)
    cc = cfg.c()
    lib().orc_phys_flux_api(ctypes.byref(cc), int(direction), _p(U), _p(F))
    return F[:cfg.nvar].copy()


def wave_speeds(cfg, U):
    """(alpha[8], cfl_den): per-field GLF constants (x fields, y fields) and max signal speed sum."""
    U = _f64(U, cfg.shape)
    a = np.zeros(8)
    den = np.zeros(1)
    cc = cfg.c()
    _check(lib().orc_wave_speeds(ctypes.byref(cc), _p(U), _p(a), _p(den)), "wave_speeds")
    return a, float(den[0])


def rhs(cfg, U, alpha=None, want_faces=False):
    """dU/dt of the full operator. With want_faces, also a dict with masks, flags, chi, face fluxes
    and the alphas used."""
    U = _f64(U, cfg.shape)
    out = np.zeros(cfg.shape)
    nv, nx, ny = cfg.nvar, cfg.nx, cfg.ny
    two_d = cfg.sys == EULER2D
    mx = np.zeros((ny, nx + 1), dtype=np.uint32)
    my = np.zeros((ny + 1, nx), dtype=np.uint32) if two_d else np.zeros(1, dtype=np.uint32)
    extra = {}
    fx = fy = cx = cy = Fx = Fy = None
    if want_faces:
        fx = np.zeros((ny, nx + 1), dtype=np.uint32)
        cx = np.zeros((ny, nx + 1, 24))
        Fx = np.zeros((nv, ny, nx + 1))
        if two_d:
            fy = np.zeros((ny + 1, nx), dtype=np.uint32)
            cy = np.zeros((ny + 1, nx, 24))
            Fy = np.zeros((nv, ny + 1, nx))
    a_in = None if alpha is None else _f64(alpha)
    a_out = np.zeros(8)
    cc = cfg.c()
    st = lib().orc_rhs(ctypes.byref(cc), _p(U), _p(a_in), _p(out), _p(mx), _p(my), _p(fx), _p(fy),
                       _p(cx), _p(cy), _p(Fx), _p(Fy), _p(a_out))
    _check(st, "rhs")
    if not want_faces:
        return out
    extra = dict(masks_x=mx, flags_x=fx, chi_x=cx, Fx=Fx, alpha=a_out)
    if two_d:
        extra.update(masks_y=my, flags_y=fy, chi_y=cy, Fy=Fy)
    return out, extra


def _masks_pair(cfg, masks_x, masks_y):
    mx = np.ascontiguousarray(masks_x, dtype=np.uint32)
    my = np.ascontiguousarray(masks_y if masks_y is not None else np.zeros(1), dtype=np.uint32)
    return mx, my


def rhs_frozen(cfg, U, alpha, masks_x, masks_y=None):
    U = _f64(U, cfg.shape)
    out = np.zeros(cfg.shape)
    mx, my = _masks_pair(cfg, masks_x, masks_y)
    a = _f64(alpha)
    cc = cfg.c()
    _check(lib().orc_rhs_frozen(ctypes.byref(cc), _p(U), _p(a), _p(mx), _p(my), _p(out)), "rhs_frozen")
    return out


def rhs_frozen_jvp(cfg, U, d, alpha, masks_x, masks_y=None, h=1e-20):
    U = _f64(U, cfg.shape)
    d = _f64(d, cfg.shape)
    out = np.zeros(cfg.shape)
    mx, my = _masks_pair(cfg, masks_x, masks_y)
    a = _f64(alpha)
    cc = cfg.c()
    st = lib().orc_rhs_frozen_jvp(ctypes.byref(cc), _p(U), _p(d), _p(a), _p(mx), _p(my), float(h), _p(out))
    _check(st, "rhs_frozen_jvp")
    return out


def run(cfg, U, nsteps, dt=0.0, cfl=0.5, record=False):
    """SSP-RK3 trajectory; returns the final state (and with record, the masks/alpha/dt)."""
    U = _f64(U, cfg.shape).copy()
    rm = ra = rd = None
    if record:
        rm = np.zeros((nsteps, 3, cfg.nfaces), dtype=np.uint32)
        ra = np.zeros((nsteps, 3, 8))
        rd = np.zeros(nsteps)
    cc = cfg.c()
    st = lib().orc_run(ctypes.byref(cc), _p(U), int(nsteps), float(dt), float(cfl), _p(rm), _p(ra), _p(rd))
    _check(st, "run")
    if record:
        return U, dict(masks=rm, alpha=ra, dt=rd)
    return U


def run_frozen(cfg, U, rec):
    U = _f64(U, cfg.shape).copy()
    n = len(rec["dt"])
    cc = cfg.c()
    st = lib().orc_run_frozen(ctypes.byref(cc), _p(U), n, _p(np.ascontiguousarray(rec["masks"])),
                              _p(np.ascontiguousarray(rec["alpha"])), _p(np.ascontiguousarray(rec["dt"])))
    _check(st, "run_frozen")
    return U


def run_frozen_jvp(cfg, U, d, rec, h=1e-20):
    U = _f64(U, cfg.shape)
    d = _f64(d, cfg.shape)
    out = np.zeros(cfg.shape)
    n = len(rec["dt"])
    cc = cfg.c()
    st = lib().orc_run_frozen_jvp(ctypes.byref(cc), _p(U), _p(d), n, _p(np.ascontiguousarray(rec["masks"])),
                                  _p(np.ascontiguousarray(rec["alpha"])), _p(np.ascontiguousarray(rec["dt"])),
                                  float(h), _p(out))
    _check(st, "run_frozen_jvp")
    return out


# ------------------------------------------------------------------------------------------------
# Drivers for large 2D states: the operator strip by strip in parallel threads, and one SSP-RK3 step
# stage by stage with every face's selection visible. Both only call the functions above in the
# order the oracle itself does, and are bitwise equal to rhs() and run() (tests/test_oracle_strips.py).
# ------------------------------------------------------------------------------------------------
HALO = 5    # a cell's derivative reads the cells within five of it along its row and column


def rk3_combine(stage, U0, Us, dU, dt):
    """In place: Us (the input of SSP-RK3 stage `stage`) becomes the stage's output, given dU = L(Us)."""
    for a in (U0, Us, dU):
        assert a.dtype == np.float64 and a.flags.c_contiguous and a.size == Us.size
    lib().orc_rk3_combine(int(stage), Us.size, _p(U0), _p(Us), _p(dU), float(dt))


def _strip(cfg, U, j0, j1):
    """Rows j0-HALO .. j1+HALO-1 of U (wrapped or clamped along y) and the matching configuration
    (outflow along y: the halo rows hold what a wider domain would give the strip's own rows)."""
    rows = np.arange(j0 - HALO, j1 + HALO)
    rows = rows % cfg.ny if cfg.bc_y == PERIODIC else np.clip(rows, 0, cfg.ny - 1)
    nr = len(rows)
    # (the cell widths, and with them eps = dx^3, dy^3, are the whole grid's exactly)
    sc = replace(cfg, ny=nr, y0=0.0, y1=1.0, bc_y=OUTFLOW, dx_=cfg.dx, dy_=cfg.dy)
    return sc, np.ascontiguousarray(U[:, rows, :])


def _strip_eval(cfg, U, alpha, j0, j1, want_faces):
    sc, Us = _strip(cfg, U, j0, j1)
    r = rhs(sc, Us, alpha=alpha, want_faces=want_faces)
    n = j1 - j0
    if not want_faces:
        return r[:, HALO:HALO + n, :], None
    d, ex = r
    fy = n + (1 if j1 == cfg.ny else 0)           # y-faces j0 .. j1-1 (and ny for the last strip)
    own = dict(masks_x=ex["masks_x"][HALO:HALO + n], flags_x=ex["flags_x"][HALO:HALO + n],
               chi_x=ex["chi_x"][HALO:HALO + n], Fx=ex["Fx"][:, HALO:HALO + n],
               masks_y=ex["masks_y"][HALO:HALO + fy], flags_y=ex["flags_y"][HALO:HALO + fy],
               chi_y=ex["chi_y"][HALO:HALO + fy], Fy=ex["Fy"][:, HALO:HALO + fy], alpha=ex["alpha"])
    return d[:, HALO:HALO + n, :], own


def rhs_strips(cfg, U, alpha, strip_rows=128, threads=1, on_faces=None):
    """The operator of a 2D Euler state evaluated strip by strip: rows [j0, j1) with HALO rows on
    either side, with the Lax-Friedrichs constants `alpha` of the whole state given. Bitwise equal to
    rhs(cfg, U, alpha). Strips run in `threads` threads (the library calls release the GIL).
    on_faces(j0, j1, faces): called in the calling thread, strip by strip, with the strip's own
    faces (x-faces of rows j0..j1-1, y-faces j0..j1-1 and, for the last strip, ny): masks, flags,
    chi, face fluxes."""
    assert cfg.sys == EULER2D
    U = _f64(U, cfg.shape)
    alpha = _f64(alpha)
    lib()
    tables()                                   # the coefficient tables set up before any thread
    out = np.empty(cfg.shape)
    spans = [(j, min(j + strip_rows, cfg.ny)) for j in range(0, cfg.ny, strip_rows)]
    want = on_faces is not None
    with ThreadPoolExecutor(max_workers=max(1, threads)) as ex:
        pending = []
        it = iter(spans)
        window = 2 * max(1, threads)           # results in flight (bounds the memory of face data)
        for sp in it:
            pending.append((sp, ex.submit(_strip_eval, cfg, U, alpha, sp[0], sp[1], want)))
            if len(pending) >= window:
                (a, b), fut = pending.pop(0)
                d, faces = fut.result()
                out[:, a:b] = d
                if want:
                    on_faces(a, b, faces)
        for (a, b), fut in pending:
            d, faces = fut.result()
            out[:, a:b] = d
            if want:
                on_faces(a, b, faces)
    return out


def step_stages(cfg, U, dt=0.0, cfl=0.5, strip_rows=None, threads=1, on_faces=None):
    """One SSP-RK3 step, stage by stage: each stage's Lax-Friedrichs constants from its own input
    (wave_speeds over the whole state), its operator (rhs, or rhs_strips for 2D Euler when
    strip_rows is given) and rk3_combine; dt > 0 is used as given, else cfl / the CFL denominator of
    U. on_faces(stage, j0, j1, faces) sees every face of every stage (faces as in rhs_strips; the
    whole domain at once without strips). Returns (U_new, dict(alpha=[3, 8], dt=dt)); bitwise equal
    to run(cfg, U, 1, dt, cfl)."""
    U0 = _f64(U, cfg.shape).copy()
    if not dt > 0.0:
        _, den = wave_speeds(cfg, U0)
        dt = cfl / den
    Us = U0.copy()
    alphas = np.zeros((3, 8))
    for stage in range(3):
        a, _ = wave_speeds(cfg, Us)
        alphas[stage] = a
        if strip_rows is not None:
            cb = None if on_faces is None else (lambda j0, j1, f, s=stage: on_faces(s, j0, j1, f))
            dU = rhs_strips(cfg, Us, a, strip_rows=strip_rows, threads=threads, on_faces=cb)
        elif on_faces is not None:
            dU, ex = rhs(cfg, Us, alpha=a, want_faces=True)
            on_faces(stage, 0, cfg.ny, ex)
        else:
            dU = rhs(cfg, Us, alpha=a)
        rk3_combine(stage, U0, Us, np.ascontiguousarray(dU), dt)
    return Us, dict(alpha=alphas, dt=dt)
