"""Seeded synthetic inputs shaped like the paper's test problems.

This module only builds initial states (and their problem parameters). It contains none of the
scheme's arithmetic, so both the GPU path and the CPU oracle consume the very same bits from it.
Random numbers come from numpy's PCG64 seeded generator; every state is float64 [nvar, ny, nx]
with ny = 1 for one-dimensional problems, conserved variables (rho, rho u, [rho v], E).

Shapes follow the paper: a smooth periodic advection wave (section "One-dimensional linear
advection problem"), a shock tube with a sinusoidal density perturbation (Shu-Osher-like,
section "Shock wave-entropy wave interaction"), and a two-dimensional four-quadrant Riemann state
with a vortex (two dimensions are not in the paper; the state combines its two ingredients,
discontinuities and smooth structure).
"""
from dataclasses import dataclass, field
import math

import numpy as np

ADV1D, EULER1D, EULER2D, BURGERS1D = 0, 1, 2, 3
PERIODIC, OUTFLOW = 0, 1
GAMMA = 1.4


@dataclass
class Problem:
    """A problem instance: system, grid, boundary conditions, time-step rule and initial state."""
    name: str
    sys: int
    nx: int
    ny: int
    x0: float
    x1: float
    y0: float
    y1: float
    bc_x: int
    bc_y: int
    U0: np.ndarray
    cfl: float = 0.5
    dt: float = 0.0            # > 0: fixed step; 0: CFL rule
    nsteps: int = 1
    gamma: float = GAMMA
    meta: dict = field(default_factory=dict)

    @property
    def dx(self):
        return (self.x1 - self.x0) / self.nx

    @property
    def dy(self):
        return (self.y1 - self.y0) / self.ny

    @property
    def ncells(self):
        return self.nx * self.ny


def cell_centres(x0, x1, n):
    dx = (x1 - x0) / n
    return x0 + (np.arange(n) + 0.5) * dx


def conserved_1d(rho, u, p, gamma=GAMMA):
    return np.stack([rho, rho * u, p / (gamma - 1.0) + 0.5 * rho * u * u])[:, None, :]


def conserved_2d(rho, u, v, p, gamma=GAMMA):
    return np.stack([rho, rho * u, rho * v, p / (gamma - 1.0) + 0.5 * rho * (u * u + v * v)])


# ------------------------------------------------------------------------------------------------
# Linear advection: u_t + u_x = 0 on [-1, 1), periodic, u0 = sin(pi x) + 0.3 sin(3 pi x + phi).
# ------------------------------------------------------------------------------------------------
def advection_wave(x, phi):
    return np.sin(np.pi * x) + 0.3 * np.sin(3.0 * np.pi * x + phi)


def advection(seed, n, cfl=0.2, t_end=2.0):
    rng = np.random.Generator(np.random.PCG64(seed))
    phi = float(rng.uniform(0.0, 2.0 * math.pi))
    x = cell_centres(-1.0, 1.0, n)
    U0 = advection_wave(x, phi)[None, None, :].astype(np.float64)
    dx = 2.0 / n
    dt = cfl * dx
    nsteps = int(round(t_end / dt))
    return Problem("advection", ADV1D, n, 1, -1.0, 1.0, 0.0, 1.0, PERIODIC, PERIODIC, U0,
                   cfl=cfl, dt=dt, nsteps=nsteps, meta=dict(phi=phi, t_end=t_end))


def advection_exact(problem, t):
    x = cell_centres(problem.x0, problem.x1, problem.nx)
    xs = (x - t - problem.x0) % (problem.x1 - problem.x0) + problem.x0
    return advection_wave(xs, problem.meta["phi"])


# ------------------------------------------------------------------------------------------------
# The paper's own linear-advection data (section "Linear advection"): u1, a Gaussian on [0, 1); u2 =
# sin(pi x)^3 on [0, 2); u3, the four-wave profile on [-1, 1). As printed, u3's pieces lie on
# [0.2, 1.6], partly outside the domain and away from their own centres; they are taken 1 to the left
# ([-0.8, -0.6] around z = -0.7, [-0.4, -0.2], [0, 0.2], [0.4, 0.6]), which puts each stated centre
# (z, 0.1, a = 0.5) inside its piece.
# ------------------------------------------------------------------------------------------------
_U3_DELTA = 0.005
_U3_ALPHA = 10.0
_U3_BETA = math.log(2.0) / (36.0 * _U3_DELTA * _U3_DELTA)


def _u3(x):
    d, al, be = _U3_DELTA, _U3_ALPHA, _U3_BETA
    z, a = -0.7, 0.5
    g = lambda c: np.exp(-be * (x - c) ** 2)
    f = lambda c: np.sqrt(np.maximum(1.0 - al * al * (x - c) ** 2, 0.0))
    u = np.zeros_like(x)
    m = (x >= -0.8) & (x <= -0.6)
    u[m] = ((g(z - d) + g(z + d) + 4.0 * g(z)) / 6.0)[m]
    u[(x >= -0.4) & (x <= -0.2)] = 1.0
    m = (x >= 0.0) & (x <= 0.2)
    u[m] = (1.0 - np.abs(10.0 * (x - 0.1)))[m]
    m = (x >= 0.4) & (x <= 0.6)
    u[m] = ((f(a - d) + f(a + d) + 4.0 * f(a)) / 6.0)[m]
    return u


PAPER_ADVECTION = {
    "u1": (0.0, 1.0, lambda x: np.exp(-300.0 * (x - 0.5) ** 2)),
    "u2": (0.0, 2.0, lambda x: np.sin(np.pi * x) ** 3),
    "u3": (-1.0, 1.0, _u3),
}


def paper_advection(kind, n, cfl=0.2, periods=1):
    """u_t + u_x = 0, periodic, with the paper's initial data `kind`, run for whole periods at a fixed
    dt = cfl dx (the exact solution is then the initial data)."""
    x0, x1, fn = PAPER_ADVECTION[kind]
    x = cell_centres(x0, x1, n)
    U0 = fn(x)[None, None, :].astype(np.float64)
    dx = (x1 - x0) / n
    dt = cfl * dx
    nsteps = int(round(periods * (x1 - x0) / dt))
    return Problem(f"advection_{kind}", ADV1D, n, 1, x0, x1, 0.0, 1.0, PERIODIC, PERIODIC, U0,
                   cfl=cfl, dt=dt, nsteps=nsteps, meta=dict(t_end=nsteps * dt))


# ------------------------------------------------------------------------------------------------
# Inviscid Burgers: u_t + (u^2/2)_x = 0 on [0, 2), periodic, u0 = 1/2 + sin(pi (x - shift)) (the
# paper's case at shift = 0; smooth until t = 1/pi, then a shock forms).
# ------------------------------------------------------------------------------------------------
def burgers_wave(x, shift=0.0):
    return 0.5 + np.sin(np.pi * (x - shift))


def burgers(n, cfl=0.5, t_end=0.5 / math.pi, shift=0.0):
    x = cell_centres(0.0, 2.0, n)
    U0 = burgers_wave(x, shift)[None, None, :].astype(np.float64)
    return Problem("burgers", BURGERS1D, n, 1, 0.0, 2.0, 0.0, 1.0, PERIODIC, PERIODIC, U0, cfl=cfl,
                   meta=dict(t_end=t_end, shift=shift))


def burgers_exact(problem, t, iters=60):
    """Smooth solution (t < 1/pi) by characteristics: u = u0(x - u t), solved by Newton's method
    started from u0(x) (the map is a contraction-free monotone root problem for t < 1/pi)."""
    x = cell_centres(problem.x0, problem.x1, problem.nx)
    shift = problem.meta.get("shift", 0.0)
    u = burgers_wave(x, shift)
    for _ in range(iters):
        ph = np.pi * (x - u * t - shift)
        g = u - 0.5 - np.sin(ph)
        dg = 1.0 + np.pi * t * np.cos(ph)
        u = u - g / dg
    return u


# ------------------------------------------------------------------------------------------------
# One-dimensional Euler: Riemann state with a sinusoidal density perturbation on the right.
# [0, 10], interface at x = 1, outflow boundaries.
# ------------------------------------------------------------------------------------------------
def euler1d(seed, n=4096, cfl=0.5, nsteps=2000):
    rng = np.random.Generator(np.random.PCG64(seed))
    rhoL, pL = rng.uniform(0.1, 2.0, size=2)
    rhoR, pR = rng.uniform(0.1, 2.0, size=2)
    uL, uR = rng.uniform(-1.0, 1.0, size=2)
    k = int(rng.integers(3, 11))
    x = cell_centres(0.0, 10.0, n)
    left = x <= 1.0
    rho = np.where(left, rhoL, rhoR * (1.0 + 0.2 * np.sin(k * x)))
    u = np.where(left, uL, uR)
    p = np.where(left, pL, pR)
    U0 = conserved_1d(rho, u, p)
    return Problem("euler1d", EULER1D, n, 1, 0.0, 10.0, 0.0, 1.0, OUTFLOW, OUTFLOW, U0,
                   cfl=cfl, nsteps=nsteps,
                   meta=dict(rhoL=rhoL, pL=pL, uL=uL, rhoR=rhoR, pR=pR, uR=uR, k=k))


# ------------------------------------------------------------------------------------------------
# Two-dimensional Euler: four-quadrant Riemann state plus an isentropic vortex, periodic [0,1]^2.
# ------------------------------------------------------------------------------------------------
def euler2d(seed, n=4096, ny=None, cfl=0.5, nsteps=100):
    ny = n if ny is None else ny
    rng = np.random.Generator(np.random.PCG64(seed))
    rho_q = rng.uniform(0.1, 1.5, size=4)
    p_q = rng.uniform(0.1, 1.5, size=4)
    u_q = rng.uniform(-1.0, 1.0, size=4)
    v_q = rng.uniform(-1.0, 1.0, size=4)
    xc, yc = rng.uniform(0.0, 1.0, size=2)
    g = GAMMA
    T_q = p_q / rho_q
    T_min = float(T_q.min())
    s_max = math.sqrt(0.5 * T_min * 8.0 * g * math.pi ** 2 / ((g - 1.0) * math.e))
    s = float(rng.uniform(0.5, 1.0)) * s_max
    r0 = 0.05

    x = cell_centres(0.0, 1.0, n)
    y = cell_centres(0.0, 1.0, ny)
    X, Y = np.meshgrid(x, y)                     # [ny, nx]
    q = (X >= 0.5).astype(int) + 2 * (Y >= 0.5).astype(int)
    rho0, p0, u0, v0, T0 = rho_q[q], p_q[q], u_q[q], v_q[q], T_q[q]
    dxv = (X - xc + 0.5) % 1.0 - 0.5             # minimum image
    dyv = (Y - yc + 0.5) % 1.0 - 0.5
    xt, yt = dxv / r0, dyv / r0
    r2 = xt * xt + yt * yt
    e1 = np.exp(0.5 * (1.0 - r2))
    du = -(s / (2.0 * math.pi)) * e1 * yt
    dv = (s / (2.0 * math.pi)) * e1 * xt
    dT = -(g - 1.0) * s * s * np.exp(1.0 - r2) / (8.0 * g * math.pi ** 2)
    T = T0 + dT
    rho = rho0 * (T / T0) ** (1.0 / (g - 1.0))
    p = rho * T
    U0 = conserved_2d(rho, u0 + du, v0 + dv, p)
    return Problem("euler2d", EULER2D, n, ny, 0.0, 1.0, 0.0, 1.0, PERIODIC, PERIODIC, U0,
                   cfl=cfl, nsteps=nsteps,
                   meta=dict(rho_q=rho_q, p_q=p_q, u_q=u_q, v_q=v_q, centre=(xc, yc), strength=s))


# ------------------------------------------------------------------------------------------------
# Batched mixture: 1D instances with N log-uniform in [256, 65536] and 2D squares with side
# log-uniform in [64, 1024]; each instance seeded from the batch seed.
# ------------------------------------------------------------------------------------------------
def batch_sizes(seed, n1d=256, n2d=256, lo1=256, hi1=65536, lo2=64, hi2=1024):
    rng = np.random.Generator(np.random.PCG64(seed))
    s1 = np.rint(np.exp(rng.uniform(math.log(lo1), math.log(hi1), size=n1d))).astype(int)
    s2 = np.rint(np.exp(rng.uniform(math.log(lo2), math.log(hi2), size=n2d))).astype(int)
    return [int(v) for v in s1], [int(v) for v in s2]


def batch(seed, n1d=256, n2d=256, lo1=256, hi1=65536, lo2=64, hi2=1024, nsteps=20):
    s1, s2 = batch_sizes(seed, n1d, n2d, lo1, hi1, lo2, hi2)
    probs = []
    for k, n in enumerate(s1):
        probs.append(euler1d(seed * 100003 + k, n=n, nsteps=nsteps))
    for k, n in enumerate(s2):
        probs.append(euler2d(seed * 100003 + 50000 + k, n=n, nsteps=nsteps))
    return probs


# ------------------------------------------------------------------------------------------------
# Adjoint target: a smooth density field rho*(x, y) = 1 + 0.2 sum_q A_q sin(2 pi (m_q x + n_q y) + psi_q).
# ------------------------------------------------------------------------------------------------
def density_target(seed, n, ny=None):
    ny = n if ny is None else ny
    rng = np.random.Generator(np.random.PCG64(seed))
    A = rng.uniform(0.0, 1.0, size=3)
    m = rng.integers(1, 5, size=3)
    k = rng.integers(1, 5, size=3)
    psi = rng.uniform(0.0, 2.0 * math.pi, size=3)
    x = cell_centres(0.0, 1.0, n)
    y = cell_centres(0.0, 1.0, ny)
    X, Y = np.meshgrid(x, y)
    t = np.ones_like(X)
    for qq in range(3):
        t = t + 0.2 * A[qq] * np.sin(2.0 * math.pi * (m[qq] * X + k[qq] * Y) + psi[qq])
    return t


def random_directions(seed, U0, count):
    """Gaussian directions scaled per conserved variable by the RMS of that variable."""
    rng = np.random.Generator(np.random.PCG64(seed))
    scale = np.sqrt(np.mean(U0 * U0, axis=tuple(range(1, U0.ndim)), keepdims=True))
    return [rng.standard_normal(U0.shape) * scale for _ in range(count)]


# ------------------------------------------------------------------------------------------------
# The paper's one-dimensional shock tubes (section "Isolated wave structure") and its shock /
# entropy-wave cases (Shu-Osher on 200 cells, Titarev-Toro on 400; domain [0, 10]).
# ------------------------------------------------------------------------------------------------
def vortex(n, cfl=0.5, strength=5.0, length=10.0):
    """Isentropic vortex in a uniform stream (rho, u, v, p) = (1, 1, 1, 1) on the periodic
    [0, length]^2, centred in it: an exact solution of the 2D Euler equations that translates with the
    stream. Point values at cell centres. (The periodic data take the nearest image of the centre; on
    [0, 10]^2 the vortex's tail at the seams is of order 1e-5, on [0, 20]^2 below 1e-20.)"""
    x = cell_centres(0.0, length, n)
    X, Y = np.meshgrid(x, x)
    rho, u, v, p = vortex_exact_primitive(X, Y, 0.0, strength, length=length)
    return Problem("vortex", EULER2D, n, n, 0.0, length, 0.0, length, PERIODIC, PERIODIC,
                   conserved_2d(rho, u, v, p), cfl=cfl, meta=dict(strength=strength, length=length))


def vortex_exact_primitive(X, Y, t, strength=5.0, gamma=GAMMA, length=10.0):
    """(rho, u, v, p) of the translating vortex at time t (nearest periodic image of the centre)."""
    h = 0.5 * length
    xc, yc = h + t, h + t
    dx = (X - xc + h) % length - h
    dy = (Y - yc + h) % length - h
    r2 = dx * dx + dy * dy
    e1 = np.exp(0.5 * (1.0 - r2))
    u = 1.0 - strength / (2.0 * math.pi) * e1 * dy
    v = 1.0 + strength / (2.0 * math.pi) * e1 * dx
    T = 1.0 - (gamma - 1.0) * strength ** 2 * np.exp(1.0 - r2) / (8.0 * gamma * math.pi ** 2)
    rho = T ** (1.0 / (gamma - 1.0))
    return rho, u, v, rho * T


def shock_tube(kind, n=200):
    x = cell_centres(0.0, 1.0, n) if kind in ("sod", "lax") else cell_centres(0.0, 10.0, n)
    if kind == "sod":
        left = x <= 0.5
        rho = np.where(left, 1.0, 0.125); u = np.zeros_like(x); p = np.where(left, 1.0, 0.1)
        t_end, x1 = 0.2, 1.0
    elif kind == "lax":
        left = x <= 0.5
        rho = np.where(left, 0.445, 0.5); u = np.where(left, 0.698, 0.0); p = np.where(left, 3.528, 0.571)
        t_end, x1 = 0.14, 1.0
    elif kind == "shu_osher":
        left = x <= 1.0
        rho = np.where(left, 3.8571, 1.0 + 0.2 * np.sin(5.0 * x))
        u = np.where(left, 2.6294, 0.0); p = np.where(left, 10.3333, 1.0)
        t_end, x1 = 1.8, 10.0
    elif kind == "titarev_toro":
        left = x <= 0.5
        rho = np.where(left, 1.515695, 1.0 + 0.1 * np.sin(20.0 * np.pi * x))
        u = np.where(left, 0.523346, 0.0); p = np.where(left, 1.80500, 1.0)
        t_end, x1 = 5.0, 10.0
    else:
        raise ValueError(kind)
    return Problem(kind, EULER1D, n, 1, 0.0, x1, 0.0, 1.0, OUTFLOW, OUTFLOW, conserved_1d(rho, u, p),
                   cfl=0.6, meta=dict(t_end=t_end))


def colliding_streams(n=200, p0=1e-4):
    """Two cold streams meeting head on (periodic, unit density, velocity +1 on [0.25, 0.75) and -1
    elsewhere, pressure p0 far below the kinetic energy): a state that the scheme, which has no
    positivity limiter, drives to a negative pressure after some steps. Used to check that a failing
    step is detected and reported."""
    x = cell_centres(0.0, 1.0, n)
    u = np.where(np.abs(x - 0.5) < 0.25, 1.0, -1.0)
    rho = np.ones_like(x)
    p = np.full_like(x, p0)
    return Problem("colliding_streams", EULER1D, n, 1, 0.0, 1.0, 0.0, 1.0, PERIODIC, PERIODIC,
                   conserved_1d(rho, u, p), cfl=0.5)
