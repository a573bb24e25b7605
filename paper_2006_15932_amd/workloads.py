"""Seeded synthetic problem generators.

This module only describes problems: species parameters, grid, boundary
conditions, time step and the initial macroscopic fields n^sigma, u, T as FP64
host arrays.  It contains none of the model's arithmetic (no moments, no
equilibria, no update), so the GPU path and the CPU oracle can both consume the
same inputs without sharing any of the method's code.

Random numbers come from SplitMix64 (Steele, Lea and Flood, OOPSLA 2014):
state_k = seed + k * 0x9E3779B97F4A7C15, output = the published 64-bit mix of
state_k; a double in [0, 1) is the top 53 bits times 2^-53.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field, replace
from typing import Optional

import numpy as np

PERIODIC, OUTFLOW, WALL = 0, 1, 2
EULER, RK3 = 0, 1
LIM_MINMOD, LIM_NONE = 0, 1
FORCE_T_EXACT, FORCE_T_SAME = 0, 1

BASE_SEED = 15932
_GOLDEN = np.uint64(0x9E3779B97F4A7C15)


def splitmix64(seed: int, n: int) -> np.ndarray:
    """First ``n`` SplitMix64 outputs of ``seed`` as doubles in [0, 1)."""
    k = np.arange(1, n + 1, dtype=np.uint64)
    with np.errstate(over="ignore"):
        z = np.uint64(seed % (1 << 64)) + k * _GOLDEN
        z = (z ^ (z >> np.uint64(30))) * np.uint64(0xBF58476D1CE4E5B9)
        z = (z ^ (z >> np.uint64(27))) * np.uint64(0x94D049BB133111EB)
        z = z ^ (z >> np.uint64(31))
    return (z >> np.uint64(11)).astype(np.float64) * (2.0 ** -53)


class Stream:
    """Sequential draws from one SplitMix64 sequence."""

    def __init__(self, seed: int):
        self.seed, self.pos = seed, 0

    def uniform(self, n: int) -> np.ndarray:
        out = splitmix64(self.seed + self.pos * int(_GOLDEN), n) if n else np.zeros(0)
        self.pos += n
        return out


@dataclass
class Species:
    m: float                 # molar mass
    I: float = 3.0           # extra degrees of freedom
    tau: float = 2e-5        # relaxation time
    a: float = 0.0           # stoichiometric coefficient
    v: tuple = (1.5, 0.8, 2.2, 2.6)      # v_a, v_b, v_c, v_d
    eta: tuple = (2.5, 0.0, 0.0, 0.0)    # eta_a .. eta_d


@dataclass
class Problem:
    name: str
    nx: int
    ny: int
    species: list
    dx: float = 1e-3
    dy: float = 1e-3
    dt: float = 1e-5
    bc_x: int = PERIODIC
    bc_y: int = PERIODIC
    reaction: Optional[dict] = None      # fuel, oxid, k_ov, Ea_over_R, Q
    mechanism: Optional[list] = None     # steps: dict(fuel, oxid, k_ov, Ea_over_R, Q, a)
    accel: tuple = (0.0, 0.0)
    scheme: int = EULER
    limiter: int = LIM_MINMOD
    force_T_mode: int = FORCE_T_EXACT
    steps: int = 1
    precision: str = "fp64"
    n_sp: np.ndarray = field(default=None, repr=False)   # [S, ny, nx]
    ux: np.ndarray = field(default=None, repr=False)     # [ny, nx]
    uy: np.ndarray = field(default=None, repr=False)
    T: np.ndarray = field(default=None, repr=False)

    @property
    def S(self) -> int:
        return len(self.species)

    @property
    def cells(self) -> int:
        return self.nx * self.ny

    def with_(self, **kw) -> "Problem":
        return replace(self, **kw)


# Velocity-set parameters.  The paper asks for v near |u| and sqrt(D T/m) and
# eta near sqrt(I T/m); these multiples of s = sqrt(T_ref/m) keep every 16x16
# moment matrix well conditioned (no two groups with equal |v|^2 + eta^2).
V_UNIT = (1.5, 0.8, 2.2, 2.6)
ETA_UNIT = (2.5, 0.0, 0.0, 0.0)


def scaled_velocities(m: float, t_ref: float = 1.0, v_unit=V_UNIT, eta_unit=ETA_UNIT):
    s = math.sqrt(t_ref / m)
    return tuple(s * x for x in v_unit), tuple(s * x for x in eta_unit)


def make_species(m, I=3.0, tau=2e-5, a=0.0, t_ref=1.0, v_unit=V_UNIT, eta_unit=ETA_UNIT):
    v, eta = scaled_velocities(m, t_ref, v_unit, eta_unit)
    return Species(m=m, I=I, tau=tau, a=a, v=v, eta=eta)


def _centres(n):
    return np.arange(n, dtype=np.float64) + 0.5


# --------------------------------------------------------------------------
# C0: two-species Sod tube, 400 x 1, outflow in x, periodic in y.
# --------------------------------------------------------------------------
def sod(nx=400, steps=1000, scheme=EULER, precision="fp64") -> Problem:
    sp = [make_species(1.0), make_species(1.0)]
    x = _centres(nx) * 1e-3
    left = x < 0.2
    n_tot = np.where(left, 1.0, 0.125)
    T = np.where(left, 1.0, 0.8)
    n_sp = np.stack([0.5 * n_tot, 0.5 * n_tot])[:, None, :]
    return Problem("sod", nx, 1, sp, dt=1e-5, bc_x=OUTFLOW, bc_y=PERIODIC,
                   scheme=scheme, steps=steps, precision=precision, n_sp=n_sp,
                   ux=np.zeros((1, nx)), uy=np.zeros((1, nx)), T=T[None, :].copy())


# --------------------------------------------------------------------------
# C1: three-species reacting premix (2 F + O -> 2 P), hot Gaussian kernel.
# --------------------------------------------------------------------------
C1_CHEM = dict(fuel=0, oxid=1, k_ov=1e3, Ea_over_R=10.0, Q=0.0)


def reacting(n=256, ny=None, steps=5000, seed=BASE_SEED + 1, tau=2e-5, t_hot=3.0,
             scheme=EULER, precision="fp32", t_ref=1.0) -> Problem:
    nx, ny = n, (ny if ny is not None else n)
    sp = [make_species(2.0, tau=tau, a=-2.0, t_ref=t_ref),
          make_species(32.0, tau=tau, a=-1.0, t_ref=t_ref),
          make_species(18.0, tau=tau, a=2.0, t_ref=t_ref)]
    Y = np.array([1.0 / 9.0, 8.0 / 9.0, 0.0])
    u = Stream(seed).uniform(nx * ny).reshape(ny, nx)
    rho = 1.0 + 0.01 * (2.0 * u - 1.0)
    n_sp = np.stack([rho * Y[k] / sp[k].m for k in range(3)])
    xc, yc = np.meshgrid(_centres(nx) - nx / 2.0, _centres(ny) - ny / 2.0)
    T = 1.0 + (t_hot - 1.0) * np.exp(-(xc ** 2 + yc ** 2) / (2.0 * 10.0 ** 2))
    return Problem("reacting", nx, ny, sp, dt=1e-5, reaction=dict(C1_CHEM),
                   scheme=scheme, steps=steps, precision=precision, n_sp=n_sp,
                   ux=np.zeros((ny, nx)), uy=np.zeros((ny, nx)), T=T)


# --------------------------------------------------------------------------
# Two-step mechanism with the same overall chemistry as C1:
#   F + O -> I (intermediate, m = 34),  F + I -> 2 P  (2 F + O -> 2 P overall).
# --------------------------------------------------------------------------
TWO_STEP = [dict(fuel=0, oxid=1, k_ov=1e3, Ea_over_R=10.0, Q=5.0, a=(-1.0, -1.0, 1.0, 0.0)),
            dict(fuel=0, oxid=2, k_ov=5e3, Ea_over_R=8.0, Q=10.0, a=(-1.0, 0.0, -1.0, 2.0))]


def two_step(n=64, ny=None, steps=200, seed=BASE_SEED + 5, tau=2e-5, t_hot=3.5,
             scheme=EULER, precision="fp64", seed_intermediate=1e-3) -> Problem:
    """Premix of F and O with a little intermediate (mass fraction
    seed_intermediate), hot Gaussian kernel, periodic, as C1 otherwise."""
    nx, ny = n, (ny if ny is not None else n)
    sp = [make_species(2.0, tau=tau), make_species(32.0, tau=tau), make_species(34.0, tau=tau),
          make_species(18.0, tau=tau)]
    Y = np.array([1.0 / 9.0, 8.0 / 9.0 - seed_intermediate, seed_intermediate, 0.0])
    u = Stream(seed).uniform(nx * ny).reshape(ny, nx)
    rho = 1.0 + 0.01 * (2.0 * u - 1.0)
    n_sp = np.stack([rho * Y[k] / sp[k].m for k in range(4)])
    xc, yc = np.meshgrid(_centres(nx) - nx / 2.0, _centres(ny) - ny / 2.0)
    T = 1.0 + (t_hot - 1.0) * np.exp(-(xc ** 2 + yc ** 2) / (2.0 * 10.0 ** 2))
    return Problem("two_step", nx, ny, sp, dt=1e-5, mechanism=[dict(st) for st in TWO_STEP],
                   scheme=scheme, steps=steps, precision=precision, n_sp=n_sp,
                   ux=np.zeros((ny, nx)), uy=np.zeros((ny, nx)), T=T)


# --------------------------------------------------------------------------
# C2: four-species Rayleigh-Taylor: heavy (m=3) over light (m=1), two passive
# tracers, gravity (0, -0.1), periodic x, specular walls in y.
# --------------------------------------------------------------------------
def rayleigh_taylor(n=1024, ny=None, steps=20000, seed=BASE_SEED + 2, scheme=EULER,
                    precision="fp32") -> Problem:
    nx, ny = n, (ny if ny is not None else n)
    g = -0.1
    sp = [make_species(3.0), make_species(1.0), make_species(3.0), make_species(1.0)]
    ux_noise = Stream(seed).uniform(nx)
    xi = _centres(nx)
    y_int = ny / 2.0 + 0.005 * nx * (np.cos(2.0 * math.pi * xi / nx) + (2.0 * ux_noise - 1.0))
    yc = _centres(ny)[:, None]
    w_heavy = 0.5 * (1.0 + np.tanh((yc - y_int[None, :]) / 4.0))
    Y = np.stack([0.98 * w_heavy, 0.98 * (1.0 - w_heavy),
                  np.full((ny, nx), 0.01), np.full((ny, nx), 0.01)])
    inv_mbar = sum(Y[k] / sp[k].m for k in range(4))
    mbar = 1.0 / inv_mbar
    T = np.ones((ny, nx))
    # Hydrostatic column: d ln p / dy = mbar g / T, trapezoid rule on cell
    # centres, then shifted so that p = 1 at the interface of each column.
    dy = 1e-3
    integrand = mbar * g / T
    lnp = np.zeros((ny, nx))
    lnp[1:] = np.cumsum(0.5 * (integrand[1:] + integrand[:-1]) * dy, axis=0)
    for x in range(nx):
        lnp[:, x] -= np.interp(y_int[x], yc[:, 0], lnp[:, x])
    p = np.exp(lnp)
    n_tot = p / T
    rho = n_tot * mbar
    n_sp = np.stack([rho * Y[k] / sp[k].m for k in range(4)])
    return Problem("rayleigh_taylor", nx, ny, sp, dt=1e-5, bc_x=PERIODIC, bc_y=WALL,
                   accel=(0.0, g), scheme=scheme, steps=steps, precision=precision,
                   n_sp=n_sp, ux=np.zeros((ny, nx)), uy=np.zeros((ny, nx)), T=T)


# --------------------------------------------------------------------------
# C3: a batch of independent reacting instances of uneven size.
# --------------------------------------------------------------------------
def batch(count=64, sizes=(64, 128, 256, 512), steps=2000, seed=BASE_SEED + 3,
          scheme=EULER, precision="fp32") -> list:
    st = Stream(seed)
    pick = st.uniform(count)
    taus = st.uniform(count)
    hots = st.uniform(count)
    out = []
    for k in range(count):
        n = sizes[min(int(pick[k] * len(sizes)), len(sizes) - 1)]
        tau = 1e-5 + 4e-5 * taus[k]
        t_hot = 2.0 + 2.0 * hots[k]
        p = reacting(n=n, steps=steps, seed=seed * 1000 + k + 1, tau=tau, t_hot=t_hot,
                     scheme=scheme, precision=precision)
        p.name = "batch[%d]" % k
        out.append(p)
    return out


# --------------------------------------------------------------------------
# C4: four reacting species (C1 chemistry + inert diluent m=28), periodic
# double shear layer u_x = +-1.5, tanh width 8 cells, +-1% transverse noise.
# --------------------------------------------------------------------------
# Velocity parameters for the supersonic layer, absolute (not scaled by m):
# the paper places v near |u| and near sqrt(D T/m); one group sits near |u|.
C4_V = (1.0, 0.7, 2.0, 1.6)


def shear_layer(n=4096, ny=None, steps=5000, seed=BASE_SEED + 4, scheme=EULER,
                precision="fp32", u0=1.5) -> Problem:
    nx, ny = n, (ny if ny is not None else n)
    ms = (2.0, 32.0, 18.0, 28.0)
    sp = []
    for k, m in enumerate(ms):
        eta_a = 2.0 * math.sqrt(3.0 / m) + 0.5
        sp.append(Species(m=m, I=3.0, tau=2e-5, a=(-2.0, -1.0, 2.0, 0.0)[k], v=C4_V,
                          eta=(eta_a, 0.0, 0.0, 0.0)))
    Y = np.array([0.3 / 9.0, 0.3 * 8.0 / 9.0, 0.0, 0.7])
    yc = _centres(ny)[:, None] * np.ones((1, nx))
    L = float(ny)
    ux = u0 * (np.tanh((yc - L / 4.0) / 8.0) - np.tanh((yc - 3.0 * L / 4.0) / 8.0) - 1.0)
    uy = 0.01 * u0 * (2.0 * Stream(seed).uniform(nx * ny).reshape(ny, nx) - 1.0)
    rho = np.ones((ny, nx))
    n_sp = np.stack([rho * Y[k] / ms[k] for k in range(4)])
    return Problem("shear_layer", nx, ny, sp, dt=1e-5, reaction=dict(C1_CHEM),
                   scheme=scheme, steps=steps, precision=precision, n_sp=n_sp,
                   ux=ux, uy=uy, T=np.ones((ny, nx)))


def fields(p: Problem):
    """The four initial field arrays, contiguous float64."""
    return (np.ascontiguousarray(p.n_sp, dtype=np.float64),
            np.ascontiguousarray(p.ux, dtype=np.float64),
            np.ascontiguousarray(p.uy, dtype=np.float64),
            np.ascontiguousarray(p.T, dtype=np.float64))


def window(p: Problem, x0: int, y0: int, w: int) -> Problem:
    """A w x w window of ``p``'s initial fields centred on (x0, y0), wrapping
    periodically, with outflow boundaries.  Its centre evolves exactly as the
    full periodic problem for (w//2 - 1)//2 steps of the 5-point-wide stencil."""
    h = w // 2
    xs = (np.arange(x0 - h, x0 - h + w)) % p.nx
    ys = (np.arange(y0 - h, y0 - h + w)) % p.ny
    sel = np.ix_(ys, xs)
    n_sp = np.stack([p.n_sp[k][sel] for k in range(p.S)])
    return p.with_(name=p.name + "-window", nx=w, ny=w, bc_x=OUTFLOW, bc_y=OUTFLOW,
                   n_sp=n_sp, ux=p.ux[sel].copy(), uy=p.uy[sel].copy(), T=p.T[sel].copy())
