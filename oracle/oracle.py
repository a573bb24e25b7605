"""ctypes front end of the FP64 CPU oracle (``dbm_oracle.c``).

TEST INFRASTRUCTURE ONLY: imported by ``tests/``, by the package smoke check and
by the CPU-baseline leg of ``bench.py``.  The GPU library never imports it, and
it imports nothing from the GPU package except the problem description passed
in by the caller (plain numbers and arrays).

Every array is float64, row-major with x fastest:
``f`` is ``[S, 16, ny, nx]``, scalar fields ``[ny, nx]``, species fields
``[S, ny, nx]``.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "dbm_oracle.c")
LIB = os.path.join(HERE, "liboracle.so")

NV = 16
ERRORS = {-1: "bad argument", -2: "singular moment matrix", -5: "unsupported"}


def build(force: bool = True) -> str:
    """Compile the oracle with gcc (FP64, no contraction, OpenMP)."""
    if not force and os.path.exists(LIB) and os.path.getmtime(LIB) >= os.path.getmtime(SRC):
        return LIB
    tmp = LIB + ".tmp%d" % os.getpid()
    cmd = ["gcc", "-O2", "-std=c11", "-ffp-contract=off", "-fno-fast-math", "-fopenmp",
           "-fPIC", "-shared", "-Wall", "-o", tmp, SRC, "-lm"]
    subprocess.run(cmd, check=True)
    os.replace(tmp, LIB)
    return LIB


class OrSpecies(ctypes.Structure):
    _fields_ = [("m", ctypes.c_double), ("I", ctypes.c_double), ("tau", ctypes.c_double),
                ("a", ctypes.c_double), ("v", ctypes.c_double * 4),
                ("eta", ctypes.c_double * 4)]


class OrReactionStep(ctypes.Structure):
    _fields_ = [("fuel", ctypes.c_int), ("oxid", ctypes.c_int), ("k", ctypes.c_double),
                ("Ea_over_R", ctypes.c_double), ("Q", ctypes.c_double),
                ("a", ctypes.c_double * 16)]


class OrConfig(ctypes.Structure):
    _fields_ = [("nx", ctypes.c_int), ("ny", ctypes.c_int), ("dx", ctypes.c_double),
                ("dy", ctypes.c_double), ("dt", ctypes.c_double), ("bc_x", ctypes.c_int),
                ("bc_y", ctypes.c_int), ("S", ctypes.c_int),
                ("sp", ctypes.POINTER(OrSpecies)), ("reaction_on", ctypes.c_int),
                ("fuel", ctypes.c_int), ("oxid", ctypes.c_int), ("k_ov", ctypes.c_double),
                ("Ea_over_R", ctypes.c_double), ("Q", ctypes.c_double),
                ("ax", ctypes.c_double), ("ay", ctypes.c_double), ("scheme", ctypes.c_int),
                ("limiter", ctypes.c_int), ("force_T_mode", ctypes.c_int),
                ("nchem", ctypes.c_int), ("chem", ctypes.POINTER(OrReactionStep))]


_lib = None
_dp = ctypes.POINTER(ctypes.c_double)


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB) or os.path.getmtime(LIB) < os.path.getmtime(SRC):
            build()
        L = ctypes.CDLL(LIB)
        L.or_create.argtypes = [ctypes.POINTER(OrConfig), ctypes.POINTER(ctypes.c_void_p)]
        L.or_destroy.argtypes = [ctypes.c_void_p]
        L.or_set_threads.argtypes = [ctypes.c_int]
        L.or_get_threads.restype = ctypes.c_int
        L.or_tables.argtypes = [ctypes.c_void_p, ctypes.c_int] + [_dp] * 5
        L.or_fhat.argtypes = [ctypes.c_double] * 5 + [_dp]
        L.or_fhat.restype = None
        L.or_feq.argtypes = [ctypes.c_void_p, ctypes.c_int] + [ctypes.c_double] * 4 + [_dp]
        L.or_cell_source.argtypes = [ctypes.c_void_p, _dp, _dp]
        L.or_init_equilibrium.argtypes = [ctypes.c_void_p] + [_dp] * 5
        L.or_rhs.argtypes = [ctypes.c_void_p, _dp, _dp]
        L.or_run.argtypes = [ctypes.c_void_p, _dp, ctypes.c_int]
        L.or_moments.argtypes = [ctypes.c_void_p] + [_dp] * 5
        L.or_noneq.argtypes = [ctypes.c_void_p, _dp, _dp, _dp]
        L.or_energy.argtypes = [ctypes.c_void_p, _dp, _dp, _dp]
        _lib = L
    return _lib


def _ptr(a):
    if a is None:
        return None
    assert a.dtype == np.float64 and a.flags["C_CONTIGUOUS"]
    return a.ctypes.data_as(_dp)


def set_threads(n: int) -> None:
    lib().or_set_threads(int(n))


def get_threads() -> int:
    return int(lib().or_get_threads())


def fhat(n, ux, uy, theta, I):
    """The 16 equilibrium moments (closed forms listed after Eq.(14))."""
    h = np.zeros(NV)
    lib().or_fhat(n, ux, uy, theta, I, _ptr(h))
    return h


class OracleError(RuntimeError):
    def __init__(self, code):
        super().__init__("oracle error %d (%s)" % (code, ERRORS.get(code, "?")))
        self.code = code


class Oracle:
    """One problem instance.  ``prob`` is a ``workloads.Problem``-like object
    (attributes nx, ny, dx, dy, dt, bc_x, bc_y, species, reaction, accel,
    scheme, limiter, force_T_mode)."""

    def __init__(self, prob):
        self.prob = prob
        S = len(prob.species)
        self.S = S
        self._sp = (OrSpecies * S)()
        for k, s in enumerate(prob.species):
            self._sp[k].m, self._sp[k].I, self._sp[k].tau, self._sp[k].a = s.m, s.I, s.tau, s.a
            for g in range(4):
                self._sp[k].v[g] = s.v[g]
                self._sp[k].eta[g] = s.eta[g]
        c = OrConfig()
        c.nx, c.ny, c.dx, c.dy, c.dt = prob.nx, prob.ny, prob.dx, prob.dy, prob.dt
        c.bc_x, c.bc_y, c.S = prob.bc_x, prob.bc_y, S
        c.sp = ctypes.cast(self._sp, ctypes.POINTER(OrSpecies))
        r = prob.reaction
        if r is not None:
            c.reaction_on, c.fuel, c.oxid = 1, r["fuel"], r["oxid"]
            c.k_ov, c.Ea_over_R, c.Q = r["k_ov"], r["Ea_over_R"], r.get("Q", 0.0)
        mech = getattr(prob, "mechanism", None)
        if mech:
            steps = (OrReactionStep * len(mech))()
            for k, st in enumerate(mech):
                steps[k].fuel, steps[k].oxid = st["fuel"], st["oxid"]
                steps[k].k, steps[k].Ea_over_R, steps[k].Q = st["k_ov"], st["Ea_over_R"], st.get("Q", 0.0)
                for j, a in enumerate(st["a"]):
                    steps[k].a[j] = a
            c.nchem = len(mech)
            c.chem = ctypes.cast(steps, ctypes.POINTER(OrReactionStep))
            self._steps = steps
        c.ax, c.ay = prob.accel
        c.scheme, c.limiter, c.force_T_mode = prob.scheme, prob.limiter, prob.force_T_mode
        self._cfg = c
        h = ctypes.c_void_p()
        rc = lib().or_create(ctypes.byref(c), ctypes.byref(h))
        if rc != 0:
            raise OracleError(rc)
        self._h = h

    def __del__(self):
        h = getattr(self, "_h", None)
        if h is not None and h.value:
            lib().or_destroy(h)
            self._h = None

    @property
    def shape_f(self):
        return (self.S, NV, self.prob.ny, self.prob.nx)

    def tables(self, s):
        vx, vy, eta = np.zeros(NV), np.zeros(NV), np.zeros(NV)
        M, Minv = np.zeros((NV, NV)), np.zeros((NV, NV))
        self._check(lib().or_tables(self._h, s, _ptr(vx), _ptr(vy), _ptr(eta), _ptr(M), _ptr(Minv)))
        return vx, vy, eta, M, Minv

    def feq(self, s, n, ux, uy, T):
        out = np.zeros(NV)
        self._check(lib().or_feq(self._h, s, n, ux, uy, T, _ptr(out)))
        return out

    def cell_source(self, fc):
        fc = np.ascontiguousarray(fc, dtype=np.float64).reshape(self.S * NV)
        out = np.zeros_like(fc)
        self._check(lib().or_cell_source(self._h, _ptr(fc), _ptr(out)))
        return out.reshape(self.S, NV)

    def init_equilibrium(self, n_sp, ux, uy, T):
        p = self.prob
        n_sp = np.ascontiguousarray(n_sp, dtype=np.float64).reshape(self.S, p.ny, p.nx)
        ux, uy, T = (np.ascontiguousarray(a, dtype=np.float64).reshape(p.ny, p.nx)
                     for a in (ux, uy, T))
        f = np.zeros(self.shape_f)
        self._check(lib().or_init_equilibrium(self._h, _ptr(n_sp), _ptr(ux), _ptr(uy),
                                              _ptr(T), _ptr(f)))
        return f

    def rhs(self, f):
        f = np.ascontiguousarray(f, dtype=np.float64)
        L = np.zeros_like(f)
        self._check(lib().or_rhs(self._h, _ptr(f), _ptr(L)))
        return L

    def run(self, f, nsteps):
        """Advance a copy of ``f`` by ``nsteps`` steps and return it."""
        g = np.array(f, dtype=np.float64, order="C", copy=True)
        self._check(lib().or_run(self._h, _ptr(g), int(nsteps)))
        return g

    def moments(self, f):
        p = self.prob
        f = np.ascontiguousarray(f, dtype=np.float64)
        rho = np.zeros((self.S, p.ny, p.nx))
        ux, uy, T = np.zeros((p.ny, p.nx)), np.zeros((p.ny, p.nx)), np.zeros((p.ny, p.nx))
        self._check(lib().or_moments(self._h, _ptr(f), _ptr(rho), _ptr(ux), _ptr(uy), _ptr(T)))
        return rho, ux, uy, T

    def noneq(self, f, want_delta=True):
        p = self.prob
        f = np.ascontiguousarray(f, dtype=np.float64)
        delta = np.zeros((self.S, 12, p.ny, p.nx)) if want_delta else None
        totals = np.zeros(self.S + 3)
        self._check(lib().or_noneq(self._h, _ptr(f), _ptr(delta), _ptr(totals)))
        return delta, totals

    def energy(self, f, want_fields=True):
        """Energies and energy fluxes [S][8] per cell and their totals."""
        p = self.prob
        f = np.ascontiguousarray(f, dtype=np.float64)
        fields = np.zeros((self.S, 8, p.ny, p.nx)) if want_fields else None
        totals = np.zeros((self.S, 8))
        self._check(lib().or_energy(self._h, _ptr(f), _ptr(fields), _ptr(totals)))
        return fields, totals

    @staticmethod
    def _check(rc):
        if rc != 0:
            raise OracleError(rc)
