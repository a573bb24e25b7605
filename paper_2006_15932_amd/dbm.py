"""ctypes binding of libdbm (include/dbm.h): the same entry points, argument
marshalling only.  Every step of the update runs in the library's HIP
kernels; PyTorch provides the device workspace and the stream.

Importing this module loads ``libdbm.so`` built in-tree by
``paper_2006_15932_amd.build``; there is no fallback implementation, so a
missing library is an error.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libdbm.so")

DBM_OK, DBM_ERR_ARG, DBM_ERR_SINGULAR_M, DBM_ERR_HIP = 0, -1, -2, -3
DBM_ERR_NONFINITE, DBM_ERR_UNSUPPORTED, DBM_ERR_WORKSPACE = -4, -5, -6
DBM_FP64, DBM_FP32_BULK, DBM_FP32X = 0, 1, 2
_PRECISIONS = {"fp64": DBM_FP64, "fp32": DBM_FP32_BULK, "fp32x": DBM_FP32X}
DBM_EULER, DBM_TVD_RK3 = 0, 1
DBM_LIM_MINMOD, DBM_LIM_NONE = 0, 1
DBM_BC_PERIODIC, DBM_BC_OUTFLOW, DBM_BC_WALL = 0, 1, 2
DBM_FORCE_T_EXACT, DBM_FORCE_T_SAME = 0, 1
DBM_OPT_PATH, DBM_OPT_GRAPH, DBM_OPT_TILE_ROWS, DBM_OPT_CHECK_EVERY = 1, 2, 3, 4
DBM_OPT_BATCH_MODE, DBM_OPT_GRAPH_CHUNK, DBM_OPT_PERSISTENT, DBM_OPT_SPLIT = 5, 6, 7, 8
DBM_OPT_PIPELINE = 9
DBM_OPT_ROUNDING = 10
DBM_OPT_CHAIN_WAVE = 11
DBM_OPT_STORAGE = 12
DBM_OPT_DRAIN = 13

NV = 16


class dbm_species(ctypes.Structure):
    _fields_ = [("m", ctypes.c_double), ("I", ctypes.c_double), ("tau", ctypes.c_double),
                ("a_stoich", ctypes.c_double), ("v", ctypes.c_double * 4),
                ("eta", ctypes.c_double * 4)]


class dbm_reaction(ctypes.Structure):
    _fields_ = [("fuel", ctypes.c_int), ("oxidiser", ctypes.c_int), ("k_ov", ctypes.c_double),
                ("Ea_over_R", ctypes.c_double), ("Q", ctypes.c_double)]


class dbm_reaction_step(ctypes.Structure):
    _fields_ = [("fuel", ctypes.c_int), ("oxidiser", ctypes.c_int), ("k_ov", ctypes.c_double),
                ("Ea_over_R", ctypes.c_double), ("Q", ctypes.c_double),
                ("a", ctypes.c_double * 16)]


class dbm_config(ctypes.Structure):
    _fields_ = [("nx", ctypes.c_int), ("ny", ctypes.c_int), ("dx", ctypes.c_double),
                ("dy", ctypes.c_double), ("dt", ctypes.c_double), ("bc_x", ctypes.c_int),
                ("bc_y", ctypes.c_int), ("nspecies", ctypes.c_int),
                ("species", ctypes.POINTER(dbm_species)),
                ("reaction", ctypes.POINTER(dbm_reaction)), ("accel", ctypes.c_double * 2),
                ("precision", ctypes.c_int), ("time_scheme", ctypes.c_int),
                ("limiter", ctypes.c_int), ("force_T_mode", ctypes.c_int),
                ("nchem", ctypes.c_int), ("chem", ctypes.POINTER(dbm_reaction_step))]


class DbmError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__("libdbm error %d: %s" % (code, msg))
        self.code = code


_lib = None
_dp = ctypes.POINTER(ctypes.c_double)
_vp = ctypes.c_void_p

# name -> (restype, argtypes); mirrors include/dbm.h
SIGNATURES = {
    "dbm_workspace_bytes": (ctypes.c_size_t, [ctypes.POINTER(dbm_config), ctypes.c_int]),
    "dbm_create": (ctypes.c_int, [ctypes.POINTER(dbm_config), ctypes.c_int, _vp, _vp,
                                  ctypes.c_size_t, ctypes.POINTER(_vp)]),
    "dbm_destroy": (ctypes.c_int, [_vp]),
    "dbm_set_fields": (ctypes.c_int, [_vp, ctypes.c_int, _dp, _dp, _dp, _dp]),
    "dbm_set_f": (ctypes.c_int, [_vp, ctypes.c_int, _dp]),
    "dbm_get_f": (ctypes.c_int, [_vp, ctypes.c_int, _dp]),
    "dbm_step": (ctypes.c_int, [_vp, ctypes.c_int]),
    "dbm_moments": (ctypes.c_int, [_vp, ctypes.c_int, _dp, _dp, _dp, _dp]),
    "dbm_noneq_moments": (ctypes.c_int, [_vp, ctypes.c_int, _dp, _dp]),
    "dbm_set_option": (ctypes.c_int, [_vp, ctypes.c_int, ctypes.c_int]),
    "dbm_get_option": (ctypes.c_int, [_vp, ctypes.c_int, ctypes.POINTER(ctypes.c_int)]),
    "dbm_energy_moments": (ctypes.c_int, [_vp, ctypes.c_int, _dp, _dp]),
    "dbm_time_stage_kernel": (ctypes.c_int, [_vp, ctypes.c_int, _dp]),
    "dbm_copy_rate": (ctypes.c_int, [_vp, _vp, ctypes.c_size_t, ctypes.c_int, ctypes.c_int,
                                     ctypes.c_int, _vp, _dp]),
    "dbm_noneq_totals_noalloc": (ctypes.c_int, [_vp, ctypes.c_int, _dp]),
    "dbm_state_bytes": (ctypes.c_size_t, [_vp, ctypes.c_int]),
    "dbm_save_state": (ctypes.c_int, [_vp, ctypes.c_int, _vp, ctypes.c_size_t]),
    "dbm_load_state": (ctypes.c_int, [_vp, ctypes.c_int, _vp, ctypes.c_size_t]),
    "dbm_last_error": (ctypes.c_char_p, []),
}


def lib():
    """Load libdbm.so (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError("libdbm.so is not built; run paper_2006_15932_amd.build.build()")
        L = ctypes.CDLL(LIB_PATH)
        for name, (res, args) in SIGNATURES.items():
            fn = getattr(L, name)
            fn.restype, fn.argtypes = res, args
        _lib = L
    return _lib


def last_error() -> str:
    return lib().dbm_last_error().decode()


def _check(rc):
    if rc != DBM_OK:
        raise DbmError(rc, last_error())


def _dptr(a):
    if a is None:
        return None
    assert a.dtype == np.float64 and a.flags["C_CONTIGUOUS"]
    return a.ctypes.data_as(_dp)


class Configs:
    """Keeps the ctypes structures of a list of problems alive."""

    def __init__(self, problems, precision=None):
        self.n = len(problems)
        self.cfg = (dbm_config * self.n)()
        self._keep = []
        for k, p in enumerate(problems):
            sp = (dbm_species * p.S)()
            for j, s in enumerate(p.species):
                sp[j].m, sp[j].I, sp[j].tau, sp[j].a_stoich = s.m, s.I, s.tau, s.a
                for g in range(4):
                    sp[j].v[g], sp[j].eta[g] = s.v[g], s.eta[g]
            c = self.cfg[k]
            c.nx, c.ny, c.dx, c.dy, c.dt = p.nx, p.ny, p.dx, p.dy, p.dt
            c.bc_x, c.bc_y, c.nspecies = p.bc_x, p.bc_y, p.S
            c.species = ctypes.cast(sp, ctypes.POINTER(dbm_species))
            if p.reaction is not None:
                r = dbm_reaction(p.reaction["fuel"], p.reaction["oxid"], p.reaction["k_ov"],
                                 p.reaction["Ea_over_R"], p.reaction.get("Q", 0.0))
                c.reaction = ctypes.pointer(r)
                self._keep.append(r)
            mech = getattr(p, "mechanism", None)
            if mech:
                steps = (dbm_reaction_step * len(mech))()
                for r, st in enumerate(mech):
                    steps[r].fuel, steps[r].oxidiser = st["fuel"], st["oxid"]
                    steps[r].k_ov, steps[r].Ea_over_R = st["k_ov"], st["Ea_over_R"]
                    steps[r].Q = st.get("Q", 0.0)
                    for j, a in enumerate(st["a"]):
                        steps[r].a[j] = a
                c.nchem = len(mech)
                c.chem = ctypes.cast(steps, ctypes.POINTER(dbm_reaction_step))
                self._keep.append(steps)
            c.accel[0], c.accel[1] = p.accel
            prec = precision if precision is not None else p.precision
            if isinstance(prec, str):
                if prec not in _PRECISIONS:
                    raise ValueError(f"unknown precision {prec!r}")
                prec = _PRECISIONS[prec]
            c.precision = int(prec)
            c.time_scheme, c.limiter, c.force_T_mode = p.scheme, p.limiter, p.force_T_mode
            self._keep.append(sp)


def dbm_workspace_bytes(configs: Configs) -> int:
    return int(lib().dbm_workspace_bytes(configs.cfg, configs.n))


def dbm_create(configs: Configs, stream_ptr: int, ws_ptr: int, ws_bytes: int) -> int:
    h = _vp()
    _check(lib().dbm_create(configs.cfg, configs.n, _vp(stream_ptr), _vp(ws_ptr),
                            ctypes.c_size_t(ws_bytes), ctypes.byref(h)))
    return h.value


def dbm_destroy(h: int) -> None:
    _check(lib().dbm_destroy(_vp(h)))


def dbm_set_fields(h, inst, n_sp, ux, uy, T) -> None:
    arrs = [np.ascontiguousarray(a, dtype=np.float64) for a in (n_sp, ux, uy, T)]
    _check(lib().dbm_set_fields(_vp(h), inst, *[_dptr(a) for a in arrs]))


def dbm_set_f(h, inst, f) -> None:
    f = np.ascontiguousarray(f, dtype=np.float64)
    _check(lib().dbm_set_f(_vp(h), inst, _dptr(f)))


def dbm_get_f(h, inst, shape) -> np.ndarray:
    f = np.zeros(shape)
    _check(lib().dbm_get_f(_vp(h), inst, _dptr(f)))
    return f


def dbm_step(h, nsteps) -> None:
    _check(lib().dbm_step(_vp(h), int(nsteps)))


def dbm_moments(h, inst, S, ny, nx):
    rho, ux, uy, T = np.zeros((S, ny, nx)), np.zeros((ny, nx)), np.zeros((ny, nx)), np.zeros((ny, nx))
    _check(lib().dbm_moments(_vp(h), inst, _dptr(rho), _dptr(ux), _dptr(uy), _dptr(T)))
    return rho, ux, uy, T


def dbm_noneq_moments(h, inst, S, ny, nx, want_delta=True):
    delta = np.zeros((S, 12, ny, nx)) if want_delta else None
    totals = np.zeros(S + 3)
    _check(lib().dbm_noneq_moments(_vp(h), inst, _dptr(delta), _dptr(totals)))
    return delta, totals


def dbm_noneq_totals_noalloc(h, inst, S):
    totals = np.zeros(S + 3)
    _check(lib().dbm_noneq_totals_noalloc(_vp(h), inst, _dptr(totals)))
    return totals


def dbm_energy_moments(h, inst, S, ny, nx, want_fields=True):
    fields = np.zeros((S, 8, ny, nx)) if want_fields else None
    totals = np.zeros((S, 8))
    _check(lib().dbm_energy_moments(_vp(h), inst, _dptr(fields), _dptr(totals)))
    return fields, totals


def dbm_set_option(h, option, value) -> None:
    _check(lib().dbm_set_option(_vp(h), option, int(value)))


def dbm_get_option(h, option) -> int:
    v = ctypes.c_int(0)
    _check(lib().dbm_get_option(_vp(h), option, ctypes.byref(v)))
    return v.value


def dbm_save_state(h, inst) -> bytes:
    n = lib().dbm_state_bytes(_vp(h), inst)
    if n == 0:
        raise DbmError(DBM_ERR_ARG, last_error())
    buf = ctypes.create_string_buffer(n)
    _check(lib().dbm_save_state(_vp(h), inst, ctypes.cast(buf, _vp), n))
    return buf.raw


def dbm_load_state(h, inst, blob: bytes) -> None:
    buf = ctypes.create_string_buffer(blob, len(blob))
    _check(lib().dbm_load_state(_vp(h), inst, ctypes.cast(buf, _vp), len(blob)))


def dbm_time_stage_kernel(h, reps) -> float:
    ms = ctypes.c_double(0.0)
    _check(lib().dbm_time_stage_kernel(_vp(h), int(reps), ctypes.byref(ms)))
    return ms.value


def dbm_copy_rate(src_ptr, dst_ptr, nbytes, grid, reps, stream_ptr, words=1) -> float:
    """Mean milliseconds of one device-to-device streaming copy of nbytes."""
    ms = ctypes.c_double(0.0)
    _check(lib().dbm_copy_rate(_vp(src_ptr), _vp(dst_ptr), ctypes.c_size_t(nbytes), int(grid),
                               int(words), int(reps), _vp(stream_ptr), ctypes.byref(ms)))
    return ms.value


def copy_rate_gbs(nbytes=1 << 30, grid=1024, reps=10, device="cuda:0", words=1) -> float:
    """Achievable HBM rate (read + write GB/s) of the library's streaming copy
    on two fresh buffers of nbytes each."""
    import torch
    a = torch.ones(nbytes // 4, dtype=torch.float32, device=device)
    b = torch.empty_like(a)
    st = torch.cuda.current_stream(device)
    ms = dbm_copy_rate(a.data_ptr(), b.data_ptr(), nbytes, grid, reps, st.cuda_stream, words)
    del a, b
    return 2.0 * nbytes / (ms * 1e-3) / 1e9


class Simulation:
    """One handle over one or more problems (``workloads.Problem``), with the
    device workspace held in a torch uint8 tensor and work ordered on a
    dedicated torch stream."""

    def __init__(self, problems, precision=None, device="cuda:0", stream=None):
        import torch

        if not isinstance(problems, (list, tuple)):
            problems = [problems]
        self.problems = list(problems)
        self.configs = Configs(self.problems, precision)
        self.device = torch.device(device)
        nbytes = dbm_workspace_bytes(self.configs)
        if nbytes == 0:
            raise DbmError(DBM_ERR_ARG, last_error())
        self.workspace = torch.empty(nbytes, dtype=torch.uint8, device=self.device)
        self.stream = stream if stream is not None else torch.cuda.Stream(device=self.device)
        self.h = dbm_create(self.configs, self.stream.cuda_stream, self.workspace.data_ptr(),
                            nbytes)

    def close(self):
        if getattr(self, "h", None):
            dbm_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _p(self, inst):
        return self.problems[inst]

    def set_fields(self, inst=0, fields=None):
        p = self._p(inst)
        n_sp, ux, uy, T = fields if fields is not None else (p.n_sp, p.ux, p.uy, p.T)
        dbm_set_fields(self.h, inst, n_sp, ux, uy, T)

    def set_f(self, f, inst=0):
        dbm_set_f(self.h, inst, f)

    def get_f(self, inst=0):
        p = self._p(inst)
        return dbm_get_f(self.h, inst, (p.S, NV, p.ny, p.nx))

    def save_state(self, inst=0) -> bytes:
        return dbm_save_state(self.h, inst)

    def load_state(self, blob, inst=0):
        dbm_load_state(self.h, inst, blob)

    def step(self, n=1):
        dbm_step(self.h, n)

    def synchronize(self):
        self.stream.synchronize()

    def moments(self, inst=0):
        p = self._p(inst)
        return dbm_moments(self.h, inst, p.S, p.ny, p.nx)

    def noneq(self, inst=0, want_delta=True):
        p = self._p(inst)
        return dbm_noneq_moments(self.h, inst, p.S, p.ny, p.nx, want_delta)

    def totals_noalloc(self, inst=0):
        return dbm_noneq_totals_noalloc(self.h, inst, self._p(inst).S)

    def energy(self, inst=0, want_fields=True):
        p = self._p(inst)
        return dbm_energy_moments(self.h, inst, p.S, p.ny, p.nx, want_fields)

    def set_option(self, option, value):
        dbm_set_option(self.h, option, value)

    def get_option(self, option):
        return dbm_get_option(self.h, option)

    def time_stage_kernel(self, reps=10):
        return dbm_time_stage_kernel(self.h, reps)
