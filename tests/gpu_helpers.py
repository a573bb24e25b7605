"""Shared helpers of the GPU parity tests: run a problem through the HIP
library and through the CPU oracle from the same seeded inputs, and compare
per field."""
import math

import numpy as np

from oracle import oracle as O
from paper_2006_15932_amd import dbm as D
from paper_2006_15932_amd import workloads as W


def gpu_run(p, steps, precision="fp64", path=0, options=None, tile_rows=None):
    sim = D.Simulation(p, precision=precision)
    if path:
        sim.set_option(D.DBM_OPT_PATH, 1)
    if tile_rows is not None:
        sim.set_option(D.DBM_OPT_TILE_ROWS, tile_rows)
    for k, v in (options or {}).items():
        sim.set_option(k, v)
    sim.set_fields()
    sim.step(steps)
    return sim


def oracle_run(p, steps, threads=8):
    O.set_threads(threads)
    o = O.Oracle(p)
    f = o.init_equilibrium(*W.fields(p))
    return o, o.run(f, steps)


def field_errors(p, mom_gpu, mom_or):
    """Normwise relative L-infinity errors per field: total rho, each rho^s,
    u (vector, denominator at least 1% of a reference sound speed), T."""
    rg, uxg, uyg, Tg = mom_gpu
    ro, uxo, uyo, To = mom_or
    out = {}
    rho_g, rho_o = rg.sum(0), ro.sum(0)
    out["rho"] = np.abs(rho_g - rho_o).max() / np.abs(rho_o).max()
    for s in range(ro.shape[0]):
        den = np.abs(ro[s]).max()
        if den > 0:
            out["rho%d" % s] = np.abs(rg[s] - ro[s]).max() / den
    mbar = rho_o.mean() / sum((ro[s] / p.species[s].m).mean() for s in range(ro.shape[0]))
    cs = math.sqrt(1.4 * To.mean() / mbar)
    du = np.hypot(uxg - uxo, uyg - uyo).max()
    umax = np.hypot(uxo, uyo).max()
    # u is a vector field that starts at rest in most setups, so its error is
    # normalised by max(max|u|, 0.01 c_s): the largest speed, but at least 1%
    # of the sound speed of the mean mixture ("u", the gate).  The error
    # relative to max(max|u|, c_s) is reported as "u_cs" for comparison only.
    floor = max(umax, 0.01 * cs)
    out["u"] = du / floor
    out["u_cs"] = du / max(umax, cs)
    out["ux"] = np.abs(uxg - uxo).max() / floor
    out["uy"] = np.abs(uyg - uyo).max() / floor
    out["T"] = np.abs(Tg - To).max() / np.abs(To).max()
    return out


def f_error(fg, fo):
    return np.abs(fg - fo).max() / np.abs(fo).max()
