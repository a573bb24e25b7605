"""GPU tests of stochastic rounding of the FP32-bulk stores
(DBM_OPT_ROUNDING = 1) against the FP64 CPU oracle.

Round-to-nearest repeats nearly the same rounding every step on slowly
varying fields, so the FP32-bulk error grows close to linearly with the step
count; unbiased stochastic rounding turns it into a random walk.  The
Rayleigh-Taylor setup over 4000 steps shows the difference at a size the
oracle runs in seconds (at 128^2 over 20000 steps the two reach 5e-5..8e-5
and 7e-7..1e-6).
"""
import numpy as np
import pytest

from gpu_helpers import f_error, field_errors, gpu_run, oracle_run
from paper_2006_15932_amd import dbm as D
from paper_2006_15932_amd import workloads as W

pytestmark = pytest.mark.gpu

FP32_TOL = 1e-5
SR = {D.DBM_OPT_ROUNDING: 1}


def _errs(p, steps, **kw):
    print("case", p.name, p.nx, p.ny, "S=%d" % p.S, "steps=%d" % steps, kw, flush=True)
    sim = gpu_run(p, steps, "fp32", **kw)
    o, fo = oracle_run(p, steps)
    e = field_errors(p, sim.moments(), o.moments(fo))
    print("errors", {k: float("%.3e" % v) for k, v in e.items()}, flush=True)
    return sim, e


def test_stochastic_rounding_removes_the_drift_of_round_to_nearest():
    """Stratified Rayleigh-Taylor, f itself stored: stochastic rounding cuts
    the errors of round-to-nearest more than fourfold.  (u is compared with
    the sound speed: the flow stays below 1% of it, where the 0.01 c_s floor
    is a known miss, test_gpu_known_misses.py.)"""
    p = W.rayleigh_taylor(n=64, steps=4000, precision="fp32")
    F = {D.DBM_OPT_STORAGE: 1}
    _, rn = _errs(p, 4000, options=F)
    sim, sr = _errs(p, 4000, options={**F, **SR})
    assert sim.get_option(D.DBM_OPT_ROUNDING) == 1
    assert sim.get_option(D.DBM_OPT_PATH) == 0
    for k in ("rho", "u_cs", "T"):
        assert sr[k] < FP32_TOL, (k, sr)
        assert sr[k] < rn[k] / 4, (k, sr[k], rn[k])


@pytest.mark.parametrize("scheme", [W.EULER, W.RK3])
def test_stochastic_rounding_reacting_within_1e5(scheme):
    p = W.reacting(n=70, ny=45, steps=500, precision="fp32", scheme=scheme)
    _, e = _errs(p, 500, options=SR)
    for k in ("rho", "u", "T"):
        assert e[k] < FP32_TOL, (k, e)


def test_stochastic_rounding_plain_path_within_1e5():
    """The plain path stores f itself: rho, T within 1e-5, u against the
    sound speed (u under the 0.01 c_s floor: test_gpu_known_misses.py)."""
    p = W.reacting(n=37, ny=29, steps=300, precision="fp32")
    sim, e = _errs(p, 300, path=1, options=SR)
    assert sim.get_option(D.DBM_OPT_PATH) == 1
    for k in ("rho", "u_cs", "T"):
        assert e[k] < FP32_TOL, (k, e)


def test_stochastic_rounding_row_pipeline_within_1e5():
    p = W.reacting(n=70, ny=45, steps=300, precision="fp32")
    on = gpu_run(p, 300, "fp32", tile_rows=4,
                 options={D.DBM_OPT_PIPELINE: 2, D.DBM_OPT_ROUNDING: 1})
    assert on.get_option(D.DBM_OPT_PIPELINE) == 2
    o, fo = oracle_run(p, 300)
    e = field_errors(p, on.moments(), o.moments(fo))
    for k in ("rho", "u_cs", "T"):       # f itself stored (see the plain path)
        assert e[k] < FP32_TOL, (k, e)


def test_stochastic_rounding_is_deterministic_and_independent_of_tiling():
    """The random bits come from the cell, species and state, so repeated
    runs, other tile shapes and eager launches give the same bits."""
    p = W.rayleigh_taylor(n=70, ny=44, steps=1, precision="fp32")
    ref = gpu_run(p, 40, "fp32", tile_rows=4, options=SR).get_f()
    for rows, graph in ((4, 1), (1, 1), (16, 0)):
        f = gpu_run(p, 40, "fp32", tile_rows=rows,
                    options={D.DBM_OPT_ROUNDING: 1, D.DBM_OPT_GRAPH: graph}).get_f()
        np.testing.assert_array_equal(f, ref)
    rn = gpu_run(p, 40, "fp32", tile_rows=4).get_f()
    assert 0 < f_error(rn, ref) < 1e-5


def test_rounding_option_rejected_where_it_does_not_apply():
    p = W.reacting(n=64, ny=16, steps=1, precision="fp64")
    for prec in ("fp64", "fp32x"):
        sim = D.Simulation(p, precision=prec)
        with pytest.raises(Exception):
            sim.set_option(D.DBM_OPT_ROUNDING, 1)
        assert sim.get_option(D.DBM_OPT_ROUNDING) == 0
    sim = D.Simulation(p, precision="fp32")
    sim.set_option(D.DBM_OPT_ROUNDING, 1)
    with pytest.raises(Exception):
        sim.set_option(D.DBM_OPT_SPLIT, 2)
    with pytest.raises(Exception):
        sim.set_option(D.DBM_OPT_ROUNDING, 2)
    sim.set_option(D.DBM_OPT_ROUNDING, 0)
    sim.set_option(D.DBM_OPT_SPLIT, 2)
    with pytest.raises(Exception):
        sim.set_option(D.DBM_OPT_ROUNDING, 1)
