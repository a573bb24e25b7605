"""GPU parity of the chain-wavefront form of the one-pass kernel (up to 3
species): one more wavefront per workgroup forms each row's mixture chain
while the species' wavefronts form their stencils.  Checked against the
FP64 oracle (bars: FP32 1e-5, FP32X 1e-7, FP64 1e-10 on rho, u, T) and
against the same runs without it."""
import numpy as np
import pytest

from gpu_helpers import f_error, field_errors, gpu_run, oracle_run
from paper_2006_15932_amd import dbm as D
from paper_2006_15932_amd import workloads as W

pytestmark = pytest.mark.gpu

TOL = 1e-5
TOLS = {"fp32": 1e-5, "fp32x": 1e-7, "fp64": 1e-10}
ON = {D.DBM_OPT_CHAIN_WAVE: 2}
OFF = {D.DBM_OPT_CHAIN_WAVE: 1, D.DBM_OPT_PIPELINE: 1}


def _check(p, steps, tile_rows=None, extra=None, precision="fp32"):
    print("case", p.name, p.nx, p.ny, "S=%d" % p.S, precision, "steps", steps, "rows", tile_rows,
          flush=True)
    off_opts = dict(OFF) if precision == "fp32" else {D.DBM_OPT_CHAIN_WAVE: 1}
    on = gpu_run(p, steps, precision, tile_rows=tile_rows, options={**ON, **(extra or {})})
    assert on.get_option(D.DBM_OPT_CHAIN_WAVE) == 2
    assert on.get_option(D.DBM_OPT_PATH) == 0
    off = gpu_run(p, steps, precision, tile_rows=tile_rows, options={**off_opts, **(extra or {})})
    assert off.get_option(D.DBM_OPT_CHAIN_WAVE) == 1
    o, fo = oracle_run(p, steps)
    errs = field_errors(p, on.moments(), o.moments(fo))
    d = f_error(on.get_f(), off.get_f())
    print("errors", {k: float("%.3e" % errs[k]) for k in ("rho", "u", "T")}, "vs off %.3e" % d,
          flush=True)
    for k in ("rho", "u", "T"):
        assert errs[k] < TOLS[precision], (k, errs)
    assert d < (1e-6 if precision == "fp32" else 1e-12)
    return on


@pytest.mark.parametrize("scheme", [W.EULER, W.RK3])
@pytest.mark.parametrize("rows", [None, 1, 3, 16])
def test_chain_wave_reacting(scheme, rows):
    _check(W.reacting(n=70, ny=45, steps=1, precision="fp32", scheme=scheme), 200, rows)


@pytest.mark.parametrize("nx,ny", [(1, 9), (7, 1), (64, 4), (129, 2), (130, 37)])
def test_chain_wave_ragged_and_degenerate(nx, ny):
    _check(W.reacting(n=nx, ny=ny, steps=1, precision="fp32"), 40)


def test_chain_wave_two_species_outflow():
    _check(W.sod(nx=400, steps=1, precision="fp32"), 200)


def test_chain_wave_stochastic_rounding_deterministic():
    p = W.reacting(n=70, ny=45, steps=1, precision="fp32")
    opts = {**ON, D.DBM_OPT_ROUNDING: 1}
    a = gpu_run(p, 100, "fp32", tile_rows=4, options=opts)
    b = gpu_run(p, 100, "fp32", tile_rows=16, options=opts)
    np.testing.assert_array_equal(a.get_f(), b.get_f())
    _check(p, 100, 4, {D.DBM_OPT_ROUNDING: 1})


def test_chain_wave_batched_instances():
    sizes = [(37, 29), (64, 64), (100, 20), (61, 61)]
    probs = [W.reacting(n=nx, ny=ny, steps=1, seed=700 + k, tau=1e-5 * (1 + k), precision="fp32")
             for k, (nx, ny) in enumerate(sizes)]
    sim = D.Simulation(probs, precision="fp32")
    sim.set_option(D.DBM_OPT_CHAIN_WAVE, 2)
    for k in range(len(probs)):
        sim.set_fields(k)
    sim.step(100)
    assert sim.get_option(D.DBM_OPT_CHAIN_WAVE) == 2
    for k, p in enumerate(probs):
        o, fo = oracle_run(p, 100)
        errs = field_errors(p, sim.moments(k), o.moments(fo))
        for key in ("rho", "u", "T"):
            assert errs[key] < TOL, (k, key, errs)


def test_chain_wave_option_rules():
    p4 = W.rayleigh_taylor(n=64, ny=16, steps=1, precision="fp32")     # 4 species
    sim = D.Simulation(p4, precision="fp32")
    with pytest.raises(Exception):
        sim.set_option(D.DBM_OPT_CHAIN_WAVE, 2)
    p3 = W.reacting(n=64, ny=16, steps=1, precision="fp64")
    D.Simulation(p3, precision="fp64").set_option(D.DBM_OPT_CHAIN_WAVE, 2)   # allowed
    sim = D.Simulation(p3, precision="fp32")
    sim.set_option(D.DBM_OPT_CHAIN_WAVE, 2)
    with pytest.raises(Exception):
        sim.set_option(D.DBM_OPT_PIPELINE, 2)
    with pytest.raises(Exception):
        sim.set_option(D.DBM_OPT_SPLIT, 2)
    with pytest.raises(Exception):
        sim.set_option(D.DBM_OPT_CHAIN_WAVE, 3)


@pytest.mark.parametrize("precision", ["fp64", "fp32x"])
@pytest.mark.parametrize("scheme,rows", [(W.EULER, None), (W.EULER, 3), (W.RK3, 1), (W.RK3, 16)])
def test_chain_wave_wide_storage(precision, scheme, rows):
    """FP64 arithmetic runs whole prefetch cycles of rows (rows past the
    tile computed, not stored); the chain wavefront runs as many."""
    p = W.reacting(n=70, ny=45, steps=1, precision=precision, scheme=scheme)
    _check(p, 60, rows, precision=precision)


@pytest.mark.parametrize("nx,ny", [(1, 9), (7, 1), (65, 3), (129, 2)])
def test_chain_wave_wide_storage_degenerate(nx, ny):
    _check(W.reacting(n=nx, ny=ny, steps=1, precision="fp64"), 20, precision="fp64")
