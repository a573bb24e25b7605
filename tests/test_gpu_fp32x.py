"""GPU parity of the FP32X storage mode (each value of f kept as an FP32
value plus a bfloat16 residual, about 32 significant bits; every operation in
FP64) against the FP64 CPU oracle.

Per stored value the split rounds with relative error at most about 2^-32
(the FP32 part leaves a residual of at most 2^-24 of the value, which bfloat16
keeps to 8 significant bits), 2^-8 of FP32's.  The FP32-bulk bar of 1e-5 scaled by
that ratio is 4e-8; the bar here is 1e-7, because in the shear layer the
temperature is the small difference of total and kinetic energy (|u| = 1.5),
which amplifies the storage rounding about tenfold (there FP32-bulk itself
reaches 1e-5 in T within 60 steps).
"""
import numpy as np
import pytest

from gpu_helpers import f_error, field_errors, gpu_run, oracle_run
from paper_2006_15932_amd import dbm as D
from paper_2006_15932_amd import workloads as W

pytestmark = pytest.mark.gpu

FP32X_TOL = 1e-7


def _check(p, steps, fields=("rho", "u", "T"), **kw):
    print("case", p.name, p.nx, p.ny, "S=%d" % p.S, "steps=%d" % steps, kw, flush=True)
    sim = gpu_run(p, steps, "fp32x", **kw)
    o, fo = oracle_run(p, steps)
    errs = field_errors(p, sim.moments(), o.moments(fo))
    ef = f_error(sim.get_f(), fo)
    print("fp32x errors", {k: float("%.3e" % v) for k, v in errs.items()}, "f %.3e" % ef,
          flush=True)
    for k in fields:
        assert errs[k] < FP32X_TOL, (k, errs)
    return sim, ef


@pytest.mark.parametrize("scheme", [W.EULER, W.RK3])
def test_fp32x_reacting(scheme):
    sim, _ = _check(W.reacting(n=64, steps=500, precision="fp32x", scheme=scheme), 500)
    assert sim.get_option(D.DBM_OPT_PATH) == 0


def test_fp32x_rayleigh_taylor():
    _check(W.rayleigh_taylor(n=64, steps=500, precision="fp32x"), 500)


def test_fp32x_two_step_mechanism():
    _check(W.two_step(n=64, steps=400, precision="fp32x"), 400)


@pytest.mark.parametrize("nx,ny", [(64, 64), (65, 33), (129, 20), (130, 37)])
def test_fp32x_ragged_sizes(nx, ny):
    _check(W.reacting(n=nx, ny=ny, steps=1, precision="fp32x"), 60)


def test_fp32x_plain_path():
    sim, _ = _check(W.reacting(n=70, ny=33, steps=1, precision="fp32x"), 60, path=1)
    assert sim.get_option(D.DBM_OPT_PATH) == 1


def test_fp32x_shear_layer_outflow_walls():
    _check(W.shear_layer(n=90, ny=64, steps=1, precision="fp32x"), 60)
    _check(W.rayleigh_taylor(n=70, ny=44, steps=1, precision="fp32x", scheme=W.RK3), 60)


def test_fp32x_tile_shape_does_not_change_bits():
    p = W.reacting(n=125, ny=41, steps=1, precision="fp32x")
    ref = None
    for rows in (1, 3, 16, 64):
        f = gpu_run(p, 15, "fp32x", tile_rows=rows).get_f()
        if ref is None:
            ref = f
        else:
            np.testing.assert_array_equal(f, ref)


def test_fp32x_storage_round_trip():
    """set_f rounds each value to the split form (relative error at most
    2^-32 (1 + 2^-15)); reading it back and storing it again changes
    nothing."""
    p = W.reacting(n=70, ny=20, steps=1, precision="fp32x")
    sim = D.Simulation(p, precision="fp32x")
    rng = np.random.default_rng(5)
    f = rng.uniform(0.5, 2.0, size=(p.S, 16, p.ny, p.nx)) * 10.0 ** rng.integers(
        -6, 3, size=(p.S, 16, p.ny, p.nx))
    sim.set_f(f)
    g = sim.get_f()
    rel = np.abs(g - f) / np.abs(f)
    assert rel.max() <= 2.0 ** -32 * (1 + 2.0 ** -15), rel.max()
    assert rel.max() > 0
    sim.set_f(g)
    np.testing.assert_array_equal(sim.get_f(), g)


def test_fp32x_checkpoint_restart_is_bit_exact():
    p = W.rayleigh_taylor(n=64, ny=40, steps=1, precision="fp32x")
    a = gpu_run(p, 20, "fp32x")
    b = gpu_run(p, 10, "fp32x")
    c = D.Simulation(p, precision="fp32x")
    c.set_f(b.get_f())
    c.step(10)
    np.testing.assert_array_equal(a.get_f(), c.get_f())


def test_fp32x_batched_instances():
    sizes = [(37, 29), (64, 64), (100, 20), (61, 61)]
    probs = [W.reacting(n=nx, ny=ny, steps=1, seed=900 + k, precision="fp32x")
             for k, (nx, ny) in enumerate(sizes)]
    sim = D.Simulation(probs, precision="fp32x")
    for k in range(len(probs)):
        sim.set_fields(k)
    sim.step(50)
    for k, p in enumerate(probs):
        o, fo = oracle_run(p, 50)
        errs = field_errors(p, sim.moments(k), o.moments(fo))
        for key in ("rho", "u", "T"):
            assert errs[key] < FP32X_TOL, (k, key, errs)


def test_fp32x_split_form_is_rejected():
    p = W.reacting(n=64, ny=16, steps=1, precision="fp32x")
    sim = D.Simulation(p, precision="fp32x")
    with pytest.raises(Exception):
        sim.set_option(D.DBM_OPT_SPLIT, 2)


@pytest.mark.parametrize("nx,ny", [(1, 9), (7, 1), (3, 2), (60, 5), (65, 3)])
@pytest.mark.parametrize("precision,opts,tol", [("fp32x", {}, FP32X_TOL),
                                                ("fp32", {}, 1e-5),
                                                ("fp32", {D.DBM_OPT_ROUNDING: 1}, 1e-5)])
def test_degenerate_sizes_narrow_storage(nx, ny, precision, opts, tol):
    """Grids narrower or shorter than the stencil (periodic wrap onto the
    same cells, one-row tiles) in the narrow storage modes."""
    p = W.reacting(n=nx, ny=ny, steps=1, precision=precision)
    sim = gpu_run(p, 12, precision, options=opts)
    o, fo = oracle_run(p, 12)
    errs = field_errors(p, sim.moments(), o.moments(fo))
    for k in ("rho", "u", "T"):
        assert errs[k] < tol, (k, errs)
