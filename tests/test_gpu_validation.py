"""The one-dimensional validations on the GPU: the same inputs as the oracle
validations, checked against the oracle and against the invariants
themselves through the library's own diagnostics."""
import numpy as np
import pytest

import validation_cases as V
from gpu_helpers import f_error, oracle_run
from paper_2006_15932_amd import dbm as D

pytestmark = pytest.mark.gpu


def _sim(p, precision, steps):
    print("validation", p.name, p.nx, p.ny, precision, steps, flush=True)
    sim = D.Simulation(p, precision=precision)
    sim.set_fields()
    _, t0 = sim.noneq(want_delta=False)
    rho0 = sim.moments()[0]
    sim.step(steps)
    return sim, t0, rho0


def test_rankine_hugoniot_shock_is_stationary_gpu():
    p, st = V.stationary_shock()
    sim, _, _ = _sim(p, "fp64", 2000)
    o, fo = oracle_run(p, 2000)
    assert f_error(sim.get_f(), fo) < 1e-10
    rho, ux, _, T = sim.moments()
    r = rho.sum(0)[0]
    x = V.shock_position(r, st["rho1"], st["rho2"])
    assert abs(x - st["x_shock"]) < 1.0
    assert abs(r[300] / st["rho2"] - 1) < 1e-9 and abs(ux[0, 100] / st["u1"] - 1) < 1e-9


@pytest.mark.parametrize("precision,tol", [("fp64", 1e-11), ("fp32", 1e-6)])
def test_reacting_wave_energy_release_gpu(precision, tol):
    p = V.reacting_wave(precision=precision)
    sim, t0, rho0 = _sim(p, precision, p.steps)
    _, t1 = sim.noneq(want_delta=False)
    rho1 = sim.moments()[0]
    cell = p.dx * p.dy / p.species[0].m
    release = p.reaction["Q"] * (rho0[0].sum() - rho1[0].sum()) * cell / 2
    assert release > 0
    assert abs((t1[-1] - t0[-1]) - release) <= tol * t0[-1]
    if precision == "fp64":
        o, fo = oracle_run(p, p.steps)
        assert f_error(sim.get_f(), fo) < 1e-10


def test_free_falling_reacting_box_gpu():
    p = V.free_falling_reacting_box()
    n = p.steps
    sim, t0, rho0 = _sim(p, "fp64", n)
    _, t1 = sim.noneq(want_delta=False)
    rho1, ux, uy, _ = sim.moments()
    t = n * p.dt
    np.testing.assert_allclose([ux.mean(), uy.mean()], np.array(p.accel) * t, rtol=1e-9)
    M = t0[:3].sum()
    work = 0.5 * M * (p.accel[0] ** 2 + p.accel[1] ** 2) * p.dt ** 2 * n * (n - 1)
    cell = p.dx * p.dy / p.species[0].m
    release = p.reaction["Q"] * (rho0[0].sum() - rho1[0].sum()) * cell / 2
    assert abs((t1[-1] - t0[-1]) - release - work) <= 1e-12 * t0[-1]
    o, fo = oracle_run(p, n)
    assert f_error(sim.get_f(), fo) < 1e-10


@pytest.mark.parametrize("precision,tol", [("fp64", 1e-11), ("fp32", 1e-6)])
def test_two_step_wave_energy_release_gpu(precision, tol):
    p = V.two_step_wave(precision=precision)
    sim, t0, rho0 = _sim(p, precision, p.steps)
    _, t1 = sim.noneq(want_delta=False)
    rho1 = sim.moments()[0]
    ms = np.array([s.m for s in p.species])
    N0 = rho0.sum(axis=(1, 2)) / ms * p.dx * p.dy
    N1 = rho1.sum(axis=(1, 2)) / ms * p.dx * p.dy
    release, x1, x2 = V.two_step_release(p, N0, N1)
    assert x1 > 0 and x2 > 0
    assert abs((t1[-1] - t0[-1]) - release) <= tol * t0[-1]
    if precision == "fp64":
        o, fo = oracle_run(p, p.steps)
        assert f_error(sim.get_f(), fo) < 1e-10
