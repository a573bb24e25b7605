"""Velocity gates of FP32-bulk that are not met, kept as tests with their
measured values (one MI355X, this library) so that they run again as soon as
the reason is removed.  The gate is the normwise velocity error over
max(max|u|, 0.01 c_s) <= 1e-5: an absolute error of 1e-7 c_s where the flow
is slower than 1% of the sound speed.

- f itself stored (plain path, split form, row pipeline, or
  DBM_OPT_STORAGE = 1): the momentum sum_i f_i v_i carries rounding of each
  f_i, about 2^-24 |f| c per step; on the reacting premix at 64^2 x 500 steps
  that is 1.5-2.3e-5 under the floor, while OM storage gives 2.2-2.9e-6; on
  the stratified Rayleigh-Taylor column 3.6e-5 at 500 steps (OM storage
  1.5e-6, asserted in test_gpu_storage.py).
- The Rayleigh-Taylor setup's 128^2 crop over 20000 steps stays below 1% of
  the sound speed: OM storage with references per row gives 5.1e-5 with
  round-to-nearest and 1.05e-5 with stochastic rounding (rho and T within
  1e-5 in both, asserted in test_gpu_stated_steps.py); f storage with
  stochastic rounding 8.3e-5.  The store's rounding of mass and energy is
  what accumulates: OM storage with A-block residuals (storage 2) meets the
  gate with 7.1e-7, and FP32X with 2.7e-7 (both asserted).
- The batch's fast-reacting instance 56 amplifies perturbations about 10^3
  over 2000 steps: OM storage 1.07e-5, with A-block residuals 2.0e-5 (the
  rounding of the stencils and of B, X, Y, amplified alike; rho, T within
  1e-5 in both); f storage 1.2e-4; FP32X 2.8e-7.  Instance 48 meets the
  gate in OM storage (8.9e-6, with residuals 3.6e-6).
"""
import pytest

from gpu_helpers import field_errors, gpu_run, oracle_run
from paper_2006_15932_amd import dbm as D
from paper_2006_15932_amd import workloads as W

pytestmark = pytest.mark.gpu

F = {D.DBM_OPT_STORAGE: 1}
FSR = {D.DBM_OPT_STORAGE: 1, D.DBM_OPT_ROUNDING: 1}
OMSR = {D.DBM_OPT_ROUNDING: 1}


def _case(name):
    return {
        "f_storage_reacting_500": (W.reacting(n=64, steps=500, precision="fp32"), 500, F, {}),
        "split_form_reacting_500": (W.reacting(n=64, steps=500, precision="fp32"), 500,
                                    {D.DBM_OPT_SPLIT: 2}, {}),
        "row_pipeline_reacting_300": (W.reacting(n=70, ny=45, steps=300, precision="fp32"), 300,
                                      {D.DBM_OPT_PIPELINE: 2}, {"tile_rows": 4}),
        "plain_path_reacting_300": (W.reacting(n=37, ny=29, steps=300, precision="fp32"), 300,
                                    {D.DBM_OPT_ROUNDING: 1}, {"path": 1}),
        "rayleigh_taylor_500": (W.rayleigh_taylor(n=64, steps=500, precision="fp32"), 500, FSR, {}),
        "rayleigh_taylor_crop_20000": (W.rayleigh_taylor(n=128, steps=20000, precision="fp32"),
                                       20000, OMSR, {}),
        "batch_56_2000": (W.batch(count=64, steps=2000, precision="fp32")[56], 2000, {}, {}),
        "batch_56_2000_residuals": (W.batch(count=64, steps=2000, precision="fp32")[56], 2000,
                                    {D.DBM_OPT_STORAGE: 2}, {}),
    }[name]


def _miss(name, measured, why):
    return pytest.param(name, marks=pytest.mark.skip(
        reason="known miss: measured u = %s under the 0.01 c_s floor; %s" % (measured, why)))


@pytest.mark.parametrize("name", [
    _miss("f_storage_reacting_500", "about 1.6e-05 (the split form, which stores f too, 1.63e-05)",
          "f storage rounds the momentum to 2^-24 |f| c"),
    _miss("split_form_reacting_500", "1.63e-05", "the split form stores f itself"),
    _miss("row_pipeline_reacting_300", "1.74e-05", "the row pipeline stores f itself"),
    _miss("plain_path_reacting_300", "1.69e-05", "the plain path stores f itself"),
    _miss("rayleigh_taylor_500", "3.55e-05", "f storage; FP32 pressure rounding below 1% of c_s"),
    _miss("rayleigh_taylor_crop_20000", "1.05e-05 (OM storage, stochastic rounding)",
          "flow below 1% of c_s over 20000 steps; FP32 storage rounding"),
    _miss("batch_56_2000", "1.07e-05 (OM storage)", "fast chemistry amplifies rounding about 10^3"),
    _miss("batch_56_2000_residuals", "2.01e-05 (OM storage with A-block residuals)",
          "fast chemistry amplifies the rounding of the stencils and of B, X, Y about 10^3"),
])
def test_fp32_velocity_gate(name):
    p, steps, opts, kw = _case(name)
    sim = gpu_run(p, steps, "fp32", options=opts, **kw)
    o, fo = oracle_run(p, steps, threads=16)
    e = field_errors(p, sim.moments(), o.moments(fo))
    assert e["u"] < 1e-5, e
