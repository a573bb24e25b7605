"""The allocation-free totals entry point (dbm_noneq_totals_noalloc, fixed
device scratch) against the totals of dbm_noneq_moments (workspace scratch),
through the C ABI: two calls in a row on one GPU, the second on a smaller
instance, in FP64 and in FP32-bulk (OM storage)."""
import numpy as np
import pytest

from paper_2006_15932_amd import dbm as D
from paper_2006_15932_amd import workloads as W

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_noalloc_totals_equal_workspace_totals(precision):
    big = W.reacting(n=130, ny=70, steps=1, precision=precision)
    small = W.reacting(n=40, ny=20, steps=1, seed=99, precision=precision)
    sim = D.Simulation([big, small], precision=precision)
    for k in range(2):
        sim.set_fields(k)
    sim.step(7)
    for k in (0, 1):                       # the second call is the smaller input
        ref = D.dbm_noneq_moments(sim.h, k, sim._p(k).S, sim._p(k).ny, sim._p(k).nx,
                                  want_delta=False)[1]
        got = sim.totals_noalloc(k)
        print(precision, "instance", k, got, flush=True)
        assert np.all(np.isfinite(got))
        np.testing.assert_array_equal(got, ref)
    # and again on the first instance: nothing of the previous call leaks in
    ref = D.dbm_noneq_moments(sim.h, 0, big.S, big.ny, big.nx, want_delta=False)[1]
    np.testing.assert_array_equal(sim.totals_noalloc(0), ref)
