"""GPU tests of the FP32-bulk storage representations and of checkpoints.

OM storage (DBM_OPT_STORAGE = 0, the default of FP32-bulk on the one-pass
path) keeps per cell and species the A-block moments of f - fref (fref an
equilibrium at rest per grid row, or one for the grid where the rows do not
differ) and the orbit components B, X, Y of f in 16 FP32 values; storage 2
adds a bfloat16 residual to each of the four A-block values (the sum is
carried in FP64, the stencils and the collision see the FP32 values); the
alternative stores the 16 values f_i.  All are checked against the FP64
oracle, against each other, for independence of the tile shape and launch
form, for conversions between them, and for bit-exact checkpoints through
dbm_save_state / dbm_load_state.
"""
import numpy as np
import pytest

from gpu_helpers import f_error, field_errors, gpu_run, oracle_run
from paper_2006_15932_amd import dbm as D
from paper_2006_15932_amd import workloads as W

pytestmark = pytest.mark.gpu

FP32_TOL = 1e-5
OM, PLAIN, ARES = 0, 1, 2


def test_storage_in_use_follows_the_options():
    p = W.reacting(n=70, ny=20, steps=1, precision="fp32")
    sim = D.Simulation(p, precision="fp32")
    assert sim.get_option(D.DBM_OPT_STORAGE) == OM
    sim.set_option(D.DBM_OPT_STORAGE, PLAIN)
    assert sim.get_option(D.DBM_OPT_STORAGE) == PLAIN
    sim.set_option(D.DBM_OPT_STORAGE, OM)
    assert sim.get_option(D.DBM_OPT_STORAGE) == OM
    for opt in (D.DBM_OPT_PATH, D.DBM_OPT_SPLIT, D.DBM_OPT_PIPELINE):
        sim.set_option(opt, 1 if opt == D.DBM_OPT_PATH else 2)
        assert sim.get_option(D.DBM_OPT_STORAGE) == PLAIN, opt
        sim.set_option(opt, 0)
        assert sim.get_option(D.DBM_OPT_STORAGE) == OM, opt
    for prec in ("fp64", "fp32x"):
        s2 = D.Simulation(p.with_(precision=prec), precision=prec)
        assert s2.get_option(D.DBM_OPT_STORAGE) == PLAIN
    sim.set_option(D.DBM_OPT_STORAGE, ARES)
    assert sim.get_option(D.DBM_OPT_STORAGE) == ARES
    with pytest.raises(D.DbmError) as e:
        sim.set_option(D.DBM_OPT_ROUNDING, 1)
    assert e.value.code == D.DBM_ERR_UNSUPPORTED
    sim.set_option(D.DBM_OPT_PIPELINE, 2)
    assert sim.get_option(D.DBM_OPT_STORAGE) == PLAIN
    sim.set_option(D.DBM_OPT_PIPELINE, 0)
    assert sim.get_option(D.DBM_OPT_STORAGE) == ARES
    sim.set_option(D.DBM_OPT_STORAGE, OM)
    sim.set_option(D.DBM_OPT_ROUNDING, 1)
    with pytest.raises(D.DbmError) as e:
        sim.set_option(D.DBM_OPT_STORAGE, ARES)
    assert e.value.code == D.DBM_ERR_UNSUPPORTED
    with pytest.raises(D.DbmError):
        sim.set_option(D.DBM_OPT_STORAGE, 3)


@pytest.mark.parametrize("case", ["reacting", "reacting_rk3", "shear4", "two_step", "outflow",
                                  "ragged"])
def test_om_storage_matches_oracle(case):
    """OM storage against the FP64 oracle (E1 metric, 1e-5) on every boundary
    type, both schemes, force, chemistry and ragged sizes."""
    p, steps = {
        "reacting": (W.reacting(n=70, ny=45, steps=1, precision="fp32"), 300),
        "reacting_rk3": (W.reacting(n=70, ny=45, steps=1, precision="fp32", scheme=W.RK3), 200),
        "shear4": (W.shear_layer(n=90, ny=64, steps=1, precision="fp32"), 40),
        "two_step": (W.two_step(n=70, ny=33, precision="fp32"), 200),
        "outflow": (W.reacting(n=61, ny=33, steps=1, precision="fp32").with_(
            bc_x=W.OUTFLOW, bc_y=W.OUTFLOW), 200),
        "ragged": (W.reacting(n=65, ny=3, steps=1, precision="fp32"), 100),
    }[case]
    print("case", case, p.nx, p.ny, "S=%d" % p.S, "steps", steps, flush=True)
    sim = gpu_run(p, steps, "fp32")
    assert sim.get_option(D.DBM_OPT_STORAGE) == OM
    assert sim.get_option(D.DBM_OPT_PATH) == 0
    o, fo = oracle_run(p, steps)
    e = field_errors(p, sim.moments(), o.moments(fo))
    print("OM errors", {k: float("%.3e" % v) for k, v in e.items()}, flush=True)
    for k in ("rho", "u", "T"):
        assert e[k] < FP32_TOL, (k, e)


@pytest.mark.parametrize("n,ny,steps", [(64, 48, 300), (64, 64, 500)])
def test_om_storage_walls_and_force(n, ny, steps):
    """OM storage on the stratified Rayleigh-Taylor column (specular walls,
    gravity; references per grid row): rho, u (E1, the flow below 1% of the
    sound speed) and T within 1e-5, with either rounding."""
    p = W.rayleigh_taylor(n=n, ny=ny, steps=1, precision="fp32")
    o, fo = oracle_run(p, steps)
    mo = o.moments(fo)
    for opts in ({}, {D.DBM_OPT_ROUNDING: 1}):
        sim = gpu_run(p, steps, "fp32", options=opts)
        assert sim.get_option(D.DBM_OPT_STORAGE) == OM
        e = field_errors(p, sim.moments(), mo)
        print("OM walls+force", n, ny, steps, opts,
              {k: float("%.3e" % e[k]) for k in ("rho", "u", "u_cs", "T")}, flush=True)
        for k in ("rho", "u", "T"):
            assert e[k] < FP32_TOL, (k, e)


@pytest.mark.parametrize("case", ["reacting", "reacting_rk3", "shear4", "walls_force", "chain3",
                                  "ragged", "two_step", "outflow"])
def test_om_residual_storage_matches_oracle(case):
    """OM storage with A-block residuals (storage 2) against the FP64 oracle
    (E1 metric, 1e-5): both schemes, four species, walls and gravity with
    references per row, the chain wavefront, ragged sizes, two-step
    chemistry, outflow boundaries."""
    p, steps, opts = {
        "reacting": (W.reacting(n=70, ny=45, steps=1, precision="fp32"), 300, {}),
        "reacting_rk3": (W.reacting(n=70, ny=45, steps=1, precision="fp32", scheme=W.RK3), 200,
                         {}),
        "shear4": (W.shear_layer(n=90, ny=64, steps=1, precision="fp32"), 40, {}),
        "walls_force": (W.rayleigh_taylor(n=64, ny=48, steps=1, precision="fp32"), 300, {}),
        "chain3": (W.reacting(n=70, ny=45, steps=1, precision="fp32"), 200,
                   {D.DBM_OPT_CHAIN_WAVE: 2}),
        "ragged": (W.reacting(n=65, ny=3, steps=1, precision="fp32"), 100, {}),
        "two_step": (W.two_step(n=70, ny=33, precision="fp32"), 200, {}),
        "outflow": (W.reacting(n=61, ny=33, steps=1, precision="fp32").with_(
            bc_x=W.OUTFLOW, bc_y=W.OUTFLOW), 200, {}),
    }[case]
    print("case", case, p.nx, p.ny, "S=%d" % p.S, "steps", steps, flush=True)
    o = dict(opts)
    o[D.DBM_OPT_STORAGE] = ARES
    sim = gpu_run(p, steps, "fp32", options=o)
    assert sim.get_option(D.DBM_OPT_STORAGE) == ARES
    assert sim.get_option(D.DBM_OPT_PATH) == 0
    if case == "chain3":
        assert sim.get_option(D.DBM_OPT_CHAIN_WAVE) == 2
    om, fo = oracle_run(p, steps)
    e = field_errors(p, sim.moments(), om.moments(fo))
    print("OM + residual errors", {k: float("%.3e" % v) for k, v in e.items()}, flush=True)
    for k in ("rho", "u", "T"):
        assert e[k] < FP32_TOL, (k, e)


def test_om_residuals_reduce_the_density_and_energy_error():
    """On the stratified column over 500 steps the A-block residuals cut the
    density and temperature errors of OM storage (the rounding of mass and
    energy at each store no longer accumulates)."""
    p = W.rayleigh_taylor(n=64, ny=48, steps=1, precision="fp32")
    o, fo = oracle_run(p, 500)
    mo = o.moments(fo)
    e = {}
    for st in (OM, ARES):
        sim = gpu_run(p, 500, "fp32", options={D.DBM_OPT_STORAGE: st})
        assert sim.get_option(D.DBM_OPT_STORAGE) == st
        e[st] = field_errors(p, sim.moments(), mo)
        print("storage", st, {k: float("%.3e" % e[st][k]) for k in ("rho", "u", "T")}, flush=True)
    assert e[ARES]["rho"] < 0.5 * e[OM]["rho"], e
    assert e[ARES]["T"] < 0.5 * e[OM]["T"], e


def test_om_residual_tile_shape_and_form_do_not_change_bits():
    """Tile rows, the chain wavefront and graph replay leave every bit of the
    state with A-block residuals unchanged."""
    p = W.reacting(n=125, ny=41, steps=1, precision="fp32")
    ref = None
    for cw in (1, 2):
        for rows in (1, 3, 16):
            for graph in (1, 0):
                o = {D.DBM_OPT_STORAGE: ARES, D.DBM_OPT_CHAIN_WAVE: cw, D.DBM_OPT_GRAPH: graph}
                sim = gpu_run(p, 15, "fp32", tile_rows=rows, options=o)
                assert sim.get_option(D.DBM_OPT_STORAGE) == ARES
                f = sim.get_f()
                if ref is None:
                    ref = f
                else:
                    np.testing.assert_array_equal(f, ref, err_msg=str((cw, rows, graph)))


@pytest.mark.parametrize("storage,case", [(OM, "shear4"), (ARES, "shear4"), (OM, "walls")])
def test_om_drain_forms_do_not_change_bits(storage, case):
    """The OM kernel's two load forms (every other row waiting for its refill
    at once, or the refills kept in flight) give identical bits at any tile
    height, ragged last tiles included (also with walls and references per
    row); the option reads back as set."""
    if case == "shear4":
        p = W.shear_layer(n=125, ny=41, steps=1, precision="fp32")
    else:
        p = W.rayleigh_taylor(n=125, ny=41, steps=1, precision="fp32")
    ref = None
    for drain in (2, 1):
        for rows in (1, 2, 3, 7, 16):
            sim = gpu_run(p, 12, "fp32", tile_rows=rows,
                          options={D.DBM_OPT_STORAGE: storage, D.DBM_OPT_DRAIN: drain})
            assert sim.get_option(D.DBM_OPT_STORAGE) == storage
            assert sim.get_option(D.DBM_OPT_DRAIN) == drain
            f = sim.get_f()
            if ref is None:
                ref = f
            else:
                np.testing.assert_array_equal(f, ref, err_msg=str((drain, rows)))
    for drain in (2, 1):   # asked for with tuned tile rows: the tuner keeps it
        sim = gpu_run(p, 12, "fp32", options={D.DBM_OPT_STORAGE: storage, D.DBM_OPT_DRAIN: drain})
        assert sim.get_option(D.DBM_OPT_DRAIN) == drain
        np.testing.assert_array_equal(sim.get_f(), ref, err_msg="tuned rows, drain %d" % drain)


def test_om_and_plain_storage_agree_to_fp32_rounding():
    p = W.reacting(n=70, ny=45, steps=1, precision="fp32")
    a = gpu_run(p, 50, "fp32")
    b = gpu_run(p, 50, "fp32", options={D.DBM_OPT_STORAGE: PLAIN})
    assert a.get_option(D.DBM_OPT_STORAGE) == OM and b.get_option(D.DBM_OPT_STORAGE) == PLAIN
    d = f_error(a.get_f(), b.get_f())
    print("OM vs f storage after 50 steps: %.3e" % d, flush=True)
    assert 0 < d < 5e-6


@pytest.mark.parametrize("case", ["reacting3", "shear4"])
def test_om_tile_shape_and_form_do_not_change_bits(case):
    """Tile rows, the chain wavefront (three species) and graph replay leave
    every bit of the OM state unchanged."""
    if case == "reacting3":
        p = W.reacting(n=125, ny=41, steps=1, precision="fp32")
        forms = [{D.DBM_OPT_CHAIN_WAVE: 1}, {D.DBM_OPT_CHAIN_WAVE: 2}]
    else:
        p = W.shear_layer(n=125, ny=41, steps=1, precision="fp32")
        forms = [{}]
    ref = None
    for opts in forms:
        for rows in (1, 2, 3, 5, 16, 64):
            for graph in (1, 0):
                o = dict(opts)
                o[D.DBM_OPT_GRAPH] = graph
                sim = gpu_run(p, 15, "fp32", tile_rows=rows, options=o)
                assert sim.get_option(D.DBM_OPT_STORAGE) == OM
                f = sim.get_f()
                if ref is None:
                    ref = f
                else:
                    np.testing.assert_array_equal(f, ref, err_msg=str((opts, rows, graph)))
                if rows not in (1, 16):
                    break


def test_four_species_f_storage_ring_tile_rows_do_not_change_bits():
    """The four-species FP32 Euler form on f storage without the row pipeline
    keeps three rows of loads in flight: tile heights 1..7 (1, 2 and 3
    complete rings, the others end mid-ring; 45 rows leave ragged last tiles)
    give identical bits, within 1e-5 of the oracle (E1)."""
    p = W.shear_layer(n=70, ny=45, steps=1, precision="fp32")
    assert p.S == 4
    opts = {D.DBM_OPT_STORAGE: PLAIN, D.DBM_OPT_PIPELINE: 1}
    ref = None
    for rows in (1, 2, 3, 4, 5, 7):
        sim = gpu_run(p, 30, "fp32", tile_rows=rows, options=opts)
        assert sim.get_option(D.DBM_OPT_STORAGE) == PLAIN
        assert sim.get_option(D.DBM_OPT_PIPELINE) == 1
        assert sim.get_option(D.DBM_OPT_TILE_ROWS) == rows
        f = sim.get_f()
        if ref is None:
            ref = f
            o, fo = oracle_run(p, 30)
            e = field_errors(p, sim.moments(), o.moments(fo))
            print("f storage, 4 species, 30 steps", {k: float("%.3e" % v) for k, v in e.items()},
                  flush=True)
            for k in ("rho", "u", "T"):
                assert e[k] < FP32_TOL, (k, e)
        else:
            np.testing.assert_array_equal(f, ref, err_msg="tile rows %d" % rows)


def test_conversion_between_representations():
    """Converting the state to f itself and back changes it by FP32 rounding
    only; stepping on OM storage afterwards stays within 1e-5 of the oracle
    (E1), and so does stepping on f storage on rho, T and u against the sound
    speed."""
    p = W.reacting(n=70, ny=45, steps=1, precision="fp32")
    sim = gpu_run(p, 20, "fp32")
    f_om = sim.get_f()
    sim.set_option(D.DBM_OPT_STORAGE, PLAIN)
    assert sim.get_option(D.DBM_OPT_STORAGE) == PLAIN
    f_pl = sim.get_f()
    assert f_error(f_pl, f_om) < 2e-7
    sim.set_option(D.DBM_OPT_STORAGE, OM)
    assert sim.get_option(D.DBM_OPT_STORAGE) == OM
    assert f_error(sim.get_f(), f_om) < 4e-7
    sim.step(40)
    o, fo = oracle_run(p, 60)
    e = field_errors(p, sim.moments(), o.moments(fo))
    for k in ("rho", "u", "T"):
        assert e[k] < FP32_TOL, (k, e)
    sim.set_option(D.DBM_OPT_STORAGE, PLAIN)
    sim.step(20)
    o, fo = oracle_run(p, 80)
    e = field_errors(p, sim.moments(), o.moments(fo))
    for k in ("rho", "u_cs", "T"):
        assert e[k] < FP32_TOL, (k, e)


def test_conversion_to_and_from_residual_storage():
    """OM storage -> with A-block residuals keeps the state to FP64 rounding
    of the stored values; -> f storage and back rounds it to FP32 (B, X, Y
    carry no residual); the residual storage then steps within 1e-5 of the
    oracle (E1)."""
    p = W.reacting(n=70, ny=45, steps=1, precision="fp32")
    sim = gpu_run(p, 20, "fp32")
    f_om = sim.get_f()
    sim.set_option(D.DBM_OPT_STORAGE, ARES)
    assert sim.get_option(D.DBM_OPT_STORAGE) == ARES
    assert f_error(sim.get_f(), f_om) < 1e-12
    sim.set_option(D.DBM_OPT_STORAGE, PLAIN)
    f_pl = sim.get_f()
    assert f_error(f_pl, f_om) < 2e-7
    sim.set_option(D.DBM_OPT_STORAGE, ARES)
    assert f_error(sim.get_f(), f_pl) < 2e-7
    sim.step(40)
    o, fo = oracle_run(p, 60)
    e = field_errors(p, sim.moments(), o.moments(fo))
    for k in ("rho", "u", "T"):
        assert e[k] < FP32_TOL, (k, e)
    f_ar = sim.get_f()
    sim.set_option(D.DBM_OPT_STORAGE, OM)
    assert sim.get_option(D.DBM_OPT_STORAGE) == OM
    assert f_error(sim.get_f(), f_ar) < 2e-7


def test_om_set_f_get_f_round_trip():
    """An arbitrary non-equilibrium f written with dbm_set_f and read back
    agrees to FP32 rounding of the stored values (and closer with A-block
    residuals, which carry mass and energy to about 33 bits)."""
    p = W.reacting(n=67, ny=23, steps=1, precision="fp32")
    rng = np.random.default_rng(2006)
    f = 0.02 * (0.5 + rng.random((p.S, 16, p.ny, p.nx)))
    f[1] *= 3.0
    sim = D.Simulation(p, precision="fp32")
    assert sim.get_option(D.DBM_OPT_STORAGE) == OM
    sim.set_f(f)
    g = sim.get_f()
    assert f_error(g, f) < 1e-6
    sim.set_option(D.DBM_OPT_STORAGE, ARES)
    sim.set_f(f)
    h = sim.get_f()
    assert f_error(h, f) < 1e-6
    mass = lambda x: x.sum(axis=(1, 2, 3))
    assert np.abs(mass(h) - mass(f)).max() < 1e-9 * np.abs(mass(f)).max()


@pytest.mark.parametrize("prec,opts", [("fp64", {}), ("fp32", {}), ("fp32x", {}),
                                       ("fp32", {D.DBM_OPT_STORAGE: PLAIN}),
                                       ("fp32", {D.DBM_OPT_ROUNDING: 1}),
                                       ("fp32", {D.DBM_OPT_STORAGE: ARES})])
def test_checkpoint_restart_is_bit_exact(prec, opts):
    """N steps equal N/2 steps, a saved state loaded into a new handle, and
    N/2 more steps, bit for bit (walls, force; every storage)."""
    p = W.rayleigh_taylor(n=64, ny=40, steps=1, precision=prec)
    a = gpu_run(p, 20, prec, options=opts)
    b = gpu_run(p, 10, prec, options=opts)
    blob = b.save_state()
    c = D.Simulation(p, precision=prec)
    for k, v in opts.items():
        c.set_option(k, v)
    c.load_state(blob)
    c.step(10)
    np.testing.assert_array_equal(a.get_f(), c.get_f())


def test_load_state_rejects_a_blob_of_another_configuration():
    p = W.reacting(n=64, ny=20, steps=1, precision="fp32")
    a = gpu_run(p, 2, "fp32")
    blob = a.save_state()
    for q, prec, opts in ((p.with_(nx=65), "fp32", {}), (p, "fp64", {}),
                          (p, "fp32", {D.DBM_OPT_STORAGE: PLAIN}),
                          (p, "fp32", {D.DBM_OPT_STORAGE: ARES})):
        b = D.Simulation(q, precision=prec)
        for k, v in opts.items():
            b.set_option(k, v)
        with pytest.raises(D.DbmError) as e:
            b.load_state(blob)
        assert e.value.code == D.DBM_ERR_ARG
    with pytest.raises(D.DbmError):
        a.load_state(blob[:100])
