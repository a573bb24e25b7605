"""The C oracle against a second, independently written NumPy statement of the
same update, on tiny grids (the two share no code)."""
import numpy as np
import pytest

from numpy_dbm import NumpyDBM
from oracle import oracle as O
from paper_2006_15932_amd import workloads as W


def _random_fields(p, seed, umax=0.3):
    r = W.splitmix64(seed, (p.S + 3) * p.cells).reshape(p.S + 3, p.ny, p.nx)
    n_sp = np.stack([(0.5 + 0.5 * r[s]) / p.species[s].m for s in range(p.S)])
    return p.with_(n_sp=n_sp, ux=umax * (2 * r[p.S] - 1), uy=umax * (2 * r[p.S + 1] - 1),
                   T=0.8 + 0.6 * r[p.S + 2])


CASES = {
    "react-force-wall-euler": dict(
        species=[W.make_species(2.0, a=-2), W.make_species(32.0, I=1.0, a=-1),
                 W.make_species(18.0, I=5.0, a=2)],
        nx=7, ny=6, bc_x=W.PERIODIC, bc_y=W.WALL, accel=(0.3, -0.6),
        reaction=dict(fuel=0, oxid=1, k_ov=5e5, Ea_over_R=2.0, Q=4.0), steps=5),
    "outflow-wallx-rk3-nolimiter-Tsame": dict(
        species=[W.make_species(1.0), W.make_species(3.0, I=2.0)],
        nx=6, ny=5, bc_x=W.WALL, bc_y=W.OUTFLOW, accel=(-0.4, 0.2), scheme=W.RK3,
        limiter=W.LIM_NONE, force_T_mode=W.FORCE_T_SAME, steps=3),
    "periodic-react-rk3": dict(
        species=[W.make_species(2.0, a=-2), W.make_species(32.0, a=-1),
                 W.make_species(18.0, a=2), W.make_species(28.0)],
        nx=8, ny=8, reaction=dict(W.C1_CHEM), scheme=W.RK3, steps=2),
}


@pytest.mark.parametrize("name", list(CASES))
def test_c_oracle_matches_numpy_transcription(name):
    kw = dict(CASES[name])
    species, nx, ny, steps = kw.pop("species"), kw.pop("nx"), kw.pop("ny"), kw.pop("steps")
    p = _random_fields(W.Problem(name, nx, ny, species, dt=2e-6, **kw), seed=sum(map(ord, name)))
    o, nd = O.Oracle(p), NumpyDBM(p)
    f0 = o.init_equilibrium(*W.fields(p))
    g0 = nd.init(*W.fields(p))
    scale = np.abs(f0).max()
    assert np.abs(f0 - g0).max() < 1e-13 * scale
    # perturb away from equilibrium so that every term is exercised
    r = W.splitmix64(7, f0.size).reshape(f0.shape)
    f0 = f0 + 0.02 * scale * (2 * r - 1)
    np.testing.assert_allclose(o.rhs(f0), nd.L(f0), rtol=0, atol=1e-12 * np.abs(nd.L(f0)).max())
    f1, g1 = o.run(f0, steps), nd.run(f0, steps)
    assert np.abs(f1 - g1).max() < 1e-13 * scale
