"""Inputs of the one-dimensional validations (synthetic, invariant forms of
the paper's shock, reacting-wave and free-falling-box tests), shared by the
oracle pins and the GPU tests.  Rankine-Hugoniot states are the textbook
normal-shock relations for a perfect gas."""
import math

import numpy as np

from paper_2006_15932_amd import workloads as W


def normal_shock(M1, gamma):
    """Density, velocity and pressure ratios across a normal shock."""
    g = gamma
    r = (g + 1) * M1 * M1 / ((g - 1) * M1 * M1 + 2)
    pr = 1 + 2 * g / (g + 1) * (M1 * M1 - 1)
    return r, 1.0 / r, pr


def stationary_shock(nx=400, M1=1.3, T1=0.5, I=3.0, x_shock=200, steps=2000):
    """Two identical species (m = 1) carrying a normal shock at rest in the
    middle of an outflow tube: upstream (x < x_shock) density 1, temperature
    T1, speed M1 c1; downstream the Rankine-Hugoniot state, gamma =
    (D+I+2)/(D+I)."""
    K = 2.0 + I
    gamma = (K + 2) / K
    sp = [W.make_species(1.0, I=I), W.make_species(1.0, I=I)]
    c1 = math.sqrt(gamma * T1)           # p = n T, rho = n (m = 1)
    u1 = M1 * c1
    r, ur, pr = normal_shock(M1, gamma)
    rho2, u2, p2 = r, u1 * ur, pr * T1
    T2 = p2 / rho2
    x = np.arange(nx)
    up = x < x_shock
    rho = np.where(up, 1.0, rho2)
    n_sp = np.stack([0.5 * rho, 0.5 * rho])[:, None, :]
    ux = np.where(up, u1, u2)[None, :]
    T = np.where(up, T1, T2)[None, :]
    p = W.Problem("shock", nx, 1, sp, dt=1e-5, bc_x=W.OUTFLOW, bc_y=W.PERIODIC,
                  steps=steps, n_sp=n_sp, ux=ux, uy=np.zeros((1, nx)), T=T)
    return p, dict(rho1=1.0, u1=u1, T1=T1, rho2=rho2, u2=u2, T2=T2, x_shock=x_shock)


def reacting_wave(nx=200, Q=20.0, steps=800, t_hot=3.5, precision="fp64"):
    """Periodic 1-D premix of the reacting configuration (2 F + O -> 2 P) with
    heat release Q per unit extent, ignited by a hot Gaussian in the middle."""
    p = W.reacting(n=nx, ny=1, steps=steps, t_hot=t_hot, precision=precision)
    chem = dict(p.reaction)
    chem["Q"] = Q
    return p.with_(reaction=chem)


def free_falling_reacting_box(n=8, Q=20.0, g=(0.3, -0.5), T=3.0, steps=300):
    """Uniform reacting premix in a periodic box under a uniform force."""
    p = W.reacting(n=n, ny=n, steps=steps)
    chem = dict(p.reaction)
    chem["Q"] = Q
    shape = (p.ny, p.nx)
    n_sp = np.stack([np.full(shape, float(p.n_sp[s].mean())) for s in range(p.S)])
    return p.with_(reaction=chem, accel=g, n_sp=n_sp, ux=np.zeros(shape), uy=np.zeros(shape),
                   T=np.full(shape, T))


def shock_position(rho, rho1, rho2):
    """Fractional cell index where the density crosses the mean of the two
    plateaus (linear interpolation between cell centres)."""
    mid = 0.5 * (rho1 + rho2)
    j = int(np.argmax(rho > mid))
    return j - 1 + (mid - rho[j - 1]) / (rho[j] - rho[j - 1])


def two_step_wave(nx=200, steps=600, precision="fp64"):
    """Periodic 1-D premix with the two-step mechanism (both steps release
    heat), ignited by a hot Gaussian."""
    return W.two_step(n=nx, ny=1, steps=steps, precision=precision)


def two_step_release(p, n0, n1):
    """Chemical energy released between species counts n0 and n1 (per
    species, integrated): step 1 uses one O, so xi_1 = -dN_O; both steps use
    one F, so xi_2 = -dN_F - xi_1."""
    x1 = n0[1] - n1[1]
    x2 = (n0[0] - n1[0]) - x1
    return p.mechanism[0]["Q"] * x1 + p.mechanism[1]["Q"] * x2, x1, x2
