"""A second, independent, vectorised NumPy statement of the D2V16 update.

Written separately from the C oracle (different structure: whole-array NumPy,
moments via matrix products, ghost cells via np.pad-style index maps) so that
a transcription slip in either one shows up as a disagreement on tiny grids.
Test infrastructure only.
"""
import numpy as np


def velocity_set(sp):
    ax = [(1, 0), (0, 1), (-1, 0), (0, -1)]
    dg = [(1, 1), (-1, 1), (-1, -1), (1, -1)]
    vx, vy, eta = [], [], []
    for g in range(4):
        for d in (ax if g in (0, 2) else dg):
            vx.append(sp.v[g] * d[0])
            vy.append(sp.v[g] * d[1])
            eta.append(sp.eta[g])
    return np.array(vx), np.array(vy), np.array(eta)


def moment_rows(vx, vy, eta):
    q = vx ** 2 + vy ** 2 + eta ** 2
    return np.array([vx ** 0, vx, vy, q, vx ** 2, vx * vy, vy ** 2, q * vx, q * vy, vx ** 3,
                     vx ** 2 * vy, vx * vy ** 2, vy ** 3, q * vx ** 2, q * vx * vy, q * vy ** 2])


def fhat(n, ux, uy, th, I):
    K = 2.0 + I
    u2 = ux ** 2 + uy ** 2
    return np.array([
        n, n * ux, n * uy, n * (K * th + u2), n * (th + ux ** 2), n * ux * uy,
        n * (th + uy ** 2), n * ux * ((K + 2) * th + u2), n * uy * ((K + 2) * th + u2),
        n * ux * (3 * th + ux ** 2), n * uy * (th + ux ** 2), n * ux * (th + uy ** 2),
        n * uy * (3 * th + uy ** 2),
        n * th * ((K + 2) * th + u2) + n * ux ** 2 * ((K + 4) * th + u2),
        n * ux * uy * ((K + 4) * th + u2),
        n * th * ((K + 2) * th + u2) + n * uy ** 2 * ((K + 4) * th + u2)])


class NumpyDBM:
    def __init__(self, p):
        self.p = p
        self.tab = []
        for sp in p.species:
            vx, vy, eta = velocity_set(sp)
            M = moment_rows(vx, vy, eta)
            mx = [int(np.where((vx == -vx[i]) & (vy == vy[i]))[0][0]) for i in range(16)]
            my = [int(np.where((vx == vx[i]) & (vy == -vy[i]))[0][0]) for i in range(16)]
            self.tab.append(dict(vx=vx, vy=vy, q=vx ** 2 + vy ** 2 + eta ** 2, M=M,
                                 Minv=np.linalg.inv(M), mx=mx, my=my))

    def feq(self, s, n, ux, uy, T):
        sp = self.p.species[s]
        h = fhat(n, ux, uy, T / sp.m, sp.I)
        return np.tensordot(self.tab[s]["Minv"], h, axes=(1, 0))

    def init(self, n_sp, ux, uy, T):
        return np.stack([self.feq(s, n_sp[s], ux, uy, T) for s in range(self.p.S)])

    def _axis_map(self, n, bc):
        idx = np.arange(-2, n + 2)
        flip = np.zeros(n + 4, dtype=bool)
        if bc == 0:
            return idx % n, flip
        if bc == 1:
            return np.clip(idx, 0, n - 1), flip
        out = idx.copy()
        for k in range(n + 4):
            j, fl = out[k], False
            while j < 0 or j >= n:
                j = -1 - j if j < 0 else 2 * n - 1 - j
                fl = not fl
            out[k], flip[k] = j, fl
        return out, flip

    def convection(self, f):
        p = self.p
        xm, xf = self._axis_map(p.nx, p.bc_x)
        ym, yf = self._axis_map(p.ny, p.bc_y)
        C = np.zeros_like(f)
        mm = lambda a, b: np.where(a * b > 0, np.where(np.abs(a) < np.abs(b), a, b), 0.0)
        for s in range(p.S):
            t = self.tab[s]
            for i in range(16):
                P = np.empty((p.ny + 4, p.nx + 4))
                for a in range(p.ny + 4):
                    for b in range(p.nx + 4):
                        k = i
                        if xf[b]:
                            k = t["mx"][k]
                        if yf[a]:
                            k = t["my"][k]
                        P[a, b] = f[s, k, ym[a], xm[b]]
                out = np.zeros((p.ny, p.nx))
                for axis, v, h in ((1, t["vx"][i], p.dx), (0, t["vy"][i], p.dy)):
                    if v == 0:
                        continue
                    g = np.moveaxis(P, axis, 0)
                    d = g[1:] - g[:-1]                      # d[j] = g[j+1] - g[j]
                    if v > 0:
                        # interface j+1/2 for padded j = 1 .. n+2
                        sl = mm(d[:-1], d[1:]) if p.limiter == 0 else d[:-1]
                        face = g[1:-1] + 0.5 * sl           # faces right of padded 1..n+2
                    else:
                        sl = mm(d[1:-1], d[2:]) if p.limiter == 0 else d[2:]
                        face = g[2:-1] - 0.5 * sl           # faces right of padded 1..n+1
                        face = np.concatenate([face, face[-1:]], axis=0)
                    deriv = (face[1:-1] - face[:-2]) / h    # cells padded 2 .. n+1
                    deriv = np.moveaxis(deriv, 0, axis)
                    if axis == 1:
                        deriv = deriv[2:-2, :]
                    else:
                        deriv = deriv[:, 2:-2]
                    out -= v * deriv
                C[s, i] = out
        return C

    def source(self, f):
        p = self.p
        S = p.S
        n = np.array([f[s].sum(0) for s in range(S)])
        jx = np.array([np.tensordot(self.tab[s]["vx"], f[s], 1) for s in range(S)])
        jy = np.array([np.tensordot(self.tab[s]["vy"], f[s], 1) for s in range(S)])
        E = np.array([np.tensordot(self.tab[s]["q"], f[s], 1) for s in range(S)])
        m = np.array([sp.m for sp in p.species])[:, None, None]
        K = np.array([2.0 + sp.I for sp in p.species])[:, None, None]
        rho = (m * n).sum(0)
        ux, uy = (m * jx).sum(0) / rho, (m * jy).sum(0) / rho
        T = ((m * E).sum(0) - rho * (ux ** 2 + uy ** 2)) / (K * n).sum(0)
        ns, Ts = n.copy(), T.copy()
        if p.reaction is not None:
            r = p.reaction
            a = np.array([sp.a for sp in p.species])
            w = r["k_ov"] * np.maximum(n[r["fuel"]], 0) * np.maximum(n[r["oxid"]], 0) * np.exp(-r["Ea_over_R"] / T)
            xi = w * p.species[0].tau
            for s in range(S):
                if a[s] < 0:
                    xi = np.minimum(xi, np.maximum(n[s], 0) / -a[s])
            ns = n + a[:, None, None] * xi
            Ts = (T * (K * n).sum(0) + 2 * r.get("Q", 0.0) * xi) / (K * ns).sum(0)
        ax, ay = p.accel
        out = np.zeros_like(f)
        for s in range(S):
            sp = p.species[s]
            g = fhat(ns[s], ux, uy, Ts / sp.m, sp.I)
            if ax != 0 or ay != 0:
                us, vs = jx[s] / n[s], jy[s] / n[s]
                Tsp = sp.m * (E[s] / n[s] - us ** 2 - vs ** 2) / (2 + sp.I)
                Td = Tsp - (sp.m * sp.tau ** 2 * (ax ** 2 + ay ** 2) / (2 + sp.I)
                            if p.force_T_mode == 0 else 0.0)
                g = g + fhat(n[s], us + sp.tau * ax, vs + sp.tau * ay, Td / sp.m, sp.I) \
                    - fhat(n[s], us, vs, Tsp / sp.m, sp.I)
            feq = np.tensordot(self.tab[s]["Minv"], g, axes=(1, 0))
            out[s] = (feq - f[s]) / sp.tau
        return out

    def L(self, f):
        return self.convection(f) + self.source(f)

    def run(self, f, steps):
        dt = self.p.dt
        for _ in range(steps):
            if self.p.scheme == 0:
                f = f + dt * self.L(f)
            else:
                f1 = f + dt * self.L(f)
                f2 = 0.75 * f + 0.25 * (f1 + dt * self.L(f1))
                f = f / 3.0 + 2.0 / 3.0 * (f2 + dt * self.L(f2))
        return f
