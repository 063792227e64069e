"""A second, independent transcription of one coupled-LB time step, in NumPy.

Test infrastructure: written from the paper's Sec. 2-3 and the readings the
step takes (div u = the central difference of the previous velocity, the
freezing term of eq. (fluid2), E_ref in the enthalpy equilibrium, the
geometric wetting ghost, halfway bounce-back and non-equilibrium
extrapolation at the wall-normal faces), as whole-array operations over the
grid instead of the oracle's cell loops.  It shares nothing with the C
oracle but the parameter dict and the state layout, and the oracle is
checked against it element by element.

State layout (as the oracle's): populations (nlat*Q, nz, ny, nx), lattice 0 =
f, 1..N = g_p, N+1 = h, post-stream values; lagged fields (N + dim + 3,
nz, ny, nx) = phi_p^{n-1}, f_s^{n-1}, u^{n-1}, D^{n-1}, q^{n-1}.
"""
from __future__ import annotations

import numpy as np

WALL, OPEN = "wall", "open"


def lattice(dim):
    """D2Q9 or D3Q19 directions (the order of the requirements) and weights."""
    if dim == 2:
        c = [(0, 0, 0), (1, 0, 0), (0, 1, 0), (-1, 0, 0), (0, -1, 0),
             (1, 1, 0), (-1, 1, 0), (-1, -1, 0), (1, -1, 0)]
        w = [4 / 9] + [1 / 9] * 4 + [1 / 36] * 4
    else:
        c = [(0, 0, 0), (1, 0, 0), (-1, 0, 0), (0, 1, 0), (0, -1, 0), (0, 0, 1), (0, 0, -1),
             (1, 1, 0), (-1, -1, 0), (1, -1, 0), (-1, 1, 0),
             (1, 0, 1), (-1, 0, -1), (1, 0, -1), (-1, 0, 1),
             (0, 1, 1), (0, -1, -1), (0, 1, -1), (0, -1, 1)]
        w = [1 / 3] + [1 / 18] * 6 + [1 / 36] * 12
    c = np.array(c, dtype=np.int64)
    w = np.array(w)
    opp = [int(np.flatnonzero((c == -ci).all(axis=1))[0]) for ci in c]
    return c, w, np.array(opp)


class Step:
    """One step of the method on a state (pop, aux) -> (pop, aux)."""

    def __init__(self, prm):
        self.P = prm
        self.d = prm["dim"]
        self.N = prm["nphase"]
        self.c, self.w, self.opp = lattice(self.d)
        self.Q = len(self.w)
        # array axes (z, y, x): x -> 2, y -> 1, z -> 0; wall-normal = y (2D) or z (3D)
        self.ax = {0: 2, 1: 1, 2: 0}
        self.wn = self.d - 1
        self.wn_ax = self.ax[self.wn]
        self.lat_dims = [a for a in range(self.d) if a != self.wn]

    # ---------- helpers ----------
    def mix(self, phi, fs, key):
        s, l = self.P[key + "_s"], self.P[key + "_l"]
        return sum(fs * phi[p] * s[p] + (1 - fs) * phi[p] * l[p] for p in range(self.N))

    def thresholds(self, phi):
        P, N = self.P, self.N
        rs = sum(phi[p] * P["rho_s"][p] for p in range(N))
        rl = sum(phi[p] * P["rho_l"][p] for p in range(N))
        cs = sum(phi[p] * P["cp_s"][p] for p in range(N))
        cl = sum(phi[p] * P["cp_l"][p] for p in range(N))
        Lv = sum(phi[p] * P["rho_l"][p] * P["latent"][p] for p in range(N))
        Tm = P["T_melt"]
        return rs * cs, rl * cl, rs * cs * Tm, rl * cl * Tm + Lv

    def invert(self, phi, rhoH):
        """Eq. (H) with the mixture's solid and liquid states."""
        a_s, a_l, Es, El = self.thresholds(phi)
        Tm = self.P["T_melt"]
        with np.errstate(divide="ignore", invalid="ignore"):
            fl_mid = np.where(El > Es, (rhoH - Es) / np.where(El > Es, El - Es, 1.0), 1.0)
            T = np.where(rhoH < Es, rhoH / a_s, np.where(rhoH > El, Tm + (rhoH - El) / a_l, Tm))
        fl = np.where(rhoH < Es, 0.0, np.where(rhoH > El, 1.0, fl_mid))
        return T, fl

    def heq(self, i, rhoH, T, rhocp, u):
        E = self.P["E_ref"]
        uu = sum(u[a] ** 2 for a in range(self.d))
        if i == 0:
            return rhoH - E * T + self.w[0] * (E * T - 1.5 * rhocp * T * uu)
        cu = sum(self.c[i, a] * u[a] for a in range(self.d))
        return self.w[i] * (E * T + rhocp * T * (3 * cu + 4.5 * cu * cu - 1.5 * uu))

    def s_i(self, i, u):
        uu = sum(u[a] ** 2 for a in range(self.d))
        cu = sum(self.c[i, a] * u[a] for a in range(self.d))
        return self.w[i] * (3 * cu + 4.5 * cu * cu - 1.5 * uu)

    def feq(self, i, p, rho, u):
        base = 3 * p * (self.w[0] - 1) if i == 0 else 3 * p * self.w[i]
        return base + rho * self.s_i(i, u)

    def geq(self, i, phi, u):
        cu = sum(self.c[i, a] * u[a] for a in range(self.d))
        return self.w[i] * phi * (1 + 3 * cu)

    def shift_nb(self, padded, i):
        """X(x + c_i) for every cell, from an array padded by one ghost layer
        on each wall-normal side; periodic along the lateral axes."""
        ci = self.c[i]
        out = padded
        for a in self.lat_dims:
            out = np.roll(out, -ci[a], axis=self.ax[a])
        n = padded.shape[self.wn_ax] - 2
        sl = [slice(None)] * 3
        sl[self.wn_ax] = slice(1 + ci[self.wn], 1 + ci[self.wn] + n)
        return out[tuple(sl)]

    def pad(self, X, lo, hi):
        return np.concatenate([lo, X, hi], axis=self.wn_ax)

    def layer(self, X, k):
        sl = [slice(None)] * 3
        sl[self.wn_ax] = slice(k, k + 1) if k >= 0 else slice(k, k + 1 if k != -1 else None)
        return X[tuple(sl)]

    def grad(self, Xp):
        g = []
        for a in range(self.d):
            g.append(3 * sum(self.w[i] * self.c[i, a] * self.shift_nb(Xp, i) for i in range(self.Q)))
        return g

    def lap(self, Xp, X):
        return 6 * sum(self.w[i] * (self.shift_nb(Xp, i) - X) for i in range(self.Q))

    # ---------- the step ----------
    def __call__(self, pop, aux):
        P, N, d, Q, c, w = self.P, self.N, self.d, self.Q, self.c, self.w
        f = pop[0:Q]
        g = [pop[(1 + p) * Q:(2 + p) * Q] for p in range(N)]
        h = pop[(N + 1) * Q:(N + 2) * Q]
        phi_prev = aux[0:N]
        fs_prev = aux[N]
        u_prev = aux[N + 1:N + 1 + d]
        D_prev = aux[N + 1 + d]
        q_prev = aux[N + 2 + d]

        # moments (Sec. 3): phi_p = sum g / (1 - D/2), rho H = sum h + q/2
        phi = np.array([g[p].sum(axis=0) / (1 - 0.5 * D_prev) for p in range(N)])
        rhoH = h.sum(axis=0) + 0.5 * q_prev
        T, fl = self.invert(phi, rhoH)
        fs = 1 - fl
        psi = sum(phi[p] for p in range(N) if P["freezes"][p])
        rho = self.mix(phi, fs, "rho")
        mu = self.mix(phi, fs, "mu")
        lam = self.mix(phi, fs, "lam")
        cp = self.mix(phi, fs, "cp")

        # ghost layers: wetting at a low wall, copies elsewhere; u mirrored at walls
        lo_b = [self.layer(X, 0) for X in phi]
        hi_b = [self.layer(X, -1) for X in phi]
        if P["flow_bc"][0] == WALL:
            ct = np.array(P["cos_theta"])
            lo_g = []
            for p in range(N):
                s = sum(lo_b[p] * lo_b[q] * ct[p][q] for q in range(N) if q != p)
                lo_g.append(lo_b[p] + 4 / P["eps"] * s)
        else:
            lo_g = lo_b
        phip = [self.pad(phi[p], lo_g[p], hi_b[p]) for p in range(N)]
        fsp = self.pad(fs, self.layer(fs, 0), self.layer(fs, -1))
        rhop = self.pad(rho, self.layer(rho, 0), self.layer(rho, -1))
        gphi = [self.grad(phip[p]) for p in range(N)]
        lphi = [self.lap(phip[p], phi[p]) for p in range(N)]
        grho = self.grad(rhop)
        gfp = []
        for p in range(N):
            gfp.append(self.grad(fsp * phip[p]) if P["freezes"][p] else [0 * rho] * d)
        sg = [-1.0 if P["flow_bc"][k] == WALL else 1.0 for k in range(2)]
        D = 0
        for a in range(d):
            up = self.pad(u_prev[a], sg[0] * self.layer(u_prev[a], 0), sg[1] * self.layer(u_prev[a], -1))
            D = D + self.grad(up)[a]

        # interface physics (Sec. 2)
        Rv = [[0 * rho for _ in range(d)] for _ in range(N)]
        for p in range(N):
            for q in range(p + 1, N):
                v = [phi[q] * gphi[p][a] - phi[p] * gphi[q][a] for a in range(d)]
                nrm = np.sqrt(sum(x * x for x in v) + 1e-24)
                k = 4 * phi[p] * phi[q] / P["eps"]
                for a in range(d):
                    Rv[p][a] = Rv[p][a] + k * (v[a] / nrm)
                    Rv[q][a] = Rv[q][a] - k * (v[a] / nrm)
        gpr = lambda x: 2 * x * (1 - x) * (1 - 2 * x)
        sig = np.array(P["sigma"])
        mup = []
        for p in range(N):
            b = sum(2 * (3 * sig[p][q] / P["eps"]) * (gpr(phi[p]) - gpr(phi[p] + phi[q]))
                    for q in range(N) if q != p)
            k = sum((-0.75 * P["eps"] * sig[p][q]) * lphi[q] for q in range(N) if q != p)
            mup.append(b - k)
        F = [sum(mup[p] * gphi[p][a] for p in range(N)) + rho * P["gravity"][a] for a in range(d)]

        # flow macros
        mom = [sum(c[i, a] * f[i] for i in range(Q)) for a in range(d)]
        ws = fs * psi
        ustar = [(mom[a] + 0.5 * F[a]) / rho for a in range(d)]
        acc = [ws * (0 - ustar[a]) for a in range(d)]
        u = [ustar[a] + 0.5 * acc[a] for a in range(d)]
        rhoa = [rho * acc[a] for a in range(d)]
        msum = 0
        for p in range(N):
            if not P["freezes"][p]:
                continue
            adv = sum(u[a] * gfp[p][a] for a in range(d))
            msum = msum + (P["rho_s"][p] - P["rho_l"][p]) * (fs * phi[p] - fs_prev * phi_prev[p] + adv)
        mdot = -msum / rho
        S = rho * mdot + sum(u[a] * grho[a] for a in range(d))
        lam_iso = (2.0 / d) * rho * (1.0 / 3.0) * S
        Fi = []
        for i in range(Q):
            cF = sum(c[i, a] * (F[a] + rhoa[a]) for a in range(d))
            qq = 0
            for a in range(d):
                for b in range(d):
                    L = u[a] * F[b] + F[a] * u[b] + (lam_iso if a == b else 0)
                    qq = qq + (c[i, a] * c[i, b] - (1 / 3 if a == b else 0)) * L
            Fi.append(w[i] * (S + 3 * cF + 4.5 * qq))
        tau_f = 3 * mu / rho + 0.5
        pr = (1 / 3) / (1 - w[0]) * (sum(f[i] for i in range(1, Q)) + 0.5 * S
                                     + (tau_f - 0.5) * Fi[0] + rho * self.s_i(0, u))

        # collisions
        fe = [self.feq(i, pr, rho, u) for i in range(Q)]
        postf = [f[i] - (f[i] - fe[i]) / tau_f + (1 - 0.5 / tau_f) * Fi[i] for i in range(Q)]
        tg = P["tau_g"]
        postg, ge = [], []
        for p in range(N):
            dpu = [phi[p] * u[a] - phi_prev[p] * u_prev[a] for a in range(d)]
            gp, gep = [], []
            for i in range(Q):
                cd = sum(c[i, a] * dpu[a] for a in range(d))
                cr = sum(c[i, a] * Rv[p][a] for a in range(d))
                Gi = w[i] * (3 * cd + cr) + w[i] * phi[p] * D
                gei = self.geq(i, phi[p], u)
                gep.append(gei)
                gp.append(g[p][i] - (g[p][i] - gei) / tg + (1 - 0.5 / tg) * Gi)
            postg.append(gp)
            ge.append(gep)
        rhocp = rho * cp
        tau_h = 3 * lam / P["E_ref"] + 0.5
        he = [self.heq(i, rhoH, T, rhocp, u) for i in range(Q)]
        posth = [h[i] - (h[i] - he[i]) / tau_h + (1 - 0.5 / tau_h) * (w[i] * rhocp * T * D) for i in range(Q)]

        # incoming values on the wall-normal faces, per face and direction
        bc = {}
        for face in (0, 1):
            k = 0 if face == 0 else -1
            into = 1 if face == 0 else -1
            L = lambda X: self.layer(X, k)
            uL = [L(x) for x in u]
            for i in range(Q):
                if c[i, self.wn] != into:
                    continue
                o = self.opp[i]
                vals = []
                if P["flow_bc"][face] == WALL:
                    vals.append(L(postf[o]))
                    vals += [L(postg[p][o]) for p in range(N)]
                else:
                    fg = self.feq(i, 0 * L(rho), L(rho), uL)
                    vals.append(fg + (1 - 1 / L(tau_f)) * (L(f[i]) - L(fe[i])))
                    for p in range(N):
                        vals.append(L(ge[p][i]) + (1 - 1 / tg) * (L(g[p][i]) - L(ge[p][i])))
                if P["flow_bc"][face] == WALL and P["therm_bc"][face] == "adiabatic":
                    vals.append(L(posth[o]))
                else:
                    Tg = 2 * P["T_face"][face] - L(T) if P["therm_bc"][face] == "dirichlet" else L(T)
                    ug = uL if P["flow_bc"][face] == OPEN else [0 * uL[0]] * d
                    hg = self.heq(i, 0.0, Tg, L(rhocp), ug)
                    vals.append(hg + (1 - 1 / L(tau_h)) * (L(h[i]) - L(he[i])))
                bc[(face, i)] = vals

        # streaming: value at x for direction i comes from x - c_i
        posts = [postf] + postg + [posth]
        new = np.empty_like(pop)
        n = pop.shape[1 + self.wn_ax]
        for i in range(Q):
            ci = c[i]
            for l, post in enumerate(posts):
                X = post[i]
                for a in self.lat_dims:
                    X = np.roll(X, ci[a], axis=self.ax[a])
                X = np.roll(X, ci[self.wn], axis=self.wn_ax)
                if ci[self.wn] == 1:
                    sl = [slice(None)] * 3
                    sl[self.wn_ax] = slice(0, 1)
                    X[tuple(sl)] = bc[(0, i)][l]
                elif ci[self.wn] == -1:
                    sl = [slice(None)] * 3
                    sl[self.wn_ax] = slice(n - 1, n)
                    X[tuple(sl)] = bc[(1, i)][l]
                new[l * Q + i] = X
        aux_new = np.concatenate([phi, fs[None], np.array(u), D[None], (rhocp * T * D)[None]])
        return new, aux_new
