"""Brute-force UGKS step: everything stored, one-shot implicit update.

TEST INFRASTRUCTURE (tiny meshes only).  This is the basic UGKS algorithm of
Section 3.1 -- time step and heat flux, reconstruction, flux evaluation for
every velocity at once with all gradients and residuals stored, macroscopic
update, then the microscopic update of Eq. microscopicUpdata in one shot --
written independently of ugks_oracle.c (numpy, velocity-vectorised, no
in-place per-velocity update, no split into the two stages of Section 3.2).
Agreement of the two pins the two-stage update and the in-place ordering of
Algorithm 1.  It uses the same readings of the paper as the oracle (listed
in the oracle's header); the slope solve uses a hand-derived closed form and
the time slope numpy's Gauss-Hermite rule.
"""
from __future__ import annotations

import math

import numpy as np
from scipy.special import erfc

R_GAS = 0.5
N_DOF = 3  # translational + internal degrees of freedom of a monatomic gas


class BruteUGKS:
    def __init__(self, case):
        m, vg, g = case["mesh"], case["vgrid"], case["gas"]
        self.D = D = int(m["dim"])
        self.M = 3 - D
        self.ncomp = 2 if self.M > 0 else 1
        self.xc = np.asarray(m["cell_centroid"], float)
        self.vol = np.asarray(m["cell_volume"], float)
        self.fc = np.asarray(m["face_cells"], int)
        self.fn = np.asarray(m["face_normal"], float)
        self.fa = np.asarray(m["face_area"], float)
        self.fx = np.asarray(m["face_centroid"], float)
        self.fs = np.asarray(m["face_shift"], float)
        self.fbc = np.asarray(m["face_bc"], int)
        self.fbid = np.asarray(m["face_bc_id"], int)
        self.u = np.asarray(vg["u"], float)
        self.w = np.asarray(vg["w"], float)
        self.Pr, self.omega, self.mu_ref = g["Pr"], g["omega"], g["mu_ref"]
        self.limiter, self.K = g["limiter"], g["limiter_k"]
        self.bcp = np.asarray(g["bc_prim"], float)
        nc, nf = len(self.vol), len(self.fa)
        # per cell: (face, sign of the outward normal, vector to the face)
        self.cell_faces = [[] for _ in range(nc)]
        self.nbrs = [[] for _ in range(nc)]
        for f in range(nf):
            l, r = self.fc[f]
            self.cell_faces[l].append((f, 1.0, self.fx[f] - self.xc[l]))
            if r >= 0:
                self.cell_faces[r].append((f, -1.0, self.fx[f] - self.fs[f] - self.xc[r]))
                self.nbrs[l].append((r, self.xc[r] + self.fs[f] - self.xc[l]))
                self.nbrs[r].append((l, self.xc[l] - self.fs[f] - self.xc[r]))
        self.lsq = []
        for i in range(nc):
            d = np.array([v for _, v in self.nbrs[i]]).reshape(-1, D)
            G = d.T @ d
            tol = 1e-10 * (np.trace(G) / D) ** D
            # a stencil of at most D neighbours is an interpolation, not a
            # least-squares fit: first order there
            ok = len(d) > D and np.linalg.det(G) > tol
            self.lsq.append(np.linalg.inv(G) @ d.T if ok else np.zeros((D, len(d))))
        self.eps2 = (self.K * self.vol ** (1.0 / D)) ** 3
        # time step
        if g["dt_override"] > 0:
            self.dt = g["dt_override"]
        else:
            best = np.inf
            for i in range(nc):
                out = np.zeros(len(self.u))
                for f, sg, _ in self.cell_faces[i]:
                    out += self.fa[f] * np.maximum(0.0, sg * (self.u @ self.fn[f]))
                ok = out > 0
                if ok.any():
                    best = min(best, (self.vol[i] / out[ok]).min())
            self.dt = g["cfl"] * best
        # initial state
        p0 = np.asarray(case["prim0"], float).copy()
        p0[:, -1] = 1.0 / p0[:, -1]
        self.f = np.zeros((nc, self.ncomp, len(self.u)))
        for i in range(nc):
            H, B = self.maxwell(p0[i])
            self.f[i, 0] = H
            if self.ncomp > 1:
                self.f[i, 1] = B
        self.W = np.array([self.moments(self.f[i]) for i in range(nc)])
        self.q = np.array([self.heat_flux(self.f[i], self.prim(self.W[i])[1:1 + D]) for i in range(nc)])
        gx, gw = np.polynomial.hermite.hermgauss(6)
        self.gh = (gx, gw)

    # ---- Section 2.1-2.2 ----------------------------------------------------
    def prim(self, W):
        D = self.D
        rho = W[0]
        U = W[1:1 + D] / rho
        lam = N_DOF * rho / (4.0 * (W[-1] - 0.5 * rho * U @ U))
        return np.concatenate([[rho], U, [lam]])

    def tau(self, p):
        T = 1.0 / p[-1]
        return self.mu_ref * T ** self.omega / (p[0] * R_GAS * T)

    def maxwell(self, p):
        D = self.D
        c2 = ((self.u - p[1:1 + D]) ** 2).sum(1)
        H = p[0] * (p[-1] / math.pi) ** (D / 2) * np.exp(-p[-1] * c2)
        return H, self.M / (2 * p[-1]) * H

    def fplus(self, p, q):
        D, lam, rho = self.D, p[-1], p[0]
        c = self.u - p[1:1 + D]
        c2 = (c ** 2).sum(1)
        H, B = self.maxwell(p)
        s = 4 * (1 - self.Pr) * lam ** 2 / (5 * rho) * (c @ q)
        out = [H + s * (2 * lam * c2 - 2 - D) * H]
        if self.ncomp > 1:
            out.append(B + s * (2 * lam * c2 - D) * self.M * H / (2 * lam))
        return np.array(out)

    def moments(self, fi):
        u2 = (self.u ** 2).sum(1)
        b = fi[1] if self.ncomp > 1 else 0.0
        return np.concatenate([[self.w @ fi[0]], (self.w * fi[0]) @ self.u, [self.w @ (0.5 * (u2 * fi[0] + b))]])

    def heat_flux(self, fi, U):
        c = self.u - U
        c2 = (c ** 2).sum(1)
        b = fi[1] if self.ncomp > 1 else 0.0
        return (self.w * 0.5 * (c2 * fi[0] + b)) @ c

    # ---- reconstruction -----------------------------------------------------
    def limited_grad(self, i, vals):
        """vals: [nc, ...] -> limited gradient [..., D] of cell i (all
        trailing entries at once)."""
        vi = vals[i]
        nb = [j for j, _ in self.nbrs[i]]
        dv = np.stack([vals[j] - vi for j in nb], 0) if nb else np.zeros((0,) + vi.shape)
        grad = np.tensordot(dv, self.lsq[i], axes=([0], [1])) if nb else np.zeros(vi.shape + (self.D,))
        if not self.limiter:
            return grad
        allv = np.stack([vi] + [vals[j] for j in nb], 0)
        vmax, vmin = allv.max(0), allv.min(0)
        phi = np.ones(vi.shape)
        for f, sg, r in self.cell_faces[i]:
            dm = grad @ r
            dp = np.where(dm > 0, vmax - vi, vmin - vi)
            e2 = self.eps2[i]
            ph = np.where(dm == 0, 1.0, (dp ** 2 + e2 + 2 * dm * dp) / (dp ** 2 + 2 * dm ** 2 + dm * dp + e2))
            phi = np.minimum(phi, ph)
        return grad * phi[..., None]

    # ---- interface equilibrium (Section 2.4) ---------------------------------
    def half(self, p, n, sign):
        D = self.D
        rho, U, lam = p[0], p[1:1 + D], p[-1]
        Un = U @ n
        Ut = U - Un * n
        a = math.sqrt(lam) * Un
        g = math.exp(-lam * Un * Un) / (2 * math.sqrt(math.pi * lam))
        m0 = 0.5 * erfc(-sign * a)
        m1 = Un * m0 + sign * g
        m2 = Un * m1 + m0 / (2 * lam)
        return rho * np.concatenate([[m0], m1 * n + Ut * m0, [0.5 * (m2 + (Ut @ Ut + (N_DOF - 1) / (2 * lam)) * m0)]])

    def slope(self, p, Dl):
        D = self.D
        lam, U = p[-1], p[1:1 + D]
        K2 = U @ U + N_DOF / (2 * lam)
        R = Dl[1:1 + D] - U * Dl[0]
        aE = 4 * lam ** 2 / N_DOF * (2 * Dl[-1] - K2 * Dl[0] - 2 * U @ R)
        am = 2 * lam * R - U * aE
        return np.concatenate([[Dl[0] - U @ am - 0.5 * aE * K2], am, [aE]])

    def time_slope(self, p, a):
        D, M = self.D, self.M
        lam, U = p[-1], p[1:1 + D]
        gx, gw = self.gh
        dims = D + M
        grids = np.meshgrid(*([gx] * dims), indexing="ij")
        wts = np.prod(np.meshgrid(*([gw] * dims), indexing="ij"), axis=0).reshape(-1) * math.pi ** (-dims / 2)
        z = np.stack([g_.reshape(-1) for g_ in grids], 1) / math.sqrt(lam)
        uu = U + z[:, :D]
        e = 0.5 * ((uu ** 2).sum(1) + (z[:, D:] ** 2).sum(1))
        psi = np.concatenate([np.ones((len(e), 1)), uu, e[:, None]], 1)
        Mm = (psi * wts[:, None]).T @ psi
        adv = sum(uu[:, d] * (psi @ a[d]) for d in range(D))
        rhs = -(psi * (wts * adv)[:, None]).sum(0)
        return np.linalg.solve(Mm, rhs)

    @staticmethod
    def time_integrals(dt, tau):
        x = dt / tau
        if x < 1.0:
            t = [x ** m / math.factorial(m) for m in range(31)]
            sg = [(-1) ** (m + 1) for m in range(31)]
            q1 = tau * sum(sg[m] * t[m] for m in range(30, 0, -1))
            q2 = tau * tau * sum(sg[m] * (m - 1) * t[m] for m in range(30, 1, -1))
            q3 = tau * sum(-sg[m] * t[m] for m in range(30, 1, -1))
            q4 = tau * tau * sum(-sg[m] * (m - 2) * t[m] for m in range(30, 2, -1))
            q5 = tau * tau * sum(sg[m] * t[m] for m in range(30, 2, -1))
            return np.array([q1, q2, q3, q4, q5])
        e, ome = math.exp(-x), -math.expm1(-x)
        return np.array([tau * ome, tau * dt * e - tau * tau * ome, dt - tau * ome,
                         2 * tau * tau * ome - tau * dt * (1 + e), 0.5 * dt * dt - tau * dt + tau * tau * ome])

    # ---- one step (Section 3.1) ----------------------------------------------
    def step(self):
        D, M, nc, nf, dt = self.D, self.M, len(self.vol), len(self.fa), self.dt
        u, w = self.u, self.w
        u2 = (u ** 2).sum(1)
        P = np.array([self.prim(self.W[i]) for i in range(nc)])
        tau_n = np.array([self.tau(P[i]) for i in range(nc)])
        # step 2: reconstruction, all stored
        gW = np.array([self.limited_grad(i, self.W) for i in range(nc)])          # [nc, D+2, D]
        for i in range(nc):
            for f, sg, r in self.cell_faces[i]:
                Wf = self.W[i] + gW[i] @ r
                if not (Wf[0] > 0 and Wf[-1] - 0.5 * (Wf[1:1 + D] @ Wf[1:1 + D]) / Wf[0] > 0):
                    gW[i] = 0.0
                    break
        gf = np.array([self.limited_grad(i, self.f) for i in range(nc)])          # [nc, ncomp, nv, D]
        # step 3: fluxes for every face and velocity
        flux = np.zeros((nf, self.ncomp, len(u)))                                # u_n int f dt
        wall_in = {}
        for f in range(nf):
            l, r = self.fc[f]
            n = self.fn[f]
            un = u @ n
            dl = self.fx[f] - self.xc[l]
            vl = self.f[l] + gf[l] @ dl
            ugl = np.einsum("ckd,kd->ck", gf[l], u)
            if r >= 0:
                dr = self.fx[f] - self.fs[f] - self.xc[r]
                vr = self.f[r] + gf[r] @ dr
                ugr = np.einsum("ckd,kd->ck", gf[r], u)
                up = un > 0
                val = np.where(up, vl, vr)
                ug = np.where(up, ugl, ugr)
                pl = self.prim(self.W[l] + gW[l] @ dl)
                pr = self.prim(self.W[r] + gW[r] @ dr)
                p0 = self.prim(self.half(pl, n, 1) + self.half(pr, n, -1))
                a = np.array([self.slope(p0, 0.5 * (gW[l][:, d] + gW[r][:, d]) / p0[0]) for d in range(D)])
                A = self.time_slope(p0, a)
                q0 = 0.5 * (self.q[l] + self.q[r])
                c = self.time_integrals(dt, self.tau(p0))
                eq = self.fplus(p0, q0)
                H0, B0 = self.maxwell(p0)
                lam = p0[-1]
                Pd = sum(u[:, d] * (a[d][0] + u @ a[d][1:1 + D] + 0.5 * a[d][-1] * u2) for d in range(D))
                Ed = sum(u[:, d] * a[d][-1] for d in range(D))
                PA = A[0] + u @ A[1:1 + D] + 0.5 * A[-1] * u2
                xi4 = M * (M + 2) / (4 * lam ** 2) * H0
                gH, tH = Pd * H0 + 0.5 * Ed * B0, PA * H0 + 0.5 * A[-1] * B0
                I = [c[0] * val[0] + c[1] * ug[0] + c[2] * eq[0] + c[3] * gH + c[4] * tH]
                if self.ncomp > 1:
                    gB, tB = Pd * B0 + 0.5 * Ed * xi4, PA * B0 + 0.5 * A[-1] * xi4
                    I.append(c[0] * val[1] + c[1] * ug[1] + c[2] * eq[1] + c[3] * gB + c[4] * tB)
                flux[f] = un * np.array(I)
                continue
            out_part = dt * vl - 0.5 * dt * dt * ugl
            bp = self.bcp[self.fbid[f]]
            if self.fbc[f] == 3:
                pw = np.concatenate([[1.0], bp[1:1 + D], [1.0 / bp[-1]]])
                Hw, Bw = self.maxwell(pw)
                sin_ = (w * un * out_part[0])[un > 0].sum()
                sout = (w * un * dt * Hw)[un <= 0].sum()
                rho_w = -sin_ / sout
                ghost = np.array([Hw, Bw][:self.ncomp]) * rho_w * dt
            else:
                pg = np.concatenate([bp[:1 + D], [1.0 / bp[-1]]]) if self.fbc[f] == 1 else P[l]
                Hg, Bg = self.maxwell(pg)
                ghost = np.array([Hg, Bg][:self.ncomp]) * dt
            flux[f] = un * np.where(un > 0, out_part, ghost)
        # residuals of every cell and velocity, stored
        res = np.zeros_like(self.f)
        for i in range(nc):
            for f, sg, _ in self.cell_faces[i]:
                res[i] -= sg * self.fa[f] * flux[f]
        # step 4: macroscopic update (Eq. macroscopicUpdata)
        Wn1 = np.array([self.W[i] + self.moments(res[i]) / self.vol[i] for i in range(nc)])
        P1 = np.array([self.prim(Wn1[i]) for i in range(nc)])
        tau1 = np.array([self.tau(P1[i]) for i in range(nc)])
        # microscopic update in one shot (Eq. microscopicUpdata); q^{n+1}
        # from the heat flux of the bracket without the f+^{n+1} term
        fnew = np.zeros_like(self.f)
        qnew = np.zeros_like(self.q)
        for i in range(nc):
            fp_n = self.fplus(P[i], self.q[i])
            rest = self.f[i] + res[i] / self.vol[i] + 0.5 * dt * (fp_n - self.f[i]) / tau_n[i]
            qnew[i] = self.heat_flux(rest, P1[i][1:1 + D]) / (1 + self.Pr * dt / (2 * tau1[i]))
            fp_1 = self.fplus(P1[i], qnew[i])
            fnew[i] = (self.f[i] + res[i] / self.vol[i]
                       + 0.5 * dt * (fp_1 / tau1[i] + (fp_n - self.f[i]) / tau_n[i])) / (1 + 0.5 * dt / tau1[i])
        self.f, self.W, self.q = fnew, Wn1, qnew
