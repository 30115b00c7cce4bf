"""Discrete adjoint of Algorithm 1 (FP64, CPU) for an ensemble-mean energy.

Objective: Phi = E_h^M = 1/2 (||<v_h>^M||^2 + ||<w_h>^M||^2) (Section 4.2).
Parameters per member j: nu_j, nu_m,j, the forcing amplitude a_j
(f_{1,j} = f_{2,j} = a_j fhat) and the coefficients of the divergence-free
initial modes of u and B (v = u + sqrt(s) B, w = u - sqrt(s) B, Section 1).

One forward step n -> n+1 is the pair of linear systems
    S_v(W^n) X_v^{n+1} = b_v(V^n, W^n),   S_w(V^n) X_w^{n+1} = b_w(W^n, V^n)
of Algorithm 1 (see ``scheme``).  The adjoint sweep solves, for n = M-1..0,
    S_v^T mu_v = [lambda_V^{n+1}; 0],     S_w^T mu_w = [lambda_W^{n+1}; 0]
and propagates lambda^n = d Phi / d(state n) through every way the step
depends on time level n: the member's own right-hand side, the ensemble mean
<z> (convection of the shared matrix and the fluctuation w_j' = w_j - <w> of
every member), and l^2 = max_j |z_j'|^2 (the eddy viscosity; the derivative
follows the maximising member, lowest index on ties).  Only the
skew-symmetric trilinear form is supported (its matrix is antisymmetric).

This is test infrastructure (no code shared with the GPU library); it stores
every forward state.
"""
from __future__ import annotations

import numpy as np
from scipy.sparse.linalg import splu

from .fem import vec2
from .scheme import Ensemble


class EnsembleAdjoint(Ensemble):
    """Algorithm 1 with parameters theta = (nu, nu_m, a, IC coefficients)."""

    def __init__(self, mesh, problem, fhat_nodal, modes_nodal):
        """fhat_nodal: (nP2, 2) forcing shape; modes_nodal: list of (nP2, 2) initial modes."""
        if problem.convective != 0:
            raise ValueError("the adjoint supports the skew-symmetric trilinear form only")
        super().__init__(mesh, problem)
        self.fhat = fhat_nodal
        self.modes = modes_nodal
        self.dmask = np.ones((mesh.nP2, 2))
        self.dmask[self.dnodes] = 0.0

    # ------------------------------------------------------------ forward
    def initial(self, coef):
        """coef (J, 2 nm): u-mode then B-mode coefficients -> V^0, W^0 (plus B = (0,1) background)."""
        pb = self.pb
        n, J = self.mesh.nP2, coef.shape[0]
        nm = len(self.modes)
        u = np.zeros((n, 2, J))
        B = np.zeros((n, 2, J))
        B[:, 1, :] = getattr(pb, "b_background", 1.0)
        for m in range(nm):
            u += self.modes[m][:, :, None] * coef[None, None, :, m]
            B += self.modes[m][:, :, None] * coef[None, None, :, nm + m]
        rs = np.sqrt(pb.s)
        return u + rs * B, u - rs * B

    def forcing_nodal(self, a):
        return self.fhat[:, :, None] * a[None, None, :]

    def forward(self, nu, num, a, coef, nsteps):
        pb = self.pb
        pb.nu, pb.nu_m = np.asarray(nu, float), np.asarray(num, float)
        V, W = self.initial(coef)
        F = self.forcing_nodal(a)
        states = [(V, W)]
        for n in range(nsteps):
            t1 = (n + 1) * pb.dt
            Gv, Gw = pb.bc(t1, self.mesh.xy)
            Sv = self.shared_matrix(W)
            Sw = self.shared_matrix(V)
            xv = self.solve_members(Sv, self.rhs(V, W, F, Gv), shared_lu=True)
            xw = self.solve_members(Sw, self.rhs(W, V, F, Gw), shared_lu=True)
            nP2 = self.mesh.nP2
            V = xv[:2 * nP2].reshape(nP2, 2, -1)
            W = xw[:2 * nP2].reshape(nP2, 2, -1)
            states.append((V, W))
        return states, self.energy(V, W)

    # ------------------------------------------------------------ building blocks
    def conv_adj(self, Z, mu):
        """Transpose of the map u -> b*(u, Z, .) applied to mu, per node and component:
        out[b, d] = 1/2 int phi_b sum_k (d_d Z_k mu_k - d_d mu_k Z_k).  Z, mu: (nP2, 2)."""
        el = self.el
        zq, mq = el.values(Z), el.values(mu)                 # (ne, 7, 2)
        gz, gm = el.grads(Z), el.grads(mu)                   # (ne, 7, k, d)
        s = 0.5 * (np.einsum('eqkd,eqk->eqd', gz, mq) - np.einsum('eqkd,eqk->eqd', gm, zq))
        loc = np.einsum('e,q,qb,eqd->ebd', el.area, el.w, el.phi, s)
        out = np.zeros((self.mesh.nP2, 2))
        np.add.at(out, self.mesh.tri, loc)
        return out

    def eddy_adj(self, Zf, mus, Xnext):
        """Adjoint of the eddy term 2 mu dt K[l^2] X (l^2 from the fluctuations Zf of
        the other variable) against the multipliers mus: d/dZ_k, all members, (nP2, 2, J)."""
        pb = self.pb
        el = self.el
        J = Zf.shape[2]
        zq = el.values(Zf)                                   # (ne, 7, 2, J)
        mag = np.sum(zq * zq, axis=2)                        # (ne, 7, J)
        jstar = np.argmax(mag, axis=2)                       # lowest index on ties
        gm = el.grads(mus.reshape(self.mesh.nP2, -1)).reshape(el.mesh.n_el, 7, 2, J, 2)
        gx = el.grads(Xnext.reshape(self.mesh.nP2, -1)).reshape(el.mesh.n_el, 7, 2, J, 2)
        psi = 2 * pb.mu * pb.dt * np.einsum('e,q,eqcjd,eqcjd->eq', el.area, el.w, gm, gx)
        ne = el.mesh.n_el
        zstar = zq[np.arange(ne)[:, None], np.arange(7)[None, :], :, jstar]     # (ne, 7, 2)
        eta = 2 * psi[:, :, None] * zstar                                       # d psi*l^2 / d z'_{j*}(x_q)
        # d l^2 / d Z_k = 2 z'_{j*} (delta_{k j*} - 1/J) phi_b
        loc = np.einsum('qb,eqd->ebd', el.phi, eta)                             # (ne, 6, 2)
        out = np.zeros((self.mesh.nP2, 2, J))
        for e in range(ne):
            for q in range(7):
                contrib = np.outer(el.phi[q], eta[e, q])                        # (6, 2)
                out[self.mesh.tri[e], :, jstar[e, q]] += contrib
        mean_part = np.zeros((self.mesh.nP2, 2))
        np.add.at(mean_part, self.mesh.tri, loc)
        out -= mean_part[:, :, None] / J
        return out

    # ------------------------------------------------------------ reverse sweep
    def gradient(self, nu, num, a, coef, nsteps):
        """Returns Phi and dPhi/d(nu, nu_m, a) (J, 3) and dPhi/d coef (J, 2 nm)."""
        pb = self.pb
        states, phi = self.forward(nu, num, a, coef, nsteps)
        nP2 = self.mesh.nP2
        J = coef.shape[0]
        M2, K2 = self.M2, self.K2
        VM, WM = states[-1]
        lamV = np.repeat((M2 @ VM.mean(axis=2).ravel()).reshape(nP2, 2)[:, :, None], J, 2) / J
        lamW = np.repeat((M2 @ WM.mean(axis=2).ravel()).reshape(nP2, 2)[:, :, None], J, 2) / J
        g = np.zeros((J, 3))
        F = self.forcing_nodal(a)
        Mf = (M2 @ self.fhat.ravel()).reshape(nP2, 2)
        nub, numb = np.mean(nu), np.mean(num)
        cminus = 0.5 * (np.asarray(nu) - np.asarray(num))
        cplus = 0.5 * ((np.asarray(nu) - nub) + (np.asarray(num) - numb))
        _ = F

        def kmul(Z):
            return np.stack([(K2 @ Z[:, :, j].ravel()).reshape(nP2, 2) for j in range(Z.shape[2])], 2)

        def mmul(Z):
            return np.stack([(M2 @ Z[:, :, j].ravel()).reshape(nP2, 2) for j in range(Z.shape[2])], 2)

        for n in range(nsteps - 1, -1, -1):
            V, W = states[n]
            V1, W1 = states[n + 1]
            Sv = self.shared_matrix(W)
            Sw = self.shared_matrix(V)
            rhs_v = np.zeros((self.mesh.n, J))
            rhs_w = np.zeros((self.mesh.n, J))
            rhs_v[:2 * nP2] = lamV.reshape(2 * nP2, J)
            rhs_w[:2 * nP2] = lamW.reshape(2 * nP2, J)
            luv, luw = splu(Sv.tocsc()), splu(Sw.tocsc())
            mv = np.stack([luv.solve(rhs_v[:, j], trans='T') for j in range(J)], 1)
            mw = np.stack([luw.solve(rhs_w[:, j], trans='T') for j in range(J)], 1)
            muv = mv[:2 * nP2].reshape(nP2, 2, J) * self.dmask[:, :, None]
            muw = mw[:2 * nP2].reshape(nP2, 2, J) * self.dmask[:, :, None]
            _, Vf = self.mean_fluct(V)
            _, Wf = self.mean_fluct(W)
            Kmv, Kmw = kmul(muv), kmul(muw)
            Mmv, Mmw = mmul(muv), mmul(muw)
            # self terms of the own right-hand side: (M/dt - N*(z'_j) - c+ K)^T mu = M mu/dt + N*(z'_j) mu - c+ K mu
            newV = Mmv / pb.dt - cplus[None, None, :] * Kmv
            newW = Mmw / pb.dt - cplus[None, None, :] * Kmw
            for j in range(J):
                Nw = vec2(self.el.convection(Wf[:, :, j], skew=True))
                Nv = vec2(self.el.convection(Vf[:, :, j], skew=True))
                newV[:, :, j] += (Nw @ muv[:, :, j].ravel()).reshape(nP2, 2)
                newW[:, :, j] += (Nv @ muw[:, :, j].ravel()).reshape(nP2, 2)
            # cross-diffusion of the other problem's right-hand side: -c- K z_other
            newV -= cminus[None, None, :] * Kmw
            newW -= cminus[None, None, :] * Kmv
            # fluctuation convection -N*(z_j - <z>) self_j: derivative w.r.t. the convecting variable
            Tw = np.stack([self.conv_adj(W[:, :, j], muw[:, :, j]) for j in range(J)], 2)
            Tv = np.stack([self.conv_adj(V[:, :, j], muv[:, :, j]) for j in range(J)], 2)
            newV += -Tw + Tw.mean(axis=2, keepdims=True)
            newW += -Tv + Tv.mean(axis=2, keepdims=True)
            # shared matrix: convection by the mean <z> of the other variable
            Tw1 = np.stack([self.conv_adj(W1[:, :, j], muw[:, :, j]) for j in range(J)], 2)
            Tv1 = np.stack([self.conv_adj(V1[:, :, j], muv[:, :, j]) for j in range(J)], 2)
            newV -= Tw1.mean(axis=2, keepdims=True)
            newW -= Tv1.mean(axis=2, keepdims=True)
            # shared matrix: eddy viscosity from l^2 of the other variable
            newV -= self.eddy_adj(Vf, muw, W1)
            newW -= self.eddy_adj(Wf, muv, V1)
            # parameter gradients (dots over all nodes and components)
            dot = lambda A, B: np.einsum('ncj,ncj->j', A, B)
            av, bv, gv_ = dot(Kmv, W), dot(Kmv, V), dot(Kmv, V1)
            aw, bw, gw_ = dot(Kmw, V), dot(Kmw, W), dot(Kmw, W1)
            common = (bv.sum() - gv_.sum() + bw.sum() - gw_.sum()) / (2 * J)
            g[:, 0] += -0.5 * av - 0.5 * bv - 0.5 * aw - 0.5 * bw + common
            g[:, 1] += +0.5 * av - 0.5 * bv + 0.5 * aw - 0.5 * bw + common
            g[:, 2] += np.einsum('nc,ncj->j', Mf, muv) + np.einsum('nc,ncj->j', Mf, muw)
            lamV, lamW = newV, newW
        nm = len(self.modes)
        gc = np.zeros((J, 2 * nm))
        rs = np.sqrt(pb.s)
        for m in range(nm):
            pv = np.einsum('nc,ncj->j', self.modes[m], lamV)
            pw = np.einsum('nc,ncj->j', self.modes[m], lamW)
            gc[:, m] = pv + pw
            gc[:, nm + m] = rs * (pv - pw)
        return phi, g, gc


def central_fd(adj, nu, num, a, coef, nsteps, which, j, h=1e-6):
    """Central finite difference of Phi w.r.t. one parameter (which in
    'nu', 'num', 'a', or ('coef', m)) of member j."""
    def run(delta):
        args = [np.array(nu, float), np.array(num, float), np.array(a, float), np.array(coef, float)]
        if which == 'nu':
            args[0][j] += delta
        elif which == 'num':
            args[1][j] += delta
        elif which == 'a':
            args[2][j] += delta
        else:
            args[3][j, which[1]] += delta
        return adj.forward(*args, nsteps)[1]
    return (run(h) - run(-h)) / (2 * h)
