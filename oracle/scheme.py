"""Algorithm 1 of the paper (Section 3, (weaknew1)-(weaknew2)), FP64, per-member LU.

One time step n -> n+1 of the decoupled ensemble scheme, for every member j:

  v-problem (weaknew1): find v_j^{n+1} (and pressure q_j^{n+1}) with
    (v^{n+1}/dt, chi) + b(<w>^n, v^{n+1}, chi) + (nu_bar+num_bar)/2 (grad v^{n+1}, grad chi)
    + (2 nu_T(w', t^n) grad v^{n+1}, grad chi) - (q, div chi)
    = (f_{1,j}(t^{n+1}), chi) + (v_j^n/dt, chi) - b(w_j'^n, v_j^n, chi)
      - (nu_j - nu_m,j)/2 (grad w_j^n, grad chi) - (nu_j' + nu_m,j')/2 (grad v_j^n, grad chi)
    (div v^{n+1}, r) = 0
  w-problem (weaknew2): the same with v and w exchanged and f_{1,j} -> f_{2,j}.

Ensemble mean / fluctuation and mean viscosities as defined in Section 1;
nu_T(z', t^n) = mu dt (l_z^n)^2 with l_z^n(x) = max_j |z_j'^n(x)| (Euclidean
length), taken pointwise at the quadrature points.

Both subproblems use time level n only, so they are independent within a
step.  The matrix of each subproblem depends on no member index; the oracle
nevertheless factors it once per member ("its own LU") unless the caller
asks for the shared factorisation, which gives identical numbers.

Readings where the paper leaves a choice (Taylor-Hood instead of
Scott-Vogelius, skew-symmetric trilinear form, Dirichlet identity rows,
pressure pin, nodal interpolation of the forcing) are listed in the
repository's design notes; the trilinear form is selectable.
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp
from scipy.sparse.linalg import splu

from .fem import Element, vecd
from .mesh import nested_dissection


class Ensemble:
    def __init__(self, mesh, problem):
        self.mesh = mesh
        self.pb = problem
        self.el = Element(mesh)
        self.M = self.el.mass()
        self.K = self.el.stiffness()
        self.B = self.el.divergence()
        self.d = d = getattr(mesh, "dim", 2)
        self.M2 = vecd(self.M, d)      # velocity operators on interleaved d-vectors
        self.K2 = vecd(self.K, d)
        self.mP1 = self.el.p1_mass_lumped()
        bxy = mesh.xy[mesh.bnd]
        self.dnodes = mesh.bnd[problem.is_dirichlet(bxy)]
        self.pin = None
        if problem.pin_pressure:
            dist = np.linalg.norm(mesh.pxy, axis=1)
            self.pin = int(np.argmin(dist))
        n = mesh.n
        keep = np.ones(n)
        for c in range(d):
            keep[d * self.dnodes + c] = 0.0
        if self.pin is not None:
            keep[d * mesh.nP2 + self.pin] = 0.0
        self.keep = keep
        self.skew = (problem.convective == 0)

    # --------------------------------------------------- ensemble statistics
    @staticmethod
    def mean_fluct(Z):
        """<z> = (1/J) sum_j z_j, z_j' = z_j - <z>  (Z: (nP2, d, J))."""
        zbar = Z.mean(axis=2)
        return zbar, Z - zbar[:, :, None]

    def eddy_l2(self, Zf):
        """l^2(x_q) = max_j |z_j'(x_q)|^2 at every quadrature point: (n_el, Q)."""
        zq = self.el.values(Zf)                     # (n_el, Q, d, J)
        return np.max(np.sum(zq * zq, axis=2), axis=2)

    # --------------------------------------------------- shared matrix
    def velocity_block(self, zbar, l2):
        pb = self.pb
        nub = pb.nu.mean()
        numb = pb.nu_m.mean()
        A = (self.M / pb.dt + self.el.convection(zbar, skew=self.skew)
             + 0.5 * (nub + numb) * self.K
             + self.el.stiffness(2.0 * pb.mu * pb.dt * l2))
        return A.tocsr()

    def saddle(self, A):
        """[[A kron I2, B^T], [B, 0]] with Dirichlet identity rows and the pressure pin."""
        S = sp.bmat([[vecd(A, self.d), self.B.T], [self.B, None]], format='csr')
        return (sp.diags(self.keep) @ S + sp.diags(1.0 - self.keep)).tocsr()

    def shared_matrix(self, Zother):
        """Matrix of the subproblem whose convecting field is the OTHER variable."""
        zbar, zf = self.mean_fluct(Zother)
        return self.saddle(self.velocity_block(zbar, self.eddy_l2(zf)))

    # --------------------------------------------------- right-hand sides
    def rhs(self, Zself, Zother, F, G, members=None):
        """Per-member right-hand sides (n, J) of the subproblem for Zself; with
        `members`, only those columns (in that order), the ensemble mean still
        taken over every member of Zother."""
        pb = self.pb
        mesh = self.mesh
        cols = range(Zself.shape[2]) if members is None else list(members)
        nub, numb = pb.nu.mean(), pb.nu_m.mean()
        cminus = 0.5 * (pb.nu - pb.nu_m)
        cplus = 0.5 * ((pb.nu - nub) + (pb.nu_m - numb))
        _, of = self.mean_fluct(Zother)
        b = np.zeros((mesh.n, len(cols)))
        d = self.d
        nu2 = d * mesh.nP2
        for i, j in enumerate(cols):
            zs = Zself[:, :, j].ravel()
            zo = Zother[:, :, j].ravel()
            Nj = vecd(self.el.convection(of[:, :, j], skew=self.skew), d)
            b[:nu2, i] = (self.M2 @ (zs / pb.dt + F[:, :, j].ravel()) - Nj @ zs
                          - cminus[j] * (self.K2 @ zo) - cplus[j] * (self.K2 @ zs))
            for c in range(d):
                b[d * self.dnodes + c, i] = G[self.dnodes, c, j]
        if self.pin is not None:
            b[nu2 + self.pin, :] = 0.0
        return b

    # --------------------------------------------------- solves
    def solve_members(self, S, b, shared_lu=False, members=None, ordering="COLAMD"):
        """Each member's system solved by its own sparse LU (or one shared LU).
        `ordering` is SuperLU's fill-reducing column ordering, or "ND" for the
        mesh's nested-dissection order applied symmetrically before a factorisation
        that prefers diagonal pivots.  It changes the rounding of the direct
        solve, not what is solved; ND keeps the fill of the larger saddle-point
        systems small."""
        cols = range(b.shape[1]) if members is None else members
        if ordering == "ND":
            p = nested_dissection(self.mesh)
            Sc = S.tocsr()[p][:, p].tocsc()
            kw = dict(permc_spec="NATURAL", diag_pivot_thresh=0.01, options=dict(SymmetricMode=True))
        else:
            p = None
            Sc = S.tocsc()
            kw = dict(permc_spec=ordering)
        x = np.zeros((b.shape[0], len(cols)))
        lu = splu(Sc, **kw) if shared_lu else None
        for i, j in enumerate(cols):
            f = lu if shared_lu else splu(Sc, **kw)
            if p is None:
                x[:, i] = f.solve(b[:, j])
            else:
                x[p, i] = f.solve(b[p, j])
        return x

    def split(self, x):
        nP2 = self.mesh.nP2
        J = x.shape[1]
        Z = x[:self.d * nP2].reshape(nP2, self.d, J)
        p = x[self.d * nP2:]
        if self.pin is not None:      # pressure determined up to a constant: report zero mean
            p = p - (self.mP1 @ p) / self.mP1.sum()
        return Z, p

    def step(self, V, W, t_next, shared_lu=False, members=None, ordering="COLAMD", log=None):
        """Algorithm 1, one step: returns V^{n+1}, W^{n+1}, q^{n+1}, r^{n+1} (zero mean when pinned).
        `log`, if given, is called with a short message before each subproblem's solve."""
        xy = self.mesh.xy
        F1, F2 = self.pb.forcing(t_next, xy)
        Gv, Gw = self.pb.bc(t_next, xy)
        Sv = self.shared_matrix(W)
        Sw = self.shared_matrix(V)
        bv = self.rhs(V, W, F1, Gv, members)
        bw = self.rhs(W, V, F2, Gw, members)
        if log:
            log("oracle: v-subproblem solve")
        xv = self.solve_members(Sv, bv, shared_lu, ordering=ordering)
        if log:
            log("oracle: w-subproblem solve")
        xw = self.solve_members(Sw, bw, shared_lu, ordering=ordering)
        V1, Q = self.split(xv)
        W1, R = self.split(xw)
        return V1, W1, Q, R

    def energy(self, V, W):
        """E_h = 1/2 (||<v_h>||^2 + ||<w_h>||^2) (Section 4.2)."""
        vb = V.mean(axis=2).ravel()
        wb = W.mean(axis=2).ravel()
        return 0.5 * (vb @ (self.M2 @ vb) + wb @ (self.M2 @ wb))

    def run(self, nsteps=None, shared_lu=False, callback=None):
        pb = self.pb
        V, W = pb.ic(self.mesh.xy)
        nsteps = pb.nsteps if nsteps is None else nsteps
        hist = [(V, W)]
        for n in range(nsteps):
            V, W, Q, R = self.step(V, W, (n + 1) * pb.dt, shared_lu)
            hist.append((V, W))
            if callback is not None:
                callback(n + 1, V, W, Q, R)
        return hist
