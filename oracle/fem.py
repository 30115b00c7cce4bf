"""Quadrature, P2 / P1 bases and global FE matrices (oracle side, FP64).

Every integral is a quadrature sum over the elements with the 7-point,
degree-5 rule of Radon (centroid plus two 3-point orbits), which is exact for
all polynomial integrands of the scheme (mass, stiffness, divergence and the
trilinear convection form of P2 fields are of degree <= 5).  The only
non-polynomial integrand, the eddy-viscosity term of Algorithm 1 (it carries
the pointwise maximum over members), is evaluated with the same rule.

Conventions:
  * barycentric coordinates (l0, l1, l2); reference triangle (0,0),(1,0),(0,1)
  * P2 basis: phi_i = l_i (2 l_i - 1) for the vertices i = 0,1,2 and
    phi_3 = 4 l0 l1, phi_4 = 4 l1 l2, phi_5 = 4 l2 l0 for the edge midpoints
  * P1 basis: psi_k = l_k
  * integral over T of f ~ |T| sum_q w_q f(x_q), weights summing to one
  * velocity unknown (P2 node i, component c) -> 2 i + c; pressure unknown k ->
    2 nP2 + k (saddle-point ordering of the coupled system); the pressure is
    continuous P1 (Taylor-Hood) or, on an Alfeld mesh, discontinuous P1
    (Scott-Vogelius), as the mesh says
"""
from __future__ import annotations

import math

import numpy as np
import scipy.sparse as sp

# ------------------------------------------------------------ quadrature
_S15 = math.sqrt(15.0)
_A1 = (6.0 - _S15) / 21.0
_A2 = (6.0 + _S15) / 21.0
_W0 = 9.0 / 40.0
_W1 = (155.0 - _S15) / 1200.0
_W2 = (155.0 + _S15) / 1200.0


def quad7():
    """Barycentric points (7, 3) and weights (7,) summing to 1."""
    pts = [(1 / 3, 1 / 3, 1 / 3)]
    wts = [_W0]
    for a, w in ((_A1, _W1), (_A2, _W2)):
        b = 1.0 - 2.0 * a
        pts += [(b, a, a), (a, b, a), (a, a, b)]
        wts += [w, w, w]
    return np.array(pts), np.array(wts)


# ------------------------------------------------------------ bases
EDGES = ((0, 1), (1, 2), (2, 0))


def p2_values(lam):
    """lam: (..., 3) barycentric -> (..., 6) P2 basis values."""
    out = [lam[..., i] * (2 * lam[..., i] - 1) for i in range(3)]
    out += [4 * lam[..., a] * lam[..., b] for a, b in EDGES]
    return np.stack(out, axis=-1)


def p2_bary_grads(lam):
    """d phi_a / d l_i: (..., 6, 3)."""
    g = np.zeros(lam.shape[:-1] + (6, 3))
    for i in range(3):
        g[..., i, i] = 4 * lam[..., i] - 1
    for s, (a, b) in enumerate(EDGES):
        g[..., 3 + s, a] = 4 * lam[..., b]
        g[..., 3 + s, b] = 4 * lam[..., a]
    return g


def geometry(xy, tri):
    """Per element: area (n_el,), gradients of barycentric coordinates (n_el, 3, 2)."""
    p = xy[tri[:, :3]]                      # (n_el, 3, 2)
    x, y = p[..., 0], p[..., 1]
    two_a = (x[:, 1] - x[:, 0]) * (y[:, 2] - y[:, 0]) - (x[:, 2] - x[:, 0]) * (y[:, 1] - y[:, 0])
    gl = np.zeros((len(tri), 3, 2))
    for i in range(3):
        j, k = (i + 1) % 3, (i + 2) % 3
        gl[:, i, 0] = (y[:, j] - y[:, k]) / two_a
        gl[:, i, 1] = (x[:, k] - x[:, j]) / two_a
    return 0.5 * np.abs(two_a), gl


class Element:
    """Quadrature-point tables of a mesh: phi (7,6), psi (7,3), dphi (n_el,7,6,2), area, points."""

    def __init__(self, mesh):
        self.mesh = mesh
        self.d = d = getattr(mesh, "dim", 2)
        if d == 2:
            lam, self.w = quad7()
            self.phi = p2_values(lam)                       # (7, 6)
            self.area, gl = geometry(mesh.xy, mesh.tri)
            dbary = p2_bary_grads(lam)                      # (7, 6, 3)
        else:   # tetrahedra (oracle.tet): "area" is the volume
            from .tet import geometry3, p2_bary_grads3, p2_values3, tet_rule
            lam, self.w = tet_rule()
            self.phi = p2_values3(lam)                      # (Q, 10)
            self.area, gl = geometry3(mesh.xy, mesh.tri)
            dbary = p2_bary_grads3(lam)                     # (Q, 10, 4)
        self.psi = lam.copy()                               # P1: the barycentric coordinates
        self.dphi = np.einsum('qai,eid->eqad', dbary, gl)
        verts = mesh.xy[mesh.tri[:, :d + 1]]                # (n_el, d+1, d)
        self.xq = np.einsum('qi,eid->eqd', lam, verts)      # (n_el, Q, d)

    # -------- fields at quadrature points
    def values(self, nodal):
        """nodal (nP2, ...) -> (n_el, 7, ...) interpolated P2 field."""
        loc = nodal[self.mesh.tri]                      # (n_el, 6, ...)
        return np.einsum('qa,ea...->eq...', self.phi, loc)

    def grads(self, nodal):
        """nodal (nP2, C) -> (n_el, 7, C, 2) gradient of each component."""
        loc = nodal[self.mesh.tri]
        return np.einsum('eqad,eac->eqcd', self.dphi, loc)

    # -------- element matrices -> global scalar P2 matrices
    def _scatter(self, ke, rows_tri, cols_tri, shape):
        r = np.repeat(rows_tri[:, :, None], cols_tri.shape[1], axis=2)
        c = np.repeat(cols_tri[:, None, :], rows_tri.shape[1], axis=1)
        return sp.coo_matrix((ke.ravel(), (r.ravel(), c.ravel())), shape=shape).tocsr()

    def mass(self):
        ke = np.einsum('e,q,qa,qb->eab', self.area, self.w, self.phi, self.phi)
        n = self.mesh.nP2
        return self._scatter(ke, self.mesh.tri, self.mesh.tri, (n, n))

    def stiffness(self, kappa=None):
        """sum_q w_q kappa_q grad phi_a . grad phi_b |T|; kappa (n_el, Q) or None (= 1)."""
        wq = self.w[None, :] * (np.ones((self.mesh.n_el, len(self.w))) if kappa is None else kappa)
        ke = np.einsum('e,eq,eqad,eqbd->eab', self.area, wq, self.dphi, self.dphi)
        n = self.mesh.nP2
        return self._scatter(ke, self.mesh.tri, self.mesh.tri, (n, n))

    def convection(self, u_nodal, skew=True):
        """Matrix of the trilinear form with convecting field u (nP2, 2):
        row a (test phi_a), column b (trial phi_b).
        plain:  (u . grad phi_b, phi_a)
        skew:   1/2 [ (u . grad phi_b, phi_a) - (u . grad phi_a, phi_b) ]"""
        uq = self.values(u_nodal)                                   # (n_el, 7, 2)
        adv = np.einsum('eqd,eqbd->eqb', uq, self.dphi)             # u . grad phi_b
        t1 = np.einsum('e,q,eqb,qa->eab', self.area, self.w, adv, self.phi)
        if skew:
            t2 = np.einsum('e,q,eqa,qb->eab', self.area, self.w, adv, self.phi)
            ke = 0.5 * (t1 - t2)
        else:
            ke = t1
        n = self.mesh.nP2
        return self._scatter(ke, self.mesh.tri, self.mesh.tri, (n, n))

    def divergence(self):
        """B (nP1, d nP2): B[k, d i + c] = -(psi_k, d phi_i / d x_c), psi_k the
        pressure basis function (continuous or, on an Alfeld mesh, per element)."""
        d = self.d
        ke = -np.einsum('e,q,qk,eqic->ekic', self.area, self.w, self.psi, self.dphi)
        ne, nloc, npl = self.mesh.n_el, self.mesh.tri.shape[1], self.mesh.ptri.shape[1]
        rows = np.repeat(self.mesh.ptri[:, :, None, None], nloc, axis=2).repeat(d, axis=3)
        cols = d * self.mesh.tri[:, None, :, None] + np.arange(d)[None, None, None, :]
        cols = np.broadcast_to(cols, (ne, npl, nloc, d))
        return sp.coo_matrix((ke.ravel(), (rows.ravel(), cols.ravel())),
                             shape=(self.mesh.nP1, d * self.mesh.nP2)).tocsr()

    def p1_mass_lumped(self):
        """m_k = integral of psi_k (exact: |T|/(d+1) per element)."""
        m = np.zeros(self.mesh.nP1)
        k = self.mesh.ptri.shape[1]
        np.add.at(m, self.mesh.ptri.ravel(), np.repeat(self.area / (self.d + 1.0), k))
        return m


def vec2(Ms):
    """Scalar P2 operator -> operator on interleaved 2-vectors (A kron I_2)."""
    return sp.kron(Ms, sp.identity(2), format='csr')


def vecd(Ms, d):
    """Scalar P2 operator -> operator on interleaved d-vectors (A kron I_d)."""
    return sp.kron(Ms, sp.identity(d), format='csr')
