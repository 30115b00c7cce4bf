"""Tetrahedral meshes, quadrature and P2 / P1 bases in three dimensions (oracle side, FP64).

Section 2 states the method and its analysis for d = 2 and 3, and Section 3.2
remarks on the rate in 3D.  This module gives the oracle the 3D pieces; the
scheme itself (Algorithm 1) is dimension-independent in `scheme.Ensemble`.

Meshes: the unit cube with N cells per side, each cube cut into the six
tetrahedra of its main diagonal (vertex (0,0,0) to (1,1,1) of the cube, one
tetrahedron per order of the three axis steps), all positively oriented.

Numbering (the oracle's own):
  * vertices in row-major order of the vertex grid (x fastest, z slowest);
  * P2 nodes = all vertices, then one node per edge in order of first
    appearance while walking the elements and their edges (01, 02, 03, 12,
    13, 23);
  * P1 (pressure) nodes = vertices, same numbers as their P2 node.
Element connectivity: (v0, v1, v2, v3, m01, m02, m03, m12, m13, m23).

Quadrature: the conical product (collapsed-coordinate) rule built from
5-point Gauss-Legendre rules, exact for polynomials of degree 7 on a
tetrahedron, so every polynomial integrand of the scheme (degree <= 5) is
integrated exactly; the eddy-viscosity term uses the same points.
"""
from __future__ import annotations

import itertools
import math

import numpy as np

EDGES3 = ((0, 1), (0, 2), (0, 3), (1, 2), (1, 3), (2, 3))


def tet_rule(n=5):
    """Barycentric points (n^3, 4) and weights (n^3,) summing to 1 on a
    tetrahedron: the map x = u, y = v (1-u), z = w (1-u)(1-v) of the unit cube
    onto the reference tetrahedron, Jacobian (1-u)^2 (1-v), with Gauss-Legendre
    points in u, v, w."""
    g, gw = np.polynomial.legendre.leggauss(n)
    t, tw = 0.5 * (g + 1.0), 0.5 * gw
    pts, wts = [], []
    for (u, wu), (v, wv), (w, ww) in itertools.product(zip(t, tw), zip(t, tw), zip(t, tw)):
        x, y, z = u, v * (1 - u), w * (1 - u) * (1 - v)
        pts.append((1.0 - x - y - z, x, y, z))
        wts.append(wu * wv * ww * (1 - u) ** 2 * (1 - v))
    wts = np.array(wts)
    return np.array(pts), wts / wts.sum()


def p2_values3(lam):
    """lam (..., 4) barycentric -> (..., 10) P2 basis values."""
    out = [lam[..., i] * (2 * lam[..., i] - 1) for i in range(4)]
    out += [4 * lam[..., a] * lam[..., b] for a, b in EDGES3]
    return np.stack(out, axis=-1)


def p2_bary_grads3(lam):
    """d phi_a / d l_i: (..., 10, 4)."""
    g = np.zeros(lam.shape[:-1] + (10, 4))
    for i in range(4):
        g[..., i, i] = 4 * lam[..., i] - 1
    for s, (a, b) in enumerate(EDGES3):
        g[..., 4 + s, a] = 4 * lam[..., b]
        g[..., 4 + s, b] = 4 * lam[..., a]
    return g


def geometry3(xyz, tet):
    """Per element: volume (n_el,), gradients of the barycentric coordinates (n_el, 4, 3)."""
    p = xyz[tet[:, :4]]                               # (n_el, 4, 3)
    E = np.transpose(p[:, 1:] - p[:, :1], (0, 2, 1))  # columns: edges from vertex 0
    det = np.linalg.det(E)
    Einv = np.linalg.inv(E)                           # rows: gradients of l1, l2, l3
    gl = np.zeros((len(tet), 4, 3))
    gl[:, 1:] = Einv
    gl[:, 0] = -Einv.sum(axis=1)
    return np.abs(det) / 6.0, gl


def cube(N: int):
    """The unit cube with N x N x N cells, six tetrahedra per cell (see module doc)."""
    from .mesh import Mesh
    h = 1.0 / N
    vid = lambda i, j, k: (k * (N + 1) + j) * (N + 1) + i
    ks, js, is_ = np.meshgrid(np.arange(N + 1), np.arange(N + 1), np.arange(N + 1), indexing="ij")
    vxyz = np.stack([is_.ravel() * h, js.ravel() * h, ks.ravel() * h], axis=1).astype(float)
    tets = []
    steps = np.eye(3, dtype=int)
    for k in range(N):
        for j in range(N):
            for i in range(N):
                for perm in itertools.permutations(range(3)):
                    c = np.array([i, j, k])
                    path = [c.copy()]
                    for axis in perm:
                        c = c + steps[axis]
                        path.append(c.copy())
                    t = [vid(*q) for q in path]
                    p = vxyz[t]
                    if np.linalg.det((p[1:] - p[0]).T) < 0:
                        t[1], t[2] = t[2], t[1]
                    tets.append(t)
    tets = np.array(tets, dtype=np.int64)
    nV = len(vxyz)
    edge_id = {}
    conn = np.zeros((len(tets), 10), dtype=np.int64)
    conn[:, :4] = tets
    for e, t in enumerate(tets):
        for s, (a, b) in enumerate(EDGES3):
            key = (min(t[a], t[b]), max(t[a], t[b]))
            if key not in edge_id:
                edge_id[key] = len(edge_id)
            conn[e, 4 + s] = nV + edge_id[key]
    keys = sorted(edge_id, key=edge_id.get)
    xyz = np.vstack([vxyz, np.array([(vxyz[a] + vxyz[b]) / 2 for a, b in keys])])
    on = np.isclose(xyz, 0.0) | np.isclose(xyz, 1.0)
    bnd = np.nonzero(on.any(axis=1))[0]
    return Mesh(xy=xyz, tri=conn, nV=nV, bnd=bnd, dim=3)


def ref_monomial(a, b, c):
    """Integral of x^a y^b z^c over the reference tetrahedron (closed form)."""
    return math.factorial(a) * math.factorial(b) * math.factorial(c) / math.factorial(a + b + c + 3)
