"""Structured triangulations and P2 / pressure node numbering (oracle side).

Meshes are the "regular triangular meshes" of Section 4: every square cell
[x_i, x_i+h] x [y_k, y_k+h] is cut by its rising diagonal into the triangles
(v00, v10, v11) and (v00, v11, v01), both counter-clockwise.  `alfeld` refines
such a mesh at the barycentres (each triangle (a, b, c) with barycentre g
becomes (a, b, g), (b, c, g), (c, a, g)), the meshes on which Section 2 places
the Scott-Vogelius pair (P2, P1 discontinuous).

Numbering (the oracle's own, unrelated to the GPU library's):
  * vertices in row-major order of the vertex grid (y slowest), only those
    that belong to a kept cell;
  * P2 nodes = all vertices, then one node per edge in order of first
    appearance while walking the elements and their edges (01, 12, 20);
  * Taylor-Hood pressure (continuous P1) nodes = vertices, same numbers as
    their P2 node;
  * Scott-Vogelius pressure (discontinuous P1): three unknowns per element,
    3 e + k belonging to its vertex k.
Element connectivity: (v0, v1, v2, m01, m12, m20) with m_ab the edge midpoint;
`ptri` (n_el, 3) gives the pressure unknown of each element vertex.
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np


@dataclass
class Mesh:
    xy: np.ndarray          # (nP2, 2) node coordinates; first nV rows are the vertices
    tri: np.ndarray         # (n_el, 6) P2 connectivity
    nV: int                 # number of vertices
    bnd: np.ndarray         # sorted P2 node ids on the boundary
    disc: bool = False      # pressure discontinuous P1 (Scott-Vogelius) instead of continuous P1
    dim: int = 2            # space dimension (3: tetrahedra with 10 P2 nodes, see oracle.tet)

    @property
    def n_el(self):
        return len(self.tri)

    @property
    def nP2(self):
        return len(self.xy)

    @property
    def nP1(self):
        """Number of pressure unknowns."""
        return 3 * self.n_el if self.disc else self.nV

    @property
    def ptri(self):
        """(n_el, 3): pressure unknown of each element vertex."""
        if self.disc:
            return np.arange(3 * self.n_el, dtype=np.int64).reshape(-1, 3)
        return self.tri[:, :self.dim + 1]

    @property
    def pxy(self):
        """(nP1, 2): location of each pressure unknown."""
        if self.disc:
            return self.xy[self.tri[:, :3]].reshape(-1, 2)
        return self.xy[:self.nV]

    @property
    def n(self):
        return self.dim * self.nP2 + self.nP1


def _build(nx, ny, h, keep, x0=0.0, y0=0.0):
    """Cells (i,k), 0<=i<nx, 0<=k<ny with keep(i,k) True, spacing h."""
    vid = -np.ones((ny + 1, nx + 1), dtype=np.int64)
    cells = [(i, k) for k in range(ny) for i in range(nx) if keep(i, k)]
    used = np.zeros((ny + 1, nx + 1), dtype=bool)
    for i, k in cells:
        used[k:k + 2, i:i + 2] = True
    ks, is_ = np.nonzero(used)            # row-major: k slowest
    vid[ks, is_] = np.arange(len(ks))
    vxy = np.stack([x0 + is_ * h, y0 + ks * h], axis=1).astype(float)
    tris = []
    for i, k in cells:
        a, b, c, d = vid[k, i], vid[k, i + 1], vid[k + 1, i + 1], vid[k + 1, i]
        tris.append((a, b, c))
        tris.append((a, c, d))
    return _p2_mesh(vxy, np.array(tris, dtype=np.int64))


def _p2_mesh(vxy, tris, disc=False):
    """P2 nodes of the triangulation (vertex coordinates vxy, counter-clockwise
    vertex triples tris): vertices, then edge midpoints in order of first use."""
    nV = len(vxy)
    edge_id = {}
    edge_count = {}
    conn = np.zeros((len(tris), 6), dtype=np.int64)
    conn[:, :3] = tris
    for e, (a, b, c) in enumerate(tris):
        for slot, (p, q) in zip((3, 4, 5), ((a, b), (b, c), (c, a))):
            key = (min(p, q), max(p, q))
            if key not in edge_id:
                edge_id[key] = len(edge_id)
                edge_count[key] = 0
            edge_count[key] += 1
            conn[e, slot] = nV + edge_id[key]
    keys = sorted(edge_id, key=edge_id.get)
    mid = np.array([(vxy[p] + vxy[q]) / 2 for p, q in keys])
    xy = np.vstack([vxy, mid])
    bset = set()
    for key in keys:
        if edge_count[key] == 1:
            bset.update((key[0], key[1], nV + edge_id[key]))
    return Mesh(xy=xy, tri=conn, nV=nV, bnd=np.array(sorted(bset), dtype=np.int64), disc=disc)


def alfeld(mesh: Mesh) -> Mesh:
    """Barycentric refinement of `mesh` with the discontinuous P1 pressure:
    vertices of `mesh` first, then the barycentres in element order; element
    e of `mesh` becomes elements 3e, 3e+1, 3e+2 = (a, b, g), (b, c, g), (c, a, g)."""
    vxy = mesh.xy[:mesh.nV]
    macro = mesh.tri[:, :3]
    g = mesh.nV + np.arange(len(macro))
    bary = vxy[macro].mean(axis=1)
    a, b, c = macro[:, 0], macro[:, 1], macro[:, 2]
    tris = np.stack([np.stack([a, b, g], 1), np.stack([b, c, g], 1), np.stack([c, a, g], 1)], 1).reshape(-1, 3)
    return _p2_mesh(np.vstack([vxy, bary]), tris, disc=True)


def unit_square(N: int) -> Mesh:
    """N x N cells on the unit square, h = 1/N."""
    return _build(N, N, 1.0 / N, lambda i, k: True)


def step_channel(m: int = 16) -> Mesh:
    """[0,30] x [0,10] minus [0,1] x [0,1] with h = 1/m."""
    return _build(30 * m, 10 * m, 1.0 / m, lambda i, k: not (i < m and k < m))


def nested_dissection(mesh: Mesh, leaf: int = 64) -> np.ndarray:
    """Fill-reducing elimination order of the saddle-point unknowns (velocity
    2i+c at P2 node i, pressure 2 nP2 + k at vertex k) by geometric nested
    dissection.  A vertex grid line crosses no element, so the unknowns lying
    on it separate those on either side: each part is ordered recursively, its
    separator after it.  Inside a part the unknowns keep their natural order
    (velocities before pressures), so every pressure is eliminated after some
    velocity it couples to.  The order only changes the rounding of a direct
    solve, not what is solved."""
    xy = np.concatenate([np.repeat(mesh.xy, 2, axis=0), mesh.pxy])
    h = float(np.min(np.diff(np.unique(np.round(mesh.xy[:mesh.nV, 0], 12)))))
    tol = 1e-6 * h
    out = []

    def part(ids):
        if len(ids) <= leaf:
            out.append(np.sort(ids))
            return
        c = xy[ids]
        lo, hi = c.min(axis=0), c.max(axis=0)
        for ax in np.argsort(lo - hi):               # longer extent first
            cut = np.round(np.median(c[:, ax]) / h) * h
            cut = min(max(cut, lo[ax] + h), hi[ax] - h)
            if lo[ax] + tol < cut < hi[ax] - tol:
                break
        else:
            out.append(np.sort(ids))
            return
        d = c[:, ax] - cut
        part(ids[d < -tol])
        part(ids[d > tol])
        out.append(np.sort(ids[np.abs(d) <= tol]))

    if mesh.disc or mesh.dim != 2:
        raise ValueError("nested dissection is defined for the unrefined 2D meshes only")
    part(np.arange(len(xy)))
    return np.concatenate(out)
