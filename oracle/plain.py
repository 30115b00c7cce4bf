"""Plain decoupled Elsasser scheme for ONE member, without ensemble machinery.

This is the single-realisation scheme that Algorithm 1 generalises: the
v-problem is convected by w^n with viscosity (nu + nu_m)/2 and the explicit
cross-diffusion -(nu - nu_m)/2 (grad w^n, grad chi); the w-problem likewise
with v and w exchanged.  There is no mean, no fluctuation and no eddy term.
For J = 1 Algorithm 1 must reduce to exactly this (Section 1: <w> = w_1,
w_1' = 0, nu_1' = nu_m,1' = 0, so l = 0).  Written separately from
``scheme`` so that the reduction test compares two independent codes.
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp
from scipy.sparse.linalg import spsolve

from .fem import Element, vec2


def run_plain(mesh, problem, member=0, nsteps=None):
    """Returns the list of (v, w) nodal arrays (nP2, 2) for steps 0..nsteps."""
    el = Element(mesh)
    M, K, B = el.mass(), el.stiffness(), el.divergence()
    nu, num = problem.nu[member], problem.nu_m[member]
    dt = problem.dt
    skew = problem.convective == 0
    xy = mesh.xy
    nP2 = mesh.nP2
    dn = mesh.bnd[problem.is_dirichlet(xy[mesh.bnd])]
    fixed = np.concatenate([2 * dn, 2 * dn + 1])
    pin = None
    if problem.pin_pressure:
        pin = 2 * nP2 + int(np.argmin(np.hypot(mesh.pxy[:, 0], mesh.pxy[:, 1])))
        fixed = np.concatenate([fixed, [pin]])
    V0, W0 = problem.ic(xy)
    v, w = V0[:, :, member].copy(), W0[:, :, member].copy()
    out = [(v, w)]
    nsteps = problem.nsteps if nsteps is None else nsteps

    def solve_one(conv_field, own, other, f, g):
        A = M / dt + el.convection(conv_field, skew=skew) + 0.5 * (nu + num) * K
        S = sp.bmat([[vec2(A), B.T], [B, None]], format='lil')
        rhs = np.zeros(mesh.n)
        rhs[:2 * nP2] = (vec2(M) @ (own.ravel() / dt + f.ravel())
                         - 0.5 * (nu - num) * (vec2(K) @ other.ravel()))
        for r in fixed:
            S.rows[r] = [r]
            S.data[r] = [1.0]
        gflat = g.ravel()
        rhs[2 * dn] = gflat[2 * dn]
        rhs[2 * dn + 1] = gflat[2 * dn + 1]
        if pin is not None:
            rhs[pin] = 0.0
        x = spsolve(S.tocsc(), rhs)
        return x[:2 * nP2].reshape(nP2, 2)

    for n in range(nsteps):
        t1 = (n + 1) * dt
        F1, F2 = problem.forcing(t1, xy)
        G1, G2 = problem.bc(t1, xy)
        v1 = solve_one(w, v, w, F1[:, :, member], G1[:, :, member])
        w1 = solve_one(v, w, v, F2[:, :, member], G2[:, :, member])
        v, w = v1, w1
        out.append((v, w))
    return out
