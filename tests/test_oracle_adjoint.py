"""Pins of the FP64 CPU adjoint: central finite differences of the oracle's
forward map (every parameter class, with an active eddy viscosity and
ensemble-mean coupling), and its J = 1 / identical-member structure."""
import numpy as np
import pytest

import workloads as wl
from oracle import mesh as om
from oracle.adjoint import EnsembleAdjoint, central_fd
from workloads import modes_and_forcing


def make(N=4, J=3, s=0.3, dt=0.05, seed=11):
    pb = wl.cavity(J=J, s=s, dt=dt, nu_mean=0.01, num_mean=0.02, ic_amp=0.3)
    ms = om.unit_square(N)
    modes, fhat = modes_and_forcing(ms.xy)
    adj = EnsembleAdjoint(ms, pb, fhat, modes)
    r = np.random.default_rng(seed)
    nu = 0.01 * (1 + r.uniform(-0.1, 0.1, J))
    num = 0.02 * (1 + r.uniform(-0.1, 0.1, J))
    a = r.uniform(0.5, 1.5, J)
    coef = 0.3 * r.uniform(-1, 1, (J, 8))
    return adj, nu, num, a, coef


def test_adjoint_matches_central_differences():
    adj, nu, num, a, coef = make()
    nsteps = 3
    phi, g, gc = adj.gradient(nu, num, a, coef, nsteps)
    assert phi > 0
    for j in range(3):
        for col, which in enumerate(("nu", "num", "a")):
            fd = central_fd(adj, nu, num, a, coef, nsteps, which, j)
            assert abs(g[j, col] - fd) <= 1e-6 * max(abs(fd), 1e-3 * np.abs(g[:, col]).max()), (which, j, g[j, col], fd)
        for m in (0, 3, 5, 7):
            fd = central_fd(adj, nu, num, a, coef, nsteps, ("coef", m), j)
            assert abs(gc[j, m] - fd) <= 1e-6 * max(abs(fd), 1e-3 * np.abs(gc).max()), (m, j, gc[j, m], fd)


def test_eddy_term_is_active_in_the_pin():
    """The finite-difference case must exercise the max over members: with the
    eddy term switched off (mu = 0) the gradient changes."""
    adj, nu, num, a, coef = make()
    g1 = adj.gradient(nu, num, a, coef, 2)[1]
    adj.pb.mu = 0.0
    g0 = adj.gradient(nu, num, a, coef, 2)[1]
    assert np.abs(g1 - g0).max() > 0.1 * np.abs(g1).max()


def test_identical_members_have_identical_gradients():
    adj, nu, num, a, coef = make(J=3)
    nu[:] = nu[0]
    num[:] = num[0]
    a[:] = a[0]
    coef[:] = coef[0]
    _, g, gc = adj.gradient(nu, num, a, coef, 2)
    assert np.abs(g - g[0]).max() <= 1e-12 * np.abs(g).max()
    assert np.abs(gc - gc[0]).max() <= 1e-12 * np.abs(gc).max()


def test_single_member_adjoint_matches_the_plain_scheme():
    """J = 1: the ensemble adjoint's gradient equals central differences of the
    plain decoupled scheme (``oracle.plain``, written without the ensemble
    machinery), with the member's parameters entering through the problem's
    own initial modes and forcing amplitude.  Pins the adjoint's reduction to
    the single-realisation scheme (Section 1)."""
    import dataclasses

    from oracle.plain import run_plain
    from oracle.fem import Element, vec2
    adj, nu, num, a, coef = make(J=1, seed=5)
    nsteps = 3
    _, g, gc = adj.gradient(nu, num, a, coef, nsteps)
    ms = adj.mesh
    M2 = vec2(Element(ms).mass())

    def energy(nu_, num_, a_, coef_):
        pb = dataclasses.replace(adj.pb, nu=np.array([nu_]), nu_m=np.array([num_]), amp=np.array([a_]),
                                 ic_coef=np.array(coef_)[None, :])
        v, w = run_plain(ms, pb, 0, nsteps)[-1]
        return 0.5 * (v.ravel() @ (M2 @ v.ravel()) + w.ravel() @ (M2 @ w.ravel()))

    h = 1e-6
    base = [nu[0], num[0], a[0], coef[0].copy()]
    for col in range(3):
        p, m = list(base), list(base)
        p[col] += h
        m[col] -= h
        fd = (energy(*p) - energy(*m)) / (2 * h)
        assert abs(g[0, col] - fd) <= 1e-6 * max(abs(fd), 1e-3 * np.abs(g).max()), (col, g[0, col], fd)
    for k in (0, 5):
        cp, cm = coef[0].copy(), coef[0].copy()
        cp[k] += h
        cm[k] -= h
        fd = (energy(nu[0], num[0], a[0], cp) - energy(nu[0], num[0], a[0], cm)) / (2 * h)
        assert abs(gc[0, k] - fd) <= 1e-6 * max(abs(fd), 1e-3 * np.abs(gc).max()), (k, gc[0, k], fd)
