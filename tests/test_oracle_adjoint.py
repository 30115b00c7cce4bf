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
