"""Pins of the FP64 CPU oracle against closed forms, the paper's theory and printed numbers.

Each test checks the oracle against something other than itself: exact
integrals, textbook element matrices, exact discrete solutions (patch tests),
the stability theorem of Section 3.1, the convergence rates and printed
errors of Section 4.1, and structural reductions of Algorithm 1.
"""
import math
import os

import numpy as np
import pytest
import scipy.sparse as sp

import workloads as wl
from oracle import fem, mesh as om, scheme
from oracle.plain import run_plain

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


# ------------------------------------------------------------ quadrature / basis
def test_quadrature_exact_to_degree_5():
    """int_ref x^a y^b = a! b! / (a+b+2)! on the unit reference triangle (area 1/2)."""
    lam, w = fem.quad7()
    x, y = lam[:, 1], lam[:, 2]
    for a in range(6):
        for b in range(6 - a):
            got = 0.5 * np.sum(w * x ** a * y ** b)
            exact = math.factorial(a) * math.factorial(b) / math.factorial(a + b + 2)
            assert abs(got - exact) < 1e-15, (a, b)
    # degree 6 is not integrated exactly (the rule really is degree 5)
    got = 0.5 * np.sum(w * x ** 6)
    assert abs(got - math.factorial(6) / math.factorial(8)) > 1e-8


def test_p2_basis_kronecker_and_partition():
    nodes = np.array([[1, 0, 0], [0, 1, 0], [0, 0, 1], [.5, .5, 0], [0, .5, .5], [.5, 0, .5]])
    assert np.allclose(fem.p2_values(nodes), np.eye(6), atol=1e-15)
    lam = np.random.default_rng(0).dirichlet([1, 1, 1], 50)
    assert np.allclose(fem.p2_values(lam).sum(axis=1), 1.0, atol=1e-14)
    el = fem.Element(om.unit_square(2))
    assert np.abs(el.dphi.sum(axis=2)).max() < 1e-13      # gradients sum to zero


def test_p2_element_mass_closed_form():
    """Textbook P2 mass: |T|/180 * [[6,-1,-1,0,-4,0], ...] (vertex-opposite-edge -4)."""
    m = om.unit_square(1)
    el = fem.Element(m)
    Mglob = el.mass().toarray()
    # rebuild the element matrix of triangle 0 from the global one restricted to it
    t = m.tri[0]
    area = el.area[0]
    ref = np.zeros((6, 6))
    for i in range(3):
        ref[i, i] = 6
        ref[3 + i, 3 + i] = 32
    for i in range(3):
        for k in range(3):
            if i != k:
                ref[i, k] = -1
    opp = {0: 4, 1: 5, 2: 3}          # vertex -> local index of the opposite edge
    for i in range(3):
        ref[i, opp[i]] = ref[opp[i], i] = -4
    for a in range(3, 6):
        for b in range(3, 6):
            if a != b:
                ref[a, b] = 16
    ref *= area / 180.0
    ke = np.einsum('q,qa,qb->ab', el.w, el.phi, el.phi) * area
    assert np.allclose(ke, ref, atol=1e-16)
    assert abs(ref.sum() - area) < 1e-15
    assert np.allclose(ref[:3].sum(axis=1), 0, atol=1e-16)   # vertex functions integrate to 0
    assert abs(Mglob.sum() - 1.0) < 1e-14
    assert t.shape == (6,)


@pytest.fixture(scope="module")
def sq4():
    m = om.unit_square(4)
    return m, fem.Element(m)


def test_stiffness_constants_and_linear(sq4):
    m, el = sq4
    K = el.stiffness()
    assert np.abs(K @ np.ones(m.nP2)).max() < 1e-13
    a, b = 0.7, -1.3
    f = a * m.xy[:, 0] + b * m.xy[:, 1]
    assert abs(f @ K @ f - (a * a + b * b)) < 1e-13


def test_divergence_exact(sq4):
    m, el = sq4
    B = el.divergence()
    const = np.tile([0.3, -0.8], m.nP2)
    assert np.abs(B @ const).max() < 1e-14
    x, y = m.xy[:, 0], m.xy[:, 1]
    # p = x, u = (x^2, 0): -int p div u = -int 2 x^2 = -2/3
    u = np.stack([x * x, 0 * x], 1).ravel()
    assert abs(x[:m.nV] @ (B @ u) + 2.0 / 3.0) < 1e-14
    # p = x + y, u = (0, y^2): -int (x+y) 2y = -7/6
    u = np.stack([0 * x, y * y], 1).ravel()
    assert abs((x + y)[:m.nV] @ (B @ u) + 7.0 / 6.0) < 1e-14


def test_convection_forms(sq4):
    m, el = sq4
    rng = np.random.default_rng(1)
    u = rng.standard_normal((m.nP2, 2))
    N = el.convection(u, skew=True).toarray()
    assert np.abs(N + N.T).max() < 1e-14
    x, y = m.xy[:, 0], m.xy[:, 1]
    # plain form, degree-5 integrand: u = (x^2, 0), v = x^2, w = y^2 -> int x^2 2x y^2 = 1/6
    Np = el.convection(np.stack([x * x, 0 * x], 1), skew=False)
    assert abs((y * y) @ (Np @ (x * x)) - 1.0 / 6.0) < 1e-14
    # u = (1, 0), v = x^2, w = y: int 2 x y = 1/2
    Np = el.convection(np.stack([1 + 0 * x, 0 * x], 1), skew=False)
    assert abs(y @ (Np @ (x * x)) - 0.5) < 1e-14


def test_mesh_counts():
    for N in (1, 4, 16):
        m = om.unit_square(N)
        assert m.nV == (N + 1) ** 2 and m.nP2 == (2 * N + 1) ** 2 and m.n_el == 2 * N * N
        assert len(m.bnd) == 8 * N
    m = om.step_channel(2)
    area = fem.Element(m).area.sum()
    assert abs(area - 299.0) < 1e-10


# ------------------------------------------------------------ patch test of a full step
class Patch(wl.Problem):
    """v_j = v*, w_j = c_j w* with v* = (x^2, -2xy) (divergence-free, quadratic),
    w* constant, q = x + 2y, r = 0.  All terms of Algorithm 1 then lie in the FE
    spaces, so one step must reproduce the data exactly (up to LU round-off)."""

    def __init__(self, J, c, **kw):
        super().__init__(J=J, **kw)
        self.c = np.asarray(c)
        self.wstar = np.array([0.4, -0.25])

    def fields(self, xy):
        x, y = xy[:, 0], xy[:, 1]
        v = np.stack([x * x, -2 * x * y], 1)
        V = np.repeat(v[:, :, None], self.J, 2)
        W = self.wstar[None, :, None] * self.c[None, None, :] * np.ones((len(x), 1, 1))
        return V, W

    def ic(self, xy):
        return self.fields(xy)

    def bc(self, t, xy):
        return self.fields(xy)

    def forcing(self, t, xy):
        x, y = xy[:, 0], xy[:, 1]
        n = len(x)
        gv = np.zeros((n, 2, 2))
        gv[:, 0, 0] = 2 * x
        gv[:, 1, 0] = -2 * y
        gv[:, 1, 1] = -2 * x
        lap_v = np.array([2.0, 0.0])
        wbar = self.wstar * self.c.mean()
        wf = self.wstar[None, :] * (self.c - self.c.mean())[:, None]     # (J, 2)
        l2w = np.max(np.sum(wf * wf, axis=1))                            # constant field
        f1 = np.zeros((n, 2, self.J))
        f2 = np.zeros((n, 2, self.J))
        for j in range(self.J):
            conv = np.einsum('d,ncd->nc', wbar + wf[j], gv)              # (<w> + w_j') . grad v*
            visc = 0.5 * (self.nu[j] + self.nu_m[j]) + 2 * self.mu * self.dt * l2w
            f1[:, :, j] = conv - visc * lap_v[None, :] + np.array([1.0, 2.0])[None, :]
            f2[:, :, j] = -0.5 * (self.nu[j] - self.nu_m[j]) * lap_v[None, :]
        return f1, f2


@pytest.mark.parametrize("convective", [0, 1])
def test_patch_full_step_exact(convective):
    m = om.unit_square(3)
    J = 3
    pb = Patch(J, c=[1.2, 0.7, 1.1], dt=0.1, nsteps=1, s=1.0, mu=1.0,
               nu=np.array([0.01, 0.012, 0.009]), nu_m=np.array([0.02, 0.018, 0.025]),
               convective=convective)
    ens = scheme.Ensemble(m, pb)
    V0, W0 = pb.ic(m.xy)
    V1, W1, Q, R = ens.step(V0, W0, 0.1)
    assert np.abs(V1 - V0).max() < 1e-11
    assert np.abs(W1 - W0).max() < 1e-11
    q = m.xy[:m.nV, 0] + 2 * m.xy[:m.nV, 1] - 1.5          # zero-mean output pressure
    assert np.abs(Q - q[:, None]).max() < 1e-10
    assert np.abs(R).max() < 1e-10


# ------------------------------------------------------------ convergence rates (Section 4.1)
class NoPressure(wl.Manufactured):
    """The Section 4.1 solution with the pressure gradient removed from the forcing."""

    def forcing(self, t, xy):
        f1, f2 = super().forcing(t, xy)
        gp = np.cos(xy[:, 0] + xy[:, 1]) * (1 + math.exp(t))
        return f1 - gp[:, None, None], f2 - gp[:, None, None]


def _errors_21(pb, N):
    ms = om.unit_square(N)
    ens = scheme.Ensemble(ms, pb)
    el = ens.el
    ev, ew = [], []

    def cb(n, V, W, Q, R):
        gv, gw = pb.base_grad(n * pb.dt, el.xq.reshape(-1, 2))
        for Z, g, acc in ((V, gv, ev), (W, gw, ew)):
            d = el.grads(Z.mean(axis=2)) - g.reshape(ms.n_el, 7, 2, 2) * pb.c.mean()
            acc.append(np.einsum('e,q,eqcd->', el.area, el.w, d * d))

    ens.run(callback=cb, shared_lu=True)
    return math.sqrt(pb.dt * sum(ev)), math.sqrt(pb.dt * sum(ew))


def test_spatial_rate_and_printed_errors():
    """Section 4.1, Table 3 (eps = 0.01, first viscosity sample).  Pressure-robust
    Scott-Vogelius velocities do not see the pressure; Taylor-Hood with the pressure
    term removed must then show the same P2 velocity errors (to 1%) and rate 2."""
    tab = np.loadtxt(os.path.join(GOLDEN, "table1_spatial_eps001.txt"))
    J = 4
    r = np.random.default_rng(5)
    nu, num = r.uniform(0.009, 0.011, J), r.uniform(0.09, 0.11, J)
    errs = []
    for N in (4, 8, 16):
        pb = NoPressure(J=J, dt=0.001 / 8, nsteps=8, s=1, mu=1, nu=nu, nu_m=num, eps=0.01)
        errs.append(_errors_21(pb, N))
        row = tab[tab[:, 0] == N][0]
        assert abs(errs[-1][0] / row[1] - 1) < 0.01, (N, errs[-1], row)
        assert abs(errs[-1][1] / row[2] - 1) < 0.01, (N, errs[-1], row)
    errs = np.array(errs)
    rates = np.log2(errs[:-1] / errs[1:])
    assert np.all(rates > 1.95), rates


def test_spatial_rate_with_pressure_taylor_hood():
    """With the pressure of Section 4.1 present, Taylor-Hood velocities carry a
    pressure-dependent error (no pressure robustness): the observed rate rises
    towards 2 and the error stays above the pressure-free one."""
    J = 2
    pbk = dict(J=J, dt=0.001 / 8, nsteps=8, s=1, mu=1, nu=np.array([0.01, 0.0105]),
               nu_m=np.array([0.1, 0.095]), eps=0.01)
    e = np.array([_errors_21(wl.Manufactured(**pbk), N)[0] for N in (8, 16, 32)])
    rates = np.log2(e[:-1] / e[1:])
    assert rates[1] > rates[0] > 1.4, rates


def test_temporal_rate_and_printed_errors():
    """Section 4.1 temporal test (T = 1, dt = T/2 ... T/16, first viscosity sample,
    eps = 0.01) on a 16x16 mesh: first order in time, and the time-dominated
    errors agree with Table 6 (v to 2 %, w to 6 %: the paper's random sample of
    20 viscosity pairs is not published)."""
    tab = np.loadtxt(os.path.join(GOLDEN, "table6_temporal_eps001.txt"))
    pbk = dict(J=2, s=1, mu=1, nu=np.array([0.0095, 0.0105]), nu_m=np.array([0.105, 0.095]),
               eps=0.01)
    e = []
    for M in (2, 4, 8, 16):
        pb = wl.Manufactured(dt=1.0 / M, nsteps=M, **pbk)
        e.append(_errors_21(pb, 16))
        row = tab[tab[:, 0] == M][0]
        assert abs(e[-1][0] / row[1] - 1) < 0.02, (M, e[-1], row)
        assert abs(e[-1][1] / row[2] - 1) < 0.06, (M, e[-1], row)
    e = np.array(e)
    rates = np.log2(e[:-1] / e[1:])
    assert np.all(rates > 0.85) and np.all(rates < 1.15), rates


# ------------------------------------------------------------ stability theorem (Section 3.1)
def _norms(ens, Z):
    M2, K2 = ens.M2, ens.K2
    l2 = np.array([Z[:, :, j].ravel() @ (M2 @ Z[:, :, j].ravel()) for j in range(Z.shape[2])])
    h1 = np.array([Z[:, :, j].ravel() @ (K2 @ Z[:, :, j].ravel()) for j in range(Z.shape[2])])
    return l2, h1


def test_stability_inequality_and_energy_decay():
    """Section 4.2 setting (f = g = 0, homogeneous BC, eps = 0.01 initial data,
    (nu, nu_m) in [0.009,0.011] x [0.09,0.11], dt = 0.05, T = 1) on a 16x16 mesh:
    the per-member bound of the stability theorem holds at every M and the
    ensemble-mean energy decays."""
    J = 4
    r = np.random.default_rng(7)
    nu, num = r.uniform(0.009, 0.011, J), r.uniform(0.09, 0.11, J)

    class Homog(wl.Manufactured):
        def forcing(self, t, xy):
            z = np.zeros((len(xy), 2, self.J))
            return z, z.copy()

        def bc(self, t, xy):
            return self.forcing(t, xy)

    pb = Homog(J=J, dt=0.05, nsteps=20, s=1, mu=1, nu=nu, nu_m=num, eps=0.01)
    ms = om.unit_square(16)
    ens = scheme.Ensemble(ms, pb)
    nub, numb = nu.mean(), num.mean()
    alpha = nub + numb - np.abs(nu - num) - np.abs((nu - nub) + (num - numb))
    assert np.all(alpha > 0)
    hist = ens.run(shared_lu=True)
    l2v0, h1v0 = _norms(ens, hist[0][0])
    l2w0, h1w0 = _norms(ens, hist[0][1])
    rhs = l2v0 + l2w0 + 0.5 * (nub + numb) * pb.dt * (h1v0 + h1w0)
    acc = np.zeros(J)
    energies = [ens.energy(*hist[0])]
    for Mstep in range(1, len(hist)):
        l2v, h1v = _norms(ens, hist[Mstep - 1][0])
        l2w, h1w = _norms(ens, hist[Mstep - 1][1])
        acc += 0.5 * alpha * pb.dt * (h1v + h1w)
        l2v, h1v = _norms(ens, hist[Mstep][0])
        l2w, h1w = _norms(ens, hist[Mstep][1])
        lhs = l2v + l2w + 0.5 * (nub + numb) * pb.dt * (h1v + h1w) + acc
        assert np.all(lhs <= rhs * (1 + 1e-12)), (Mstep, lhs, rhs)
        energies.append(ens.energy(*hist[Mstep]))
    assert np.all(np.diff(energies[1:]) < 0)


# ------------------------------------------------------------ structural reductions
def test_energy_closed_form():
    """E_h = 1/2 (||<v_h>||^2 + ||<w_h>||^2) (Section 4.2) on member fields whose
    mean is known in closed form: v_j = c_j (x, y^2), w_j = d_j (1, -2) with
    mean(c) = 3, mean(d) = -1, so ||<v>||^2 = 9 (1/3 + 1/5) and ||<w>||^2 = 5
    on the unit square (P2 interpolation and the P2 mass matrix are exact for
    these fields); on the step channel the constant field measures the area
    30 * 10 - 1.  A dropped 1/2, a mean of member norms instead of the norm of
    the mean, a single velocity component or a swapped variable all fail."""
    c = np.array([1.0, 2.0, 6.0])
    d = np.array([0.0, 1.0, -4.0])
    pb = wl.cavity(J=3, s=0.1, dt=0.01)
    m = om.unit_square(6)
    ens = scheme.Ensemble(m, pb)
    x, y = m.xy[:, 0], m.xy[:, 1]
    V = np.stack([x, y * y], axis=1)[:, :, None] * c[None, None, :]
    W = np.array([1.0, -2.0])[None, :, None] * d[None, None, :] * np.ones((m.nP2, 1, 1))
    assert abs(ens.energy(V, W) - 0.5 * (9.0 * (1.0 / 3.0 + 1.0 / 5.0) + 5.0)) < 1e-13
    assert abs(ens.energy(W, V) - ens.energy(V, W)) < 1e-13
    assert abs(ens.energy(V, 0 * W) - 0.5 * 9.0 * 8.0 / 15.0) < 1e-13
    pc = wl.step_channel(J=2, delta=0.1, s=0.01, dt=0.02, nsteps=1)
    mc = om.step_channel(1)
    ec = scheme.Ensemble(mc, pc)
    Vc = np.array([1.0, -2.0])[None, :, None] * np.array([0.5, 1.5])[None, None, :] * np.ones((mc.nP2, 1, 1))
    assert abs(ec.energy(Vc, 0 * Vc) - 0.5 * 5.0 * 299.0) < 1e-9


def test_J1_reduces_to_plain_scheme():
    pb = wl.manufactured(J=1, eps=0.0, dt=0.01, nsteps=4)
    ms = om.unit_square(6)
    hist = scheme.Ensemble(ms, pb).run()
    plain = run_plain(ms, pb)
    for (V, W), (v, w) in zip(hist, plain):
        assert np.abs(V[:, :, 0] - v).max() < 1e-12
        assert np.abs(W[:, :, 0] - w).max() < 1e-12


def test_identical_members_equal_single_run():
    base = wl.cavity(J=1, s=0.5, dt=0.02, nsteps=3, nu_mean=0.01, num_mean=0.02, ic_amp=0.05)
    J = 3
    pb = wl.Cavity(J=J, dt=base.dt, nsteps=3, s=base.s, mu=1.0, nu=np.repeat(base.nu, J),
                   nu_m=np.repeat(base.nu_m, J), ic_coef=np.repeat(base.ic_coef, J, 0))
    ms = om.unit_square(6)
    h1 = scheme.Ensemble(ms, base).run()
    hJ = scheme.Ensemble(ms, pb).run()
    for (V, W), (v, w) in zip(hJ, h1):
        for j in range(J):
            assert np.abs(V[:, :, j] - v[:, :, 0]).max() < 1e-12
            assert np.abs(W[:, :, j] - w[:, :, 0]).max() < 1e-12


def test_v_w_swap_symmetry_s0():
    """s = 0 makes v = w = u in the data; the scheme is symmetric under v <-> w."""
    pb = wl.cavity(J=3, s=0.0, dt=0.05, nsteps=3, nu_mean=0.01, num_mean=0.01, ic_amp=0.1)
    pb.nu_m = pb.nu.copy()
    hist = scheme.Ensemble(om.unit_square(6), pb).run()
    for V, W in hist:
        assert np.abs(V - W).max() < 1e-12


def test_member_permutation_equivariance():
    pb = wl.cavity(J=4, s=0.3, dt=0.05, nsteps=2, nu_mean=0.01, num_mean=0.02, ic_amp=0.1)
    perm = np.array([2, 0, 3, 1])
    pp = wl.Cavity(J=4, dt=pb.dt, nsteps=2, s=pb.s, mu=1.0, nu=pb.nu[perm], nu_m=pb.nu_m[perm],
                   ic_coef=pb.ic_coef[perm])
    ms = om.unit_square(5)
    a = scheme.Ensemble(ms, pb).run()[-1]
    b = scheme.Ensemble(ms, pp).run()[-1]
    assert np.abs(a[0][:, :, perm] - b[0]).max() < 1e-12
    assert np.abs(a[1][:, :, perm] - b[1]).max() < 1e-12


def test_shared_lu_equals_per_member_lu():
    pb = wl.cavity(J=3, s=0.1, dt=0.01, nsteps=1, nu_mean=0.01, num_mean=0.01, ic_amp=0.1)
    ms = om.unit_square(6)
    ens = scheme.Ensemble(ms, pb)
    V, W = pb.ic(ms.xy)
    a = ens.step(V, W, 0.01, shared_lu=False)
    b = ens.step(V, W, 0.01, shared_lu=True)
    for x, y in zip(a, b):
        assert np.abs(x - y).max() < 1e-13


@pytest.mark.parametrize("kind", ["square", "channel"])
def test_nested_dissection_order(kind):
    """The nested-dissection order is a permutation whose separators split the
    matrix graph (no entry couples the two halves of a dissection), and a
    solve in that order matches the default SuperLU ordering to rounding, with
    a do-nothing outflow (channel) and with the pressure pin (square)."""
    if kind == "square":
        pb = wl.cavity(J=2, s=0.1, dt=0.01, nsteps=1, nu_mean=0.01, num_mean=0.01, ic_amp=0.1)
        ms = om.unit_square(8)
    else:
        pb = wl.step_channel(J=2, delta=1e-2, s=0.01, dt=0.02)
        ms = om.step_channel(2)
    ens = scheme.Ensemble(ms, pb)
    p = om.nested_dissection(ms, leaf=16)
    assert np.array_equal(np.sort(p), np.arange(ms.n))
    V, W = pb.ic(ms.xy)
    S = ens.shared_matrix(W).tocsr()
    # first split: the unknowns strictly either side of the first cut never couple
    nV = ms.nV
    xy = np.concatenate([np.repeat(ms.xy, 2, axis=0), ms.xy[:nV]])
    ax = int(np.argmax(xy.max(0) - xy.min(0)))
    sep = p[-np.count_nonzero(np.isclose(xy[:, ax], xy[p[-1], ax])):]
    cut = xy[sep[0], ax]
    assert np.allclose(xy[sep, ax], cut)
    side = np.sign(np.round(xy[:, ax] - cut, 9))
    r, c = S.nonzero()
    assert not np.any(side[r] * side[c] < 0)
    assert np.any(side < 0) and np.any(side > 0)
    a = ens.step(V, W, pb.dt, shared_lu=True, ordering="ND")
    b = ens.step(V, W, pb.dt, shared_lu=True)
    for x, y in zip(a, b):
        assert np.abs(x - y).max() <= 1e-11 * max(1.0, np.abs(y).max())


def test_member_subset_solve():
    pb = wl.cavity(J=4, s=0.1, dt=0.01, nsteps=1, nu_mean=0.01, num_mean=0.01, ic_amp=0.1)
    ms = om.unit_square(5)
    ens = scheme.Ensemble(ms, pb)
    V, W = pb.ic(ms.xy)
    full = ens.step(V, W, 0.01)
    sub = ens.step(V, W, 0.01, members=[1, 3])
    assert np.abs(full[0][:, :, [1, 3]] - sub[0]).max() < 1e-13


def test_dirichlet_rows_and_pin():
    pb = wl.cavity(J=2, s=0.1)
    ms = om.unit_square(4)
    ens = scheme.Ensemble(ms, pb)
    V, W = pb.ic(ms.xy)
    S = ens.shared_matrix(W).tocsr()
    for i in ens.dnodes:
        for c in (0, 1):
            row = S.getrow(2 * i + c)
            assert row.nnz == 1 and row.indices[0] == 2 * i + c and row.data[0] == 1.0
    prow = S.getrow(2 * ms.nP2 + ens.pin)
    assert prow.nnz == 1 and prow.data[0] == 1.0
    assert np.allclose(ms.xy[ens.pin], [0, 0])


# ------------------------------------------------------------ problem data
def test_manufactured_forcing_matches_symbolic():
    """The hand-derived forcing of the Section 4.1 solution against sympy."""
    sy = pytest.importorskip("sympy")
    x, y, t, nu, nm, c = sy.symbols('x y t nu nm c')
    a = 1 + sy.exp(t)
    v = sy.Matrix([sy.cos(y) + a * sy.sin(y), sy.sin(x) + a * sy.cos(x)]) * c
    w = sy.Matrix([sy.cos(y) - a * sy.sin(y), sy.sin(x) - a * sy.cos(x)]) * c
    p = sy.sin(x + y) * a

    def conv(u, z):
        return sy.Matrix([u[0] * sy.diff(z[i], x) + u[1] * sy.diff(z[i], y) for i in range(2)])

    def lap(z):
        return sy.Matrix([sy.diff(z[i], x, 2) + sy.diff(z[i], y, 2) for i in range(2)])

    gp = sy.Matrix([sy.diff(p, x), sy.diff(p, y)])
    f1 = sy.diff(v, t) + conv(w, v) - (nu + nm) / 2 * lap(v) - (nu - nm) / 2 * lap(w) + gp
    f2 = sy.diff(w, t) + conv(v, w) - (nu + nm) / 2 * lap(w) - (nu - nm) / 2 * lap(v) + gp
    F = sy.lambdify((x, y, t, nu, nm, c), [f1[0], f1[1], f2[0], f2[1]], 'numpy')
    pb = wl.Manufactured(J=2, dt=0.1, nsteps=1, s=1, mu=1, nu=np.array([0.01, 0.02]),
                         nu_m=np.array([0.1, 0.05]), eps=0.3)
    xy = np.random.default_rng(3).uniform(0, 1, (20, 2))
    tt = 0.37
    g1, g2 = pb.forcing(tt, xy)
    for j in range(2):
        vals = F(xy[:, 0], xy[:, 1], tt, pb.nu[j], pb.nu_m[j], pb.c[j])
        assert np.allclose(g1[:, 0, j], vals[0], atol=1e-13)
        assert np.allclose(g1[:, 1, j], vals[1], atol=1e-13)
        assert np.allclose(g2[:, 0, j], vals[2], atol=1e-13)
        assert np.allclose(g2[:, 1, j], vals[3], atol=1e-13)


def test_member_factor_pattern():
    """c_j = 1 + (-1)^(j+1) ceil(j/2) eps/5 (Section 4.1): +, -, ++, --, ..."""
    c = wl.member_factor(6, 0.5)
    assert np.allclose(c, [1.1, 0.9, 1.2, 0.8, 1.3, 0.7])
    assert abs(wl.member_factor(20, 0.01).mean() - 1) < 1e-15


def test_modes_divergence_free_and_vanish_on_boundary():
    ms = om.unit_square(8)
    pts = np.random.default_rng(4).uniform(0.05, 0.95, (30, 2))
    h = 1e-5
    ex, ey = np.array([h, 0.0]), np.array([0.0, h])
    for k, l in wl.MODES:
        f = wl.mode_field(k, l, ms.xy)
        assert np.abs(f[ms.bnd]).max() < 1e-12
        div = ((wl.mode_field(k, l, pts + ex)[:, 0] - wl.mode_field(k, l, pts - ex)[:, 0])
               + (wl.mode_field(k, l, pts + ey)[:, 1] - wl.mode_field(k, l, pts - ey)[:, 1])) / (2 * h)
        assert np.abs(div).max() < 1e-6
