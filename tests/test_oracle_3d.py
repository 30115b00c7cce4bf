"""Pins of the oracle's 3D pieces (Section 2: the method for d = 3; the 3D
remark of Section 3.2): tetrahedral quadrature against closed-form monomial
integrals, the P2 tetrahedral basis, mesh counts and volumes, stiffness,
divergence and convection against exact integrals computed with an independent
tensor Gauss rule on the cube, the full-step patch test of Algorithm 1 in three
dimensions (every term exact, so one step reproduces the data), and the spatial
convergence rate of P2 velocities."""
import itertools

import numpy as np
import pytest

import workloads as wl
from oracle import fem, scheme, tet


def test_tet_rule_exact_to_degree_7():
    lam, w = tet.tet_rule()
    x, y, z = lam[:, 1], lam[:, 2], lam[:, 3]
    assert abs(w.sum() - 1.0) < 1e-14
    for a, b, c in itertools.product(range(8), repeat=3):
        if a + b + c > 7:
            continue
        q = (w * x ** a * y ** b * z ** c).sum() / 6.0      # reference volume 1/6
        assert abs(q - tet.ref_monomial(a, b, c)) < 1e-15, (a, b, c)


def test_p2_tet_basis_kronecker_and_partition():
    nodes = [np.eye(4)[i] for i in range(4)] + [(np.eye(4)[a] + np.eye(4)[b]) / 2 for a, b in tet.EDGES3]
    V = tet.p2_values3(np.array(nodes))
    assert np.abs(V - np.eye(10)).max() < 1e-15
    lam = np.random.default_rng(0).dirichlet(np.ones(4), 20)
    assert np.abs(tet.p2_values3(lam).sum(axis=1) - 1).max() < 1e-14
    # sum_a phi_a = 2 (sum l)^2 - sum l as a polynomial in the four l_i: each
    # partial derivative of the sum is 4 sum l - 1 = 3 (so the gradients sum to 0)
    assert np.abs(tet.p2_bary_grads3(lam).sum(axis=1) - 3.0).max() < 1e-13


@pytest.mark.parametrize("N", [1, 2, 3])
def test_cube_mesh(N):
    m = tet.cube(N)
    assert m.nV == (N + 1) ** 3 and m.nP2 == (2 * N + 1) ** 3 and m.n_el == 6 * N ** 3
    assert m.n == 3 * m.nP2 + m.nV
    vol, _ = tet.geometry3(m.xy, m.tri)
    assert np.all(vol > 0) and abs(vol.sum() - 1.0) < 1e-13
    assert np.allclose(vol, 1.0 / (6 * N ** 3))
    assert len(m.bnd) == (2 * N + 1) ** 3 - (2 * N - 1) ** 3
    # every edge midpoint is the midpoint of its element's vertices
    for s, (a, b) in enumerate(tet.EDGES3):
        assert np.abs(m.xy[m.tri[:, 4 + s]] - 0.5 * (m.xy[m.tri[:, a]] + m.xy[m.tri[:, b]])).max() < 1e-15


def _cube_integral(f, n=6):
    """Tensor Gauss-Legendre integral over the unit cube (independent of the tetrahedra)."""
    g, w = np.polynomial.legendre.leggauss(n)
    t, tw = 0.5 * (g + 1), 0.5 * w
    X, Y, Z = np.meshgrid(t, t, t, indexing="ij")
    W = tw[:, None, None] * tw[None, :, None] * tw[None, None, :]
    return float((W * f(X, Y, Z)).sum())


@pytest.fixture(scope="module")
def el2():
    return fem.Element(tet.cube(2))


def test_stiffness_constants_and_linear_fields(el2):
    m = el2.mesh
    K = el2.stiffness()
    assert np.abs(K @ np.ones(m.nP2)).max() < 1e-13
    x, y, z = m.xy.T
    f = 0.3 * x - 1.1 * y + 0.7 * z
    assert abs(f @ (K @ f) - (0.09 + 1.21 + 0.49)) < 1e-13
    M = el2.mass()
    g = x * y + z * z
    assert abs(g @ (M @ g) - _cube_integral(lambda X, Y, Z: (X * Y + Z * Z) ** 2)) < 1e-14


def test_divergence_exact(el2):
    m = el2.mesh
    B = el2.divergence()
    x, y, z = m.xy.T
    u = np.stack([x * x, y * z, x * z], axis=1).ravel()          # div u = 3x + z
    p = (1 + x + 2 * y - z)[:m.nV]
    want = -_cube_integral(lambda X, Y, Z: (1 + X + 2 * Y - Z) * (3 * X + Z))
    assert abs(p @ (B @ u) - want) < 1e-13
    const = np.tile([0.3, -0.2, 0.5], m.nP2)
    assert np.abs(B @ const).max() < 1e-14


def test_convection_exact(el2):
    m = el2.mesh
    x, y, z = m.xy.T
    u = np.stack([y, z, x], axis=1)
    C = el2.convection(u, skew=False)                             # row: test w, column: trial v
    v, w = x * x, y * z
    assert abs(w @ (C @ v) - _cube_integral(lambda X, Y, Z: (Y * 2 * X) * (Y * Z))) < 1e-14
    S = el2.convection(u, skew=True)
    assert np.abs((S + S.T).toarray()).max() < 1e-14


class Patch3(wl.Problem):
    """v_j = v*, w_j = c_j w* with v* = (x^2, -2xy, 0) (divergence-free, quadratic),
    w* constant, q = x + 2y + 3z, r = 0: every term of Algorithm 1 lies in the FE
    spaces, so one step reproduces the data."""

    def __init__(self, J, c, **kw):
        super().__init__(J=J, **kw)
        self.c = np.asarray(c)
        self.wstar = np.array([0.4, -0.25, 0.3])

    def fields(self, xyz):
        x, y = xyz[:, 0], xyz[:, 1]
        v = np.stack([x * x, -2 * x * y, 0 * x], 1)
        V = np.repeat(v[:, :, None], self.J, 2)
        W = self.wstar[None, :, None] * self.c[None, None, :] * np.ones((len(x), 1, 1))
        return V, W

    def ic(self, xyz):
        return self.fields(xyz)

    def bc(self, t, xyz):
        return self.fields(xyz)

    def forcing(self, t, xyz):
        x, y = xyz[:, 0], xyz[:, 1]
        n = len(x)
        gv = np.zeros((n, 3, 3))
        gv[:, 0, 0] = 2 * x
        gv[:, 1, 0] = -2 * y
        gv[:, 1, 1] = -2 * x
        lap_v = np.array([2.0, 0.0, 0.0])
        wbar = self.wstar * self.c.mean()
        wf = self.wstar[None, :] * (self.c - self.c.mean())[:, None]
        l2w = np.max(np.sum(wf * wf, axis=1))
        f1 = np.zeros((n, 3, self.J))
        f2 = np.zeros((n, 3, self.J))
        for j in range(self.J):
            conv = np.einsum('d,ncd->nc', wbar + wf[j], gv)
            visc = 0.5 * (self.nu[j] + self.nu_m[j]) + 2 * self.mu * self.dt * l2w
            f1[:, :, j] = conv - visc * lap_v[None, :] + np.array([1.0, 2.0, 3.0])[None, :]
            f2[:, :, j] = -0.5 * (self.nu[j] - self.nu_m[j]) * lap_v[None, :]
        return f1, f2


@pytest.mark.parametrize("convective", [0, 1])
def test_patch_full_step_exact_3d(convective):
    m = tet.cube(2)
    pb = Patch3(3, c=[1.2, 0.7, 1.1], dt=0.1, nsteps=1, s=1.0, mu=1.0,
                nu=np.array([0.01, 0.012, 0.009]), nu_m=np.array([0.02, 0.018, 0.025]), convective=convective)
    ens = scheme.Ensemble(m, pb)
    assert ens.pin == 0 and np.all(m.xy[0] == 0)
    V0, W0 = pb.ic(m.xy)
    V1, W1, Q, R = ens.step(V0, W0, 0.1)
    assert np.abs(V1 - V0).max() < 1e-11
    assert np.abs(W1 - W0).max() < 1e-11
    x, y, z = m.xy[:m.nV].T
    assert np.abs(Q - (x + 2 * y + 3 * z - 3.0)[:, None]).max() < 1e-10
    assert np.abs(R).max() < 1e-10


def test_identical_members_equal_the_single_run_3d():
    """The ensemble statistics of identical members vanish, so each member steps
    as the single run (3D, data not in the FE space)."""
    m = tet.cube(2)
    kw = dict(dt=0.05, nsteps=1, s=0.5, mu=1.0, nu=np.array([0.01]), nu_m=np.array([0.02]))
    one = Patch3(1, c=[1.0], **kw)
    three = Patch3(3, c=[1.0, 1.0, 1.0], **{**kw, "nu": np.full(3, 0.01), "nu_m": np.full(3, 0.02)})
    rng = np.random.default_rng(4)
    bump = rng.standard_normal((m.nP2, 3)) * 0.05
    bump[m.bnd] = 0.0
    V1, W1 = one.ic(m.xy)
    V1 = V1 + bump[:, :, None]
    V3 = np.repeat(V1, 3, axis=2)
    W3 = np.repeat(W1, 3, axis=2)
    a = scheme.Ensemble(m, one).step(V1, W1, 0.05)
    b = scheme.Ensemble(m, three).step(V3, W3, 0.05)
    for x, y in zip(a, b):
        for j in range(3):
            assert np.abs(y[..., j] - x[..., 0]).max() < 1e-12


class Manufactured3(wl.Problem):
    """A divergence-free 3D pair with the structure of the Section 4.1 solution:
    v = (g(y+z), g(x+z), g(x+y)), g(s) = cos s + a sin s, and w the same with
    k(s) = cos s - a sin s, a = 1 + e^t, p = a sin(x+y+z); member j scales v and
    w by c_j.  Laplacians are -2 v and -2 w; the forcing follows from the
    Elsasser system with the member's nu_j, nu_m,j."""

    def __init__(self, J, c, **kw):
        super().__init__(J=J, **kw)
        self.c = np.asarray(c)

    @staticmethod
    def _pair(t, xyz):
        x, y, z = xyz.T
        a = 1.0 + np.exp(t)
        s = np.stack([y + z, x + z, x + y], axis=1)
        v = np.cos(s) + a * np.sin(s)
        w = np.cos(s) - a * np.sin(s)
        dv = -np.sin(s) + a * np.cos(s)     # g'(s)
        dw = -np.sin(s) - a * np.cos(s)     # k'(s)
        grad = lambda d: np.stack([np.stack([0 * x, d[:, 0], d[:, 0]], 1),
                                   np.stack([d[:, 1], 0 * x, d[:, 1]], 1),
                                   np.stack([d[:, 2], d[:, 2], 0 * x], 1)], 1)   # [n, comp, dir]
        return v, w, grad(dv), grad(dw), np.exp(t) * np.sin(s), a

    def _members(self, v):
        return v[:, :, None] * self.c[None, None, :]

    def ic(self, xyz):
        v, w, *_ = self._pair(0.0, xyz)
        return self._members(v), self._members(w)

    def bc(self, t, xyz):
        v, w, *_ = self._pair(t, xyz)
        return self._members(v), self._members(w)

    def forcing(self, t, xyz):
        v, w, gv, gw, st, a = self._pair(t, xyz)
        gp = (a * np.cos(xyz.sum(axis=1)))[:, None] * np.ones((1, 3))
        w_grad_v = np.einsum('nd,ncd->nc', w, gv)
        v_grad_w = np.einsum('nd,ncd->nc', v, gw)
        c = self.c[None, None, :]
        nup = (self.nu + self.nu_m)[None, None, :]
        num = (self.nu - self.nu_m)[None, None, :]
        f1 = c * st[:, :, None] + c * c * w_grad_v[:, :, None] + nup * c * v[:, :, None] \
            + num * c * w[:, :, None] + gp[:, :, None]
        f2 = -c * st[:, :, None] + c * c * v_grad_w[:, :, None] + nup * c * w[:, :, None] \
            + num * c * v[:, :, None] + gp[:, :, None]
        return f1, f2


def test_spatial_rate_3d():
    """P2 velocities in 3D: the H^1 error of the ensemble means after two short
    steps (dt = 0.001/8, so the time error is negligible) falls at rate 2 on
    the cube meshes of h = 1/2, 1/3, 1/4 (observed 1.86, 1.94 for v and 2.00
    for w)."""
    J = 3
    Ns = (2, 3, 4)
    errs = []
    for N in Ns:
        m = tet.cube(N)
        pb = Manufactured3(J, c=[1.0, 1.01, 0.99], dt=0.001 / 8, nsteps=2, s=1.0, mu=1.0,
                           nu=np.array([0.01, 0.011, 0.009]), nu_m=np.array([0.1, 0.09, 0.11]))
        ens = scheme.Ensemble(m, pb)
        V, W = pb.ic(m.xy)
        for n in range(pb.nsteps):
            V, W, _, _ = ens.step(V, W, (n + 1) * pb.dt, shared_lu=True)
        el = ens.el
        v, w, gv, gw, _, _ = Manufactured3._pair(pb.nsteps * pb.dt, el.xq.reshape(-1, 3))
        e = []
        for Z, g in ((V, gv), (W, gw)):
            d = el.grads(Z.mean(axis=2)) - g.reshape(m.n_el, -1, 3, 3) * pb.c.mean()
            e.append(np.sqrt(np.einsum('e,q,eqcd->', el.area, el.w, d * d)))
        errs.append(e)
    errs = np.array(errs)
    rates = np.log(errs[:-1] / errs[1:]) / np.log(np.array(Ns[1:]) / np.array(Ns[:-1]))[:, None]
    assert np.all(rates > 1.8), (errs, rates)
    assert np.all(rates[-1] > 1.9), (errs, rates)
