"""Pins of the oracle's 3D pieces (Section 2: the method for d = 3; the 3D
remark of Section 3.2): tetrahedral quadrature against closed-form monomial
integrals, the P2 tetrahedral basis, mesh counts and volumes, stiffness,
divergence and convection against exact integrals computed with an independent
tensor Gauss rule on the cube, and the full-step patch test of Algorithm 1 in
three dimensions (every term exact, so one step reproduces the data)."""
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
