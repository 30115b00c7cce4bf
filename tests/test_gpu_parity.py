"""GPU parity: the HIP path through the C ABI against the FP64 CPU oracle.

Node numberings differ (each side meshes on its own); entries are mapped by
node coordinates.  Bars: assembly entries to 1e-13 relative to the largest
entry; FP64 solves and steps to relative L2 (P2 mass norm) 1e-10; FP32 inner
solves with FP64 refinement to 1e-6 per step from identical inputs.
"""
import sys

import numpy as np
import pytest

import workloads as wl
from oracle import mesh as om, scheme
from tests.maps import csr_from_view, mass_rel_err, node_map, p1_map, unknown_perm

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def L():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2108_05110_amd import _lib
    _lib.lib()
    return _lib


def setup_pair(L, N, pb):
    from paper_2108_05110_amd.ensemble import Mesh
    gm = Mesh(L.MHD_MESH_UNIT_SQUARE, N)
    om_ = om.unit_square(N)
    ens = scheme.Ensemble(om_, pb)
    pm2 = node_map(gm.xy, om_.xy, 1.0 / N)
    pm1 = p1_map(gm.xy, om_, 1.0 / N)
    perm = unknown_perm(pm2, pm1, om_.nP2)
    return gm, om_, ens, pm2, pm1, perm


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float64)).cuda()


def to_gpu_order(Z, pm2):
    """oracle-numbered (nP2, 2, J) -> GPU numbering"""
    return Z[pm2]


def random_state(pb, xy, seed):
    V, W = pb.ic(xy)
    r = np.random.default_rng(seed)
    V = V + 0.05 * r.standard_normal(V.shape)
    W = W + 0.05 * r.standard_normal(W.shape)
    return V, W


def test_mesh_coordinates_and_dirichlet(L):
    from paper_2108_05110_amd.ensemble import Mesh
    for N in (3, 8):
        say("mesh", N)
        gm = Mesh(L.MHD_MESH_UNIT_SQUARE, N)
        om_ = om.unit_square(N)
        pm = node_map(gm.xy, om_.xy, 1.0 / N)
        assert len(np.unique(pm)) == om_.nP2
        assert sorted(pm[gm.dir_nodes]) == sorted(om_.bnd)
        gm.close()


@pytest.mark.parametrize("J,convective", [(3, 0), (3, 1), (70, 0)])
def test_shared_matrix_parity(L, J, convective):
    say("shared matrix", J, convective)
    N = 6
    pb = wl.cavity(J=J, s=0.3, dt=0.02, nu_mean=0.01, num_mean=0.02, ic_amp=0.2, convective=convective)
    gm, om_, ens, pm2, pm1, perm = setup_pair(L, N, pb)
    V, W = random_state(pb, om_.xy, 1)
    S_orc = ens.shared_matrix(W).tocsr()
    A = L.mhd_ens_shared_create(gm.handle, J, 4)
    c = L.Coeffs(pb.dt, pb.mu, float(pb.nu.mean()), float(pb.nu_m.mean()), convective)
    L.mhd_ens_assemble_shared(gm.handle, c, dev(to_gpu_order(W, pm2)), J, A)
    S_gpu = csr_from_view(torch, L.mhd_ens_shared_csr(A))
    P = np.zeros(len(perm), dtype=np.int64)
    P[perm] = np.arange(len(perm))
    S_g_in_o = S_gpu[P][:, P]           # oracle ordering
    D = (S_g_in_o - S_orc).tocsr()
    scale = abs(S_orc).max()
    assert abs(D).max() <= 1e-13 * scale, abs(D).max() / scale
    L.mhd_ens_shared_free(A)
    gm.close()


@pytest.mark.parametrize("J,which", [(3, 0), (3, 1), (33, 0), (1, 1)])
def test_rhs_parity(L, J, which):
    say("rhs", J, which)
    N = 6
    pb = wl.manufactured(J=J, eps=0.3, dt=0.05)
    gm, om_, ens, pm2, pm1, perm = setup_pair(L, N, pb)
    V, W = random_state(pb, om_.xy, 2)
    t1 = 0.05
    F1, F2 = pb.forcing(t1, om_.xy)
    Gv, Gw = pb.bc(t1, om_.xy)
    selfZ, otherZ, F, G = (V, W, F1, Gv) if which == 0 else (W, V, F2, Gw)
    b_orc = ens.rhs(selfZ, otherZ, F, G)
    n = gm.n
    rhs = torch.zeros((n, J), dtype=torch.float64, device="cuda")
    c = L.Coeffs(pb.dt, pb.mu, float(pb.nu.mean()), float(pb.nu_m.mean()), 0)
    Gdir = to_gpu_order(G, pm2)[gm.dir_nodes]
    L.mhd_ens_assemble_rhs(gm.handle, c, which, J, dev(to_gpu_order(selfZ, pm2)), dev(to_gpu_order(otherZ, pm2)),
                           dev(pb.nu), dev(pb.nu_m), dev(to_gpu_order(F, pm2)), dev(Gdir), rhs)
    b_gpu = rhs.cpu().numpy()
    b_g_in_o = np.zeros_like(b_gpu)
    b_g_in_o[perm] = b_gpu
    scale = np.abs(b_orc).max()
    assert np.abs(b_g_in_o - b_orc).max() <= 1e-13 * scale
    # FP32 output: the same FP64 arithmetic, rounded once when stored
    r32 = torch.full((n, J), float("nan"), dtype=torch.float32, device="cuda")
    L.mhd_ens_assemble_rhs(gm.handle, c, which, J, dev(to_gpu_order(selfZ, pm2)), dev(to_gpu_order(otherZ, pm2)),
                           dev(pb.nu), dev(pb.nu_m), dev(to_gpu_order(F, pm2)), dev(Gdir), r32)
    assert torch.equal(r32, rhs.to(torch.float32))
    gm.close()


@pytest.mark.parametrize("m,J", [(2, 20), (1, 70)])
def test_rhs_parity_step_channel(L, m, J):
    """Right-hand sides on the step channel (cells missing under the step, a
    do-nothing outflow) against the oracle, J spanning several member slices
    with a ragged last one."""
    from paper_2108_05110_amd.ensemble import Mesh
    say("rhs channel", m, J)
    pb = wl.step_channel(J=J, delta=0.1, s=0.01, dt=0.02)
    gm = Mesh(L.MHD_MESH_STEP_CHANNEL, m, 1)
    om_ = om.step_channel(m)
    ens = scheme.Ensemble(om_, pb)
    h = 1.0 / m
    pm2 = node_map(gm.xy, om_.xy, h)
    pm1 = p1_map(gm.xy, om_, h)
    perm = unknown_perm(pm2, pm1, om_.nP2)
    V, W = random_state(pb, om_.xy, 5)
    Gv, _ = pb.bc(pb.dt, om_.xy)
    F1, _ = pb.forcing(pb.dt, om_.xy)
    b_orc = ens.rhs(V, W, F1, Gv)
    rhs = torch.full((gm.n, J), float("nan"), dtype=torch.float64, device="cuda")
    c = L.Coeffs(pb.dt, pb.mu, float(pb.nu.mean()), float(pb.nu_m.mean()), 0)
    L.mhd_ens_assemble_rhs(gm.handle, c, 0, J, dev(to_gpu_order(V, pm2)), dev(to_gpu_order(W, pm2)), dev(pb.nu),
                           dev(pb.nu_m), dev(to_gpu_order(F1, pm2)), dev(to_gpu_order(Gv, pm2)[gm.dir_nodes]), rhs)
    b_gpu = rhs.cpu().numpy()
    assert np.isfinite(b_gpu).all()
    b_g_in_o = np.zeros_like(b_gpu)
    b_g_in_o[perm] = b_gpu
    assert np.abs(b_g_in_o - b_orc).max() <= 1e-13 * np.abs(b_orc).max()
    gm.close()


# J = 16 (FP32 inner solves) takes the matrix-core coarse-grid solve, J = 4 the vector one
@pytest.mark.parametrize("precision,tol,J", [(0, 1e-10, 4), (1, 1e-9, 4), (1, 1e-9, 16)])
def test_solve_parity(L, precision, tol, J):
    say("solve", precision, J)
    N = 8
    pb = wl.cavity(J=J, s=0.3, dt=0.01, nu_mean=0.001, num_mean=0.001, ic_amp=0.05)
    gm, om_, ens, pm2, pm1, perm = setup_pair(L, N, pb)
    V, W = random_state(pb, om_.xy, 3)
    Sv = ens.shared_matrix(W)
    Gv, _ = pb.bc(0.01, om_.xy)
    F1, _ = pb.forcing(0.01, om_.xy)
    b = ens.rhs(V, W, F1, Gv)
    x_orc = ens.solve_members(Sv, b)
    A = L.mhd_ens_shared_create(gm.handle, J, 30)
    c = L.Coeffs(pb.dt, pb.mu, float(pb.nu.mean()), float(pb.nu_m.mean()), 0)
    L.mhd_ens_assemble_shared(gm.handle, c, dev(to_gpu_order(W, pm2)), J, A)
    bg = b[perm]
    x = torch.zeros((gm.n, J), dtype=torch.float64, device="cuda")
    L.mhd_ens_prepare(A, J, precision)       # the tuned kernel plans, as a context would use them
    st, _ = L.mhd_ens_solve(A, dev(bg), x, J, L.solver_opts(precision))
    say("  iters", st.iters, "cycles", st.cycles, "relres", st.max_relres)
    xo = np.zeros_like(bg)
    xo[perm] = x.cpu().numpy()
    err = np.linalg.norm(xo - x_orc) / np.linalg.norm(x_orc)
    assert err <= tol, err
    L.mhd_ens_shared_free(A)
    gm.close()


def run_pair(L, N, pb, nsteps, precision):
    from paper_2108_05110_amd.ensemble import Stepper
    gm, om_, ens, pm2, pm1, perm = setup_pair(L, N, pb)
    stp = Stepper(gm, pb, opts=L.solver_opts(precision))
    V, W = pb.ic(om_.xy)
    errs = []
    for n in range(nsteps):
        st = stp.step()
        V, W, Q, R = ens.step(V, W, (n + 1) * pb.dt, shared_lu=True)
        Vg = np.zeros_like(V)
        Wg = np.zeros_like(W)
        Vg[pm2] = stp.V.cpu().numpy()
        Wg[pm2] = stp.W.cpu().numpy()
        errs.append((mass_rel_err(ens, Vg, V), mass_rel_err(ens, Wg, W)))
        say("  step", n + 1, errs[-1], st.v.iters, st.w.iters)
    qg = stp.Q.cpu().numpy()
    qo = np.zeros_like(qg)
    qo[pm1] = qg
    stp.close()
    gm.close()
    return np.array(errs), qo, Q


def test_step_parity_manufactured_fp64(L):
    """Config of the 16x16 manufactured run: J = 2, dt = 0.01, 10 steps, FP64."""
    say("step C1 fp64")
    pb = wl.manufactured(J=2, eps=0.01, dt=0.01, nsteps=10)
    errs, qg, qo = run_pair(L, 16, pb, 10, 0)
    assert errs.max() <= 1e-10, errs.max()
    assert np.abs(qg - qo).max() <= 1e-7 * np.abs(qo).max()


def test_step_parity_cavity_fp32ir(L):
    say("step cavity fp32+IR")
    pb = wl.cavity(J=5, s=0.1, dt=0.01, nsteps=4, ic_amp=1e-2)
    errs, _, _ = run_pair(L, 16, pb, 4, 1)
    assert errs.max() <= 1e-6, errs.max()


def test_identical_members_bitwise(L):
    from paper_2108_05110_amd.ensemble import Mesh, Stepper
    say("identical members")
    base = wl.cavity(J=1, s=0.5, dt=0.02, nu_mean=0.01, num_mean=0.02, ic_amp=0.05)
    J = 4
    pb = wl.Cavity(J=J, dt=base.dt, nsteps=3, s=base.s, mu=1.0, nu=np.repeat(base.nu, J),
                   nu_m=np.repeat(base.nu_m, J), ic_coef=np.repeat(base.ic_coef, J, 0))
    gm = Mesh(L.MHD_MESH_UNIT_SQUARE, 8)
    s = Stepper(gm, pb)
    s1 = Stepper(gm, base)
    for _ in range(3):
        s.step()
        s1.step()
    V = s.V.cpu().numpy()
    v1 = s1.V.cpu().numpy()
    for j in range(J):
        assert np.array_equal(V[:, :, j], V[:, :, 0])
    assert np.abs(V[:, :, 0] - v1[:, :, 0]).max() < 1e-11
    s.close()
    s1.close()
    gm.close()


def test_single_step_cavity_128(L):
    """128x128 cavity, J = 20, one step from the initial state, members 0, 7, 19."""
    from paper_2108_05110_amd.ensemble import Mesh, Stepper
    say("single step 128^2 J=20")
    N, J = 128, 20
    pb = wl.cavity(J=J, s=0.1, dt=0.01)
    gm = Mesh(L.MHD_MESH_UNIT_SQUARE, N)
    for prec, tol in ((0, 1e-10), (1, 1e-6)):
        stp = Stepper(gm, pb, opts=L.solver_opts(prec))
        st = stp.step()
        say("  prec", prec, "iters", st.v.iters, st.w.iters, "cycles", st.v.cycles)
        Vg = stp.V.cpu().numpy()
        stp.close()
        if prec == 0:
            om_ = om.unit_square(N)
            ens = scheme.Ensemble(om_, pb)
            pm2 = node_map(gm.xy, om_.xy, 1.0 / N)
            V0, W0 = pb.ic(om_.xy)
            members = [0, 7, 19]
            V1, W1, _, _ = ens.step(V0, W0, pb.dt, shared_lu=True, members=members)
        Vo = np.zeros((len(pm2), 2, len(members)))
        Vo[pm2] = Vg[:, :, members]
        err = mass_rel_err(ens, Vo, V1)
        say("  err", err)
        assert err <= tol, (prec, err)
    gm.close()


def test_step_parity_step_channel_natural_outflow(L):
    """Step channel [0,30]x[0,10] minus the unit inlet step, h = 1/2, do-nothing
    outflow (no pressure pin), J = 3, two FP64 steps; pressures compared as is."""
    from paper_2108_05110_amd.ensemble import Mesh, Stepper
    say("step channel")
    m = 2
    pb = wl.step_channel(J=3, delta=0.1, s=0.01, dt=0.02, nsteps=2)
    gm = Mesh(L.MHD_MESH_STEP_CHANNEL, m, 1)
    om_ = om.step_channel(m)
    ens = scheme.Ensemble(om_, pb)
    assert ens.pin is None and gm.info.pin == -1
    h = 1.0 / m
    pm2 = node_map(gm.xy, om_.xy, h)
    pm1 = p1_map(gm.xy, om_, h)
    assert len(gm.dir_nodes) == len(ens.dnodes)
    stp = Stepper(gm, pb, opts=L.solver_opts(L.MHD_FP64))
    V, W = pb.ic(om_.xy)
    for n in range(2):
        st = stp.step()
        V, W, Q, R = ens.step(V, W, (n + 1) * pb.dt, shared_lu=True)
        Vg = np.zeros_like(V)
        Vg[pm2] = stp.V.cpu().numpy()
        Wg = np.zeros_like(W)
        Wg[pm2] = stp.W.cpu().numpy()
        ev, ew = mass_rel_err(ens, Vg, V), mass_rel_err(ens, Wg, W)
        say("  step", n + 1, ev, ew, st.v.iters, st.w.iters)
        assert max(ev, ew) <= 1e-10
    qg = np.zeros_like(Q)
    qg[pm1] = stp.Q.cpu().numpy()
    assert np.abs(qg - Q).max() <= 1e-8 * np.abs(Q).max()
    stp.close()
    gm.close()
