"""Block GMRES (one Krylov space shared by the J right-hand sides, deflation of
dependent directions) against the FP64 oracle and against the per-member
Arnoldi solver over the same shared SpMM (paper, Section 1: the one matrix for
all J members invites block solvers)."""
import sys

import numpy as np
import pytest

import workloads as wl
from oracle import mesh as om, scheme
from tests.maps import node_map, p1_map, unknown_perm

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


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float64)).cuda()


@pytest.mark.parametrize("precision,tol", [(0, 1e-10), (1, 1e-9)])
def test_block_gmres_parity(L, precision, tol):
    from paper_2108_05110_amd.ensemble import Mesh
    N, J = 8, 16
    say("block gmres parity", precision)
    pb = wl.cavity(J=J, s=0.3, dt=0.01, nu_mean=0.001, num_mean=0.001, ic_amp=0.05)
    gm = Mesh(L.MHD_MESH_UNIT_SQUARE, N)
    om_ = om.unit_square(N)
    ens = scheme.Ensemble(om_, pb)
    pm2 = node_map(gm.xy, om_.xy, 1.0 / N)
    perm = unknown_perm(pm2, p1_map(gm.xy, om_, 1.0 / N), om_.nP2)
    V, W = pb.ic(om_.xy)
    r = np.random.default_rng(3)
    V = V + 0.05 * r.standard_normal(V.shape)
    W = W + 0.05 * r.standard_normal(W.shape)
    Sv = ens.shared_matrix(W)
    Gv, _ = pb.bc(0.01, om_.xy)
    F1, _ = pb.forcing(0.01, om_.xy)
    b = ens.rhs(V, W, F1, Gv)
    x_orc = ens.solve_members(Sv, b)
    A = L.mhd_ens_shared_create(gm.handle, J, 30)
    c = L.Coeffs(pb.dt, pb.mu, float(pb.nu.mean()), float(pb.nu_m.mean()), 0)
    L.mhd_ens_assemble_shared(gm.handle, c, dev(W[pm2]), J, A)
    L.mhd_ens_prepare(A, J, precision)
    x = torch.zeros((gm.n, J), dtype=torch.float64, device="cuda")
    st, _ = L.mhd_ens_solve(A, dev(b[perm]), x, J, L.solver_opts(precision, restart=10, block_krylov=1))
    say("  block iters", st.iters, "cycles", st.cycles, "relres", st.max_relres, "rank", st.min_block_rank)
    xo = np.zeros_like(b)
    xo[perm] = x.cpu().numpy()
    err = np.linalg.norm(xo - x_orc) / np.linalg.norm(x_orc)
    say("  error vs oracle", err)
    assert st.converged == 1
    assert err <= tol, err
    L.mhd_ens_shared_free(A)
    gm.close()


@pytest.mark.parametrize("precision", [0, 1])
def test_block_gmres_deflates_identical_members(L, precision):
    """Right-hand sides in four groups of four identical columns: the first
    block has rank 4, and every member's solution equals the per-member
    solver's to the solve tolerance."""
    from paper_2108_05110_amd.ensemble import Mesh, to_dev
    N, J = 16, 16
    say("block gmres deflation", precision)
    pb = wl.cavity(J=J, s=0.3, dt=0.01, ic_amp=0.05)
    gm = Mesh(L.MHD_MESH_UNIT_SQUARE, N)
    V, W = pb.ic(gm.xy)
    A = L.mhd_ens_shared_create(gm.handle, J, 30)
    c = L.Coeffs(pb.dt, pb.mu, float(pb.nu.mean()), float(pb.nu_m.mean()), 0)
    L.mhd_ens_assemble_shared(gm.handle, c, to_dev(W), J, A)
    g = torch.Generator("cuda").manual_seed(11)
    b4 = torch.randn((gm.n, 4), dtype=torch.float64, device="cuda", generator=g)
    b = b4.repeat_interleave(4, dim=1).contiguous()
    xb = torch.zeros_like(b)
    st, _ = L.mhd_ens_solve(A, b, xb, J, L.solver_opts(precision, restart=10, block_krylov=1, rtol=1e-10))
    say("  block iters", st.iters, "rank", st.min_block_rank, "relres", st.max_relres)
    assert st.converged == 1 and st.min_block_rank <= 4
    xm = torch.zeros_like(b)
    sm, _ = L.mhd_ens_solve(A, b, xm, J, L.solver_opts(precision, restart=10, rtol=1e-10))
    say("  per-member iters", sm.iters)
    rel = float(torch.linalg.norm(xb - xm) / torch.linalg.norm(xm))
    assert rel < 1e-8, rel
    for grp in range(4):
        cols = xb[:, 4 * grp:4 * grp + 4]
        spread = float((cols - cols[:, :1]).abs().max() / cols.abs().max())
        assert spread < 1e-9, spread
    L.mhd_ens_shared_free(A)
    gm.close()


def test_block_gmres_iterations_vs_per_member(L):
    """On the 32 x 32 cavity with J = 32 distinct right-hand sides, the block
    Krylov space (dimension k J after k steps) contains every member's own
    space, so its least-squares residuals after k steps are no larger than
    one Arnoldi process per member reaches; both test them after every step
    and stop a cycle at the same bar, so the block method needs no more
    iterations."""
    from paper_2108_05110_amd.ensemble import Mesh, to_dev
    N, J = 32, 32
    say("block vs per-member iterations")
    pb = wl.cavity(J=J, s=0.3, dt=0.01, ic_amp=0.05)
    gm = Mesh(L.MHD_MESH_UNIT_SQUARE, N)
    V, W = pb.ic(gm.xy)
    A = L.mhd_ens_shared_create(gm.handle, J, 30)
    c = L.Coeffs(pb.dt, pb.mu, float(pb.nu.mean()), float(pb.nu_m.mean()), 0)
    L.mhd_ens_assemble_shared(gm.handle, c, to_dev(W), J, A)
    g = torch.Generator("cuda").manual_seed(5)
    b = torch.randn((gm.n, J), dtype=torch.float64, device="cuda", generator=g)
    its = {}
    for blk in (0, 1):
        x = torch.zeros_like(b)
        st, _ = L.mhd_ens_solve(A, b, x, J, L.solver_opts(0, restart=30, block_krylov=blk, rtol=1e-10))
        its[blk] = st.iters
        say("  block" if blk else "  per-member", st.iters, st.cycles, st.max_relres)
        assert st.converged == 1
    assert its[1] <= its[0], its
    L.mhd_ens_shared_free(A)
    gm.close()
