"""GPU tests of the C ABI's promises: solves and steps allocate no device
memory (only creation and the explicit tuning calls do), per-member solver
statistics, the stability-condition warnings of Section 3.1, and non-finite
residual detection under the fixed (graph-capturable) schedule."""
import sys

import numpy as np
import pytest

import workloads as wl

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


def test_steps_and_solves_allocate_nothing(L):
    from paper_2108_05110_amd.ensemble import Mesh, Stepper, fixed_schedule_opts, to_dev
    N, J = 32, 16
    say("alloc-free: 32^2, J=16, graph fixed schedule and eager adaptive steps")
    pb = wl.cavity(J=J, s=0.1, dt=0.01, ic_amp=0.05)
    gm = Mesh(L.MHD_MESH_UNIT_SQUARE, N)
    g = Stepper(gm, pb, opts=fixed_schedule_opts(), time_dependent_data=False, graph=True)
    e = Stepper(gm, pb, opts=L.solver_opts(L.MHD_FP32_IR), time_dependent_data=False)
    torch.cuda.synchronize()
    n0, b0 = L.mhd_ens_alloc_stats()
    for _ in range(2):
        g.step(stats=True)      # the first call captures the step graph
        e.step(stats=True)
    torch.cuda.synchronize()
    n1, b1 = L.mhd_ens_alloc_stats()
    assert (n1, b1) == (n0, b0), (n0, n1, b0, b1)
    # a bare solve: prepare allocates (tilings, packed entries), the solve does not
    A = L.mhd_ens_shared_create(gm.handle, J, 8)
    c = L.Coeffs(pb.dt, pb.mu, float(pb.nu.mean()), float(pb.nu_m.mean()), 0)
    L.mhd_ens_assemble_shared(gm.handle, c, e.W.reshape(-1), J, A)
    L.mhd_ens_prepare(A, J, L.MHD_FP32_IR)
    b = torch.randn((gm.n, J), dtype=torch.float64, device="cuda")
    x = torch.zeros_like(b)
    torch.cuda.synchronize()
    n2, _ = L.mhd_ens_alloc_stats()
    st, _ = L.mhd_ens_solve(A, b, x, J, L.solver_opts(L.MHD_FP32_IR, restart=8))
    st2, _ = L.mhd_ens_solve(A, b, torch.zeros_like(b), J - 3, L.solver_opts(L.MHD_FP32_IR, restart=8))
    torch.cuda.synchronize()
    n3, _ = L.mhd_ens_alloc_stats()
    assert n3 == n2, (n2, n3)
    L.mhd_ens_shared_free(A)
    g.close()
    e.close()
    gm.close()


def test_per_member_statistics(L):
    from paper_2108_05110_amd.ensemble import Mesh, Stepper, fixed_schedule_opts
    N, J = 16, 8
    say("per-member statistics: adaptive solve and fixed-schedule step")
    pb = wl.cavity(J=J, s=0.1, dt=0.01, ic_amp=0.05)
    gm = Mesh(L.MHD_MESH_UNIT_SQUARE, N)
    a = Stepper(gm, pb, opts=L.solver_opts(L.MHD_FP64), time_dependent_data=False)
    st = a.step(stats=True)
    for q in (st.v, st.w):
        rel, its = L.member_stats(q, J)
        say("  adaptive", q.iters, q.max_relres, rel[:3], its[:3])
        assert q.converged == 1 and q.nonfinite == 0
        assert max(rel) == pytest.approx(q.max_relres, rel=1e-12)
        assert all(0 <= r <= 1e-12 for r in rel)
        assert all(1 <= k <= q.iters for k in its)
    f = Stepper(gm, pb, opts=fixed_schedule_opts(), time_dependent_data=False, graph=True)
    for _ in range(2):
        st = f.step(stats=True)
    for q in (st.v, st.w):
        rel, its = L.member_stats(q, J)
        say("  fixed", q.iters, q.max_relres, rel[:3])
        assert q.converged == -1 and q.nonfinite == 0
        assert all(np.isfinite(r) and 0 <= r < 1e-3 for r in rel)
        assert max(rel) == pytest.approx(q.max_relres, rel=1e-12)
        assert its == [q.iters] * J
    a.close()
    f.close()
    gm.close()


def test_stability_warnings(L):
    from paper_2108_05110_amd.ensemble import Mesh, Stepper
    N, J = 8, 3
    say("warnings: alpha_j <= 0, mu <= 1/2")
    pb = wl.cavity(J=J, s=0.1, dt=0.01)
    gm = Mesh(L.MHD_MESH_UNIT_SQUARE, N)
    ok = Stepper(gm, pb, opts=L.solver_opts(L.MHD_FP64), time_dependent_data=False)
    st = ok.step(stats=True)
    assert st.warnings == 0 and st.min_alpha > 0
    ok.close()
    pb.nu = np.array([1e-3, 1e-3, 1e-1])
    pb.nu_m = np.array([1e-3, 1e-3, 1e-3])
    pb.mu = 0.4
    nub, numb = pb.nu.mean(), pb.nu_m.mean()
    alpha = nub + numb - np.abs(pb.nu - pb.nu_m) - np.abs((pb.nu - nub) + (pb.nu_m - numb))
    bad = Stepper(gm, pb, opts=L.solver_opts(L.MHD_FP64), time_dependent_data=False)
    st = bad.step(stats=True)
    say("  warnings", st.warnings, st.min_alpha, alpha)
    assert st.warnings & L.MHD_WARN_ALPHA and st.warnings & L.MHD_WARN_MU
    assert st.min_alpha == pytest.approx(alpha.min(), rel=1e-12)
    bad.close()
    gm.close()


def test_nonfinite_state_reported_under_fixed_schedule(L):
    """A NaN planted in the state (from the host) reaches the residuals of the
    fixed schedule, which looks at none while it runs: the step's statistics
    flag it and the call returns MHD_ENOCONV."""
    from paper_2108_05110_amd.ensemble import Mesh, Stepper, fixed_schedule_opts
    N, J = 16, 8
    say("non-finite detection, fixed schedule")
    pb = wl.cavity(J=J, s=0.1, dt=0.01)
    gm = Mesh(L.MHD_MESH_UNIT_SQUARE, N)
    f = Stepper(gm, pb, opts=fixed_schedule_opts(), time_dependent_data=False, graph=True)
    f.step(stats=False)
    f.V[100, 0, 3] = float("nan")
    with pytest.raises(L.MhdError) as ei:
        f.step(stats=True)
    assert ei.value.status == L.MHD_ENOCONV
    assert "non-finite" in str(ei.value)
    st = f.step(stats=True, allow_noconv=True)
    assert st.warnings & L.MHD_WARN_NONFINITE
    assert st.v.nonfinite + st.w.nonfinite > 0
    f.close()
    gm.close()


def test_later_handles_on_a_mesh_match_the_first(L):
    """A shared-matrix handle created after another one on the same mesh, and
    after the mesh's pressure Schur hierarchy was recomputed for the time step,
    must carry the hierarchy for its own (dt, nu) and solve exactly as the first:
    same iterations, bit-identical iterates.  The same holds for whole graph-
    captured steps of a second stepper started after the first was closed."""
    from paper_2108_05110_amd.ensemble import Mesh, Stepper, fixed_schedule_opts, to_dev
    N, J = 32, 8
    say("later handles: 32^2, J=8, FP64 solves and fixed-schedule steppers")
    pb = wl.cavity(J=J, s=0.1, dt=0.01, ic_amp=0.05)
    gm = Mesh(L.MHD_MESH_UNIT_SQUARE, N)
    V, W = pb.ic(gm.xy)
    c = L.Coeffs(pb.dt, pb.mu, float(pb.nu.mean()), float(pb.nu_m.mean()), 0)
    g = torch.Generator("cuda").manual_seed(3)
    b = torch.randn((gm.n, J), dtype=torch.float64, device="cuda", generator=g)
    out = []
    for k in range(3):
        A = L.mhd_ens_shared_create(gm.handle, J, 30)
        L.mhd_ens_assemble_shared(gm.handle, c, to_dev(W), J, A)
        x = torch.zeros_like(b)
        st, _ = L.mhd_ens_solve(A, b, x, J, L.solver_opts(L.MHD_FP64, rtol=1e-10))
        say(f"  handle {k}: {st.iters} iterations, relres {st.max_relres:.2e}")
        out.append((st.iters, x))
        L.mhd_ens_shared_free(A)
    for its, x in out[1:]:
        assert its == out[0][0]
        assert torch.equal(x, out[0][1])
    states = []
    for k in range(2):
        s = Stepper(gm, pb, opts=fixed_schedule_opts(), time_dependent_data=False, graph=True)
        for _ in range(3):
            st = s.step(stats=True)
        say(f"  stepper {k}: final relres {st.v.max_relres:.2e} {st.w.max_relres:.2e}")
        states.append((s.V.clone(), s.W.clone()))
        s.close()
    assert torch.equal(states[0][0], states[1][0]) and torch.equal(states[0][1], states[1][1])
    gm.close()


def test_gram_schmidt_variants(L):
    """The three Gram-Schmidt variants of the FP32 inner solve (one pass with
    the norm taken directly, two passes, one fused pass with the norm from the
    dot products) reach the FP64 solution on one handle, in the order 2, 1, 3,
    so that a single direct pass runs after two-pass solves have filled the
    second pass's coefficients (which it must not read).  Only the fused pass
    may report norm clamps; restart 12 is past the cycle length the fused pass
    is validated for, so only its count is checked there."""
    from paper_2108_05110_amd.ensemble import Mesh, to_dev
    N, J = 32, 16
    say("Gram-Schmidt variants: 32^2, J=16, FP32 inner solves")
    pb = wl.cavity(J=J, s=0.1, dt=0.01, ic_amp=0.05)
    gm = Mesh(L.MHD_MESH_UNIT_SQUARE, N)
    V, W = pb.ic(gm.xy)
    c = L.Coeffs(pb.dt, pb.mu, float(pb.nu.mean()), float(pb.nu_m.mean()), 0)
    g = torch.Generator("cuda").manual_seed(11)
    b = torch.randn((gm.n, J), dtype=torch.float64, device="cuda", generator=g)
    A = L.mhd_ens_shared_create(gm.handle, J, 12)
    L.mhd_ens_assemble_shared(gm.handle, c, to_dev(W), J, A)
    ref = torch.zeros_like(b)
    L.mhd_ens_solve(A, b, ref, J, L.solver_opts(L.MHD_FP64, rtol=1e-12, restart=12))
    rel = lambda x: float(torch.linalg.norm(x - ref) / torch.linalg.norm(ref))
    for cgs in (2, 1, 3):
        for restart, cycles in ((6, 0), (6, 3), (12, 3)):
            x = torch.zeros_like(b)
            opts = L.solver_opts(L.MHD_FP32_IR, restart=restart, fixed_cycles=cycles, cgs_passes=cgs, rtol=1e-10)
            st, _ = L.mhd_ens_solve(A, b, x, J, opts, allow_noconv=True)
            e = rel(x)
            say(f"  cgs {cgs} restart {restart} cycles {cycles}: error {e:.2e}, iterations {st.iters}, "
                f"norm clamps {st.norm_clamps}")
            if cgs != 3:
                assert st.norm_clamps == 0 or (cycles > 0 and st.norm_clamps == -1)
            if cgs != 3 or restart <= 8:
                assert e <= (1e-8 if cycles == 0 else 1e-5), (cgs, restart, cycles, e)
    L.mhd_ens_shared_free(A)
    gm.close()


def test_converged_members_are_compacted_out(L):
    """Adaptive per-member solver: members whose iterate already meets rtol drop
    out and the others continue as a compacted block.  Half the members start
    from their converged solution: they are left bit for bit as they were, the
    statistics report the compacted block, and the others reach the same
    solution as with every column kept (keep_converged = 1)."""
    from paper_2108_05110_amd.ensemble import Mesh, to_dev
    N, J = 16, 8
    say("compaction of converged members: 16^2, J=8, FP64 and FP32+IR adaptive")
    pb = wl.cavity(J=J, s=0.1, dt=0.01, ic_amp=0.05)
    gm = Mesh(L.MHD_MESH_UNIT_SQUARE, N)
    V, W = pb.ic(gm.xy)
    c = L.Coeffs(pb.dt, pb.mu, float(pb.nu.mean()), float(pb.nu_m.mean()), 0)
    g = torch.Generator("cuda").manual_seed(21)
    b = torch.randn((gm.n, J), dtype=torch.float64, device="cuda", generator=g)
    A = L.mhd_ens_shared_create(gm.handle, J, 30)
    L.mhd_ens_assemble_shared(gm.handle, c, to_dev(W), J, A)
    ref = torch.zeros_like(b)
    st, _ = L.mhd_ens_solve(A, b, ref, J, L.solver_opts(L.MHD_FP64, rtol=1e-13, keep_converged=1))
    assert st.compacted == 0
    for prec, rtol in ((L.MHD_FP64, 1e-11), (L.MHD_FP32_IR, 1e-10)):
        out = {}
        for keep in (0, 1):
            x = torch.zeros_like(b)
            x[:, :4] = ref[:, :4]
            x0 = x.clone()
            st, _ = L.mhd_ens_solve(A, b, x, J, L.solver_opts(prec, rtol=rtol, keep_converged=keep))
            rel, its = L.member_stats(st, J)
            say(f"  precision {prec} keep {keep}: iterations {st.iters}, compacted {st.compacted}, "
                f"max relres {st.max_relres:.2e}, member iterations {its}")
            assert st.converged == 1 and st.max_relres <= rtol
            out[keep] = (x, st)
            if keep == 0:
                assert st.compacted == 4
                assert torch.equal(x[:, :4], x0[:, :4])
            else:
                assert st.compacted == 0
        err = float(torch.linalg.norm(out[0][0] - ref) / torch.linalg.norm(ref))
        assert err <= 1e3 * rtol, err
    L.mhd_ens_shared_free(A)
    gm.close()


def test_extra_post_smoothing_option(L):
    """mg_post adds damped Jacobi post-smoothing sweeps on the finest pressure
    level: a stronger Schur part, the same solution, no more iterations."""
    from paper_2108_05110_amd.ensemble import Mesh, to_dev
    N, J = 64, 16   # at least two pressure levels (32^2 has only the dense one)
    say("extra post-smoothing: 64^2, J=16, FP64 adaptive")
    pb = wl.cavity(J=J, s=0.1, dt=0.01, ic_amp=0.05)
    gm = Mesh(L.MHD_MESH_UNIT_SQUARE, N)
    V, W = pb.ic(gm.xy)
    c = L.Coeffs(pb.dt, pb.mu, float(pb.nu.mean()), float(pb.nu_m.mean()), 0)
    g = torch.Generator("cuda").manual_seed(13)
    b = torch.randn((gm.n, J), dtype=torch.float64, device="cuda", generator=g)
    A = L.mhd_ens_shared_create(gm.handle, J, 30)
    L.mhd_ens_assemble_shared(gm.handle, c, to_dev(W), J, A)
    xs, its = [], []
    for post in (0, 3):
        x = torch.zeros_like(b)
        st, _ = L.mhd_ens_solve(A, b, x, J, L.solver_opts(L.MHD_FP64, rtol=1e-11, mg_post=post))
        say(f"  mg_post {post}: {st.iters} iterations, relres {st.max_relres:.2e}")
        assert st.converged == 1
        xs.append(x)
        its.append(st.iters)
    assert its[1] <= its[0]
    assert not torch.equal(xs[1], xs[0])      # the option reached the multigrid
    assert float(torch.linalg.norm(xs[1] - xs[0]) / torch.linalg.norm(xs[0])) <= 1e-9
    L.mhd_ens_shared_free(A)
    gm.close()


def test_kernel_timer_selects_the_operator(L):
    """mhd_ens_timer_op: the timer counts the SpMM launches of a solve (one per
    inner iteration) or the velocity Jacobi sweeps that update the previous
    iterate (sweeps - 2 per preconditioner application with the paired-row
    plans, sweeps - 1 otherwise); other operators are refused."""
    from paper_2108_05110_amd.ensemble import Mesh, to_dev
    N, J, sweeps = 32, 16, 7
    say("kernel timer: SpMM and Jacobi sweep launches of a fixed-schedule FP32 solve")
    pb = wl.cavity(J=J, s=0.1, dt=0.01, ic_amp=0.05)
    gm = Mesh(L.MHD_MESH_UNIT_SQUARE, N)
    V, W = pb.ic(gm.xy)
    c = L.Coeffs(pb.dt, pb.mu, float(pb.nu.mean()), float(pb.nu_m.mean()), 0)
    b = torch.ones((gm.n, J), dtype=torch.float64, device="cuda")
    A = L.mhd_ens_shared_create(gm.handle, J, 6)
    L.mhd_ens_assemble_shared(gm.handle, c, to_dev(W), J, A)
    opts = L.solver_opts(L.MHD_FP32_IR, restart=6, fixed_cycles=2, jacobi_sweeps=sweeps)
    counts = {}
    for op in (L.TUNE_SADDLE, L.TUNE_JACOBI):
        L.mhd_ens_timer_op(op)
        L.mhd_ens_timer_enable(True)
        x = torch.zeros_like(b)
        st, _ = L.mhd_ens_solve(A, b, x, J, opts)
        ms, launches, _, _ = L.mhd_ens_timer_read()
        L.mhd_ens_timer_enable(False)
        counts[op] = (launches, st.iters, ms)
        say(f"  op {op}: {launches} launches, {ms:.3f} ms, {st.iters} iterations")
    L.mhd_ens_timer_op(L.TUNE_SADDLE)
    launches, iters, ms = counts[L.TUNE_SADDLE]
    assert launches == iters and ms > 0
    launches, iters, ms = counts[L.TUNE_JACOBI]
    assert launches in ((sweeps - 2) * iters, (sweeps - 1) * iters) and ms > 0
    with pytest.raises(L.MhdError):
        L.mhd_ens_timer_op(L.TUNE_RESIDUAL)
    L.mhd_ens_shared_free(A)
    gm.close()
