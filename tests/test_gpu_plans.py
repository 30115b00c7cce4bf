"""GPU: every launch plan of the node-row operators (saddle-point SpMM, FP64
residual, velocity-block Jacobi sweeps) gives the same result, and the
autotuner's report is consistent.

The plans differ in how rows are mapped to lanes and workgroups (members per
lane per load, units per wavefront, LDS-staged row tiles), not in arithmetic,
so the planned kernels must agree exactly with each other and, within FP
rounding, with the operator rebuilt on the host from the device CSR arrays.
The mesh (12 x 12 cells: 625 P2 + 169 P1 units) leaves a ragged last
workgroup for every units-per-wavefront choice and cut tiles at its edges.
"""
import sys

import numpy as np
import pytest

import workloads as wl
from tests.maps import csr_from_view

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

N = 12


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


def candidates(J, word):
    """(vec, group, deep, tile, waves): generic, gather, pipelined and LDS-staged plans."""
    out = [(0, 0, 0, 0, 4)]
    vecs = [v for v in ((4, 2, 1) if word == 4 else (2, 1)) if J % (32 * v) == 0]
    for v in vecs:
        out += [(v, g, 0, 0, 4) for g in (0, 1, 2, 4)]
        out += [(v, g, 1, 0, 4) for g in (1, 2, 4, 8)]
    if J % (256 // word) == 0:
        out += [(16 // word, g, 2, 0, 4) for g in (4, 8)]
    for v in (2, 1):
        if J % (32 * v) == 0 and (v == 1 or word == 4):
            out += [(v, 0, dp, t, w) for dp in (0, 3) for t in (8, 12, 16) for w in (4, 8)]
    return out


def ell_candidates(J, word):
    """Row-per-lane tiles (FP32): tile code tx * 100 + ty (+ 10000: 8 members per workgroup)."""
    if word != 4 or J % 8:
        return []
    codes = (11616, 13208, 11608) + ((1616, 3208, 1608) if J % 16 == 0 else ())
    return [(4, 0, 6, code, 0) for code in codes]


def set_plan(L, A, J, precision, op, plan):
    """False if the device cannot hold this LDS tile."""
    try:
        L.mhd_ens_set_plan(A, J, precision, op, *plan)
    except RuntimeError as e:
        if "LDS" in str(e):
            return False
        raise
    return True


def shared(L, J, seed=0):
    from paper_2108_05110_amd.ensemble import Mesh, to_dev
    pb = wl.cavity(J=J, s=0.1, dt=0.01)
    gm = Mesh(L.MHD_MESH_UNIT_SQUARE, N)
    V, W = pb.ic(gm.xy)
    W = W + 0.05 * np.random.default_rng(seed).standard_normal(W.shape)
    A = L.mhd_ens_shared_create(gm.handle, J, 30)
    c = L.Coeffs(pb.dt, pb.mu, float(pb.nu.mean()), float(pb.nu_m.mean()), 0)
    L.mhd_ens_assemble_shared(gm.handle, c, to_dev(W), J, A)
    return pb, gm, A, V, W


@pytest.mark.parametrize("precision,J", [(1, 64), (1, 128), (1, 32), (0, 64), (0, 32)])
def test_every_spmm_plan(L, precision, J):
    say("spmm plans", precision, J)
    pb, gm, A, _, _ = shared(L, J)
    S = csr_from_view(torch, L.mhd_ens_shared_csr(A))
    word = 4 if precision == 1 else 8
    dt = torch.float32 if word == 4 else torch.float64
    x = torch.from_numpy(np.random.default_rng(1).standard_normal((gm.n, J))).to("cuda", dt)
    ref = S @ x.double().cpu().numpy()
    tol = 2e-6 if word == 4 else 1e-14
    planned = {}
    for plan in candidates(J, word) + ell_candidates(J, word):
        if not set_plan(L, A, J, precision, L.TUNE_SADDLE, plan):
            say("  plan", plan, "does not fit in LDS")
            continue
        y = torch.full((gm.n, J), float("nan"), dtype=dt, device="cuda")
        L.mhd_ens_spmm(A, x, y, J, precision)
        torch.cuda.synchronize()
        yh = y.double().cpu().numpy()
        err = np.abs(yh - ref).max() / np.abs(ref).max()
        say("  plan", plan, "err", err)
        assert err <= tol, (plan, err)
        if plan[0]:
            planned[plan] = y
    base = next(iter(planned.values()))
    for k, y in planned.items():
        assert torch.equal(y, base), k
    L.mhd_ens_shared_free(A)
    gm.close()


@pytest.mark.parametrize("precision", [1, 0])
def test_every_solver_plan_same_solution(L, precision):
    """Jacobi (first and later sweeps) and FP64-residual plans inside a full
    adaptive solve: identical iterates, so identical solutions and counts."""
    J = 64
    say("solver plans", precision)
    pb, gm, A, V, W = shared(L, J, seed=2)
    word = 4 if precision == 1 else 8
    rng = np.random.default_rng(3)
    b = torch.from_numpy(rng.standard_normal((gm.n, J))).cuda()
    results = {}
    for plan in candidates(J, word) + ell_candidates(J, word):
        if plan[0] == 0:
            continue
        if plan[2] == 6:   # FP32 plans: the FP64 residual keeps a gather plan
            ok = all([set_plan(L, A, J, precision, op, plan)
                      for op in (L.TUNE_SADDLE, L.TUNE_JACOBI_FIRST, L.TUNE_JACOBI)])
            ok = set_plan(L, A, J, precision, L.TUNE_RESIDUAL, (1, 1, 0, 0, 4)) and ok
        else:
            ok = all([set_plan(L, A, J, precision, op, plan)
                      for op in (L.TUNE_SADDLE, L.TUNE_JACOBI_FIRST, L.TUNE_JACOBI)])
            # FP64 residual: LDS tiles take vec 1, paired rows need J a multiple of 32
            resid = (1,) + plan[1:] if plan[3] else (min(plan[0], 2),) + plan[1:]
            ok = set_plan(L, A, J, precision, L.TUNE_RESIDUAL, resid) and ok
        if not ok:
            say("  plan", plan, "does not fit in LDS")
            continue
        x = torch.zeros((gm.n, J), dtype=torch.float64, device="cuda")
        st, _ = L.mhd_ens_solve(A, b, x, J, L.solver_opts(precision, rtol=1e-10))
        say("  plan", plan, "iters", st.iters, "relres", st.max_relres)
        assert st.converged == 1
        results[plan] = (x, st.iters)
    x0, it0 = next(iter(results.values()))
    for k, (x, it) in results.items():
        assert it == it0, k
        assert torch.equal(x, x0), k
    L.mhd_ens_shared_free(A)
    gm.close()


def test_unaligned_solution_vector(L):
    """x at an 8-byte offset (not 16-byte aligned): the FP64 residual takes one
    member per lane and the FP32 inner solve adds its correction to x in a pass
    of its own instead of inside the last basis combination; the iterates are
    the same as with an aligned x."""
    J = 64
    pb, gm, A, V, W = shared(L, J, seed=4)
    rng = np.random.default_rng(5)
    b = torch.from_numpy(rng.standard_normal((gm.n, J))).cuda()
    x0 = torch.zeros((gm.n, J), dtype=torch.float64, device="cuda")
    st0, _ = L.mhd_ens_solve(A, b, x0, J, L.solver_opts(1, rtol=1e-10))
    big = torch.zeros(gm.n * J + 2, dtype=torch.float64, device="cuda")
    x1 = big[1:1 + gm.n * J].view(gm.n, J)
    assert x1.data_ptr() % 16 == 8
    st1, _ = L.mhd_ens_solve(A, b, x1, J, L.solver_opts(1, rtol=1e-10))
    say("  aligned iters", st0.iters, "cycles", st0.cycles, "unaligned iters", st1.iters, "cycles", st1.cycles)
    assert st0.converged == 1 and st1.converged == 1
    assert (st1.iters, st1.cycles) == (st0.iters, st0.cycles)
    assert torch.equal(x1, x0)
    L.mhd_ens_shared_free(A)
    gm.close()


def test_autotune_report(L):
    J = 64
    pb, gm, A, _, _ = shared(L, J)
    rep = L.mhd_ens_autotune(A, J, 1)
    ops = {}
    for e in rep:
        assert (e["us"] > 0 or (e["us"] == -1 and not e["chosen"])) and e["J"] == J
        ops.setdefault((e["op"], e["word"]), []).append(e)
    assert set(ops) == {("saddle", 4), ("jacobi_first", 4), ("jacobi", 4), ("residual", 8)}
    for key, es in ops.items():
        chosen = [e for e in es if e["chosen"]]
        assert len(chosen) == 1, key
        assert chosen[0]["us"] == min(e["us"] for e in es if e["us"] > 0), key
        say(key, [(e["vec"], e["group"], e["deep"], e["tile"], e["waves"], round(e["us"], 2)) for e in es])
    # a J with no vector shape tunes nothing and solves with the generic kernels
    assert L.mhd_ens_autotune(A, 5, 1) == []
    L.mhd_ens_shared_free(A)
    gm.close()


def test_row_tile_values_follow_assembly(L):
    """The row-per-lane SpMM keeps its own copy of the A values in tile order:
    a new assembly of the same handle must reach it."""
    from paper_2108_05110_amd.ensemble import to_dev
    J = 32
    pb, gm, A, V, W = shared(L, J, seed=4)
    assert set_plan(L, A, J, 1, L.TUNE_SADDLE, (4, 0, 6, 1608, 0))
    x = torch.from_numpy(np.random.default_rng(5).standard_normal((gm.n, J))).to("cuda", torch.float32)
    for step in range(2):
        if step:
            W2 = W + 0.3 * np.random.default_rng(6).standard_normal(W.shape)
            c = L.Coeffs(pb.dt, pb.mu, float(pb.nu.mean()), float(pb.nu_m.mean()), 0)
            L.mhd_ens_assemble_shared(gm.handle, c, to_dev(W2), J, A)
        S = csr_from_view(torch, L.mhd_ens_shared_csr(A))
        y = torch.full((gm.n, J), float("nan"), dtype=torch.float32, device="cuda")
        L.mhd_ens_spmm(A, x, y, J, 1)
        torch.cuda.synchronize()
        ref = S @ x.double().cpu().numpy()
        err = np.abs(y.double().cpu().numpy() - ref).max() / np.abs(ref).max()
        say("  assembly", step, "err", err)
        assert err <= 2e-6
    L.mhd_ens_shared_free(A)
    gm.close()


@pytest.mark.parametrize("precision", [1, 0])
def test_fused_multigrid_matches_sweeps(L, precision):
    """The V-cycle levels as their two fused sparse operators against the same
    cycle run sweep by sweep: the same solution (to the solve tolerance) and
    iteration counts within rounding effects, and one fixed-schedule FP32 cycle
    agreeing to FP32 rounding."""
    from paper_2108_05110_amd.ensemble import Mesh, to_dev
    N, J = 64, 64
    say("fused multigrid", precision)
    pb = wl.cavity(J=J, s=0.3, dt=0.01, ic_amp=0.05)
    gm = Mesh(L.MHD_MESH_UNIT_SQUARE, N)
    V, W = pb.ic(gm.xy)
    A = L.mhd_ens_shared_create(gm.handle, J, 30)
    c = L.Coeffs(pb.dt, pb.mu, float(pb.nu.mean()), float(pb.nu_m.mean()), 0)
    L.mhd_ens_assemble_shared(gm.handle, c, to_dev(W), J, A)
    L.mhd_ens_prepare(A, J, precision)
    b = torch.randn((gm.n, J), dtype=torch.float64, device="cuda", generator=torch.Generator("cuda").manual_seed(3))
    out = {}
    for unf in (0, 1):
        x = torch.zeros_like(b)
        st, _ = L.mhd_ens_solve(A, b, x, J, L.solver_opts(precision, rtol=1e-10, mg_unfused=unf))
        out[unf] = (x, st.iters)
        say("  unfused" if unf else "  fused", st.iters, st.max_relres)
    rel = float(torch.linalg.norm(out[0][0] - out[1][0]) / torch.linalg.norm(out[1][0]))
    assert rel < 1e-8, rel
    # FP32 inner cycles stop at a residual reduction, so rounding may move a
    # cycle's end by a few iterations; a wrong operator would change the rate
    assert abs(out[0][1] - out[1][1]) <= max(2, out[1][1] // 10), (out[0][1], out[1][1])
    if precision == 1:
        xs = []
        for unf in (0, 1):
            x = torch.zeros_like(b)
            L.mhd_ens_solve(A, b, x, J, L.solver_opts(1, restart=6, fixed_cycles=1, jacobi_sweeps=5,
                                                        mg_unfused=unf))
            xs.append(x)
        d = float(torch.linalg.norm(xs[0] - xs[1]) / torch.linalg.norm(xs[1]))
        say("  one fixed cycle: fused vs sweeps", d)
        assert d < 1e-3, d
    L.mhd_ens_shared_free(A)
    gm.close()
