"""GPU parity at full size: the kernels the throughput figures run, against
the FP64 CPU oracle (Algorithm 1, per-member sparse LU).

* The 128 x 128 cavity with J = 64 members on the graph-captured fixed
  schedule (FP32 inner GMRES, FP64 refinement, tuned node-row plans): after
  three steps of flow development on the GPU, one more step is compared with
  the oracle's step from the same GPU state for members 0, 31 and 63 (the
  means and eddy-viscosity maxima still over all 64 members).
* The step channel at h = 1/16 with J = 64, FP32 inner solves: one step from
  a GPU state on a member subset, adaptive refinement and the fixed schedule.
* A fixed-schedule FP32 solve with J = 16 (the matrix-core coarse-level
  solve) against the same solve of its first 15 members (vector coarse
  solve) and against the oracle, so that a defect in the matrix-core product
  shows in the iterate instead of being refined away.

Bar (FP32 inner solves with FP64 refinement): relative L2 error in the P2
mass norm 1e-6 per step from identical inputs.
"""
import sys
import time

import numpy as np
import pytest

import workloads as wl
from oracle import mesh as om, scheme
from tests.maps import mass_rel_err, node_map, p1_map, unknown_perm

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


def oracle_step_subset(ens, pm2, Vg, Wg, t_next, members):
    """Oracle step from a GPU state (GPU numbering) for a member subset; returns
    the subset's V, W at t_next in the oracle numbering."""
    V = np.empty_like(Vg)
    W = np.empty_like(Wg)
    V[pm2] = Vg
    W[pm2] = Wg
    t0 = time.time()
    V1, W1, _, _ = ens.step(V, W, t_next, shared_lu=True, members=members, ordering="ND",
                            log=lambda msg: say("  " + msg))
    say(f"  oracle step ({len(members)} members) {time.time() - t0:.1f} s")
    return V1, W1


def gpu_subset(pm2, Zg, members):
    Z = np.empty((len(pm2), 2, len(members)))
    Z[pm2] = Zg[:, :, members]
    return Z


@pytest.mark.timeout(600)
def test_headline_cavity128_J64_graph_step_vs_oracle(L):
    from paper_2108_05110_amd.ensemble import Mesh, Stepper, fixed_schedule_opts
    N, J = 128, 64
    members = [0, 31, 63]
    say("headline: cavity 128^2, J=64, FP32+IR fixed schedule, graph step")
    pb = wl.cavity(J=J, s=0.1, dt=0.01)
    gm = Mesh(L.MHD_MESH_UNIT_SQUARE, N)
    opts = fixed_schedule_opts()
    stp = Stepper(gm, pb, opts=opts, time_dependent_data=False, graph=True)
    for _ in range(3):
        stp.step(stats=False)
    Vn, Wn = stp.V.cpu().numpy(), stp.W.cpu().numpy()
    st = stp.step(stats=True)
    say("  krylov iterations", st.v.iters, st.w.iters)
    V1g, W1g = stp.V.cpu().numpy(), stp.W.cpu().numpy()
    # which SpMM plan the captured step used: the process-wide tuner table
    A = L.mhd_ens_shared_create(gm.handle, J, 6)
    from paper_2108_05110_amd.ensemble import to_dev
    c = L.Coeffs(pb.dt, pb.mu, float(pb.nu.mean()), float(pb.nu_m.mean()), 0)
    L.mhd_ens_assemble_shared(gm.handle, c, to_dev(Wn), J, A)
    rep = L.mhd_ens_plan(A, J, L.MHD_FP32_IR)
    L.mhd_ens_shared_free(A)
    say("  plans", rep)
    assert rep["saddle"]["deep"] in (2, 6), rep          # paired-row or row-per-lane SpMM
    assert rep["jacobi"]["vec"] > 0, rep                  # a specialised Jacobi plan, not the generic one
    stp.close()
    om_ = om.unit_square(N)
    ens = scheme.Ensemble(om_, pb)
    pm2 = node_map(gm.xy, om_.xy, 1.0 / N)
    V1o, W1o = oracle_step_subset(ens, pm2, Vn, Wn, 4 * pb.dt, members)
    ev = mass_rel_err(ens, gpu_subset(pm2, V1g, members), V1o)
    ew = mass_rel_err(ens, gpu_subset(pm2, W1g, members), W1o)
    say(f"  rel. L2 (mass) error v {ev:.3e} w {ew:.3e}")
    assert max(ev, ew) <= 1e-6, (ev, ew)
    gm.close()


@pytest.mark.timeout(600)
def test_step_channel_h16_J64_step_vs_oracle(L):
    """Two adaptive FP32+IR steps on the GPU, then from that state one step with
    the adaptive solver and one with the graph-captured fixed schedule, both
    against one oracle step of members 0 and 63."""
    from paper_2108_05110_amd.ensemble import Mesh, Stepper, fixed_schedule_opts
    m, J = 16, 64
    members = [0, 63]
    say("step channel h=1/16, J=64, FP32+IR adaptive and fixed schedule")
    pb = wl.step_channel(J=J, delta=1e-2, s=0.01, dt=0.02)
    gm = Mesh(L.MHD_MESH_STEP_CHANNEL, m, 1)
    ada = Stepper(gm, pb, opts=L.solver_opts(L.MHD_FP32_IR), time_dependent_data=False)
    fix = Stepper(gm, pb, opts=fixed_schedule_opts(), time_dependent_data=False, graph=True)
    for _ in range(2):
        ada.step(stats=False)
    Vn, Wn = ada.V.cpu().numpy(), ada.W.cpu().numpy()
    for a, b in ((ada.V, fix.V), (ada.W, fix.W), (ada.Q, fix.Q), (ada.R, fix.R)):
        b.copy_(a)
    fix.n = ada.n
    out = {}
    for name, stp in (("adaptive", ada), ("fixed", fix)):
        st = stp.step(stats=True)
        say(f"  {name}: krylov iterations", st.v.iters, st.w.iters, "relres", st.v.max_relres, st.w.max_relres)
        out[name] = (stp.V.cpu().numpy(), stp.W.cpu().numpy())
        stp.close()
    om_ = om.step_channel(m)
    ens = scheme.Ensemble(om_, pb)
    pm2 = node_map(gm.xy, om_.xy, 1.0 / m)
    V1o, W1o = oracle_step_subset(ens, pm2, Vn, Wn, 3 * pb.dt, members)
    errs = {}
    for name, (V1g, W1g) in out.items():
        ev = mass_rel_err(ens, gpu_subset(pm2, V1g, members), V1o)
        ew = mass_rel_err(ens, gpu_subset(pm2, W1g, members), W1o)
        errs[name] = max(ev, ew)
        say(f"  {name}: rel. L2 (mass) error v {ev:.3e} w {ew:.3e}")
    assert max(errs.values()) <= 1e-6, errs
    gm.close()


def test_fixed_schedule_fp32_solve_matrix_core_coarse(L):
    """J = 16 takes the matrix-core coarse solve, J = 15 the vector one; one
    fixed refinement cycle of 6 FP32 iterations leaves the preconditioner's
    imprint on the iterate."""
    from paper_2108_05110_amd.ensemble import Mesh, to_dev
    N, J = 32, 16
    say("fixed-schedule FP32 solve, J=16 vs J=15 vs oracle")
    pb = wl.cavity(J=J, s=0.3, dt=0.01, ic_amp=0.05)
    gm = Mesh(L.MHD_MESH_UNIT_SQUARE, N)
    om_ = om.unit_square(N)
    ens = scheme.Ensemble(om_, pb)
    pm2 = node_map(gm.xy, om_.xy, 1.0 / N)
    pm1 = p1_map(gm.xy, om_, 1.0 / N)
    perm = unknown_perm(pm2, pm1, om_.nP2)
    V, W = pb.ic(om_.xy)
    r = np.random.default_rng(7)
    V = V + 0.05 * r.standard_normal(V.shape)
    W = W + 0.05 * r.standard_normal(W.shape)
    Sv = ens.shared_matrix(W)
    Gv, _ = pb.bc(pb.dt, om_.xy)
    F1, _ = pb.forcing(pb.dt, om_.xy)
    b = ens.rhs(V, W, F1, Gv)
    x_orc = ens.solve_members(Sv, b, shared_lu=True)
    c = L.Coeffs(pb.dt, pb.mu, float(pb.nu.mean()), float(pb.nu_m.mean()), 0)
    opts = L.solver_opts(L.MHD_FP32_IR, restart=6, fixed_cycles=1, jacobi_sweeps=5)
    bg = b[perm]
    xs = {}
    for Jr in (16, 15):
        A = L.mhd_ens_shared_create(gm.handle, 16, 6)
        L.mhd_ens_assemble_shared(gm.handle, c, to_dev(W[pm2]), J, A)    # matrix from all 16 members
        x = torch.zeros((gm.n, Jr), dtype=torch.float64, device="cuda")
        L.mhd_ens_solve(A, to_dev(bg[:, :Jr]), x, Jr, opts)
        xo = np.zeros((gm.n, Jr))
        xo[perm] = x.cpu().numpy()
        xs[Jr] = xo
        L.mhd_ens_shared_free(A)
    rel = lambda a, b_: np.linalg.norm(a - b_) / np.linalg.norm(b_)
    e16, e15 = rel(xs[16], x_orc), rel(xs[15], x_orc[:, :15])
    agree = rel(xs[16][:, :15], xs[15])
    say(f"  error vs oracle: J=16 {e16:.3e}, J=15 {e15:.3e}; J=16 vs J=15 {agree:.3e}")
    # one cycle of 6 iterations: the solve is unfinished.  The two coarse solves
    # sum in different orders, and GMRES carries that FP32 rounding into the
    # iterate (observed 2.8e-5 relative, 6e-4 of the iterate's own error); a
    # defective product changes the preconditioner itself and so moves the
    # iterate by the order of its error
    assert agree <= 1e-2 * e15, agree
    assert e16 <= 1.05 * e15 + 1e-7
    assert e16 < 0.1
    gm.close()


@pytest.mark.timeout(900)
def test_headline_four_steps_vs_oracle_trajectory(L):
    """The headline configuration over several steps: 128 x 128 cavity, J = 64,
    the graph-captured fixed schedule from the initial state for 4 steps, against
    the oracle's own 4-step trajectory of all 64 members (shared sparse LU per
    subproblem and step, nested-dissection order); members 0, 31 and 63 compared
    after every second step, bar 1e-6 in the P2 mass norm (errors of every step
    accumulated)."""
    from paper_2108_05110_amd.ensemble import Mesh, Stepper, fixed_schedule_opts
    N, J, nsteps = 128, 64, 4
    members = [0, 31, 63]
    say("headline trajectory: cavity 128^2, J=64, 4 graph steps vs 4 oracle steps")
    pb = wl.cavity(J=J, s=0.1, dt=0.01)
    gm = Mesh(L.MHD_MESH_UNIT_SQUARE, N)
    stp = Stepper(gm, pb, opts=fixed_schedule_opts(), time_dependent_data=False, graph=True)
    om_ = om.unit_square(N)
    ens = scheme.Ensemble(om_, pb)
    pm2 = node_map(gm.xy, om_.xy, 1.0 / N)
    V, W = pb.ic(om_.xy)
    for n in range(1, nsteps + 1):
        stp.step(stats=False)
        t0 = time.time()
        V, W, _, _ = ens.step(V, W, n * pb.dt, shared_lu=True, ordering="ND")
        if n % 2 == 0:
            Vg, Wg = stp.V.cpu().numpy(), stp.W.cpu().numpy()
            ev = mass_rel_err(ens, gpu_subset(pm2, Vg, members), V[:, :, members])
            ew = mass_rel_err(ens, gpu_subset(pm2, Wg, members), W[:, :, members])
            say(f"  step {n}: rel. L2 (mass) error v {ev:.3e} w {ew:.3e} (oracle step {time.time() - t0:.1f} s)")
            assert max(ev, ew) <= 1e-6, (n, ev, ew)
        else:
            say(f"  step {n}: oracle step {time.time() - t0:.1f} s")
    stp.close()
    gm.close()
