#!/usr/bin/env python3
"""Throughput of the ensemble MHD time step on one MI355X.

A step is one pass of Algorithm 1 (paper, Section 3) for every member: the
ensemble statistics, both shared saddle-point matrices, both batched
right-hand sides, both batched solves (FP32 inner Krylov, FP64 refinement),
state update and pressure normalisation -- one mhd_ens_step call.  Workload:
lid-driven cavity on the unit square, 128x128 cells, Taylor-Hood P2-P1,
J = 64 members, s = 0.1, dt = 0.01, mean Re = 1000 with +-10 % member
viscosities (synthetic, seeded).  Inputs are resident in device memory before
the timed region.

The timed step is the HIP graph of one step with a fixed solver schedule
(default 2 refinement cycles of 6 right-preconditioned GMRES iterations, 7
velocity Jacobi sweeps damped by 0.6, two V-cycles for the Schur part); its
error against FP64 solves is reported after one step and after 8 steps, and
its final residual along a 200-step trajectory.  The node-row kernels are chosen by the library's autotuner
first; the chosen plans are part of the output.

Reported beside it on the same GPU: the J-separate form (the same shared
matrices and schedule, each member solved by its own single-column solve,
also graph-captured), the roofline of the saddle-point SpMM (algorithmic bytes
per launch over the launch time from HIP events recorded around every launch
of an eager pass of the same schedule), and the FP64 CPU oracle timed on a
bounded sample on the host.

Other workloads: --workload adjoint (gradients of the ensemble-mean energy
through 50 steps with checkpointing), --workload large (a 512x512 ensemble
of 128 members and four 128x128 ensembles of 16 in one graph launch) and
--workload sv (the cavity ensemble with Scott-Vogelius elements on the
barycentric refinement of a 64x64 mesh) and --workload channel (the step
channel at h = 1/16 with 64 members).
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
T_START = time.perf_counter()


def log(msg):
    """Progress line on stderr (the JSON result is the only stdout line)."""
    print(f"[bench {time.perf_counter() - T_START:7.1f} s] {msg}", file=sys.stderr, flush=True)


def spmm_bytes(info, J, word):
    """Algorithmic bytes of one saddle-point SpMM y = S x on an (n, J) block:
    compact operator (A shared by both velocity components, B and B^T with two
    values per entry, pressure diagonal) read once, x read once, y written once."""
    nP2, nP1 = info.nP2, info.nP1
    nnzA, nnzB = info.nnz_A, info.nnz_B
    idx = 4
    matrix = ((nP2 + 1) * idx + nnzA * (idx + word)            # A
              + (nP2 + 1) * idx + nnzB * (idx + 2 * word)      # B^T
              + (nP1 + 1) * idx + nnzB * (idx + 2 * word)      # B
              + nP1 * word)                                     # pressure diagonal
    return matrix + 2 * info.n * J * word


def spmm_bytes_csr(info, J, word):
    """Algorithmic bytes of one SpMM with the full saddle-point CSR (the count
    the throughput targets are stated in): value + int32 column per nonzero,
    row pointers, x read once and y written once."""
    return (word + 4) * info.nnz + 4 * (info.n + 1) + 2 * word * info.n * J


def velo_sweep_bytes(info, J, word):
    """Algorithmic bytes of one velocity Jacobi sweep z' = z + w D^-1 (t - A z)
    on both components: the scalar P2 block A as CSR (value + int32 column per
    nonzero, row pointers), D^-1, and t and z read once and z' written once."""
    return (word + 4) * info.nnz_A + 4 * (info.nP2 + 1) + word * info.nP2 + 3 * 2 * word * info.nP2 * J


def jacobi_roofline(info, J, word, ms, launches, plan):
    """Roofline of the velocity Jacobi sweep (the largest share of the step's
    kernel time) from the HIP events of its launches in an eager pass."""
    if not launches:
        return None
    avg = ms / 1e3 / launches
    b = velo_sweep_bytes(info, J, word)
    return {"bound": "hbm", "kernel": f"velocity Jacobi sweep ({saddle_kernel_name(plan).replace('saddle', 'velo')})",
            "achieved": b / avg / 1e9, "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": b / avg / 1e9 / HBM_PEAK_GBS, "bytes_per_launch": b, "avg_launch_us": avg * 1e6,
            "launches": launches}


def source_hash():
    """Hash of the code that decides the SpMM's memory traffic: the row-per-lane
    (sliced-ELL) kernels of solve.hip and the host code that lays out their
    tiles.  A change anywhere else leaves recorded counter values valid."""
    h = hashlib.sha256()
    with open(os.path.join(ROOT, "paper_2108_05110_amd", "csrc", "solve.hip"), "rb") as f:
        src = f.read()
    begin = src.index(b"// ------------------------------------------------------------------ row-per-lane tiles")
    end = src.index(b"// ------------------------------------------------------------------", begin + 10)
    h.update(src[begin:end])
    with open(os.path.join(ROOT, "paper_2108_05110_amd", "csrc", "tiling.cpp"), "rb") as f:
        h.update(f.read())
    return h.hexdigest()[:16]


def traffic_from_profiles(J, N, plan):
    """HBM bytes per SpMM launch measured with rocprofv3 counters (FETCH_SIZE +
    WRITE_SIZE, scaled by the same counters on a copy of known size), if they
    were recorded for the current kernel source, shape and launch plan; else
    None."""
    path = os.path.join(ROOT, "profiles", f"spmm_traffic_cavity{N}_J{J}.json")
    if not os.path.exists(path):
        return None
    with open(path) as f:
        prof = json.load(f)
    if prof.get("source_hash") != source_hash() or prof.get("J") != J or prof.get("N") != N or plan is None:
        return None
    for rec in prof.get("records", []):   # one record per profiled launch plan
        if all(rec.get("plan", {}).get(k) == plan.get(k) for k in ("vec", "group", "deep", "tile", "waves")):
            return rec.get("bytes_per_launch")
    return None


def _oracle_v_member(task):
    """The v-subproblem of one member in the first step of the cavity, as the
    FP64 oracle computes it: the shared matrix from all J members, that member's
    right-hand side and its own sparse LU (half a member-step); seconds."""
    N, J, j = task
    import workloads as wl
    from oracle import mesh as om, scheme
    pb = wl.cavity(J=J, s=0.1, dt=0.01)
    ms = om.unit_square(N)
    ens = scheme.Ensemble(ms, pb)
    V, W = pb.ic(ms.xy)
    F1, _ = pb.forcing(pb.dt, ms.xy)
    G, _ = pb.bc(pb.dt, ms.xy)
    t0 = time.perf_counter()
    Sv = ens.shared_matrix(W)
    b = ens.rhs(V, W, F1, G, members=[j])
    ens.solve_members(Sv, b)
    return time.perf_counter() - t0


def _oracle_v_shared_lu(task):
    """The same v-subproblem for all J members with one LU shared by them (the
    paper's saving); seconds."""
    N, J = task
    import workloads as wl
    from oracle import mesh as om, scheme
    pb = wl.cavity(J=J, s=0.1, dt=0.01)
    ms = om.unit_square(N)
    ens = scheme.Ensemble(ms, pb)
    V, W = pb.ic(ms.xy)
    F1, _ = pb.forcing(pb.dt, ms.xy)
    G, _ = pb.bc(pb.dt, ms.xy)
    t0 = time.perf_counter()
    Sv = ens.shared_matrix(W)
    b = ens.rhs(V, W, F1, G)
    ens.solve_members(Sv, b, shared_lu=True)
    return time.perf_counter() - t0


def cpu_model():
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline(N, J, max_workers=16):
    """FP64 oracle on the host, on a bounded sample of the first step: P worker
    processes (one thread each) each solve the v-subproblem of one member with
    that member's own sparse LU, all at once (P half member-steps); beside them
    one more process solves the same v-subproblem for all J members with one
    shared LU.  P = the host's CPU count, at most the 16-core
    share of one GPU."""
    import multiprocessing as mp
    try:
        ncpu = len(os.sched_getaffinity(0))
    except AttributeError:
        ncpu = os.cpu_count() or 1
    P = max(1, min(ncpu, max_workers))
    keys = ("OMP_NUM_THREADS", "OPENBLAS_NUM_THREADS", "MKL_NUM_THREADS")
    saved = {k: os.environ.get(k) for k in keys}
    for k in keys:
        os.environ[k] = "1"
    try:
        ctx = mp.get_context("spawn")
        with ctx.Pool(P + 1) as pool:
            t0 = time.perf_counter()
            shared = pool.apply_async(_oracle_v_shared_lu, ((N, J),))
            times = pool.map(_oracle_v_member, [(N, J, j % J) for j in range(P)], chunksize=1)
            t_shared = shared.get()
            wall = time.perf_counter() - t0
    finally:
        for k, v in saved.items():
            if v is None:
                os.environ.pop(k, None)
            else:
                os.environ[k] = v
    return {"value": 0.5 * P / max(times), "unit": "member-steps/s", "cores": P, "kind": "oracle",
            "cpu": cpu_model(),
            "sample": f"{P} processes x 1 thread at once, each the v-subproblem (half a member-step) of one member "
                      f"in step 1 of the {N}x{N} cavity with J={J} members in the ensemble statistics, with that "
                      f"member's own SuperLU; value = {P} x 0.5 / slowest process ({max(times):.1f} s; wall with "
                      f"start-up {wall:.1f} s)",
            "shared_lu": {"value": 0.5 * J / t_shared, "unit": "member-steps/s", "cores": 1,
                          "sample": f"one more process at the same time: the same v-subproblem for all J={J} members "
                                    f"with one SuperLU factorisation shared by them, {t_shared:.1f} s"}}


class Separate:
    """J-separate form on the same GPU: the same shared matrices and right-hand
    sides as the ensemble step, then every member solved by its own
    single-column solve with the same solver schedule; the whole step is
    captured in a graph and replayed, like the ensemble step."""

    def __init__(self, L, mesh, stp, opts):
        import torch
        self.L, self.mesh, self.stp, self.opts = L, mesh, stp, opts
        J = stp.J
        self.Av = L.mhd_ens_shared_create(mesh.handle, J, opts.restart)
        self.Aw = L.mhd_ens_shared_create(mesh.handle, J, opts.restart)
        n = mesh.n
        self.bv = torch.zeros((n, J), dtype=torch.float64, device="cuda")
        self.bw = torch.zeros_like(self.bv)
        self.nu = torch.from_numpy(stp.nu).cuda()
        self.nu_m = torch.from_numpy(stp.nu_m).cuda()
        self.graph = None

    def _body(self):
        import torch
        L, m, s = self.L, self.mesh, self.stp
        J = s.J
        c = L.Coeffs(s.pb.dt, s.pb.mu, float(s.nu.mean()), float(s.nu_m.mean()), int(s.pb.convective))
        L.mhd_ens_assemble_shared(m.handle, c, s.W, J, self.Av)
        L.mhd_ens_assemble_shared(m.handle, c, s.V, J, self.Aw)
        L.mhd_ens_assemble_rhs(m.handle, c, L.MHD_V_PROBLEM, J, s.V, s.W, self.nu, self.nu_m, s.f1, s.gv, self.bv)
        L.mhd_ens_assemble_rhs(m.handle, c, L.MHD_W_PROBLEM, J, s.W, s.V, self.nu, self.nu_m, s.f2, s.gw, self.bw)
        nvel = 2 * m.nP2
        for A, b, Z, P in ((self.Av, self.bv, s.V, s.Q), (self.Aw, self.bw, s.W, s.R)):
            xs = []
            for j in range(J):
                b1 = b[:, j].contiguous()
                x1 = torch.cat([Z[:, :, j].reshape(-1), P[:, j]])
                L.mhd_ens_solve(A, b1, x1, 1, self.opts, allow_noconv=True)
                xs.append(x1)
            X = torch.stack(xs, 1)
            Z.copy_(X[:nvel].view(m.nP2, 2, J))
            P.copy_(X[nvel:])

    def step(self):
        import torch
        s = self.stp
        s.set_data((s.n + 1) * s.pb.dt)
        if self.opts.fixed_cycles > 0:
            if self.graph is None:
                self._body()                     # warm-up outside the capture
                torch.cuda.synchronize()
                self.graph = torch.cuda.CUDAGraph()
                with torch.cuda.graph(self.graph):
                    self._body()
            self.graph.replay()
        else:
            self._body()
        s.n += 1

    def close(self):
        self.L.mhd_ens_shared_free(self.Av)
        self.L.mhd_ens_shared_free(self.Aw)


def step_accuracy(L, mesh, pb, opts):
    """Relative L2 difference of one step with `opts` against an FP64 solve to
    1e-12 from the same state (after a few steps of flow development)."""
    import torch
    from paper_2108_05110_amd.ensemble import Stepper
    a = Stepper(mesh, pb, opts=opts, time_dependent_data=False, graph=opts.fixed_cycles > 0)
    for _ in range(3):
        a.step(stats=False)
    b = Stepper(mesh, pb, opts=fp64_reference_opts(L), time_dependent_data=False)
    for t_src, t_dst in ((a.V, b.V), (a.W, b.W), (a.Q, b.Q), (a.R, b.R)):
        t_dst.copy_(t_src)
    b.n = a.n
    a.step(stats=False)
    b.step(stats=False)
    rel = lambda x, y: float(torch.linalg.norm(x - y) / torch.linalg.norm(y))
    out = max(rel(a.V, b.V), rel(a.W, b.W))
    a.close()
    b.close()
    return out


def fp64_reference_opts(L):
    """FP64 solves to a relative residual of 1e-11 with a preconditioner that
    stays convergent in the developed cavity flow (Jacobi damping 0.5, two
    V-cycles for the Schur part)."""
    return L.solver_opts(L.MHD_FP64, rtol=1e-11, jacobi_omega=0.5, mg_cycles=2)


def multi_step_error(L, mesh, pb, opts, checkpoints=(8,)):
    """Relative L2 difference after each of `checkpoints` steps from the initial
    state with `opts` against FP64 solves (errors of every step accumulated),
    the largest final residual of the reference, and its time per step."""
    import torch
    from paper_2108_05110_amd.ensemble import Stepper
    a = Stepper(mesh, pb, opts=opts, time_dependent_data=False, graph=opts.fixed_cycles > 0)
    b = Stepper(mesh, pb, opts=fp64_reference_opts(L), time_dependent_data=False)
    rel = lambda x, y: float(torch.linalg.norm(x - y) / torch.linalg.norm(y))
    out, t64, worst = {}, 0.0, 0.0
    for n in range(1, max(checkpoints) + 1):
        a.step(stats=False)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        st = b.step(stats=True, allow_noconv=True)
        torch.cuda.synchronize()
        worst = max(worst, st.v.max_relres, st.w.max_relres)
        if n > 1:
            t64 += time.perf_counter() - t0
        if n in checkpoints:
            out[n] = max(rel(a.V, b.V), rel(a.W, b.W))
        if n % 25 == 0:
            log(f"  trajectory step {n}: error {max(rel(a.V, b.V), rel(a.W, b.W)):.2e}")
    out["reference_max_relres"] = worst
    a.close()
    b.close()
    return out, t64 / max(1, max(checkpoints) - 1)


def residual_track(L, mesh, pb, opts, nsteps=200, every=50):
    """Final relative residuals (max over members and both subproblems) of the
    graph-captured schedule at every `every`-th of `nsteps` steps."""
    from paper_2108_05110_amd.ensemble import Stepper
    a = Stepper(mesh, pb, opts=opts, time_dependent_data=False, graph=True)
    out = {}
    for n in range(1, nsteps + 1):
        st = a.step(stats=(n % every == 0), allow_noconv=True)
        if n % every == 0:
            out[n] = max(st.v.max_relres, st.w.max_relres)
    a.close()
    return out


def trajectory_workload(args, L, wl, torch):
    """The headline schedule against FP64 solves over `traj_steps` steps of the
    cavity from the same initial state: relative L2 difference of the member
    states at checkpoints, and the reference's largest final residual."""
    from paper_2108_05110_amd.ensemble import Mesh
    prec = L.MHD_FP32_IR if args.precision == "fp32ir" else L.MHD_FP64
    opts = L.solver_opts(prec, restart=args.restart, fixed_cycles=args.cycles, jacobi_sweeps=args.sweeps,
                         jacobi_omega=args.omega, mg_cycles=args.mg_cycles, cgs_passes=args.cgs)
    pb = wl.cavity(J=args.J, s=0.1, dt=0.01)
    mesh = Mesh(L.MHD_MESH_UNIT_SQUARE, args.N)
    tuned_plans(L, wl, mesh, args.J, prec)
    n = args.traj_steps
    cps = tuple(sorted({1, 8, 25, 50, 100, 150, n} & set(range(1, n + 1))))
    err, t64 = multi_step_error(L, mesh, pb, opts, cps)
    mesh.close()
    return {"metric": "relative L2 difference of the member states against FP64 solves", "value": err.get(n),
            "unit": "", "n_gpus": 1, "higher_is_better": False, "dtype": "f32", "data": "synthetic",
            "config": {"workload": f"cavity {args.N}x{args.N}, J={args.J}, {n} steps dt=0.01",
                       "schedule": f"{args.cycles}x{args.restart}, {args.sweeps} sweeps damping {args.omega}, "
                                   f"{args.mg_cycles} V-cycles"},
            "errors": {str(k): v for k, v in err.items()}, "fp64_ms_per_step": 1e3 * t64}


def member_problem(pb, j):
    """Member j of an ensemble problem as a one-member problem (its own data)."""
    import dataclasses
    import numpy as np
    kw = {}
    for f in dataclasses.fields(pb):
        v = getattr(pb, f.name)
        if isinstance(v, np.ndarray) and v.ndim >= 1 and v.shape[0] == pb.J:
            kw[f.name] = v[j:j + 1].copy()
    kw["J"] = 1
    return dataclasses.replace(pb, **kw)


def independent_runs(L, mesh, pb, opts, steps):
    """J independent plain runs on the same GPU: each member advanced by its own
    one-member step (its own matrices from its own fields and viscosities: the
    plain decoupled scheme), every step graph-captured; member-steps/s."""
    import torch
    from paper_2108_05110_amd.ensemble import Stepper
    runs = [Stepper(mesh, member_problem(pb, j), opts=opts, time_dependent_data=False,
                    graph=opts.fixed_cycles > 0) for j in range(pb.J)]
    for r in runs:
        r.step(stats=False)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        for r in runs:
            r.step(stats=False)
    torch.cuda.synchronize()
    el = time.perf_counter() - t0
    for r in runs:
        r.close()
    return pb.J * steps / el


def independent_runs_concurrent(L, mesh, pb, opts, steps):
    """The same J independent one-member runs advanced together: one context
    per member in a multi-ensemble group, so that each step is one graph launch
    whose J branches the GPU runs concurrently (fixed schedule only);
    member-steps/s."""
    import torch
    from paper_2108_05110_amd.ensemble import Stepper
    runs = [Stepper(mesh, member_problem(pb, j), opts=opts, time_dependent_data=False) for j in range(pb.J)]
    for r in runs:
        r.set_data(pb.dt)
    grp = L.mhd_ens_group_create([r.ctx for r in runs])
    stream = torch.cuda.Stream()

    def go():
        L.mhd_ens_group_step(grp, [r.V for r in runs], [r.W for r in runs], [r.Q for r in runs], [r.R for r in runs],
                             [r.inputs() for r in runs], stream=stream)

    go()
    stream.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        go()
    stream.synchronize()
    el = time.perf_counter() - t0
    L.mhd_ens_group_free(grp)
    for r in runs:
        r.close()
    return pb.J * steps / el


def spmm_large(L, wl, torch, N=512, J=128, plan="4,0,6,1608,0"):
    """The saddle-point SpMM of the 512 x 512 cavity with J = 128 members (FP32),
    whose operands do not fit the last-level cache: launch time from the HIP
    events of each dispatch, bytes as the full-CSR count.  The plan is the
    row-per-lane kernel with 16 x 8 half-step tiles and 16 members per
    workgroup (the autotuner's pick at this size; pinned so that the bench does
    not build every candidate's tiling), or "tune"."""
    from paper_2108_05110_amd.ensemble import Mesh, to_dev
    log("512^2 SpMM: mesh")
    mesh = Mesh(L.MHD_MESH_UNIT_SQUARE, N)
    pb = wl.cavity(J=J, s=0.1, dt=0.01, cfg=4)
    V, W = pb.ic(mesh.xy)
    A = L.mhd_ens_shared_create(mesh.handle, J, 1)
    c = L.Coeffs(pb.dt, pb.mu, float(pb.nu.mean()), float(pb.nu_m.mean()), 0)
    L.mhd_ens_assemble_shared(mesh.handle, c, to_dev(W), J, A)
    log("512^2 SpMM: plan")
    if plan == "tune":
        rep = L.mhd_ens_autotune(A, J, L.MHD_FP32_IR)
        plan = next((e for e in rep if e["chosen"] and e["op"] == L.TUNE_SADDLE), None)
    else:
        vec, group, deep, tile, waves = (int(v) for v in plan.split(","))
        L.mhd_ens_set_plan(A, J, L.MHD_FP32_IR, L.TUNE_SADDLE, vec, group, deep, tile, waves)
        plan = dict(vec=vec, group=group, deep=deep, tile=tile, waves=waves)
    log("512^2 SpMM: timing")
    x = torch.randn((mesh.n, J), device="cuda", dtype=torch.float32)
    y = torch.empty_like(x)
    for _ in range(3):
        L.mhd_ens_spmm(A, x, y, J, L.MHD_FP32_IR)
    torch.cuda.synchronize()
    L.mhd_ens_timer_enable(True)
    for _ in range(20):
        L.mhd_ens_spmm(A, x, y, J, L.MHD_FP32_IR)
    ms, launches, _, _ = L.mhd_ens_timer_read()
    L.mhd_ens_timer_enable(False)
    L.mhd_ens_shared_free(A)
    avg = ms / 1e3 / max(1, launches)
    b8 = spmm_bytes_csr(mesh.info, J, 4)
    out = {"workload": f"cavity {N}x{N} P2-P1, J={J}, FP32", "n_unknowns": int(mesh.n), "nnz": int(mesh.info.nnz),
           "bytes_per_launch": b8, "avg_launch_us": avg * 1e6, "launches": launches,
           "achieved": b8 / avg / 1e9, "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": b8 / avg / 1e9 / HBM_PEAK_GBS,
           "compact_bytes_per_launch": spmm_bytes(mesh.info, J, 4),
           "traffic": traffic_from_profiles(J, N, plan),
           "kernel": saddle_kernel_name(plan), "plan": {k: plan[k] for k in ("vec", "group", "deep", "tile", "waves")}
           if plan else None}
    mesh.close()
    return out


KERNEL_NAMES = {0: "k_saddle_v", 1: "k_saddle_p", 2: "k_saddle_h"}


def tuned_plans(L, wl, mesh, J, prec):
    """Runs the kernel autotuner for this mesh and J (the step contexts use the
    same process-wide table) and returns the chosen plan per operator."""
    import torch
    from paper_2108_05110_amd.ensemble import to_dev
    pb = wl.cavity(J=J, s=0.1, dt=0.01)
    V, W = pb.ic(mesh.xy)
    A = L.mhd_ens_shared_create(mesh.handle, J, 8)
    c = L.Coeffs(pb.dt, pb.mu, float(pb.nu.mean()), float(pb.nu_m.mean()), 0)
    L.mhd_ens_assemble_shared(mesh.handle, c, to_dev(W), J, A)
    rep = L.mhd_ens_autotune(A, J, prec)
    torch.cuda.synchronize()
    L.mhd_ens_shared_free(A)
    plans = {}
    for e in rep:
        if e["chosen"]:
            plans[e["op"]] = {k: e[k] for k in ("word", "vec", "group", "deep", "tile", "waves", "us")}
            plans[e["op"]]["candidates"] = sum(1 for f in rep if f["op"] == e["op"])
    return plans


def saddle_kernel_name(plan):
    if plan is None:
        return "k_saddle"
    if plan["deep"] == 6:
        return "k_saddle_e"
    if plan["tile"]:
        return "k_saddle_t" if plan["deep"] == 3 else "k_saddle_lds"
    if plan["deep"]:
        return KERNEL_NAMES[plan["deep"]]
    return "k_saddle_g" if plan["group"] else "k_saddle_v"


def rhs_timing(L, wl, torch, mesh, J, reps=20):
    """One subproblem's batched right-hand sides (mhd_ens_assemble_rhs) at the
    headline shape, FP64 and FP32 output, timed with events around `reps`
    launches on the current stream.  Algorithmic bytes: the member states of
    both variables read once (FP64), the ensemble mean and boundary values,
    the right-hand sides written once; the cavity has no body force."""
    import numpy as np
    pb = wl.cavity(J=J, s=0.1, dt=0.01)
    V, W = pb.ic(mesh.xy)
    dev = lambda a: torch.as_tensor(np.ascontiguousarray(a), device="cuda")
    Vd, Wd, nu, num = dev(V), dev(W), dev(pb.nu), dev(pb.nu_m)
    Gv, _ = pb.bc(pb.dt, mesh.xy[mesh.dir_nodes])
    g = dev(Gv)
    c = L.Coeffs(pb.dt, pb.mu, float(pb.nu.mean()), float(pb.nu_m.mean()), 0)
    out = {}
    nP2, n, ndir = V.shape[0], int(mesh.n), len(mesh.dir_nodes)
    for name, dt in (("fp64", torch.float64), ("fp32", torch.float32)):
        rhs = torch.empty((n, J), dtype=dt, device="cuda")
        for _ in range(3):
            L.mhd_ens_assemble_rhs(mesh.handle, c, L.MHD_V_PROBLEM, J, Vd, Wd, nu, num, None, g, rhs)
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(reps):
            L.mhd_ens_assemble_rhs(mesh.handle, c, L.MHD_V_PROBLEM, J, Vd, Wd, nu, num, None, g, rhs)
        e1.record()
        torch.cuda.synchronize()
        us = 1e3 * e0.elapsed_time(e1) / reps
        word = 8 if dt == torch.float64 else 4
        b = 8 * (2 * 2 * nP2 * J + 2 * nP2 + 2 * ndir * J) + word * n * J
        out[name] = {"us": us, "bytes": b, "GB_s": b / us / 1e3, "frac_hbm": b / us / 1e3 / HBM_PEAK_GBS}
    out["kernel"] = "k_rhs_strip"
    return out


def timed_steps(stp, steps):
    import torch
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        stp.step(stats=False)
    torch.cuda.synchronize()
    return time.perf_counter() - t0


def headline(args, L, wl, torch):
    from paper_2108_05110_amd.ensemble import Mesh, Stepper
    prec = L.MHD_FP32_IR if args.precision == "fp32ir" else L.MHD_FP64
    if args.schedule == "fixed":
        opts = L.solver_opts(prec, restart=args.restart, fixed_cycles=args.cycles, jacobi_sweeps=args.sweeps,
                             jacobi_omega=args.omega, mg_cycles=args.mg_cycles, cgs_passes=args.cgs)
    else:
        opts = L.solver_opts(prec, rtol=args.rtol, jacobi_sweeps=args.sweeps, jacobi_omega=args.omega,
                             mg_cycles=args.mg_cycles)
    graph = args.schedule == "fixed"
    pb = wl.cavity(J=args.J, s=0.1, dt=0.01)
    mesh = Mesh(L.MHD_MESH_UNIT_SQUARE, args.N)
    log("autotune")
    plans = tuned_plans(L, wl, mesh, args.J, prec)
    if args.plan:
        # study option: pin the SpMM plan after tuning (the table is process-wide)
        from paper_2108_05110_amd.ensemble import to_dev
        vec, group, deep, tile, waves = (int(v) for v in args.plan.split(","))
        A = L.mhd_ens_shared_create(mesh.handle, args.J, 8)
        L.mhd_ens_set_plan(A, args.J, prec, L.TUNE_SADDLE, vec, group, deep, tile, waves)
        L.mhd_ens_shared_free(A)
        plans["saddle"] = {"word": 4 if prec == L.MHD_FP32_IR else 8, "vec": vec, "group": group, "deep": deep,
                           "tile": tile, "waves": waves, "us": None, "candidates": 0}
    # timed region: the graph-captured step (fixed schedule) or the adaptive step
    log("timed steps")
    stp = Stepper(mesh, pb, opts=opts, time_dependent_data=False, graph=graph)
    for _ in range(args.warmup):
        stp.step(stats=False)
    elapsed = timed_steps(stp, args.steps)
    value = args.J * args.steps / elapsed
    stp.close()
    # the same schedule eager with the two subproblems one after the other, so that
    # each SpMM runs alone, timed by events its dispatch records
    log("eager pass with SpMM events")
    eag = Stepper(mesh, pb, opts=opts, time_dependent_data=False, serial=True)
    eag.step(stats=False)
    L.mhd_ens_timer_enable(True)
    e_elapsed = timed_steps(eag, max(2, args.steps // 2))
    ms, launches, _, _ = L.mhd_ens_timer_read()
    L.mhd_ens_timer_enable(False)
    # the same eager pass timing the velocity Jacobi sweeps, the step's largest kernel time
    L.mhd_ens_timer_op(L.TUNE_JACOBI)
    L.mhd_ens_timer_enable(True)
    timed_steps(eag, max(2, args.steps // 2))
    ms_j, launches_j, _, _ = L.mhd_ens_timer_read()
    L.mhd_ens_timer_enable(False)
    L.mhd_ens_timer_op(L.TUNE_SADDLE)
    st = eag.step(stats=True)
    iters = st.v.iters + st.w.iters
    eag.close()
    word = 4 if prec == L.MHD_FP32_IR else 8
    bpl_compact = spmm_bytes(mesh.info, args.J, word)
    bpl = spmm_bytes_csr(mesh.info, args.J, word)
    avg_s = (ms / 1e3) / max(launches, 1)
    achieved = bpl / avg_s / 1e9 if launches else None
    log("right-hand side timing")
    rhs_us = rhs_timing(L, wl, torch, mesh, args.J)
    log("one-step accuracy")
    acc = step_accuracy(L, mesh, pb, opts)
    log("8-step trajectory against FP64")
    traj, fp64_s = multi_step_error(L, mesh, pb, opts, (8,))
    log(f"final residuals over {args.traj_steps} steps")
    track = residual_track(L, mesh, pb, opts, args.traj_steps, 50) if graph else {}
    separate = None
    if not args.no_separate:
        log("J-separate solves")
        sstp = Stepper(mesh, pb, opts=opts, time_dependent_data=False)
        sp = Separate(L, mesh, sstp, opts)
        sp.step()                       # warm-up (and capture)
        torch.cuda.synchronize()
        s0 = time.perf_counter()
        for _ in range(args.separate_steps):
            sp.step()
        torch.cuda.synchronize()
        sv = args.J * args.separate_steps / (time.perf_counter() - s0)
        separate = {"value": sv, "unit": "member-steps/s", "steps": args.separate_steps,
                    "form": "same shared matrices and schedule, J single-column solves per subproblem, "
                            + ("graph-captured" if graph else "eager"),
                    "shared_over_separate": value / sv}
        sp.close()
        sstp.close()
        log("J independent runs")
        iv = independent_runs(L, mesh, pb, opts, args.separate_steps)
        separate["independent_runs"] = {
            "value": iv, "unit": "member-steps/s", "steps": args.separate_steps,
            "form": "J plain one-member runs, each with its own matrices (own fields and viscosities), same schedule, "
                    "each step graph-captured", "shared_over_independent": value / iv}
        if graph:
            log("J independent runs, concurrent")
            ic = independent_runs_concurrent(L, mesh, pb, opts, args.separate_steps)
            separate["independent_runs_concurrent"] = {
                "value": ic, "unit": "member-steps/s", "steps": args.separate_steps,
                "form": "the same J one-member runs as one multi-ensemble group: one graph launch per step, the J "
                        "runs as concurrent branches", "shared_over_independent": value / ic}
    out = {
        "metric": "member-steps/s at 128^2 P2-P1, J=64 (shared vs J-separate); SpMM HBM GB/s",
        "value": value,
        "unit": "member-steps/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": 1e3 * elapsed / args.steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32" if prec == L.MHD_FP32_IR else "f64",
        "data": "synthetic",
        "config": {"workload": f"lid-driven cavity, unit square {args.N}x{args.N} cells, Taylor-Hood P2-P1, "
                               f"J={args.J} members, s=0.1, dt=0.01, Re=1000 (nu, nu_m +-10% uniform)",
                   "n_unknowns": int(mesh.n), "J": args.J,
                   "precision": ("FP32 inner GMRES + FP64 refinement" if prec == L.MHD_FP32_IR else "FP64"),
                   "schedule": (f"hipGraph step, fixed {args.cycles} refinement cycles x {args.restart} GMRES "
                                f"iterations, {args.sweeps} Jacobi sweeps (damping {args.omega or 0.6:g}), "
                                f"{args.mg_cycles} V-cycle(s)" if graph else
                                f"adaptive, rtol {args.rtol:g}, {args.sweeps} Jacobi sweeps (damping {args.omega or 0.6:g})"),
                   "krylov_iterations_per_step": iters,
                   "eager_serial_member_steps_per_s": args.J * max(2, args.steps // 2) / e_elapsed,
                   "step_rel_l2_vs_fp64": acc,
                   "rel_l2_vs_fp64_after_8_steps": traj.get(8),
                   "reference_max_relres": traj.get("reference_max_relres"),
                   "final_relres_by_step": {str(k): v for k, v in track.items()},
                   "fp64_mode": {"ms_per_step": 1e3 * fp64_s, "member_steps_per_s": args.J / fp64_s,
                                 "schedule": "FP64 GMRES with FP64 refinement to rtol 1e-11, adaptive, eager, "
                                             "Jacobi damping 0.5, two V-cycles"}},
        "autotune": plans,
        "roofline": {"bound": "hbm",
                     "kernel": f"saddle-point SpMM ({saddle_kernel_name(plans.get('saddle'))})",
                     "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": (achieved / HBM_PEAK_GBS) if achieved else None,
                     "traffic": traffic_from_profiles(args.J, args.N, plans.get("saddle")), "bytes_per_launch": bpl,
                     "bytes": "full saddle-point CSR: (word + 4) nnz + 4 (n + 1) + 2 word n J",
                     "compact_bytes_per_launch": bpl_compact,
                     "compact_frac": (bpl_compact / avg_s / 1e9 / HBM_PEAK_GBS) if launches else None,
                     "avg_launch_us": avg_s * 1e6, "launches": launches},
        "rhs": rhs_us,
        "roofline_jacobi": jacobi_roofline(mesh.info, args.J, word, ms_j, launches_j, plans.get("jacobi")),
        "spmm_512_J128": None if args.no_large_spmm else spmm_large(L, wl, torch, plan=args.large_plan),
        "multi_ensemble": None if (args.no_multi or not graph) else multi_summary(args, L, wl, torch),
        "adjoint": None if args.no_adjoint else adjoint_summary(args, L, wl, torch),
        "scott_vogelius": None if args.no_sv else sv_workload(args, L, wl, torch),
        "step_channel": None if (args.no_channel or not graph) else channel_workload(args, L, wl, torch),
        "separate": separate,
        "cpu_baseline": None,
    }
    if not args.no_cpu_baseline:
        log("CPU oracle baseline")
        out["cpu_baseline"] = cpu_baseline(args.N, args.J)
    mesh.close()
    return out


def step_workload(args, L, wl, torch):
    """Only the graph-captured step of the headline configuration, replayed
    `steps` times after the warm-up: the run the per-step kernel profile is
    taken from (tuning and capture happen before the replays)."""
    from paper_2108_05110_amd.ensemble import Mesh, Stepper
    prec = L.MHD_FP32_IR if args.precision == "fp32ir" else L.MHD_FP64
    opts = L.solver_opts(prec, restart=args.restart, fixed_cycles=args.cycles, jacobi_sweeps=args.sweeps,
                         jacobi_omega=args.omega, mg_cycles=args.mg_cycles, cgs_passes=args.cgs)
    pb = wl.cavity(J=args.J, s=0.1, dt=0.01)
    mesh = Mesh(L.MHD_MESH_UNIT_SQUARE, args.N)
    plans = tuned_plans(L, wl, mesh, args.J, prec)
    stp = Stepper(mesh, pb, opts=opts, time_dependent_data=False, graph=True)
    for _ in range(args.warmup):
        stp.step(stats=False)
    torch.cuda.synchronize()
    time.sleep(0.25)   # an idle gap that separates the replays from tuning and capture in a kernel trace
    log("replays")
    elapsed = timed_steps(stp, args.steps)
    stp.close()
    mesh.close()
    # a plain device copy of known size after the replays: the reference for hardware byte counters
    src = torch.ones((256 << 20) // 4, device="cuda", dtype=torch.float32)
    dst = torch.empty_like(src)
    for _ in range(3):
        dst.copy_(src)
    torch.cuda.synchronize()
    return {"metric": "member-steps/s (graph replays only)", "value": args.J * args.steps / elapsed,
            "unit": "member-steps/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
            "ms_per_step": 1e3 * elapsed / args.steps, "higher_is_better": True, "scaling": "weak",
            "vs_baseline": None, "dtype": "f32" if prec == L.MHD_FP32_IR else "f64", "data": "synthetic",
            "config": {"workload": f"lid-driven cavity {args.N}x{args.N}, J={args.J}, graph step replays"},
            "autotune": plans}


def block_workload(args, L, wl, torch):
    """Block GMRES (one Krylov space for the J members, with deflation) against
    one Arnoldi process per member over the same shared SpMM and
    preconditioner: the first-step systems of the cavity at J = 16 ... 128,
    FP32 inner solves with FP64 refinement to rtol 1e-10 from x = 0; inner
    iterations (one SpMM over the J columns each), solve time and final
    residual."""
    from paper_2108_05110_amd.ensemble import Mesh, to_dev
    N = args.N
    mesh = Mesh(L.MHD_MESH_UNIT_SQUARE, N)
    rows = []
    for J in (16, 32, 64, 128):
        pb = wl.cavity(J=J, s=0.1, dt=0.01)
        V, W = pb.ic(mesh.xy)
        V, W = to_dev(V), to_dev(W)
        A = L.mhd_ens_shared_create(mesh.handle, J, args.restart)
        c = L.Coeffs(pb.dt, pb.mu, float(pb.nu.mean()), float(pb.nu_m.mean()), 0)
        L.mhd_ens_assemble_shared(mesh.handle, c, W, J, A)
        Gv, _ = pb.bc(pb.dt, mesh.xy[mesh.dir_nodes])
        b = torch.empty((mesh.n, J), dtype=torch.float64, device="cuda")
        L.mhd_ens_assemble_rhs(mesh.handle, c, L.MHD_V_PROBLEM, J, V, W, to_dev(pb.nu), to_dev(pb.nu_m), None,
                               to_dev(Gv), b)
        prec = L.MHD_FP32_IR if args.precision == "fp32ir" else L.MHD_FP64
        L.mhd_ens_prepare(A, J, prec)
        row = {"J": J}
        for name, blk in (("per_member", 0), ("block", 1)):
            opts = L.solver_opts(prec, rtol=1e-10, restart=args.restart, block_krylov=blk)
            x = torch.zeros_like(b)
            L.mhd_ens_solve(A, b, x, J, opts)            # warm-up
            x.zero_()
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            st, _ = L.mhd_ens_solve(A, b, x, J, opts)
            torch.cuda.synchronize()
            row[name] = {"iters": st.iters, "cycles": st.cycles, "ms": 1e3 * (time.perf_counter() - t0),
                         "max_relres": st.max_relres, "min_block_rank": st.min_block_rank}
        log(f"block J={J}: {row}")
        rows.append(row)
        L.mhd_ens_shared_free(A)
    mesh.close()
    return {"metric": "block GMRES vs per-member Arnoldi (first-step v-systems of the cavity)", "value": None,
            "unit": "ms", "n_gpus": 1, "dtype": "f32" if args.precision == "fp32ir" else "f64", "data": "synthetic",
            "config": {"workload": f"cavity {N}x{N}, restart {args.restart}, rtol 1e-10"}, "rows": rows}


def spmm_workload(args, L, wl, torch):
    """The saddle-point SpMM alone at the headline shape with the tuned plan,
    and a plain device copy of known size beside it (the reference for
    hardware byte counters): the run profiled for HBM traffic."""
    from paper_2108_05110_amd.ensemble import Mesh, to_dev
    prec = L.MHD_FP32_IR if args.precision == "fp32ir" else L.MHD_FP64
    dt = torch.float32 if prec == L.MHD_FP32_IR else torch.float64
    mesh = Mesh(L.MHD_MESH_UNIT_SQUARE, args.N)
    pb = wl.cavity(J=args.J, s=0.1, dt=0.01)
    V, W = pb.ic(mesh.xy)
    A = L.mhd_ens_shared_create(mesh.handle, args.J, 8)
    c = L.Coeffs(pb.dt, pb.mu, float(pb.nu.mean()), float(pb.nu_m.mean()), 0)
    L.mhd_ens_assemble_shared(mesh.handle, c, to_dev(W), args.J, A)
    if args.plan:
        # a pinned plan (under counter collection the tuner's timings are not representative)
        vec, group, deep, tile, waves = (int(v) for v in args.plan.split(","))
        L.mhd_ens_set_plan(A, args.J, prec, L.TUNE_SADDLE, vec, group, deep, tile, waves)
        plans = {"saddle": {"word": 4 if prec == L.MHD_FP32_IR else 8, "vec": vec, "group": group, "deep": deep,
                            "tile": tile, "waves": waves, "us": None, "candidates": 0}}
    else:
        plans = tuned_plans(L, wl, mesh, args.J, prec)
    x = torch.randn((mesh.n, args.J), device="cuda", dtype=torch.float64).to(dt)
    y = torch.empty_like(x)
    copy_bytes = 256 << 20
    src = torch.ones(copy_bytes // 4, device="cuda", dtype=torch.float32)
    dst = torch.empty_like(src)
    for _ in range(args.warmup):
        L.mhd_ens_spmm(A, x, y, args.J, prec)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        L.mhd_ens_spmm(A, x, y, args.J, prec)
    torch.cuda.synchronize()
    el = (time.perf_counter() - t0) / args.steps
    for _ in range(3):
        dst.copy_(src)
    torch.cuda.synchronize()
    L.mhd_ens_shared_free(A)
    word = 4 if prec == L.MHD_FP32_IR else 8
    bpl = spmm_bytes_csr(mesh.info, args.J, word)
    out = {"metric": "saddle-point SpMM algorithmic GB/s", "value": bpl / el / 1e9, "unit": "GB/s",
           "n_gpus": 1, "steps": args.steps, "warmup": args.warmup, "ms_per_step": el * 1e3,
           "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
           "dtype": "f32" if word == 4 else "f64", "data": "synthetic",
           "config": {"workload": f"saddle-point SpMM, unit square {args.N}x{args.N} P2-P1, J={args.J}",
                      "bytes_per_launch": bpl, "compact_bytes_per_launch": spmm_bytes(mesh.info, args.J, word),
                      "copy_reference_bytes": copy_bytes,
                      "kernel": saddle_kernel_name(plans.get("saddle"))},
           "autotune": plans}
    mesh.close()
    return out


def adjoint_workload(args, L, wl, torch, fd_checks=True):
    """128x128 cavity, J = 32, 50 FP64 steps, gradients of the final ensemble-mean
    energy w.r.t. (nu, nu_m, forcing amplitude, 8 IC coefficients) of every
    member, checkpoints every 10 steps; two entries checked by central
    differences of the GPU forward map."""
    import numpy as np
    from workloads import modes_and_forcing
    from paper_2108_05110_amd.autograd import EnsembleEnergy, Rollout
    from paper_2108_05110_amd.ensemble import Mesh
    J, N, nsteps = 32, args.N, 50
    pb = wl.cavity(J=J, s=0.1, dt=0.01, nsteps=nsteps, cfg=3)
    r = wl.rng(3, 3)
    a = r.uniform(0.5, 1.5, J)
    params = torch.tensor(np.column_stack([pb.nu, pb.nu_m, a, pb.ic_coef]), dtype=torch.float64, device="cuda")
    mesh = Mesh(L.MHD_MESH_UNIT_SQUARE, N)
    modes, fhat = modes_and_forcing(mesh.xy)
    ro = Rollout(mesh, pb, modes, fhat, opts=L.solver_opts(L.MHD_FP64), checkpoint_every=10)
    p = params.clone().requires_grad_(True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    phi = EnsembleEnergy.apply(p, ro)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    phi.backward()
    torch.cuda.synchronize()
    t2 = time.perf_counter()
    g = p.grad.cpu().numpy()
    checks = []
    h = 1e-6
    for (j, k) in (((0, 0), (5, 2), (9, 4)) if fd_checks else ()):
        pp, pm = params.clone(), params.clone()
        pp[j, k] += h
        pm[j, k] -= h
        fd = (ro.forward(pp, keep_checkpoints=False)[0] - ro.forward(pm, keep_checkpoints=False)[0]) / (2 * h)
        checks.append({"member": j, "param": k, "adjoint": float(g[j, k]), "central_fd": fd,
                       "rel_err": abs(g[j, k] - fd) / max(abs(fd), 1e-300)})
    ro.close()
    mesh.close()
    return {"metric": "adjoint gradient wall time (forward + checkpointed reverse)", "value": t2 - t0,
            "unit": "s", "higher_is_better": False, "n_gpus": 1, "dtype": "f64", "data": "synthetic",
            "config": {"workload": f"cavity {N}x{N} P2-P1, J={J}, {nsteps} steps dt=0.01, checkpoint every 10, "
                                   f"objective E_h^M, 11 parameters per member"},
            "forward_s": t1 - t0, "backward_s": t2 - t1, "phi": float(phi.detach()), "fd_checks": checks}


def adjoint_summary(args, L, wl, torch):
    """The adjoint workload (128 x 128, J = 32, 50 FP64 steps, checkpoints every
    10) as a sub-result of the headline run: wall times of the forward pass and
    the checkpointed reverse pass (its finite-difference checks are a GPU test
    and the adjoint workload's own output)."""
    log("adjoint: 50 steps forward and reverse")
    r = adjoint_workload(args, L, wl, torch, fd_checks=False)
    return {"value": r["value"], "unit": r["unit"], "forward_s": r["forward_s"], "backward_s": r["backward_s"],
            "workload": r["config"]["workload"]}


def sv_workload(args, L, wl, torch):
    """Scott-Vogelius elements (P2 velocity, discontinuous P1 pressure on the
    barycentric refinement of the sv_N x sv_N unit square; Sections 2 and 4):
    the lid-driven cavity ensemble with FP32 inner solves and FP64 refinement,
    graph-captured with a fixed schedule longer than the Taylor-Hood one (the
    discontinuous pressure level of the Schur preconditioner converges more
    slowly: 4 x 7 against 2 x 6), or adaptive eager steps to rtol.  SpMM and
    velocity-sweep rooflines from HIP events of an eager step; one-step
    accuracy against an FP64 solve."""
    from paper_2108_05110_amd.ensemble import Mesh, Stepper
    N, J = args.sv_N, args.J
    prec = L.MHD_FP32_IR
    graph = bool(args.sv_fixed)
    if graph:   # study option: a fixed schedule "cycles,restart", graph-captured
        cyc, rst = (int(v) for v in args.sv_fixed.split(","))
        opts = L.solver_opts(prec, restart=rst, fixed_cycles=cyc, jacobi_sweeps=args.sweeps,
                             jacobi_omega=args.omega, mg_cycles=args.sv_mg_cycles, cgs_passes=args.cgs,
                             mg_post=args.sv_mg_post)
    else:
        opts = L.solver_opts(prec, rtol=args.rtol, jacobi_sweeps=args.sweeps, jacobi_omega=args.omega,
                             mg_cycles=args.sv_mg_cycles, mg_post=args.sv_mg_post)
    pb = wl.cavity(J=J, s=0.1, dt=0.01)
    log(f"Scott-Vogelius {N}x{N}: mesh and autotune")
    mesh = Mesh(L.MHD_MESH_UNIT_SQUARE, N, 0, L.MHD_ELEMENT_SCOTT_VOGELIUS)
    plans = tuned_plans(L, wl, mesh, J, prec)
    stp = Stepper(mesh, pb, opts=opts, time_dependent_data=False, graph=graph)
    stp.step(stats=False)
    steps = max(2, args.sv_steps)
    elapsed = timed_steps(stp, steps)
    stp.close()
    stp = Stepper(mesh, pb, opts=opts, time_dependent_data=False, serial=True)
    st = stp.step(stats=True)
    iters = st.v.iters + st.w.iters
    L.mhd_ens_timer_enable(True)
    timed_steps(stp, 1)
    ms, launches, _, _ = L.mhd_ens_timer_read()
    L.mhd_ens_timer_enable(False)
    L.mhd_ens_timer_op(L.TUNE_JACOBI)
    L.mhd_ens_timer_enable(True)
    timed_steps(stp, 1)
    ms_j, launches_j, _, _ = L.mhd_ens_timer_read()
    L.mhd_ens_timer_enable(False)
    L.mhd_ens_timer_op(L.TUNE_SADDLE)
    stp.close()
    log("Scott-Vogelius one-step accuracy and 8-step trajectory against FP64")
    acc = step_accuracy(L, mesh, pb, opts)
    traj, _ = multi_step_error(L, mesh, pb, opts, (8,))
    bpl = spmm_bytes_csr(mesh.info, J, 4)
    avg_s = (ms / 1e3) / max(launches, 1)
    ach = bpl / avg_s / 1e9 if launches else None
    out = {"value": J * steps / elapsed, "unit": "member-steps/s", "ms_per_step": 1e3 * elapsed / steps,
           "steps": steps,
           "workload": f"lid-driven cavity, unit square {N}x{N} cells refined at the barycentres, Scott-Vogelius "
                       f"P2-P1disc, J={J}, s=0.1, dt=0.01, FP32 inner GMRES + FP64 refinement, "
                       + (f"hipGraph step, fixed {cyc} refinement cycles x {rst} GMRES iterations" if graph else
                          f"adaptive to rtol {args.rtol:g}, eager") + f", {args.sv_mg_cycles} V-cycle(s)",
           "n_unknowns": int(mesh.n), "nnz": int(mesh.info.nnz), "krylov_iterations_per_step": iters,
           "step_rel_l2_vs_fp64": acc, "rel_l2_vs_fp64_after_8_steps": traj.get(8),
           "roofline": {"bound": "hbm", "kernel": f"saddle-point SpMM ({saddle_kernel_name(plans.get('saddle'))})",
                        "achieved": ach, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                        "frac": ach / HBM_PEAK_GBS if ach else None, "bytes_per_launch": bpl,
                        "bytes": "full saddle-point CSR: (word + 4) nnz + 4 (n + 1) + 2 word n J",
                        "avg_launch_us": avg_s * 1e6, "launches": launches},
           "roofline_jacobi": jacobi_roofline(mesh.info, J, 4, ms_j, launches_j, plans.get("jacobi")),
           "autotune": plans}
    mesh.close()
    return out


def channel_workload(args, L, wl, torch):
    """The step channel [0,30]x[0,10] minus the unit step (Section 4.4 setting)
    at h = 1/channel_m with a do-nothing outflow, J members, FP32 inner solves
    with FP64 refinement on the bench's fixed schedule, graph-captured: step
    throughput, the SpMM roofline from HIP events of an eager step (the operands
    exceed the last-level cache), and one-step accuracy against FP64."""
    from paper_2108_05110_amd.ensemble import Mesh, Stepper
    m, J = args.channel_m, args.J
    opts = L.solver_opts(L.MHD_FP32_IR, restart=args.restart, fixed_cycles=args.cycles, jacobi_sweeps=args.sweeps,
                         jacobi_omega=args.omega, mg_cycles=args.mg_cycles, cgs_passes=args.cgs)
    pb = wl.step_channel(J=J, delta=1e-2, s=0.01, dt=0.02)
    log(f"step channel h=1/{m}: mesh and autotune")
    mesh = Mesh(L.MHD_MESH_STEP_CHANNEL, m, 1)
    plans = tuned_plans(L, wl, mesh, J, L.MHD_FP32_IR)
    stp = Stepper(mesh, pb, opts=opts, time_dependent_data=False, graph=True)
    stp.step(stats=False)
    steps = max(2, args.channel_steps)
    elapsed = timed_steps(stp, steps)
    stp.close()
    eag = Stepper(mesh, pb, opts=opts, time_dependent_data=False, serial=True)
    eag.step(stats=False)
    L.mhd_ens_timer_enable(True)
    timed_steps(eag, 1)
    ms, launches, _, _ = L.mhd_ens_timer_read()
    L.mhd_ens_timer_enable(False)
    eag.close()
    log("step channel one-step accuracy")
    acc = step_accuracy(L, mesh, pb, opts)
    bpl = spmm_bytes_csr(mesh.info, J, 4)
    avg_s = (ms / 1e3) / max(launches, 1)
    ach = bpl / avg_s / 1e9 if launches else None
    out = {"value": J * steps / elapsed, "unit": "member-steps/s", "ms_per_step": 1e3 * elapsed / steps,
           "steps": steps,
           "workload": f"step channel [0,30]x[0,10] minus [0,1]x[0,1], h=1/{m}, do-nothing outflow, Taylor-Hood "
                       f"P2-P1, J={J}, s=0.01, dt=0.02, nu=1/600, FP32 inner GMRES + FP64 refinement, hipGraph step, "
                       f"fixed {args.cycles} refinement cycles x {args.restart} GMRES iterations",
           "n_unknowns": int(mesh.n), "nnz": int(mesh.info.nnz), "step_rel_l2_vs_fp64": acc,
           "roofline": {"bound": "hbm", "kernel": f"saddle-point SpMM ({saddle_kernel_name(plans.get('saddle'))})",
                        "achieved": ach, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                        "frac": ach / HBM_PEAK_GBS if ach else None, "bytes_per_launch": bpl,
                        "bytes": "full saddle-point CSR: (word + 4) nnz + 4 (n + 1) + 2 word n J",
                        "avg_launch_us": avg_s * 1e6, "launches": launches},
           "autotune": plans}
    mesh.close()
    return out


def multi_summary(args, L, wl, torch):
    """The multi-ensemble workload (512 x 512, J = 128 plus four 128 x 128, J = 16,
    one graph launch per step) as a sub-result of the headline run."""
    log("multi-ensemble group step")
    r = large_workload(args, L, wl, torch, steps=3)
    return {"value": r["value"], "unit": r["unit"], "ms_per_step": r["ms_per_step"], "steps": r["steps"],
            "workload": r["config"]["workload"], "spmm_512_frac": r["roofline"]["frac"]}


def large_workload(args, L, wl, torch, steps=None):
    """512x512 cavity with J = 128 plus four 128x128 cavities with J = 16 (distinct
    seeds, s in {0.01, 0.1, 1, 1}), all advanced by one graph launch per step.
    The ensembles with s = 1 take the strong-field schedule (three refinement
    cycles, damping 0.5), the others the bench schedule."""
    nsteps = args.steps if steps is None else steps
    from paper_2108_05110_amd.ensemble import Mesh, Stepper, STRONG_FIELD_SCHEDULE
    opts = L.solver_opts(L.MHD_FP32_IR, restart=args.restart, fixed_cycles=args.cycles, jacobi_sweeps=args.sweeps,
                         jacobi_omega=args.omega, mg_cycles=args.mg_cycles, cgs_passes=args.cgs)
    strong = L.solver_opts(L.MHD_FP32_IR, **STRONG_FIELD_SCHEDULE)
    specs = [(512, wl.cavity(J=128, s=0.1, dt=0.01, cfg=4))]
    for i, sc in enumerate((0.01, 0.1, 1.0, 1.0)):
        specs.append((128, wl.cavity(J=16, s=sc, dt=0.01, cfg=10 + i)))
    meshes, steppers = [], []
    for N, pb in specs:
        m = Mesh(L.MHD_MESH_UNIT_SQUARE, N)
        meshes.append(m)
        s = Stepper(m, pb, opts=strong if pb.s >= 1.0 else opts, time_dependent_data=False)
        s.set_data(pb.dt)
        steppers.append(s)
    grp = L.mhd_ens_group_create([s.ctx for s in steppers])
    stream = torch.cuda.Stream()

    def go():
        L.mhd_ens_group_step(grp, [s.V for s in steppers], [s.W for s in steppers], [s.Q for s in steppers],
                             [s.R for s in steppers], [s.inputs() for s in steppers], stream=stream)

    go()
    stream.synchronize()
    t0 = time.perf_counter()
    for _ in range(nsteps):
        go()
    stream.synchronize()
    el = time.perf_counter() - t0
    total_members = sum(s.J for s in steppers)
    # SpMM of the 512^2 ensemble alone, eager, with HIP events
    big = Stepper(meshes[0], specs[0][1], opts=opts, time_dependent_data=False, serial=True)
    big.step(stats=False)
    L.mhd_ens_timer_enable(True)
    timed_steps(big, 1)
    ms, launches, _, _ = L.mhd_ens_timer_read()
    L.mhd_ens_timer_enable(False)
    big.close()
    bpl = spmm_bytes_csr(meshes[0].info, 128, 4)
    avg_s = (ms / 1e3) / max(launches, 1)
    L.mhd_ens_group_free(grp)
    for s in steppers:
        s.close()
    for m in meshes:
        m.close()
    ach = bpl / avg_s / 1e9
    return {"metric": "member-steps/s, one graph launch per step over 5 ensembles", "value": total_members *
            nsteps / el, "unit": "member-steps/s", "higher_is_better": True, "n_gpus": 1, "dtype": "f32",
            "data": "synthetic", "steps": nsteps, "ms_per_step": 1e3 * el / nsteps,
            "config": {"workload": "cavity 512x512 J=128 + 4 x cavity 128x128 J=16, FP32 inner + FP64 refinement, "
                                   f"fixed {args.cycles}x{args.restart} schedule (3x6, damping 0.5 for s = 1)"},
            "roofline": {"bound": "hbm", "kernel": "saddle-point SpMM at 512^2, J=128", "achieved": ach,
                         "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": ach / HBM_PEAK_GBS,
                         "bytes_per_launch": bpl, "avg_launch_us": avg_s * 1e6, "launches": launches}}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--N", type=int, default=128)
    ap.add_argument("--J", type=int, default=64)
    ap.add_argument("--precision", choices=["fp32ir", "fp64"], default="fp32ir")
    ap.add_argument("--schedule", choices=["fixed", "adaptive"], default="fixed")
    ap.add_argument("--restart", type=int, default=6)
    ap.add_argument("--cycles", type=int, default=2)
    ap.add_argument("--sweeps", type=int, default=7)
    ap.add_argument("--omega", type=float, default=0.6, help="Jacobi damping (0: the library default 0.6)")
    ap.add_argument("--mg-cycles", type=int, default=2, help="V-cycles per Schur-part application")
    ap.add_argument("--cgs", type=int, default=3,
                    help="Gram-Schmidt: 1 or 2 passes with the direct norm, 3 the fused single pass")
    ap.add_argument("--rtol", type=float, default=1e-10)
    ap.add_argument("--workload", choices=["cavity", "adjoint", "large", "spmm", "step", "block", "trajectory", "sv",
                                           "channel"],
                    default="cavity")
    ap.add_argument("--separate-steps", type=int, default=5)
    ap.add_argument("--traj-steps", type=int, default=200,
                    help="steps of the residual track (and of the trajectory workload)")
    ap.add_argument("--no-large-spmm", action="store_true")
    ap.add_argument("--large-plan", default="4,0,6,1608,0", help="SpMM plan at 512^2 (or 'tune')")
    ap.add_argument("--no-separate", action="store_true")
    ap.add_argument("--no-multi", action="store_true", help="skip the multi-ensemble sub-result")
    ap.add_argument("--no-adjoint", action="store_true", help="skip the adjoint sub-result")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-sv", action="store_true", help="skip the Scott-Vogelius sub-result")
    ap.add_argument("--no-channel", action="store_true", help="skip the step-channel sub-result")
    ap.add_argument("--channel-m", type=int, default=16, help="cells per unit length of the step channel")
    ap.add_argument("--channel-steps", type=int, default=3, help="timed steps of the step-channel workload")
    ap.add_argument("--sv-N", type=int, default=64, help="cells per side of the Scott-Vogelius workload")
    ap.add_argument("--sv-steps", type=int, default=3, help="timed steps of the Scott-Vogelius workload")
    ap.add_argument("--sv-mg-cycles", type=int, default=1, help="V-cycles per Schur-part application in the "
                    "Scott-Vogelius workload")
    ap.add_argument("--sv-mg-post", type=int, default=0, help="extra post-smoothing sweeps on the finest pressure "
                    "level in the Scott-Vogelius workload")
    ap.add_argument("--sv-fixed", default="4,7", help="fixed schedule 'cycles,restart' for the Scott-Vogelius "
                    "workload, graph-captured ('' for adaptive eager steps to --rtol)")
    ap.add_argument("--plan", default="", help="pinned SpMM plan vec,group,deep,tile,waves (spmm workload; study "
                    "option for the step)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py: this build runs on one GPU only (asked for --gpus {args.gpus}); "
              "member sharding over several GPUs is a design note, not implemented.", file=sys.stderr)
        sys.exit(2)
    rank = int(os.environ.get("RANK", "0"))
    import torch
    import workloads as wl
    from paper_2108_05110_amd import _lib as L
    torch.cuda.init()
    if args.workload == "adjoint":
        out = adjoint_workload(args, L, wl, torch)
    elif args.workload == "large":
        out = large_workload(args, L, wl, torch)
    elif args.workload == "spmm":
        out = spmm_workload(args, L, wl, torch)
    elif args.workload == "step":
        out = step_workload(args, L, wl, torch)
    elif args.workload == "block":
        out = block_workload(args, L, wl, torch)
    elif args.workload == "trajectory":
        out = trajectory_workload(args, L, wl, torch)
    elif args.workload == "sv":
        out = sv_workload(args, L, wl, torch)
    elif args.workload == "channel":
        out = channel_workload(args, L, wl, torch)
    else:
        if rank != 0:
            args.no_cpu_baseline = True
        out = headline(args, L, wl, torch)
    if rank == 0:
        print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
