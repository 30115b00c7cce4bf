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

Reported beside it on the same GPU: the J-separate form (the same shared
matrices, each member solved by its own single-column solve), the roofline of
the saddle-point SpMM (algorithmic bytes per launch over the launch time from
HIP events recorded around every launch inside the timed region), and the
FP64 CPU oracle timed on a bounded sample on the host.
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


def source_hash():
    h = hashlib.sha256()
    with open(os.path.join(ROOT, "paper_2108_05110_amd", "csrc", "solve.hip"), "rb") as f:
        h.update(f.read())
    return h.hexdigest()[:16]


def traffic_from_profiles(J, N):
    """HBM bytes per SpMM launch measured with rocprofv3 counters, if recorded for
    the current kernel source; else None."""
    path = os.path.join(ROOT, "profiles", "spmm_traffic_cavity128_J64.json")
    if not os.path.exists(path):
        return None
    with open(path) as f:
        rec = json.load(f)
    if rec.get("source_hash") != source_hash() or rec.get("J") != J or rec.get("N") != N:
        return None
    return rec.get("bytes_per_launch")


def cpu_baseline(N, J, seconds_hint=30.0):
    """FP64 oracle (its own per-member sparse LU) on a bounded sample of the same
    workload: the v-subproblem of one member in the first step (shared matrix
    from all J members, that member's right-hand side, its own LU)."""
    import numpy as np
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
    b = ens.rhs(V[:, :, :1], W[:, :, :1], F1[:, :, :1], G[:, :, :1])
    ens.solve_members(Sv, b, members=[0])
    dt = time.perf_counter() - t0
    _ = np
    return {"value": 0.5 / dt, "unit": "member-steps/s", "cores": 1, "kind": "oracle",
            "sample": f"v-subproblem of 1 member, step 1, {N}x{N} cavity with J={J} members in the "
                      f"ensemble statistics (= 0.5 member-step), per-member SuperLU, "
                      f"{dt:.1f} s on one host core"}


class Separate:
    """J-separate form on the same GPU: shared matrices and right-hand sides as in
    the ensemble step, then every member solved by its own single-column solve."""

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
        self.iters = 0

    def step(self):
        import torch
        L, m, s = self.L, self.mesh, self.stp
        J = s.J
        s.set_data((s.n + 1) * s.pb.dt)
        c = L.Coeffs(s.pb.dt, s.pb.mu, float(s.nu.mean()), float(s.nu_m.mean()), int(s.pb.convective))
        L.mhd_ens_assemble_shared(m.handle, c, s.W, J, self.Av)
        L.mhd_ens_assemble_shared(m.handle, c, s.V, J, self.Aw)
        L.mhd_ens_assemble_rhs(m.handle, c, L.MHD_V_PROBLEM, J, s.V, s.W, self.nu, self.nu_m, s.f1, s.gv, self.bv)
        L.mhd_ens_assemble_rhs(m.handle, c, L.MHD_W_PROBLEM, J, s.W, s.V, self.nu, self.nu_m, s.f2, s.gw, self.bw)
        nvel = 2 * m.nP2
        newV = torch.empty_like(s.V)
        newW = torch.empty_like(s.W)
        for A, b, Z, P, out in ((self.Av, self.bv, s.V, s.Q, newV), (self.Aw, self.bw, s.W, s.R, newW)):
            for j in range(J):
                b1 = b[:, j].contiguous()
                x1 = torch.cat([Z[:, :, j].reshape(-1), P[:, j]])
                st, _ = L.mhd_ens_solve(A, b1, x1, 1, self.opts, allow_noconv=True)
                self.iters += st.iters
                out[:, :, j] = x1[:nvel].view(m.nP2, 2)
                P[:, j] = x1[nvel:]
        s.V.copy_(newV)
        s.W.copy_(newW)
        s.n += 1

    def close(self):
        self.L.mhd_ens_shared_free(self.Av)
        self.L.mhd_ens_shared_free(self.Aw)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--N", type=int, default=128)
    ap.add_argument("--J", type=int, default=64)
    ap.add_argument("--precision", choices=["fp32ir", "fp64"], default="fp32ir")
    ap.add_argument("--separate-steps", type=int, default=1)
    ap.add_argument("--no-separate", action="store_true")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py: this build runs on one GPU only (asked for --gpus {args.gpus}); "
              "member sharding over several GPUs is a design note, not implemented.", file=sys.stderr)
        sys.exit(2)
    rank = int(os.environ.get("RANK", "0"))

    import numpy as np
    import torch
    import workloads as wl
    from paper_2108_05110_amd import _lib as L
    from paper_2108_05110_amd.ensemble import Mesh, Stepper

    torch.cuda.init()
    prec = L.MHD_FP32_IR if args.precision == "fp32ir" else L.MHD_FP64
    opts = L.solver_opts(prec)
    pb = wl.cavity(J=args.J, s=0.1, dt=0.01)
    mesh = Mesh(L.MHD_MESH_UNIT_SQUARE, args.N)
    stp = Stepper(mesh, pb, opts=opts, time_dependent_data=False)
    for _ in range(args.warmup):
        stp.step(stats=False)
    L.mhd_ens_timer_enable(True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    iters = 0
    for _ in range(args.steps):
        st = stp.step(stats=True)
        iters += st.v.iters + st.w.iters
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    ms, launches, nJ32, nJ64 = L.mhd_ens_timer_read()
    L.mhd_ens_timer_enable(False)
    elapsed = t1 - t0
    value = args.J * args.steps / elapsed
    word = 4 if prec == L.MHD_FP32_IR else 8
    bpl = spmm_bytes(mesh.info, args.J, word)
    avg_s = (ms / 1e3) / max(launches, 1)
    achieved = bpl / avg_s / 1e9 if launches else None
    traffic = traffic_from_profiles(args.J, args.N)

    separate = None
    if not args.no_separate:
        sp = Separate(L, mesh, stp, opts)
        sp.step()                       # warm-up
        torch.cuda.synchronize()
        s0 = time.perf_counter()
        for _ in range(args.separate_steps):
            sp.step()
        torch.cuda.synchronize()
        s1 = time.perf_counter()
        sv = args.J * args.separate_steps / (s1 - s0)
        separate = {"value": sv, "unit": "member-steps/s", "steps": args.separate_steps,
                    "form": "same shared matrices, J single-column solves per subproblem",
                    "shared_over_separate": value / sv}
        sp.close()

    cpu = None
    if rank == 0 and not args.no_cpu_baseline:
        cpu = cpu_baseline(args.N, args.J)

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
                   "precision": "FP32 inner GMRES + FP64 refinement" if prec == L.MHD_FP32_IR else "FP64",
                   "krylov_iterations_per_step": iters / args.steps},
        "roofline": {"bound": "hbm", "kernel": "saddle-point SpMM (k_saddle)",
                     "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": (achieved / HBM_PEAK_GBS) if achieved else None,
                     "traffic": traffic, "bytes_per_launch": bpl, "avg_launch_us": avg_s * 1e6,
                     "launches": launches},
        "separate": separate,
        "cpu_baseline": cpu,
    }
    if rank == 0:
        print(json.dumps(out), flush=True)
    stp.close()
    mesh.close()
    _ = np


if __name__ == "__main__":
    main()
