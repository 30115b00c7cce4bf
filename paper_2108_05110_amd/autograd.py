"""Gradients of an ensemble-mean objective through the C ABI's adjoint step.

``EnsembleEnergy.apply(params, problem)`` runs Algorithm 1 for ``problem.nsteps``
steps from initial data built from the parameters and returns
Phi = E_h^M = (||<v_h>^M||^2 + ||<w_h>^M||^2)/2 (Section 4.2) as a 0-dim
tensor.  params is a (J, 11) float64 tensor per member:
[nu, nu_m, a (forcing amplitude: f_1 = f_2 = a fhat), 4 u-mode and 4 B-mode
initial coefficients].  The backward pass replays the forward from
checkpoints stored every ``checkpoint_every`` steps (device memory bounded by
the segment length) and runs mhd_ens_adjoint_step in reverse.
"""
from __future__ import annotations

import ctypes as C

import numpy as np
import torch

from . import _lib as L
from .ensemble import Mesh, to_dev


class Rollout:
    """Forward/adjoint driver for one mesh, problem and parameter set."""

    def __init__(self, mesh: Mesh, problem, modes, fhat, opts=None, checkpoint_every=10):
        self.mesh, self.pb = mesh, problem
        self.J = problem.J
        self.opts = opts if opts is not None else L.solver_opts(L.MHD_FP64)
        self.K = max(1, int(checkpoint_every))
        desc = L.CtxDesc(L.Coeffs(problem.dt, problem.mu, float(np.mean(problem.nu)), float(np.mean(problem.nu_m)),
                                  0), self.opts, self.J, 1)
        self.ctx = L.mhd_ens_ctx_create(mesh.handle, desc)
        self.modes_np = np.stack(modes)                           # (nm, nP2, 2)
        self.modes = to_dev(self.modes_np)
        self.fhat_np = fhat
        self.fhat = to_dev(fhat)
        xy = mesh.xy
        Gv, Gw = problem.bc(problem.dt, xy[mesh.dir_nodes])       # time-independent boundary data
        self.gv, self.gw = to_dev(Gv), to_dev(Gw)

    def initial(self, coef):
        nm = self.modes_np.shape[0]
        u = np.einsum('mnc,jm->ncj', self.modes_np, coef[:, :nm])
        B = np.einsum('mnc,jm->ncj', self.modes_np, coef[:, nm:2 * nm])
        B[:, 1, :] += 1.0
        rs = np.sqrt(self.pb.s)
        return to_dev(u + rs * B), to_dev(u - rs * B)

    def _step(self, V, W, Q, R, nu, num, F):
        inp = L.StepInputs(nu.ctypes.data_as(C.POINTER(C.c_double)), num.ctypes.data_as(C.POINTER(C.c_double)),
                           L.ptr(F), L.ptr(F), L.ptr(self.gv), L.ptr(self.gw), self.J)
        return L.mhd_ens_step(self.ctx, V, W, Q, R, inp, stats=True)

    def forward(self, params, keep_checkpoints=True):
        p = params.detach().cpu().numpy().astype(np.float64)
        nu, num, a = np.ascontiguousarray(p[:, 0]), np.ascontiguousarray(p[:, 1]), p[:, 2]
        coef = p[:, 3:]
        V, W = self.initial(coef)
        F = to_dev(self.fhat_np[:, :, None] * a[None, None, :])
        Q = torch.zeros((self.mesh.nP1, self.J), dtype=torch.float64, device="cuda")
        R = torch.zeros_like(Q)
        ckpt = {}
        energy = None
        for n in range(self.pb.nsteps):
            if keep_checkpoints and n % self.K == 0:
                ckpt[n] = (V.clone(), W.clone(), Q.clone(), R.clone())
            st = self._step(V, W, Q, R, nu, num, F)
            energy = st.energy
        return energy, ckpt, (nu, num, F)

    def backward(self, params, ckpt, data):
        nu, num, F = data
        J = self.J
        V_end = None
        lamV = torch.empty((self.mesh.nP2, 2, J), dtype=torch.float64, device="cuda")
        lamW = torch.empty_like(lamV)
        grad = torch.zeros((J, 3), dtype=torch.float64, device="cuda")
        adj_in = L.AdjointInputs(nu.ctypes.data_as(C.POINTER(C.c_double)), num.ctypes.data_as(C.POINTER(C.c_double)),
                                 L.ptr(self.fhat), J)
        N = self.pb.nsteps
        starts = sorted(ckpt)
        first = True
        for s0 in reversed(starts):
            s1 = min(s0 + self.K, N)
            V, W, Q, R = (t.clone() for t in ckpt[s0])
            seg = [(V.clone(), W.clone())]
            for n in range(s0, s1):                  # recompute the segment's states
                self._step(V, W, Q, R, nu, num, F)
                seg.append((V.clone(), W.clone()))
            if first:
                V_end = seg[-1]
                L.mhd_ens_adjoint_terminal(self.ctx, V_end[0], V_end[1], lamV, lamW, J)
                first = False
            for k in range(s1 - s0 - 1, -1, -1):
                Vn, Wn = seg[k]
                V1, W1 = seg[k + 1]
                L.mhd_ens_adjoint_step(self.ctx, Vn, Wn, V1, W1, lamV, lamW, lamV, lamW, adj_in, grad)
        nm = self.modes_np.shape[0]
        gic = torch.zeros((J, 2 * nm), dtype=torch.float64, device="cuda")
        L.mhd_ens_adjoint_ic(self.ctx, lamV, lamW, self.modes, nm, float(self.pb.s), gic, J)
        return torch.cat([grad, gic], dim=1)

    def close(self):
        if self.ctx:
            L.mhd_ens_ctx_free(self.ctx)
            self.ctx = None


class EnsembleEnergy(torch.autograd.Function):
    @staticmethod
    def forward(ctx, params, rollout):
        energy, ckpt, data = rollout.forward(params)
        ctx.rollout, ctx.ckpt, ctx.data = rollout, ckpt, data
        ctx.save_for_backward(params)
        return torch.tensor(energy, dtype=torch.float64, device=params.device)

    @staticmethod
    def backward(ctx, grad_out):
        (params,) = ctx.saved_tensors
        g = ctx.rollout.backward(params, ctx.ckpt, ctx.data)
        return grad_out * g.to(params.device), None
