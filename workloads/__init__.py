"""Seeded synthetic inputs for the ensemble MHD time step (problem data only).

This module is the one place that both the FP64 CPU oracle and the GPU path
take their inputs from.  It holds problem data and nothing of the numerical
method: member parameters drawn from seeded generators, and closed-form
initial, boundary and forcing functions evaluated at whatever node
coordinates the caller passes in (each side evaluates them on its own mesh).
No assembly, no time stepping and no linear algebra lives here.

Problems (paper, Section 4):

* ``Manufactured`` -- the convergence-rate test of Section 4.1: the smooth
  Elsasser pair (v, w) and pressure given there, member copies scaled by the
  factor c_j of Section 4.1, forcing derived from the Elsasser system
  (els1)-(els2) with each member's own viscosities.
* ``Cavity`` -- a lid-driven cavity on the unit square with the magnetic
  boundary data of Section 4.3 (B = (0, 1) on all walls), small random
  divergence-free initial perturbations, Re = 1000 mean viscosities with
  uniform +-10 % member perturbations.
* ``StepChannel`` -- flow over a forward step in [0,30]x[0,10] minus the unit
  square at the inlet corner, parabolic inflow with a member perturbation.

Seeds: ``numpy.random.default_rng(2108_05110 + 100 * cfg + k)`` with k the
index of the array drawn (0: nu, 1: nu_m, 2: initial-condition coefficients,
3: forcing amplitudes, 4: inflow perturbation).
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np

SEED_BASE = 2108_05110


def rng(cfg: int, k: int) -> np.random.Generator:
    return np.random.default_rng(SEED_BASE + 100 * cfg + k)


def member_factor(J: int, eps: float) -> np.ndarray:
    """c_j = 1 + (-1)^(j+1) ceil(j/2) eps / 5 for j = 1..J (Section 4.1)."""
    j = np.arange(1, J + 1)
    return 1.0 + ((-1.0) ** (j + 1)) * np.ceil(j / 2.0) * eps / 5.0


# ---------------------------------------------------------------- modes
# Divergence-free modes that vanish on the boundary of the unit square:
# phi_kl = curl psi_kl = (d psi/dy, -d psi/dx), psi_kl = sin^2(k pi x) sin^2(l pi y).
MODES = ((1, 1), (1, 2), (2, 1), (2, 2))


def mode_field(k: int, l: int, xy: np.ndarray) -> np.ndarray:
    x, y = xy[:, 0], xy[:, 1]
    a, b = k * math.pi, l * math.pi
    sx, sy = np.sin(a * x), np.sin(b * y)
    # d/dy sin^2(b y) = b sin(2 b y); d/dx sin^2(a x) = a sin(2 a x)
    ux = sx * sx * b * np.sin(2 * b * y)
    uy = -a * np.sin(2 * a * x) * sy * sy
    return np.stack([ux, uy], axis=1)


def modes_and_forcing(xy: np.ndarray):
    """The four initial modes of the parameter study (nodal fields at xy) and
    the forcing shape fhat = curl(sin^2(pi x) sin^2(pi y))."""
    modes = [mode_field(k, l, xy) for (k, l) in MODES]
    return modes, mode_field(1, 1, xy)


def _on(val, target, tol=1e-12):
    return np.abs(val - target) < tol


@dataclass
class Problem:
    """Common interface.  Vector nodal arrays are (n_nodes, 2, J); scalars (n, J)."""
    J: int
    dt: float
    nsteps: int
    s: float
    mu: float
    nu: np.ndarray
    nu_m: np.ndarray
    convective: int = 0          # 0: skew-symmetric trilinear form, 1: plain (u.grad v, w)
    pin_pressure: bool = True    # all-Dirichlet problems pin the pressure at (0,0)
    natural_outflow: bool = False

    def ic(self, xy):
        raise NotImplementedError

    def forcing(self, t, xy):
        raise NotImplementedError

    def bc(self, t, xy):
        raise NotImplementedError

    def is_dirichlet(self, xy_boundary):
        """Mask over boundary nodes that carry Dirichlet data (all, unless a natural outflow)."""
        return np.ones(len(xy_boundary), dtype=bool)


# ------------------------------------------------------- manufactured
@dataclass
class Manufactured(Problem):
    """Section 4.1: v, w, p closed forms with lambda = 0, scaled per member by c_j."""
    eps: float = 0.0
    c: np.ndarray = field(default=None)

    def __post_init__(self):
        if self.c is None:
            self.c = member_factor(self.J, self.eps)

    @staticmethod
    def base(t, xy):
        x, y = xy[:, 0], xy[:, 1]
        a = 1.0 + math.exp(t)
        v = np.stack([np.cos(y) + a * np.sin(y), np.sin(x) + a * np.cos(x)], axis=1)
        w = np.stack([np.cos(y) - a * np.sin(y), np.sin(x) - a * np.cos(x)], axis=1)
        p = np.sin(x + y) * a
        return v, w, p

    @staticmethod
    def base_grad(t, xy):
        """Gradients G[n, c, d] = d v_c / d x_d of the unscaled v and w."""
        x, y = xy[:, 0], xy[:, 1]
        a = 1.0 + math.exp(t)
        z = np.zeros_like(x)
        gv = np.stack([np.stack([z, -np.sin(y) + a * np.cos(y)], 1),
                       np.stack([np.cos(x) - a * np.sin(x), z], 1)], 1)
        gw = np.stack([np.stack([z, -np.sin(y) - a * np.cos(y)], 1),
                       np.stack([np.cos(x) + a * np.sin(x), z], 1)], 1)
        return gv, gw

    def exact(self, t, xy):
        v, w, p = self.base(t, xy)
        V = v[:, :, None] * self.c[None, None, :]
        W = w[:, :, None] * self.c[None, None, :]
        P = np.repeat(p[:, None], self.J, axis=1)
        return V, W, P

    def ic(self, xy):
        V, W, _ = self.exact(0.0, xy)
        return V, W

    def bc(self, t, xy):
        V, W, _ = self.exact(t, xy)
        return V, W

    def forcing(self, t, xy):
        """f_{1,j}, f_{2,j} from the Elsasser system with the member's nu_j, nu_m,j.

        With v_j = c_j v, w_j = c_j w, q_j = r_j = p:
          f1 = c v_t + c^2 w.grad v - (nu+nu_m)/2 c lap v - (nu-nu_m)/2 c lap w + grad p
        and lap v = -v, lap w = -w for this pair.
        """
        x, y = xy[:, 0], xy[:, 1]
        et = math.exp(t)
        a = 1.0 + et
        v, w, p = self.base(t, xy)
        vt = np.stack([et * np.sin(y), et * np.cos(x)], axis=1)
        wt = -vt
        gv, gw = self.base_grad(t, xy)
        w_grad_v = np.einsum('nd,ncd->nc', w, gv)
        v_grad_w = np.einsum('nd,ncd->nc', v, gw)
        gp = np.stack([np.cos(x + y) * a, np.cos(x + y) * a], axis=1)
        c = self.c[None, None, :]
        nup = ((self.nu + self.nu_m) / 2)[None, None, :]
        num = ((self.nu - self.nu_m) / 2)[None, None, :]
        f1 = (c * vt[:, :, None] + c * c * w_grad_v[:, :, None]
              + nup * c * v[:, :, None] + num * c * w[:, :, None] + gp[:, :, None])
        f2 = (c * wt[:, :, None] + c * c * v_grad_w[:, :, None]
              + nup * c * w[:, :, None] + num * c * v[:, :, None] + gp[:, :, None])
        return f1, f2


def manufactured(J=2, eps=0.01, h_inv=16, dt=0.01, nsteps=10, s=1.0, mu=1.0,
                 nu_mean=0.01, num_mean=0.01, spread=0.1, cfg=0, convective=0):
    """Config C1 family: nu_j = nu_mean(1+e_j), nu_m,j = num_mean(1+eta_j), e,eta ~ U[-spread, spread]."""
    e = rng(cfg, 0).uniform(-spread, spread, J)
    eta = rng(cfg, 1).uniform(-spread, spread, J)
    return Manufactured(J=J, dt=dt, nsteps=nsteps, s=s, mu=mu,
                        nu=nu_mean * (1 + e), nu_m=num_mean * (1 + eta), eps=eps,
                        convective=convective)


# --------------------------------------------------------------- cavity
@dataclass
class Cavity(Problem):
    """Lid-driven cavity, unit square: u = (1,0) on the lid y = 1 (0 < x < 1, corners
    take the wall value), u = 0 on the other walls, B = (0,1) on every wall, f = g = 0,
    initial B = (0,1) plus small modes, initial u = small modes."""
    ic_coef: np.ndarray = None      # (J, 8): 4 velocity-mode and 4 magnetic-mode coefficients
    amp: np.ndarray = None          # (J,) forcing amplitude a_j (f_j = a_j fhat); zero by default
    lid: float = 1.0

    def _uB_bc(self, xy):
        x, y = xy[:, 0], xy[:, 1]
        u = np.zeros((len(x), 2))
        top = _on(y, 1.0) & (x > 1e-12) & (x < 1 - 1e-12)
        u[top, 0] = self.lid
        B = np.zeros((len(x), 2))
        B[:, 1] = 1.0
        return u, B

    def ic(self, xy):
        n = len(xy)
        u = np.zeros((n, 2, self.J))
        B = np.zeros((n, 2, self.J))
        B[:, 1, :] = 1.0
        for m, (k, l) in enumerate(MODES):
            ph = mode_field(k, l, xy)[:, :, None]
            u += ph * self.ic_coef[None, None, :, m]
            B += ph * self.ic_coef[None, None, :, 4 + m]
        rs = math.sqrt(self.s)
        return u + rs * B, u - rs * B

    def bc(self, t, xy):
        u, B = self._uB_bc(xy)
        rs = math.sqrt(self.s)
        v = (u + rs * B)[:, :, None].repeat(self.J, axis=2)
        w = (u - rs * B)[:, :, None].repeat(self.J, axis=2)
        return v, w

    def forcing(self, t, xy):
        n = len(xy)
        if self.amp is None or not np.any(self.amp):
            z = np.zeros((n, 2, self.J))
            return z, z.copy()
        fh = mode_field(1, 1, xy)[:, :, None] * self.amp[None, None, :]
        return fh, fh.copy()


def cavity(J=20, s=0.1, dt=0.01, nsteps=200, mu=1.0, nu_mean=1e-3, num_mean=1e-3,
           spread=0.1, ic_amp=1e-3, cfg=1, convective=0, amp=None):
    e = rng(cfg, 0).uniform(-spread, spread, J)
    eta = rng(cfg, 1).uniform(-spread, spread, J)
    coef = ic_amp * rng(cfg, 2).uniform(-1.0, 1.0, (J, 8))
    return Cavity(J=J, dt=dt, nsteps=nsteps, s=s, mu=mu, nu=nu_mean * (1 + e),
                  nu_m=num_mean * (1 + eta), ic_coef=coef, amp=amp, convective=convective)


# ---------------------------------------------------------- step channel
@dataclass
class StepChannel(Problem):
    """[0,30]x[0,10] minus [0,1]x[0,1]; inlet x = 0, y in [1,10]:
    u = (y' (9 - y') 4/81 + delta (1 + e_j) sin(pi y/10), 0), y' = y - 1 (a parabola of
    peak 1 across the inlet); walls u = 0; B = (0,1) on inlet and walls; natural
    outflow at x = 30.  Initial u = inlet profile extended in x (zero on walls),
    initial B = 0."""
    delta: float = 1e-2
    e: np.ndarray = None

    def _inflow(self, y):
        yp = y - 1.0
        base = np.clip(yp * (9.0 - yp) * 4.0 / 81.0, 0.0, None)
        pert = self.delta * (1.0 + self.e)[None, :] * np.sin(math.pi * y / 10.0)[:, None]
        return base[:, None] + pert * (yp > 0)[:, None] * (yp < 9)[:, None]

    def is_dirichlet(self, xy_boundary):
        return ~_on(xy_boundary[:, 0], 30.0)

    def _uB_bc(self, xy):
        x, y = xy[:, 0], xy[:, 1]
        n = len(x)
        u = np.zeros((n, 2, self.J))
        inlet = _on(x, 0.0) & (y > 1 + 1e-12) & (y < 10 - 1e-12)
        u[inlet, 0, :] = self._inflow(y[inlet])
        B = np.zeros((n, 2, self.J))
        B[:, 1, :] = 1.0
        return u, B

    def bc(self, t, xy):
        u, B = self._uB_bc(xy)
        rs = math.sqrt(self.s)
        return u + rs * B, u - rs * B

    def ic(self, xy):
        x, y = xy[:, 0], xy[:, 1]
        n = len(x)
        u = np.zeros((n, 2, self.J))
        inside = (y > 1 + 1e-12) & (y < 10 - 1e-12)
        u[inside, 0, :] = self._inflow(y[inside])
        B = np.zeros((n, 2, self.J))
        rs = math.sqrt(self.s)
        return u + rs * B, u - rs * B

    def forcing(self, t, xy):
        z = np.zeros((len(xy), 2, self.J))
        return z, z.copy()


def step_channel(J=64, delta=1e-2, s=0.01, dt=0.02, nsteps=300, mu=1.0, nu=1.0 / 600,
                 spread=0.1, cfg=2):
    e = rng(cfg, 4).uniform(-spread, spread, J)
    return StepChannel(J=J, dt=dt, nsteps=nsteps, s=s, mu=mu, nu=np.full(J, nu),
                       nu_m=np.full(J, nu), delta=delta, e=e, pin_pressure=False,
                       natural_outflow=True)
