"""GPU adjoint (mhd_ens_adjoint_* through torch.autograd) against the FP64 CPU
adjoint and against central differences of the GPU forward map."""
import sys

import numpy as np
import pytest

import workloads as wl
from oracle import mesh as om
from oracle.adjoint import EnsembleAdjoint
from workloads import modes_and_forcing

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def setup(N=4, J=3, nsteps=3, seed=11, K=10):
    from paper_2108_05110_amd import _lib as L
    from paper_2108_05110_amd.autograd import Rollout
    from paper_2108_05110_amd.ensemble import Mesh
    pb = wl.cavity(J=J, s=0.3, dt=0.05, nsteps=nsteps, nu_mean=0.01, num_mean=0.02, ic_amp=0.3)
    r = np.random.default_rng(seed)
    nu = 0.01 * (1 + r.uniform(-0.1, 0.1, J))
    num = 0.02 * (1 + r.uniform(-0.1, 0.1, J))
    a = r.uniform(0.5, 1.5, J)
    coef = 0.3 * r.uniform(-1, 1, (J, 8))
    pb.nu, pb.nu_m = nu.copy(), num.copy()
    gm = Mesh(L.MHD_MESH_UNIT_SQUARE, N)
    modes, fhat = modes_and_forcing(gm.xy)
    ro = Rollout(gm, pb, modes, fhat, opts=L.solver_opts(L.MHD_FP64), checkpoint_every=K)
    params = torch.tensor(np.column_stack([nu, num, a, coef]), dtype=torch.float64, device="cuda")
    return pb, gm, ro, params, (nu, num, a, coef)


@pytest.fixture(scope="module")
def gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


def test_adjoint_matches_cpu_adjoint(gpu):
    from paper_2108_05110_amd.autograd import EnsembleEnergy
    say("adjoint vs CPU adjoint")
    pb, gm, ro, params, (nu, num, a, coef) = setup()
    p = params.clone().requires_grad_(True)
    phi = EnsembleEnergy.apply(p, ro)
    phi.backward()
    g_gpu = p.grad.cpu().numpy()
    ms = om.unit_square(4)
    modes, fhat = modes_and_forcing(ms.xy)
    adj = EnsembleAdjoint(ms, pb, fhat, modes)
    phi_c, g, gc = adj.gradient(nu, num, a, coef, pb.nsteps)
    g_cpu = np.column_stack([g, gc])
    say("  phi", float(phi), phi_c)
    assert abs(float(phi) - phi_c) <= 1e-11 * abs(phi_c)
    err = np.abs(g_gpu - g_cpu).max() / np.abs(g_cpu).max()
    say("  max rel grad diff", err)
    assert err <= 1e-8, err
    ro.close()
    gm.close()


def test_adjoint_matches_gpu_central_differences(gpu):
    from paper_2108_05110_amd.autograd import EnsembleEnergy
    say("adjoint vs GPU central differences")
    pb, gm, ro, params, _ = setup(J=4, nsteps=4, seed=3)
    p = params.clone().requires_grad_(True)
    EnsembleEnergy.apply(p, ro).backward()
    g = p.grad.cpu().numpy()
    h = 1e-5
    for (j, k) in ((0, 0), (1, 1), (2, 2), (3, 3), (0, 7), (2, 10)):
        pp, pm = params.clone(), params.clone()
        pp[j, k] += h
        pm[j, k] -= h
        fd = (ro.forward(pp, keep_checkpoints=False)[0] - ro.forward(pm, keep_checkpoints=False)[0]) / (2 * h)
        say("  param", j, k, g[j, k], fd)
        assert abs(g[j, k] - fd) <= 1e-5 * max(abs(fd), 1e-3 * np.abs(g).max()), (j, k, g[j, k], fd)
    ro.close()
    gm.close()


def test_checkpoint_interval_does_not_change_gradient(gpu):
    from paper_2108_05110_amd.autograd import EnsembleEnergy
    say("checkpoint intervals")
    grads = []
    for K in (1, 2, 10):
        pb, gm, ro, params, _ = setup(J=3, nsteps=5, seed=5, K=K)
        p = params.clone().requires_grad_(True)
        EnsembleEnergy.apply(p, ro).backward()
        grads.append(p.grad.cpu().numpy())
        ro.close()
        gm.close()
    assert np.array_equal(grads[0], grads[1]) and np.array_equal(grads[0], grads[2])


@pytest.mark.timeout(600)
def test_adjoint_at_full_size_matches_gpu_central_differences(gpu):
    """The adjoint workload at its full size: 128 x 128 cavity, J = 32, 50 FP64
    steps, checkpoints every 10, gradient of the final ensemble-mean energy with
    respect to all 11 parameters of every member; three entries (a viscosity,
    a forcing amplitude, an initial-mode coefficient) against central
    differences of the GPU forward map, bar 1e-5 relative."""
    from paper_2108_05110_amd import _lib as L
    from paper_2108_05110_amd.autograd import EnsembleEnergy, Rollout
    from paper_2108_05110_amd.ensemble import Mesh
    N, J, nsteps = 128, 32, 50
    say("adjoint at full size: 128^2, J=32, 50 steps, checkpoints every 10")
    pb = wl.cavity(J=J, s=0.1, dt=0.01, nsteps=nsteps, cfg=3)
    a = wl.rng(3, 3).uniform(0.5, 1.5, J)
    params = torch.tensor(np.column_stack([pb.nu, pb.nu_m, a, pb.ic_coef]), dtype=torch.float64, device="cuda")
    gm = Mesh(L.MHD_MESH_UNIT_SQUARE, N)
    modes, fhat = modes_and_forcing(gm.xy)
    ro = Rollout(gm, pb, modes, fhat, opts=L.solver_opts(L.MHD_FP64), checkpoint_every=10)
    p = params.clone().requires_grad_(True)
    EnsembleEnergy.apply(p, ro).backward()
    g = p.grad.cpu().numpy()
    say("  gradient done")
    h = 1e-6
    for (j, k) in ((0, 0), (5, 2), (9, 4)):
        pp, pm = params.clone(), params.clone()
        pp[j, k] += h
        pm[j, k] -= h
        fd = (ro.forward(pp, keep_checkpoints=False)[0] - ro.forward(pm, keep_checkpoints=False)[0]) / (2 * h)
        rel = abs(g[j, k] - fd) / abs(fd)
        say(f"  member {j} parameter {k}: adjoint {g[j, k]:.10e}, central difference {fd:.10e}, rel {rel:.2e}")
        assert rel <= 1e-5, (j, k, g[j, k], fd)
    ro.close()
    gm.close()
