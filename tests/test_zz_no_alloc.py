"""GPU test of the allocation-free right-hand side entry point.

mhd_ens_assemble_rhs_noalloc runs the kernels of mhd_ens_assemble_rhs with
its scratch (member coefficients, ensemble mean) in a fixed device array of
the library; its output must equal the allocating call's bit for bit, also
when a second, smaller call follows (the array keeps the first call's
contents).
"""
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


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float64)).cuda()


def rhs_pair(L, gm, pb, which, seed):
    """(allocating call, allocation-free call) right-hand sides for a random state."""
    J = pb.J
    V, W = pb.ic(gm.xy)
    r = np.random.default_rng(seed)
    V = V + 0.05 * r.standard_normal(V.shape)
    W = W + 0.05 * r.standard_normal(W.shape)
    t1 = pb.dt
    F1, F2 = pb.forcing(t1, gm.xy)
    Gv, Gw = pb.bc(t1, gm.xy)
    selfZ, otherZ, F, G = (V, W, F1, Gv) if which == 0 else (W, V, F2, Gw)
    c = L.Coeffs(pb.dt, pb.mu, float(pb.nu.mean()), float(pb.nu_m.mean()), 0)
    args = (dev(selfZ), dev(otherZ), dev(pb.nu), dev(pb.nu_m), dev(F), dev(G[gm.dir_nodes]))
    ref = torch.full((gm.n, J), np.nan, dtype=torch.float64, device="cuda")
    out = torch.full((gm.n, J), np.nan, dtype=torch.float64, device="cuda")
    L.mhd_ens_assemble_rhs(gm.handle, c, which, J, *args, ref)
    L.mhd_ens_assemble_rhs_noalloc(gm.handle, c, which, J, *args, out)
    torch.cuda.synchronize()
    return ref, out


def test_noalloc_rhs_equals_allocating_call_twice(L):
    from paper_2108_05110_amd.ensemble import Mesh
    cases = [(24, 40, 0, 11), (8, 5, 1, 12)]     # (N, J, which, seed): the second call is smaller
    for N, J, which, seed in cases:
        say(f"noalloc rhs: unit square {N}x{N}, J={J}, which={which}")
        pb = wl.manufactured(J=J, eps=0.3, dt=0.05)
        gm = Mesh(L.MHD_MESH_UNIT_SQUARE, N)
        ref, out = rhs_pair(L, gm, pb, which, seed)
        assert torch.isfinite(ref).all()
        assert torch.equal(ref, out), (ref - out).abs().max().item()
        gm.close()
