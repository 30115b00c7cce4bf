"""HIP-graph step and multi-ensemble group launch: replays reproduce eager
fixed-schedule steps bitwise (replayed several times with eager work between
the replays) and stay within the FP32+IR bar against the oracle."""
import sys

import numpy as np
import pytest

import workloads as wl
from oracle import mesh as om, scheme
from tests.maps import mass_rel_err, node_map

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


def fixed_opts(L, precision=1):
    return L.solver_opts(precision, restart=10, fixed_cycles=3)


def test_graph_replay_bitwise_equals_eager(L):
    from paper_2108_05110_amd.ensemble import Mesh, Stepper
    say("graph vs eager")
    pb = wl.cavity(J=5, s=0.1, dt=0.01, ic_amp=1e-2)
    gm = Mesh(L.MHD_MESH_UNIT_SQUARE, 16)
    eager = Stepper(gm, pb, opts=fixed_opts(L))
    graph = Stepper(gm, pb, opts=fixed_opts(L), graph=True)
    junk = torch.ones(1 << 20, dtype=torch.float64, device="cuda")
    for n in range(4):
        eager.step(stats=False)
        graph.step(stats=False)
        junk.mul_(1.0001).add_(0.5)          # eager work between the replays
        torch.cuda.synchronize()
        assert torch.equal(eager.V, graph.V) and torch.equal(eager.W, graph.W), n
        assert torch.equal(eager.Q, graph.Q) and torch.equal(eager.R, graph.R), n
    eager.close()
    graph.close()
    gm.close()


def test_graph_fixed_schedule_accuracy(L):
    from paper_2108_05110_amd.ensemble import Mesh, Stepper
    say("graph accuracy")
    N = 16
    pb = wl.cavity(J=5, s=0.1, dt=0.01, ic_amp=1e-2)
    gm = Mesh(L.MHD_MESH_UNIT_SQUARE, N)
    stp = Stepper(gm, pb, opts=fixed_opts(L), graph=True)
    om_ = om.unit_square(N)
    ens = scheme.Ensemble(om_, pb)
    pm2 = node_map(gm.xy, om_.xy, 1.0 / N)
    V, W = pb.ic(om_.xy)
    for n in range(3):
        stp.step(stats=False)
        V, W, _, _ = ens.step(V, W, (n + 1) * pb.dt, shared_lu=True)
        Vg = np.zeros_like(V)
        Vg[pm2] = stp.V.cpu().numpy()
        err = mass_rel_err(ens, Vg, V)
        say("  step", n + 1, err)
        assert err <= 1e-6
    stp.close()
    gm.close()


def test_group_launch_equals_individual_steps(L):
    from paper_2108_05110_amd.ensemble import Mesh, Stepper
    say("group launch")
    pa = wl.cavity(J=4, s=0.1, dt=0.01, ic_amp=1e-2, cfg=5)
    pbb = wl.cavity(J=3, s=1.0, dt=0.01, ic_amp=1e-2, cfg=6)
    ma, mb = Mesh(L.MHD_MESH_UNIT_SQUARE, 16), Mesh(L.MHD_MESH_UNIT_SQUARE, 8)
    ref = [Stepper(ma, pa, opts=fixed_opts(L)), Stepper(mb, pbb, opts=fixed_opts(L))]
    grp = [Stepper(ma, pa, opts=fixed_opts(L)), Stepper(mb, pbb, opts=fixed_opts(L))]
    for s in grp:
        s.set_data(s.pb.dt)
    g = L.mhd_ens_group_create([s.ctx for s in grp])
    stream = torch.cuda.Stream()
    for n in range(3):
        for s in ref:
            s.step(stats=False)
        torch.cuda.synchronize()
        L.mhd_ens_group_step(g, [s.V for s in grp], [s.W for s in grp], [s.Q for s in grp], [s.R for s in grp],
                             [s.inputs() for s in grp], stream=stream)
        stream.synchronize()
        for r, s in zip(ref, grp):
            assert torch.equal(r.V, s.V) and torch.equal(r.W, s.W), n
    L.mhd_ens_group_free(g)
    for s in ref + grp:
        s.close()
    ma.close()
    mb.close()


def test_group_on_one_mesh_with_different_viscosities(L):
    """Two ensembles on one mesh whose mean viscosities differ (each shared
    matrix handle keeps its own Schur-approximation values): one group launch
    equals the two contexts stepped alone, bitwise, over three steps, and the
    alternating contexts keep their values (no refresh between their steps)."""
    from paper_2108_05110_amd.ensemble import Mesh, Stepper
    say("group, one mesh, different viscosities")
    pa = wl.cavity(J=4, s=0.1, dt=0.01, ic_amp=1e-2, cfg=7, nu_mean=1e-2, num_mean=1e-2)
    pbb = wl.cavity(J=4, s=0.1, dt=0.01, ic_amp=1e-2, cfg=8, nu_mean=2e-3, num_mean=3e-3)
    m = Mesh(L.MHD_MESH_UNIT_SQUARE, 16)
    ref = [Stepper(m, pa, opts=fixed_opts(L)), Stepper(m, pbb, opts=fixed_opts(L))]
    grp = [Stepper(m, pa, opts=fixed_opts(L)), Stepper(m, pbb, opts=fixed_opts(L))]
    for s in grp:
        s.set_data(s.pb.dt)
    g = L.mhd_ens_group_create([s.ctx for s in grp])
    stream = torch.cuda.Stream()
    for n in range(3):
        for s in ref:                 # alternate the two contexts on the one mesh
            s.step(stats=False)
        torch.cuda.synchronize()
        L.mhd_ens_group_step(g, [s.V for s in grp], [s.W for s in grp], [s.Q for s in grp], [s.R for s in grp],
                             [s.inputs() for s in grp], stream=stream)
        stream.synchronize()
        for r, s in zip(ref, grp):
            assert torch.equal(r.V, s.V) and torch.equal(r.W, s.W), n
    assert not torch.equal(grp[0].V, grp[1].V)
    L.mhd_ens_group_free(g)
    for s in ref + grp:
        s.close()
    m.close()
