"""The library's Scott-Vogelius mesh (Alfeld refinement, Section 2), built by
its host code (tests/cpp/sv_mesh_dump.cpp compiled against csrc/mesh.cpp),
against the oracle's independently written refinement: counts, node
coordinates, elements as sets of node positions in the stated local order,
Dirichlet nodes, the pressure pin, and the interpolation of the unrefined
vertex grid into the discontinuous pressure space (exact for linear
functions)."""
import os
import shutil
import subprocess

import numpy as np
import pytest

from oracle import mesh as om

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_2108_05110_amd", "csrc")


@pytest.fixture(scope="module")
def dump_exe(tmp_path_factory):
    if shutil.which("g++") is None:
        pytest.skip("no host C++ compiler")
    exe = str(tmp_path_factory.mktemp("sv") / "sv_mesh_dump")
    subprocess.run(["g++", "-O1", "-std=c++17", "-I", CSRC, os.path.join(ROOT, "tests", "cpp", "sv_mesh_dump.cpp"),
                    os.path.join(CSRC, "mesh.cpp"), "-o", exe], check=True)
    return exe


def _read(exe, N, tmp_path):
    out = str(tmp_path / f"sv{N}.bin")
    subprocess.run([exe, str(N), out], check=True, timeout=120)
    raw = open(out, "rb").read()
    head = np.frombuffer(raw[:48], dtype=np.int64)
    nP2, nP1, n_el, levels, pin, nnzA = (int(v) for v in head)
    o = 48
    xy = np.frombuffer(raw[o:o + 16 * nP2], dtype=np.float64).reshape(nP2, 2); o += 16 * nP2
    tri = np.frombuffer(raw[o:o + 24 * n_el], dtype=np.int32).reshape(n_el, 6); o += 24 * n_el
    dirf = np.frombuffer(raw[o:o + nP2], dtype=np.uint8); o += nP2
    pv = np.frombuffer(raw[o:o + 8 * nP1], dtype=np.float64); o += 8 * nP1
    pv1 = np.frombuffer(raw[o:o + 8 * (nP1 // 3)], dtype=np.float64)
    return dict(nP2=nP2, nP1=nP1, n_el=n_el, levels=levels, pin=pin, xy=xy, tri=tri, dir=dirf, pv=pv, pv1=pv1)


def _keys(xy, h):
    return [tuple(int(round(c * 6 / h)) for c in p) for p in xy]


@pytest.mark.parametrize("N", [4, 8, 16])
def test_sv_mesh_matches_the_oracle_refinement(dump_exe, tmp_path, N):
    lib = _read(dump_exe, N, tmp_path)
    ref = om.alfeld(om.unit_square(N))
    h = 1.0 / N
    assert (lib["nP2"], lib["n_el"], lib["nP1"]) == (ref.nP2, ref.n_el, ref.nP1)
    # nodes: the same positions, numbered row-major on the sixth-step grid
    kl, kr = _keys(lib["xy"], h), _keys(ref.xy, h)
    assert np.abs(lib["xy"] - np.array(kl) * h / 6).max() < 1e-15
    assert set(kl) == set(kr)
    assert kl == sorted(kl, key=lambda p: (p[1], p[0]))
    # elements: the same node-position sextuples in the same local order
    # (v0, v1, v2, m01, m12, m20), counter-clockwise, in the same element order
    el_lib = [tuple(kl[i] for i in t) for t in lib["tri"]]
    el_ref = [tuple(kr[i] for i in t) for t in ref.tri]
    assert el_lib == el_ref
    p = lib["xy"][lib["tri"][:, :3]]
    two_a = (p[:, 1, 0] - p[:, 0, 0]) * (p[:, 2, 1] - p[:, 0, 1]) - (p[:, 2, 0] - p[:, 0, 0]) * (p[:, 1, 1] - p[:, 0, 1])
    assert np.all(two_a > 0)
    assert np.allclose(two_a.sum() / 2, 1.0, atol=1e-13)
    # Dirichlet nodes = boundary nodes (whole boundary Dirichlet)
    assert set(map(tuple, np.array(kl)[lib["dir"] == 1])) == set(kr[i] for i in ref.bnd)
    # the pin: pressure unknown 0, at vertex 0 of element 0, the corner (0, 0)
    assert lib["pin"] == 0 and kl[lib["tri"][0, 0]] == (0, 0)
    # the hierarchy's transfers are exact for x + 2y (the pinned unknowns' rows,
    # and the columns of pinned coarse unknowns, are empty): unrefined triangles ->
    # every element vertex, and vertex grid -> the unrefined triangles' vertices
    pxy = lib["xy"][lib["tri"][:, :3]].reshape(-1, 2)
    want = pxy[:, 0] + 2 * pxy[:, 1]
    if lib["levels"] > 1:
        assert lib["pv"][0] == 0.0
        assert np.abs(lib["pv"][1:] - want[1:]).max() < 1e-13
    if lib["levels"] > 2:
        w1 = lib["xy"][lib["tri"][:, 0]]          # vertex 0 of element 3E + q: vertex q of triangle E
        w1 = w1[:, 0] + 2 * w1[:, 1]
        assert lib["pv1"][0] == 0.0
        assert np.abs(lib["pv1"][1:] - w1[1:]).max() < 1e-13
    assert lib["levels"] == {4: 1, 8: 2, 16: 3}[N]
