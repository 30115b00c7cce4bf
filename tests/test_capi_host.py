"""Host-side checks of libmhd_ens.so that need no GPU: the library loads, exports
every entry point the public header declares, computes mesh counts that match
closed forms, and rejects invalid arguments before touching a device."""
import os
import re

import pytest

from paper_2108_05110_amd import _lib as L

HEADER = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))), "include", "mhd_ens.h")


def declared():
    txt = open(HEADER).read()
    return sorted(set(re.findall(r"\b(mhd_ens_[a-z0-9_]+)\s*\(", txt)))


def test_header_symbols_exported():
    lib = L.lib()
    names = declared()
    assert len(names) >= 10
    for n in names:
        assert hasattr(lib, n), n
    assert set(names) == set(L.EXPORTS)
    assert lib.mhd_ens_version().startswith(b"mhd_ens")


@pytest.mark.parametrize("N", [1, 2, 5, 16, 128])
def test_unit_square_counts(N):
    i = L.mhd_ens_mesh_counts(L.MHD_MESH_UNIT_SQUARE, N)
    assert i.n_el == 2 * N * N
    assert i.nP2 == (2 * N + 1) ** 2 and i.nP1 == (N + 1) ** 2
    assert i.n == 2 * i.nP2 + i.nP1
    assert i.nnz_A == 46 * N * N + 16 * N + 1
    assert i.nnz_B == 19 * N * N + 10 * N + 1
    assert i.nnz == 2 * i.nnz_A + 4 * i.nnz_B + 1
    assert i.n_bd == 8 * N and i.n_dir == 8 * N and i.pin == 0


def test_step_channel_counts():
    m = 16
    i = L.mhd_ens_mesh_counts(L.MHD_MESH_STEP_CHANNEL, m, 1)
    assert i.nP1 == (30 * m + 1) * (10 * m + 1) - m * m
    assert i.n == 692099 and i.nnz == 12882438
    assert i.pin == -1
    # Dirichlet nodes: boundary minus the outflow edge x = 30 (2*10*m + 1 nodes)
    assert i.n_dir == i.n_bd - (2 * 10 * m + 1)
    j = L.mhd_ens_mesh_counts(L.MHD_MESH_STEP_CHANNEL, m, 0)
    assert j.n_dir == j.n_bd and j.pin == 0


@pytest.mark.parametrize("kind,nx,out", [(7, 4, 0), (0, 0, 0), (0, 5000, 0), (0, 4, 1)])
def test_invalid_mesh_rejected(kind, nx, out):
    with pytest.raises(L.MhdError) as e:
        L.mhd_ens_mesh_counts(kind, nx, out)
    assert e.value.status == L.MHD_EINVAL


def test_null_handles_rejected_without_device():
    lib = L.lib()
    import ctypes as C
    assert lib.mhd_ens_mesh(None, None, None) == L.MHD_EINVAL
    assert lib.mhd_ens_shared_create(None, 4, 4, C.byref(C.c_void_p())) == L.MHD_EINVAL
    assert lib.mhd_ens_solve(None, None, None, 1, None, None, None) == L.MHD_EINVAL
    assert lib.mhd_ens_step(None, None, None, None, None, None, None, None) == L.MHD_EINVAL
    assert lib.mhd_ens_mesh_free(None) == L.MHD_OK
    assert b"null" in lib.mhd_ens_last_error()


def _patterns(ms):
    """Distinct P2-P2 pairs and pressure-P2 pairs that share an element."""
    aa, bb = set(), set()
    for e, t in enumerate(ms.tri):
        for a in t:
            for b in t:
                aa.add((a, b))
            for k in ms.ptri[e]:
                bb.add((k, a))
    return len(aa), len(bb)


@pytest.mark.parametrize("kind,nx,outflow", [(0, 2, 0), (0, 4, 0), (0, 8, 0), (1, 1, 1), (1, 2, 0)])
def test_scott_vogelius_counts_match_the_oracle_refinement(kind, nx, outflow):
    """Counts of the library's Scott-Vogelius meshes (built on the host) against
    the oracle's barycentric refinement: elements, nodes, discontinuous pressure
    unknowns, the P2 and divergence patterns, boundary and Dirichlet nodes."""
    from oracle import mesh as om
    i = L.mhd_ens_mesh_counts(kind, nx, outflow, L.MHD_ELEMENT_SCOTT_VOGELIUS)
    base = om.unit_square(nx) if kind == 0 else om.step_channel(nx)
    ms = om.alfeld(base)
    assert (i.n_el, i.nP2, i.nP1, i.n) == (ms.n_el, ms.nP2, ms.nP1, ms.n)
    assert i.nP1 == 3 * i.n_el
    nA, nB = _patterns(ms)
    assert (i.nnz_A, i.nnz_B) == (nA, nB)
    assert i.nnz == 2 * i.nnz_A + 4 * i.nnz_B + (1 if i.pin >= 0 else 0)
    assert i.n_bd == len(ms.bnd)
    assert i.pin == (-1 if outflow else 0)
    if not outflow:
        assert i.n_dir == i.n_bd


def test_scott_vogelius_rejects_an_unknown_element():
    with pytest.raises(RuntimeError):
        L.mhd_ens_mesh_counts(L.MHD_MESH_UNIT_SQUARE, 4, 0, 7)
