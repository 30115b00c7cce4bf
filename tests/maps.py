"""Test helpers: map GPU node numbering to the oracle's by coordinates, rebuild
the GPU's compact saddle-point operator as a scipy matrix, and norms."""
import numpy as np
import scipy.sparse as sp


def node_map(xy_gpu, xy_orc, h):
    """perm[i_gpu] = i_orc for P2 nodes (coordinates on the half-step grid)."""
    s = 2.0 / h
    key = lambda xy: np.round(xy[:, 0] * s).astype(np.int64) * 1000003 + np.round(xy[:, 1] * s).astype(np.int64)
    ko = {k: i for i, k in enumerate(key(xy_orc))}
    return np.array([ko[k] for k in key(xy_gpu)])


def p1_map(xy_gpu, orc_mesh, h):
    """P1 nodes: GPU P1 node k is the k-th P2 node at an even half-step position."""
    s = 2.0 / h
    ij = np.round(xy_gpu * s).astype(np.int64)
    verts = np.nonzero((ij[:, 0] % 2 == 0) & (ij[:, 1] % 2 == 0))[0]
    pm = node_map(xy_gpu[verts], orc_mesh.xy[:orc_mesh.nV], h)
    return pm


def unknown_perm(pmap2, pmap1, nP2_orc):
    """GPU unknown index -> oracle unknown index."""
    vel = np.stack([2 * pmap2, 2 * pmap2 + 1], axis=1).ravel()
    return np.concatenate([vel, 2 * nP2_orc + pmap1])


def csr_from_view(torch, v):
    """Full saddle-point matrix (GPU numbering) from the compact device arrays."""
    import ctypes as C

    import ctypes as C
    hip = C.CDLL("libamdhip64.so")
    hip.hipMemcpy.argtypes = [C.c_void_p, C.c_void_p, C.c_size_t, C.c_int]
    hip.hipMemcpy.restype = C.c_int
    torch.cuda.synchronize()

    def dev(ptr, n, dtype):
        out = np.empty(n, dtype=dtype)
        rc = hip.hipMemcpy(out.ctypes.data, ptr, out.nbytes, 2)     # device to host
        assert rc == 0, rc
        return out

    nP2, nP1 = v.nP2, v.nP1
    Arp = dev(v.rowptr_A, nP2 + 1, np.int32)
    Acol = dev(v.col_A, v.nnz_A, np.int32)
    Aval = dev(v.val_A, v.nnz_A, np.float64)
    Btrp = dev(v.rowptr_Bt, nP2 + 1, np.int32)
    Btcol = dev(v.col_Bt, v.nnz_Bt, np.int32)
    Btval = dev(v.val_Bt, 2 * v.nnz_Bt, np.float64)
    Brp = dev(v.rowptr_B, nP1 + 1, np.int32)
    Bcol = dev(v.col_B, v.nnz_B, np.int32)
    Bval = dev(v.val_B, 2 * v.nnz_B, np.float64)
    dp = dev(v.diag_p, nP1, np.float64)
    rows, cols, vals = [], [], []
    rA = np.repeat(np.arange(nP2), np.diff(Arp))
    for c in (0, 1):
        rows.append(2 * rA + c)
        cols.append(2 * Acol + c)
        vals.append(Aval)
    rBt = np.repeat(np.arange(nP2), np.diff(Btrp))
    for c in (0, 1):
        rows.append(2 * rBt + c)
        cols.append(2 * nP2 + Btcol)
        vals.append(Btval[c::2])
    rB = np.repeat(np.arange(nP1), np.diff(Brp))
    for c in (0, 1):
        rows.append(2 * nP2 + rB)
        cols.append(2 * Bcol + c)
        vals.append(Bval[c::2])
    rows.append(2 * nP2 + np.arange(nP1))
    cols.append(2 * nP2 + np.arange(nP1))
    vals.append(dp)
    n = 2 * nP2 + nP1
    S = sp.coo_matrix((np.concatenate(vals), (np.concatenate(rows), np.concatenate(cols))), shape=(n, n)).tocsr()
    S.eliminate_zeros()
    return S


def mass_rel_err(ens, Za, Zb):
    """||a - b||_M / ||b||_M over all members and components (P2 mass, oracle numbering)."""
    num = den = 0.0
    for j in range(Za.shape[2]):
        d = (Za[:, :, j] - Zb[:, :, j]).ravel()
        b = Zb[:, :, j].ravel()
        num += d @ (ens.M2 @ d)
        den += b @ (ens.M2 @ b)
    return float(np.sqrt(num / den))
