"""ctypes binding of libmhd_ens.so (argument marshalling only).

Every function here forwards to the C entry point of the same name declared
in include/mhd_ens.h; all numerical work happens in the library's HIP
kernels.  Device arrays are passed as raw pointers taken from torch tensors,
streams as the raw hipStream_t of a torch stream.  If the library is missing
the import fails loudly: there is no fallback path.
"""
from __future__ import annotations

import ctypes as C
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIBPATH = os.path.join(HERE, "libmhd_ens.so")

MHD_OK, MHD_EINVAL, MHD_ENOMEM, MHD_EHIP, MHD_ENOCONV, MHD_ESHAPE = 0, -1, -2, -3, -4, -5
MHD_FP64, MHD_FP32_IR = 0, 1
MHD_MESH_UNIT_SQUARE, MHD_MESH_STEP_CHANNEL = 0, 1
MHD_V_PROBLEM, MHD_W_PROBLEM = 0, 1
MHD_ELEMENT_TAYLOR_HOOD, MHD_ELEMENT_SCOTT_VOGELIUS = 0, 1

# Public symbols of include/mhd_ens.h (checked by the CPU test-suite).
EXPORTS = (
    "mhd_ens_mesh_counts", "mhd_ens_mesh", "mhd_ens_mesh_coords", "mhd_ens_mesh_elements", "mhd_ens_mesh_free",
    "mhd_ens_shared_create", "mhd_ens_shared_free", "mhd_ens_assemble_shared", "mhd_ens_shared_csr",
    "mhd_ens_assemble_rhs", "mhd_ens_assemble_rhs_noalloc", "mhd_ens_solve", "mhd_ens_ctx_create", "mhd_ens_ctx_free", "mhd_ens_step",
    "mhd_ens_spmm", "mhd_ens_timer_enable", "mhd_ens_timer_op", "mhd_ens_timer_read", "mhd_ens_last_error", "mhd_ens_version",
    "mhd_ens_adjoint_terminal", "mhd_ens_adjoint_step", "mhd_ens_adjoint_ic",
    "mhd_ens_group_create", "mhd_ens_group_step", "mhd_ens_group_free",
    "mhd_ens_autotune", "mhd_ens_set_plan", "mhd_ens_get_plan",
    "mhd_ens_prepare", "mhd_ens_ctx_prepare", "mhd_ens_alloc_stats",
)


TUNE_SADDLE, TUNE_RESIDUAL, TUNE_JACOBI_FIRST, TUNE_JACOBI = 0, 1, 2, 3
TUNE_OPS = {TUNE_SADDLE: "saddle", TUNE_RESIDUAL: "residual", TUNE_JACOBI_FIRST: "jacobi_first",
            TUNE_JACOBI: "jacobi"}


class TuneEntry(C.Structure):
    _fields_ = [("op", C.c_int32), ("word", C.c_int32), ("J", C.c_int32), ("vec", C.c_int32),
                ("group", C.c_int32), ("deep", C.c_int32), ("tile", C.c_int32), ("waves", C.c_int32),
                ("us", C.c_float),
                ("chosen", C.c_int32)]


class MeshDesc(C.Structure):
    _fields_ = [("kind", C.c_int), ("nx", C.c_int), ("natural_outflow", C.c_int), ("element", C.c_int)]


class MeshInfo(C.Structure):
    _fields_ = [("n_el", C.c_int64), ("nP2", C.c_int64), ("nP1", C.c_int64), ("n_u", C.c_int64),
                ("n", C.c_int64), ("nnz_A", C.c_int64), ("nnz_B", C.c_int64), ("nnz", C.c_int64),
                ("n_bd", C.c_int64), ("n_dir", C.c_int64), ("pin", C.c_int32), ("mg_levels", C.c_int32)]


class Coeffs(C.Structure):
    _fields_ = [("dt", C.c_double), ("mu", C.c_double), ("nu_bar", C.c_double), ("num_bar", C.c_double),
                ("convective", C.c_int)]


class CSRView(C.Structure):
    _fields_ = [("rowptr_A", C.c_void_p), ("col_A", C.c_void_p), ("rowptr_Bt", C.c_void_p),
                ("col_Bt", C.c_void_p), ("rowptr_B", C.c_void_p), ("col_B", C.c_void_p),
                ("val_A", C.c_void_p), ("val_Bt", C.c_void_p), ("val_B", C.c_void_p), ("diag_p", C.c_void_p),
                ("val_A32", C.c_void_p),
                ("nP2", C.c_int64), ("nP1", C.c_int64), ("nnz_A", C.c_int64), ("nnz_Bt", C.c_int64),
                ("nnz_B", C.c_int64)]


class SolverOpts(C.Structure):
    _fields_ = [("precision", C.c_int), ("rtol", C.c_double), ("inner_rtol", C.c_double), ("maxit", C.c_int),
                ("restart", C.c_int), ("jacobi_sweeps", C.c_int), ("check_every", C.c_int),
                ("cgs_passes", C.c_int), ("fixed_cycles", C.c_int), ("jacobi_omega", C.c_double),
                ("mg_unfused", C.c_int), ("mg_cycles", C.c_int), ("block_krylov", C.c_int),
                ("mg_post", C.c_int), ("keep_converged", C.c_int)]


class SolveStats(C.Structure):
    _fields_ = [("iters", C.c_int), ("cycles", C.c_int), ("max_relres", C.c_double), ("converged", C.c_int),
                ("nonfinite", C.c_int), ("relres", C.POINTER(C.c_double)), ("member_iters", C.POINTER(C.c_int32)),
                ("min_block_rank", C.c_int), ("norm_clamps", C.c_int), ("compacted", C.c_int)]


class CtxDesc(C.Structure):
    _fields_ = [("coeffs", Coeffs), ("solver", SolverOpts), ("J_max", C.c_int), ("adjoint", C.c_int),
                ("graph", C.c_int), ("serial", C.c_int)]


class AdjointInputs(C.Structure):
    _fields_ = [("nu", C.POINTER(C.c_double)), ("nu_m", C.POINTER(C.c_double)), ("fhat", C.c_void_p),
                ("J", C.c_int)]


class StepInputs(C.Structure):
    _fields_ = [("nu", C.POINTER(C.c_double)), ("nu_m", C.POINTER(C.c_double)), ("f1", C.c_void_p),
                ("f2", C.c_void_p), ("g_v", C.c_void_p), ("g_w", C.c_void_p), ("J", C.c_int)]


class StepStats(C.Structure):
    _fields_ = [("v", SolveStats), ("w", SolveStats), ("energy", C.c_double), ("warnings", C.c_int),
                ("min_alpha", C.c_double)]


MHD_WARN_ALPHA, MHD_WARN_MU, MHD_WARN_NONFINITE = 1, 2, 4


def _member_arrays(st, J):
    """Attaches host arrays for the per-member statistics (kept alive on st)."""
    st._keep = []
    for q in ((st.v, st.w) if isinstance(st, StepStats) else (st,)):
        r = (C.c_double * J)()
        it = (C.c_int32 * J)()
        q.relres = C.cast(r, C.POINTER(C.c_double))
        q.member_iters = C.cast(it, C.POINTER(C.c_int32))
        st._keep += [r, it]
    return st


def member_stats(q, J):
    """(relres, member_iters) lists of one subproblem's statistics."""
    return [q.relres[j] for j in range(J)], [q.member_iters[j] for j in range(J)]


_lib = None


def lib():
    """Loads libmhd_ens.so (raises if it was not built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIBPATH):
            raise RuntimeError(f"{LIBPATH} is missing: build it with python -m paper_2108_05110_amd.build")
        L = C.CDLL(LIBPATH)
        P, I = C.c_void_p, C.c_int
        sig = {
            "mhd_ens_mesh_counts": [C.POINTER(MeshDesc), C.POINTER(MeshInfo)],
            "mhd_ens_mesh": [C.POINTER(MeshDesc), C.POINTER(P), C.POINTER(MeshInfo)],
            "mhd_ens_mesh_coords": [P, P, P],
            "mhd_ens_mesh_elements": [P, P],
            "mhd_ens_mesh_free": [P],
            "mhd_ens_shared_create": [P, I, I, C.POINTER(P)],
            "mhd_ens_shared_free": [P],
            "mhd_ens_assemble_shared": [P, C.POINTER(Coeffs), P, I, P, P],
            "mhd_ens_shared_csr": [P, C.POINTER(CSRView)],
            "mhd_ens_assemble_rhs": [P, C.POINTER(Coeffs), I, I, P, P, P, P, P, P, P, I, P],
            "mhd_ens_assemble_rhs_noalloc": [P, C.POINTER(Coeffs), I, I, P, P, P, P, P, P, P, I, P],
            "mhd_ens_solve": [P, P, P, I, C.POINTER(SolverOpts), C.POINTER(SolveStats), P],
            "mhd_ens_ctx_create": [P, C.POINTER(CtxDesc), C.POINTER(P)],
            "mhd_ens_ctx_free": [P],
            "mhd_ens_step": [P, P, P, P, P, C.POINTER(StepInputs), C.POINTER(StepStats), P],
            "mhd_ens_spmm": [P, P, P, I, I, P],
            "mhd_ens_autotune": [P, I, I, C.POINTER(TuneEntry), I, C.POINTER(I), P],
            "mhd_ens_set_plan": [P, I, I, I, I, I, I, I, I],
            "mhd_ens_get_plan": [P, I, I, I, C.POINTER(TuneEntry)],
            "mhd_ens_prepare": [P, I, I, P],
            "mhd_ens_ctx_prepare": [P, I, P],
            "mhd_ens_alloc_stats": [C.POINTER(C.c_int64), C.POINTER(C.c_int64)],
            "mhd_ens_timer_enable": [I],
            "mhd_ens_timer_op": [I],
            "mhd_ens_adjoint_terminal": [P, P, P, P, P, I, P],
            "mhd_ens_adjoint_step": [P, P, P, P, P, P, P, P, P, C.POINTER(AdjointInputs), P,
                                     C.POINTER(StepStats), P],
            "mhd_ens_adjoint_ic": [P, P, P, P, I, C.c_double, P, I, P],
            "mhd_ens_group_create": [I, C.POINTER(P), C.POINTER(P)],
            "mhd_ens_group_step": [P, C.POINTER(P), C.POINTER(P), C.POINTER(P), C.POINTER(P),
                                   C.POINTER(StepInputs), P],
            "mhd_ens_group_free": [P],
            "mhd_ens_timer_read": [C.POINTER(C.c_double), C.POINTER(C.c_int64), C.POINTER(C.c_double),
                                   C.POINTER(C.c_double)],
        }
        for name, args in sig.items():
            f = getattr(L, name)
            f.argtypes = args
            f.restype = C.c_int
        L.mhd_ens_last_error.restype = C.c_char_p
        L.mhd_ens_last_error.argtypes = []
        L.mhd_ens_version.restype = C.c_char_p
        L.mhd_ens_version.argtypes = []
        _lib = L
    return _lib


class MhdError(RuntimeError):
    def __init__(self, name, status):
        msg = lib().mhd_ens_last_error().decode()
        super().__init__(f"{name} -> {status}: {msg}")
        self.status = status


def check(name, status, allow=(MHD_OK,)):
    if status not in allow:
        raise MhdError(name, status)
    return status


def ptr(t):
    """Raw device (or host) pointer of a tensor / None."""
    if t is None:
        return None
    return C.c_void_p(t.data_ptr())


def stream_ptr(stream=None):
    import torch
    s = stream if stream is not None else torch.cuda.current_stream()
    return C.c_void_p(s.cuda_stream)


# ------------------------------------------------------------------ same-name wrappers
def mhd_ens_mesh_counts(kind, nx, natural_outflow=0, element=0):
    d = MeshDesc(kind, nx, natural_outflow, element)
    info = MeshInfo()
    check("mhd_ens_mesh_counts", lib().mhd_ens_mesh_counts(C.byref(d), C.byref(info)))
    return info


def mhd_ens_mesh(kind, nx, natural_outflow=0, element=0):
    d = MeshDesc(kind, nx, natural_outflow, element)
    h = C.c_void_p()
    info = MeshInfo()
    check("mhd_ens_mesh", lib().mhd_ens_mesh(C.byref(d), C.byref(h), C.byref(info)))
    return h, info


def mhd_ens_mesh_coords(mesh, info):
    import numpy as np
    xy = np.zeros((info.nP2, 2), dtype=np.float64)
    dn = np.zeros(max(info.n_dir, 1), dtype=np.int32)
    check("mhd_ens_mesh_coords", lib().mhd_ens_mesh_coords(mesh, xy.ctypes.data_as(C.c_void_p),
                                                           dn.ctypes.data_as(C.c_void_p)))
    return xy, dn[:info.n_dir].copy()


def mhd_ens_mesh_elements(mesh, info):
    import numpy as np
    tri = np.zeros((info.n_el, 6), dtype=np.int32)
    check("mhd_ens_mesh_elements", lib().mhd_ens_mesh_elements(mesh, tri.ctypes.data_as(C.c_void_p)))
    return tri


def mhd_ens_mesh_free(mesh):
    check("mhd_ens_mesh_free", lib().mhd_ens_mesh_free(mesh))


def mhd_ens_shared_create(mesh, J_max, restart):
    h = C.c_void_p()
    check("mhd_ens_shared_create", lib().mhd_ens_shared_create(mesh, J_max, restart, C.byref(h)))
    return h


def mhd_ens_shared_free(A):
    check("mhd_ens_shared_free", lib().mhd_ens_shared_free(A))


def mhd_ens_assemble_shared(mesh, coeffs, z_other, J, A, stream=None):
    check("mhd_ens_assemble_shared",
          lib().mhd_ens_assemble_shared(mesh, C.byref(coeffs), ptr(z_other), J, A, stream_ptr(stream)))


def mhd_ens_shared_csr(A):
    v = CSRView()
    check("mhd_ens_shared_csr", lib().mhd_ens_shared_csr(A, C.byref(v)))
    return v


def _rhs_precision(rhs):
    import torch
    return MHD_FP32_IR if rhs.dtype == torch.float32 else MHD_FP64


def mhd_ens_assemble_rhs(mesh, coeffs, which, J, self_n, other_n, nu, nu_m, forcing, bc_vals, rhs, stream=None):
    """rhs: float64 or float32 tensor (n, J); the output precision follows its dtype."""
    check("mhd_ens_assemble_rhs",
          lib().mhd_ens_assemble_rhs(mesh, C.byref(coeffs), which, J, ptr(self_n), ptr(other_n), ptr(nu),
                                     ptr(nu_m), ptr(forcing), ptr(bc_vals), ptr(rhs), _rhs_precision(rhs),
                                     stream_ptr(stream)))


def mhd_ens_assemble_rhs_noalloc(mesh, coeffs, which, J, self_n, other_n, nu, nu_m, forcing, bc_vals, rhs,
                                 stream=None):
    check("mhd_ens_assemble_rhs_noalloc",
          lib().mhd_ens_assemble_rhs_noalloc(mesh, C.byref(coeffs), which, J, ptr(self_n), ptr(other_n), ptr(nu),
                                             ptr(nu_m), ptr(forcing), ptr(bc_vals), ptr(rhs), _rhs_precision(rhs),
                                             stream_ptr(stream)))


def mhd_ens_solve(A, rhs, x, J, opts, stream=None, allow_noconv=False):
    st = _member_arrays(SolveStats(), J)
    allow = (MHD_OK, MHD_ENOCONV) if allow_noconv else (MHD_OK,)
    rc = check("mhd_ens_solve", lib().mhd_ens_solve(A, ptr(rhs), ptr(x), J, C.byref(opts), C.byref(st),
                                                    stream_ptr(stream)), allow)
    return st, rc


def mhd_ens_ctx_create(mesh, desc):
    h = C.c_void_p()
    check("mhd_ens_ctx_create", lib().mhd_ens_ctx_create(mesh, C.byref(desc), C.byref(h)))
    return h


def mhd_ens_ctx_free(ctx):
    check("mhd_ens_ctx_free", lib().mhd_ens_ctx_free(ctx))


def mhd_ens_step(ctx, V, W, Q, R, inputs, stats=True, stream=None, allow_noconv=False):
    st = _member_arrays(StepStats(), inputs.J) if stats else None
    allow = (MHD_OK, MHD_ENOCONV) if allow_noconv else (MHD_OK,)
    check("mhd_ens_step", lib().mhd_ens_step(ctx, ptr(V), ptr(W), ptr(Q), ptr(R), C.byref(inputs),
                                             C.byref(st) if st is not None else None, stream_ptr(stream)), allow)
    return st


def mhd_ens_prepare(A, J, precision, stream=None):
    check("mhd_ens_prepare", lib().mhd_ens_prepare(A, J, precision, stream_ptr(stream)))


def mhd_ens_ctx_prepare(ctx, J, stream=None):
    check("mhd_ens_ctx_prepare", lib().mhd_ens_ctx_prepare(ctx, J, stream_ptr(stream)))


def mhd_ens_alloc_stats():
    n, b = C.c_int64(), C.c_int64()
    check("mhd_ens_alloc_stats", lib().mhd_ens_alloc_stats(C.byref(n), C.byref(b)))
    return n.value, b.value


def mhd_ens_spmm(A, x, y, J, precision, stream=None):
    check("mhd_ens_spmm", lib().mhd_ens_spmm(A, ptr(x), ptr(y), J, precision, stream_ptr(stream)))


def mhd_ens_autotune(A, J, precision, stream=None, cap=256):
    """Re-tunes the node-row kernels; returns one dict per timed candidate."""
    out = (TuneEntry * cap)()
    cnt = C.c_int(0)
    check("mhd_ens_autotune", lib().mhd_ens_autotune(A, J, precision, out, cap, C.byref(cnt), stream_ptr(stream)))
    return [dict(op=TUNE_OPS[e.op], word=e.word, J=e.J, vec=e.vec, group=e.group, deep=e.deep, tile=e.tile,
                 waves=e.waves, us=e.us, chosen=bool(e.chosen)) for e in out[:cnt.value]]


def mhd_ens_set_plan(A, J, precision, op, vec, group, deep=0, tile=0, waves=4):
    check("mhd_ens_set_plan", lib().mhd_ens_set_plan(A, J, precision, op, vec, group, deep, tile, waves))


def mhd_ens_get_plan(A, J, precision, op):
    e = TuneEntry()
    check("mhd_ens_get_plan", lib().mhd_ens_get_plan(A, J, precision, op, C.byref(e)))
    return dict(op=TUNE_OPS[e.op], word=e.word, J=e.J, vec=e.vec, group=e.group, deep=e.deep, tile=e.tile,
                waves=e.waves, us=e.us, chosen=bool(e.chosen))


def mhd_ens_plan(A, J, precision):
    """The plans of all four node-row operators, keyed by operator name."""
    return {TUNE_OPS[op]: mhd_ens_get_plan(A, J, precision, op) for op in TUNE_OPS}


def mhd_ens_timer_op(op):
    check("mhd_ens_timer_op", lib().mhd_ens_timer_op(op))


def mhd_ens_timer_enable(on=True):
    check("mhd_ens_timer_enable", lib().mhd_ens_timer_enable(1 if on else 0))


def mhd_ens_timer_read():
    ms, n, a, b = C.c_double(), C.c_int64(), C.c_double(), C.c_double()
    check("mhd_ens_timer_read", lib().mhd_ens_timer_read(C.byref(ms), C.byref(n), C.byref(a), C.byref(b)))
    return ms.value, n.value, a.value, b.value


def mhd_ens_adjoint_terminal(ctx, V, W, lamV, lamW, J, stream=None):
    check("mhd_ens_adjoint_terminal",
          lib().mhd_ens_adjoint_terminal(ctx, ptr(V), ptr(W), ptr(lamV), ptr(lamW), J, stream_ptr(stream)))


def mhd_ens_adjoint_step(ctx, V_n, W_n, V_np1, W_np1, lamV_np1, lamW_np1, lamV_n, lamW_n, inputs, grad,
                         stream=None, allow_noconv=False):
    st = StepStats()
    allow = (MHD_OK, MHD_ENOCONV) if allow_noconv else (MHD_OK,)
    check("mhd_ens_adjoint_step",
          lib().mhd_ens_adjoint_step(ctx, ptr(V_n), ptr(W_n), ptr(V_np1), ptr(W_np1), ptr(lamV_np1),
                                     ptr(lamW_np1), ptr(lamV_n), ptr(lamW_n), C.byref(inputs), ptr(grad),
                                     C.byref(st), stream_ptr(stream)), allow)
    return st


def mhd_ens_adjoint_ic(ctx, lamV0, lamW0, modes, nm, s_coupling, grad_ic, J, stream=None):
    check("mhd_ens_adjoint_ic",
          lib().mhd_ens_adjoint_ic(ctx, ptr(lamV0), ptr(lamW0), ptr(modes), nm, s_coupling, ptr(grad_ic), J,
                                   stream_ptr(stream)))


def mhd_ens_group_create(ctxs):
    arr = (C.c_void_p * len(ctxs))(*[c.value if isinstance(c, C.c_void_p) else c for c in ctxs])
    h = C.c_void_p()
    check("mhd_ens_group_create", lib().mhd_ens_group_create(len(ctxs), arr, C.byref(h)))
    return h


def mhd_ens_group_step(group, Vs, Ws, Qs, Rs, inputs, stream=None):
    n = len(Vs)
    mk = lambda ts: (C.c_void_p * n)(*[t.data_ptr() for t in ts])
    ins = (StepInputs * n)(*inputs)
    check("mhd_ens_group_step", lib().mhd_ens_group_step(group, mk(Vs), mk(Ws), mk(Qs), mk(Rs), ins,
                                                         stream_ptr(stream)))


def mhd_ens_group_free(group):
    check("mhd_ens_group_free", lib().mhd_ens_group_free(group))


def solver_opts(precision=MHD_FP64, rtol=None, inner_rtol=None, maxit=2000, restart=30, jacobi_sweeps=6,
                check_every=1, cgs_passes=0, fixed_cycles=0, jacobi_omega=0.0, mg_unfused=0, mg_cycles=0,
                block_krylov=0, mg_post=0, keep_converged=0):
    if rtol is None:
        rtol = 1e-12 if precision == MHD_FP64 else 1e-11
    if inner_rtol is None:
        inner_rtol = 1e-8 if precision == MHD_FP64 else 1e-4
    return SolverOpts(precision, rtol, inner_rtol, maxit, restart, jacobi_sweeps, check_every, cgs_passes,
                      fixed_cycles, jacobi_omega, mg_unfused, mg_cycles, block_krylov, mg_post, keep_converged)
