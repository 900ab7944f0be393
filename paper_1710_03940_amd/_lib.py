"""ctypes binding of libdfamg.so: the C ABI declared in include/dfamg.h.

Argument marshalling only.  Every numerical step of setup and solve runs in
the library (host C++ for setup, HIP kernels on the GPU for the solve); if the
library is missing this module raises instead of falling back to anything.
"""
import ctypes
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libdfamg.so")

OK, EINVAL, ENOMEM, ESINGULAR, ENOCONV, EBREAKDOWN, ENAN, EHIP, ENOGPU = range(9)
STATUS_NAMES = {OK: "OK", EINVAL: "EINVAL", ENOMEM: "ENOMEM", ESINGULAR: "ESINGULAR",
                ENOCONV: "ENOCONV", EBREAKDOWN: "EBREAKDOWN", ENAN: "ENAN",
                EHIP: "EHIP", ENOGPU: "ENOGPU"}
SOLVER_CG, SOLVER_BICGSTAB, SOLVER_BICGSTAB2, SOLVER_FGMRES = 0, 1, 2, 3
COARSE_EXACT, COARSE_FP32, COARSE_CG = 0, 1, 2
PREC_FP64, PREC_MIXED = 0, 1
SMOOTHER_SPAI0, SMOOTHER_JACOBI, SMOOTHER_BLOCK_SPAI0 = 0, 1, 2
FORMAT_AUTO, FORMAT_CSR, FORMAT_SELL, FORMAT_CSR_GATHER, FORMAT_BSR4, FORMAT_COLUMN_TILED = 0, 1, 2, 3, 4, 5
PRECOND_AMG, PRECOND_NONE, PRECOND_SPAI0 = 0, 1, 2
OP_SPMV, OP_PROJECT, OP_PRECOND, OP_RECOVER = 0, 1, 2, 3
NOALLOC_MAX_N = 512
KERNEL_NAMES = ["spmv", "project", "update", "test", "presmooth0", "restrict0", "coarser",
                "prolong0", "postsmooth0", "direction", "restrict1", "deep", "up1"]

EXPORTED = [
    "dfamg_params_default", "dfamg_setup", "dfamg_setup_batched", "dfamg_solve",
    "dfamg_solve_batched", "dfamg_apply", "dfamg_get_stats", "dfamg_destroy",
    "dfamg_last_error", "dfamg_plan_create", "dfamg_plan_levels",
    "dfamg_plan_aggregates", "dfamg_plan_level_matrix",
    "dfamg_plan_coarse_operator", "dfamg_plan_destroy", "dfamg_coarse_inverse",
    "dfamg_dense_inverse", "dfamg_setup_schur", "dfamg_coarse_operator",
    "dfamg_dense_inverse_noalloc",
]


class DfamgError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"{STATUS_NAMES.get(status, status)}: {msg}")
        self.status = status


class Params(ctypes.Structure):
    _fields_ = [
        ("solver", ctypes.c_int32), ("maxiter", ctypes.c_int32),
        ("rtol", ctypes.c_double), ("precision", ctypes.c_int32),
        ("smoother", ctypes.c_int32), ("jacobi_omega", ctypes.c_double),
        ("coarse_enough", ctypes.c_int32), ("eps_strong", ctypes.c_double),
        ("max_levels", ctypes.c_int32), ("block_size", ctypes.c_int32),
        ("precond", ctypes.c_int32), ("spmv_format", ctypes.c_int32),
        ("autotune", ctypes.c_int32), ("graph_iters", ctypes.c_int32), ("host_threads", ctypes.c_int32),
        ("verbose", ctypes.c_int32), ("profile", ctypes.c_int32),
        ("restart", ctypes.c_int32), ("coarse_solve", ctypes.c_int32),
        ("coarse_rtol", ctypes.c_double), ("coarse_maxiter", ctypes.c_int32),
        ("flexible_cg", ctypes.c_int32), ("npre", ctypes.c_int32), ("npost", ctypes.c_int32),
        ("setup_device", ctypes.c_int32),
    ]


class Stats(ctypes.Structure):
    _fields_ = [
        ("n", ctypes.c_int64), ("nnz", ctypes.c_int64),
        ("nsys", ctypes.c_int32), ("nsub", ctypes.c_int32),
        ("ndv", ctypes.c_int32), ("m_total", ctypes.c_int32),
        ("nlevels_max", ctypes.c_int32),
        ("level_rows", ctypes.c_int64 * 20), ("level_nnz", ctypes.c_int64 * 20),
        ("level_p_nnz", ctypes.c_int64 * 20),
        ("format_outer", ctypes.c_int32), ("format_level", ctypes.c_int32 * 20),
        ("lanes_level", ctypes.c_int32 * 20),
        ("setup_host_s", ctypes.c_double), ("setup_device_s", ctypes.c_double),
        ("solve_s", ctypes.c_double), ("device_bytes", ctypes.c_int64),
        ("bytes_per_iter", ctypes.c_double),
        ("kernel_calls", ctypes.c_int64 * 16), ("kernel_ms", ctypes.c_double * 16),
        ("kernel_bytes", ctypes.c_double * 16), ("profile_in_graph", ctypes.c_int32),
        ("layouts", ctypes.c_char * 1024), ("outer_layout_bytes", ctypes.c_double),
        ("coarse_iters", ctypes.c_int64), ("schur_inner_iters", ctypes.c_int64 * 2),
        ("setup_hierarchy_s", ctypes.c_double), ("setup_hierarchy_device", ctypes.c_int32),
    ]


_lib = None


def load():
    """Load libdfamg.so; raises if it has not been built."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is missing: run `python -m paper_1710_03940_amd.build`")
    lib = ctypes.CDLL(LIB_PATH)
    P, I32, I64, D = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.c_double
    H = ctypes.c_void_p
    lib.dfamg_params_default.argtypes = [ctypes.POINTER(Params)]
    lib.dfamg_params_default.restype = None
    lib.dfamg_setup.argtypes = [ctypes.POINTER(Params), I64, P, P, P, P, I32, I32, P, P,
                                ctypes.POINTER(H)]
    lib.dfamg_setup_batched.argtypes = [ctypes.POINTER(Params), I32, P, I64, P, P, P, P,
                                        I32, I32, P, P, ctypes.POINTER(H)]
    lib.dfamg_solve.argtypes = [H, P, P, P, P, P, P, I32]
    lib.dfamg_solve_batched.argtypes = [H, P, P, P, P, P]
    lib.dfamg_apply.argtypes = [H, I32, P, P]
    lib.dfamg_get_stats.argtypes = [H, ctypes.POINTER(Stats)]
    lib.dfamg_destroy.argtypes = [H]
    lib.dfamg_last_error.argtypes = [H]
    lib.dfamg_last_error.restype = ctypes.c_char_p
    lib.dfamg_plan_create.argtypes = [ctypes.POINTER(Params), I32, P, I64, P, P, P, P,
                                      I32, I32, P, ctypes.POINTER(H)]
    lib.dfamg_plan_levels.argtypes = [H, I32, I32, P, P, P, P, P]
    lib.dfamg_plan_aggregates.argtypes = [H, I32, I32, I64, P, P]
    lib.dfamg_plan_level_matrix.argtypes = [H, I32, I32, I32, P, P, P, P, P, P]
    lib.dfamg_plan_coarse_operator.argtypes = [H, I32, P, P, I64]
    lib.dfamg_plan_destroy.argtypes = [H]
    lib.dfamg_coarse_inverse.argtypes = [H, I32, P, P, I64]
    lib.dfamg_coarse_operator.argtypes = [H, I32, P, P, I64]
    lib.dfamg_dense_inverse.argtypes = [P, I32, I32, P]
    lib.dfamg_dense_inverse_noalloc.argtypes = [P, I32, P, P]
    lib.dfamg_setup_schur.argtypes = [ctypes.POINTER(Params), I64, P, P, P, P, P, I32, I32, P, P,
                                      ctypes.POINTER(H)]
    for name in EXPORTED:
        f = getattr(lib, name)
        if name not in ("dfamg_params_default", "dfamg_last_error"):
            f.restype = ctypes.c_int
    _lib = lib
    return lib


def _ptr(a):
    return None if a is None else ctypes.c_void_p(a.ctypes.data)


def _check(status, handle=None):
    if status != OK:
        msg = load().dfamg_last_error(handle)
        raise DfamgError(status, msg.decode() if msg else "")


def dfamg_params_default(**overrides):
    p = Params()
    load().dfamg_params_default(ctypes.byref(p))
    for k, v in overrides.items():
        if not hasattr(p, k):
            raise AttributeError(k)
        setattr(p, k, v)
    return p


def _csr_arrays(A):
    ptr = np.ascontiguousarray(A.indptr, dtype=np.int64)
    col = np.ascontiguousarray(A.indices, dtype=np.int32)
    val = np.ascontiguousarray(A.data, dtype=np.float64)
    return ptr, col, val


def dfamg_setup(prm, A, part, nsub, Z, stream=None):
    """Returns an opaque handle (int).  A: scipy CSR; part: int32 [n];
    Z: float64 [n, ndv]; stream: hipStream_t as int (None = null stream)."""
    lib = load()
    ptr, col, val = _csr_arrays(A)
    part = np.ascontiguousarray(part, dtype=np.int32)
    Z = np.ascontiguousarray(Z, dtype=np.float64)
    h = ctypes.c_void_p()
    st = lib.dfamg_setup(ctypes.byref(prm), A.shape[0], _ptr(ptr), _ptr(col), _ptr(val),
                         _ptr(part), nsub, Z.shape[1], _ptr(Z) if Z.size else None,
                         ctypes.c_void_p(stream or 0), ctypes.byref(h))
    _check(st)
    return h.value


def dfamg_setup_batched(prm, sys_row_off, A, part, nsub, Z, stream=None):
    lib = load()
    ptr, col, val = _csr_arrays(A)
    part = np.ascontiguousarray(part, dtype=np.int32)
    Z = np.ascontiguousarray(Z, dtype=np.float64)
    off = np.ascontiguousarray(sys_row_off, dtype=np.int64)
    h = ctypes.c_void_p()
    st = lib.dfamg_setup_batched(ctypes.byref(prm), len(off) - 1, _ptr(off), A.shape[0],
                                 _ptr(ptr), _ptr(col), _ptr(val), _ptr(part), nsub,
                                 Z.shape[1], _ptr(Z) if Z.size else None,
                                 ctypes.c_void_p(stream or 0), ctypes.byref(h))
    _check(st)
    return h.value


def dfamg_solve(h, rhs_ptr, x_ptr, history_cap=0, raise_on_error=True):
    """rhs_ptr, x_ptr: device addresses (int) of n float64 values."""
    lib = load()
    iters = ctypes.c_int32()
    rr = ctypes.c_double()
    rt = ctypes.c_double()
    hist = np.zeros(max(history_cap, 1))
    st = lib.dfamg_solve(ctypes.c_void_p(h), ctypes.c_void_p(rhs_ptr), ctypes.c_void_p(x_ptr),
                         ctypes.byref(iters), ctypes.byref(rr), ctypes.byref(rt),
                         _ptr(hist) if history_cap else None, history_cap)
    if raise_on_error and st not in (OK, ENOCONV):
        _check(st, ctypes.c_void_p(h))
    out = {"status": st, "iters": iters.value, "relres": rr.value, "relres_true": rt.value}
    if history_cap:
        out["history"] = hist[:min(history_cap, iters.value + 1)].copy()
    return out


def dfamg_solve_batched(h, rhs_ptr, x_ptr, nsys):
    lib = load()
    iters = np.zeros(nsys, dtype=np.int32)
    rt = np.zeros(nsys)
    status = np.zeros(nsys, dtype=np.int32)
    st = lib.dfamg_solve_batched(ctypes.c_void_p(h), ctypes.c_void_p(rhs_ptr),
                                 ctypes.c_void_p(x_ptr), _ptr(iters), _ptr(rt), _ptr(status))
    if st not in (OK, ENOCONV):
        _check(st, ctypes.c_void_p(h))
    return {"status": st, "iters": iters, "relres_true": rt, "sys_status": status}


def dfamg_apply(h, op, in_ptr, out_ptr):
    st = load().dfamg_apply(ctypes.c_void_p(h), op, ctypes.c_void_p(in_ptr), ctypes.c_void_p(out_ptr))
    _check(st, ctypes.c_void_p(h))


def dfamg_get_stats(h):
    s = Stats()
    _check(load().dfamg_get_stats(ctypes.c_void_p(h), ctypes.byref(s)), ctypes.c_void_p(h))
    L = s.nlevels_max
    return {"n": s.n, "nnz": s.nnz, "nsys": s.nsys, "nsub": s.nsub, "ndv": s.ndv,
            "m_total": s.m_total, "nlevels_max": L,
            "level_rows": list(s.level_rows[:L]), "level_nnz": list(s.level_nnz[:L]),
            "level_p_nnz": list(s.level_p_nnz[:L]),
            "format_outer": s.format_outer, "format_level": list(s.format_level[:L]),
            "lanes_level": list(s.lanes_level[:L]),
            "setup_host_s": s.setup_host_s, "setup_device_s": s.setup_device_s,
            "solve_s": s.solve_s, "device_bytes": s.device_bytes,
            "bytes_per_iter": s.bytes_per_iter, "profile_in_graph": bool(s.profile_in_graph),
            "layouts": s.layouts.decode(), "outer_layout_bytes": s.outer_layout_bytes,
            "coarse_iters": int(s.coarse_iters),
            "schur_inner_iters": [int(s.schur_inner_iters[0]), int(s.schur_inner_iters[1])],
            "setup_hierarchy_s": float(s.setup_hierarchy_s),
            "setup_hierarchy_device": int(s.setup_hierarchy_device),
            "kernels": {name: {"calls": int(s.kernel_calls[i]), "ms": float(s.kernel_ms[i]),
                               "bytes": float(s.kernel_bytes[i])}
                        for i, name in enumerate(KERNEL_NAMES)}}


def dfamg_destroy(h):
    if h:
        load().dfamg_destroy(ctypes.c_void_p(h))


def dfamg_last_error(h=None):
    msg = load().dfamg_last_error(ctypes.c_void_p(h) if h else None)
    return msg.decode() if msg else ""


# --------------------------------------------------------------------------
# host-only plan inspection (no GPU needed)
# --------------------------------------------------------------------------

def dfamg_plan_create(prm, A, part, nsub, Z, sys_row_off=None):
    lib = load()
    ptr, col, val = _csr_arrays(A)
    part = np.ascontiguousarray(part, dtype=np.int32)
    Z = np.ascontiguousarray(Z, dtype=np.float64)
    off = None if sys_row_off is None else np.ascontiguousarray(sys_row_off, dtype=np.int64)
    nsys = 1 if off is None else len(off) - 1
    h = ctypes.c_void_p()
    st = lib.dfamg_plan_create(ctypes.byref(prm), nsys, _ptr(off), A.shape[0], _ptr(ptr),
                               _ptr(col), _ptr(val), _ptr(part), nsub, Z.shape[1],
                               _ptr(Z) if Z.size else None, ctypes.byref(h))
    _check(st)
    return h.value


def dfamg_plan_levels(p, sub, cap=20):
    nl = ctypes.c_int32()
    rows = np.zeros(cap, dtype=np.int64)
    nnz = np.zeros(cap, dtype=np.int64)
    pnnz = np.zeros(cap, dtype=np.int64)
    om = np.zeros(cap)
    _check(load().dfamg_plan_levels(ctypes.c_void_p(p), sub, cap, ctypes.byref(nl), _ptr(rows),
                                    _ptr(nnz), _ptr(pnnz), _ptr(om)))
    L = nl.value
    return [(int(rows[l]), int(nnz[l]), int(pnnz[l]), float(om[l])) for l in range(L)]


def dfamg_plan_aggregates(p, sub, level):
    lib = load()
    cnt = ctypes.c_int64()
    _check(lib.dfamg_plan_aggregates(ctypes.c_void_p(p), sub, level, 0, None, ctypes.byref(cnt)))
    agg = np.zeros(cnt.value, dtype=np.int32)
    _check(lib.dfamg_plan_aggregates(ctypes.c_void_p(p), sub, level, cnt.value, _ptr(agg),
                                     ctypes.byref(cnt)))
    return agg


def dfamg_plan_level_matrix(p, sub, level, which):
    """Returns (row_ptr, col, val, shape) of A_l (which=0), P_l (which=1),
    B_l = R_l (I - A_l diag(m_l)) (which=2) or the smoother M_l (which=3)."""
    lib = load()
    nr, nc, nz = ctypes.c_int64(), ctypes.c_int64(), ctypes.c_int64()
    _check(lib.dfamg_plan_level_matrix(ctypes.c_void_p(p), sub, level, which, ctypes.byref(nr),
                                       ctypes.byref(nc), ctypes.byref(nz), None, None, None))
    ptr = np.zeros(nr.value + 1, dtype=np.int64)
    col = np.zeros(nz.value, dtype=np.int32)
    val = np.zeros(nz.value)
    _check(lib.dfamg_plan_level_matrix(ctypes.c_void_p(p), sub, level, which, None, None, None,
                                       _ptr(ptr), _ptr(col), _ptr(val)))
    return ptr, col, val, (nr.value, nc.value)


def dfamg_plan_coarse_operator(p, sys=0):
    lib = load()
    m = ctypes.c_int32()
    _check(lib.dfamg_plan_coarse_operator(ctypes.c_void_p(p), sys, ctypes.byref(m), None, 0))
    E = np.zeros((m.value, m.value))
    _check(lib.dfamg_plan_coarse_operator(ctypes.c_void_p(p), sys, ctypes.byref(m), _ptr(E),
                                          E.size))
    return E


def dfamg_setup_schur(prm, A, pmask, part, nsub, Z, stream=None):
    """Schur pressure-correction handle.  A: scipy CSR of the whole system;
    pmask: nonzero for pressure unknowns; part / Z: subdomain ids and
    deflation vectors of the pressure unknowns (ascending index order)."""
    lib = load()
    ptr, col, val = _csr_arrays(A)
    pmask = np.ascontiguousarray(pmask, dtype=np.int32)
    part = np.ascontiguousarray(part, dtype=np.int32)
    Z = np.ascontiguousarray(Z, dtype=np.float64)
    h = ctypes.c_void_p()
    st = lib.dfamg_setup_schur(ctypes.byref(prm), A.shape[0], _ptr(ptr), _ptr(col), _ptr(val), _ptr(pmask),
                               _ptr(part), int(nsub), Z.shape[1], _ptr(Z),
                               ctypes.c_void_p(stream or 0), ctypes.byref(h))
    _check(st)
    return h.value


def dfamg_coarse_inverse(h, sys=0):
    """E^{-1} of system `sys` as held on the device (numpy array)."""
    lib = load()
    m = ctypes.c_int32()
    _check(lib.dfamg_coarse_inverse(ctypes.c_void_p(h), sys, ctypes.byref(m), None, 0))
    X = np.zeros((m.value, m.value))
    _check(lib.dfamg_coarse_inverse(ctypes.c_void_p(h), sys, ctypes.byref(m), _ptr(X), X.size))
    return X


def dfamg_coarse_operator(h, sys=0):
    """E of system `sys` assembled on the device from the handle's operator."""
    lib = load()
    m = ctypes.c_int32()
    _check(lib.dfamg_coarse_operator(ctypes.c_void_p(h), sys, ctypes.byref(m), None, 0))
    E = np.zeros((m.value, m.value))
    _check(lib.dfamg_coarse_operator(ctypes.c_void_p(h), sys, ctypes.byref(m), _ptr(E), E.size))
    return E


def dfamg_dense_inverse(a, method=0):
    """Inverse of a dense float64 matrix computed on the GPU (method 0 blocked,
    1 unblocked)."""
    lib = load()
    a = np.ascontiguousarray(a, dtype=np.float64)
    out = np.zeros_like(a)
    _check(lib.dfamg_dense_inverse(_ptr(a), a.shape[0], method, _ptr(out)))
    return out


def dfamg_dense_inverse_noalloc(a, out, stream=None):
    """Inverse of the n x n float64 device tensor `a` into the device tensor
    `out`, computed without any device allocation by the library (method 1 of
    dfamg_dense_inverse); `stream` is a torch stream (default: current)."""
    import torch
    if not (a.is_cuda and out.is_cuda and a.dtype == torch.float64 and out.dtype == torch.float64
            and a.is_contiguous() and out.is_contiguous() and a.dim() == 2 and a.shape[0] == a.shape[1]
            and out.shape == a.shape):
        raise ValueError("a and out must be contiguous square float64 CUDA tensors of the same shape")
    st = stream if stream is not None else torch.cuda.current_stream(a.device)
    _check(load().dfamg_dense_inverse_noalloc(ctypes.c_void_p(a.data_ptr()), a.shape[0],
                                              ctypes.c_void_p(out.data_ptr()),
                                              ctypes.c_void_p(st.cuda_stream)))
    return out


def dfamg_plan_destroy(p):
    if p:
        load().dfamg_plan_destroy(ctypes.c_void_p(p))
