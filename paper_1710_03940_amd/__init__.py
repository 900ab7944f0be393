"""MI355X-native subdomain-deflated local-AMG Krylov solver (Python binding).

The solver itself is the C ABI library `libdfamg.so` (host C++ setup, HIP
kernels for gfx950); this package only marshals arguments.  PyTorch supplies
device memory and the stream.

    from paper_1710_03940_amd import Solver
    S = Solver(A, part, nsub, Z, precision="mixed")
    info = S.solve(b_dev, x_dev)      # torch float64 CUDA tensors
"""
from . import _lib
from ._lib import (DfamgError, dfamg_params_default, dfamg_setup, dfamg_setup_batched,
                   dfamg_solve, dfamg_solve_batched, dfamg_apply, dfamg_get_stats,
                   dfamg_destroy, dfamg_last_error, dfamg_plan_create, dfamg_plan_levels,
                   dfamg_plan_aggregates, dfamg_plan_level_matrix,
                   dfamg_plan_coarse_operator, dfamg_plan_destroy, dfamg_coarse_inverse,
                   dfamg_dense_inverse, dfamg_setup_schur, dfamg_coarse_operator,
                   dfamg_dense_inverse_noalloc)

__all__ = ["Solver", "BatchedSolver", "SchurSolver", "make_params", "DfamgError"] + [
    n for n in dir(_lib) if n.startswith("dfamg_")]

_ENUMS = {
    "solver": {"cg": _lib.SOLVER_CG, "bicgstab": _lib.SOLVER_BICGSTAB, "bicgstab2": _lib.SOLVER_BICGSTAB2,
               "fgmres": _lib.SOLVER_FGMRES},
    "coarse_solve": {"exact": _lib.COARSE_EXACT, "fp32": _lib.COARSE_FP32, "cg": _lib.COARSE_CG},
    "precision": {"fp64": _lib.PREC_FP64, "mixed": _lib.PREC_MIXED},
    "smoother": {"spai0": _lib.SMOOTHER_SPAI0, "jacobi": _lib.SMOOTHER_JACOBI,
                 "block_spai0": _lib.SMOOTHER_BLOCK_SPAI0},
    "spmv_format": {"auto": _lib.FORMAT_AUTO, "csr": _lib.FORMAT_CSR, "sell": _lib.FORMAT_SELL,
                    "csr_gather": _lib.FORMAT_CSR_GATHER, "bsr4": _lib.FORMAT_BSR4,
                    "column_tiled": _lib.FORMAT_COLUMN_TILED},
    "precond": {"amg": _lib.PRECOND_AMG, "none": _lib.PRECOND_NONE, "spai0": _lib.PRECOND_SPAI0},
}


def make_params(**kw):
    """dfamg_params with defaults; string values are mapped to the enums."""
    conv = {}
    for k, v in kw.items():
        if k in _ENUMS and isinstance(v, str):
            v = _ENUMS[k][v]
        conv[k] = v
    return dfamg_params_default(**conv)


def _stream():
    import torch
    return torch.cuda.current_stream().cuda_stream


def _dev_ptr(t, n):
    import torch
    if not (t.is_cuda and t.dtype == torch.float64 and t.is_contiguous() and t.numel() == n):
        raise ValueError("expected a contiguous float64 CUDA tensor of length n")
    return t.data_ptr()


class Solver:
    """Setup once (host hierarchy + device upload), solve many right-hand sides."""

    def __init__(self, A, part, nsub, Z, **params):
        self.n = A.shape[0]
        self.params = make_params(**params)
        self.h = dfamg_setup(self.params, A, part, nsub, Z, stream=_stream())

    def solve(self, b, x, history=True):
        cap = self.params.maxiter + 1 if history else 0
        return dfamg_solve(self.h, _dev_ptr(b, self.n), _dev_ptr(x, self.n), history_cap=cap)

    def apply(self, op, v, out):
        dfamg_apply(self.h, op, _dev_ptr(v, self.n), _dev_ptr(out, self.n))

    def stats(self):
        return dfamg_get_stats(self.h)

    def coarse_operator(self, sys=0):
        """E of one system assembled on the device (host numpy copy)."""
        return dfamg_coarse_operator(self.h, sys)

    def coarse_inverse(self, sys=0):
        """E^{-1} of one system as the device holds it (host numpy copy)."""
        return dfamg_coarse_inverse(self.h, sys)

    def close(self):
        if self.h:
            dfamg_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class BatchedSolver(Solver):
    """Many independent systems in one block-diagonal handle."""

    def __init__(self, A, part, nsub, Z, sys_row_off, **params):
        self.n = A.shape[0]
        self.nsys = len(sys_row_off) - 1
        self.params = make_params(**params)
        self.h = dfamg_setup_batched(self.params, sys_row_off, A, part, nsub, Z, stream=_stream())

    def solve(self, b, x, history=False):
        return dfamg_solve_batched(self.h, _dev_ptr(b, self.n), _dev_ptr(x, self.n), self.nsys)


class SchurSolver(Solver):
    """Flexible GMRES on a velocity-pressure system with the Schur
    pressure-correction preconditioner (inner solvers as in dfamg.h)."""

    def __init__(self, A, pmask, part, nsub, Z, **params):
        self.n = A.shape[0]
        params.setdefault("solver", "fgmres")
        params.setdefault("restart", 50)
        self.params = make_params(**params)
        self.h = dfamg_setup_schur(self.params, A, pmask, part, nsub, Z, stream=_stream())
