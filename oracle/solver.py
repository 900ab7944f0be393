"""Setup + solve with the library's calling conventions (oracle).

TEST INFRASTRUCTURE ONLY (see the package docstring).

Mirrors the usage of Listing 1: the solver is built once from a CSR matrix and
parameters, then `solve(rhs, x)` takes x as the initial guess and returns the
iteration count and the relative residual.  Here setup also takes the
subdomain partition and the local deflation blocks, as in the subdomain
deflation solver of section "Implementation".
"""
from dataclasses import dataclass

import numpy as np
import scipy.sparse as sp

from .deflation import Deflation, DeflationError, CoarseSolve, adef1_preconditioner
from .krylov import deflated_cg, deflated_bicgstab, deflated_bicgstabl, fgmres, OK, NOCONV, BREAKDOWN
from .vcycle import BlockAMG


class OracleError(Exception):
    pass


@dataclass
class OracleParams:
    solver: str = "cg"              # "cg", "bicgstab", "bicgstabl" or "fgmres"
    ell: int = 2                    # BiCGStab(ell)
    restart: int = 30               # FGMRES cycle length
    coarse_solve: str = "exact"     # FGMRES: "exact", "fp32" or "cg" E_hat
    coarse_rtol: float = 1e-2       # "cg": relative residual of the coarse solve
    coarse_maxiter: int = 100       # "cg": step limit of the coarse solve
    rtol: float = 1e-8
    maxiter: int = 1000
    smoother: str = "spai0"         # "spai0", "jacobi" or "block_spai0"
    jacobi_omega: float = 0.8
    coarse_enough: int = 500
    eps_strong: float = 0.08
    max_levels: int = 20
    block_size: int = 1
    flexible: bool = False          # CG: Polak-Ribiere beta (flexible CG)
    npre: int = 1                   # V-cycle pre-smoothing sweeps
    npost: int = 1                  # V-cycle post-smoothing sweeps
    precond: str = "amg"            # "amg", "identity" or "spai0" (diagonal)


def validate(A, part, nsub, Z):
    n = A.shape[0]
    if A.shape[1] != n:
        raise OracleError("matrix must be square")
    if part.shape != (n,) or Z.shape[0] != n:
        raise OracleError("partition / deflation sizes do not match the matrix")
    if n and (part.min() < 0 or part.max() >= nsub):
        raise OracleError("partition id out of range")
    if np.any(np.bincount(part, minlength=nsub) == 0):
        raise OracleError("empty subdomain")
    if not (np.all(np.isfinite(A.data)) and np.all(np.isfinite(Z))):
        raise OracleError("non-finite input")


class OracleSolver:
    def __init__(self, A, part, nsub, Z, prm=None):
        self.prm = prm or OracleParams()
        A = sp.csr_matrix(A, dtype=np.float64)
        A.sort_indices()
        part = np.asarray(part, dtype=np.int64)
        Z = np.asarray(Z, dtype=np.float64)
        validate(A, part, nsub, Z)
        self.A, self.part, self.nsub, self.Zloc = A, part, nsub, Z
        try:
            self.defl = Deflation(A, part, nsub, Z,
                                  symmetric=(self.prm.solver == "cg"))
        except DeflationError as exc:
            raise OracleError(str(exc))
        if self.prm.precond == "amg":
            self.M = BlockAMG(A, part, nsub, npre=self.prm.npre, npost=self.prm.npost,
                              eps_strong=self.prm.eps_strong,
                              coarse_enough=self.prm.coarse_enough,
                              max_levels=self.prm.max_levels,
                              smoother=self.prm.smoother,
                              jacobi_omega=self.prm.jacobi_omega,
                              bs=self.prm.block_size)
            self.precond = self.M.apply
        elif self.prm.precond == "spai0":
            # purely local SPAI-0: m_i = a_ii / sum_j a_ij^2
            self.M = None
            m = A.diagonal() / np.asarray(A.multiply(A).sum(axis=1)).ravel()
            self.precond = lambda r: m * r
        else:
            self.M = None
            self.precond = lambda r: r.copy()

    def solve(self, b, x0=None, rtol=None, maxiter=None):
        prm = self.prm
        b = np.asarray(b, dtype=np.float64)
        y0 = np.zeros_like(b) if x0 is None else np.asarray(x0, dtype=np.float64)
        if not (np.all(np.isfinite(b)) and np.all(np.isfinite(y0))):
            raise OracleError("non-finite right-hand side or initial guess")
        rtol = prm.rtol if rtol is None else rtol
        maxiter = prm.maxiter if maxiter is None else maxiter
        if prm.solver == "cg":
            y, iters, hist, status = deflated_cg(
                self.A, self.defl, self.precond, b, y0, rtol, maxiter,
                flexible=prm.flexible)
        elif prm.solver == "bicgstab":
            y, iters, hist, status = deflated_bicgstab(
                self.A, self.defl, self.precond, b, y0, rtol, maxiter)
        elif prm.solver == "bicgstabl":
            y, iters, hist, status = deflated_bicgstabl(
                self.A, self.defl, self.precond, b, y0, rtol, maxiter, ell=prm.ell)
        elif prm.solver == "fgmres":
            # the original system, preconditioned by the deflation combined
            # with the block AMG; no recovery step
            B = adef1_preconditioner(self.defl, CoarseSolve(self.defl, prm.coarse_solve,
                                                            prm.coarse_rtol, prm.coarse_maxiter),
                                     self.precond)
            y, iters, hist, status = fgmres(self.A, B, b, y0, rtol, maxiter, prm.restart)
        else:
            raise OracleError(prm.solver)
        bnorm = np.linalg.norm(b)
        if bnorm == 0.0:
            x = np.zeros_like(b)
            true = 0.0
        else:
            x = y if prm.solver == "fgmres" else self.defl.recover(b, y)
            true = np.linalg.norm(b - self.A @ x) / bnorm
        return {"x": x, "y": y, "iters": iters, "history": np.array(hist),
                "relres": hist[-1], "relres_true": true, "status": status}

    # component access for unit parity checks
    def project(self, v):
        return self.defl.project(np.asarray(v, dtype=np.float64))

    def apply_precond(self, r):
        return self.precond(np.asarray(r, dtype=np.float64))

    def hierarchy_summary(self):
        """Per subdomain: list of (n_l, nnz(A_l), nnz(P_l), omega_l)."""
        out = []
        for H in self.M.hierarchies:
            rows = []
            for lvl in H.levels:
                rows.append((lvl.A.shape[0], lvl.A.nnz,
                             0 if lvl.P is None else lvl.P.nnz, lvl.omega))
            out.append(rows)
        return out
