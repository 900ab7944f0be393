"""Schur pressure-correction preconditioner for the Navier-Stokes-shaped
block system (oracle).

TEST INFRASTRUCTURE ONLY (see the package docstring).

Section "Navier-Stokes problem": the system [K G; D S] [u; p] = [b_u; b_p]
(velocity block K, gradient G, divergence D, stabilisation S; the pressure
unknowns are marked by a mask) is solved by flexible GMRES preconditioned by
an inexact pressure-Schur step, each application being
  1. u_hat ~ K^{-1} r_u,
  2. p ~ solve of (S - D diag(K)^{-1} G) p = r_p - D u_hat,
  3. u ~ K^{-1} (r_u - G p);
steps 1 and 3 use GMRES preconditioned by a purely local SPAI-0, step 2 uses
flexible GMRES preconditioned by subdomain deflation with local AMG, and the
settings of the paper's JSON listing are the defaults (top level FGMRES(50)
to 1e-4; K solves to 1e-3 in at most 5 steps; pressure solves to 1e-2 in at
most 20 steps, coarse_enough 500).  Readings:

* the approximate Schur complement S_hat = S - D diag(K)^{-1} G is formed
  explicitly (the paper applies it matrix-free; the product is the same) and
  the pressure preconditioner -- the deflation combined with the block AMG,
  inside flexible GMRES -- is built from S_hat rather than from S;
* GMRES with the fixed SPAI-0 preconditioner is the flexible GMRES of
  `krylov` (identical when the preconditioner does not change);
* every inner solve starts from zero; a solve that stops at its step limit
  returns its last iterate.
"""
import numpy as np
import scipy.sparse as sp

from .krylov import fgmres
from .solver import OracleSolver, OracleParams


def split_blocks(A, pmask):
    """K, G, D, S of the system with the unknowns in two groups: velocity
    (pmask == 0) and pressure (pmask != 0), each in ascending index order."""
    A = sp.csr_matrix(A)
    pmask = np.asarray(pmask) != 0
    u = np.flatnonzero(~pmask)
    p = np.flatnonzero(pmask)
    K = A[u][:, u].tocsr()
    G = A[u][:, p].tocsr()
    D = A[p][:, u].tocsr()
    S = A[p][:, p].tocsr()
    return u, p, K, G, D, S


def schur_complement_approx(K, G, D, S):
    """S_hat = S - D diag(K)^{-1} G."""
    dinv = sp.diags(1.0 / K.diagonal())
    Sh = (S - D @ dinv @ G).tocsr()
    Sh.sum_duplicates()
    Sh.sort_indices()
    return Sh


def spai0_diagonal(M):
    """m_i = a_ii / sum_j a_ij^2 (SPAI-0, section "Implementation")."""
    M = sp.csr_matrix(M)
    return M.diagonal() / np.asarray(M.multiply(M).sum(axis=1)).ravel()


class SchurPressureCorrection:
    """The preconditioner r -> (u, p) of the three steps above."""

    def __init__(self, A, pmask, part_p, nsub, Zp, u_rtol=1e-3, u_maxiter=5,
                 p_rtol=1e-2, p_maxiter=20, coarse_enough=500, k_solve=None, p_solve=None):
        self.u, self.p, self.K, self.G, self.D, self.S = split_blocks(A, pmask)
        self.n = A.shape[0]
        self.Sh = schur_complement_approx(self.K, self.G, self.D, self.S)
        self.mK = spai0_diagonal(self.K)
        self.u_rtol, self.u_maxiter = u_rtol, u_maxiter
        self.P = OracleSolver(self.Sh, part_p, nsub, Zp,
                              OracleParams(solver="fgmres", restart=p_maxiter, rtol=p_rtol,
                                           maxiter=p_maxiter, coarse_enough=coarse_enough))
        # replacements of the inner solves (exact ones in the pins)
        self.k_solve = k_solve or self._k_solve
        self.p_solve = p_solve or (lambda rhs: self.P.solve(rhs)["x"])

    def _k_solve(self, rhs):
        x, *_ = fgmres(self.K, lambda v: self.mK * v, rhs, np.zeros_like(rhs), self.u_rtol,
                       self.u_maxiter, self.u_maxiter)
        return x

    def __call__(self, r):
        ru, rp = r[self.u], r[self.p]
        uh = self.k_solve(ru)
        p = self.p_solve(rp - self.D @ uh)
        u = self.k_solve(ru - self.G @ p)
        out = np.empty(self.n)
        out[self.u] = u
        out[self.p] = p
        return out


def schur_fgmres(A, b, pmask, part_p, nsub, Zp, rtol=1e-4, maxiter=500, restart=50, x0=None, **kw):
    """Top-level flexible GMRES with the Schur pressure-correction
    preconditioner.  Returns the result dict of the other solvers' form."""
    A = sp.csr_matrix(A)
    B = SchurPressureCorrection(A, pmask, part_p, nsub, Zp, **kw)
    x0 = np.zeros(A.shape[0]) if x0 is None else x0
    x, it, hist, status = fgmres(A, B, b, x0, rtol, maxiter, restart)
    bn = np.linalg.norm(b)
    true = np.linalg.norm(b - A @ x) / bn if bn > 0 else 0.0
    return {"x": x, "iters": it, "history": np.array(hist), "relres": hist[-1],
            "relres_true": true, "status": status}
