"""Deflation basis, coarse operator, projector and solution recovery (oracle).

TEST INFRASTRUCTURE ONLY (see the package docstring).

Follows section "Subdomain deflation":
* x = y + Z lambda with Z an n x m basis (eq. (2));
* E = Z^T A Z, invertible when A is and Z has independent columns (eqs. (3),
  (4) and the remark after them);
* the deflated system P(A y) = P(b) with P = I - A Z E^{-1} Z^T (eqs. (6)-(7));
* lambda recovered from the first block row of eq. (4).  The printed formula
  for lambda is dimensionally inconsistent; the reading used is
  lambda = E^{-1} Z^T (b - A y), which is what eq. (3) gives, so that
  b - A x = P(b - A y);
and section "Implementation": the projector applied matrix-free as
t1 = Z^T r, t2 = E^{-1} t1, r* = r - (AZ) t2 with AZ and E formed explicitly,
and E solved exactly (section "On precision of the coarse system solution").

Z is given as its local blocks: row i of `Zloc` holds the ndv deflation
vectors of the subdomain part[i] evaluated at unknown i; the full basis has
column part[i]*ndv + k for the k-th vector (sections "Constant deflation",
"Linear deflation").
"""
import numpy as np
import scipy.linalg as sla
import scipy.sparse as sp


class DeflationError(Exception):
    pass


def full_basis(part, nsub, Zloc):
    """Sparse n x (nsub*ndv) basis Z from its local blocks."""
    n, ndv = Zloc.shape
    rows = np.repeat(np.arange(n), ndv)
    cols = (np.asarray(part, dtype=np.int64)[:, None] * ndv
            + np.arange(ndv)).ravel()
    return sp.csr_matrix((Zloc.ravel(), (rows, cols)), shape=(n, nsub * ndv))


def local_rank_check(part, nsub, Zloc, rtol=1e-12):
    """Return the first subdomain whose local block has dependent columns
    (numerical rank below ndv with tolerance rtol * largest singular value),
    or -1 when every block has full column rank."""
    ndv = Zloc.shape[1]
    if ndv == 0:
        return -1
    order = np.argsort(part, kind="stable")
    bounds = np.searchsorted(part[order], np.arange(nsub + 1))
    for s in range(nsub):
        Zs = Zloc[order[bounds[s]:bounds[s + 1]]]
        if Zs.shape[0] < ndv:
            return s
        sv = np.linalg.svd(Zs, compute_uv=False)
        if sv[0] == 0.0 or np.sum(sv > rtol * sv[0]) < ndv:
            return s
    return -1


class Deflation:
    """P = I - A Z E^{-1} Z^T with exact FP64 E solves."""

    def __init__(self, A, part, nsub, Zloc, symmetric=True):
        self.A = A
        self.Z = full_basis(part, nsub, Zloc)
        bad = local_rank_check(np.asarray(part), nsub, Zloc)
        if bad >= 0:
            raise DeflationError(f"deflation block of subdomain {bad} is rank deficient")
        self.AZ = (A @ self.Z).tocsr()
        self.E = (self.Z.T @ self.AZ).toarray()
        self.symmetric = symmetric
        self.m = self.E.shape[0]
        if self.m == 0:              # no deflation vectors: P = I
            self._fac = None
            return
        try:
            if symmetric:
                self._fac = sla.cho_factor(self.E, lower=True, check_finite=True)
            else:
                self._fac = sla.lu_factor(self.E, check_finite=True)
                if np.any(np.diag(self._fac[0]) == 0.0):
                    raise np.linalg.LinAlgError("singular E")
        except np.linalg.LinAlgError as exc:
            raise DeflationError(f"E = Z^T A Z is not factorizable: {exc}")

    def solve_E(self, t1):
        if self.m == 0:
            return np.zeros(0)
        if self.symmetric:
            return sla.cho_solve(self._fac, t1)
        return sla.lu_solve(self._fac, t1)

    def project(self, v):
        """P v = v - AZ E^{-1} Z^T v."""
        t1 = self.Z.T @ v
        t2 = self.solve_E(t1)
        return v - self.AZ @ t2

    def recover(self, b, y):
        """x = y + Z E^{-1} Z^T (b - A y)."""
        lam = self.solve_E(self.Z.T @ (b - self.A @ y))
        return y + self.Z @ lam


class CoarseSolve:
    """t -> E_hat t, an approximation of E^{-1} t.

    Section "On precision of the coarse system solution": an inexact inverse
    E_hat of E is allowed once the projector is used as part of a (variable)
    preconditioner of the original system instead of defining the deflated
    system.  Kinds:
    * "exact": the FP64 factorisation of `Deflation` (E^{-1} t to rounding);
    * "fp32": E^{-1}, formed in FP64, rounded to single precision and applied
      to the single-precision rounding of t in single-precision arithmetic
      (a solve whose relative error is of the order of the single-precision
      unit roundoff times the condition of the product);
    * "cg": an iterative solve to a relaxed tolerance (symmetric positive
      definite E), the Krylov option the section discusses.
    """

    def __init__(self, defl, kind="exact", rtol=1e-3, maxiter=100):
        if kind not in ("exact", "fp32", "cg"):
            raise ValueError(kind)
        self.defl, self.kind = defl, kind
        self.rtol, self.maxiter = rtol, maxiter
        self.iters = []                      # CG steps of every call (kind "cg")
        if kind == "fp32" and defl.m > 0:
            self.Einv32 = np.linalg.inv(defl.E).astype(np.float32)

    def __call__(self, t1):
        if self.defl.m == 0:
            return np.zeros(0)
        if self.kind == "exact":
            return self.defl.solve_E(t1)
        if self.kind == "cg":
            return self._cg(t1)
        return (self.Einv32 @ t1.astype(np.float32)).astype(np.float64)

    def _cg(self, t):
        """Jacobi-preconditioned CG on E t2 = t from t2 = 0 (Hestenes and
        Stiefel's method with the diagonal of E as preconditioner), stopped at
        the first step with ||t - E t2|| <= rtol ||t|| or after maxiter steps:
        a solve whose accuracy, and hence the preconditioner it belongs to,
        changes from call to call."""
        E = self.defl.E
        d = np.diag(E)
        x = np.zeros_like(t)
        r = t.copy()
        tn = np.linalg.norm(t)
        k = 0
        if tn == 0.0:
            self.iters.append(0)
            return x
        z = r / d
        p = z.copy()
        rho = r @ z
        while k < self.maxiter and np.linalg.norm(r) > self.rtol * tn:
            q = E @ p
            alpha = rho / (p @ q)
            x = x + alpha * p
            r = r - alpha * q
            k += 1
            z = r / d
            rho_new = r @ z
            p = z + (rho_new / rho) * p
            rho = rho_new
        self.iters.append(k)
        return x


def adef1_preconditioner(defl, coarse, precond):
    """Multiplicative combination of the deflation and a preconditioner M.

    Section "On precision of the coarse system solution": the projector acts
    as a preconditioner of the original system, combined multiplicatively with
    the other preconditioners.  Reading (Tang, Nabben, Vuik and Erlangga 2009,
    the variant they call A-DEF1): with Q_hat = Z E_hat Z^T,

        B(v) = Q_hat v + M^{-1} (v - A Q_hat v),

    the coarse correction first, then M applied to the residual it leaves,
    computed as t1 = Z^T v, t2 = E_hat t1, u = Z t2, v - (AZ) t2 (the
    projector's own steps, section "Implementation"), s = M^{-1}(v - (AZ) t2),
    B(v) = u + s.  With the exact E^{-1}, B(A Z c) = Z c.
    """
    def apply(v):
        t2 = coarse(defl.Z.T @ v)
        return defl.Z @ t2 + precond(v - defl.AZ @ t2)
    return apply
