"""Deflated preconditioned Krylov iterations (oracle).

TEST INFRASTRUCTURE ONLY (see the package docstring).

The method solves P(A y) = P(b) (section "Subdomain deflation", eq. (7)) with
a Krylov method preconditioned by the block AMG (section "Implementation":
the algorithm is equivalent to solving the deflated system preconditioned
with block AMG), then recovers x = y + Z lambda.  Readings:

* preconditioned CG (Listing 1's solver) on M^{-1} P A y = M^{-1} P b; P A is
  symmetric positive semi-definite for SPD A, so CG applies;
* BiCGStab in the right-preconditioned form of Barrett et al. (1994,
  "Templates", which the paper cites for CG) on the operator P A;
* stop at the first iteration whose recurrence residual satisfies
  ||r_k|| <= rtol ||b|| (2-norms; the paper's tolerance is a relative
  residual norm, Listing 1); r_0 = P(b - A y_0) with y_0 the initial guess;
* one loop pass (one operator product for CG, two for BiCGStab) counts as one
  iteration; the preconditioner application before the loop is not counted;
* b = 0 returns x = 0 after 0 iterations; exact zeros of rho or omega in
  BiCGStab are breakdowns.
"""
import numpy as np

OK, NOCONV, BREAKDOWN = "ok", "noconv", "breakdown"


def deflated_cg(A, defl, precond, b, y0, rtol, maxiter, flexible=False):
    """Returns (y, iters, history, status); history[k] = ||r_k|| / ||b||."""
    bnorm = np.linalg.norm(b)
    y = y0.copy()
    if bnorm == 0.0:
        return np.zeros_like(b), 0, [0.0], OK
    r = defl.project(b - A @ y)
    hist = [np.linalg.norm(r) / bnorm]
    if hist[0] <= rtol:
        return y, 0, hist, OK
    s = precond(r)
    p = s.copy()
    rho = r @ s
    for k in range(1, maxiter + 1):
        q = defl.project(A @ p)
        alpha = rho / (p @ q)
        y += alpha * p
        r -= alpha * q
        hist.append(np.linalg.norm(r) / bnorm)
        if hist[-1] <= rtol:
            return y, k, hist, OK
        s_old = s
        s = precond(r)
        rho_new = r @ s
        if flexible:
            beta = (r @ (s - s_old)) / rho
        else:
            beta = rho_new / rho
        p = s + beta * p
        rho = rho_new
    return y, maxiter, hist, NOCONV


def deflated_bicgstab(A, defl, precond, b, y0, rtol, maxiter):
    """Right-preconditioned BiCGStab on P A; returns (y, iters, history, status)."""
    bnorm = np.linalg.norm(b)
    y = y0.copy()
    if bnorm == 0.0:
        return np.zeros_like(b), 0, [0.0], OK
    r = defl.project(b - A @ y)
    hist = [np.linalg.norm(r) / bnorm]
    if hist[0] <= rtol:
        return y, 0, hist, OK
    rt = r.copy()
    rho_old = alpha = omega = 1.0
    v = np.zeros_like(b)
    p = np.zeros_like(b)
    for k in range(1, maxiter + 1):
        rho = rt @ r
        if rho == 0.0:
            return y, k - 1, hist, BREAKDOWN
        beta = (rho / rho_old) * (alpha / omega)
        p = r + beta * (p - omega * v)
        ph = precond(p)
        v = defl.project(A @ ph)
        alpha = rho / (rt @ v)
        s = r - alpha * v
        snorm = np.linalg.norm(s) / bnorm
        if snorm <= rtol:
            y += alpha * ph
            hist.append(snorm)
            return y, k, hist, OK
        sh = precond(s)
        t = defl.project(A @ sh)
        tt = t @ t
        omega = (t @ s) / tt if tt != 0.0 else 0.0
        if omega == 0.0:
            return y, k, hist, BREAKDOWN
        y += alpha * ph + omega * sh
        r = s - omega * t
        hist.append(np.linalg.norm(r) / bnorm)
        if hist[-1] <= rtol:
            return y, k, hist, OK
        rho_old = rho
    return y, maxiter, hist, NOCONV
