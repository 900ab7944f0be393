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


def deflated_bicgstabl(A, defl, precond, b, y0, rtol, maxiter, ell=2, observe=None):
    """BiCGStab(ell) of Sleijpen & Fokkema (1993) on the right-preconditioned
    deflated operator K = P A M^{-1}; returns (y, iters, history, status).

    This is the solver of the paper's Poisson runs.  Readings: the iteration
    solves K d = r_0 from d = 0, r_0 = P(b - A y_0), and y = y_0 + M^{-1} d is
    formed once at the end (M^{-1}, one V-cycle from a zero guess, is linear);
    one iteration is one cycle (ell BiCG steps, then the minimal-residual
    polynomial step over r_1 .. r_ell orthogonalised by modified Gram-Schmidt),
    i.e. 2 ell operator products; the stopping test runs after each cycle;
    r~ = r_0; exact zeros of rho, gamma or sigma are breakdowns.
    `observe(k, r_before, r_after, rt)` (tests only) sees, per cycle, copies of
    r^_0 .. r^_ell as the BiCG part leaves them and the cycle's new residual.
    """
    bnorm = np.linalg.norm(b)
    y = y0.copy()
    if bnorm == 0.0:
        return np.zeros_like(b), 0, [0.0], OK

    def K(v):
        return defl.project(A @ precond(v))

    r0 = defl.project(b - A @ y)
    hist = [np.linalg.norm(r0) / bnorm]
    if hist[0] <= rtol:
        return y, 0, hist, OK
    rt = r0.copy()
    d = np.zeros_like(b)                 # the iterate of K d = r_0
    r = [r0.copy()] + [None] * ell       # r^_0 .. r^_ell
    u = [np.zeros_like(b)] + [None] * ell
    rho0, alpha, omega = 1.0, 0.0, 1.0

    def finish(status, k):
        return y + precond(d), k, hist, status

    for k in range(1, maxiter + 1):
        rho0 = -omega * rho0
        # BiCG part: ell steps, each extending the u and r sequences by one
        for j in range(ell):
            rho1 = r[j] @ rt
            if rho0 == 0.0 or rho1 == 0.0:
                return finish(BREAKDOWN, k - 1)
            beta = alpha * rho1 / rho0
            rho0 = rho1
            for i in range(j + 1):
                u[i] = r[i] - beta * u[i]
            u[j + 1] = K(u[j])
            gamma = u[j + 1] @ rt
            if gamma == 0.0:
                return finish(BREAKDOWN, k - 1)
            alpha = rho0 / gamma
            for i in range(j + 1):
                r[i] = r[i] - alpha * u[i + 1]
            r[j + 1] = K(r[j])
            d = d + alpha * u[0]
        before = [v.copy() for v in r] if observe else None
        # minimal-residual part: orthogonalise r_1 .. r_ell (modified
        # Gram-Schmidt) and minimise ||r_0 - sum_j g_j r_j|| over g
        tau = np.zeros((ell + 1, ell + 1))
        sigma = np.zeros(ell + 1)
        gp = np.zeros(ell + 1)           # gamma'
        for j in range(1, ell + 1):
            for i in range(1, j):
                tau[i, j] = (r[j] @ r[i]) / sigma[i]
                r[j] = r[j] - tau[i, j] * r[i]
            sigma[j] = r[j] @ r[j]
            if sigma[j] == 0.0:
                return finish(BREAKDOWN, k)
            gp[j] = (r[0] @ r[j]) / sigma[j]
        g = np.zeros(ell + 1)            # gamma, by back substitution
        g[ell] = gp[ell]
        omega = g[ell]
        for j in range(ell - 1, 0, -1):
            g[j] = gp[j] - sum(tau[j, i] * g[i] for i in range(j + 1, ell + 1))
        gpp = np.zeros(ell + 1)          # gamma''
        for j in range(1, ell):
            gpp[j] = g[j + 1] + sum(tau[j, i] * g[i + 1] for i in range(j + 1, ell))
        d = d + g[1] * r[0]
        r[0] = r[0] - gp[ell] * r[ell]
        u[0] = u[0] - g[ell] * u[ell]
        for j in range(1, ell):
            u[0] = u[0] - g[j] * u[j]
            d = d + gpp[j] * r[j]
            r[0] = r[0] - gp[j] * r[j]
        if observe:
            observe(k, before, r[0].copy(), rt)
        hist.append(np.linalg.norm(r[0]) / bnorm)
        if not np.isfinite(hist[-1]):
            return finish(BREAKDOWN, k)
        if hist[-1] <= rtol:
            return finish(OK, k)
        if omega == 0.0:
            return finish(BREAKDOWN, k)
    return finish(NOCONV, maxiter)


def fgmres(A, precond, b, x0, rtol, maxiter, restart, observe=None):
    """Restarted flexible GMRES, right-preconditioned, on A x = b.

    Section "On precision of the coarse system solution": when the coarse
    operator is solved inexactly the projector becomes part of a variable
    preconditioner, which needs a flexible Krylov method such as flexible
    GMRES; the same passage and the Navier-Stokes section name FGMRES.  The
    iteration is Saad's flexible GMRES (Iterative Methods for Sparse Linear
    Systems, 2nd ed., section 9.4.1): Arnoldi with modified Gram-Schmidt on the
    vectors A z_j, where z_j = precond(v_j) may change from call to call, the
    preconditioned vectors z_j kept, and x = x0 + Z_k y_k with y_k the
    least-squares solution of the Hessenberg system, obtained with Givens
    rotations.  Readings:

    * one Arnoldi step (one preconditioner application, one product with A)
      is one iteration; history[k] = |g_{k}| / ||b||, the residual norm of the
      least-squares problem after k iterations (equal to ||b - A x_k|| in
      exact arithmetic); history[0] = ||b - A x0|| / ||b||;
    * stop at the first iteration with history[k] <= rtol, or at maxiter, or
      when h_{j+1,j} = 0 (the Krylov space is invariant: the residual of the
      least-squares problem is then zero); x is formed from the vectors of
      the current cycle whenever the loop leaves it;
    * after `restart` steps without convergence x is formed, r = b - A x is
      recomputed and a new cycle starts from v_0 = r / ||r||;
    * a zero diagonal after the rotations (singular Hessenberg) is a
      breakdown; b = 0 returns x = 0 after 0 iterations.

    observe(k, x_k, z_list), when given, is called at the end of every cycle
    with the iterate and the preconditioned vectors of that cycle.
    Returns (x, iters, history, status).
    """
    bnorm = np.linalg.norm(b)
    if bnorm == 0.0:
        return np.zeros_like(b), 0, [0.0], OK
    x = x0.copy()
    r = b - A @ x
    beta = np.linalg.norm(r)
    hist = [beta / bnorm]
    if hist[0] <= rtol:
        return x, 0, hist, OK
    if maxiter <= 0:
        return x, 0, hist, NOCONV
    it = 0
    m = restart
    while True:
        V = [r / beta]
        Zs = []
        H = np.zeros((m + 1, m))
        cs = np.zeros(m)
        sn = np.zeros(m)
        g = np.zeros(m + 1)
        g[0] = beta
        k = 0
        status = None
        for j in range(m):
            z = precond(V[j])
            Zs.append(z)
            w = A @ z
            for i in range(j + 1):              # modified Gram-Schmidt
                H[i, j] = w @ V[i]
                w = w - H[i, j] * V[i]
            H[j + 1, j] = np.linalg.norm(w)
            hnext = H[j + 1, j]
            for i in range(j):                  # earlier rotations on column j
                a, c = H[i, j], H[i + 1, j]
                H[i, j] = cs[i] * a + sn[i] * c
                H[i + 1, j] = -sn[i] * a + cs[i] * c
            d = np.hypot(H[j, j], H[j + 1, j])
            k = j + 1
            it += 1
            if d == 0.0:
                status = BREAKDOWN
                k = j                            # column j is not usable
                hist.append(hist[-1])
                break
            cs[j] = H[j, j] / d
            sn[j] = H[j + 1, j] / d
            H[j, j] = d
            H[j + 1, j] = 0.0
            g[j + 1] = -sn[j] * g[j]
            g[j] = cs[j] * g[j]
            res = abs(g[j + 1])
            hist.append(res / bnorm)
            if not np.isfinite(res):
                status = "nan"
                break
            if hist[-1] <= rtol or hnext == 0.0:
                status = OK
                break
            if it >= maxiter:
                status = NOCONV
                break
            V.append(w / hnext)
        if k > 0:
            # back substitution with the rotated (upper triangular) H
            yk = np.zeros(k)
            for i in range(k - 1, -1, -1):
                yk[i] = (g[i] - H[i, i + 1:k] @ yk[i + 1:k]) / H[i, i]
            for i in range(k):
                x = x + yk[i] * Zs[i]
        if observe is not None:
            observe(it, x.copy(), Zs[:k])
        if status is not None:
            return x, it, hist, status
        r = b - A @ x
        beta = np.linalg.norm(r)
        if beta == 0.0:
            return x, it, hist, OK
