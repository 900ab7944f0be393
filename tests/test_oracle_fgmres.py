"""Pins of the oracle's flexible GMRES, inexact coarse solve and multiplicative
deflation preconditioner against facts that do not come from the oracle:
least-squares minima over explicitly built subspaces (numpy's lstsq), the
textbook minimal-residual iteration, dense solves, algebraic identities of the
combined preconditioner and the rounding-error bound of a single-precision
matrix-vector product."""
import numpy as np
import pytest

from workloads import tiny_problem, make_problem
from workloads.convdiff import convection_diffusion7
from oracle import OracleSolver, OracleParams
from oracle.deflation import CoarseSolve, adef1_preconditioner
from oracle.krylov import fgmres


def _nonsym(n=14, seed=0):
    rng = np.random.default_rng(seed)
    A = 4.0 * np.eye(n) + 0.6 * rng.standard_normal((n, n))
    return A, rng.standard_normal(n)


def _min_residual(A, r0, basis):
    """min over c of ||r0 - A B c|| with B the given columns."""
    B = np.column_stack(basis)
    Q, _ = np.linalg.qr(B)                   # the same span, well conditioned
    AQ = A @ Q
    c, *_ = np.linalg.lstsq(AQ, r0, rcond=None)
    return np.linalg.norm(r0 - AQ @ c)


def test_fgmres_identity_is_minimal_residual_over_krylov_space():
    A, b = _nonsym()
    n = len(b)
    x, it, hist, st = fgmres(A, lambda v: v.copy(), b, np.zeros(n), 1e-13, 40, restart=n)
    assert st == "ok"
    K = [b]
    for k in range(1, it + 1):
        ref = _min_residual(A, b, K)
        assert abs(hist[k] * np.linalg.norm(b) - ref) <= 1e-10 * np.linalg.norm(b)
        K.append(A @ K[-1])
    assert np.linalg.norm(x - np.linalg.solve(A, b)) <= 1e-11 * np.linalg.norm(x)


def test_fgmres_fixed_preconditioner_minimises_over_preconditioned_space():
    A, b = _nonsym(seed=1)
    n = len(b)
    d = np.linspace(0.5, 2.0, n)
    x0 = np.random.default_rng(5).standard_normal(n)
    r0 = b - A @ x0
    x, it, hist, st = fgmres(A, lambda v: d * v, b, x0, 1e-13, 40, restart=n)
    assert st == "ok"
    K = [r0]                                  # Krylov space of A M^{-1} from r0
    for k in range(1, it + 1):
        ref = _min_residual(A, r0, [d * v for v in K])
        assert abs(hist[k] * np.linalg.norm(b) - ref) <= 1e-10 * np.linalg.norm(b)
        K.append(A @ (d * K[-1]))


@pytest.mark.parametrize("k", [1, 3, 6, 9])
def test_fgmres_variable_preconditioner_minimises_over_its_own_vectors(k):
    """With a preconditioner that changes at every call, x_k minimises the
    residual over x0 + span(z_0 .. z_{k-1}) of the vectors actually produced
    (the flexible property), and the recurrence residual is the true one."""
    A, b = _nonsym(seed=2)
    n = len(b)
    rng = np.random.default_rng(11)
    scales = [np.exp(0.8 * rng.standard_normal(n)) for _ in range(20)]
    calls = [0]

    def varying(v):
        s = scales[calls[0]]
        calls[0] += 1
        return s * v

    seen = {}
    x, it, hist, st = fgmres(A, varying, b, np.zeros(n), 1e-14, k, restart=n,
                             observe=lambda i, xk, zs: seen.update(x=xk, z=zs))
    assert it == k and st == "noconv"
    ref = _min_residual(A, b, seen["z"])
    true = np.linalg.norm(b - A @ x)
    assert abs(true - ref) <= 1e-10 * np.linalg.norm(b)
    assert abs(hist[-1] * np.linalg.norm(b) - true) <= 1e-10 * np.linalg.norm(b)


def test_fgmres_restart_one_is_the_minimal_residual_iteration():
    """FGMRES(1) with M = I: x += a r with a = (r, A r) / (A r, A r)."""
    A, b = _nonsym(seed=3)
    n = len(b)
    x, it, hist, st = fgmres(A, lambda v: v.copy(), b, np.zeros(n), 1e-30, 12, restart=1)
    xr = np.zeros(n)
    for _ in range(12):
        r = b - A @ xr
        Ar = A @ r
        xr = xr + (r @ Ar) / (Ar @ Ar) * r
    assert np.linalg.norm(x - xr) <= 1e-12 * np.linalg.norm(xr)
    assert abs(hist[-1] - np.linalg.norm(b - A @ xr) / np.linalg.norm(b)) <= 1e-12


def test_fgmres_restarts_match_dense_solve():
    A, b = _nonsym(n=30, seed=4)
    x, it, hist, st = fgmres(A, lambda v: v.copy(), b, np.zeros(30), 1e-12, 500, restart=4)
    assert st == "ok" and it > 4
    assert np.linalg.norm(x - np.linalg.solve(A, b)) <= 1e-9 * np.linalg.norm(x)
    assert all(hist[i + 1] <= hist[i] * (1 + 1e-12) for i in range(len(hist) - 1))


def test_fgmres_exits():
    A, b = _nonsym(seed=6)
    n = len(b)
    x, it, hist, st = fgmres(A, lambda v: v, np.zeros(n), np.ones(n), 1e-8, 10, restart=5)
    assert it == 0 and st == "ok" and not x.any()
    x, it, hist, st = fgmres(A, lambda v: v, b, np.zeros(n), 1e-8, 0, restart=5)
    assert it == 0 and st == "noconv"
    x, it, hist, st = fgmres(A, lambda v: v, b, np.zeros(n), 1e-14, 7, restart=5)
    assert it == 7 and st == "noconv" and len(hist) == 8
    assert abs(hist[-1] * np.linalg.norm(b) - np.linalg.norm(b - A @ x)) <= 1e-10 * np.linalg.norm(b)


def _convdiff_case(defl="linear"):
    A = convection_diffusion7(8, peclet=3.0)
    base = tiny_problem(N=8, pieces=(2, 2, 1), deflation=defl, seed=2)
    return A, base


@pytest.mark.parametrize("coarse", ["exact", "fp32"])
@pytest.mark.parametrize("restart", [3, 30])
def test_fgmres_deflated_amg_matches_dense_solve(coarse, restart):
    A, base = _convdiff_case()
    S = OracleSolver(A, base.part, base.nsub, base.Z,
                     OracleParams(solver="fgmres", coarse_solve=coarse, restart=restart,
                                  rtol=1e-12, coarse_enough=10))
    res = S.solve(base.b)
    xd = np.linalg.solve(A.toarray(), base.b)
    assert res["status"] == "ok"
    assert np.linalg.norm(res["x"] - xd) <= 1e-9 * np.linalg.norm(xd)
    assert res["relres_true"] <= 2e-12


def test_adef1_maps_range_of_AZ_to_Z():
    """B(A Z c) = Z c: the coarse correction solves A Z c exactly and leaves
    a zero residual for M (nonsymmetric A, so a transposed E would fail)."""
    A, base = _convdiff_case()
    S = OracleSolver(A, base.part, base.nsub, base.Z, OracleParams(solver="fgmres", coarse_enough=10))
    B = adef1_preconditioner(S.defl, CoarseSolve(S.defl, "exact"), S.precond)
    c = np.random.default_rng(0).standard_normal(S.defl.m)
    Zc = S.defl.Z @ c
    assert np.linalg.norm(B(A @ Zc) - Zc) <= 1e-10 * np.linalg.norm(Zc)


def test_adef1_hands_M_a_residual_orthogonal_to_Z():
    A, base = _convdiff_case()
    S = OracleSolver(A, base.part, base.nsub, base.Z, OracleParams(solver="fgmres", coarse_enough=10))
    seen = []

    def M(u):
        seen.append(u.copy())
        return S.precond(u)

    B = adef1_preconditioner(S.defl, CoarseSolve(S.defl, "exact"), M)
    v = np.random.default_rng(1).standard_normal(A.shape[0])
    z = B(v)
    u = seen[0]
    assert np.linalg.norm(S.defl.Z.T @ u) <= 1e-10 * np.linalg.norm(v)
    # the result is the coarse correction plus M applied to that residual
    t2 = np.linalg.solve(S.defl.E, S.defl.Z.T @ v)
    assert np.linalg.norm(u - (v - A @ (S.defl.Z @ t2))) <= 1e-10 * np.linalg.norm(v)
    assert np.linalg.norm(z - S.defl.Z @ t2 - S.precond(u)) <= 1e-10 * np.linalg.norm(z)


def test_fp32_coarse_solve_within_single_precision_bound():
    A, base = _convdiff_case()
    S = OracleSolver(A, base.part, base.nsub, base.Z, OracleParams(solver="fgmres", coarse_enough=10))
    E = S.defl.E
    m = E.shape[0]
    t = np.random.default_rng(2).standard_normal(m)
    exact = np.linalg.solve(E, t)
    approx = CoarseSolve(S.defl, "fp32")(t)
    u = 2.0 ** -24
    Einv = np.linalg.inv(E)
    bound = (m + 3) * u * (np.abs(Einv) @ np.abs(t))
    assert np.all(np.abs(approx - exact) <= bound)
    assert np.linalg.norm(approx - exact) > 1e-12 * np.linalg.norm(exact)   # genuinely inexact


def test_inexact_coarse_solve_breaks_the_projector_but_not_fgmres():
    """Section "On precision of the coarse system solution": with an inexact
    E the deflated system no longer determines x, so the projected CG does
    not reach the tolerance, while the deflation used as a preconditioner of
    the original system inside FGMRES still does."""
    P = make_problem("p", (24, 24, 24), (2, 2, 2), deflation="linear", sigma=2.0, coef_seed=1)
    S = OracleSolver(P.A, P.part, P.nsub, P.Z, OracleParams(solver="cg"))
    S.defl.solve_E = CoarseSolve(S.defl, "fp32")
    bad = S.solve(P.b, maxiter=200)
    assert bad["relres_true"] > 1e-6
    F = OracleSolver(P.A, P.part, P.nsub, P.Z, OracleParams(solver="fgmres", coarse_solve="fp32"))
    good = F.solve(P.b)
    assert good["status"] == "ok" and good["relres_true"] <= 1.01e-8


def _spd_coarse():
    P = make_problem("p", (10, 10, 10), (2, 2, 2), deflation="linear", sigma=1.0, coef_seed=3)
    S = OracleSolver(P.A, P.part, P.nsub, P.Z, OracleParams(solver="fgmres", coarse_enough=30))
    return P, S


def test_cg_coarse_solve_finite_termination_and_first_step():
    P, S = _spd_coarse()
    E = S.defl.E
    m = E.shape[0]
    t = np.random.default_rng(3).standard_normal(m)
    exact = np.linalg.solve(E, t)
    C = CoarseSolve(S.defl, "cg", rtol=1e-14, maxiter=4 * m)
    assert np.linalg.norm(C(t) - exact) <= 1e-10 * np.linalg.norm(exact)
    # one step: x1 = a D^{-1} t with a = (t, D^{-1} t) / (D^{-1} t, E D^{-1} t)
    z = t / np.diag(E)
    x1 = (t @ z) / (z @ E @ z) * z
    C1 = CoarseSolve(S.defl, "cg", rtol=0.0, maxiter=1)
    assert np.linalg.norm(C1(t) - x1) <= 1e-13 * np.linalg.norm(x1)


@pytest.mark.parametrize("rtol", [1e-1, 1e-2, 1e-4])
def test_cg_coarse_solve_stops_at_first_step_below_tolerance(rtol):
    P, S = _spd_coarse()
    E = S.defl.E
    t = np.random.default_rng(4).standard_normal(E.shape[0])
    C = CoarseSolve(S.defl, "cg", rtol=rtol, maxiter=500)
    x = C(t)
    k = C.iters[-1]
    assert np.linalg.norm(t - E @ x) <= rtol * np.linalg.norm(t)
    assert k >= 1
    Cp = CoarseSolve(S.defl, "cg", rtol=0.0, maxiter=k - 1)
    xp = Cp(t)
    assert np.linalg.norm(t - E @ xp) > rtol * np.linalg.norm(t)
    assert not CoarseSolve(S.defl, "cg")(np.zeros_like(t)).any()


def test_fgmres_with_iterative_coarse_solve_matches_dense_solve():
    """A coarse solve to 1e-1 changes the preconditioner from call to call;
    the flexible method still converges to the solution."""
    P, S = _spd_coarse()
    F = OracleSolver(P.A, P.part, P.nsub, P.Z,
                     OracleParams(solver="fgmres", coarse_solve="cg", coarse_rtol=1e-1,
                                  rtol=1e-12, coarse_enough=30))
    res = F.solve(P.b)
    xd = np.linalg.solve(P.A.toarray(), P.b)
    assert res["status"] == "ok"
    assert np.linalg.norm(res["x"] - xd) <= 1e-9 * np.linalg.norm(xd)
