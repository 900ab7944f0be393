"""Pins of the oracle's V(npre, npost) cycle and of its flexible CG.

* Two-grid identity: with an exact coarse solve, one V-cycle from a zero
  guess is the linear map x = (I - E) A^{-1} f, where the error propagation
  operator is E = S^npost (I - P A_c^{-1} R A) S^npre with the smoothing
  iteration matrix S = I - M A (a textbook fact of multigrid theory, e.g.
  Trottenberg, Oosterlee, Schueller, "Multigrid", section 2.4).  The test
  forms E densely and compares, for several sweep counts; a dropped sweep, a
  swapped pre/post count or a residual taken from the wrong iterate fails it.
* Three levels: the same identity with the coarse solve replaced by the
  coarse level's own V-cycle matrix, which pins the recursion passing the
  sweep counts down.
* Flexible CG (Polak-Ribiere beta): with a fixed symmetric positive
  definite preconditioner it generates the same iterates as the standard
  (Fletcher-Reeves) form in exact arithmetic, since the new residual is
  orthogonal to the previous preconditioned one; with a preconditioner that
  changes from one application to the next the standard form stagnates
  while the flexible one still converges (Notay, SIAM J. Sci. Comput. 22,
  2000).  A wrong sign or a dropped previous-residual term fails one of them.
"""
import numpy as np
import pytest
import scipy.sparse as sp

from oracle import sa
from oracle.vcycle import vcycle
from oracle.krylov import deflated_cg
from workloads.poisson import poisson7


def _hier(N, coarse_enough, sigma=1.0, seed=7):
    k = np.exp(sigma * np.random.default_rng(seed).standard_normal(N ** 3))
    A = poisson7(N, k=k).tocsr()
    return A, sa.build_hierarchy(A, eps_strong=0.08, coarse_enough=coarse_enough)


def _dense_level(H, l):
    lvl = H.levels[l]
    A = lvl.A.toarray()
    M = np.diag(lvl.m) if isinstance(lvl.m, np.ndarray) else lvl.m.toarray()
    return A, M, lvl.P.toarray(), lvl.R.toarray()


def _vcycle_matrix(H, l, npre, npost):
    """Dense matrix B_l with V(l, f) = B_l f, from the error propagation
    operator: B_l = (I - E_l) A_l^{-1}, E_l = S^npost (I - P B_{l+1} R A) S^npre."""
    A = H.levels[l].A.toarray()
    if l == H.nlevels - 1:
        return np.linalg.inv(A)
    A, M, P, R = _dense_level(H, l)
    n = A.shape[0]
    S = np.eye(n) - M @ A
    Bc = _vcycle_matrix(H, l + 1, npre, npost)
    E = np.linalg.matrix_power(S, npost) @ (np.eye(n) - P @ Bc @ R @ A) @ np.linalg.matrix_power(S, npre)
    return (np.eye(n) - E) @ np.linalg.inv(A)


@pytest.mark.parametrize("npre,npost", [(0, 1), (1, 1), (2, 2), (3, 1), (1, 3)])
def test_two_grid_identity(npre, npost):
    A, H = _hier(6, coarse_enough=60)
    assert H.nlevels == 2
    # the coarse operator is the Galerkin product
    _, _, P, R = _dense_level(H, 0)
    assert np.allclose(H.levels[1].A.toarray(), R @ A.toarray() @ P, rtol=0, atol=1e-12)
    f = np.random.default_rng(3).uniform(-1, 1, A.shape[0])
    x = vcycle(H, 0, f, npre, npost)
    want = _vcycle_matrix(H, 0, npre, npost) @ f
    assert np.allclose(x, want, rtol=0, atol=1e-11 * np.abs(want).max())


@pytest.mark.parametrize("npre,npost", [(1, 1), (2, 2), (0, 2)])
def test_three_level_identity(npre, npost):
    A, H = _hier(9, coarse_enough=12)
    assert H.nlevels >= 3
    f = np.random.default_rng(4).uniform(-1, 1, A.shape[0])
    x = vcycle(H, 0, f, npre, npost)
    want = _vcycle_matrix(H, 0, npre, npost) @ f
    assert np.allclose(x, want, rtol=0, atol=1e-10 * np.abs(want).max())


def test_more_sweeps_reduce_the_two_grid_error():
    # the spectral radius of E shrinks as sweeps are added (SPAI-0 on an SPD
    # M-matrix is a convergent smoother)
    A, H = _hier(6, coarse_enough=60)
    n = A.shape[0]
    rho = []
    for nu in (1, 2, 3):
        B = _vcycle_matrix(H, 0, nu, nu)
        rho.append(max(abs(np.linalg.eigvals(np.eye(n) - B @ A.toarray()))))
    assert rho[0] > rho[1] > rho[2] and rho[0] < 1.0


class _NoDeflation:
    def project(self, v):
        return v


def _spd_1d(n=200):
    return (sp.diags([-np.ones(n - 1), 2.0 * np.ones(n), -np.ones(n - 1)], [-1, 0, 1]) +
            0.01 * sp.eye(n)).tocsr()


def test_flexible_cg_equals_standard_for_a_fixed_preconditioner():
    # 8^3 Poisson (well enough conditioned that rounding stays small over
    # the whole run) with a fixed SPD diagonal preconditioner
    A = poisson7(8).tocsr()
    n = A.shape[0]
    b = np.random.default_rng(0).uniform(-1, 1, n)
    d = 1.0 + 0.5 * np.random.default_rng(1).uniform(-1, 1, n)
    out = [deflated_cg(A, _NoDeflation(), lambda r: d * r, b, np.zeros(n), 1e-10, 1000, flexible=f)
           for f in (False, True)]
    (y0, it0, h0, s0), (y1, it1, h1, s1) = out
    assert s0 == s1 == "ok" and it0 == it1
    assert np.allclose(h0, h1, rtol=1e-8, atol=0)
    assert np.linalg.norm(y0 - y1) <= 1e-12 * np.linalg.norm(y0)


def test_flexible_cg_converges_with_a_varying_preconditioner():
    A = _spd_1d()
    n = A.shape[0]
    b = np.random.default_rng(0).uniform(-1, 1, n)

    def run(flexible):
        rng = np.random.default_rng(1)

        def prec(r):   # a different SPD diagonal at every application
            return (1.0 + 0.5 * rng.uniform(-1, 1, n)) * r
        return deflated_cg(A, _NoDeflation(), prec, b, np.zeros(n), 1e-8, 2000, flexible=flexible)

    y, it, h, st = run(True)
    assert st == "ok" and it < 700
    assert np.linalg.norm(b - A @ y) <= 1.01e-8 * np.linalg.norm(b)
    _, it_std, _, st_std = run(False)
    assert st_std == "noconv" or it_std > 2 * it
