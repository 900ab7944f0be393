"""Pins of the oracle's Schur pressure-correction preconditioner against
block algebra that does not come from the oracle: with exact inner solves
the three steps are the block-LU inverse of the system; the approximate
Schur complement is the exact one when K is diagonal; SPAI-0 on a hand
example; the top-level flexible GMRES against a sparse direct solve."""
import numpy as np
import pytest
import scipy.sparse as sp
import scipy.sparse.linalg as spla

from workloads import oseen_q1
from workloads.partition import box_partition
from oracle.schur import (split_blocks, schur_complement_approx, spai0_diagonal,
                          SchurPressureCorrection, schur_fgmres)


def _oseen(N, pieces=(2, 1, 1)):
    A, _ = oseen_q1(N)
    n = A.shape[0]
    pmask = (np.arange(n) % 4 == 3).astype(np.int32)
    part_p, nsub = box_partition(N, N, N, *pieces)
    return A, pmask, part_p, nsub, np.ones((N ** 3, 1))


def test_split_blocks_reassemble():
    A, pmask, *_ = _oseen(4)
    u, p, K, G, D, S = split_blocks(A, pmask)
    B = sp.bmat([[K, G], [D, S]]).toarray()
    order = np.concatenate([u, p])
    assert np.array_equal(B, A.toarray()[np.ix_(order, order)])
    assert len(p) == 64 and np.all(p % 4 == 3)


def test_exact_inner_solves_give_the_inverse():
    """With K^{-1} and (S - D K^{-1} G)^{-1} exact, the three steps are the
    block-LU solve: B(r) = A^{-1} r and FGMRES stops after one step."""
    A, pmask, part_p, nsub, Zp = _oseen(4)
    u, p, K, G, D, S = split_blocks(A, pmask)
    Kd = K.toarray()
    Sx = S.toarray() - D.toarray() @ np.linalg.solve(Kd, G.toarray())
    B = SchurPressureCorrection(A, pmask, part_p, nsub, Zp, coarse_enough=20,
                                k_solve=lambda r: np.linalg.solve(Kd, r),
                                p_solve=lambda r: np.linalg.solve(Sx, r))
    r = np.random.default_rng(0).standard_normal(A.shape[0])
    x = spla.spsolve(A.tocsc(), r)
    assert np.linalg.norm(B(r) - x) <= 1e-10 * np.linalg.norm(x)
    from oracle.krylov import fgmres
    xs, it, hist, st = fgmres(A, B, r, np.zeros_like(r), 1e-9, 10, 10)
    assert it == 1 and st == "ok"


def test_approximate_schur_complement_is_exact_for_diagonal_K():
    rng = np.random.default_rng(1)
    nu, npr = 12, 5
    K = sp.diags(rng.uniform(1.0, 3.0, nu))
    G = sp.random(nu, npr, density=0.4, random_state=2)
    D = sp.random(npr, nu, density=0.4, random_state=3)
    S = sp.random(npr, npr, density=0.5, random_state=4)
    Sh = schur_complement_approx(sp.csr_matrix(K), sp.csr_matrix(G), sp.csr_matrix(D), sp.csr_matrix(S))
    exact = S.toarray() - D.toarray() @ np.linalg.solve(K.toarray(), G.toarray())
    assert np.allclose(Sh.toarray(), exact, rtol=0, atol=1e-14)


def test_spai0_hand_example():
    m = spai0_diagonal(sp.csr_matrix(np.array([[2.0, 1.0], [1.0, 3.0]])))
    assert np.allclose(m, [2.0 / 5.0, 3.0 / 10.0], rtol=0, atol=1e-16)


@pytest.mark.parametrize("N,pieces", [(5, (1, 1, 1)), (6, (2, 2, 1))])
def test_schur_fgmres_matches_direct_solve(N, pieces):
    A, pmask, part_p, nsub, Zp = _oseen(N, pieces)
    b = np.random.default_rng(N).uniform(-1, 1, A.shape[0])
    res = schur_fgmres(A, b, pmask, part_p, nsub, Zp, rtol=1e-11, coarse_enough=30)
    x = spla.spsolve(A.tocsc(), b)
    assert res["status"] == "ok"
    assert np.linalg.norm(res["x"] - x) <= 1e-8 * np.linalg.norm(x)
