"""Pins of the oracle's point-block smoothed aggregation (block size b > 1).

The point-block hierarchy (section "Implementation": block-local AMG of the
square diagonal sub-blocks; section "Navier-Stokes problem": the non-scalar
system) runs strength, aggregation, filtering, omega and the tentative
prolongation on the node graph.  These tests pin every block branch of
oracle/sa.py to facts that do not come from the oracle itself:

* a b = 2 case worked out by hand with non-identity, nonsymmetric diagonal
  blocks, so that the Frobenius strength test, the lumping of weak blocks,
  the side D^{-1} is applied on, the infinity norm in the Gershgorin bound,
  the smoothed prolongator and the Galerkin product all have literal values;
* a singular diagonal block, which must leave the Gershgorin bound and get
  no smoothing term;
* Kronecker invariance: for A = A_s kron I_b the block hierarchy is the
  scalar one kron I_b (same aggregates and omega, P = P_s kron I_b,
  A_c = A_c,s kron I_b), which ties the block code to the scalar code that
  the closed forms of tests/test_oracle_pins.py pin;
* a whole block solve on a small Oseen system against a dense direct solve.
"""
from fractions import Fraction

import numpy as np
import pytest
import scipy.sparse as sp

from oracle import sa
from oracle import OracleSolver, OracleParams


# ---------------------------------------------------------------------------
# the hand-derived b = 2 case
# ---------------------------------------------------------------------------
#
# Three nodes in a chain, b = 2, node blocks
#   D = [[4, 1], [0, 2]]     (every diagonal block)
#   C = [[-1, -1], [0, -1]]  (nodes 0-1, both directions)
#   W = [[-1/2, 0], [0, 0]]  (nodes 1-2, both directions)
# and eps = 1/7 (eps^2 = 1/49).
#
# Strength, ||A_IJ||_F^2 >= eps^2 ||A_II||_F ||A_JJ||_F, with ||D||_F^2 = 21:
#   0-1: ||C||_F^2 = 3    >= 21/49 = 3/7   strong
#   1-2: ||W||_F^2 = 1/4  <  3/7           weak   (node 2 has no strong
#                                                   neighbour: isolated)
# Aggregation: pass 1 at node 0 makes {0, 1}; node 2 stays out: agg = [0, 0, -1].
# Filtered matrix: the weak blocks go into their row's diagonal block:
#   A_F,00 = D, A_F,11 = A_F,22 = D + W = [[7/2, 1], [0, 2]],
#   A_F,01 = A_F,10 = C, A_F,12 = A_F,21 = 0.
# Block inverses: D^{-1} = [[1/4, -1/8], [0, 1/2]],
#                 (D + W)^{-1} = [[2/7, -1/7], [0, 1/2]].
# Gershgorin: sum_J ||D_I^{-1} A_F,IJ||_inf (row sums of absolute values):
#   node 0: 1 + ||[[-1/4, -1/8], [0, -1/2]]||_inf = 1 + 1/2 = 3/2
#   node 1: 1 + ||[[-2/7, -1/7], [0, -1/2]]||_inf = 1 + 1/2 = 3/2
#   node 2: 1
#   rho = 3/2, omega = (4/3) / (3/2) = 8/9.
#   (With the 1-norm node 1 would give 1 + 9/14 = 23/14; with the inverse
#   applied on the right, A_F,01 (D + W)^{-1}, node 0 would give 23/14.)
# Prolongator P = P_t - omega D^{-1} A_F P_t, P_t = [I; I; 0]:
#   A_F P_t: node 0: D + C = [[3, 0], [0, 1]]; node 1: C + D + W = [[5/2, 0], [0, 1]];
#            node 2: 0
#   P_0 = I - 8/9 [[3/4, -1/8], [0, 1/2]] = [[1/3, 1/9], [0, 5/9]]
#   P_1 = I - 8/9 [[5/7, -1/7], [0, 1/2]] = [[23/63, 8/63], [0, 5/9]]
#   P_2 = 0
# Galerkin product with the unfiltered A (R = P^T):
#   (A P)_0 = D P_0 + C P_1 = [[61/63, 20/63], [0, 5/9]]
#   (A P)_1 = C P_0 + D P_1 = [[71/63, 25/63], [0, 5/9]]
#   A_c = P_0^T (A P)_0 + P_1^T (A P)_1 = [[2914, 995], [995, 2790]] / 3969

F = Fraction
D2 = [[4, 1], [0, 2]]
C2 = [[-1, -1], [0, -1]]
W2 = [[F(-1, 2), 0], [0, 0]]
EPS = 1.0 / 7.0


def _blocks_to_csr(blocks, nn, b):
    A = np.zeros((nn * b, nn * b))
    for (I, J), blk in blocks.items():
        A[I * b:(I + 1) * b, J * b:(J + 1) * b] = np.array(blk, dtype=float)
    M = sp.csr_matrix(A)
    M.eliminate_zeros()
    M.sort_indices()
    return M, A


def _hand_case():
    blocks = {(0, 0): D2, (0, 1): C2, (1, 0): C2, (1, 1): D2, (1, 2): W2, (2, 1): W2, (2, 2): D2}
    return _blocks_to_csr(blocks, 3, 2)


def _fl(rows):
    return np.array([[float(v) for v in r] for r in rows])


P_HAND = _fl([[F(1, 3), F(1, 9)],
              [0, F(5, 9)],
              [F(23, 63), F(8, 63)],
              [0, F(5, 9)],
              [0, 0],
              [0, 0]])
AC_HAND = np.array([[2914.0, 995.0], [995.0, 2790.0]]) / 3969.0


def test_hand_b2_strength_decisions():
    A, _ = _hand_case()
    Fm, strong = sa.strong_graph(A, EPS, bs=2)
    rows = np.repeat(np.arange(3), np.diff(Fm.indptr))
    pairs = {(int(r), int(c)) for r, c, s in zip(rows, Fm.indices, strong) if s}
    assert pairs == {(0, 1), (1, 0)}
    # the node matrix holds the squared block Frobenius norms
    dense = Fm.toarray()
    assert np.allclose(dense, [[21, 3, 0], [3, 21, 0.25], [0, 0.25, 21]], rtol=0, atol=1e-15)


def test_hand_b2_aggregates():
    A, _ = _hand_case()
    Fm, strong = sa.strong_graph(A, EPS, bs=2)
    agg, n_agg = sa.plain_aggregation(Fm, strong)
    assert list(agg) == [0, 0, -1] and n_agg == 1
    Pt = sa.tentative_prolongation(agg, n_agg, bs=2).toarray()
    assert np.array_equal(Pt, np.vstack([np.eye(2), np.eye(2), np.zeros((2, 2))]))


def test_hand_b2_filtered_matrix():
    A, _ = _hand_case()
    Fm, strong = sa.strong_graph(A, EPS, bs=2)
    AF = sa.filtered_matrix(A, Fm, strong, bs=2).toarray()
    want = np.zeros((6, 6))
    want[0:2, 0:2] = D2
    want[0:2, 2:4] = C2
    want[2:4, 0:2] = C2
    want[2:4, 2:4] = [[3.5, 1], [0, 2]]
    want[4:6, 4:6] = [[3.5, 1], [0, 2]]
    assert np.array_equal(AF, want)
    # row sums of A are preserved
    assert np.allclose(AF.sum(axis=1), A.toarray().sum(axis=1), rtol=0, atol=1e-15)


def test_hand_b2_block_inverse_and_omega():
    A, _ = _hand_case()
    Fm, strong = sa.strong_graph(A, EPS, bs=2)
    AF = sa.filtered_matrix(A, Fm, strong, bs=2)
    Dinv, ok = sa.block_diag_inverse(AF, bs=2)
    want = np.zeros((6, 6))
    want[0:2, 0:2] = [[0.25, -0.125], [0, 0.5]]
    want[2:4, 2:4] = [[2 / 7, -1 / 7], [0, 0.5]]
    want[4:6, 4:6] = [[2 / 7, -1 / 7], [0, 0.5]]
    assert np.allclose(Dinv.toarray(), want, rtol=0, atol=1e-15)
    assert list(ok) == [True, True, True]
    omega = sa.gershgorin_omega(AF, Dinv, ok, bs=2)
    assert abs(omega - 8.0 / 9.0) <= 1e-15


def test_hand_b2_prolongator_and_coarse_operator():
    A, _ = _hand_case()
    H = sa.build_hierarchy(A, eps_strong=EPS, coarse_enough=2, bs=2)
    assert H.nlevels == 2
    L0 = H.levels[0]
    assert abs(L0.omega - 8.0 / 9.0) <= 1e-15
    assert np.allclose(L0.P.toarray(), P_HAND, rtol=0, atol=1e-15)
    assert np.allclose(L0.R.toarray(), P_HAND.T, rtol=0, atol=1e-15)
    assert np.allclose(H.levels[1].A.toarray(), AC_HAND, rtol=0, atol=1e-14)
    # scalar SPAI-0 rows of the expanded matrix: row 0 = [4, 1, -1, -1]
    assert abs(L0.m[0] - 4.0 / 19.0) <= 1e-16


def test_singular_diagonal_block_is_left_out():
    # two nodes, D_0 = [[1, 1], [1, 1]] (singular), D_1 = D, coupled by C,
    # one aggregate {0, 1}; node 0 is excluded from rho and gets no smoothing term:
    #   rho = node 1's 3/2 (as in the hand case), omega = 8/9,
    #   P_0 = I (tentative), P_1 = [[1/3, 1/9], [0, 5/9]]
    # (a pseudo-inverse of D_0 would add node 0 with
    #  ||pinv(D_0) D_0||_inf + ||pinv(D_0) C||_inf = 1 + 3/4 = 7/4 > 3/2.)
    blocks = {(0, 0): [[1, 1], [1, 1]], (0, 1): C2, (1, 0): C2, (1, 1): D2}
    A, _ = _blocks_to_csr(blocks, 2, 2)
    # strength 0-1: ||C||_F^2 = 3 >= (1/49) * 2 * sqrt(21) ~ 0.187
    Fm, strong = sa.strong_graph(A, EPS, bs=2)
    AF = sa.filtered_matrix(A, Fm, strong, bs=2)
    Dinv, ok = sa.block_diag_inverse(AF, bs=2)
    assert list(ok) == [False, True]
    assert np.all(Dinv.toarray()[0:2] == 0.0)
    omega = sa.gershgorin_omega(AF, Dinv, ok, bs=2)
    assert abs(omega - 8.0 / 9.0) <= 1e-15
    H = sa.build_hierarchy(A, eps_strong=EPS, coarse_enough=2, bs=2)
    want = np.vstack([np.eye(2), [[1 / 3, 1 / 9], [0, 5 / 9]]])
    assert np.allclose(H.levels[0].P.toarray(), want, rtol=0, atol=1e-15)


def test_ill_conditioned_diagonal_block_is_inverted():
    # D_0 = [[1, 1], [1, 1 + d]] with d = 2^-20 is invertible (det = d), with
    # the exact inverse (1/d) [[1 + d, -1], [-1, 1]]: only an exactly singular
    # block may be left out, whatever its condition number (here ~4e6), so a
    # rank test with a loose tolerance must not drop it
    d = 2.0 ** -20
    blocks = {(0, 0): [[1, 1], [1, 1 + d]], (0, 1): C2, (1, 0): C2, (1, 1): D2}
    A, _ = _blocks_to_csr(blocks, 2, 2)
    Fm, strong = sa.strong_graph(A, EPS, bs=2)
    AF = sa.filtered_matrix(A, Fm, strong, bs=2)
    Dinv, ok = sa.block_diag_inverse(AF, bs=2)
    assert list(ok) == [True, True]
    want = np.array([[1 + d, -1.0], [-1.0, 1.0]]) / d
    assert np.allclose(Dinv.toarray()[0:2, 0:2], want, rtol=1e-8, atol=0)


# ---------------------------------------------------------------------------
# Kronecker invariance
# ---------------------------------------------------------------------------

def _scalar_test_matrix():
    from workloads.poisson import poisson7
    rng = np.random.default_rng(41)
    N = 9
    k = np.exp(1.5 * rng.standard_normal(N ** 3))
    A = poisson7(N, N, N, k=k)
    return _csr64(A)


def _csr64(M):
    M = sp.csr_matrix(M)
    return sp.csr_matrix((M.data, M.indices.astype(np.int64), M.indptr.astype(np.int64)), shape=M.shape)


def _kron_identity(M, b):
    """M kron I_b with interleaved unknowns: entry (i b + p, j b + q) = m_ij d_pq."""
    C = sp.coo_matrix(M)
    r = (C.row.astype(np.int64)[:, None] * b + np.arange(b)).ravel()
    c = (C.col.astype(np.int64)[:, None] * b + np.arange(b)).ravel()
    v = np.repeat(C.data, b)
    out = sp.csr_matrix((v, (r, c)), shape=(M.shape[0] * b, M.shape[1] * b))
    out.sort_indices()
    return out


@pytest.mark.parametrize("b", [2, 4])
def test_block_hierarchy_of_kronecker_product_is_scalar_hierarchy_kron_identity(b):
    As = _scalar_test_matrix()
    Ab = _kron_identity(As, b)
    Hs = sa.build_hierarchy(As, coarse_enough=40)
    Hb = sa.build_hierarchy(Ab, coarse_enough=40 * b, bs=b)
    assert Hs.nlevels >= 3
    assert Hb.nlevels == Hs.nlevels
    for l in range(Hs.nlevels - 1):
        ls, lb = Hs.levels[l], Hb.levels[l]
        assert np.array_equal(ls.agg, lb.agg)
        assert ls.n_agg == lb.n_agg
        assert abs(ls.omega - lb.omega) <= 1e-14 * ls.omega
        Pk = _kron_identity(ls.P, b)
        assert abs(Pk - lb.P).max() <= 1e-14 * abs(Pk).max()
        Ak = _kron_identity(Hs.levels[l + 1].A, b)
        assert abs(Ak - Hb.levels[l + 1].A).max() <= 1e-14 * abs(Ak).max()


# ---------------------------------------------------------------------------
# whole block solve
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("N,smoother", [(5, "spai0"), (6, "spai0"), (5, "block_spai0")])
def test_block_size4_oseen_solve_matches_direct_solve(N, smoother):
    from workloads.oseen import oseen_q1, field_deflation
    A, _ = oseen_q1(N, seed=3)
    A = sp.csr_matrix(A)
    part, nsub, Z = field_deflation(N, (1, 1, 2))
    b = np.random.default_rng(42).uniform(-1, 1, A.shape[0])
    S = OracleSolver(A, part, nsub, Z, OracleParams(solver="bicgstab", block_size=4, rtol=1e-13,
                                                    coarse_enough=40, smoother=smoother))
    # the block hierarchy really coarsens (point-block aggregates of nodes)
    assert S.M.hierarchies[0].nlevels >= 2
    out = S.solve(b)
    assert out["status"] == "ok"
    x = np.linalg.solve(A.toarray(), b)
    assert np.linalg.norm(out["x"] - x) <= 1e-10 * np.linalg.norm(x)
