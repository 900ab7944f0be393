"""Pins of the CPU oracle against facts that do not come from the oracle itself:
values printed in the paper, closed forms, algebraic invariants, textbook
special cases and brute-force dense solves on tiny inputs."""
import numpy as np
import pytest
import scipy.sparse as sp
import scipy.sparse.linalg as spla

from workloads import (poisson7, box_partition, constant_deflation,
                       linear_deflation, grid_coords, tiny_problem,
                       make_problem, config_small_poisson)
from workloads.convdiff import convection_diffusion7
from oracle import OracleSolver, OracleParams, OracleError
from oracle import sa, _aggregate
from oracle.deflation import Deflation, full_basis
from oracle.krylov import deflated_cg


# --------------------------------------------------------------------------
# generator: sizes printed in the paper
# --------------------------------------------------------------------------

def test_poisson_150_sizes_match_paper():
    # Implementation section: the 150^3 problem has 3,375,000 unknowns and
    # 23,490,000 nonzeros.
    A = poisson7(150)
    assert A.shape == (3375000, 3375000)
    assert A.nnz == 23490000


def test_poisson_32_size_and_stencil():
    A = poisson7(32)
    assert A.nnz == 7 * 32**3 - 6 * 32**2 == 223232
    assert np.all(A.diagonal() == 6.0)
    off = A - sp.diags(A.diagonal())
    assert set(np.unique(off.data)) == {-1.0}


def test_partition_piece_sizes():
    part, nsub = box_partition(150, 150, 150, 4, 4, 4)
    assert nsub == 64
    cnt = np.bincount(part)
    assert cnt.min() == 37**3 and cnt.max() == 38**3


# --------------------------------------------------------------------------
# deflation: closed forms and projector invariants
# --------------------------------------------------------------------------

def test_E_closed_form_slabs():
    # 32^3 unit Poisson, 8 slabs of 32x32x4, constant Z: E_ss = 1^T A_ss 1 =
    # number of faces leaving the slab = 4*32*4 (side walls) + 2*32*32
    # (neighbouring slab or end wall) = 2560; E_{s,s+1} = -(faces shared) = -1024.
    P = config_small_poisson()
    D = Deflation(P.A, P.part, P.nsub, P.Z)
    expect = (np.diag(np.full(8, 2560.0)) + np.diag(np.full(7, -1024.0), 1)
              + np.diag(np.full(7, -1024.0), -1))
    assert np.array_equal(D.E, expect)
    # sum of all entries = 1^T A 1 = number of Dirichlet faces = 6 N^2
    assert D.E.sum() == 6 * 32**2


@pytest.mark.parametrize("defl", ["constant", "linear"])
def test_projector_invariants(defl):
    P = tiny_problem(N=8, pieces=(2, 2, 1), deflation=defl, sigma=1.0, seed=3)
    D = Deflation(P.A, P.part, P.nsub, P.Z)
    rng = np.random.default_rng(5)
    v = rng.standard_normal(P.n)
    Pv = D.project(v)
    # P is a projection (eq. after the deflated system)
    assert np.linalg.norm(D.project(Pv) - Pv) <= 1e-12 * np.linalg.norm(v)
    # Z^T P v = 0
    assert np.linalg.norm(D.Z.T @ Pv) <= 1e-12 * np.linalg.norm(v) * np.abs(P.Z).max()
    # P A symmetric for symmetric A; E symmetric positive definite
    Ad = P.A.toarray()
    PA = np.column_stack([D.project(Ad[:, j]) for j in range(P.n)])
    assert np.abs(PA - PA.T).max() <= 1e-12 * np.abs(Ad).max()
    assert np.abs(D.E - D.E.T).max() <= 1e-13 * np.abs(D.E).max()
    assert np.linalg.eigvalsh(D.E).min() > 0
    # exact coarse solve
    t1 = rng.standard_normal(D.m)
    t2 = D.solve_E(t1)
    assert np.linalg.norm(D.E @ t2 - t1) <= 1e-12 * np.linalg.norm(t1)


def _laplace_eigvec(N, k):
    i = np.arange(1, N + 1)
    s = [np.sin(kd * np.pi * i / (N + 1)) for kd in k]
    v = np.einsum("k,j,i->kji", s[2], s[1], s[0]).ravel()
    lam = sum(4 * np.sin(kd * np.pi / (2 * (N + 1))) ** 2 for kd in k)
    return v, lam


def test_eigenvalue_deflation_removes_eigenvalues():
    # Section "Subdomain deflation", remarks: with Z = eigenvectors of A the
    # deflated operator P A has those eigenvalues replaced by zero.
    N = 6
    A = poisson7(N)
    modes = [(1, 1, 1), (2, 1, 1), (1, 2, 1), (1, 1, 2), (2, 2, 1)]
    Z = np.column_stack([_laplace_eigvec(N, k)[0] for k in modes])
    lams = np.array([_laplace_eigvec(N, k)[1] for k in modes])
    D = Deflation(A, np.zeros(N**3, dtype=np.int32), 1, Z)
    Ad = A.toarray()
    PA = np.column_stack([D.project(Ad[:, j]) for j in range(N**3)])
    spec_pa = np.sort(np.linalg.eigvalsh(0.5 * (PA + PA.T)))
    spec_a = list(np.sort(np.linalg.eigvalsh(Ad)))
    for lam in lams:          # remove one copy of each deflated eigenvalue
        j = int(np.argmin(np.abs(np.array(spec_a) - lam)))
        assert abs(spec_a[j] - lam) < 1e-10
        spec_a.pop(j)
    expect = np.sort(np.r_[np.zeros(len(modes)), spec_a])
    assert np.abs(spec_pa - expect).max() < 1e-10


def test_rank_deficient_Z_rejected():
    # linear deflation on a one-plane-thick slab: the z column is constant
    # (zero after centering), so the local block has rank 3 < 4
    P = make_problem("slab", (6, 6, 4), (1, 1, 4), deflation="linear")
    with pytest.raises(OracleError):
        OracleSolver(P.A, P.part, P.nsub, P.Z)


# --------------------------------------------------------------------------
# smoothed aggregation: closed forms and hand-derived cases
# --------------------------------------------------------------------------

def test_spai0_and_omega_closed_forms():
    # SPAI-0 of the unit stencil: interior row 6 / (36 + 6) = 1/7; a row
    # missing one neighbour (Dirichlet or dropped): 6 / (36 + 5) = 6/41.
    A = poisson7(6)
    m = sa.smoother_diagonal(A, "spai0")
    idx = np.arange(216).reshape(6, 6, 6)
    assert m[idx[2, 2, 2]] == pytest.approx(1 / 7, rel=1e-15)
    assert m[idx[2, 2, 0]] == pytest.approx(6 / 41, rel=1e-15)
    assert m[idx[0, 0, 0]] == pytest.approx(6 / 39, rel=1e-15)
    mj = sa.smoother_diagonal(A, "jacobi", 0.8)
    assert np.allclose(mj, 0.8 / 6)
    # all connections strong (1 >= 0.0064 * 36); Gershgorin bound of
    # D^{-1} A: interior row (6 + 6) / 6 = 2, so omega = (4/3) / 2 = 2/3
    F, strong = sa.strong_graph(A, 0.08)
    assert strong.sum() == A.nnz - A.shape[0]
    AF = sa.filtered_matrix(A, F, strong)
    assert (AF != A).nnz == 0
    Dinv, ok = sa.block_diag_inverse(AF)
    assert sa.gershgorin_omega(AF, Dinv, ok) == pytest.approx(2 / 3, rel=1e-14)


def _chain(n):
    return sp.diags([-np.ones(n - 1), 2 * np.ones(n), -np.ones(n - 1)],
                    [-1, 0, 1], format="csr")


def test_aggregation_hand_derived_chain():
    # 1D chain of 7: pass 1 takes {0,1}, skips 2 (neighbour 1 taken), takes
    # {2,3,4} from node 3, skips 5, takes {5,6} from node 6.
    A = _chain(7)
    F, strong = sa.strong_graph(A, 0.08)
    agg, nagg = sa.plain_aggregation(F, strong)
    assert nagg == 3
    assert agg.tolist() == [0, 0, 1, 1, 1, 2, 2]


def test_aggregation_hand_derived_grid():
    # 3x3 grid (5-point): pass 1 takes {0,1,3} from node 0 and {2,4,5,8} from
    # node 5; pass 2 puts 6 with its first aggregated neighbour 3 (equal
    # weights) and 7 with 4.
    n = 3
    T = _chain(n)
    A = (sp.kron(sp.eye(n), T) + sp.kron(T, sp.eye(n))).tocsr()
    A.sort_indices()
    F, strong = sa.strong_graph(A, 0.08)
    agg, nagg = sa.plain_aggregation(F, strong)
    assert nagg == 2
    assert agg.tolist() == [0, 0, 1, 0, 1, 1, 0, 1, 1]


def test_aggregation_pass2_weight_rule():
    # path 0-1-2 and 3 attached to 1 and 2, with node 4 attached to 0
    # (light) and 2 (heavy); after pass 1 = {0,1,3? }, hand-traced below.
    # Adjacency (symmetric weights):
    #   0-1:1  1-2:1  0-4:1  2-4:4  2-3:1  3-5:1  5-6:1
    edges = {(0, 1): 1, (1, 2): 1, (0, 4): 1, (2, 4): 4, (2, 3): 1,
             (3, 5): 1, (5, 6): 1}
    n = 7
    Ad = np.zeros((n, n))
    for (i, j), w in edges.items():
        Ad[i, j] = Ad[j, i] = -w
    np.fill_diagonal(Ad, -Ad.sum(axis=1) + 1.0)
    A = sp.csr_matrix(Ad)
    A.sort_indices()
    F, strong = sa.strong_graph(A, 0.08)
    agg, nagg = sa.plain_aggregation(F, strong)
    # pass 1: node 0 (nbrs 1,4) free -> agg0 = {0,1,4}
    #         node 2 (nbrs 1,3,4): taken; node 3 (nbrs 2,5) free -> agg1 = {2,3,5}
    #         node 6 (nbr 5): taken
    # pass 2: node 6 -> aggregate of 5 (agg1)
    assert agg.tolist() == [0, 0, 1, 1, 0, 1, 1]
    assert nagg == 2


def test_aggregation_pass2_heaviest_and_tie():
    # node 4 sees aggregated neighbours 1 (agg0, weight 1) and 3 (agg1,
    # weight 2): joins agg1.  Node 5 sees 0 (agg0) and 2 (agg1) with equal
    # weights: joins agg0 (smaller index).
    edges = {(0, 1): 1, (2, 3): 1, (1, 4): 1, (3, 4): 2, (0, 5): 1, (2, 5): 1,
             (4, 5): 1}
    n = 6
    Ad = np.zeros((n, n))
    for (i, j), w in edges.items():
        Ad[i, j] = Ad[j, i] = -w
    np.fill_diagonal(Ad, -Ad.sum(axis=1) + 1.0)
    A = sp.csr_matrix(Ad)
    A.sort_indices()
    F, strong = sa.strong_graph(A, 0.08)
    agg, _ = sa.plain_aggregation(F, strong)
    # pass 1: node 0 (nbrs 1,5) -> agg0 = {0,1,5}; node 2 (nbrs 3,5): 5 taken;
    # node 3 (nbrs 2,4) -> agg1 = {2,3,4}.  All aggregated in pass 1.
    assert agg.tolist() == [0, 0, 1, 1, 1, 0]


def test_aggregation_pass2_and_pass3_hand_case():
    # 0-1, 1-2, 2-3, 3-4, 4-5 chain plus isolated node 6 (no strong link)
    # and a pendant node 7 attached to 2 only.
    edges = {(0, 1): 1, (1, 2): 1, (2, 3): 1, (3, 4): 1, (4, 5): 1, (2, 7): 1}
    n = 8
    Ad = np.zeros((n, n))
    for (i, j), w in edges.items():
        Ad[i, j] = Ad[j, i] = -w
    np.fill_diagonal(Ad, -Ad.sum(axis=1) + 1.0)
    A = sp.csr_matrix(Ad)
    A.sort_indices()
    F, strong = sa.strong_graph(A, 0.08)
    agg, nagg = sa.plain_aggregation(F, strong)
    # pass 1: 0 -> {0,1}; 2 (nbrs 1,3,7): 1 taken; 3 (nbrs 2,4) -> {2,3,4};
    #         5 (nbr 4) taken; 7 (nbr 2) taken.
    # pass 2: 5 -> agg of 4 (1); 7 -> agg of 2 (1).  6 isolated.
    assert agg.tolist() == [0, 0, 1, 1, 1, 1, -1, 1]
    assert nagg == 2


def test_aggregation_pass3_never_needed():
    # A node skipped by pass 1 had an aggregated strong neighbour at that
    # moment, so pass 2 always places it; pass 3 therefore leaves every
    # aggregate as pass 2 left it.  Check on random asymmetric graphs that
    # after pass 2 no node with a neighbourhood is left.
    rng = np.random.default_rng(3)
    for trial in range(5):
        n = 300
        M = sp.random(n, n, density=0.02, random_state=trial, format="csr")
        M.sort_indices()
        rows = np.repeat(np.arange(n), np.diff(M.indptr))
        strong = (rng.random(M.nnz) < 0.5) & (M.indices != rows)
        agg, nagg = _aggregate.aggregate_py(M.indptr, M.indices, np.ones(M.nnz), strong)
        has = np.bincount(rows[strong], minlength=n) > 0
        assert np.all(agg[has] >= 0)


@pytest.mark.parametrize("seed", range(6))
def test_c_aggregation_matches_definition(seed):
    rng = np.random.default_rng(seed)
    n = 400
    dens = 0.01 + 0.02 * seed
    M = sp.random(n, n, density=dens, random_state=seed, format="csr")
    if seed % 2 == 0:
        M = M + M.T
    M = M.tocsr()
    M.sort_indices()
    strong = rng.random(M.nnz) < 0.6
    rows = np.repeat(np.arange(n), np.diff(M.indptr))
    strong &= M.indices != rows
    w = np.round(rng.random(M.nnz) * 4) + 1     # many ties
    a1, n1 = _aggregate.aggregate_py(M.indptr, M.indices, w, strong)
    a2, n2 = _aggregate.aggregate_c(M.indptr, M.indices, w, strong)
    assert n1 == n2
    assert np.array_equal(a1, a2)


def test_aggregates_partition_non_isolated_nodes():
    P = tiny_problem(N=10, pieces=(1, 1, 1), sigma=2.0, seed=4)
    A = P.A
    for eps in (0.08, 0.25, 0.5):
        F, strong = sa.strong_graph(A, eps)
        agg, nagg = sa.plain_aggregation(F, strong)
        rows = np.repeat(np.arange(A.shape[0]), np.diff(F.indptr))
        has_nbr = np.bincount(rows[strong], minlength=A.shape[0]) > 0
        assert np.all(agg[has_nbr] >= 0)
        assert set(np.unique(agg[agg >= 0])) == set(range(nagg))


def test_smoothed_prolongation_chain_hand_values():
    # 1D chain of 7, aggregates [0,0,1,1,1,2,2], omega = 2/3, D = 2:
    # P = (I - (1/3) A) P_t.  Row 0: (A P_t)[0] = (2-1, 0, 0) -> P = (2/3, 0, 0)
    # row 1: (A P_t)[1] = (-1+2, -1, 0) -> (2/3, 1/3, 0)
    # row 3: (A P_t)[3] = (0, -1+2-1, 0) -> (0, 1, 0)
    A = _chain(7)
    H = sa.build_hierarchy(A, coarse_enough=2)
    lvl = H.levels[0]
    assert lvl.omega == pytest.approx(2 / 3, rel=1e-14)
    P = lvl.P.toarray()
    assert np.allclose(P[0], [2 / 3, 0, 0], atol=1e-15)
    assert np.allclose(P[1], [2 / 3, 1 / 3, 0], atol=1e-15)
    assert np.allclose(P[3], [0, 1, 0], atol=1e-15)
    assert np.allclose(P[2], [1 / 3, 2 / 3, 0], atol=1e-15)
    # Galerkin coarse operator is P^T A P, symmetric
    Ac = H.levels[1].A.toarray()
    assert np.allclose(Ac, Ac.T, atol=1e-15)


def test_smoothed_constant_preserved():
    # rows of A_F with zero row sum keep P 1_c = 1 (constant preserved)
    P = tiny_problem(N=8, pieces=(1, 1, 1), sigma=1.0, seed=2)
    A = P.A
    F, strong = sa.strong_graph(A, 0.08)
    agg, nagg = sa.plain_aggregation(F, strong)
    Pt = sa.tentative_prolongation(agg, nagg)
    AF = sa.filtered_matrix(A, F, strong)
    assert np.allclose(AF @ np.ones(A.shape[0]), A @ np.ones(A.shape[0]))
    Dinv, ok = sa.block_diag_inverse(AF)
    om = sa.gershgorin_omega(AF, Dinv, ok)
    Pm = sa.smoothed_prolongation(AF, Pt, om, Dinv)
    rs = AF @ np.ones(A.shape[0])
    Pt1 = Pt @ np.ones(nagg)
    # a row with zero A_F row sum whose stencil lies inside aggregated nodes
    rows_ok = np.flatnonzero((np.abs(rs) < 1e-12) & (Pt1 == 1))
    nbr_all_agg = np.array([np.all(Pt1[AF.indices[AF.indptr[i]:AF.indptr[i + 1]]] == 1)
                            for i in rows_ok], dtype=bool)
    sel = rows_ok[nbr_all_agg]
    assert sel.size > 0
    assert np.allclose((Pm @ np.ones(nagg))[sel], 1.0, atol=1e-13)


# --------------------------------------------------------------------------
# preconditioner: symmetry and positivity of the V-cycle
# --------------------------------------------------------------------------

@pytest.mark.parametrize("smoother", ["spai0", "jacobi"])
def test_vcycle_symmetric_positive(smoother):
    P = tiny_problem(N=10, pieces=(2, 1, 1), sigma=1.0, seed=7)
    S = OracleSolver(P.A, P.part, P.nsub, P.Z,
                     OracleParams(coarse_enough=20, smoother=smoother))
    assert max(len(h) for h in S.hierarchy_summary()) >= 3
    rng = np.random.default_rng(0)
    for _ in range(3):
        u, v = rng.standard_normal((2, P.n))
        Mu, Mv = S.apply_precond(u), S.apply_precond(v)
        assert abs(u @ Mv - v @ Mu) <= 1e-12 * np.linalg.norm(u) * np.linalg.norm(v)
        assert u @ Mu > 0


# --------------------------------------------------------------------------
# whole solves: brute force, textbook reductions, manufactured solution
# --------------------------------------------------------------------------

@pytest.mark.parametrize("N,pieces,defl", [
    (4, (1, 1, 1), "constant"), (6, (1, 1, 2), "constant"),
    (6, (2, 2, 1), "linear"), (8, (2, 2, 2), "constant"),
    (8, (2, 2, 2), "linear"), (8, (1, 1, 8), "constant")])
def test_cg_matches_dense_solve(N, pieces, defl):
    P = tiny_problem(N=N, pieces=pieces, deflation=defl, sigma=1.0, seed=N)
    S = OracleSolver(P.A, P.part, P.nsub, P.Z,
                     OracleParams(rtol=1e-13, coarse_enough=8))
    res = S.solve(P.b)
    xd = np.linalg.solve(P.A.toarray(), P.b)
    assert res["status"] == "ok"
    assert np.linalg.norm(res["x"] - xd) <= 1e-10 * np.linalg.norm(xd)
    assert res["relres_true"] <= 1e-12


@pytest.mark.parametrize("pieces,defl", [((1, 1, 1), "constant"),
                                         ((2, 1, 2), "constant"),
                                         ((2, 2, 1), "linear")])
def test_bicgstab_nonsymmetric_matches_dense_solve(pieces, defl):
    N = 8
    A = convection_diffusion7(N, peclet=3.0)
    base = tiny_problem(N=N, pieces=pieces, deflation=defl, seed=1)
    S = OracleSolver(A, base.part, base.nsub, base.Z,
                     OracleParams(solver="bicgstab", rtol=1e-13, coarse_enough=10))
    res = S.solve(base.b)
    xd = np.linalg.solve(A.toarray(), base.b)
    assert res["status"] == "ok"
    assert np.linalg.norm(res["x"] - xd) <= 1e-10 * np.linalg.norm(xd)


@pytest.mark.parametrize("ell", [1, 2, 3])
@pytest.mark.parametrize("pieces,defl", [((1, 1, 1), "constant"), ((2, 2, 1), "linear")])
def test_bicgstabl_nonsymmetric_matches_dense_solve(ell, pieces, defl):
    N = 8
    A = convection_diffusion7(N, peclet=3.0)
    base = tiny_problem(N=N, pieces=pieces, deflation=defl, seed=2)
    S = OracleSolver(A, base.part, base.nsub, base.Z,
                     OracleParams(solver="bicgstabl", ell=ell, rtol=1e-13, coarse_enough=10))
    res = S.solve(base.b)
    xd = np.linalg.solve(A.toarray(), base.b)
    assert res["status"] == "ok"
    assert np.linalg.norm(res["x"] - xd) <= 1e-10 * np.linalg.norm(xd)


def test_bicgstabl_with_ell_1_is_bicgstab():
    """BiCGStab(1) is BiCGStab: the same residual after every full step
    (Sleijpen & Fokkema's construction reduces to van der Vorst's)."""
    N = 10
    A = convection_diffusion7(N, peclet=2.0)
    base = tiny_problem(N=N, pieces=(2, 1, 1), deflation="linear", seed=3)
    kw = dict(rtol=1e-11, coarse_enough=20)
    r1 = OracleSolver(A, base.part, base.nsub, base.Z,
                      OracleParams(solver="bicgstab", **kw)).solve(base.b)
    rl = OracleSolver(A, base.part, base.nsub, base.Z,
                      OracleParams(solver="bicgstabl", ell=1, **kw)).solve(base.b)
    k = min(len(r1["history"]), len(rl["history"])) - 1   # the last may be a half step
    assert k >= 5
    assert np.allclose(rl["history"][:k], r1["history"][:k], rtol=1e-8, atol=0)
    assert np.linalg.norm(rl["x"] - r1["x"]) <= 1e-8 * np.linalg.norm(r1["x"])


@pytest.mark.parametrize("ell", [2, 3])
def test_bicgstabl_cycle_properties(ell):
    """Per cycle: the BiCG part leaves the last residual orthogonal to the
    shadow vector, and the minimal-residual part returns the least-squares
    residual of r_0 over r_1 .. r_ell (orthogonal to each of them, and equal
    to the one numpy's lstsq gives)."""
    from oracle.krylov import deflated_bicgstabl
    N = 8
    A = convection_diffusion7(N, peclet=4.0)
    base = tiny_problem(N=N, pieces=(2, 1, 1), deflation="constant", seed=4)
    S = OracleSolver(A, base.part, base.nsub, base.Z, OracleParams(coarse_enough=10))
    seen = []

    def observe(k, before, after, rt):
        R = np.column_stack(before[1:])
        g, *_ = np.linalg.lstsq(R, before[0], rcond=None)
        ls = before[0] - R @ g
        scale = np.linalg.norm(before[0])
        assert np.linalg.norm(after - ls) <= 1e-9 * scale
        for j in range(1, ell + 1):
            assert abs(after @ before[j]) <= 1e-9 * scale * np.linalg.norm(before[j])
        assert abs(before[ell - 1] @ rt) <= 1e-9 * np.linalg.norm(before[ell - 1]) * np.linalg.norm(rt)
        seen.append(k)

    deflated_bicgstabl(A, S.defl, S.precond, base.b, np.zeros(A.shape[0]), 1e-10, 50,
                       ell=ell, observe=observe)
    assert len(seen) >= 2


def test_plain_cg_reduction_matches_scipy():
    # Z empty and M = I: textbook CG; scipy's cg counts the same iterations
    P = tiny_problem(N=12, pieces=(1, 1, 1), sigma=1.0, seed=9)
    Z0 = np.zeros((P.n, 0))
    S = OracleSolver(P.A, P.part, 1, Z0, OracleParams(precond="identity"))
    res = S.solve(P.b)
    count = [0]
    x, info = spla.cg(P.A, P.b, rtol=1e-8, atol=0.0, maxiter=1000,
                      callback=lambda xk: count.__setitem__(0, count[0] + 1))
    assert info == 0
    assert abs(res["iters"] - count[0]) <= 1
    assert np.linalg.norm(res["x"] - x) <= 1e-6 * np.linalg.norm(x)


def test_manufactured_solution_second_order():
    # u = sin(pi x) sin(pi y) sin(pi z), -Lap u = 3 pi^2 u, b = h^2 f for the
    # unscaled stencil; the max error should drop ~4x when h halves
    errs = []
    for N in (15, 31):
        h = 1.0 / (N + 1)
        X = grid_coords(N, N, N, h)
        u = np.prod(np.sin(np.pi * X), axis=1)
        b = h * h * 3 * np.pi**2 * u
        part, nsub = box_partition(N, N, N, 2, 2, 2)
        Z = linear_deflation(X, part, nsub)
        A = poisson7(N)
        S = OracleSolver(A, part, nsub, Z, OracleParams(rtol=1e-12))
        res = S.solve(b)
        errs.append(np.abs(res["x"] - u).max())
    ratio = errs[0] / errs[1]
    assert 3.6 < ratio < 4.4


def test_cg_energy_error_monotone_and_Z_orthogonal_residual():
    P = tiny_problem(N=10, pieces=(2, 2, 1), deflation="linear", sigma=1.0, seed=11)
    S = OracleSolver(P.A, P.part, P.nsub, P.Z, OracleParams(coarse_enough=30))
    xs = np.linalg.solve(P.A.toarray(), P.b)
    prev = np.inf
    full = S.solve(P.b)
    for k in range(1, full["iters"] + 1):
        r = S.solve(P.b, maxiter=k)
        x = r["x"]
        e = x - xs
        en = np.sqrt(e @ (P.A @ e))
        assert en <= prev * (1 + 1e-12)
        prev = en
        res_true = P.b - P.A @ x
        # b - A x = P(b - A y) lies in the null space of Z^T
        assert np.linalg.norm(S.defl.Z.T @ res_true) <= 1e-10 * np.linalg.norm(P.b)


def test_recovery_residual_equals_projected_residual():
    P = tiny_problem(N=8, pieces=(2, 1, 1), deflation="linear", sigma=1.0, seed=6)
    S = OracleSolver(P.A, P.part, P.nsub, P.Z)
    y = np.random.default_rng(1).standard_normal(P.n)
    x = S.defl.recover(P.b, y)
    lhs = P.b - P.A @ x
    rhs = S.defl.project(P.b - P.A @ y)
    assert np.linalg.norm(lhs - rhs) <= 1e-12 * np.linalg.norm(P.b - P.A @ y)


def test_basis_invariance():
    # P and therefore every iterate depend on span(Z) only: scaling and
    # mixing the columns of each local block leaves the solve unchanged
    P = tiny_problem(N=10, pieces=(2, 1, 2), deflation="linear", sigma=1.0, seed=8)
    S1 = OracleSolver(P.A, P.part, P.nsub, P.Z, OracleParams(coarse_enough=30))
    R = np.array([[2.0, 0.5, 0, 0], [0, 3.0, 0, 0.1], [0, 0.2, 0.5, 0],
                  [1.0, 0, 0, 4.0]])
    S2 = OracleSolver(P.A, P.part, P.nsub, P.Z @ R, OracleParams(coarse_enough=30))
    r1, r2 = S1.solve(P.b), S2.solve(P.b)
    assert r1["iters"] == r2["iters"]
    assert np.linalg.norm(r1["x"] - r2["x"]) <= 1e-10 * np.linalg.norm(r1["x"])
    assert np.allclose(r1["history"], r2["history"], rtol=1e-7, atol=0)


def test_zero_rhs_and_maxiter():
    P = tiny_problem(N=8, pieces=(2, 1, 1))
    S = OracleSolver(P.A, P.part, P.nsub, P.Z)
    r = S.solve(np.zeros(P.n))
    assert r["iters"] == 0 and np.all(r["x"] == 0) and r["status"] == "ok"
    r = S.solve(P.b, maxiter=1)
    assert r["iters"] == 1 and r["status"] == "noconv"


def test_invalid_inputs():
    P = tiny_problem(N=4, pieces=(1, 1, 2))
    with pytest.raises(OracleError):
        OracleSolver(P.A, P.part, 3, P.Z)                # empty subdomain 2
    bad = P.part.copy(); bad[0] = 7
    with pytest.raises(OracleError):
        OracleSolver(P.A, bad, 2, P.Z)
    S = OracleSolver(P.A, P.part, P.nsub, P.Z)
    b = P.b.copy(); b[3] = np.nan
    with pytest.raises(OracleError):
        S.solve(b)


# --------------------------------------------------------------------------
# qualitative trends stated in the paper
# --------------------------------------------------------------------------

def _iters(dims, pieces, defl, precond="amg"):
    P = make_problem("t", dims, pieces, deflation=defl)
    S = OracleSolver(P.A, P.part, P.nsub, P.Z, OracleParams(precond=precond,
                                                             coarse_enough=50))
    return S.solve(P.b)["iters"]


def test_trend_more_subdomains_fewer_iterations_with_deflation():
    # Section "Domain decomposition approaches": more subdomains improve the
    # deflation space and reduce iterations (deflated CG without AMG)
    it = [_iters((16, 16, 16), (k, k, k), "linear", "identity") for k in (1, 2, 4)]
    assert it[0] > it[1] > it[2]


def test_trend_linear_not_worse_than_constant():
    # Section "Linear deflation": the better approximation needs fewer
    # iterations
    assert _iters((16, 16, 16), (2, 2, 2), "linear") <= \
        _iters((16, 16, 16), (2, 2, 2), "constant")


def test_two_grid_error_propagation_textbook_form():
    # For a two-level hierarchy with exact coarse solve the V(1,1) cycle
    # B satisfies the textbook identity
    #   I - B A = (I - M A)(I - P A_c^{-1} R A)(I - M A),  M = diag(m)
    # and its error propagation is a contraction in the A-norm.
    from oracle.vcycle import vcycle
    P = tiny_problem(N=7, pieces=(1, 1, 1), sigma=1.0, seed=12)
    H = sa.build_hierarchy(P.A, coarse_enough=100)
    assert H.nlevels == 2
    A = P.A.toarray()
    n = A.shape[0]
    B = np.column_stack([vcycle(H, 0, e) for e in np.eye(n)])
    lvl = H.levels[0]
    M = np.diag(lvl.m)
    Pm, Rm = lvl.P.toarray(), lvl.R.toarray()
    Ac = Rm @ A @ Pm
    I = np.eye(n)
    S = I - M @ A
    C = I - Pm @ np.linalg.solve(Ac, Rm @ A)
    assert np.abs((I - B @ A) - S @ C @ S).max() < 1e-12
    rho = np.abs(np.linalg.eigvals(I - B @ A)).max()
    assert rho < 1.0


def test_single_level_is_exact_solve():
    # a block no larger than coarse_enough is solved exactly
    P = tiny_problem(N=5, pieces=(1, 1, 1), sigma=1.0, seed=1)
    H = sa.build_hierarchy(P.A, coarse_enough=500)
    from oracle.vcycle import vcycle
    assert H.nlevels == 1
    f = np.random.default_rng(0).standard_normal(P.n)
    assert np.allclose(P.A @ vcycle(H, 0, f), f, atol=1e-12)


# --------------------------------------------------------------------------
# block SPAI-0
# --------------------------------------------------------------------------

def test_block_spai0_scalar_case_is_spai0():
    A = sp.csr_matrix(convection_diffusion7(5, peclet=2.0))
    Mb = sa.block_spai0(A, 1)
    assert np.allclose(Mb.diagonal(), sa.smoother_diagonal(A, "spai0"), rtol=1e-14, atol=0)
    assert Mb.nnz == A.shape[0]


def test_block_spai0_inverts_block_diagonal_matrices():
    rng = np.random.default_rng(3)
    blocks = [rng.standard_normal((4, 4)) + 4 * np.eye(4) for _ in range(5)]
    A = sp.block_diag(blocks, format="csr")
    M = sa.block_spai0(A, 4)
    assert np.allclose((M @ A).toarray(), np.eye(20), atol=1e-12)


def test_block_spai0_is_the_frobenius_minimiser():
    """||I - M A||_F grows under any perturbation of the diagonal blocks
    (least-squares optimality), and its gradient vanishes."""
    from workloads import config_oseen
    A = config_oseen(N=4, pieces=(1, 1, 1)).A
    M = sa.block_spai0(A, 4).toarray()
    Ad = A.toarray()
    n = Ad.shape[0]
    base = np.linalg.norm(np.eye(n) - M @ Ad)
    rng = np.random.default_rng(5)
    mask = sp.block_diag([np.ones((4, 4))] * (n // 4)).toarray()
    for _ in range(5):
        D = rng.standard_normal((n, n)) * mask * 1e-3
        assert np.linalg.norm(np.eye(n) - (M + D) @ Ad) > base
    grad = ((np.eye(n) - M @ Ad) @ Ad.T) * mask
    assert np.abs(grad).max() <= 1e-10 * np.abs(Ad).max()
