"""CSR rows at the edges of the row loop's chunks (eight entries per lane):
a Poisson operator with hub rows whose lengths sit on either side of one,
two and several chunks for 8 lanes per row (64, 65, 128, 129, 200 entries)
and of the short-row forms (8, 9 entries), kept symmetric positive definite.
The outer operator product in the fixed CSR layout (8 lanes) against A v
element by element; every tuner candidate of every operator against the
first (DFAMG_TUNE_VERIFY); whole CG solves in both against the oracle."""
import os

import numpy as np
import pytest
import scipy.sparse as sp

from workloads import make_problem
from oracle import OracleSolver, OracleParams

torch = pytest.importorskip("torch")
pytestmark = [pytest.mark.gpu,
              pytest.mark.skipif(not torch.cuda.is_available(), reason="needs a GPU")]

HUB_LENGTHS = (8, 9, 64, 65, 128, 129, 200)


def _t(a):
    return torch.tensor(np.ascontiguousarray(a, dtype=np.float64), device=torch.device("cuda:0"))


def _hub_problem():
    P = make_problem("hubs", (14, 13, 12), (2, 1, 1), deflation="linear", sigma=1.0, coef_seed=31,
                     rhs="uniform", rhs_seed=32)
    A = sp.lil_matrix(P.A)
    rng = np.random.default_rng(33)
    used = set()
    hubs = []
    for length in HUB_LENGTHS:
        # a hub in subdomain 0 coupled to nodes of its own subdomain, plus a few
        # in the other one (couplings of the outer operator), as a weighted
        # graph Laplacian added to A: symmetric, diagonal dominance kept
        cand = np.flatnonzero(P.part == 0)
        h = int(rng.choice([c for c in cand if c not in used]))
        used.add(h)
        have = A.rows[h]
        extra = length - len(have)
        pool_own = [c for c in cand if c not in used and c not in have]
        pool_other = [c for c in np.flatnonzero(P.part == 1) if c not in have]
        n_other = min(3, extra // 4)
        js = list(rng.choice(pool_own, extra - n_other, replace=False)) + \
            list(rng.choice(pool_other, n_other, replace=False))
        for j in js:
            w = 0.05 * (1.0 + rng.random())
            A[h, j] = A[h, j] - w
            A[j, h] = A[j, h] - w
            A[h, h] = A[h, h] + w
            A[j, j] = A[j, j] + w
        hubs.append(h)
    A = sp.csr_matrix(A)
    A.sort_indices()
    lengths = np.diff(A.indptr)[hubs]
    assert list(lengths) == list(HUB_LENGTHS), lengths
    assert abs(A - A.T).max() == 0.0
    return P.__class__(P.name, A, P.part, P.nsub, P.Z, P.b, P.x0), hubs


def test_csr_chunk_edges_product_and_solve():
    import paper_1710_03940_amd as L
    P, hubs = _hub_problem()
    v = np.random.default_rng(5).standard_normal(P.n)
    ref = P.A @ v
    S = L.Solver(P.A, P.part, P.nsub, P.Z, coarse_enough=40, spmv_format="csr", autotune=0)
    out = _t(np.zeros(P.n))
    S.apply(L._lib.OP_SPMV, _t(v), out)
    got = out.cpu().numpy()
    assert np.abs(got - ref).max() <= 1e-13 * np.abs(ref).max()
    assert np.abs(got[hubs] - ref[hubs]).max() <= 1e-13 * np.abs(ref).max()
    x = _t(np.zeros(P.n))
    res = S.solve(_t(P.b), x)
    lay = S.stats()["layouts"]
    S.close()
    assert "csr8" in lay, lay
    orc = OracleSolver(P.A, P.part, P.nsub, P.Z, OracleParams(coarse_enough=40)).solve(P.b)
    assert res["status"] == 0 and abs(res["iters"] - orc["iters"]) <= 2
    assert np.linalg.norm(x.cpu().numpy() - orc["x"]) <= 1e-6 * np.linalg.norm(orc["x"])


def test_csr_chunk_edges_every_candidate(capfd):
    import paper_1710_03940_amd as L
    P, hubs = _hub_problem()
    os.environ["DFAMG_TUNE_VERIFY"] = "1"
    try:
        S = L.Solver(P.A, P.part, P.nsub, P.Z, coarse_enough=40, spmv_format="csr", autotune=1, verbose=2)
    finally:
        del os.environ["DFAMG_TUNE_VERIFY"]
    v = np.random.default_rng(6).standard_normal(P.n)
    out = _t(np.zeros(P.n))
    S.apply(L._lib.OP_SPMV, _t(v), out)
    x = _t(np.zeros(P.n))
    res = S.solve(_t(P.b), x)
    S.close()
    err = capfd.readouterr().err
    assert err.count("layout check") >= 10
    ref = P.A @ v
    assert np.abs(out.cpu().numpy() - ref).max() <= 1e-13 * np.abs(ref).max()
    assert res["status"] == 0 and res["relres_true"] <= 1e-8 * 1.01
