"""The BSR4 layout (4 x 4 blocks, one column index per block) on the
point-block Oseen operator: whole solves against the oracle with every
operator forced into BSR4, the single operator product element by element,
and BSR4 among the tuner's candidates."""
import numpy as np
import pytest

from workloads import config_oseen
from oracle import OracleSolver, OracleParams

torch = pytest.importorskip("torch")
pytestmark = [pytest.mark.gpu,
              pytest.mark.skipif(not torch.cuda.is_available(), reason="needs a GPU")]


def _t(a):
    return torch.tensor(np.ascontiguousarray(a, dtype=np.float64), device=torch.device("cuda:0"))


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_bsr4_bicgstab_parity(precision):
    import paper_1710_03940_amd as L
    P = config_oseen(N=12, pieces=(2, 2, 1))
    ref = OracleSolver(P.A, P.part, P.nsub, P.Z, OracleParams(solver="bicgstab", block_size=4,
                                                              coarse_enough=100)).solve(P.b)
    S = L.Solver(P.A, P.part, P.nsub, P.Z, solver="bicgstab", block_size=4, coarse_enough=100,
                 spmv_format="bsr4", precision=precision)
    x = _t(np.zeros(P.n))
    out = S.solve(_t(P.b), x)
    lay = S.stats()["layouts"]
    S.close()
    print(lay, out["iters"], ref["iters"], out["relres_true"], flush=True)
    assert lay.count("bsr4") >= 4 and "sell" not in lay and "csr" not in lay, lay
    assert out["status"] == 0 and out["relres_true"] <= 1e-8
    if precision == "fp64":
        assert abs(out["iters"] - ref["iters"]) <= 2
    else:
        assert out["iters"] <= 1.15 * ref["iters"] + 1
    xs = x.cpu().numpy()
    assert np.linalg.norm(xs - ref["x"]) <= 1e-6 * np.linalg.norm(ref["x"])


def test_bsr4_operator_product():
    import paper_1710_03940_amd as L
    P = config_oseen(N=10, pieces=(2, 1, 1))
    S = L.Solver(P.A, P.part, P.nsub, P.Z, solver="bicgstab", block_size=4, spmv_format="bsr4")
    v = np.random.default_rng(3).uniform(-1, 1, P.n)
    out = _t(np.zeros(P.n))
    S.apply(L._lib.OP_SPMV, _t(v), out)
    S.close()
    want = P.A @ v
    assert np.allclose(out.cpu().numpy(), want, rtol=0, atol=1e-13 * np.abs(want).max())


def test_bsr4_among_tuner_candidates():
    # the tuner times BSR4 beside SELL and CSR for every operator of a
    # point-block hierarchy; whichever it keeps, the solve matches the oracle
    import paper_1710_03940_amd as L
    P = config_oseen(N=12, pieces=(2, 2, 1))
    ref = OracleSolver(P.A, P.part, P.nsub, P.Z, OracleParams(solver="bicgstab", block_size=4,
                                                              coarse_enough=100)).solve(P.b)
    S = L.Solver(P.A, P.part, P.nsub, P.Z, solver="bicgstab", block_size=4, coarse_enough=100, verbose=2)
    x = _t(np.zeros(P.n))
    out = S.solve(_t(P.b), x)
    print(S.stats()["layouts"], flush=True)
    S.close()
    assert out["status"] == 0 and abs(out["iters"] - ref["iters"]) <= 2
