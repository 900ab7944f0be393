"""GPU parity of the solver options of the nested parameter listing: the
flexible (Polak-Ribiere) CG and the V(npre, npost) cycle, through the C ABI
against the CPU FP64 oracle with the same options."""
import numpy as np
import pytest

from workloads import tiny_problem, make_problem
from oracle import OracleSolver, OracleParams

torch = pytest.importorskip("torch")
pytestmark = [pytest.mark.gpu,
              pytest.mark.skipif(not torch.cuda.is_available(), reason="needs a GPU")]


def _t(a):
    return torch.tensor(np.ascontiguousarray(a, dtype=np.float64), device=torch.device("cuda:0"))


def _pair(P, okw, gkw):
    import paper_1710_03940_amd as L
    ref = OracleSolver(P.A, P.part, P.nsub, P.Z, OracleParams(**okw)).solve(P.b)
    S = L.Solver(P.A, P.part, P.nsub, P.Z, **gkw)
    x = _t(np.zeros(P.n))
    out = S.solve(_t(P.b), x)
    out["x"] = x.cpu().numpy()
    S.close()
    rel = np.linalg.norm(out["x"] - ref["x"]) / np.linalg.norm(ref["x"])
    print(f"{gkw}: gpu iters {out['iters']} oracle {ref['iters']} relres_true {out['relres_true']:.2e} "
          f"|x - x_oracle|/|x| {rel:.2e}", flush=True)
    return ref, out, rel


def _problem():
    # two levels of tiles in every subdomain plus ragged tails
    return tiny_problem(N=22, pieces=(2, 2, 2), deflation="linear", sigma=2.0, seed=31)


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_flexible_cg_parity(precision):
    P = _problem()
    ref, out, rel = _pair(P, dict(coarse_enough=40, flexible=True),
                          dict(coarse_enough=40, flexible_cg=1, precision=precision))
    assert out["status"] == 0
    assert out["relres_true"] <= 1e-8
    if precision == "fp64":
        assert abs(out["iters"] - ref["iters"]) <= 2
        assert rel <= 1e-6
        # the residual history follows the oracle's iterate by iterate
        k = min(len(out["history"]), len(ref["history"])) - 3
        assert np.allclose(out["history"][:k], ref["history"][:k], rtol=1e-6, atol=0)
    else:
        assert out["iters"] <= 1.15 * ref["iters"] + 1
        assert rel <= 1e-6


@pytest.mark.parametrize("npre,npost", [(2, 2), (0, 1), (3, 1), (1, 2)])
@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_vcycle_sweeps_parity(npre, npost, precision):
    P = _problem()
    solver = "cg" if npre == npost else "bicgstab"   # CG needs the symmetric V(nu, nu)
    ref, out, rel = _pair(P, dict(coarse_enough=40, npre=npre, npost=npost, solver=solver),
                          dict(coarse_enough=40, npre=npre, npost=npost, precision=precision, solver=solver))
    assert out["status"] == 0
    assert out["relres_true"] <= 1e-8
    if precision == "fp64":
        assert abs(out["iters"] - ref["iters"]) <= 2
    else:
        assert out["iters"] <= 1.15 * ref["iters"] + 1
    assert rel <= 1e-6


def test_vcycle_sweeps_operator_matches_oracle():
    # M^{-1} applied once (DFAMG_OP_PRECOND) with V(2, 2): element by element
    import paper_1710_03940_amd as L
    P = _problem()
    o = OracleSolver(P.A, P.part, P.nsub, P.Z, OracleParams(coarse_enough=40, npre=2, npost=2))
    v = np.random.default_rng(5).uniform(-1, 1, P.n)
    want = o.precond(v)
    S = L.Solver(P.A, P.part, P.nsub, P.Z, coarse_enough=40, npre=2, npost=2)
    out = _t(np.zeros(P.n))
    S.apply(L._lib.OP_PRECOND, _t(v), out)
    got = out.cpu().numpy()
    S.close()
    assert np.allclose(got, want, rtol=0, atol=1e-11 * np.abs(want).max())


def test_two_sweeps_reduce_iterations():
    P = make_problem("p", (24, 24, 24), (2, 2, 2), deflation="linear", sigma=1.0, coef_seed=3,
                     rhs="uniform", rhs_seed=4)
    import paper_1710_03940_amd as L
    its = []
    for nu in (1, 2):
        S = L.Solver(P.A, P.part, P.nsub, P.Z, npre=nu, npost=nu)
        x = _t(np.zeros(P.n))
        its.append(S.solve(_t(P.b), x)["iters"])
        S.close()
    print("iterations V(1,1), V(2,2):", its, flush=True)
    assert its[1] < its[0]


@pytest.mark.parametrize("graph_iters", [16, 0])
def test_cg_profile_events_first_graph_only(graph_iters):
    # profile = 1 records its events in the first captured graph of every
    # solve (later chunks replay a graph without event nodes), every
    # iteration with direct launches; profile = 2 every span of every
    # iteration.  The iterate is bitwise that of the unprofiled solve.
    import paper_1710_03940_amd as L
    P = make_problem("p20", (20, 20, 20), (2, 2, 1), deflation="linear", sigma=2.0, coef_seed=11,
                     rhs="uniform", rhs_seed=12)
    kw = dict(coarse_enough=40, autotune=0, graph_iters=graph_iters)
    xs, its, calls = [], [], {}
    for prof in (0, 1, 2):
        S = L.Solver(P.A, P.part, P.nsub, P.Z, profile=prof, **kw)
        for _ in range(2):
            x = _t(np.zeros(P.n))
            out = S.solve(_t(P.b), x)
        st = S.stats()
        S.close()
        assert out["status"] == 0
        xs.append(x.cpu().numpy())
        its.append(out["iters"])
        calls[prof] = st["kernels"]["spmv"]["calls"]
        if prof:
            assert st["kernels"]["presmooth0"]["calls"] == calls[prof] and st["kernels"]["spmv"]["ms"] > 0
    assert its[0] == its[1] == its[2] and its[0] > 16
    assert np.array_equal(xs[0], xs[1]) and np.array_equal(xs[0], xs[2])
    print("iterations", its[0], "spmv spans", calls, flush=True)
    # the iteration that meets the tolerance may go uncounted once per solve
    every = range(2 * (its[0] - 1), 2 * its[0] + 1)
    assert calls[1] == 2 * 16 if graph_iters else calls[1] in every
    assert calls[2] in every
