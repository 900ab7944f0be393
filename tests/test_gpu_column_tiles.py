"""The column-tiled restriction (spmv_format = COLUMN_TILED: every
restriction operator B = R (I - A diag(m)) split by column tiles of 512
unknowns of the finer vector, each tile staged once in LDS, one partial sum
per row segment, the partials added per row in tile order) against the CPU
FP64 oracle, on ragged cases where subdomains span several column tiles and
the last tile of each is short: one preconditioner application element by
element, whole CG and BiCGStab solves in FP64 and mixed precision, and
batched systems against their standalone solves."""
import numpy as np
import pytest

from workloads import tiny_problem, make_problem, concat_problems
from oracle import OracleSolver, OracleParams

torch = pytest.importorskip("torch")
pytestmark = [pytest.mark.gpu,
              pytest.mark.skipif(not torch.cuda.is_available(), reason="needs a GPU")]


def _t(a):
    return torch.tensor(np.ascontiguousarray(a, dtype=np.float64), device=torch.device("cuda:0"))


def _problem():
    # 8 subdomains of 1,400-1,900 unknowns: three or four column tiles each
    return make_problem("p25", (25, 23, 26), (2, 2, 2), deflation="linear", sigma=2.0, coef_seed=21,
                        rhs="uniform", rhs_seed=22)


def _layouts(S):
    return S.stats()["layouts"]


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_column_tiled_operator_matches_oracle(precision):
    import paper_1710_03940_amd as L
    P = _problem()
    o = OracleSolver(P.A, P.part, P.nsub, P.Z, OracleParams(coarse_enough=30))
    v = np.random.default_rng(7).uniform(-1, 1, P.n)
    want = o.precond(v)
    S = L.Solver(P.A, P.part, P.nsub, P.Z, coarse_enough=30, spmv_format="column_tiled", precision=precision)
    lay = _layouts(S)
    out = _t(np.zeros(P.n))
    S.apply(L._lib.OP_PRECOND, _t(v), out)
    got = out.cpu().numpy()
    S.close()
    print(precision, lay, flush=True)
    assert "B seg512" in lay and "L1{" in lay, lay
    tol = 1e-11 if precision == "fp64" else 2e-5
    assert np.allclose(got, want, rtol=0, atol=tol * np.abs(want).max())


@pytest.mark.parametrize("solver,precision", [("cg", "fp64"), ("cg", "mixed"), ("bicgstab", "fp64")])
def test_column_tiled_solve_matches_oracle(solver, precision):
    import paper_1710_03940_amd as L
    P = _problem()
    ref = OracleSolver(P.A, P.part, P.nsub, P.Z, OracleParams(coarse_enough=30, solver=solver)).solve(P.b)
    S = L.Solver(P.A, P.part, P.nsub, P.Z, coarse_enough=30, solver=solver, spmv_format="column_tiled",
                 precision=precision)
    x = _t(np.zeros(P.n))
    out = S.solve(_t(P.b), x)
    S.close()
    print(solver, precision, "iterations", out["iters"], "oracle", ref["iters"], flush=True)
    assert out["status"] == 0 and out["relres_true"] <= 1e-8 * 1.01
    if precision == "fp64":
        assert abs(out["iters"] - ref["iters"]) <= 2
    else:
        assert out["iters"] <= 1.15 * ref["iters"] + 1
    assert np.linalg.norm(x.cpu().numpy() - ref["x"]) <= 1e-6 * np.linalg.norm(ref["x"])


def test_column_tiled_batched_equals_standalone():
    # systems of different sizes in one handle: the column tiles never
    # straddle subdomains, so each system's iterate is its standalone one
    import paper_1710_03940_amd as L
    probs = [tiny_problem(N=n, pieces=pc, deflation="linear", sigma=1.5, seed=s)
             for n, pc, s in ((17, (2, 1, 1), 1), (23, (2, 2, 1), 2), (11, (1, 1, 1), 3))]
    A, part, nsub, Z, b, x0, off = concat_problems(probs)
    kw = dict(coarse_enough=25, spmv_format="column_tiled")
    S = L.BatchedSolver(A, part, nsub, Z, off, **kw)
    x = _t(np.zeros(A.shape[0]))
    out = S.solve(_t(b), x)
    S.close()
    xs = x.cpu().numpy()
    for s_, P in enumerate(probs):
        T = L.Solver(P.A, P.part, P.nsub, P.Z, **kw)
        y = _t(np.zeros(P.n))
        o1 = T.solve(_t(P.b), y)
        T.close()
        assert int(out["iters"][s_]) == o1["iters"]
        assert np.array_equal(xs[off[s_]:off[s_ + 1]], y.cpu().numpy())
        ref = OracleSolver(P.A, P.part, P.nsub, P.Z, OracleParams(coarse_enough=25)).solve(P.b)
        assert np.linalg.norm(y.cpu().numpy() - ref["x"]) <= 1e-6 * np.linalg.norm(ref["x"])
