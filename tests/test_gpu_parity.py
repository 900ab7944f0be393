"""GPU parity: the HIP path (through the C ABI) against the CPU FP64 oracle on
the same seeded inputs."""
import numpy as np
import pytest

from workloads import (tiny_problem, config_small_poisson, make_problem)
from oracle import OracleSolver, OracleParams

torch = pytest.importorskip("torch")
pytestmark = [pytest.mark.gpu,
              pytest.mark.skipif(not torch.cuda.is_available(), reason="needs a GPU")]


def _dev():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch.device("cuda:0")


def _lib():
    import paper_1710_03940_amd as L
    return L


def _t(a):
    return torch.tensor(np.ascontiguousarray(a, dtype=np.float64), device=_dev())


def _solve_pair(P, oracle_kw=None, gpu_kw=None, x0=None):
    L = _lib()
    okw = dict(oracle_kw or {})
    gkw = dict(gpu_kw or {})
    ref = OracleSolver(P.A, P.part, P.nsub, P.Z, OracleParams(**okw)).solve(P.b, x0=x0)
    S = L.Solver(P.A, P.part, P.nsub, P.Z, **gkw)
    b = _t(P.b)
    x = _t(np.zeros(P.n) if x0 is None else x0)
    out = S.solve(b, x)
    out["x"] = x.cpu().numpy()
    out["stats"] = S.stats()
    S.close()
    return ref, out


def _assert_parity(ref, out, iters_tol=2, sol_tol=1e-6):
    print(f"gpu iters {out['iters']} oracle {ref['iters']} relres_true {out['relres_true']:.3e}",
          flush=True)
    assert out["status"] == 0, out
    assert abs(out["iters"] - ref["iters"]) <= iters_tol
    assert out["relres_true"] <= 1e-8
    rel = np.linalg.norm(out["x"] - ref["x"]) / np.linalg.norm(ref["x"])
    assert rel <= sol_tol, rel


def test_small_poisson_fp64_parity():
    P = config_small_poisson()
    ref, out = _solve_pair(P)
    _assert_parity(ref, out)
    # the residual history follows the oracle's iterate by iterate
    h = out["history"]
    k = min(len(h), len(ref["history"]))
    assert np.allclose(h[:k], ref["history"][:k], rtol=1e-6, atol=0)


@pytest.mark.parametrize("fmt,tune", [("auto", 1), ("sell", 1), ("csr", 1), ("sell", 0), ("csr", 0),
                                      ("csr_gather", 1), ("csr_gather", 0)])
def test_layouts_fp64_parity(fmt, tune):
    P = tiny_problem(N=20, pieces=(2, 2, 2), deflation="linear", sigma=2.0, seed=20)
    ref, out = _solve_pair(P, dict(coarse_enough=40),
                           dict(coarse_enough=40, spmv_format=fmt, autotune=tune))
    _assert_parity(ref, out)
    lay = out["stats"]["layouts"]
    print(lay, flush=True)
    if fmt == "csr_gather":
        # every multigrid operator is CSR staged from a gather list (or
        # unstaged CSR), the outer operator CSR
        outer, levels = lay.split(";", 1)
        assert "csr" in outer and "/glist" not in outer, lay
        assert "/glist" in levels and "/stage" not in levels and "sell" not in levels, lay


def test_autotuned_batched_matches_standalone_closely():
    # independent autotuning may regroup partial sums: results agree to
    # rounding, iteration counts exactly or within one
    L = _lib()
    from workloads import concat_problems
    probs = [tiny_problem(N=n, pieces=pc, deflation="linear", sigma=1.0, seed=n)
             for n, pc in [(16, (2, 2, 1)), (20, (2, 1, 2))]]
    A, part, nsub, Z, b, x0, off = concat_problems(probs)
    SB = L.BatchedSolver(A, part, nsub, Z, off, coarse_enough=30)
    xb = _t(np.zeros(A.shape[0]))
    outb = SB.solve(_t(b), xb)
    xb = xb.cpu().numpy()
    SB.close()
    for i, p in enumerate(probs):
        S = L.Solver(p.A, p.part, p.nsub, p.Z, coarse_enough=30)
        x = _t(np.zeros(p.n))
        o = S.solve(_t(p.b), x)
        S.close()
        assert abs(o["iters"] - outb["iters"][i]) <= 1
        xs = x.cpu().numpy()
        assert np.linalg.norm(xs - xb[off[i]:off[i + 1]]) <= 1e-9 * np.linalg.norm(xs)


@pytest.mark.parametrize("case", [
    dict(N=10, pieces=(2, 1, 1), deflation="constant", sigma=1.0, ce=20),
    dict(N=13, pieces=(2, 2, 2), deflation="linear", sigma=2.0, ce=30),
    dict(N=17, pieces=(3, 1, 2), deflation="linear", sigma=1.0, ce=60),
    dict(N=9, pieces=(1, 1, 3), deflation="constant", sigma=0.0, ce=500),   # level-0 direct solves
])
def test_tiny_problems_fp64_parity(case):
    P = tiny_problem(N=case["N"], pieces=case["pieces"], deflation=case["deflation"],
                     sigma=case["sigma"], seed=case["N"])
    ref, out = _solve_pair(P, dict(coarse_enough=case["ce"]), dict(coarse_enough=case["ce"]))
    _assert_parity(ref, out)


def test_operators_match_oracle():
    L = _lib()
    P = tiny_problem(N=14, pieces=(2, 2, 1), deflation="linear", sigma=2.0, seed=21)
    ora = OracleSolver(P.A, P.part, P.nsub, P.Z, OracleParams(coarse_enough=40))
    S = L.Solver(P.A, P.part, P.nsub, P.Z, coarse_enough=40)
    v = np.random.default_rng(0).standard_normal(P.n)
    vin, out = _t(v), _t(np.zeros(P.n))
    S.apply(L._lib.OP_SPMV, vin, out)
    ref = P.A @ v
    assert np.abs(out.cpu().numpy() - ref).max() <= 1e-13 * np.abs(ref).max()
    S.apply(L._lib.OP_PROJECT, vin, out)
    ref = ora.project(v)
    assert np.linalg.norm(out.cpu().numpy() - ref) <= 1e-11 * np.linalg.norm(ref)
    S.apply(L._lib.OP_PRECOND, vin, out)
    ref = ora.apply_precond(v)
    assert np.linalg.norm(out.cpu().numpy() - ref) <= 1e-10 * np.linalg.norm(ref)
    S.close()


def test_zero_rhs_and_maxiter():
    L = _lib()
    P = tiny_problem(N=8, pieces=(2, 1, 1))
    S = L.Solver(P.A, P.part, P.nsub, P.Z, coarse_enough=20)
    x = _t(np.ones(P.n))
    out = S.solve(_t(np.zeros(P.n)), x)
    assert out["status"] == 0 and out["iters"] == 0
    assert np.all(x.cpu().numpy() == 0.0)
    S.close()
    S = L.Solver(P.A, P.part, P.nsub, P.Z, coarse_enough=20, maxiter=2)
    out = S.solve(_t(P.b), _t(np.zeros(P.n)))
    assert out["status"] == L._lib.ENOCONV and out["iters"] == 2
    S.close()


def _mixed_bound(ref_iters):
    # mixed precision must reach the same FP64 residual within +15 % iterations
    return int(np.floor(ref_iters * 1.15)) + 1


@pytest.mark.parametrize("fmt,tune", [("auto", 1), ("csr_gather", 0)])
def test_small_poisson_mixed_reaches_fp64_residual(fmt, tune):
    P = config_small_poisson()
    ref, out = _solve_pair(P, gpu_kw=dict(precision="mixed", spmv_format=fmt, autotune=tune))
    print(f"mixed iters {out['iters']} oracle fp64 {ref['iters']} {out['stats']['layouts']}", flush=True)
    if fmt == "csr_gather":
        assert "/glist" in out["stats"]["layouts"].split(";", 1)[1]
    assert out["status"] == 0
    assert out["relres_true"] <= 1e-8
    assert out["iters"] <= _mixed_bound(ref["iters"])
    rel = np.linalg.norm(out["x"] - ref["x"]) / np.linalg.norm(ref["x"])
    assert rel <= 1e-6


@pytest.mark.parametrize("precision,fmt", [("fp64", "auto"), ("mixed", "auto"), ("mixed", "csr_gather")])
def test_batched_equals_standalone(precision, fmt):
    L = _lib()
    from workloads import concat_problems
    probs = [tiny_problem(N=n, pieces=pc, deflation="linear", sigma=1.0, seed=n)
             for n, pc in [(9, (2, 1, 1)), (12, (2, 2, 1)), (7, (1, 1, 2)), (15, (3, 1, 1))]]
    A, part, nsub, Z, b, x0, off = concat_problems(probs)
    # one layout family so that both handles sum every row in the same order
    kw = dict(precision=precision, coarse_enough=30, autotune=0, spmv_format=fmt)
    SB = L.BatchedSolver(A, part, nsub, Z, off, **kw)
    xb = _t(np.zeros(A.shape[0]))
    outb = SB.solve(_t(b), xb)
    xb = xb.cpu().numpy()
    SB.close()
    assert outb["status"] == 0
    for i, p in enumerate(probs):
        S = L.Solver(p.A, p.part, p.nsub, p.Z, **kw)
        x = _t(np.zeros(p.n))
        o = S.solve(_t(p.b), x)
        S.close()
        assert o["iters"] == outb["iters"][i]
        assert np.array_equal(x.cpu().numpy(), xb[off[i]:off[i + 1]])
        assert outb["relres_true"][i] <= 1e-8


def test_no_preconditioner_and_no_deflation():
    # M = I with deflation: deflated CG; ndv = 0: plain AMG-PCG
    P = tiny_problem(N=12, pieces=(2, 2, 1), deflation="linear", sigma=1.0, seed=4)
    ref, out = _solve_pair(P, dict(precond="identity"), dict(precond="none"))
    _assert_parity(ref, out)
    Z0 = np.zeros((P.n, 0))
    P0 = P.__class__(P.name, P.A, P.part, P.nsub, Z0, P.b, P.x0)
    ref, out = _solve_pair(P0, dict(coarse_enough=30), dict(coarse_enough=30))
    _assert_parity(ref, out)


def test_jacobi_smoother_parity():
    P = tiny_problem(N=13, pieces=(1, 2, 2), deflation="constant", sigma=1.0, seed=13)
    ref, out = _solve_pair(P, dict(smoother="jacobi", coarse_enough=40),
                           dict(smoother="jacobi", coarse_enough=40))
    _assert_parity(ref, out)


def test_nonzero_initial_guess():
    P = tiny_problem(N=11, pieces=(2, 1, 1), deflation="linear", sigma=1.0, seed=2)
    x0 = np.random.default_rng(3).standard_normal(P.n)
    ref, out = _solve_pair(P, dict(coarse_enough=30), dict(coarse_enough=30), x0=x0)
    _assert_parity(ref, out)


def test_graph_and_direct_launch_agree():
    L = _lib()
    P = tiny_problem(N=12, pieces=(2, 2, 1), deflation="linear", sigma=1.0, seed=8)
    res = []
    for g in (0, 1, 16):
        S = L.Solver(P.A, P.part, P.nsub, P.Z, coarse_enough=30, graph_iters=g, autotune=0)
        x = _t(np.zeros(P.n))
        for _ in range(3):             # repeated replays give identical results
            x.zero_()
            o = S.solve(_t(P.b), x)
            res.append((o["iters"], x.cpu().numpy().copy()))
        S.close()
    for it, xv in res[1:]:
        assert it == res[0][0]
        assert np.array_equal(xv, res[0][1])


@pytest.mark.parametrize("ndv", [2, 6, 8])
def test_other_deflation_counts(ndv):
    # Z with ndv columns per subdomain: linear vectors plus bilinear and
    # trilinear ones (8, the most the library takes)
    P = tiny_problem(N=12, pieces=(2, 2, 1), deflation="linear", sigma=1.0, seed=ndv)
    Zx = np.column_stack([P.Z, P.Z[:, 1] * P.Z[:, 2], P.Z[:, 2] * P.Z[:, 3], P.Z[:, 1] * P.Z[:, 3],
                          P.Z[:, 1] * P.Z[:, 2] * P.Z[:, 3]])[:, :ndv]
    P2 = P.__class__(P.name, P.A, P.part, P.nsub, np.ascontiguousarray(Zx), P.b, P.x0)
    ref, out = _solve_pair(P2, dict(coarse_enough=30), dict(coarse_enough=30))
    _assert_parity(ref, out)


def test_general_deflation_vectors():
    # deflation columns with more than 256 distinct values per subdomain
    # (the operator epilogue then reads Z as plain FP64 rather than as
    # per-subdomain value tables)
    P = tiny_problem(N=12, pieces=(2, 2, 1), deflation="constant", sigma=1.0, seed=31)
    g = np.random.default_rng(5).standard_normal((P.n, 2))
    Zx = np.column_stack([P.Z[:, 0], g[:, 0], g[:, 1]])
    P2 = P.__class__(P.name, P.A, P.part, P.nsub, np.ascontiguousarray(Zx), P.b, P.x0)
    assert min(len(np.unique(Zx[P.part == s, 1])) for s in range(P.nsub)) > 256
    ref, out = _solve_pair(P2, dict(coarse_enough=30), dict(coarse_enough=30))
    _assert_parity(ref, out)


@pytest.mark.parametrize("solver", ["cg", "bicgstab", "bicgstab2"])
def test_one_and_two_row_subdomains(solver):
    """Subdomains of one and two rows (solved directly on level 0) beside a
    large one with a hierarchy; constant deflation."""
    P = tiny_problem(N=6, pieces=(1, 1, 1), deflation="constant", sigma=1.0, seed=8)
    part = np.full(P.n, 2, dtype=np.int32)
    part[0] = 0
    part[1:3] = 1
    Z = np.ones((P.n, 1))
    P2 = P.__class__("ragged", P.A, part, 3, Z, P.b, P.x0)
    okw = dict(coarse_enough=10, solver="bicgstabl" if solver == "bicgstab2" else solver)
    if solver == "bicgstab2":
        okw["ell"] = 2
    L = _lib()
    ref = OracleSolver(P2.A, P2.part, P2.nsub, P2.Z, OracleParams(**okw)).solve(P2.b)
    S = L.Solver(P2.A, P2.part, P2.nsub, P2.Z, coarse_enough=10, solver=solver)
    x = _t(np.zeros(P2.n))
    out = S.solve(_t(P2.b), x)
    out["x"] = x.cpu().numpy()
    S.close()
    _assert_parity(ref, out)


def test_bicgstab2_zero_rhs_and_maxiter():
    L = _lib()
    P = tiny_problem(N=8, pieces=(2, 1, 1))
    S = L.Solver(P.A, P.part, P.nsub, P.Z, coarse_enough=20, solver="bicgstab2")
    x = _t(np.ones(P.n))
    out = S.solve(_t(np.zeros(P.n)), x)
    assert out["status"] == 0 and out["iters"] == 0
    assert np.all(x.cpu().numpy() == 0.0)
    S.close()
    S = L.Solver(P.A, P.part, P.nsub, P.Z, coarse_enough=20, solver="bicgstab2", maxiter=1, rtol=1e-14)
    out = S.solve(_t(P.b), _t(np.zeros(P.n)))
    S.close()
    assert out["status"] == L._lib.ENOCONV and out["iters"] == 1
