"""GPU parity of restarted flexible GMRES on A x = b preconditioned by the
deflation combined multiplicatively with the block AMG, with the exact FP64
coarse solve and the inexact single-precision one, against the oracle."""
import numpy as np
import pytest

from workloads import tiny_problem, config_oseen, convection_diffusion7, config_small_poisson
from oracle import OracleSolver, OracleParams

torch = pytest.importorskip("torch")
pytestmark = [pytest.mark.gpu,
              pytest.mark.skipif(not torch.cuda.is_available(), reason="needs a GPU")]


def _t(a):
    return torch.tensor(np.ascontiguousarray(a, dtype=np.float64), device="cuda:0")


def _convdiff(N, pieces, deflation, peclet, seed):
    base = tiny_problem(N=N, pieces=pieces, deflation=deflation, seed=seed)
    A = convection_diffusion7(N, peclet=peclet)
    return base.__class__(f"cd{N}", A, base.part, base.nsub, base.Z, base.b, base.x0)


def _pair(P, kw, gpu_extra=None, x0=None, oracle_extra=None):
    import paper_1710_03940_amd as L
    print(f"case {P.name} n={P.n} nsub={P.nsub} ndv={P.ndv} {kw} {gpu_extra}", flush=True)
    ref = OracleSolver(P.A, P.part, P.nsub, P.Z,
                       OracleParams(**{**kw, **(oracle_extra or {})})).solve(P.b, x0=x0)
    S = L.Solver(P.A, P.part, P.nsub, P.Z, **{**kw, **(gpu_extra or {})})
    x = _t(np.zeros(P.n) if x0 is None else x0)
    out = S.solve(_t(P.b), x)
    out["x"] = x.cpu().numpy()
    S.close()
    print(f"  gpu iters {out['iters']} status {out['status']} relres_true {out['relres_true']:.3e}"
          f" | oracle iters {ref['iters']} {ref['status']}", flush=True)
    return ref, out


def _check(ref, out, iters_tol=2, sol_tol=1e-6, rtol=1e-8):
    assert ref["status"] == "ok"
    assert out["status"] == 0, out
    assert abs(out["iters"] - ref["iters"]) <= iters_tol
    assert out["relres_true"] <= rtol * (1 + 1e-6)
    rel = np.linalg.norm(out["x"] - ref["x"]) / np.linalg.norm(ref["x"])
    assert rel <= sol_tol, rel


@pytest.mark.parametrize("coarse", ["exact", "fp32"])
@pytest.mark.parametrize("restart", [30, 4])
@pytest.mark.parametrize("N,pieces,deflation,peclet,ce", [
    (12, (2, 2, 1), "linear", 2.0, 40),
    (10, (2, 1, 1), "constant", 5.0, 20),
])
def test_fgmres_convdiff_parity(N, pieces, deflation, peclet, ce, restart, coarse):
    P = _convdiff(N, pieces, deflation, peclet, seed=N)
    ref, out = _pair(P, dict(solver="fgmres", restart=restart, coarse_solve=coarse, coarse_enough=ce))
    _check(ref, out)
    # the least-squares residual follows the oracle's step by step
    h, g = out["history"], ref["history"]
    k = min(len(h), len(g), 8)
    assert np.allclose(h[:k], g[:k], rtol=1e-7 if coarse == "exact" else 1e-5)


def test_fgmres_largest_restart():
    # restart 64, the largest the device state holds: one full cycle of 64
    # steps, then a second one (the oracle takes 111 steps)
    P = _convdiff(20, (1, 1, 2), "constant", 1.0, seed=20)
    ref, out = _pair(P, dict(solver="fgmres", restart=64, precond="none", coarse_enough=40))
    assert ref["iters"] > 64
    _check(ref, out)


@pytest.mark.parametrize("coarse", ["exact", "fp32"])
def test_fgmres_poisson_slabs_parity(coarse):
    P = config_small_poisson()
    ref, out = _pair(P, dict(solver="fgmres", coarse_solve=coarse))
    _check(ref, out)


def test_fgmres_oseen_fp64_and_mixed():
    P = config_oseen(N=16, pieces=(2, 2, 1))
    kw = dict(solver="fgmres", block_size=4, coarse_solve="fp32")
    ref, out = _pair(P, kw)
    _check(ref, out)
    ref, out = _pair(P, kw, dict(precision="mixed"))
    assert out["status"] == 0
    assert out["relres_true"] <= 1e-8 * (1 + 1e-6)
    assert out["iters"] <= int(np.floor(ref["iters"] * 1.15)) + 1
    assert np.linalg.norm(out["x"] - ref["x"]) <= 1e-6 * np.linalg.norm(ref["x"])


@pytest.mark.parametrize("rtol", [1e-2, 1e-3, 1e-4, 1e-5, 1e-6, 1e-7])
def test_fgmres_stops_like_oracle_at_any_tolerance(rtol):
    """Stops inside a cycle and at its last step (restart 5) like the oracle."""
    P = _convdiff(9, (3, 1, 1), "constant", 3.0, seed=4)
    ref, out = _pair(P, dict(solver="fgmres", restart=5, coarse_enough=30, rtol=rtol))
    _check(ref, out, iters_tol=0, sol_tol=1e-9, rtol=rtol)


def test_fgmres_initial_guess_no_preconditioner_no_deflation():
    P = _convdiff(11, (1, 2, 2), "linear", 2.0, seed=6)
    x0 = np.random.default_rng(8).standard_normal(P.n)
    ref, out = _pair(P, dict(solver="fgmres", restart=10, coarse_enough=30), x0=x0)
    _check(ref, out)
    ref, out = _pair(P, dict(solver="fgmres", restart=20), dict(precond="none"),
                     oracle_extra=dict(precond="identity"))
    _check(ref, out)
    Q = P.__class__(P.name, P.A, P.part, P.nsub, np.zeros((P.n, 0)), P.b, P.x0)
    ref, out = _pair(Q, dict(solver="fgmres", restart=8, coarse_enough=30))
    _check(ref, out)


def test_fgmres_zero_rhs_and_maxiter():
    import paper_1710_03940_amd as L
    P = _convdiff(9, (2, 1, 1), "linear", 2.0, seed=3)
    S = L.Solver(P.A, P.part, P.nsub, P.Z, solver="fgmres", restart=4, coarse_enough=20, maxiter=6)
    x = _t(np.ones(P.n))
    out = S.solve(_t(np.zeros(P.n)), x)
    assert out["iters"] == 0 and out["status"] == 0
    assert not x.cpu().numpy().any()
    # maxiter in the second cycle: the iterate formed from the steps taken
    x = _t(np.zeros(P.n))
    out = S.solve(_t(P.b), x)
    S.close()
    ref = OracleSolver(P.A, P.part, P.nsub, P.Z,
                       OracleParams(solver="fgmres", restart=4, coarse_enough=20)).solve(P.b, maxiter=6)
    assert out["iters"] == 6 and ref["iters"] == 6 and ref["status"] == "noconv"
    assert out["status"] == 4                      # DFAMG_ENOCONV
    assert np.linalg.norm(x.cpu().numpy() - ref["x"]) <= 1e-9 * np.linalg.norm(ref["x"])


def test_fgmres_batched_equals_standalone_and_graph_equals_direct():
    import paper_1710_03940_amd as L
    from workloads import concat_problems
    probs = [_convdiff(n, pc, "linear", 2.0, seed=n) for n, pc in [(9, (2, 1, 1)), (12, (2, 2, 1))]]
    A, part, nsub, Z, b, x0, off = concat_problems(probs)
    kw = dict(solver="fgmres", restart=6, coarse_solve="fp32", coarse_enough=30, autotune=0)
    S = L.BatchedSolver(A, part, nsub, Z, off, **kw)
    xb = _t(np.zeros(A.shape[0]))
    outb = S.solve(_t(b), xb)
    S.close()
    xb = xb.cpu().numpy()
    for s, p in enumerate(probs):
        xs = []
        for gi in (16, 0):
            S1 = L.Solver(p.A, p.part, p.nsub, p.Z, graph_iters=gi, **kw)
            x1 = _t(np.zeros(p.n))
            o1 = S1.solve(_t(p.b), x1)
            S1.close()
            assert int(outb["iters"][s]) == o1["iters"]
            xs.append(x1.cpu().numpy())
        assert np.array_equal(xb[off[s]:off[s + 1]], xs[0])
        assert np.array_equal(xs[0], xs[1])


@pytest.mark.parametrize("profile,graph_iters", [(2, 16), (2, 0), (1, 16)])
def test_fgmres_profiled_solve_unchanged(profile, graph_iters):
    """Event spans recorded inside the cycle graph (or around direct launches)
    leave the iterate bitwise unchanged and report the outer operator."""
    import paper_1710_03940_amd as L
    P = _convdiff(10, (2, 1, 1), "linear", 2.0, seed=5)
    kw = dict(solver="fgmres", restart=7, coarse_enough=30, autotune=0, graph_iters=graph_iters)
    xs = []
    for prof in (0, profile):
        S = L.Solver(P.A, P.part, P.nsub, P.Z, profile=prof, **kw)
        x = _t(np.zeros(P.n))
        out = S.solve(_t(P.b), x)
        st = S.stats()
        S.close()
        assert out["status"] == 0
        xs.append(x.cpu().numpy())
        if prof:
            assert st["kernels"]["spmv"]["calls"] > 0 and st["kernels"]["spmv"]["ms"] > 0
    assert np.array_equal(xs[0], xs[1])


@pytest.mark.parametrize("crtol", [1e-1, 1e-2, 1e-4])
def test_fgmres_iterative_coarse_solve_parity(crtol):
    """The CG coarse solve to a relaxed tolerance (a preconditioner that
    changes from call to call) against the oracle's."""
    from workloads import make_problem
    P = make_problem("p16", (16, 16, 16), (2, 2, 2), deflation="linear", sigma=1.0, coef_seed=3,
                     rhs="uniform", rhs_seed=4)
    kw = dict(solver="fgmres", restart=12, coarse_solve="cg", coarse_rtol=crtol, coarse_enough=60)
    ref, out = _pair(P, kw)
    _check(ref, out)
    h, g = out["history"], ref["history"]
    k = min(len(h), len(g), 6)
    assert np.allclose(h[:k], g[:k], rtol=1e-6)


def test_fgmres_iterative_coarse_solve_reports_steps_and_rejects_nonsymmetric_E():
    import paper_1710_03940_amd as L
    from workloads import make_problem
    P = make_problem("p12", (12, 12, 12), (2, 2, 1), deflation="linear", sigma=1.0, coef_seed=5)
    S = L.Solver(P.A, P.part, P.nsub, P.Z, solver="fgmres", coarse_solve="cg", coarse_enough=60)
    x = _t(np.zeros(P.n))
    out = S.solve(_t(P.b), x)
    st = S.stats()
    S.close()
    assert out["status"] == 0
    assert st["coarse_iters"] >= out["iters"]          # at least one CG step per application
    Q = _convdiff(9, (2, 1, 1), "linear", 4.0, seed=2)
    with pytest.raises(L.DfamgError) as ei:
        L.Solver(Q.A, Q.part, Q.nsub, Q.Z, solver="fgmres", coarse_solve="cg", coarse_enough=20)
    assert ei.value.status == 1                          # DFAMG_EINVAL


def test_fgmres_restart_one():
    """FGMRES(1): a preconditioned minimal-residual iteration, one step per
    cycle (every kernel of the cycle runs with a single basis vector)."""
    P = _convdiff(9, (2, 1, 1), "linear", 2.0, seed=11)
    ref, out = _pair(P, dict(solver="fgmres", restart=1, coarse_enough=30, maxiter=400))
    _check(ref, out, iters_tol=0)
