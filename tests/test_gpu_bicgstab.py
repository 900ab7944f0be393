"""GPU parity of the deflated BiCGStab path on nonsymmetric operators: upwind
convection-diffusion (scalar SA) and the stabilised Q1 Oseen operator (4x4
point-block SA, per-field deflation, nonsymmetric E)."""
import numpy as np
import pytest

from workloads import tiny_problem, config_oseen, convection_diffusion7
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


def _pair(P, kw, gpu_extra=None, x0=None):
    import paper_1710_03940_amd as L
    print(f"case {P.name} n={P.n} nsub={P.nsub} ndv={P.ndv} {kw} {gpu_extra}", flush=True)
    ref = OracleSolver(P.A, P.part, P.nsub, P.Z, OracleParams(**kw)).solve(P.b, x0=x0)
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


@pytest.mark.parametrize("N,pieces,deflation,peclet,ce", [
    (12, (2, 2, 1), "linear", 2.0, 40),
    (10, (2, 1, 1), "constant", 5.0, 20),
    (15, (1, 3, 1), "linear", 1.0, 500),
])
def test_bicgstab_convdiff_fp64_parity(N, pieces, deflation, peclet, ce):
    P = _convdiff(N, pieces, deflation, peclet, seed=N)
    ref, out = _pair(P, dict(solver="bicgstab", coarse_enough=ce))
    _check(ref, out)
    # the residual history follows the oracle's iterate by iterate
    h, g = out["history"], ref["history"]
    k = min(len(h), len(g), 6)
    assert np.allclose(h[:k], g[:k], rtol=1e-7)


@pytest.mark.parametrize("N,pieces", [(16, (2, 2, 1)), (12, (2, 2, 2))])
def test_bicgstab_oseen_fp64_parity(N, pieces):
    P = config_oseen(N=N, pieces=pieces)
    ref, out = _pair(P, dict(solver="bicgstab", block_size=4))
    _check(ref, out)


def test_bicgstab_oseen_mixed_reaches_fp64_residual():
    P = config_oseen(N=16, pieces=(2, 2, 1))
    ref, out = _pair(P, dict(solver="bicgstab", block_size=4), dict(precision="mixed"))
    assert out["status"] == 0
    assert out["relres_true"] <= 1e-8 * (1 + 1e-6)
    assert out["iters"] <= int(np.floor(ref["iters"] * 1.15)) + 1
    rel = np.linalg.norm(out["x"] - ref["x"]) / np.linalg.norm(ref["x"])
    assert rel <= 1e-6


@pytest.mark.parametrize("rtol", [1e-2, 3e-3, 1e-3, 3e-4, 1e-4, 3e-5, 1e-5, 3e-6])
def test_bicgstab_stops_like_oracle_at_any_tolerance(rtol):
    """A sweep of tolerances hits both exits (after the half step on s and
    after the full step on r); either way the iterate must be the oracle's."""
    P = _convdiff(9, (3, 1, 1), "constant", 3.0, seed=4)
    ref, out = _pair(P, dict(solver="bicgstab", coarse_enough=30, rtol=rtol))
    _check(ref, out, iters_tol=0, sol_tol=1e-9, rtol=rtol)


def test_bicgstab_nonzero_initial_guess_and_no_preconditioner():
    P = _convdiff(11, (1, 2, 2), "linear", 2.0, seed=6)
    x0 = np.random.default_rng(8).standard_normal(P.n)
    ref, out = _pair(P, dict(solver="bicgstab", coarse_enough=30), x0=x0)
    _check(ref, out)
    ref, out = _pair(P, dict(solver="bicgstab", precond="identity"),
                     dict(precond="none"))  # oracle name / library name
    _check(ref, out)


def test_bicgstab_operators_match_oracle():
    """Projection with the nonsymmetric (LU-solved) E, and the block V-cycle."""
    import paper_1710_03940_amd as L
    P = config_oseen(N=8, pieces=(2, 2, 1))
    kw = dict(solver="bicgstab", block_size=4)
    ora = OracleSolver(P.A, P.part, P.nsub, P.Z, OracleParams(**kw))
    S = L.Solver(P.A, P.part, P.nsub, P.Z, **kw)
    v = np.random.default_rng(1).standard_normal(P.n)
    vin, out = _t(v), _t(np.zeros(P.n))
    S.apply(L._lib.OP_SPMV, vin, out)
    ref = P.A @ v
    assert np.abs(out.cpu().numpy() - ref).max() <= 1e-13 * np.abs(ref).max()
    S.apply(L._lib.OP_PROJECT, vin, out)
    ref = ora.project(v)
    assert np.linalg.norm(out.cpu().numpy() - ref) <= 1e-11 * np.linalg.norm(ref)
    # the projected vector is orthogonal to the deflation space
    got = out.cpu().numpy()
    for s in range(P.nsub):
        rows = P.part == s
        assert np.abs(P.Z[rows].T @ got[rows]).max() <= 1e-10 * np.linalg.norm(v)
    S.apply(L._lib.OP_PRECOND, vin, out)
    ref = ora.apply_precond(v)
    assert np.linalg.norm(out.cpu().numpy() - ref) <= 1e-10 * np.linalg.norm(ref)
    S.close()


def test_bicgstab_maxiter():
    import paper_1710_03940_amd as L
    P = _convdiff(8, (2, 1, 1), "constant", 2.0, seed=2)
    S = L.Solver(P.A, P.part, P.nsub, P.Z, solver="bicgstab", coarse_enough=20, maxiter=2)
    out = S.solve(_t(P.b), _t(np.zeros(P.n)))
    S.close()
    assert out["status"] == L._lib.ENOCONV and out["iters"] == 2


# --------------------------------------------------------------------------
# BiCGStab(2): the library's "bicgstab2" against the oracle's BiCGStab(ell=2)
# --------------------------------------------------------------------------

def _pair2(P, kw, gpu_extra=None, x0=None):
    return _pair_named(P, dict(kw, solver="bicgstabl", ell=2), dict(kw, solver="bicgstab2", **(gpu_extra or {})),
                       x0=x0)


def _pair_named(P, okw, gkw, x0=None):
    import paper_1710_03940_amd as L
    print(f"case {P.name} n={P.n} nsub={P.nsub} ndv={P.ndv} {gkw}", flush=True)
    ref = OracleSolver(P.A, P.part, P.nsub, P.Z, OracleParams(**okw)).solve(P.b, x0=x0)
    S = L.Solver(P.A, P.part, P.nsub, P.Z, **gkw)
    x = _t(np.zeros(P.n) if x0 is None else x0)
    out = S.solve(_t(P.b), x)
    out["x"] = x.cpu().numpy()
    S.close()
    print(f"  gpu iters {out['iters']} status {out['status']} relres_true {out['relres_true']:.3e}"
          f" | oracle iters {ref['iters']} {ref['status']}", flush=True)
    return ref, out


@pytest.mark.parametrize("N,pieces,deflation,peclet,ce", [
    (12, (2, 2, 1), "linear", 2.0, 40),
    (10, (2, 1, 1), "constant", 5.0, 20),
    (15, (1, 3, 1), "linear", 0.0, 500),      # symmetric (pure diffusion)
])
def test_bicgstab2_fp64_parity(N, pieces, deflation, peclet, ce):
    P = _convdiff(N, pieces, deflation, peclet, seed=N + 1)
    ref, out = _pair2(P, dict(coarse_enough=ce))
    _check(ref, out)
    h, g = out["history"], ref["history"]
    k = min(len(h), len(g), 5)
    assert np.allclose(h[:k], g[:k], rtol=1e-7)


def test_bicgstab2_oseen_fp64_and_mixed():
    P = config_oseen(N=16, pieces=(2, 2, 1))
    ref, out = _pair2(P, dict(block_size=4))
    _check(ref, out)
    ref, out = _pair2(P, dict(block_size=4), dict(precision="mixed"))
    assert out["status"] == 0
    assert out["relres_true"] <= 1e-8 * (1 + 1e-6)
    assert out["iters"] <= int(np.floor(ref["iters"] * 1.15)) + 1
    assert np.linalg.norm(out["x"] - ref["x"]) <= 1e-6 * np.linalg.norm(ref["x"])


@pytest.mark.parametrize("rtol", [1e-3, 1e-5, 1e-7])
def test_bicgstab2_stops_like_oracle(rtol):
    P = _convdiff(9, (3, 1, 1), "constant", 3.0, seed=4)
    ref, out = _pair2(P, dict(coarse_enough=30, rtol=rtol))
    _check(ref, out, iters_tol=0, sol_tol=1e-9, rtol=rtol)


def test_bicgstab2_initial_guess_and_no_preconditioner():
    P = _convdiff(11, (1, 2, 2), "linear", 2.0, seed=6)
    x0 = np.random.default_rng(9).standard_normal(P.n)
    ref, out = _pair2(P, dict(coarse_enough=30), x0=x0)
    _check(ref, out)
    ref, out = _pair_named(P, dict(solver="bicgstabl", ell=2, precond="identity"),
                           dict(solver="bicgstab2", precond="none"))
    _check(ref, out)


def test_bicgstab2_batched_equals_standalone():
    import paper_1710_03940_amd as L
    from workloads import concat_problems
    probs = [_convdiff(n, pc, "linear", 2.0, seed=n) for n, pc in [(9, (2, 1, 1)), (12, (2, 2, 1))]]
    A, part, nsub, Z, b, x0, off = concat_problems(probs)
    kw = dict(solver="bicgstab2", coarse_enough=30, autotune=0)
    S = L.BatchedSolver(A, part, nsub, Z, off, **kw)
    xb = _t(np.zeros(A.shape[0]))
    outb = S.solve(_t(b), xb)
    S.close()
    xb = xb.cpu().numpy()
    for s, p in enumerate(probs):
        S1 = L.Solver(p.A, p.part, p.nsub, p.Z, **kw)
        x1 = _t(np.zeros(p.n))
        o1 = S1.solve(_t(p.b), x1)
        S1.close()
        assert int(outb["iters"][s]) == o1["iters"]
        assert np.array_equal(xb[off[s]:off[s + 1]], x1.cpu().numpy())
