"""GPU tests of the status paths of dfamg_solve and of the recovery operator.

* A non-finite right-hand side or initial guess must end the solve with
  DFAMG_ENAN (the relative residual ||r_0|| / ||b|| is not a number), not be
  taken for the b = 0 shortcut, and every kernel must still exit through the
  device stop flags: the handle solves a finite system correctly afterwards.
* A BiCGStab breakdown is forced from the host: with M = I, no deflation,
  A = diag(+1, -1, +1, -1, ...) and b = 1, the shadow residual r~ = r_0 = b is
  orthogonal to v = A r_0, so (r~, v) = sum_i d_i = 0 exactly and the first
  alpha = rho / (r~, v) cannot be formed (BiCGStab(2): the first BiCG step's
  sigma = (r~, A r_0) is the same number).
* DFAMG_OP_RECOVER (x = y + Z E^{-1} Z^T (b - A y), section "Subdomain
  deflation", eqs. (2)-(5)) against the oracle's recovery.
"""
import numpy as np
import pytest
import scipy.sparse as sp

from workloads import tiny_problem, convection_diffusion7
from oracle import OracleSolver, OracleParams

torch = pytest.importorskip("torch")
pytestmark = [pytest.mark.gpu,
              pytest.mark.skipif(not torch.cuda.is_available(), reason="needs a GPU")]


def _t(a):
    return torch.tensor(np.ascontiguousarray(a, dtype=np.float64), device="cuda:0")


def _lib():
    import paper_1710_03940_amd as L
    return L


def _problem(solver):
    if solver == "cg":
        return tiny_problem(N=12, pieces=(2, 2, 1), deflation="linear", sigma=1.0, seed=31)
    base = tiny_problem(N=12, pieces=(2, 2, 1), deflation="linear", seed=31)
    A = convection_diffusion7(12, peclet=2.0)
    return base.__class__("cd12", A, base.part, base.nsub, base.Z, base.b, base.x0)


@pytest.mark.parametrize("solver", ["cg", "bicgstab", "bicgstab2", "fgmres"])
@pytest.mark.parametrize("where", ["rhs", "guess"])
def test_non_finite_input_reports_enan_and_handle_recovers(solver, where):
    L = _lib()
    P = _problem(solver)
    print(f"case nan-{where} solver={solver} n={P.n}", flush=True)
    S = L.Solver(P.A, P.part, P.nsub, P.Z, solver=solver, coarse_enough=40, graph_iters=4)
    b = P.b.copy()
    x0 = np.zeros(P.n)
    if where == "rhs":
        b[P.n // 3] = np.nan
    else:
        x0[P.n // 2] = np.inf
    x = _t(x0)
    out = L._lib.dfamg_solve(S.h, _t(b).data_ptr(), x.data_ptr(), history_cap=0, raise_on_error=False)
    print(f"  status {out['status']} iters {out['iters']}", flush=True)
    assert out["status"] == L._lib.ENAN, out
    assert out["iters"] == 0
    # the same handle then solves a finite system like the oracle
    okw = dict(solver="bicgstabl" if solver == "bicgstab2" else solver, coarse_enough=40)
    ref = OracleSolver(P.A, P.part, P.nsub, P.Z, OracleParams(**okw)).solve(P.b)
    x = _t(np.zeros(P.n))
    out = S.solve(_t(P.b), x)
    S.close()
    assert out["status"] == 0, out
    assert abs(out["iters"] - ref["iters"]) <= 2
    xs = x.cpu().numpy()
    assert np.linalg.norm(xs - ref["x"]) <= 1e-6 * np.linalg.norm(ref["x"])


def test_nan_rhs_batched_flags_only_that_system():
    L = _lib()
    from workloads import concat_problems
    probs = [tiny_problem(N=n, pieces=pc, deflation="linear", sigma=1.0, seed=n)
             for n, pc in [(10, (2, 1, 1)), (12, (2, 2, 1)), (9, (1, 1, 2))]]
    A, part, nsub, Z, b, x0, off = concat_problems(probs)
    b = b.copy()
    b[off[1] + 5] = np.nan
    print(f"case nan-batched n={A.shape[0]} systems={len(probs)}", flush=True)
    S = L.BatchedSolver(A, part, nsub, Z, off, coarse_enough=30)
    x = _t(np.zeros(A.shape[0]))
    st = L._lib.load().dfamg_solve_batched
    iters = np.zeros(3, dtype=np.int32)
    rt = np.zeros(3)
    status = np.zeros(3, dtype=np.int32)
    import ctypes
    ret = st(ctypes.c_void_p(S.h), ctypes.c_void_p(_t(b).data_ptr()), ctypes.c_void_p(x.data_ptr()),
             iters.ctypes.data_as(ctypes.c_void_p), rt.ctypes.data_as(ctypes.c_void_p),
             status.ctypes.data_as(ctypes.c_void_p))
    S.close()
    print(f"  ret {ret} status {status} iters {iters}", flush=True)
    assert ret == L._lib.ENAN
    assert list(status) == [0, L._lib.ENAN, 0]
    xs = x.cpu().numpy()
    for i in (0, 2):
        p = probs[i]
        ref = OracleSolver(p.A, p.part, p.nsub, p.Z, OracleParams(coarse_enough=30)).solve(p.b)
        assert abs(int(iters[i]) - ref["iters"]) <= 1
        seg = xs[off[i]:off[i + 1]]
        assert np.linalg.norm(seg - ref["x"]) <= 1e-6 * np.linalg.norm(ref["x"])


@pytest.mark.parametrize("solver", ["bicgstab", "bicgstab2"])
def test_bicgstab_breakdown_forced_from_host(solver):
    L = _lib()
    n = 64
    d = np.where(np.arange(n) % 2 == 0, 1.0, -1.0)
    A = sp.csr_matrix(sp.diags(d))
    b = np.ones(n)
    # (r~, A r_0) with r~ = r_0 = b is exactly zero: the breakdown the test wants
    assert b @ (A @ b) == 0.0
    print(f"case breakdown solver={solver} n={n}", flush=True)
    S = L.Solver(A, np.zeros(n, dtype=np.int32), 1, np.zeros((n, 0)), solver=solver,
                 precond="none", graph_iters=4)
    x = _t(np.zeros(n))
    out = L._lib.dfamg_solve(S.h, _t(b).data_ptr(), x.data_ptr(), history_cap=0, raise_on_error=False)
    S.close()
    print(f"  status {out['status']} iters {out['iters']}", flush=True)
    assert out["status"] == L._lib.EBREAKDOWN, out
    assert out["iters"] == 0
    xs = x.cpu().numpy()
    assert np.all(np.isfinite(xs))
    assert np.all(xs == 0.0)     # no step was taken: the initial guess comes back


@pytest.mark.parametrize("solver,ndv_kind", [("cg", "linear"), ("bicgstab", "linear"), ("cg", "constant")])
def test_recover_operator_matches_oracle(solver, ndv_kind):
    L = _lib()
    if solver == "cg":
        P = tiny_problem(N=14, pieces=(2, 2, 1), deflation=ndv_kind, sigma=2.0, seed=41)
    else:
        base = tiny_problem(N=14, pieces=(2, 2, 1), deflation=ndv_kind, seed=41)
        P = base.__class__("cd14", convection_diffusion7(14, peclet=3.0), base.part, base.nsub,
                           base.Z, base.b, base.x0)
    print(f"case recover solver={solver} {ndv_kind} n={P.n}", flush=True)
    ora = OracleSolver(P.A, P.part, P.nsub, P.Z, OracleParams(solver=solver, coarse_enough=40))
    S = L.Solver(P.A, P.part, P.nsub, P.Z, solver=solver, coarse_enough=40, maxiter=3)
    # a solve records b on the device (RECOVER uses the last right-hand side)
    x = _t(np.zeros(P.n))
    L._lib.dfamg_solve(S.h, _t(P.b).data_ptr(), x.data_ptr(), raise_on_error=False)
    rng = np.random.default_rng(7)
    for _ in range(2):
        y = rng.standard_normal(P.n)
        out = _t(np.zeros(P.n))
        S.apply(L._lib.OP_RECOVER, _t(y), out)
        ref = ora.defl.recover(P.b, y)
        got = out.cpu().numpy()
        assert np.linalg.norm(got - ref) <= 1e-11 * np.linalg.norm(ref)
        # the recovered iterate's residual is deflated: Z^T (b - A x) = 0
        zt = ora.defl.Z.T @ (P.b - P.A @ got)
        assert np.abs(zt).max() <= 1e-9 * np.linalg.norm(P.b) * np.sqrt(P.n)
    S.close()


def test_recover_without_previous_solve_is_rejected():
    L = _lib()
    P = tiny_problem(N=8, pieces=(2, 1, 1))
    S = L.Solver(P.A, P.part, P.nsub, P.Z, coarse_enough=20)
    with pytest.raises(L.DfamgError):
        S.apply(L._lib.OP_RECOVER, _t(np.ones(P.n)), _t(np.zeros(P.n)))
    S.close()
