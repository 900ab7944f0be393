"""GPU parity of the dense FP64 inverses of the coarse operator E (the blocked
panel + GEMM elimination and the unblocked one) against numpy's LAPACK
inverse, on ragged sizes around the panel width, a case that needs pivoting,
a singular matrix and the largest supported size; and the E^{-1} a handle
holds against the inverse of the setup's E."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")
pytestmark = [pytest.mark.gpu,
              pytest.mark.skipif(not torch.cuda.is_available(), reason="needs a GPU")]


def _matrix(n, seed):
    rng = np.random.default_rng(seed)
    return rng.standard_normal((n, n)) + 2.0 * np.sqrt(n) * np.eye(n)


def _check(A, X, tol=1e-12):
    n = A.shape[0]
    ref = np.linalg.inv(A)
    assert np.linalg.norm(X - ref) <= tol * np.linalg.norm(ref)
    assert np.abs(A @ X - np.eye(n)).max() <= tol * np.sqrt(n) * 10


@pytest.mark.parametrize("n", [1, 2, 63, 64, 65, 127, 128, 130, 200, 513, 1024])
@pytest.mark.parametrize("method", [0, 1])
def test_dense_inverse_matches_lapack(n, method):
    import paper_1710_03940_amd as L
    print(f"case n={n} method={method}", flush=True)
    A = _matrix(n, seed=n)
    _check(A, L.dfamg_dense_inverse(A, method))


@pytest.mark.parametrize("method", [0, 1])
def test_dense_inverse_needs_pivoting(method):
    """Zero diagonal: without row interchanges the first pivot is zero."""
    import paper_1710_03940_amd as L
    n = 150
    rng = np.random.default_rng(1)
    perm = rng.permutation(n)
    while np.any(perm == np.arange(n)):
        perm = rng.permutation(n)
    A = np.zeros((n, n))
    A[np.arange(n), perm] = 3.0 + rng.random(n)
    A += 0.05 * rng.standard_normal((n, n)) * (A == 0)
    np.fill_diagonal(A, 0.0)
    _check(A, L.dfamg_dense_inverse(A, method), tol=1e-11)


@pytest.mark.parametrize("method", [0, 1])
def test_dense_inverse_singular(method):
    import paper_1710_03940_amd as L
    A = _matrix(140, seed=3)
    A[:, 77] = 0.0                       # a zero column stays zero: exact breakdown
    with pytest.raises(L.DfamgError) as ei:
        L.dfamg_dense_inverse(A, method)
    assert ei.value.status == 3          # DFAMG_ESINGULAR


def test_dense_inverse_largest_size_blocked():
    import paper_1710_03940_amd as L
    A = _matrix(4096, seed=9)
    X = L.dfamg_dense_inverse(A, 0)
    assert np.abs(A @ X - np.eye(4096)).max() <= 1e-10


def test_handle_coarse_inverse_blocked_and_unblocked():
    """m = 1024 (blocked) for the Oseen operator with 256 subdomains, m = 64
    (unblocked) for a small Poisson problem."""
    import paper_1710_03940_amd as L
    from workloads import config_oseen, make_problem
    for P, kw in [(config_oseen(N=32, pieces=(8, 8, 4)), dict(solver="bicgstab", block_size=4)),
                  (make_problem("p", (16, 16, 16), (4, 2, 2), deflation="linear"), dict())]:
        plan = L.dfamg_plan_create(L.make_params(**kw), P.A, P.part, P.nsub, P.Z)
        E = L.dfamg_plan_coarse_operator(plan)
        L.dfamg_plan_destroy(plan)
        S = L.Solver(P.A, P.part, P.nsub, P.Z, **kw)
        X = S.coarse_inverse()
        S.close()
        print(f"m={E.shape[0]}", flush=True)
        assert X.shape == E.shape
        _check(E, X, tol=1e-10)


def test_coarse_operator_assembled_on_device_matches_setup():
    """E = Z^T A Z from one operator product per column on the device against
    the host setup's E (linear deflation, coded Z; per-field deflation of the
    Oseen operator, m = 1024, the size the setup assembles on the device)."""
    import paper_1710_03940_amd as L
    from workloads import config_oseen, make_problem
    for P, kw in [(make_problem("p", (16, 16, 16), (4, 2, 2), deflation="linear", sigma=1.0, coef_seed=2), dict()),
                  (config_oseen(N=32, pieces=(8, 8, 4)), dict(solver="bicgstab", block_size=4))]:
        plan = L.dfamg_plan_create(L.make_params(**kw), P.A, P.part, P.nsub, P.Z)
        E = L.dfamg_plan_coarse_operator(plan)
        L.dfamg_plan_destroy(plan)
        S = L.Solver(P.A, P.part, P.nsub, P.Z, **kw)
        Ed = S.coarse_operator()
        X = S.coarse_inverse()
        S.close()
        print(f"m={E.shape[0]}", flush=True)
        assert np.abs(Ed - E).max() <= 1e-12 * np.abs(E).max()
        _check(E, X, tol=1e-10)
