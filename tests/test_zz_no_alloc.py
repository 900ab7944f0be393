"""dfamg_dense_inverse_noalloc: the dense FP64 inverse computed in a static
per-device workspace, checked against dfamg_dense_inverse (method 1, which
allocates its workspace) through the C ABI.

Both run the same unblocked Gauss-Jordan kernels on the same input, so the
bar is bitwise equality; each inverse is also checked as A X = I.  Two calls
in a row, the second smaller, show that the shared workspace keeps nothing of
the first call that matters to the second.
"""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

import paper_1710_03940_amd as L  # noqa: E402
from paper_1710_03940_amd import _lib  # noqa: E402

pytestmark = pytest.mark.gpu


def _matrix(n, seed):
    rng = np.random.default_rng(seed)
    # diagonally weighted so that the inverse is well conditioned, with row
    # interchanges still needed (the largest entry of a column is off the diagonal
    # in some rows)
    A = rng.standard_normal((n, n)) + 0.5 * np.sqrt(n) * np.eye(n)
    A[[0, n - 1]] = A[[n - 1, 0]]
    return A


def _noalloc(A):
    dev = torch.device("cuda:0")
    a = torch.tensor(A, device=dev)
    out = torch.full_like(a, float("nan"))
    L.dfamg_dense_inverse_noalloc(a, out)
    torch.cuda.synchronize()
    assert torch.equal(a.cpu(), torch.tensor(A)), "input modified"
    return out.cpu().numpy()


def _check_inverse(A, X, tol=1e-11):
    R = A @ X - np.eye(A.shape[0])
    assert np.abs(R).max() <= tol * max(1.0, np.abs(A).max() * np.abs(X).max() * A.shape[0] ** 0.5)


def test_noalloc_matches_allocating_inverse_two_calls():
    for n, seed in ((_lib.NOALLOC_MAX_N, 11), (77, 12)):
        print(f"noalloc inverse n={n} seed={seed}", flush=True)
        A = _matrix(n, seed)
        X = _noalloc(A)
        Xref = L.dfamg_dense_inverse(A, 1)
        assert np.array_equal(X, Xref), np.abs(X - Xref).max()
        _check_inverse(A, X)


def test_noalloc_singular_then_regular():
    n = 40
    A = _matrix(n, 13)
    A[:, 5] = 0.0
    dev = torch.device("cuda:0")
    with pytest.raises(L.DfamgError) as ei:
        L.dfamg_dense_inverse_noalloc(torch.tensor(A, device=dev), torch.empty((n, n), dtype=torch.float64,
                                                                               device=dev))
    assert ei.value.status == _lib.ESINGULAR
    # the singular flag of the previous call does not leak into the next one
    B = _matrix(33, 14)
    X = _noalloc(B)
    assert np.array_equal(X, L.dfamg_dense_inverse(B, 1))


def test_noalloc_rejects_size_beyond_workspace():
    n = _lib.NOALLOC_MAX_N + 1
    dev = torch.device("cuda:0")
    a = torch.eye(n, dtype=torch.float64, device=dev)
    with pytest.raises(L.DfamgError) as ei:
        L.dfamg_dense_inverse_noalloc(a, torch.empty_like(a))
    assert ei.value.status == _lib.EINVAL
    assert "workspace limit" in str(ei.value)
