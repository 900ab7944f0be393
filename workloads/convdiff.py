"""Small nonsymmetric test operators: 7-point diffusion plus first-order upwind
convection with a constant velocity on the same grid and ordering as
`poisson7` (Dirichlet nodes eliminated).  Used to exercise the nonsymmetric
(BiCGStab, LU) paths on inputs small enough for dense checks.
"""
import numpy as np
import scipy.sparse as sp

from .poisson import poisson7


def convection_diffusion7(nx, ny=None, nz=None, velocity=(1.0, 0.5, 0.25),
                          peclet=2.0):
    """A = L + peclet * C with L the unit 7-point Laplacian and C the upwind
    convection matrix for `velocity` (grid units)."""
    ny = nx if ny is None else ny
    nz = nx if nz is None else nz
    L = poisson7(nx, ny, nz)
    n = nx * ny * nz
    idx = np.arange(n).reshape(nz, ny, nx)
    rows, cols, vals = [], [], []
    diag = np.zeros(n)
    for axis, v in zip((2, 1, 0), velocity):   # x is the last array axis
        a = abs(v)
        if a == 0.0:
            continue
        diag += a
        # upwind neighbour: i - e for v > 0, i + e for v < 0
        sl_row = [slice(None)] * 3
        sl_nbr = [slice(None)] * 3
        if v > 0:
            sl_row[axis] = slice(1, None)
            sl_nbr[axis] = slice(0, -1)
        else:
            sl_row[axis] = slice(0, -1)
            sl_nbr[axis] = slice(1, None)
        r = idx[tuple(sl_row)].ravel()
        c = idx[tuple(sl_nbr)].ravel()
        rows.append(r)
        cols.append(c)
        vals.append(np.full(r.size, -a))
    rows.append(np.arange(n))
    cols.append(np.arange(n))
    vals.append(diag)
    C = sp.coo_matrix((np.concatenate(vals),
                       (np.concatenate(rows), np.concatenate(cols))),
                      shape=(n, n)).tocsr()
    A = (L + peclet * C).tocsr()
    A.sum_duplicates()
    A.sort_indices()
    A.indptr = A.indptr.astype(np.int64)
    A.indices = A.indices.astype(np.int32)
    return A
