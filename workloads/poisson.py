"""7-point finite-difference Poisson operators on a structured grid.

Unknowns are the interior nodes of an (nx+2) x (ny+2) x (nz+2) lattice; the
boundary layer carries homogeneous Dirichlet values and is eliminated, which is
how the paper's 150^3 problem has 3,375,000 unknowns and 23,490,000 nonzeros
(implementation section, single-node OpenMP/CUDA comparison).

Ordering is lexicographic with x fastest: i = ix + nx * (iy + ny * iz).

Coefficients are cellwise (one positive value per unknown).  The coupling
between two neighbouring unknowns is the harmonic mean of their coefficients;
a face on the Dirichlet boundary contributes the unknown's own coefficient to
the diagonal only.  With unit coefficients this is the plain unscaled stencil
(6 on the diagonal, -1 off it).  No h^2 scaling is applied.
"""
import numpy as np
import scipy.sparse as sp


def grid_coords(nx, ny, nz, h=None):
    """Node coordinates ((ix+1)h, (iy+1)h, (iz+1)h) in the unknown ordering.

    h defaults to 1/(max(nx,ny,nz)+1), i.e. isotropic spacing that equals
    1/(N+1) on a cube.
    """
    if h is None:
        h = 1.0 / (max(nx, ny, nz) + 1)
    iz, iy, ix = np.meshgrid(np.arange(nz), np.arange(ny), np.arange(nx),
                             indexing="ij")
    return np.stack([(ix.ravel() + 1) * h, (iy.ravel() + 1) * h,
                     (iz.ravel() + 1) * h], axis=1)


def poisson7(nx, ny=None, nz=None, k=None):
    """Assemble the 7-point operator as a canonical scipy CSR matrix.

    k: None (unit coefficients) or an array of n positive cell coefficients.
    Returns a CSR matrix with sorted column indices, int64 row pointers and
    int32 column indices.
    """
    ny = nx if ny is None else ny
    nz = nx if nz is None else nz
    n = nx * ny * nz
    if k is None:
        k = np.ones(n)
    k = np.asarray(k, dtype=np.float64).reshape(nz, ny, nx)
    idx = np.arange(n, dtype=np.int64).reshape(nz, ny, nx)

    diag = np.zeros((nz, ny, nx))
    rows, cols, vals = [], [], []
    for axis in range(3):
        # interior faces between idx[..., i] and idx[..., i+1] along `axis`
        lo = [slice(None)] * 3
        hi = [slice(None)] * 3
        lo[axis] = slice(0, -1)
        hi[axis] = slice(1, None)
        lo, hi = tuple(lo), tuple(hi)
        ka, kb = k[lo], k[hi]
        face = 2.0 * ka * kb / (ka + kb)
        diag[lo] += face
        diag[hi] += face
        a, b = idx[lo].ravel(), idx[hi].ravel()
        f = face.ravel()
        rows += [a, b]
        cols += [b, a]
        vals += [-f, -f]
        # Dirichlet faces at both ends of the axis use the cell coefficient
        first = [slice(None)] * 3
        last = [slice(None)] * 3
        first[axis] = 0
        last[axis] = -1
        diag[tuple(first)] += k[tuple(first)]
        diag[tuple(last)] += k[tuple(last)]
    rows.append(idx.ravel())
    cols.append(idx.ravel())
    vals.append(diag.ravel())
    A = sp.coo_matrix((np.concatenate(vals),
                       (np.concatenate(rows), np.concatenate(cols))),
                      shape=(n, n)).tocsr()
    A.sum_duplicates()
    A.sort_indices()
    A.indptr = A.indptr.astype(np.int64)
    A.indices = A.indices.astype(np.int32)
    return A
