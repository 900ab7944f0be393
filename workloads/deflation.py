"""Local deflation blocks Z^l (one row per unknown, ndv columns).

Only the block local to each subdomain is stored: row i holds the values of
the deflation vectors of the subdomain that owns unknown i.  The full
n x (nsub*ndv) basis is implied by the partition.

* constant ("subdomain") deflation: a single column of ones
  (section "Constant deflation");
* linear deflation: four columns 1, x - c_x, y - c_y, z - c_z with c the
  barycenter of the subdomain, taken as the unweighted mean of the node
  coordinates of the subdomain (section "Linear deflation").
"""
import numpy as np


def constant_deflation(n):
    return np.ones((n, 1), dtype=np.float64)


def linear_deflation(coords, part, nsub):
    coords = np.asarray(coords, dtype=np.float64)
    part = np.asarray(part)
    cnt = np.bincount(part, minlength=nsub).astype(np.float64)
    if np.any(cnt == 0):
        raise ValueError("empty subdomain")
    Z = np.empty((coords.shape[0], 4))
    Z[:, 0] = 1.0
    for d in range(3):
        c = np.bincount(part, weights=coords[:, d], minlength=nsub) / cnt
        Z[:, 1 + d] = coords[:, d] - c[part]
    return Z
