"""Box partitions of a structured grid into subdomains.

Along an axis with N nodes split into p pieces, node i belongs to piece
floor(i * p / N); for N = 150, p = 4 this gives piece sizes 38, 37, 38, 37.
Subdomain ids are lexicographic over the pieces with x fastest.
"""
import numpy as np


def box_partition(nx, ny, nz, px, py, pz):
    """Return (part, nsub): part[i] in [0, px*py*pz) for every unknown."""
    if not (1 <= px <= nx and 1 <= py <= ny and 1 <= pz <= nz):
        raise ValueError("each axis needs at least one node per piece")
    iz, iy, ix = np.meshgrid(np.arange(nz), np.arange(ny), np.arange(nx),
                             indexing="ij")
    bx = (ix * px) // nx
    by = (iy * py) // ny
    bz = (iz * pz) // nz
    part = (bx + px * (by + py * bz)).ravel().astype(np.int32)
    return part, px * py * pz


def slab_partition(nx, ny, nz, nslabs):
    """Slabs normal to z: part = floor(iz * nslabs / nz)."""
    return box_partition(nx, ny, nz, 1, 1, nslabs)
