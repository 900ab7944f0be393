"""The benchmark workloads, generated from fixed seeds.

* small Poisson: 32^3 unit-coefficient 7-point Poisson, right-hand side of ones
  (the paper's -Laplace u = 1 problem), 8 slabs of 32x32x4, constant deflation;
* log-normal Poisson: 150^3 grid (the paper's single-node size, 3,375,000
  unknowns), cellwise coefficients exp(2 g) with g standard normal (seed 0),
  right-hand side uniform in [-1, 1] (seed 1), 4x4x4 boxes, linear deflation;
* batched: 48 independent log-normal (sigma = 1) Poisson systems with grid
  edges drawn uniformly from [16, 96] and 2..4 pieces per axis (seed 2),
  coefficients from seed 1000+s, right-hand sides from seed 2000+s, linear
  deflation with isotropic spacing 1/(max edge + 1);
* Oseen: the stabilised equal-order Q1 Oseen operator on 64^3 interior nodes
  (4 interleaved unknowns per node, 1,048,576 rows), convection from seed 3,
  nu = 1e-2, right-hand side U[-1,1] from seed 4, 8x8x4 boxes of 8x8x16 nodes,
  per-field constant deflation (4 vectors per subdomain).
"""
from dataclasses import dataclass, field
from typing import Optional

import numpy as np
import scipy.sparse as sp

from .poisson import poisson7, grid_coords
from .partition import box_partition
from .deflation import constant_deflation, linear_deflation
from .oseen import oseen_q1, field_deflation


@dataclass
class Problem:
    name: str
    A: sp.csr_matrix
    part: np.ndarray          # int32 [n]
    nsub: int
    Z: np.ndarray             # float64 [n, ndv]
    b: np.ndarray             # float64 [n]
    x0: np.ndarray            # float64 [n]
    dims: tuple = ()
    pieces: tuple = ()
    meta: dict = field(default_factory=dict)

    @property
    def n(self):
        return self.A.shape[0]

    @property
    def ndv(self):
        return self.Z.shape[1]


def make_problem(name, dims, pieces, deflation="linear", sigma=0.0,
                 coef_seed=None, rhs="ones", rhs_seed=None, h=None):
    """Build one Poisson problem on a box grid.

    sigma > 0 draws cellwise coefficients exp(sigma * g), g ~ N(0,1) from
    default_rng(coef_seed); rhs is "ones" or "uniform" (U[-1,1] from
    default_rng(rhs_seed)).
    """
    nx, ny, nz = dims
    n = nx * ny * nz
    k = None
    if sigma:
        g = np.random.default_rng(coef_seed).standard_normal(n)
        k = np.exp(sigma * g)
    A = poisson7(nx, ny, nz, k)
    part, nsub = box_partition(nx, ny, nz, *pieces)
    if deflation == "constant":
        Z = constant_deflation(n)
    elif deflation == "linear":
        Z = linear_deflation(grid_coords(nx, ny, nz, h), part, nsub)
    else:
        raise ValueError(deflation)
    if rhs == "ones":
        b = np.ones(n)
    elif rhs == "uniform":
        b = np.random.default_rng(rhs_seed).uniform(-1.0, 1.0, n)
    else:
        raise ValueError(rhs)
    return Problem(name, A, part, nsub, Z, b, np.zeros(n), tuple(dims),
                   tuple(pieces), {"sigma": sigma, "deflation": deflation})


def config_small_poisson():
    """32^3 unit Poisson, b = 1, 8 slabs, constant deflation."""
    return make_problem("poisson32_slabs8_constant", (32, 32, 32), (1, 1, 8),
                        deflation="constant")


def config_lognormal_poisson(N=150, pieces=(4, 4, 4)):
    """150^3 log-normal (sigma = 2) Poisson, 64 boxes, linear deflation."""
    return make_problem(f"poisson{N}_lognormal2_boxes{np.prod(pieces)}_linear",
                        (N, N, N), pieces, deflation="linear", sigma=2.0,
                        coef_seed=0, rhs="uniform", rhs_seed=1)


def batched_recipe(nsys=48, seed=2):
    rng = np.random.default_rng(seed)
    edges = rng.integers(16, 97, (nsys, 3))
    pieces = rng.integers(2, 5, (nsys, 3))
    return edges, pieces


def config_batched(nsys=48, seed=2, systems=None):
    """List of the batched systems (a prefix or subset via `systems`)."""
    edges, pieces = batched_recipe(nsys, seed)
    out = []
    for s in (range(nsys) if systems is None else systems):
        dims = tuple(int(v) for v in edges[s])
        pc = tuple(int(v) for v in pieces[s])
        h = 1.0 / (max(dims) + 1)
        out.append(make_problem(f"batched{s}", dims, pc, deflation="linear",
                                sigma=1.0, coef_seed=1000 + s, rhs="uniform",
                                rhs_seed=2000 + s, h=h))
    return out


def concat_problems(problems):
    """Concatenate independent systems into one block-diagonal input.

    Returns (A, part, nsub_total, Z, b, x0, sys_row_off); subdomain ids are
    offset so that they are global across the batch.
    """
    ptrs, cols, vals = [np.zeros(1, dtype=np.int64)], [], []
    row0 = nz0 = 0
    for p in problems:
        ptrs.append(p.A.indptr[1:].astype(np.int64) + nz0)
        cols.append(p.A.indices.astype(np.int64) + row0)
        vals.append(p.A.data)
        row0 += p.n
        nz0 += p.A.nnz
    A = sp.csr_matrix((np.concatenate(vals), np.concatenate(cols).astype(np.int32),
                       np.concatenate(ptrs)), shape=(row0, row0))
    parts, off = [], 0
    for p in problems:
        parts.append(p.part + off)
        off += p.nsub
    ndv = problems[0].ndv
    if any(p.ndv != ndv for p in problems):
        raise ValueError("all systems need the same number of deflation vectors")
    sys_row_off = np.zeros(len(problems) + 1, dtype=np.int64)
    sys_row_off[1:] = np.cumsum([p.n for p in problems])
    return (A, np.concatenate(parts).astype(np.int32), off,
            np.concatenate([p.Z for p in problems]),
            np.concatenate([p.b for p in problems]),
            np.concatenate([p.x0 for p in problems]), sys_row_off)


def tiny_problem(N=6, pieces=(1, 1, 2), deflation="constant", sigma=0.0,
                 seed=0, rhs="uniform", dims=None):
    """Small cases for brute-force checks."""
    dims = (N, N, N) if dims is None else dims
    return make_problem(f"tiny{dims}", dims, pieces, deflation=deflation,
                        sigma=sigma, coef_seed=seed, rhs=rhs,
                        rhs_seed=seed + 17)


def config_oseen(N=64, pieces=(8, 8, 4), nu=1e-2, dt=None):
    """Oseen Q1 system with per-field constant deflation (block size 4)."""
    A, _ = oseen_q1(N, nu=nu, seed=3, dt=dt)
    part, nsub, Z = field_deflation(N, pieces)
    n = A.shape[0]
    b = np.random.default_rng(4).uniform(-1.0, 1.0, n)
    return Problem(f"oseen{N}_boxes{nsub}_field", A, part, nsub, Z, b,
                   np.zeros(n), (N, N, N), tuple(pieces),
                   {"nu": nu, "dt": dt, "block_size": 4, "deflation": "field"})


def config_oseen_schur(N=64, pieces=(8, 8, 4), nu=1e-2, dt=0.1):
    """The Oseen system of config_oseen, as one backward-Euler step of size dt
    (the mass term of a transient solver), split for the Schur pressure
    correction: pressure mask (every fourth unknown), box partition of the
    pressure nodes and one constant deflation vector per subdomain."""
    P = config_oseen(N=N, pieces=pieces, nu=nu, dt=dt)
    pmask = (np.arange(P.n) % 4 == 3).astype(np.int32)
    part_p, nsub = box_partition(N, N, N, *pieces)
    return P, pmask, part_p, nsub, np.ones((N ** 3, 1))

