"""Stabilised equal-order Q1 Oseen operator (a Navier-Stokes-shaped system).

The paper's Navier-Stokes matrix (equal-order elements with ASGS-type
stabilisation) is not available, so this synthetic stand-in has the same
shape: trilinear hexahedra on a uniform grid of the unit cube, four unknowns
per node interleaved as (u, v, w, p), homogeneous Dirichlet conditions on every
boundary node (all four fields eliminated), a constant convection vector per
element and viscosity nu.  With test function phi_i and trial phi_j
(2x2x2 Gauss quadrature):

  velocity-velocity (each component)  nu (grad phi_j, grad phi_i)
                                      + (phi_i, a . grad phi_j)
                                      + tau (a . grad phi_i, a . grad phi_j)
  velocity d - pressure               -(d_d phi_i, phi_j) + tau (a . grad phi_i, d_d phi_j)
  pressure - velocity d               (phi_i, d_d phi_j) + tau (d_d phi_i, a . grad phi_j)
  pressure - pressure                 tau (grad phi_j, grad phi_i)

with tau_e = (4 nu / h^2 + 2 |a_e| / h)^-1.  Every 4x4 node block has 10
structural nonzeros.  `dt` adds the backward-Euler mass term (phi_i, phi_j)/dt
to the velocity blocks.
"""
import itertools

import numpy as np
import scipy.sparse as sp

from .partition import box_partition


def _reference_q1():
    """Values and reference gradients of the 8 Q1 shape functions at the 8
    Gauss points of [0,1]^3 (weights 1/8)."""
    g = (1.0 - 1.0 / np.sqrt(3.0)) / 2.0
    gp = np.array(list(itertools.product([g, 1.0 - g], repeat=3)))[:, ::-1]   # (q, xyz)
    corners = np.array(list(itertools.product([0, 1], repeat=3)))[:, ::-1]     # (a, xyz) x fastest
    phi = np.ones((8, 8))
    dphi = np.ones((8, 8, 3))
    for q in range(8):
        for a in range(8):
            f = [gp[q, d] if corners[a, d] else 1.0 - gp[q, d] for d in range(3)]
            df = [1.0 if corners[a, d] else -1.0 for d in range(3)]
            phi[q, a] = f[0] * f[1] * f[2]
            for d in range(3):
                prod = df[d]
                for e in range(3):
                    if e != d:
                        prod *= f[e]
                dphi[q, a, d] = prod
    w = np.full(8, 1.0 / 8.0)
    return corners, phi, dphi, w


def oseen_q1(N, nu=1e-2, seed=3, dt=None):
    """Assemble the operator on N^3 interior nodes ((N+1)^3 elements).

    Returns (A as CSR with 4N^3 rows, node coordinates (N^3, 3)).
    """
    h = 1.0 / (N + 1)
    ne = N + 1
    nel = ne ** 3
    corners, phi, dphi_ref, w = _reference_q1()
    dphi = dphi_ref / h                      # physical gradients
    vol = h ** 3
    # element tensors (a = test, b = trial), quadrature summed
    Mab = vol * np.einsum("q,qa,qb->ab", w, phi, phi)
    Lab = vol * np.einsum("q,qad,qbd->ab", w, dphi, dphi)
    Cd = vol * np.einsum("q,qa,qbd->abd", w, phi, dphi)        # phi_a d_d phi_b
    Gdd = vol * np.einsum("q,qad,qbe->abde", w, dphi, dphi)    # d_d phi_a d_e phi_b
    # convection per element: |a| ~ U[0,1], direction uniform on the sphere
    rng = np.random.default_rng(seed)
    mag = rng.uniform(0.0, 1.0, nel)
    d = rng.standard_normal((nel, 3))
    d /= np.linalg.norm(d, axis=1, keepdims=True)
    a = mag[:, None] * d
    tau = 1.0 / (4.0 * nu / h ** 2 + 2.0 * mag / h)
    # element blocks, shape (nel, 8, 8)
    conv = np.einsum("abd,xd->xab", Cd, a)                      # (phi_a, a . grad phi_b)
    supg = np.einsum("abde,xd,xe->xab", Gdd, a, a)              # (a . grad phi_a, a . grad phi_b)
    Kv = nu * Lab[None] + conv + tau[:, None, None] * supg
    if dt is not None:
        Kv = Kv + Mab[None] / dt
    # velocity d (test a) - pressure (trial b)
    Gv = -np.einsum("bad->abd", Cd)[None] + tau[:, None, None, None] * np.einsum("abed,xe->xabd", Gdd, a)
    # pressure (test a) - velocity d (trial b)
    Dv = Cd[None] + tau[:, None, None, None] * np.einsum("abde,xe->xabd", Gdd, a)
    Sp = tau[:, None, None] * Lab[None]
    # global node ids of the element corners ((N+2)^3 lattice, interior 1..N)
    ex, ey, ez = np.meshgrid(np.arange(ne), np.arange(ne), np.arange(ne), indexing="ij")
    ex, ey, ez = ex.transpose(2, 1, 0).ravel(), ey.transpose(2, 1, 0).ravel(), ez.transpose(2, 1, 0).ravel()
    cx = ex[:, None] + corners[None, :, 0]
    cy = ey[:, None] + corners[None, :, 1]
    cz = ez[:, None] + corners[None, :, 2]
    interior = (cx >= 1) & (cx <= N) & (cy >= 1) & (cy <= N) & (cz >= 1) & (cz <= N)
    node = (cx - 1) + N * ((cy - 1) + N * (cz - 1))
    node = np.where(interior, node, -1)
    # scatter the 10 block entries of every (a, b) corner pair
    ia = np.broadcast_to(node[:, :, None], (nel, 8, 8))
    ib = np.broadcast_to(node[:, None, :], (nel, 8, 8))
    keep = (ia >= 0) & (ib >= 0)
    I, J = ia[keep], ib[keep]
    rows, cols, vals = [], [], []
    for c in range(3):                       # u-u, v-v, w-w
        rows.append(4 * I + c)
        cols.append(4 * J + c)
        vals.append(Kv[keep])
    for c in range(3):                       # velocity c - pressure
        rows.append(4 * I + c)
        cols.append(4 * J + 3)
        vals.append(Gv[..., c][keep])
    for c in range(3):                       # pressure - velocity c
        rows.append(4 * I + 3)
        cols.append(4 * J + c)
        vals.append(Dv[..., c][keep])
    rows.append(4 * I + 3)                   # pressure - pressure
    cols.append(4 * J + 3)
    vals.append(Sp[keep])
    n = 4 * N ** 3
    A = sp.coo_matrix((np.concatenate(vals), (np.concatenate(rows), np.concatenate(cols))),
                      shape=(n, n)).tocsr()
    A.sum_duplicates()
    A.sort_indices()
    A.indptr = A.indptr.astype(np.int64)
    A.indices = A.indices.astype(np.int32)
    iz, iy, ix = np.meshgrid(np.arange(N), np.arange(N), np.arange(N), indexing="ij")
    coords = np.stack([(ix.ravel() + 1) * h, (iy.ravel() + 1) * h, (iz.ravel() + 1) * h], axis=1)
    return A, coords


def field_deflation(N, pieces):
    """Per-field constant deflation on a box partition of the nodes: 4 vectors
    per subdomain, the indicator of each of u, v, w, p."""
    part_nodes, nsub = box_partition(N, N, N, *pieces)
    part = np.repeat(part_nodes, 4).astype(np.int32)
    Z = np.zeros((4 * N ** 3, 4))
    for c in range(4):
        Z[c::4, c] = 1.0
    return part, nsub, Z
