"""Smoothed-aggregation AMG hierarchy for one subdomain block (oracle).

TEST INFRASTRUCTURE ONLY (see the package docstring).

The paper builds one AMG preconditioner per subdomain from the square diagonal
block of A (non-local columns dropped, which acts as a Dirichlet condition),
with smoothed aggregation as the coarsening and SPAI-0 (one sweep) or damped
Jacobi (damping 0.8) as the relaxation (sections "Implementation" and
"Benchmarks"; Listing 1).  The paper names these components but does not spell
out their internals, so the oracle fixes the following readings:

* strength of connection at level l with eps_l = 0.08 / 2^l:
  j is a strong neighbour of i (j != i) when |A_ij|^2 >= eps_l^2 |A_ii| |A_jj|,
  where for point-block matrices |.| is the Frobenius norm of the b x b block
  and the test runs on the node graph;
* plain aggregation in three passes over nodes in ascending order
  (Vanek, Mandel & Brezina 1996):
  1. an unaggregated node with a non-empty strong neighbourhood that is
     entirely unaggregated starts a new aggregate {i} + N_i;
  2. every node still unaggregated after pass 1 with a non-empty
     neighbourhood joins the pass-1 aggregate of its strong neighbour with the
     largest |A_ij| (smallest j on ties), judged against the pass-1 result;
  3. every node still unaggregated with a non-empty neighbourhood starts an
     aggregate with itself and its still unaggregated strong neighbours;
  nodes with no strong neighbour stay out of every aggregate (their row of
  the prolongation is zero); aggregate ids follow creation order;
* coarsening stops when the level has at most `coarse_enough` scalar unknowns,
  when no aggregate forms or when aggregation does not reduce the size, or
  after `max_levels` levels;
* tentative prolongation P_t = (aggregate indicator) kron I_b, unnormalised;
* filtered matrix A_F: strong off-diagonal blocks kept, weak off-diagonal
  blocks added to the diagonal block, so A_F has the row sums of A;
* omega = (4/3) / rho, rho = max_i sum_j ||D_i^{-1} A_F,ij||_inf with D the
  block diagonal of A_F (for b = 1: sum_j |a^F_ij| / |a^F_ii|), rows with a
  singular diagonal block excluded, computed per subdomain and level;
* P = P_t - omega D^{-1} A_F P_t, R = P^T, A_{l+1} = R A_l P;
* smoother on every non-coarsest level: SPAI-0 m_i = a_ii / sum_j a_ij^2
  (Broeker & Grote 2002, scalar rows even for block matrices), damped
  Jacobi m_i = 0.8 / a_ii, or block SPAI-0 (b x b diagonal blocks, see
  block_spai0) for point-block matrices;
* the coarsest level is solved exactly (dense LU with partial pivoting).
"""
from dataclasses import dataclass, field
from typing import List, Optional

import numpy as np
import scipy.linalg as sla
import scipy.sparse as sp

from . import _aggregate


@dataclass
class Level:
    A: sp.csr_matrix
    P: Optional[sp.csr_matrix] = None      # n_l x n_{l+1}
    R: Optional[sp.csr_matrix] = None      # n_{l+1} x n_l
    m: Optional[np.ndarray] = None         # smoother diagonal
    eps: float = 0.0
    omega: float = 0.0
    agg: Optional[np.ndarray] = None       # node -> aggregate id (-1 isolated)
    n_agg: int = 0


@dataclass
class Hierarchy:
    levels: List[Level] = field(default_factory=list)
    coarse_lu: object = None               # scipy lu_factor of the coarsest A

    @property
    def nlevels(self):
        return len(self.levels)


def _node_frobenius_sq(A, bs):
    """Node-level matrix holding ||A_IJ||_F^2 for every stored block."""
    n = A.shape[0]
    rows = np.repeat(np.arange(n), np.diff(A.indptr))
    F = sp.coo_matrix((A.data * A.data, (rows // bs, A.indices // bs)),
                      shape=(n // bs, n // bs)).tocsr()
    F.sum_duplicates()
    F.sort_indices()
    return F


def strong_graph(A, eps, bs=1):
    """Node graph of strong connections.

    Returns (F, strong) with F the node-level CSR of squared block Frobenius
    norms and `strong` a boolean mask over F's stored entries.
    """
    F = _node_frobenius_sq(A, bs)
    nn = F.shape[0]
    dnorm = np.sqrt(F.diagonal())
    rows = np.repeat(np.arange(nn), np.diff(F.indptr))
    cols = F.indices
    strong = (cols != rows) & (F.data >= eps * eps * dnorm[rows] * dnorm[cols])
    return F, strong


def plain_aggregation(F, strong):
    """Three-pass aggregation on the strong node graph (ascending order).

    Returns (agg, n_agg) with agg[i] = -1 for nodes left out of every
    aggregate.
    """
    return _aggregate.aggregate(F.indptr, F.indices, np.sqrt(F.data), strong)


def tentative_prolongation(agg, n_agg, bs=1):
    nn = agg.shape[0]
    keep = agg >= 0
    rows = np.arange(nn)[keep]
    cols = agg[keep]
    if bs == 1:
        return sp.csr_matrix((np.ones(rows.size), (rows, cols)),
                             shape=(nn, n_agg))
    r = (rows[:, None] * bs + np.arange(bs)).ravel()
    c = (cols[:, None] * bs + np.arange(bs)).ravel()
    return sp.csr_matrix((np.ones(r.size), (r, c)), shape=(nn * bs, n_agg * bs))


def filtered_matrix(A, F, strong, bs=1):
    """A_F: strong off-diagonal blocks kept, weak ones lumped into the
    diagonal block (row sums preserved)."""
    n = A.shape[0]
    rows = np.repeat(np.arange(n), np.diff(A.indptr))
    cols = A.indices.astype(np.int64)
    I, J = rows // bs, cols // bs
    # strong flag per scalar entry: look up the node pair (I, J) in F, whose
    # entries are sorted by (row, column)
    nn = F.shape[0]
    keyF = np.repeat(np.arange(nn, dtype=np.int64), np.diff(F.indptr)) * nn \
        + F.indices
    pos = np.searchsorted(keyF, I.astype(np.int64) * nn + J)
    weak = (I != J) & ~strong[pos]
    new_cols = np.where(weak, I * bs + cols % bs, cols)
    AF = sp.coo_matrix((A.data, (rows, new_cols)), shape=A.shape).tocsr()
    AF.sum_duplicates()
    AF.sort_indices()
    return AF


def block_diag_inverse(AF, bs=1):
    """Block-diagonal D^{-1} of A_F (singular blocks replaced by zero) and a
    mask of rows (nodes) whose block is invertible."""
    n = AF.shape[0]
    nn = n // bs
    D = np.zeros((nn, bs, bs))
    rows = np.repeat(np.arange(n), np.diff(AF.indptr))
    cols = AF.indices
    same = (rows // bs) == (cols // bs)
    D[rows[same] // bs, rows[same] % bs, cols[same] % bs] = AF.data[same]
    Dinv = np.zeros_like(D)
    ok = np.zeros(nn, dtype=bool)
    for I in range(nn) if bs > 1 else []:
        try:
            if np.linalg.matrix_rank(D[I]) == bs:
                Dinv[I] = np.linalg.inv(D[I])
                ok[I] = True
        except np.linalg.LinAlgError:
            pass
    if bs == 1:
        d = D[:, 0, 0]
        ok = d != 0
        Dinv[ok, 0, 0] = 1.0 / d[ok]
    r = (np.arange(nn)[:, None, None] * bs + np.arange(bs)[None, :, None])
    c = (np.arange(nn)[:, None, None] * bs + np.arange(bs)[None, None, :])
    r, c = np.broadcast_arrays(r, c)
    Dinv_mat = sp.csr_matrix((Dinv.ravel(), (r.ravel(), c.ravel())),
                             shape=(n, n))
    Dinv_mat.eliminate_zeros()
    return Dinv_mat, ok


def gershgorin_omega(AF, Dinv, ok, bs=1):
    """omega = (4/3) / max_I sum_J ||D_I^{-1} A_F,IJ||_inf."""
    B = (Dinv @ AF).tocsr()
    n = B.shape[0]
    rows = np.repeat(np.arange(n), np.diff(B.indptr))
    # row abs sums per (scalar row, node column), then inf-norm per block
    T = sp.coo_matrix((np.abs(B.data), (rows, B.indices // bs)),
                      shape=(n, n // bs)).tocsr()
    T.sum_duplicates()
    # ||block||_inf = max over the block's scalar rows of the abs row sum
    Trows = np.repeat(np.arange(n), np.diff(T.indptr))
    node = Trows // bs
    key = node.astype(np.int64) * (n // bs) + T.indices
    order = np.lexsort((T.data, key))
    key_s, val_s = key[order], T.data[order]
    last = np.r_[key_s[1:] != key_s[:-1], True]
    blk_key, blk_inf = key_s[last], val_s[last]
    rho_node = np.bincount(blk_key // (n // bs), weights=blk_inf,
                           minlength=n // bs)
    rho = rho_node[ok].max() if np.any(ok) else 1.0
    return (4.0 / 3.0) / rho


def smoothed_prolongation(AF, Ptent, omega, Dinv):
    P = (Ptent - omega * (Dinv @ (AF @ Ptent))).tocsr()
    P.sum_duplicates()
    P.sort_indices()
    return P


def smoother_diagonal(A, kind="spai0", jacobi_omega=0.8, bs=1):
    """The smoother M of one level: a vector (diagonal SPAI-0 or damped
    Jacobi) or, for "block_spai0", a block-diagonal sparse matrix."""
    d = A.diagonal()
    if kind == "spai0":
        sq = np.asarray(A.multiply(A).sum(axis=1)).ravel()
        return d / sq
    if kind == "jacobi":
        return jacobi_omega / d
    if kind == "block_spai0":
        return block_spai0(A, bs)
    raise ValueError(kind)


def block_spai0(A, bs):
    """Block SPAI-0: the block-diagonal M minimising ||I - M A||_F over
    matrices with b x b diagonal blocks (the block form of the SPAI-0 of
    Broeker and Grote).  Row block i of I - M A is E_i - M_i A_(i,:), whose
    least-squares minimiser is M_i = A_ii^T (A_(i,:) A_(i,:)^T)^{-1}; for b = 1
    this is a_ii / sum_j a_ij^2."""
    A = sp.csr_matrix(A)
    n = A.shape[0]
    nb = n // bs
    blocks = []
    for i in range(nb):
        rows = A[i * bs:(i + 1) * bs]
        G = (rows @ rows.T).toarray()
        Aii = rows[:, i * bs:(i + 1) * bs].toarray()
        blocks.append(np.linalg.solve(G.T, Aii).T)         # A_ii^T G^{-1}
    return sp.block_diag(blocks, format="csr")


def build_hierarchy(A, eps_strong=0.08, coarse_enough=500, max_levels=20,
                    smoother="spai0", jacobi_omega=0.8, bs=1):
    """Build the SA hierarchy of one subdomain block A (scipy CSR, FP64)."""
    A = sp.csr_matrix(A, dtype=np.float64)
    A.sort_indices()
    H = Hierarchy()
    eps = eps_strong
    while True:
        lvl = Level(A=A, eps=eps)
        H.levels.append(lvl)
        n = A.shape[0]
        if n <= coarse_enough or len(H.levels) >= max_levels:
            break
        F, strong = strong_graph(A, eps, bs)
        agg, n_agg = plain_aggregation(F, strong)
        if n_agg == 0 or n_agg * bs >= n:
            break
        Pt = tentative_prolongation(agg, n_agg, bs)
        AF = filtered_matrix(A, F, strong, bs)
        Dinv, ok = block_diag_inverse(AF, bs)
        omega = gershgorin_omega(AF, Dinv, ok, bs)
        P = smoothed_prolongation(AF, Pt, omega, Dinv)
        R = P.T.tocsr()
        R.sort_indices()
        Ac = (R @ A @ P).tocsr()
        Ac.sum_duplicates()
        Ac.sort_indices()
        lvl.P, lvl.R, lvl.agg, lvl.n_agg, lvl.omega = P, R, agg, n_agg, omega
        lvl.m = smoother_diagonal(A, smoother, jacobi_omega, bs)
        A = Ac
        eps = eps * 0.5
    H.coarse_lu = sla.lu_factor(H.levels[-1].A.toarray(), check_finite=True)
    return H
