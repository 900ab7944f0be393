"""V(npre, npost) cycle and the block-diagonal local AMG preconditioner (oracle).

TEST INFRASTRUCTURE ONLY (see the package docstring).

The preconditioner is block AMG without overlap: one AMG per subdomain, built
on the square diagonal block of A, applied independently to the residual
restricted to each subdomain (section "Implementation", last paragraphs).
One application is one V-cycle starting from a zero guess on every level,
with an exact solve on the coarsest level.  The paper's runs use one pre- and
one post-smoothing step (V(1,1), the default); the sweep counts are the
solver parameters npre / npost of the nested parameter listing.  A sweep of
the smoother M is x <- x + M (f - A x); from the zero guess the first
pre-smoothing sweep is x = M f.
"""
import numpy as np
import scipy.linalg as sla

from .sa import build_hierarchy


def vcycle(H, l, f, npre=1, npost=1):
    """x = V(l, f) on hierarchy H with npre pre- and npost post-smoothing sweeps."""
    if l == H.nlevels - 1:
        return sla.lu_solve(H.coarse_lu, f)
    lvl = H.levels[l]
    M = (lambda v: lvl.m * v) if isinstance(lvl.m, np.ndarray) else (lambda v: lvl.m @ v)
    x = np.zeros_like(f)
    for k in range(npre):                           # pre-smooth from x = 0
        x = M(f) if k == 0 else x + M(f - lvl.A @ x)
    r = f - lvl.A @ x
    x = x + lvl.P @ vcycle(H, l + 1, lvl.R @ r, npre, npost)
    for _ in range(npost):                          # post-smooth
        x = x + M(f - lvl.A @ x)
    return x


class BlockAMG:
    """s = M^{-1} r, M^{-1} = blockdiag_s(V-cycle of A[S_s, S_s])."""

    def __init__(self, A, part, nsub, npre=1, npost=1, **sa_params):
        self.npre, self.npost = npre, npost
        part = np.asarray(part)
        self.sets = []
        self.hierarchies = []
        for s in range(nsub):
            S = np.flatnonzero(part == s)            # ascending global index
            self.sets.append(S)
            A_ss = A[S][:, S].tocsr()
            self.hierarchies.append(build_hierarchy(A_ss, **sa_params))

    def apply(self, r):
        out = np.zeros_like(r)
        for S, H in zip(self.sets, self.hierarchies):
            out[S] = vcycle(H, 0, r[S], self.npre, self.npost)
        return out
