"""Block-diagonal preconditioners of Sec. III.B (oracle; test infrastructure).

The paper builds M as a block-diagonal section of A itself and names the
choices by the index that is held fixed inside a block.  M^u has one block
per n_u, holding every basis function with that n_u: the matrix elements
A_{(d, n_g, n_u), (d', n_g', n_u)}.  Blocks couple along n_g only.

paper_blocks(Ng, Nu, fixed) gives all six of the paper's choices: the
indices named in ``fixed`` (a string over "d", "g", "u") are held fixed
inside a block, so "g" is M^g (blocks 2 N_u x 2 N_u, fixed n_g), "u" is M^u,
"d" is M^d, and "dg", "gu", "du" are the small-block ones (N_u x N_u, 2 x 2,
N_g x N_g).

segmented_blocks(Ng, Nu, s) splits every block of M^u further into pieces of
s consecutive n_g (and one state d each; at fixed n_u the two states lie in
different symmetry sectors, so A has no element between them there and the
split by d drops nothing).  s = Ng gives M^u itself, s = 1 gives diag(A).

Everything here is the plain definition: the blocks are slices of the
assembled matrix, M^{-1} v is a dense LU solve per block.  Indices refer to
the full layout of model2d (state-major, then n_g, then n_u).
"""
import numpy as np
import scipy.linalg as sla
import scipy.sparse as sp


def segmented_blocks(Ng, Nu, s):
    """Index arrays of the blocks of fixed (d, n_u) and n_g in [g0, g0 + s)."""
    if s < 1:
        raise ValueError("segment length must be >= 1")
    n = Ng * Nu
    out = []
    for d in range(2):
        for u in range(Nu):
            for g0 in range(0, Ng, s):
                g = np.arange(g0, min(Ng, g0 + s))
                out.append(d * n + g * Nu + u)
    return out


def paper_blocks(Ng, Nu, fixed):
    """Index arrays of the blocks of M^{fixed}: the basis functions grouped
    by the values of the indices named in ``fixed``."""
    if not fixed or set(fixed) - set("dgu"):
        raise ValueError("fixed must name indices among d, g, u")
    n = Ng * Nu
    groups = {}
    for d in range(2):
        for g in range(Ng):
            for u in range(Nu):
                key = tuple({"d": d, "g": g, "u": u}[c] for c in "dgu" if c in fixed)
                groups.setdefault(key, []).append(d * n + g * Nu + u)
    return [np.array(groups[k]) for k in sorted(groups)]


def block_matrix(A, blocks):
    """M: the block-diagonal section of A on the given index sets (sparse)."""
    A = sp.csr_matrix(A)
    rows, cols, vals = [], [], []
    for idx in blocks:
        B = A[idx][:, idx].toarray()
        r, c = np.meshgrid(idx, idx, indexing="ij")
        rows.append(r.ravel())
        cols.append(c.ravel())
        vals.append(B.ravel())
    return sp.csr_matrix((np.concatenate(vals), (np.concatenate(rows), np.concatenate(cols))),
                         shape=A.shape)


class BlockInverse:
    """v -> M^{-1} v for M the block-diagonal section of A (LU per block)."""

    def __init__(self, A, blocks):
        A = sp.csr_matrix(A)
        self.blocks = [(idx, sla.lu_factor(A[idx][:, idx].toarray())) for idx in blocks]
        self.n = A.shape[0]

    def __call__(self, v):
        v = np.asarray(v, dtype=np.complex128)
        out = np.zeros_like(v)
        for idx, lu in self.blocks:
            out[idx] = sla.lu_solve(lu, v[idx])
        return out
