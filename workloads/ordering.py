"""Fill-reducing symmetric orderings.

An ordering is an int64 array ``q`` with ``A[q][:, q]`` the reordered matrix
(position k holds original unknown q[k]). The paper leaves the ordering of
the block ILDL open (it only lists ordering among the error sources of the
factorization, Section 2.5); these are the choices used for the synthetic
workloads: reverse Cuthill-McKee for the small 2D case and the random graphs,
and a geometric nested dissection that also orders every separator by nested
dissection of its own lower-dimensional box (which keeps the dependency DAG
of the incomplete factor shallow).
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp
from scipy.sparse.csgraph import reverse_cuthill_mckee


def rcm(A) -> np.ndarray:
    """Reverse Cuthill-McKee ordering of the symmetric pattern of ``A``."""
    A = sp.csr_matrix(A)
    B = sp.csr_matrix((np.ones(A.nnz), A.indices.astype(np.int32), A.indptr.astype(np.int32)),
                      shape=A.shape)
    return np.asarray(reverse_cuthill_mckee(B, symmetric_mode=True), dtype=np.int64)


def nested_dissection_grid(shape, leaf: int = 1) -> np.ndarray:
    """Geometric nested dissection of a lexicographic (x fastest) grid.

    The box is split along its longest axis at the midpoint plane; the two
    halves are ordered first (recursively), then the separator plane, which is
    itself ordered by nested dissection of its own box (one dimension lower).
    Boxes with at most ``leaf`` nodes are numbered lexicographically.
    """
    shape = tuple(int(s) for s in shape)
    dims = len(shape)
    strides = [1]
    for a in range(1, dims):
        strides.append(strides[-1] * shape[a - 1])
    out = np.empty(int(np.prod(shape)), dtype=np.int64)
    pos = 0
    # explicit stack of (lo, hi, phase) boxes; phase 0 = expand, else emit
    stack = [(tuple(0 for _ in shape), shape)]
    # iterative post-order: we push in reverse so that left, right, separator
    # come out in that order
    while stack:
        lo, hi = stack.pop()
        ext = [h - l for l, h in zip(lo, hi)]
        size = int(np.prod(ext))
        if size == 0:
            continue
        if size == 1:
            out[pos] = sum(l * s for l, s in zip(lo, strides))
            pos += 1
            continue
        if size <= leaf:
            grids = np.meshgrid(*[np.arange(l, h) for l, h in zip(lo, hi)], indexing="ij")
            idx = sum(g.transpose(*reversed(range(dims))).ravel() * s
                      for g, s in zip(grids, strides))
            out[pos:pos + size] = idx
            pos += size
            continue
        a = int(np.argmax(ext))
        mid = (lo[a] + hi[a]) // 2
        left_hi = list(hi)
        left_hi[a] = mid
        right_lo = list(lo)
        right_lo[a] = mid + 1
        sep_lo = list(lo)
        sep_lo[a] = mid
        sep_hi = list(hi)
        sep_hi[a] = mid + 1
        # pushed in reverse of the emission order
        stack.append((tuple(sep_lo), tuple(sep_hi)))
        stack.append((tuple(right_lo), tuple(hi)))
        stack.append((tuple(lo), tuple(left_hi)))
    assert pos == len(out)
    return out


def nested_multicolor_grid(shape) -> np.ndarray:
    """Nested multicolor ordering of a lexicographic (x fastest) grid.

    Unknowns are sorted by their bit-reversed Morton key: the lowest bit of
    every coordinate is the most significant digit, then the next bit, and so
    on. The first sort digit is the 2^d parity colouring (no two unknowns of a
    colour are stencil neighbours for the 5/7/9/27-point stencils), and each
    colour class is ordered the same way on the grid coarsened by two. For
    incomplete factors this keeps the dependency DAG of the selected-inversion
    sweep O(log N) deep instead of the O(N^(d-1)) separator chains of nested
    dissection, at the same fill.
    """
    shape = tuple(int(s) for s in shape)
    dims = len(shape)
    n = int(np.prod(shape))
    idx = np.arange(n, dtype=np.int64)
    coords = []
    rem = idx
    for a in range(dims):
        coords.append(rem % shape[a])
        rem = rem // shape[a]
    nb = max(1, int(np.ceil(np.log2(max(shape)))))
    key = np.zeros(n, dtype=np.int64)
    for b in range(nb):
        for a in range(dims):
            key |= ((coords[a] >> b) & 1) << (dims * (nb - 1 - b) + a)
    return np.argsort(key, kind="stable").astype(np.int64)


def apply_symmetric_perm(A, q):
    """Return A[q][:, q] as canonical CSR (int64 indptr, int32 indices)."""
    A = sp.csr_matrix(A)
    B = A[q][:, q].tocsr()
    B.sort_indices()
    B.indptr = B.indptr.astype(np.int64)
    B.indices = B.indices.astype(np.int32)
    return B
