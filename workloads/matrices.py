"""Seeded synthetic sparse symmetric matrices.

Every generator returns a ``scipy.sparse.csr_matrix`` holding both triangles,
with int64 row pointers, int32 column indices (sorted within each row) and
float64 values. Grid unknowns are numbered lexicographically with x fastest:
node(x, y[, z]) = x + nx*y [+ nx*ny*z].

The workloads stand in for the paper's SuiteSparse test set (Section 3.2,
table of test matrices): SPD finite-volume/finite-difference operators for the
structural/FE class, a shifted Laplacian with a prescribed number of negative
eigenvalues for the indefinite class, and strongly diagonally dominant random
graphs for the microbenchmark class. Randomness comes only from
``numpy.random.default_rng(seed)``, drawn in the order documented per function.
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp


def _csr(n, rows, cols, vals):
    A = sp.coo_matrix((vals, (rows, cols)), shape=(n, n)).tocsr()
    A.sum_duplicates()
    A.sort_indices()
    A.indptr = A.indptr.astype(np.int64)
    A.indices = A.indices.astype(np.int32)
    A.data = A.data.astype(np.float64)
    return A


def _grid_pairs(shape, offset):
    """Pairs (p, p+offset) of in-grid nodes for a lexicographic grid (x fastest).

    ``shape`` is (nx, ny[, nz]) and ``offset`` the integer displacement per axis.
    Returns the flat indices of both endpoints and the base coordinates.
    """
    dims = len(shape)
    ranges = []
    for a in range(dims):
        lo = max(0, -offset[a])
        hi = min(shape[a], shape[a] - offset[a])
        ranges.append(np.arange(lo, hi))
    grids = np.meshgrid(*ranges, indexing="ij")
    coords = [g.ravel() for g in grids]
    strides = [1]
    for a in range(1, dims):
        strides.append(strides[-1] * shape[a - 1])
    p = sum(c * s for c, s in zip(coords, strides))
    q = sum((c + o) * s for c, o, s in zip(coords, offset, strides))
    return p.astype(np.int64), q.astype(np.int64), coords


def laplace2d(nx: int, ny: int | None = None, shift: float = 0.0):
    """5-point Dirichlet Laplacian on an nx-by-ny grid plus ``shift`` * I.

    Diagonal 4 + shift, neighbours -1. Used as 32x32 with shift 0.01 (the small
    SPD case) and, with a negative shift, as the indefinite case.
    """
    ny = nx if ny is None else ny
    n = nx * ny
    rows = [np.arange(n)]
    cols = [np.arange(n)]
    vals = [np.full(n, 4.0 + shift)]
    for off in [(1, 0), (0, 1)]:
        p, q, _ = _grid_pairs((nx, ny), off)
        rows += [p, q]
        cols += [q, p]
        vals += [-np.ones(len(p)), -np.ones(len(p))]
    return _csr(n, np.concatenate(rows), np.concatenate(cols), np.concatenate(vals))


def laplace2d_eigenvalues(nx: int, ny: int | None = None):
    """Closed-form eigenvalues 4 sin^2(p pi/(2(nx+1))) + 4 sin^2(q pi/(2(ny+1))), sorted."""
    ny = nx if ny is None else ny
    lx = 4.0 * np.sin(np.arange(1, nx + 1) * np.pi / (2 * (nx + 1))) ** 2
    ly = 4.0 * np.sin(np.arange(1, ny + 1) * np.pi / (2 * (ny + 1))) ** 2
    return np.sort((lx[:, None] + ly[None, :]).ravel())


def shifted_laplace2d_indefinite(N: int = 512, n_negative: int = 20):
    """5-point Dirichlet Laplacian on N x N minus sigma*I, indefinite.

    sigma is the midpoint of the n_negative-th and (n_negative+1)-th smallest
    closed-form eigenvalues, so exactly ``n_negative`` eigenvalues are negative.
    Returns (A, sigma).
    """
    lam = laplace2d_eigenvalues(N)
    gap = lam[n_negative] - lam[n_negative - 1]
    if gap <= 1e-9 * lam[n_negative]:
        raise ValueError(f"eigenvalues {n_negative} and {n_negative + 1} coincide; "
                         "sigma would make the matrix singular")
    sigma = 0.5 * (lam[n_negative - 1] + lam[n_negative])
    return laplace2d(N, N, -sigma), float(sigma)


def diffusion3d_7pt(N: int = 64, sigma: float = 1.0, seed: int = 2):
    """3D 7-point finite-volume diffusion on N^3 with lognormal face coefficients.

    Face coefficients c = exp(sigma * xi), xi ~ N(0,1), are drawn as three
    arrays indexed (x, y, z): x-faces of shape (N+1, N, N), then y-faces
    (N, N+1, N), then z-faces (N, N, N+1); face i along an axis lies between
    cells i-1 and i. Boundary faces add their coefficient to the diagonal
    (Dirichlet); A_ii is the sum of the cell's six face coefficients and
    A_ij = -c for an interior face. The result is SPD with DoDD = 1.
    """
    rng = np.random.default_rng(seed)
    cx = np.exp(sigma * rng.standard_normal((N + 1, N, N)))
    cy = np.exp(sigma * rng.standard_normal((N, N + 1, N)))
    cz = np.exp(sigma * rng.standard_normal((N, N, N + 1)))
    n = N ** 3
    # diagonal: sum of the six faces of every cell, flattened x fastest
    diag = (cx[:-1, :, :] + cx[1:, :, :] + cy[:, :-1, :] + cy[:, 1:, :]
            + cz[:, :, :-1] + cz[:, :, 1:])
    diag = diag.transpose(2, 1, 0).ravel()  # (x,y,z) -> flat x + N y + N^2 z
    rows = [np.arange(n)]
    cols = [np.arange(n)]
    vals = [diag]
    for axis, c in enumerate((cx, cy, cz)):
        off = [0, 0, 0]
        off[axis] = 1
        p, q, coords = _grid_pairs((N, N, N), off)
        idx = list(coords)
        idx[axis] = idx[axis] + 1  # face between cell and its +axis neighbour
        w = c[idx[0], idx[1], idx[2]]
        rows += [p, q]
        cols += [q, p]
        vals += [-w, -w]
    return _csr(n, np.concatenate(rows), np.concatenate(cols), np.concatenate(vals))


STENCIL27_DIRECTIONS = [
    (1, 0, 0), (0, 1, 0), (0, 0, 1),
    (1, 1, 0), (1, -1, 0), (1, 0, 1), (1, 0, -1), (0, 1, 1), (0, 1, -1),
    (1, 1, 1), (1, 1, -1), (1, -1, 1), (1, -1, -1),
]


def stencil27_3d(N: int = 128, sigma: float = 0.5, seed: int = 5):
    """3D 27-point stencil on N^3 with lognormal coupling coefficients.

    For each of the 13 half-space directions d (in ``STENCIL27_DIRECTIONS``
    order) a padded (N+2)^3 array C_d = exp(sigma * xi) indexed (x, y, z) is
    drawn; the pair {q, q+d} with base q in [-1, N]^3 has coefficient
    C_d[q + 1]. Ghost neighbours outside the grid keep their coefficients, so
    A_ii is the sum of all 26 couplings of node i and A_ij = -c for in-grid
    pairs: SPD with DoDD = 1.
    """
    rng = np.random.default_rng(seed)
    n = N ** 3
    P = N + 2
    diag = np.zeros((N, N, N))
    rows = []
    cols = []
    vals = []
    for d in STENCIL27_DIRECTIONS:
        C = np.exp(sigma * rng.standard_normal((P, P, P)))
        # coupling to +d: base q = p, padded index p + 1
        diag += C[1:N + 1, 1:N + 1, 1:N + 1]
        # coupling to -d: base q = p - d, padded index p - d + 1
        diag += C[1 - d[0]:N + 1 - d[0], 1 - d[1]:N + 1 - d[1], 1 - d[2]:N + 1 - d[2]]
        p, q, coords = _grid_pairs((N, N, N), d)
        w = C[coords[0] + 1, coords[1] + 1, coords[2] + 1]
        rows += [p, q]
        cols += [q, p]
        vals += [-w, -w]
        del C
    rows.append(np.arange(n))
    cols.append(np.arange(n))
    vals.append(diag.transpose(2, 1, 0).ravel())
    return _csr(n, np.concatenate(rows), np.concatenate(cols), np.concatenate(vals))


def random_dd_symmetric(seed: int, n: int | None = None, per_row: int = 5,
                        dominance: float = 1.05):
    """Random sparse symmetric, strictly diagonally dominant matrix.

    Draw order from ``default_rng(seed)``: n = integers(2000, 20001) unless
    given; then for every row i in order, ``per_row`` distinct partners
    j != i chosen uniformly; the union of unordered pairs (sorted
    lexicographically) gets one N(0,1) value each; a_ii = dominance * sum_j |a_ij|.
    About 2 * per_row off-diagonals per row.
    """
    rng = np.random.default_rng(seed)
    if n is None:
        n = int(rng.integers(2000, 20001))
    k = min(per_row, n - 1)
    pick = np.empty((n, k), dtype=np.int64)
    for i in range(n):
        c = rng.choice(n - 1, size=k, replace=False)
        pick[i] = c + (c >= i)
    ii = np.repeat(np.arange(n, dtype=np.int64), k)
    jj = pick.ravel()
    lo = np.minimum(ii, jj)
    hi = np.maximum(ii, jj)
    key = np.unique(lo * n + hi)
    lo = key // n
    hi = key % n
    v = rng.standard_normal(len(key))
    absrow = np.bincount(lo, weights=np.abs(v), minlength=n) + \
        np.bincount(hi, weights=np.abs(v), minlength=n)
    diag = dominance * absrow
    diag[diag == 0] = 1.0
    rows = np.concatenate([lo, hi, np.arange(n)])
    cols = np.concatenate([hi, lo, np.arange(n)])
    vals = np.concatenate([v, v, diag])
    return _csr(n, rows, cols, vals)


def kkt_matrix(m: int, k: int, seed: int, density: float = 0.3):
    """Saddle-point matrix [[0_k, B], [B^T, I_m]] with a random k-by-m block B.

    The zero block comes first, so factoring in the natural order meets zero
    pivots and forces Bunch-Kaufman 2x2 pivots. B has N(0,1) values with the
    given density and at least one entry per row.
    """
    rng = np.random.default_rng(seed)
    B = rng.standard_normal((k, m)) * (rng.random((k, m)) < density)
    for r in range(k):
        if not B[r].any():
            B[r, rng.integers(m)] = 1.0 + rng.random()
    K = np.zeros((m + k, m + k))
    K[k:, k:] = np.eye(m)
    K[:k, k:] = B
    K[k:, :k] = B.T
    r, c = np.nonzero(K)
    return _csr(m + k, r, c, K[r, c])


def saddle2d(N: int = 160, seed: int = 7, scale: float = 8.0):
    """Sparse saddle-point matrix [[A, B^T], [B, 0]] and an ordering for it.

    A: the 5-point Dirichlet Laplacian on an N x N grid (diagonal 4, N even),
    unknowns 0 .. N^2 - 1 lexicographic (x fastest). B: one constraint per
    2 x 2 cell (N^2 / 4 of them, unknowns N^2 + cell index, cells
    lexicographic) coupling the cell's four grid unknowns with weights
    s scale (0.5 + U(0, 1)), s a random sign; drawn from
    numpy.random.default_rng(seed), cell by cell, the four corners in the order
    (0,0), (1,0), (0,1), (1,1), the magnitude before the sign. The zero
    diagonal of the constraints makes a symmetric indefinite matrix; with
    couplings larger than the Laplacian's diagonal (the default scale) the
    grid unknown a constraint meets fails the Bunch-Kaufman 1x1 test as well,
    and the threshold factorization takes (constraint, grid unknown) 2x2
    pivots.

    Returns (K, q): q orders the cells by the nested multicolor ordering of the
    (N/2 x N/2) cell grid, each cell's constraint first and its four grid
    unknowns after it, so the factorization meets every constraint's zero
    pivot beside the unknowns it couples.
    """
    from .ordering import nested_multicolor_grid
    if N % 2:
        raise ValueError("N must be even")
    rng = np.random.default_rng(seed)
    L2 = laplace2d(N, N, 0.0)
    A_row = np.repeat(np.arange(N * N), np.diff(L2.indptr))
    nu, M = N * N, N // 2
    nc = M * M
    cx, cy = np.meshgrid(np.arange(M), np.arange(M), indexing="xy")
    cx, cy = cx.ravel(), cy.ravel()  # cell c = cx + M cy
    corners = [(0, 0), (1, 0), (0, 1), (1, 1)]
    rows, cols, vals = [], [], []
    draws = rng.random((nc, 4, 2))
    for k, (dx, dy) in enumerate(corners):
        u = (2 * cx + dx) + N * (2 * cy + dy)
        w = scale * (0.5 + draws[:, k, 0]) * np.where(draws[:, k, 1] < 0.5, -1.0, 1.0)
        rows += [nu + np.arange(nc), u]
        cols += [u, nu + np.arange(nc)]
        vals += [w, w]
    r = np.concatenate([A_row] + rows)
    c = np.concatenate([L2.indices.astype(np.int64)] + cols)
    v = np.concatenate([L2.data] + vals)
    K = _csr(nu + nc, r, c, v)
    cell_order = nested_multicolor_grid((M, M))
    q = np.empty(nu + nc, np.int64)
    pos = 0
    for c0 in cell_order:
        x, y = c0 % M, c0 // M
        q[pos] = nu + c0
        for dx, dy in corners:
            q[pos + 1 + (dx + 2 * dy)] = (2 * x + dx) + N * (2 * y + dy)
        pos += 5
    return K, q


def dodd(A) -> float:
    """Degree of diagonal dominance min_i |a_ii| / sum_{j != i} |a_ij| (Section 3.2)."""
    A = sp.csr_matrix(A)
    d = np.abs(A.diagonal())
    off = np.asarray(abs(A).sum(axis=1)).ravel() - d
    with np.errstate(divide="ignore"):
        r = np.where(off > 0, d / np.where(off > 0, off, 1), np.inf)
    return float(r.min())


def covariance_grid(N: int = 200, alpha: float = 3.0, beta: float = 4.0):
    """Covariance-type matrix on an N-by-N grid (the paper's covariance and
    uncertainty-quantification example): c_ij = (1 - d(i, j) / alpha)^beta
    where the Euclidean grid distance d(i, j) <= alpha, 0 otherwise.

    The diagonal is 1. For beta >= 3/2 the truncated power function is a
    positive definite kernel in two dimensions, so the matrix is SPD; with
    alpha = 3, beta = 4 it has 25 entries per interior row and is not
    diagonally dominant (off-diagonal row sums about 1.19). Deterministic.
    """
    n = N * N
    r = int(np.floor(alpha))
    rows = [np.arange(n)]
    cols = [np.arange(n)]
    vals = [np.ones(n)]
    for dy in range(0, r + 1):
        for dx in range(-r, r + 1):
            if dy == 0 and dx <= 0:
                continue  # each unordered pair once
            d = float(np.hypot(dx, dy))
            if d > alpha:
                continue
            c = (1.0 - d / alpha) ** beta
            if c == 0.0:
                continue
            p, q, _ = _grid_pairs((N, N), (dx, dy))
            rows += [p, q]
            cols += [q, p]
            vals += [np.full(len(p), c), np.full(len(p), c)]
    return _csr(n, np.concatenate(rows), np.concatenate(cols), np.concatenate(vals))
