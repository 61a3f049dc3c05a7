"""ctypes front end of the C oracle (csrc/oracle.c) — test infrastructure only.

Every function takes plain numpy arrays and returns numpy arrays over the
pattern S = {(i, j) : (L + D + L^T)_ij != 0} in S's CSR layout (both
triangles, sorted columns), in the factor ordering.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from dataclasses import dataclass

import numpy as np
import scipy.sparse as sp

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "csrc", "oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")

ORC_ERRORS = {1: "pattern", 2: "singular D block", 3: "allocation"}


_NATIVE = os.path.join(_HERE, "liboracle_native.so")

# Single-threaded, no fast-math: no reassociation, and no contraction of a
# product and a sum into one rounding (-ffp-contract=off), so every build
# gives the same bits. The shipped copy targets x86-64-v3 (it may run on a
# host other than the one that built it); the timed CPU baseline rebuilds for
# the CPU it runs on (use_host_tuned).
_FLAGS = ["-O3", "-ffp-contract=off", "-std=c11", "-fPIC", "-shared"]


def build(force: bool = True) -> str:
    """Compile the oracle with gcc (-O3 -march=x86-64-v3)."""
    if force or not os.path.exists(_LIB):
        tmp = _LIB + ".tmp"
        subprocess.run(["gcc", *_FLAGS, "-march=x86-64-v3", "-o", tmp, _SRC, "-lm"], check=True)
        os.replace(tmp, _LIB)
    return _LIB


_lib = None
_lib_path = None
_P = ctypes.c_void_p


def use_host_tuned() -> str:
    """Rebuild the oracle for this host's CPU (-O3 -march=native) and load that
    copy instead: for timing it as the CPU baseline on the machine that runs
    it. Same source and floating-point flags, so the same results."""
    global _lib
    tmp = f"{_NATIVE}.{os.getpid()}.tmp"
    subprocess.run(["gcc", *_FLAGS, "-march=native", "-o", tmp, _SRC, "-lm"], check=True)
    os.replace(tmp, _NATIVE)
    _lib = None
    _load(_NATIVE)
    return "gcc -O3 -march=native -ffp-contract=off"


def _load(path=None):
    global _lib, _lib_path
    if _lib is None:
        path = path or _LIB
        if path == _LIB and not os.path.exists(_LIB):
            build(force=False)
        _lib_path = path
        lib = ctypes.CDLL(path)
        i32, i64, f64 = ctypes.c_int32, ctypes.c_int64, ctypes.c_double
        lib.orc_pattern.argtypes = [i32, _P, _P, _P, _P, _P, ctypes.POINTER(i64)]
        lib.orc_selinv.argtypes = [i32, _P, _P, _P, _P, _P, _P, _P, _P, _P, i32]
        lib.orc_linv.argtypes = [i32, _P, _P, _P, i32, f64, i64, _P, _P, _P, ctypes.POINTER(i64)]
        lib.orc_ninv_product.argtypes = [i32, _P, _P, _P, _P, _P, _P, _P, _P, _P]
        lib.orc_mix.argtypes = [i32, _P, _P, _P, _P, f64, _P]
        lib.orc_mix.restype = None
        lib.orc_spai.argtypes = [i32, _P, _P, _P, _P, _P, _P, i32, _P]
        lib.orc_lowrank.argtypes = [i32, i32, _P, _P, _P, _P, _P, _P]
        lib.orc_lowrank.restype = None
        _lib = lib
    return _lib


def _p(a):
    return a.ctypes.data


def _check(rc):
    if rc != 0:
        raise ValueError(f"oracle error: {ORC_ERRORS.get(rc, rc)}")


@dataclass
class Pattern:
    """S in CSR form (both triangles)."""
    n: int
    rowptr: np.ndarray  # int64 [n+1]
    col: np.ndarray     # int32 [nnzS]

    @property
    def nnz(self) -> int:
        return int(self.rowptr[-1])

    def rows(self) -> np.ndarray:
        return np.repeat(np.arange(self.n, dtype=np.int64), np.diff(self.rowptr))

    def diag_positions(self) -> np.ndarray:
        r = self.rows()
        return np.nonzero(r == self.col)[0]

    def to_csr(self, vals) -> sp.csr_matrix:
        return sp.csr_matrix((np.asarray(vals, dtype=np.float64), self.col, self.rowptr),
                             shape=(self.n, self.n))

    def gather(self, M) -> np.ndarray:
        """Values of a (dense or sparse) matrix at the positions of S."""
        if sp.issparse(M):
            M = sp.csr_matrix(M)
            return np.asarray(M[self.rows(), self.col]).ravel()
        return np.asarray(M)[self.rows(), self.col]


def _f(F, name):
    return np.ascontiguousarray(getattr(F, name))


def pattern(F) -> Pattern:
    """S = pattern(L + D + L^T) with the 2x2 union rule (Section 1)."""
    lib = _load()
    n = F.n
    Lp, Li, piv = _f(F, "L_rowptr"), _f(F, "L_col"), _f(F, "piv")
    rowptr = np.zeros(n + 1, np.int64)
    nnz = ctypes.c_int64()
    _check(lib.orc_pattern(n, _p(Lp), _p(Li), _p(piv), _p(rowptr), None, ctypes.byref(nnz)))
    col = np.zeros(max(1, nnz.value), np.int32)
    _check(lib.orc_pattern(n, _p(Lp), _p(Li), _p(piv), _p(rowptr), _p(col), ctypes.byref(nnz)))
    return Pattern(n, rowptr, col[:nnz.value])


def selinv(F, S: Pattern, sentinel: bool = False, wrong_order: bool = False) -> np.ndarray:
    """Takahashi/SelInv recursion on S (Section 2.1). sentinel: start from NaN
    on S, so a read before a write shows as a non-finite result.
    wrong_order: visit the blocks first to last (a planted mistake, only for
    the test that shows the sentinel catches it)."""
    lib = _load()
    Z = np.zeros(max(1, S.nnz))
    flags = (1 if sentinel else 0) | (2 if wrong_order else 0)
    _check(lib.orc_selinv(F.n, _p(_f(F, "L_rowptr")), _p(_f(F, "L_col")), _p(_f(F, "L_val")),
                          _p(_f(F, "d_diag")), _p(_f(F, "d_sub")), _p(_f(F, "piv")),
                          _p(S.rowptr), _p(S.col), _p(Z), flags))
    return Z[:S.nnz]


def linv(F, p: int, delta: float):
    """Columns of the truncated, delta-sparsified Neumann series of L^-1 (Section 2.2).

    Returns CSC arrays (colptr int64, rows int32, vals float64), rows sorted.
    """
    lib = _load()
    n = F.n
    need = ctypes.c_int64()
    args = (n, _p(_f(F, "L_rowptr")), _p(_f(F, "L_col")), _p(_f(F, "L_val")), int(p), float(delta))
    _check(lib.orc_linv(*args, 0, None, None, None, ctypes.byref(need)))
    cap = max(1, need.value)
    Vp = np.zeros(n + 1, np.int64)
    Vi = np.zeros(cap, np.int32)
    Vx = np.zeros(cap)
    _check(lib.orc_linv(*args, cap, _p(Vp), _p(Vi), _p(Vx), ctypes.byref(need)))
    return Vp, Vi[:need.value], Vx[:need.value]


def ninv(F, S: Pattern, p: int, delta: float, linv_cols=None) -> np.ndarray:
    """NInv on S: (L^inv)^T D^-1 L^inv evaluated at the positions of S (Section 2.2)."""
    lib = _load()
    Vp, Vi, Vx = linv(F, p, delta) if linv_cols is None else linv_cols
    N = np.zeros(max(1, S.nnz))
    Vi = np.ascontiguousarray(Vi) if len(Vi) else np.zeros(1, np.int32)
    Vx = np.ascontiguousarray(Vx) if len(Vx) else np.zeros(1)
    _check(lib.orc_ninv_product(F.n, _p(Vp), _p(Vi), _p(Vx), _p(_f(F, "d_diag")),
                                _p(_f(F, "d_sub")), _p(_f(F, "piv")), _p(S.rowptr), _p(S.col),
                                _p(N)))
    return N[:S.nnz]


def dinv_matrix(F) -> sp.csr_matrix:
    """D^-1 as a sparse block-diagonal matrix (1x1 and 2x2 blocks, Section 2.1),
    2x2 inverses as [d, -c; -c, a] / (a d - c^2)."""
    n = F.n
    rows, cols, vals = [], [], []
    j = 0
    while j < n:
        if F.piv[j] == 1:
            a, c, d = F.d_diag[j], F.d_sub[j], F.d_diag[j + 1]
            det = a * d - c * c
            rows += [j, j, j + 1, j + 1]
            cols += [j, j + 1, j, j + 1]
            vals += [d / det, -c / det, -c / det, a / det]
            j += 2
        else:
            rows.append(j)
            cols.append(j)
            vals.append(1.0 / F.d_diag[j])
            j += 1
    return sp.csr_matrix((vals, (rows, cols)), shape=(n, n))


def ninv_full(F, p: int, delta: float, drop: float, linv_cols=None):
    """NInv on its own pattern (Section 2.2): N = (L^inv)^T D^-1 L^inv over
    every pair of columns of L^inv that meet a common D block, with the
    off-diagonal entries |N_ij| < drop sqrt(|N_ii N_jj|) removed (the product
    drop of Section 2.2). Returns the lower triangle (diagonal included) as
    CSR arrays (rowptr int64, col int32 sorted, val float64)."""
    n = F.n
    Vp, Vi, Vx = linv(F, p, delta) if linv_cols is None else linv_cols
    Li = sp.csc_matrix((Vx, Vi, Vp), shape=(n, n))
    Di = dinv_matrix(F)
    N = (Li.T @ Di @ Li).tocsr()
    # structure without cancellation: the same product over indicator matrices
    B = sp.csc_matrix((np.ones(len(Vi)), Vi, Vp), shape=(n, n))
    C = sp.csr_matrix((np.ones(Di.nnz), Di.indices, Di.indptr), shape=(n, n))
    Pt = sp.tril(B.T @ C @ B).tocsr()
    Pt.sort_indices()
    r = np.repeat(np.arange(n), np.diff(Pt.indptr))
    c = Pt.indices.astype(np.int64)
    v = np.asarray(N[r, c]).ravel()
    d = N.diagonal()
    keep = (r == c) | (np.abs(v) >= drop * np.sqrt(np.abs(d[r] * d[c])))
    r, c, v = r[keep], c[keep], v[keep]
    rowptr = np.zeros(n + 1, np.int64)
    np.add.at(rowptr, r + 1, 1)
    return np.cumsum(rowptr), c.astype(np.int32), v


def mix_full(S: Pattern, Z: np.ndarray, Nfull, eps: float):
    """Mix on NInv's own pattern (Section 2.3): Z_ij for (i, j) in S_eps =
    {|Z_ij| > eps sqrt(|Z_ii Z_jj|)}, N_ij elsewhere on N's pattern; the
    pattern is N's joined with S_eps. Nfull and the result are lower
    triangles (diagonal included) as CSR arrays (rowptr, col, val)."""
    n = S.n
    r = S.rows()
    c = S.col.astype(np.int64)
    zd = np.asarray(Z)[S.diag_positions()]
    sel = (c <= r) & (np.abs(Z) > eps * np.sqrt(np.abs(zd[r] * zd[c])))
    out = {}
    Np, Nc, Nv = Nfull
    for i in range(n):
        for q in range(Np[i], Np[i + 1]):
            out[(i, int(Nc[q]))] = Nv[q]
    for q in np.nonzero(sel)[0]:
        out[(int(r[q]), int(c[q]))] = Z[q]
    keys = sorted(out)
    rowptr = np.zeros(n + 1, np.int64)
    for (i, _) in keys:
        rowptr[i + 1] += 1
    return (np.cumsum(rowptr), np.array([k[1] for k in keys], dtype=np.int32),
            np.array([out[k] for k in keys], dtype=np.float64))


def spmv(S: Pattern, X: np.ndarray, x: np.ndarray) -> np.ndarray:
    """y = X x for X on S (Section 2.5: the second term of E x)."""
    return S.to_csr(X) @ np.asarray(x, dtype=np.float64)


def error_eigenpairs(Ahat, S: Pattern, X: np.ndarray, k: int):
    """The k eigenpairs of largest |lambda| of the inverse-error operator
    E = Ah^-1 - X (Section 2.5, Algorithm 1), by its definition: Ah^-1 as a
    dense inverse, X as the dense matrix of its values on S, the symmetric
    eigendecomposition of E. Returns (lambda [k] in decreasing |lambda|, ties
    by ascending lambda, V [n, k] orthonormal). Dense: small n only."""
    Ainv = np.linalg.inv(np.asarray(sp.csr_matrix(Ahat).todense(), dtype=np.float64))
    E = Ainv - np.asarray(S.to_csr(X).todense())
    lam, V = np.linalg.eigh(0.5 * (E + E.T))
    order = np.argsort(-np.abs(lam), kind="stable")[:k]
    return lam[order], np.ascontiguousarray(V[:, order])


def za_diag(S: Pattern, Z: np.ndarray, Ahat) -> np.ndarray:
    """(Z Ah)_ii = sum_k Z_ik Ah_ki for Z on S (1 where Z is exact on the
    rows' reach, Section 2.1)."""
    return np.asarray((S.to_csr(Z) @ sp.csr_matrix(Ahat)).diagonal()).ravel()


def unit_lower(F) -> sp.csr_matrix:
    """L with its unit diagonal (the factor stores the strictly lower part)."""
    L = sp.csr_matrix(F.L_csr())
    return (L + sp.identity(F.n, format="csr")).tocsr()


def ldl_solve(F, x: np.ndarray) -> np.ndarray:
    """y = (L D L^T)^-1 x: the incomplete factorization as a preconditioner
    (Section 2.5), by two triangular solves around the D-block inverses."""
    from scipy.sparse.linalg import spsolve_triangular
    L = unit_lower(F)
    z = spsolve_triangular(L, np.asarray(x, dtype=np.float64), lower=True, unit_diagonal=True)
    w = dinv_matrix(F) @ z
    return spsolve_triangular(sp.csr_matrix(L.T), w, lower=False, unit_diagonal=True)


def mix(S: Pattern, Z: np.ndarray, N: np.ndarray, eps: float) -> np.ndarray:
    """Mix (Section 2.3): Z where |Z_ij| > eps sqrt(|Z_ii Z_jj|), else N."""
    lib = _load()
    M = np.zeros(max(1, S.nnz))
    Z = np.ascontiguousarray(Z, dtype=np.float64)
    N = np.ascontiguousarray(N, dtype=np.float64)
    lib.orc_mix(S.n, _p(S.rowptr), _p(S.col), _p(Z), _p(N), float(eps), _p(M))
    return M[:S.nnz]


def spai(Ahat, S: Pattern, M: np.ndarray, iters: int) -> np.ndarray:
    """Mix-SPAI (Section 2.4): per-column CG refinement on S, then (X + X^T)/2.

    ``Ahat`` = P^T A P in the factor ordering (both triangles).
    """
    lib = _load()
    Ahat = sp.csr_matrix(Ahat)
    Ahat.sort_indices()
    Ap = np.ascontiguousarray(Ahat.indptr, dtype=np.int64)
    Aj = np.ascontiguousarray(Ahat.indices, dtype=np.int32)
    Ax = np.ascontiguousarray(Ahat.data, dtype=np.float64)
    R = np.zeros(max(1, S.nnz))
    M = np.ascontiguousarray(M, dtype=np.float64)
    _check(lib.orc_spai(S.n, _p(Ap), _p(Aj), _p(Ax), _p(S.rowptr), _p(S.col), _p(M), int(iters),
                        _p(R)))
    return R[:S.nnz]


def lowrank(S: Pattern, V: np.ndarray, lam: np.ndarray, X: np.ndarray) -> np.ndarray:
    """Rank-k correction on S (Section 2.5): X_ij + sum_m lam_m V_im V_jm."""
    lib = _load()
    V = np.ascontiguousarray(V, dtype=np.float64)
    lam = np.ascontiguousarray(lam, dtype=np.float64)
    X = np.ascontiguousarray(X, dtype=np.float64)
    out = np.zeros(max(1, S.nnz))
    lib.orc_lowrank(S.n, V.shape[1], _p(V), _p(lam), _p(S.rowptr), _p(S.col), _p(X), _p(out))
    return out[:S.nnz]


def diag(S: Pattern, X: np.ndarray) -> np.ndarray:
    return np.asarray(X)[S.diag_positions()]


def err1(d: np.ndarray, dhat: np.ndarray) -> float:
    """Relative diagonal 1-norm error ||d - dhat||_1 / ||d||_1 (Section 2.6)."""
    return float(np.abs(d - dhat).sum() / np.abs(d).sum())


def selinv_block_check(F, S: Pattern, Z: np.ndarray, blocks) -> np.ndarray:
    """Largest entry error, per block J in `blocks` (first columns), between a
    result Z on S and the SelInv recursion of Section 2.1 evaluated from Z's
    own entries on S: Z(R_J, J) = -Zhat(R_J, R_J) L(R_J, J) with Zhat = Z on S
    and 0 off S, and Z_JJ = D_J^-1 - L(R_J, J)^T Z(R_J, J) (2x2 off-diagonal:
    the mean of its two expressions). A Z that satisfies this at every block
    is the SelInv result; checking a sample of blocks is a property test that
    holds at any size."""
    Lc = F.L_csr().tocsc()
    Lc.sort_indices()
    Z = np.asarray(Z)
    dpos = S.diag_positions()

    def zval(rows, cols):
        # Z at (rows[k], cols[k]) when stored in S, else 0
        out = np.zeros(len(rows))
        for k, (r, c) in enumerate(zip(rows, cols)):
            seg = S.col[S.rowptr[r]:S.rowptr[r + 1]]
            q = np.searchsorted(seg, c)
            if q < len(seg) and seg[q] == c:
                out[k] = Z[S.rowptr[r] + q]
        return out

    errs = []
    for j in blocks:
        j = int(j)
        J = [j, j + 1] if F.piv[j] == 1 else [j]
        last = J[-1]
        R = sorted(set(int(r) for c in J for r in Lc.indices[Lc.indptr[c]:Lc.indptr[c + 1]] if r > last))
        c = len(R)
        LRJ = np.zeros((c, len(J)))
        for b, col in enumerate(J):
            rows = Lc.indices[Lc.indptr[col]:Lc.indptr[col + 1]]
            vals = Lc.data[Lc.indptr[col]:Lc.indptr[col + 1]]
            for r, v in zip(rows, vals):
                if r > last:
                    LRJ[R.index(int(r)), b] = v
        if c:
            rr, ll = np.meshgrid(R, R, indexing="ij")
            Zh = zval(rr.ravel(), ll.ravel()).reshape(c, c)
        else:
            Zh = np.zeros((0, 0))
        y = -Zh @ LRJ
        if len(J) == 1:
            Dinv = np.array([[1.0 / F.d_diag[j]]])
        else:
            a, b2, d = F.d_diag[j], F.d_sub[j], F.d_diag[j + 1]
            Dinv = np.array([[d, -b2], [-b2, a]]) / (a * d - b2 * b2)
        ZJJ = Dinv - LRJ.T @ y
        if len(J) == 2:
            ZJJ[0, 1] = ZJJ[1, 0] = 0.5 * (ZJJ[0, 1] + ZJJ[1, 0])
        got_y = np.stack([zval(R, [col] * c) for col in J], axis=1) if c else np.zeros((0, len(J)))
        got_J = np.array([[zval([a1], [b1])[0] for b1 in J] for a1 in J])
        def zd(i):
            return abs(Z[dpos[i]])
        e = 0.0
        for k, r in enumerate(R):
            for b, col in enumerate(J):
                sc = max(np.sqrt(zd(r) * zd(col)), abs(y[k, b]))
                e = max(e, abs(got_y[k, b] - y[k, b]) / (sc if sc > 0 else 1.0))
        for a1 in range(len(J)):
            for b1 in range(len(J)):
                sc = max(np.sqrt(zd(J[a1]) * zd(J[b1])), abs(ZJJ[a1, b1]))
                e = max(e, abs(got_J[a1, b1] - ZJJ[a1, b1]) / (sc if sc > 0 else 1.0))
        errs.append(e)
    return np.array(errs)


def dag_levels(F, S: Pattern) -> np.ndarray:
    """Level of every unknown in the SelInv dependency DAG (Section 2.1; the
    schedule reading for an incomplete pattern): the blocks J of D (1x1, or
    the two columns of a 2x2 pivot) are visited last to first, R_J is the set
    of rows of S below J outside J, level(J) = 0 when R_J is empty and
    1 + max level over R_J otherwise; both columns of a 2x2 block carry the
    block's level."""
    n = F.n
    piv = np.asarray(F.piv)
    lev = np.zeros(n, dtype=np.int64)
    j = n - 1
    while j >= 0:
        j0 = j - 1 if piv[j] == 2 else j
        R = set()
        for c in range(j0, j + 1):
            cols = S.col[S.rowptr[c]:S.rowptr[c + 1]]
            R.update(int(r) for r in cols if r > j)
        lev[j0:j + 1] = 1 + max(lev[r] for r in R) if R else 0
        j = j0 - 1
    return lev


def corrected_diag(dhat: np.ndarray, V: np.ndarray, lam: np.ndarray) -> np.ndarray:
    """Diagonal of the rank-k corrected approximation (Section 2.6):
    dhat_i + sum_m lam_m V_im^2."""
    dk = np.array(dhat, dtype=np.float64)
    for m in range(len(lam)):
        dk += lam[m] * V[:, m] * V[:, m]
    return dk


def err1_sums(d: np.ndarray, dhat: np.ndarray, V=None, lam=None):
    """(||d - dhat^k||_1, ||d||_1), the two sums of err_1 (Section 2.6) for the
    diagonal corrected by the modes (V, lam) (none when V is None)."""
    dk = dhat if V is None else corrected_diag(dhat, V, lam)
    return float(np.abs(d - dk).sum()), float(np.abs(d).sum())


def trace_sums(S, X: np.ndarray, V=None, lam=None):
    """(tr, ||diag||_1) of the approximation X on S, corrected by the modes
    (V, lam) when given: the trace estimate of the covariance A^-1 as the sum
    of the approximate diagonal (Section 3.5)."""
    d = diag(S, X)
    dk = d if V is None else corrected_diag(d, V, lam)
    return float(dk.sum()), float(np.abs(dk).sum())


def accept_modes(d: np.ndarray, dhat: np.ndarray, V: np.ndarray, lam: np.ndarray):
    """Acceptance test of Algorithm 1, read per mode: candidates are taken in
    order of decreasing |lam| (ties by index); each is kept only if adding it to
    the modes kept so far makes ||d - dhat^k||_1 strictly smaller (Section 3,
    safeguard on the diagonal error). Returns (indices kept, err_1 before,
    err_1 after)."""
    order = sorted(range(len(lam)), key=lambda m: (-abs(lam[m]), m))
    kept = []
    cur = np.array(dhat, dtype=np.float64)
    base, dn = err1_sums(d, cur)
    best = base
    for m in order:
        cand = cur + lam[m] * V[:, m] * V[:, m]
        e = float(np.abs(d - cand).sum())
        if e < best:
            kept.append(m)
            cur, best = cand, e
    return kept, base / dn, best / dn


def entry_error(S: Pattern, X: np.ndarray, Y: np.ndarray) -> np.ndarray:
    """Per-entry error |x_ij - y_ij| / sqrt(|y_ii y_jj|) on S (Y is the reference).

    For indefinite inputs a diagonal entry of the inverse can vanish; the
    scale is then max(sqrt(|y_ii y_jj|), |y_ij|), and 1 where both are zero
    (the error becomes absolute). For SPD inputs |y_ij| <= sqrt(y_ii y_jj), so
    the scale is the plain one.
    """
    X = np.asarray(X)
    Y = np.asarray(Y)
    dy = diag(S, Y)
    r = S.rows()
    scale = np.maximum(np.sqrt(np.abs(dy[r] * dy[S.col])), np.abs(Y))
    scale = np.where(scale > 0, scale, 1.0)
    return np.abs(X - Y) / scale


def permuted(A, perm) -> sp.csr_matrix:
    """P^T A P = A[perm][:, perm] in the factor ordering."""
    A = sp.csr_matrix(A)
    B = A[perm][:, perm].tocsr()
    B.sort_indices()
    return B
