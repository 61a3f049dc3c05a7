"""Python front end of the host threshold ILDL (Bunch-Kaufman) input producer.

``ildl_bk(A, q, tau)`` factors the symmetrically ordered A[q][:, q] and
returns L, D and the composed permutation ``perm`` with
A[perm][:, perm] ~ L D L^T, in the layouts the selected-inversion library
takes: L strictly lower CSR (int64 rowptr, int32 col, float64 val), D as
d_diag / d_sub / piv arrays (piv 0 = 1x1, 1 and 2 = first and second index
of a 2x2 block, d_sub[j] = D[j+1, j] at a block start, else 0).
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from dataclasses import dataclass, field

import numpy as np
import scipy.sparse as sp

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "csrc", "ildl_bk.c")
_LIB = os.path.join(_HERE, "libildl.so")


def build(force: bool = True) -> str:
    """Compile the ILDL shared library in-tree with gcc (host code only)."""
    if force or not os.path.exists(_LIB):
        tmp = _LIB + ".tmp"
        subprocess.run(["gcc", "-O3", "-std=c11", "-fPIC", "-shared", "-o", tmp, _SRC, "-lm"],
                       check=True)
        os.replace(tmp, _LIB)
    return _LIB


class _Res(ctypes.Structure):
    _fields_ = [
        ("n", ctypes.c_int32),
        ("nnzL", ctypes.c_int64),
        ("L_rowptr", ctypes.POINTER(ctypes.c_int64)),
        ("L_col", ctypes.POINTER(ctypes.c_int32)),
        ("L_val", ctypes.POINTER(ctypes.c_double)),
        ("d_diag", ctypes.POINTER(ctypes.c_double)),
        ("d_sub", ctypes.POINTER(ctypes.c_double)),
        ("piv", ctypes.POINTER(ctypes.c_int8)),
        ("order", ctypes.POINTER(ctypes.c_int32)),
        ("n_perturbed", ctypes.c_int64),
        ("n_2x2", ctypes.c_int64),
        ("peak_schur", ctypes.c_int64),
    ]


_lib = None


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB):
            build(force=False)
        lib = ctypes.CDLL(_LIB)
        lib.ildl_bk.restype = ctypes.c_int
        lib.ildl_bk.argtypes = [ctypes.c_int32, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p,
                                ctypes.c_double, ctypes.c_int, ctypes.POINTER(_Res)]
        lib.ildl_set_progress.restype = None
        lib.ildl_set_progress.argtypes = [ctypes.c_int32]
        lib.ildl_free.restype = None
        lib.ildl_free.argtypes = [ctypes.POINTER(_Res)]
        _lib = lib
    return _lib


@dataclass
class IldlFactors:
    """P^T A P ~ L D L^T with A[perm][:, perm] = P^T A P."""
    n: int
    perm: np.ndarray          # int32 [n]
    L_rowptr: np.ndarray      # int64 [n+1]
    L_col: np.ndarray         # int32 [nnzL]
    L_val: np.ndarray         # float64 [nnzL]
    d_diag: np.ndarray        # float64 [n]
    d_sub: np.ndarray         # float64 [n]
    piv: np.ndarray           # int8 [n]
    tau: float
    n_perturbed: int = 0
    n_2x2: int = 0
    stats: dict = field(default_factory=dict)

    @property
    def nnzL(self) -> int:
        return int(self.L_rowptr[-1])

    @property
    def nnzS(self) -> int:
        """nnz(L + D + L^T) counted over both triangles (2x2 blocks add 2)."""
        return 2 * self.nnzL + self.n + 2 * int(np.count_nonzero(self.piv == 1))

    def trailing(self, k: int) -> "IldlFactors":
        """The factor of the trailing unknowns k..n-1 (rows and columns of L,
        D and piv from k on, renumbered from 0; k must not split a 2x2 block).
        L is lower triangular, so every result of the method on the trailing
        unknowns depends on this part only: it is a sub-problem whose result
        is the trailing block of the whole result."""
        if not 0 <= k < self.n or self.piv[k] == 2:
            raise ValueError("k must start a block")
        rows = np.repeat(np.arange(self.n), np.diff(self.L_rowptr))
        keep = (rows >= k) & (self.L_col >= k)
        n2 = self.n - k
        rp = np.zeros(n2 + 1, np.int64)
        np.add.at(rp, rows[keep] - k + 1, 1)
        return IldlFactors(n=n2, perm=np.arange(n2, dtype=np.int32), L_rowptr=np.cumsum(rp),
                           L_col=(self.L_col[keep] - k).astype(np.int32), L_val=self.L_val[keep].copy(),
                           d_diag=self.d_diag[k:].copy(), d_sub=self.d_sub[k:].copy(), piv=self.piv[k:].copy(),
                           tau=self.tau, n_2x2=int(np.count_nonzero(self.piv[k:] == 1)))

    def L_csr(self):
        return sp.csr_matrix((self.L_val, self.L_col, self.L_rowptr), shape=(self.n, self.n))

    def D_csr(self):
        n = self.n
        rows = [np.arange(n)]
        cols = [np.arange(n)]
        vals = [self.d_diag]
        s = np.nonzero(self.piv == 1)[0]
        rows += [s, s + 1]
        cols += [s + 1, s]
        vals += [self.d_sub[s], self.d_sub[s]]
        return sp.csr_matrix((np.concatenate(vals), (np.concatenate(rows), np.concatenate(cols))),
                             shape=(n, n))


def ildl_bk(A, q=None, tau: float = 1e-3, pivoting: bool = True, progress: bool = False) -> IldlFactors:
    """Threshold ILDL with Bunch-Kaufman pivots of A ordered by q.

    ``q`` is a fill-reducing ordering (identity if None); the returned
    ``perm`` composes q with the pivoting swaps. ``progress`` prints a line
    to stderr every 5 % of the pivots.
    """
    A = sp.csr_matrix(A)
    n = A.shape[0]
    if q is None:
        q = np.arange(n, dtype=np.int64)
    q = np.asarray(q, dtype=np.int64)
    B = A[q][:, q].tocsr()
    B.sort_indices()
    rowptr = np.ascontiguousarray(B.indptr, dtype=np.int64)
    col = np.ascontiguousarray(B.indices, dtype=np.int32)
    val = np.ascontiguousarray(B.data, dtype=np.float64)
    lib = _load()
    lib.ildl_set_progress(max(1, n // 20) if progress else 0)
    res = _Res()
    rc = lib.ildl_bk(n, rowptr.ctypes.data, col.ctypes.data, val.ctypes.data, float(tau),
                     1 if pivoting else 0, ctypes.byref(res))
    if rc != 0:
        raise RuntimeError(f"ildl_bk failed with code {rc}")
    try:
        nnzL = int(res.nnzL)
        L_rowptr = np.ctypeslib.as_array(res.L_rowptr, shape=(n + 1,)).copy()
        L_col = (np.ctypeslib.as_array(res.L_col, shape=(nnzL,)).copy() if nnzL
                 else np.zeros(0, np.int32))
        L_val = (np.ctypeslib.as_array(res.L_val, shape=(nnzL,)).copy() if nnzL
                 else np.zeros(0, np.float64))
        d_diag = np.ctypeslib.as_array(res.d_diag, shape=(n,)).copy()
        d_sub = np.ctypeslib.as_array(res.d_sub, shape=(n,)).copy()
        piv = np.ctypeslib.as_array(res.piv, shape=(n,)).copy()
        order = np.ctypeslib.as_array(res.order, shape=(n,)).copy()
        npert, n2 = int(res.n_perturbed), int(res.n_2x2)
    finally:
        lib.ildl_free(ctypes.byref(res))
    perm = q[order].astype(np.int32)
    return IldlFactors(n=n, perm=perm, L_rowptr=L_rowptr, L_col=L_col, L_val=L_val,
                       d_diag=d_diag, d_sub=d_sub, piv=piv, tau=float(tau),
                       n_perturbed=npert, n_2x2=n2)


def random_dd_factors(seed: int, taus):
    """The random dominant matrix of `seed` (`random_dd_symmetric`), its RCM
    ordering and its threshold ILDL-BK at each tau in `taus`: a module-level
    function, so that process pools can produce a set of matrices in
    parallel. Returns (seed, A, q, [factors])."""
    from .matrices import random_dd_symmetric
    from .ordering import rcm
    A = random_dd_symmetric(seed)
    q = rcm(A)
    return seed, A, q, [ildl_bk(A, q, t) for t in taus]
