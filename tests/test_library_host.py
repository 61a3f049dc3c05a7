"""Host-side checks of libasi that need no GPU: the library loads, exports every
symbol include/asi.h declares, and its host-only analysis validates inputs
and reports the pattern size and dependency levels."""
import ctypes
import os
import re

import numpy as np
import pytest

from oracle import core as oc
from paper_2609_11363_amd import asi
from workloads import (diffusion3d_7pt, ildl_bk, kkt_matrix, laplace2d, nested_multicolor_grid,
                       random_dd_symmetric, rcm)

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared_symbols():
    txt = open(os.path.join(ROOT, "include", "asi.h")).read()
    return sorted(set(re.findall(r"\b(asi_[a-z0-9_]+)\s*\(", txt)))


def test_exports_every_declared_symbol():
    lib = asi.load_library()
    names = _declared_symbols()
    assert set(names) == set(asi.EXPORTS)
    for name in names:
        assert hasattr(lib, name), name


class HostHandle:
    def __init__(self):
        self.lib = asi.load_library()
        self.h = ctypes.c_void_p()
        assert self.lib.asi_create(ctypes.byref(self.h), -1, None) == 0

    def analyze(self, n, rowptr, col, piv):
        rowptr = np.ascontiguousarray(rowptr, np.int64)
        col = np.ascontiguousarray(col if len(col) else np.zeros(1), np.int32)
        piv = np.ascontiguousarray(piv, np.int8)
        nnz = ctypes.c_int64()
        ws = ctypes.c_size_t()
        rc = self.lib.asi_analyze(self.h, n, rowptr.ctypes.data, col.ctypes.data, piv.ctypes.data,
                                  ctypes.byref(nnz), ctypes.byref(ws))
        return rc, nnz.value, ws.value

    def info(self):
        inf = asi.Info()
        assert self.lib.asi_get_info(self.h, ctypes.byref(inf)) == 0
        return inf.as_dict()

    def error(self):
        return self.lib.asi_last_error(self.h).decode()

    def __del__(self):
        self.lib.asi_destroy(self.h)


@pytest.mark.parametrize("case", ["lap", "kkt", "rand", "diff"])
def test_host_analysis_matches_oracle_pattern_size(case):
    if case == "lap":
        A = laplace2d(20, 20, 0.01)
        F = ildl_bk(A, rcm(A), 1e-2)
    elif case == "kkt":
        F = ildl_bk(kkt_matrix(30, 12, 1), None, 0.05)
        assert F.n_2x2 > 0
    elif case == "rand":
        A = random_dd_symmetric(2, n=500)
        F = ildl_bk(A, rcm(A), 1e-2)
    else:
        A = diffusion3d_7pt(12, 1.0, 2)
        F = ildl_bk(A, nested_multicolor_grid((12, 12, 12)), 1e-3)
    h = HostHandle()
    rc, nnz, ws = h.analyze(F.n, F.L_rowptr, F.L_col, F.piv)
    assert rc == 0, h.error()
    S = oc.pattern(F)
    assert nnz == S.nnz == F.nnzS
    inf = h.info()
    assert inf["n"] == F.n and inf["nnz_L"] == F.nnzL
    assert inf["n_blocks"] == F.n - int((F.piv == 1).sum())
    assert 1 <= inf["n_levels"] <= inf["n_blocks"]
    assert inf["gather_hits"] <= inf["gather_pairs"]
    assert ws >= inf["workspace_min"]


def test_levels_of_a_chain_and_of_a_diagonal():
    # tridiagonal L: every column depends on the next -> n levels
    n = 50
    rowptr = np.concatenate([[0, 0], np.arange(1, n)]).astype(np.int64)
    col = np.arange(0, n - 1, dtype=np.int32)
    h = HostHandle()
    assert h.analyze(n, rowptr, col, np.zeros(n, np.int8))[0] == 0
    assert h.info()["n_levels"] == n
    # empty L: one level, |S| = n
    rc, nnz, _ = h.analyze(n, np.zeros(n + 1, np.int64), np.zeros(0, np.int32), np.zeros(n, np.int8))
    assert rc == 0 and nnz == n and h.info()["n_levels"] == 1


def test_host_analysis_rejects_bad_patterns():
    h = HostHandle()
    n = 4
    piv = np.zeros(n, np.int8)
    # upper entry
    rc, _, _ = h.analyze(n, [0, 1, 1, 1, 1], [2], piv)
    assert rc == 2 and "strictly lower" in h.error()
    # unsorted row
    rc, _, _ = h.analyze(n, [0, 0, 0, 0, 2], [2, 1], piv)
    assert rc == 2
    # duplicate
    rc, _, _ = h.analyze(n, [0, 0, 0, 0, 2], [1, 1], piv)
    assert rc == 2
    # piv 1 not followed by 2
    rc, _, _ = h.analyze(n, [0, 0, 0, 0, 0], [], np.array([1, 0, 0, 0], np.int8))
    assert rc == 2
    # (j+1, j) stored inside a 2x2 block
    rc, _, _ = h.analyze(n, [0, 0, 1, 1, 1], [0], np.array([1, 2, 0, 0], np.int8))
    assert rc == 2 and "2x2" in h.error()
    # bad n
    rc, _, _ = h.analyze(0, [0], [], np.zeros(1, np.int8))
    assert rc == 1


def test_host_handle_has_no_device_calls():
    h = HostHandle()
    assert h.analyze(3, [0, 0, 1, 2], [0, 1], np.zeros(3, np.int8))[0] == 0
    rc = h.lib.asi_selinv(h.h, None, None, None, 0, None)
    assert rc == 5  # ASI_E_STATE: no workspace on a host-only handle
    rc = h.lib.asi_set_workspace(h.h, ctypes.c_void_p(256), 1 << 20)
    assert rc == 5


def test_check_matrix_accepts_valid_and_rejects_invalid_input():
    import scipy.sparse as sp
    from workloads import covariance_grid
    h = HostHandle()
    A = covariance_grid(6)
    n = A.shape[0]
    perm = np.random.default_rng(0).permutation(n).astype(np.int32)

    def check(M, p=perm, tol=0.0, nn=None):
        ip = np.ascontiguousarray(M.indptr, np.int64)
        ic = np.ascontiguousarray(M.indices, np.int32)
        iv = np.ascontiguousarray(M.data, np.float64)
        pp = None if p is None else np.ascontiguousarray(p, np.int32)
        return h.lib.asi_check_matrix(h.h, M.shape[0] if nn is None else nn, ip.ctypes.data, ic.ctypes.data,
                                      iv.ctypes.data, None if pp is None else pp.ctypes.data, ctypes.c_double(tol))

    assert check(A) == 0 and check(A, None) == 0
    bad = perm.copy()
    bad[1] = bad[0]
    assert check(A, bad) == 2 and "permutation" in h.error()
    B = A.tolil()
    B[0, 5] = 0.125  # pattern no longer symmetric
    assert check(sp.csr_matrix(B)) == 2 and "structurally" in h.error()
    C = A.copy()
    C.data = C.data.copy()
    q = C.indptr[1] - 1  # last entry of row 0, an off-diagonal
    C.data[q] *= 1 + 1e-9
    assert check(C) == 2 and "values" in h.error()
    assert check(C, tol=1e-8) == 0
    D = A.copy()
    D.indices = D.indices.copy()
    D.indices[[0, 1]] = D.indices[[1, 0]]  # unsorted row
    assert check(D) == 2 and "sorted" in h.error()
    E = A.copy()
    E.data = E.data.copy()
    E.data[3] = np.nan
    assert check(E) == 4  # ASI_E_NONFINITE


def test_sweep_plan_reaches_every_variant():
    """asi_sweep_plan on the layered factor (host-only handle): every level
    launch variant occurs, and the counts add up to one small-block launch per
    level with small blocks plus one large-block launch per level with large
    blocks."""
    from workloads.layered import layered_factor
    F = layered_factor(seed=1)
    h = HostHandle()
    rc, nnz, _ = h.analyze(F.n, F.L_rowptr, F.L_col, F.piv)
    assert rc == 0, h.error()
    counts = np.zeros(7, np.int64)
    assert h.lib.asi_sweep_plan(h.h, counts.ctypes.data) == 0
    plan = dict(zip(asi.SWEEP_VARIANTS, counts.tolist()))
    assert all(v > 0 for v in plan.values()), plan
    # levels computed by the oracle's definition: per level, whether it has
    # blocks with |R_J| <= 128 and with |R_J| > 128
    S = oc.pattern(F)
    lev = oc.dag_levels(F, S)
    firsts = np.nonzero(F.piv != 2)[0]
    last = np.where(F.piv[firsts] == 1, firsts + 1, firsts)
    diagpos = S.diag_positions()
    c = S.rowptr[last + 1] - diagpos[last] - 1
    small = {int(lev[j]) for j, cj in zip(firsts, c) if cj <= 128}
    big = {int(lev[j]) for j, cj in zip(firsts, c) if cj > 128}
    assert sum(plan.values()) == len(small) + len(big)
    assert plan["big256"] + plan["big1024"] == len(big)
    assert h.info()["n_levels"] == int(lev.max()) + 1
