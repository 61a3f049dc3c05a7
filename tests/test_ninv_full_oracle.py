"""Pins of the oracle's NInv and Mix on their own pattern (Section 2.2, the
product drop; Section 2.3, Mix keeps NInv's structure): dense products of
the dense Neumann series with the drop applied entry by entry, the exact
inverse when the series is complete, agreement with NInv on S where both are
defined, and the Mix selection by brute force."""
import numpy as np
import pytest

from oracle import core as oc
from oracle import dense as od
from workloads import ildl_bk, kkt_matrix, laplace2d, random_dd_symmetric, rcm


def _dense_lower(n, full):
    rp, c, v = full
    M = np.zeros((n, n))
    r = np.repeat(np.arange(n), np.diff(rp))
    M[r, c] = v
    return M, r, c


@pytest.mark.parametrize("delta,drop", [(0.1, 0.1), (1e-2, 1e-2), (1e-2, 0.0)])
def test_ninv_full_matches_dense_product_with_drop(delta, drop):
    A = random_dd_symmetric(5, n=60, per_row=3, dominance=0.7)
    F = ildl_bk(A, rcm(A), 1e-2)
    L = od.dense_L(F)
    Li = od.neumann_linv(L, 3, delta)
    D = od.dense_D(F.d_diag, F.d_sub, F.piv)
    Nd = Li.T @ np.linalg.inv(D) @ Li
    # structure: pairs of columns of L^inv meeting a common D block
    Bs = (Li != 0).astype(float)
    Cs = (D != 0).astype(float)
    struct = np.tril((Bs.T @ Cs @ Bs) > 0)
    d = np.diag(Nd)
    keep = struct & ((np.abs(Nd) >= drop * np.sqrt(np.abs(np.outer(d, d)))) | np.eye(F.n, dtype=bool))
    full = oc.ninv_full(F, 3, delta, drop)
    M, r, c = _dense_lower(F.n, full)
    got = np.zeros((F.n, F.n), dtype=bool)
    got[r, c] = True
    np.testing.assert_array_equal(got, keep)
    np.testing.assert_allclose(M[keep], Nd[keep], rtol=1e-12, atol=1e-14 * np.abs(Nd).max())
    for i in range(F.n):  # columns sorted within rows, lower triangle only
        cols = full[1][full[0][i]:full[0][i + 1]]
        assert np.all(np.diff(cols) > 0) and (len(cols) == 0 or cols[-1] <= i)


def test_ninv_full_complete_series_is_inverse():
    # nilpotent E: p >= n - 1 and no drops give N = (L D L^T)^-1 (2x2 pivots included)
    K = kkt_matrix(10, 5, 3)
    F = ildl_bk(K, None, 0.0)
    full = oc.ninv_full(F, F.n, 0.0, 0.0)
    M, r, c = _dense_lower(F.n, full)
    L = od.dense_L(F)
    D = od.dense_D(F.d_diag, F.d_sub, F.piv)
    inv = np.linalg.inv(L @ D @ L.T)
    np.testing.assert_allclose(M[r, c], inv[r, c], rtol=1e-9, atol=1e-12 * np.abs(inv).max())
    outside = np.ones((F.n, F.n), dtype=bool)
    outside[r, c] = False
    assert np.abs(np.tril(inv)[outside]).max() <= 1e-12 * np.abs(inv).max()


def test_ninv_full_agrees_with_ninv_on_s():
    A = laplace2d(14, 14, 0.05)
    F = ildl_bk(A, rcm(A), 1e-2)
    S = oc.pattern(F)
    Ns = oc.ninv(F, S, 3, 0.1)
    full = oc.ninv_full(F, 3, 0.1, 0.0)
    M, r, c = _dense_lower(F.n, full)
    present = np.zeros((F.n, F.n), dtype=bool)
    present[r, c] = True
    sr, sc = S.rows(), S.col.astype(np.int64)
    low = sc <= sr
    inside = present[sr[low], sc[low]]
    np.testing.assert_allclose(M[sr[low], sc[low]][inside], Ns[low][inside], rtol=1e-12, atol=1e-15)
    assert np.all(Ns[low][~inside] == 0.0)  # S entries NInv does not reach are exact zeros


@pytest.mark.parametrize("eps", [0.0, 1e-2, 2.0])
def test_mix_full_brute_force(eps):
    A = laplace2d(9, 9, 0.1)
    F = ildl_bk(A, rcm(A), 3e-2)
    S = oc.pattern(F)
    Z = oc.selinv(F, S)
    full = oc.ninv_full(F, 3, 0.1, 0.1)
    out = oc.mix_full(S, Z, full, eps)
    Nd, _, _ = _dense_lower(F.n, full)
    npat = np.zeros((F.n, F.n), dtype=bool)
    npat[np.repeat(np.arange(F.n), np.diff(full[0])), full[1]] = True
    Zd = S.to_csr(Z).toarray()
    zd = np.diag(Zd)
    spat = S.to_csr(np.ones(S.nnz)).toarray() > 0
    sel = np.tril(spat & (np.abs(Zd) > eps * np.sqrt(np.abs(np.outer(zd, zd)))))
    ref = np.where(sel, Zd, Nd)
    Md, r, c = _dense_lower(F.n, out)
    got = np.zeros((F.n, F.n), dtype=bool)
    got[r, c] = True
    np.testing.assert_array_equal(got, npat | sel)
    np.testing.assert_array_equal(Md, np.where(npat | sel, ref, 0.0))
    if eps >= 1.0:  # S_eps is empty: Mix is NInv
        np.testing.assert_array_equal(out[2], full[2])
