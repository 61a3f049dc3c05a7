"""Pins of the fixed-pattern numeric factorization in the oracle (Section 2.1:
the incomplete factorization P^T A P ~ L D L^T, with its pattern and pivot
sequence taken as given). Checks: exact L D L^T at full fill; the defining
identity (L D L^T)_ij = Ah_ij on every kept entry and every D block on
arbitrary patterns; and agreement with both threshold ILDL-BK
implementations (the host C factorization and the dense one in the oracle)
when given the pattern and pivots they chose."""
import numpy as np
import pytest

from oracle import dense as od
from workloads import diffusion3d_7pt, ildl_bk, kkt_matrix, laplace2d, random_dd_symmetric, rcm


def _lpat(F):
    P = np.zeros((F.n, F.n), bool)
    for i in range(F.n):
        P[i, F.L_col[F.L_rowptr[i]:F.L_rowptr[i + 1]]] = True
    return P


def _ah(A, perm):
    A = A.toarray() if hasattr(A, "toarray") else np.asarray(A)
    return A[np.ix_(perm, perm)]


def _vals(L, F):
    rows = np.repeat(np.arange(F.n), np.diff(F.L_rowptr))
    return L[rows, F.L_col]


@pytest.mark.parametrize("case", ["kkt", "laplace2d"])
def test_full_fill_is_the_exact_ldlt(case):
    A = kkt_matrix(14, 6, 1) if case == "kkt" else laplace2d(9)
    F = ildl_bk(A, None if case == "kkt" else rcm(A), 0.0)
    if case == "kkt":
        assert (F.piv == 1).any()  # 2x2 blocks present
    Ah = _ah(A, F.perm)
    L, dd, ds = od.fixed_pattern_ldl(Ah, _lpat(F), F.piv)
    D = od.dense_D(dd, ds, F.piv)
    assert np.abs(L @ D @ L.T - Ah).max() <= 1e-12 * np.abs(Ah).max()


@pytest.mark.parametrize("seed", [0, 1, 2])
def test_kept_entries_satisfy_the_defining_identity(seed):
    rng = np.random.default_rng(seed)
    n = 40
    A = random_dd_symmetric(seed, n).toarray()
    piv = np.zeros(n, np.int8)
    for j in range(0, n - 1, 7):  # a few 2x2 blocks
        piv[j], piv[j + 1] = 1, 2
    P = np.tril(rng.random((n, n)) < 0.25, -1)
    for j in range(n - 1):  # both columns of a 2x2 block in every row that holds one
        if piv[j] == 1:
            P[j + 1, j] = False
            both = P[:, j] | P[:, j + 1]
            both[: j + 2] = False
            P[:, j] = P[:, j + 1] = both
    L, dd, ds = od.fixed_pattern_ldl(A, P, piv)
    D = od.dense_D(dd, ds, piv)
    R = L @ D @ L.T - A
    scale = np.abs(A).max()
    assert np.abs(R[P]).max() <= 1e-12 * scale
    assert np.abs(np.diag(R)).max() <= 1e-12 * scale
    blk = piv == 1
    assert np.abs(R[np.flatnonzero(blk) + 1, np.flatnonzero(blk)]).max() <= 1e-12 * scale
    assert not (L[np.tril(~P, -1)] != 0).any()
    # the identity fails off the pattern (entries were dropped), so it is a real constraint
    assert np.abs(R[np.tril(~P, -1) & (A != 0)]).max() > 1e-8 * scale


@pytest.mark.parametrize("case,tau", [("diffusion", 1e-2), ("diffusion", 1e-3), ("kkt", 1e-2),
                                      ("random", 5e-2)])
def test_matches_the_host_threshold_factor(case, tau):
    if case == "diffusion":
        A = diffusion3d_7pt(6, 1.0, 3)
        q = rcm(A)
    elif case == "kkt":
        A, q = kkt_matrix(20, 8, 2), None
    else:
        A = random_dd_symmetric(5, 150)
        q = rcm(A)
    F = ildl_bk(A, q, tau)
    assert F.n_perturbed == 0
    if case == "kkt":
        assert (F.piv == 1).any()
    L, dd, ds = od.fixed_pattern_ldl(_ah(A, F.perm), _lpat(F), F.piv)
    lv = _vals(L, F)
    assert np.abs(lv - F.L_val).max() <= 1e-10 * max(1.0, np.abs(F.L_val).max())
    assert np.abs(dd - F.d_diag).max() <= 1e-10 * np.abs(F.d_diag).max()
    two = F.piv == 1
    assert np.abs(ds[two] - F.d_sub[two]).max(initial=0.0) <= 1e-10 * np.abs(F.d_diag).max()


def test_matches_the_dense_threshold_factor():
    A = kkt_matrix(12, 5, 4).toarray()
    order, Lr, Lpat, dd_r, ds_r, piv = od.dense_ildl_bk(A, tau=3e-2)
    L, dd, ds = od.fixed_pattern_ldl(A[np.ix_(order, order)], Lpat, piv)
    assert np.abs(L - Lr).max() <= 1e-10 * np.abs(Lr).max()
    assert np.abs(dd - dd_r).max() <= 1e-10 * np.abs(dd_r).max()
    assert np.abs(ds - ds_r).max() <= 1e-10 * np.abs(dd_r).max()
