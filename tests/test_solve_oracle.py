"""Pins of the oracle's operator applications of the eigen step (Section 2.5):
the preconditioner solve satisfies L D L^T y = x (with 2x2 pivots), and the
product with X on S equals a dense product."""
import numpy as np
import pytest

from oracle import core as oc
from oracle import dense as od
from workloads import covariance_grid, ildl_bk, kkt_matrix, nested_multicolor_grid


@pytest.mark.parametrize("case", ["cov", "kkt"])
def test_ldl_solve_inverts_the_factor(case):
    if case == "cov":
        F = ildl_bk(covariance_grid(12), nested_multicolor_grid((12, 12)), 1e-3)
    else:
        F = ildl_bk(kkt_matrix(30, 20, 4), None, 1e-2)
        assert F.n_2x2 > 0
    L = od.dense_L(F)
    D = od.dense_D(F.d_diag, F.d_sub, F.piv)
    x = np.random.default_rng(1).standard_normal(F.n)
    y = oc.ldl_solve(F, x)
    r = L @ (D @ (L.T @ y)) - x
    assert np.abs(r).max() <= 1e-12 * np.abs(x).max() * max(1.0, np.abs(L).max() ** 2 * np.abs(D).max())
    np.testing.assert_allclose(y, np.linalg.solve(L @ D @ L.T, x), rtol=1e-9, atol=1e-12 * np.abs(y).max())


def test_spmv_dense():
    F = ildl_bk(covariance_grid(9), nested_multicolor_grid((9, 9)), 1e-3)
    S = oc.pattern(F)
    X = np.random.default_rng(2).standard_normal(S.nnz)
    x = np.random.default_rng(3).standard_normal(F.n)
    np.testing.assert_allclose(oc.spmv(S, X, x), S.to_csr(X).toarray() @ x, rtol=1e-13, atol=1e-13)


def test_za_diag_is_one_for_the_exact_inverse_on_a_closed_pattern():
    # tau = 0: pattern(Ah) is inside S and Z = A^-1 on S, so (Z Ah)_ii = 1 (Section 2.1)
    A = covariance_grid(10)
    F = ildl_bk(A, nested_multicolor_grid((10, 10)), 0.0)
    S = oc.pattern(F)
    Z = oc.selinv(F, S)
    d = oc.za_diag(S, Z, oc.permuted(A, F.perm))
    np.testing.assert_allclose(d, 1.0, rtol=0, atol=1e-12)
    # NInv with drops on an incomplete pattern: equal to a dense product's diagonal, not all ones
    F2 = ildl_bk(A, nested_multicolor_grid((10, 10)), 1e-2)
    S2 = oc.pattern(F2)
    N2 = oc.ninv(F2, S2, 3, 0.1)
    Ah = oc.permuted(A, F2.perm).toarray()
    d2 = oc.za_diag(S2, N2, Ah)
    np.testing.assert_allclose(d2, np.diag(S2.to_csr(N2).toarray() @ Ah), rtol=1e-13)
    assert np.abs(d2 - 1).max() > 1e-6
