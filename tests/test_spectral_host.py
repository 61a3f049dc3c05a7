"""Host side of the spectral correction (Section 2.5, Algorithm 1, Section 2.6).

Pins: the closed-form shifted-Laplacian inverse against a dense inverse, the
oracle's corrected diagonal and err_1 sums against hand-built cases, the
per-mode acceptance on a case worked out by hand, the package's acceptance
loop against the oracle's, and the host eigen step against a dense
eigendecomposition of A^-1 - X.
"""
import numpy as np
import pytest

from oracle import core as oc
from workloads import ShiftedLaplace2DExact, shifted_laplace2d_indefinite
from workloads.matrices import laplace2d_eigenvalues as lap_eigs


@pytest.mark.parametrize("N,neg", [(6, 3), (12, 4)])
def test_exact_inverse_matches_dense(N, neg):
    A, sigma = shifted_laplace2d_indefinite(N, neg)
    ex = ShiftedLaplace2DExact(N, sigma)
    Ainv = np.linalg.inv(A.toarray())
    rng = np.random.default_rng(N)
    X = rng.standard_normal((N * N, 3))
    np.testing.assert_allclose(ex.solve(X), Ainv @ X, rtol=0, atol=1e-10 * np.abs(Ainv).max())
    np.testing.assert_allclose(ex.solve(X[:, 1]), Ainv @ X[:, 1], rtol=0, atol=1e-10 * np.abs(Ainv).max())
    np.testing.assert_allclose(ex.inverse_diag(), np.diag(Ainv), rtol=1e-10)
    ev = np.linalg.eigvalsh(A.toarray())
    np.testing.assert_allclose(ex.eigenvalues(), ev, rtol=0, atol=1e-12)
    assert int((ev < 0).sum()) == neg
    np.testing.assert_allclose(ex.eigenvalues() + sigma, lap_eigs(N), rtol=0, atol=1e-12)


def test_corrected_diag_and_err1_sums():
    rng = np.random.default_rng(0)
    n, k = 50, 5
    V = rng.standard_normal((n, k))
    lam = rng.standard_normal(k)
    d = rng.standard_normal(n) + 3.0
    # a base diagonal that the k modes correct exactly
    dhat = d - (V * V) @ lam
    e, dn = oc.err1_sums(d, dhat, V, lam)
    assert e <= 1e-13 * dn
    assert dn == pytest.approx(np.abs(d).sum())
    e0, _ = oc.err1_sums(d, dhat)
    assert e0 / dn == pytest.approx(oc.err1(d, dhat))
    # one mode by hand: d^1_i = dhat_i + lam_0 V_i0^2
    np.testing.assert_allclose(oc.corrected_diag(dhat, V[:, :1], lam[:1]), dhat + lam[0] * V[:, 0] ** 2)


def test_accept_modes_worked_example():
    # d = 0; dhat = (1, 1); modes e_1 (lam -1), e_1 + e_2 scaled (lam 5), e_2 (lam -0.5)
    d = np.zeros(2)
    dhat = np.ones(2)
    V = np.array([[1.0, np.sqrt(0.5), 0.0], [0.0, np.sqrt(0.5), 1.0]])
    lam = np.array([-1.0, 5.0, -0.5])
    kept, before, after = oc.accept_modes(d + 1.0, dhat, V, lam)
    # reference diagonal (1, 1) equals dhat: nothing can improve it
    assert kept == [] and before == 0.0 and after == 0.0
    kept, before, after = oc.accept_modes(np.array([0.0, 0.5]), dhat, V, lam)
    # order by |lam|: mode 1 (5: error grows, rejected), mode 0 (-1: |0-0| + |0.5-1| = 0.5 < 1.5,
    # kept), mode 2 (-0.5: second entry becomes 0.5, error 0, kept)
    assert kept == [0, 2]
    assert before == pytest.approx(1.5 / 0.5)
    assert after == pytest.approx(0.0)


def test_package_acceptance_loop_matches_oracle():
    from paper_2609_11363_amd.spectral import greedy_accept
    rng = np.random.default_rng(3)
    for trial in range(20):
        n, k = 40, 8
        V = rng.standard_normal((n, k)) * 0.3
        lam = rng.standard_normal(k)
        d = rng.standard_normal(n)
        dhat = d + rng.standard_normal(n) * 0.5

        def evaluate(w):
            return oc.err1_sums(d, dhat, V, w)

        kept, w, e0, e1 = greedy_accept(lam, evaluate)
        ko, o0, o1 = oc.accept_modes(d, dhat, V, lam)
        assert kept == ko
        assert e0 == pytest.approx(o0) and e1 == pytest.approx(o1)
        assert np.all(w[kept] == lam[kept]) and np.count_nonzero(w) == len(kept)


def test_inverse_error_eigenpairs_match_dense():
    from paper_2609_11363_amd.spectral import inverse_error_eigenpairs
    import scipy.sparse as sp
    N = 10
    A, sigma = shifted_laplace2d_indefinite(N, 3)
    ex = ShiftedLaplace2DExact(N, sigma)
    # a diagonal approximate inverse with random scales (they split the
    # degenerate eigenvalues of the grid, so the eigenvectors are unique)
    Ad = A.toarray()
    r = np.random.default_rng(2).uniform(0.8, 1.2, N * N)
    X = sp.csr_matrix(np.diag(r / np.diag(Ad)))
    E = np.linalg.inv(Ad) - X.toarray()
    ev, W = np.linalg.eigh(E)
    order = np.argsort(-np.abs(ev))
    k = 5
    lam, V, res, napp = inverse_error_eigenpairs(ex.solve, X, k, tol=1e-12, seed=1)
    np.testing.assert_allclose(lam, ev[order[:k]], rtol=1e-9)
    for m in range(k):
        w = W[:, order[m]]
        assert abs(abs(w @ V[:, m]) - 1.0) <= 1e-8
    assert np.all(res <= 1e-8) and napp > 0
