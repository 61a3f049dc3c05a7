"""Covariance-type workload (Section 3.6) and the trace output of the
covariance / uncertainty-quantification application (Section 3.5), on the CPU.

Pins: the generator against its defining formula evaluated by brute force
over all pairs of grid points, positive definiteness (the truncated power
kernel with beta >= 3/2 is positive definite in two dimensions), and the
oracle's trace sums against the closed-form trace of the inverse 1D Laplacian
and against the trace identity of an orthonormal rank-k term.
"""
import numpy as np
import pytest
import scipy.sparse as sp

from oracle import core as oc
from workloads import covariance_grid, ildl_bk, nested_dissection_grid, rcm


@pytest.mark.parametrize("N,alpha,beta", [(12, 3.0, 4.0), (9, 2.5, 2.0), (7, 1.0, 4.0)])
def test_covariance_grid_matches_definition(N, alpha, beta):
    A = covariance_grid(N, alpha, beta)
    n = N * N
    x = np.arange(n) % N
    y = np.arange(n) // N
    d = np.hypot(x[:, None] - x[None, :], y[:, None] - y[None, :])
    ref = np.where(d <= alpha, np.clip(1.0 - d / alpha, 0.0, None) ** beta, 0.0)
    D = A.toarray()
    np.testing.assert_array_equal(D, D.T)
    np.testing.assert_allclose(D, ref, rtol=1e-15, atol=0)
    assert np.linalg.eigvalsh(D).min() > 0


def test_covariance_grid_sizes():
    import os
    golden = os.path.join(os.path.dirname(__file__), "golden", "covariance_sizes.txt")
    for line in open(golden):
        if line.strip() and not line.startswith("#"):
            N, n = (int(x) for x in line.split())
            assert covariance_grid(N, 3.0, 4.0).shape == (n, n)
    A = covariance_grid(200)
    assert A.shape == (40000, 40000)
    counts = np.diff(A.indptr)
    # interior points: the 25 grid points at distance < 3 (distance exactly 3 gives 0)
    assert counts.max() == 25 and np.median(counts) == 25
    assert A.indptr.dtype == np.int64 and A.indices.dtype == np.int32


def test_trace_sums_closed_form_and_rank_k_identity():
    # tr(A^-1) of tridiag(-1, 2, -1) of order n is n (n + 2) / 6
    n = 30
    A = sp.diags([-np.ones(n - 1), 2 * np.ones(n), -np.ones(n - 1)], [-1, 0, 1]).tocsr()
    F = ildl_bk(A, None, 0.0)
    S = oc.pattern(F)
    Z = oc.selinv(F, S)
    tr, a1 = oc.trace_sums(S, Z)
    assert tr == pytest.approx(n * (n + 2) / 6, rel=1e-13)
    assert a1 == pytest.approx(tr, rel=1e-15)  # SPD: positive diagonal
    # an orthonormal rank-k term adds sum(lambda) to the trace
    rng = np.random.default_rng(0)
    V, _ = np.linalg.qr(rng.standard_normal((n, 4)))
    lam = np.array([0.5, -0.25, 2.0, 0.0])
    tk, _ = oc.trace_sums(S, Z, V, lam)
    assert tk == pytest.approx(tr + lam.sum(), rel=1e-13)


def test_selinv_on_covariance_tau0_is_exact_inverse():
    """At tau = 0 the pattern is closed, so SelInv gives A^-1 on S (Section
    2.1) on the covariance workload too; its trace is tr(A^-1)."""
    N = 10
    A = covariance_grid(N)
    F = ildl_bk(A, nested_dissection_grid((N, N)), 0.0)
    S = oc.pattern(F)
    Z = oc.selinv(F, S)
    Ainv = np.linalg.inv(A.toarray())[np.ix_(F.perm, F.perm)]
    ref = Ainv[S.rows(), S.col]
    np.testing.assert_allclose(Z, ref, rtol=0, atol=1e-12 * np.abs(Ainv).max())
    tr, _ = oc.trace_sums(S, Z)
    assert tr == pytest.approx(np.trace(Ainv), rel=1e-12)
