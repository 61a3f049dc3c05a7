"""Pins of the oracle's eigen step (Section 2.5, Algorithm 1): the
eigenpairs of E = Ah^-1 - X against closed forms: a diagonal A and X (E
diagonal, eigenvalues 1/a_i - x_i, signs mixed), the 1D Laplacian
(eigenvalues of its inverse in closed form, eigenvectors sine vectors, moved
by the permutation), and the trace and Frobenius identities of E when X
holds A^-1's own values on S."""
import numpy as np
import scipy.sparse as sp

from oracle import core as oc


def _diag_pattern(n):
    return oc.Pattern(n, np.arange(n + 1, dtype=np.int64), np.arange(n, dtype=np.int32))


def _tridiag_pattern(n):
    rows, cols = [], []
    for i in range(n):
        for j in (i - 1, i, i + 1):
            if 0 <= j < n:
                rows.append(i)
                cols.append(j)
    rp = np.zeros(n + 1, dtype=np.int64)
    np.add.at(rp, np.array(rows) + 1, 1)
    return oc.Pattern(n, np.cumsum(rp), np.array(cols, dtype=np.int32))


def test_oracle_eigenpairs_diagonal_closed_form():
    n = 9
    a = np.array([1.0, 2.0, 4.0, 0.5, 8.0, 3.0, 1.5, 0.25, 5.0])
    x = np.array([0.5, 0.1, 0.25, 4.0, 0.0, 0.3, 0.2, 3.4, -0.1])
    lam_exact = 1.0 / a - x                  # E = diag(1/a - x)
    lam, V = oc.error_eigenpairs(sp.diags(a), _diag_pattern(n), x, 4)
    order = np.argsort(-np.abs(lam_exact), kind="stable")[:4]
    np.testing.assert_allclose(lam, lam_exact[order], rtol=1e-14)
    assert lam[0] < 0  # the largest |lambda| is the negative 1/0.5 - 4 = -2
    for t in range(4):  # eigenvectors are +- unit vectors
        assert abs(abs(V[order[t], t]) - 1.0) < 1e-14


def test_oracle_eigenpairs_laplacian_with_permutation():
    n = 30
    A = sp.diags([-np.ones(n - 1), 2 * np.ones(n), -np.ones(n - 1)], [-1, 0, 1]).tocsr()
    perm = np.random.default_rng(3).permutation(n).astype(np.int32)
    Ah = oc.permuted(A, perm)
    S = oc.Pattern(n, Ah.indptr.astype(np.int64), Ah.indices.astype(np.int32))  # X = 0 on Ah's pattern
    lam, V = oc.error_eigenpairs(Ah, S, np.zeros(S.nnz), 3)
    j = np.arange(1, 4)
    np.testing.assert_allclose(lam, 1.0 / (2.0 - 2.0 * np.cos(j * np.pi / (n + 1))), rtol=1e-12)
    i = np.arange(1, n + 1)
    for t in range(3):
        v = np.sin(i * (t + 1) * np.pi / (n + 1))
        v /= np.linalg.norm(v)
        assert abs(abs(v[perm] @ V[:, t]) - 1.0) < 1e-12  # Ah's eigenvector is v permuted


def test_oracle_eigenpairs_trace_and_frobenius_identities():
    n = 25
    rng = np.random.default_rng(4)
    off = -rng.uniform(0.1, 1.0, n - 1)
    A = sp.diags([off, 3.0 + rng.uniform(0, 1, n), off], [-1, 0, 1]).tocsr()
    S = _tridiag_pattern(n)
    Ainv = np.linalg.inv(A.toarray())
    X = S.gather(Ainv)             # A^-1's own values on S
    lam, _ = oc.error_eigenpairs(A, S, X, n)
    # E = A^-1 with the entries on S set to 0: zero diagonal, and its
    # Frobenius norm is that of A^-1 off S
    assert abs(lam.sum()) < 1e-13 * np.abs(lam).max()
    mask = np.ones((n, n), dtype=bool)
    mask[S.rows(), S.col] = False
    np.testing.assert_allclose((lam ** 2).sum(), (Ainv[mask] ** 2).sum(), rtol=1e-12)
