"""Exact inverse of the shifted 2D Dirichlet Laplacian in closed form.

For A = T (x) I + I (x) T - sigma I on an N x N grid, with T = tridiag(-1, 2, -1)
of order N, the eigenvectors of T are the discrete sine vectors
    q_p(i) = sqrt(2 / (N + 1)) sin((i + 1)(p + 1) pi / (N + 1)),
with eigenvalues mu_p = 4 sin^2((p + 1) pi / (2 (N + 1))), so
    A^-1 = (Q (x) Q) diag(1 / (mu_p + mu_q - sigma)) (Q (x) Q).
Applying it to a grid vector X (X[y, x], x fastest as in the generators) is
Q ((Q X Q) / K) Q with K[y, x] = mu_y + mu_x - sigma, four dense N x N
products, and the diagonal of A^-1 is (Q o Q) (1 / K) (Q o Q)^T.

These are the reference quantities of the indefinite workload: the paper
computes the exact diagonal of A^-1 in advance with a direct solver (Section
2.6) and replaces A^-1 x in the inverse-error operator by a preconditioned
Krylov solve (Section 2.5); for this matrix both are available exactly.
"""
from __future__ import annotations

import numpy as np


class ShiftedLaplace2DExact:
    """Exact A^-1 products and diag(A^-1) for laplace2d(N, N, -sigma)."""

    def __init__(self, N: int, sigma: float):
        self.N = int(N)
        self.sigma = float(sigma)
        i = np.arange(1, N + 1)
        self.Q = np.sqrt(2.0 / (N + 1)) * np.sin(np.outer(i, i) * np.pi / (N + 1))
        self.mu = 4.0 * np.sin(i * np.pi / (2 * (N + 1))) ** 2
        K = self.mu[:, None] + self.mu[None, :] - self.sigma
        if np.min(np.abs(K)) == 0.0:
            raise ValueError("sigma is an eigenvalue: A is singular")
        self.Kinv = 1.0 / K

    @property
    def n(self) -> int:
        return self.N * self.N

    def solve(self, X: np.ndarray) -> np.ndarray:
        """A^-1 X for X of shape (n,) or (n, b), in the grid ordering."""
        N, Q = self.N, self.Q
        one = X.ndim == 1
        Xb = np.asarray(X, dtype=np.float64).reshape(N, N, -1).transpose(2, 0, 1)  # (b, y, x)
        Y = Q @ ((Q @ Xb @ Q) * self.Kinv) @ Q
        out = Y.transpose(1, 2, 0).reshape(N * N, -1)
        return out[:, 0] if one else out

    def inverse_diag(self) -> np.ndarray:
        """diag(A^-1) in the grid ordering."""
        Q2 = self.Q * self.Q
        return (Q2 @ self.Kinv @ Q2.T).ravel()

    def eigenvalues(self) -> np.ndarray:
        """All eigenvalues of A, sorted ascending."""
        return np.sort((self.mu[:, None] + self.mu[None, :] - self.sigma).ravel())
