"""Spectral correction of an approximate inverse (Section 2.5, Algorithm 1).

The dominant eigenpairs of the inverse-error operator E = A^-1 - X are found
matrix-free, either on the device by the library's thick-restart Lanczos
iteration (Solver.eigs_error: A^-1 x by PCG or SQMR preconditioned with the
incomplete factor, the paper's choice) or here on the host (ARPACK's
implicitly restarted Lanczos through scipy) with A^-1 x supplied by the
caller, where any solver more accurate than X serves.
Everything that touches S runs in libasi's kernels: the rank-k update on S
(asi_lowrank), the diagonals (asi_diag) and the err_1 sums of the
acceptance test (asi_diag_err1).
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np


def inverse_error_eigenpairs(apply_inv, X_csr, k: int, tol: float = 1e-8, seed: int = 0,
                             ncv: int | None = None, maxiter: int | None = None, apply_E=None):
    """k eigenpairs of E = A^-1 - X of largest |lambda| (Section 2.5).

    apply_inv(x) returns A^-1 x (float64, same ordering as X_csr); or
    apply_E(x) returns E x directly (then apply_inv and X_csr are not used
    for products, X_csr only gives n). Returns (lam [k], V [n, k]
    orthonormal columns, ordered by decreasing |lam|, relative residuals
    ||E v - lam v|| / |lam|, number of applications of E).
    """
    from scipy.sparse.linalg import LinearOperator, eigsh
    n = X_csr.shape[0]
    count = [0]

    def mv(x):
        count[0] += 1
        x = np.asarray(x, dtype=np.float64).ravel()
        if apply_E is not None:
            return apply_E(x)
        return apply_inv(x) - X_csr @ x

    op = LinearOperator((n, n), matvec=mv, dtype=np.float64)
    v0 = np.random.default_rng(seed).standard_normal(n)
    lam, V = eigsh(op, k=k, which="LM", v0=v0, tol=tol, ncv=ncv, maxiter=maxiter)
    order = np.argsort(-np.abs(lam), kind="stable")
    lam = lam[order]
    V = np.ascontiguousarray(V[:, order])
    res = np.array([np.linalg.norm(mv(V[:, m]) - lam[m] * V[:, m]) / abs(lam[m]) for m in range(k)])
    return lam, V, res, count[0]


def greedy_accept(lam, evaluate):
    """Acceptance test of Algorithm 1, per mode: candidates in order of
    decreasing |lam| (ties by index); a mode is kept only if the error with it
    added to the modes kept so far is strictly smaller (Section 3, diagonal
    safeguard). evaluate(weights) returns (||d - d^k||_1, ||d||_1) for the
    correction sum_m weights_m v_m v_m^T. Returns (kept indices, weights of
    the kept modes (0 elsewhere), err_1 before, err_1 after)."""
    k = len(lam)
    w = np.zeros(k)
    base, dn = evaluate(w)
    best = base
    kept = []
    for m in sorted(range(k), key=lambda m: (-abs(lam[m]), m)):
        trial = w.copy()
        trial[m] = lam[m]
        e, _ = evaluate(trial)
        if e < best:
            kept.append(m)
            w, best = trial, e
    return kept, w, base / dn, best / dn


@dataclass
class Correction:
    kept: list
    weights: np.ndarray   # lam_m for kept modes, 0 for the others
    err1_before: float
    err1_after: float


def accept_on_device(solver, d_ref, d_hat, V_dev, lam) -> Correction:
    """Run the acceptance test with the library's err_1 reduction.

    d_ref, d_hat: device float64 [n] (factor ordering); V_dev: device [n, k];
    lam: host float64 [k]."""
    import torch
    sums = torch.empty(2, dtype=torch.float64, device=solver.device)

    def evaluate(w):
        wd = torch.as_tensor(np.asarray(w, dtype=np.float64), device=solver.device)
        solver.diag_err1(d_ref, d_hat, V_dev, wd, sums=sums)
        solver.sync()
        a, b = sums.tolist()
        return a, b

    kept, w, e0, e1 = greedy_accept(np.asarray(lam, dtype=np.float64), evaluate)
    return Correction(kept=kept, weights=w, err1_before=e0, err1_after=e1)
