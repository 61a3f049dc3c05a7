"""Pins of the learned-correction reference (oracle/mlp.py): bfloat16 rounding
against torch's conversion, gradients against central finite differences,
Adam's first step, the zero-last-layer identity and the features against a
per-entry brute force."""
import numpy as np
import pytest
import torch

from oracle import core as oc
from oracle import mlp as om
from workloads import ildl_bk, laplace2d, rcm


def test_bf16_rounding_matches_torch():
    rng = np.random.default_rng(0)
    x = np.concatenate([(rng.standard_normal(10000) * 10.0 ** rng.integers(-5, 5, 10000)).astype(np.float32),
                        np.array([1.0, -1.0, 0.0, 1 + 2 ** -8, 1 + 3 * 2 ** -9], np.float32)])
    ref = torch.from_numpy(x).to(torch.bfloat16).to(torch.float32).numpy()
    np.testing.assert_array_equal(om.bf16(x), ref)


def test_gradients_match_finite_differences():
    rng = np.random.default_rng(1)
    theta = om.init_params(3).astype(np.float64)
    X = rng.standard_normal((40, om.NF))
    dy = rng.standard_normal(40)
    g = om.backward_exact(theta, X, dy)
    h = 1e-6
    idx = rng.choice(om.NPARAMS, 60, replace=False)
    for i in idx:
        tp, tm = theta.copy(), theta.copy()
        tp[i] += h
        tm[i] -= h
        fd = (dy @ om.forward_exact(tp, X) - dy @ om.forward_exact(tm, X)) / (2 * h)
        assert abs(fd - g[i]) <= 1e-6 * max(1.0, abs(fd)), (i, fd, g[i])


def test_quantized_backward_close_to_exact():
    rng = np.random.default_rng(2)
    theta = om.init_params(4)
    X = om.bf16(rng.standard_normal((256, om.NF)).astype(np.float32))
    dy = rng.standard_normal(256)
    gq = om.backward(theta, X, dy)
    P = om.unpack(theta)
    Pr = {k: (om.bf16(v) if k in ("W1", "W2", "w3") else v) for k, v in P.items()}
    ge = om.backward_exact(om.pack(Pr), X.astype(np.float64), dy)
    assert np.linalg.norm(gq - ge) <= 2e-2 * np.linalg.norm(ge)


def test_adam_first_step_is_signed_lr():
    rng = np.random.default_rng(3)
    theta = rng.standard_normal(100)
    g = rng.standard_normal(100)
    t1, m, v = om.adam(theta, np.zeros(100), np.zeros(100), g, 1, lr=1e-3, eps=0.0)
    np.testing.assert_allclose(t1, theta - 1e-3 * np.sign(g), rtol=0, atol=1e-15)


def test_zero_last_layer_is_identity():
    theta = om.init_params(5, zero_last=True)
    X = om.bf16(np.random.default_rng(6).standard_normal((50, om.NF)).astype(np.float32))
    y = om.forward(theta, X)
    assert np.all(y == 0.0)


def test_features_match_per_entry_brute_force():
    A = laplace2d(10, 10, 0.05)
    F = ildl_bk(A, rcm(A), 5e-2)
    S = oc.pattern(F)
    Z = oc.selinv(F, S)
    N = oc.ninv(F, S, 3, 0.1)
    eps = 1e-2
    M = oc.mix(S, Z, N, eps)
    level = np.zeros(F.n, np.int64)
    ucount = np.zeros(F.n, np.int64)
    rows = S.rows()
    for j in range(F.n - 1, -1, -1):
        R = [c for c in S.col[S.rowptr[j]:S.rowptr[j + 1]] if c > j]
        ucount[j] = len(R)
        level[j] = 0 if not R else 1 + max(level[r] for r in R)
    X, s = om.features(S, Z, N, M, eps, F, level, ucount)
    Ld = np.eye(F.n)
    Lm = F.L_csr().toarray()
    Dinv = np.linalg.inv(F.D_csr().toarray())
    dpos = S.diag_positions()
    for q in np.random.default_rng(0).choice(S.nnz, 200, replace=False):
        i, j = rows[q], S.col[q]
        sij = np.sqrt(abs(M[dpos[i]] * M[dpos[j]])) or 1.0
        want = [M[q] / sij, (Z[q] - N[q]) / sij,
                float(abs(Z[q]) > eps * np.sqrt(abs(Z[dpos[i]] * Z[dpos[j]]))), float(i == j),
                np.log(abs(Dinv[i, i]) + 1e-30), np.log(abs(Dinv[j, j]) + 1e-30),
                np.log(np.linalg.norm(Lm[i]) + 1e-30), np.log(np.linalg.norm(Lm[j]) + 1e-30),
                np.log(np.linalg.norm(Lm[:, i]) + 1e-30), np.log(np.linalg.norm(Lm[:, j]) + 1e-30),
                abs(Lm[max(i, j), min(i, j)]), np.log1p(abs(N[q]) / sij), np.log1p(abs(Z[q]) / sij),
                level[i] / level.max(), level[j] / level.max(), np.log1p(ucount[min(i, j)])]
        np.testing.assert_array_equal(X[q], om.bf16(np.array(want, np.float32)))
        assert s[q] == np.float32(sij)
    del Ld


def test_dag_levels_chain_and_brute_force():
    from workloads import kkt_matrix
    # tridiagonal in natural order, no drops: column j depends on j + 1 only
    A = laplace2d(12, 1, 0.5)
    F = ildl_bk(A, np.arange(12), 0.0)
    S = oc.pattern(F)
    np.testing.assert_array_equal(oc.dag_levels(F, S), np.arange(11, -1, -1))
    # 1x1 pivots only: the per-column recursion written out directly
    A = laplace2d(9, 9, 0.05)
    F = ildl_bk(A, rcm(A), 5e-2)
    S = oc.pattern(F)
    assert int(np.sum(F.piv != 0)) == 0
    want = np.zeros(F.n, np.int64)
    for j in range(F.n - 1, -1, -1):
        R = [c for c in S.col[S.rowptr[j]:S.rowptr[j + 1]] if c > j]
        want[j] = 0 if not R else 1 + max(want[r] for r in R)
    np.testing.assert_array_equal(oc.dag_levels(F, S), want)
    # 2x2 pivots: both columns of a block share its level, which exceeds the
    # level of every row below the block
    A = kkt_matrix(30, 20, 1)
    F = ildl_bk(A, None, 1e-2)
    S = oc.pattern(F)
    lev = oc.dag_levels(F, S)
    first = np.nonzero(F.piv == 1)[0]
    assert len(first) > 0
    for j0 in first:
        assert lev[j0] == lev[j0 + 1]
        R = [c for c in np.concatenate([S.col[S.rowptr[j0]:S.rowptr[j0 + 1]],
                                        S.col[S.rowptr[j0 + 1]:S.rowptr[j0 + 2]]]) if c > j0 + 1]
        assert all(lev[j0] > lev[r] for r in R)
