"""Pins of the CPU oracle against what the paper and the mathematics fix.

Each test checks an oracle function against something other than itself:
closed-form inverses, the exactness of the Takahashi recursion when the
pattern is closed (Section 2.1), the finite Neumann series of a nilpotent E
(Section 2.2), the Mix limits (Section 2.3), least-squares optima for SPAI
(Section 2.4), a dense masked statement of every recursion, and the
Eckart-Young optimality of the spectral correction (Section 2.5).
"""
import numpy as np
import pytest
import scipy.sparse as sp

from oracle import core as oc
from oracle import dense as od
from workloads import (ildl_bk, kkt_matrix, laplace2d, random_dd_symmetric, rcm,
                       shifted_laplace2d_indefinite, nested_multicolor_grid, diffusion3d_7pt)
from workloads.ildl import IldlFactors


def _factors_from_dense(L, D, piv, keep_mask=None):
    """IldlFactors from a dense unit-lower L (pattern = nonzeros or keep_mask)."""
    n = L.shape[0]
    mask = (L != 0) if keep_mask is None else keep_mask
    mask = np.tril(mask, -1)
    rows, cols = np.nonzero(mask)
    order = np.lexsort((cols, rows))
    rows, cols = rows[order], cols[order]
    rowptr = np.zeros(n + 1, np.int64)
    np.add.at(rowptr, rows + 1, 1)
    rowptr = np.cumsum(rowptr)
    d_diag = np.diag(D).copy()
    d_sub = np.zeros(n)
    for j in range(n - 1):
        if piv[j] == 1:
            d_sub[j] = D[j + 1, j]
    return IldlFactors(n=n, perm=np.arange(n, dtype=np.int32), L_rowptr=rowptr,
                       L_col=cols.astype(np.int32), L_val=L[rows, cols].astype(np.float64),
                       d_diag=d_diag, d_sub=d_sub, piv=np.asarray(piv, np.int8), tau=0.0)


def _random_band_factors(n, bw, seed, with_2x2=True):
    """Random unit-lower banded L and block-diagonal D (1x1 and 2x2 blocks)."""
    rng = np.random.default_rng(seed)
    piv = np.zeros(n, np.int8)
    j = 0
    while j < n:
        if with_2x2 and j + 1 < n and rng.random() < 0.3:
            piv[j], piv[j + 1] = 1, 2
            j += 2
        else:
            j += 1
    L = np.eye(n)
    for i in range(n):
        for c in range(max(0, i - bw), i):
            if piv[c] == 1 and i == c + 1:
                continue
            L[i, c] = rng.normal() * 0.5
    D = np.zeros((n, n))
    for j in range(n):
        if piv[j] == 0:
            D[j, j] = rng.choice([-1, 1]) * (1.0 + rng.random())
        elif piv[j] == 1:
            a, c, b = rng.normal(), rng.normal(), 1.0 + rng.random()
            D[j:j + 2, j:j + 2] = [[a, b], [b, c]]
    # the union rule: both columns of a 2x2 block share one row set
    mask = L != 0
    for j in range(n - 1):
        if piv[j] == 1:
            u = mask[:, j] | mask[:, j + 1]
            u[: j + 2] = False
            mask[:, j] = mask[:, j] | u
            mask[:, j + 1] = mask[:, j + 1] | u
    return L, D, piv, mask


# ---------------------------------------------------------------- SelInv ---

def test_selinv_1d_laplacian_closed_form():
    # (A^-1)_ij = min(i,j) (n+1-max(i,j)) / (n+1), 1-based, for tridiag(-1, 2, -1)
    n = 40
    A = sp.diags([-np.ones(n - 1), 2 * np.ones(n), -np.ones(n - 1)], [-1, 0, 1]).tocsr()
    F = ildl_bk(A, None, 0.0)
    S = oc.pattern(F)
    Z = oc.selinv(F, S)
    i = S.rows() + 1
    j = S.col.astype(np.int64) + 1
    ref = np.minimum(i, j) * (n + 1 - np.maximum(i, j)) / (n + 1)
    np.testing.assert_allclose(Z, ref, rtol=1e-12, atol=0)


def _sine_series_inverse(N, shift, xs, ys, xps, yps):
    """(A^-1) of the N x N Dirichlet 5-point Laplacian + shift I by its eigenbasis."""
    p = np.arange(1, N + 1)
    h = np.pi / (N + 1)
    lam = 4 * np.sin(p * h / 2) ** 2
    den = lam[:, None] + lam[None, :] + shift
    out = np.empty(len(xs))
    for t, (x, y, xp, yp) in enumerate(zip(xs, ys, xps, yps)):
        sx = np.sin(p * h * x) * np.sin(p * h * xp)
        sy = np.sin(p * h * y) * np.sin(p * h * yp)
        out[t] = (2.0 / (N + 1)) ** 2 * np.sum(sx[:, None] * sy[None, :] / den)
    return out


def test_selinv_exact_on_2d_laplacian_tau0():
    # Takahashi exactness (Section 2.1): exact factor -> SelInv = A^-1 on S
    N = 32
    A = laplace2d(N, N, 0.01)
    F = ildl_bk(A, rcm(A), 0.0)
    S = oc.pattern(F)
    Z = oc.selinv(F, S)
    r, c = S.rows(), S.col.astype(np.int64)
    orig_r, orig_c = F.perm[r], F.perm[c]
    rng = np.random.default_rng(0)
    pick = rng.choice(S.nnz, 400, replace=False)
    x, y = orig_r[pick] % N + 1, orig_r[pick] // N + 1
    xp, yp = orig_c[pick] % N + 1, orig_c[pick] // N + 1
    ref = _sine_series_inverse(N, 0.01, x, y, xp, yp)
    d = oc.diag(S, Z)
    err = np.abs(Z[pick] - ref) / np.sqrt(np.abs(d[r[pick]] * d[c[pick]]))
    assert err.max() < 1e-12
    # and against LAPACK's dense inverse on every entry of S
    Ainv = np.linalg.inv(oc.permuted(A, F.perm).toarray())
    assert oc.entry_error(S, Z, S.gather(Ainv)).max() < 1e-12


@pytest.mark.parametrize("seed", [0, 1, 2])
def test_selinv_exact_on_closed_band_pattern(seed):
    # a band pattern is closed under the recursion (R_J x R_J in S), so SelInv
    # equals (L D L^T)^-1 on S for arbitrary L, D values, 2x2 blocks included
    L, D, piv, mask = _random_band_factors(48, 4, seed)
    F = _factors_from_dense(L, D, piv, mask)
    S = oc.pattern(F)
    Z = oc.selinv(F, S)
    ref = S.gather(np.linalg.inv(L @ D @ L.T))
    np.testing.assert_allclose(Z, ref, rtol=1e-9, atol=1e-9 * np.abs(ref).max())


@pytest.mark.parametrize("seed", [0, 1, 2, 3])
def test_selinv_matches_dense_masked_recursion(seed):
    # any tau: dense boolean-mask statement of the same recursion
    A = random_dd_symmetric(seed, n=60, per_row=3, dominance=0.6)
    F = ildl_bk(A, rcm(A), 0.05)
    S = oc.pattern(F)
    Z = oc.selinv(F, S)
    mask = od.pattern_mask(F)
    assert mask.sum() == S.nnz
    Zd = od.masked_selinv(od.dense_L(F), od.dense_D(F.d_diag, F.d_sub, F.piv), F.piv, mask)
    np.testing.assert_allclose(Z, S.gather(Zd), rtol=1e-11, atol=1e-13)


def test_selinv_kkt_2x2_pivots_exact():
    for seed in range(4):
        K = kkt_matrix(14, 6, seed)
        F = ildl_bk(K, None, 0.0)
        assert F.n_2x2 > 0
        S = oc.pattern(F)
        Z = oc.selinv(F, S)
        Kinv = np.linalg.inv(oc.permuted(K, F.perm).toarray())
        np.testing.assert_allclose(Z, S.gather(Kinv), rtol=1e-10, atol=1e-12)


def test_selinv_properties_tau0():
    A = laplace2d(20, 20, 0.01)
    F = ildl_bk(A, rcm(A), 0.0)
    S = oc.pattern(F)
    Z = oc.selinv(F, S)
    Zm = S.to_csr(Z)
    assert abs(Zm - Zm.T).max() == 0.0                        # symmetric
    d = oc.diag(S, Z)
    assert (d > 0).all()                                      # SPD
    r, c = S.rows(), S.col
    assert (np.abs(Z) <= np.sqrt(d[r] * d[c]) * (1 + 1e-12)).all()
    # (Z A)_ii = 1 since pattern(P^T A P) is inside S at tau = 0
    Ap = oc.permuted(A, F.perm)
    ZA = (Zm @ Ap).diagonal()
    np.testing.assert_allclose(ZA, 1.0, rtol=0, atol=1e-12)


def test_selinv_pattern_count():
    A = random_dd_symmetric(7, n=300)
    F = ildl_bk(A, rcm(A), 1e-2)
    S = oc.pattern(F)
    assert S.nnz == 2 * F.nnzL + F.n + 2 * int((F.piv == 1).sum())
    M = S.to_csr(np.ones(S.nnz))
    assert abs(M - M.T).max() == 0


# ------------------------------------------------------------------ NInv ---

def test_ninv_delta0_dense_formula():
    A = laplace2d(12, 12, 0.01)
    F = ildl_bk(A, rcm(A), 1e-2)
    S = oc.pattern(F)
    L = od.dense_L(F)
    D = od.dense_D(F.d_diag, F.d_sub, F.piv)
    for p in (1, 2, 3):
        E = np.eye(F.n) - L
        Li = sum(np.linalg.matrix_power(E, m) for m in range(p + 1))
        ref = S.gather(Li.T @ np.linalg.inv(D) @ Li)
        np.testing.assert_allclose(oc.ninv(F, S, p, 0.0), ref, rtol=1e-12, atol=1e-14)


def test_ninv_full_series_is_exact_inverse():
    # E is nilpotent: with p >= n-1 and no drops, L^inv = L^-1 and NInv = SelInv at tau 0
    K = kkt_matrix(10, 5, 3)
    F = ildl_bk(K, None, 0.0)
    S = oc.pattern(F)
    N = oc.ninv(F, S, F.n, 0.0)
    Z = oc.selinv(F, S)
    np.testing.assert_allclose(N, Z, rtol=1e-9, atol=1e-12)


@pytest.mark.parametrize("delta", [1e-1, 1e-2])
def test_ninv_drops_match_dense_emulation(delta):
    A = random_dd_symmetric(3, n=50, per_row=3, dominance=0.7)
    F = ildl_bk(A, rcm(A), 1e-2)
    S = oc.pattern(F)
    L = od.dense_L(F)
    Li = od.neumann_linv(L, 3, delta)
    Vp, Vi, Vx = oc.linv(F, 3, delta)
    Lo = sp.csc_matrix((Vx, Vi, Vp), shape=(F.n, F.n)).toarray()
    np.testing.assert_allclose(Lo, Li, rtol=1e-13, atol=1e-15)
    D = od.dense_D(F.d_diag, F.d_sub, F.piv)
    np.testing.assert_allclose(oc.ninv(F, S, 3, delta), S.gather(Li.T @ np.linalg.inv(D) @ Li),
                               rtol=1e-12, atol=1e-14)


# ------------------------------------------------------------------- Mix ---

def test_mix_limits():
    A = laplace2d(16, 16, 0.01)
    F = ildl_bk(A, rcm(A), 0.0)
    S = oc.pattern(F)
    Z = oc.selinv(F, S)
    N = oc.ninv(F, S, 3, 1e-1)
    M0 = oc.mix(S, Z, N, 0.0)
    np.testing.assert_array_equal(M0, np.where(Z != 0, Z, N))
    # eps >= 1 on SPD at tau 0: |Z_ij| <= sqrt(Z_ii Z_jj) and '>' is strict
    M1 = oc.mix(S, Z, N, 1.0)
    np.testing.assert_array_equal(M1, N)
    # brute force on a middle threshold
    eps = 0.05
    d = oc.diag(S, Z)
    keep = np.abs(Z) > eps * np.sqrt(np.abs(d[S.rows()] * d[S.col]))
    np.testing.assert_array_equal(oc.mix(S, Z, N, eps), np.where(keep, Z, N))
    assert 0 < keep.mean() < 1


# ------------------------------------------------------------------ SPAI ---

def test_spai_dense_pattern_converges_to_inverse():
    # a full pattern with enough CG steps gives m_j = A^-1 e_j
    A = random_dd_symmetric(4, n=24, per_row=3, dominance=2.0)
    Ad = A.toarray()
    L = np.tril(np.ones((24, 24)), -1)
    F = _factors_from_dense(np.eye(24) + 0.0 * L, np.eye(24), np.zeros(24, np.int8),
                            keep_mask=L.astype(bool))
    S = oc.pattern(F)
    assert S.nnz == 24 * 24
    R = oc.spai(A, S, np.zeros(S.nnz), 200)
    np.testing.assert_allclose(R, S.gather(np.linalg.inv(Ad)), rtol=1e-8, atol=1e-10)


def test_spai_diagonal_pattern_one_step():
    A = random_dd_symmetric(5, n=30, per_row=2)
    Ad = A.toarray()
    F = _factors_from_dense(np.eye(30), np.eye(30), np.zeros(30, np.int8))
    S = oc.pattern(F)
    R = oc.spai(A, S, np.zeros(S.nnz), 3)
    ref = np.diag(Ad) / (Ad ** 2).sum(axis=0)
    np.testing.assert_allclose(R, ref, rtol=1e-13)


def test_spai_matches_least_squares_and_is_symmetric():
    A = laplace2d(8, 8, 0.3)
    F = ildl_bk(A, rcm(A), 1e-1)
    S = oc.pattern(F)
    Ah = oc.permuted(A, F.perm)
    M = oc.selinv(F, S)
    R = oc.spai(Ah, S, M, 200)
    Rm = S.to_csr(R)
    assert abs(Rm - Rm.T).max() < 1e-15
    mask = od.pattern_mask(F)
    X = np.zeros((F.n, F.n))
    for j in range(F.n):
        X[:, j] = od.spai_lstsq(Ah.toarray(), mask, j)
    np.testing.assert_allclose(R, S.gather(0.5 * (X + X.T)), rtol=1e-9, atol=1e-12)


# --------------------------------------------------------------- low rank ---

def test_lowrank_equals_masked_dense():
    A = laplace2d(10, 10, 0.1)
    F = ildl_bk(A, rcm(A), 1e-2)
    S = oc.pattern(F)
    rng = np.random.default_rng(1)
    V = rng.standard_normal((F.n, 5))
    lam = rng.standard_normal(5)
    X = rng.standard_normal(S.nnz)
    out = oc.lowrank(S, V, lam, X)
    np.testing.assert_allclose(out, X + S.gather(V @ np.diag(lam) @ V.T), rtol=1e-13, atol=1e-14)
    # diagonal follows d_i + sum_j lam_j v_ij^2 (Section 2.6)
    np.testing.assert_allclose(oc.diag(S, out), oc.diag(S, X) + (V ** 2) @ lam, rtol=1e-13)


# ------------------------------------------------------ host factorization ---

@pytest.mark.parametrize("tau", [0.0, 1e-2, 1e-1])
def test_host_ildl_matches_dense_reference(tau):
    for seed in range(3):
        K = kkt_matrix(9, 4, seed)
        F = ildl_bk(K, None, tau)
        order, L, Lpat, d_diag, d_sub, piv = od.dense_ildl_bk(K.toarray(), tau)
        np.testing.assert_array_equal(F.perm, order)
        np.testing.assert_array_equal(F.piv, piv)
        np.testing.assert_array_equal(F.L_csr().toarray() != 0 | False, np.tril(Lpat, -1) & (L != 0))
        np.testing.assert_allclose(od.dense_L(F), L, rtol=1e-12, atol=1e-14)
        np.testing.assert_allclose(F.d_diag, d_diag, rtol=1e-12)
        np.testing.assert_allclose(F.d_sub, d_sub, rtol=1e-12)


def test_host_ildl_exact_and_inertia():
    A, sigma = shifted_laplace2d_indefinite(24, 4)
    F = ildl_bk(A, nested_multicolor_grid((24, 24)), 0.0)
    L = od.dense_L(F)
    D = od.dense_D(F.d_diag, F.d_sub, F.piv)
    Ap = oc.permuted(A, F.perm).toarray()
    assert np.abs(Ap - L @ D @ L.T).max() < 1e-12 * np.abs(Ap).max()
    assert (np.linalg.eigvalsh(D) < 0).sum() == 4        # Sylvester
    assert (np.linalg.eigvalsh(A.toarray()) < 0).sum() == 4
    assert F.n_perturbed == 0


def test_host_ildl_dominant_spd_is_1x1_positive():
    A = diffusion3d_7pt(8, 1.0, 2)
    F = ildl_bk(A, nested_multicolor_grid((8, 8, 8)), 1e-3)
    assert (F.piv == 0).all() and (F.d_diag > 0).all() and F.n_perturbed == 0


@pytest.mark.parametrize("seed", [0, 1, 2])
def test_selinv_2x2_incomplete_matches_dense_masked_recursion(seed):
    # incomplete factor with 2x2 pivots: dense masked statement of the recursion
    K = kkt_matrix(16, 7, seed, density=0.5)
    F = ildl_bk(K, None, 0.1)
    assert F.n_2x2 > 0
    S = oc.pattern(F)
    mask = od.pattern_mask(F)
    Zd = od.masked_selinv(od.dense_L(F), od.dense_D(F.d_diag, F.d_sub, F.piv), F.piv, mask)
    np.testing.assert_allclose(oc.selinv(F, S), S.gather(Zd), rtol=1e-11, atol=1e-13)


def test_selinv_block_check_accepts_selinv_and_flags_a_planted_error():
    """The sampled-block property checker (used where the full oracle is too
    slow) returns rounding-level errors on the oracle's SelInv, with 1x1 and
    2x2 blocks, and flags one perturbed entry in the blocks that read it."""
    from workloads import kkt_matrix
    for A, q in [(laplace2d(20, 20, 0.05), "rcm"), (kkt_matrix(40, 25, 2), None)]:
        F = ildl_bk(A, rcm(A) if q == "rcm" else None, 1e-2)
        S = oc.pattern(F)
        Z = oc.selinv(F, S)
        blocks = [j for j in range(F.n) if F.piv[j] != 2]
        assert oc.selinv_block_check(F, S, Z, blocks).max() <= 1e-13
        Zb = Z.copy()
        p = S.rowptr[10] + 1  # an off-diagonal entry of row 10
        Zb[p] *= 1.0 + 1e-6
        assert oc.selinv_block_check(F, S, Zb, blocks).max() >= 1e-8


def test_selinv_nan_sentinel_run_is_finite_and_catches_a_planted_order_mistake():
    """NaN-sentinel run (Section 2.1 reads only entries of Zhat that later
    blocks have written): starting from NaN on S instead of zero gives a
    finite result, bit for bit the ordinary one, on 1x1 and 2x2 incomplete
    factors. The same run with the blocks visited in the wrong order (first
    to last, a mistake planted in the oracle) turns non-finite, while the
    zero-started run with that mistake stays finite: the sentinel is what
    exposes it."""
    cases = [ildl_bk(laplace2d(12, 12, 0.05), rcm(laplace2d(12, 12, 0.05)), 1e-2),
             ildl_bk(kkt_matrix(30, 18, 3), None, 1e-2),
             ildl_bk(diffusion3d_7pt(6, 1.0, 4), nested_multicolor_grid((6, 6, 6)), 1e-3)]
    assert cases[1].n_2x2 > 0
    for F in cases:
        S = oc.pattern(F)
        Z = oc.selinv(F, S)
        Zs = oc.selinv(F, S, sentinel=True)
        assert np.isfinite(Zs).all()
        assert np.array_equal(Zs, Z)
        wrong = oc.selinv(F, S, wrong_order=True)
        assert np.isfinite(wrong).all()
        assert not np.isfinite(oc.selinv(F, S, sentinel=True, wrong_order=True)).all()


def test_saddle2d_generator_and_its_2x2_pivots():
    """The saddle-point input: symmetric, the Laplacian block and one
    constraint per 2 x 2 cell coupling exactly the cell's four grid unknowns,
    a zero constraint block, q a permutation that puts each constraint before
    its cell's unknowns; the host factorization then takes 2x2 pivots (and a
    dense LDL^T of the same matrix confirms its inertia: N^2 positive and N^2/4
    negative eigenvalues)."""
    from workloads import saddle2d
    N = 12
    K, q = saddle2d(N)
    n, nu = N * N + N * N // 4, N * N
    assert K.shape == (n, n) and abs(K - K.T).max() == 0
    Kd = K.toarray()
    np.testing.assert_array_equal(Kd[:nu, :nu], laplace2d(N, N, 0.0).toarray())
    assert not Kd[nu:, nu:].any()
    for c in range(N * N // 4):
        x, y = c % (N // 2), c // (N // 2)
        cells = sorted((2 * x + dx) + N * (2 * y + dy) for dx in (0, 1) for dy in (0, 1))
        assert sorted(np.nonzero(Kd[nu + c, :nu])[0].tolist()) == cells
    assert sorted(q.tolist()) == list(range(n))
    pos = np.empty(n, np.int64)
    pos[q] = np.arange(n)
    for c in range(N * N // 4):
        assert all(pos[nu + c] < pos[u] for u in np.nonzero(Kd[nu + c, :nu])[0])
    F = ildl_bk(K, q, 1e-3)
    assert F.n_2x2 > 0
    ev = np.linalg.eigvalsh(Kd)
    assert (ev > 0).sum() == nu and (ev < 0).sum() == N * N // 4
    # the inertia of D equals that of K (Sylvester) for the complete factor
    G = ildl_bk(K, q, 0.0)
    D = od.dense_D(G.d_diag, G.d_sub, G.piv)
    evd = np.linalg.eigvalsh(D)
    assert (evd > 0).sum() == nu and (evd < 0).sum() == N * N // 4
