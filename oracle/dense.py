"""Dense numpy references for tiny inputs — test infrastructure only.

These are second, independent statements of the definitions (dense matrices,
boolean masks, library linear algebra) used to pin the C oracle and the host
factorization on inputs small enough for O(n^3) work.
"""
from __future__ import annotations

import numpy as np

ALPHA_BK = (1.0 + np.sqrt(17.0)) / 8.0


def block_starts(piv):
    piv = np.asarray(piv)
    out = []
    j = 0
    n = len(piv)
    while j < n:
        out.append(j)
        j += 2 if piv[j] == 1 else 1
    return out


def dense_D(d_diag, d_sub, piv):
    n = len(d_diag)
    D = np.diag(np.asarray(d_diag, dtype=np.float64))
    for j in range(n):
        if piv[j] == 1:
            D[j + 1, j] = D[j, j + 1] = d_sub[j]
    return D


def dense_L(F):
    L = np.eye(F.n)
    for i in range(F.n):
        for q in range(F.L_rowptr[i], F.L_rowptr[i + 1]):
            L[i, F.L_col[q]] = F.L_val[q]
    return L


def pattern_mask(F):
    """Boolean S of L + D + L^T with the 2x2 union rule."""
    n = F.n
    M = np.eye(n, dtype=bool)
    piv = F.piv
    for i in range(n):
        for q in range(F.L_rowptr[i], F.L_rowptr[i + 1]):
            j = F.L_col[q]
            J = j - 1 if piv[j] == 2 else j
            for jj in ([J, J + 1] if piv[J] == 1 else [J]):
                M[i, jj] = M[jj, i] = True
    for j in range(n):
        if piv[j] == 1:
            M[j, j + 1] = M[j + 1, j] = True
    return M


def masked_selinv(L, D, piv, mask):
    """Takahashi recursion on a dense boolean pattern (Section 2.1).

    Blocks from last to first; Z(R, J) = -(Z o mask)(R, R) L(R, J),
    Z(J, J) = D_J^-1 - L(R, J)^T Z(R, J) (off-diagonal of a 2x2 averaged).
    """
    n = L.shape[0]
    Z = np.zeros((n, n))
    for J in reversed(block_starts(piv)):
        cols = [J, J + 1] if piv[J] == 1 else [J]
        last = cols[-1]
        R = [r for r in range(last + 1, n) if mask[r, J]]
        Zr = (Z * mask)[np.ix_(R, R)]
        Lr = L[np.ix_(R, cols)]
        Y = -Zr @ Lr
        Z[np.ix_(R, cols)] = Y
        Z[np.ix_(cols, R)] = Y.T
        ZJ = np.linalg.inv(D[np.ix_(cols, cols)]) - Lr.T @ Y
        ZJ = 0.5 * (ZJ + ZJ.T)
        Z[np.ix_(cols, cols)] = ZJ
    return Z


def neumann_linv(L, p, delta):
    """Truncated, delta-sparsified Neumann series of L^-1 (Section 2.2)."""
    n = L.shape[0]
    E = np.eye(n) - L
    T = np.eye(n)
    S = np.eye(n)
    for _ in range(p):
        T = E @ T
        T[np.abs(T) < delta] = 0.0
        S = S + T
    return S


def spai_lstsq(Ahat, mask, j):
    """Exact minimiser of ||Ahat m - e_j||_2 over m supported on column j of mask."""
    J = np.nonzero(mask[:, j])[0]
    e = np.zeros(Ahat.shape[0])
    e[j] = 1.0
    m, *_ = np.linalg.lstsq(Ahat[:, J], e, rcond=None)
    out = np.zeros(Ahat.shape[0])
    out[J] = m
    return out


def dense_ildl_bk(A, tau=0.0, pivoting=True):
    """Dense threshold ILDL with Bunch-Kaufman pivots — the reference for the host factor.

    Same readings as the host factorization (symmetric scaling by
    1/sqrt(max_j |a_ij|), drop |l_ik| < tau on the scaled factor, a 2x2 row
    dropped only when both entries are below tau, tiny-pivot replacement),
    written on a dense Schur complement with a boolean structure mask that
    tracks structural fill. Returns (perm, L, d_diag, d_sub, piv) with
    A[perm][:, perm] ~ L D L^T.
    """
    A = np.array(A, dtype=np.float64)
    n = A.shape[0]
    s = 1.0 / np.sqrt(np.maximum(np.abs(A).max(axis=1), 1e-300))
    s[np.abs(A).max(axis=1) == 0] = 1.0
    S = s[:, None] * A * s[None, :]
    amax = np.abs(S).max()
    struct = A != 0
    active = np.ones(n, bool)
    order = list(range(n))
    where = list(range(n))
    Lh = np.zeros((n, n))       # indexed by (unknown id, position)
    Lmask = np.zeros((n, n), bool)
    dd = np.zeros(n)
    ds = np.zeros(n)
    piv = np.zeros(n, np.int8)

    def colmax(p):
        best, arg = 0.0, -1
        ids = [i for i in range(n) if active[i] and i != p and struct[i, p]]
        for i in sorted(ids, key=lambda i: where[i]):
            if abs(S[i, p]) > best:
                best, arg = abs(S[i, p]), i
        return best, arg

    def swap(a, b):
        ia, ib = order[a], order[b]
        order[a], order[b] = ib, ia
        where[ib], where[ia] = a, b

    k = 0
    while k < n:
        p = order[k]
        two = False
        if pivoting:
            lam, r = colmax(p)
            if lam > 0 and abs(S[p, p]) < ALPHA_BK * lam:
                sig, _ = colmax(r)
                if abs(S[p, p]) * sig >= ALPHA_BK * lam * lam:
                    pass
                elif abs(S[r, r]) >= ALPHA_BK * sig:
                    swap(k, where[r])
                    p = r
                else:
                    two = True
                    swap(k + 1, where[r])
        if not two:
            d = S[p, p]
            if abs(d) < 1e-14 * amax:
                d = (1.0 if d >= 0 else -1.0) * 1e-8 * amax
            nb = [i for i in range(n) if active[i] and i != p and struct[i, p]]
            kept = [i for i in nb if not abs(S[i, p] / d) < tau]
            lv = np.array([S[i, p] / d for i in kept])
            dd[k] = d
            active[p] = False
            for a, i in enumerate(kept):
                Lh[i, k] = lv[a]
                Lmask[i, k] = True
            for a, i in enumerate(kept):
                la = lv[a] * d
                for b, i2 in enumerate(kept):
                    S[i, i2] -= la * lv[b]
                    struct[i, i2] = True
            k += 1
        else:
            a11, a22, b = S[p, p], S[r, r], S[p, r]
            al, ga = a11 / b, a22 / b
            den = b * (al * ga - 1.0)
            nb = [i for i in range(n) if active[i] and i not in (p, r)
                  and (struct[i, p] or struct[i, r])]
            rows = []
            for i in nb:
                w0, w1 = S[i, p], S[i, r]
                l0 = (w0 * ga - w1) / den
                l1 = (-w0 + w1 * al) / den
                if abs(l0) < tau and abs(l1) < tau:
                    continue
                rows.append((i, l0, l1, w0, w1))
            dd[k], dd[k + 1], ds[k] = a11, a22, b
            piv[k], piv[k + 1] = 1, 2
            active[p] = active[r] = False
            for (i, l0, l1, w0, w1) in rows:
                Lh[i, k], Lh[i, k + 1] = l0, l1
                Lmask[i, k] = Lmask[i, k + 1] = True
            for (i, l0, l1, _, _) in rows:
                for (i2, _, _, v0, v1) in rows:
                    S[i, i2] -= l0 * v0 + l1 * v1
                    struct[i, i2] = True
            k += 2
    # final positions and unscaling
    order = np.array(order)
    where = np.array(where)
    L = np.eye(n)
    Lpat = np.zeros((n, n), bool)
    for i in range(n):
        for c in range(n):
            if Lmask[i, c]:
                L[where[i], c] = Lh[i, c] * s[order[c]] / s[i]
                Lpat[where[i], c] = True
    sq = s[order]
    d_diag = dd / sq ** 2
    d_sub = np.zeros(n)
    for j in range(n - 1):
        if piv[j] == 1:
            d_sub[j] = ds[j] / (sq[j] * sq[j + 1])
    return order, L, Lpat, d_diag, d_sub, piv


def fixed_pattern_ldl(Ah, Lpat, piv):
    """Numeric phase of the incomplete factorization P^T A P ~ L D L^T
    (Section 2.1) on a given strictly lower pattern and 1x1/2x2 partition.

    The pivot sequence and the kept entries are the symbolic result of a
    threshold factorization; given them, each block B = {j} or {j, j+1} of D
    and each kept entry of L follow from the Crout recurrence, in block order:
        W(:, B) = Ah(:, B) - L(:, <j) D(<j, <j) L(B, <j)^T,
        D_B = W(B, B),
        L(i, B) = W(i, B) D_B^-1 where (i, B) is kept, 0 elsewhere.
    Dense matrices, library matrix products, no reordering. Returns
    (L with unit diagonal, d_diag, d_sub) with d_sub[j] = D(j+1, j) at the
    first index of each 2x2 block.
    """
    Ah = np.asarray(Ah, dtype=np.float64)
    n = Ah.shape[0]
    L = np.eye(n)
    D = np.zeros((n, n))
    d_diag = np.zeros(n)
    d_sub = np.zeros(n)
    for j in block_starts(piv):
        B = [j, j + 1] if piv[j] == 1 else [j]
        e = j + len(B)
        W = Ah[:, B] - L[:, :j] @ (D[:j, :j] @ L[B, :j].T)
        if len(B) == 1:
            d = W[j, 0]
            D[j, j] = d_diag[j] = d
            L[e:, j] = np.where(Lpat[e:, j], W[e:, 0] / d, 0.0)
        else:
            d0, d1, s = W[j, 0], W[j + 1, 1], W[j + 1, 0]
            D[j, j], D[j + 1, j + 1] = d0, d1
            D[j + 1, j] = D[j, j + 1] = s
            d_diag[j], d_diag[j + 1], d_sub[j] = d0, d1, s
            det = d0 * d1 - s * s
            inv = np.array([[d1, -s], [-s, d0]]) / det
            L[e:, B] = np.where(Lpat[e:, B], W[e:, :] @ inv, 0.0)
    return L, d_diag, d_sub
