"""Learned per-entry correction — CPU reference (test infrastructure only).

The paper has no learned component; this correction is an addition to the
method. A small MLP predicts a correction of the Mix value of every entry of S from
local features, as a stand-in for tightening the drop tolerance:

    M'_ij = M_ij + y_ij * s_ij,   s_ij = sqrt(|M_ii M_jj|)   (1 where that is 0)

Features (16 per entry (i, j) of S), in this order:
  0  M_ij / s_ij
  1  (Z_ij - N_ij) / s_ij
  2  1 if |Z_ij| > eps sqrt(|Z_ii Z_jj|) (Mix took the SelInv value) else 0
  3  1 if i == j else 0
  4  log(|(D^-1)_ii| + 1e-30)   5  same for j   (with 2x2 pivots a diagonal
     entry of D^-1 can vanish; the offset keeps the feature finite)
  6  log(||L(i, :)||_2 + 1e-30)   7  same for row j   (strict lower part of L)
  8  log(||L(:, i)||_2 + 1e-30)   9  same for column j
  10 |L(max(i,j), min(i,j))| (the first Neumann term at the entry; 0 if not stored)
  11 log(1 + |N_ij| / s_ij)   12 log(1 + |Z_ij| / s_ij)
  13 level(i) / max level     14 level(j) / max level   (SelInv dependency levels)
  15 log(1 + |R_min(i,j)|)    (rows below the block of column min(i, j))
Each feature is computed in float64, rounded to float32 and then to bfloat16
(round to nearest even) — the values the network sees.

Network: 16 -> 64 -> 64 -> 1 with ReLU. Weights are bfloat16 copies (round to
nearest even) of float32 master weights; biases stay float32. The inputs of
every layer are bfloat16 (features, bf16(relu(z1)), bf16(relu(z2))); layer
sums are accumulated in float32, as on the device. Training minimises the
mean squared error of y against t_ij = (Z_tight_ij - M_ij) / s_ij with Adam.
The backward pass treats the bfloat16 roundings as identity.

Parameter vector (float32, 5313 entries): W1 (64 x 16, row = output unit),
b1 (64), W2 (64 x 64), b2 (64), w3 (64), b3 (1).
"""
from __future__ import annotations

import numpy as np

NF, NH = 16, 64
SIZES = [("W1", (NH, NF)), ("b1", (NH,)), ("W2", (NH, NH)), ("b2", (NH,)), ("w3", (NH,)), ("b3", (1,))]
NPARAMS = sum(int(np.prod(s)) for _, s in SIZES)


def unpack(theta):
    out, o = {}, 0
    for name, shape in SIZES:
        k = int(np.prod(shape))
        out[name] = np.asarray(theta[o:o + k]).reshape(shape)
        o += k
    return out


def pack(params):
    return np.concatenate([np.asarray(params[name], dtype=np.float64).ravel() for name, _ in SIZES])


def bf16(x):
    """Round float32 values to bfloat16 (nearest even), returned as float32."""
    x = np.ascontiguousarray(x, dtype=np.float32)
    b = x.view(np.uint32).astype(np.uint64)
    b = (b + 0x7FFF + ((b >> 16) & 1)) & 0xFFFF0000
    return b.astype(np.uint32).view(np.float32)


def init_params(seed=0, zero_last=False):
    """He-style initialisation of the master weights (float32)."""
    rng = np.random.default_rng(seed)
    p = {"W1": rng.standard_normal((NH, NF)) * np.sqrt(2.0 / NF), "b1": np.zeros(NH),
         "W2": rng.standard_normal((NH, NH)) * np.sqrt(2.0 / NH), "b2": np.zeros(NH),
         "w3": rng.standard_normal(NH) * (0.0 if zero_last else np.sqrt(1.0 / NH)),
         "b3": np.zeros(1)}
    return pack(p).astype(np.float32)


def features(S, Z, N, M, eps, F, level, ucount):
    """The 16 features of every entry of S (float32 after bfloat16 rounding).

    S: oracle Pattern; Z, N, M: values on S; F: the factors (IldlFactors);
    level: SelInv DAG level per unknown; ucount: |R| of the block of each
    unknown's column (the entries of its row's upper part).
    Returns (features [|S|, 16] float32 bf16-valued, scale s [|S|] float32).
    """
    n = F.n
    r = S.rows()
    c = S.col.astype(np.int64)
    dpos = S.diag_positions()
    md, zd = M[dpos], Z[dpos]
    s = np.sqrt(np.abs(md[r] * md[c]))
    s = np.where(s > 0, s, 1.0)
    # diagonal of D^-1
    dinv = np.empty(n)
    j = 0
    while j < n:
        if F.piv[j] == 1:
            # [[a, c], [c, d]]^-1 = [[d, -c], [-c, a]] / (a d - c^2): exact zeros
            # where a or d is zero
            ba, bc, bd = F.d_diag[j], F.d_sub[j], F.d_diag[j + 1]
            det = ba * bd - bc * bc
            dinv[j], dinv[j + 1] = bd / det, ba / det
            j += 2
        else:
            dinv[j] = 1.0 / F.d_diag[j]
            j += 1
    Lm = F.L_csr()
    rn = np.sqrt(np.asarray(Lm.multiply(Lm).sum(axis=1)).ravel())
    cn = np.sqrt(np.asarray(Lm.multiply(Lm).sum(axis=0)).ravel())
    lo, hi = np.minimum(r, c), np.maximum(r, c)
    Lval = np.asarray(Lm[hi, lo]).ravel()
    maxlev = max(int(level.max()), 1)
    f = np.empty((S.nnz, NF))
    f[:, 0] = M / s
    f[:, 1] = (Z - N) / s
    f[:, 2] = (np.abs(Z) > eps * np.sqrt(np.abs(zd[r] * zd[c]))).astype(float)
    f[:, 3] = (r == c).astype(float)
    f[:, 4] = np.log(np.abs(dinv[r]) + 1e-30)
    f[:, 5] = np.log(np.abs(dinv[c]) + 1e-30)
    f[:, 6] = np.log(rn[r] + 1e-30)
    f[:, 7] = np.log(rn[c] + 1e-30)
    f[:, 8] = np.log(cn[r] + 1e-30)
    f[:, 9] = np.log(cn[c] + 1e-30)
    f[:, 10] = np.abs(Lval)
    f[:, 11] = np.log1p(np.abs(N) / s)
    f[:, 12] = np.log1p(np.abs(Z) / s)
    f[:, 13] = level[r] / maxlev
    f[:, 14] = level[c] / maxlev
    f[:, 15] = np.log1p(ucount[lo].astype(float))
    return bf16(f.astype(np.float32)), s.astype(np.float32)


def forward(theta, X, want_cache=False):
    """y for feature rows X (bf16-valued float32); float32 accumulation."""
    P = unpack(np.asarray(theta, dtype=np.float32))
    W1, W2, w3 = bf16(P["W1"]), bf16(P["W2"]), bf16(P["w3"])
    b1, b2, b3 = (P[k].astype(np.float32) for k in ("b1", "b2", "b3"))
    X = np.asarray(X, dtype=np.float32)
    z1 = (X @ W1.T).astype(np.float32) + b1
    h1 = bf16(np.maximum(z1, 0))
    z2 = (h1 @ W2.T).astype(np.float32) + b2
    h2 = bf16(np.maximum(z2, 0))
    y = (h2 @ w3).astype(np.float32) + b3[0]
    if want_cache:
        return y, (X, z1, h1, z2, h2, W1, W2, w3)
    return y


def backward(theta, X, dy):
    """Gradient of sum(dy * y) with respect to the float32 master parameters.

    The bfloat16 roundings are treated as identity (straight-through)."""
    _, (X, z1, h1, z2, h2, W1, W2, w3) = forward(theta, X, want_cache=True)
    dy = np.asarray(dy, dtype=np.float64)
    g = {}
    g["w3"] = h2.astype(np.float64).T @ dy
    g["b3"] = np.array([dy.sum()])
    dz2 = (dy[:, None] * w3[None, :].astype(np.float64)) * (z2 > 0)
    g["W2"] = dz2.T @ h1.astype(np.float64)
    g["b2"] = dz2.sum(axis=0)
    dz1 = (dz2 @ W2.astype(np.float64)) * (z1 > 0)
    g["W1"] = dz1.T @ X.astype(np.float64)
    g["b1"] = dz1.sum(axis=0)
    return pack(g)


def forward_exact(theta, X):
    """Float64 forward without any rounding (for finite-difference checks)."""
    P = unpack(np.asarray(theta, dtype=np.float64))
    h1 = np.maximum(X @ P["W1"].T + P["b1"], 0)
    h2 = np.maximum(h1 @ P["W2"].T + P["b2"], 0)
    return h2 @ P["w3"] + P["b3"][0]


def backward_exact(theta, X, dy):
    """Float64 gradient of sum(dy * y) for forward_exact."""
    P = unpack(np.asarray(theta, dtype=np.float64))
    z1 = X @ P["W1"].T + P["b1"]
    h1 = np.maximum(z1, 0)
    z2 = h1 @ P["W2"].T + P["b2"]
    h2 = np.maximum(z2, 0)
    g = {"w3": h2.T @ dy, "b3": np.array([dy.sum()])}
    dz2 = dy[:, None] * P["w3"][None, :] * (z2 > 0)
    g["W2"] = dz2.T @ h1
    g["b2"] = dz2.sum(axis=0)
    dz1 = (dz2 @ P["W2"]) * (z1 > 0)
    g["W1"] = dz1.T @ X
    g["b1"] = dz1.sum(axis=0)
    return pack(g)


def mse_grad(y, t):
    """Loss sum((y - t)^2) / B and its gradient with respect to y."""
    d = np.asarray(y, dtype=np.float64) - np.asarray(t, dtype=np.float64)
    return float((d * d).mean()), 2.0 * d / len(d)


def adam(theta, m, v, g, t, lr=1e-3, b1=0.9, b2=0.999, eps=1e-8):
    """One Adam step (bias-corrected), float64 arithmetic on float32 state."""
    m = b1 * m + (1 - b1) * g
    v = b2 * v + (1 - b2) * g * g
    mh = m / (1 - b1 ** t)
    vh = v / (1 - b2 ** t)
    return theta - lr * mh / (np.sqrt(vh) + eps), m, v
