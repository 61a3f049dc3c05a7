"""Seeded factors (L, D) with a prescribed dependency-level structure.

The method takes L and D as given (Section 1), so a factor can also be drawn
directly instead of computed from a matrix. This generator builds one whose
SelInv dependency levels (Section 2.1: block J waits for every block holding a
row of R_J) have chosen widths and row-set sizes, so that a single small
input exercises level launches of every width band and every block size the
device sweep distinguishes:

  - a dense "top" of ``top`` columns at the end of the ordering (every entry
    of its strictly lower triangle stored), which forms a chain of one-block
    levels;
  - below it, layers of blocks, each layer one level: every block of a layer
    holds the top's first column (or, below the first layer, a column of the
    layer above it) plus random top columns, so all its blocks sit one level
    above the layer it reads.

A layer is (count, kind): kind "light" draws |R_J| in [8, 24] (at most 276
hits of the sweep per block), "heavy" makes every tenth block draw
|R_J| in [36, 60] (more than 512 hits), "big" draws |R_J| in [130, 190] (more
than 128 rows). A fraction of the blocks are 2x2 pivots whose two columns
share their rows (the union rule), half of them indefinite.

Values: L(r, j) ~ U(-1, 1) * 0.5 / sqrt(|R_J|); 1x1 D ~ U(1, 2); 2x2 blocks
[[a, b], [b, c]] with a, c ~ U(1, 2) and b = 0.3 (definite) or 2.5
(indefinite). Random draws from numpy.random.default_rng(seed) in layer
order, block by block: the kind's |R_J|, the rows, the L values, then D.
It holds none of the method's arithmetic.
"""
from __future__ import annotations

import numpy as np

from .ildl import IldlFactors

DEFAULT_LAYERS = (("light", 3500), ("heavy", 3500), ("light", 2000), ("light", 1000), ("light", 300),
                  ("big", 1100), ("big", 40))


def layered_factor(layers=DEFAULT_LAYERS, top: int = 200, frac_2x2: float = 0.1, seed: int = 0) -> IldlFactors:
    """Factor whose layers (first entry: the first layer below the top, which
    the sweep reaches first) become consecutive levels of the given widths."""
    rng = np.random.default_rng(seed)
    if top < 191:
        raise ValueError("top must hold at least 191 columns (big blocks draw up to 190 of them)")
    # plan the unknowns: layers from the bottom of the ordering upwards are
    # the reverse of the given order; each block is 1 or 2 unknowns
    plan = []  # per layer, list of (first index, width) of its blocks
    kinds = [k for k, _ in layers]
    sizes = []
    for kind, count in layers:
        w = (rng.random(count) < frac_2x2).astype(np.int64) + 1
        sizes.append(w)
    nbelow = int(sum(int(w.sum()) for w in sizes))
    n = nbelow + top
    t0 = nbelow  # first top column
    start = nbelow
    for w in sizes:
        start -= int(w.sum())
        firsts = start + np.concatenate(([0], np.cumsum(w)[:-1]))
        plan.append(list(zip(firsts.tolist(), w.tolist())))
    cols = {}  # column j -> (rows, values)
    piv = np.zeros(n, np.int8)
    d_diag = np.zeros(n)
    d_sub = np.zeros(n)
    # the dense top: column t0 + a holds every later top row
    for a in range(top):
        j = t0 + a
        rows = np.arange(j + 1, n, dtype=np.int64)
        c = max(len(rows), 1)
        cols[j] = (rows, rng.uniform(-1.0, 1.0, len(rows)) * 0.5 / np.sqrt(c))
        d_diag[j] = rng.uniform(1.0, 2.0)
    above = None  # unknowns of the layer above (the one the sweep reached before)
    for li, (kind, blocks) in enumerate(zip(kinds, plan)):
        mine = []
        for bi, (j, w) in enumerate(blocks):
            if kind == "big":
                c = int(rng.integers(130, 191))
            elif kind == "heavy" and bi % 10 == 0:
                c = int(rng.integers(36, 61))
            else:
                c = int(rng.integers(8, 25))
            anchor = t0 if above is None else int(above[rng.integers(len(above))])
            pool = np.arange(t0 + 1, n)
            extra = rng.choice(pool, size=c - 1, replace=False)
            rows = np.unique(np.concatenate(([anchor], extra))).astype(np.int64)
            for q in range(w):
                cols[j + q] = (rows, rng.uniform(-1.0, 1.0, len(rows)) * 0.5 / np.sqrt(len(rows)))
            if w == 1:
                d_diag[j] = rng.uniform(1.0, 2.0)
            else:
                d_diag[j] = rng.uniform(1.0, 2.0)
                d_diag[j + 1] = rng.uniform(1.0, 2.0)
                d_sub[j] = 0.3 if rng.random() < 0.5 else 2.5
                piv[j], piv[j + 1] = 1, 2
            mine.extend(range(j, j + w))
        above = np.array(mine, dtype=np.int64)
    # CSR of the strictly lower L (row r holds column j for every r in R_j)
    ent_r, ent_c, ent_v = [], [], []
    for j, (rows, vals) in cols.items():
        ent_r.append(rows)
        ent_c.append(np.full(len(rows), j, np.int64))
        ent_v.append(vals)
    r = np.concatenate(ent_r)
    c = np.concatenate(ent_c)
    v = np.concatenate(ent_v)
    order = np.lexsort((c, r))
    r, c, v = r[order], c[order], v[order]
    rowptr = np.zeros(n + 1, np.int64)
    np.add.at(rowptr, r + 1, 1)
    rowptr = np.cumsum(rowptr)
    return IldlFactors(n=n, perm=np.arange(n, dtype=np.int32), L_rowptr=rowptr, L_col=c.astype(np.int32),
                       L_val=v.astype(np.float64), d_diag=d_diag, d_sub=d_sub, piv=piv, tau=0.0,
                       n_2x2=int(np.count_nonzero(piv == 1)))
