"""Learned per-entry correction of the Mix result: data, training, inference.

The network and its training run in libasi's kernels (asi_mlp_*); this module
only orchestrates them: it builds training pairs from the method itself (Mix
of a loose incomplete factor as input, SelInv of a tight factor of the same
matrix and ordering as target), runs Adam over mini-batches, keeps the
parameters with the best validation error and falls back to plain Mix when
the network does not beat it.

Target of entry (i, j) in S_loose that is also in S_tight:
    t_ij = (Z_tight_ij - M_ij) / s_ij,   s_ij = sqrt(|M_ii M_jj|),
and the corrected value is M'_ij = M_ij + y_ij s_ij.
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np

from .asi import MLP_PARAMS, Solver, upload_factors

# master parameter layout: W1 [64][16], b1, W2 [64][64], b2, w3, b3
_LAYOUT = [(64, 16), (64,), (64, 64), (64,), (64,), (1,)]


# offsets of the last layer in the master vector
_W3, _B3 = 5248, 5312


def init_theta(seed: int = 0) -> np.ndarray:
    """He-initialised hidden layers, zero biases and a zero output layer, so
    the untrained network returns y = 0 (the corrected values equal Mix)."""
    rng = np.random.default_rng(seed)
    parts = []
    for shape in _LAYOUT:
        if len(shape) == 2:
            parts.append(rng.standard_normal(shape).ravel() * np.sqrt(2.0 / shape[1]))
        else:
            parts.append(np.zeros(shape))
    theta = np.concatenate(parts).astype(np.float32)
    assert theta.size == MLP_PARAMS
    return theta


def fold_scale(theta, sigma):
    """Parameters whose output is sigma times the input parameters' output."""
    out = theta.clone()
    out[_W3:_B3 + 1] *= sigma
    return out


@dataclass
class Sample:
    """One matrix of the data set, resident on the device."""
    solver: Solver
    F: object            # features of every entry of S_loose (int16 bf16 words)
    scale: object        # s_ij (float32)
    M: object            # Mix values on S_loose (float64)
    rows: object         # indices of the entries of S_loose that are in S_tight (int64, device)
    target: object       # t_ij on those entries (float32, device)
    Zt: np.ndarray       # tight SelInv on those entries (host, float64)
    meta: dict = field(default_factory=dict)


def _keys(rowptr, col, n):
    r = np.repeat(np.arange(n, dtype=np.int64), np.diff(rowptr))
    return r * n + col.astype(np.int64)


def build_sample(A, q, tau_loose=1e-2, tau_tight=3e-4, p=3, delta=0.1, eps=1e-2, device=0, ildl=None):
    """Mix at tau_loose (input) and SelInv at tau_tight (target) of one matrix."""
    import torch
    if ildl is None:
        from workloads import ildl_bk as ildl
    Fl = ildl(A, q, tau_loose)
    Ft = ildl(A, q, tau_tight)
    if not np.array_equal(Fl.perm, Ft.perm):
        raise ValueError("the loose and tight factors use different permutations")
    sl = Solver(device)
    sl.analyze(Fl.n, Fl.L_rowptr, Fl.L_col, Fl.piv)
    Lv, dd, ds = upload_factors(Fl, f"cuda:{device}")
    Z = sl.selinv(Lv, dd, ds)
    N = sl.ninv(Lv, dd, ds, p=p, delta=delta)
    M = sl.mix(Z, N, eps)
    F, sc = sl.mlp_features(Z, N, M, eps, Lv, dd, ds)
    st = Solver(device)
    st.analyze(Ft.n, Ft.L_rowptr, Ft.L_col, Ft.piv)
    Lt, dt, dst = upload_factors(Ft, f"cuda:{device}")
    Zt = st.selinv(Lt, dt, dst)
    sl.sync()
    st.sync()
    rpl, cll = (x.cpu().numpy() for x in sl.pattern())
    rpt, clt = (x.cpu().numpy() for x in st.pattern())
    kl = _keys(rpl, cll, Fl.n)
    kt = _keys(rpt, clt, Fl.n)
    pos = np.searchsorted(kt, kl)
    pos = np.minimum(pos, len(kt) - 1)
    ok = kt[pos] == kl
    rows = np.nonzero(ok)[0]
    zt = Zt.cpu().numpy()[pos[ok]]
    m = M.cpu().numpy()[rows]
    s = sc.cpu().numpy()[rows].astype(np.float64)
    target = ((zt - m) / s).astype(np.float32)
    dev = torch.device("cuda", device)
    del st, Lt, dt, dst, Zt
    return Sample(solver=sl, F=F, scale=sc, M=M, rows=torch.as_tensor(rows, device=dev),
                  target=torch.as_tensor(target, device=dev), Zt=zt,
                  meta={"n": Fl.n, "nnz_S_loose": int(len(kl)), "nnz_S_tight": int(len(kt)),
                        "matched": int(len(rows))})


def entry_errors(sample: Sample, corrected) -> np.ndarray:
    """|x_ij - Z_tight_ij| / s_ij on the matched entries."""
    x = corrected.cpu().numpy()[sample.rows.cpu().numpy()]
    s = sample.scale.cpu().numpy()[sample.rows.cpu().numpy()].astype(np.float64)
    return np.abs(x - sample.Zt) / s


def predict(sample: Sample, packed):
    """M' = M + y s on all of S_loose (device)."""
    y = sample.solver.mlp_forward(packed, sample.F)
    return sample.solver.mlp_apply(sample.M, y, sample.scale)


def mean_error(samples, packed=None):
    errs = []
    for smp in samples:
        x = smp.M if packed is None else predict(smp, packed)
        errs.append(entry_errors(smp, x))
    e = np.concatenate(errs)
    return float(e.mean()), float(np.quantile(e, 0.99))


def train(train_set, val_set, epochs=30, batch=65536, lr=1e-3, seed=0, log=None):
    """Adam on the squared error of y against the targets divided by their
    standard deviation sigma (sigma is folded back into the output layer for
    inference); returns (packed weights or None for the plain-Mix fallback,
    float32 masters with sigma folded in, history)."""
    import torch
    solver = train_set[0].solver
    dev = solver.device
    theta = torch.as_tensor(init_theta(seed), device=dev)
    m = torch.zeros_like(theta)
    v = torch.zeros_like(theta)
    grad = torch.zeros_like(theta)
    loss = torch.zeros(1, dtype=torch.float64, device=dev)
    packed = solver.mlp_pack(theta)
    # gather the matched rows of every training matrix into one batch source
    Fs = torch.cat([smp.F.index_select(0, smp.rows) for smp in train_set])
    Ts = torch.cat([smp.target for smp in train_set])
    sigma = float(Ts.double().std().item()) or 1.0
    Ts = (Ts / sigma).contiguous()
    eval_packed = torch.empty_like(packed)
    rows = Fs.shape[0]
    gen = torch.Generator(device="cpu").manual_seed(seed)
    base_val = mean_error(val_set)[0]
    best = (base_val, None, None)
    history = {"base_val": base_val, "loss": [], "val": [], "sigma": sigma}
    step = 0
    for ep in range(epochs):
        order = torch.randperm(rows, generator=gen).to(dev)
        ep_loss = 0.0
        nb = 0
        for b0 in range(0, rows, batch):
            idx = order[b0:b0 + batch]
            Fb = Fs.index_select(0, idx)
            Tb = Ts.index_select(0, idx)
            y = solver.mlp_forward(packed, Fb)
            dy = torch.empty_like(y)
            loss.zero_()
            grad.zero_()
            solver.mlp_loss(y, Tb, dy, loss)
            solver.mlp_backward(packed, Fb, dy, grad)
            step += 1
            solver.mlp_adam(theta, m, v, grad, step, lr=lr)
            solver.mlp_pack(theta, packed)
            ep_loss += float(loss.item())
            nb += 1
        folded = fold_scale(theta, sigma)
        solver.mlp_pack(folded, eval_packed)
        val = mean_error(val_set, eval_packed)[0]
        history["loss"].append(ep_loss / max(nb, 1))
        history["val"].append(val)
        if log:
            log(f"epoch {ep}: loss {ep_loss / max(nb, 1):.4e} val {val:.4e} (plain Mix {base_val:.4e})")
        if val < best[0]:
            best = (val, eval_packed.clone(), folded)
    return best[1], best[2], history
