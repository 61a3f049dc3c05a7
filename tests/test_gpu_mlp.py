"""GPU parity of the learned correction's kernels against oracle/mlp.py, and a
small end-to-end training run showing what the trained network gains over
plain Mix on held-out matrices.

Forward: both sides use the same bfloat16 features and weights and float32
accumulation; the rare bfloat16 re-rounding flips of a hidden activation
(different float32 summation order) bound the tolerance. Gradients: relative
Frobenius error <= 1e-3 per tensor against the oracle's float64 backward with
the same quantisation points.
"""
import numpy as np
import pytest

from oracle import core as oc
from oracle import mlp as om
from workloads import ildl_bk, laplace2d, random_dd_symmetric, rcm

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def solver():
    from paper_2609_11363_amd import Solver
    A = laplace2d(8, 8, 0.1)
    F = ildl_bk(A, rcm(A), 1e-2)
    s = Solver(0)
    s.analyze(F.n, F.L_rowptr, F.L_col, F.piv)
    return s


def _bf16_words(x):
    """float32 bf16-valued array -> int16 words (the device layout)."""
    b = np.ascontiguousarray(x, dtype=np.float32).view(np.uint32) >> 16
    return b.astype(np.uint16).view(np.int16)


def _random_inputs(rows, seed):
    rng = np.random.default_rng(seed)
    X = om.bf16((rng.standard_normal((rows, om.NF)) * 1.5).astype(np.float32))
    theta = om.init_params(seed)
    return X, theta


@pytest.mark.parametrize("rows", [1, 63, 64, 1000, 70001])
def test_forward_parity(solver, rows):
    import torch
    print(f"[mlp forward] rows={rows}", flush=True)
    X, theta = _random_inputs(rows, rows)
    dev = solver.device
    th = torch.as_tensor(theta, device=dev)
    packed = solver.mlp_pack(th)
    y = solver.mlp_forward(packed, torch.as_tensor(_bf16_words(X), device=dev)).cpu().numpy()
    ref = om.forward(theta, X)
    err = np.abs(y - ref)
    scale = np.abs(ref).max() + 1e-6
    rel = err / (np.abs(ref) + 1e-3 * scale)
    print(f"  max abs {err.max():.2e} (scale {scale:.2e}) median rel {np.median(rel):.2e}")
    assert np.median(rel) <= 1e-5
    assert err.max() <= 2e-2 * scale
    assert (rel > 1e-4).mean() <= 0.01


def test_backward_loss_adam_parity(solver):
    import torch
    rows = 5000
    X, theta = _random_inputs(rows, 7)
    t = np.random.default_rng(8).standard_normal(rows).astype(np.float32)
    dev = solver.device
    th = torch.as_tensor(theta, device=dev)
    packed = solver.mlp_pack(th)
    Xd = torch.as_tensor(_bf16_words(X), device=dev)
    y = solver.mlp_forward(packed, Xd)
    dy = torch.empty_like(y)
    loss = torch.zeros(1, dtype=torch.float64, device=dev)
    solver.mlp_loss(y, torch.as_tensor(t, device=dev), dy, loss)
    grad = torch.zeros(om.NPARAMS, dtype=torch.float32, device=dev)
    solver.mlp_backward(packed, Xd, dy, grad)
    solver.sync()
    yo = om.forward(theta, X)
    lo, dyo = om.mse_grad(yo, t)
    assert abs(loss.item() - lo) <= 1e-4 * lo
    np.testing.assert_allclose(dy.cpu().numpy(), dyo, rtol=1e-3, atol=1e-6 * np.abs(dyo).max())
    gov = om.backward(theta, X, dyo)
    go = om.unpack(gov)
    gg = om.unpack(grad.cpu().numpy().astype(np.float64))
    for k in go:
        e = np.linalg.norm(gg[k] - go[k]) / max(np.linalg.norm(go[k]), 1e-30)
        print(f"  grad {k}: rel {e:.2e}")
        assert e <= 1e-3, k
    # one Adam step from zero moments
    m = torch.zeros_like(th)
    v = torch.zeros_like(th)
    solver.mlp_adam(th, m, v, grad, 1, lr=1e-3)
    solver.sync()
    t1, _, _ = om.adam(theta.astype(np.float64), 0 * theta, 0 * theta, gov, 1)
    big = np.abs(gov) > 1e-3 * np.abs(gov).max()  # where the gradient's sign is unambiguous
    np.testing.assert_allclose(th.cpu().numpy()[big], t1[big], rtol=1e-6, atol=1e-7)


@pytest.mark.parametrize("rows", [1, 17, 1000, 70001])
def test_backward_sizes_and_accumulation(solver, rows):
    """The backward pass (bfloat16 MFMA products, float32 sums) against the
    oracle's float64 backward at ragged sizes (a single entry; one block and
    one entry; many workgroups with a partial last block), and grad += on a
    second call."""
    import torch
    X, theta = _random_inputs(rows, 11)
    dyo = np.random.default_rng(12).standard_normal(rows).astype(np.float32) / max(rows, 1)
    dev = solver.device
    packed = solver.mlp_pack(torch.as_tensor(theta, device=dev))
    Xd = torch.as_tensor(_bf16_words(X), device=dev)
    dy = torch.as_tensor(dyo, device=dev)
    grad = torch.zeros(om.NPARAMS, dtype=torch.float32, device=dev)
    solver.mlp_backward(packed, Xd, dy, grad)
    solver.sync()
    g1 = grad.cpu().numpy().astype(np.float64)
    solver.mlp_backward(packed, Xd, dy, grad)
    solver.sync()
    g2 = grad.cpu().numpy().astype(np.float64)
    go = om.unpack(om.backward(theta, X, dyo.astype(np.float64)))
    for tag, g, f in (("one call", g1, 1.0), ("two calls", g2, 2.0)):
        gg = om.unpack(g)
        for k in go:
            ref = f * go[k]
            e = np.linalg.norm(gg[k] - ref) / max(np.linalg.norm(ref), 1e-30)
            print(f"  rows={rows} {tag} grad {k}: rel {e:.2e}")
            assert e <= 1e-3, (tag, k)


def test_features_parity_and_zero_layer_identity():
    import torch
    from paper_2609_11363_amd import Solver, upload_factors
    A = random_dd_symmetric(3, n=2500)
    F = ildl_bk(A, rcm(A), 1e-2)
    s = Solver(0)
    s.analyze(F.n, F.L_rowptr, F.L_col, F.piv)
    Lv, dd, ds = upload_factors(F)
    eps = 1e-2
    Z = s.selinv(Lv, dd, ds)
    N = s.ninv(Lv, dd, ds, p=3, delta=0.1)
    M = s.mix(Z, N, eps)
    Fe, sc = s.mlp_features(Z, N, M, eps, Lv, dd, ds)
    s.sync()
    S = oc.pattern(F)
    Zo = oc.selinv(F, S)
    No = oc.ninv(F, S, 3, 0.1)
    Mo = oc.mix(S, Zo, No, eps)
    ucount = np.array([int((S.col[S.rowptr[j]:S.rowptr[j + 1]] > j).sum()) for j in range(F.n)])
    Xo, so = om.features(S, Zo, No, Mo, eps, F, oc.dag_levels(F, S), ucount)
    Xg = (Fe.cpu().numpy().view(np.uint16).astype(np.uint32) << 16).view(np.float32)
    same = Xg == Xo
    print(f"  features identical: {same.mean():.6f}")
    assert same.mean() >= 0.9999
    diff = np.abs(Xg - Xo)[~same]
    assert np.all(diff <= np.abs(Xo[~same]) * 2 ** -7 + 1e-30)
    np.testing.assert_allclose(sc.cpu().numpy(), so, rtol=1e-6)
    # zero last layer: the corrected values equal Mix bit for bit
    theta = torch.as_tensor(om.init_params(1, zero_last=True), device=s.device)
    y = s.mlp_forward(s.mlp_pack(theta), Fe)
    out = s.mlp_apply(M, y, sc)
    s.sync()
    assert torch.equal(out, M)


def test_training_gain_on_held_out_matrices():
    """Train on Mix (tau 1e-2) -> SelInv (tau 3e-4) pairs; report the gain."""
    from paper_2609_11363_amd import learned
    sizes = [2000, 2600, 3200, 2300, 2900, 3500, 2100, 3300]
    samples = []
    for seed, n in enumerate(sizes):
        A = random_dd_symmetric(100 + seed, n=n)
        samples.append(learned.build_sample(A, rcm(A)))
        print(f"  sample {seed}: {samples[-1].meta}", flush=True)
    train, val, test = samples[:5], samples[5:6], samples[6:]
    packed, theta, hist = learned.train(train, val, epochs=30, lr=1e-3, seed=0,
                                        log=lambda m: print("  " + m, flush=True))
    assert hist["loss"][-1] < hist["loss"][0]
    base = learned.mean_error(test)
    if packed is None:
        print(f"  fallback to plain Mix: test error {base[0]:.4e}")
        return
    got = learned.mean_error(test, packed)
    print(f"  held-out mean entry error vs tight SelInv: Mix {base[0]:.4e} -> Mix+learned {got[0]:.4e} "
          f"(gain {base[0] / got[0]:.2f}x); p99 {base[1]:.3e} -> {got[1]:.3e}")
    assert got[0] < base[0]


@pytest.mark.parametrize("case", ["rand2500", "kkt"])
def test_fused_correction_matches_three_calls_and_oracle(case):
    """asi_mlp_correct equals features -> forward -> apply bit for bit, and the
    oracle's features -> network -> M + y s within the forward tolerance."""
    import torch
    from paper_2609_11363_amd import Solver, upload_factors
    from workloads import kkt_matrix
    print(f"[mlp correct] case={case}", flush=True)
    if case == "rand2500":
        A = random_dd_symmetric(4, n=2500)
        F = ildl_bk(A, rcm(A), 1e-2)
    else:
        A = kkt_matrix(60, 40, 3)
        F = ildl_bk(A, None, 1e-2)
    s = Solver(0)
    s.analyze(F.n, F.L_rowptr, F.L_col, F.piv)
    Lv, dd, ds = upload_factors(F)
    eps = 1e-2
    Z = s.selinv(Lv, dd, ds)
    N = s.ninv(Lv, dd, ds, p=3, delta=0.1)
    M = s.mix(Z, N, eps)
    theta_h = om.init_params(11)
    theta_h[5248:5313] *= 0.01  # a correction of the size the trained network makes
    theta = torch.as_tensor(theta_h, device=s.device)
    packed = s.mlp_pack(theta)
    Fe, sc = s.mlp_features(Z, N, M, eps, Lv, dd, ds)
    y = s.mlp_forward(packed, Fe)
    out3 = s.mlp_apply(M, y, sc)
    outF = s.mlp_correct(packed, Z, N, M, eps, Lv, dd, ds)
    Ma = M.clone()
    s.mlp_correct(packed, Z, N, Ma, eps, Lv, dd, ds, out=Ma)  # out may alias M
    s.sync()
    diff = (out3 != outF).nonzero().flatten()
    if diff.numel():
        d = (out3 - outF).abs()
        k = int(diff[0])
        print(f"  fused vs three calls: {diff.numel()} of {out3.numel()} differ, max {d.max().item():.3e}; "
              f"first at {k}: {out3[k].item()!r} vs {outF[k].item()!r}, M {M[k].item()!r}, y {y[k].item()!r}, "
              f"s {sc[k].item()!r}")
    assert torch.equal(out3, outF)
    assert torch.equal(outF, Ma)
    # oracle: its own SelInv, NInv, Mix and features, then the network
    S = oc.pattern(F)
    Zo = oc.selinv(F, S)
    No = oc.ninv(F, S, 3, 0.1)
    Mo = oc.mix(S, Zo, No, eps)
    ucount = np.array([int((S.col[S.rowptr[j]:S.rowptr[j + 1]] > j).sum()) for j in range(F.n)])
    Xo, so = om.features(S, Zo, No, Mo, eps, F, oc.dag_levels(F, S), ucount)
    yo = om.forward(theta_h, Xo)
    want = Mo + yo.astype(np.float64) * so.astype(np.float64)
    got = outF.cpu().numpy()
    # scale of the correction: |y| s; compare the corrections themselves
    d_got, d_want = got - Mo, want - Mo
    err = np.abs(d_got - d_want)
    scale = np.abs(d_want).max() + 1e-300
    rel = err / (np.abs(d_want) + 1e-3 * scale)
    print(f"  |S|={S.nnz} max |correction| {scale:.3e} max abs err {err.max():.2e} median rel {np.median(rel):.2e}")
    assert np.median(rel) <= 1e-5
    assert err.max() <= 2e-2 * scale
    assert (rel > 1e-4).mean() <= 0.01


@pytest.mark.parametrize("case", ["rand2500", "kkt", "diff12_mixed"])
def test_mix_and_correction_in_one_pass(case):
    """asi_mlp_correct_mix writes M = Mix(Z, N) and M + y s equal to asi_mix
    followed by asi_mlp_correct bit for bit (1x1 and 2x2 pivots, float64 and
    mixed-precision SelInv; factor loaded or passed; M not requested); M and
    out must differ."""
    import torch
    from paper_2609_11363_amd import AsiError, Solver, upload_factors
    from workloads import diffusion3d_7pt, kkt_matrix, nested_multicolor_grid
    print(f"[mix+mlp] case={case}", flush=True)
    prec = "fp64"
    if case == "rand2500":
        A = random_dd_symmetric(6, n=2500)
        F = ildl_bk(A, rcm(A), 1e-2)
    elif case == "kkt":
        A = kkt_matrix(60, 40, 3)
        F = ildl_bk(A, None, 1e-2)
    else:
        A = diffusion3d_7pt(12, 1.0, 2)
        F = ildl_bk(A, nested_multicolor_grid((12, 12, 12)), 1e-3)
        prec = "mixed"
    s = Solver(0)
    s.analyze(F.n, F.L_rowptr, F.L_col, F.piv)
    Lv, dd, ds = upload_factors(F)
    eps = 1e-2
    Z = s.selinv(Lv, dd, ds, precision=prec)
    N = s.ninv(Lv, dd, ds, p=3, delta=0.1)
    theta_h = om.init_params(13)
    theta_h[5248:5313] *= 0.01
    packed = s.mlp_pack(torch.as_tensor(theta_h, device=s.device))
    M1 = s.mix(Z, N, eps)
    out1 = s.mlp_correct(packed, Z, N, M1, eps, Lv, dd, ds)
    M2 = torch.full_like(Z, float("nan"))
    out2 = s.mlp_correct_mix(packed, Z, N, eps, Lv, dd, ds, M=M2)
    s.load_factor(Lv, dd, ds)
    out3 = s.mlp_correct_mix(packed, Z, N, eps)  # loaded factor, M not written
    s.sync()
    print(f"  |S|={Z.numel()} M differs at {int((M1 != M2).sum())}, out at {int((out1 != out2).sum())}",
          flush=True)
    assert torch.equal(M1, M2) and torch.equal(out1, out2) and torch.equal(out1, out3)
    with pytest.raises(AsiError, match="ASI_E_ARG"):
        s.mlp_correct_mix(packed, Z, N, eps, M=M2, out=M2)
