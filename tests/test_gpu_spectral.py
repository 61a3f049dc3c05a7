"""GPU parity of the spectral-correction pieces (Section 2.5, Algorithm 1,
Section 2.6): the err_1 reduction of the acceptance test, and a small
indefinite case run end to end (SelInv -> NInv -> Mix -> SPAI -> eigenpairs
of A^-1 - X on the host -> acceptance -> rank-k update on S).

Every input of the oracle comes from the oracle or from the host eigen step
run on the oracle's result; the device receives the same inputs.
"""
import numpy as np
import pytest

from oracle import core as oc
from workloads import ShiftedLaplace2DExact, ildl_bk, nested_multicolor_grid, shifted_laplace2d_indefinite

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("n,k", [(1, 0), (1000, 0), (1000, 1), (3001, 16), (300000, 16), (70000, 64)])
def test_diag_err1_parity_and_determinism(n, k):
    import torch
    from paper_2609_11363_amd import Solver
    from workloads import laplace2d
    print(f"[diag_err1] n={n} k={k}", flush=True)
    # the reduction only needs a handle with an analysis of some matrix of order n
    A = laplace2d(n, 1, 0.5)
    F = ildl_bk(A, np.arange(n), 0.0)
    s = Solver(0)
    s.analyze(F.n, F.L_rowptr, F.L_col, F.piv)
    rng = np.random.default_rng(n + k)
    d = rng.standard_normal(n)
    dhat = d + 0.1 * rng.standard_normal(n)
    V = rng.standard_normal((n, k)) / np.sqrt(max(n, 1))
    lam = rng.standard_normal(k)
    if k > 2:
        lam[1] = 0.0
    dev = torch.device("cuda", 0)
    td = torch.as_tensor(d, device=dev)
    th = torch.as_tensor(dhat, device=dev)
    Vt = torch.as_tensor(V, device=dev) if k else None
    lt = torch.as_tensor(lam, device=dev) if k else None
    a = s.diag_err1(td, th, Vt, lt)
    b = s.diag_err1(td, th, Vt, lt)
    s.sync()
    want = oc.err1_sums(d, dhat, V, lam) if k else oc.err1_sums(d, dhat)
    got = a.cpu().numpy()
    print(f"  sums {got} oracle {want}")
    assert torch.equal(a, b)
    np.testing.assert_allclose(got, want, rtol=1e-12)


def test_indefinite_pipeline_small():
    import torch
    from paper_2609_11363_amd import Solver, upload_factors
    from paper_2609_11363_amd.spectral import accept_on_device, inverse_error_eigenpairs
    N, neg, k = 24, 4, 6
    print(f"[spectral] indefinite {N}^2 neg={neg} k={k}", flush=True)
    A, sigma = shifted_laplace2d_indefinite(N, neg)
    F = ildl_bk(A, nested_multicolor_grid((N, N)), 1e-2)
    S = oc.pattern(F)
    Ahat = oc.permuted(A, F.perm)
    Zo = oc.selinv(F, S)
    No = oc.ninv(F, S, 3, 0.1)
    Mo = oc.mix(S, Zo, No, 1e-2)
    Ro = oc.spai(Ahat, S, Mo, 10)
    # device pipeline on the same factors
    dev = torch.device("cuda", 0)
    s = Solver(0)
    s.analyze(F.n, F.L_rowptr, F.L_col, F.piv)
    Lv, dd, ds = upload_factors(F)
    Z = s.selinv(Lv, dd, ds)
    Nn = s.ninv(Lv, dd, ds, p=3, delta=0.1)
    M = s.mix(Z, Nn, 1e-2)
    Ar = torch.as_tensor(A.indptr.astype(np.int64), device=dev)
    Ac = torch.as_tensor(A.indices.astype(np.int32), device=dev)
    Av = torch.as_tensor(A.data, device=dev)
    perm = torch.as_tensor(F.perm.astype(np.int32), device=dev)
    R = s.spai(Ar, Ac, Av, perm, M, cg_iters=10)
    s.sync()
    eR = oc.entry_error(S, R.cpu().numpy(), Ro)
    print(f"  Mix-SPAI e_max {eR.max():.2e}")
    assert eR.max() <= 1e-10
    # host eigen step on the oracle's result, exact A^-1 in the factor ordering
    ex = ShiftedLaplace2DExact(N, sigma)
    p = F.perm

    def apply_inv(x):
        y = np.empty_like(x)
        y[p] = x
        return ex.solve(y)[p]

    lam, V, res, napp = inverse_error_eigenpairs(apply_inv, S.to_csr(Ro), k, tol=1e-10, seed=0)
    print(f"  eigenpairs |lam| {np.abs(lam).round(3)} residual max {res.max():.1e} ({napp} applications)")
    assert res.max() <= 1e-6
    d_ref = ex.inverse_diag()[p]
    dhat = oc.diag(S, Ro)
    kept, e0, e1 = oc.accept_modes(d_ref, dhat, V, lam)
    Vt = torch.as_tensor(V, device=dev)
    corr = accept_on_device(s, torch.as_tensor(d_ref, device=dev), torch.as_tensor(dhat, device=dev), Vt, lam)
    print(f"  kept {kept} err_1 {e0:.3e} -> {e1:.3e}; device kept {corr.kept}")
    assert corr.kept == kept
    assert corr.err1_before == pytest.approx(e0, rel=1e-12)
    assert corr.err1_after == pytest.approx(e1, rel=1e-12)
    assert e1 < e0  # the near-null modes are what an incomplete factor misses
    w = torch.as_tensor(corr.weights, device=dev)
    out = s.lowrank(Vt, w, torch.as_tensor(Ro, device=dev))
    dk = s.diag(out)
    s.sync()
    want = oc.lowrank(S, V, corr.weights, Ro)
    e = oc.entry_error(S, out.cpu().numpy(), want)
    print(f"  corrected e_max {e.max():.2e}")
    assert e.max() <= 1e-10
    assert oc.err1(d_ref, dk.cpu().numpy()) == pytest.approx(e1, rel=1e-10)
