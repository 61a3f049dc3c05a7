"""GPU parity on the covariance-type workload (Section 3.6) and of the trace
output (Section 3.5): SelInv, NInv, Mix and Mix-SPAI against the oracle on
the same factors, and the trace sums (with and without a rank-k term)
against the oracle's, repeatable bit for bit."""
import numpy as np
import pytest

from oracle import core as oc
from workloads import covariance_grid, ildl_bk, laplace2d, nested_multicolor_grid

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("N,tau", [(30, 1e-3), (17, 1e-4)])
def test_covariance_pipeline_and_trace(N, tau):
    import torch
    from paper_2609_11363_amd import Solver, upload_factors
    print(f"[covariance] N={N} tau={tau}", flush=True)
    A = covariance_grid(N)
    F = ildl_bk(A, nested_multicolor_grid((N, N)), tau)
    S = oc.pattern(F)
    Ahat = oc.permuted(A, F.perm)
    Zo = oc.selinv(F, S)
    No = oc.ninv(F, S, 3, 0.1)
    Mo = oc.mix(S, Zo, No, 1e-2)
    Ro = oc.spai(Ahat, S, Mo, 10)
    dev = torch.device("cuda", 0)
    s = Solver(0)
    s.analyze(F.n, F.L_rowptr, F.L_col, F.piv)
    Lv, dd, ds = upload_factors(F)
    s.load_factor(Lv, dd, ds)
    Z, Nn = s.selinv_ninv(p=3, delta=0.1)
    M = s.mix(Z, Nn, 1e-2)
    Ar = torch.as_tensor(A.indptr.astype(np.int64), device=dev)
    Ac = torch.as_tensor(A.indices.astype(np.int32), device=dev)
    Av = torch.as_tensor(A.data, device=dev)
    perm = torch.as_tensor(F.perm.astype(np.int32), device=dev)
    R = s.spai(Ar, Ac, Av, perm, M, cg_iters=10)
    t0 = s.trace(R)
    t1 = s.trace(R)
    rng = np.random.default_rng(N)
    V = rng.standard_normal((F.n, 3)) / np.sqrt(F.n)
    lam = np.array([0.3, -0.2, 0.05])
    tk = s.trace(R, torch.as_tensor(V, device=dev), torch.as_tensor(lam, device=dev))
    s.sync()
    for name, g, o in (("selinv", Z, Zo), ("ninv", Nn, No), ("mix", M, Mo), ("mix_spai", R, Ro)):
        e = oc.entry_error(S, g.cpu().numpy(), o).max()
        print(f"  {name} e_max {e:.2e}")
        assert e <= 1e-10, name
    assert torch.equal(t0, t1)
    np.testing.assert_allclose(t0.cpu().numpy(), oc.trace_sums(S, Ro), rtol=1e-12)
    np.testing.assert_allclose(tk.cpu().numpy(), oc.trace_sums(S, Ro, V, lam), rtol=1e-12)


def test_trace_single_unknown():
    import torch
    from paper_2609_11363_amd import Solver
    A = laplace2d(1, 1, 0.5)
    F = ildl_bk(A, np.arange(1), 0.0)
    s = Solver(0)
    s.analyze(F.n, F.L_rowptr, F.L_col, F.piv)
    X = torch.tensor([-2.5], dtype=torch.float64, device=s.device)
    t = s.trace(X)
    s.sync()
    assert t.cpu().numpy().tolist() == [-2.5, 2.5]
