"""GPU parity: the HIP path through the C ABI against the CPU oracle.

Every case runs SelInv, NInv and Mix on the device and compares, entry by
entry on S, with the oracle on the same (L, D, P): float64 mode within a
relative entry error e_ij = |x_ij - y_ij| / sqrt(|y_ii y_jj|) of 1e-10, the
mixed float32/float64 mode within 1e-4 (the stated bound; the measured value
is printed). Patterns are compared bit-exactly.
"""
import numpy as np
import pytest
import scipy.sparse as sp

from oracle import core as oc
from workloads import (diffusion3d_7pt, ildl_bk, kkt_matrix, laplace2d, nested_multicolor_grid,
                       random_dd_symmetric, rcm)
from workloads.ildl import IldlFactors

pytestmark = pytest.mark.gpu

FP64_TOL = 1e-10
MIXED_TOL = 1e-4


def _arrow(n, seed):
    """Arrowhead SPD matrix whose hub is eliminated first: |R_0| = n - 1."""
    rng = np.random.default_rng(seed)
    A = sp.lil_matrix((n, n))
    for i in range(n):
        A[i, i] = 4.0 + rng.random()
    for i in range(1, n):
        v = 0.5 * rng.standard_normal() / np.sqrt(n)
        A[0, i] = A[i, 0] = v
        if i + 1 < n:
            A[i, i + 1] = A[i + 1, i] = -1.0
    return sp.csr_matrix(A)


def _case(name):
    if name == "lap32_tau0":
        A = laplace2d(32, 32, 0.01)
        return ildl_bk(A, rcm(A), 0.0)
    if name == "lap32_tau1e-2":
        A = laplace2d(32, 32, 0.01)
        return ildl_bk(A, rcm(A), 1e-2)
    if name == "kkt_tau0":
        return ildl_bk(kkt_matrix(60, 25, 3, density=0.15), None, 0.0)
    if name == "kkt_tau5e-2":
        return ildl_bk(kkt_matrix(60, 25, 4, density=0.15), None, 5e-2)
    if name == "diff16_tau1e-3":
        A = diffusion3d_7pt(16, 1.0, 2)
        return ildl_bk(A, nested_multicolor_grid((16, 16, 16)), 1e-3)
    if name == "rand3000_tau1e-2":
        A = random_dd_symmetric(11, n=3000)
        return ildl_bk(A, rcm(A), 1e-2)
    if name == "arrow600":
        return ildl_bk(_arrow(600, 0), None, 0.0, pivoting=False)
    if name == "n1":
        return IldlFactors(n=1, perm=np.zeros(1, np.int32), L_rowptr=np.zeros(2, np.int64),
                           L_col=np.zeros(0, np.int32), L_val=np.zeros(0), d_diag=np.array([2.5]),
                           d_sub=np.zeros(1), piv=np.zeros(1, np.int8), tau=0.0)
    if name == "2x2_only":
        return IldlFactors(n=2, perm=np.arange(2, dtype=np.int32), L_rowptr=np.zeros(3, np.int64),
                           L_col=np.zeros(0, np.int32), L_val=np.zeros(0),
                           d_diag=np.array([0.0, 1e-3]), d_sub=np.array([1.5, 0.0]),
                           piv=np.array([1, 2], np.int8), tau=0.0)
    raise KeyError(name)


CASES = ["n1", "2x2_only", "lap32_tau0", "lap32_tau1e-2", "kkt_tau0", "kkt_tau5e-2",
         "diff16_tau1e-3", "rand3000_tau1e-2", "arrow600"]


@pytest.fixture(scope="module")
def torch_mod():
    import torch
    assert torch.cuda.is_available()
    return torch


def _run(torch_mod, F, p, delta, eps, precision):
    from paper_2609_11363_amd import Solver, upload_factors
    s = Solver(0)
    s.analyze(F.n, F.L_rowptr, F.L_col, F.piv, pool_entries=F.n * min(F.n, 1024))
    Lv, dd, ds = upload_factors(F)
    Z = s.selinv(Lv, dd, ds, precision=precision)
    N = s.ninv(Lv, dd, ds, p=p, delta=delta, precision=precision)
    M = s.mix(Z, N, eps)
    s.sync()
    rp, cl = s.pattern()
    return s, (rp.cpu().numpy(), cl.cpu().numpy()), Z.cpu().numpy(), N.cpu().numpy(), M.cpu().numpy()


@pytest.mark.parametrize("name", CASES)
def test_parity_fp64(torch_mod, name):
    print(f"[parity fp64] case={name}", flush=True)
    F = _case(name)
    p, delta, eps = 3, (0.0 if F.n < 2000 else 0.1), 1e-2
    S = oc.pattern(F)
    s, (rp, cl), Z, N, M = _run(torch_mod, F, p, delta, eps, "fp64")
    np.testing.assert_array_equal(rp, S.rowptr)
    np.testing.assert_array_equal(cl, S.col)
    Zo = oc.selinv(F, S)
    No = oc.ninv(F, S, p, delta)
    Mo = oc.mix(S, Zo, No, eps)
    ez = oc.entry_error(S, Z, Zo).max()
    en = oc.entry_error(S, N, No).max()
    em = oc.entry_error(S, M, Mo).max()
    print(f"  n={F.n} |S|={S.nnz} levels={s.info()['n_levels']} e_Z={ez:.2e} e_N={en:.2e} e_M={em:.2e}")
    assert ez <= FP64_TOL and en <= FP64_TOL and em <= FP64_TOL


@pytest.mark.parametrize("name", ["lap32_tau1e-2", "diff16_tau1e-3", "rand3000_tau1e-2", "arrow600"])
def test_parity_mixed(torch_mod, name):
    print(f"[parity mixed] case={name}", flush=True)
    F = _case(name)
    p, delta, eps = 3, 0.1, 1e-2
    S = oc.pattern(F)
    s, _, Z, N, M = _run(torch_mod, F, p, delta, eps, "mixed")
    Zo = oc.selinv(F, S)
    No = oc.ninv(F, S, p, delta)
    ez = oc.entry_error(S, Z, Zo)
    en = oc.entry_error(S, N, No)
    # the Mix mask is taken from the device's own Z: compare M with that mask
    d = oc.diag(S, Z)
    keep = np.abs(Z) > eps * np.sqrt(np.abs(d[S.rows()] * d[S.col]))
    em = oc.entry_error(S, M, np.where(keep, Zo, No))
    flips = int((keep != (oc.mix(S, Zo, No, eps) == Zo)).sum())
    print(f"  e_Z max={ez.max():.2e} p99={np.quantile(ez, .99):.2e} e_N max={en.max():.2e} "
          f"e_M max={em.max():.2e} mask flips={flips}")
    assert ez.max() <= MIXED_TOL and en.max() <= MIXED_TOL and em.max() <= MIXED_TOL


def test_singular_d_is_reported(torch_mod):
    from paper_2609_11363_amd import AsiError, Solver, upload_factors
    F = _case("lap32_tau1e-2")
    F.d_diag = F.d_diag.copy()
    F.d_diag[17] = 0.0
    s = Solver(0)
    s.analyze(F.n, F.L_rowptr, F.L_col, F.piv)
    Lv, dd, ds = upload_factors(F)
    s.selinv(Lv, dd, ds)
    with pytest.raises(AsiError) as ei:
        s.sync()
    assert ei.value.code in (3, 4)
    s.sync()  # the latched status was cleared


def test_small_pool_is_reported(torch_mod):
    from paper_2609_11363_amd import AsiError, Solver, upload_factors
    F = _case("lap32_tau0")
    s = Solver(0)
    s.analyze(F.n, F.L_rowptr, F.L_col, F.piv)
    info = s.info()
    s.set_workspace(info["workspace_min"])
    Lv, dd, ds = upload_factors(F)
    s.ninv(Lv, dd, ds, p=3, delta=0.0)
    with pytest.raises(AsiError) as ei:
        s.sync()
    assert ei.value.code == 6


@pytest.mark.parametrize("name", ["lap32_tau0", "kkt_tau0", "diff16_tau1e-3", "rand3000_tau1e-2"])
@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_sweep_schedules_agree(torch_mod, name, precision):
    """Level-by-level and dataflow sweeps both match the oracle."""
    from paper_2609_11363_amd import Solver, upload_factors
    print(f"[sweeps] case={name} precision={precision}", flush=True)
    F = _case(name)
    S = oc.pattern(F)
    Zo = oc.selinv(F, S)
    tol = FP64_TOL if precision == "fp64" else MIXED_TOL
    s = Solver(0)
    s.analyze(F.n, F.L_rowptr, F.L_col, F.piv)
    Lv, dd, ds = upload_factors(F)
    for mode in ("levels", "dataflow"):
        s.set_sweep(mode)
        for rep in range(2):  # the second call reuses the flags with a new epoch
            Z = s.selinv(Lv, dd, ds, precision=precision)
            s.sync()
            e = oc.entry_error(S, Z.cpu().numpy(), Zo).max()
            print(f"  {mode} call {rep}: e_Z={e:.2e}")
            assert e <= tol
