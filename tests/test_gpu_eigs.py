"""GPU parity of the device eigen step (Section 2.5, Algorithm 1): the k
eigenpairs of largest |lambda| of E = Ah^-1 - X by the library's
thick-restart Lanczos iteration (A^-1 by PCG for positive definite A, by
SQMR for indefinite A, both preconditioned with the incomplete factor)
against the oracle's dense eigendecomposition of E: eigenvalues, the
spanned subspace, orthonormality and the true residual; repeatability bit
for bit; a second call with a smaller problem in the same work buffer; the
argument checks."""
import numpy as np
import pytest

from oracle import core as oc
from workloads import covariance_grid, ildl_bk, kkt_matrix, nested_multicolor_grid, shifted_laplace2d_indefinite

pytestmark = pytest.mark.gpu


def _case(name):
    if name == "cov20":      # positive definite, X = SelInv
        A = covariance_grid(20)
        F = ildl_bk(A, nested_multicolor_grid((20, 20)), 1e-3)
        return A, F, oc.selinv(F, oc.pattern(F))
    if name == "indef24":    # indefinite shifted Laplacian, X = Mix
        A, _ = shifted_laplace2d_indefinite(24, 4)
        F = ildl_bk(A, nested_multicolor_grid((24, 24)), 1e-2)
        S = oc.pattern(F)
        return A, F, oc.mix(S, oc.selinv(F, S), oc.ninv(F, S, 3, 0.1), 1e-2)
    A = kkt_matrix(60, 40, 3)  # saddle point with 2x2 pivots, X = NInv
    F = ildl_bk(A, None, 1e-2)
    return A, F, oc.ninv(F, oc.pattern(F), 3, 0.1)


def _setup(name):
    import torch
    from paper_2609_11363_amd import Solver, upload_factors
    A, F, X = _case(name)
    s = Solver(0)
    s.analyze(F.n, F.L_rowptr, F.L_col, F.piv)
    s.load_factor(*upload_factors(F))
    dev = s.device
    t = lambda a, dt: torch.as_tensor(np.ascontiguousarray(a, dtype=dt), device=dev)
    args = (t(A.indptr, np.int64), t(A.indices, np.int32), t(A.data, np.float64), t(F.perm, np.int32),
            t(X, np.float64))
    return A, F, X, s, args


def _check(A, F, X, lam, V, k, rtol):
    S = oc.pattern(F)
    Ah = oc.permuted(A, F.perm)
    lam_o, V_o = oc.error_eigenpairs(Ah, S, X, k)
    E = np.linalg.inv(Ah.toarray()) - S.to_csr(X).toarray()
    Vd = V.cpu().numpy()
    lam_err = np.abs(lam - lam_o).max() / np.abs(lam_o).max()
    orth = np.abs(Vd.T @ Vd - np.eye(k)).max()
    sv = np.linalg.svd(Vd.T @ V_o, compute_uv=False).min()
    res = max(np.linalg.norm(E @ Vd[:, t] - lam[t] * Vd[:, t]) / abs(lam[t]) for t in range(k))
    print(f"  lambda {lam} (oracle {lam_o}); rel err {lam_err:.1e}, orth {orth:.1e}, subspace {sv:.12f}, "
          f"residual {res:.1e}", flush=True)
    assert lam_err <= rtol
    assert orth <= 1e-10
    assert sv >= 1 - 1e-6
    assert res <= 1e-6


@pytest.mark.parametrize("name,method,k,m,block", [("cov20", "cg", 3, 20, 1), ("cov20", "cg", 6, 14, 1),
                                                   ("indef24", "sqmr", 3, 20, 1), ("kkt", "sqmr", 2, 16, 1),
                                                   ("cov20", "cg", 3, 24, 4), ("cov20", "cg", 6, 21, 3),
                                                   ("indef24", "sqmr", 3, 24, 4), ("kkt", "sqmr", 2, 16, 8)])
def test_eigs_matches_oracle(name, method, k, m, block):
    A, F, X, s, args = _setup(name)
    print(f"[eigs] {name} n={F.n} method={method} k={k} m={m} block={block}", flush=True)
    solve_tol = 1e-12 if method == "cg" else 1e-11
    lam, V, res, st = s.eigs_error(*args, k, m=m, block=block, tol=1e-10, method=method, solve_tol=solve_tol,
                                   solve_maxit=3000)
    s.sync()
    print(f"  stats {st}, estimated residuals {res}", flush=True)
    assert st["converged"] == k and st["max_solve_relres"] <= solve_tol
    assert np.all(np.diff(np.abs(lam)) <= 0)
    _check(A, F, X, lam, V, k, 1e-8 if method == "cg" else 1e-6)


def test_eigs_repeatable_and_second_smaller_call():
    import torch
    A, F, X, s, args = _setup("cov20")
    print(f"[eigs] repeat cov20 n={F.n}", flush=True)
    work = torch.empty(F.n * 64, dtype=torch.float64, device=s.device)
    lam1, V1, _, st1 = s.eigs_error(*args, 4, m=16, work=work)
    lam2, V2, _, st2 = s.eigs_error(*args, 4, m=16, work=work)
    s.sync()
    assert np.array_equal(lam1, lam2) and torch.equal(V1, V2) and st1 == st2
    # a smaller problem in the same (dirty) work buffer
    lam3, V3, _, st3 = s.eigs_error(*args, 2, m=8, work=work, tol=1e-10)
    s.sync()
    assert st3["converged"] == 2
    _check(A, F, X, lam3, V3, 2, 1e-8)


def test_eigs_argument_checks():
    import torch
    from paper_2609_11363_amd import AsiError, Solver
    A, F, X, s, args = _setup("cov20")
    with pytest.raises(AsiError, match="ASI_E_ARG"):
        s.eigs_error(*args, 3, m=4)                      # m < k + 2
    with pytest.raises(AsiError, match="ASI_E_ARG"):
        s.eigs_error(*args, 3, m=7, block=4)             # m < k + block + 1
    with pytest.raises(AsiError, match="ASI_E_ARG"):    # dependent start columns
        s.eigs_error(*args, 2, m=12, block=2, v0=torch.ones((2, F.n), dtype=torch.float64, device=s.device))
    with pytest.raises(AsiError, match="ASI_E_ARG"):
        s.eigs_error(*args, 65, m=200)                   # k > 64
    with pytest.raises(AsiError, match="ASI_E_ARG"):
        s.eigs_error(*args, 1, v0=torch.zeros(F.n, dtype=torch.float64, device=s.device))
    s2 = Solver(0)
    s2.analyze(F.n, F.L_rowptr, F.L_col, F.piv)
    with pytest.raises(AsiError, match="ASI_E_STATE"):  # no factor loaded
        s2.eigs_error(*args, 2, m=8)
    import ctypes
    small = torch.empty(1024, dtype=torch.float64, device=s.device)
    lam = np.zeros(2)
    V = torch.empty((F.n, 2), dtype=torch.float64, device=s.device)
    v0 = torch.ones(F.n, dtype=torch.float64, device=s.device)
    p = lambda x: ctypes.c_void_p(x.data_ptr())
    rc = s.lib.asi_eigs_error(s.h, *[p(a) for a in args], p(v0), 2, 8, 1, 1e-8, 10, 0, 1e-12, 100, p(small),
                              small.numel() * 8, lam.ctypes.data_as(ctypes.c_void_p), p(V), None, None)
    assert rc == 6  # ASI_E_WORKSPACE


def test_eigs_edge_cases():
    """The smallest basis a block allows (m = k + b + 1), a run stopped by
    max_restarts = 0 before convergence (it returns its best Ritz pairs with
    honest residual estimates), and k = 1 with b = 1."""
    A, F, X, s, args = _setup("cov20")
    print(f"[eigs] edge cases n={F.n}", flush=True)
    # minimal basis for k = 1, b = 2
    lam, V, res, st = s.eigs_error(*args, 1, m=4, block=2, tol=1e-9, max_restarts=500)
    s.sync()
    print(f"  m=4 b=2: {lam} {st}", flush=True)
    assert st["converged"] == 1
    _check(A, F, X, lam, V, 1, 1e-7)
    # stopped early: the estimates say so
    lam0, V0, res0, st0 = s.eigs_error(*args, 3, m=8, block=1, tol=1e-14, max_restarts=0)
    s.sync()
    print(f"  max_restarts=0: {lam0} residual estimates {res0} {st0}", flush=True)
    assert st0["restarts"] == 0 and st0["applications"] == 8
    assert np.all(np.isfinite(lam0)) and np.all(res0 >= 0)
    assert st0["converged"] == int((res0 <= 1e-14).sum())
    Vd = V0.cpu().numpy()
    assert np.abs(Vd.T @ Vd - np.eye(3)).max() <= 1e-10
    S = oc.pattern(F)
    E = np.linalg.inv(oc.permuted(A, F.perm).toarray()) - S.to_csr(X).toarray()
    true = [np.linalg.norm(E @ Vd[:, t] - lam0[t] * Vd[:, t]) / abs(lam0[t]) for t in range(3)]
    np.testing.assert_allclose(true, res0, rtol=1e-3, atol=1e-9)  # the estimates are the true residuals
    # k = 1, b = 1
    lam1, V1, _, st1 = s.eigs_error(*args, 1, m=6, tol=1e-10)
    s.sync()
    assert st1["converged"] == 1
    _check(A, F, X, lam1, V1, 1, 1e-8)
