"""GPU parity of the eigen step's operator applications (Section 2.5): y = X x
on S, the preconditioner solve (L D L^T)^-1 x by the level schedule (1x1 and
2x2 pivots, blocks of both record kinds), conjugate gradients on P^T A P
preconditioned by the factor, and the eigenpairs of A^-1 - X computed with
those device solves against the same computation with a host direct solver."""
import numpy as np
import pytest
import scipy.sparse as sp

from oracle import core as oc
from workloads import (covariance_grid, diffusion3d_7pt, ildl_bk, kkt_matrix, nested_multicolor_grid,
                       stencil27_3d)

pytestmark = pytest.mark.gpu


def _case(name):
    if name == "cov20":
        A = covariance_grid(20)
        return A, ildl_bk(A, nested_multicolor_grid((20, 20)), 1e-3)
    if name == "diff12":
        A = diffusion3d_7pt(12, 1.0, 2)
        return A, ildl_bk(A, nested_multicolor_grid((12, 12, 12)), 1e-3)
    if name == "st27_tight":  # blocks with |R_J| > 128 (the large-block records)
        A = stencil27_3d(10, 0.5, 3)
        return A, ildl_bk(A, nested_multicolor_grid((10, 10, 10)), 1e-5)
    A = kkt_matrix(60, 40, 3)
    return A, ildl_bk(A, None, 1e-2)


@pytest.mark.parametrize("name", ["cov20", "diff12", "st27_tight", "kkt"])
def test_spmv_and_ldl_solve(name):
    import torch
    from paper_2609_11363_amd import Solver, upload_factors
    A, F = _case(name)
    S = oc.pattern(F)
    s = Solver(0)
    s.analyze(F.n, F.L_rowptr, F.L_col, F.piv)
    info = s.info()
    print(f"[solve] {name} n={F.n} levels={info['n_levels']} max|R_J|={info['max_cols']} 2x2={F.n_2x2}", flush=True)
    Lv, dd, ds = upload_factors(F)
    dev = s.device
    rng = np.random.default_rng(5)
    X = rng.standard_normal(S.nnz)
    x = rng.standard_normal(F.n)
    xt = torch.as_tensor(x, device=dev)
    y = s.spmv(torch.as_tensor(X, device=dev), xt)
    s.load_factor(Lv, dd, ds)
    z = s.ldl_solve(xt)
    z2 = s.ldl_solve(xt)
    zi = xt.clone()
    s.ldl_solve(zi, zi)  # in place
    s.sync()
    yo = oc.spmv(S, X, x)
    np.testing.assert_allclose(y.cpu().numpy(), yo, rtol=1e-12, atol=1e-13 * np.abs(yo).max())
    zo = oc.ldl_solve(F, x)
    err = np.abs(z.cpu().numpy() - zo).max() / np.abs(zo).max()
    print(f"  spmv ok; ldl solve max rel error {err:.1e}")
    assert err <= 1e-11
    assert torch.equal(z, z2) and torch.equal(z, zi)


@pytest.mark.parametrize("name", ["cov20", "diff12"])
def test_pcg(name):
    import torch
    from paper_2609_11363_amd import Solver, upload_factors
    A, F = _case(name)
    s = Solver(0)
    s.analyze(F.n, F.L_rowptr, F.L_col, F.piv)
    Lv, dd, ds = upload_factors(F)
    s.load_factor(Lv, dd, ds)
    dev = s.device
    Ar = torch.as_tensor(A.indptr.astype(np.int64), device=dev)
    Ac = torch.as_tensor(A.indices.astype(np.int32), device=dev)
    Av = torch.as_tensor(A.data, device=dev)
    perm = torch.as_tensor(F.perm.astype(np.int32), device=dev)
    b = np.random.default_rng(7).standard_normal(F.n)
    x, it, rr = s.pcg(Ar, Ac, Av, perm, torch.as_tensor(b, device=dev), tol=1e-12, maxit=500)
    s.sync()
    Ah = oc.permuted(A, F.perm)
    xo = sp.linalg.spsolve(sp.csc_matrix(Ah), b)
    err = np.abs(x.cpu().numpy() - xo).max() / np.abs(xo).max()
    res = np.linalg.norm(Ah @ x.cpu().numpy() - b) / np.linalg.norm(b)
    print(f"[pcg] {name}: {it} steps, reported {rr:.1e}, true residual {res:.1e}, error {err:.1e}")
    assert rr <= 1e-12 and res <= 1e-11 and err <= 1e-9
    # with other work on the stream between calls, a second call repeats the
    # first bit for bit
    bd = torch.as_tensor(b, device=dev)
    ze = s.ldl_solve(bd)
    x2, it2, rr2 = s.pcg(Ar, Ac, Av, perm, bd, tol=1e-12, maxit=500)
    ze2 = s.ldl_solve(bd)
    s.sync()
    assert torch.equal(x, x2) and it2 == it and rr2 == rr and torch.equal(ze, ze2)
    # zero right-hand side: zero steps, zero solution
    x0, it0, _ = s.pcg(Ar, Ac, Av, perm, torch.zeros(F.n, dtype=torch.float64, device=dev))
    s.sync()
    assert it0 == 0 and not x0.abs().max().item()


def test_eigenpairs_with_device_solves_match_host():
    import scipy.sparse.linalg as spla
    import torch
    from paper_2609_11363_amd import Solver, upload_factors
    from paper_2609_11363_amd.spectral import inverse_error_eigenpairs
    A, F = _case("cov20")
    S = oc.pattern(F)
    s = Solver(0)
    s.analyze(F.n, F.L_rowptr, F.L_col, F.piv)
    Lv, dd, ds = upload_factors(F)
    s.load_factor(Lv, dd, ds)
    dev = s.device
    Ar = torch.as_tensor(A.indptr.astype(np.int64), device=dev)
    Ac = torch.as_tensor(A.indices.astype(np.int32), device=dev)
    Av = torch.as_tensor(A.data, device=dev)
    perm = torch.as_tensor(F.perm.astype(np.int32), device=dev)
    Zo = oc.selinv(F, S)
    X = S.to_csr(Zo)

    def dev_inv(v):
        x, _, _ = s.pcg(Ar, Ac, Av, perm, torch.as_tensor(np.ascontiguousarray(v), device=dev), tol=1e-13, maxit=500)
        return x.cpu().numpy()

    lu = spla.splu(sp.csc_matrix(oc.permuted(A, F.perm)))
    lam_d, V_d, res_d, _ = inverse_error_eigenpairs(dev_inv, X, 3, tol=1e-10, seed=0)
    lam_h, V_h, res_h, _ = inverse_error_eigenpairs(lu.solve, X, 3, tol=1e-10, seed=0)
    print(f"[eig] device {lam_d} host {lam_h}")
    np.testing.assert_allclose(lam_d, lam_h, rtol=1e-8)
    # the spanned subspaces agree (degenerate eigenvalues make single vectors arbitrary)
    sv = np.linalg.svd(V_d.T @ V_h, compute_uv=False)
    assert sv.min() >= 1 - 1e-6


@pytest.mark.parametrize("name", ["indef24", "kkt", "cov20"])
def test_sqmr(name):
    import torch
    from paper_2609_11363_amd import Solver, upload_factors
    from workloads import shifted_laplace2d_indefinite
    if name == "indef24":
        A, _ = shifted_laplace2d_indefinite(24, 4)
        F = ildl_bk(A, nested_multicolor_grid((24, 24)), 1e-2)
    else:
        A, F = _case(name)
    s = Solver(0)
    s.analyze(F.n, F.L_rowptr, F.L_col, F.piv)
    Lv, dd, ds = upload_factors(F)
    s.load_factor(Lv, dd, ds)
    dev = s.device
    Ar = torch.as_tensor(A.indptr.astype(np.int64), device=dev)
    Ac = torch.as_tensor(A.indices.astype(np.int32), device=dev)
    Av = torch.as_tensor(A.data, device=dev)
    perm = torch.as_tensor(F.perm.astype(np.int32), device=dev)
    b = np.random.default_rng(9).standard_normal(F.n)
    x, it, rr = s.sqmr(Ar, Ac, Av, perm, torch.as_tensor(b, device=dev), tol=1e-11, maxit=2000)
    s.sync()
    Ah = oc.permuted(A, F.perm)
    xo = sp.linalg.spsolve(sp.csc_matrix(Ah), b)
    xg = x.cpu().numpy()
    res = np.linalg.norm(Ah @ xg - b) / np.linalg.norm(b)
    err = np.abs(xg - xo).max() / np.abs(xo).max()
    print(f"[sqmr] {name}: {it} steps, reported {rr:.1e}, true residual {res:.1e}, error {err:.1e}")
    assert rr <= 1e-11 and res <= 2e-11
    cond = np.linalg.cond(Ah.toarray())
    assert err <= 1e-11 * cond * 10


def test_sqmr_restarts_when_the_true_residual_stalls():
    """A right-hand side made of the eigenvectors of Ah nearest zero (an
    indefinite 48 x 48 shifted Laplacian, condition ~2e3) and a tolerance
    close to the attainable accuracy: the recursion's quasi-residual keeps
    falling while the true residual stalls just above 1e-12, so without a
    fresh recursion from the iterate SQMR never meets the tolerance (a
    float64 host run of the same steps stalls for 2,000 steps; with the
    restart it stops after 150). The block form takes the same restarts:
    each of its columns equals the one-vector solve bit for bit."""
    import torch
    from paper_2609_11363_amd import Solver, upload_factors
    from workloads import shifted_laplace2d_indefinite
    A, _ = shifted_laplace2d_indefinite(48, 20)
    F = ildl_bk(A, nested_multicolor_grid((48, 48)), 1e-2)
    Ah = oc.permuted(A, F.perm)
    w, V = np.linalg.eigh(Ah.toarray())
    near = np.argsort(np.abs(w))[:8]
    rng = np.random.default_rng(3)
    B = np.stack([V[:, near] @ rng.standard_normal(8) + 1e-3 * rng.standard_normal(F.n) for _ in range(3)])
    s = Solver(0)
    s.analyze(F.n, F.L_rowptr, F.L_col, F.piv)
    s.load_factor(*upload_factors(F))
    dev = s.device
    Ar = torch.as_tensor(A.indptr.astype(np.int64), device=dev)
    Ac = torch.as_tensor(A.indices.astype(np.int32), device=dev)
    Av = torch.as_tensor(A.data, device=dev)
    perm = torch.as_tensor(F.perm.astype(np.int32), device=dev)
    Bt = torch.as_tensor(B, device=dev)
    tol, maxit = 1e-12, 600
    print(f"[sqmr stall] n={F.n} cond={np.abs(w).max() / np.abs(w).min():.0f} tol={tol:g}", flush=True)
    X, iters, rel = s.sqmr_block(Ar, Ac, Av, perm, Bt, tol=tol, maxit=maxit)
    s.sync()
    for v in range(3):
        x1, it1, rr1 = s.sqmr(Ar, Ac, Av, perm, Bt[v].contiguous(), tol=tol, maxit=maxit)
        s.sync()
        res = np.linalg.norm(Ah @ x1.cpu().numpy() - B[v]) / np.linalg.norm(B[v])
        print(f"  vector {v}: {it1} steps, reported {rr1:.1e}, true {res:.1e}", flush=True)
        assert rr1 <= tol and it1 < maxit and res <= 2 * tol
        assert torch.equal(X[v], x1) and iters[v] == it1 and rel[v] == rr1


@pytest.mark.parametrize("name", ["cov20", "kkt"])
def test_za_diag(name):
    import torch
    from paper_2609_11363_amd import Solver
    A, F = _case(name)
    S = oc.pattern(F)
    Z = oc.ninv(F, S, 3, 0.1)  # an approximation whose (Z Ah)_ii are not all 1
    s = Solver(0)
    s.analyze(F.n, F.L_rowptr, F.L_col, F.piv)
    dev = s.device
    d = s.za_diag(torch.as_tensor(A.indptr.astype(np.int64), device=dev),
                  torch.as_tensor(A.indices.astype(np.int32), device=dev), torch.as_tensor(A.data, device=dev),
                  torch.as_tensor(F.perm.astype(np.int32), device=dev), torch.as_tensor(Z, device=dev))
    s.sync()
    want = oc.za_diag(S, Z, oc.permuted(A, F.perm))
    np.testing.assert_allclose(d.cpu().numpy(), want, rtol=1e-12, atol=1e-14)


@pytest.mark.parametrize("name,method,nrhs", [("cov20", "cg", 3), ("diff12", "cg", 8), ("indef24", "sqmr", 4),
                                              ("kkt", "sqmr", 2)])
def test_block_solves_equal_single_solves(name, method, nrhs):
    """Several right-hand sides at once: each column equals the one-vector
    solve bit for bit (same kernels' arithmetic, per-vector scalars and
    stopping), including a zero column that never starts."""
    import torch
    from paper_2609_11363_amd import Solver, upload_factors
    from workloads import shifted_laplace2d_indefinite
    if name == "indef24":
        A, _ = shifted_laplace2d_indefinite(24, 4)
        F = ildl_bk(A, nested_multicolor_grid((24, 24)), 1e-2)
    else:
        A, F = _case(name)
    s = Solver(0)
    s.analyze(F.n, F.L_rowptr, F.L_col, F.piv)
    s.load_factor(*upload_factors(F))
    dev = s.device
    Ar = torch.as_tensor(A.indptr.astype(np.int64), device=dev)
    Ac = torch.as_tensor(A.indices.astype(np.int32), device=dev)
    Av = torch.as_tensor(A.data, device=dev)
    perm = torch.as_tensor(F.perm.astype(np.int32), device=dev)
    B = np.random.default_rng(11).standard_normal((nrhs, F.n))
    B[nrhs - 1] = 0.0
    Bt = torch.as_tensor(B, device=dev)
    tol = 1e-11
    print(f"[block] {name} {method} nrhs={nrhs} n={F.n}", flush=True)
    blk = s.pcg_block if method == "cg" else s.sqmr_block
    one = s.pcg if method == "cg" else s.sqmr
    X, iters, rel = blk(Ar, Ac, Av, perm, Bt, tol=tol, maxit=3000)
    s.sync()
    Ah = oc.permuted(A, F.perm)
    for v in range(nrhs):
        x1, it1, rr1 = one(Ar, Ac, Av, perm, Bt[v].contiguous(), tol=tol, maxit=3000)
        s.sync()
        print(f"  vector {v}: block {iters[v]} steps {rel[v]:.1e}, single {it1} steps {rr1:.1e}", flush=True)
        assert torch.equal(X[v], x1) and iters[v] == it1 and rel[v] == rr1
        if v < nrhs - 1:
            xg = X[v].cpu().numpy()
            assert np.linalg.norm(Ah @ xg - B[v]) / np.linalg.norm(B[v]) <= 2 * tol
    assert not X[nrhs - 1].abs().max().item() and iters[nrhs - 1] == 0


def test_block_solve_edge_cases():
    """One right-hand side (equal to asi_pcg bit for bit), maxit = 0 (X = 0,
    no steps), and the argument checks (nrhs above 8, work too small)."""
    import ctypes

    import torch
    from paper_2609_11363_amd import AsiError, Solver, upload_factors
    A, F = _case("cov20")
    s = Solver(0)
    s.analyze(F.n, F.L_rowptr, F.L_col, F.piv)
    s.load_factor(*upload_factors(F))
    dev = s.device
    Ar = torch.as_tensor(A.indptr.astype(np.int64), device=dev)
    Ac = torch.as_tensor(A.indices.astype(np.int32), device=dev)
    Av = torch.as_tensor(A.data, device=dev)
    perm = torch.as_tensor(F.perm.astype(np.int32), device=dev)
    B = torch.as_tensor(np.random.default_rng(13).standard_normal((1, F.n)), device=dev)
    print(f"[block] edge cases n={F.n}", flush=True)
    X, iters, rel = s.pcg_block(Ar, Ac, Av, perm, B, tol=1e-12, maxit=500)
    x1, it1, rr1 = s.pcg(Ar, Ac, Av, perm, B[0].contiguous(), tol=1e-12, maxit=500)
    s.sync()
    assert torch.equal(X[0], x1) and iters[0] == it1 and rel[0] == rr1
    X0, it0, _ = s.sqmr_block(Ar, Ac, Av, perm, B, tol=1e-12, maxit=0)
    s.sync()
    assert it0[0] == 0 and not X0.abs().max().item()
    with pytest.raises(AsiError, match="ASI_E_ARG"):
        s.pcg_block(Ar, Ac, Av, perm, torch.zeros((9, F.n), dtype=torch.float64, device=dev))
    small = torch.empty(64, dtype=torch.float64, device=dev)
    Xs = torch.empty((1, F.n), dtype=torch.float64, device=dev)
    it = np.zeros(1, dtype=np.int32)
    rr = np.zeros(1)
    p = lambda t: ctypes.c_void_p(t.data_ptr())
    rc = s.lib.asi_pcg_block(s.h, p(Ar), p(Ac), p(Av), p(perm), 1, p(B), p(Xs), 1e-10, 10, p(small), 512,
                             it.ctypes.data_as(ctypes.c_void_p), rr.ctypes.data_as(ctypes.c_void_p))
    assert rc == 6  # ASI_E_WORKSPACE
