"""asi_unpermute_noalloc (static device scratch, no allocation) against
asi_unpermute (workspace scratch), through the C ABI.

Two calls in a row, the second with a smaller input, so the second reuses a
scratch that still holds the first call's inverse permutation; both must
equal the workspace variant bit for bit (the operation is index work and a
copy of values). Sizes above the static scratch are refused synchronously.
"""
import ctypes

import numpy as np
import pytest

from workloads import diffusion3d_7pt, ildl_bk, laplace2d, nested_multicolor_grid, rcm
from workloads.ildl import IldlFactors

pytestmark = pytest.mark.gpu


def _ptr(t):
    return ctypes.c_void_p(t.data_ptr())


def _both(F):
    import torch
    from paper_2609_11363_amd import Solver, upload_factors
    s = Solver(0)
    s.analyze(F.n, F.L_rowptr, F.L_col, F.piv)
    Z = s.selinv(*upload_factors(F))
    perm = torch.as_tensor(F.perm.astype(np.int32), device=s.device)
    ref = s.unpermute(perm, Z)
    out = (torch.full((F.n + 1,), -7, dtype=torch.int64, device=s.device),
           torch.full((s.nnz_S,), -7, dtype=torch.int32, device=s.device),
           torch.full((s.nnz_S,), np.nan, dtype=torch.float64, device=s.device))
    s._stream()
    rc = s.lib.asi_unpermute_noalloc(s.h, _ptr(perm), _ptr(Z), *(_ptr(t) for t in out))
    assert rc == 0, s.lib.asi_last_error(s.h)
    s.sync()
    return s, ref, out


def test_noalloc_matches_workspace_variant_twice():
    import torch
    cases = [("diff16", lambda: ildl_bk(diffusion3d_7pt(16, 1.0, 2), nested_multicolor_grid((16, 16, 16)), 1e-3)),
             ("lap32", lambda: (lambda A: ildl_bk(A, rcm(A), 1e-2))(laplace2d(32, 32, 0.01)))]
    sizes = []
    for name, make in cases:
        print(f"[noalloc] case={name}", flush=True)
        F = make()
        s, ref, out = _both(F)
        sizes.append(F.n)
        for a, b in zip(ref, out):
            assert torch.equal(a, b), name
    assert sizes[1] < sizes[0]


def test_noalloc_refuses_sizes_above_its_scratch():
    from paper_2609_11363_amd import Solver
    import torch
    n = (1 << 21) + 1
    F = IldlFactors(n=n, perm=np.arange(n, dtype=np.int32), L_rowptr=np.zeros(n + 1, np.int64),
                    L_col=np.zeros(0, np.int32), L_val=np.zeros(0), d_diag=np.ones(n), d_sub=np.zeros(n),
                    piv=np.zeros(n, np.int8), tau=0.0)
    s = Solver(0)
    s.analyze(F.n, F.L_rowptr, F.L_col, F.piv)
    X = torch.ones(s.nnz_S, dtype=torch.float64, device=s.device)
    perm = torch.arange(n, dtype=torch.int32, device=s.device)
    rp = torch.empty(n + 1, dtype=torch.int64, device=s.device)
    cl = torch.empty(s.nnz_S, dtype=torch.int32, device=s.device)
    vl = torch.empty(s.nnz_S, dtype=torch.float64, device=s.device)
    rc = s.lib.asi_unpermute_noalloc(s.h, _ptr(perm), _ptr(X), _ptr(rp), _ptr(cl), _ptr(vl))
    assert rc == 1
    assert b"2,097,152" in s.lib.asi_last_error(s.h)
    s.sync()
