"""Mix selection (Section 2.3) on the device: the two-entries-per-thread
kernel (16-byte aligned arrays) and the one-entry kernel (8-byte aligned
views) give the same bits, and the oracle's selection; the 7 x 7 case has an
odd number of entries (the tail entry done alone)."""
import numpy as np
import pytest

from oracle import core as oc
from workloads import ildl_bk, laplace2d, rcm

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("nx,ny", [(7, 7), (12, 13)])
def test_mix_aligned_and_unaligned(nx, ny):
    import torch
    from paper_2609_11363_amd import Solver, upload_factors
    A = laplace2d(nx, ny, 0.05)
    F = ildl_bk(A, rcm(A), 1e-2)
    S = oc.pattern(F)
    print(f"[mix] {nx}x{ny} |S|={S.nnz}", flush=True)
    Zo = oc.selinv(F, S)
    No = oc.ninv(F, S, 3, 0.1)
    s = Solver(0)
    s.analyze(F.n, F.L_rowptr, F.L_col, F.piv)
    dev = s.device
    Z = torch.as_tensor(Zo, device=dev)
    N = torch.as_tensor(No, device=dev)
    M = s.mix(Z, N, 1e-2)
    # the same values at an 8-byte offset
    buf = torch.zeros(3, S.nnz + 1, dtype=torch.float64, device=dev)
    buf[0, 1:] = Z
    buf[1, 1:] = N
    Mu = s.mix(buf[0, 1:], buf[1, 1:], 1e-2, out=buf[2, 1:])
    s.sync()
    assert buf[2, 1:].data_ptr() % 16 == 8
    assert torch.equal(M, Mu)
    np.testing.assert_array_equal(M.cpu().numpy(), oc.mix(S, Zo, No, 1e-2))
