"""The trailing sub-factor (unknowns k..n-1) is a sub-problem of the method:
L is lower triangular, so SelInv's recursion for the blocks from k on reads
only rows and columns from k on (Section 2.1), and so do NInv's series
columns and their product (Section 2.2) and Mix (Section 2.3). The oracle on
the sub-factor must therefore give the trailing block of the oracle's whole
result exactly (same operations in the same order). The benchmark's CPU
baseline and its full-size parity check rest on this."""
import numpy as np
import pytest

from oracle import core as oc
from workloads import diffusion3d_7pt, ildl_bk, kkt_matrix, nested_multicolor_grid


@pytest.mark.parametrize("name", ["diff16", "kkt"])
def test_trailing_subfactor_gives_the_trailing_block(name):
    if name == "diff16":
        F = ildl_bk(diffusion3d_7pt(16, 1.0, 2), nested_multicolor_grid((16, 16, 16)), 1e-3)
    else:
        F = ildl_bk(kkt_matrix(60, 25, 3, density=0.15), None, 0.0)
        assert (F.piv == 1).any()
    S = oc.pattern(F)
    Z = oc.selinv(F, S)
    N = oc.ninv(F, S, 3, 0.1)
    M = oc.mix(S, Z, N, 1e-2)
    for frac in (0.1, 0.5):
        k = int(F.n * (1 - frac))
        while F.piv[k] == 2:
            k -= 1
        G = F.trailing(k)
        S2 = oc.pattern(G)
        for whole, sub in ((Z, oc.selinv(G, S2)), (N, oc.ninv(G, S2, 3, 0.1))):
            B = S.to_csr(whole)[k:, k:]
            B.sort_indices()
            np.testing.assert_array_equal(B.indptr, S2.rowptr)
            np.testing.assert_array_equal(B.indices, S2.col)
            np.testing.assert_array_equal(B.data, sub)
        B = S.to_csr(M)[k:, k:]
        B.sort_indices()
        Z2, N2 = oc.selinv(G, S2), oc.ninv(G, S2, 3, 0.1)
        np.testing.assert_array_equal(B.data, oc.mix(S2, Z2, N2, 1e-2))
