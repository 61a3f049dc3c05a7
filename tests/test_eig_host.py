"""Host parts of the device eigen step (Section 2.5, Algorithm 1): the
library's Jacobi routine for the Lanczos iteration's projected problem
against LAPACK, a 2 x 2 closed form and degenerate inputs; the work size of
the device iteration against its stated layout."""
import ctypes

import numpy as np
import pytest

from paper_2609_11363_amd import AsiError, dense_symeig, load_library


@pytest.mark.parametrize("m", [1, 2, 3, 17, 64])
def test_dense_symeig_matches_lapack(m):
    rng = np.random.default_rng(m)
    B = rng.standard_normal((m, m))
    T = B + B.T
    theta, Y = dense_symeig(T)
    ref = np.linalg.eigvalsh(T)
    scale = max(1.0, np.abs(ref).max())
    assert np.abs(theta - ref).max() <= 1e-13 * scale
    assert np.abs(T @ Y - Y * theta).max() <= 1e-13 * scale
    assert np.abs(Y.T @ Y - np.eye(m)).max() <= 1e-13


def test_dense_symeig_closed_form_and_degenerate_inputs():
    a, b, d = 3.0, 2.0, -1.0
    theta, Y = dense_symeig(np.array([[a, b], [b, d]]))
    r = np.sqrt(((a - d) / 2) ** 2 + b * b)
    np.testing.assert_allclose(theta, [(a + d) / 2 - r, (a + d) / 2 + r], rtol=1e-15)
    # identity: repeated eigenvalues, the unit vectors (no rotation happens)
    theta, Y = dense_symeig(np.eye(5))
    assert np.array_equal(theta, np.ones(5)) and np.array_equal(Y, np.eye(5))
    # diagonal input: sorted ascending, ties by position
    theta, Y = dense_symeig(np.diag([2.0, -1.0, 2.0, 0.0]))
    assert np.array_equal(theta, [-1.0, 0.0, 2.0, 2.0])
    assert np.array_equal(np.argmax(np.abs(Y), axis=0), [1, 3, 0, 2])
    # an unsymmetric input is read as (T + T^T) / 2
    T = np.array([[1.0, 3.0], [1.0, 1.0]])
    theta, _ = dense_symeig(T)
    np.testing.assert_allclose(theta, [-1.0, 3.0], rtol=1e-15)
    with pytest.raises(AsiError):
        dense_symeig(np.array([[1.0, np.nan], [np.nan, 1.0]]))
    with pytest.raises(AsiError):
        dense_symeig(np.zeros((0, 0)))


def test_eigs_and_block_solve_work_bytes_layout():
    lib = load_library()
    out = ctypes.c_size_t(0)
    up = lambda x: (x + 31) // 32 * 32
    n = 100000
    dotb = min(1024, (n + 255) // 256)
    for nrhs in (1, 3, 8):
        assert lib.asi_block_solve_work_bytes(n, nrhs, ctypes.byref(out)) == 0
        solve = 7 * up(nrhs * n) + up(nrhs * dotb) + up(6 * nrhs) + up(2 * nrhs) + 2 * up(nrhs)
        assert out.value == 8 * solve
    assert lib.asi_block_solve_work_bytes(n, 9, ctypes.byref(out)) == 1
    for m, b in ((20, 1), (40, 4)):
        assert lib.asi_eigs_work_bytes(n, m, b, ctypes.byref(out)) == 0
        nb = max(1, min(1024, (n + 1023) // 1024))
        cols = m + b
        part = max(cols * nb, dotb)
        solve = 7 * up(b * n) + up(b * dotb) + up(6 * b) + up(2 * b) + 2 * up(b)
        expect = 8 * (2 * up(cols * n) + up(b * n) + up(part) + up(2 * cols + 1) + up(m * m) + solve)
        assert out.value == expect
    assert lib.asi_eigs_work_bytes(n, 257, 1, ctypes.byref(out)) == 1  # m above the basis limit
    assert lib.asi_eigs_work_bytes(n, 20, 9, ctypes.byref(out)) == 1   # block above 8
    assert lib.asi_eigs_work_bytes(1, 2, 1, ctypes.byref(out)) == 1
