"""Block-diagonal sparsity (Section 5.3): the oracle of a scan over
block-diagonal products is the plain d x d matrix-product scan of the full
matrices (oracle.matd_scan / matd_scan_vjp on diag(M^0, ..., M^{k-1})).
These pins tie it to something else: the k block positions scanned on their
own by the independent C oracle (q = 1: scan of *, q = 2: the 2x2 product),
the vanishing off-diagonal blocks of every product, and the BDS rule itself
(the adjoint of block j needs only block j's Jacobians)."""
from __future__ import annotations

import numpy as np
import pytest

import oracle
from workloads import o2_matrices, orthogonal_matrices


def block_diag(B):
    """B (n, k, q, q) -> (n, k q, k q) block-diagonal matrices"""
    n, k, q, _ = B.shape
    M = np.zeros((n, k * q, k * q))
    for j in range(k):
        M[:, j * q:(j + 1) * q, j * q:(j + 1) * q] = B[:, j]
    return M


def diag_blocks(M, k, q):
    return np.stack([M[:, j * q:(j + 1) * q, j * q:(j + 1) * q] for j in range(k)], axis=1)


def blocks(rng, n, k, q):
    if q == 1:
        x = rng.choice([-1.0, 1.0], (n, k)) * np.exp(rng.uniform(-0.01, 0.01, (n, k)))
        return x.astype(np.float32).reshape(n, k, 1, 1)
    if q == 2:
        return o2_matrices(rng, n * k).reshape(n, k, 2, 2)
    return orthogonal_matrices(rng, n * k, q).reshape(n, k, q, q)


@pytest.mark.parametrize("q,k", [(1, 3), (2, 2), (2, 3), (3, 2), (2, 1)])
def test_full_scan_equals_blockwise_scans(q, k):
    rng = np.random.default_rng(100 * q + k)
    n = 257
    B = blocks(rng, n, k, q)
    Pb = rng.standard_normal((n, k, q, q)).astype(np.float32)
    M = block_diag(B.astype(np.float64))
    P, c = oracle.matd_scan(M)
    # off-diagonal blocks of every prefix product are exactly zero
    mask = block_diag(np.ones((1, k, q, q)))[0] == 0
    assert np.all(P[:, mask] == 0.0)
    PD = diag_blocks(P, k, q)
    # the full adjoint given a block-diagonal P_bar
    Mb, _ = oracle.matd_scan_vjp(M, block_diag(Pb.astype(np.float64)))
    MbD = diag_blocks(Mb, k, q)
    for j in range(k):
        if q == 1:
            rs, _ = oracle.scan_fwd("mul", B[:, j, 0, 0])
            np.testing.assert_allclose(PD[:, j, 0, 0], rs[:, 0], rtol=1e-12, atol=0)
            xb, _ = oracle.scan_vjp("mul", Pb[:, j, 0, 0], B[:, j, 0, 0])
            np.testing.assert_allclose(MbD[:, j, 0, 0], xb[:, 0], rtol=1e-10, atol=1e-12)
        elif q == 2:
            rs, _ = oracle.scan_fwd("mat2", B[:, j].reshape(n, 4))
            np.testing.assert_allclose(PD[:, j].reshape(n, 4), rs, rtol=1e-12, atol=1e-14)
            xb, _ = oracle.scan_vjp("mat2", Pb[:, j].reshape(n, 4), B[:, j].reshape(n, 4))
            np.testing.assert_allclose(MbD[:, j].reshape(n, 4), xb, rtol=1e-10, atol=1e-12)
        else:
            Pj, _ = oracle.matd_scan(B[:, j])
            np.testing.assert_allclose(PD[:, j], Pj, rtol=1e-12, atol=1e-14)
            Mj, _ = oracle.matd_scan_vjp(B[:, j], Pb[:, j])
            np.testing.assert_allclose(MbD[:, j], Mj, rtol=1e-10, atol=1e-12)
    # companion: the spectral norm of a block-diagonal matrix is its largest
    # block's, so c_i = prod_{t<=i} max_j ||M_t^j||_2
    norms = np.linalg.norm(B.astype(np.float64), 2, axis=(2, 3)).max(axis=1)
    np.testing.assert_allclose(c, np.cumprod(norms), rtol=1e-12)


def test_bds_adjoint_needs_only_its_blocks_jacobians():
    """The BDS rule: with M = diag(B^0, B^1), the adjoint of block 0 is
    unchanged when block 1's factors and output adjoint are replaced."""
    rng = np.random.default_rng(7)
    n, q = 120, 2
    B = blocks(rng, n, 2, q).astype(np.float64)
    Pb = rng.standard_normal((n, 2, q, q))
    Mb1, _ = oracle.matd_scan_vjp(block_diag(B), block_diag(Pb))
    B2, Pb2 = B.copy(), Pb.copy()
    B2[:, 1] = blocks(rng, n, 1, q)[:, 0]
    Pb2[:, 1] = rng.standard_normal((n, q, q))
    Mb2, _ = oracle.matd_scan_vjp(block_diag(B2), block_diag(Pb2))
    np.testing.assert_array_equal(diag_blocks(Mb1, 2, q)[:, 0], diag_blocks(Mb2, 2, q)[:, 0])
    assert not np.allclose(diag_blocks(Mb1, 2, q)[:, 1], diag_blocks(Mb2, 2, q)[:, 1])
