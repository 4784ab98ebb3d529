"""Scans of block-diagonal matrix products (Section 5.3, Block-Diagonal
Sparsity) through the C-ABI, against the oracle's plain d x d product scan
of the full block-diagonal matrices (d = k q): P's blocks and the diagonal
blocks of M_bar, over several tiles with ragged tails, batched rows, and
PCAD_ACCUMULATE.  Factors are orthogonal blocks (q >= 2) or multipliers
+-exp(U[-0.01, 0.01]) (q = 1), so products neither overflow nor underflow and
every output is gated element by element."""
from __future__ import annotations

import numpy as np
import pytest
import torch

import oracle
from oracle.gate import RTOL, assert_discriminates, assert_gate
from test_oracle_bds import block_diag, blocks, diag_blocks

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def pcad():
    import paper_2310_03568_amd as p
    p.lib()
    assert torch.cuda.is_available()
    return p


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def host(t):
    torch.cuda.synchronize()
    return t.cpu().numpy()


def block_companions(B, Pb):
    """Companions of every block position's own scan (n, k), forward and
    adjoint: the norm-wise companion of the full d x d product takes the
    largest block's norm at every factor, which compounds far beyond any
    one block's products, so each block is gated with the companion of its
    own q x q scan (the same bound, taken block by block)."""
    n, k, q, _ = B.shape
    cf, cb = np.empty((n, k)), np.empty((n, k))
    for j in range(k):
        if q == 1:
            _, c = oracle.scan_fwd("mul", B[:, j, 0, 0])
            cf[:, j] = c[:, 0]
            _, c = oracle.scan_vjp("mul", Pb[:, j, 0, 0], B[:, j, 0, 0])
            cb[:, j] = c[:, 0]
        elif q == 2:
            _, c = oracle.scan_fwd("mat2", B[:, j].reshape(n, 4))
            cf[:, j] = c.max(axis=1)
            _, c = oracle.scan_vjp("mat2", Pb[:, j].reshape(n, 4), B[:, j].reshape(n, 4))
            cb[:, j] = c.max(axis=1)
        else:
            _, cf[:, j] = oracle.matd_scan(B[:, j])
            _, cb[:, j] = oracle.matd_scan_vjp(B[:, j], Pb[:, j])
    return cf, cb


def gate_blocks(g, r, c, k, q, what):
    """g (n, k, q, q) float32 against the blocks of the oracle's d x d r
    (n, d, d), companions c (n, k) per block"""
    n = g.shape[0]
    rb = diag_blocks(r, k, q)
    cc = np.broadcast_to(c[:, :, None, None], rb.shape)
    assert_gate(g, rb, cc, RTOL["mat2"], what=what)
    if n > 600:
        assert_discriminates(g.reshape(n, -1), rb.reshape(n, -1), cc.reshape(n, -1),
                             RTOL["mat2"], width=k * q * q, what=what)


@pytest.mark.parametrize("q,k,batch,n", [(2, 2, 1, 1), (2, 2, 1, 9000), (2, 3, 2, 4097),
                                         (1, 4, 1, 30_011), (1, 2, 3, 8193),
                                         (3, 2, 1, 3000), (5, 2, 2, 1100), (3, 1, 1, 2049)])
def test_bds_scan(pcad, q, k, batch, n):
    rng = np.random.default_rng(1000 * q + 10 * k + batch)
    B = np.stack([blocks(rng, n, k, q) for _ in range(batch)])
    Pb = rng.standard_normal(B.shape).astype(np.float32)
    print(f"bds q={q} k={k} batch={batch} n={n}", flush=True)
    M = dev(B)
    P, saved = pcad.bds_scan_fwd(M)
    Mb = pcad.bds_scan_vjp(M, saved, dev(Pb))
    P, Mb = host(P), host(Mb)
    for r in range(batch):
        Mfull = block_diag(B[r].astype(np.float64))
        cf, cb = block_companions(B[r], Pb[r])
        rs, _ = oracle.matd_scan(Mfull)
        gate_blocks(P[r], rs, cf, k, q, f"bds fwd row {r}")
        xb, _ = oracle.matd_scan_vjp(Mfull, block_diag(Pb[r].astype(np.float64)))
        gate_blocks(Mb[r], xb, cb, k, q, f"bds vjp row {r}")


def test_bds_accumulate_and_errors(pcad):
    rng = np.random.default_rng(3)
    n, k, q = 5000, 2, 2
    B = blocks(rng, n, k, q)
    Pb = rng.standard_normal(B.shape).astype(np.float32)
    M = dev(B)
    P, saved = pcad.bds_scan_fwd(M)
    ref = host(pcad.bds_scan_vjp(M, saved, dev(Pb)))
    out = dev(np.full(B.shape, 0.5, np.float32))
    pcad.bds_scan_vjp(M, saved, dev(Pb), out=out, accumulate=True)
    np.testing.assert_allclose(host(out), ref + 0.5, rtol=0, atol=2e-6)
    # empty rows: nothing to do
    E = torch.empty((0, 3, 2, 2), device="cuda")
    P0, _ = pcad.bds_scan_fwd(E)
    assert P0.shape == E.shape
    # unsupported block size and too many block floats are refused
    st = pcad.lib().pcad_bds_query(4, 2, 1, 10, 0, None, None, None, None)
    assert st == 1  # PCAD_E_INVALID_ARG
    st = pcad.lib().pcad_bds_query(5, 200, 1, 10, 0, None, None, None, None)
    assert st == 5  # PCAD_E_SIZE
