"""pcad_scan_vjp_noalloc (the scan adjoint whose look-back workspace is a
static device array) against pcad_scan_vjp with a caller's workspace, both
called through the C-ABI on the same inputs, two calls in a row with the
second on a smaller input (the array keeps the first call's status words).

Both results must pass the oracle's gate, and the two must agree within
twice its companion-scaled bound (they need not be bit-identical: which
predecessors a look-back finds already resolved depends on timing, and so
does the association of the sums it forms).
"""
from __future__ import annotations

import numpy as np
import pytest
import torch

import oracle
from oracle.gate import RTOL, assert_gate, chain_rtol

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


def inputs(op, n, rng):
    if op == "linrec":
        return (rng.uniform(0.9, 1.0, n).astype(np.float32),
                rng.standard_normal(n).astype(np.float32))
    if op == "mat2":
        from workloads import o2_matrices
        return o2_matrices(rng, n).reshape(n, 4), None
    if op == "mul":
        from workloads import mul_finite
        return mul_finite((n,), seed=int(rng.integers(1 << 30)))["x"], None
    x = rng.uniform(0.5, 2.0, n)
    if op in ("min", "max"):
        x = np.floor(x * 8) / 8
    return x.astype(np.float32), None


def noalloc_vjp(pcad, op, X0, X1, saved, YB, outs):
    st = torch.cuda.current_stream().cuda_stream
    n = X0.shape[0]
    return pcad.lib().pcad_scan_vjp_noalloc(
        pcad.OPS[op], 1, n, X0.data_ptr(), X1.data_ptr() if X1 is not None else None,
        saved.data_ptr(), YB.data_ptr(), None, outs[0].data_ptr(),
        outs[1].data_ptr() if len(outs) > 1 else None, 0, st)


@pytest.mark.parametrize("op", ["linrec", "add", "mul", "min", "max", "mat2"])
def test_scan_vjp_noalloc_matches_workspace_call(pcad, op):
    rng = np.random.default_rng(20231003 + pcad.OPS[op])
    # first call beyond one round of the persistent grid, second much smaller
    for n in (4_200_017, 30_011):
        x0, x1 = inputs(op, n, rng)
        yb = rng.standard_normal((n, 4) if op == "mat2" else n).astype(np.float32)
        X0, X1, YB = dev(x0), (dev(x1) if x1 is not None else None), dev(yb)
        _, _, saved = pcad.scan_fwd(op, X0, X1)
        ref = pcad.scan_vjp(op, X0, X1, saved, YB)
        ref = [host(t) for t in ref] if op == "linrec" else [host(ref)]
        outs = [torch.full_like(X0, np.nan)] + ([torch.full_like(X1, np.nan)] if op == "linrec" else [])
        st = noalloc_vjp(pcad, op, X0, X1, saved, YB, outs)
        assert st == 0, pcad.lib().pcad_status_string(st)
        got = [host(t) for t in outs]
        ybo = np.stack([np.zeros(n), yb], 1) if op == "linrec" else yb
        xb, cx = oracle.scan_vjp(op, ybo, x0, x1)
        rt = RTOL[op]
        if op in ("mul", "mat2"):  # products of up to n factors
            rt = chain_rtol(n, rt, width=4 if op == "mat2" else 1, adjoint=True)
        if op == "linrec":
            pairs = [(got[0], ref[0], xb[:, 0], cx[:, 0]), (got[1], ref[1], xb[:, 1], cx[:, 1])]
        elif op == "mat2":
            pairs = [(got[0], ref[0], xb, cx)]
        else:
            pairs = [(got[0], ref[0], xb[:, 0], cx[:, 0])]
        for g, r, o, c in pairs:
            assert_gate(g, o, c, rt, what=f"noalloc {op} n={n}")
            assert_gate(r, o, c, rt, what=f"workspace {op} n={n}")
            d = np.abs(g.astype(np.float64) - r.astype(np.float64))
            cc = c if c.shape == g.shape else np.repeat(c, 4).reshape(g.shape)
            assert np.all(d.reshape(-1) <= 2 * np.asarray(rt) * cc.reshape(-1) + 2.0 ** -125), (
                f"{op} n={n}: calls disagree")


def test_scan_vjp_noalloc_rejects_oversize(pcad):
    """A workspace beyond the static array is refused before any launch."""
    PCAD_E_SIZE = 5
    n = 1 << 28  # MAT2 at 2^28 elements needs about 12 MB of status words
    # null pointers: were the size not refused first, the call would fail
    # with PCAD_E_NULLPTR, still before any launch
    st = pcad.lib().pcad_scan_vjp_noalloc(pcad.OPS["mat2"], 1, n, None, None, None, None, None,
                                          None, None, 0, None)
    assert st == PCAD_E_SIZE
