"""The comparison gate and the parity ensembles, on the CPU.

A parity test is only as strict as its inputs let it be: on inputs whose
outputs under- or overflow float32, an output that stopped being computed
after a few hundred elements passes the gate.  These tests show, with the
oracle's own float32-rounded results standing in for a GPU result, that the
ensembles the GPU tests use make the gate reject such an output, and that
the workload ensembles they replace do not.
"""
from __future__ import annotations

import numpy as np
import pytest

import oracle
from oracle.gate import RTOL, assert_discriminates, assert_gate, gate


def as32(r):
    return np.asarray(r).astype(np.float32)


def test_gaussian_mat2_products_are_vacuous_and_o2_are_not():
    from workloads import mat2
    n = 20_000
    for ens, vacuous in (("gauss", True), ("o2", False)):
        w = mat2(n=n, ensemble=ens)
        rs, c = oracle.scan_fwd("mat2", w["M"])
        xb, cx = oracle.scan_vjp("mat2", w["Pbar"], w["M"])
        assert_gate(as32(rs), rs, c, RTOL["mat2"], max_range_exceeded=None)
        for g, r, cc in ((rs, rs, c), (xb, xb, cx)):
            if vacuous:
                with pytest.raises(AssertionError, match="passes the gate"):
                    assert_discriminates(as32(g), r, cc, RTOL["mat2"], width=4)
            else:
                assert_discriminates(as32(g), r, cc, RTOL["mat2"], width=4)


def test_mul_scan_with_early_zeros_is_vacuous_and_finite_ensemble_is_not():
    from workloads import mul_finite, small
    w = small(n=30_000)
    x = w["x_mul"]
    rs, c = oracle.scan_fwd("mul", x)
    assert np.count_nonzero(rs[:, 0]) < 600  # the first zero comes early
    with pytest.raises(AssertionError, match="passes the gate"):
        assert_discriminates(as32(rs[:, 0]), rs[:, 0], c[:, 0], RTOL["mul"])
    w = mul_finite(30_000, zeros_after=3 * 8192, n_zeros=2)
    rs, c = oracle.scan_fwd("mul", w["x"])
    assert np.count_nonzero(rs[:, 0]) >= 3 * 8192
    assert_discriminates(as32(rs[:, 0]), rs[:, 0], c[:, 0], RTOL["mul"])
    xb, cx = oracle.scan_vjp("mul", w["ybar"], w["x"])
    assert_discriminates(as32(xb[:, 0]), xb[:, 0], cx[:, 0], RTOL["mul"])
    # exactly the two zero positions and everything before the first zero
    # carry non-zero adjoints; after the second zero every x_bar is 0
    z = np.flatnonzero(w["x"] == 0)
    assert z.size == 2 and np.all(xb[z[1] + 1:, 0] == 0)


def test_gate_rejects_wrong_sign_and_nan():
    r = np.array([1.0, -2.0, 3.0])
    c = np.abs(r)
    assert gate(as32(r), r, c, 1e-5)["ok"]
    assert not gate(-as32(r), r, c, 1e-5)["ok"]
    g = as32(r)
    g[1] = np.nan
    assert not gate(g, r, c, 1e-5)["ok"]


def test_segmented_argmin_against_brute_force():
    """The chained workload's decision: per instance and bin the lowest
    index of the minimum of the given float32 values, the instance length
    when empty; -0.0 and +0.0 tie and the earlier one's sign is kept."""
    rng = np.random.default_rng(5)
    L = [0, 1, 7, 40, 3, 25]
    off = np.concatenate([[0], np.cumsum(L)]).astype(np.int64)
    N, m = int(off[-1]), 5
    y = (rng.integers(-3, 4, N) * 0.5).astype(np.float32)
    y[rng.choice(N, 10, replace=False)] = -0.0
    y[rng.choice(N, 10, replace=False)] = 0.0
    idx = rng.integers(-1, m + 1, N).astype(np.int32)
    argk, h = oracle.segmented_argmin(off, idx, y, m)
    for s in range(len(L)):
        lo = off[s]
        for k in range(m):
            pos = [i for i in range(L[s]) if idx[lo + i] == k]
            if not pos:
                assert argk[s, k] == L[s] and np.isinf(h[s, k]) and h[s, k] > 0
                continue
            best = pos[0]
            for i in pos[1:]:
                if y[lo + i] < y[lo + best]:
                    best = i
            assert argk[s, k] == best
            assert np.float32(h[s, k]).view(np.uint32) == y[lo + best].view(np.uint32)


def test_segmented_decisions_flags_a_wrong_index():
    """The decision check accepts the oracle's own decisions and rejects a
    later index among equal minima and a value that is not y at argk."""
    from oracle.gate import segmented_decisions
    from workloads import segmented_ties
    w = segmented_ties(S=6, m=4, median=50, cap=200)
    off, idx, m = w["offsets"], w["idx"], w["m"]
    f = oracle.segmented_fwd(off, w["a"], w["b"], idx, m)
    y = f["y"].astype(np.float32)
    argk, h = oracle.segmented_argmin(off, idx, y, m)
    d = segmented_decisions(off, idx, m, y, h.astype(np.float32), argk, f)
    assert d["argk_ok"] and d["h_ok"] and d["diff_ok"] and d["n_diff_oracle"] == 0
    # a tie broken the wrong way: the last equal minimum of a bin
    done = False
    for s in range(6):
        lo, hi = off[s], off[s + 1]
        for k in range(m):
            pos = np.flatnonzero(idx[lo:hi] == k)
            if pos.size and np.count_nonzero(y[lo + pos] == y[lo + argk[s, k]]) > 1:
                bad = argk.copy()
                bad[s, k] = pos[y[lo + pos] == y[lo + argk[s, k]]][-1]
                assert not segmented_decisions(off, idx, m, y, h.astype(np.float32), bad)["argk_ok"]
                done = True
                break
        if done:
            break
    assert done
    hb = h.astype(np.float32).copy()
    j = np.flatnonzero(np.isfinite(hb.reshape(-1)))[0]
    hb.reshape(-1)[j] = np.nextafter(hb.reshape(-1)[j], np.float32(np.inf))
    assert not segmented_decisions(off, idx, m, y, hb, argk)["h_ok"]
