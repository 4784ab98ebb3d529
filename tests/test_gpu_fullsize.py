"""Parity at the full sizes of the measured workloads, with the calls and
launch configurations that bench.py times, against the float64 oracle over
every output (the C oracle finishes these sizes in seconds):

  * linear-recurrence scan, n = 2^26, a ~ U[0.9, 1), b ~ N(0, 1);
  * 2x2 matrix-product scan, n = 2^24: on random orthogonal factors, where
    every output stays in the float32 range and is gated element by element;
    and on the workload's N(0, 0.5) entries, whose products underflow within
    a few hundred factors (gated norm-wise: a check of the shape of the
    workload, not of the arithmetic);
  * scans of + * min max at n = 2^24 (more than one round of the persistent
    grid; * on multipliers that keep the products finite), both adjoint
    forms;
  * reduce-by-index, n = 2^26, m in {256, 65536, 2^22} x {uniform, Zipf(1.1)}
    keys, + * min max (min/max and arg-extrema bit-exact, zero counts
    bit-exact), and the ordered 2x2 product per bin (orthogonal factors
    where N(0, 1) ones would overflow float32);
  * the batched segmented workload, 4096 instances (about 2^26 elements),
    with every bin's arg-minimum checked bit for bit against the GPU's y;
  * int32 reduce and scan of + * min max at n = 2^24 + 13 (more tiles than
    one block of the tile-carry scan covers), bit-exact.

Where a check could pass vacuously, the test also shows on the CPU that a
copy of the GPU output zeroed past element 600 fails the same gate.
"""
from __future__ import annotations

import numpy as np
import pytest
import torch

import oracle
from oracle.gate import RTOL, assert_discriminates, assert_gate, chain_rtol, segmented_decisions

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


def ws_error(p):
    return p.ws_status_all()  # raises if a look-back wait timed out


def test_linrec_scan_2e26(pcad):
    from workloads import linrec
    n = 1 << 26
    print(f"linrec scan n={n}", flush=True)
    w = linrec(n=n)
    A, B = dev(w["a"]), dev(w["b"])
    y, _, saved = pcad.scan_fwd("linrec", A, B)
    ab, bb = pcad.scan_vjp("linrec", A, B, saved, dev(w["ybar"]))
    y, ab, bb = host(y), host(ab), host(bb)
    rs, c = oracle.scan_fwd("linrec", w["a"], w["b"])
    assert_gate(y, rs[:, 1], c[:, 1], RTOL["linrec"], what="linrec y")
    yt = np.zeros((n, 2))
    yt[:, 1] = w["ybar"]
    xb, cx = oracle.scan_vjp("linrec", yt, w["a"], w["b"])
    assert_gate(ab, xb[:, 0], cx[:, 0], RTOL["linrec"], what="linrec a_bar")
    assert_gate(bb, xb[:, 1], cx[:, 1], RTOL["linrec"], what="linrec b_bar")
    assert_discriminates(y, rs[:, 1], c[:, 1], RTOL["linrec"], what="linrec y")
    assert_discriminates(ab, xb[:, 0], cx[:, 0], RTOL["linrec"], what="linrec a_bar")
    assert ws_error(pcad) == 0


def test_mat2_scan_2e24_orthogonal(pcad):
    """The 2x2 product scan and its adjoint at 2^24 on random orthogonal
    factors: no output leaves the float32 range, so every P_i and M_bar_i is
    gated element by element (Section 5.3, redundant block-diagonal
    sparsity of the adjoint maps)."""
    from workloads import mat2
    n = 1 << 24
    print(f"mat2 O(2) scan n={n}", flush=True)
    w = mat2(n=n, ensemble="o2")
    M = dev(w["M"])
    P, _, saved = pcad.scan_fwd("mat2", M)
    Mb = pcad.scan_vjp("mat2", M, None, saved, dev(w["Pbar"]))
    Mc = pcad.scan_vjp_checkpoint("mat2", M, None, P, None, dev(w["Pbar"]))
    P, Mb, Mc = host(P), host(Mb), host(Mc)
    # products of up to 2^24 factors: the tolerance grows with the chain
    # length as the rounding error of any evaluation does
    rf = chain_rtol(n, RTOL["mat2"], width=4)
    rb = chain_rtol(n, RTOL["mat2"], width=4, adjoint=True)
    rs, c = oracle.scan_fwd("mat2", w["M"])
    assert_gate(P, rs, c, rf, max_range_exceeded=0, what="O(2) P")
    assert_discriminates(P, rs, c, rf, width=4, what="O(2) P")
    xb, cx = oracle.scan_vjp("mat2", w["Pbar"], w["M"])
    assert_gate(Mb, xb, cx, rb, max_range_exceeded=0, what="O(2) M_bar")
    assert_gate(Mc, xb, cx, rb, max_range_exceeded=0, what="O(2) M_bar (checkpoint)")
    assert_discriminates(Mb, xb, cx, rb, width=4, what="O(2) M_bar")
    assert ws_error(pcad) == 0


def _scalar_scan_inputs(op, n):
    from workloads import BASE_SEED, f32, mul_finite, round_to_grid, _streams
    if op == "mul":
        w = mul_finite(n, seed=BASE_SEED + 70)
        return w["x"], w["ybar"]
    r = _streams(BASE_SEED + 71 + ["add", "min", "max"].index(op), 2)
    if op in ("min", "max"):
        # a trend from 2 down to 0.5 (max: up) under U[0, 2e-4] noise on a
        # 2^-14 grid: the running extremum is renewed about every 700
        # elements all the way (about 24,500 positions with a non-zero
        # adjoint) and equals later elements about 3 million times, where
        # the earlier index must keep it
        t = np.arange(n) / n
        noise = r[0].uniform(0.0, 2e-4, n)
        x = (2.0 - 1.5 * t + noise) if op == "min" else (0.5 + 1.5 * t - noise)
        return f32(round_to_grid(x, -14)), f32(r[1].standard_normal(n))
    x = r[0].uniform(0.5, 2.0, n)
    return f32(x), f32(r[1].standard_normal(n))


@pytest.mark.parametrize("op", ["add", "mul", "min", "max"])
def test_scalar_scan_2e24(pcad, op):
    """Scans of + * min max at 2^24 elements, 2048 tiles: every persistent
    block runs several rounds, so the b + G path of the look-back (a tile
    resolved against its own block's previous tile) is exercised; both
    adjoint forms (recomputed prefixes and the checkpointed forward)."""
    n = 1 << 24
    print(f"scan {op} n={n}", flush=True)
    x, yb = _scalar_scan_inputs(op, n)
    X = dev(x)
    y, _, saved = pcad.scan_fwd(op, X)
    g = pcad.scan_vjp(op, X, None, saved, dev(yb))
    gc = pcad.scan_vjp_checkpoint(op, X, None, y, None, dev(yb))
    y, g, gc = host(y), host(g), host(gc)
    rs, c = oracle.scan_fwd(op, x)
    xb, cx = oracle.scan_vjp(op, yb, x)
    rt = rtb = RTOL[op]
    if op == "mul":  # products of up to 2^24 factors
        rt, rtb = chain_rtol(n, RTOL[op]), chain_rtol(n, RTOL[op], adjoint=True)
    if op in ("min", "max"):
        np.testing.assert_array_equal(y, rs[:, 0].astype(np.float32))
        assert_gate(g, xb[:, 0], cx[:, 0], rt, what=f"scan {op} x_bar")
        assert_gate(gc, xb[:, 0], cx[:, 0], rt, what=f"scan {op} x_bar (checkpoint)")
        # the adjoint sums y_bar over runs of equal prefix minima: non-zero far
        # beyond the first elements
        assert np.count_nonzero(xb[600:, 0]) > 10_000
        assert_discriminates(g, xb[:, 0], cx[:, 0], rt, what=f"scan {op} x_bar", sparse=True)
    else:
        assert np.count_nonzero(rs[:, 0]) == n
        assert_gate(y, rs[:, 0], c[:, 0], rt, what=f"scan {op} y")
        assert_discriminates(y, rs[:, 0], c[:, 0], rt, what=f"scan {op} y")
        assert_gate(g, xb[:, 0], cx[:, 0], rtb, what=f"scan {op} x_bar")
        assert_gate(gc, xb[:, 0], cx[:, 0], rtb, what=f"scan {op} x_bar (checkpoint)")
        assert_discriminates(g, xb[:, 0], cx[:, 0], rtb, what=f"scan {op} x_bar")
    assert ws_error(pcad) == 0


def test_mat2_scan_2e24(pcad):
    from workloads import mat2
    n = 1 << 24
    print(f"mat2 scan n={n}", flush=True)
    w = mat2(n=n)
    M = dev(w["M"])
    P, _, saved = pcad.scan_fwd("mat2", M)
    Mb = pcad.scan_vjp("mat2", M, None, saved, dev(w["Pbar"]))
    P, Mb = host(P), host(Mb)
    rs, c = oracle.scan_fwd("mat2", w["M"])
    assert_gate(P, rs, c, RTOL["mat2"], max_range_exceeded=None, what="mat2 P")
    xb, cx = oracle.scan_vjp("mat2", w["Pbar"], w["M"])
    assert_gate(Mb, xb, cx, RTOL["mat2"], max_range_exceeded=None, what="mat2 M_bar")
    assert ws_error(pcad) == 0


RBI_FULL = [(op, m, dist) for op in ("add", "mul", "min", "max")
            for m in (256, 65536, 1 << 22) for dist in ("uniform", "zipf")]


@pytest.mark.parametrize("op,m,dist", RBI_FULL)
def test_rbi_2e26(pcad, op, m, dist):
    from workloads import rbi
    n = 1 << 26
    print(f"rbi {op} n={n} m={m} {dist}", flush=True)
    w = rbi(op, n=n, m=m, dist=dist)
    I, V = dev(w["idx"]), dev(w["v"])
    h, saved = pcad.rbi_fwd(op, I, V, m)
    vb = pcad.rbi_vjp(op, I, V, m, saved, dev(w["hbar"]))
    h, vb, sv = host(h), host(vb), host(saved)
    o = oracle.rbi_fwd(op, w["idx"], m, w["v"])
    xb, cx = oracle.rbi_vjp(op, w["idx"], m, w["hbar"], w["v"])
    rt = RTOL[op]
    if op in ("min", "max"):
        np.testing.assert_array_equal(sv[: 4 * m].view(np.int32), o["argk"])
        np.testing.assert_array_equal(h, o["hist"][:, 0].astype(np.float32))
        np.testing.assert_array_equal(vb, xb[:, 0].astype(np.float32))
    else:
        if op == "mul":
            np.testing.assert_array_equal(sv[: 4 * m].view(np.uint32), o["n0"])
        assert_gate(h, o["hist"][:, 0], o["c"][:, 0], rt, what=f"rbi {op} hist")
        if op == "add":
            np.testing.assert_array_equal(vb, xb[:, 0].astype(np.float32))
        else:
            assert_gate(vb, xb[:, 0], cx[:, 0], rt, what=f"rbi {op} v_bar")
    assert ws_error(pcad) == 0


@pytest.mark.parametrize("m,ens", [(65536, "mat2o2"), (1 << 22, "mat2")])
def test_rbi_mat2_per_bin_2e26(pcad, m, ens):
    """The generic 2x2 product per bin (ordered by element index).  With
    N(0, 1) entries a bin of about 1024 factors (m = 65536) overflows float32
    (its float64 product reaches 1e40 and beyond), where no float32 result
    is meaningful, so that bin count runs on random orthogonal factors; the
    16 factors per bin of m = 2^22 stay in range with N(0, 1) entries."""
    from workloads import rbi
    n = 1 << 26
    print(f"rbi mat2 n={n} m={m} {ens}", flush=True)
    w = rbi(ens, n=n, m=m)
    I, V = dev(w["idx"]), dev(w["v"])
    h, saved = pcad.rbi_fwd("mat2", I, V, m)
    vb = pcad.rbi_vjp("mat2", I, V, m, saved, dev(w["hbar"]))
    h, vb = host(h), host(vb)
    o = oracle.rbi_fwd("mat2", w["idx"], m, w["v"])
    # both ensembles keep every bin's product in range (16 N(0, 1) factors
    # per bin at m = 2^22, orthogonal factors at m = 65536)
    assert_gate(h, o["hist"], o["c"], RTOL["mat2"], max_range_exceeded=0, what="rbi mat2 hist")
    xb, cx = oracle.rbi_vjp("mat2", w["idx"], m, w["hbar"], w["v"])
    assert_gate(vb, xb, cx, RTOL["mat2"], max_range_exceeded=0, what="rbi mat2 v_bar")
    assert_discriminates(vb, xb, cx, RTOL["mat2"], width=4, what="rbi mat2 v_bar")
    assert ws_error(pcad) == 0


def test_segmented_4096_instances(pcad):
    """The batched workload as bench.py runs it: one graph per phase.  y is
    gated against the oracle; every bin's arg-minimum must be the lowest
    index of the minimum of the GPU's own float32 y, and h that y bit for
    bit; the adjoint runs on the plan's own decisions."""
    from workloads import segmented
    print("segmented S=4096", flush=True)
    w = segmented()
    plan = pcad.BatchedPlan(w["offsets"], w["m"])
    plan.load(a=w["a"], b=w["b"], idx=w["idx"], ybar=w["ybar"], hbar=w["hbar"])
    N, S, m = plan.n, plan.nseg, plan.m
    plan.run(pcad.PHASE_FWD)
    torch.cuda.synchronize()
    y = plan.y[:N].cpu().numpy()
    h = plan.h.cpu().numpy()
    argk = plan.argk.cpu().numpy()
    f = oracle.segmented_fwd(w["offsets"], w["a"], w["b"], w["idx"], m)
    assert_gate(y, f["y"], f["cy"], 1e-4, what="segmented y")
    d = segmented_decisions(w["offsets"], w["idx"], m, y, h, argk, f)
    assert d["argk_ok"] and d["h_ok"] and d["diff_ok"], d
    assert d["n_diff_oracle"] <= max(2, S * m // 5000), d
    plan.run(pcad.PHASE_BWD)
    torch.cuda.synchronize()
    ab, bb, cab, cbb = oracle.segmented_vjp(w["offsets"], w["a"], w["b"], w["idx"], m,
                                            w["ybar"], w["hbar"], argk.reshape(S, m))
    a_bar, b_bar = plan.abar[:N].cpu().numpy(), plan.bbar[:N].cpu().numpy()
    assert_gate(a_bar, ab, cab, 1e-4, what="segmented a_bar")
    assert_gate(b_bar, bb, cbb, 1e-4, what="segmented b_bar")
    assert_discriminates(b_bar, bb, cbb, 1e-4, what="segmented b_bar")
    assert plan.ws_error() == 0
    plan.close()


@pytest.mark.parametrize("op", ["add", "mul", "min", "max"])
def test_i32_scan_2e24(pcad, op):
    """int32 reduce and scan, wrapping mod 2^32, bit for bit against the
    oracle at a size whose tile carries take several rounds."""
    rng = np.random.default_rng(231003568 + len(op))
    n = (1 << 24) + 13
    if op == "mul":
        x = rng.choice(np.array([-3, -1, 1, 3, 5, 7], np.int64), size=n).astype(np.int32)
    else:
        x = rng.integers(-2**31, 2**31, size=n, dtype=np.int64).astype(np.int32)
    print(f"i32 {op} n={n}", flush=True)
    X = dev(x)
    y = host(pcad.i32_fwd(pcad.REDUCE, op, X))
    s = host(pcad.i32_fwd(pcad.SCAN, op, X))
    assert int(y) == oracle.i32_reduce(op, x)
    np.testing.assert_array_equal(s, oracle.i32_scan(op, x))
    assert ws_error(pcad) == 0
