"""Parity of the HIP path (through the C-ABI) with the CPU FP64 oracle.

Floats pass the companion-scaled gate |g - r| <= rtol*c + 2^-126 with
rtol 1e-5 for + min max and 1e-4 for *, the linear recurrence and the 2x2
matrix product; integer results (indices, counts) and pure copies (min/max
values, gathered adjoints) are compared bit for bit.  Sizes span several
tiles with ragged tails; batches use row lengths that misalign the rows.
"""
from __future__ import annotations

import numpy as np
import pytest
import torch

import oracle
from oracle.gate import RTOL, assert_discriminates, assert_gate, chain_rtol

pytestmark = pytest.mark.gpu

SCALAR = ["add", "mul", "min", "max"]
ALL = SCALAR + ["linrec", "mat2"]


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


def ws_error():
    """0 unless a look-back wait timed out on a cached workspace (then
    pcad_ws_status reports it and the binding raises)"""
    import paper_2310_03568_amd as p
    return p.ws_status_all()


# Products of N(0, 0.5) 2x2 factors underflow float32 after a few hundred
# factors, after which every output is 0 and any result passes; beyond this
# many elements per row, 2x2 inputs are random orthogonal factors instead
MAT2_GAUSS_MAX = 256


def mat2_o2(rows_n):
    return rows_n > MAT2_GAUSS_MAX


def make_inputs(op, shape, rng, ties=False):
    """Inputs of the small workload's distributions, shaped (..., n)."""
    if op == "linrec":
        a = rng.uniform(0.9, 1.0, shape).astype(np.float32)
        b = rng.standard_normal(shape).astype(np.float32)
        return a, b
    if op == "mat2":
        if mat2_o2(shape[-1]):
            from workloads import o2_matrices
            return o2_matrices(rng, int(np.prod(shape))).reshape(shape + (4,)), None
        return (rng.standard_normal(shape + (4,)) * np.sqrt(0.5)).astype(np.float32), None
    x = rng.uniform(0.5, 2.0, shape)
    if op == "mul":
        flat = x.reshape(-1)
        z = rng.choice(flat.size, max(flat.size // 100, 0), replace=False)
        flat[z] = 0.0
    if ties:
        x = np.floor(x * 4) / 4
    return x.astype(np.float32), None


def rows(a, batch):
    return a.reshape(batch, -1) if a.ndim == 1 or a.shape[-1] != 4 else a.reshape(batch, -1, 4)


# ---------------------------------------------------------------------------
# scan
# ---------------------------------------------------------------------------
SCAN_SIZES = [1, 2, 5, 63, 64, 65, 1023, 1024, 1025, 4095, 4096, 4097, 12293, 100_000]


def check_scan(pcad, op, batch, n, seed, ties=False, abar=False, ckpt=False, rt_f=None, rt_b=None):
    rng = np.random.default_rng(seed)
    shape = (batch, n) if batch > 1 else (n,)
    x0, x1 = make_inputs(op, shape, rng, ties)
    d = oracle.DIM[op]
    yb = rng.standard_normal(shape + ((4,) if op == "mat2" else ())).astype(np.float32)
    Ab = rng.standard_normal(shape).astype(np.float32) if abar else None
    X0, X1 = dev(x0), (dev(x1) if x1 is not None else None)
    y, A, saved = pcad.scan_fwd(op, X0, X1, want_A=(op == "linrec"))
    if ckpt:
        # the checkpoint form reads y (and A) instead of the tile prefixes;
        # the linear recurrence's offsets are not passed at all
        g = pcad.scan_vjp_checkpoint(op, X0, None, y, A if abar else None, dev(yb),
                                     dev(Ab) if abar else None)
    else:
        g = pcad.scan_vjp(op, X0, X1, saved, dev(yb), dev(Ab) if abar else None)
    y = host(y)
    A = host(A) if A is not None else None
    g = [host(t) for t in g] if op == "linrec" else host(g)
    rt = RTOL[op] if rt_f is None else rt_f
    rtb = rt if rt_b is None else rt_b
    max_rx = n * batch if op == "mul" else 0
    for r in range(batch):
        sl = (r,) if batch > 1 else ()
        xr0 = x0[sl] if batch > 1 else x0
        xr1 = (x1[sl] if batch > 1 else x1) if x1 is not None else None
        rs, c = oracle.scan_fwd(op, xr0, xr1)
        mx2 = 0 if mat2_o2(n) else None
        if op == "linrec":
            assert_gate(y[sl], rs[:, 1], c[:, 1], rt, what=f"scan linrec y row {r}")
            assert_discriminates(y[sl], rs[:, 1], c[:, 1], rt, what=f"scan linrec y row {r}")
            assert_gate(A[sl], rs[:, 0], c[:, 0], rt, what=f"scan linrec A row {r}")
            ybo = np.stack([Ab[sl] if abar else np.zeros(n), yb[sl]], 1)
        elif op == "mat2":
            assert_gate(y[sl], rs, c, rt, max_range_exceeded=mx2, what=f"scan mat2 row {r}")
            if mx2 == 0:
                assert_discriminates(y[sl], rs, c, rt, width=4, what=f"scan mat2 row {r}")
            ybo = yb[sl]
        elif op in ("min", "max"):
            np.testing.assert_array_equal(y[sl], rs[:, 0].astype(np.float32))
            ybo = yb[sl]
        else:
            assert_gate(y[sl], rs[:, 0], c[:, 0], rt, max_range_exceeded=max_rx,
                        what=f"scan {op} row {r}")
            if op == "add":
                assert_discriminates(y[sl], rs[:, 0], c[:, 0], rt, what=f"scan add row {r}")
            ybo = yb[sl]
        xb, cx = oracle.scan_vjp(op, ybo, xr0, xr1)
        if op == "linrec":
            assert_gate(g[0][sl], xb[:, 0], cx[:, 0], rtb, what=f"scan_vjp linrec a_bar row {r}")
            assert_gate(g[1][sl], xb[:, 1], cx[:, 1], rtb, what=f"scan_vjp linrec b_bar row {r}")
            assert_discriminates(g[0][sl], xb[:, 0], cx[:, 0], rtb, what=f"linrec a_bar row {r}")
            assert_discriminates(g[1][sl], xb[:, 1], cx[:, 1], rtb, what=f"linrec b_bar row {r}")
        elif op == "mat2":
            assert_gate(g[sl], xb, cx, rtb, max_range_exceeded=mx2, what=f"scan_vjp mat2 row {r}")
            if mx2 == 0:
                assert_discriminates(g[sl], xb, cx, rtb, width=4, what=f"scan_vjp mat2 row {r}")
        else:
            assert_gate(g[sl], xb[:, 0], cx[:, 0], rtb, max_range_exceeded=max_rx,
                        what=f"scan_vjp {op} row {r}")
            if op == "add":
                assert_discriminates(g[sl], xb[:, 0], cx[:, 0], rtb, what=f"scan_vjp add row {r}")
    assert ws_error() == 0


@pytest.mark.parametrize("op,batch,tiles", [("add", 3, 258), ("linrec", 3, 258), ("mat2", 2, 300)])
def test_scan_rows_past_a_round(pcad, op, batch, tiles):
    """Rows of more tiles than one round of the persistent grid (about one
    512-thread block per CU): a tile's look-back then takes the prefix one
    round back from its block's own previous tile, which has to lie in the
    same row, and row boundaries fall inside rounds.  The 2x2 products are
    orthogonal chains of up to 6e5 factors, gated with the chain tolerance."""
    tile = 2048 if op == "mat2" else 8192
    n = tiles * tile + 5
    print(f"scan rows past a round: {op} batch={batch} n={n}", flush=True)
    kw = {}
    if op == "mat2":
        kw = dict(rt_f=chain_rtol(n, RTOL["mat2"], width=4),
                  rt_b=chain_rtol(n, RTOL["mat2"], width=4, adjoint=True))
    check_scan(pcad, op, batch, n, 7100 + tiles, **kw)


@pytest.mark.parametrize("op", ALL)
@pytest.mark.parametrize("n", SCAN_SIZES)
def test_scan(pcad, op, n):
    check_scan(pcad, op, 1, n, seed=n)


@pytest.mark.parametrize("op", ALL)
def test_scan_batched_misaligned(pcad, op):
    check_scan(pcad, op, 3, 5001, seed=7)


MUL_TILE = 8192  # elements per tile of the scalar scans


def check_scan_mul_finite(pcad, batch, n, seed, n_zeros=0, ckpt=False):
    """* scans whose prefix products stay finite and non-zero across many
    tiles (multipliers +-exp(U[-0.01, 0.01])), so that the cross-tile
    carries of the forward products and of the adjoint maps are compared
    on non-zero values; with ``n_zeros``, exact zeros only past the first
    three tiles (the zero-prefix guard of the adjoint and the three zero
    cases of Section 3.2 then act inside a long non-zero run)."""
    from workloads import mul_finite
    shape = (batch, n) if batch > 1 else (n,)
    w = mul_finite(shape, seed=seed, zeros_after=3 * MUL_TILE, n_zeros=n_zeros)
    x, yb = w["x"], w["ybar"]
    X = dev(x)
    y, _, saved = pcad.scan_fwd("mul", X)
    if ckpt:
        g = pcad.scan_vjp_checkpoint("mul", X, None, y, None, dev(yb))
    else:
        g = pcad.scan_vjp("mul", X, None, saved, dev(yb))
    y, g = host(y).reshape(batch, n), host(g).reshape(batch, n)
    # products of up to n factors: the tolerance grows with the chain length
    rf, rb = chain_rtol(n, RTOL["mul"]), chain_rtol(n, RTOL["mul"], adjoint=True)
    for r in range(batch):
        xr, ybr = x.reshape(batch, n)[r], yb.reshape(batch, n)[r]
        rs, c = oracle.scan_fwd("mul", xr)
        nz = int(np.count_nonzero(rs[:, 0]))
        assert nz >= min(n, 3 * MUL_TILE), nz  # the ensemble does what it claims
        assert_gate(y[r], rs[:, 0], c[:, 0], rf, what=f"scan mul row {r}")
        assert_discriminates(y[r], rs[:, 0], c[:, 0], rf, what=f"scan mul row {r}")
        xb, cx = oracle.scan_vjp("mul", ybr, xr)
        assert_gate(g[r], xb[:, 0], cx[:, 0], rb, what=f"scan_vjp mul row {r}")
        assert_discriminates(g[r], xb[:, 0], cx[:, 0], rb, what=f"scan_vjp mul row {r}")
    assert ws_error() == 0


@pytest.mark.parametrize("n", [3 * MUL_TILE + 77, 100_003, (1 << 21) + 5])
@pytest.mark.parametrize("ckpt", [False, True])
def test_scan_mul_finite_prefixes(pcad, n, ckpt):
    check_scan_mul_finite(pcad, 1, n, seed=300 + n % 1000, ckpt=ckpt)


@pytest.mark.parametrize("n_zeros", [1, 2, 3])
@pytest.mark.parametrize("ckpt", [False, True])
def test_scan_mul_zeros_after_three_tiles(pcad, n_zeros, ckpt):
    check_scan_mul_finite(pcad, 1, 5 * MUL_TILE + 123, seed=310 + n_zeros, n_zeros=n_zeros, ckpt=ckpt)
    check_scan_mul_finite(pcad, 2, 4 * MUL_TILE + 9, seed=320 + n_zeros, n_zeros=n_zeros, ckpt=ckpt)


@pytest.mark.parametrize("op", ["min", "max"])
def test_scan_ties(pcad, op):
    check_scan(pcad, op, 1, 50_000, seed=11, ties=True)
    check_scan(pcad, op, 2, 4099, seed=12, ties=True)


@pytest.mark.parametrize("op", ALL)
@pytest.mark.parametrize("n", [1, 5, 65, 4097, 12293, 100_000])
def test_scan_checkpoint(pcad, op, n):
    check_scan(pcad, op, 1, n, seed=100 + n, ckpt=True)


@pytest.mark.parametrize("op", ALL)
def test_scan_checkpoint_batched_misaligned(pcad, op):
    check_scan(pcad, op, 3, 5001, seed=17, ckpt=True)


def test_scan_checkpoint_ties_and_abar(pcad):
    check_scan(pcad, "min", 2, 20_001, seed=18, ties=True, ckpt=True)
    check_scan(pcad, "max", 1, 20_001, seed=19, ties=True, ckpt=True)
    check_scan(pcad, "linrec", 2, 9001, seed=20, abar=True, ckpt=True)


def test_scan_linrec_abar(pcad):
    check_scan(pcad, "linrec", 1, 70_001, seed=13, abar=True)
    check_scan(pcad, "linrec", 2, 4097, seed=14, abar=True)


def test_scan_mat2_orthogonal(pcad):
    from workloads import mat2
    w = mat2(n=50_000, ensemble="o2")
    M = dev(w["M"])
    P, _, saved = pcad.scan_fwd("mat2", M)
    Mb = pcad.scan_vjp("mat2", M, None, saved, dev(w["Pbar"]))
    rs, c = oracle.scan_fwd("mat2", w["M"])
    assert_gate(host(P), rs, c, RTOL["mat2"], what="O(2) products")
    xb, cx = oracle.scan_vjp("mat2", w["Pbar"], w["M"])
    assert_gate(host(Mb), xb, cx, RTOL["mat2"], what="O(2) adjoint")


def test_scan_signed_zero_ties(pcad):
    """-0.0 and +0.0 tie; the earlier element's bit pattern is kept."""
    x = np.array([1.0, -0.0, 0.0, 2.0, 0.0, -0.0], np.float32)
    y, _, s = pcad.scan_fwd("min", dev(x))
    yy = host(y)
    np.testing.assert_array_equal(np.signbit(yy), [False, True, True, True, True, True])
    xb = host(pcad.scan_vjp("min", dev(x), None, s, dev(np.ones(6, np.float32))))
    np.testing.assert_array_equal(xb, [1, 5, 0, 0, 0, 0])


def test_ws_status_reports_and_clears_a_timeout_word(pcad):
    """The control block's error word names the launch whose look-back wait
    timed out.  Planting the tag of the launch that just finished (as if one
    of its waits had run out) must not disturb the next launches, whose tags
    differ, and pcad_ws_status reports it once and clears it.  No wait is
    made to time out here: the word is written from the host."""
    rng = np.random.default_rng(77)
    x = rng.integers(-8, 8, 50_000).astype(np.float32)
    X = dev(x)
    y, _, s = pcad.scan_fwd("add", X)
    torch.cuda.synchronize()
    assert pcad.ws_status_all() == 0
    key = (X.device.index, torch.cuda.current_stream(X.device).cuda_stream)
    ws = pcad._ws[key]
    ctl = ws[:16].view(torch.int32)
    epoch = int(ctl[1].item())
    assert epoch != 0
    ctl[2] = epoch  # the tag of the finished launch
    torch.cuda.synchronize()
    for _ in range(3):
        y, _, s = pcad.scan_fwd("add", X)
        np.testing.assert_array_equal(host(y), np.cumsum(x.astype(np.float64)).astype(np.float32))
    with pytest.raises(pcad.PcadError, match="timed out"):
        pcad.ws_status(ws, clear=True)
    assert pcad.ws_status(ws) == 0
    assert int(ws[:16].view(torch.int32)[2].item()) == 0


def test_scan_accumulate(pcad):
    rng = np.random.default_rng(3)
    x = rng.uniform(0.5, 2, 9000).astype(np.float32)
    yb = rng.standard_normal(9000).astype(np.float32)
    X = dev(x)
    _, _, s = pcad.scan_fwd("add", X)
    base = rng.standard_normal(9000).astype(np.float32)
    out = dev(base)
    pcad.scan_vjp("add", X, None, s, dev(yb), out=(out,), accumulate=True)
    xb, cx = oracle.scan_vjp("add", yb, x)
    assert_gate(host(out), xb[:, 0] + base, cx[:, 0] + np.abs(base), 1e-5, what="accumulate")


@pytest.mark.parametrize("op,n,ckpt", [("add", 100_003, False), ("linrec", 2_500_007, False),
                                       ("linrec", 300_001, True), ("max", 200_003, True),
                                       ("mat2", 300_001, False), ("mat2", 100_001, True)])
def test_scan_vjp_accumulate(pcad, op, n, ckpt):
    """PCAD_ACCUMULATE (the paper's +=) in every scan-adjoint kernel: the
    delayed group-major and lane-major kernels (recompute form), and the
    checkpoint forms, over several tiles and, for LINREC, several rounds."""
    rng = np.random.default_rng(4000 + n)
    x0, x1 = make_inputs(op, (n,), rng)
    yb = rng.standard_normal((n, 4) if op == "mat2" else n).astype(np.float32)
    X0, X1 = dev(x0), (dev(x1) if x1 is not None else None)
    y, A, saved = pcad.scan_fwd(op, X0, X1, want_A=(op == "linrec"))
    k = 2 if op == "linrec" else 1
    base = [rng.standard_normal(x0.shape).astype(np.float32) for _ in range(k)]
    out = tuple(dev(b) for b in base)
    if ckpt:
        pcad.scan_vjp_checkpoint(op, X0, None, y, None, dev(yb), out=out, accumulate=True)
    else:
        pcad.scan_vjp(op, X0, X1, saved, dev(yb), out=out, accumulate=True)
    ybo = np.stack([np.zeros(n), yb], 1) if op == "linrec" else yb
    xb, cx = oracle.scan_vjp(op, ybo, x0, x1)
    rt = RTOL[op]
    if op == "mat2":
        rt = chain_rtol(n, RTOL["mat2"], width=4, adjoint=True)
        assert_gate(host(out[0]), xb + base[0], cx + np.abs(base[0]), rt, max_range_exceeded=0,
                    what="mat2 accumulate")
        return
    for c in range(k):
        assert_gate(host(out[c]), xb[:, c] + base[c], cx[:, c] + np.abs(base[c]), rt,
                    what=f"{op} accumulate {c}")
    assert ws_error() == 0


def test_scan_repeat_reuses_workspace(pcad):
    """Self-resetting counters and epoch tags: many launches on one
    workspace, alternating directions and sizes, stay exact."""
    rng = np.random.default_rng(5)
    for it in range(20):
        n = int(rng.integers(1, 40_000))
        x = rng.integers(-8, 8, n).astype(np.float32)
        X = dev(x)
        y, _, s = pcad.scan_fwd("add", X)
        np.testing.assert_array_equal(host(y), np.cumsum(x.astype(np.float64)).astype(np.float32))
        yb = rng.integers(-8, 8, n).astype(np.float32)
        g = pcad.scan_vjp("add", X, None, s, dev(yb))
        np.testing.assert_array_equal(host(g), np.cumsum(yb[::-1].astype(np.float64))[::-1].astype(np.float32))
    assert ws_error() == 0


# ---------------------------------------------------------------------------
# reduce
# ---------------------------------------------------------------------------
RED_SIZES = [1, 3, 4, 5, 1000, 4096, 16385, 100_000, 1 << 20]


def check_reduce(pcad, op, batch, n, seed, ties=False):
    rng = np.random.default_rng(seed)
    shape = (batch, n) if batch > 1 else (n,)
    x0, x1 = make_inputs(op, shape, rng, ties)
    d = oracle.DIM[op]
    yb = rng.standard_normal((batch, d) if batch > 1 else (d,)).astype(np.float32)
    if d == 1:
        yb = yb.reshape(shape[:-1]) if batch > 1 else yb.reshape(())
        yb = np.atleast_1d(yb)
    X0, X1 = dev(x0), (dev(x1) if x1 is not None else None)
    y, saved = pcad.reduce_fwd(op, X0, X1)
    g = pcad.reduce_vjp(op, X0, X1, saved, dev(yb))
    y = host(y).reshape(batch, d)
    g = [host(t) for t in g] if op == "linrec" else host(g)
    sv = host(saved)
    rt = RTOL[op]
    for r in range(batch):
        sl = (r,) if batch > 1 else ()
        xr0 = x0[sl] if batch > 1 else x0
        xr1 = (x1[sl] if batch > 1 else x1) if x1 is not None else None
        o = oracle.reduce_fwd(op, xr0, xr1)
        ybr = yb.reshape(batch, d)[r]
        if op in ("min", "max"):
            assert y[r, 0] == np.float32(o["y"][0])
            assert sv[: 4 * batch].view(np.int32)[r] == o["k"]
        elif op == "mul":
            assert sv[: 8 * batch].view(np.uint32)[2 * r] == o["n0"]
            ypos = sv[: 8 * batch].view(np.float32)[2 * r + 1]
            assert_gate([ypos], [o["ypos"]], [abs(o["ypos"])], rt, max_range_exceeded=1, what="ypos")
            assert_gate(y[r], o["y"], o["c"], rt, max_range_exceeded=1, what="reduce mul")
        else:
            mx2 = None if (op == "mat2" and not mat2_o2(n)) else 0
            assert_gate(y[r], o["y"], o["c"], rt, max_range_exceeded=mx2, what=f"reduce {op}")
            if op == "mat2" and mx2 == 0:
                # a wrong product (here: the identity, or zero) must fail
                assert not any(gate_ok(z, o["y"], o["c"], rt) for z in ([1, 0, 0, 1], [0, 0, 0, 0]))
        xb, cx = oracle.reduce_vjp(op, ybr, xr0, xr1)
        if op == "linrec":
            assert_gate(g[0][sl], xb[:, 0], cx[:, 0], rt, what="reduce_vjp linrec a")
            assert_gate(g[1][sl], xb[:, 1], cx[:, 1], rt, what="reduce_vjp linrec b")
            # b_bar_i = y_bar times the later multipliers (a < 1): negligible
            # beyond a few thousand elements from the end
            assert_discriminates(g[1][sl], xb[:, 1], cx[:, 1], rt, what="reduce_vjp linrec b",
                                 sparse=True)
        elif op == "mat2":
            mx2 = 0 if mat2_o2(n) else None
            assert_gate(g[sl], xb, cx, rt, max_range_exceeded=mx2, what="reduce_vjp mat2")
            if mx2 == 0:
                assert_discriminates(g[sl], xb, cx, rt, width=4, what="reduce_vjp mat2")
        elif op in ("add", "min", "max"):
            np.testing.assert_array_equal(g[sl], xb[:, 0].astype(np.float32))
        else:
            assert_gate(g[sl], xb[:, 0], cx[:, 0], rt, max_range_exceeded=n, what="reduce_vjp mul")
    assert ws_error() == 0


def gate_ok(g, r, c, rtol):
    from oracle.gate import gate
    return gate(g, r, c, rtol)["ok"]


@pytest.mark.parametrize("op", ALL)
@pytest.mark.parametrize("n", RED_SIZES)
def test_reduce(pcad, op, n):
    # 2x2 products beyond MAT2_GAUSS_MAX factors run on orthogonal factors
    check_reduce(pcad, op, 1, n, seed=100 + n)


@pytest.mark.parametrize("op", ALL)
def test_reduce_batched(pcad, op):
    check_reduce(pcad, op, 5, 3001, seed=21)


@pytest.mark.parametrize("op", ["min", "max"])
def test_reduce_ties(pcad, op):
    check_reduce(pcad, op, 1, 300_000, seed=22, ties=True)
    check_reduce(pcad, op, 3, 777, seed=23, ties=True)


@pytest.mark.parametrize("zeros", [0, 1, 2])
def test_reduce_mul_zero_cases(pcad, zeros):
    rng = np.random.default_rng(30 + zeros)
    x = rng.uniform(0.95, 1.05, 50_000).astype(np.float32)
    pos = rng.choice(50_000, zeros, replace=False)
    x[pos] = 0.0
    X = dev(x)
    y, s = pcad.reduce_fwd("mul", X)
    g = host(pcad.reduce_vjp("mul", X, None, s, dev(np.array([1.5], np.float32))))
    xb, cx = oracle.reduce_vjp("mul", np.array([1.5]), x)
    assert_gate(g, xb[:, 0], cx[:, 0], 1e-4, what=f"reduce mul {zeros} zeros")
    if zeros >= 2:
        assert not g.any()


def test_reduce_empty(pcad):
    for op in ALL:
        shape = (3, 0, 4) if op == "mat2" else (3, 0)
        x = torch.zeros(shape, device="cuda")
        y, s = pcad.reduce_fwd(op, x, torch.zeros(shape, device="cuda") if op == "linrec" else None)
        y = host(y)
        e = {"add": 0, "mul": 1, "min": np.inf, "max": -np.inf}
        if op in e:
            np.testing.assert_array_equal(y, np.full(3, e[op], np.float32))
        elif op == "linrec":
            np.testing.assert_array_equal(y, np.tile([1, 0], (3, 1)))
        else:
            np.testing.assert_array_equal(y, np.tile([1, 0, 0, 1], (3, 1)))


# ---------------------------------------------------------------------------
# reduce-by-index
# ---------------------------------------------------------------------------
def check_rbi(pcad, op, batch, n, m, seed, dist="uniform", oob=True, ties=False):
    rng = np.random.default_rng(seed)
    shape = (batch, n) if batch > 1 else (n,)
    v = rng.standard_normal(shape)
    if op == "mul":
        fl = v.reshape(-1)
        fl[rng.choice(fl.size, fl.size // 50, replace=False)] = 0.0
        v = rng.uniform(0.9, 1.1, shape) * np.sign(v) * (v != 0)
    if ties or op in ("min", "max"):
        v = np.round(v * 256) / 256
    v = v.astype(np.float32)
    if dist == "zipf":
        from workloads import zipf_keys
        idx = zipf_keys(rng, batch * n, m).reshape(shape)
    else:
        idx = rng.integers(0, max(m, 1), shape).astype(np.int32)
    if oob and n > 0:
        fl = idx.reshape(-1)
        k = rng.choice(fl.size, max(fl.size // 97, 1), replace=False)
        fl[k] = rng.choice([-1, m, m + 5, -1000], k.size)
    hb = rng.standard_normal((batch, m) if batch > 1 else (m,)).astype(np.float32)
    I, V = dev(idx.astype(np.int32)), dev(v)
    h, saved = pcad.rbi_fwd(op, I, V, m)
    vb = pcad.rbi_vjp(op, I, V, m, saved, dev(hb))
    h = host(h).reshape(batch, m)
    vb = host(vb).reshape(batch, n)
    sv = host(saved)
    rt = RTOL[op]
    for r in range(batch):
        ir = idx.reshape(batch, n)[r]
        vr = v.reshape(batch, n)[r]
        o = oracle.rbi_fwd(op, ir, m, vr)
        if op in ("min", "max"):
            ak = sv[: 4 * batch * m].view(np.int32).reshape(batch, m)[r]
            np.testing.assert_array_equal(ak, o["argk"])
            np.testing.assert_array_equal(h[r], o["hist"][:, 0].astype(np.float32))
        elif op == "mul":
            n0 = sv[: 4 * batch * m].view(np.uint32).reshape(batch, m)[r]
            np.testing.assert_array_equal(n0, o["n0"])
            yp = sv[4 * batch * m: 8 * batch * m].view(np.float32).reshape(batch, m)[r]
            assert_gate(yp, o["ypos"], np.abs(o["ypos"]), rt, what="rbi mul ypos")
            assert_gate(h[r], o["hist"][:, 0], o["c"][:, 0], rt, what="rbi mul hist")
        else:
            assert_gate(h[r], o["hist"][:, 0], o["c"][:, 0], rt, what="rbi add hist")
        xb, cx = oracle.rbi_vjp(op, ir, m, hb.reshape(batch, m)[r], vr)
        if op == "mul":
            assert_gate(vb[r], xb[:, 0], cx[:, 0], rt, what="rbi_vjp mul")
        else:
            np.testing.assert_array_equal(vb[r], xb[:, 0].astype(np.float32))
    assert ws_error() == 0


RBI_CASES = [(0, 5), (1, 1), (1000, 7), (10_000, 1), (100_000, 1024), (100_000, 4096),
             (100_000, 4097), (100_000, 8192), (100_000, 8193), (300_000, 65536), (200_003, 100_000),
             (70_000, 1 << 20)]


@pytest.mark.parametrize("op", SCALAR)
@pytest.mark.parametrize("n,m", RBI_CASES)
def test_rbi(pcad, op, n, m):
    check_rbi(pcad, op, 1, n, m, seed=n + m)


@pytest.mark.parametrize("op", SCALAR)
def test_rbi_batched(pcad, op):
    check_rbi(pcad, op, 4, 5003, 333, seed=41)
    check_rbi(pcad, op, 2, 9001, 20_000, seed=42)


@pytest.mark.parametrize("op", SCALAR)
@pytest.mark.parametrize("m", [256, 65536])
def test_rbi_zipf(pcad, op, m):
    check_rbi(pcad, op, 1, 200_000, m, seed=43, dist="zipf")


@pytest.mark.parametrize("op", SCALAR)
@pytest.mark.parametrize("dist", ["uniform", "zipf"])
def test_rbi_many_bins(pcad, op, dist):
    """Bin counts far beyond the LDS capacity: hundreds of bin ranges (the
    partitioned path), skewed keys splitting the hot range over many blocks"""
    check_rbi(pcad, op, 1, 1 << 21, 1 << 22, seed=46, dist=dist)
    check_rbi(pcad, op, 1, 999_999, 3 * 8192 + 5, seed=47, dist=dist)


@pytest.mark.parametrize("op", SCALAR)
@pytest.mark.parametrize("m", [700, 3000, 20_011])
def test_rbi_vjp_without_workspace(pcad, op, m):
    """The adjoint of + * min max may be called with ws = NULL (direct gathers
    from the saved arrays); it must equal the call with a workspace (LDS or
    packed per-bin records) bit for bit, and also accumulate the same way."""
    rng = np.random.default_rng(m)
    n = 50_001
    v = rng.standard_normal(n).astype(np.float32)
    if op == "mul":
        v[rng.choice(n, 300, replace=False)] = 0.0
    if op in ("min", "max"):
        v = np.round(v * 16) / 16
    idx = rng.integers(-3, m + 3, n).astype(np.int32)
    I, V = dev(idx), dev(v)
    hb = dev(rng.standard_normal(m).astype(np.float32))
    h, saved = pcad.rbi_fwd(op, I, V, m)
    ref = pcad.rbi_vjp(op, I, V, m, saved, hb)
    for acc in (0, pcad.ACCUMULATE):
        out = dev(np.ones(n, np.float32)) if acc else torch.empty_like(V)
        pcad.check(pcad.lib().pcad_rbi_vjp(pcad.OPS[op], 1, n, m, I.data_ptr(), V.data_ptr(),
                                           saved.data_ptr(), hb.data_ptr(), out.data_ptr(), acc,
                                           None, 0, torch.cuda.current_stream().cuda_stream),
                   "pcad_rbi_vjp")
        expect = host(ref) + (1.0 if acc else 0.0)
        np.testing.assert_array_equal(host(out), expect.astype(np.float32))


def test_rbi_zero_bins(pcad):
    for op in SCALAR:
        I = dev(np.array([0, 3, -1], np.int32))
        V = dev(np.array([1, 2, 3], np.float32))
        h, s = pcad.rbi_fwd(op, I, V, 0)
        assert h.numel() == 0
        vb = host(pcad.rbi_vjp(op, I, V, 0, s, torch.zeros(0, device="cuda")))
        np.testing.assert_array_equal(vb, [0, 0, 0])


# ---------------------------------------------------------------------------
# reduce-by-index of the ordered (non-commutative) operators: per-bin folds in
# ascending element order, through the sort-based path
# ---------------------------------------------------------------------------
def check_rbi_ordered(pcad, op, batch, n, m, seed, dist="uniform"):
    rng = np.random.default_rng(seed)
    d = oracle.DIM[op]
    if op == "linrec":
        a = rng.uniform(0.9, 1.0, (batch, n))
        b = rng.standard_normal((batch, n))
        v = np.stack([a, b], -1).astype(np.float32)
    else:
        v = (rng.standard_normal((batch, n, 4)) * np.sqrt(0.5)).astype(np.float32)
    if dist == "zipf":
        from workloads import zipf_keys
        idx = zipf_keys(rng, batch * n, m).reshape(batch, n)
    else:
        idx = rng.integers(0, max(m, 1), (batch, n)).astype(np.int32)
    if n > 0:
        fl = idx.reshape(-1)
        k = rng.choice(fl.size, max(fl.size // 97, 1), replace=False)
        fl[k] = rng.choice([-1, m, m + 5], k.size)
    hb = rng.standard_normal((batch, m, d)).astype(np.float32)
    I, V = dev(idx.astype(np.int32)), dev(v)
    h, saved = pcad.rbi_fwd(op, I, V, m)
    vb = pcad.rbi_vjp(op, I, V, m, saved, dev(hb))
    h, vb = host(h).reshape(batch, m, d), host(vb).reshape(batch, n, d)
    rt = RTOL[op]
    for r in range(batch):
        args = (v[r, :, 0], v[r, :, 1]) if op == "linrec" else (v[r],)
        o = oracle.rbi_fwd(op, idx[r], m, *args)
        # MAT2 products over long runs of N(0, 0.5) factors leave the float32
        # range: those bins are checked norm-wise
        mx = None if op == "mat2" else 0
        assert_gate(h[r], o["hist"], o["c"], rt, max_range_exceeded=mx, what=f"rbi {op} hist row {r}")
        xb, cx = oracle.rbi_vjp(op, idx[r], m, hb[r], *args)
        assert_gate(vb[r], xb, cx, rt, max_range_exceeded=mx, what=f"rbi_vjp {op} row {r}")
    assert ws_error() == 0


@pytest.mark.parametrize("op", ["linrec", "mat2"])
@pytest.mark.parametrize("n,m", [(0, 3), (1, 1), (2049, 1), (2049, 7), (50_001, 300),
                                 (50_001, 70_000), (200_000, 1 << 20)])
def test_rbi_ordered(pcad, op, n, m):
    check_rbi_ordered(pcad, op, 1, n, m, seed=n + 3 * m)


@pytest.mark.parametrize("op", ["linrec", "mat2"])
def test_rbi_ordered_batched_and_skewed(pcad, op):
    check_rbi_ordered(pcad, op, 3, 7001, 129, seed=44)
    check_rbi_ordered(pcad, op, 1, 100_000, 1000, seed=45, dist="zipf")


# ---------------------------------------------------------------------------
# sumOfProd (Section 3.3) for reduce and reduce-by-index (Section 4.2,
# Invertible Operators)
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("batch,n", [(1, 0), (1, 1), (1, 2), (1, 1000), (1, 100_003), (3, 70_001),
                                     (1, 1 << 20)])
def test_reduce_sumprod(pcad, batch, n):
    rng = np.random.default_rng(n + 7 * batch)
    x = rng.standard_normal((batch, n)).astype(np.float32)
    yb = rng.standard_normal(batch).astype(np.float32)
    X = dev(x if batch > 1 else x[0])
    y, saved = pcad.reduce_fwd("sumprod", X)
    g = pcad.reduce_vjp("sumprod", X, None, saved, dev(yb if batch > 1 else yb[:1]))
    y = host(y).reshape(batch)
    g = host(g).reshape(batch, n)
    s = host(saved)[: 4 * batch].view(np.float32)
    for r in range(batch):
        o = oracle.sumprod_reduce(x[r])
        assert_gate([y[r]], [o["y"]], [o["c"]], RTOL["sumprod"], what=f"sumprod row {r}")
        assert_gate([s[r]], [o["s"]], [np.abs(x[r].astype(np.float64)).sum()], RTOL["add"],
                    what="sumprod s")
        xb, cx = oracle.sumprod_reduce_vjp(x[r], float(yb[r]))
        assert_gate(g[r], xb, cx, RTOL["sumprod"], what=f"sumprod vjp row {r}")


@pytest.mark.parametrize("dist", ["uniform", "zipf"])
@pytest.mark.parametrize("n,m", [(0, 9), (1000, 7), (100_000, 256), (100_000, 4096),
                                 (100_000, 4097), (300_000, 65536), (200_000, 1 << 20)])
def test_rbi_sumprod(pcad, n, m, dist):
    """LDS table of (p, s) pairs up to 4096 bins, the partitioned path
    beyond; out-of-range keys; skew puts most elements into a few bins."""
    rng = np.random.default_rng(n + m)
    v = rng.standard_normal(n).astype(np.float32)
    if dist == "zipf":
        from workloads import zipf_keys
        idx = zipf_keys(rng, n, m) if n else np.zeros(0, np.int32)
    else:
        idx = rng.integers(0, m, n).astype(np.int32)
    if n:
        k = rng.choice(n, max(n // 97, 1), replace=False)
        idx[k] = rng.choice([-1, m, m + 5], k.size)
    hb = rng.standard_normal(m).astype(np.float32)
    I, V = dev(idx), dev(v)
    h, saved = pcad.rbi_fwd("sumprod", I, V, m)
    vb = pcad.rbi_vjp("sumprod", I, V, m, saved, dev(hb))
    h, vb, s = host(h), host(vb), host(saved)[: 4 * m].view(np.float32)
    o = oracle.sumprod_rbi_fwd(idx, m, v)
    assert_gate(h, o["hist"], o["c"], RTOL["sumprod"], what="rbi sumprod hist")
    cs = np.zeros(m)
    ok = (idx >= 0) & (idx < m)
    np.add.at(cs, idx[ok], np.abs(v[ok].astype(np.float64)))
    assert_gate(s, o["s"], cs, RTOL["add"], what="rbi sumprod s")
    xb, cx = oracle.sumprod_rbi_vjp(idx, m, hb, v)
    assert_gate(vb, xb, cx, RTOL["sumprod"], what="rbi sumprod vjp")
    assert ws_error() == 0


def test_rbi_sumprod_batched_and_accumulate(pcad):
    rng = np.random.default_rng(3)
    batch, n, m = 3, 50_001, 9000
    v = rng.standard_normal((batch, n)).astype(np.float32)
    idx = rng.integers(-1, m + 1, (batch, n)).astype(np.int32)
    hb = rng.standard_normal((batch, m)).astype(np.float32)
    I, V = dev(idx), dev(v)
    h, saved = pcad.rbi_fwd("sumprod", I, V, m)
    base = dev(np.full((batch, n), 0.5, np.float32))
    pcad.rbi_vjp("sumprod", I, V, m, saved, dev(hb), out=base, accumulate=True)
    h, vb = host(h), host(base)
    for r in range(batch):
        o = oracle.sumprod_rbi_fwd(idx[r], m, v[r])
        assert_gate(h[r], o["hist"], o["c"], RTOL["sumprod"], what=f"row {r}")
        xb, cx = oracle.sumprod_rbi_vjp(idx[r], m, hb[r], v[r])
        assert_gate(vb[r], xb + 0.5, cx + 0.5, RTOL["sumprod"], what=f"vjp row {r}")


# ---------------------------------------------------------------------------
# vectorised operators (Sections 3.2, 4.2, 5.3, Vectorized Operators)
# ---------------------------------------------------------------------------
VEC_SHAPES = [(1, 5000, 1), (1, 20_011, 3), (2, 9001, 16), (1, 3000, 100), (1, 70_000, 64)]


def _vec_values(op, shape, rng):
    x = rng.standard_normal(shape)
    if op == "mul":
        x = rng.uniform(0.9, 1.1, shape) * np.sign(x)
        x.reshape(-1)[rng.choice(x.size, max(x.size // 500, 1), replace=False)] = 0.0
    if op in ("min", "max"):
        x = np.round(x * 64) / 64
    return x.astype(np.float32)


def _check_cols(g, r, c, op, what):
    if op in ("min", "max"):
        np.testing.assert_array_equal(g, r.astype(np.float32), err_msg=what)
    else:
        assert_gate(g, r, c, RTOL[op], max_range_exceeded=g.size if op == "mul" else 0, what=what)


@pytest.mark.parametrize("op", SCALAR)
@pytest.mark.parametrize("batch,n,d", VEC_SHAPES)
def test_vreduce(pcad, op, batch, n, d):
    rng = np.random.default_rng(n + d + batch)
    x = _vec_values(op, (batch, n, d), rng)
    yb = rng.standard_normal((batch, d)).astype(np.float32)
    X = dev(x)
    y, saved = pcad.vreduce_fwd(op, X)
    g = pcad.vreduce_vjp(op, X, saved, dev(yb))
    y, g = host(y), host(g)
    for b in range(batch):
        o = oracle.vreduce_fwd(op, x[b])
        _check_cols(y[b], o["y"], o["c"], op, f"vreduce {op}")
        xb, cx = oracle.vreduce_vjp(op, yb[b], x[b])
        _check_cols(g[b], xb, cx, op, f"vreduce_vjp {op}")


@pytest.mark.parametrize("op", SCALAR)
@pytest.mark.parametrize("batch,n,d", VEC_SHAPES)
def test_vscan(pcad, op, batch, n, d):
    rng = np.random.default_rng(2 * n + d + batch)
    x = _vec_values(op, (batch, n, d), rng)
    yb = rng.standard_normal((batch, n, d)).astype(np.float32)
    X = dev(x)
    y, saved = pcad.vscan_fwd(op, X)
    base = dev(np.full((batch, n, d), 0.25, np.float32))
    pcad.vscan_vjp(op, X, saved, dev(yb), out=base, accumulate=True)
    y, g = host(y), host(base)
    for b in range(batch):
        Y, CY = oracle.vscan_fwd(op, x[b])
        _check_cols(y[b], Y, CY, op, f"vscan {op}")
        xb, cx = oracle.vscan_vjp(op, yb[b], x[b])
        # min/max adjoints of a scan are sums of y_bar (the running extremum
        # collects them), so every operator goes through the gate here
        assert_gate(g[b], xb + 0.25, cx + 0.25, RTOL[op], max_range_exceeded=g[b].size if op == "mul" else 0,
                    what=f"vscan_vjp {op}")


@pytest.mark.parametrize("op", SCALAR)
@pytest.mark.parametrize("batch,n,d,m", [(1, 5000, 1, 7), (1, 20_011, 3, 300), (2, 9001, 16, 1000),
                                         (1, 40_000, 8, 20_000), (1, 3000, 100, 64)])
def test_vrbi(pcad, op, batch, n, d, m):
    rng = np.random.default_rng(n + d + m)
    v = _vec_values(op, (batch, n, d), rng)
    idx = rng.integers(-2, m + 2, (batch, n)).astype(np.int32)
    hb = rng.standard_normal((batch, m, d)).astype(np.float32)
    I, V = dev(idx), dev(v)
    h, saved = pcad.vrbi_fwd(op, I, V, m)
    g = pcad.vrbi_vjp(op, I, V, m, saved, dev(hb))
    h, g = host(h), host(g)
    for b in range(batch):
        o = oracle.vrbi_fwd(op, idx[b], m, v[b])
        _check_cols(h[b], o["hist"], o["c"], op, f"vrbi {op}")
        xb, cx = oracle.vrbi_vjp(op, idx[b], m, hb[b], v[b])
        _check_cols(g[b], xb, cx, op, f"vrbi_vjp {op}")
    assert ws_error() == 0


def test_vectorised_rejects_other_operators(pcad):
    X = dev(np.ones((10, 4), np.float32))
    with pytest.raises(pcad.PcadError):
        pcad.vreduce_fwd("linrec", X)


# ---------------------------------------------------------------------------
# saturated addition (the evaluation's operator figure): scan (both adjoint
# forms), reduce (the general rule) and reduce-by-index (the sort-based
# general rule).  Values are positive multiples of 3: every partial sum is
# an exact float32 integer and none equals the cap 1e6, so the saturation
# decisions, and the bracketing-independent derivatives, agree exactly with
# the oracle's.
# ---------------------------------------------------------------------------
def _sat_values(rng, shape, hi):
    return (3 * rng.integers(1, hi, shape)).astype(np.float32)


@pytest.mark.parametrize("batch,n,hi", [(1, 1, 10), (1, 100_003, 11), (3, 30_001, 40), (2, 9000, 30_000),
                                        (1, 1 << 20, 3)])
def test_scan_satadd(pcad, batch, n, hi):
    rng = np.random.default_rng(n + hi)
    x = _sat_values(rng, (batch, n), hi)
    yb = rng.standard_normal((batch, n)).astype(np.float32)
    X = dev(x)
    y, _, saved = pcad.scan_fwd("satadd", X)
    g = pcad.scan_vjp("satadd", X, None, saved, dev(yb))
    gc = pcad.scan_vjp_checkpoint("satadd", X, None, y, None, dev(yb))
    y, g, gc = host(y), host(g), host(gc)
    for r in range(batch):
        rs, _ = oracle.scan_fwd("satadd", x[r])
        np.testing.assert_array_equal(y[r], rs[:, 0].astype(np.float32))
        xb, cx = oracle.scan_vjp("satadd", yb[r], x[r])
        assert_gate(g[r], xb[:, 0], cx[:, 0], RTOL["add"], what="scan satadd vjp")
        assert_gate(gc[r], xb[:, 0], cx[:, 0], RTOL["add"], what="scan satadd vjp checkpoint")
    assert ws_error() == 0


@pytest.mark.parametrize("batch,n,hi", [(1, 1, 10), (1, 50_000, 11), (1, 100_003, 5), (4, 20_001, 9)])
def test_reduce_satadd(pcad, batch, n, hi):
    """n*hi*3/2 against 1e6 puts some rows below the cap and some above."""
    rng = np.random.default_rng(7 * n + hi)
    x = _sat_values(rng, (batch, n), hi)
    yb = rng.standard_normal(batch).astype(np.float32)
    X = dev(x)
    y, saved = pcad.reduce_fwd("satadd", X)
    g = pcad.reduce_vjp("satadd", X, None, saved, dev(yb))
    y, g = host(y).reshape(batch), host(g).reshape(batch, n)
    for r in range(batch):
        o = oracle.reduce_fwd("satadd", x[r])
        assert y[r] == np.float32(o["y"][0])
        xb, _ = oracle.reduce_vjp("satadd", yb[r:r + 1], x[r])
        np.testing.assert_array_equal(g[r], xb[:, 0].astype(np.float32))


@pytest.mark.parametrize("n,m,hi", [(1000, 7, 30_000), (100_000, 64, 40), (200_003, 5000, 3_000),
                                    (100_000, 1 << 20, 300_000)])
def test_rbi_satadd(pcad, n, m, hi):
    rng = np.random.default_rng(n + m)
    v = _sat_values(rng, n, hi)
    idx = rng.integers(-2, m + 2, n).astype(np.int32)
    hb = rng.standard_normal(m).astype(np.float32)
    I, V = dev(idx), dev(v)
    h, saved = pcad.rbi_fwd("satadd", I, V, m)
    vb = pcad.rbi_vjp("satadd", I, V, m, saved, dev(hb))
    h, vb = host(h), host(vb)
    o = oracle.rbi_fwd("satadd", idx, m, v)
    np.testing.assert_array_equal(h, o["hist"][:, 0].astype(np.float32))
    xb, _ = oracle.rbi_vjp("satadd", idx, m, hb, v)
    np.testing.assert_array_equal(vb, xb[:, 0].astype(np.float32))
    assert ws_error() == 0


@pytest.mark.parametrize("batch,n", [(1, 1), (1, 5000), (1, 100_003), (3, 30_001), (1, 1 << 20)])
def test_scan_sumprod(pcad, batch, n):
    """Scans with sumOfProd (Section 3.3's operator, lifted pairs (p, s)):
    y_i = sum over j<k<=i of x_j x_k, and the adjoint by the right-to-left
    scan of lower-triangular adjoint maps."""
    rng = np.random.default_rng(n + batch)
    x = (rng.standard_normal((batch, n)) / np.sqrt(max(n, 1)) * 8).astype(np.float32)
    yb = rng.standard_normal((batch, n)).astype(np.float32)
    X = dev(x)
    y, _, saved = pcad.scan_fwd("sumprod", X)
    g = pcad.scan_vjp("sumprod", X, None, saved, dev(yb))
    y, g = host(y), host(g)
    for r in range(batch):
        Y, CY = oracle.sumprod_scan(x[r])
        assert_gate(y[r], Y, CY, RTOL["sumprod"], what="scan sumprod")
        xb, cx = oracle.sumprod_scan_vjp(x[r], yb[r])
        assert_gate(g[r], xb, cx, RTOL["sumprod"], what="scan sumprod vjp")
    assert ws_error() == 0
    with pytest.raises(pcad.PcadError):
        pcad.scan_vjp_checkpoint("sumprod", X, None, dev(y), None, dev(yb))


# ---------------------------------------------------------------------------
# scans of d x d matrix products (3x3, 5x5)
# ---------------------------------------------------------------------------
def _matd_gate(g, r, c, what):
    d = r.shape[-1]
    cc = np.repeat(c[:, None], d * d, axis=1).reshape(r.shape)
    assert_gate(g, r, cc, RTOL["mat2"], what=what)


def _ws_clear(pcad):
    """Zero every cached workspace (other calls leave tagged status words
    there, which the product scans may overwrite but need not clear)."""
    torch.cuda.synchronize()
    for buf in pcad._ws.values():
        buf.zero_()
    torch.cuda.synchronize()


def _ws_tail_zero(pcad, d, batch, n):
    """The product scans leave no temporaries behind them."""
    _, w_b = pcad.matd_query(d, batch, n)
    torch.cuda.synchronize()
    for buf in pcad._ws.values():
        assert int(buf[256:w_b].count_nonzero().item()) == 0


@pytest.mark.parametrize("d", [3, 5])
@pytest.mark.parametrize("batch,n,ens", [(1, 1, "orth"), (1, 700, "near"), (2, 3 * 1024 + 37, "orth"),
                                         (3, 2 * 512 + 1, "near"), (1, -1, "orth"), (2, -2, "orth")])
def test_matd_scan(pcad, d, batch, n, ens):
    """P_i = M_0 ... M_i and M_bar_i = P_{i-1}^T R_bar_i against the float64
    loops, over several tiles, a ragged tail and (n < 0) more tiles per row
    than one chunk of the tile scan holds (256 tiles of 1024 3x3 or 512 5x5
    elements)."""
    from workloads import matd
    if n < 0:
        n = (256 * -n + 1) * (1024 if d == 3 else 512) + 11
    w = matd(d, n, batch, ensemble=ens)
    print(f"matd d={d} batch={batch} n={n} {ens}", flush=True)
    M = dev(w["M"])
    _ws_clear(pcad)
    P, saved = pcad.matd_scan_fwd(M)
    Mb = pcad.matd_scan_vjp(M, saved, dev(w["Pbar"]))
    P, Mb = host(P), host(Mb)
    for r in range(batch):
        rs, c = oracle.matd_scan(w["M"][r])
        _matd_gate(P[r], rs, c, f"matd{d} scan row {r}")
        xb, cx = oracle.matd_scan_vjp(w["M"][r], w["Pbar"][r])
        _matd_gate(Mb[r], xb, cx, f"matd{d} vjp row {r}")
    _ws_tail_zero(pcad, d, batch, n)


@pytest.mark.parametrize("d", [3, 5])
def test_matd_scan_accumulate_and_empty(pcad, d):
    from workloads import matd
    w = matd(d, 1500, 2, ensemble="near")
    M = dev(w["M"])
    P, saved = pcad.matd_scan_fwd(M)
    base = np.random.default_rng(d).standard_normal(w["M"].shape).astype(np.float32)
    out = dev(base)
    pcad.matd_scan_vjp(M, saved, dev(w["Pbar"]), out=out, accumulate=True)
    g = host(out) - base
    for r in range(2):
        xb, cx = oracle.matd_scan_vjp(w["M"][r], w["Pbar"][r])
        cc = np.repeat(cx[:, None], d * d, axis=1).reshape(xb.shape) + np.abs(base[r])
        assert_gate(g[r], xb, cc, RTOL["mat2"], what=f"matd{d} accumulate")
    E = torch.empty((3, 0, d, d), device="cuda")
    P0, s0 = pcad.matd_scan_fwd(E)
    assert P0.shape == E.shape
    assert pcad.matd_scan_vjp(E, s0, E).shape == E.shape
    with pytest.raises(pcad.PcadError):
        pcad.matd_scan_fwd(torch.empty((4, 4, 4), device="cuda"))


@pytest.mark.parametrize("d", [3, 5])
@pytest.mark.parametrize("batch,n", [(1, 1), (2, 777), (3, 2 * 1024 + 5), (1, -1)])
def test_matd_reduce(pcad, d, batch, n):
    """Y = M_0 ... M_{n-1} and Mbar_i = L_i^T Ybar R_i^T (Section 3.1's rule)
    against the float64 oracle; n < 0: more tiles than one chunk holds."""
    from workloads import matd
    if n < 0:
        n = 257 * (1024 if d == 3 else 512) + 3
    w = matd(d, n, batch, ensemble="orth")
    print(f"matd reduce d={d} batch={batch} n={n}", flush=True)
    yb = np.random.default_rng(n + d).standard_normal((batch, d, d)).astype(np.float32)
    M = dev(w["M"])
    _ws_clear(pcad)
    Y, saved = pcad.matd_reduce_fwd(M)
    base = np.random.default_rng(d).standard_normal(w["M"].shape).astype(np.float32)
    out = dev(base)
    pcad.matd_reduce_vjp(M, saved, dev(yb), out=out, accumulate=True)
    Y, g = host(Y), host(out) - base
    for r in range(batch):
        ry, cy = oracle.matd_reduce(w["M"][r])
        assert_gate(Y[r], ry, np.full(ry.shape, cy), RTOL["mat2"], what=f"matd{d} reduce row {r}")
        xb, cx = oracle.matd_reduce_vjp(w["M"][r], yb[r])
        cc = np.repeat(cx[:, None], d * d, axis=1).reshape(xb.shape) + np.abs(base[r])
        assert_gate(g[r], xb, cc, RTOL["mat2"], what=f"matd{d} reduce vjp row {r}")
    _ws_tail_zero(pcad, d, batch, n)
    Y0, s0 = pcad.matd_reduce_fwd(torch.empty((2, 0, d, d), device="cuda"))
    np.testing.assert_array_equal(host(Y0), np.broadcast_to(np.eye(d, dtype=np.float32), (2, d, d)))


# ---------------------------------------------------------------------------
# int32 forward combinators (+ * min max wrapping mod 2^32): bit-exact
# ---------------------------------------------------------------------------
def _i32_inputs(op, shape, rng):
    if op == "mul":  # small factors: products wrap many times without going to 0
        x = rng.choice(np.array([-3, -1, 1, 3, 5, 7], np.int64), size=shape)
    else:
        x = rng.integers(-2**31, 2**31, size=shape, dtype=np.int64)
    return x.astype(np.int32)


@pytest.mark.parametrize("op", SCALAR)
@pytest.mark.parametrize("batch,n", [(1, 1), (1, 4095), (2, 4097), (3, 50_001), (1, 1_050_011)])
def test_i32_reduce_and_scan(pcad, op, batch, n):
    rng = np.random.default_rng(n + len(op))
    x = _i32_inputs(op, (batch, n), rng)
    X = dev(x)
    y = host(pcad.i32_fwd(pcad.REDUCE, op, X))
    s = host(pcad.i32_fwd(pcad.SCAN, op, X))
    for r in range(batch):
        assert int(y[r]) == oracle.i32_reduce(op, x[r])
        if n <= 60_000 or r == 0:
            np.testing.assert_array_equal(s[r], oracle.i32_scan(op, x[r]))
    assert ws_error() == 0


@pytest.mark.parametrize("op", SCALAR)
@pytest.mark.parametrize("batch,n,m", [(1, 0, 5), (1, 1, 1), (2, 30_001, 300), (1, 100_000, 8192),
                                       (1, 100_000, 8193), (1, 700_001, 100_000), (2, 20_000, 9000),
                                       (1, 60_000, 1 << 20)])
def test_i32_rbi(pcad, op, batch, n, m):
    rng = np.random.default_rng(n + m + len(op))
    x = _i32_inputs(op, (batch, n), rng)
    idx = rng.integers(-2, m + 2, size=(batch, n)).astype(np.int32)
    h = host(pcad.i32_fwd(pcad.RBI, op, dev(x), dev(idx), m))
    for r in range(batch):
        np.testing.assert_array_equal(h[r], oracle.i32_rbi(op, idx[r], m, x[r]))


def test_i32_empty_and_rejects(pcad):
    y = host(pcad.i32_fwd(pcad.REDUCE, "min", torch.empty((3, 0), dtype=torch.int32, device="cuda")))
    np.testing.assert_array_equal(y, np.full(3, 2**31 - 1, np.int32))
    with pytest.raises(pcad.PcadError):
        pcad.i32_fwd(pcad.SCAN, "linrec", torch.zeros(10, dtype=torch.int32, device="cuda"))
    with pytest.raises(pcad.PcadError):
        pcad.i32_fwd(pcad.SCAN, "add", torch.zeros(10, dtype=torch.float32, device="cuda"))
