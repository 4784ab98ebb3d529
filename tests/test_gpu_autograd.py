"""Autograd Functions over the HIP kernels against the oracle.

The autograd workload (64 sequences of 2^16; loss = sum log|y| of the
linear recurrence + sum over non-empty bins of max-by-index) runs in both
saved-state forms; every Function is also checked on small random cases
with a random cotangent.  The scan adjoint's seed is taken from autograd
itself (a hook on y), so the oracle sees the float32 seed the kernels saw.
"""
from __future__ import annotations

import numpy as np
import pytest
import torch

import oracle
from oracle.gate import RTOL, assert_discriminates, assert_gate

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ag():
    import paper_2310_03568_amd as p
    p.lib()
    import paper_2310_03568_amd.autograd as a
    return a


def dev(x, grad=False):
    t = torch.from_numpy(np.ascontiguousarray(x)).cuda()
    return t.requires_grad_(grad) if grad else t


def host(t):
    torch.cuda.synchronize()
    return t.detach().cpu().numpy()


def run_loss(ag, w, mode):
    a, b, v = dev(w["a"], True), dev(w["b"], True), dev(w["v"], True)
    idx = dev(w["idx"])
    seed = {}
    y = ag.scan_linrec(a, b, mode=mode)
    y.register_hook(lambda g: seed.setdefault("ybar", g.detach().clone()))
    h = ag.reduce_by_index("max", idx, v, w["m"])
    loss = torch.log(torch.abs(y)).sum() + torch.where(torch.isfinite(h), h, 0).sum()
    loss.backward()
    return host(a.grad), host(b.grad), host(v.grad), host(seed["ybar"]), float(loss.detach())


@pytest.mark.parametrize("mode", ["recompute", "checkpoint"])
def test_autograd_workload(ag, mode):
    from workloads import autograd
    w = autograd()
    B, T, m = w["a"].shape[0], w["a"].shape[1], w["m"]
    print(f"autograd workload B={B} T={T} m={m} mode={mode}", flush=True)
    torch.cuda.reset_peak_memory_stats()
    ga, gb, gv, ybar, loss = run_loss(ag, w, mode)
    print(f"peak bytes {torch.cuda.max_memory_allocated()} loss {loss}", flush=True)
    ref_loss = 0.0
    for s in range(B):
        ref_loss += oracle.autograd_loss(w["a"][s], w["b"][s], w["v"][s], w["idx"][s], m)
        ab, bb, vb, ca, cb, cv = oracle.autograd_grad(w["a"][s], w["b"][s], w["v"][s],
                                                      w["idx"][s], m, ybar=ybar[s])
        assert_gate(ga[s], ab, ca, RTOL["linrec"], what=f"a_bar seq {s}")
        assert_gate(gb[s], bb, cb, RTOL["linrec"], what=f"b_bar seq {s}")
        np.testing.assert_array_equal(gv[s], vb.astype(np.float32))
    # the loss sums 4M float32 logs: compare in relative terms
    assert abs(loss - ref_loss) <= 1e-4 * (abs(ref_loss) + B * T), (loss, ref_loss)


def loss64_gpu(a, b, v, idx, m, chunk=256):
    """The autograd workload's loss of ONE sequence in float64 on the GPU with
    plain torch operations (finite-difference reference): the recurrence in
    chunks (sequential inside a chunk, vectorised across chunks, then the
    chunk carries), and the max per bin by scatter_reduce."""
    T = a.shape[0]
    C = T // chunk
    A = a.view(C, chunk)
    B = b.view(C, chunk)
    yl = torch.empty_like(B)
    Al = torch.empty_like(A)
    prev_y = torch.zeros(C, dtype=a.dtype, device=a.device)
    prev_A = torch.ones(C, dtype=a.dtype, device=a.device)
    for i in range(chunk):
        prev_y = A[:, i] * prev_y + B[:, i]
        prev_A = A[:, i] * prev_A
        yl[:, i] = prev_y
        Al[:, i] = prev_A
    carry = torch.zeros(C, dtype=a.dtype, device=a.device)
    c = torch.zeros((), dtype=a.dtype, device=a.device)
    for k in range(1, C):
        c = Al[k - 1, -1] * c + yl[k - 1, -1]
        carry[k] = c
    y = yl + Al * carry[:, None]
    h = torch.full((m,), -float("inf"), dtype=v.dtype, device=v.device)
    h = h.scatter_reduce(0, idx.long(), v, reduce="amax", include_self=True)
    return float(torch.log(torch.abs(y)).sum() + h[torch.isfinite(h)].sum())


def test_autograd_central_differences_fp64(ag):
    """Gradient through the autograd Functions against FP64 central
    differences on the GPU at 32 coordinates drawn from a, b and v (a v
    coordinate within 2h of another value of its bin is redrawn)."""
    from workloads import autograd
    w = autograd()
    B, T, m = w["a"].shape[0], w["a"].shape[1], w["m"]
    ga, gb, gv, ybar, _ = run_loss(ag, w, "recompute")
    rng = np.random.default_rng(2310)
    picked = 0
    while picked < 32:
        which = int(rng.integers(0, 3))
        s, j = int(rng.integers(0, B)), int(rng.integers(0, T))
        x = (w["a"], w["b"], w["v"])[which][s].astype(np.float64)
        h = 1e-6 * max(1.0, abs(x[j]))
        if which == 2:
            same = np.flatnonzero(w["idx"][s] == w["idx"][s][j])
            if np.any(np.abs(x[same[same != j]] - x[j]) <= 2 * h):
                continue
        picked += 1
        args = [torch.from_numpy(w[k][s].astype(np.float64)).cuda() for k in ("a", "b", "v")]
        idx = torch.from_numpy(w["idx"][s]).cuda()
        args[which][j] += h
        fp = loss64_gpu(args[0], args[1], args[2], idx, m)
        args[which][j] -= 2 * h
        fm = loss64_gpu(args[0], args[1], args[2], idx, m)
        fd = (fp - fm) / (2 * h)
        g = (ga, gb, gv)[which][s, j]
        # the float32 gradient's own bound (the oracle companion) plus the
        # difference quotient's rounding (eps * |loss| / h) and truncation
        _, _, _, ca, cb, cv = oracle.autograd_grad(w["a"][s], w["b"][s], w["v"][s], w["idx"][s], m,
                                                   ybar=ybar[s])
        comp = (ca, cb, cv)[which][j]
        tol = 1e-4 * comp + 1e-15 * abs(fp) / h * 8 + 1e-6 * abs(fd)
        print(f"coord {'abv'[which]}[{s},{j}] fd {fd:.9g} grad {g:.9g} tol {tol:.3g}", flush=True)
        assert abs(fd - g) <= tol, (which, s, j, fd, g, tol)


def test_modes_agree(ag):
    from workloads import autograd
    w = autograd(B=4, T=1 << 14, m=1 << 14, seed=11)
    r = run_loss(ag, w, "recompute")
    c = run_loss(ag, w, "checkpoint")
    np.testing.assert_array_equal(r[2], c[2])
    for g, h, what in ((r[0], c[0], "a_bar"), (r[1], c[1], "b_bar")):
        scale = np.abs(g).max()
        assert np.max(np.abs(g - h)) <= 1e-4 * scale, what


SCAN_OPS = ["add", "mul", "min", "max", "linrec", "mat2"]


@pytest.mark.parametrize("op", SCAN_OPS)
@pytest.mark.parametrize("mode", ["recompute", "checkpoint"])
def test_scan_function(ag, op, mode):
    # a fixed seed per case (Python's string hash changes between runs)
    rng = np.random.default_rng(1000 + 10 * SCAN_OPS.index(op) + (mode == "checkpoint"))
    n = 20_001
    if op == "linrec":
        x0 = rng.uniform(0.9, 1.0, (2, n)).astype(np.float32)
        x1 = rng.standard_normal((2, n)).astype(np.float32)
    elif op == "mat2":
        # orthogonal factors: every product and adjoint stays in range
        from workloads import o2_matrices
        x0 = o2_matrices(rng, 2 * n).reshape(2, n, 4)
        x1 = None
    elif op == "mul":
        # +-exp(U[-0.01, 0.01]): finite, non-zero products over all of n
        x0 = (rng.choice([-1.0, 1.0], (2, n)) * np.exp(rng.uniform(-0.01, 0.01, (2, n)))).astype(np.float32)
        x1 = None
    else:
        x0 = rng.uniform(0.5, 2.0, (2, n)).astype(np.float32)
        x1 = None
    X0 = dev(x0, True)
    X1 = dev(x1, True) if x1 is not None else None
    out = ag.scan(op, X0, X1, mode=mode, return_A=(op == "linrec"))
    yb = rng.standard_normal(x0.shape).astype(np.float32)
    if op == "linrec":
        y, A = out
        Ab = rng.standard_normal(x0.shape).astype(np.float32)
        torch.autograd.backward([y, A], [dev(yb), dev(Ab)])
    else:
        out.backward(dev(yb))
    g0 = host(X0.grad)
    g1 = host(X1.grad) if X1 is not None else None
    for r in range(2):
        if op == "linrec":
            xb, cx = oracle.scan_vjp(op, np.stack([Ab[r], yb[r]], 1), x0[r], x1[r])
            assert_gate(g0[r], xb[:, 0], cx[:, 0], RTOL[op], what=f"{op} a_bar")
            assert_gate(g1[r], xb[:, 1], cx[:, 1], RTOL[op], what=f"{op} b_bar")
        elif op == "mat2":
            xb, cx = oracle.scan_vjp(op, yb[r], x0[r])
            assert_gate(g0[r], xb, cx, RTOL[op], max_range_exceeded=0, what="mat2")
            assert_discriminates(g0[r], xb, cx, RTOL[op], width=4, what="mat2")
        else:
            xb, cx = oracle.scan_vjp(op, yb[r], x0[r])
            assert_gate(g0[r], xb[:, 0], cx[:, 0], RTOL[op], what=op)
            if op in ("add", "mul"):
                assert_discriminates(g0[r], xb[:, 0], cx[:, 0], RTOL[op], what=op)


@pytest.mark.parametrize("op", SCAN_OPS)
def test_reduce_function(ag, op):
    rng = np.random.default_rng(2000 + SCAN_OPS.index(op))
    n = 30_001
    x1 = None
    if op == "linrec":
        x0 = rng.uniform(0.9, 1.0, (3, n)).astype(np.float32)
        x1 = rng.standard_normal((3, n)).astype(np.float32)
    elif op == "mat2":
        from workloads import o2_matrices
        x0 = o2_matrices(rng, 3 * n).reshape(3, n, 4)
    elif op == "mul":
        # finite non-zero products; one row with a single exact zero
        x0 = (rng.choice([-1.0, 1.0], (3, n)) * np.exp(rng.uniform(-0.01, 0.01, (3, n)))).astype(np.float32)
        x0[1, 17] = 0.0
    else:
        x0 = rng.uniform(0.5, 2.0, (3, n)).astype(np.float32)
    X0 = dev(x0, True)
    X1 = dev(x1, True) if x1 is not None else None
    y = ag.reduce(op, X0, X1)
    yb = rng.standard_normal(tuple(y.shape)).astype(np.float32)
    y.backward(dev(yb))
    g0 = host(X0.grad)
    for r in range(3):
        xb, cx = oracle.reduce_vjp(op, yb[r], x0[r], None if x1 is None else x1[r])
        if op == "linrec":
            assert_gate(g0[r], xb[:, 0], cx[:, 0], RTOL[op], what="reduce linrec a_bar")
            assert_gate(host(X1.grad)[r], xb[:, 1], cx[:, 1], RTOL[op], what="reduce linrec b_bar")
        elif op == "mat2":
            assert_gate(g0[r], xb, cx, RTOL[op], max_range_exceeded=0, what="reduce mat2")
            assert_discriminates(g0[r], xb, cx, RTOL[op], width=4, what="reduce mat2")
        else:
            assert_gate(g0[r], xb[:, 0], cx[:, 0], RTOL[op], what=f"reduce {op}")


@pytest.mark.parametrize("op", ["add", "mul", "min", "max"])
def test_reduce_by_index_function(ag, op):
    rng = np.random.default_rng(40 + len(op))
    n, m = 50_000, 777
    v = rng.uniform(0.5, 2.0, n).astype(np.float32)
    if op in ("min", "max"):
        v = np.floor(v * 8) / 8  # ties
    if op == "mul":
        v[rng.choice(n, 50, replace=False)] = 0.0
    idx = rng.integers(-3, m + 3, n).astype(np.int32)  # some keys out of range
    V = dev(v, True)
    out = ag.reduce_by_index(op, dev(idx), V, m, return_argk=op in ("min", "max"))
    h = out[0] if isinstance(out, tuple) else out
    hb = rng.standard_normal(m).astype(np.float32)
    h.backward(dev(hb))
    vb, cv = oracle.rbi_vjp(op, idx, m, hb, v)
    g = host(V.grad)
    if op in ("add", "min", "max"):
        np.testing.assert_array_equal(g, vb[:, 0].astype(np.float32))
        if op != "add":
            r = oracle.rbi_fwd(op, idx, m, v)
            np.testing.assert_array_equal(host(out[1]).astype(np.int64), r["argk"])
    else:
        assert_gate(g, vb[:, 0], cv[:, 0], RTOL[op], what="rbi mul")


def test_sumprod_functions(ag):
    """sumOfProd through the autograd Functions: the gradient of
    sum_{i<j} a_i a_j is S - a (Section 3.3), and of sum_k w_k hist_k over a
    reduce-by-index it is (s_k - v_i) w_k (Section 4.2); both against the
    oracle's reverse sweep."""
    rng = np.random.default_rng(17)
    a_np = rng.standard_normal(30_001).astype(np.float32)
    a = torch.from_numpy(a_np).cuda().requires_grad_(True)
    y = ag.reduce("sumprod", a)
    y.backward()
    o = oracle.sumprod_reduce(a_np)
    assert_gate([y.item()], [o["y"]], [o["c"]], RTOL["sumprod"], what="sumprod y")
    xb, cx = oracle.sumprod_reduce_vjp(a_np, 1.0)
    assert_gate(a.grad.cpu().numpy(), xb, cx, RTOL["sumprod"], what="sumprod grad")

    m = 5000
    v_np = rng.standard_normal(40_000).astype(np.float32)
    idx_np = rng.integers(-1, m + 1, 40_000).astype(np.int32)
    w_np = rng.standard_normal(m).astype(np.float32)
    v = torch.from_numpy(v_np).cuda().requires_grad_(True)
    h = ag.reduce_by_index("sumprod", torch.from_numpy(idx_np).cuda(), v, m)
    (h * torch.from_numpy(w_np).cuda()).sum().backward()
    vb, cv = oracle.sumprod_rbi_vjp(idx_np, m, w_np, v_np)
    assert_gate(v.grad.cpu().numpy(), vb, cv, RTOL["sumprod"], what="sumprod rbi grad")


@pytest.mark.parametrize("d", [3, 5])
def test_matd_functions(ag, d):
    """3x3 / 5x5 products through autograd: the gradient of sum(W * P) for the
    scan and of sum(V * Y) for the reduce against the oracle's reverse
    sweeps, on orthogonal factors."""
    from workloads import matd
    w = matd(d, 3001, 2, ensemble="near")
    M = torch.from_numpy(w["M"]).cuda().requires_grad_(True)
    W = torch.from_numpy(w["Pbar"]).cuda()
    (ag.scan_matd(M) * W).sum().backward()
    g = host(M.grad)
    for r in range(2):
        xb, cx = oracle.matd_scan_vjp(w["M"][r], w["Pbar"][r])
        cc = np.repeat(cx[:, None], d * d, axis=1).reshape(xb.shape)
        assert_gate(g[r], xb, cc, RTOL["mat2"], what=f"matd{d} scan grad")
    M.grad = None
    V = np.random.default_rng(d).standard_normal((2, d, d)).astype(np.float32)
    (ag.reduce_matd(M) * torch.from_numpy(V).cuda()).sum().backward()
    g = host(M.grad)
    for r in range(2):
        xb, cx = oracle.matd_reduce_vjp(w["M"][r], V[r])
        cc = np.repeat(cx[:, None], d * d, axis=1).reshape(xb.shape)
        assert_gate(g[r], xb, cc, RTOL["mat2"], what=f"matd{d} reduce grad")


@pytest.mark.parametrize("op", ["add", "mul", "min", "max"])
def test_vectorised_functions(ag, op):
    """map2 operators through autograd against the oracle's per-component
    adjoints."""
    rng = np.random.default_rng(len(op) + 40)
    n, d, m = 5000, 7, 300
    x = rng.uniform(0.5, 2.0, (n, d)).astype(np.float32)
    if op in ("min", "max"):
        x = np.floor(x * 8) / 8
    X = dev(x, True)
    wy = rng.standard_normal((n, d)).astype(np.float32)
    (ag.vscan(op, X) * dev(wy)).sum().backward()
    # products of thousands of factors in [0.5, 2) leave the float32 range
    rx = n * d if op == "mul" else 0
    xb, cx = oracle.vscan_vjp(op, wy, x)
    assert_gate(host(X.grad), xb, cx, RTOL[op], max_range_exceeded=rx, what=f"vscan {op}")
    X.grad = None
    wr = rng.standard_normal(d).astype(np.float32)
    (ag.vreduce(op, X) * dev(wr)).sum().backward()
    xb, cx = oracle.vreduce_vjp(op, wr, x)
    assert_gate(host(X.grad), xb, cx, RTOL[op], max_range_exceeded=rx, what=f"vreduce {op}")
    X.grad = None
    idx = rng.integers(-1, m + 1, n).astype(np.int32)
    wh = rng.standard_normal((m, d)).astype(np.float32)
    (ag.vreduce_by_index(op, torch.from_numpy(idx).cuda(), X, m) * dev(wh)).sum().backward()
    xb, cx = oracle.vrbi_vjp(op, idx, m, wh, x)
    assert_gate(host(X.grad), xb, cx, RTOL[op], what=f"vrbi {op}")
