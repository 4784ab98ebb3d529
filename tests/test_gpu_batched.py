"""Batched segmented plan (one hipGraph per phase) against the oracle.

Per instance: y = linear-recurrence scan of (a, b); (h, argk) = min-by-index
of y into m bins; adjoint with y_bar and h_bar.  The min decision is taken on
float32 values on both sides; where the oracle's two best candidates of a bin
lie within rounding of each other either index is a valid argmin, so argk is
compared exactly only where the minimum is unique beyond rounding, and the
adjoint is checked with the oracle's decision written into argk.
"""
from __future__ import annotations

import numpy as np
import pytest
import torch

import oracle
from oracle.gate import assert_gate

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def pcad():
    import paper_2310_03568_amd as p
    p.lib()
    return p


def workload(lengths, m, seed):
    rng = np.random.default_rng(seed)
    off = np.zeros(len(lengths) + 1, np.int64)
    np.cumsum(lengths, out=off[1:])
    N = int(off[-1])
    return dict(
        offsets=off, m=m,
        a=rng.uniform(0.9, 1.0, N).astype(np.float32),
        b=rng.standard_normal(N).astype(np.float32),
        idx=rng.integers(0, m, N).astype(np.int32),
        ybar=rng.standard_normal(N).astype(np.float32),
        hbar=rng.standard_normal(len(lengths) * m).astype(np.float32),
    )


def ragged_lengths(seed):
    from workloads import segment_lengths
    rng = np.random.default_rng(seed)
    L = list(segment_lengths(rng, 40, median=700, cap=30_000))
    # edge cases: single element, exact window, one past it, a long instance, empty
    return L + [1, 8192, 8193, 25_001, 0, 3]


def check_forward(p, w, y, h, argk, what):
    off, m = w["offsets"], w["m"]
    S = len(off) - 1
    f = oracle.segmented_fwd(off, w["a"], w["b"], w["idx"], m)
    assert_gate(y, f["y"], f["cy"], 1e-4, what=f"{what} y")
    h = h.reshape(S, m)
    argk = argk.reshape(S, m)
    ambiguous = 0
    for s in range(S):
        lo, hi = int(off[s]), int(off[s + 1])
        L = hi - lo
        for k in np.flatnonzero(argk[s] != f["argk"][s]):
            g, r = int(argk[s, k]), int(f["argk"][s, k])
            assert g < L and r < L, (s, k, g, r)
            assert w["idx"][lo + g] == k
            # both positions must tie within rounding in the oracle
            assert abs(f["y"][lo + g] - f["y"][lo + r]) <= 1e-4 * (f["cy"][lo + g] + f["cy"][lo + r])
            ambiguous += 1
        ok = argk[s] < L
        # h is the float32 y at the chosen position, bit for bit
        np.testing.assert_array_equal(h[s][ok], y[lo + argk[s][ok]])
        assert np.all(np.isinf(h[s][~ok])) and np.all(argk[s][~ok] == L)
    assert ambiguous <= max(2, S * m // 5000), ambiguous
    return f


def check_backward(w, f, abar, bbar, what):
    ab, bb, cab, cbb = oracle.segmented_vjp(w["offsets"], w["a"], w["b"], w["idx"], w["m"],
                                            w["ybar"], w["hbar"], f["argk"])
    assert_gate(abar, ab, cab, 1e-4, what=f"{what} a_bar")
    assert_gate(bbar, bb, cbb, 1e-4, what=f"{what} b_bar")


@pytest.mark.parametrize("m", [16, 512])
def test_plan_matches_oracle(pcad, m):
    w = workload(ragged_lengths(1), m, seed=2)
    plan = pcad.BatchedPlan(w["offsets"], m, per_segment=True)
    plan.load(a=w["a"], b=w["b"], idx=w["idx"], ybar=w["ybar"], hbar=w["hbar"])
    N = plan.n
    f = None
    for rep in range(3):
        plan.run(pcad.PHASE_FWD)
        torch.cuda.synchronize()
        y = plan.y[:N].cpu().numpy()
        f = check_forward(pcad, w, y, plan.h.cpu().numpy(), plan.argk.cpu().numpy(), f"graph fwd #{rep}")
        # eager work between replays
        _ = (plan.y[:N] * 2).sum().item()
    # adjoint with the oracle's decision in argk
    plan.argk.copy_(torch.from_numpy(f["argk"].reshape(-1).astype(np.int32)))
    for rep in range(3):
        plan.run(pcad.PHASE_BWD)
        torch.cuda.synchronize()
        check_backward(w, f, plan.abar[:N].cpu().numpy(), plan.bbar[:N].cpu().numpy(), f"graph bwd #{rep}")
    # both phases in one launch, then the per-instance path
    plan.run(pcad.PHASE_BOTH)
    torch.cuda.synchronize()
    f2 = check_forward(pcad, w, plan.y[:N].cpu().numpy(), plan.h.cpu().numpy(),
                       plan.argk.cpu().numpy(), "graph both")
    plan.run_per_segment(pcad.PHASE_FWD)
    torch.cuda.synchronize()
    check_forward(pcad, w, plan.y[:N].cpu().numpy(), plan.h.cpu().numpy(), plan.argk.cpu().numpy(),
                  "per-instance fwd")
    plan.argk.copy_(torch.from_numpy(f["argk"].reshape(-1).astype(np.int32)))
    plan.run_per_segment(pcad.PHASE_BWD)
    torch.cuda.synchronize()
    check_backward(w, f, plan.abar[:N].cpu().numpy(), plan.bbar[:N].cpu().numpy(), "per-instance bwd")
    assert plan.ws_error() == 0
    plan.close()


def test_plan_segmented_workload_scaled(pcad):
    """The segmented workload's distributions at 1/16 of its instance count."""
    from workloads import segmented
    w = segmented(S=256)
    plan = pcad.BatchedPlan(w["offsets"], w["m"])
    plan.load(a=w["a"], b=w["b"], idx=w["idx"], ybar=w["ybar"], hbar=w["hbar"])
    plan.run(pcad.PHASE_FWD)
    torch.cuda.synchronize()
    N = plan.n
    f = check_forward(pcad, w, plan.y[:N].cpu().numpy(), plan.h.cpu().numpy(),
                      plan.argk.cpu().numpy(), "segmented fwd")
    plan.argk.copy_(torch.from_numpy(f["argk"].reshape(-1).astype(np.int32)))
    plan.run(pcad.PHASE_BWD)
    torch.cuda.synchronize()
    check_backward(w, f, plan.abar[:N].cpu().numpy(), plan.bbar[:N].cpu().numpy(), "segmented bwd")
    assert plan.ws_error() == 0
    plan.close()


def test_plan_argument_errors(pcad):
    import ctypes
    L = pcad.lib()
    h = ctypes.c_void_p()
    off = np.array([0, 5, 3], np.int64)  # decreasing
    assert L.pcad_plan_create(ctypes.byref(h), 2, off.ctypes.data, 8, 0) == 1
    off = np.array([0, 5, 9], np.int64)
    assert L.pcad_plan_create(ctypes.byref(h), 2, off.ctypes.data, 5000, 0) == 5
    assert L.pcad_plan_create(ctypes.byref(h), 2, off.ctypes.data, 8, 1 << 4) == 1
    assert L.pcad_plan_create(ctypes.byref(h), 2, off.ctypes.data, 8, 0) == 0
    assert L.pcad_plan_run(h, 1, None) == 1  # not bound
    L.pcad_plan_destroy(h)


def test_plan_many_instances_both_paths_interleaved(pcad):
    """4096 short instances (the instance count of the segmented workload):
    graph and per-instance runs interleaved on one plan, each checked; the
    per-instance calls share the plan's workspace with the graph kernels'
    instance tables, which must stay intact."""
    from workloads import segment_lengths
    rng = np.random.default_rng(41)
    L = list(segment_lengths(rng, 4096, median=96, cap=4000))
    w = workload(L, 512, seed=42)
    plan = pcad.BatchedPlan(w["offsets"], 512, per_segment=True)
    plan.load(a=w["a"], b=w["b"], idx=w["idx"], ybar=w["ybar"], hbar=w["hbar"])
    N = plan.n
    f = None
    for rnd in range(2):
        for path in ("graph", "per-instance"):
            run = plan.run if path == "graph" else plan.run_per_segment
            run(pcad.PHASE_FWD)
            torch.cuda.synchronize()
            f = check_forward(pcad, w, plan.y[:N].cpu().numpy(), plan.h.cpu().numpy(),
                              plan.argk.cpu().numpy(), f"{path} fwd round {rnd}")
            plan.argk.copy_(torch.from_numpy(f["argk"].reshape(-1).astype(np.int32)))
            run(pcad.PHASE_BWD)
            torch.cuda.synchronize()
            check_backward(w, f, plan.abar[:N].cpu().numpy(), plan.bbar[:N].cpu().numpy(),
                           f"{path} bwd round {rnd}")
    assert plan.ws_error() == 0
    plan.close()
