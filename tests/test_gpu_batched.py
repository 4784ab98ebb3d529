"""Batched segmented plan (one hipGraph per phase) against the oracle.

Per instance: y = linear-recurrence scan of (a, b); (h, argk) = min-by-index
of y into m bins; adjoint with y_bar and h_bar.

y is gated against the oracle's float64 recurrence.  The min-by-index
consumes the GPU's own float32 y, so its decisions are checked exactly
against the oracle's min-by-index of that same y (Section 4.2: lowest index
of the bin's minimum, bit for bit, every bin); h must be y at argk bit for
bit, except that a -0.0 winner reads +0.0 (the packed 64-bit keys fold the
two zeros).  Where the oracle's float64 y would choose another position, the
two candidates must tie within rounding.  The adjoint runs on the plan's own
argk and is gated against the oracle's adjoint for that decision.
"""
from __future__ import annotations

import numpy as np
import pytest
import torch

import oracle
from oracle.gate import assert_gate, segmented_decisions

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


def check_forward(p, w, y, h, argk, what, exact_decisions=False):
    off, m = w["offsets"], w["m"]
    S = len(off) - 1
    f = oracle.segmented_fwd(off, w["a"], w["b"], w["idx"], m)
    assert_gate(y, f["y"], f["cy"], 1e-4, what=f"{what} y")
    d = segmented_decisions(off, w["idx"], m, y, h, argk, f)
    assert d["argk_ok"], f"{what}: {d['argk_bad_bins']} bins whose argk is not the lowest-index minimum"
    assert d["h_ok"], f"{what}: h is not y at argk"
    assert d["diff_ok"], f"{what}: a decision differs from the oracle's without a tie"
    if exact_decisions:
        assert d["n_diff_oracle"] == 0, (what, d)
    assert d["n_diff_oracle"] <= max(2, S * m // 5000), d
    return f


def check_backward(w, argk, abar, bbar, what):
    """adjoint for the decision ``argk`` (the plan's own, already checked)"""
    S = len(w["offsets"]) - 1
    ab, bb, cab, cbb = oracle.segmented_vjp(w["offsets"], w["a"], w["b"], w["idx"], w["m"],
                                            w["ybar"], w["hbar"], argk.reshape(S, w["m"]))
    assert_gate(abar, ab, cab, 1e-4, what=f"{what} a_bar")
    assert_gate(bbar, bb, cbb, 1e-4, what=f"{what} b_bar")


@pytest.mark.parametrize("m", [16, 512])
def test_plan_matches_oracle(pcad, m):
    w = workload(ragged_lengths(1), m, seed=2)
    plan = pcad.BatchedPlan(w["offsets"], m, per_segment=True)
    plan.load(a=w["a"], b=w["b"], idx=w["idx"], ybar=w["ybar"], hbar=w["hbar"])
    N = plan.n
    for rep in range(3):
        plan.run(pcad.PHASE_FWD)
        torch.cuda.synchronize()
        y = plan.y[:N].cpu().numpy()
        check_forward(pcad, w, y, plan.h.cpu().numpy(), plan.argk.cpu().numpy(), f"graph fwd #{rep}")
        # eager work between replays
        _ = (plan.y[:N] * 2).sum().item()
    # adjoint on the plan's own argk
    ak = plan.argk.cpu().numpy()
    for rep in range(3):
        plan.run(pcad.PHASE_BWD)
        torch.cuda.synchronize()
        check_backward(w, ak, plan.abar[:N].cpu().numpy(), plan.bbar[:N].cpu().numpy(), f"graph bwd #{rep}")
    # both phases in one launch, then the per-instance path
    plan.run(pcad.PHASE_BOTH)
    torch.cuda.synchronize()
    check_forward(pcad, w, plan.y[:N].cpu().numpy(), plan.h.cpu().numpy(),
                  plan.argk.cpu().numpy(), "graph both")
    check_backward(w, plan.argk.cpu().numpy(), plan.abar[:N].cpu().numpy(),
                   plan.bbar[:N].cpu().numpy(), "graph both")
    plan.run_per_segment(pcad.PHASE_FWD)
    torch.cuda.synchronize()
    check_forward(pcad, w, plan.y[:N].cpu().numpy(), plan.h.cpu().numpy(), plan.argk.cpu().numpy(),
                  "per-instance fwd")
    plan.run_per_segment(pcad.PHASE_BWD)
    torch.cuda.synchronize()
    check_backward(w, plan.argk.cpu().numpy(), plan.abar[:N].cpu().numpy(),
                   plan.bbar[:N].cpu().numpy(), "per-instance bwd")
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
    check_forward(pcad, w, plan.y[:N].cpu().numpy(), plan.h.cpu().numpy(),
                  plan.argk.cpu().numpy(), "segmented fwd")
    plan.run(pcad.PHASE_BWD)
    torch.cuda.synchronize()
    check_backward(w, plan.argk.cpu().numpy(), plan.abar[:N].cpu().numpy(),
                   plan.bbar[:N].cpu().numpy(), "segmented bwd")
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
    for rnd in range(2):
        for path in ("graph", "per-instance"):
            run = plan.run if path == "graph" else plan.run_per_segment
            run(pcad.PHASE_FWD)
            torch.cuda.synchronize()
            check_forward(pcad, w, plan.y[:N].cpu().numpy(), plan.h.cpu().numpy(),
                          plan.argk.cpu().numpy(), f"{path} fwd round {rnd}")
            run(pcad.PHASE_BWD)
            torch.cuda.synchronize()
            check_backward(w, plan.argk.cpu().numpy(), plan.abar[:N].cpu().numpy(),
                           plan.bbar[:N].cpu().numpy(), f"{path} bwd round {rnd}")
    assert plan.ws_error() == 0
    plan.close()


@pytest.mark.parametrize("m", [3, 16, 512])
def test_plan_exact_ties(pcad, m):
    """a in {0, 1} and integer offsets: y is exact in float32 on both sides,
    equal minima fill many bins and the lowest index must win every one of them;
    the oracle's decisions then coincide with the plan's exactly.  Graph and
    per-instance paths, forward and adjoint."""
    from workloads import segmented_ties
    w = segmented_ties(S=48, m=m)
    lens = list(np.diff(w["offsets"]))
    plan = pcad.BatchedPlan(w["offsets"], m, per_segment=True)
    plan.load(a=w["a"], b=w["b"], idx=w["idx"], ybar=w["ybar"], hbar=w["hbar"])
    N = plan.n
    for path in ("graph", "per-instance"):
        run = plan.run if path == "graph" else plan.run_per_segment
        run(pcad.PHASE_FWD)
        torch.cuda.synchronize()
        y = plan.y[:N].cpu().numpy()
        # exact integers: a tie of the minimum in at least a quarter of the
        # non-empty bins
        ties = nonempty = 0
        off = w["offsets"]
        for s in range(len(lens)):
            ys, ks = y[off[s]:off[s + 1]], w["idx"][off[s]:off[s + 1]]
            for k in range(m):
                v = ys[ks == k]
                nonempty += v.size > 0
                ties += v.size > 0 and np.count_nonzero(v == v.min()) > 1
        assert ties >= nonempty // 4, (ties, nonempty)
        check_forward(pcad, w, y, plan.h.cpu().numpy(), plan.argk.cpu().numpy(), f"ties {path} fwd",
                      exact_decisions=True)
        run(pcad.PHASE_BWD)
        torch.cuda.synchronize()
        check_backward(w, plan.argk.cpu().numpy(), plan.abar[:N].cpu().numpy(),
                       plan.bbar[:N].cpu().numpy(), f"ties {path} bwd")
    assert plan.ws_error() == 0
    plan.close()
