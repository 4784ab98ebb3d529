"""Host-side pins of the autograd workload: the oracle's gradient of
loss = sum log|y| + sum over non-empty bins of max-by-index, against FP64
central differences of the oracle's own forward (no GPU)."""
from __future__ import annotations

import numpy as np
import pytest

import oracle


def small_workload(T=4096, m=4096, seed=7):
    from workloads import autograd
    w = autograd(B=1, T=T, m=m, seed=seed)
    return w["a"][0], w["b"][0], w["v"][0], w["idx"][0], m


def fd_coords(rng, a, b, v, idx, h_rel=1e-6, count=32):
    """Coordinates over a, b and v; a v coordinate within 2h of another value
    of its bin is redrawn (the max would switch inside the stencil)."""
    n = len(a)
    out = []
    while len(out) < count:
        which = int(rng.integers(0, 3))
        j = int(rng.integers(0, n))
        if which == 2:
            h = h_rel * max(1.0, abs(float(v[j])))
            same = np.flatnonzero(idx == idx[j])
            others = v[same[same != j]].astype(np.float64)
            if np.any(np.abs(others - v[j]) <= 2 * h):
                continue
        out.append((which, j))
    return out


def test_gradient_matches_central_differences():
    a, b, v, idx, m = small_workload()
    ab, bb, vb, _, _, _ = oracle.autograd_grad(a, b, v, idx, m)
    rng = np.random.default_rng(3)
    base = [a.astype(np.float64), b.astype(np.float64), v.astype(np.float64)]
    grads = [ab, bb, vb]
    for which, j in fd_coords(rng, a, b, v, idx):
        x = base[which]
        h = 1e-6 * max(1.0, abs(x[j]))
        args_p = [t.copy() for t in base]
        args_m = [t.copy() for t in base]
        args_p[which][j] += h
        args_m[which][j] -= h
        fp = oracle.autograd_loss(*args_p, idx, m)
        fm = oracle.autograd_loss(*args_m, idx, m)
        fd = (fp - fm) / (2 * h)
        g = grads[which][j]
        # central-difference truncation O(h^2) plus cancellation eps*|loss|/h
        tol = 1e-6 * max(1.0, abs(g)) + 1e-16 * abs(fp) / h * 8
        assert abs(fd - g) <= tol, (which, j, fd, g)


def test_max_by_index_gradient_is_one_hot_on_nonempty_bins():
    a, b, v, idx, m = small_workload(T=2048, m=4096, seed=9)
    _, _, vb, _, _, _ = oracle.autograd_grad(a, b, v, idx, m)
    r = oracle.rbi_fwd("max", idx, m, v)
    full = np.flatnonzero(r["argk"] < len(v))
    expect = np.zeros(len(v))
    expect[r["argk"][full]] = 1.0
    np.testing.assert_array_equal(vb, expect)
    # about e^-(T/m) of the bins stay empty
    assert 0.5 < (m - len(full)) / m < 0.7


def test_pick_mode():
    import paper_2310_03568_amd.autograd as ag
    assert ag.pick_mode("auto", 1 << 20) == "checkpoint"
    assert ag.pick_mode("auto", ag.CHECKPOINT_BUDGET_BYTES + 1) == "recompute"
    assert ag.pick_mode("recompute", 1) == "recompute"
    with pytest.raises(Exception):
        ag.pick_mode("tape", 1)
