"""Comparison gate between a float32 result and the float64 oracle.

TEST INFRASTRUCTURE ONLY (used by the tests and the benchmark's parity leg).

For each float output g (float32) against the oracle value r (float64) with
companion c >= |r| (the same multilinear expression on absolute values):

    |g - r| <= rtol * c + 2^-126

* If |r| > FLT_MAX the float32 result must be the same-signed infinity.
* If c > FLT_MAX (or r, c are not finite) while r is in range, the element is
  "range-exceeded": no float32 method can be held to it; it is excluded and
  counted, and the caller decides how many are acceptable.
* A NaN where the oracle is finite fails.

The tolerance is relative to the companion rather than to |r| because plain
element-wise relative error is unattainable for any float32 method where
cancellation makes |r| much smaller than the terms that produce it (suffix
sums of N(0,1) adjoints, linear recurrences crossing zero).
"""
from __future__ import annotations

import numpy as np

FLT_MAX = float(np.finfo(np.float32).max)
TINY = 2.0 ** -126

RTOL = {"add": 1e-5, "min": 1e-5, "max": 1e-5, "mul": 1e-4, "linrec": 1e-4, "mat2": 1e-4,
        # sumOfProd accumulates pairwise products s1*s2 of partial sums: the
        # error bound of a dot product, like the product-type folds above
        "sumprod": 1e-4}


def chain_rtol(n: int, rtol: float, width: int = 1, adjoint: bool = False, k: float = 4.0):
    """Per-element tolerance for scans whose outputs are products of many
    factors (*, the 2x2 and d x d matrix products): any evaluation of the
    product of i+1 factors rounds i times, so with factors that neither
    shrink nor grow the relative error of element i grows like
    sqrt(i+1) * 2^-24 (a random walk of independent roundings; measured at
    0.3-0.7 times that on orthogonal 2x2 chains), and no float32 method keeps
    it below a fixed rtol along millions of factors.  Element i gets
    max(rtol, k sqrt(L_i) 2^-24) with L_i = i+1 for the forward and
    max(i+1, n-i) for the adjoint, whose element i multiplies the prefix of
    i factors by sums over chains of up to n-i of them.  Equal to ``rtol``
    (1e-4) up to L_i of about 1.75e5 with k = 4.  Returns an array of n *
    ``width`` tolerances in element order."""
    i = np.arange(n, dtype=np.float64)
    L = np.maximum(i + 1.0, n - i) if adjoint else i + 1.0
    return np.repeat(np.maximum(rtol, k * np.sqrt(L) * 2.0 ** -24), width)


def gate(g, r, c, rtol):
    g = np.asarray(g, dtype=np.float64).reshape(-1)
    r = np.asarray(r, dtype=np.float64).reshape(-1)
    c = np.asarray(c, dtype=np.float64).reshape(-1)
    assert g.shape == r.shape == c.shape, (g.shape, r.shape, c.shape)
    over = np.isfinite(r) & (np.abs(r) > FLT_MAX)
    rng_ex = (~over) & (~np.isfinite(r) | ~np.isfinite(c) | (c > FLT_MAX))
    normal = ~over & ~rng_ex
    ok = np.ones(g.shape, dtype=bool)
    ok[over] = np.isinf(g[over]) & (np.sign(g[over]) == np.sign(r[over]))
    with np.errstate(invalid="ignore", over="ignore"):
        err = np.abs(g - r)
        bound = rtol * c + TINY
        ok[normal] = np.isfinite(g[normal]) & (err[normal] <= bound[normal])
        sel = normal & (np.abs(r) >= 1e-3 * c) & (np.abs(r) > 0)
        max_rel = float(np.max(err[sel] / np.abs(r[sel]))) if sel.any() else 0.0
        rn = np.linalg.norm(r[normal])
        normwise = float(np.linalg.norm((g - r)[normal]) / rn) if rn > 0 else 0.0
        ratio = np.where(normal, err / bound, 0.0)
    bad = np.flatnonzero(~ok)
    worst = int(np.argmax(ratio)) if ratio.size else -1
    return dict(
        ok=bool(bad.size == 0), n=int(g.size), n_fail=int(bad.size),
        first_fail=[int(i) for i in bad[:8]], n_range_exceeded=int(rng_ex.sum()),
        max_rel=max_rel, normwise=normwise,
        worst=worst, worst_ratio=float(ratio[worst]) if worst >= 0 else 0.0,
    )


def assert_gate(g, r, c, rtol, max_range_exceeded=0, what: str = ""):
    """Gate every element.  ``max_range_exceeded`` bounds how many elements
    may fall outside the float32 range of the companion; ``None`` allows any
    number but then holds those elements to a norm-wise relative error
    ||g - r||_2 <= rtol ||r||_2 + 2^-126 sqrt(count) (products of matrices
    whose norm product overflows while the product itself underflows)."""
    res = gate(g, r, c, rtol)
    gg = np.asarray(g, dtype=np.float64).reshape(-1)
    rr = np.asarray(r, dtype=np.float64).reshape(-1)
    cc = np.asarray(c, dtype=np.float64).reshape(-1)
    detail = ", ".join(f"[{i}] g={gg[i]!r} r={rr[i]!r} c={cc[i]!r}" for i in res["first_fail"][:4])
    assert res["ok"], f"{what}: {res['n_fail']}/{res['n']} outside the gate: {detail}"
    if max_range_exceeded is None:
        over = np.isfinite(rr) & (np.abs(rr) > FLT_MAX)
        ex = (~over) & (~np.isfinite(rr) | ~np.isfinite(cc) | (cc > FLT_MAX))
        if ex.any():
            assert np.all(np.isfinite(rr[ex])), f"{what}: oracle not finite"
            err = float(np.linalg.norm(gg[ex] - rr[ex]))
            bound = rtol * float(np.linalg.norm(rr[ex])) + TINY * np.sqrt(ex.sum())
            res["normwise_range_exceeded"] = err / max(float(np.linalg.norm(rr[ex])), TINY)
            assert err <= bound, f"{what}: norm-wise error {err} > {bound} on range-exceeded part"
    else:
        assert res["n_range_exceeded"] <= max_range_exceeded, (
            f"{what}: {res['n_range_exceeded']} range-exceeded elements")
    return res


def assert_discriminates(g, r, c, rtol, start: int = 600, width: int = 1, what: str = "",
                         sparse: bool = False):
    """Self-check of a parity test on the CPU: the gate that accepted ``g``
    must reject a copy of ``g`` whose elements from ``start`` on (``width``
    floats per element) are zero, i.e. an output that stopped being computed
    after a few hundred elements.  A gate that lets such a copy through
    (outputs that under- or overflow, or a companion far above |r|) would
    make the comparison vacuous.  The copy must fail at 1% of the zeroed
    floats, or, for outputs that are negligible by nature almost everywhere
    (``sparse``: a min/max scan adjoint is non-zero only where the running
    extremum was renewed; the reduce adjoint of a contracting recurrence
    decays geometrically away from the last element), at 99% of the zeroed
    floats where |r| >= 2^-100."""
    gz = np.array(g, dtype=np.float64, copy=True).reshape(-1)
    if gz.size <= start * width:
        return
    gz[start * width:] = 0.0
    res = gate(gz, r, c, rtol)
    assert not res["ok"], f"{what}: a copy zeroed past element {start} passes the gate"
    if sparse:
        rr = np.abs(np.asarray(r, dtype=np.float64).reshape(-1)[start * width:])
        need = int(0.99 * np.count_nonzero(rr >= 2.0 ** -100))
    else:
        need = (gz.size - start * width) // 100
    assert res["n_fail"] >= need, (
        f"{what}: a copy zeroed past element {start} fails only {res['n_fail']} elements")


def segmented_decisions(offsets, idx, m: int, y32, h, argk, f=None) -> dict:
    """Checks of the chained workload's min-by-index decisions, which are
    taken on the implementation's own float32 y (Section 4.2, Min/Max):

    * argk_ok: every bin's argk is the lowest instance-relative index of the
      minimum of y32 over the instance's positions with that key (the
      oracle's min-by-index of y32), the instance length for an empty bin;
    * h_ok: h is y32 at argk bit for bit (+inf for an empty bin), except that
      a -0.0 winner may read +0.0;
    * with ``f`` (the oracle's segmented_fwd on the float64 recurrence):
      n_diff_oracle counts bins where the float64 decision differs, and
      diff_ok says every such pair of candidates ties within 1e-4 of their
      companions.
    """
    import oracle
    off = np.asarray(offsets, dtype=np.int64)
    S = off.shape[0] - 1
    lens = np.diff(off)
    y32 = np.asarray(y32, dtype=np.float32)
    h = np.asarray(h, dtype=np.float32).reshape(S, m)
    argk = np.asarray(argk).reshape(S, m)
    ak_y, h_y = oracle.segmented_argmin(off, idx, y32, m)
    out = dict(argk_ok=bool(np.array_equal(argk, ak_y)),
               argk_bad_bins=int(np.count_nonzero(argk != ak_y)))
    want = h_y.astype(np.float32)
    neg0 = (want == 0) & np.signbit(want)
    out["h_ok"] = bool(np.array_equal(h.view(np.uint32)[~neg0], want.view(np.uint32)[~neg0])
                       and np.all(h[neg0] == 0)
                       and np.array_equal(argk == lens[:, None], np.isinf(want)))
    if f is not None:
        diff = np.argwhere(argk != f["argk"])
        ok = True
        for s, k in diff:
            lo = int(off[s])
            g, r = int(argk[s, k]), int(f["argk"][s, k])
            ok = ok and g < lens[s] and r < lens[s] and int(idx[lo + g]) == k and (
                abs(f["y"][lo + g] - f["y"][lo + r]) <= 1e-4 * (f["cy"][lo + g] + f["cy"][lo + r]))
        out["n_diff_oracle"] = int(len(diff))
        out["diff_ok"] = bool(ok)
    return out
