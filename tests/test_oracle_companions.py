"""Pins of the oracle's absolute-value companions against their closed forms.

Every float gate of the parity tests is |g - r| <= rtol*c + 2^-126, so a
companion c that is too large loosens every check made with it.  The
companion of a result is the same multilinear expression as the result,
evaluated on absolute values (|inputs|, |output adjoints|, spectral norms
for 2x2 factors and Frobenius norms for 2x2 adjoints), with the discrete
decisions (which element wins a min/max, which steps of a saturated sum
saturate) taken from the real run -- the quantity that bounds the rounding
error of any evaluation order of that expression (Section 2.2's vjp
composed from the operator's partials, applied to absolute values).

Each expectation below is written out as a sum over paths -- for a scan
output i, sum over j <= i of |term j| times the product of the absolute
multipliers between j and i -- evaluated by plain double loops in numpy,
never by the oracle's left-to-right recurrences.  Equality (to float64
rounding) pins the companion from above as well as from below: a factor
planted anywhere in a companion recurrence fails here.
"""
from __future__ import annotations

import numpy as np
import pytest

import oracle

REL = 1e-12


def close(got, exp, what=""):
    got = np.asarray(got, dtype=np.float64)
    exp = np.asarray(exp, dtype=np.float64)
    assert got.shape == exp.shape, (what, got.shape, exp.shape)
    np.testing.assert_allclose(got, exp, rtol=REL, atol=0, err_msg=what)


def prod(v):
    return float(np.prod(np.asarray(v, dtype=np.float64))) if len(v) else 1.0


def paths_fwd(w, mult):
    """t_i = sum_{j<=i} w_j * prod_{k=j+1..i} mult_k (double loop)."""
    n = len(w)
    return np.array([sum(w[j] * prod(mult[j + 1:i + 1]) for j in range(i + 1)) for i in range(n)])


def paths_rev(w, mult):
    """s_i = sum_{j>=i} w_j * prod_{k=i+1..j} mult_k (double loop)."""
    n = len(w)
    return np.array([sum(w[j] * prod(mult[i + 1:j + 1]) for j in range(i, n)) for i in range(n)])


def spec(M):
    return np.array([np.linalg.norm(m.reshape(2, 2), 2) for m in M])


def frob(M):
    return np.array([np.linalg.norm(m.reshape(2, 2)) for m in M])


def first_extremum(x, op):
    """lowest index of the minimum (maximum) of x"""
    return int(np.argmin(x)) if op == "min" else int(np.argmax(x))


# ---------------------------------------------------------------------------
# closed forms per operator: forward companions of the inclusive scan and the
# adjoint companions for output adjoints ybar (one per scan output)
# ---------------------------------------------------------------------------
def scan_fwd_comp(op, X):
    """X: (n, d) elements -> (n, d) companions of the inclusive scan."""
    n = X.shape[0]
    if op == "add":
        return np.array([[np.sum(np.abs(X[: i + 1, 0]))] for i in range(n)])
    if op == "mul":
        return np.array([[prod(np.abs(X[: i + 1, 0]))] for i in range(n)])
    if op in ("min", "max"):
        return np.array([[abs(X[first_extremum(X[: i + 1, 0], op), 0])] for i in range(n)])
    if op == "linrec":
        a, b = np.abs(X[:, 0]), np.abs(X[:, 1])
        return np.stack([np.array([prod(a[: i + 1]) for i in range(n)]), paths_fwd(b, a)], 1)
    if op == "mat2":
        s = spec(X)
        c = np.array([prod(s[: i + 1]) for i in range(n)])
        return np.repeat(c[:, None], 4, 1)
    raise ValueError(op)


def scan_vjp_comp(op, X, Yb):
    """Companions of x_bar for output adjoints Yb (n, d)."""
    n = X.shape[0]
    if op == "add":
        return np.array([[np.sum(np.abs(Yb[i:, 0]))] for i in range(n)])
    if op == "mul":
        ax = np.abs(X[:, 0])
        return np.array([[sum(abs(Yb[j, 0]) * prod(np.delete(ax[: j + 1], i)) for j in range(i, n))]
                         for i in range(n)])
    if op in ("min", "max"):
        c = np.zeros((n, 1))
        for j in range(n):
            c[first_extremum(X[: j + 1, 0], op), 0] += abs(Yb[j, 0])
        return c
    if op == "linrec":
        a, b = np.abs(X[:, 0]), np.abs(X[:, 1])
        lam_y = paths_rev(np.abs(Yb[:, 1]), a)   # companion of b_bar
        lam_A = paths_rev(np.abs(Yb[:, 0]), a)
        cA = np.array([prod(a[:i]) for i in range(n)])       # |A_{i-1}|, empty product at 0
        cy = np.concatenate([[0.0], paths_fwd(b, a)[:-1]])   # |y_{i-1}| path sum, y_{-1} = 0
        ca = cA * lam_A + cy * lam_y
        ca[0] = lam_A[0]  # x_bar_0 = lam_0: a_0 enters A_0 only
        return np.stack([ca, lam_y], 1)
    if op == "mat2":
        s, f = spec(X), frob(Yb)
        cR = paths_rev(f, s)
        c = np.array([prod(s[:i]) * cR[i] for i in range(n)])
        return np.repeat(c[:, None], 4, 1)
    raise ValueError(op)


def reduce_vjp_comp(op, X, yb):
    """Companions of x_bar of the fold for the output adjoint yb (d,)."""
    n, d = X.shape
    Yb = np.zeros((n, d))
    Yb[-1] = yb
    if op in ("min", "max"):
        c = np.zeros((n, 1))
        c[first_extremum(X[:, 0], op), 0] = abs(yb[0])
        return c
    if op == "mul":
        ax = np.abs(X[:, 0])
        return np.array([[abs(yb[0]) * prod(np.delete(ax, i))] for i in range(n)])
    if op == "mat2":
        s = spec(X)
        fy = np.linalg.norm(np.asarray(yb).reshape(2, 2))
        c = np.array([prod(s[:i]) * fy * prod(s[i + 1:]) for i in range(n)])
        return np.repeat(c[:, None], 4, 1)
    return scan_vjp_comp(op, X, Yb)


def elems(op, n, rng):
    if op == "linrec":
        return np.stack([rng.uniform(-1.5, 1.5, n), rng.standard_normal(n)], 1)
    if op == "mat2":
        return rng.standard_normal((n, 4))
    if op == "mul":
        return (rng.uniform(0.5, 2.0, n) * rng.choice([-1.0, 1.0], n))[:, None]
    if op in ("min", "max"):
        return (np.round(rng.standard_normal(n) * 2) / 2)[:, None]  # ties
    return rng.standard_normal(n)[:, None]


def args(op, X):
    if op == "linrec":
        return (X[:, 0], X[:, 1])
    if op == "mat2":
        return (X,)
    return (X[:, 0],)


OPS = ["add", "mul", "min", "max", "linrec", "mat2"]


@pytest.mark.parametrize("op", OPS)
@pytest.mark.parametrize("n", [1, 2, 9, 40])
def test_scan_companions(op, n):
    rng = np.random.default_rng(1000 + 7 * n + OPS.index(op))
    X = elems(op, n, rng)
    d = oracle.DIM[op]
    _, c = oracle.scan_fwd(op, *args(op, X))
    close(c, scan_fwd_comp(op, X), f"scan {op} forward companion")
    Yb = rng.standard_normal((n, d))
    _, cx = oracle.scan_vjp(op, Yb, *args(op, X))
    close(cx, scan_vjp_comp(op, X, Yb), f"scan {op} adjoint companion")


@pytest.mark.parametrize("op", OPS)
@pytest.mark.parametrize("n", [1, 2, 9, 40])
def test_reduce_companions(op, n):
    rng = np.random.default_rng(2000 + 7 * n + OPS.index(op))
    X = elems(op, n, rng)
    d = oracle.DIM[op]
    r = oracle.reduce_fwd(op, *args(op, X))
    close(r["c"], scan_fwd_comp(op, X)[-1], f"reduce {op} forward companion")
    yb = rng.standard_normal(d)
    _, cx = oracle.reduce_vjp(op, yb, *args(op, X))
    close(cx, reduce_vjp_comp(op, X, yb), f"reduce {op} adjoint companion")


@pytest.mark.parametrize("op", OPS)
def test_rbi_companions(op):
    """Per bin, the companions of the fold of the bin's elements in
    ascending index; elements with an out-of-range key get 0."""
    rng = np.random.default_rng(3000 + OPS.index(op))
    n, m = 90, 6
    X = elems(op, n, rng)
    d = oracle.DIM[op]
    idx = rng.integers(-1, m + 1, n).astype(np.int32)
    r = oracle.rbi_fwd(op, idx, m, *args(op, X))
    hb = rng.standard_normal((m, d))
    _, cv = oracle.rbi_vjp(op, idx, m, hb, *args(op, X))
    exp_cv = np.zeros((n, d))
    for k in range(m):
        mem = np.flatnonzero(idx == k)
        if mem.size == 0:
            continue
        close(r["c"][k], scan_fwd_comp(op, X[mem])[-1], f"rbi {op} bin {k} forward companion")
        exp_cv[mem] = reduce_vjp_comp(op, X[mem], hb[k])
    close(cv, exp_cv, f"rbi {op} adjoint companion")


def test_linrec_companion_with_A_adjoint():
    """The cumulative multiplier's adjoint enters a_bar through |A_{i-1}|."""
    rng = np.random.default_rng(4000)
    n = 25
    X = elems("linrec", n, rng)
    Yb = rng.standard_normal((n, 2))
    _, cx = oracle.scan_vjp("linrec", Yb, X[:, 0], X[:, 1])
    close(cx, scan_vjp_comp("linrec", X, Yb), "linrec companion with A_bar")


def test_scan_companion_with_seeded_adjoint_companion():
    """scan_vjp's optional cybar replaces |y_bar| as the companion seed (the
    chained workload seeds |y_bar| + |h_bar| at the argmin)."""
    rng = np.random.default_rng(4001)
    n = 30
    X = elems("linrec", n, rng)
    Yb = np.zeros((n, 2))
    Yb[:, 1] = rng.standard_normal(n)
    seed = np.abs(Yb) + np.stack([np.zeros(n), rng.uniform(0, 2, n)], 1)
    _, cx = oracle.scan_vjp("linrec", Yb, X[:, 0], X[:, 1], cybar=seed)
    a = np.abs(X[:, 0])
    lam_y = paths_rev(seed[:, 1], a)
    cy = np.concatenate([[0.0], paths_fwd(np.abs(X[:, 1]), a)[:-1]])
    exp = np.stack([cy * lam_y, lam_y], 1)
    exp[0, 0] = 0.0
    close(cx, exp, "seeded companion")


def test_satadd_companions():
    """Saturated addition: the companion follows the real run's saturation
    decisions; an unsaturated step adds |x|, a saturated step is the cap."""
    rng = np.random.default_rng(4002)
    cap = oracle.SAT_CAP
    x = rng.integers(0, 90_000, 40).astype(np.float64) * 3
    rs, c = oracle.scan_fwd("satadd", x)
    np.testing.assert_array_equal(c[:, 0], rs[:, 0])  # non-negative inputs: c == y
    sat = np.zeros(40, bool)
    acc = x[0]
    for i in range(1, 40):
        sat[i] = acc + x[i] > cap
        acc = cap if sat[i] else acc + x[i]
    assert sat.any() and not sat.all()
    yb = rng.standard_normal(40)
    _, cx = oracle.scan_vjp("satadd", yb, x)
    exp = np.array([sum(abs(yb[j]) * prod((~sat[max(i, 1):j + 1]).astype(float)) for j in range(i, 40))
                    for i in range(40)])
    close(cx[:, 0], exp, "satadd adjoint companion")


@pytest.mark.parametrize("n", [1, 2, 17])
def test_sumprod_companions(n):
    """p = sum_{j<k} a_j a_k: forward companion sum_{j<k} |a_j||a_k|; the
    invertible rule's adjoint s - a_i rounds relative to |ybar| sum |a|."""
    rng = np.random.default_rng(4003 + n)
    a = rng.standard_normal(n)
    aa = np.abs(a)
    pair = lambda v: sum(v[j] * v[k] for j in range(len(v)) for k in range(j + 1, len(v)))
    r = oracle.sumprod_reduce(a)
    close([r["c"]], [pair(aa)], "sumprod reduce forward companion")
    _, c = oracle.sumprod_reduce_vjp(a, -1.7)
    close(c, np.full(n, 1.7 * aa.sum()), "sumprod reduce adjoint companion")
    y, c = oracle.sumprod_scan(a)
    close(c, [pair(aa[: i + 1]) for i in range(n)], "sumprod scan forward companion")
    yb = rng.standard_normal(n)
    _, c = oracle.sumprod_scan_vjp(a, yb)
    exp = [sum(abs(yb[j]) * (aa[: j + 1].sum() - aa[i]) for j in range(i, n)) for i in range(n)]
    close(c, exp, "sumprod scan adjoint companion")
    m = 3
    idx = rng.integers(-1, m + 1, n).astype(np.int32)
    hb = rng.standard_normal(m)
    r = oracle.sumprod_rbi_fwd(idx, m, a)
    _, cv = oracle.sumprod_rbi_vjp(idx, m, hb, a)
    exp = np.zeros(n)
    for k in range(m):
        mem = np.flatnonzero(idx == k)
        close([r["c"][k]], [pair(aa[mem])], f"sumprod rbi bin {k}")
        exp[mem] = abs(hb[k]) * aa[mem].sum()
    close(cv, exp, "sumprod rbi adjoint companion")


@pytest.mark.parametrize("d", [2, 3, 5])
def test_matd_companions(d):
    """d x d products: prod ||M_j||_2 forward; the adjoint companion
    ||P_{i-1}||-bound times the path sum of ||Pbar_j||_2 through the later
    factors' norms (scan), or the two-sided norm product (reduce)."""
    rng = np.random.default_rng(4010 + d)
    n = 12
    M = rng.standard_normal((n, d, d)) / np.sqrt(d)
    s = np.array([np.linalg.norm(m, 2) for m in M])
    _, c = oracle.matd_scan(M)
    close(c, [prod(s[: i + 1]) for i in range(n)], "matd scan forward companion")
    Pb = rng.standard_normal((n, d, d))
    fb = np.array([np.linalg.norm(p, 2) for p in Pb])
    _, c = oracle.matd_scan_vjp(M, Pb)
    cR = paths_rev(fb, s)
    close(c, [prod(s[:i]) * cR[i] for i in range(n)], "matd scan adjoint companion")
    _, c = oracle.matd_reduce(M)
    close([c], [prod(s)], "matd reduce forward companion")
    Yb = rng.standard_normal((d, d))
    _, c = oracle.matd_reduce_vjp(M, Yb)
    close(c, [prod(s[:i]) * np.linalg.norm(Yb, 2) * prod(s[i + 1:]) for i in range(n)],
          "matd reduce adjoint companion")


def test_segmented_companions():
    """The chained workload: y's companion is the linrec path sum, h's the
    companion at the chosen position, and the adjoint companions use
    |y_bar| + |h_bar at the argmin| as the seed."""
    from workloads import segmented
    w = segmented(S=5, m=4, median=20, cap=60)
    off = w["offsets"]
    f = oracle.segmented_fwd(off, w["a"], w["b"], w["idx"], 4)
    ab, bb, cab, cbb = oracle.segmented_vjp(off, w["a"], w["b"], w["idx"], 4, w["ybar"], w["hbar"],
                                            f["argk"])
    hb = np.asarray(w["hbar"], np.float64).reshape(5, 4)
    for s in range(5):
        lo, hi = int(off[s]), int(off[s + 1])
        L = hi - lo
        a = np.abs(w["a"][lo:hi].astype(np.float64))
        b = np.abs(w["b"][lo:hi].astype(np.float64))
        cy = paths_fwd(b, a)
        close(f["cy"][lo:hi], cy, f"segment {s} y companion")
        seed = np.abs(w["ybar"][lo:hi].astype(np.float64))
        for k in range(4):
            g = int(f["argk"][s, k])
            if g < L:
                close([f["ch"][s, k]], [cy[g]], f"segment {s} bin {k} h companion")
                seed[g] += abs(hb[s, k])
        lam = paths_rev(seed, a)
        close(cbb[lo:hi], lam, f"segment {s} b_bar companion")
        exp = np.concatenate([[0.0], cy[:-1]]) * lam
        close(cab[lo:hi], exp, f"segment {s} a_bar companion")
