"""Pins of the CPU oracle against things other than itself.

Each check is chosen so that a plausible mistake in the oracle (a dropped
term, a wrong sign or index, a transposed operand, a wrong tie rule) fails at
least one of them:

* hand-derived worked examples under ``tests/golden`` (each cites the rule it
  follows);
* library primitives for the forward (numpy cumsum / cumprod / accumulate /
  matmul / bincount / ufunc.at / argmin);
* closed forms for the adjoints (broadcast, suffix sums, the three zero cases
  of multiplication, one-hot at the lowest-index argmin, the linear-recurrence
  sums, the matrix embedding of the linear recurrence, determinants);
* forward-mode dual numbers over independently written operator definitions
  (a brute-force Jacobian, so x_bar = J^T y_bar is checked without any
  reverse sweep) for n <= 16;
* central finite differences of the oracle forward;
* the paper's alternative rules for the same adjoint: the general reduce rule
  (exclusive scans l and r, then the local vjp of l (.) x (.) r), the general
  scan rule (Jacobians cs, a scan with linear-function composition, then a
  map), PPAD's scan rule (appendix figure) and the sort-based
  reduce-by-index rule (its rule figure).
"""
from __future__ import annotations

import glob
import itertools
import json
import os

import numpy as np
import pytest

import oracle

HERE = os.path.dirname(os.path.abspath(__file__))
OPS = ["add", "mul", "min", "max", "linrec", "mat2"]
D = oracle.DIM


# ---------------------------------------------------------------------------
# independent operator definitions (Section 6.1 operator figure) and duals
# ---------------------------------------------------------------------------
class Dual:
    __slots__ = ("v", "t")

    def __init__(self, v, t):
        self.v = v
        self.t = t

    @staticmethod
    def lift(o, N):
        return o if isinstance(o, Dual) else Dual(float(o), np.zeros(N))

    def __add__(self, o):
        o = Dual.lift(o, self.t.size)
        return Dual(self.v + o.v, self.t + o.t)

    __radd__ = __add__

    def __mul__(self, o):
        o = Dual.lift(o, self.t.size)
        return Dual(self.v * o.v, self.v * o.t + o.v * self.t)

    __rmul__ = __mul__

    def __le__(self, o):
        return self.v <= (o.v if isinstance(o, Dual) else o)

    def __ge__(self, o):
        return self.v >= (o.v if isinstance(o, Dual) else o)


def py_op(op, p, q):
    """p (.) q on lists of components; min/max keep the left operand on ties."""
    if op == "add":
        return [p[0] + q[0]]
    if op == "mul":
        return [p[0] * q[0]]
    if op == "min":
        return [p[0] if p[0] <= q[0] else q[0]]
    if op == "max":
        return [p[0] if p[0] >= q[0] else q[0]]
    if op == "linrec":
        # linFnComp (b1,c1) (b2,c2) = (b2 + c2*b1, c2*c1); stored as (c, b)
        c1, b1 = p
        c2, b2 = q
        return [c2 * c1, b2 + c2 * b1]
    if op == "mat2":
        a1, b1, c1, d1 = p
        a2, b2, c2, d2 = q
        return [a1 * a2 + b1 * c2, a1 * b2 + b1 * d2, c1 * a2 + d1 * c2, c1 * b2 + d1 * d2]
    raise ValueError(op)


def py_neutral(op):
    return {"add": [0.0], "mul": [1.0], "min": [np.inf], "max": [-np.inf],
            "linrec": [1.0, 0.0], "mat2": [1.0, 0.0, 0.0, 1.0]}[op]


def dual_inputs(X):
    n, d = X.shape
    N = n * d
    out = []
    for i in range(n):
        row = []
        for t in range(d):
            tan = np.zeros(N)
            tan[i * d + t] = 1.0
            row.append(Dual(float(X[i, t]), tan))
        out.append(row)
    return out


def jac_rows(elems, N):
    return np.array([[e.t if isinstance(e, Dual) else np.zeros(N) for e in el] for el in elems])


def dual_scan(op, X):
    xs = dual_inputs(X)
    rs = [xs[0]]
    for i in range(1, len(xs)):
        rs.append(py_op(op, rs[-1], xs[i]))
    N = X.size
    J = jac_rows(rs, N).reshape(-1, N)
    vals = np.array([[e.v for e in el] for el in rs])
    return vals, J


def dual_reduce(op, X):
    xs = dual_inputs(X)
    acc = xs[0]
    for i in range(1, len(xs)):
        acc = py_op(op, acc, xs[i])
    N = X.size
    return np.array([e.v for e in acc]), np.array([e.t for e in acc]).reshape(-1, N)


def dual_rbi(op, idx, m, V):
    xs = dual_inputs(V)
    N = V.size
    d = V.shape[1]
    hist = [None] * m
    for i, k in enumerate(idx):
        if 0 <= k < m:
            hist[k] = xs[i] if hist[k] is None else py_op(op, hist[k], xs[i])
    J = np.zeros((m * d, N))
    for k in range(m):
        if hist[k] is not None:
            for t in range(d):
                J[k * d + t] = hist[k][t].t
    return J


def rand_elems(op, n, rng, nonneg=False):
    d = D[op]
    if op == "linrec":
        a = rng.uniform(0.5, 1.5, n)
        b = rng.standard_normal(n)
        return np.stack([a, b], 1).astype(np.float32).astype(np.float64)
    X = rng.standard_normal((n, d))
    if op == "mul":
        X = rng.uniform(0.5, 2.0, (n, 1)) * rng.choice([-1.0, 1.0], (n, 1))
    return X.astype(np.float32).astype(np.float64)


def as_args(op, X):
    if op == "linrec":
        return (X[:, 0], X[:, 1])
    if op == "mat2":
        return (X,)
    return (X[:, 0],)


# ---------------------------------------------------------------------------
# golden worked examples
# ---------------------------------------------------------------------------
def _golden():
    return [json.load(open(p)) for p in sorted(glob.glob(os.path.join(HERE, "golden", "*.json")))]


def _f(v):
    return np.array([np.inf if x == "inf" else x for x in v], dtype=np.float64)


@pytest.mark.parametrize("g", _golden(), ids=lambda g: g["name"])
def test_golden(g):
    op, comb = g["op"], g["combinator"]
    assert g.get("cite"), "every fixture cites the rule it follows"
    if comb == "reduce" and op == "sumprod":
        r = oracle.sumprod_reduce(np.array(g["x"]))
        assert r["y"] == g["y"][0] and r["s"] == g["s"]
        xb, _ = oracle.sumprod_reduce_vjp(np.array(g["x"]), g["ybar"][0])
        np.testing.assert_array_equal(xb, g["xbar"])
    elif comb == "rbi" and op == "sumprod":
        idx = np.array(g["idx"], np.int32)
        r = oracle.sumprod_rbi_fwd(idx, g["m"], np.array(g["v"]))
        np.testing.assert_array_equal(r["hist"], g["hist"])
        np.testing.assert_array_equal(r["s"], g["s"])
        np.testing.assert_array_equal(r["count"], g["count"])
        vb, _ = oracle.sumprod_rbi_vjp(idx, g["m"], np.array(g["hbar"]), np.array(g["v"]))
        np.testing.assert_array_equal(vb, g["vbar"])
    elif comb == "reduce":
        r = oracle.reduce_fwd(op, np.array(g["x"]))
        np.testing.assert_array_equal(r["y"], g["y"])
        if "y_signbit" in g:  # -0.0 == +0.0: the bit pattern is checked apart
            np.testing.assert_array_equal(np.signbit(r["y"]), g["y_signbit"])
        if "k" in g:
            assert r["k"] == g["k"]
        if "n0" in g:
            assert r["n0"] == g["n0"] and r["ypos"] == g["ypos"]
        xb, _ = oracle.reduce_vjp(op, np.array(g["ybar"]), np.array(g["x"]))
        np.testing.assert_allclose(xb[:, 0], g["xbar"], rtol=1e-15)
    elif comb == "scan" and op == "linrec":
        rs, _ = oracle.scan_fwd(op, np.array(g["a"]), np.array(g["b"]))
        np.testing.assert_allclose(rs[:, 1], g["y"], rtol=1e-15)
        np.testing.assert_allclose(rs[:, 0], g["A"], rtol=1e-15)
        yb = np.stack([np.zeros(3), np.array(g["ybar"])], 1)
        xb, _ = oracle.scan_vjp(op, yb, np.array(g["a"]), np.array(g["b"]))
        np.testing.assert_allclose(xb[:, 0], g["abar"], rtol=1e-15)
        np.testing.assert_allclose(xb[:, 1], g["bbar"], rtol=1e-15)
    elif comb == "scan" and op == "mat2":
        rs, _ = oracle.scan_fwd(op, np.array(g["M"]))
        np.testing.assert_allclose(rs, g["P"], rtol=1e-15)
        xb, _ = oracle.scan_vjp(op, np.array(g["Pbar"], dtype=float), np.array(g["M"]))
        np.testing.assert_allclose(xb, g["Mbar"], rtol=1e-15, atol=0)
    elif comb == "scan":
        rs, _ = oracle.scan_fwd(op, np.array(g["x"]))
        np.testing.assert_array_equal(rs[:, 0], g["y"])
        if "y_signbit" in g:
            np.testing.assert_array_equal(np.signbit(rs[:, 0]), g["y_signbit"])
        xb, _ = oracle.scan_vjp(op, np.array(g["ybar"]), np.array(g["x"]))
        np.testing.assert_allclose(xb[:, 0], g["xbar"], rtol=1e-15)
    elif comb == "rbi":
        idx = np.array(g["idx"], np.int32)
        r = oracle.rbi_fwd(op, idx, g["m"], np.array(g["v"]))
        np.testing.assert_array_equal(r["hist"][:, 0], _f(g["hist"]))
        if "hist_signbit" in g:
            np.testing.assert_array_equal(np.signbit(r["hist"][:, 0]), g["hist_signbit"])
        for key in ("count", "argk", "n0", "ypos"):
            if key in g:
                np.testing.assert_array_equal(r[key], g[key])
        vb, _ = oracle.rbi_vjp(op, idx, g["m"], np.array(g["hbar"]), np.array(g["v"]))
        np.testing.assert_allclose(vb[:, 0], g["vbar"], rtol=1e-15)
    else:
        raise AssertionError(comb)


# ---------------------------------------------------------------------------
# forward against library primitives
# ---------------------------------------------------------------------------
def test_scan_fwd_library():
    rng = np.random.default_rng(1)
    x = rng.uniform(0.5, 2.0, 500).astype(np.float32)
    xd = x.astype(np.float64)
    np.testing.assert_allclose(oracle.scan_fwd("add", x)[0][:, 0], np.cumsum(xd), rtol=1e-13)
    np.testing.assert_allclose(oracle.scan_fwd("mul", x[:60])[0][:, 0], np.cumprod(xd[:60]), rtol=1e-13)
    np.testing.assert_array_equal(oracle.scan_fwd("min", x)[0][:, 0], np.minimum.accumulate(xd))
    np.testing.assert_array_equal(oracle.scan_fwd("max", x)[0][:, 0], np.maximum.accumulate(xd))
    M = rng.standard_normal((40, 4)).astype(np.float32)
    P = oracle.scan_fwd("mat2", M)[0]
    acc = np.eye(2)
    for i in range(40):
        acc = acc @ M[i].astype(np.float64).reshape(2, 2)
        np.testing.assert_allclose(P[i].reshape(2, 2), acc, rtol=1e-12, atol=1e-14)


def test_reduce_fwd_library():
    rng = np.random.default_rng(2)
    x = rng.uniform(-2.0, 2.0, 333).astype(np.float32)
    xd = x.astype(np.float64)
    r = oracle.reduce_fwd("add", x)
    np.testing.assert_allclose(r["y"][0], np.sum(xd), rtol=1e-13)
    assert r["c"][0] == pytest.approx(np.sum(np.abs(xd)), rel=1e-13)
    r = oracle.reduce_fwd("min", x)
    assert r["y"][0] == xd.min() and r["k"] == int(np.argmin(xd))
    r = oracle.reduce_fwd("max", x)
    assert r["y"][0] == xd.max() and r["k"] == int(np.argmax(xd))
    xm = x[:50].copy()
    xm[[3, 17]] = 0
    r = oracle.reduce_fwd("mul", xm)
    nz = xm[xm != 0].astype(np.float64)
    assert r["y"][0] == 0.0 and r["n0"] == 2
    assert r["ypos"] == pytest.approx(np.prod(nz), rel=1e-13)
    # empty input: neutral, sentinel index n = 0
    r = oracle.reduce_fwd("min", np.zeros(0, np.float32))
    assert r["y"][0] == np.inf and r["k"] == 0


def test_rbi_fwd_library():
    rng = np.random.default_rng(3)
    n, m = 2000, 37
    idx = rng.integers(-3, m + 3, n).astype(np.int32)
    v = np.round(rng.standard_normal(n) * 8) / 8
    v = v.astype(np.float32)
    vd = v.astype(np.float64)
    ok = (idx >= 0) & (idx < m)
    r = oracle.rbi_fwd("add", idx, m, v)
    np.testing.assert_allclose(r["hist"][:, 0], np.bincount(idx[ok], vd[ok], minlength=m), rtol=1e-12, atol=1e-12)
    np.testing.assert_array_equal(r["count"], np.bincount(idx[ok], minlength=m))
    for op, uf, init in (("min", np.minimum, np.inf), ("max", np.maximum, -np.inf)):
        r = oracle.rbi_fwd(op, idx, m, v)
        h = np.full(m, init)
        uf.at(h, idx[ok], vd[ok])
        np.testing.assert_array_equal(r["hist"][:, 0], h)
        for k in range(m):
            members = np.flatnonzero(ok & (idx == k))
            if members.size == 0:
                assert r["argk"][k] == n
            else:
                win = members[np.flatnonzero(vd[members] == h[k])[0]]
                assert r["argk"][k] == win
    vm = vd.copy()
    vm[rng.choice(n, 100, replace=False)] = 0.0
    r = oracle.rbi_fwd("mul", idx, m, vm)
    n0 = np.bincount(idx[ok & (vm == 0)], minlength=m)
    np.testing.assert_array_equal(r["n0"], n0)
    yp = np.ones(m)
    np.multiply.at(yp, idx[ok & (vm != 0)], vm[ok & (vm != 0)])
    np.testing.assert_allclose(r["ypos"], yp, rtol=1e-12)
    np.testing.assert_allclose(r["hist"][:, 0], np.where(n0 > 0, 0.0, yp), rtol=1e-12)


# ---------------------------------------------------------------------------
# closed forms of the adjoints
# ---------------------------------------------------------------------------
def test_closed_form_add():
    rng = np.random.default_rng(4)
    x = rng.standard_normal(300).astype(np.float32)
    yb = rng.standard_normal(300)
    xb, _ = oracle.scan_vjp("add", yb, x)
    np.testing.assert_allclose(xb[:, 0], np.cumsum(yb[::-1])[::-1], rtol=1e-12, atol=1e-12)
    xb, _ = oracle.reduce_vjp("add", np.array([0.7]), x)
    np.testing.assert_array_equal(xb[:, 0], np.full(300, 0.7))


@pytest.mark.parametrize("zeros", [0, 1, 2, 5])
def test_closed_form_reduce_mul(zeros):
    rng = np.random.default_rng(10 + zeros)
    x = rng.uniform(0.5, 2.0, 40) * rng.choice([-1, 1], 40)
    pos = rng.choice(40, zeros, replace=False)
    x[pos] = 0.0
    x = x.astype(np.float32).astype(np.float64)
    yb = 1.3
    xb, _ = oracle.reduce_vjp("mul", np.array([yb]), x)
    nz = np.prod(x[x != 0])
    if zeros == 0:
        exp = np.prod(x) / x * yb
    elif zeros == 1:
        exp = np.zeros(40)
        exp[pos[0]] = nz * yb
    else:
        exp = np.zeros(40)
    np.testing.assert_allclose(xb[:, 0], exp, rtol=1e-12, atol=0)


@pytest.mark.parametrize("op", ["min", "max"])
def test_min_max_all_tie_patterns(op):
    """Every pattern over {0,1,2} for n <= 7: reduce adjoint is the one-hot
    at the lowest-index extremum; scan adjoint of position k sums y_bar over
    the prefixes whose lowest-index extremum is k."""
    sel = np.argmin if op == "min" else np.argmax
    for n in range(1, 8):
        for pat in itertools.product([0.0, 1.0, 2.0], repeat=n):
            x = np.array(pat)
            r = oracle.reduce_fwd(op, x)
            k = int(sel(x))
            assert r["k"] == k
            xb, _ = oracle.reduce_vjp(op, np.array([3.0]), x)
            exp = np.zeros(n)
            exp[k] = 3.0
            np.testing.assert_array_equal(xb[:, 0], exp)
            if n <= 6:
                yb = 2.0 ** np.arange(n)
                xb, _ = oracle.scan_vjp(op, yb, x)
                exp = np.zeros(n)
                for j in range(n):
                    exp[int(sel(x[: j + 1]))] += yb[j]
                np.testing.assert_array_equal(xb[:, 0], exp)


def test_closed_form_linrec():
    """y_i = sum_j b_j prod_{k=j+1..i} a_k; lam_i = sum_{j>=i} ybar_j
    prod_{k=i+1..j} a_k; b_bar = lam; a_bar_i = lam_i y_{i-1} (+ Abar part)."""
    rng = np.random.default_rng(5)
    n = 30
    a = rng.uniform(0.5, 1.5, n)
    b = rng.standard_normal(n)
    yb = rng.standard_normal(n)
    Ab = rng.standard_normal(n)
    y = np.array([sum(b[j] * np.prod(a[j + 1:i + 1]) for j in range(i + 1)) for i in range(n)])
    A = np.array([np.prod(a[: i + 1]) for i in range(n)])
    rs, _ = oracle.scan_fwd("linrec", a, b)
    np.testing.assert_allclose(rs[:, 1], y, rtol=1e-12, atol=1e-13)
    np.testing.assert_allclose(rs[:, 0], A, rtol=1e-12)
    lam = np.array([sum(yb[j] * np.prod(a[i + 1:j + 1]) for j in range(i, n)) for i in range(n)])
    lamA = np.array([sum(Ab[j] * np.prod(a[i + 1:j + 1]) for j in range(i, n)) for i in range(n)])
    yprev = np.concatenate([[0.0], y[:-1]])
    Aprev = np.concatenate([[1.0], A[:-1]])
    xb, _ = oracle.scan_vjp("linrec", np.stack([Ab, yb], 1), a, b)
    np.testing.assert_allclose(xb[:, 1], lam, rtol=1e-11, atol=1e-12)
    np.testing.assert_allclose(xb[:, 0], lam * yprev + lamA * Aprev, rtol=1e-11, atol=1e-12)
    # a == 1: scan(+) of b;  a == 0: y = b
    rs, _ = oracle.scan_fwd("linrec", np.ones(n), b)
    np.testing.assert_allclose(rs[:, 1], np.cumsum(b), rtol=1e-12, atol=1e-13)
    rs, _ = oracle.scan_fwd("linrec", np.zeros(n), b)
    np.testing.assert_array_equal(rs[:, 1], b)
    # reduce of linrec = last scan element; its adjoint = scan adjoint with
    # y_bar only at the end
    r = oracle.reduce_fwd("linrec", a, b)
    np.testing.assert_allclose(r["y"], rs[-1] * 0 + oracle.scan_fwd("linrec", a, b)[0][-1], rtol=1e-13)


def test_mat2_embeds_linrec_and_mul():
    rng = np.random.default_rng(6)
    n = 50
    a = rng.uniform(0.5, 1.5, n)
    b = rng.standard_normal(n)
    # [[a,0],[b,1]] products: entry (0,0) = A, entry (1,0) = y
    M = np.stack([a, np.zeros(n), b, np.ones(n)], 1)
    P, _ = oracle.scan_fwd("mat2", M)
    rs, _ = oracle.scan_fwd("linrec", a, b)
    np.testing.assert_allclose(P[:, 0], rs[:, 0], rtol=1e-12)
    np.testing.assert_allclose(P[:, 2], rs[:, 1], rtol=1e-12, atol=1e-13)
    yb, Ab = rng.standard_normal(n), rng.standard_normal(n)
    Pb = np.zeros((n, 4))
    Pb[:, 0] = Ab
    Pb[:, 2] = yb
    Mb, _ = oracle.scan_vjp("mat2", Pb, M)
    xb, _ = oracle.scan_vjp("linrec", np.stack([Ab, yb], 1), a, b)
    np.testing.assert_allclose(Mb[:, 0], xb[:, 0], rtol=1e-11, atol=1e-12)
    np.testing.assert_allclose(Mb[:, 2], xb[:, 1], rtol=1e-11, atol=1e-12)
    # diagonal matrices are two independent scans with *
    p, q = rng.uniform(0.5, 2, n), rng.uniform(0.5, 2, n)
    M = np.stack([p, np.zeros(n), np.zeros(n), q], 1)
    P, _ = oracle.scan_fwd("mat2", M)
    np.testing.assert_allclose(P[:, 0], np.cumprod(p), rtol=1e-12)
    np.testing.assert_allclose(P[:, 3], np.cumprod(q), rtol=1e-12)
    Pb = rng.standard_normal((n, 4))
    Mb, _ = oracle.scan_vjp("mat2", Pb, M)
    np.testing.assert_allclose(Mb[:, 0], oracle.scan_vjp("mul", Pb[:, 0], p)[0][:, 0], rtol=1e-11)
    np.testing.assert_allclose(Mb[:, 3], oracle.scan_vjp("mul", Pb[:, 3], q)[0][:, 0], rtol=1e-11)
    # det P_i = prod det M_j
    M = rng.standard_normal((n, 4)) * 0.8
    P, _ = oracle.scan_fwd("mat2", M)
    det = lambda X: X[:, 0] * X[:, 3] - X[:, 1] * X[:, 2]
    scale = np.abs(P[:, 0] * P[:, 3]) + np.abs(P[:, 1] * P[:, 2])
    assert np.all(np.abs(det(P) - np.cumprod(det(M))) <= 1e-12 * scale)


def test_rbi_closed_forms():
    rng = np.random.default_rng(7)
    n, m = 3000, 41
    idx = rng.integers(-2, m + 2, n).astype(np.int32)
    ok = (idx >= 0) & (idx < m)
    v = rng.standard_normal(n).astype(np.float32)
    hb = rng.standard_normal(m)
    vb, _ = oracle.rbi_vjp("add", idx, m, hb, v)
    exp = np.where(ok, hb[np.clip(idx, 0, m - 1)], 0.0)
    np.testing.assert_array_equal(vb[:, 0], exp)
    cnt = np.bincount(idx[ok], minlength=m)
    assert np.sum(vb) == pytest.approx(np.sum(cnt * hb), rel=1e-12)
    for op in ("min", "max"):
        r = oracle.rbi_fwd(op, idx, m, v)
        vb, _ = oracle.rbi_vjp(op, idx, m, hb, v)
        exp = np.zeros(n)
        hit = r["argk"] < n
        exp[r["argk"][hit]] = hb[hit]
        np.testing.assert_array_equal(vb[:, 0], exp)
    vm = v.astype(np.float64)
    vm[rng.choice(n, 120, replace=False)] = 0.0
    r = oracle.rbi_fwd("mul", idx, m, vm)
    vb, _ = oracle.rbi_vjp("mul", idx, m, hb, vm)
    for i in range(n):
        if not ok[i]:
            assert vb[i, 0] == 0.0
            continue
        k = idx[i]
        if r["n0"][k] == 0:
            e = r["ypos"][k] / vm[i] * hb[k]
        elif r["n0"][k] == 1 and vm[i] == 0.0:
            e = r["ypos"][k] * hb[k]
        else:
            e = 0.0
        assert vb[i, 0] == pytest.approx(e, rel=1e-12, abs=0)


# ---------------------------------------------------------------------------
# brute-force Jacobians with dual numbers
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("op", OPS)
@pytest.mark.parametrize("n", [1, 2, 3, 7, 16])
def test_dual_jacobian_scan_reduce(op, n):
    rng = np.random.default_rng(100 + n)
    X = rand_elems(op, n, rng)
    vals, J = dual_scan(op, X)
    rs, crs = oracle.scan_fwd(op, *as_args(op, X))
    np.testing.assert_allclose(rs, vals, rtol=1e-13, atol=1e-15)
    assert np.all(crs >= np.abs(rs) * (1 - 1e-15))
    yb = rng.standard_normal(X.shape)
    xb, cxb = oracle.scan_vjp(op, yb, *as_args(op, X))
    np.testing.assert_allclose(xb.reshape(-1), J.T @ yb.reshape(-1), rtol=1e-12, atol=1e-13)
    assert np.all(cxb >= np.abs(xb) * (1 - 1e-12))
    # reduce
    y, Jr = dual_reduce(op, X)
    r = oracle.reduce_fwd(op, *as_args(op, X))
    np.testing.assert_allclose(r["y"], y, rtol=1e-13, atol=1e-15)
    ybr = rng.standard_normal(D[op])
    xb, _ = oracle.reduce_vjp(op, ybr, *as_args(op, X))
    np.testing.assert_allclose(xb.reshape(-1), Jr.T @ ybr, rtol=1e-12, atol=1e-13)


@pytest.mark.parametrize("op", OPS)
def test_dual_jacobian_rbi(op):
    rng = np.random.default_rng(200)
    n, m = 16, 5
    X = rand_elems(op, n, rng)
    if op in ("min", "max"):
        X = np.round(X * 2) / 2  # force ties
    idx = rng.integers(-1, m + 1, n).astype(np.int32)
    J = dual_rbi(op, idx, m, X)
    hb = rng.standard_normal((m, D[op]))
    vb, _ = oracle.rbi_vjp(op, idx, m, hb, *as_args(op, X))
    np.testing.assert_allclose(vb.reshape(-1), J.T @ hb.reshape(-1), rtol=1e-12, atol=1e-13)


# ---------------------------------------------------------------------------
# finite differences of the oracle forward (smooth operators)
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("op", ["add", "mul", "linrec", "mat2"])
def test_finite_differences(op):
    rng = np.random.default_rng(300)
    n = 12
    X = rand_elems(op, n, rng)
    yb = rng.standard_normal(X.shape)
    xb, _ = oracle.scan_vjp(op, yb, *as_args(op, X))
    h = 1e-6
    fd = np.zeros(X.size)
    for j in range(X.size):
        Xp, Xm = X.copy().reshape(-1), X.copy().reshape(-1)
        Xp[j] += h
        Xm[j] -= h
        fp = oracle.scan_fwd(op, *as_args(op, Xp.reshape(X.shape)))[0]
        fm = oracle.scan_fwd(op, *as_args(op, Xm.reshape(X.shape)))[0]
        fd[j] = np.sum((fp - fm) * yb) / (2 * h)
    np.testing.assert_allclose(xb.reshape(-1), fd, rtol=1e-6, atol=1e-7)


# ---------------------------------------------------------------------------
# the paper's alternative rules for the same adjoints
# ---------------------------------------------------------------------------
def local_vjp(f, x, ybar):
    """VJP of f at x (a list of floats) by forward-mode duals."""
    d = len(x)
    xs = [Dual(float(x[t]), np.eye(d)[t]) for t in range(d)]
    out = f(xs)
    J = np.array([o.t if isinstance(o, Dual) else np.zeros(d) for o in out])
    return J.T @ np.asarray(ybar, dtype=float)


@pytest.mark.parametrize("op", OPS)
def test_general_reduce_rule(op):
    """Reduce rule figure: l = exclusive scan, r = reversed exclusive scan with
    the flipped operator, then x_bar_i = vjp(x -> l_i (.) x (.) r_i)(x_i, y_bar)."""
    rng = np.random.default_rng(400)
    n = 25
    X = rand_elems(op, n, rng)
    yb = rng.standard_normal(D[op])
    e = py_neutral(op)
    ls, acc = [], list(e)
    for i in range(n):
        ls.append(acc)
        acc = py_op(op, acc, list(X[i]))
    rs, acc = [None] * n, list(e)
    for i in range(n - 1, -1, -1):
        rs[i] = acc
        acc = py_op(op, list(X[i]), acc)  # flipped operator: y (.) x with x the new element on the left
    exp = np.array([local_vjp(lambda x, i=i: py_op(op, py_op(op, ls[i], x), rs[i]), X[i], yb)
                    for i in range(n)])
    xb, _ = oracle.reduce_vjp(op, yb, *as_args(op, X))
    np.testing.assert_allclose(xb, exp, rtol=1e-11, atol=1e-12)


def _mat_vec_lin(c2, c1):
    return c2 @ c1


@pytest.mark.parametrize("op", OPS)
def test_general_scan_rule(op):
    """Scan rule figure: cs_i = d(rs_i (.) as_{i+1})/d rs_i (cs_{n-1} = I),
    then a scan of reversed (y_bar, cs) pairs with linear-function
    composition lin_o (b1,c1)(b2,c2) = (b2 + c2.b1, c2 x c1), then the map
    a_bar_i = vjp(x -> rs_{i-1} (.) x)(as_i, rs_bar_i), a_bar_0 = rs_bar_0.
    The Jacobians act transposed (the paper's notation caveat)."""
    rng = np.random.default_rng(500)
    n = 20
    X = rand_elems(op, n, rng)
    d = D[op]
    yb = rng.standard_normal((n, d))
    rs = [list(X[0])]
    for i in range(1, n):
        rs.append(py_op(op, rs[-1], list(X[i])))
    cs = []
    for i in range(n):
        if i == n - 1:
            cs.append(np.eye(d))
        else:
            xs = [Dual(float(rs[i][t]), np.eye(d)[t]) for t in range(d)]
            out = py_op(op, xs, list(X[i + 1]))
            cs.append(np.array([o.t if isinstance(o, Dual) else np.zeros(d) for o in out]))
    # scan over the reversed sequence with lin_o, via recursive doubling
    elems = [(yb[n - 1 - j].copy(), cs[n - 1 - j].T.copy()) for j in range(n)]

    def lin_o(p, q):
        b1, c1 = p
        b2, c2 = q
        return (b2 + c2 @ b1, _mat_vec_lin(c2, c1))

    cur = list(elems)
    step = 1
    while step < n:
        cur = [cur[j] if j < step else lin_o(cur[j - step], cur[j]) for j in range(n)]
        step *= 2
    rsbar = np.array([cur[n - 1 - i][0] for i in range(n)])
    exp = np.zeros((n, d))
    for i in range(n):
        if i == 0:
            exp[i] = rsbar[0]
        else:
            exp[i] = local_vjp(lambda x, i=i: py_op(op, rs[i - 1], x), X[i], rsbar[i])
    xb, _ = oracle.scan_vjp(op, yb, *as_args(op, X))
    np.testing.assert_allclose(xb, exp, rtol=1e-11, atol=1e-12)


@pytest.mark.parametrize("op", OPS)
def test_ppad_scan_rule(op):
    """PPAD's rule (appendix figure): a right scan with op_lft over
    (x, u_lft, x_bar) triples, then op_bar_2 against the shifted prefixes."""
    rng = np.random.default_rng(600)
    n = 18
    X = rand_elems(op, n, rng)
    d = D[op]
    e = py_neutral(op)
    xb_in = rng.standard_normal((n, d))
    xs = [list(X[0])]
    for i in range(1, n):
        xs.append(py_op(op, xs[-1], list(X[i])))

    def op_bar_1(x, y, rb):  # vjp of (a -> a (.) y) at x
        return local_vjp(lambda a: py_op(op, a, y), x, rb)

    def op_bar_2(x, y, rb):  # vjp of (b -> x (.) b) at y
        return local_vjp(lambda b: py_op(op, x, b), y, rb)

    def op_lft(p, q):
        x1, a1, y1h = p
        _, a2, y2h = q
        return (x1, py_op(op, a1, a2), op_bar_1(x1, a1, y2h) + y1h)

    u_lft = [list(X[i + 1]) if i < n - 1 else list(e) for i in range(n)]
    m = [(xs[i], u_lft[i], xb_in[i]) for i in range(n)]
    acc = (list(e), list(e), np.zeros(d))
    xhat = [None] * n
    for i in range(n - 1, -1, -1):
        acc = op_lft(m[i], acc)
        xhat[i] = acc[2]
    x_rht = [list(e) if i == 0 else xs[i - 1] for i in range(n)]
    exp = np.array([op_bar_2(x_rht[i], list(X[i]), xhat[i]) for i in range(n)])
    xb, _ = oracle.scan_vjp(op, xb_in, *as_args(op, X))
    np.testing.assert_allclose(xb, exp, rtol=1e-11, atol=1e-12)


@pytest.mark.parametrize("op", OPS)
def test_sort_based_rbi_rule(op):
    """Reduce-by-index rule figure: stable sort of iota by key, forward and
    reverse exclusive segmented scans, per-element vjp of l (.) x (.) r with
    the bin's adjoint, scattered back; out-of-range keys get zero."""
    rng = np.random.default_rng(700)
    n, m = 60, 7
    X = rand_elems(op, n, rng)
    if op in ("min", "max"):
        X = np.round(X * 2) / 2
    d = D[op]
    idx = rng.integers(-1, m + 1, n).astype(np.int32)
    hb = rng.standard_normal((m, d))
    e = py_neutral(op)
    siota = np.argsort(idx, kind="stable")
    sks = idx[siota]
    svs = X[siota]
    flag = np.array([i == 0 or sks[i - 1] != sks[i] for i in range(n)])
    ls, acc = [], None
    for i in range(n):
        if flag[i]:
            acc = list(e)
        ls.append(acc)
        acc = py_op(op, acc, list(svs[i]))
    rsr = [None] * n
    acc = None
    for i in range(n - 1, -1, -1):
        if i == n - 1 or flag[i + 1]:
            acc = list(e)
        rsr[i] = acc
        acc = py_op(op, list(svs[i]), acc)
    sbar = np.zeros((n, d))
    for i in range(n):
        k = sks[i]
        if 0 <= k < m:
            sbar[i] = local_vjp(lambda x, i=i: py_op(op, py_op(op, ls[i], x), rsr[i]), svs[i], hb[k])
    exp = np.zeros((n, d))
    exp[siota] = sbar
    vb, _ = oracle.rbi_vjp(op, idx, m, hb, *as_args(op, X))
    np.testing.assert_allclose(vb, exp, rtol=1e-11, atol=1e-12)


def test_segmented_matches_per_instance():
    from workloads import segmented
    w = segmented(S=6, m=8, median=40, cap=200)
    f = oracle.segmented_fwd(w["offsets"], w["a"], w["b"], w["idx"], 8)
    off = w["offsets"]
    for s in range(6):
        lo, hi = off[s], off[s + 1]
        rs, _ = oracle.scan_fwd("linrec", w["a"][lo:hi], w["b"][lo:hi])
        np.testing.assert_array_equal(f["y"][lo:hi], rs[:, 1])
        for k in range(8):
            mem = np.flatnonzero(w["idx"][lo:hi] == k)
            if mem.size == 0:
                assert f["argk"][s, k] == hi - lo
            else:
                y32 = rs[mem, 1].astype(np.float32)
                assert f["argk"][s, k] == mem[np.argmin(y32)]
    ab, bb, cab, cbb = oracle.segmented_vjp(off, w["a"], w["b"], w["idx"], 8, w["ybar"], w["hbar"], f["argk"])
    assert np.all(cab >= np.abs(ab)) and np.all(cbb >= np.abs(bb))
    # the min-by-index adjoint plus y_bar, pushed through the linrec adjoint
    s = 2
    lo, hi = off[s], off[s + 1]
    yt = w["ybar"][lo:hi].astype(np.float64).copy()
    for k in range(8):
        j = f["argk"][s, k]
        if j < hi - lo:
            yt[j] += w["hbar"][s * 8 + k]
    xb, _ = oracle.scan_vjp("linrec", np.stack([np.zeros(hi - lo), yt], 1), w["a"][lo:hi], w["b"][lo:hi])
    np.testing.assert_allclose(bb[lo:hi], xb[:, 1], rtol=1e-13)


# -------------------------------------------------------------------------
# sumOfProd (Section 3.3; reduce-by-index: Section 4.2, Invertible Operators)
# -------------------------------------------------------------------------
def _sp_comb(a, b):
    """The operator as Section 3.3 defines it, written independently."""
    return (a[0] + b[0] + a[1] * b[1], a[1] + b[1])


def _sp_inv(z, b):
    """Its left inverse: z = a (.) b  =>  a = z inv b."""
    return (z[0] - b[0] - (z[1] - b[1]) * b[1], z[1] - b[1])


@pytest.mark.parametrize("seed", range(6))
def test_sumprod_reduce_closed_forms(seed):
    """Small integers keep float64 exact: p equals the brute-force pair sum
    and (S^2 - sum a^2)/2, s equals S, a_bar equals (S - a) y_bar."""
    rng = np.random.default_rng(seed)
    n = int(rng.integers(1, 40))
    a = rng.integers(-9, 10, n).astype(np.float64)
    r = oracle.sumprod_reduce(a)
    brute = sum(a[i] * a[j] for i in range(n) for j in range(i + 1, n))
    S = a.sum()
    assert r["y"] == brute == (S * S - (a * a).sum()) / 2
    assert r["s"] == S
    assert r["c"] >= abs(r["y"])
    xb, c = oracle.sumprod_reduce_vjp(a, 3.0)
    np.testing.assert_array_equal(xb, (S - a) * 3.0)
    # the companion of the invertible rule's s - a_i: every |a_j| counts
    np.testing.assert_array_equal(c, np.full(n, np.abs(a).sum() * 3.0))
    assert np.all(c >= np.abs(xb))


def test_sumprod_reduce_fd_and_empty():
    rng = np.random.default_rng(11)
    a = rng.standard_normal(25)
    xb, _ = oracle.sumprod_reduce_vjp(a, 1.0)
    h = 1e-6
    for k in range(0, 25, 4):
        e = np.zeros_like(a)
        e[k] = h
        fd = (oracle.sumprod_reduce(a + e)["y"] - oracle.sumprod_reduce(a - e)["y"]) / (2 * h)
        assert abs(fd - xb[k]) <= 1e-7 * (1 + abs(xb[k]))
    r = oracle.sumprod_reduce(np.zeros(0))
    assert r["y"] == 0.0 and r["s"] == 0.0
    r = oracle.sumprod_reduce(np.array([7.0]))
    assert r["y"] == 0.0 and r["s"] == 7.0


@pytest.mark.parametrize("seed", range(4))
def test_sumprod_rbi_against_brute_force_and_the_invertible_rule(seed):
    """Per bin the pair sum and value sum by brute force; the adjoint by the
    paper's invertible-operator rule (b_i = hist[k] inv (0, v_i), then the
    derivative of b_i (.) (0, x) in x, which is b_i's s), written here
    from the operator alone, and by its closed form (s_k - v_i) h_bar[k]."""
    rng = np.random.default_rng(100 + seed)
    n, m = 60, 7
    v = rng.integers(-5, 6, n).astype(np.float64)
    idx = rng.integers(-2, m + 2, n).astype(np.int32)
    hb = rng.integers(-4, 5, m).astype(np.float64)
    r = oracle.sumprod_rbi_fwd(idx, m, v)
    for k in range(m):
        vk = v[idx == k]
        assert r["hist"][k] == sum(vk[i] * vk[j] for i in range(len(vk)) for j in range(i + 1, len(vk)))
        assert r["s"][k] == vk.sum() and r["count"][k] == len(vk)
    vb, c = oracle.sumprod_rbi_vjp(idx, m, hb, v)
    for i in range(n):
        k = idx[i]
        if k < 0 or k >= m:
            assert vb[i] == 0.0
            continue
        b = _sp_inv((r["hist"][k], r["s"][k]), (0.0, v[i]))
        assert _sp_comb(b, (0.0, v[i])) == (r["hist"][k], r["s"][k])
        assert vb[i] == b[1] * hb[k] == (r["s"][k] - v[i]) * hb[k]
    assert np.all(c >= np.abs(vb))


def test_sumprod_operator_is_associative_commutative_invertible():
    rng = np.random.default_rng(5)
    for _ in range(50):
        x, y, z = (tuple(rng.integers(-20, 21, 2).astype(float)) for _ in range(3))
        assert _sp_comb(_sp_comb(x, y), z) == _sp_comb(x, _sp_comb(y, z))
        assert _sp_comb(x, y) == _sp_comb(y, x)
        assert _sp_inv(_sp_comb(x, y), y) == x
    # the oracle's fold agrees with the operator applied left to right
    a = rng.integers(-9, 10, 12).astype(float)
    acc = (0.0, 0.0)
    for t in a:
        acc = _sp_comb(acc, (0.0, t))
    r = oracle.sumprod_reduce(a)
    assert (r["y"], r["s"]) == acc


# -------------------------------------------------------------------------
# vectorised operators (Sections 3.2, 4.2, 5.3 Vectorized Operators)
# -------------------------------------------------------------------------
def test_vectorised_forwards_against_numpy_axis0():
    """Small integers keep float64 exact: column folds, scans and histograms
    against numpy's axis-0 reductions and scatter-updates."""
    rng = np.random.default_rng(21)
    n, d, m = 23, 5, 6
    X = rng.integers(-4, 5, (n, d)).astype(float)
    X[X == 0] = 1.0
    idx = rng.integers(-1, m + 1, n).astype(np.int32)
    for op, red, acc in (("add", np.sum, np.add.accumulate), ("mul", np.prod, np.multiply.accumulate),
                         ("min", np.min, np.minimum.accumulate), ("max", np.max, np.maximum.accumulate)):
        r = oracle.vreduce_fwd(op, X)
        np.testing.assert_array_equal(r["y"], red(X, axis=0))
        if op in ("min", "max"):
            ref = np.argmin(X, axis=0) if op == "min" else np.argmax(X, axis=0)
            np.testing.assert_array_equal(r["k"], ref)  # numpy returns the first extremum
        Y, _ = oracle.vscan_fwd(op, X)
        np.testing.assert_array_equal(Y, acc(X, axis=0))
        h = oracle.vrbi_fwd(op, idx, m, X)["hist"]
        ref = np.full((m, d), {"add": 0.0, "mul": 1.0, "min": np.inf, "max": -np.inf}[op])
        ok = (idx >= 0) & (idx < m)
        {"add": np.add, "mul": np.multiply, "min": np.minimum, "max": np.maximum}[op].at(ref, idx[ok], X[ok])
        np.testing.assert_array_equal(h, ref)


def test_vectorised_adjoints_are_per_component():
    """Perturbing one component column leaves the other columns' adjoints
    unchanged, and central differences of the forward match the adjoint."""
    rng = np.random.default_rng(22)
    n, d, m = 17, 4, 5
    X = rng.uniform(0.5, 1.5, (n, d))
    yb = rng.standard_normal(d)
    Yb = rng.standard_normal((n, d))
    idx = rng.integers(0, m, n).astype(np.int32)
    Hb = rng.standard_normal((m, d))
    for op in ("add", "mul"):
        g, _ = oracle.vreduce_vjp(op, yb, X)
        gs, _ = oracle.vscan_vjp(op, Yb, X)
        gr, _ = oracle.vrbi_vjp(op, idx, m, Hb, X)
        X2 = X.copy()
        X2[:, 1] *= 1.3
        np.testing.assert_array_equal(oracle.vreduce_vjp(op, yb, X2)[0][:, 0], g[:, 0])
        np.testing.assert_array_equal(oracle.vscan_vjp(op, Yb, X2)[0][:, 2], gs[:, 2])
        np.testing.assert_array_equal(oracle.vrbi_vjp(op, idx, m, Hb, X2)[0][:, 3], gr[:, 3])
        h = 1e-6
        for (i, j) in ((0, 0), (5, 2), (16, 3)):
            E = np.zeros_like(X)
            E[i, j] = h
            f = lambda Z: float(oracle.vreduce_fwd(op, Z)["y"] @ yb)
            assert abs((f(X + E) - f(X - E)) / (2 * h) - g[i, j]) <= 1e-7 * (1 + abs(g[i, j]))
            fs = lambda Z: float((oracle.vscan_fwd(op, Z)[0] * Yb).sum())
            assert abs((fs(X + E) - fs(X - E)) / (2 * h) - gs[i, j]) <= 1e-7 * (1 + abs(gs[i, j]))
            fr = lambda Z: float((oracle.vrbi_fwd(op, idx, m, Z)["hist"] * Hb).sum())
            assert abs((fr(X + E) - fr(X - E)) / (2 * h) - gr[i, j]) <= 1e-7 * (1 + abs(gr[i, j]))


# -------------------------------------------------------------------------
# saturated addition (the evaluation's operator figure, Section 6.1)
# -------------------------------------------------------------------------
CAP = 1e6


def _sat_loop_with_jacobian(x):
    """Sequential saturated sums and their Jacobian by forward-mode
    derivative vectors, written from the operator's definition alone."""
    n = len(x)
    ys, J = [], np.zeros((n, n))
    acc, dacc = 0.0, np.zeros(n)
    for i, v in enumerate(x):
        e = np.zeros(n)
        e[i] = 1.0
        if i == 0:
            acc, dacc = v, e
        elif acc + v > CAP:
            acc, dacc = CAP, np.zeros(n)
        else:
            acc, dacc = acc + v, dacc + e
        ys.append(acc)
        J[i] = dacc
    return np.array(ys), J


@pytest.mark.parametrize("seed", range(6))
def test_satadd_scan_and_reduce_against_brute_force(seed):
    rng = np.random.default_rng(300 + seed)
    n = int(rng.integers(1, 30))
    x = rng.integers(0, 4, n).astype(float) * rng.choice([1.0, 1e5, 3e5], n)
    yb = rng.standard_normal(n)
    Y, J = _sat_loop_with_jacobian(x)
    rs, c = oracle.scan_fwd("satadd", x)
    np.testing.assert_array_equal(rs[:, 0], Y)
    assert np.all(c[:, 0] >= np.abs(Y))
    xb, _ = oracle.scan_vjp("satadd", yb, x)
    np.testing.assert_allclose(xb[:, 0], J.T @ yb, rtol=1e-12, atol=1e-12)
    r = oracle.reduce_fwd("satadd", x)
    assert r["y"][0] == Y[-1]
    g, _ = oracle.reduce_vjp("satadd", np.array([1.5]), x)
    np.testing.assert_allclose(g[:, 0], 1.5 * J[-1], rtol=1e-12, atol=1e-12)


def test_satadd_reduce_general_rule():
    """The general reduce rule (Section 3.1): x_bar_i = d(l_i (.) x_i (.) r_i)/d x_i
    y_bar with exclusive prefix l_i and suffix r_i.  For non-negative values
    the operator is associative, but its derivative depends on the
    bracketing where a bracket lands exactly on the cap (a kink: a zero
    prefix meeting a saturated suffix, or a partial sum equal to 1e6).  The
    values here are positive multiples of 3e5, whose sums never equal 1e6,
    and then the rule equals the reverse sweep."""
    rng = np.random.default_rng(9)
    for _ in range(20):
        n = int(rng.integers(2, 25))
        x = rng.integers(1, 4, n).astype(float) * 3e5
        sat = lambda a, b: CAP if a + b > CAP else a + b
        g, _ = oracle.reduce_vjp("satadd", np.array([1.0]), x)
        for i in range(n):
            l = 0.0
            for t in x[:i]:
                l = sat(l, t)
            r = 0.0
            for t in x[i + 1:][::-1]:
                r = sat(t, r)
            lx = sat(l, x[i])
            d = (0.0 if l + x[i] > CAP else 1.0) * (0.0 if lx + r > CAP else 1.0)
            assert g[i, 0] == d, (x, i)


def test_satadd_rbi_against_per_bin_loops():
    rng = np.random.default_rng(10)
    n, m = 80, 5
    v = rng.integers(0, 4, n).astype(float) * 2e5
    idx = rng.integers(-1, m + 1, n).astype(np.int32)
    hb = rng.standard_normal(m)
    r = oracle.rbi_fwd("satadd", idx, m, v)
    vb, _ = oracle.rbi_vjp("satadd", idx, m, hb, v)
    for k in range(m):
        sel = np.flatnonzero(idx == k)
        if sel.size == 0:
            assert r["hist"][k, 0] == 0.0
            continue
        Y, J = _sat_loop_with_jacobian(v[sel])
        assert r["hist"][k, 0] == Y[-1]
        np.testing.assert_allclose(vb[sel, 0], hb[k] * J[-1], rtol=1e-12, atol=1e-12)
    assert np.all(vb[(idx < 0) | (idx >= m), 0] == 0.0)


@pytest.mark.parametrize("seed", range(4))
def test_sumprod_scan_closed_forms(seed):
    """y_i = sum_{j<k<=i} a_j a_k by brute force, and the adjoint
    d/da_m sum_i ybar_i y_i = sum_{i>=m} ybar_i (S_i - a_m), S_i = a_0+..+a_i."""
    rng = np.random.default_rng(500 + seed)
    n = int(rng.integers(1, 30))
    a = rng.integers(-6, 7, n).astype(float)
    yb = rng.integers(-3, 4, n).astype(float)
    y, c = oracle.sumprod_scan(a)
    for i in range(n):
        assert y[i] == sum(a[j] * a[k] for j in range(i + 1) for k in range(j + 1, i + 1))
    assert np.all(c >= np.abs(y))
    S = np.cumsum(a)
    xb, cx = oracle.sumprod_scan_vjp(a, yb)
    ref = np.array([sum(yb[i] * (S[i] - a[m_]) for i in range(m_, n)) for m_ in range(n)])
    np.testing.assert_array_equal(xb, ref)
    assert np.all(cx >= np.abs(xb))


# -------------------------------------------------------------------------
# d x d matrix-product scans (the evaluation's matMul3x3 / matMul5x5)
# -------------------------------------------------------------------------
@pytest.mark.parametrize("d", [2, 3, 5])
def test_matd_scan_against_products_and_the_2x2_oracle(d):
    rng = np.random.default_rng(40 + d)
    n = 9
    M = rng.integers(-2, 3, (n, d, d)).astype(float)
    P, c = oracle.matd_scan(M)
    for i in range(n):
        np.testing.assert_array_equal(P[i], np.linalg.multi_dot(list(M[: i + 1])) if i > 0 else M[0])
        assert c[i] >= np.abs(P[i]).max() - 1e-12
    if d == 2:
        rs, _ = oracle.scan_fwd("mat2", M.reshape(n, 4))
        np.testing.assert_array_equal(P.reshape(n, 4), rs)
        Pb = rng.integers(-2, 3, (n, 2, 2)).astype(float)
        xb, _ = oracle.scan_vjp("mat2", Pb.reshape(n, 4), M.reshape(n, 4))
        Mb, _ = oracle.matd_scan_vjp(M, Pb)
        np.testing.assert_array_equal(Mb.reshape(n, 4), xb)


@pytest.mark.parametrize("d", [3, 5])
def test_matd_scan_vjp_central_differences_and_embedding(d):
    rng = np.random.default_rng(50 + d)
    n = 7
    M = rng.standard_normal((n, d, d)) * 0.6
    Pb = rng.standard_normal((n, d, d))
    Mb, c = oracle.matd_scan_vjp(M, Pb)
    assert np.all(c >= np.abs(Mb).max(axis=(1, 2)) - 1e-12)
    f = lambda Z: float((oracle.matd_scan(Z)[0] * Pb).sum())
    h = 1e-6
    for (i, a, b) in ((0, 0, 1), (3, d - 1, 0), (6, 1, 2)):
        E = np.zeros_like(M)
        E[i, a, b] = h
        fd = (f(M + E) - f(M - E)) / (2 * h)
        assert abs(fd - Mb[i, a, b]) <= 1e-6 * (1 + abs(fd))
    # a 2x2 block embedded with an identity block scans (and adjoints) as the 2x2 product
    M2 = rng.standard_normal((n, 2, 2))
    Pb2 = rng.standard_normal((n, 2, 2))
    Me = np.tile(np.eye(d), (n, 1, 1))
    Me[:, :2, :2] = M2
    Pbe = np.zeros((n, d, d))
    Pbe[:, :2, :2] = Pb2
    Pe, _ = oracle.matd_scan(Me)
    rs, _ = oracle.scan_fwd("mat2", M2.reshape(n, 4))
    np.testing.assert_allclose(Pe[:, :2, :2].reshape(n, 4), rs, rtol=1e-13, atol=1e-13)
    Mbe, _ = oracle.matd_scan_vjp(Me, Pbe)
    xb, _ = oracle.scan_vjp("mat2", Pb2.reshape(n, 4), M2.reshape(n, 4))
    np.testing.assert_allclose(Mbe[:, :2, :2].reshape(n, 4), xb, rtol=1e-12, atol=1e-12)


@pytest.mark.parametrize("d", [2, 3, 5])
def test_matd_reduce_against_products_scan_and_differences(d):
    """The reduce is the scan's last prefix; its adjoint is the scan adjoint
    seeded at the last element only (Section 3.1's rule and Section 5's
    recurrence must agree); central differences; the 2x2 case against the
    2x2 reduce oracle; the empty reduce is the identity."""
    rng = np.random.default_rng(60 + d)
    n = 8
    M = rng.integers(-2, 3, (n, d, d)).astype(float)
    Y, c = oracle.matd_reduce(M)
    np.testing.assert_array_equal(Y, np.linalg.multi_dot(list(M)))
    assert c >= np.abs(Y).max() - 1e-12
    Yb = rng.integers(-2, 3, (d, d)).astype(float)
    Mb, cm = oracle.matd_reduce_vjp(M, Yb)
    Pb = np.zeros((n, d, d))
    Pb[-1] = Yb
    Ms, _ = oracle.matd_scan_vjp(M, Pb)
    np.testing.assert_array_equal(Mb, Ms)
    assert np.all(cm >= np.abs(Mb).max(axis=(1, 2)) - 1e-12)
    Mg = rng.standard_normal((n, d, d)) * 0.7
    Mbg, _ = oracle.matd_reduce_vjp(Mg, Yb)
    f = lambda Z: float((oracle.matd_reduce(Z)[0] * Yb).sum())
    h = 1e-6
    for (i, a, b) in ((0, 1, 0), (4, 0, d - 1), (7, d - 1, 1)):
        E = np.zeros_like(Mg)
        E[i, a, b] = h
        fd = (f(Mg + E) - f(Mg - E)) / (2 * h)
        assert abs(fd - Mbg[i, a, b]) <= 1e-6 * (1 + abs(fd))
    if d == 2:
        y2 = oracle.reduce_fwd("mat2", M.reshape(n, 4))["y"]
        np.testing.assert_array_equal(y2.reshape(2, 2), Y)
        xb, _ = oracle.reduce_vjp("mat2", Yb.reshape(4), M.reshape(n, 4))
        np.testing.assert_array_equal(xb.reshape(n, 2, 2), Mb)
    Y0, c0 = oracle.matd_reduce(np.zeros((0, d, d)))
    np.testing.assert_array_equal(Y0, np.eye(d))
    assert c0 == 1.0


# -------------------------------------------------------------------------
# int32 forward combinators (wrapping mod 2^32)
# -------------------------------------------------------------------------
@pytest.mark.parametrize("op", ["add", "mul", "min", "max"])
def test_i32_against_numpy_wrapping_arithmetic(op):
    """numpy's int32 arithmetic wraps mod 2^32 (two's complement): its
    accumulate and ufunc.at must agree with the oracle's loops, including
    on values that overflow."""
    rng = np.random.default_rng(70 + len(op))
    x = rng.integers(-2**31, 2**31, 500, dtype=np.int64).astype(np.int32)
    if op == "mul":
        x = rng.integers(-7, 8, 500).astype(np.int32)  # products wrap many times
    uf = {"add": np.add, "mul": np.multiply, "min": np.minimum, "max": np.maximum}[op]
    with np.errstate(over="ignore"):
        ref_scan = uf.accumulate(x, dtype=np.int32)
    np.testing.assert_array_equal(oracle.i32_scan(op, x), ref_scan)
    assert oracle.i32_reduce(op, x) == int(ref_scan[-1])
    m = 37
    idx = rng.integers(-3, m + 3, 500).astype(np.int32)
    h = np.full(m, oracle._I32_NEUTRAL[op], dtype=np.int32)
    ok = (idx >= 0) & (idx < m)
    with np.errstate(over="ignore"):
        uf.at(h, idx[ok], x[ok])
    np.testing.assert_array_equal(oracle.i32_rbi(op, idx, m, x), h)


def test_i32_closed_forms():
    n = 100_000
    x = np.arange(n, dtype=np.int32)
    assert oracle.i32_reduce("add", x) == (n * (n - 1) // 2 + 2**31) % 2**32 - 2**31
    assert oracle.i32_reduce("add", np.zeros(0, np.int32)) == 0
    assert oracle.i32_reduce("mul", np.zeros(0, np.int32)) == 1
    assert oracle.i32_reduce("min", np.zeros(0, np.int32)) == 2**31 - 1
    assert oracle.i32_reduce("max", np.array([-2**31, -5], np.int32)) == -5
    # 2^31 wraps to -2^31; 2^32 wraps to 0
    assert oracle.i32_reduce("mul", np.array([2**16, 2**15], np.int32)) == -2**31
    assert oracle.i32_reduce("mul", np.array([2**16, 2**16], np.int32)) == 0
