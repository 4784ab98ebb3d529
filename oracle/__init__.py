"""CPU FP64 oracle for reduce / scan / reduce-by-index and their adjoints.

TEST INFRASTRUCTURE ONLY.  Only the test-suite, ``__graft_entry__.smoke()``
and the CPU-baseline leg of ``bench.py`` may import this package.  It shares
no code with the GPU library and never imports it.

The arithmetic lives in ``oracle.c`` (plain single-threaded float64, built
with gcc, no fast-math, no FMA contraction); this module only marshals numpy
arrays through ctypes and composes the C calls for the chained segmented
workload.  Every function widens its float32 inputs exactly to float64.

Operators (names used throughout): ``add``, ``mul``, ``min``, ``max``,
``linrec`` (linear-function composition, Section 6.1 operator figure, with
multiplier a and offset b, y_i = a_i*y_{i-1} + b_i), ``mat2`` (row-major
2x2 matrix product, Section 6.1 operator figure) and ``sumprod`` (the
invertible operator sumOfProd of Section 3.3 on lifted pairs (p, s); the
``sumprod_*`` functions below take the scalar inputs, lift each a to (0, a)
and return the p component, as that section composes them) and ``satadd``
(saturated addition at 1e6, the evaluation's operator figure).
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")

OPS = {"add": 0, "mul": 1, "min": 2, "max": 3, "linrec": 4, "mat2": 5, "sumprod": 6, "satadd": 7}
DIM = {"add": 1, "mul": 1, "min": 1, "max": 1, "linrec": 2, "mat2": 4, "sumprod": 2, "satadd": 1}
SAT_CAP = 1e6


def build(force: bool = True) -> str:
    """Compile oracle.c into liboracle.so with gcc (plain -O2, no contraction)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp"
        subprocess.check_call([
            "gcc", "-O2", "-std=c99", "-ffp-contract=off", "-fno-fast-math", "-fPIC",
            "-shared", _SRC, "-o", tmp, "-lm",
        ])
        os.replace(tmp, _LIB)
    return _LIB


_lib = None


def lib():
    global _lib
    if _lib is None:
        build(force=False)
        L = ctypes.CDLL(_LIB)
        P = ctypes.c_void_p
        I = ctypes.c_int
        I64 = ctypes.c_int64
        L.orc_scan_fwd.argtypes = [I, I64, P, P, P]
        L.orc_scan_vjp.argtypes = [I, I64, P, P, P, P, P]
        L.orc_reduce_fwd.argtypes = [I, I64, P, P, P, P, P, P]
        L.orc_reduce_vjp.argtypes = [I, I64, P, P, P, P]
        L.orc_rbi_fwd.argtypes = [I, I64, I64, P, P, P, P, P, P, P, P]
        L.orc_rbi_vjp.argtypes = [I, I64, I64, P, P, P, P, P]
        for f in (L.orc_scan_fwd, L.orc_scan_vjp, L.orc_reduce_fwd, L.orc_reduce_vjp,
                  L.orc_rbi_fwd, L.orc_rbi_vjp):
            f.restype = I
        _lib = L
    return _lib


def _p(a):
    return None if a is None else a.ctypes.data


def _f64(a) -> np.ndarray:
    return np.ascontiguousarray(np.asarray(a), dtype=np.float64)


def pack(op: str, x0, x1=None) -> np.ndarray:
    """Element array (n, d) float64.  linrec: x0 = a (multiplier), x1 = b
    (offset).  mat2: x0 has shape (n, 4).  Scalar ops: x0 has shape (n,)."""
    d = DIM[op]
    if op == "linrec":
        a, b = _f64(x0).reshape(-1), _f64(x1).reshape(-1)
        return np.ascontiguousarray(np.stack([a, b], axis=1))
    if op == "sumprod":
        # the lifting map of Section 3.3: a -> (0, a); a (n, 2) array is
        # taken as already lifted
        x = _f64(x0)
        if x.ndim == 2 and x.shape[1] == 2:
            return np.ascontiguousarray(x)
        a = x.reshape(-1)
        return np.ascontiguousarray(np.stack([np.zeros_like(a), a], axis=1))
    if d == 4:
        return _f64(x0).reshape(-1, 4)
    return _f64(x0).reshape(-1, 1)


def _check(rc):
    if rc != 0:
        raise RuntimeError(f"oracle error {rc}")


# -------------------------------------------------------------------------
# scan
# -------------------------------------------------------------------------
def scan_fwd(op: str, x0, x1=None):
    """Inclusive scan.  Returns (rs, c), both (n, d) float64.  For linrec
    the columns are (A, y): the cumulative multiplier and the recurrence."""
    X = pack(op, x0, x1)
    n, d = X.shape
    rs = np.empty((n, d))
    c = np.empty((n, d))
    _check(lib().orc_scan_fwd(OPS[op], n, _p(X), _p(rs), _p(c)))
    return rs, c


def scan_vjp(op: str, ybar, x0, x1=None, cybar=None):
    """Adjoint of the inclusive scan.  ``ybar`` is (n, d) (for linrec the
    columns are (A_bar, y_bar)).  ``cybar`` optionally seeds the companion
    of the output adjoint (default |ybar|).  Returns (xbar, c), (n, d)
    float64; for linrec the columns are (a_bar, b_bar)."""
    X = pack(op, x0, x1)
    n, d = X.shape
    Y = _f64(ybar).reshape(n, d)
    CY = None if cybar is None else _f64(cybar).reshape(n, d)
    xb = np.empty((n, d))
    c = np.empty((n, d))
    _check(lib().orc_scan_vjp(OPS[op], n, _p(X), _p(Y), _p(CY), _p(xb), _p(c)))
    return xb, c


# -------------------------------------------------------------------------
# reduce
# -------------------------------------------------------------------------
def reduce_fwd(op: str, x0, x1=None):
    """Left fold.  Returns dict(y (d,), c (d,), k, n0, ypos)."""
    X = pack(op, x0, x1)
    n, d = X.shape
    y = np.empty(d)
    c = np.empty(d)
    k = np.zeros(1, np.int64)
    n0 = np.zeros(1, np.int64)
    yp = np.zeros(1)
    _check(lib().orc_reduce_fwd(OPS[op], n, _p(X), _p(y), _p(c), _p(k), _p(n0), _p(yp)))
    return dict(y=y, c=c, k=int(k[0]), n0=int(n0[0]), ypos=float(yp[0]))


def reduce_vjp(op: str, ybar, x0, x1=None):
    X = pack(op, x0, x1)
    n, d = X.shape
    Y = _f64(ybar).reshape(d)
    xb = np.empty((n, d))
    c = np.empty((n, d))
    _check(lib().orc_reduce_vjp(OPS[op], n, _p(X), _p(Y), _p(xb), _p(c)))
    return xb, c


# -------------------------------------------------------------------------
# reduce-by-index
# -------------------------------------------------------------------------
def rbi_fwd(op: str, idx, m: int, v0, v1=None):
    """Sequential histogram.  Returns dict(hist (m,d), c, count, argk, n0, ypos)."""
    V = pack(op, v0, v1)
    n, d = V.shape
    ix = np.ascontiguousarray(np.asarray(idx, dtype=np.int32).reshape(-1))
    assert ix.shape[0] == n
    mm = max(int(m), 0)
    h = np.empty((mm, d))
    c = np.empty((mm, d))
    cnt = np.empty(mm, np.int64)
    ak = np.empty(mm, np.int64)
    n0 = np.empty(mm, np.int64)
    yp = np.empty(mm)
    _check(lib().orc_rbi_fwd(OPS[op], n, mm, _p(ix), _p(V), _p(h), _p(c), _p(cnt), _p(ak),
                             _p(n0), _p(yp)))
    return dict(hist=h, c=c, count=cnt, argk=ak, n0=n0, ypos=yp)


def rbi_vjp(op: str, idx, m: int, hbar, v0, v1=None):
    V = pack(op, v0, v1)
    n, d = V.shape
    ix = np.ascontiguousarray(np.asarray(idx, dtype=np.int32).reshape(-1))
    H = _f64(hbar).reshape(max(int(m), 0), d)
    vb = np.empty((n, d))
    c = np.empty((n, d))
    _check(lib().orc_rbi_vjp(OPS[op], n, int(m), _p(ix), _p(V), _p(H), _p(vb), _p(c)))
    return vb, c


# -------------------------------------------------------------------------
# chained segmented workload: per instance s,
#   y_s = linrec scan of (a_s, b_s);  (h_s, argk_s) = min-by-index(y_s, idx_s, m)
# and the adjoint of both given y_bar (per element) and h_bar (per bin).
# -------------------------------------------------------------------------
def segmented_fwd(offsets, a, b, idx, m: int):
    """Returns dict(y, cy, h, ch, argk, count) with argk relative to the
    instance start (sentinel = instance length for an empty bin).

    The min-by-index decision is taken on the float32 rounding of the
    float64 recurrence (the precision of the paper's evaluation), with the
    lowest index winning among equal float32 values; h is then the float64
    value at that position."""
    off = np.asarray(offsets, dtype=np.int64)
    S = off.shape[0] - 1
    N = int(off[-1])
    y = np.empty(N)
    cy = np.empty(N)
    h = np.empty((S, m))
    ch = np.empty((S, m))
    argk = np.empty((S, m), np.int64)
    for s in range(S):
        lo, hi = int(off[s]), int(off[s + 1])
        rs, c = scan_fwd("linrec", a[lo:hi], b[lo:hi])
        y[lo:hi] = rs[:, 1]
        cy[lo:hi] = c[:, 1]
        y32 = rs[:, 1].astype(np.float32).astype(np.float64)
        r = rbi_fwd("min", idx[lo:hi], m, y32)
        ak = r["argk"]
        argk[s] = ak
        L = hi - lo
        ok = ak < L
        hs = np.full(m, np.inf)
        chs = np.full(m, np.inf)
        hs[ok] = rs[ak[ok], 1]
        chs[ok] = c[ak[ok], 1]
        h[s] = hs
        ch[s] = chs
    return dict(y=y, cy=cy, h=h, ch=ch, argk=argk)


def segmented_argmin(offsets, idx, y32, m: int):
    """Per instance s and bin k, the lowest instance-relative index of the
    minimum of the float32 values ``y32`` over the positions of s whose key
    is k (the instance length for an empty bin), and that value: the
    sequential min-by-index (Section 4 with Section 4.2's lifted min) of the
    given values, one instance at a time.  Returns (argk (S, m) int64,
    h (S, m) float64, the winner's value with its sign bit)."""
    off = np.asarray(offsets, dtype=np.int64)
    S = off.shape[0] - 1
    y = np.asarray(y32, dtype=np.float32)
    argk = np.empty((S, m), np.int64)
    h = np.empty((S, m))
    for s in range(S):
        lo, hi = int(off[s]), int(off[s + 1])
        r = rbi_fwd("min", idx[lo:hi], m, y[lo:hi])
        argk[s] = r["argk"]
        h[s] = r["hist"][:, 0]
    return argk, h


def segmented_vjp(offsets, a, b, idx, m: int, ybar, hbar, argk):
    """Adjoint of the chained workload for a given per-bin decision
    ``argk`` (S, m) (instance-relative, >= length means empty).  The
    min-by-index adjoint adds h_bar[s,k] at position argk[s,k]; that sum is
    the adjoint of y fed to the linrec scan adjoint.  Returns (abar, bbar,
    cabar, cbbar) float64 arrays of length N."""
    off = np.asarray(offsets, dtype=np.int64)
    S = off.shape[0] - 1
    N = int(off[-1])
    hb = np.asarray(hbar, dtype=np.float64).reshape(S, m)
    ab = np.empty(N)
    bb = np.empty(N)
    cab = np.empty(N)
    cbb = np.empty(N)
    for s in range(S):
        lo, hi = int(off[s]), int(off[s + 1])
        L = hi - lo
        yt = np.zeros((L, 2))
        yt[:, 1] = ybar[lo:hi]
        ak = np.asarray(argk[s], dtype=np.int64)
        ok = ak < L
        # each element is the argmin of at most one bin, so no collisions
        yt[ak[ok], 1] += hb[s][ok]
        # companion of the summed adjoint: |y_bar| + |h_bar|
        yc = np.zeros((L, 2))
        yc[:, 1] = np.abs(ybar[lo:hi])
        yc[ak[ok], 1] += np.abs(hb[s][ok])
        xb, c = scan_vjp("linrec", yt, a[lo:hi], b[lo:hi], cybar=yc)
        ab[lo:hi] = xb[:, 0]
        bb[lo:hi] = xb[:, 1]
        cab[lo:hi] = c[:, 0]
        cbb[lo:hi] = c[:, 1]
    return ab, bb, cab, cbb


# -------------------------------------------------------------------------
# autograd workload: per sequence, loss = sum_i log|y_i| over the linear
# recurrence y of (a, b), plus the sum over non-empty bins of the
# max-by-index of v (an empty bin holds the neutral -inf and is left out).
# The gradient composes the two adjoints by the chain rule of reverse mode
# (Section 2): the scan adjoint seeded with d log|y|/dy = 1/y and the
# max-by-index adjoint seeded with 1 on every non-empty bin.
# -------------------------------------------------------------------------
def autograd_loss(a, b, v, idx, m: int) -> float:
    rs, _ = scan_fwd("linrec", a, b)
    r = rbi_fwd("max", idx, m, v)
    n = len(np.asarray(v).reshape(-1))
    full = r["argk"] < n
    return float(np.sum(np.log(np.abs(rs[:, 1]))) + np.sum(r["hist"][full, 0]))


def autograd_grad(a, b, v, idx, m: int, ybar=None):
    """Returns (a_bar, b_bar, v_bar, c_a, c_b, c_v) float64.  ``ybar``
    replaces the seed 1/y of the scan adjoint when given (e.g. the float32
    seed another implementation used)."""
    a = np.asarray(a).reshape(-1)
    n = a.shape[0]
    rs, _ = scan_fwd("linrec", a, b)
    yb = 1.0 / rs[:, 1] if ybar is None else _f64(ybar).reshape(-1)
    xb, cx = scan_vjp("linrec", np.stack([np.zeros(n), yb], 1), a, b)
    r = rbi_fwd("max", idx, m, v)
    hb = (r["argk"] < n).astype(np.float64)
    vb, cv = rbi_vjp("max", idx, m, hb, v)
    return xb[:, 0], xb[:, 1], vb[:, 0], cx[:, 0], cx[:, 1], cv[:, 0]


# -------------------------------------------------------------------------
# sumOfProd: the invertible-operator example of Section 3.3 as the
# composition lift -> fold with the lifted operator -> project to p, for
# reduce and reduce-by-index (Section 4.2, Invertible Operators).  The
# adjoints are the reverse sweep of that composition: the output adjoint
# enters as (p_bar, 0) and an input's adjoint is the s component of its
# lifted adjoint (the lifting a -> (0, a) passes only the s slot).
#
# Companions of the adjoints: the rule these adjoints specialise (Section
# 3.3, and Section 4.2 for reduce-by-index) obtains the rest of the fold by
# inverting the total with the element, i.e. it evaluates s - a_i with s the
# total sum.  Rounding in s and in that subtraction is bounded relative to
# sum_j |a_j| * |y_bar| (all elements, a_i included), not relative to the
# reverse sweep's sum over j != i; the companions returned below are
# therefore the sweep's plus |a_i| * |y_bar|.
# -------------------------------------------------------------------------
def sumprod_reduce(a):
    """Returns dict(y = p = sum_{i<j} a_i a_j, s = sum a_i, c = companion of p)."""
    r = reduce_fwd("sumprod", a)
    return dict(y=float(r["y"][0]), s=float(r["y"][1]), c=float(r["c"][0]))


def sumprod_reduce_vjp(a, ybar: float):
    """Returns (a_bar, c) for y = sum_{i<j} a_i a_j and output adjoint ybar."""
    xb, c = reduce_vjp("sumprod", np.array([float(ybar), 0.0]), a)
    av = np.abs(_f64(a).reshape(-1))
    return xb[:, 1].copy(), c[:, 1] + av * abs(float(ybar))


def sumprod_scan(a):
    """Inclusive scan with sumOfProd (Section 3.3's operator under the scan of
    Section 5.1): returns (y, c) with y_i = sum over j<k<=i of a_j a_k."""
    rs, c = scan_fwd("sumprod", a)
    return rs[:, 0].copy(), c[:, 0].copy()


def sumprod_scan_vjp(a, ybar):
    """Adjoint of sumprod_scan: the reverse sweep of the lifted scan with
    output adjoints (ybar_i, 0); an input's adjoint is the s slot."""
    yb = _f64(ybar).reshape(-1)
    yl = np.stack([yb, np.zeros_like(yb)], axis=1)
    xb, c = scan_vjp("sumprod", yl, a)
    return xb[:, 1].copy(), c[:, 1].copy()


def sumprod_rbi_fwd(idx, m: int, a):
    """Per bin: hist (p_k), s (sum of the bin's values), c (companion of p_k),
    count."""
    r = rbi_fwd("sumprod", idx, m, a)
    return dict(hist=r["hist"][:, 0].copy(), s=r["hist"][:, 1].copy(), c=r["c"][:, 0].copy(),
                count=r["count"])


def sumprod_rbi_vjp(idx, m: int, hbar, a):
    """Returns (v_bar, c): the adjoint of every value for bin adjoints hbar."""
    H = _f64(hbar).reshape(-1)
    hb = np.stack([H, np.zeros(max(int(m), 0))], axis=1)
    vb, c = rbi_vjp("sumprod", idx, m, hb, a)
    ix = np.asarray(idx, dtype=np.int64).reshape(-1)
    ok = (ix >= 0) & (ix < m)
    extra = np.zeros(ix.shape[0])
    extra[ok] = np.abs(_f64(a).reshape(-1)[ok]) * np.abs(H[ix[ok]])
    return vb[:, 1].copy(), c[:, 1] + extra


# -------------------------------------------------------------------------
# vectorised operators (Sections 3.2, 4.2 and 5.3, Vectorized Operators):
# elements are vectors of d values combined component-wise (map2 (.)).  A
# component-wise operator folds, scans or histograms each component on its
# own, so every function below applies the scalar definition to each column
# of an (n, d) array; the adjoints are per column as well (the Jacobian of a
# component-wise program is block-diagonal by component).
# -------------------------------------------------------------------------
def _cols(a):
    a = _f64(a)
    return a.reshape(a.shape[0], -1) if a.ndim > 1 else a.reshape(-1, 1)


def vreduce_fwd(op: str, X):
    """X (n, d) -> dict(y (d,), c (d,), k (d,) int, n0 (d,) int, ypos (d,))."""
    X = _cols(X)
    rs = [reduce_fwd(op, X[:, j]) for j in range(X.shape[1])]
    return dict(y=np.array([r["y"][0] for r in rs]), c=np.array([r["c"][0] for r in rs]),
                k=np.array([r["k"] for r in rs], np.int64), n0=np.array([r["n0"] for r in rs], np.int64),
                ypos=np.array([r["ypos"] for r in rs]))


def vreduce_vjp(op: str, ybar, X):
    X = _cols(X)
    yb = _f64(ybar).reshape(-1)
    out = [reduce_vjp(op, yb[j:j + 1], X[:, j]) for j in range(X.shape[1])]
    return (np.stack([o[0][:, 0] for o in out], 1) if out else np.zeros(X.shape),
            np.stack([o[1][:, 0] for o in out], 1) if out else np.zeros(X.shape))


def vscan_fwd(op: str, X):
    X = _cols(X)
    out = [scan_fwd(op, X[:, j]) for j in range(X.shape[1])]
    return np.stack([o[0][:, 0] for o in out], 1), np.stack([o[1][:, 0] for o in out], 1)


def vscan_vjp(op: str, Ybar, X):
    X = _cols(X)
    Y = _cols(Ybar)
    out = [scan_vjp(op, Y[:, j], X[:, j]) for j in range(X.shape[1])]
    return np.stack([o[0][:, 0] for o in out], 1), np.stack([o[1][:, 0] for o in out], 1)


def vrbi_fwd(op: str, idx, m: int, V):
    """idx (n,), V (n, d) -> dict(hist (m, d), c, argk (m, d), n0 (m, d), ypos (m, d))."""
    V = _cols(V)
    rs = [rbi_fwd(op, idx, m, V[:, j]) for j in range(V.shape[1])]
    return {key: np.stack([(r[key][:, 0] if r[key].ndim > 1 else r[key]) for r in rs], 1)
            for key in ("hist", "c", "argk", "n0", "ypos", "count")}


def vrbi_vjp(op: str, idx, m: int, Hbar, V):
    V = _cols(V)
    H = _f64(Hbar).reshape(max(int(m), 0), V.shape[1])
    out = [rbi_vjp(op, idx, m, H[:, j], V[:, j]) for j in range(V.shape[1])]
    return np.stack([o[0][:, 0] for o in out], 1), np.stack([o[1][:, 0] for o in out], 1)


# -------------------------------------------------------------------------
# d x d matrix-product scans, d >= 3 (the evaluation's matMul3x3 and
# matMul5x5, Section 6.1 operator figure; their adjoint by the redundant
# block-diagonal sparsity of Section 5.3): plain float64 loops.
#   forward : P_0 = M_0, P_i = P_{i-1} M_i;
#   adjoint : the reverse sweep of that loop -- Rbar_{n-1} = Pbar_{n-1},
#             Rbar_i = Pbar_i + Rbar_{i+1} M_{i+1}^T, Mbar_i = P_{i-1}^T Rbar_i
#             with P_{-1} = I (the adjoint of P_i = P_{i-1} M_i with respect
#             to both factors).
# Companions are norm-wise: every entry of a product chain is bounded by the
# product of the factors' spectral norms (Frobenius norms would grow as
# sqrt(d) per factor even for orthogonal factors and leave the float range).
# -------------------------------------------------------------------------
def matd_scan(M):
    """M (n, d, d) -> (P (n, d, d), c (n,)): inclusive products and the
    companion prod_{j<=i} ||M_j||_2 (spectral norm: it bounds ||P_i||_2 and
    so every entry, and it stays 1 along chains of orthogonal factors)."""
    M = _f64(M)
    n, d = M.shape[0], M.shape[1]
    P = np.empty_like(M)
    c = np.empty(n)
    acc, ca = np.eye(d), 1.0
    for i in range(n):
        acc = M[i].copy() if i == 0 else acc @ M[i]
        ca = (np.linalg.norm(M[i], 2) if i == 0 else ca * np.linalg.norm(M[i], 2))
        P[i], c[i] = acc, ca
    return P, c


def matd_scan_vjp(M, Pbar):
    """M, Pbar (n, d, d) -> (Mbar (n, d, d), c (n,)) with the norm-wise
    companion ||P_{i-1}|| * (sum_{j>=i} ||Pbar_j|| prod_{i<k<=j} ||M_k||),
    spectral norms throughout."""
    M, Pb = _f64(M), _f64(Pbar)
    n, d = M.shape[0], M.shape[1]
    P, cP = matd_scan(M)
    Mb = np.empty_like(M)
    c = np.empty(n)
    R, cR = None, 0.0
    for i in range(n - 1, -1, -1):
        if i == n - 1:
            R, cR = Pb[i].copy(), np.linalg.norm(Pb[i], 2)
        else:
            R = Pb[i] + R @ M[i + 1].T
            cR = np.linalg.norm(Pb[i], 2) + cR * np.linalg.norm(M[i + 1], 2)
        prev = P[i - 1] if i > 0 else np.eye(d)
        Mb[i] = prev.T @ R
        c[i] = (cP[i - 1] if i > 0 else 1.0) * cR
    return Mb, c


def matd_reduce(M):
    """M (n, d, d) -> (Y = M_0 M_1 ... M_{n-1}, c = prod ||M_j||_2); the
    identity (c = 1) for n = 0 (the operator's neutral element)."""
    M = _f64(M)
    n, d = M.shape[0], M.shape[1]
    Y, c = np.eye(d), 1.0
    for i in range(n):
        Y = Y @ M[i]
        c *= np.linalg.norm(M[i], 2)
    return Y, c


def matd_reduce_vjp(M, Ybar):
    """Section 3.1's rule for a general associative operator, written out for
    the matrix product: with L_i = M_0 ... M_{i-1} and R_i = M_{i+1} ... M_{n-1}
    (identities when empty), Mbar_i = L_i^T Ybar R_i^T; companion
    ||L_i|| ||Ybar|| ||R_i|| (spectral norms, each bounded by the product of
    its factors' norms)."""
    M, Yb = _f64(M), _f64(Ybar)
    n, d = M.shape[0], M.shape[1]
    L = np.empty((n, d, d))
    cL = np.empty(n)
    acc, ca = np.eye(d), 1.0
    for i in range(n):
        L[i], cL[i] = acc, ca
        acc = acc @ M[i]
        ca *= np.linalg.norm(M[i], 2)
    Mb = np.empty_like(M)
    c = np.empty(n)
    acc, ca = np.eye(d), 1.0
    yn = np.linalg.norm(Yb, 2)
    for i in range(n - 1, -1, -1):
        Mb[i] = L[i].T @ Yb @ acc.T
        c[i] = cL[i] * yn * ca
        acc = M[i] @ acc
        ca *= np.linalg.norm(M[i], 2)
    return Mb, c


# -------------------------------------------------------------------------
# int32 forward combinators for + * min max, results wrapping mod 2^32 (the
# evaluation's integer element types; forward only, as integer arithmetic
# has no derivative).  Plain loops over Python integers, reduced mod 2^32 and
# read back in two's complement after every step: exact by construction.
# -------------------------------------------------------------------------
_I32_NEUTRAL = {"add": 0, "mul": 1, "min": 2**31 - 1, "max": -2**31}


def _wrap32(x: int) -> int:
    x &= 0xFFFFFFFF
    return x - (1 << 32) if x >= (1 << 31) else x


def _i32_comb(op: str, a: int, b: int) -> int:
    if op == "add":
        return _wrap32(a + b)
    if op == "mul":
        return _wrap32(a * b)
    if op == "min":
        return a if a <= b else b
    if op == "max":
        return a if a >= b else b
    raise ValueError(op)


def i32_reduce(op: str, x) -> int:
    """Left fold of x (int32) from the neutral element."""
    acc = _I32_NEUTRAL[op]
    for v in np.asarray(x, dtype=np.int64).reshape(-1).tolist():
        acc = _i32_comb(op, acc, v)
    return acc


def i32_scan(op: str, x) -> np.ndarray:
    """Inclusive scan of x (int32)."""
    out = np.empty(len(x), dtype=np.int32)
    acc = _I32_NEUTRAL[op]
    for i, v in enumerate(np.asarray(x, dtype=np.int64).reshape(-1).tolist()):
        acc = _i32_comb(op, acc, v)
        out[i] = acc
    return out


def i32_rbi(op: str, idx, m: int, v) -> np.ndarray:
    """hist[k] = fold of v[i] over idx[i] == k from the neutral element; keys
    outside [0, m) are skipped (Section 4's sequential loop)."""
    h = [_I32_NEUTRAL[op]] * max(int(m), 0)
    for k, x in zip(np.asarray(idx).reshape(-1).tolist(), np.asarray(v, dtype=np.int64).reshape(-1).tolist()):
        if 0 <= k < m:
            h[k] = _i32_comb(op, h[k], x)
    return np.array(h, dtype=np.int32)
