"""Seeded synthetic inputs for the reduce / scan / reduce-by-index workloads.

This module only draws data.  It holds none of the arithmetic of the method
(no combine, no adjoint), so both the CPU oracle and the HIP path may take
their inputs from here without sharing any computation.

The paper evaluates on "randomly generated arrays" of FP32 values (Section 5.1,
Datasets; no distributions stated).  The five workloads below fix those
distributions; every array is drawn in float64 with numpy's PCG64 and rounded
once to float32 (indices are int32).  Sub-streams come from
``SeedSequence.spawn`` in the order the arrays are listed in each function, so
a workload is fully determined by its seed.

Workload names and default sizes:

* ``small``      -- n=100000, x ~ U[0.5,2), 1% exact zeros for ``*``, m=1024 bins.
* ``linrec``     -- linear-recurrence pairs (a ~ U[0.9,1), b ~ N(0,1)), n=2^26.
* ``mat2``       -- 2x2 matrices with entries ~ N(0, variance 0.5), n=2^24,
                    plus a norm-preserving O(2) companion ensemble.
* ``rbi``        -- n=2^26 values ~ N(0,1), uniform or Zipf(1.1) keys over m bins.
* ``segmented``  -- 4096 instances with lognormal lengths (median 4096).
* ``autograd``   -- 64 sequences of length 2^16 with a 65536-bin histogram.

Parity ensembles (inputs on which every output stays inside the float32
range, so a comparison with the oracle constrains every element):

* ``mul_finite``     -- multipliers +-exp(U[-0.01, 0.01]), optional exact
                        zeros past a given position.
* ``mat2(ensemble="o2")`` -- random orthogonal 2x2 factors.
* ``segmented_ties`` -- the segmented workload with a in {0, 1} and small integer
                        offsets, so that equal minima are common.
"""
from __future__ import annotations

import math

import numpy as np

BASE_SEED = 231003568


def _streams(seed: int, k: int):
    ss = np.random.SeedSequence(seed)
    return [np.random.Generator(np.random.PCG64(s)) for s in ss.spawn(k)]


def f32(a) -> np.ndarray:
    return np.ascontiguousarray(np.asarray(a, dtype=np.float64).astype(np.float32))


def exact_zero_positions(rng, n: int, count: int) -> np.ndarray:
    """``count`` distinct positions in [0, n), drawn without replacement."""
    count = min(int(count), n)
    if count <= 0:
        return np.zeros(0, dtype=np.int64)
    return np.sort(rng.choice(n, size=count, replace=False))


def zipf_keys(rng, n: int, m: int, s: float = 1.1) -> np.ndarray:
    """Keys with P(bin = r-1) proportional to r^-s for r in 1..m.

    Hot bins are the low indices (no permutation).  Sampled by inverse CDF
    from the generator's uniform stream.
    """
    w = np.arange(1, m + 1, dtype=np.float64) ** (-s)
    cdf = np.cumsum(w)
    cdf /= cdf[-1]
    u = rng.random(n)
    k = np.searchsorted(cdf, u, side="right")
    return np.minimum(k, m - 1).astype(np.int32)


def round_to_grid(v: np.ndarray, step_log2: int = -8) -> np.ndarray:
    """Round float64 values to multiples of 2^step_log2 (half to even)."""
    scale = 2.0 ** (-step_log2)
    return np.rint(v * scale) / scale


def o2_matrices(rng, n: int) -> np.ndarray:
    """n random orthogonal 2x2 matrices, row-major (n, 4), float32.

    A rotation by theta ~ U[0, 2pi), composed with the reflection
    diag(1, -1) with probability 1/2.  Products of such matrices keep unit
    spectral norm, so long chains neither overflow nor underflow.
    """
    th = rng.random(n) * (2.0 * math.pi)
    refl = rng.random(n) < 0.5
    c, s = np.cos(th), np.sin(th)
    m = np.empty((n, 4), dtype=np.float64)
    m[:, 0] = c
    m[:, 1] = -s
    m[:, 2] = s
    m[:, 3] = c
    # right-multiplying by diag(1,-1) negates the second column
    m[refl, 1] *= -1.0
    m[refl, 3] *= -1.0
    return f32(m)


# --------------------------------------------------------------------------
# workload: small (all four scalar operators, all three combinators)
# --------------------------------------------------------------------------
def small(n: int = 100_000, m: int = 1024, seed: int = BASE_SEED + 1, zero_frac: float = 0.01):
    """x ~ U[0.5, 2); x_mul = x with floor(zero_frac*n) exact zeros;
    keys ~ U{0..m-1}; adjoints ~ N(0,1) for a reduce (1), a scan (n) and a
    histogram (m)."""
    r = _streams(seed, 6)
    x = r[0].uniform(0.5, 2.0, n)
    zpos = exact_zero_positions(r[1], n, math.floor(zero_frac * n))
    x_mul = x.copy()
    x_mul[zpos] = 0.0
    idx = r[2].integers(0, m, n, dtype=np.int64).astype(np.int32) if m > 0 else np.zeros(n, np.int32)
    return dict(
        x=f32(x), x_mul=f32(x_mul), idx=idx, m=m,
        ybar_reduce=f32(r[3].standard_normal(1)),
        ybar_scan=f32(r[4].standard_normal(n)),
        ybar_rbi=f32(r[5].standard_normal(max(m, 0))),
    )


# --------------------------------------------------------------------------
# workload: large linear-recurrence scan
# --------------------------------------------------------------------------
def linrec(n: int = 1 << 26, seed: int = BASE_SEED + 2, with_abar: bool = False):
    """y_i = a_i*y_{i-1} + b_i with a ~ U[0.9, 1), b ~ N(0,1); adjoint of y
    ~ N(0,1); adjoint of the cumulative product A is zero unless
    ``with_abar``, in which case it is ~ N(0,1) as well."""
    r = _streams(seed, 4)
    out = dict(
        a=f32(r[0].uniform(0.9, 1.0, n)),
        b=f32(r[1].standard_normal(n)),
        ybar=f32(r[2].standard_normal(n)),
    )
    out["Abar"] = f32(r[3].standard_normal(n)) if with_abar else None
    return out


def mat2(n: int = 1 << 24, seed: int = BASE_SEED + 2, ensemble: str = "gauss"):
    """2x2 matrices row-major (n,4).  ``gauss``: entries ~ N(0, variance
    0.5).  ``o2``: random orthogonal matrices.  Output adjoint entries
    ~ N(0,1)."""
    r = _streams(seed + 1000, 3)
    if ensemble == "gauss":
        M = f32(r[0].standard_normal((n, 4)) * math.sqrt(0.5))
    elif ensemble == "o2":
        M = o2_matrices(r[0], n)
    else:
        raise ValueError(ensemble)
    return dict(M=M, Pbar=f32(r[1].standard_normal((n, 4))))


def mul_finite(shape, seed: int = BASE_SEED + 7, zeros_after: int = -1, n_zeros: int = 0):
    """Multipliers x = sign * exp(v) with sign = +-1 equally likely and
    v ~ U[-0.01, 0.01]: log |product| is a driftless random walk with a
    standard deviation of 5.8e-3 per factor, so prefix products stay finite
    and non-zero over 2^24 and more elements (|log| below about 25 there).
    Factors much closer to 1 (spread 1e-3) would make float32 products in
    a tree order drop their second-order terms systematically, an error
    that grows linearly with the chain instead of as its square root.
    With ``n_zeros`` > 0, that many exact zeros at distinct positions >=
    ``zeros_after`` along the last axis.  Output adjoint y_bar ~ N(0,1) of
    the same shape."""
    r = _streams(seed, 4)
    shape = tuple(shape) if isinstance(shape, (tuple, list)) else (int(shape),)
    x = r[0].choice([-1.0, 1.0], shape) * np.exp(r[1].uniform(-0.01, 0.01, shape))
    if n_zeros > 0:
        n = shape[-1]
        lo = max(int(zeros_after), 0)
        flat = x.reshape(-1, n)
        for row in flat:
            row[lo + exact_zero_positions(r[2], n - lo, n_zeros)] = 0.0
    return dict(x=f32(x), ybar=f32(r[3].standard_normal(shape)))


# --------------------------------------------------------------------------
# workload: large reduce-by-index
# --------------------------------------------------------------------------
def rbi(op: str, n: int = 1 << 26, m: int = 1 << 22, dist: str = "uniform",
        seed: int = BASE_SEED + 3, zero_frac: float = 0.001):
    """Values ~ N(0,1) (4 entries per element for ``mat2``); keys uniform or
    Zipf(1.1) over m bins.  ``mul``: floor(zero_frac*n) exact zeros.
    ``min``/``max``: values rounded to multiples of 2^-8 so ties occur.
    ``mat2o2``: orthogonal matrices.  Histogram adjoint ~ N(0,1) per bin."""
    r = _streams(seed, 4)
    if op in ("mat2", "mat2o2"):
        v = r[0].standard_normal((n, 4)) if op == "mat2" else None
        v = f32(v) if v is not None else o2_matrices(r[0], n)
    else:
        v = r[0].standard_normal(n)
        if op == "mul":
            zpos = exact_zero_positions(r[1], n, math.floor(zero_frac * n))
            v[zpos] = 0.0
        if op in ("min", "max"):
            v = round_to_grid(v, -8)
        v = f32(v)
    if dist == "uniform":
        idx = r[2].integers(0, m, n, dtype=np.int64).astype(np.int32)
    elif dist == "zipf":
        idx = zipf_keys(r[2], n, m)
    else:
        raise ValueError(dist)
    d = 4 if op in ("mat2", "mat2o2") else 1
    hbar = f32(r[3].standard_normal(m * d).reshape((m, d) if d > 1 else (m,)))
    return dict(v=v, idx=idx, m=m, hbar=hbar)


# --------------------------------------------------------------------------
# workload: batched segmented instances
# --------------------------------------------------------------------------
def segment_lengths(rng, S: int, median: int = 4096, cap: int = 1 << 20) -> np.ndarray:
    """clamp(rint(LogNormal(ln median, sigma)), 1, cap) with
    sigma = sqrt(2 ln 4), so that the mean length is 4x the median."""
    sigma = math.sqrt(2.0 * math.log(4.0))
    L = np.rint(rng.lognormal(math.log(median), sigma, S))
    return np.clip(L, 1, cap).astype(np.int64)


def segmented(S: int = 4096, m: int = 512, seed: int = BASE_SEED + 4,
              median: int = 4096, cap: int = 1 << 20):
    """S instances; per instance a linear recurrence (a ~ U[0.9,1),
    b ~ N(0,1)) whose outputs feed a min-by-index into m bins with keys
    ~ U{0..m-1}.  Adjoints: y ~ N(0,1) per element, h ~ N(0,1) per
    (instance, bin).  Returns concatenated arrays and int64 offsets[S+1]."""
    r = _streams(seed, 6)
    L = segment_lengths(r[0], S, median, cap)
    off = np.zeros(S + 1, dtype=np.int64)
    np.cumsum(L, out=off[1:])
    N = int(off[-1])
    return dict(
        offsets=off, lengths=L, m=m, n_total=N,
        a=f32(r[1].uniform(0.9, 1.0, N)),
        b=f32(r[2].standard_normal(N)),
        idx=r[3].integers(0, m, N, dtype=np.int64).astype(np.int32),
        ybar=f32(r[4].standard_normal(N)),
        hbar=f32(r[5].standard_normal(S * m)),
    )


def segmented_ties(S: int = 64, m: int = 16, seed: int = BASE_SEED + 8, median: int = 700,
                   cap: int = 30_000):
    """Like ``segmented`` but with multipliers a in {0, 1} (each 0 with
    probability 1/2, which restarts the recurrence at y_i = b_i) and small
    integer offsets b ~ U{-1, 0, 1}: every y is an exact float32 integer of
    small magnitude, so equal minima occur in about half of the bins with
    several elements and the lowest-index rule decides them."""
    r = _streams(seed, 6)
    L = segment_lengths(r[0], S, median, cap)
    off = np.zeros(S + 1, dtype=np.int64)
    np.cumsum(L, out=off[1:])
    N = int(off[-1])
    return dict(
        offsets=off, lengths=L, m=m, n_total=N,
        a=(r[5].random(N) >= 0.5).astype(np.float32),
        b=f32(r[1].integers(-1, 2, N)),
        idx=r[2].integers(0, m, N, dtype=np.int64).astype(np.int32),
        ybar=f32(r[3].standard_normal(N)),
        hbar=f32(r[4].standard_normal(S * m)),
    )


# --------------------------------------------------------------------------
# workload: autograd end-to-end
# --------------------------------------------------------------------------
def autograd(B: int = 64, T: int = 1 << 16, m: int = 65536, seed: int = BASE_SEED + 5):
    """B sequences of length T: a ~ U[0.9,1), b ~ N(0,1), v ~ N(0,1),
    keys ~ U{0..m-1}; shapes (B, T)."""
    r = _streams(seed, 4)
    return dict(
        a=f32(r[0].uniform(0.9, 1.0, (B, T))),
        b=f32(r[1].standard_normal((B, T))),
        v=f32(r[2].standard_normal((B, T))),
        idx=r[3].integers(0, m, (B, T), dtype=np.int64).astype(np.int32),
        m=m,
    )


# --------------------------------------------------------------------------
# workload: d x d matrix-product scans (3x3, 5x5)
# --------------------------------------------------------------------------
def orthogonal_matrices(rng, n: int, d: int) -> np.ndarray:
    """n Haar-random orthogonal d x d matrices (n, d, d), float32: the Q of
    a QR factorisation of a Gaussian matrix, columns signed so that R has a
    positive diagonal."""
    G = rng.standard_normal((n, d, d))
    Q, R = np.linalg.qr(G)
    sgn = np.sign(np.diagonal(R, axis1=1, axis2=2))
    sgn[sgn == 0] = 1.0
    return f32(Q * sgn[:, None, :])


def matd(d: int, n: int, batch: int = 1, seed: int = BASE_SEED + 6, ensemble: str = "orth"):
    """M (batch, n, d, d) and an output adjoint Pbar ~ N(0, 1) of the same
    shape.  ``orth``: Haar-orthogonal factors (products keep unit spectral
    norm); ``near``: orthogonal factors times (1 + 0.01 N(0, 1)) entrywise
    perturbations, so that the products drift slowly in norm."""
    r = _streams(seed + 100 * d, 3)
    M = orthogonal_matrices(r[0], batch * n, d).astype(np.float64)
    if ensemble == "near":
        M = M * (1.0 + 0.01 * r[2].standard_normal(M.shape))
    elif ensemble != "orth":
        raise ValueError(ensemble)
    return dict(M=f32(M).reshape(batch, n, d, d),
                Pbar=f32(r[1].standard_normal((batch, n, d, d))))
