// reduce (Section 3) and its adjoint.
//
// + * min max and sumOfProd: a lifted grid reduction.  Each block folds a contiguous chunk
// of a row into one lifted partial -- the sum; (zero count, product of the
// non-zeros) for * (Section 3.2 Multiplication); (value, lowest index) for
// min/max (Section 3.2 Min/Max); (p, s) for sumOfProd (Section 3.3) --
// and a second, stream-ordered launch
// folds each row's partials.  The
// adjoints are single elementwise passes (broadcast, the three zero cases,
// the one-hot at k).
//
// linear recurrence / 2x2 matrix product / saturated addition: the general
// rule of Section 3.1
// (reduce rule figure).  The forward is the look-back scan kernel run without
// per-element outputs; it saves every tile's exclusive prefix l_t.  The
// adjoint takes tiles right to left, recomputes in registers the in-tile
// exclusive prefix and suffix of every element, gets the tile's exclusive
// suffix r_t by a right-to-left look-back over tile aggregates, and applies
// x_bar_i = d(l_i (.) x_i (.) r_i)/dx_i^T y_bar (Eq. 2).  No l/r arrays are
// materialised: 2 reads + 1 write per element instead of the rule's ~8.
#include "adjoint.hpp"
#include "internal.hpp"

namespace pcad {

// ---------------------------------------------------------------------------
// lifted values for + * min max: f = value, u = count (mul) or index (min/max)
// ---------------------------------------------------------------------------
struct LV {
  float f;
  uint32_t u;
};

template <int OP>
struct Lift;

template <>
struct Lift<ADD> {
  __device__ static LV id() { return {0.0f, 0u}; }
  __device__ static LV elem(float x, uint32_t) { return {x, 0u}; }
  __device__ static LV comb(const LV &a, const LV &b) { return {a.f + b.f, 0u}; }
};

template <>
struct Lift<MUL> {
  __device__ static LV id() { return {1.0f, 0u}; }
  __device__ static LV elem(float x, uint32_t) { return x == 0.0f ? LV{1.0f, 1u} : LV{x, 0u}; }
  __device__ static LV comb(const LV &a, const LV &b) { return {a.f * b.f, a.u + b.u}; }
};

template <>
struct Lift<MIN> {
  __device__ static LV id() { return {__builtin_inff(), 0xffffffffu}; }
  __device__ static LV elem(float x, uint32_t i) { return {x, i}; }
  __device__ static LV comb(const LV &a, const LV &b) {
    return (b.f < a.f || (b.f == a.f && b.u < a.u)) ? b : a;
  }
};

template <>
struct Lift<MAX> {
  __device__ static LV id() { return {-__builtin_inff(), 0xffffffffu}; }
  __device__ static LV elem(float x, uint32_t i) { return {x, i}; }
  __device__ static LV comb(const LV &a, const LV &b) {
    return (b.f > a.f || (b.f == a.f && b.u < a.u)) ? b : a;
  }
};

// sumOfProd (Section 3.3): f = p, u = the bits of s
template <>
struct Lift<SUMPROD> {
  __device__ static LV id() { return {0.0f, 0u}; }
  __device__ static LV elem(float x, uint32_t) { return {0.0f, __float_as_uint(x)}; }
  __device__ static LV comb(const LV &a, const LV &b) {
    const SP r = sp_comb(SP{a.f, __uint_as_float(a.u)}, SP{b.f, __uint_as_float(b.u)});
    return {r.p, __float_as_uint(r.s)};
  }
};

__device__ __forceinline__ LV shfl_down_lv(const LV &v, int d) {
  LV r;
  r.f = __shfl_down(v.f, d, WAVE);
  r.u = (uint32_t)__shfl_down((int)v.u, d, WAVE);
  return r;
}

// block-wide reduction of a commutative lifted value; result valid in thread 0
template <int OP>
__device__ LV block_reduce_lv(LV v, LV *s_w) {
  const int lane = lane_id(), wave = threadIdx.x / WAVE;
#pragma unroll
  for (int d = WAVE / 2; d > 0; d >>= 1) v = Lift<OP>::comb(v, shfl_down_lv(v, d));
  if (lane == 0) s_w[wave] = v;
  __syncthreads();
  if (threadIdx.x == 0) {
    v = s_w[0];
    for (int w = 1; w < WAVES; ++w) v = Lift<OP>::comb(v, s_w[w]);
  }
  __syncthreads();
  return v;
}

struct RedArgs {
  const float *x;
  float *y;
  void *saved;
  int64_t n;
  int64_t chunk;  // elements per block (multiple of 4)
  int bpr;        // blocks per row
  LV *parts;      // [batch][bpr] lifted partials
};

// pass 1: every block folds its chunk of a row into one lifted partial
template <int OP>
__global__ __launch_bounds__(BLOCK) void k_reduce_part(RedArgs a) {
  __shared__ LV s_w[WAVES];
  const int tid = threadIdx.x;
  const int64_t row = blockIdx.y;
  const int b = blockIdx.x;
  const float *xr = a.x + row * a.n;
  const int64_t lo = (int64_t)b * a.chunk;
  const int64_t hi = lo + a.chunk < a.n ? lo + a.chunk : a.n;
  const bool vec_ok = ((row * a.n) & 3) == 0;
  LV acc = Lift<OP>::id();
  for (int64_t i = lo + (int64_t)tid * 4; i < hi; i += (int64_t)BLOCK * 4) {
    if (vec_ok && i + 4 <= hi) {
      const float4 v = ld_stream<float4>(xr + i);
      acc = Lift<OP>::comb(acc, Lift<OP>::elem(v.x, (uint32_t)i));
      acc = Lift<OP>::comb(acc, Lift<OP>::elem(v.y, (uint32_t)(i + 1)));
      acc = Lift<OP>::comb(acc, Lift<OP>::elem(v.z, (uint32_t)(i + 2)));
      acc = Lift<OP>::comb(acc, Lift<OP>::elem(v.w, (uint32_t)(i + 3)));
    } else {
#pragma unroll
      for (int j = 0; j < 4; ++j)
        if (i + j < hi) acc = Lift<OP>::comb(acc, Lift<OP>::elem(xr[i + j], (uint32_t)(i + j)));
    }
  }
  acc = block_reduce_lv<OP>(acc, s_w);
  if (tid == 0) a.parts[row * a.bpr + b] = acc;
}

// pass 2 (stream-ordered after pass 1): one block per row folds the partials
template <int OP>
__global__ __launch_bounds__(BLOCK) void k_reduce_fold(RedArgs a) {
  __shared__ LV s_w[WAVES];
  const int64_t row = blockIdx.x;
  LV r = Lift<OP>::id();
  for (int p = threadIdx.x; p < a.bpr; p += BLOCK) {
    r = Lift<OP>::comb(r, a.parts[row * a.bpr + p]);
    a.parts[row * a.bpr + p] = LV{};  // leave the workspace holding no data between calls
  }
  r = block_reduce_lv<OP>(r, s_w);
  if (threadIdx.x == 0) {
    if (OP == ADD) {
      a.y[row] = r.f;
    } else if (OP == SUMPROD) {
      a.y[row] = r.f;
      reinterpret_cast<float *>(a.saved)[row] = __uint_as_float(r.u);  // s = sum of the row
    } else if (OP == MUL) {
      a.y[row] = r.u > 0 ? 0.0f : r.f;
      uint32_t *sv = reinterpret_cast<uint32_t *>(a.saved) + row * 2;
      sv[0] = r.u;
      reinterpret_cast<float *>(sv)[1] = r.f;
    } else {
      a.y[row] = r.f;
      reinterpret_cast<int32_t *>(a.saved)[row] = (int32_t)r.u;
    }
  }
}

// neutral results for rows of length 0
__global__ void k_reduce_empty(int op, int64_t batch, int d, float *y, void *saved) {
  const int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (r >= batch) return;
  switch (op) {
  case ADD: y[r] = 0.0f; break;
  case MUL:
    y[r] = 1.0f;
    reinterpret_cast<uint32_t *>(saved)[2 * r] = 0u;
    reinterpret_cast<float *>(saved)[2 * r + 1] = 1.0f;
    break;
  case MIN:
  case MAX:
    y[r] = op == MIN ? __builtin_inff() : -__builtin_inff();
    reinterpret_cast<int32_t *>(saved)[r] = 0;  // sentinel n = 0
    break;
  case LINREC:
    y[2 * r] = 1.0f;
    y[2 * r + 1] = 0.0f;
    break;
  case MAT2:
    y[4 * r] = 1.0f; y[4 * r + 1] = 0.0f; y[4 * r + 2] = 0.0f; y[4 * r + 3] = 1.0f;
    break;
  case SUMPROD:
    y[r] = 0.0f;
    reinterpret_cast<float *>(saved)[r] = 0.0f;
    break;
  case SATADD: y[r] = 0.0f; break;
  }
  (void)d;
}

// adjoint of + * min max: one elementwise pass per row
template <int OP>
__global__ __launch_bounds__(BLOCK) void k_reduce_vjp(const float *x, const void *saved,
                                                      const float *ybar, float *xb, int64_t n,
                                                      int accumulate) {
  const int64_t row = blockIdx.y;
  const float yb = ybar[row];
  uint32_t n0 = 0;
  float ypos = 0.0f;
  int64_t k = -1;
  if (OP == MUL) {
    n0 = reinterpret_cast<const uint32_t *>(saved)[2 * row];
    ypos = reinterpret_cast<const float *>(saved)[2 * row + 1];
  }
  if (OP == MIN || OP == MAX) k = reinterpret_cast<const int32_t *>(saved)[row];
  // sumOfProd: d p / d x_i = s - x_i (the invertible-operator rule of
  // Section 3.3: the rest of the fold is s - x_i)
  const float ssum = OP == SUMPROD ? reinterpret_cast<const float *>(saved)[row] : 0.0f;
  const float *xr = x + row * n;
  float *xbr = xb + row * n;
  const bool vec_ok = ((row * n) & 3) == 0;
  const int64_t stride = (int64_t)gridDim.x * BLOCK * 4;
  for (int64_t i = ((int64_t)blockIdx.x * BLOCK + threadIdx.x) * 4; i < n; i += stride) {
    float v[4], o[4];
    const bool full = vec_ok && i + 4 <= n;
    if (OP == MUL || OP == SUMPROD) {
      if (full) {
        const float4 t = ld_stream<float4>(xr + i);
        v[0] = t.x; v[1] = t.y; v[2] = t.z; v[3] = t.w;
      } else {
        for (int j = 0; j < 4; ++j) v[j] = (i + j < n) ? xr[i + j] : 1.0f;
      }
    }
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      if (OP == ADD) o[j] = yb;
      if (OP == MUL)
        o[j] = n0 == 0 ? (ypos / v[j]) * yb : ((n0 == 1 && v[j] == 0.0f) ? ypos * yb : 0.0f);
      if (OP == MIN || OP == MAX) o[j] = (i + j == k) ? yb : 0.0f;
      if (OP == SUMPROD) o[j] = (ssum - v[j]) * yb;
    }
    if (accumulate) {
      for (int j = 0; j < 4; ++j)
        if (i + j < n) o[j] += xbr[i + j];
    }
    if (full) {
      *reinterpret_cast<float4 *>(xbr + i) = make_float4(o[0], o[1], o[2], o[3]);
    } else {
      for (int j = 0; j < 4; ++j)
        if (i + j < n) xbr[i + j] = o[j];
    }
  }
}

// ---------------------------------------------------------------------------
// general rule for the linear recurrence and the 2x2 matrix product
// ---------------------------------------------------------------------------
// the forward operator run right to left: comb(earlier = right, later = left)
template <int OP>
struct RevLB {
  using T = typename Fwd<OP>::T;
  using P = T;
  static constexpr int NA = Fwd<OP>::N, NP = Fwd<OP>::N;
  __device__ static T id() { return Fwd<OP>::id(); }
  __device__ static T comb(const T &e, const T &l) { return Fwd<OP>::comb(l, e); }
  __device__ static T from_pre(const P &p) { return p; }
};

// x_bar of one element from l (everything before), x and r (everything after)
template <int OP>
struct LocalVjp;

template <>
struct LocalVjp<LINREC> {
  using T = Fwd<LINREC>::T;
  // out = l x r: (lA a rA, rA (a lB + b) + rB); ybar = (ybar_A, ybar_B)
  __device__ static void apply(const T &l, const T &x, const T &r, const float *yb, float *xb) {
    const float ra = r.f[0];
    xb[0] = ra * __builtin_fmaf(yb[0], l.f[0], yb[1] * l.f[1]);  // a_bar
    xb[1] = yb[1] * ra;                                          // b_bar
    (void)x;
  }
};

template <>
struct LocalVjp<MAT2> {
  using T = Fwd<MAT2>::T;
  // Y = L X R  ->  X_bar = L^T Y_bar R^T
  __device__ static void apply(const T &l, const T &x, const T &r, const float *yb, float *xb) {
    float lt[4] = {l.f[0], l.f[2], l.f[1], l.f[3]};
    float rt[4] = {r.f[0], r.f[2], r.f[1], r.f[3]};
    float t[4];
    MapMat::mm(lt, yb, t);
    MapMat::mm(t, rt, xb);
    (void)x;
  }
};

template <>
struct LocalVjp<SATADD> {
  using T = Fwd<SATADD>::T;
  // out = (l (.) x) (.) r: the two steps' partials in x, each 0 if saturated
  __device__ static void apply(const T &l, const T &x, const T &r, const float *yb, float *xb) {
    const float lx = l.f[0] + x.f[0];
    const float lxs = lx > kSatCap ? kSatCap : lx;
    const bool pass = !(lx > kSatCap) && !(lxs + r.f[0] > kSatCap);
    xb[0] = pass ? yb[0] : 0.0f;
    xb[1] = 0.0f;
  }
};

struct RedGenArgs {
  const float *x0, *x1;
  const float *saved;  // exclusive prefix per tile (forward)
  const float *ybar;   // N floats per row
  float *xb0, *xb1;
  int64_t n;
  int tpr;
  int accumulate;
  Ctl *ctl;
  uint64_t *status;
};

template <int OP>
__global__ __launch_bounds__(Shape<OP>::THREADS) void k_reduce_vjp_gen(RedGenArgs a) {
  using F = FwdLB<OP>;
  using R = RevLB<OP>;
  using T = typename F::T;
  using Io = IO<OP>;
  constexpr int EPL = Shape<OP>::EPL, K = Shape<OP>::K, TILE = Shape<OP>::TILE;
  constexpr int TH = Shape<OP>::THREADS, W = Shape<OP>::W;
  constexpr int NIN = Io::NIN, S = Io::S, N = Fwd<OP>::N;

  __shared__ T s_ftot[K][W];
  __shared__ T s_fpre[K][W];
  __shared__ T s_rtot[K][W];
  __shared__ T s_rpre[K][W];
  __shared__ T s_carry;
  __shared__ unsigned s_epoch;

  const int tid = threadIdx.x, lane = lane_id(), wave = tid / WAVE;
  if (tid == 0) s_epoch = ctl_load(&a.ctl->epoch);
  // descending tile order: dispatch order runs right to left
  const TileInfo ti = tile_info(gridDim.x - 1 - blockIdx.x, a.n, a.tpr, TILE);

  T xe[K][EPL];
#pragma unroll
  for (int g = 0; g < K; ++g) {
    const int el = g * TH * EPL + tid * EPL;
    const int v = ti.valid - el;
    const float *src[2] = {a.x0, a.x1};
    float4 in[NIN];
#pragma unroll
    for (int s = 0; s < NIN; ++s)
      in[s] = load_group<S>(src[s], ti.base, el, v, ti.vec_ok, Io::fill(s));
#pragma unroll
    for (int j = 0; j < EPL; ++j) xe[g][j] = Io::elem(in, j);
  }

  // in-thread inclusive prefixes and exclusive suffixes, then wave scans
  T locp[K][EPL], sufx[K][EPL];
  T inf_[K], inr_[K];
#pragma unroll
  for (int g = 0; g < K; ++g) {
    T acc = xe[g][0];
    locp[g][0] = acc;
#pragma unroll
    for (int j = 1; j < EPL; ++j) {
      acc = F::comb(acc, xe[g][j]);
      locp[g][j] = acc;
    }
    T sacc = F::id();
#pragma unroll
    for (int j = EPL - 1; j >= 0; --j) {
      sufx[g][j] = sacc;
      sacc = F::comb(xe[g][j], sacc);
    }
    inf_[g] = wave_scan_fwd<F>(acc);
    inr_[g] = wave_scan_rev<R>(sacc);
    if (lane == WAVE - 1) s_ftot[g][wave] = inf_[g];
    if (lane == 0) s_rtot[g][wave] = inr_[g];
  }
  __syncthreads();
  const uint32_t tag = next_tag(s_epoch);

  if (wave == 0) {
    // forward side: l = saved tile prefix (.) in-tile exclusive prefix
    T lcar;
#pragma unroll
    for (int i = 0; i < N; ++i) lcar.f[i] = a.saved[ti.tile * N + i];
    wave0_block_prefix<F, K, W, false>(s_ftot, s_fpre, lcar);
    // reverse side: in-tile suffixes, the tile total, and a right-to-left
    // look-back over tile totals for the tile's exclusive suffix
    const T tile_agg = wave0_block_prefix<R, K, W, true>(s_rtot, s_rpre, R::id());
    uint64_t *st = a.status + ti.tile * (R::NA + R::NP);
    const int dist_max = a.tpr - 1 - ti.lt;
    T c = R::id();
    if (dist_max == 0) {
      if (lane == 0) publish<N>(st + R::NA, tag, tile_agg);
    } else {
      if (lane == 0) publish<N>(st, tag, tile_agg);
      c = lookback<R>(a.status, ti.tile, -1, dist_max, tag, a.ctl);
      if (lane == 0) publish<N>(st + R::NA, tag, R::comb(c, tile_agg));
    }
    if (lane == 0) {
      s_carry = c;
      if (ti.lt == 0) ctl_row_done(a.ctl, gridDim.x / a.tpr, tag);
    }
  }
  __syncthreads();
  const T carry = s_carry;

  float yb[4];
#pragma unroll
  for (int i = 0; i < N; ++i) yb[i] = a.ybar[ti.row * N + i];

#pragma unroll
  for (int g = 0; g < K; ++g) {
    T exf = shift_up1(inf_[g]);
    if (lane == 0) exf = F::id();
    T exr = shift_down1(inr_[g]);
    if (lane == WAVE - 1) exr = R::id();
    const T lth = F::comb(s_fpre[g][wave], exf);                 // everything before this thread
    const T rth = R::comb(R::comb(carry, s_rpre[g][wave]), exr);  // everything after this thread
    float4 o[2];
    o[0] = make_float4(0, 0, 0, 0);
    o[1] = make_float4(0, 0, 0, 0);
#pragma unroll
    for (int j = 0; j < EPL; ++j) {
      const T l = j == 0 ? lth : F::comb(lth, locp[g][j - 1]);
      const T r = F::comb(sufx[g][j], rth);
      float xb[4];
      LocalVjp<OP>::apply(l, xe[g][j], r, yb, xb);
      if (S == 4) {
        o[0] = make_float4(xb[0], xb[1], xb[2], xb[3]);
      } else {
        f4set(o[0], j, xb[0]);
        f4set(o[1], j, xb[1]);
      }
    }
    const int el = g * TH * EPL + tid * EPL;
    const int v = ti.valid - el;
    float *dst[2] = {a.xb0, a.xb1};
    constexpr int NS = (OP == LINREC) ? 2 : 1;
#pragma unroll
    for (int s = 0; s < NS; ++s) {
      float4 val = o[s];
      if (a.accumulate) {
        const float4 old = load_group<S>(dst[s], ti.base, el, v, ti.vec_ok, make_float4(0, 0, 0, 0));
        val.x += old.x; val.y += old.y; val.z += old.z; val.w += old.w;
      }
      store_group<S>(dst[s], ti.base, el, v, ti.vec_ok, val);
    }
  }
}

// ---------------------------------------------------------------------------
// host side
// ---------------------------------------------------------------------------
int reduce_blocks_per_row(int64_t batch, int64_t n) {
  int64_t bpr = (n + 16383) / 16384;
  int64_t cap = 4096 / (batch > 0 ? batch : 1);
  if (cap < 1) cap = 1;
  if (bpr > cap) bpr = cap;
  if (bpr < 1) bpr = 1;
  return (int)bpr;
}

size_t reduce_ws_bytes(int op, int64_t batch, int64_t n) {
  if (op == LINREC || op == MAT2 || op == SATADD) {
    const int tile = scan_tile_size(op);
    const int64_t tiles = batch * ((n + tile - 1) / tile);
    return kCtlBytes + (size_t)tiles * 2 * scan_elem_floats(op) * sizeof(uint64_t);
  }
  const int bpr = reduce_blocks_per_row(batch, n);
  return kCtlBytes + (size_t)batch * bpr * sizeof(LV);
}

hipError_t reduce_fwd_launch(int op, int64_t batch, int64_t n, const float *x0, const float *x1,
                             float *y, void *saved, void *ws, hipStream_t s) {
  if (batch == 0) return hipSuccess;
  if (n == 0) {
    hipLaunchKernelGGL(k_reduce_empty, dim3((unsigned)((batch + 255) / 256)), dim3(256), 0, s,
                       op, batch, scan_elem_floats(op), y, saved);
    return hipGetLastError();
  }
  if (op == LINREC || op == MAT2 || op == SATADD)
    return scan_fwd_launch(op, batch, n, x0, x1, nullptr, nullptr, static_cast<float *>(saved), y,
                           true, ws, s);
  RedArgs a;
  a.x = x0; a.y = y; a.saved = saved; a.n = n;
  a.bpr = reduce_blocks_per_row(batch, n);
  a.chunk = ((n + a.bpr - 1) / a.bpr + 3) / 4 * 4;
  a.parts = reinterpret_cast<LV *>(static_cast<char *>(ws) + kCtlBytes);
  const dim3 grid((unsigned)a.bpr, (unsigned)batch);
  const dim3 fold((unsigned)batch);
#define PCAD_RED(OPV)                                                          \
  case OPV:                                                                    \
    hipLaunchKernelGGL(k_reduce_part<OPV>, grid, dim3(BLOCK), 0, s, a);        \
    hipLaunchKernelGGL(k_reduce_fold<OPV>, fold, dim3(BLOCK), 0, s, a);        \
    break;
  switch (op) {
    PCAD_RED(ADD)
    PCAD_RED(MUL)
    PCAD_RED(MIN)
    PCAD_RED(MAX)
    PCAD_RED(SUMPROD)
  default: return hipErrorInvalidValue;
  }
#undef PCAD_RED
  return hipGetLastError();
}

hipError_t reduce_vjp_launch(int op, int64_t batch, int64_t n, const float *x0, const float *x1,
                             const void *saved, const float *ybar, float *xb0, float *xb1,
                             bool accumulate, void *ws, hipStream_t s) {
  if (batch == 0 || n == 0) return hipSuccess;
  if (op == LINREC || op == MAT2 || op == SATADD) {
    const int tile = scan_tile_size(op);
    const int tpr = (int)((n + tile - 1) / tile);
    RedGenArgs a;
    a.x0 = x0; a.x1 = x1; a.saved = static_cast<const float *>(saved); a.ybar = ybar;
    a.xb0 = xb0; a.xb1 = xb1; a.n = n; a.tpr = tpr; a.accumulate = accumulate ? 1 : 0;
    a.ctl = reinterpret_cast<Ctl *>(ws);
    a.status = reinterpret_cast<uint64_t *>(static_cast<char *>(ws) + kCtlBytes);
    const dim3 grid((unsigned)(batch * tpr));
    if (op == LINREC) hipLaunchKernelGGL(k_reduce_vjp_gen<LINREC>, grid, dim3(Shape<LINREC>::THREADS), 0, s, a);
    else if (op == SATADD) hipLaunchKernelGGL(k_reduce_vjp_gen<SATADD>, grid, dim3(Shape<SATADD>::THREADS), 0, s, a);
    else hipLaunchKernelGGL(k_reduce_vjp_gen<MAT2>, grid, dim3(Shape<MAT2>::THREADS), 0, s, a);
    return hipGetLastError();
  }
  int64_t bx = (n + BLOCK * 4 * 4 - 1) / (BLOCK * 4 * 4);
  if (bx > 65535) bx = 65535;
  const dim3 grid((unsigned)bx, (unsigned)batch);
  const int acc = accumulate ? 1 : 0;
  switch (op) {
  case ADD: hipLaunchKernelGGL(k_reduce_vjp<ADD>, grid, dim3(BLOCK), 0, s, x0, saved, ybar, xb0, n, acc); break;
  case MUL: hipLaunchKernelGGL(k_reduce_vjp<MUL>, grid, dim3(BLOCK), 0, s, x0, saved, ybar, xb0, n, acc); break;
  case MIN: hipLaunchKernelGGL(k_reduce_vjp<MIN>, grid, dim3(BLOCK), 0, s, x0, saved, ybar, xb0, n, acc); break;
  case MAX: hipLaunchKernelGGL(k_reduce_vjp<MAX>, grid, dim3(BLOCK), 0, s, x0, saved, ybar, xb0, n, acc); break;
  case SUMPROD: hipLaunchKernelGGL(k_reduce_vjp<SUMPROD>, grid, dim3(BLOCK), 0, s, x0, saved, ybar, xb0, n, acc); break;
  default: return hipErrorInvalidValue;
  }
  (void)x1; (void)xb1;
  return hipGetLastError();
}

}  // namespace pcad
