// Sort-based reduce-by-index (Section 4, the general rule by sorting): after a
// stable sort of the element indices by bin (sort.hip), the bins are the runs
// of equal keys, and every bin's value is the ordered fold of its run.  The
// fold is a segmented scan over the sorted sequence with the operator
// lifted to (key, value) pairs -- two pairs combine when their keys agree and
// the later pair restarts otherwise, which is associative on a sorted
// sequence -- solved tile by tile with the decoupled look-back; the position
// that ends a run writes its bin.  This serves every operator, the
// non-commutative ones (LINREC, MAT2: per-bin products in ascending element
// order) and, for bin counts beyond an LDS histogram, the commutative ones
// without hot-bin atomics.
//
// Adjoint of the ordered operators (the same rule figure): the exclusive run
// prefix L_i (forward pass), the exclusive run suffix R_i (reverse pass,
// right-to-left look-back) and x_bar_i = d(L_i (.) x_i (.) R_i)/dx_i^T
// applied to the bin adjoint, scattered back through the permutation.
#include "../../include/pcad.h"
#include "device.hpp"
#include "internal.hpp"

namespace pcad {

constexpr int RS_TH = 256, RS_EPL = 8, RS_W = RS_TH / WAVE;
constexpr int RS_TILE = RS_TH * RS_EPL;

__device__ __forceinline__ bool same_key(float a, float b) {
  return __float_as_uint(a) == __float_as_uint(b);
}

// value part of a bin, by operator: payload words, neutral, ordered combine
// (a earlier), and the lift of element `e` (original index) of v
template <int OP>
struct RsBase;

template <>
struct RsBase<ADD> {
  static constexpr int N = 1;
  __device__ static void id(float *p) { p[0] = 0.0f; }
  __device__ static void comb(const float *a, const float *b, float *r) { r[0] = a[0] + b[0]; }
  __device__ static void lift(const float *v, int64_t e, float *p) { p[0] = v[e]; }
};

// (zero count, product of the non-zeros)
template <>
struct RsBase<MUL> {
  static constexpr int N = 2;
  __device__ static void id(float *p) { p[0] = __uint_as_float(0u); p[1] = 1.0f; }
  __device__ static void comb(const float *a, const float *b, float *r) {
    r[0] = __uint_as_float(__float_as_uint(a[0]) + __float_as_uint(b[0]));
    r[1] = a[1] * b[1];
  }
  __device__ static void lift(const float *v, int64_t e, float *p) {
    const float x = v[e];
    p[0] = __uint_as_float(x == 0.0f ? 1u : 0u);
    p[1] = x == 0.0f ? 1.0f : x;
  }
};

// packed 64-bit (ord(value), index) key, as (high, low) words
template <int OP>
struct RsMinMax {
  static constexpr int N = 2;
  __device__ static uint64_t join(const float *p) {
    return ((uint64_t)__float_as_uint(p[0]) << 32) | __float_as_uint(p[1]);
  }
  __device__ static void split(uint64_t k, float *p) {
    p[0] = __uint_as_float((uint32_t)(k >> 32));
    p[1] = __uint_as_float((uint32_t)k);
  }
  __device__ static void id(float *p) { split(key_init<OP>(), p); }
  __device__ static void comb(const float *a, const float *b, float *r) {
    const uint64_t x = join(a), y = join(b);
    split(OP == MIN ? (x < y ? x : y) : (x > y ? x : y), r);
  }
  __device__ static void lift(const float *v, int64_t e, float *p) {
    split(key_of<OP>(v[e], (uint32_t)e), p);
  }
};
template <>
struct RsBase<MIN> : RsMinMax<MIN> {};
template <>
struct RsBase<MAX> : RsMinMax<MAX> {};

// saturated addition (the evaluation's operator figure)
template <>
struct RsBase<SATADD> {
  static constexpr int N = 1;
  __device__ static void id(float *p) { p[0] = 0.0f; }
  __device__ static void comb(const float *a, const float *b, float *r) {
    const float t = a[0] + b[0];
    r[0] = t > kSatCap ? kSatCap : t;
  }
  __device__ static void lift(const float *v, int64_t e, float *p) { p[0] = v[e]; }
};

template <>
struct RsBase<LINREC> {
  static constexpr int N = 2;  // (A, y); elements (a, b) interleaved in v
  __device__ static void id(float *p) { p[0] = 1.0f; p[1] = 0.0f; }
  __device__ static void comb(const float *a, const float *b, float *r) {
    const float A = a[0] * b[0], y = __builtin_fmaf(b[0], a[1], b[1]);
    r[0] = A;
    r[1] = y;
  }
  __device__ static void lift(const float *v, int64_t e, float *p) {
    const float2 t = *reinterpret_cast<const float2 *>(v + e * 2);
    p[0] = t.x;
    p[1] = t.y;
  }
};

template <>
struct RsBase<MAT2> {
  static constexpr int N = 4;  // row-major 2x2, elements as float4 in v
  __device__ static void id(float *p) { p[0] = 1.0f; p[1] = 0.0f; p[2] = 0.0f; p[3] = 1.0f; }
  __device__ static void comb(const float *a, const float *b, float *r) {
    const float r0 = __builtin_fmaf(a[0], b[0], a[1] * b[2]);
    const float r1 = __builtin_fmaf(a[0], b[1], a[1] * b[3]);
    const float r2 = __builtin_fmaf(a[2], b[0], a[3] * b[2]);
    const float r3 = __builtin_fmaf(a[2], b[1], a[3] * b[3]);
    r[0] = r0; r[1] = r1; r[2] = r2; r[3] = r3;
  }
  __device__ static void lift(const float *v, int64_t e, float *p) {
    const float4 t = *reinterpret_cast<const float4 *>(v + e * 4);
    p[0] = t.x; p[1] = t.y; p[2] = t.z; p[3] = t.w;
  }
};

// the lifted segmented operator: word 0 holds the key's bits.  REV: the
// scan runs right to left (the accumulated part is the later one).
template <int OP, bool REV>
struct RsSeg {
  using B = RsBase<OP>;
  static constexpr int N = 1 + B::N;
  using T = Vec<N>;
  using P = T;
  static constexpr int NA = N, NP = N;
  __device__ static T id() {
    T t;
    t.f[0] = __uint_as_float(0xffffffffu);  // no key
    B::id(t.f + 1);
    return t;
  }
  // the neutral element (no key) is an identity on both sides; otherwise a
  // later pair with another key restarts the run
  __device__ static T comb(const T &a, const T &b) {
    if (__float_as_uint(b.f[0]) == 0xffffffffu) return a;
    if (!same_key(a.f[0], b.f[0])) return b;
    T r;
    r.f[0] = b.f[0];
    if (REV) B::comb(b.f + 1, a.f + 1, r.f + 1);
    else B::comb(a.f + 1, b.f + 1, r.f + 1);
    return r;
  }
  __device__ static T from_pre(const P &p) { return p; }
};

struct RsArgs {
  const int32_t *sk, *perm;  // sorted keys (m: out of range) and permutation
  const float *v;            // element values (d floats per element)
  int64_t n, m;
  int64_t ntiles;
  // forward outputs (mode 0)
  float *hist;               // ADD, LINREC, MAT2: bins (d floats each)
  uint32_t *n0;              // MUL
  float *ypos;               // MUL
  uint64_t *keys;            // MIN/MAX
  // adjoint (mode 1 writes L; the reverse pass reads it): L_i of sorted
  // position i lives at lpre[perm[i]] -- the element's own output slot when
  // the adjoint is overwritten, so no scratch is needed
  float *lpre;               // [n][B::N], original element order
  const float *hbar;         // [m][d] bin adjoints
  float *vbar;               // [n][d] element adjoints, original order
  int accumulate;
  Ctl *ctl;
  uint64_t *status;
};

// MODE 0: bins at run ends.  MODE 1: exclusive run prefixes L_i.
template <int OP, int MODE>
__global__ __launch_bounds__(RS_TH) void k_rbi_sorted(RsArgs a) {
  using Tr = RsSeg<OP, false>;
  using T = typename Tr::T;
  using B = RsBase<OP>;
  constexpr int N = Tr::N;
  __shared__ T s_tot[1][RS_W];
  __shared__ T s_pre[1][RS_W];
  __shared__ T s_carry;
  __shared__ unsigned s_epoch;
  const int tid = threadIdx.x, lane = lane_id(), wave = tid / WAVE;
  if (tid == 0) s_epoch = ctl_load(&a.ctl->epoch);
  const int64_t tile = blockIdx.x;
  const int64_t p0 = tile * RS_TILE + (int64_t)tid * RS_EPL;

  T loc[RS_EPL];
  int32_t key[RS_EPL + 1];
#pragma unroll
  for (int j = 0; j <= RS_EPL; ++j) key[j] = p0 + j < a.n ? a.sk[p0 + j] : -1;
  T acc = Tr::id();
#pragma unroll
  for (int j = 0; j < RS_EPL; ++j) {
    T x = Tr::id();
    if (p0 + j < a.n) {
      x.f[0] = __int_as_float(key[j]);
      if (key[j] < a.m) B::lift(a.v, a.perm[p0 + j], x.f + 1);
    }
    acc = j == 0 ? x : Tr::comb(acc, x);
    loc[j] = acc;
  }
  const T incl = wave_scan_fwd<Tr>(acc);
  if (lane == WAVE - 1) s_tot[0][wave] = incl;
  __syncthreads();
  const uint32_t tag = next_tag(s_epoch);
  if (wave == 0) {
    const T agg = wave0_block_prefix<Tr, 1, RS_W, false>(s_tot, s_pre, Tr::id());
    uint64_t *st = a.status + tile * (Tr::NA + Tr::NP);
    T c = Tr::id();
    if (tile == 0) {
      if (lane == 0) publish<N>(st + Tr::NA, tag, agg);
    } else {
      if (lane == 0) publish<N>(st, tag, agg);
      c = lookback<Tr>(a.status, tile, +1, (int)(tile < 0x7fffffff ? tile : 0x7fffffff), tag, a.ctl);
      if (lane == 0) publish<N>(st + Tr::NA, tag, Tr::comb(c, agg));
    }
    if (lane == 0) {
      s_carry = c;
      if (tile == a.ntiles - 1) ctl_row_done(a.ctl, 1u, tag);
    }
  }
  __syncthreads();
  T ex = shift_up1(incl);
  if (lane == 0) ex = Tr::id();
  const T full = Tr::comb(Tr::comb(s_carry, s_pre[0][wave]), ex);
#pragma unroll
  for (int j = 0; j < RS_EPL; ++j) {
    const int64_t p = p0 + j;
    if (p >= a.n || key[j] >= a.m) continue;
    if (MODE == 0) {
      if (p + 1 < a.n && key[j + 1] == key[j]) continue;  // not the run's end
      const T r = Tr::comb(full, loc[j]);
      const int64_t k = key[j];
      if (OP == ADD || OP == SATADD) a.hist[k] = r.f[1];
      if (OP == MUL) { a.n0[k] = __float_as_uint(r.f[1]); a.ypos[k] = r.f[2]; }
      if (OP == MIN || OP == MAX) a.keys[k] = RsMinMax<OP>::join(r.f + 1);
      if (OP == LINREC || OP == MAT2) {
#pragma unroll
        for (int t = 0; t < B::N; ++t) a.hist[k * B::N + t] = r.f[1 + t];
      }
    } else {
      // exclusive prefix: the inclusive value one position earlier, if it
      // belongs to the same run
      const T prev = j == 0 ? full : Tr::comb(full, loc[j - 1]);
      float l[B::N];
      if (same_key(prev.f[0], __int_as_float(key[j]))) {
#pragma unroll
        for (int t = 0; t < B::N; ++t) l[t] = prev.f[1 + t];
      } else {
        B::id(l);
      }
      const int64_t e = a.perm[p];
#pragma unroll
      for (int t = 0; t < B::N; ++t) a.lpre[e * B::N + t] = l[t];
    }
  }
}

// adjoint of the ordered operators: reverse pass over the sorted sequence
template <int OP>
__device__ __forceinline__ void rs_local_vjp(const float *l, const float *x, const float *r,
                                             const float *hb, float *xb) {
  if (OP == SATADD) {
    // out = (l (.) x) (.) r: both steps' partials in x, 0 where saturated
    const float lx = l[0] + x[0];
    const float lxs = lx > kSatCap ? kSatCap : lx;
    xb[0] = (!(lx > kSatCap) && !(lxs + r[0] > kSatCap)) ? hb[0] : 0.0f;
  } else if (OP == LINREC) {
    // out = (l (.) x) (.) r = (A_l a A_r, (y_l a + b) A_r + y_r)
    xb[0] = (hb[0] * l[0] + hb[1] * l[1]) * r[0];
    xb[1] = hb[1] * r[0];
  } else {
    // out = l x r: x_bar = l^T hb r^T
    const float t0 = __builtin_fmaf(hb[0], r[0], hb[1] * r[1]);  // (hb r^T) row 0
    const float t1 = __builtin_fmaf(hb[0], r[2], hb[1] * r[3]);
    const float t2 = __builtin_fmaf(hb[2], r[0], hb[3] * r[1]);  // row 1
    const float t3 = __builtin_fmaf(hb[2], r[2], hb[3] * r[3]);
    xb[0] = __builtin_fmaf(l[0], t0, l[2] * t2);
    xb[1] = __builtin_fmaf(l[0], t1, l[2] * t3);
    xb[2] = __builtin_fmaf(l[1], t0, l[3] * t2);
    xb[3] = __builtin_fmaf(l[1], t1, l[3] * t3);
  }
}

template <int OP>
__global__ __launch_bounds__(RS_TH) void k_rbi_sorted_vjp(RsArgs a) {
  using Tr = RsSeg<OP, true>;
  using T = typename Tr::T;
  using B = RsBase<OP>;
  constexpr int N = Tr::N, D = B::N;
  __shared__ T s_tot[1][RS_W];
  __shared__ T s_pre[1][RS_W];
  __shared__ T s_carry;
  __shared__ unsigned s_epoch;
  const int tid = threadIdx.x, lane = lane_id(), wave = tid / WAVE;
  if (tid == 0) s_epoch = ctl_load(&a.ctl->epoch);
  const int64_t tile = a.ntiles - 1 - blockIdx.x;  // right to left
  const int64_t p0 = tile * RS_TILE + (int64_t)tid * RS_EPL;

  T loc[RS_EPL];     // inclusive run suffix from the thread's right end
  int32_t key[RS_EPL];
  float xs[RS_EPL][D];
#pragma unroll
  for (int j = 0; j < RS_EPL; ++j) {
    key[j] = p0 + j < a.n ? a.sk[p0 + j] : -1;
    if (p0 + j < a.n && key[j] < a.m) B::lift(a.v, a.perm[p0 + j], xs[j]);
    else B::id(xs[j]);
  }
  T acc = Tr::id();
#pragma unroll
  for (int j = RS_EPL - 1; j >= 0; --j) {
    T x = Tr::id();
    if (p0 + j < a.n) {
      x.f[0] = __int_as_float(key[j]);
#pragma unroll
      for (int t = 0; t < D; ++t) x.f[1 + t] = xs[j][t];
    }
    acc = j == RS_EPL - 1 ? x : Tr::comb(acc, x);
    loc[j] = acc;
  }
  const T incl = wave_scan_rev<Tr>(acc);
  if (lane == 0) s_tot[0][wave] = incl;
  __syncthreads();
  const uint32_t tag = next_tag(s_epoch);
  if (wave == 0) {
    const T agg = wave0_block_prefix<Tr, 1, RS_W, true>(s_tot, s_pre, Tr::id());
    uint64_t *st = a.status + tile * (Tr::NA + Tr::NP);
    T c = Tr::id();
    const int64_t dist = a.ntiles - 1 - tile;
    if (dist == 0) {
      if (lane == 0) publish<N>(st + Tr::NA, tag, agg);
    } else {
      if (lane == 0) publish<N>(st, tag, agg);
      c = lookback<Tr>(a.status, tile, -1, (int)(dist < 0x7fffffff ? dist : 0x7fffffff), tag, a.ctl);
      if (lane == 0) publish<N>(st + Tr::NA, tag, Tr::comb(c, agg));
    }
    if (lane == 0) {
      s_carry = c;
      if (tile == 0) ctl_row_done(a.ctl, 1u, tag);
    }
  }
  __syncthreads();
  T ex = shift_down1(incl);
  if (lane == WAVE - 1) ex = Tr::id();
  const T full = Tr::comb(Tr::comb(s_carry, s_pre[0][wave]), ex);  // everything right of the thread
#pragma unroll
  for (int j = 0; j < RS_EPL; ++j) {
    const int64_t p = p0 + j;
    if (p >= a.n) continue;
    const int64_t e = a.perm[p];
    float xb[D];
    if (key[j] < a.m) {
      // exclusive suffix: the inclusive suffix one position later, if it
      // belongs to the same run
      const T nxt = j == RS_EPL - 1 ? full : Tr::comb(full, loc[j + 1]);
      float r[D];
      if (same_key(nxt.f[0], __int_as_float(key[j]))) {
#pragma unroll
        for (int t = 0; t < D; ++t) r[t] = nxt.f[1 + t];
      } else {
        B::id(r);
      }
      float l[D], hb[D];
#pragma unroll
      for (int t = 0; t < D; ++t) {
        l[t] = a.lpre[e * D + t];
        hb[t] = a.hbar[(int64_t)key[j] * D + t];
      }
      rs_local_vjp<OP>(l, xs[j], r, hb, xb);
    } else {
#pragma unroll
      for (int t = 0; t < D; ++t) xb[t] = 0.0f;  // out-of-range key: no adjoint
    }
#pragma unroll
    for (int t = 0; t < D; ++t) {
      float o = xb[t];
      if (a.accumulate) o += a.vbar[e * D + t];
      a.vbar[e * D + t] = o;
    }
  }
}

// ---------------------------------------------------------------------------
// host
// ---------------------------------------------------------------------------
static int rs_words(int op) {
  switch (op) {
  case ADD: return 2 * (1 + RsBase<ADD>::N);
  case MUL: return 2 * (1 + RsBase<MUL>::N);
  case MIN: case MAX: return 2 * (1 + 2);
  case LINREC: return 2 * (1 + RsBase<LINREC>::N);
  case MAT2: return 2 * (1 + RsBase<MAT2>::N);
  case SATADD: return 2 * (1 + RsBase<SATADD>::N);
  }
  return 0;
}

static size_t al256(size_t x) { return (x + 255) / 256 * 256; }

// Per row, in the caller's saved state: the sorted keys, the permutation and
// the sort's scratch (the ordered adjoint reuses the sort), so the workspace
// holds nothing but look-back status words between calls.
size_t rbi_sort_area_bytes(int64_t n, int64_t m) {
  return 2 * al256((size_t)n * 4) + al256(sort_ws_bytes(n, m));
}

// workspace of one row: the look-back status words and, for an accumulating
// ordered adjoint, L (zeroed again before the call returns)
size_t rbi_sorted_ws_bytes(int op, int64_t n, int64_t m) {
  (void)m;
  const int64_t nt = (n + RS_TILE - 1) / RS_TILE;
  size_t b = al256((size_t)(nt > 0 ? nt : 1) * rs_words(op) * 8);
  if (op == LINREC || op == MAT2 || op == SATADD)
    b += al256((size_t)n * (op == LINREC ? 2 : (op == MAT2 ? 4 : 1)) * 4);
  return b;
}

__global__ void k_zero_f32(float *p, int64_t n) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x)
    p[i] = 0.0f;
}

hipError_t rbi_sorted_fwd_row(int op, int64_t n, int64_t m, const int32_t *idx, const float *v,
                              float *hist, uint32_t *n0, float *ypos, uint64_t *keys, void *ctl,
                              void *region, void *area, hipStream_t s) {
  if (n == 0) return hipSuccess;
  char *ar = static_cast<char *>(area);
  int32_t *sk = reinterpret_cast<int32_t *>(ar);
  int32_t *perm = reinterpret_cast<int32_t *>(ar + al256((size_t)n * 4));
  hipError_t e = sort_by_key(idx, n, m, sk, perm, ar + 2 * al256((size_t)n * 4), s);
  if (e != hipSuccess) return e;
  RsArgs a{};
  a.sk = sk; a.perm = perm; a.v = v; a.n = n; a.m = m;
  a.ntiles = (n + RS_TILE - 1) / RS_TILE;
  a.hist = hist; a.n0 = n0; a.ypos = ypos; a.keys = keys;
  a.ctl = reinterpret_cast<Ctl *>(ctl);
  a.status = reinterpret_cast<uint64_t *>(region);
  const dim3 g((unsigned)a.ntiles);
  switch (op) {
  case ADD: hipLaunchKernelGGL((k_rbi_sorted<ADD, 0>), g, dim3(RS_TH), 0, s, a); break;
  case MUL: hipLaunchKernelGGL((k_rbi_sorted<MUL, 0>), g, dim3(RS_TH), 0, s, a); break;
  case MIN: hipLaunchKernelGGL((k_rbi_sorted<MIN, 0>), g, dim3(RS_TH), 0, s, a); break;
  case MAX: hipLaunchKernelGGL((k_rbi_sorted<MAX, 0>), g, dim3(RS_TH), 0, s, a); break;
  case LINREC: hipLaunchKernelGGL((k_rbi_sorted<LINREC, 0>), g, dim3(RS_TH), 0, s, a); break;
  case MAT2: hipLaunchKernelGGL((k_rbi_sorted<MAT2, 0>), g, dim3(RS_TH), 0, s, a); break;
  case SATADD: hipLaunchKernelGGL((k_rbi_sorted<SATADD, 0>), g, dim3(RS_TH), 0, s, a); break;
  default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

// adjoint of one row by the general rule (LINREC, MAT2, SATADD), from the sort the
// forward left in `area`
hipError_t rbi_sorted_vjp_row(int op, int64_t n, int64_t m, const float *v, const float *hbar,
                              float *vbar, bool accumulate, void *ctl, void *region,
                              const void *area, hipStream_t s) {
  if (n == 0) return hipSuccess;
  const char *ar = static_cast<const char *>(area);
  const int d = op == LINREC ? 2 : (op == MAT2 ? 4 : 1);
  const int64_t nt = (n + RS_TILE - 1) / RS_TILE;
  RsArgs a{};
  a.sk = reinterpret_cast<const int32_t *>(ar);
  a.perm = reinterpret_cast<const int32_t *>(ar + al256((size_t)n * 4));
  a.v = v; a.n = n; a.m = m;
  a.ntiles = nt;
  a.hbar = hbar; a.vbar = vbar; a.accumulate = accumulate ? 1 : 0;
  a.ctl = reinterpret_cast<Ctl *>(ctl);
  a.status = reinterpret_cast<uint64_t *>(region);
  float *scratch = reinterpret_cast<float *>(static_cast<char *>(region) +
                                             al256((size_t)(nt > 0 ? nt : 1) * rs_words(op) * 8));
  a.lpre = accumulate ? scratch : vbar;
  const dim3 g((unsigned)nt);
  if (op == LINREC) {
    hipLaunchKernelGGL((k_rbi_sorted<LINREC, 1>), g, dim3(RS_TH), 0, s, a);
    hipLaunchKernelGGL(k_rbi_sorted_vjp<LINREC>, g, dim3(RS_TH), 0, s, a);
  } else if (op == MAT2) {
    hipLaunchKernelGGL((k_rbi_sorted<MAT2, 1>), g, dim3(RS_TH), 0, s, a);
    hipLaunchKernelGGL(k_rbi_sorted_vjp<MAT2>, g, dim3(RS_TH), 0, s, a);
  } else if (op == SATADD) {
    hipLaunchKernelGGL((k_rbi_sorted<SATADD, 1>), g, dim3(RS_TH), 0, s, a);
    hipLaunchKernelGGL(k_rbi_sorted_vjp<SATADD>, g, dim3(RS_TH), 0, s, a);
  } else {
    return hipErrorInvalidValue;
  }
  if (accumulate) {
    // leave the workspace as found: no data beyond status words
    int64_t g2 = ((int64_t)n * d + 255) / 256;
    if (g2 > 16384) g2 = 16384;
    hipLaunchKernelGGL(k_zero_f32, dim3((unsigned)g2), dim3(256), 0, s, scratch, (int64_t)n * d);
  }
  return hipGetLastError();
}

}  // namespace pcad
