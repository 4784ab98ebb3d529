// Scans of d x d matrix products for d = 3 and 5 (the evaluation's 3x3 and
// 5x5 matrix multiplication operators) and their adjoints, by the redundant
// block-diagonal sparsity of Section 5.3: the adjoint state of P_i is a
// d x d matrix Rbar_i and its recurrence r -> Pbar_i + r M_{i+1}^T is an
// affine map with a d x d linear part, so an adjoint map carries 2 d^2
// floats instead of the d^4 of a dense Jacobian.
//
//   forward : P_i = P_{i-1} M_i
//   adjoint : rho_i = (Pbar_i + rho_{i+1}) M_i^T carried right to left,
//             Rbar_i = Pbar_i + rho_{i+1},  Mbar_i = P_{i-1}^T Rbar_i
//
// Elements are large (36 or 100 bytes), so these kernels reduce and then
// scan instead of looking back.  Per direction:
//   1. per tile (TPT consecutive elements per thread, 256 threads) the
//      ordered product of the tile (forward) or the composition of its
//      adjoint maps (reverse);
//   2. per chunk of 256 tiles, one block scans the tile values (exclusive
//      prefixes in scan order) and emits the chunk's value;
//   3. one block per row scans the chunk values;
//   4. every tile is rescanned from its entry value and written out.
// Tiles move between HBM and LDS in coalesced runs; each thread's elements
// sit in LDS at an odd stride (no bank conflicts) and the in-block scans run
// in registers through DPP (wave) and a 4-entry LDS table (waves).
//
// The forward saves the exclusive prefix product of every tile; the adjoint
// recomputes the forward prefixes inside each tile from it.  The reduce runs
// passes 1-3 (the row product falls out of pass 3) and its adjoint is the
// scan adjoint seeded with Ybar at the last element only, which is Section
// 3.1's rule L_i^T Ybar R_i^T.  Workspace
// temporaries are zeroed by the pass that consumes them (the last one by a
// small fill kernel), so the workspace holds only zeros between calls.
#include "device.hpp"
#include "internal.hpp"

namespace pcad {
namespace {

constexpr int MD_TH = 256;
constexpr int MD_W = MD_TH / WAVE;  // waves per block
constexpr int MD_CH = MD_TH;        // tiles per chunk (one per thread)

template <int D>
struct MD {
  static constexpr int D2 = D * D;
  static constexpr int TPT = D == 3 ? 4 : 2;  // elements per thread
  static constexpr int TILE = MD_TH * TPT;
  static constexpr int GF = TPT * D2;         // floats of one thread's elements
  static constexpr int GS = GF + 1;           // their LDS stride (odd)
  static constexpr int LDS = MD_TH * GS;

  __device__ static void eye(float *a) {
#pragma unroll
    for (int i = 0; i < D2; ++i) a[i] = (i % (D + 1) == 0) ? 1.0f : 0.0f;
  }
  // r = a b (r must not alias a or b)
  __device__ static void mul(const float *a, const float *b, float *r) {
#pragma unroll
    for (int i = 0; i < D; ++i)
#pragma unroll
      for (int j = 0; j < D; ++j) {
        float s = a[i * D] * b[j];
#pragma unroll
        for (int k = 1; k < D; ++k) s = __builtin_fmaf(a[i * D + k], b[k * D + j], s);
        r[i * D + j] = s;
      }
  }
  // r = a b^T
  __device__ static void mul_bt(const float *a, const float *b, float *r) {
#pragma unroll
    for (int i = 0; i < D; ++i)
#pragma unroll
      for (int j = 0; j < D; ++j) {
        float s = a[i * D] * b[j * D];
#pragma unroll
        for (int k = 1; k < D; ++k) s = __builtin_fmaf(a[i * D + k], b[j * D + k], s);
        r[i * D + j] = s;
      }
  }
  // r = a^T b
  __device__ static void mul_at(const float *a, const float *b, float *r) {
#pragma unroll
    for (int i = 0; i < D; ++i)
#pragma unroll
      for (int j = 0; j < D; ++j) {
        float s = a[i] * b[j];
#pragma unroll
        for (int k = 1; k < D; ++k) s = __builtin_fmaf(a[k * D + i], b[k * D + j], s);
        r[i * D + j] = s;
      }
  }
  // adjoint maps h(r) = o + r W, stored as o[D2] then W[D2]
  __device__ static void map_id(float *h) {
#pragma unroll
    for (int i = 0; i < D2; ++i) h[i] = 0.0f;
    eye(h + D2);
  }
  // r = l o e (e applied first): o = o_l + o_e W_l, W = W_e W_l
  __device__ static void map_comb(const float *l, const float *e, float *r) {
    mul(e, l + D2, r);
#pragma unroll
    for (int i = 0; i < D2; ++i) r[i] += l[i];
    mul(e + D2, l + D2, r + D2);
  }
  // r = h(v) = o + v W
  __device__ static void map_apply(const float *h, const float *v, float *r) {
    mul(v, h + D2, r);
#pragma unroll
    for (int i = 0; i < D2; ++i) r[i] += h[i];
  }
};

// scan operators for the DPP wave scans (comb(earlier, later))
template <int D>
struct TrMat {
  using T = Vec<D * D>;
  __device__ static T id() {
    T r;
    MD<D>::eye(r.f);
    return r;
  }
  __device__ static T comb(const T &a, const T &b) {
    T r;
    MD<D>::mul(a.f, b.f, r.f);
    return r;
  }
};

// adjoint maps in right-to-left order: the earlier (right) map acts first
template <int D>
struct TrMap {
  using T = Vec<2 * D * D>;
  __device__ static T id() {
    T r;
    MD<D>::map_id(r.f);
    return r;
  }
  __device__ static T comb(const T &earlier, const T &later) {
    T r;
    MD<D>::map_comb(later.f, earlier.f, r.f);
    return r;
  }
};

template <int D>
using Mat = Vec<D * D>;
template <int D>
using Map = Vec<2 * D * D>;

struct MdArgs {
  const float *x;     // M [rows][n][d*d]
  const float *pbar;  // adjoint input [rows][n][d*d]
  float *y;           // forward output / adjoint output
  float *pre;         // saved: exclusive prefix per tile [tiles][d*d]
  float *agg;         // workspace: tile values [tiles][2 d*d]
  float *cagg;        // workspace: chunk values [chunks][2 d*d]
  float *cvec;        // workspace: chunk entry values [chunks][d*d]
  float *total;       // reduce: the product of each row [rows][d*d] (else null)
  const float *ybar_last;  // reduce adjoint: Ybar per row; Pbar_i = Ybar at
                           // i = n-1, else 0 (pbar unused)
  int64_t n;
  int64_t tpr;        // tiles per row
  int64_t cpr;        // chunks per row
  int accumulate;
};

struct TileRange {
  int64_t row, lt, base;  // base: global element index of the tile's first element
  int64_t chunk;          // global chunk index
  int valid;
};

template <int D>
__device__ __forceinline__ TileRange md_tile(const MdArgs &a, int64_t tile) {
  TileRange t;
  t.row = tile / a.tpr;
  t.lt = tile - t.row * a.tpr;
  const int64_t s = t.lt * MD<D>::TILE;
  t.base = t.row * a.n + s;
  t.chunk = t.row * a.cpr + t.lt / MD_CH;
  const int64_t rem = a.n - s;
  t.valid = (int)(rem < MD<D>::TILE ? rem : MD<D>::TILE);
  return t;
}

// global run of cnt floats -> LDS, thread groups of GF floats at stride GS
template <int D>
__device__ __forceinline__ void stage_in(const float *__restrict__ src, int cnt, float *lds) {
  using C = MD<D>;
#pragma unroll 4
  for (int f = threadIdx.x; f < cnt; f += MD_TH) lds[f + f / C::GF] = src[f];
}

template <int D>
__device__ __forceinline__ void stage_out(float *__restrict__ dst, int cnt, const float *lds,
                                          bool accumulate) {
  using C = MD<D>;
#pragma unroll 4
  for (int f = threadIdx.x; f < cnt; f += MD_TH) {
    const float v = lds[f + f / C::GF];
    dst[f] = accumulate ? dst[f] + v : v;
  }
}

// the adjoint input of a tile: Pbar from memory, or for the reduce adjoint
// Ybar at the row's last element and zeros elsewhere
template <int D>
__device__ __forceinline__ void stage_pbar(const MdArgs &a, const TileRange &t, float *lds) {
  using C = MD<D>;
  if (!a.ybar_last) {
    stage_in<D>(a.pbar + t.base * C::D2, t.valid * C::D2, lds);
    return;
  }
  const int cnt = t.valid * C::D2;
  const int64_t last = a.n - 1 - t.lt * C::TILE;  // the row's last element, tile-relative
  const float *yb = a.ybar_last + t.row * C::D2;
  for (int f = threadIdx.x; f < cnt; f += MD_TH) {
    const int e = f / C::D2;
    lds[f + f / C::GF] = (e == last) ? yb[f - e * C::D2] : 0.0f;
  }
}

// this thread's element j in LDS
template <int D>
__device__ __forceinline__ float *lds_el(float *lds, int j) {
  return lds + threadIdx.x * MD<D>::GS + j * MD<D>::D2;
}

template <int N>
__device__ __forceinline__ void copy_in(Vec<N> &v, const float *p) {
#pragma unroll
  for (int i = 0; i < N; ++i) v.f[i] = p[i];
}

template <int N>
__device__ __forceinline__ void put(float *g, const Vec<N> &v) {
#pragma unroll
  for (int i = 0; i < N; ++i) g[i] = v.f[i];
}

template <int N>
__device__ __forceinline__ void zero(float *g) {
#pragma unroll
  for (int i = 0; i < N; ++i) g[i] = 0.0f;
}

// the thread's ordered product of its elements (identity past the end)
template <int D>
__device__ __forceinline__ Mat<D> thread_product(float *lds, int valid) {
  using C = MD<D>;
  Mat<D> acc = TrMat<D>::id();
#pragma unroll
  for (int j = 0; j < C::TPT; ++j) {
    const int e = threadIdx.x * C::TPT + j;
    if (e >= valid) break;
    Mat<D> m;
    copy_in(m, lds_el<D>(lds, j));
    acc = j == 0 ? m : TrMat<D>::comb(acc, m);
  }
  return acc;
}

// the thread's composed adjoint map h_first o ... o h_last with
// h_i(r) = (Pbar_i + r) M_i^T; M from registers, Pbar from LDS
template <int D>
__device__ __forceinline__ Map<D> thread_map(const Mat<D> (&m)[MD<D>::TPT], float *lds, int valid) {
  using C = MD<D>;
  Map<D> acc = TrMap<D>::id();
  bool first = true;
#pragma unroll
  for (int j = C::TPT - 1; j >= 0; --j) {
    const int e = threadIdx.x * C::TPT + j;
    if (e >= valid) continue;
    float q[C::D2];
    const float *p = lds_el<D>(lds, j);
#pragma unroll
    for (int i = 0; i < C::D2; ++i) q[i] = p[i] + (first ? 0.0f : acc.f[i]);
    Map<D> r;
    C::mul_bt(q, m[j].f, r.f);  // o = (Pbar + o_acc) M^T
    if (first) {
#pragma unroll
      for (int i = 0; i < D; ++i)
#pragma unroll
        for (int k = 0; k < D; ++k) r.f[C::D2 + i * D + k] = m[j].f[k * D + i];  // W = M^T
    } else {
      C::mul_bt(acc.f + C::D2, m[j].f, r.f + C::D2);  // W = W_acc M^T
    }
    acc = r;
    first = false;
  }
  return acc;
}

// pass 1, forward: the ordered product of every tile
template <int D>
__global__ __launch_bounds__(MD_TH) void k_md_agg(MdArgs a) {
  using C = MD<D>;
  using Tr = TrMat<D>;
  __shared__ float s_t[C::LDS];
  __shared__ Mat<D> s_w[MD_W];
  const TileRange t = md_tile<D>(a, blockIdx.x);
  stage_in<D>(a.x + t.base * C::D2, t.valid * C::D2, s_t);
  __syncthreads();
  const Mat<D> inc = wave_scan_fwd<Tr>(thread_product<D>(s_t, t.valid));
  if (lane_id() == WAVE - 1) s_w[threadIdx.x / WAVE] = inc;
  __syncthreads();
  if (threadIdx.x == 0) {
    Mat<D> tot = s_w[0];
#pragma unroll
    for (int w = 1; w < MD_W; ++w) tot = Tr::comb(tot, s_w[w]);
    put(a.agg + blockIdx.x * 2 * C::D2, tot);
  }
}

// pass 1, adjoint: the composed adjoint map of every tile
template <int D>
__global__ __launch_bounds__(MD_TH) void k_md_vagg(MdArgs a) {
  using C = MD<D>;
  using Tr = TrMap<D>;
  __shared__ float s_t[C::LDS];
  __shared__ Map<D> s_w[MD_W];
  const TileRange t = md_tile<D>(a, blockIdx.x);
  stage_in<D>(a.x + t.base * C::D2, t.valid * C::D2, s_t);
  __syncthreads();
  Mat<D> m[C::TPT];
#pragma unroll
  for (int j = 0; j < C::TPT; ++j) copy_in(m[j], lds_el<D>(s_t, j));
  __syncthreads();
  stage_pbar<D>(a, t, s_t);
  __syncthreads();
  const Map<D> inc = wave_scan_rev<Tr>(thread_map<D>(m, s_t, t.valid));
  if (lane_id() == 0) s_w[threadIdx.x / WAVE] = inc;
  __syncthreads();
  if (threadIdx.x == 0) {
    Map<D> tot = s_w[MD_W - 1];
#pragma unroll
    for (int w = MD_W - 2; w >= 0; --w) tot = Tr::comb(tot, s_w[w]);
    put(a.agg + blockIdx.x * 2 * C::D2, tot);
  }
}

// pass 2 (one block per chunk of tiles): forward, the chunk-local exclusive
// prefix of every tile into `pre`; adjoint, the composed map of the tiles
// right of each tile within the chunk, in place of the tile's value
template <int D, bool REV>
__global__ __launch_bounds__(MD_TH) void k_md_scan_tiles(MdArgs a) {
  using C = MD<D>;
  const int lane = lane_id(), wave = threadIdx.x / WAVE;
  const int64_t row = blockIdx.x / a.cpr, ch = blockIdx.x - row * a.cpr;
  const int64_t tl = ch * MD_CH + threadIdx.x;
  const bool ok = tl < a.tpr;
  float *g = a.agg + (row * a.tpr + tl) * 2 * C::D2;
  if constexpr (!REV) {
    using Tr = TrMat<D>;
    __shared__ Mat<D> s_w[MD_W];
    Mat<D> v = Tr::id();
    if (ok) {
      copy_in(v, g);
      zero<C::D2>(g);  // consumed
    }
    const Mat<D> inc = wave_scan_fwd<Tr>(v);
    if (lane == WAVE - 1) s_w[wave] = inc;
    __syncthreads();
    Mat<D> r = shift_up1(inc);
    if (lane == 0) r = Tr::id();
    for (int w = wave - 1; w >= 0; --w) r = Tr::comb(s_w[w], r);
    if (ok) put(a.pre + (row * a.tpr + tl) * C::D2, r);
    if (threadIdx.x == 0) {
      Mat<D> tot = s_w[0];
#pragma unroll
      for (int w = 1; w < MD_W; ++w) tot = Tr::comb(tot, s_w[w]);
      put(a.cagg + blockIdx.x * 2 * C::D2, tot);
    }
  } else {
    using Tr = TrMap<D>;
    __shared__ Map<D> s_w[MD_W];
    Map<D> v = Tr::id();
    if (ok) copy_in(v, g);
    const Map<D> inc = wave_scan_rev<Tr>(v);
    if (lane == 0) s_w[wave] = inc;
    __syncthreads();
    Map<D> r = shift_down1(inc);
    if (lane == WAVE - 1) r = Tr::id();
    for (int w = wave + 1; w < MD_W; ++w) r = Tr::comb(s_w[w], r);
    if (ok) put(g, r);
    if (threadIdx.x == 0) {
      Map<D> tot = s_w[MD_W - 1];
#pragma unroll
      for (int w = MD_W - 2; w >= 0; --w) tot = Tr::comb(tot, s_w[w]);
      put(a.cagg + blockIdx.x * 2 * C::D2, tot);
    }
  }
}

// pass 3 (one block per row): the entry value of every chunk -- forward, the
// product of the chunks before it; adjoint, the adjoint entering it from the
// right
template <int D, bool REV>
__global__ __launch_bounds__(MD_TH) void k_md_scan_chunks(MdArgs a) {
  using C = MD<D>;
  const int lane = lane_id(), wave = threadIdx.x / WAVE;
  const int64_t row = blockIdx.x;
  if constexpr (!REV) {
    using Tr = TrMat<D>;
    __shared__ Mat<D> s_w[MD_W];
    Mat<D> carry = Tr::id();
    for (int64_t c0 = 0; c0 < a.cpr; c0 += MD_TH) {
      const int64_t c = c0 + threadIdx.x;
      const bool ok = c < a.cpr;
      float *g = a.cagg + (row * a.cpr + c) * 2 * C::D2;
      Mat<D> v = Tr::id();
      if (ok) {
        copy_in(v, g);
        zero<C::D2>(g);
      }
      const Mat<D> inc = wave_scan_fwd<Tr>(v);
      if (lane == WAVE - 1) s_w[wave] = inc;
      __syncthreads();
      Mat<D> r = shift_up1(inc);
      if (lane == 0) r = Tr::id();
      for (int w = wave - 1; w >= 0; --w) r = Tr::comb(s_w[w], r);
      if (ok) put(a.cvec + (row * a.cpr + c) * C::D2, Tr::comb(carry, r));
#pragma unroll
      for (int w = 0; w < MD_W; ++w) carry = Tr::comb(carry, s_w[w]);
      __syncthreads();
    }
    if (a.total && threadIdx.x == 0) put(a.total + row * C::D2, carry);
  } else {
    using Tr = TrMap<D>;
    __shared__ Map<D> s_w[MD_W];
    Mat<D> carry;
#pragma unroll
    for (int i = 0; i < C::D2; ++i) carry.f[i] = 0.0f;
    for (int64_t c1 = a.cpr; c1 > 0; c1 -= MD_TH) {
      // thread i holds chunk c1 - MD_TH + i
      const int64_t c = c1 - MD_TH + threadIdx.x;
      const bool ok = c >= 0;
      float *g = a.cagg + (row * a.cpr + c) * 2 * C::D2;
      Map<D> v = Tr::id();
      if (ok) {
        copy_in(v, g);
        zero<2 * C::D2>(g);
      }
      const Map<D> inc = wave_scan_rev<Tr>(v);
      if (lane == 0) s_w[wave] = inc;
      __syncthreads();
      Map<D> ex = shift_down1(inc);
      if (lane == WAVE - 1) ex = Tr::id();
      Mat<D> u = carry, t2;
      for (int w = MD_W - 1; w > wave; --w) {
        C::map_apply(s_w[w].f, u.f, t2.f);
        u = t2;
      }
      C::map_apply(ex.f, u.f, t2.f);
      if (ok) put(a.cvec + (row * a.cpr + c) * C::D2, t2);
#pragma unroll
      for (int w = MD_W - 1; w >= 0; --w) {
        C::map_apply(s_w[w].f, carry.f, t2.f);
        carry = t2;
      }
      __syncthreads();
    }
  }
}

// pass 4, forward: rescan every tile from its entry value, write P_i, and
// complete the saved tile prefix
template <int D>
__global__ __launch_bounds__(MD_TH) void k_md_apply(MdArgs a) {
  using C = MD<D>;
  using Tr = TrMat<D>;
  __shared__ float s_t[C::LDS];
  __shared__ Mat<D> s_w[MD_W];
  const int lane = lane_id(), wave = threadIdx.x / WAVE;
  const TileRange t = md_tile<D>(a, blockIdx.x);
  stage_in<D>(a.x + t.base * C::D2, t.valid * C::D2, s_t);
  __syncthreads();
  const Mat<D> inc = wave_scan_fwd<Tr>(thread_product<D>(s_t, t.valid));
  if (lane == WAVE - 1) s_w[wave] = inc;
  Mat<D> loc, cv;
  copy_in(loc, a.pre + blockIdx.x * C::D2);
  copy_in(cv, a.cvec + t.chunk * C::D2);
  Mat<D> cur = Tr::comb(cv, loc);  // exclusive prefix of the tile
  __syncthreads();
  if (threadIdx.x == 0) put(a.pre + blockIdx.x * C::D2, cur);
  for (int w = 0; w < wave; ++w) cur = Tr::comb(cur, s_w[w]);
  Mat<D> ex = shift_up1(inc);
  if (lane == 0) ex = Tr::id();
  cur = Tr::comb(cur, ex);
#pragma unroll
  for (int j = 0; j < C::TPT; ++j) {
    const int e = threadIdx.x * C::TPT + j;
    if (e >= t.valid) break;
    float *p = lds_el<D>(s_t, j);
    Mat<D> m;
    copy_in(m, p);
    cur = Tr::comb(cur, m);
    put(p, cur);
  }
  __syncthreads();
  stage_out<D>(a.y + t.base * C::D2, t.valid * C::D2, s_t, false);
}

// pass 4, adjoint: per tile, the adjoint entering every thread from the
// right, the forward prefixes from the saved tile prefix, and the serial
// right-to-left sweep writing Mbar
template <int D>
__global__ __launch_bounds__(MD_TH) void k_md_vapply(MdArgs a) {
  using C = MD<D>;
  __shared__ float s_t[C::LDS];
  __shared__ Map<D> s_w[MD_W];
  __shared__ Mat<D> s_f[MD_W];
  const int lane = lane_id(), wave = threadIdx.x / WAVE;
  const TileRange t = md_tile<D>(a, blockIdx.x);
  stage_in<D>(a.x + t.base * C::D2, t.valid * C::D2, s_t);
  __syncthreads();
  Mat<D> m[C::TPT];
#pragma unroll
  for (int j = 0; j < C::TPT; ++j) copy_in(m[j], lds_el<D>(s_t, j));
  __syncthreads();
  stage_pbar<D>(a, t, s_t);
  __syncthreads();

  // reverse side: rho entering this thread's last element from the right
  Mat<D> rho;
  {
    using Tr = TrMap<D>;
    const Map<D> inc = wave_scan_rev<Tr>(thread_map<D>(m, s_t, t.valid));
    if (lane == 0) s_w[wave] = inc;
    Map<D> h;
    Mat<D> cv;
    float *g = a.agg + blockIdx.x * 2 * C::D2;
    copy_in(h, g);
    copy_in(cv, a.cvec + t.chunk * C::D2);
    Mat<D> u, t2;
    C::map_apply(h.f, cv.f, u.f);  // the adjoint entering the tile
    __syncthreads();
    if (threadIdx.x == 0) zero<2 * C::D2>(g);  // consumed
    for (int w = MD_W - 1; w > wave; --w) {
      C::map_apply(s_w[w].f, u.f, t2.f);
      u = t2;
    }
    Map<D> ex = shift_down1(inc);
    if (lane == WAVE - 1) ex = Tr::id();
    C::map_apply(ex.f, u.f, rho.f);
  }
  // forward side: the prefix before each of the thread's elements
  Mat<D> pv[C::TPT];
  {
    using Tr = TrMat<D>;
    Mat<D> acc = Tr::id();
#pragma unroll
    for (int j = 0; j < C::TPT; ++j) {
      const int e = threadIdx.x * C::TPT + j;
      if (e >= t.valid) break;
      acc = j == 0 ? m[0] : Tr::comb(acc, m[j]);
    }
    const Mat<D> inc = wave_scan_fwd<Tr>(acc);
    if (lane == WAVE - 1) s_f[wave] = inc;
    Mat<D> cur;
    copy_in(cur, a.pre + blockIdx.x * C::D2);
    __syncthreads();
    for (int w = 0; w < wave; ++w) cur = Tr::comb(cur, s_f[w]);
    Mat<D> ex = shift_up1(inc);
    if (lane == 0) ex = Tr::id();
    pv[0] = Tr::comb(cur, ex);
#pragma unroll
    for (int j = 1; j < C::TPT; ++j) pv[j] = Tr::comb(pv[j - 1], m[j - 1]);
  }
  // right-to-left sweep: Rbar = Pbar + rho, Mbar = P_{i-1}^T Rbar, rho = Rbar M^T
#pragma unroll
  for (int j = C::TPT - 1; j >= 0; --j) {
    const int e = threadIdx.x * C::TPT + j;
    if (e >= t.valid) continue;
    float *p = lds_el<D>(s_t, j);
    Mat<D> rb, mb;
#pragma unroll
    for (int i = 0; i < C::D2; ++i) rb.f[i] = p[i] + rho.f[i];
    C::mul_at(pv[j].f, rb.f, mb.f);
    put(p, mb);
    C::mul_bt(rb.f, m[j].f, rho.f);
  }
  __syncthreads();
  stage_out<D>(a.y + t.base * C::D2, t.valid * C::D2, s_t, a.accumulate != 0);
}

// reduce forward: complete the saved tile prefixes (chunk prefix times the
// chunk-local prefix), which the scan forward does in its last pass
template <int D>
__global__ __launch_bounds__(256) void k_md_fix_pre(MdArgs a, int64_t tiles) {
  using Tr = TrMat<D>;
  constexpr int D2 = D * D;
  for (int64_t tile = (int64_t)blockIdx.x * 256 + threadIdx.x; tile < tiles;
       tile += (int64_t)gridDim.x * 256) {
    const int64_t row = tile / a.tpr, lt = tile - row * a.tpr;
    Mat<D> loc, cv;
    copy_in(loc, a.pre + tile * D2);
    copy_in(cv, a.cvec + (row * a.cpr + lt / MD_CH) * D2);
    put(a.pre + tile * D2, Tr::comb(cv, loc));
  }
}

// reduce of empty rows: the identity
__global__ __launch_bounds__(256) void k_md_eye(float *y, int64_t count, int d) {
  for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < count;
       i += (int64_t)gridDim.x * 256) {
    const int k = (int)(i % (d * d));
    y[i] = (k % (d + 1) == 0) ? 1.0f : 0.0f;
  }
}

__global__ __launch_bounds__(256) void k_md_zero(float *p, int64_t count) {
  for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < count;
       i += (int64_t)gridDim.x * 256)
    p[i] = 0.0f;
}

size_t al256(size_t x) { return (x + 255) / 256 * 256; }

int64_t md_tile_size(int d) { return d == 3 ? MD<3>::TILE : MD<5>::TILE; }

int64_t md_chunks(int d, int64_t batch, int64_t n) {
  const int64_t tile = md_tile_size(d);
  const int64_t tpr = (n + tile - 1) / tile;
  return batch * ((tpr + MD_CH - 1) / MD_CH);
}

}  // namespace

int64_t matd_tiles(int d, int64_t batch, int64_t n) {
  const int64_t tile = md_tile_size(d);
  return batch * ((n + tile - 1) / tile);
}

size_t matd_saved_bytes(int d, int64_t batch, int64_t n) {
  return (size_t)matd_tiles(d, batch, n) * d * d * 4;
}

size_t matd_ws_bytes(int d, int64_t batch, int64_t n) {
  const size_t tiles = (size_t)matd_tiles(d, batch, n);
  const size_t chunks = (size_t)md_chunks(d, batch, n);
  return kCtlBytes + al256(tiles * 2 * d * d * 4) + al256(chunks * 2 * d * d * 4) +
         al256(chunks * d * d * 4);
}

// reduce (forward): y = null, total = the row products; reduce (adjoint):
// pbar = null, ybar_last = Ybar per row
template <int D>
static hipError_t matd_run(bool vjp, int64_t batch, int64_t n, const float *x, const float *pbar,
                           float *y, float *saved, bool accumulate, void *ws, hipStream_t s,
                           float *total = nullptr, const float *ybar_last = nullptr) {
  constexpr int D2 = D * D;
  MdArgs a;
  a.x = x;
  a.pbar = pbar;
  a.y = y;
  a.pre = saved;
  a.total = total;
  a.ybar_last = ybar_last;
  a.n = n;
  a.tpr = (n + MD<D>::TILE - 1) / MD<D>::TILE;
  a.cpr = (a.tpr + MD_CH - 1) / MD_CH;
  a.accumulate = accumulate ? 1 : 0;
  const int64_t tiles = batch * a.tpr, chunks = batch * a.cpr;
  char *w = static_cast<char *>(ws) + kCtlBytes;
  a.agg = reinterpret_cast<float *>(w);
  w += al256((size_t)tiles * 2 * D2 * 4);
  a.cagg = reinterpret_cast<float *>(w);
  w += al256((size_t)chunks * 2 * D2 * 4);
  a.cvec = reinterpret_cast<float *>(w);
  if (tiles == 0) return hipSuccess;
  if (tiles > 2147483647LL || batch > 2147483647LL) return hipErrorInvalidValue;
  const dim3 gt((unsigned)tiles), gc((unsigned)chunks), gr((unsigned)batch), th(MD_TH);
  if (!vjp) {
    hipLaunchKernelGGL(k_md_agg<D>, gt, th, 0, s, a);
    hipLaunchKernelGGL((k_md_scan_tiles<D, false>), gc, th, 0, s, a);
    hipLaunchKernelGGL((k_md_scan_chunks<D, false>), gr, th, 0, s, a);
    if (total) {
      const int64_t fb = (tiles + 255) / 256;
      hipLaunchKernelGGL(k_md_fix_pre<D>, dim3((unsigned)(fb < 4096 ? fb : 4096)), dim3(256), 0,
                         s, a, tiles);
    } else {
      hipLaunchKernelGGL(k_md_apply<D>, gt, th, 0, s, a);
    }
  } else {
    hipLaunchKernelGGL(k_md_vagg<D>, gt, th, 0, s, a);
    hipLaunchKernelGGL((k_md_scan_tiles<D, true>), gc, th, 0, s, a);
    hipLaunchKernelGGL((k_md_scan_chunks<D, true>), gr, th, 0, s, a);
    hipLaunchKernelGGL(k_md_vapply<D>, gt, th, 0, s, a);
  }
  const int64_t zc = chunks * D2;
  const int64_t zb = (zc + 255) / 256;
  hipLaunchKernelGGL(k_md_zero, dim3((unsigned)(zb < 1024 ? zb : 1024)), dim3(256), 0, s, a.cvec,
                     zc);
  return hipGetLastError();
}

hipError_t matd_fwd_launch(int d, int64_t batch, int64_t n, const float *x, float *y,
                           float *saved, void *ws, hipStream_t s) {
  if (batch == 0 || n == 0) return hipSuccess;
  if (d == 3) return matd_run<3>(false, batch, n, x, nullptr, y, saved, false, ws, s);
  if (d == 5) return matd_run<5>(false, batch, n, x, nullptr, y, saved, false, ws, s);
  return hipErrorInvalidValue;
}

hipError_t matd_vjp_launch(int d, int64_t batch, int64_t n, const float *x, const float *saved,
                           const float *ybar, float *xbar, bool accumulate, void *ws,
                           hipStream_t s) {
  if (batch == 0 || n == 0) return hipSuccess;
  float *sv = const_cast<float *>(saved);  // read only in the adjoint passes
  if (d == 3) return matd_run<3>(true, batch, n, x, ybar, xbar, sv, accumulate, ws, s);
  if (d == 5) return matd_run<5>(true, batch, n, x, ybar, xbar, sv, accumulate, ws, s);
  return hipErrorInvalidValue;
}

hipError_t matd_reduce_fwd_launch(int d, int64_t batch, int64_t n, const float *x, float *y,
                                  float *saved, void *ws, hipStream_t s) {
  if (batch == 0) return hipSuccess;
  if (n == 0) {
    const int64_t cnt = batch * d * d, nb = (cnt + 255) / 256;
    hipLaunchKernelGGL(k_md_eye, dim3((unsigned)(nb < 4096 ? nb : 4096)), dim3(256), 0, s, y, cnt,
                       d);
    return hipGetLastError();
  }
  if (d == 3) return matd_run<3>(false, batch, n, x, nullptr, nullptr, saved, false, ws, s, y);
  if (d == 5) return matd_run<5>(false, batch, n, x, nullptr, nullptr, saved, false, ws, s, y);
  return hipErrorInvalidValue;
}

hipError_t matd_reduce_vjp_launch(int d, int64_t batch, int64_t n, const float *x,
                                  const float *saved, const float *ybar, float *xbar,
                                  bool accumulate, void *ws, hipStream_t s) {
  if (batch == 0 || n == 0) return hipSuccess;
  float *sv = const_cast<float *>(saved);
  if (d == 3)
    return matd_run<3>(true, batch, n, x, nullptr, xbar, sv, accumulate, ws, s, nullptr, ybar);
  if (d == 5)
    return matd_run<5>(true, batch, n, x, nullptr, xbar, sv, accumulate, ws, s, nullptr, ybar);
  return hipErrorInvalidValue;
}

}  // namespace pcad
