// Scans of d x d matrix products for d = 3 and 5 (the evaluation's matMul3x3
// and matMul5x5) and their adjoints, by the redundant block-diagonal
// sparsity of Section 5.3: the adjoint state of P_i is a d x d matrix Rbar_i
// and its recurrence is r -> Pbar_i + r M_{i+1}^T, an affine map with a d x d
// linear part, so an adjoint map carries 2 d^2 floats instead of the d^4 of a
// dense Jacobian.
//
// Elements are large (36 or 100 bytes), so these kernels reduce and then
// scan instead of looking back: per tile (TPT elements per thread) the
// ordered product (forward) or the composed adjoint map (reverse) of the
// tile, one block per row scanning the tile values (forward: exclusive
// prefixes, which are also the saved state; reverse: the adjoint entering
// each tile from the right), and a pass that rescans each tile from its
// entry value.  Inside a block the thread values are combined in LDS in
// element order.
//
//   forward : P_i = P_{i-1} M_i
//   adjoint : rho_i = (Pbar_i + rho_{i+1}) M_i^T carried right to left,
//             Rbar_i = Pbar_i + rho_{i+1},  Mbar_i = P_{i-1}^T Rbar_i
// Scratch words in the workspace (tile values) are zeroed by the pass that
// consumes them.
#include "device.hpp"
#include "internal.hpp"

namespace pcad {
namespace {

constexpr int MD_TH = 256;

template <int D>
struct MD {
  static constexpr int DIM = D;
  static constexpr int D2 = D * D;
  static constexpr int TPT = D == 3 ? 4 : 2;  // elements per thread
  static constexpr int TILE = MD_TH * TPT;
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

struct MdArgs {
  const float *x;      // M [rows][n][d*d]
  const float *pbar;   // adjoint input [rows][n][d*d]
  float *y;            // forward output / adjoint output
  float *pre;          // saved: exclusive prefix per tile [tiles][d*d]
  float *agg;          // workspace: tile values [tiles][2 d*d]
  float *rin;          // workspace: adjoint entering each tile [tiles][d*d]
  int64_t n;
  int64_t tpr;         // tiles per row
  int accumulate;
};

struct TileRange {
  int64_t row, lt, base;  // base: global element index of the tile's first element
  int valid;
};

template <int D>
__device__ __forceinline__ TileRange md_tile(const MdArgs &a, int64_t tile) {
  TileRange t;
  t.row = tile / a.tpr;
  t.lt = tile - t.row * a.tpr;
  const int64_t s = t.lt * MD<D>::TILE;
  t.base = t.row * a.n + s;
  const int64_t rem = a.n - s;
  t.valid = (int)(rem < MD<D>::TILE ? rem : MD<D>::TILE);
  return t;
}

// this thread's ordered product of its elements (identity past the end)
template <int D>
__device__ __forceinline__ void thread_product(const MdArgs &a, const TileRange &t, float *acc) {
  using C = MD<D>;
  C::eye(acc);
#pragma unroll
  for (int j = 0; j < C::TPT; ++j) {
    const int e = threadIdx.x * C::TPT + j;
    if (e >= t.valid) break;
    float m[C::D2], r[C::D2];
    const float *p = a.x + (t.base + e) * C::D2;
#pragma unroll
    for (int i = 0; i < C::D2; ++i) m[i] = p[i];
    C::mul(acc, m, r);
#pragma unroll
    for (int i = 0; i < C::D2; ++i) acc[i] = r[i];
  }
}

// this thread's composed adjoint map h_first o ... o h_last, h_i(r) = (Pbar_i + r) M_i^T
template <int D>
__device__ __forceinline__ void thread_map(const MdArgs &a, const TileRange &t, float *acc) {
  using C = MD<D>;
  C::map_id(acc);
#pragma unroll
  for (int j = C::TPT - 1; j >= 0; --j) {
    const int e = threadIdx.x * C::TPT + j;
    if (e >= t.valid) continue;
    float m[C::D2], h[2 * C::D2], r[2 * C::D2];
    const float *p = a.x + (t.base + e) * C::D2;
    const float *q = a.pbar + (t.base + e) * C::D2;
#pragma unroll
    for (int i = 0; i < C::D2; ++i) {
      m[i] = p[i];
      r[i] = q[i];
    }
    C::mul_bt(r, m, h);  // o = Pbar M^T
#pragma unroll
    for (int i = 0; i < D; ++i)
#pragma unroll
      for (int k = 0; k < D; ++k) h[C::D2 + i * D + k] = m[k * D + i];  // W = M^T
    C::map_comb(h, acc, r);
#pragma unroll
    for (int i = 0; i < 2 * C::D2; ++i) acc[i] = r[i];
  }
}

// In-order block scan of NF-float values in LDS (stride NF + 1).  FWD: the
// inclusive value of thread t combines threads 0..t (left to right);
// otherwise threads t..TH-1 with `comb(left, right)`.  Returns in `out` the
// inclusive value of thread t; the whole scan stays in `s` afterwards.
template <int NF, bool FWD, class Comb>
__device__ __forceinline__ void block_scan(float *s, const float *mine, float *out, Comb comb) {
  constexpr int ST = NF + 1;
  const int t = threadIdx.x;
  float v[NF];
#pragma unroll
  for (int i = 0; i < NF; ++i) {
    v[i] = mine[i];
    s[t * ST + i] = v[i];
  }
  __syncthreads();
  for (int d = 1; d < MD_TH; d <<= 1) {
    float r[NF];
    const int o = FWD ? t - d : t + d;
    const bool has = FWD ? (o >= 0) : (o < MD_TH);
    if (has) {
      float w[NF];
#pragma unroll
      for (int i = 0; i < NF; ++i) w[i] = s[o * ST + i];
      if (FWD) comb(w, v, r);  // earlier block of threads first
      else comb(v, w, r);
    }
    __syncthreads();
    if (has) {
#pragma unroll
      for (int i = 0; i < NF; ++i) {
        v[i] = r[i];
        s[t * ST + i] = r[i];
      }
    }
    __syncthreads();
  }
#pragma unroll
  for (int i = 0; i < NF; ++i) out[i] = v[i];
}

// forward pass 1: the ordered product of every tile
template <int D>
__global__ __launch_bounds__(MD_TH) void k_md_agg(MdArgs a) {
  using C = MD<D>;
  __shared__ float s[MD_TH * (C::D2 + 1)];
  const TileRange t = md_tile<D>(a, blockIdx.x);
  float acc[C::D2], incl[C::D2];
  thread_product<D>(a, t, acc);
  block_scan<C::D2, true>(s, acc, incl, [](const float *l, const float *r, float *o) { C::mul(l, r, o); });
  if (threadIdx.x == MD_TH - 1) {
#pragma unroll
    for (int i = 0; i < C::D2; ++i) a.agg[blockIdx.x * 2 * C::D2 + i] = incl[i];
  }
}

// forward pass 2 (one block per row): exclusive prefix of every tile
template <int D>
__global__ __launch_bounds__(MD_TH) void k_md_scan_tiles(MdArgs a) {
  using C = MD<D>;
  __shared__ float s[MD_TH * (C::D2 + 1)];
  const int64_t row = blockIdx.x;
  float carry[C::D2];
  C::eye(carry);
  for (int64_t c0 = 0; c0 < a.tpr; c0 += MD_TH) {
    const int64_t tl = c0 + threadIdx.x;
    float v[C::D2], incl[C::D2];
    if (tl < a.tpr) {
      float *g = a.agg + (row * a.tpr + tl) * 2 * C::D2;
#pragma unroll
      for (int i = 0; i < C::D2; ++i) {
        v[i] = g[i];
        g[i] = 0.0f;  // consumed
      }
    } else {
      C::eye(v);
    }
    block_scan<C::D2, true>(s, v, incl, [](const float *l, const float *r, float *o) { C::mul(l, r, o); });
    if (tl < a.tpr) {
      float ex[C::D2];
      if (threadIdx.x == 0) {
#pragma unroll
        for (int i = 0; i < C::D2; ++i) ex[i] = carry[i];
      } else {
        float w[C::D2];
#pragma unroll
        for (int i = 0; i < C::D2; ++i) w[i] = s[(threadIdx.x - 1) * (C::D2 + 1) + i];
        C::mul(carry, w, ex);
      }
#pragma unroll
      for (int i = 0; i < C::D2; ++i) a.pre[(row * a.tpr + tl) * C::D2 + i] = ex[i];
    }
    float last[C::D2], nc[C::D2];
#pragma unroll
    for (int i = 0; i < C::D2; ++i) last[i] = s[(MD_TH - 1) * (C::D2 + 1) + i];
    C::mul(carry, last, nc);
#pragma unroll
    for (int i = 0; i < C::D2; ++i) carry[i] = nc[i];
    __syncthreads();
  }
}

// forward pass 3: rescan every tile from its exclusive prefix and write P_i
template <int D>
__global__ __launch_bounds__(MD_TH) void k_md_apply(MdArgs a) {
  using C = MD<D>;
  __shared__ float s[MD_TH * (C::D2 + 1)];
  const TileRange t = md_tile<D>(a, blockIdx.x);
  float acc[C::D2], incl[C::D2];
  thread_product<D>(a, t, acc);
  block_scan<C::D2, true>(s, acc, incl, [](const float *l, const float *r, float *o) { C::mul(l, r, o); });
  float cur[C::D2], ex[C::D2];
  if (threadIdx.x == 0) {
    C::eye(ex);
  } else {
#pragma unroll
    for (int i = 0; i < C::D2; ++i) ex[i] = s[(threadIdx.x - 1) * (C::D2 + 1) + i];
  }
  float tp[C::D2];
#pragma unroll
  for (int i = 0; i < C::D2; ++i) tp[i] = a.pre[blockIdx.x * C::D2 + i];
  C::mul(tp, ex, cur);
#pragma unroll
  for (int j = 0; j < C::TPT; ++j) {
    const int e = threadIdx.x * C::TPT + j;
    if (e >= t.valid) break;
    float m[C::D2], r[C::D2];
    const float *p = a.x + (t.base + e) * C::D2;
#pragma unroll
    for (int i = 0; i < C::D2; ++i) m[i] = p[i];
    C::mul(cur, m, r);
    float *o = a.y + (t.base + e) * C::D2;
#pragma unroll
    for (int i = 0; i < C::D2; ++i) {
      cur[i] = r[i];
      o[i] = r[i];
    }
  }
}

// adjoint pass 1: the composed adjoint map of every tile
template <int D>
__global__ __launch_bounds__(MD_TH) void k_md_vagg(MdArgs a) {
  using C = MD<D>;
  __shared__ float s[MD_TH * (2 * C::D2 + 1)];
  const TileRange t = md_tile<D>(a, blockIdx.x);
  float acc[2 * C::D2], incl[2 * C::D2];
  thread_map<D>(a, t, acc);
  block_scan<2 * C::D2, false>(s, acc, incl,
                               [](const float *l, const float *r, float *o) { C::map_comb(l, r, o); });
  if (threadIdx.x == 0) {
#pragma unroll
    for (int i = 0; i < 2 * C::D2; ++i) a.agg[blockIdx.x * 2 * C::D2 + i] = incl[i];
  }
}

// adjoint pass 2 (one block per row, right to left): rin[t] = the adjoint
// handed into tile t from the tiles right of it
template <int D>
__global__ __launch_bounds__(MD_TH) void k_md_vscan_tiles(MdArgs a) {
  using C = MD<D>;
  __shared__ float s[MD_TH * (2 * C::D2 + 1)];
  const int64_t row = blockIdx.x;
  float carry[C::D2];
#pragma unroll
  for (int i = 0; i < C::D2; ++i) carry[i] = 0.0f;
  for (int64_t c1 = a.tpr; c1 > 0; c1 -= MD_TH) {
    // chunk [c1 - MD_TH, c1): thread i holds tile c1 - MD_TH + i
    const int64_t tl = c1 - MD_TH + threadIdx.x;
    float v[2 * C::D2], incl[2 * C::D2];
    if (tl >= 0) {
      float *g = a.agg + (row * a.tpr + tl) * 2 * C::D2;
#pragma unroll
      for (int i = 0; i < 2 * C::D2; ++i) {
        v[i] = g[i];
        g[i] = 0.0f;  // consumed
      }
    } else {
      C::map_id(v);
    }
    block_scan<2 * C::D2, false>(s, v, incl,
                                 [](const float *l, const float *r, float *o) { C::map_comb(l, r, o); });
    if (tl >= 0) {
      float r[C::D2];
      if (threadIdx.x == MD_TH - 1) {
#pragma unroll
        for (int i = 0; i < C::D2; ++i) r[i] = carry[i];
      } else {
        float h[2 * C::D2];
#pragma unroll
        for (int i = 0; i < 2 * C::D2; ++i) h[i] = s[(threadIdx.x + 1) * (2 * C::D2 + 1) + i];
        C::map_apply(h, carry, r);
      }
#pragma unroll
      for (int i = 0; i < C::D2; ++i) a.rin[(row * a.tpr + tl) * C::D2 + i] = r[i];
    }
    float h0[2 * C::D2], nc[C::D2];
#pragma unroll
    for (int i = 0; i < 2 * C::D2; ++i) h0[i] = s[i];
    C::map_apply(h0, carry, nc);
#pragma unroll
    for (int i = 0; i < C::D2; ++i) carry[i] = nc[i];
    __syncthreads();
  }
}

// adjoint pass 3: per tile, forward prefixes from the saved tile prefix, the
// adjoint entering each thread from the right, and the serial sweep
template <int D>
__global__ __launch_bounds__(MD_TH) void k_md_vapply(MdArgs a) {
  using C = MD<D>;
  __shared__ float s[MD_TH * (2 * C::D2 + 1)];
  const TileRange t = md_tile<D>(a, blockIdx.x);
  // forward side: the prefix before this thread's first element
  float fp[C::D2];
  {
    float acc[C::D2], incl[C::D2], ex[C::D2], tp[C::D2];
    thread_product<D>(a, t, acc);
    block_scan<C::D2, true>(s, acc, incl, [](const float *l, const float *r, float *o) { C::mul(l, r, o); });
    if (threadIdx.x == 0) {
      C::eye(ex);
    } else {
#pragma unroll
      for (int i = 0; i < C::D2; ++i) ex[i] = s[(threadIdx.x - 1) * (C::D2 + 1) + i];
    }
#pragma unroll
    for (int i = 0; i < C::D2; ++i) tp[i] = a.pre[blockIdx.x * C::D2 + i];
    C::mul(tp, ex, fp);
    __syncthreads();
  }
  // reverse side: rho entering this thread's last element from the right
  float rho[C::D2];
  {
    float acc[2 * C::D2], incl[2 * C::D2], rt[C::D2];
    thread_map<D>(a, t, acc);
    block_scan<2 * C::D2, false>(s, acc, incl,
                                 [](const float *l, const float *r, float *o) { C::map_comb(l, r, o); });
#pragma unroll
    for (int i = 0; i < C::D2; ++i) rt[i] = a.rin[blockIdx.x * C::D2 + i];
    if (threadIdx.x == MD_TH - 1) {
#pragma unroll
      for (int i = 0; i < C::D2; ++i) rho[i] = rt[i];
    } else {
      float h[2 * C::D2];
#pragma unroll
      for (int i = 0; i < 2 * C::D2; ++i) h[i] = s[(threadIdx.x + 1) * (2 * C::D2 + 1) + i];
      C::map_apply(h, rt, rho);
    }
    __syncthreads();
    if (threadIdx.x < C::D2) a.rin[blockIdx.x * C::D2 + threadIdx.x] = 0.0f;  // consumed
  }
  // forward prefixes of the thread's elements
  float pv[C::TPT][C::D2];
  {
    float cur[C::D2];
#pragma unroll
    for (int i = 0; i < C::D2; ++i) cur[i] = fp[i];
#pragma unroll
    for (int j = 0; j < C::TPT; ++j) {
#pragma unroll
      for (int i = 0; i < C::D2; ++i) pv[j][i] = cur[i];
      const int e = threadIdx.x * C::TPT + j;
      if (e < t.valid && j + 1 < C::TPT) {
        float m[C::D2], r[C::D2];
        const float *p = a.x + (t.base + e) * C::D2;
#pragma unroll
        for (int i = 0; i < C::D2; ++i) m[i] = p[i];
        C::mul(cur, m, r);
#pragma unroll
        for (int i = 0; i < C::D2; ++i) cur[i] = r[i];
      }
    }
  }
  // right-to-left sweep: Rbar = Pbar + rho, Mbar = P_{i-1}^T Rbar, rho = Rbar M^T
#pragma unroll
  for (int j = C::TPT - 1; j >= 0; --j) {
    const int e = threadIdx.x * C::TPT + j;
    if (e >= t.valid) continue;
    float m[C::D2], rb[C::D2], mb[C::D2];
    const float *p = a.x + (t.base + e) * C::D2;
    const float *q = a.pbar + (t.base + e) * C::D2;
#pragma unroll
    for (int i = 0; i < C::D2; ++i) {
      m[i] = p[i];
      rb[i] = q[i] + rho[i];
    }
    C::mul_at(pv[j], rb, mb);
    float *o = a.y + (t.base + e) * C::D2;
#pragma unroll
    for (int i = 0; i < C::D2; ++i) o[i] = a.accumulate ? o[i] + mb[i] : mb[i];
    C::mul_bt(rb, m, rho);
  }
}

}  // namespace

int64_t matd_tiles(int d, int64_t batch, int64_t n) {
  const int64_t tile = d == 3 ? MD<3>::TILE : MD<5>::TILE;
  return batch * ((n + tile - 1) / tile);
}

size_t matd_saved_bytes(int d, int64_t batch, int64_t n) {
  return (size_t)matd_tiles(d, batch, n) * d * d * 4;
}

size_t matd_ws_bytes(int d, int64_t batch, int64_t n) {
  const size_t tiles = (size_t)matd_tiles(d, batch, n);
  auto al = [](size_t x) { return (x + 255) / 256 * 256; };
  return kCtlBytes + al(tiles * 2 * d * d * 4) + al(tiles * d * d * 4);
}

template <int D>
static hipError_t matd_run(bool vjp, int64_t batch, int64_t n, const float *x, const float *pbar,
                           float *y, float *saved, bool accumulate, void *ws, hipStream_t s) {
  MdArgs a;
  a.x = x; a.pbar = pbar; a.y = y; a.pre = saved;
  a.n = n;
  a.tpr = (n + MD<D>::TILE - 1) / MD<D>::TILE;
  a.accumulate = accumulate ? 1 : 0;
  const int64_t tiles = batch * a.tpr;
  auto al = [](size_t v) { return (v + 255) / 256 * 256; };
  char *w = static_cast<char *>(ws) + kCtlBytes;
  a.agg = reinterpret_cast<float *>(w);
  a.rin = reinterpret_cast<float *>(w + al((size_t)tiles * 2 * D * D * 4));
  if (tiles == 0) return hipSuccess;
  if (tiles > 2147483647LL) return hipErrorInvalidValue;
  const dim3 gt((unsigned)tiles), gr((unsigned)batch);
  if (!vjp) {
    hipLaunchKernelGGL(k_md_agg<D>, gt, dim3(MD_TH), 0, s, a);
    hipLaunchKernelGGL(k_md_scan_tiles<D>, gr, dim3(MD_TH), 0, s, a);
    hipLaunchKernelGGL(k_md_apply<D>, gt, dim3(MD_TH), 0, s, a);
  } else {
    hipLaunchKernelGGL(k_md_vagg<D>, gt, dim3(MD_TH), 0, s, a);
    hipLaunchKernelGGL(k_md_vscan_tiles<D>, gr, dim3(MD_TH), 0, s, a);
    hipLaunchKernelGGL(k_md_vapply<D>, gt, dim3(MD_TH), 0, s, a);
  }
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

}  // namespace pcad
