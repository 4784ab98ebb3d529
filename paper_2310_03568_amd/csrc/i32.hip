// int32 forward combinators for + * min max (the evaluation's integer element
// types; forward only).  + and * wrap mod 2^32 in two's complement.  Integer
// + * min max are associative and commutative with exact results, so partial
// results combine in any order (block partials through atomics) and every
// result is bit-exact.
//
//   reduce : per block a partial over its chunk of the row (a serial pass per
//            thread, a wave butterfly, an LDS step across waves), then one
//            atomic into the row's result, initialised to the neutral element;
//   scan   : reduce-then-scan over tiles of 4096 elements -- tile totals, one
//            block per row scanning them, a rescan of every tile from its
//            exclusive prefix (workspace entries cleared after use);
//   reduce_by_index : LDS histograms of up to 8192 bins merged with one
//            atomic per non-neutral bin; one row of up to 131072 bins split
//            into 128 KB LDS tables, one block per (table, chunk); global
//            atomics beyond.
#include "device.hpp"
#include "internal.hpp"

namespace pcad {
namespace {

constexpr int I_TH = 256;
constexpr int I_EPT = 16;                  // scan elements per thread
constexpr int I_TILE = I_TH * I_EPT;       // scan tile
constexpr int kI32LdsBins = 8192;

template <int OP>
__device__ __forceinline__ int32_t ineutral() {
  return OP == ADD ? 0 : (OP == MUL ? 1 : (OP == MIN ? 0x7fffffff : (int32_t)0x80000000));
}

template <int OP>
__device__ __forceinline__ int32_t icomb(int32_t a, int32_t b) {
  if (OP == ADD) return (int32_t)((uint32_t)a + (uint32_t)b);
  if (OP == MUL) return (int32_t)((uint32_t)a * (uint32_t)b);
  if (OP == MIN) return a < b ? a : b;
  return a > b ? a : b;
}

// atomic combine into global or LDS memory
template <int OP>
__device__ __forceinline__ void iatomic(int32_t *p, int32_t v) {
  if (OP == ADD) atomicAdd(p, v);
  else if (OP == MIN) atomicMin(p, v);
  else if (OP == MAX) atomicMax(p, v);
  else {
    int32_t old = *p;
    for (;;) {
      const int32_t prev = atomicCAS(p, old, icomb<MUL>(old, v));
      if (prev == old) return;
      old = prev;
    }
  }
}

template <int OP>
__device__ __forceinline__ int32_t wave_fold(int32_t v) {
#pragma unroll
  for (int d = 1; d < WAVE; d <<= 1) v = icomb<OP>(v, __shfl_xor(v, d, WAVE));
  return v;
}

template <int OP>
__global__ __launch_bounds__(I_TH) void k_i32_fill(int32_t *y, int64_t count) {
  for (int64_t i = (int64_t)blockIdx.x * I_TH + threadIdx.x; i < count;
       i += (int64_t)gridDim.x * I_TH)
    y[i] = ineutral<OP>();
}

// grid (blocks per row, rows)
template <int OP>
__global__ __launch_bounds__(I_TH) void k_i32_reduce(const int32_t *x, int32_t *y, int64_t n) {
  __shared__ int32_t s_w[I_TH / WAVE];
  const int64_t row = blockIdx.y;
  const int32_t *xr = x + row * n;
  int32_t acc = ineutral<OP>();
  for (int64_t i = (int64_t)blockIdx.x * I_TH + threadIdx.x; i < n; i += (int64_t)gridDim.x * I_TH)
    acc = icomb<OP>(acc, xr[i]);
  acc = wave_fold<OP>(acc);
  if (lane_id() == 0) s_w[threadIdx.x / WAVE] = acc;
  __syncthreads();
  if (threadIdx.x == 0) {
    int32_t t = s_w[0];
#pragma unroll
    for (int w = 1; w < I_TH / WAVE; ++w) t = icomb<OP>(t, s_w[w]);
    if (t != ineutral<OP>()) iatomic<OP>(&y[row], t);
  }
}

// exclusive block scan of one int per thread (Hillis-Steele in LDS); returns
// the block total in *tot
template <int OP>
__device__ __forceinline__ int32_t block_excl(int32_t v, int32_t *s, int32_t *tot) {
  const int t = threadIdx.x;
  s[t] = v;
  __syncthreads();
  for (int d = 1; d < I_TH; d <<= 1) {
    const int32_t o = t >= d ? s[t - d] : ineutral<OP>();
    __syncthreads();
    if (t >= d) s[t] = icomb<OP>(o, s[t]);
    __syncthreads();
  }
  const int32_t ex = t > 0 ? s[t - 1] : ineutral<OP>();
  *tot = s[I_TH - 1];
  __syncthreads();
  return ex;
}

struct I32ScanArgs {
  const int32_t *x;
  int32_t *y;
  int32_t *agg;  // workspace: tile totals, then tile exclusive prefixes
  int64_t n, tpr;
};

// pass 1: every tile's total
template <int OP>
__global__ __launch_bounds__(I_TH) void k_i32_tiles(I32ScanArgs a) {
  __shared__ int32_t s_w[I_TH / WAVE];
  const int64_t tile = blockIdx.x;
  const int64_t row = tile / a.tpr, lt = tile - row * a.tpr;
  const int64_t s0 = lt * I_TILE;
  const int64_t e0 = s0 + I_TILE < a.n ? s0 + I_TILE : a.n;
  const int32_t *xr = a.x + row * a.n;
  int32_t acc = ineutral<OP>();
  for (int64_t i = s0 + threadIdx.x; i < e0; i += I_TH) acc = icomb<OP>(acc, xr[i]);
  acc = wave_fold<OP>(acc);
  if (lane_id() == 0) s_w[threadIdx.x / WAVE] = acc;
  __syncthreads();
  if (threadIdx.x == 0) {
    int32_t t = s_w[0];
#pragma unroll
    for (int w = 1; w < I_TH / WAVE; ++w) t = icomb<OP>(t, s_w[w]);
    a.agg[tile] = t;
  }
}

// pass 2 (one block per row): tile totals -> tile exclusive prefixes, in
// place; each thread takes TS consecutive tiles per round
template <int OP>
__global__ __launch_bounds__(I_TH) void k_i32_tile_scan(I32ScanArgs a) {
  constexpr int TS = 8;
  __shared__ int32_t s[I_TH];
  const int64_t row = blockIdx.x;
  int32_t *g = a.agg + row * a.tpr;
  int32_t carry = ineutral<OP>();
  for (int64_t c0 = 0; c0 < a.tpr; c0 += (int64_t)I_TH * TS) {
    const int64_t t0 = c0 + (int64_t)threadIdx.x * TS;
    int32_t v[TS];
    int32_t acc = ineutral<OP>();
#pragma unroll
    for (int j = 0; j < TS; ++j) {
      v[j] = t0 + j < a.tpr ? g[t0 + j] : ineutral<OP>();
      acc = icomb<OP>(acc, v[j]);
    }
    int32_t tot;
    int32_t run = icomb<OP>(carry, block_excl<OP>(acc, s, &tot));
#pragma unroll
    for (int j = 0; j < TS; ++j) {
      if (t0 + j < a.tpr) g[t0 + j] = run;
      run = icomb<OP>(run, v[j]);
    }
    carry = icomb<OP>(carry, tot);
  }
}

// pass 3: rescan every tile from its prefix; clears the prefix afterwards
template <int OP>
__global__ __launch_bounds__(I_TH) void k_i32_apply(I32ScanArgs a) {
  __shared__ int32_t s[I_TH];
  const int64_t tile = blockIdx.x;
  const int64_t row = tile / a.tpr, lt = tile - row * a.tpr;
  const int64_t s0 = lt * I_TILE + (int64_t)threadIdx.x * I_EPT;
  const int32_t *xr = a.x + row * a.n;
  int32_t *yr = a.y + row * a.n;
  int32_t v[I_EPT];
  int32_t acc = ineutral<OP>();
  if (((row * a.n) & 3) == 0 && s0 + I_EPT <= a.n) {
    // 16-byte loads (the row start and s0 are multiples of 4 elements)
#pragma unroll
    for (int q = 0; q < I_EPT / 4; ++q) {
      const int4 w = ld_stream<int4>(xr + s0 + 4 * q);
      v[4 * q] = w.x; v[4 * q + 1] = w.y; v[4 * q + 2] = w.z; v[4 * q + 3] = w.w;
    }
  } else {
#pragma unroll
    for (int j = 0; j < I_EPT; ++j) v[j] = s0 + j < a.n ? xr[s0 + j] : ineutral<OP>();
  }
#pragma unroll
  for (int j = 0; j < I_EPT; ++j) acc = icomb<OP>(acc, v[j]);
  const int32_t pre = a.agg[tile];
  int32_t tot;
  const int32_t ex = block_excl<OP>(acc, s, &tot);
  if (threadIdx.x == 0) a.agg[tile] = 0;  // every thread read it before block_excl's barriers
  int32_t run = icomb<OP>(pre, ex);
#pragma unroll
  for (int j = 0; j < I_EPT; ++j) {
    run = icomb<OP>(run, v[j]);
    v[j] = run;
  }
  if (((row * a.n) & 3) == 0 && s0 + I_EPT <= a.n) {
#pragma unroll
    for (int q = 0; q < I_EPT / 4; ++q)
      *reinterpret_cast<int4 *>(yr + s0 + 4 * q) =
          make_int4(v[4 * q], v[4 * q + 1], v[4 * q + 2], v[4 * q + 3]);
  } else {
#pragma unroll
    for (int j = 0; j < I_EPT; ++j)
      if (s0 + j < a.n) yr[s0 + j] = v[j];
  }
}

// reduce-by-index with a private LDS histogram per block (m <= kI32LdsBins)
template <int OP>
__global__ __launch_bounds__(I_TH) void k_i32_rbi_lds(const int32_t *idx, const int32_t *x,
                                                      int32_t *h, int64_t n, int m) {
  __shared__ int32_t s_h[kI32LdsBins];
  const int64_t row = blockIdx.y;
  for (int k = threadIdx.x; k < m; k += I_TH) s_h[k] = ineutral<OP>();
  __syncthreads();
  const int32_t *ir = idx + row * n;
  const int32_t *xr = x + row * n;
  for (int64_t i = (int64_t)blockIdx.x * I_TH + threadIdx.x; i < n; i += (int64_t)gridDim.x * I_TH) {
    const int32_t k = ir[i];
    if (k >= 0 && k < m) iatomic<OP>(&s_h[k], xr[i]);
  }
  __syncthreads();
  for (int k = threadIdx.x; k < m; k += I_TH) {
    const int32_t v = s_h[k];
    if (v != ineutral<OP>()) iatomic<OP>(&h[row * (int64_t)m + k], v);
  }
}

template <int OP>
__global__ __launch_bounds__(I_TH) void k_i32_rbi_global(const int32_t *idx, const int32_t *x,
                                                         int32_t *h, int64_t n, int64_t m) {
  const int64_t row = blockIdx.y;
  const int32_t *ir = idx + row * n;
  const int32_t *xr = x + row * n;
  for (int64_t i = (int64_t)blockIdx.x * I_TH + threadIdx.x; i < n; i += (int64_t)gridDim.x * I_TH) {
    const int32_t k = ir[i];
    if (k >= 0 && k < m) iatomic<OP>(&h[row * m + k], xr[i]);
  }
}

// one row with up to four 128 KB LDS tables' worth of bins: block (part,
// chunk) keeps the keys of its contiguous bin range in LDS and merges its
// non-neutral bins with global atomics; the blocks of a chunk sit on one
// XCD (blocks are dealt to the XCDs round robin), so the chunk is read from
// HBM about once
constexpr int I_PARTS_TH = 1024;
constexpr int kI32PartBins = 32768;  // 128 KB
constexpr int kI32Xcds = 8;

template <int OP>
__global__ __launch_bounds__(I_PARTS_TH) void k_i32_rbi_parts(const int32_t *idx, const int32_t *x,
                                                              int32_t *h, int64_t n, int64_t m,
                                                              int64_t chunk, int P) {
  __shared__ int32_t s_h[kI32PartBins];
  const int b = blockIdx.x;
  const int xcd = b % kI32Xcds, slot = b / kI32Xcds;
  const int c = xcd + kI32Xcds * (slot / P), p = slot % P;
  const int64_t kb0 = (int64_t)p * kI32PartBins;
  const int lim = (int)(m - kb0 < kI32PartBins ? m - kb0 : kI32PartBins);
  for (int k = threadIdx.x; k < kI32PartBins; k += I_PARTS_TH) s_h[k] = ineutral<OP>();
  __syncthreads();
  const int64_t lo = (int64_t)c * chunk;
  const int64_t hi = lo + chunk < n ? lo + chunk : n;
  for (int64_t i = lo + threadIdx.x; i < hi; i += I_PARTS_TH) {
    const int64_t k = (int64_t)idx[i] - kb0;
    if (k >= 0 && k < lim) iatomic<OP>(&s_h[k], x[i]);
  }
  __syncthreads();
  for (int k = threadIdx.x; k < lim; k += I_PARTS_TH) {
    const int32_t v = s_h[k];
    if (v != ineutral<OP>()) iatomic<OP>(&h[kb0 + k], v);
  }
}

size_t al256(size_t x) { return (x + 255) / 256 * 256; }

unsigned grid_cap(int64_t g, int64_t cap) { return (unsigned)(g < 1 ? 1 : (g > cap ? cap : g)); }

template <int OP>
hipError_t i32_run(int comb, int64_t batch, int64_t n, int64_t m, const int32_t *idx,
                   const int32_t *x, int32_t *y, void *ws, hipStream_t s) {
  if (comb == 0) {  // reduce
    hipLaunchKernelGGL(k_i32_fill<OP>, dim3(grid_cap((batch + I_TH - 1) / I_TH, 1024)), dim3(I_TH),
                       0, s, y, batch);
    if (n > 0) {
      const unsigned bx = grid_cap((n + I_TH * 64 - 1) / (I_TH * 64), 2048 / (batch < 2048 ? batch : 2048));
      hipLaunchKernelGGL(k_i32_reduce<OP>, dim3(bx, (unsigned)batch), dim3(I_TH), 0, s, x, y, n);
    }
  } else if (comb == 1) {  // scan
    if (n == 0) return hipSuccess;
    I32ScanArgs a;
    a.x = x; a.y = y; a.n = n;
    a.tpr = (n + I_TILE - 1) / I_TILE;
    a.agg = reinterpret_cast<int32_t *>(static_cast<char *>(ws) + kCtlBytes);
    const int64_t tiles = batch * a.tpr;
    hipLaunchKernelGGL(k_i32_tiles<OP>, dim3((unsigned)tiles), dim3(I_TH), 0, s, a);
    hipLaunchKernelGGL(k_i32_tile_scan<OP>, dim3((unsigned)batch), dim3(I_TH), 0, s, a);
    hipLaunchKernelGGL(k_i32_apply<OP>, dim3((unsigned)tiles), dim3(I_TH), 0, s, a);
  } else {  // reduce_by_index
    if (m == 0) return hipSuccess;
    const int64_t total = batch * m;
    hipLaunchKernelGGL(k_i32_fill<OP>, dim3(grid_cap((total + I_TH - 1) / I_TH, 16384)), dim3(I_TH),
                       0, s, y, total);
    if (n > 0) {
      if (m <= kI32LdsBins) {
        const unsigned bx = grid_cap((n + 16383) / 16384, 2048 / (batch < 2048 ? batch : 2048));
        hipLaunchKernelGGL(k_i32_rbi_lds<OP>, dim3(bx, (unsigned)batch), dim3(I_TH), 0, s, idx, x, y,
                           n, (int)m);
      } else if (batch == 1 && m <= 4 * kI32PartBins) {
        const int P = (int)((m + kI32PartBins - 1) / kI32PartBins);
        int64_t cl = 32 / P;
        const int64_t want = (n + (int64_t)kI32Xcds * 65536 - 1) / ((int64_t)kI32Xcds * 65536);
        if (cl > want) cl = want;
        if (cl < 1) cl = 1;
        const int64_t C = kI32Xcds * cl;
        const int64_t chunk = (n + C - 1) / C;
        hipLaunchKernelGGL(k_i32_rbi_parts<OP>, dim3((unsigned)(C * P)), dim3(I_PARTS_TH), 0, s, idx,
                           x, y, n, m, chunk, P);
      } else {
        const unsigned bx = grid_cap((n + I_TH * 16 - 1) / (I_TH * 16), 65535 / (batch < 65535 ? batch : 65535));
        hipLaunchKernelGGL(k_i32_rbi_global<OP>, dim3(bx, (unsigned)batch), dim3(I_TH), 0, s, idx, x,
                           y, n, m);
      }
    }
  }
  return hipGetLastError();
}

}  // namespace

int64_t i32_scan_tiles(int64_t batch, int64_t n) { return batch * ((n + I_TILE - 1) / I_TILE); }

size_t i32_ws_bytes(int comb, int64_t batch, int64_t n) {
  if (comb != 1 || batch == 0 || n == 0) return 0;
  return kCtlBytes + al256((size_t)i32_scan_tiles(batch, n) * 4);
}

hipError_t i32_fwd_launch(int comb, int op, int64_t batch, int64_t n, int64_t m,
                          const int32_t *idx, const int32_t *x, int32_t *y, void *ws,
                          hipStream_t s) {
  if (batch == 0) return hipSuccess;
  switch (op) {
  case ADD: return i32_run<ADD>(comb, batch, n, m, idx, x, y, ws, s);
  case MUL: return i32_run<MUL>(comb, batch, n, m, idx, x, y, ws, s);
  case MIN: return i32_run<MIN>(comb, batch, n, m, idx, x, y, ws, s);
  case MAX: return i32_run<MAX>(comb, batch, n, m, idx, x, y, ws, s);
  }
  return hipErrorInvalidValue;
}

}  // namespace pcad
