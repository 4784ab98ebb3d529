// Partitioned reduce-by-index (Section 4) for + * min max and sumOfProd
// (Section 3.3, applied to reduce-by-index in Section 4.2) when the bins do
// not fit one LDS histogram.  The paper's construct handles large
// histograms with a multi-pass technique: each pass re-reads the input and
// updates one partition of the bins.  Here the input is partitioned once
// instead, so every later step works on one LDS-sized bin range:
//
//   bins are cut into buckets of W consecutive bins (W * element <= 64 KB);
//   1. count   -- elements per (bucket, input block), counted in LDS;
//   2. offsets -- an exclusive scan of the counts in bucket-major order gives
//                 every input block its output position per bucket; a
//                 one-block pass turns the bucket totals into work items of
//                 at most T elements (buckets with more are split, so skewed
//                 keys spread over many blocks);
//   3. scatter -- each in-range element goes to its bucket's region as a
//                 record (bin, value); for min/max (bin, packed key);
//   4. bins    -- one block per work item builds the bucket's LDS histogram
//                 from the item's records.  The only item of a bucket writes
//                 the final bins (and the saved state) itself; the items of a
//                 split bucket write partial histograms, which a last pass
//                 folds in item order.
//
// There are no global atomics.  Ranks within a block come from LDS atomics;
// the lanes of a wave that share the first active lane's bucket (the hot
// bucket under skewed keys) take one atomic together.  The scatter stages
// each round of records in LDS in bucket order, so its global writes leave
// as contiguous runs per bucket rather than single records.
//
// Workspace data left behind never looks like a look-back status word
// (whose upper 32 bits are a tag in [1, 2^31)): every 8-byte word of the
// records and of the item table has its upper half >= 2^31; the counts, the
// scan's block totals and the partial histograms are zeroed once read.
#include "device.hpp"
#include "internal.hpp"

namespace pcad {
namespace {

constexpr int PT_TH = 512;          // count / scatter block
constexpr int PH_TH = 1024;         // histogram block
constexpr int PC_TH = 256;          // fold block
constexpr int PT_NB_MAX = 2048;     // buckets
constexpr int64_t PT_ITEMS = 512;   // target work items per row
constexpr int64_t PT_MIN_T = 8192;  // smallest work item
constexpr uint32_t kHi = 0x80000000u;

// log2 of the bucket width: 64 KB of LDS per bucket
template <int OP>
constexpr int part_lw() {
  return OP == ADD ? 14 : 13;  // + : 16384 floats; * : 8192 (count, product); min/max: 8192 keys;
                               // sumOfProd: 8192 (p, s) pairs
}

int part_lw_rt(int op) { return op == ADD ? 14 : 13; }

struct PartArgs {
  const int32_t *idx;
  const float *v;
  int64_t n, m;
  int nbk;             // buckets
  int nb1;             // count / scatter blocks
  int64_t ch;          // elements per count / scatter block (multiple of 4*PT_TH)
  int64_t T;           // largest work item
  bool vec;            // idx and v 16-byte aligned
  uint32_t *counts;    // nbk*nb1 + 1 entries
  uint64_t *rec;       // records, 8 or 16 bytes each
  uint64_t *tab;       // [0] items; per bucket 5 words: start, count, first item, items, first slot
  void *partial;       // partial histograms: slot-major, W entries per slot
  float *hist;
  uint32_t *n0;
  float *ypos;
  int32_t *argk;
  float *ssum;
};

__device__ __forceinline__ uint64_t tword(uint32_t x) { return ((uint64_t)0xffffffffu << 32) | x; }
__device__ __forceinline__ uint32_t tval(const uint64_t *t, int64_t i) { return (uint32_t)t[i]; }

__device__ __forceinline__ uint64_t lanes_below() {
  const int lane = lane_id();
  return lane == 0 ? 0ull : (~0ull >> (WAVE - lane));
}

// cnt[d] += 1 for every lane with ok; returns the lane's old value (its rank
// among this block's elements of bucket d).  The lanes whose bucket equals
// the first active lane's are served by one atomic.
template <bool RET>
__device__ __forceinline__ uint32_t lds_count(uint32_t *cnt, uint32_t d, bool ok) {
  const uint64_t act = __ballot(ok);
  if (act == 0) return 0u;
  const int first = __builtin_ctzll(act);
  const uint32_t d0 = (uint32_t)__builtin_amdgcn_readlane((int)d, first);
  const bool hot = ok && d == d0;
  const uint64_t hm = __ballot(hot);
  uint32_t r = 0;
  if (lane_id() == first) {
    if (RET) r = atomicAdd(&cnt[d0], (uint32_t)__popcll(hm));
    else atomicAdd(&cnt[d0], (uint32_t)__popcll(hm));
  }
  if (RET) r = (uint32_t)__builtin_amdgcn_readlane((int)r, first) + (uint32_t)__popcll(hm & lanes_below());
  if (ok && !hot) {
    if (RET) r = atomicAdd(&cnt[d], 1u);
    else atomicAdd(&cnt[d], 1u);
  }
  return r;
}

// four consecutive (key, value) pairs of the block's chunk starting at i
__device__ __forceinline__ void load4(const PartArgs &a, int64_t i, int64_t hi, bool with_v,
                                      int32_t k[4], float x[4]) {
  if (a.vec && i + 4 <= hi) {
    const int4 k4 = ld_stream<int4>(a.idx + i);
    k[0] = k4.x; k[1] = k4.y; k[2] = k4.z; k[3] = k4.w;
    if (with_v) {
      const float4 v4 = ld_stream<float4>(a.v + i);
      x[0] = v4.x; x[1] = v4.y; x[2] = v4.z; x[3] = v4.w;
    }
  } else {
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      k[j] = i + j < hi ? a.idx[i + j] : -1;
      if (with_v) x[j] = i + j < hi ? a.v[i + j] : 0.0f;
    }
  }
}

__global__ __launch_bounds__(PT_TH) void k_part_count(PartArgs a, int lw) {
  __shared__ uint32_t s_c[PT_NB_MAX];
  for (int b = threadIdx.x; b < a.nbk; b += PT_TH) s_c[b] = 0u;
  __syncthreads();
  const int64_t lo = (int64_t)blockIdx.x * a.ch;
  const int64_t hi = lo + a.ch < a.n ? lo + a.ch : a.n;
  for (int64_t i = lo + (int64_t)threadIdx.x * 4; i - (int64_t)threadIdx.x * 4 < hi;
       i += (int64_t)PT_TH * 4) {
    int32_t k[4];
    float x[4];
    load4(a, i, hi, false, k, x);
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const bool ok = k[j] >= 0 && k[j] < a.m;
      lds_count<false>(s_c, ok ? (uint32_t)k[j] >> lw : 0u, ok);
    }
  }
  __syncthreads();
  for (int b = threadIdx.x; b < a.nbk; b += PT_TH)
    a.counts[(int64_t)b * a.nb1 + blockIdx.x] = s_c[b];
  if (blockIdx.x == 0 && threadIdx.x == 0) a.counts[(int64_t)a.nbk * a.nb1] = 0u;
}

// one block: bucket starts and sizes from the scanned counts, then work items
// (q_b = max(1, ceil(c_b / T))) and partial-histogram slots (q_b of them for
// a split bucket) by exclusive scans over the buckets
constexpr int PI_TH = 1024;
constexpr int PI_PER = PT_NB_MAX / PI_TH;

__device__ __forceinline__ uint32_t block_excl(uint32_t x, uint32_t *s_w, uint32_t *total) {
  const int lane = lane_id(), wave = threadIdx.x / WAVE;
  uint32_t inc = x;
#pragma unroll
  for (int d = 1; d < WAVE; d <<= 1) {
    const uint32_t o = __shfl_up(inc, d, WAVE);
    if (lane >= d) inc += o;
  }
  if (lane == WAVE - 1) s_w[wave] = inc;
  __syncthreads();
  if (threadIdx.x == 0) {
    uint32_t run = 0;
    for (int w = 0; w < PI_TH / WAVE; ++w) {
      const uint32_t t = s_w[w];
      s_w[w] = run;
      run += t;
    }
    s_w[PI_TH / WAVE] = run;
  }
  __syncthreads();
  const uint32_t r = s_w[wave] + inc - x;
  *total = s_w[PI_TH / WAVE];
  __syncthreads();
  return r;
}

__global__ __launch_bounds__(PI_TH) void k_part_items(PartArgs a) {
  __shared__ uint32_t s_w[PI_TH / WAVE + 1];
  uint32_t st[PI_PER], c[PI_PER], q[PI_PER], sq = 0, ss = 0;
#pragma unroll
  for (int j = 0; j < PI_PER; ++j) {
    const int b = threadIdx.x * PI_PER + j;
    st[j] = c[j] = 0u;
    q[j] = 0u;
    if (b < a.nbk) {
      st[j] = a.counts[(int64_t)b * a.nb1];
      c[j] = a.counts[(int64_t)(b + 1) * a.nb1] - st[j];
      const uint32_t qq = (uint32_t)((c[j] + a.T - 1) / a.T);
      q[j] = qq > 1u ? qq : 1u;
    }
    sq += q[j];
    ss += q[j] > 1u ? q[j] : 0u;
  }
  uint32_t nitems, nslots;
  uint32_t iq = block_excl(sq, s_w, &nitems);
  uint32_t is = block_excl(ss, s_w, &nslots);
#pragma unroll
  for (int j = 0; j < PI_PER; ++j) {
    const int b = threadIdx.x * PI_PER + j;
    if (b < a.nbk) {
      uint64_t *t = a.tab + 1 + (int64_t)b * 5;
      t[0] = tword(st[j]);
      t[1] = tword(c[j]);
      t[2] = tword(iq);
      t[3] = tword(q[j]);
      t[4] = tword(is);
    }
    iq += q[j];
    is += q[j] > 1u ? q[j] : 0u;
  }
  if (threadIdx.x == 0) a.tab[0] = tword(nitems);
}

// exclusive scan of in[0..nb) into out (nb <= PT_NB_MAX), by a PT_TH block;
// returns the total
__device__ __forceinline__ uint32_t block_scan_buckets(const uint32_t *in, uint32_t *out, int nb,
                                                       uint32_t *s_w) {
  constexpr int PER = PT_NB_MAX / PT_TH;
  const int lane = lane_id(), wave = threadIdx.x / WAVE;
  const int b0 = threadIdx.x * PER;
  uint32_t x[PER], sum = 0;
#pragma unroll
  for (int j = 0; j < PER; ++j) {
    x[j] = b0 + j < nb ? in[b0 + j] : 0u;
    sum += x[j];
  }
  uint32_t inc = sum;
#pragma unroll
  for (int d = 1; d < WAVE; d <<= 1) {
    const uint32_t o = __shfl_up(inc, d, WAVE);
    if (lane >= d) inc += o;
  }
  if (lane == WAVE - 1) s_w[wave] = inc;
  __syncthreads();
  uint32_t before = 0, total = 0;
#pragma unroll
  for (int w = 0; w < PT_TH / WAVE; ++w) {
    const uint32_t t = s_w[w];
    before += w < wave ? t : 0u;
    total += t;
  }
  uint32_t run = before + inc - sum;
#pragma unroll
  for (int j = 0; j < PER; ++j) {
    if (b0 + j < nb) out[b0 + j] = run;
    run += x[j];
  }
  return total;
}

// records: + and * (bin | 2^31, value bits); min/max (lo32(key), bin | 2^31)
// then (hi32(key), bin | 2^31).  Each round of R elements is ranked per
// bucket, staged in LDS in bucket order with its destinations, and written
// out in stage order.
template <int OP>
__global__ __launch_bounds__(PT_TH) void k_part_scatter(PartArgs a, int lw) {
  constexpr bool KEYS = OP == MIN || OP == MAX;
  constexpr int R = KEYS ? 2048 : 4096;  // elements per round
  constexpr int G = R / (PT_TH * 4);     // int4 groups per thread and round
  __shared__ uint32_t s_gb[PT_NB_MAX];   // the block's next output position per bucket
  __shared__ uint32_t s_rc[PT_NB_MAX];   // this round's count per bucket
  __shared__ uint32_t s_ro[PT_NB_MAX];   // this round's stage offset per bucket
  __shared__ uint32_t s_dst[R];
  __shared__ uint64_t s_st[KEYS ? 2 * R : R];
  __shared__ uint32_t s_w[PT_TH / WAVE];
  for (int b = threadIdx.x; b < a.nbk; b += PT_TH) {
    const int64_t e = (int64_t)b * a.nb1 + blockIdx.x;
    s_gb[b] = a.counts[e];
    a.counts[e] = 0u;
    s_rc[b] = 0u;
  }
  if (blockIdx.x == 0 && threadIdx.x == 0) a.counts[(int64_t)a.nbk * a.nb1] = 0u;
  __syncthreads();
  const int64_t lo = (int64_t)blockIdx.x * a.ch;
  const int64_t hi = lo + a.ch < a.n ? lo + a.ch : a.n;
  for (int64_t r0 = lo; r0 < hi; r0 += R) {
    int32_t k[G][4];
    float x[G][4];
    uint32_t rk[G][4];
#pragma unroll
    for (int g = 0; g < G; ++g) {
      const int64_t i = r0 + (int64_t)g * PT_TH * 4 + (int64_t)threadIdx.x * 4;
      load4(a, i, hi, true, k[g], x[g]);
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        const bool ok = k[g][j] >= 0 && k[g][j] < a.m;
        rk[g][j] = lds_count<true>(s_rc, ok ? (uint32_t)k[g][j] >> lw : 0u, ok);
      }
    }
    __syncthreads();
    const uint32_t nr = block_scan_buckets(s_rc, s_ro, a.nbk, s_w);
    __syncthreads();
#pragma unroll
    for (int g = 0; g < G; ++g) {
      const int64_t i = r0 + (int64_t)g * PT_TH * 4 + (int64_t)threadIdx.x * 4;
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        if (k[g][j] < 0 || k[g][j] >= a.m) continue;
        const uint32_t d = (uint32_t)k[g][j] >> lw;
        const uint32_t slot = s_ro[d] + rk[g][j];
        const uint32_t kb = (uint32_t)k[g][j] | kHi;
        s_dst[slot] = s_gb[d] + rk[g][j];
        if (KEYS) {
          const uint64_t key = key_of<OP>(x[g][j], (uint32_t)(i + j));
          s_st[2 * slot] = ((uint64_t)kb << 32) | (uint32_t)key;
          s_st[2 * slot + 1] = ((uint64_t)kb << 32) | (uint32_t)(key >> 32);
        } else {
          s_st[slot] = ((uint64_t)kb << 32) | __float_as_uint(x[g][j]);
        }
      }
    }
    __syncthreads();
    for (uint32_t t = threadIdx.x; t < nr; t += PT_TH) {
      if (KEYS) {
        const uint64_t w0 = s_st[2 * t], w1 = s_st[2 * t + 1];
        uint4 r;
        r.x = (uint32_t)w0; r.y = (uint32_t)(w0 >> 32); r.z = (uint32_t)w1; r.w = (uint32_t)(w1 >> 32);
        reinterpret_cast<uint4 *>(a.rec)[s_dst[t]] = r;
      } else {
        a.rec[s_dst[t]] = s_st[t];
      }
    }
    for (int b = threadIdx.x; b < a.nbk; b += PT_TH) {
      s_gb[b] += s_rc[b];
      s_rc[b] = 0u;
    }
    __syncthreads();
  }
}

// the final value of bin g (global bin index) from its folded state
template <int OP>
__device__ __forceinline__ void put_bin(const PartArgs &a, int64_t g, float f, uint32_t cnt,
                                        uint64_t key) {
  if (OP == ADD) a.hist[g] = f;
  if (OP == MUL) {
    a.n0[g] = cnt;
    a.ypos[g] = f;
    a.hist[g] = cnt > 0u ? 0.0f : f;
  }
  if (OP == SUMPROD) {
    const SP r = sp_unpack(key);
    a.hist[g] = r.p;
    a.ssum[g] = r.s;
  }
  if (OP == MIN || OP == MAX) {
    if (key == key_init<OP>()) {
      a.argk[g] = (int32_t)a.n;
      a.hist[g] = OP == MIN ? __builtin_inff() : -__builtin_inff();
    } else {
      const uint32_t lo = (uint32_t)key;
      const uint32_t i = OP == MIN ? lo : ~lo;
      a.argk[g] = (int32_t)i;
      a.hist[g] = a.v[i];
    }
  }
}

template <int OP>
__global__ __launch_bounds__(PH_TH) void k_part_hist(PartArgs a) {
  constexpr int LW = part_lw<OP>();
  constexpr int W = 1 << LW;
  constexpr bool KEYS = OP == MIN || OP == MAX;
  __shared__ float s_f[KEYS ? 1 : W];
  __shared__ uint32_t s_c[OP == MUL ? W : 1];
  __shared__ unsigned long long s_k[KEYS ? W : 1];
  const uint32_t t = blockIdx.x;
  if (t >= tval(a.tab, 0)) return;
  const uint64_t *tb = a.tab + 1;
  // the bucket of item t: the last bucket whose first item is <= t
  int lo = 0, hi = a.nbk - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (tval(tb, (int64_t)mid * 5 + 2) <= t) lo = mid;
    else hi = mid - 1;
  }
  const int b = lo;
  const uint32_t start = tval(tb, (int64_t)b * 5), cnt = tval(tb, (int64_t)b * 5 + 1);
  const uint32_t j = t - tval(tb, (int64_t)b * 5 + 2), q = tval(tb, (int64_t)b * 5 + 3);
  const uint32_t per = q > 1u ? (cnt + q - 1u) / q : cnt;
  const int64_t e0 = (int64_t)start + (int64_t)j * per;
  const int64_t e1 = e0 + per < (int64_t)start + cnt ? e0 + per : (int64_t)start + cnt;
  for (int i = threadIdx.x; i < W; i += PH_TH) {
    if (OP == ADD) s_f[i] = 0.0f;
    if (OP == MUL) { s_f[i] = 1.0f; s_c[i] = 0u; }
    if (KEYS) s_k[i] = key_init<OP>();
  }
  __syncthreads();
  constexpr int U = 4;
  for (int64_t p0 = e0 + threadIdx.x; p0 < e1; p0 += (int64_t)PH_TH * U) {
    uint64_t r0[U], r1[U];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int64_t p = p0 + (int64_t)u * PH_TH;
      r0[u] = r1[u] = 0;
      if (p < e1) {
        if (KEYS) {
          const uint4 r = reinterpret_cast<const uint4 *>(a.rec)[p];
          r0[u] = ((uint64_t)r.y << 32) | r.x;
          r1[u] = r.z;
        } else {
          r0[u] = a.rec[p];
        }
      }
    }
#pragma unroll
    for (int u = 0; u < U; ++u) {
      if (p0 + (int64_t)u * PH_TH >= e1) break;
      const uint32_t bin = (uint32_t)(r0[u] >> 32) & (uint32_t)(W - 1);
      if (OP == ADD) lds_add_f32(&s_f[bin], __uint_as_float((uint32_t)r0[u]));
      if (OP == MUL) {
        const float x = __uint_as_float((uint32_t)r0[u]);
        if (x == 0.0f) atomicAdd(&s_c[bin], 1u);
        else {
          unsigned *w = reinterpret_cast<unsigned *>(&s_f[bin]);
          unsigned old = __hip_atomic_load(w, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
          for (;;) {
            const unsigned nw = __float_as_uint(__uint_as_float(old) * x);
            if (__hip_atomic_compare_exchange_strong(w, &old, nw, __ATOMIC_RELAXED, __ATOMIC_RELAXED,
                                                     __HIP_MEMORY_SCOPE_WORKGROUP))
              break;
          }
        }
      }
      if (KEYS) {
        const unsigned long long key = (r1[u] << 32) | (uint32_t)r0[u];
        if (OP == MIN) atomicMin(&s_k[bin], key);
        else atomicMax(&s_k[bin], key);
      }
    }
  }
  __syncthreads();
  const int64_t g0 = (int64_t)b << LW;
  const int nb = a.m - g0 < W ? (int)(a.m - g0) : W;
  if (q == 1u) {
    for (int i = threadIdx.x; i < nb; i += PH_TH)
      put_bin<OP>(a, g0 + i, KEYS ? 0.0f : s_f[i], OP == MUL ? s_c[i] : 0u,
                  KEYS ? s_k[i] : 0ull);
  } else {
    const int64_t slot = (int64_t)tval(tb, (int64_t)b * 5 + 4) + j;
    for (int i = threadIdx.x; i < nb; i += PH_TH) {
      if (OP == ADD) static_cast<float *>(a.partial)[slot * W + i] = s_f[i];
      if (OP == MUL)
        static_cast<uint2 *>(a.partial)[slot * W + i] = make_uint2(s_c[i], __float_as_uint(s_f[i]));
      if (KEYS) static_cast<uint64_t *>(a.partial)[slot * W + i] = s_k[i];
    }
  }
}

// sumOfProd: the bucket's LDS table of packed (p, s) pairs; every lane of
// the block takes every round (sp_wave_update works on whole waves)
__global__ __launch_bounds__(PH_TH) void k_part_hist_sp(PartArgs a) {
  constexpr int LW = part_lw<SUMPROD>();
  constexpr int W = 1 << LW;
  __shared__ uint64_t s_t[W];
  const uint32_t t = blockIdx.x;
  if (t >= tval(a.tab, 0)) return;
  const uint64_t *tb = a.tab + 1;
  int lo = 0, hi = a.nbk - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (tval(tb, (int64_t)mid * 5 + 2) <= t) lo = mid;
    else hi = mid - 1;
  }
  const int b = lo;
  const uint32_t start = tval(tb, (int64_t)b * 5), cnt = tval(tb, (int64_t)b * 5 + 1);
  const uint32_t j = t - tval(tb, (int64_t)b * 5 + 2), q = tval(tb, (int64_t)b * 5 + 3);
  const uint32_t per = q > 1u ? (cnt + q - 1u) / q : cnt;
  const int64_t e0 = (int64_t)start + (int64_t)j * per;
  const int64_t e1 = e0 + per < (int64_t)start + cnt ? e0 + per : (int64_t)start + cnt;
  for (int i = threadIdx.x; i < W; i += PH_TH) s_t[i] = 0ull;
  __syncthreads();
  for (int64_t p = e0 + threadIdx.x; p - threadIdx.x < e1; p += PH_TH) {
    const bool ok = p < e1;
    const uint64_t r = ok ? a.rec[p] : 0ull;
    sp_wave_update(s_t, (uint32_t)(r >> 32) & (uint32_t)(W - 1), __uint_as_float((uint32_t)r), ok);
  }
  __syncthreads();
  const int64_t g0 = (int64_t)b << LW;
  const int nb = a.m - g0 < W ? (int)(a.m - g0) : W;
  if (q == 1u) {
    for (int i = threadIdx.x; i < nb; i += PH_TH) put_bin<SUMPROD>(a, g0 + i, 0.0f, 0u, s_t[i]);
  } else {
    const int64_t slot = (int64_t)tval(tb, (int64_t)b * 5 + 4) + j;
    for (int i = threadIdx.x; i < nb; i += PH_TH)
      static_cast<uint64_t *>(a.partial)[slot * W + i] = s_t[i];
  }
}

// split buckets: fold the partial histograms in item order, then zero them
template <int OP>
__global__ __launch_bounds__(PC_TH) void k_part_fold(PartArgs a) {
  constexpr int LW = part_lw<OP>();
  constexpr int W = 1 << LW;
  constexpr bool KEYS = OP == MIN || OP == MAX;
  const int i = blockIdx.x * PC_TH + threadIdx.x;
  const uint64_t *tb = a.tab + 1;
  for (int b = blockIdx.y; b < a.nbk; b += gridDim.y) {
    const uint32_t q = tval(tb, (int64_t)b * 5 + 3);
    const int64_t g = ((int64_t)b << LW) + i;
    if (q <= 1u || g >= a.m) continue;
    const int64_t s0 = tval(tb, (int64_t)b * 5 + 4);
    float f = OP == MUL ? 1.0f : 0.0f;
    uint32_t c = 0;
    uint64_t key = OP == SUMPROD ? 0ull : key_init<OP>();
    for (uint32_t j = 0; j < q; ++j) {
      const int64_t e = (s0 + j) * W + i;
      if (OP == ADD) {
        float *p = static_cast<float *>(a.partial);
        f += p[e];
        p[e] = 0.0f;
      }
      if (OP == MUL) {
        uint2 *p = static_cast<uint2 *>(a.partial);
        const uint2 u = p[e];
        c += u.x;
        f *= __uint_as_float(u.y);
        p[e] = make_uint2(0u, 0u);
      }
      if (KEYS) {
        uint64_t *p = static_cast<uint64_t *>(a.partial);
        const uint64_t k = p[e];
        key = OP == MIN ? (k < key ? k : key) : (k > key ? k : key);
        p[e] = 0ull;
      }
      if (OP == SUMPROD) {
        uint64_t *p = static_cast<uint64_t *>(a.partial);
        key = sp_pack(sp_comb(sp_unpack(key), sp_unpack(p[e])));
        p[e] = 0ull;
      }
    }
    put_bin<OP>(a, g, f, c, key);
  }
}

struct PartCfg {
  int lw, nbk, nb1;
  int64_t ch, T, slots;
  size_t rec_b, cnt_b, tot_b, tab_b, part_b;
};

size_t al256(size_t x) { return (x + 255) / 256 * 256; }

PartCfg part_cfg(int op, int64_t n, int64_t m) {
  PartCfg c{};
  c.lw = part_lw_rt(op);
  c.nbk = (int)((m + ((int64_t)1 << c.lw) - 1) >> c.lw);
  c.ch = 16384;
  while ((int64_t)c.nbk * ((n + c.ch - 1) / c.ch) + 1 > (int64_t)1 << 24) c.ch *= 2;
  c.nb1 = (int)((n + c.ch - 1) / c.ch);
  if (c.nb1 < 1) c.nb1 = 1;
  c.T = (n + PT_ITEMS - 1) / PT_ITEMS;
  if (c.T < PT_MIN_T) c.T = PT_MIN_T;
  // split buckets hold more than T elements each, so there are at most n/T
  // of them and their items number at most n/T + n/T
  c.slots = 2 * ((n + c.T - 1) / c.T) + 1;
  const bool keys = op == MIN || op == MAX;
  const int64_t ne = (int64_t)c.nbk * c.nb1 + 1;
  c.rec_b = al256((size_t)n * (keys ? 16 : 8));
  c.cnt_b = al256((size_t)ne * 4);
  c.tot_b = al256((size_t)iscan_totals(ne) * 4);
  c.tab_b = al256((size_t)(1 + 5 * (int64_t)c.nbk) * 8);
  c.part_b = al256((size_t)c.slots * ((size_t)1 << c.lw) * (op == ADD ? 4 : 8));
  return c;
}

}  // namespace

bool rbi_part_may(int op, int64_t m) {
  if (op != ADD && op != MUL && op != MIN && op != MAX && op != SUMPROD) return false;
  const int lw = part_lw_rt(op);
  return m > 0 && ((m + ((int64_t)1 << lw) - 1) >> lw) <= PT_NB_MAX;
}

size_t rbi_part_ws_bytes(int op, int64_t n, int64_t m) {
  if (!rbi_part_may(op, m)) return 0;
  const PartCfg c = part_cfg(op, n, m);
  return c.rec_b + c.cnt_b + c.tot_b + c.tab_b + c.part_b;
}

hipError_t rbi_part_fwd_row(int op, int64_t n, int64_t m, const int32_t *idx, const float *v,
                            float *hist, uint32_t *n0, float *ypos, int32_t *argk, float *ssum,
                            void *region, hipStream_t s) {
  if (n <= 0 || !rbi_part_may(op, m)) return hipErrorInvalidValue;
  const PartCfg c = part_cfg(op, n, m);
  PartArgs a;
  a.idx = idx; a.v = v; a.n = n; a.m = m;
  a.nbk = c.nbk; a.nb1 = c.nb1; a.ch = c.ch; a.T = c.T;
  a.vec = ((uintptr_t)idx % 16 == 0) && ((uintptr_t)v % 16 == 0);
  char *w = static_cast<char *>(region);
  a.rec = reinterpret_cast<uint64_t *>(w);
  a.counts = reinterpret_cast<uint32_t *>(w + c.rec_b);
  uint32_t *tot = reinterpret_cast<uint32_t *>(w + c.rec_b + c.cnt_b);
  a.tab = reinterpret_cast<uint64_t *>(w + c.rec_b + c.cnt_b + c.tot_b);
  a.partial = w + c.rec_b + c.cnt_b + c.tot_b + c.tab_b;
  a.hist = hist; a.n0 = n0; a.ypos = ypos; a.argk = argk; a.ssum = ssum;
  const int64_t ne = (int64_t)c.nbk * c.nb1 + 1;
  if (!iscan_fits(ne)) return hipErrorInvalidValue;
  const int64_t items_max = c.nbk + (n + c.T - 1) / c.T;
  const int W = 1 << c.lw;
  const dim3 gf((unsigned)(W / PC_TH), (unsigned)(c.nbk < 64 ? c.nbk : 64));
  hipLaunchKernelGGL(k_part_count, dim3(c.nb1), dim3(PT_TH), 0, s, a, c.lw);
  hipError_t e = iscan_u32(a.counts, ne, tot, s);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_part_items, dim3(1), dim3(PI_TH), 0, s, a);
#define PCAD_PART(OPV)                                                                   \
  case OPV:                                                                              \
    hipLaunchKernelGGL(k_part_scatter<OPV>, dim3(c.nb1), dim3(PT_TH), 0, s, a, c.lw);    \
    hipLaunchKernelGGL(k_part_hist<OPV>, dim3((unsigned)items_max), dim3(PH_TH), 0, s, a); \
    hipLaunchKernelGGL(k_part_fold<OPV>, gf, dim3(PC_TH), 0, s, a);                      \
    break;
  switch (op) {
    PCAD_PART(ADD)
    PCAD_PART(MUL)
    PCAD_PART(MIN)
    PCAD_PART(MAX)
  case SUMPROD:
    hipLaunchKernelGGL(k_part_scatter<SUMPROD>, dim3(c.nb1), dim3(PT_TH), 0, s, a, c.lw);
    hipLaunchKernelGGL(k_part_hist_sp, dim3((unsigned)items_max), dim3(PH_TH), 0, s, a);
    hipLaunchKernelGGL(k_part_fold<SUMPROD>, gf, dim3(PC_TH), 0, s, a);
    break;
  default: return hipErrorInvalidValue;
  }
#undef PCAD_PART
  return hipGetLastError();
}

}  // namespace pcad
