// reduce_by_index (Section 4) for + * min max and sumOfProd, and its adjoint
// (Section 4.2).
//
// Forward, three launches: neutral initialisation of the bins, the update
// pass, and (min/max, *) a per-bin finalisation.
//   update pass, small m: every block owns a contiguous chunk of one row and
//     a private sub-histogram in LDS (the paper's multi-histogram idea,
//     Section 4.2 Discussing Performance), merged into the global bins with
//     one atomic per touched bin;
//   update pass, large m: global atomics per element.
// Lifted operators:
//   min/max -- a packed 64-bit key {ord(v):32 | index:32} (index complemented
//     for max) updated with 64-bit atomic min/max, so "smallest value, then
//     smallest index" is a single native atomic instead of the mutex the
//     paper's lifted (index, value) operator needs; the value is re-read from
//     v at the winning index, so its bit pattern is kept;
//   *       -- (zero count, product of non-zeros): an atomic add on the count
//     and a compare-and-swap product.
// Adjoint: one elementwise pass -- gather (+), three zero cases (*),
// one-hot against the saved argk (min/max).
#include "device.hpp"
#include "internal.hpp"

namespace pcad {

// LDS sub-histogram limits (bins per block)
constexpr int kLdsBinsF32 = 8192;   // + and *: 32 KB of values (+ 32 KB counts for *)
constexpr int kLdsBinsU64 = 4096;   // min/max: 32 KB of keys

// CAS-loop product on global or LDS memory
__device__ __forceinline__ void atomic_mul_f32(float *p, float v) {
  unsigned *u = reinterpret_cast<unsigned *>(p);
  unsigned old = __hip_atomic_load(u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  for (;;) {
    const unsigned nw = __float_as_uint(__uint_as_float(old) * v);
    if (__hip_atomic_compare_exchange_strong(u, &old, nw, __ATOMIC_RELAXED, __ATOMIC_RELAXED,
                                             __HIP_MEMORY_SCOPE_AGENT))
      return;
  }
}

__device__ __forceinline__ void lds_mul_f32(float *p, float v) {
  unsigned *u = reinterpret_cast<unsigned *>(p);
  unsigned old = __hip_atomic_load(u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
  for (;;) {
    const unsigned nw = __float_as_uint(__uint_as_float(old) * v);
    if (__hip_atomic_compare_exchange_strong(u, &old, nw, __ATOMIC_RELAXED, __ATOMIC_RELAXED,
                                             __HIP_MEMORY_SCOPE_WORKGROUP))
      return;
  }
}

struct RbiArgs {
  const int32_t *idx;
  const float *v;
  float *hist;        // ADD: bins; MUL: finalised values
  uint32_t *n0;       // MUL: zero counts (saved)
  float *ypos;        // MUL: product of non-zeros (saved)
  uint64_t *keys;     // MIN/MAX: packed keys; SUMPROD: packed (p, s) pairs (workspace)
  int32_t *argk;      // MIN/MAX: saved
  float *ssum;        // SUMPROD: sum of each bin's values (saved)
  int64_t n, m;
  int64_t chunk;      // elements per block (multiple of 4)
  int bpr;
};

// neutral initialisation of the bins
template <int OP>
__global__ __launch_bounds__(BLOCK) void k_rbi_init(RbiArgs a, int64_t total) {
  for (int64_t k = (int64_t)blockIdx.x * BLOCK + threadIdx.x; k < total;
       k += (int64_t)gridDim.x * BLOCK) {
    if (OP == ADD) a.hist[k] = 0.0f;
    if (OP == MUL) { a.n0[k] = 0u; a.ypos[k] = 1.0f; }
    if (OP == MIN || OP == MAX) a.keys[k] = key_init<OP>();
    if (OP == LINREC) { a.hist[2 * k] = 1.0f; a.hist[2 * k + 1] = 0.0f; }
    if (OP == SATADD) a.hist[k] = 0.0f;
    if (OP == MAT2) {
      a.hist[4 * k] = 1.0f; a.hist[4 * k + 1] = 0.0f;
      a.hist[4 * k + 2] = 0.0f; a.hist[4 * k + 3] = 1.0f;
    }
  }
}

// visit the (key, value, index) triples of this block's chunk
template <class F>
__device__ __forceinline__ void for_chunk(const RbiArgs &a, int64_t row, F &&f) {
  const int64_t lo = (int64_t)blockIdx.x * a.chunk;
  const int64_t hi = lo + a.chunk < a.n ? lo + a.chunk : a.n;
  const int32_t *ir = a.idx + row * a.n;
  const float *vr = a.v + row * a.n;
  const bool vec_ok = ((row * a.n) & 3) == 0;
  for (int64_t i = lo + (int64_t)threadIdx.x * 4; i < hi; i += (int64_t)BLOCK * 4) {
    if (vec_ok && i + 4 <= hi) {
      const int4 k4 = ld_stream<int4>(ir + i);
      const float4 v4 = ld_stream<float4>(vr + i);
      f(k4.x, v4.x, (uint32_t)i);
      f(k4.y, v4.y, (uint32_t)(i + 1));
      f(k4.z, v4.z, (uint32_t)(i + 2));
      f(k4.w, v4.w, (uint32_t)(i + 3));
    } else {
      for (int j = 0; j < 4; ++j)
        if (i + j < hi) f(ir[i + j], vr[i + j], (uint32_t)(i + j));
    }
  }
}

// update pass with an LDS sub-histogram per block
template <int OP>
__global__ __launch_bounds__(BLOCK) void k_rbi_lds(RbiArgs a) {
  extern __shared__ __align__(16) unsigned char smem[];
  const int64_t row = blockIdx.y;
  const int m = (int)a.m;
  float *sf = reinterpret_cast<float *>(smem);
  unsigned *sc = reinterpret_cast<unsigned *>(smem + (size_t)m * 4);
  unsigned long long *sk = reinterpret_cast<unsigned long long *>(smem);
  for (int k = threadIdx.x; k < m; k += BLOCK) {
    if (OP == ADD) sf[k] = 0.0f;
    if (OP == MUL) { sf[k] = 1.0f; sc[k] = 0u; }
    if (OP == MIN || OP == MAX) sk[k] = key_init<OP>();
  }
  __syncthreads();
  for_chunk(a, row, [&](int32_t k, float v, uint32_t i) {
    if (k < 0 || k >= m) return;
    if (OP == ADD) lds_add_f32(&sf[k], v);
    if (OP == MUL) {
      if (v == 0.0f) atomicAdd(&sc[k], 1u);
      else lds_mul_f32(&sf[k], v);
    }
    if (OP == MIN) atomicMin(&sk[k], (unsigned long long)key_of<MIN>(v, i));
    if (OP == MAX) atomicMax(&sk[k], (unsigned long long)key_of<MAX>(v, i));
  });
  __syncthreads();
  const int64_t gb = row * a.m;
  for (int k = threadIdx.x; k < m; k += BLOCK) {
    if (OP == ADD) {
      const float s = sf[k];
      if (s != 0.0f) unsafeAtomicAdd(&a.hist[gb + k], s);
    }
    if (OP == MUL) {
      if (sc[k]) atomicAdd(&a.n0[gb + k], sc[k]);
      if (sf[k] != 1.0f) atomic_mul_f32(&a.ypos[gb + k], sf[k]);
    }
    if (OP == MIN) {
      const unsigned long long key = sk[k];
      if (key != key_init<MIN>()) atomicMin(reinterpret_cast<unsigned long long *>(&a.keys[gb + k]), key);
    }
    if (OP == MAX) {
      const unsigned long long key = sk[k];
      if (key != key_init<MAX>()) atomicMax(reinterpret_cast<unsigned long long *>(&a.keys[gb + k]), key);
    }
  }
}

// sumOfProd (Section 3.3) with an LDS table of packed (p, s) pairs per
// block; the chunk is walked in rounds that every lane of the block takes
// (sp_wave_update needs whole waves), then the table goes to the block's own
// slot of the workspace (a global compare-and-swap merge of many blocks
// into few bins would serialise on those bins)
__global__ __launch_bounds__(BLOCK) void k_rbi_lds_sp(RbiArgs a) {
  extern __shared__ __align__(16) unsigned char smem[];
  uint64_t *tab = reinterpret_cast<uint64_t *>(smem);
  const int64_t row = blockIdx.y;
  const int m = (int)a.m;
  for (int k = threadIdx.x; k < m; k += BLOCK) tab[k] = 0ull;
  __syncthreads();
  const int64_t lo = (int64_t)blockIdx.x * a.chunk;
  const int64_t hi = lo + a.chunk < a.n ? lo + a.chunk : a.n;
  const int32_t *ir = a.idx + row * a.n;
  const float *vr = a.v + row * a.n;
  for (int64_t i = lo + threadIdx.x; i - threadIdx.x < hi; i += BLOCK) {
    const bool in = i < hi;
    const int32_t k = in ? ir[i] : -1;
    const float x = in ? vr[i] : 0.0f;
    const bool ok = k >= 0 && k < m;
    sp_wave_update(tab, ok ? (uint32_t)k : 0u, x, ok);
  }
  __syncthreads();
  uint64_t *slot = a.keys + (row * a.bpr + blockIdx.x) * a.m;
  for (int k = threadIdx.x; k < m; k += BLOCK) slot[k] = tab[k];
}

// fold the blocks' tables of every bin in block order (the fold order is
// fixed, so results repeat bit for bit), then zero them
__global__ __launch_bounds__(BLOCK) void k_rbi_fold_sp(RbiArgs a, int64_t total) {
  for (int64_t t = (int64_t)blockIdx.x * BLOCK + threadIdx.x; t < total;
       t += (int64_t)gridDim.x * BLOCK) {
    const int64_t row = t / a.m, k = t - row * a.m;
    SP r = {0.0f, 0.0f};
    for (int j = 0; j < a.bpr; ++j) {
      uint64_t *w = a.keys + (row * a.bpr + j) * a.m + k;
      r = sp_comb(r, sp_unpack(*w));
      *w = 0ull;
    }
    a.hist[t] = r.p;
    a.ssum[t] = r.s;
  }
}

// Update pass for bin counts beyond a full LDS histogram: each block keeps
// an LDS hash table of the bins it meets (open addressing, linear probing),
// so repeated bins -- skewed keys -- combine in LDS and reach global memory
// once per block; a key that finds no slot within kProbes probes goes
// straight to a global atomic (distinct bins contend little).
constexpr int kHashSlots = 4096;
constexpr int kProbes = 8;

template <int OP>
__device__ __forceinline__ void rbi_global_update(const RbiArgs &a, int64_t g, float v,
                                                  uint32_t i) {
  if (OP == ADD) unsafeAtomicAdd(&a.hist[g], v);
  if (OP == MUL) {
    if (v == 0.0f) atomicAdd(&a.n0[g], 1u);
    else atomic_mul_f32(&a.ypos[g], v);
  }
  if (OP == MIN)
    atomicMin(reinterpret_cast<unsigned long long *>(&a.keys[g]),
              (unsigned long long)key_of<MIN>(v, i));
  if (OP == MAX)
    atomicMax(reinterpret_cast<unsigned long long *>(&a.keys[g]),
              (unsigned long long)key_of<MAX>(v, i));
}

template <int OP>
__global__ __launch_bounds__(BLOCK) void k_rbi_hash(RbiArgs a) {
  constexpr bool KEYS = OP == MIN || OP == MAX;
  __shared__ int32_t s_bin[kHashSlots];
  __shared__ float s_f[KEYS ? 1 : kHashSlots];
  __shared__ unsigned s_c[OP == MUL ? kHashSlots : 1];
  __shared__ unsigned long long s_k[KEYS ? kHashSlots : 1];
  const int64_t row = blockIdx.y;
  const int64_t gb = row * a.m;
  const int64_t m = a.m;
  for (int t = threadIdx.x; t < kHashSlots; t += BLOCK) {
    s_bin[t] = -1;
    if (OP == ADD) s_f[t] = 0.0f;
    if (OP == MUL) { s_f[t] = 1.0f; s_c[t] = 0u; }
    if (KEYS) s_k[t] = key_init<OP>();
  }
  __syncthreads();
  for_chunk(a, row, [&](int32_t k, float v, uint32_t i) {
    if (k < 0 || k >= m) return;
    uint32_t h = ((uint32_t)k * 2654435761u) >> (32 - 12);  // kHashSlots = 2^12
#pragma unroll 1
    for (int p = 0; p < kProbes; ++p) {
      int32_t cur = __hip_atomic_load(&s_bin[h], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
      if (cur == -1) {
        int32_t expect = -1;
        __hip_atomic_compare_exchange_strong(&s_bin[h], &expect, k, __ATOMIC_RELAXED,
                                             __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
        cur = expect == -1 ? k : expect;  // the slot is ours, or holds the winner's bin
      }
      if (cur == k) {
        if (OP == ADD) lds_add_f32(&s_f[h], v);
        if (OP == MUL) {
          if (v == 0.0f) atomicAdd(&s_c[h], 1u);
          else lds_mul_f32(&s_f[h], v);
        }
        if (OP == MIN) atomicMin(&s_k[h], (unsigned long long)key_of<MIN>(v, i));
        if (OP == MAX) atomicMax(&s_k[h], (unsigned long long)key_of<MAX>(v, i));
        return;
      }
      h = (h + 1) & (kHashSlots - 1);
    }
    rbi_global_update<OP>(a, gb + k, v, i);
  });
  __syncthreads();
  for (int t = threadIdx.x; t < kHashSlots; t += BLOCK) {
    const int32_t k = s_bin[t];
    if (k < 0) continue;
    const int64_t g = gb + k;
    if (OP == ADD) unsafeAtomicAdd(&a.hist[g], s_f[t]);
    if (OP == MUL) {
      if (s_c[t]) atomicAdd(&a.n0[g], s_c[t]);
      if (s_f[t] != 1.0f) atomic_mul_f32(&a.ypos[g], s_f[t]);
    }
    if (OP == MIN) atomicMin(reinterpret_cast<unsigned long long *>(&a.keys[g]), s_k[t]);
    if (OP == MAX) atomicMax(reinterpret_cast<unsigned long long *>(&a.keys[g]), s_k[t]);
  }
}

// per-bin finalisation: value and argk (min/max), value (mul)
template <int OP>
__global__ __launch_bounds__(BLOCK) void k_rbi_fin(RbiArgs a, int64_t total) {
  for (int64_t t = (int64_t)blockIdx.x * BLOCK + threadIdx.x; t < total;
       t += (int64_t)gridDim.x * BLOCK) {
    if (OP == MUL) {
      a.hist[t] = a.n0[t] > 0 ? 0.0f : a.ypos[t];
    } else {
      const uint64_t key = a.keys[t];
      a.keys[t] = 0;  // leave the workspace holding no data between calls
      const int64_t row = t / a.m;
      if (key == key_init<OP>()) {
        a.argk[t] = (int32_t)a.n;
        a.hist[t] = OP == MIN ? __builtin_inff() : -__builtin_inff();
      } else {
        const uint32_t lo = (uint32_t)key;
        const uint32_t i = OP == MIN ? lo : ~lo;
        a.argk[t] = (int32_t)i;
        a.hist[t] = a.v[row * a.n + i];
      }
    }
  }
}

// adjoint: one elementwise pass per row.  What an element needs from its
// bin comes from one place per element:
//   GATHER -- the saved arrays and hbar directly (one gather per array);
//   LDS    -- a per-bin record table the block builds in LDS (small m);
//   TABLE  -- the same records built once in the workspace by k_rbi_vjp_tab
//             (large m: one gather per element instead of one per array).
// Records: + : hbar;  * : {y_pos, n0 | 2^31, hbar, 2^31};
// min/max: {hbar, argk | 2^31}.  Every 8-byte word of a record left in the
// workspace has its upper half >= 2^31.
struct RbiVjpArgs {
  const int32_t *idx;
  const float *v;
  const float *hbar;
  const uint32_t *n0;
  const float *ypos;
  const int32_t *argk;
  const float *ssum;
  float *vbar;
  void *tab;
  int64_t n, m;
  int accumulate;
};

enum { VJP_GATHER = 0, VJP_LDS = 1, VJP_TABLE = 2 };
constexpr uint32_t kRecHi = 0x80000000u;

template <int OP>
__device__ __forceinline__ uint4 vjp_rec(const RbiVjpArgs &a, int64_t t) {
  uint4 r;
  if (OP == MUL) {
    r.x = __float_as_uint(a.ypos[t]); r.y = a.n0[t] | kRecHi;
    r.z = __float_as_uint(a.hbar[t]); r.w = kRecHi;
  } else {  // SUMPROD
    r.x = __float_as_uint(a.ssum[t]); r.y = __float_as_uint(a.hbar[t]);  // LDS only
    r.z = r.w = 0u;
  }
  return r;
}

template <int OP>
__global__ __launch_bounds__(BLOCK) void k_rbi_vjp_tab(RbiVjpArgs a, int64_t total) {
  for (int64_t t = (int64_t)blockIdx.x * BLOCK + threadIdx.x; t < total;
       t += (int64_t)gridDim.x * BLOCK) {
    static_cast<uint4 *>(a.tab)[t] = vjp_rec<OP>(a, t);  // MUL
  }
}

// + and sumOfProd adjoints beyond the 16 KB tables: 1024-thread blocks (one
// per CU, 16 waves) keep the records of the first up to kBigBins bins in
// 144 KB of LDS and gather the rest from memory, so that at m = 65536 most
// lookups stay out of the L2 -> L1 path (a random 4-byte gather moves a
// whole line there)
constexpr int VJP_BIG_TH = 1024;
constexpr int kBigLdsBytes = 147456;

template <int OP>
__global__ __launch_bounds__(VJP_BIG_TH) void k_rbi_vjp_big(RbiVjpArgs a, int64_t lm) {
  constexpr int REC = OP == ADD ? 4 : 8;  // ADD: hbar; SUMPROD: (s, hbar)
  __shared__ __align__(16) unsigned char s_tab[kBigLdsBytes];
  const int64_t row = blockIdx.y;
  const int32_t *ir = a.idx + row * a.n;
  const float *vr = a.v + row * a.n;
  float *ob = a.vbar + row * a.n;
  const int64_t gb = row * a.m;
  for (int64_t k = threadIdx.x; k < lm; k += VJP_BIG_TH) {
    if (OP == ADD) reinterpret_cast<float *>(s_tab)[k] = a.hbar[gb + k];
    else reinterpret_cast<float2 *>(s_tab)[k] = make_float2(a.ssum[gb + k], a.hbar[gb + k]);
  }
  __syncthreads();
  static_assert(REC == 4 || REC == 8, "record size");
  const bool vec_ok = ((row * a.n) & 3) == 0;
  const int64_t stride = (int64_t)gridDim.x * VJP_BIG_TH * 4;
  for (int64_t i = ((int64_t)blockIdx.x * VJP_BIG_TH + threadIdx.x) * 4; i < a.n; i += stride) {
    const bool full = vec_ok && i + 4 <= a.n;
    int kk[4];
    float vv[4] = {0.0f, 0.0f, 0.0f, 0.0f}, o[4];
    if (full) {
      const int4 k4 = ld_stream<int4>(ir + i);
      kk[0] = k4.x; kk[1] = k4.y; kk[2] = k4.z; kk[3] = k4.w;
      if (OP == SUMPROD) {
        const float4 v4 = ld_stream<float4>(vr + i);
        vv[0] = v4.x; vv[1] = v4.y; vv[2] = v4.z; vv[3] = v4.w;
      }
    } else {
      for (int j = 0; j < 4; ++j) {
        kk[j] = (i + j < a.n) ? ir[i + j] : -1;
        if (OP == SUMPROD && i + j < a.n) vv[j] = vr[i + j];
      }
    }
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const int k = kk[j];
      float r = 0.0f;
      if (k >= 0 && k < a.m) {
        if (OP == ADD) {
          r = k < lm ? reinterpret_cast<const float *>(s_tab)[k] : a.hbar[gb + k];
        } else {
          float sk, h;
          if (k < lm) {
            const float2 q = reinterpret_cast<const float2 *>(s_tab)[k];
            sk = q.x; h = q.y;
          } else {
            sk = a.ssum[gb + k]; h = a.hbar[gb + k];
          }
          r = (sk - vv[j]) * h;  // the invertible-operator rule
        }
      }
      o[j] = r;
    }
    if (a.accumulate) {
      for (int j = 0; j < 4; ++j)
        if (i + j < a.n) o[j] += ob[i + j];
    }
    if (full) {
      *reinterpret_cast<float4 *>(ob + i) = make_float4(o[0], o[1], o[2], o[3]);
    } else {
      for (int j = 0; j < 4; ++j)
        if (i + j < a.n) ob[i + j] = o[j];
    }
  }
}

// min/max adjoint as the min rule figure of Section 4.2 states it: the bin
// adjoint goes to the bin's arg-extremum by a scatter (positions are unique
// within a row, and an empty bin's sentinel n selects nothing); every other
// element's adjoint is zero (a fill first unless accumulating).  The keys are
// never read.
__global__ __launch_bounds__(BLOCK) void k_rbi_vjp_fill0(float *vbar, int64_t total) {
  const int64_t t4 = total / 4;
  for (int64_t t = (int64_t)blockIdx.x * BLOCK + threadIdx.x; t < t4;
       t += (int64_t)gridDim.x * BLOCK)
    reinterpret_cast<float4 *>(vbar)[t] = make_float4(0.0f, 0.0f, 0.0f, 0.0f);
  const int64_t r = t4 * 4 + (int64_t)blockIdx.x * BLOCK + threadIdx.x;
  if (r < total) vbar[r] = 0.0f;
}

__global__ __launch_bounds__(BLOCK) void k_rbi_vjp_scatter(RbiVjpArgs a, int64_t total) {
  for (int64_t t = (int64_t)blockIdx.x * BLOCK + threadIdx.x; t < total;
       t += (int64_t)gridDim.x * BLOCK) {
    const int64_t row = t / a.m;
    const int32_t k = a.argk[t];
    if (k >= 0 && k < a.n) {
      float *o = a.vbar + row * a.n + k;
      *o = a.accumulate ? *o + a.hbar[t] : a.hbar[t];
    }
  }
}

template <int OP, int SRC>
__global__ __launch_bounds__(BLOCK) void k_rbi_vjp(RbiVjpArgs a) {
  extern __shared__ __align__(16) unsigned char smem[];
  const int64_t row = blockIdx.y;
  const int32_t *ir = a.idx + row * a.n;
  const float *vr = a.v + row * a.n;
  float *ob = a.vbar + row * a.n;
  const int64_t gb = row * a.m;
  if (SRC == VJP_LDS) {
    for (int64_t k = threadIdx.x; k < a.m; k += BLOCK) {
      if (OP == ADD) reinterpret_cast<float *>(smem)[k] = a.hbar[gb + k];
      else if (OP == MUL) reinterpret_cast<uint4 *>(smem)[k] = vjp_rec<OP>(a, gb + k);
      else {  // SUMPROD: (s, hbar)
        const uint4 r = vjp_rec<OP>(a, gb + k);
        reinterpret_cast<uint2 *>(smem)[k] = make_uint2(r.x, r.y);
      }
    }
    __syncthreads();
  }
  const bool vec_ok = ((row * a.n) & 3) == 0;
  const int64_t stride = (int64_t)gridDim.x * BLOCK * 4;
  for (int64_t i = ((int64_t)blockIdx.x * BLOCK + threadIdx.x) * 4; i < a.n; i += stride) {
    const bool full = vec_ok && i + 4 <= a.n;
    int kk[4];
    float vv[4] = {1.0f, 1.0f, 1.0f, 1.0f}, o[4];
    if (full) {
      const int4 k4 = ld_stream<int4>(ir + i);
      kk[0] = k4.x; kk[1] = k4.y; kk[2] = k4.z; kk[3] = k4.w;
      if (OP == MUL || OP == SUMPROD) {
        const float4 v4 = ld_stream<float4>(vr + i);
        vv[0] = v4.x; vv[1] = v4.y; vv[2] = v4.z; vv[3] = v4.w;
      }
    } else {
      for (int j = 0; j < 4; ++j) {
        kk[j] = (i + j < a.n) ? ir[i + j] : -1;
        if ((OP == MUL || OP == SUMPROD) && i + j < a.n) vv[j] = vr[i + j];
      }
    }
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const int k = kk[j];
      float r = 0.0f;
      if (k >= 0 && k < a.m) {
        if (OP == ADD) {
          r = SRC == VJP_LDS ? reinterpret_cast<const float *>(smem)[k] : a.hbar[gb + k];
        } else if (OP == MUL) {
          uint32_t z;
          float p, h;
          if (SRC == VJP_GATHER) {
            z = a.n0[gb + k]; p = a.ypos[gb + k]; h = a.hbar[gb + k];
          } else {
            const uint4 q = SRC == VJP_LDS ? reinterpret_cast<const uint4 *>(smem)[k]
                                           : static_cast<const uint4 *>(a.tab)[gb + k];
            p = __uint_as_float(q.x); z = q.y & ~kRecHi; h = __uint_as_float(q.z);
          }
          r = z == 0 ? (p / vv[j]) * h : ((z == 1 && vv[j] == 0.0f) ? p * h : 0.0f);
        } else if (OP == SUMPROD) {
          float sk, h;
          if (SRC == VJP_LDS) {
            const uint2 q = reinterpret_cast<const uint2 *>(smem)[k];
            sk = __uint_as_float(q.x); h = __uint_as_float(q.y);
          } else {
            sk = a.ssum[gb + k]; h = a.hbar[gb + k];
          }
          // the invertible-operator rule: the bin without v_i keeps s - v_i
          r = (sk - vv[j]) * h;
        }
      }
      o[j] = r;
    }
    if (a.accumulate) {
      for (int j = 0; j < 4; ++j)
        if (i + j < a.n) o[j] += ob[i + j];
    }
    if (full) {
      *reinterpret_cast<float4 *>(ob + i) = make_float4(o[0], o[1], o[2], o[3]);
    } else {
      for (int j = 0; j < 4; ++j)
        if (i + j < a.n) ob[i + j] = o[j];
    }
  }
}

// ---------------------------------------------------------------------------
// Bin counts of a few LDS tables: the bins are split into P <= 4 parts of
// one 128 KB table each, and one 1024-thread block per CU owns a (part,
// chunk of elements) pair, keeping only the keys of its part.  Blocks are
// dealt to the XCDs round robin, so the P blocks of a chunk are placed on
// one XCD: the chunk comes from HBM about once and from that XCD's L2 for
// the other parts.  Each block writes its table to its own slot; a fold
// combines a bin's chunks in chunk order (deterministic) and clears the
// slots.  For one row; the slots live where the partition's records would.
// ---------------------------------------------------------------------------
constexpr int PARTS_TH = 1024;
constexpr int kPartsLdsBytes = 131072;
constexpr int kPartsMax = 4;
constexpr int kXcds = 8;  // gfx950: blocks go to the 8 XCDs round robin

template <int OP>
constexpr int parts_bins() {
  return OP == ADD ? kPartsLdsBytes / 4 : kPartsLdsBytes / 8;
}

struct PartsArgs {
  const int32_t *idx;
  const float *v;
  float *hist;
  int32_t *argk;
  void *slots;
  int64_t n, m, chunk;
  int P, C;
};

template <int OP>
__global__ __launch_bounds__(PARTS_TH) void k_rbi_parts(PartsArgs a) {
  constexpr int L = parts_bins<OP>();
  constexpr bool KEYS = OP == MIN || OP == MAX;
  __shared__ __align__(16) unsigned char s_raw[kPartsLdsBytes];
  static_assert(OP == ADD || KEYS, "+ and min/max only");
  float *sf = reinterpret_cast<float *>(s_raw);                    // + values
  unsigned long long *sk = reinterpret_cast<unsigned long long *>(s_raw);  // min/max keys
  const int b = blockIdx.x;
  const int xcd = b % kXcds, slot = b / kXcds;
  const int c = xcd + kXcds * (slot / a.P), p = slot % a.P;
  for (int k = threadIdx.x; k < L; k += PARTS_TH) {
    if (OP == ADD) sf[k] = 0.0f;
    if (KEYS) sk[k] = key_init<OP>();
  }
  __syncthreads();
  const int64_t lo = (int64_t)c * a.chunk;
  const int64_t hi = lo + a.chunk < a.n ? lo + a.chunk : a.n;
  // +: bins are dealt to the parts round robin (bin g: part g mod P, entry
  // g / P), so the hot low bins of a skewed key distribution spread over
  // the parts instead of loading one of them (Zipf keys at m = 65536:
  // 0.54 -> 0.37 ms); min/max keep contiguous ranges, which measured faster
  // for them (0.28 against 0.34 ms)
  constexpr bool INTER = OP == ADD;
  const int lp = a.P == 4 ? 2 : (a.P == 2 ? 1 : 0);
  const int64_t kb0 = (int64_t)p * L;
  auto upd = [&](int32_t key, float v, uint32_t i) {
    if (key < 0 || key >= a.m) return;
    int k;
    if (INTER) {
      if ((key & (a.P - 1)) != p) return;
      k = key >> lp;
    } else {
      const int64_t kk = (int64_t)key - kb0;
      if (kk < 0 || kk >= L) return;
      k = (int)kk;
    }
    if (OP == ADD) lds_add_f32(&sf[k], v);
    if (OP == MIN) atomicMin(&sk[k], (unsigned long long)key_of<MIN>(v, i));
    if (OP == MAX) atomicMax(&sk[k], (unsigned long long)key_of<MAX>(v, i));
  };
  for (int64_t i = lo + (int64_t)threadIdx.x * 4; i < hi; i += (int64_t)PARTS_TH * 4) {
    if (i + 4 <= hi) {  // lo, chunk and the row start are multiples of 4
      const int4 k4 = ld_stream<int4>(a.idx + i);
      const float4 v4 = ld_stream<float4>(a.v + i);
      upd(k4.x, v4.x, (uint32_t)i);
      upd(k4.y, v4.y, (uint32_t)(i + 1));
      upd(k4.z, v4.z, (uint32_t)(i + 2));
      upd(k4.w, v4.w, (uint32_t)(i + 3));
    } else {
      for (int64_t j = i; j < hi; ++j) upd(a.idx[j], a.v[j], (uint32_t)j);
    }
  }
  __syncthreads();
  // only the part's bins below m: the fold clears exactly what was written
  const int64_t base = ((int64_t)p * a.C + c) * L;
  const int lim = INTER ? (int)((a.m - p + a.P - 1) >> lp)  // entries of bins below m
                        : (int)(a.m - kb0 < L ? a.m - kb0 : L);
  for (int k = threadIdx.x; k < lim; k += PARTS_TH) {
    if (OP == ADD) static_cast<float *>(a.slots)[base + k] = sf[k];
    if (KEYS) static_cast<uint64_t *>(a.slots)[base + k] = sk[k];
  }
}

template <int OP>
__global__ __launch_bounds__(BLOCK) void k_rbi_parts_fold(PartsArgs a) {
  constexpr int L = parts_bins<OP>();
  for (int64_t g = (int64_t)blockIdx.x * BLOCK + threadIdx.x; g < a.m;
       g += (int64_t)gridDim.x * BLOCK) {
    const int64_t p = OP == ADD ? (g & (a.P - 1)) : g / L;
    const int64_t k = OP == ADD ? (g >> (a.P == 4 ? 2 : (a.P == 2 ? 1 : 0))) : g - p * L;
    float f = 0.0f;
    uint64_t key = key_init<OP == MAX ? MAX : MIN>();
    for (int c = 0; c < a.C; ++c) {
      const int64_t e = (p * a.C + c) * L + k;
      if (OP == ADD) {
        float *s = static_cast<float *>(a.slots);
        f += s[e];
        s[e] = 0.0f;
      }
      if (OP == MIN || OP == MAX) {
        uint64_t *s = static_cast<uint64_t *>(a.slots);
        const uint64_t q = s[e];
        key = OP == MIN ? (q < key ? q : key) : (q > key ? q : key);
        s[e] = 0ull;
      }
    }
    if (OP == ADD) a.hist[g] = f;
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
}

// ---------------------------------------------------------------------------
// host side
// ---------------------------------------------------------------------------
static bool use_lds(int op, int64_t m) {
  if (op == SUMPROD) return m <= kLdsBinsU64;  // no hash path: the knob does not apply
  if (op == MIN || op == MAX) return m <= kLdsBinsU64 && m <= knob_rbi_lds_max_bins(true);
  return m <= kLdsBinsF32 && m <= knob_rbi_lds_max_bins(false);
}

static size_t lds_bytes(int op, int64_t m) {
  if (op == MIN || op == MAX || op == SUMPROD) return (size_t)m * 8;
  if (op == MUL) return (size_t)m * 8;
  return (size_t)m * 4;
}

static size_t op_saved_bytes(int op, int64_t batch, int64_t m) {
  if (op == MUL) return (size_t)batch * m * 8;
  if (op == MIN || op == MAX || op == SUMPROD) return (size_t)batch * m * 4;
  return 0;
}

// the sort-based path: always for the ordered operators; for the others
// beyond the LDS capacity (a fixed bound, so the workspace size does not
// depend on the knobs), from the knob's bin count on
// (the general rule: the ordered operators and saturated addition, which has
// no specialised rule)
static bool general_rule(int op) { return op == LINREC || op == MAT2 || op == SATADD; }

static bool sorted_may(int op, int64_t m) {
  if (op == SUMPROD) return false;
  if (general_rule(op)) return true;
  return m > ((op == MIN || op == MAX) ? kLdsBinsU64 : kLdsBinsF32);
}

static bool use_sorted(int op, int64_t m) {
  if (general_rule(op)) return true;
  return sorted_may(op, m) && m >= knob_rbi_sort_min_bins();
}

// the partitioned path: the commutative operators beyond the LDS capacity
// (a fixed bound, like sorted_may), unless the knob picks the hash table
static bool part_may(int op, int64_t m) {
  if (general_rule(op)) return false;
  const bool u64 = op == MIN || op == MAX || op == SUMPROD;
  return m > (u64 ? kLdsBinsU64 : kLdsBinsF32) && rbi_part_may(op, m);
}

// sumOfProd has no other path beyond the LDS histogram
static bool use_part(int op, int64_t n, int64_t m) {
  if (op == SUMPROD) return n > 0 && part_may(op, m);
  return n > 0 && part_may(op, m) && knob_rbi_partition() && !use_sorted(op, m);
}

// the LDS-table parts (see k_rbi_parts): one row, at most kPartsMax tables
struct PartsCfg {
  int P = 0, C = 0;
  int64_t chunk = 0;
  size_t bytes = 0;
};

static PartsCfg parts_cfg(int op, int64_t n, int64_t m) {
  PartsCfg c;
  const int64_t L = op == ADD ? kPartsLdsBytes / 4 : kPartsLdsBytes / 8;
  int64_t P = (m + L - 1) / L;
  if (P == 3 && op == ADD) P = 4;  // +: a power of two (part = bin mod P, entry = bin / P)
  if (P < 1 || P > kPartsMax) return c;
  // chunks per XCD: fill the 256 CUs, but give every block at least 64K elements
  int64_t cl = 32 / P;
  const int64_t want = (n + (int64_t)kXcds * 65536 - 1) / ((int64_t)kXcds * 65536);
  if (cl > want) cl = want;
  if (cl < 1) cl = 1;
  c.P = (int)P;
  c.C = (int)(kXcds * cl);
  c.chunk = ((n + c.C - 1) / c.C + 3) / 4 * 4;
  c.bytes = (size_t)P * c.C * L * (op == ADD ? 4 : 8);
  return c;
}

// (not for *: its LDS product is a compare-and-swap loop, which hot bins of
// skewed keys serialise in these large blocks -- 2.7 ms against the
// partition's 1.0 ms at m = 65536 with Zipf keys)
static bool use_parts(int op, int64_t batch, int64_t n, int64_t m) {
  if (op != ADD && op != MIN && op != MAX) return false;
  if (batch != 1 || n <= 0 || !knob_rbi_parts() || !part_may(op, m) || use_sorted(op, m))
    return false;
  const PartsCfg c = parts_cfg(op, n, m);
  return c.P > 0 && c.bytes <= rbi_part_ws_bytes(op, n, m);
}

// control block, then the per-bin region: min/max keys (forward) or
// adjoint records (8 bytes per bin), * adjoint records (16 bytes per bin),
// sumOfProd's per-block tables
// sumOfProd with the LDS table: blocks per row, each writing its table to
// its own slot of the workspace (at most 2^22 pairs, 32 MB, in all)
static int64_t sp_blocks_per_row(int64_t batch, int64_t n, int64_t m) {
  int64_t cap = ((int64_t)1 << 22) / (batch * m > 0 ? batch * m : 1);
  if (cap > 1024) cap = 1024;
  if (cap < 1) cap = 1;
  int64_t bpr = (n + 16383) / 16384;
  if (bpr > cap) bpr = cap;
  if (bpr < 1) bpr = 1;
  return bpr;
}

static size_t base_ws_bytes(int op, int64_t batch, int64_t n, int64_t m) {
  size_t b = kCtlBytes;
  if (op == MIN || op == MAX) b += (size_t)batch * m * 8;
  if (op == SUMPROD && m <= kLdsBinsU64)
    b += (size_t)(batch * sp_blocks_per_row(batch, n, m) * m) * 8;
  if (op == MUL) b += (size_t)batch * m * 16;
  return (b + 255) / 256 * 256;
}

size_t rbi_ws_bytes(int op, int64_t batch, int64_t n, int64_t m) {
  // one row at a time: the sort's or the partition's scratch (whichever
  // may run) after the operator's own workspace
  const size_t so = sorted_may(op, m) ? rbi_sorted_ws_bytes(op, n, m) : 0;
  const size_t pa = part_may(op, m) ? rbi_part_ws_bytes(op, n, m) : 0;
  return base_ws_bytes(op, batch, n, m) + (so > pa ? so : pa);
}

// saved state: the operator's own (zero counts and products; arg-extrema)
// then, where the sort-based path may run, each row's sort
static size_t op_saved_aligned(int op, int64_t batch, int64_t m) {
  return (op_saved_bytes(op, batch, m) + 255) / 256 * 256;
}

size_t rbi_saved_bytes(int op, int64_t batch, int64_t n, int64_t m) {
  size_t b = op_saved_bytes(op, batch, m);
  if (sorted_may(op, m)) b = op_saved_aligned(op, batch, m) + (size_t)batch * rbi_sort_area_bytes(n, m);
  return b;
}

static int64_t grid1d(int64_t total) {
  int64_t g = (total + BLOCK - 1) / BLOCK;
  if (g > 16384) g = 16384;
  if (g < 1) g = 1;
  return g;
}

hipError_t rbi_fwd_launch(int op, int64_t batch, int64_t n, int64_t m, const int32_t *idx,
                          const float *v, float *hist, void *saved, void *ws, hipStream_t s) {
  if (batch == 0 || m == 0) return hipSuccess;
  RbiArgs a;
  a.idx = idx; a.v = v; a.hist = hist; a.n = n; a.m = m;
  a.n0 = nullptr; a.ypos = nullptr; a.keys = nullptr; a.argk = nullptr; a.ssum = nullptr;
  const int64_t total = batch * m;
  if (op == MUL) {
    a.n0 = static_cast<uint32_t *>(saved);
    a.ypos = reinterpret_cast<float *>(static_cast<uint32_t *>(saved) + total);
  }
  if (op == MIN || op == MAX) {
    a.keys = reinterpret_cast<uint64_t *>(static_cast<char *>(ws) + kCtlBytes);
    a.argk = static_cast<int32_t *>(saved);
  }
  if (op == SUMPROD) {
    a.keys = reinterpret_cast<uint64_t *>(static_cast<char *>(ws) + kCtlBytes);
    a.ssum = static_cast<float *>(saved);
  }
  if (use_sorted(op, m)) {
    const int d = op == LINREC ? 2 : (op == MAT2 ? 4 : 1);
    void *sws = static_cast<char *>(ws) + base_ws_bytes(op, batch, n, m);
    const dim3 gi((unsigned)grid1d(total));
#define PCAD_RBI_INIT(OPV) \
  case OPV: hipLaunchKernelGGL(k_rbi_init<OPV>, gi, dim3(BLOCK), 0, s, a, total); break;
    switch (op) {
      PCAD_RBI_INIT(ADD)
      PCAD_RBI_INIT(MUL)
      PCAD_RBI_INIT(MIN)
      PCAD_RBI_INIT(MAX)
      PCAD_RBI_INIT(LINREC)
      PCAD_RBI_INIT(MAT2)
      PCAD_RBI_INIT(SATADD)
    default: return hipErrorInvalidValue;
    }
#undef PCAD_RBI_INIT
    char *area = static_cast<char *>(saved) + op_saved_aligned(op, batch, m);
    const size_t ab = rbi_sort_area_bytes(n, m);
    for (int64_t r = 0; r < batch; ++r) {
      hipError_t e = rbi_sorted_fwd_row(
          op, n, m, idx + r * n, v + r * n * d, hist ? hist + r * m * d : nullptr,
          a.n0 ? a.n0 + r * m : nullptr, a.ypos ? a.ypos + r * m : nullptr,
          a.keys ? a.keys + r * m : nullptr, ws, sws, area + r * ab, s);
      if (e != hipSuccess) return e;
    }
    switch (op) {
    case MUL: hipLaunchKernelGGL(k_rbi_fin<MUL>, gi, dim3(BLOCK), 0, s, a, total); break;
    case MIN: hipLaunchKernelGGL(k_rbi_fin<MIN>, gi, dim3(BLOCK), 0, s, a, total); break;
    case MAX: hipLaunchKernelGGL(k_rbi_fin<MAX>, gi, dim3(BLOCK), 0, s, a, total); break;
    default: break;
    }
    return hipGetLastError();
  }
  if (use_parts(op, batch, n, m)) {
    const PartsCfg c = parts_cfg(op, n, m);
    PartsArgs q;
    q.idx = idx; q.v = v; q.hist = hist; q.argk = a.argk;
    q.slots = static_cast<char *>(ws) + base_ws_bytes(op, batch, n, m);
    q.n = n; q.m = m; q.chunk = c.chunk; q.P = c.P; q.C = c.C;
    const dim3 gp((unsigned)(c.P * c.C)), gf((unsigned)grid1d(m));
#define PCAD_PARTS(OPV)                                                              \
  case OPV:                                                                          \
    hipLaunchKernelGGL(k_rbi_parts<OPV>, gp, dim3(PARTS_TH), 0, s, q);               \
    hipLaunchKernelGGL(k_rbi_parts_fold<OPV>, gf, dim3(BLOCK), 0, s, q);             \
    break;
    switch (op) {
      PCAD_PARTS(ADD)
      PCAD_PARTS(MIN)
      PCAD_PARTS(MAX)
    default: return hipErrorInvalidValue;
    }
#undef PCAD_PARTS
    return hipGetLastError();
  }
  if (use_part(op, n, m)) {
    void *region = static_cast<char *>(ws) + base_ws_bytes(op, batch, n, m);
    for (int64_t r = 0; r < batch; ++r) {
      hipError_t e = rbi_part_fwd_row(op, n, m, idx + r * n, v + r * n, hist + r * m,
                                      a.n0 ? a.n0 + r * m : nullptr,
                                      a.ypos ? a.ypos + r * m : nullptr,
                                      a.argk ? a.argk + r * m : nullptr,
                                      a.ssum ? a.ssum + r * m : nullptr, region, s);
      if (e != hipSuccess) return e;
    }
    return hipGetLastError();
  }
  const bool lds = use_lds(op, m);
  // blocks per row: enough to fill the chip, few enough that the LDS
  // sub-histogram of each block sees many elements
  const int64_t epb = knob_rbi_elems_per_block();
  int64_t bpr = (n + epb - 1) / epb;
  int64_t cap = (lds ? 2048 : 65535) / (batch > 0 ? batch : 1);
  if (cap < 1) cap = 1;
  if (bpr > cap) bpr = cap;
  if (bpr < 1) bpr = 1;
  a.bpr = (int)bpr;
  a.chunk = ((n + bpr - 1) / bpr + 3) / 4 * 4;
  const dim3 gi((unsigned)grid1d(total));
  const dim3 gu((unsigned)bpr, (unsigned)batch);
  const size_t shm = lds_bytes(op, m);
#define PCAD_RBI(OPV)                                                               \
  case OPV:                                                                         \
    hipLaunchKernelGGL(k_rbi_init<OPV>, gi, dim3(BLOCK), 0, s, a, total);           \
    if (n > 0) {                                                                    \
      if (lds) hipLaunchKernelGGL(k_rbi_lds<OPV>, gu, dim3(BLOCK), shm, s, a);      \
      else hipLaunchKernelGGL(k_rbi_hash<OPV>, gu, dim3(BLOCK), 0, s, a);           \
    }                                                                               \
    if (OPV != ADD) hipLaunchKernelGGL(k_rbi_fin<OPV>, gi, dim3(BLOCK), 0, s, a, total); \
    break;
  if (op == SUMPROD) {
    // n > 0 beyond the LDS table took the partitioned path above
    if (n > 0 && !lds) return hipErrorInvalidValue;
    a.bpr = n > 0 ? (int)sp_blocks_per_row(batch, n, m) : 0;
    a.chunk = n > 0 ? ((n + a.bpr - 1) / a.bpr + 3) / 4 * 4 : 0;
    if (n > 0) hipLaunchKernelGGL(k_rbi_lds_sp, dim3((unsigned)a.bpr, (unsigned)batch), dim3(BLOCK),
                                  shm, s, a);
    hipLaunchKernelGGL(k_rbi_fold_sp, gi, dim3(BLOCK), 0, s, a, total);
    return hipGetLastError();
  }
  switch (op) {
    PCAD_RBI(ADD)
    PCAD_RBI(MUL)
    PCAD_RBI(MIN)
    PCAD_RBI(MAX)
  default: return hipErrorInvalidValue;
  }
#undef PCAD_RBI
  return hipGetLastError();
}

hipError_t rbi_vjp_launch(int op, int64_t batch, int64_t n, int64_t m, const int32_t *idx,
                          const float *v, const void *saved, const float *hbar, float *vbar,
                          bool accumulate, void *ws, hipStream_t s) {
  if (batch == 0 || n == 0) return hipSuccess;
  if (general_rule(op)) {
    const int d = op == LINREC ? 2 : (op == MAT2 ? 4 : 1);
    void *sws = static_cast<char *>(ws) + base_ws_bytes(op, batch, n, m);
    const char *area = static_cast<const char *>(saved) + op_saved_aligned(op, batch, m);
    const size_t ab = rbi_sort_area_bytes(n, m);
    for (int64_t r = 0; r < batch; ++r) {
      hipError_t e = rbi_sorted_vjp_row(op, n, m, v + r * n * d, hbar + r * m * d,
                                        vbar + r * n * d, accumulate, ws, sws, area + r * ab, s);
      if (e != hipSuccess) return e;
    }
    return hipSuccess;
  }
  RbiVjpArgs a;
  a.idx = idx; a.v = v; a.hbar = hbar; a.vbar = vbar; a.n = n; a.m = m;
  a.accumulate = accumulate ? 1 : 0;
  a.n0 = nullptr; a.ypos = nullptr; a.argk = nullptr; a.ssum = nullptr; a.tab = nullptr;
  const int64_t total = batch * m;
  if (op == MUL) {
    a.n0 = static_cast<const uint32_t *>(saved);
    a.ypos = reinterpret_cast<const float *>(static_cast<const uint32_t *>(saved) + total);
  }
  if (op == MIN || op == MAX) a.argk = static_cast<const int32_t *>(saved);
  if (op == SUMPROD) a.ssum = static_cast<const float *>(saved);
  if (op == MIN || op == MAX) {
    if (!accumulate) {
      const int64_t nt = batch * n;
      hipLaunchKernelGGL(k_rbi_vjp_fill0, dim3((unsigned)grid1d((nt + 3) / 4)), dim3(BLOCK), 0, s,
                         vbar, nt);
    }
    if (total > 0)
      hipLaunchKernelGGL(k_rbi_vjp_scatter, dim3((unsigned)grid1d(total)), dim3(BLOCK), 0, s, a,
                         total);
    return hipGetLastError();
  }
  // bins per row up to which a block builds its record table in LDS (16 KB)
  const int64_t lds_max = op == ADD ? 4096 : (op == MUL ? 1024 : 2048);
  if ((op == ADD || op == SUMPROD) && m > lds_max) {
    const int64_t lm_cap = kBigLdsBytes / (op == ADD ? 4 : 8);
    const int64_t lm = m < lm_cap ? m : lm_cap;
    int dev = 0, cus = 0;
    if (hipGetDevice(&dev) != hipSuccess ||
        hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess)
      return hipErrorInvalidDevice;
    int64_t bx = (cus + batch - 1) / batch;
    const int64_t need = (n + VJP_BIG_TH * 4 - 1) / (VJP_BIG_TH * 4);
    if (bx > need) bx = need;
    if (bx < 1) bx = 1;
    const dim3 grid((unsigned)bx, (unsigned)batch);
    if (op == ADD) hipLaunchKernelGGL(k_rbi_vjp_big<ADD>, grid, dim3(VJP_BIG_TH), 0, s, a, lm);
    else hipLaunchKernelGGL(k_rbi_vjp_big<SUMPROD>, grid, dim3(VJP_BIG_TH), 0, s, a, lm);
    return hipGetLastError();
  }
  const size_t rec = op == ADD ? 4 : (op == MUL ? 16 : 8);  // SUMPROD: 8
  int src = VJP_GATHER;
  if (m <= lds_max) src = VJP_LDS;
  else if (op == MUL && ws != nullptr) src = VJP_TABLE;
  int64_t bx = (n + BLOCK * 4 * 4 - 1) / (BLOCK * 4 * 4);
  // an LDS table is built once per block: fewer, longer blocks
  const int64_t bx_cap = src == VJP_LDS ? 2048 / (batch < 2048 ? batch : 2048) : 65535;
  if (bx > bx_cap) bx = bx_cap;
  if (bx < 1) bx = 1;
  const dim3 grid((unsigned)bx, (unsigned)batch);
  const size_t shm = src == VJP_LDS ? (size_t)m * rec : 0;
  if (src == VJP_TABLE) {
    a.tab = static_cast<char *>(ws) + kCtlBytes;
    const dim3 gi((unsigned)grid1d(total));
    switch (op) {
    case MUL: hipLaunchKernelGGL(k_rbi_vjp_tab<MUL>, gi, dim3(BLOCK), 0, s, a, total); break;
    default: return hipErrorInvalidValue;
    }
  }
  // here + and sumOfProd have m <= lds_max (the 144 KB tables took the rest)
  switch (op) {
  case ADD: hipLaunchKernelGGL((k_rbi_vjp<ADD, VJP_LDS>), grid, dim3(BLOCK), shm, s, a); break;
  case SUMPROD: hipLaunchKernelGGL((k_rbi_vjp<SUMPROD, VJP_LDS>), grid, dim3(BLOCK), shm, s, a); break;
  case MUL:
    if (src == VJP_LDS) hipLaunchKernelGGL((k_rbi_vjp<MUL, VJP_LDS>), grid, dim3(BLOCK), shm, s, a);
    else if (src == VJP_TABLE) hipLaunchKernelGGL((k_rbi_vjp<MUL, VJP_TABLE>), grid, dim3(BLOCK), 0, s, a);
    else hipLaunchKernelGGL((k_rbi_vjp<MUL, VJP_GATHER>), grid, dim3(BLOCK), 0, s, a);
    break;
  default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

}  // namespace pcad
