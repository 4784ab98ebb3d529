// Stable sort of element indices by bin (least-significant-digit radix sort,
// 8-bit digits), the first step of the sort-based reduce-by-index of
// Section 4 (its rule figure sorts iota by key).  Keys outside [0, m) sort
// to the end as bin m.  Output: the keys in ascending order and the
// permutation (original element index of every sorted position); equal keys
// keep ascending original index.
//
// One pass: per-block digit counts (LDS), an exclusive scan of the counts in
// digit-major, block-minor order, and a stable scatter in which every block
// walks its chunk in rounds of one element per thread, ranking each element
// among the round's equal digits with eight ballots (lanes of a wave whose
// digit bits all agree) and a per-digit prefix over the block's waves; the
// chunk is staged in LDS in digit order and written out run by run.
#include "device.hpp"
#include "internal.hpp"

namespace pcad {

constexpr int SORT_TH = 256;                // threads per block
constexpr int SORT_CH = 8192;               // elements per block and pass (staged in LDS)
constexpr int SORT_D = 256;                 // digit values
constexpr int SORT_W = SORT_TH / WAVE;
constexpr int SCAN_TH = 1024, SCAN_PER = 4; // integer scan: entries per block = 4096

__device__ __forceinline__ int32_t clamp_key(int32_t k, int64_t m) {
  return (k < 0 || k >= m) ? (int32_t)m : k;
}

// keys: the caller's keys on the first pass (clamped), else the previous
// pass's sorted keys
__global__ __launch_bounds__(SORT_TH) void k_sort_hist(const int32_t *keys, int64_t n, int64_t m,
                                                       bool first, int shift, int nb,
                                                       uint32_t *counts) {
  __shared__ uint32_t s_c[SORT_D];
  s_c[threadIdx.x] = 0u;  // SORT_TH == SORT_D
  __syncthreads();
  const int64_t lo = (int64_t)blockIdx.x * SORT_CH;
  const int64_t hi = lo + SORT_CH < n ? lo + SORT_CH : n;
  for (int64_t i = lo + threadIdx.x; i < hi; i += SORT_TH) {
    int32_t k = keys[i];
    if (first) k = clamp_key(k, m);
    atomicAdd(&s_c[(k >> shift) & (SORT_D - 1)], 1u);
  }
  __syncthreads();
  counts[(int64_t)threadIdx.x * nb + blockIdx.x] = s_c[threadIdx.x];
}

// exclusive scan of uint32 entries, three kernels: block-local scans with
// block totals, a scan of the totals (one block; at most SCAN_TH*SCAN_PER of
// them), and the add-back
__global__ __launch_bounds__(SCAN_TH) void k_iscan_local(uint32_t *v, int64_t n, uint32_t *tot) {
  __shared__ uint32_t s_w[SCAN_TH / WAVE];
  const int64_t base = (int64_t)blockIdx.x * SCAN_TH * SCAN_PER + (int64_t)threadIdx.x * SCAN_PER;
  uint32_t x[SCAN_PER], s = 0;
#pragma unroll
  for (int j = 0; j < SCAN_PER; ++j) {
    x[j] = base + j < n ? v[base + j] : 0u;
    s += x[j];
  }
  // inclusive wave scan of the thread sums
  const int lane = lane_id(), wave = threadIdx.x / WAVE;
  uint32_t inc = s;
#pragma unroll
  for (int d = 1; d < WAVE; d <<= 1) {
    const uint32_t o = __shfl_up(inc, d, WAVE);
    if (lane >= d) inc += o;
  }
  if (lane == WAVE - 1) s_w[wave] = inc;
  __syncthreads();
  if (threadIdx.x == 0) {
    uint32_t run = 0;
    for (int w = 0; w < SCAN_TH / WAVE; ++w) {
      const uint32_t t = s_w[w];
      s_w[w] = run;
      run += t;
    }
    tot[blockIdx.x] = run;
  }
  __syncthreads();
  uint32_t run = s_w[wave] + inc - s;
#pragma unroll
  for (int j = 0; j < SCAN_PER; ++j) {
    if (base + j < n) v[base + j] = run;
    run += x[j];
  }
}

__global__ __launch_bounds__(SCAN_TH) void k_iscan_totals(uint32_t *tot, int64_t nt) {
  // nt <= SCAN_TH * SCAN_PER: one block scans them like k_iscan_local
  __shared__ uint32_t s_w[SCAN_TH / WAVE];
  const int64_t base = (int64_t)threadIdx.x * SCAN_PER;
  uint32_t x[SCAN_PER], s = 0;
#pragma unroll
  for (int j = 0; j < SCAN_PER; ++j) {
    x[j] = base + j < nt ? tot[base + j] : 0u;
    s += x[j];
  }
  const int lane = lane_id(), wave = threadIdx.x / WAVE;
  uint32_t inc = s;
#pragma unroll
  for (int d = 1; d < WAVE; d <<= 1) {
    const uint32_t o = __shfl_up(inc, d, WAVE);
    if (lane >= d) inc += o;
  }
  if (lane == WAVE - 1) s_w[wave] = inc;
  __syncthreads();
  if (threadIdx.x == 0) {
    uint32_t run = 0;
    for (int w = 0; w < SCAN_TH / WAVE; ++w) {
      const uint32_t t = s_w[w];
      s_w[w] = run;
      run += t;
    }
  }
  __syncthreads();
  uint32_t run = s_w[wave] + inc - s;
#pragma unroll
  for (int j = 0; j < SCAN_PER; ++j) {
    if (base + j < nt) tot[base + j] = run;
    run += x[j];
  }
}

// the block totals are cleared once read (workspace data is not left
// behind)
__global__ __launch_bounds__(SCAN_TH) void k_iscan_add(uint32_t *v, int64_t n, uint32_t *tot) {
  const uint32_t add = tot[blockIdx.x];
  const int64_t base = (int64_t)blockIdx.x * SCAN_TH * SCAN_PER;
  for (int j = threadIdx.x; j < SCAN_TH * SCAN_PER; j += SCAN_TH)
    if (base + j < n) v[base + j] += add;
  __syncthreads();
  if (threadIdx.x == 0) tot[blockIdx.x] = 0u;
}

int64_t iscan_totals(int64_t ne) { return (ne + SCAN_TH * SCAN_PER - 1) / (SCAN_TH * SCAN_PER); }

bool iscan_fits(int64_t ne) { return iscan_totals(ne) <= SCAN_TH * SCAN_PER; }

hipError_t iscan_u32(uint32_t *v, int64_t ne, uint32_t *tot, hipStream_t s) {
  if (ne <= 0) return hipSuccess;
  const int64_t nt = iscan_totals(ne);
  hipLaunchKernelGGL(k_iscan_local, dim3((unsigned)nt), dim3(SCAN_TH), 0, s, v, ne, tot);
  hipLaunchKernelGGL(k_iscan_totals, dim3(1), dim3(SCAN_TH), 0, s, tot, nt);
  hipLaunchKernelGGL(k_iscan_add, dim3((unsigned)nt), dim3(SCAN_TH), 0, s, v, ne, tot);
  return hipGetLastError();
}

// stable scatter of (key, perm) by digit; perm_in == nullptr means the
// identity (first pass).  The block's chunk is staged in LDS in digit order
// first (its digit counts follow from the scanned offsets), then written
// out slot by slot, so each digit's elements leave as one contiguous run
// instead of single scattered words.
__global__ __launch_bounds__(SORT_TH) void k_sort_scatter(const int32_t *keys_in,
                                                          const int32_t *perm_in, int64_t n,
                                                          int64_t m, bool first, int shift, int nb,
                                                          const uint32_t *offsets,
                                                          int32_t *keys_out, int32_t *perm_out) {
  __shared__ uint32_t s_base[SORT_D];          // block's first output position per digit
  __shared__ uint32_t s_rb[SORT_D];            // first stage slot per digit
  __shared__ uint32_t s_cnt[SORT_W][SORT_D];   // this round's count per wave and digit
  __shared__ uint32_t s_off[SORT_W][SORT_D];   // this round's offset per wave and digit
  __shared__ uint32_t s_w[SORT_W];
  __shared__ int32_t s_k[SORT_CH];
  __shared__ int32_t s_p[SORT_CH];
  const int tid = threadIdx.x, lane = lane_id(), wave = tid / WAVE;
  const int64_t ne = (int64_t)SORT_D * nb;
  {
    // digit tid: the block's output base and count; stage bases by an
    // exclusive scan of the counts over the digits
    const int64_t e = (int64_t)tid * nb + blockIdx.x;
    const uint32_t base = offsets[e];
    const uint32_t cnt = (e + 1 < ne ? offsets[e + 1] : (uint32_t)n) - base;
    s_base[tid] = base;
    uint32_t inc = cnt;
#pragma unroll
    for (int dd = 1; dd < WAVE; dd <<= 1) {
      const uint32_t o = __shfl_up(inc, dd, WAVE);
      if (lane >= dd) inc += o;
    }
    if (lane == WAVE - 1) s_w[wave] = inc;
    __syncthreads();
    uint32_t before = 0;
#pragma unroll
    for (int w = 0; w < SORT_W; ++w) before += w < wave ? s_w[w] : 0u;
    s_rb[tid] = before + inc - cnt;
  }
#pragma unroll
  for (int w = 0; w < SORT_W; ++w) s_cnt[w][tid] = 0u;
  uint32_t run = 0;  // thread `tid` tracks digit `tid`: elements placed in earlier rounds
  __syncthreads();
  const int64_t lo = (int64_t)blockIdx.x * SORT_CH;
  const int64_t hi = lo + SORT_CH < n ? lo + SORT_CH : n;
  const uint64_t lt = (lane == 0) ? 0ull : (~0ull >> (WAVE - lane));  // lanes below this one
  for (int64_t r0 = lo; r0 < hi; r0 += SORT_TH) {
    const int64_t i = r0 + tid;
    const bool valid = i < hi;
    int32_t k = 0, p = 0;
    if (valid) {
      k = keys_in[i];
      if (first) k = clamp_key(k, m);
      p = perm_in ? perm_in[i] : (int32_t)i;
    }
    const int d = (k >> shift) & (SORT_D - 1);
    uint64_t peers = __ballot(valid);
#pragma unroll
    for (int b = 0; b < 8; ++b) {
      const uint64_t bb = __ballot((d >> b) & 1);
      peers &= ((d >> b) & 1) ? bb : ~bb;
    }
    const uint32_t rank = (uint32_t)__popcll(peers & lt);
    if (valid && rank == 0) s_cnt[wave][d] = (uint32_t)__popcll(peers);
    __syncthreads();
    {
      uint32_t acc = run;
#pragma unroll
      for (int w = 0; w < SORT_W; ++w) {
        const uint32_t c = s_cnt[w][tid];
        s_off[w][tid] = acc;
        acc += c;
        s_cnt[w][tid] = 0u;
      }
      run = acc;
    }
    __syncthreads();
    if (valid) {
      const uint32_t slot = s_rb[d] + s_off[wave][d] + rank;
      s_k[slot] = k;
      s_p[slot] = p;
    }
  }
  __syncthreads();
  const int len = (int)(hi - lo);
  for (int t = tid; t < len; t += SORT_TH) {
    const int32_t k = s_k[t];
    const int d = (k >> shift) & (SORT_D - 1);
    const uint32_t pos = s_base[d] + (uint32_t)t - s_rb[d];
    keys_out[pos] = k;
    perm_out[pos] = s_p[t];
  }
}

int sort_passes(int64_t m) {
  int bits = 0;
  while (((int64_t)1 << bits) <= m) ++bits;  // keys take values 0..m
  return (bits + 7) / 8;
}

size_t sort_ws_bytes(int64_t n, int64_t m) {
  const int64_t nb = (n + SORT_CH - 1) / SORT_CH;
  const int64_t ne = nb * SORT_D;
  const int64_t nt = (ne + SCAN_TH * SCAN_PER - 1) / (SCAN_TH * SCAN_PER);
  (void)m;
  auto al = [](size_t x) { return (x + 255) / 256 * 256; };
  return al((size_t)n * 4) * 2 + al((size_t)ne * 4) + al((size_t)nt * 4);
}

bool sort_supported(int64_t n) {
  const int64_t nb = (n + SORT_CH - 1) / SORT_CH;
  const int64_t nt = (nb * SORT_D + SCAN_TH * SCAN_PER - 1) / (SCAN_TH * SCAN_PER);
  return n <= 2147483647LL && nt <= SCAN_TH * SCAN_PER;
}

// keys_out/perm_out: n entries each (the sorted keys and the permutation);
// ws: sort_ws_bytes(n, m)
hipError_t sort_by_key(const int32_t *keys, int64_t n, int64_t m, int32_t *keys_out,
                       int32_t *perm_out, void *ws, hipStream_t s) {
  if (n == 0) return hipSuccess;
  const int nb = (int)((n + SORT_CH - 1) / SORT_CH);
  const int64_t ne = (int64_t)nb * SORT_D;
  auto al = [](size_t x) { return (x + 255) / 256 * 256; };
  char *w = static_cast<char *>(ws);
  int32_t *tk = reinterpret_cast<int32_t *>(w);
  int32_t *tp = reinterpret_cast<int32_t *>(w + al((size_t)n * 4));
  uint32_t *counts = reinterpret_cast<uint32_t *>(w + 2 * al((size_t)n * 4));
  uint32_t *tot = reinterpret_cast<uint32_t *>(w + 2 * al((size_t)n * 4) + al((size_t)ne * 4));
  const int passes = sort_passes(m);
  // ping-pong so that the last pass lands in the outputs
  const int32_t *ik = keys;
  const int32_t *ip = nullptr;
  for (int p = 0; p < passes; ++p) {
    const bool last = p == passes - 1;
    const bool odd_from_end = ((passes - 1 - p) & 1) != 0;
    int32_t *ok = last ? keys_out : (odd_from_end ? tk : keys_out);
    int32_t *op = last ? perm_out : (odd_from_end ? tp : perm_out);
    const int shift = 8 * p;
    hipLaunchKernelGGL(k_sort_hist, dim3(nb), dim3(SORT_TH), 0, s, ik, n, m, p == 0, shift, nb, counts);
    hipError_t e = iscan_u32(counts, ne, tot, s);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_sort_scatter, dim3(nb), dim3(SORT_TH), 0, s, ik, ip, n, m, p == 0, shift,
                       nb, counts, ok, op);
    ik = ok;
    ip = op;
  }
  return hipGetLastError();
}

}  // namespace pcad
