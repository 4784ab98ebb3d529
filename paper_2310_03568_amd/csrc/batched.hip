// Batched segmented forward and adjoint of a chained workload: for every
// instance s of a ragged batch,
//   y_s = scan of (a_s, b_s) under linear-function composition
//         (y_i = a_i*y_{i-1} + b_i),
//   (h_s, argk_s) = reduce_by_index(min) of y_s into m bins with keys idx_s,
// and the adjoint of both: y_bar_total = y_bar + onehot(h_bar at argk) fed to
// the scan adjoint (Section 5.2), with the min-by-index adjoint
// (Section 4.2 Min/Max) fused in.
//
// Work items are windows of SEG_T elements aligned to multiples of SEG_T in
// the concatenated array and clipped to an instance, so 16-byte accesses stay
// aligned whatever the instance offsets are.  Items run in dispatch order;
// each instance carries its own look-back chain over its items.  A forward
// item folds its outputs into an LDS sub-histogram of 64-bit (ord(y), index)
// keys; an instance with one item finalises h/argk itself, longer instances
// merge their keys with 64-bit atomic min and a small pass finalises them
// (and resets the keys for the next launch).
#include <algorithm>
#include <vector>

#include "../../include/pcad.h"
#include "adjoint.hpp"
#include "internal.hpp"

namespace pcad {

// Items of SEG_T elements (4096 or 8192) and the block sizes of the forward
// and adjoint kernels (256, 512 or 1024 threads) are template parameters; a
// plan picks one instantiation of each from the tuning knobs when it is
// created (seg.tile, seg.fwd.threads, seg.vjp.threads).
constexpr int SEG_EPL = 4;
constexpr int SEG_MAX_BINS = 1024;

// one record per work item, built on the host at bind time
struct alignas(16) ItemRec {
  int64_t wbase;   // first element of the aligned window
  int64_t start;   // first element of the instance
  int32_t lo, hi;  // the instance's part of the window, relative to wbase
  int32_t s;       // instance
  int32_t li, nli; // item index within the instance, items of the instance
  int32_t len;     // elements of the instance
};

struct SegTables {
  const ItemRec *items;      // [nitems]
  const int64_t *seg_off;    // [S+1] element offsets
  const int32_t *seg_item0;  // [S+1] first item of each instance
};

struct SegItem {
  int64_t s;
  int li, nli;           // item index within the instance, items of the instance
  int64_t wbase;         // first element of the aligned window
  int64_t lo, hi;        // elements of the instance inside the window
  int64_t start, len;    // the instance
  int lo_r, hi_r;        // lo, hi relative to wbase
  int wofs;              // wbase - start: instance index of the window's first element
};

// a block-uniform 64-bit value, held in scalar registers: the item record is
// then read through the scalar cache, so reading it never waits for vector
// loads in flight
__device__ __forceinline__ int64_t uniform64(int64_t v) {
  const uint32_t lo = __builtin_amdgcn_readfirstlane((uint32_t)v);
  const uint32_t hi = __builtin_amdgcn_readfirstlane((uint32_t)((uint64_t)v >> 32));
  return (int64_t)(((uint64_t)hi << 32) | lo);
}

__device__ __forceinline__ SegItem seg_item(const SegTables &t, int64_t item) {
  // the table is never written during a launch: read it as constant memory
  // (the host pass only parses this function)
#if defined(__HIP_DEVICE_COMPILE__)
  typedef const __attribute__((address_space(4))) ItemRec ConstRec;
  const ItemRec r = ((ConstRec *)(t.items))[uniform64(item)];
#else
  const ItemRec r = t.items[item];
#endif
  SegItem q;
  q.s = r.s;
  q.li = r.li;
  q.nli = r.nli;
  q.wbase = r.wbase;
  q.lo = r.wbase + r.lo;
  q.hi = r.wbase + r.hi;
  q.start = r.start;
  q.len = r.len;
  q.lo_r = r.lo;
  q.hi_r = r.hi;
  q.wofs = (int)(r.wbase - r.start);
  return q;
}

// Window loads are split in two so that no lane ever writes a register
// that a load in flight targets (a wave that straddles an instance boundary
// would otherwise have to drain every load it has in flight, once per
// array):
//  * ld_raw issues one 16-byte load for a lane whose group [e, e+4) meets
//    the window's [lo, hi) -- the group of the window at element wbase of an
//    array of N >= 4 elements, or, for a group that runs past the array's
//    end, the array's last four elements -- and leaves the other lanes'
//    registers undefined (no fill is written at load time, and no byte of
//    another instance is fetched);
//  * win_fix, applied where the data is first used (the loads have landed
//    by then anyway), shifts that last group into place and replaces the
//    elements outside [lo, hi) by `fill`.
template <class V, class S>
__device__ __forceinline__ V ld_raw(const S *__restrict__ arr, int64_t N, int64_t wbase, int e,
                                    int lo, int hi) {
  V v;
  if (e + 4 > lo && e < hi) {
    const int64_t i0 = wbase + e;
    v = ld_stream<V>(arr + (i0 + 4 <= N ? i0 : N - 4));
  }
  return v;
}

// which of the group's four elements [e, e+4) lie in the window's [lo, hi)
struct WinMask {
  bool in[4];
};
__device__ __forceinline__ WinMask win_mask(int e, int lo, int hi) {
  WinMask m;
#pragma unroll
  for (int j = 0; j < 4; ++j) m.in[j] = (unsigned)(e + j - lo) < (unsigned)(hi - lo);
  return m;
}

// `tail`: the window reaches past the array's end (a uniform condition, so
// the shifting costs nothing elsewhere)
template <class V, class S>
__device__ __forceinline__ V win_fix(const V &v, const WinMask &m, bool tail, int64_t N,
                                     int64_t wbase, int e, S fill) {
  S x[4] = {v.x, v.y, v.z, v.w};
  if (tail) {
    const int64_t i0 = wbase + e;
    const int64_t sh = i0 + 4 <= N ? 0 : i0 - (N - 4);
    const int s = (int)(sh < 4 ? sh : 4);
    const S y0 = x[0], y1 = x[1], y2 = x[2], y3 = x[3];
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const int q = j + s;
      x[j] = q == 0 ? y0 : (q == 1 ? y1 : (q == 2 ? y2 : (q == 3 ? y3 : fill)));
    }
  }
  V o;
  o.x = m.in[0] ? x[0] : fill;
  o.y = m.in[1] ? x[1] : fill;
  o.z = m.in[2] ? x[2] : fill;
  o.w = m.in[3] ? x[3] : fill;
  return o;
}

__device__ __forceinline__ void st_range(float *__restrict__ w, int e, int lo, int hi, float4 v) {
  const unsigned o = (unsigned)e;
  if (e >= lo && e + 4 <= hi) {
    typedef float v4f __attribute__((ext_vector_type(4)));
    v4f x = {v.x, v.y, v.z, v.w};
    __builtin_nontemporal_store(x, reinterpret_cast<v4f *>(w + o));
    return;
  }
  const float r[4] = {v.x, v.y, v.z, v.w};
#pragma unroll
  for (int j = 0; j < 4; ++j)
    if (e + j >= lo && e + j < hi) w[o + j] = r[j];
}

__device__ __forceinline__ int i4get(const int4 &v, int j) {
  return j == 0 ? v.x : (j == 1 ? v.y : (j == 2 ? v.z : v.w));
}

// ---------------------------------------------------------------------------
// forward
// ---------------------------------------------------------------------------
struct SegFwdArgs {
  SegTables tab;
  int64_t nitems;
  int64_t n;           // elements of the concatenated arrays
  int S, m;
  int nrows;           // instances with at least one element
  const float *a, *b;
  const int32_t *idx;
  float *y, *h;
  int32_t *argk;
  float *carry;        // [nitems][2] exclusive prefix (A, y) of every item
  uint64_t *keys;      // [S][m] merge keys of multi-item instances, ~0 between launches
  Ctl *ctl;
  uint64_t *status;
};

// Persistent: the grid holds the resident blocks; block b takes items
// b, b+G, ... in item order.  As in the plain scan, an item's look-back runs
// one iteration after its aggregate was published (the block scans and
// publishes its next item in between).  The pending item's item-local
// prefixes and keys wait in LDS; its outputs and LDS sub-histogram follow
// the look-back.
template <int SEG_T, int TH>
__global__ __launch_bounds__(TH) void k_seg_fwd(SegFwdArgs a) {
  using Op = FwdLB<LINREC>;
  using T = Op::T;
  constexpr int EPL = SEG_EPL, K = SEG_T / (TH * EPL), W = TH / WAVE;
  static_assert(K >= 1 && K * TH * EPL == SEG_T, "items must be whole groups of the block");

  __shared__ T s_tot[K][W];
  __shared__ T s_pre[K][W];
  __shared__ T s_carry;
  __shared__ unsigned s_epoch;
  __shared__ unsigned long long s_keys[SEG_MAX_BINS];
  __shared__ float4 s_pv[SEG_T / 2];  // pending item: (A, y) item-local prefix per element
  __shared__ int4 s_pix[SEG_T / 4];   // pending item: bin keys

  const int tid = threadIdx.x, lane = lane_id(), wave = tid / WAVE;
  const int64_t G = gridDim.x;
  if (tid == 0) s_epoch = ctl_load(&a.ctl->epoch);

  float4 ca[K], cb[K];  // the prefetched item
  int4 ci[K];
  auto load_grp = [&](const SegItem &it, int g) {
    const int e = g * TH * EPL + tid * EPL;
    ca[g] = ld_raw<float4>(a.a, a.n, it.wbase, e, it.lo_r, it.hi_r);
    cb[g] = ld_raw<float4>(a.b, a.n, it.wbase, e, it.lo_r, it.hi_r);
    ci[g] = ld_raw<int4>(a.idx, a.n, it.wbase, e, it.lo_r, it.hi_r);
  };
  auto load = [&](const SegItem &it) {
#pragma unroll
    for (int g = 0; g < K; ++g) load_grp(it, g);
  };
  int64_t i = blockIdx.x;  // the item whose outputs are pending
  SegItem it = seg_item(a.tab, i);
  load(it);
  __syncthreads();
  const uint32_t tag = next_tag(s_epoch);

  // scans the prefetched item into item-local inclusive prefixes (v) and its
  // fixed keys (ix) and, in wave 0, the item aggregate (ag), which is
  // published (an instance's first item publishes it as its inclusive
  // prefix).  after(g) runs once group g of the prefetch registers has been
  // read for the last time: the next item's loads for that group go out
  // there, a group at a time, instead of all at once after the scan.
  auto phase1 = [&](const SegItem &jt, int64_t item, T (&v)[K][EPL], int4 (&ix)[K], T &ag,
                    auto &&after) {
    T incl[K];
    const bool tail = jt.wbase + SEG_T > a.n;
#pragma unroll
    for (int g = 0; g < K; ++g) {
      const int e = g * TH * EPL + tid * EPL;
      const WinMask wm = win_mask(e, jt.lo_r, jt.hi_r);
      ca[g] = win_fix(ca[g], wm, tail, a.n, jt.wbase, e, 1.0f);
      cb[g] = win_fix(cb[g], wm, tail, a.n, jt.wbase, e, 0.0f);
      ci[g] = win_fix(ci[g], wm, tail, a.n, jt.wbase, e, -1);
    }
#pragma unroll
    for (int g = 0; g < K; ++g) {
      T acc = {{f4get(ca[g], 0), f4get(cb[g], 0)}};
      v[g][0] = acc;
#pragma unroll
      for (int j = 1; j < EPL; ++j) {
        acc = Op::comb(acc, T{{f4get(ca[g], j), f4get(cb[g], j)}});
        v[g][j] = acc;
      }
      ix[g] = ci[g];
      after(g);
      incl[g] = wave_scan_fwd<Op>(acc);
      if (lane == WAVE - 1) s_tot[g][wave] = incl[g];
    }
    __syncthreads();
    if (wave == 0) {
      ag = wave0_block_prefix<Op, K, W, false>(s_tot, s_pre, Op::id());
      uint64_t *st = a.status + item * (Op::NA + Op::NP);
      if (lane == 0) publish<2>(jt.li == 0 ? st + Op::NA : st, tag, ag);
    }
    __syncthreads();
#pragma unroll
    for (int g = 0; g < K; ++g) {
      T ex = shift_up1(incl[g]);
      if (lane == 0) ex = Op::id();
      const T thr = Op::comb(s_pre[g][wave], ex);
#pragma unroll
      for (int j = 0; j < EPL; ++j) v[g][j] = Op::comb(thr, v[g][j]);
    }
  };
  // element el of an item: group el / (TH*EPL), thread (el % (TH*EPL)) / EPL
  auto put_pending = [&](const T (&v)[K][EPL], const int4 (&ix)[K]) {
#pragma unroll
    for (int g = 0; g < K; ++g) {
      const int q = g * TH + tid;  // 4-element group index
      s_pv[q * 2 + 0] = make_float4(v[g][0].f[0], v[g][0].f[1], v[g][1].f[0], v[g][1].f[1]);
      s_pv[q * 2 + 1] = make_float4(v[g][2].f[0], v[g][2].f[1], v[g][3].f[0], v[g][3].f[1]);
      s_pix[q] = ix[g];
    }
  };

  T pagg = Op::id();       // wave 0: aggregate of the pending item
  T prev_incl = Op::id();  // wave 0: inclusive prefix of the block's previous item
  int64_t in = i + G;
  SegItem nt = it;
  {
    const bool has = in < a.nitems;
    if (has) nt = seg_item(a.tab, in);
    T v[K][EPL];
    int4 iv[K];
    phase1(it, i, v, iv, pagg, [&](int g) {
      if (has) load_grp(nt, g);
    });
    put_pending(v, iv);
  }
  for (;;) {
    const bool more = in < a.nitems;
    T nv[K][EPL];
    int4 niv[K];
    T nagg = Op::id();
    SegItem nnt = nt;
    if (more) {
      const bool has = in + G < a.nitems;
      if (has) nnt = seg_item(a.tab, in + G);
      phase1(nt, in, nv, niv, nagg, [&](int g) {
        if (has) load_grp(nnt, g);
      });
    }

    if (wave == 0) {
      T c = Op::id();
      if (it.li > 0) {
        // predecessors at distances 1..G-1 belong to other blocks; the one at
        // distance G is this block's previous item, in the same instance
        const int win = it.li < G ? it.li : (int)(G - 1);
        bool hit = false;
        if (win > 0) c = lookback<Op>(a.status, i, +1, win, tag, a.ctl, &hit);
        if (!hit) c = win > 0 ? Op::comb(prev_incl, c) : prev_incl;
        if (lane == 0) publish<2>(a.status + i * (Op::NA + Op::NP) + Op::NA, tag, Op::comb(c, pagg));
      }
      prev_incl = Op::comb(c, pagg);
      if (lane == 0) {
        s_carry = c;
        if (it.li == it.nli - 1) ctl_row_done(a.ctl, (unsigned)a.nrows, tag);
        a.carry[i * 2 + 0] = c.f[0];
        a.carry[i * 2 + 1] = c.f[1];
      }
    }
    for (int k = tid; k < a.m; k += TH) s_keys[k] = key_init<MIN>();
    __syncthreads();
    const T carry = s_carry;

#pragma unroll
    for (int g = 0; g < K; ++g) {
      const int q = g * TH + tid;
      const float4 p0 = s_pv[q * 2 + 0], p1 = s_pv[q * 2 + 1];
      const int4 ix = s_pix[q];
      const float pa[4] = {p0.x, p0.z, p1.x, p1.z}, py[4] = {p0.y, p0.w, p1.y, p1.w};
      const int e = g * TH * EPL + tid * EPL;
      float4 o;
#pragma unroll
      for (int j = 0; j < EPL; ++j) {
        const float yv = Op::comb(carry, T{{pa[j], py[j]}}).f[1];
        f4set(o, j, yv);
        const int k = i4get(ix, j);
        if (k >= 0 && k < a.m) {  // elements outside the instance carry key -1
          const unsigned long long key = key_of<MIN>(yv, (uint32_t)(it.wofs + e + j));
          atomicMin(&s_keys[k], key);
        }
      }
      st_range(a.y + it.wbase, e, it.lo_r, it.hi_r, o);
    }
    __syncthreads();
    // the pending slot is free: the next item waits there
    if (more) put_pending(nv, niv);

    const int64_t hb = it.s * a.m;
    if (it.nli == 1) {
      // the item holds the whole instance: finalise directly
      for (int k = tid; k < a.m; k += TH) {
        const uint64_t key = s_keys[k];
        if (key == key_init<MIN>()) {
          a.h[hb + k] = __builtin_inff();
          a.argk[hb + k] = (int32_t)it.len;
        } else {
          a.h[hb + k] = ord_inv((uint32_t)(key >> 32));
          a.argk[hb + k] = (int32_t)(uint32_t)key;
        }
      }
    } else {
      for (int k = tid; k < a.m; k += TH) {
        const unsigned long long key = s_keys[k];
        if (key != key_init<MIN>())
          __hip_atomic_fetch_min(reinterpret_cast<unsigned long long *>(&a.keys[hb + k]), key,
                                 __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      }
    }
    if (!more) break;
    // s_keys, s_pv, s_carry and s_pre are rewritten only after barriers that
    // every thread reaches after its reads above
    i = in;
    it = nt;
    in = i + G;
    nt = nnt;
    pagg = nagg;
  }
}

// finalise the instances spanning several items; reset their keys
__global__ __launch_bounds__(256) void k_seg_fin(SegFwdArgs a) {
  const int64_t total = (int64_t)a.S * a.m;
  for (int64_t t = (int64_t)blockIdx.x * 256 + threadIdx.x; t < total;
       t += (int64_t)gridDim.x * 256) {
    const int64_t s = t / a.m;
    const int nli = a.tab.seg_item0[s + 1] - a.tab.seg_item0[s];
    if (nli == 1) continue;  // finalised by its only item
    if (nli == 0) {          // empty instance: neutral bin, sentinel 0
      a.h[t] = __builtin_inff();
      a.argk[t] = 0;
      continue;
    }
    const uint64_t key = a.keys[t];
    if (key == key_init<MIN>()) {
      a.h[t] = __builtin_inff();
      a.argk[t] = (int32_t)(a.tab.seg_off[s + 1] - a.tab.seg_off[s]);
    } else {
      a.h[t] = ord_inv((uint32_t)(key >> 32));
      a.argk[t] = (int32_t)(uint32_t)key;
      a.keys[t] = key_init<MIN>();
    }
  }
}

__global__ void k_fill_u64(uint64_t *p, int64_t n, uint64_t v) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x)
    p[i] = v;
}

// ---------------------------------------------------------------------------
// adjoint
// ---------------------------------------------------------------------------
struct SegBwdArgs {
  SegTables tab;
  int64_t nitems;
  int64_t n;             // elements of the concatenated arrays
  int S, m;
  int nrows;
  const float *a, *b;
  const int32_t *idx;
  const float *y;        // forward output (read for the prefixes y_{i-1})
  const int32_t *argk;
  const float *ybar, *hbar;
  float *abar, *bbar;
  Ctl *ctl;
  uint64_t *status;
};

// Persistent: block b takes items nitems-1-b, nitems-1-b-G, ... (right to
// left).  One iteration prefetches the next item (a, the forward output y,
// y_bar, keys, and the bins' argk / h_bar entries), resolves the current
// item's look-back, sweeps and stores it, then scans the next item:
// y_bar_total = y_bar + h_bar at the bin's argmin, the adjoint maps of the
// recurrence scanned right to left and the item aggregate published.  The
// forward prefix y_{i-1} that a_bar needs is read from the forward output
// (the forward of this workload stores y anyway), so the adjoint never
// re-runs the forward recurrence and never reads b.
template <int SEG_T, int TH>
__global__ __launch_bounds__(TH) void k_seg_bwd(SegBwdArgs a) {
  using FT = Fwd<LINREC>::T;
  using M = MapScalT<false>;
  using MT = M::T;
  using A = Adj<LINREC, false>;
  constexpr int EPL = SEG_EPL, K = SEG_T / (TH * EPL), W = TH / WAVE;
  static_assert(K >= 1 && K * TH * EPL == SEG_T, "items must be whole groups of the block");
  constexpr int TPT = (SEG_MAX_BINS + TH - 1) / TH;  // bin entries per thread

  __shared__ MT s_mtot[K][W];
  __shared__ MT s_mpre[K][W];
  __shared__ MT s_carry;
  __shared__ unsigned s_epoch;
  __shared__ int2 s_bin[SEG_MAX_BINS];  // (argk, h_bar bits) of the item's instance, per bin

  const int tid = threadIdx.x, lane = lane_id(), wave = tid / WAVE;
  const int64_t G = gridDim.x;
  if (tid == 0) s_epoch = ctl_load(&a.ctl->epoch);

  // what the scan of an item reads: raw window loads, fixed where first used
  struct Buf {
    float4 a[K], yb[K];
    int4 ix[K];
    int32_t ak[TPT];
    float hb[TPT];
  };
  // what only its sweep reads: the forward output
  struct YBuf {
    float4 y[K];
    float yp0[K];  // lane 0: y of the element before the lane's group (0 at an instance start)
  };
  auto load_grp = [&](const SegItem &it, Buf &B, int g) {
    const int e = g * TH * EPL + tid * EPL;
    B.a[g] = ld_raw<float4>(a.a, a.n, it.wbase, e, it.lo_r, it.hi_r);
    B.yb[g] = ld_raw<float4>(a.ybar, a.n, it.wbase, e, it.lo_r, it.hi_r);
    B.ix[g] = ld_raw<int4>(a.idx, a.n, it.wbase, e, it.lo_r, it.hi_r);
  };
  auto load_bins = [&](const SegItem &it, Buf &B) {
    const int64_t hb = it.s * a.m;
#pragma unroll
    for (int r = 0; r < TPT; ++r) {
      // every lane loads (entries past m are never put in LDS)
      const int k = tid + r * TH;
      const int kc = k < a.m ? k : a.m - 1;
      B.ak[r] = a.argk[hb + kc];
      B.hb[r] = a.hbar[hb + kc];
    }
  };
  auto load_y = [&](const SegItem &it, YBuf &Y) {
#pragma unroll
    for (int g = 0; g < K; ++g) {
      const int e = g * TH * EPL + tid * EPL;
      Y.y[g] = ld_raw<float4>(a.y, a.n, it.wbase, e, it.lo_r, it.hi_r);
      // element e-1 lies in the instance iff its instance index is >= 0 and
      // it is before the instance's end in this window
      Y.yp0[g] = 0.0f;
      if (lane == 0 && it.wofs + e - 1 >= 0 && e - 1 < it.hi_r) Y.yp0[g] = a.y[it.wbase + e - 1];
    }
  };
  auto item_of = [&](int64_t kk) { return a.nitems - 1 - kk; };

  uint32_t tag = 0;  // this launch's tag, set once the epoch has been read
  MT mincl[K];
  MT agg = M::id();        // wave 0: map aggregate of the current item
  MT prev_incl = M::id();  // wave 0: carry into the block's previous item, combined with it

  // Scans the item in B (its bin entries already in LDS).  After each group,
  // `after(g)` may issue that group's loads for a later item.
  auto phase1 = [&](const SegItem &jt, int64_t item, Buf &B, auto &&after) {
    const bool tail = jt.wbase + SEG_T > a.n;
#pragma unroll
    for (int g = 0; g < K; ++g) {
      const int e = g * TH * EPL + tid * EPL;
      const WinMask wm = win_mask(e, jt.lo_r, jt.hi_r);
      const float4 av = win_fix(B.a[g], wm, tail, a.n, jt.wbase, e, 1.0f);
      float4 ybv = win_fix(B.yb[g], wm, tail, a.n, jt.wbase, e, 0.0f);
      const int4 ixv = win_fix(B.ix[g], wm, tail, a.n, jt.wbase, e, -1);
      // the group's four bin records, read together (one LDS round trip)
      int2 bv[EPL];
#pragma unroll
      for (int j = 0; j < EPL; ++j) {
        const int kb = i4get(ixv, j);
        bv[j] = s_bin[(unsigned)kb < (unsigned)a.m ? kb : 0];
      }
      MT acc = M::id();
#pragma unroll
      for (int j = EPL - 1; j >= 0; --j) {
        // y_bar_total = y_bar + h_bar at the bin's argmin (fused min-by-index adjoint)
        const int kb = i4get(ixv, j);
        const bool hit = (unsigned)kb < (unsigned)a.m && bv[j].x == jt.wofs + e + j;
        const float y0 = f4get(ybv, j);
        f4set(ybv, j, hit ? y0 + __int_as_float(bv[j].y) : y0);
        const float yb[2] = {f4get(ybv, j), 0.0f};
        const MT hm = A::make(FT{{1.0f, 0.0f}}, FT{{f4get(av, j), 0.0f}}, yb, false);
        acc = (j == EPL - 1) ? hm : M::comb(acc, hm);
      }
      // the sweep reads the fixed values
      B.a[g] = av;
      B.yb[g] = ybv;
      after(g);
      mincl[g] = wave_scan_rev<M>(acc);
      if (lane == 0) s_mtot[g][wave] = mincl[g];
    }
    __syncthreads();
    if (wave == 0) {
      agg = wave0_block_prefix<M, K, W, true>(s_mtot, s_mpre, M::id());
      uint64_t *st = a.status + item * (M::NA + M::NP);
      if (lane == 0) {
        if (jt.li == jt.nli - 1)
          publish<M::NP>(st + M::NA, tag, M::apply0(M::comb(M::from_pre(M::P{{0.0f}}), agg)));
        else
          publish<M::NA>(st, tag, agg);
      }
    }
  };
  auto put_bins = [&](const Buf &B) {
#pragma unroll
    for (int r = 0; r < TPT; ++r) {
      const int kb = tid + r * TH;
      if (kb < a.m) s_bin[kb] = make_int2(B.ak[r], __float_as_int(B.hb[r]));
    }
  };

  // Two register buffers alternate roles: `cur` holds the scanned item k,
  // `nxt` the loads of item k+G.  Once item k is swept, the loads of item
  // k+2G go into `cur` a group at a time while item k+G is scanned, so the
  // memory requests of the next items are in flight through the scan, the
  // look-back and the sweep, and no wave stalls issuing a whole item's loads
  // at once.  The loop is unrolled by two so that no register of a load in
  // flight is ever copied.  The forward output y, which only the sweep
  // reads, has one buffer of its own, loaded for item k+G as soon as item k
  // is swept.
  int64_t k = blockIdx.x;
  SegItem it = seg_item(a.tab, item_of(k));
  Buf b0, b1;
  YBuf yv;
#pragma unroll
  for (int g = 0; g < K; ++g) load_grp(it, b0, g);
  load_bins(it, b0);
  __syncthreads();
  tag = next_tag(s_epoch);
  put_bins(b0);
  __syncthreads();
  SegItem nt = it;
  const bool has1 = k + G < a.nitems;
  if (has1) nt = seg_item(a.tab, item_of(k + G));
  phase1(it, item_of(k), b0, [&](int g) {
    if (has1) load_grp(nt, b1, g);
  });
  if (has1) load_bins(nt, b1);
  load_y(it, yv);

  auto step = [&](Buf &cur, Buf &nxt) -> bool {
    const int64_t item = item_of(k);
    if (wave == 0) {
      MT c = M::from_pre(M::P{{0.0f}});
      const int dist_max = it.nli - 1 - it.li;
      if (dist_max > 0) {
        // successors at distances 1..G-1 belong to other blocks; the one at
        // distance G is this block's previous item, in the same instance
        const int win = dist_max < G ? dist_max : (int)(G - 1);
        bool hit = false;
        if (win > 0) c = lookback<M>(a.status, item, -1, win, tag, a.ctl, &hit);
        if (!hit) c = win > 0 ? M::comb(prev_incl, c) : prev_incl;
        if (lane == 0)
          publish<M::NP>(a.status + item * (M::NA + M::NP) + M::NA, tag, M::apply0(M::comb(c, agg)));
      }
      prev_incl = M::from_pre(M::apply0(M::comb(c, agg)));
      if (lane == 0) {
        s_carry = c;
        if (it.li == 0) ctl_row_done(a.ctl, (unsigned)a.nrows, tag);
      }
    }
    __syncthreads();
    const MT carry = s_carry;
    const bool tail = it.wbase + SEG_T > a.n;

#pragma unroll
    for (int g = 0; g < K; ++g) {
      MT ex = shift_down1(mincl[g]);
      if (lane == WAVE - 1) ex = M::id();
      M::P rho = M::apply0(M::comb(M::comb(carry, s_mpre[g][wave]), ex));
      const int e = g * TH * EPL + tid * EPL;
      const float4 yg = win_fix(yv.y[g], win_mask(e, it.lo_r, it.hi_r), tail, a.n, it.wbase, e, 0.0f);
      // y_{i-1} of the four slots: the left neighbour's last y for the first
      float yprev0 = dpp_f<kDppWaveShr1>(yg.w);
      if (lane == 0) yprev0 = yv.yp0[g];
      const float yprev[4] = {yprev0, yg.x, yg.y, yg.z};
      float4 oa, ob;
#pragma unroll
      for (int j = EPL - 1; j >= 0; --j) {
        const float yb[2] = {f4get(cur.yb[g], j), 0.0f};
        float xb[2];
        A::step(FT{{1.0f, yprev[j]}}, FT{{f4get(cur.a[g], j), 0.0f}}, yb, false, rho, xb);
        f4set(oa, j, xb[0]);
        f4set(ob, j, xb[1]);
      }
      st_range(a.abar + it.wbase, e, it.lo_r, it.hi_r, oa);
      st_range(a.bbar + it.wbase, e, it.lo_r, it.hi_r, ob);
    }
    if (k + G >= a.nitems) return false;
    // the next item's forward output first (its sweep comes first)
    load_y(nt, yv);
    const bool has2 = k + 2 * G < a.nitems;
    SegItem nnt = nt;
    if (has2) nnt = seg_item(a.tab, item_of(k + 2 * G));
    __syncthreads();  // LDS of the finished item is rewritten below
    put_bins(nxt);
    __syncthreads();
    phase1(nt, item_of(k + G), nxt, [&](int g) {
      if (has2) load_grp(nnt, cur, g);
    });
    if (has2) load_bins(nnt, cur);
    k += G;
    it = nt;
    nt = nnt;
    return true;
  };
  for (;;) {
    if (!step(b0, b1)) break;
    if (!step(b1, b0)) break;
  }
}

}  // namespace pcad

// ---------------------------------------------------------------------------
// plan (host)
// ---------------------------------------------------------------------------
using namespace pcad;

struct pcad_plan {
  int64_t S = 0, N = 0, m = 0, nitems = 0, nrows = 0;
  unsigned flags = 0;
  int tile = 8192, thf = 512, thb = 512;  // item size and block sizes, fixed at creation
  std::vector<int64_t> off;
  std::vector<ItemRec> item_rec;
  std::vector<int32_t> seg_item0;
  // workspace layout
  size_t ws_status = 0, ws_keys = 0, ws_tab = 0, ws_plain = 0, ws_bytes = 0;
  size_t tab_off = 0, tab_item0 = 0;  // table offsets inside the table region
  size_t sv_carry = 0, sv_plain = 0, saved_bytes = 0;
  size_t plain_ws_bytes = 0;
  // bound buffers
  bool bound = false;
  const float *a = nullptr, *b = nullptr, *ybar = nullptr, *hbar = nullptr;
  const int32_t *idx = nullptr;
  float *y = nullptr, *h = nullptr, *abar = nullptr, *bbar = nullptr;
  int32_t *argk = nullptr;
  char *saved = nullptr, *ws = nullptr;
  SegFwdArgs fa;
  SegBwdArgs ba;
  hipGraphExec_t g[4] = {nullptr, nullptr, nullptr, nullptr};
  // graphs are captured on this private stream: the caller's stream may be
  // the legacy null stream, which cannot be captured
  hipStream_t cap = nullptr;
};

namespace {

thread_local int g_plan_hip = 0;

size_t align256(size_t x) { return (x + 255) / 256 * 256; }

int plan_hip(hipError_t e) {
  if (e == hipSuccess) return PCAD_OK;
  g_plan_hip = (int)e;
  return hip_status(e);
}

// persistent grids: as many blocks as can be resident at once (a block waits
// only on items of lower order in its direction, owned by resident blocks)
template <class F>
int64_t seg_grid(F kernel, int threads, int64_t nitems) {
  int dev = 0, cus = 0, occ = 0;
  if (hipGetDevice(&dev) != hipSuccess) return 0;
  if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess) return 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&occ, kernel, threads, 0) != hipSuccess) return 0;
  const int64_t cap = (int64_t)cus * (occ > 0 ? occ : 1);
  return nitems < cap ? nitems : cap;
}

template <int T, int TH>
hipError_t launch_fwd_t(pcad_plan *p, hipStream_t s) {
  const int64_t grid = seg_grid(k_seg_fwd<T, TH>, TH, p->nitems);
  if (grid == 0) return hipErrorInvalidDevice;
  hipLaunchKernelGGL((k_seg_fwd<T, TH>), dim3((unsigned)grid), dim3(TH), 0, s, p->fa);
  return hipGetLastError();
}

template <int T, int TH>
hipError_t launch_bwd_t(pcad_plan *p, hipStream_t s) {
  const int64_t grid = seg_grid(k_seg_bwd<T, TH>, TH, p->nitems);
  if (grid == 0) return hipErrorInvalidDevice;
  hipLaunchKernelGGL((k_seg_bwd<T, TH>), dim3((unsigned)grid), dim3(TH), 0, s, p->ba);
  return hipGetLastError();
}

template <int T>
hipError_t launch_fwd_tile(pcad_plan *p, hipStream_t s) {
  switch (p->thf) {
  case 256: return launch_fwd_t<T, 256>(p, s);
  case 1024: return launch_fwd_t<T, 1024>(p, s);
  default: return launch_fwd_t<T, 512>(p, s);
  }
}

template <int T>
hipError_t launch_bwd_tile(pcad_plan *p, hipStream_t s) {
  switch (p->thb) {
  case 256: return launch_bwd_t<T, 256>(p, s);
  case 1024: return launch_bwd_t<T, 1024>(p, s);
  default: return launch_bwd_t<T, 512>(p, s);
  }
}

hipError_t launch_fwd_nodes(pcad_plan *p, hipStream_t s) {
  if (p->nitems > 0) {
    const hipError_t e = p->tile == 4096 ? launch_fwd_tile<4096>(p, s) : launch_fwd_tile<8192>(p, s);
    if (e != hipSuccess) return e;
  }
  hipLaunchKernelGGL(k_seg_fin, dim3(2048), dim3(256), 0, s, p->fa);
  return hipGetLastError();
}

hipError_t launch_bwd_nodes(pcad_plan *p, hipStream_t s) {
  if (p->nitems > 0)
    return p->tile == 4096 ? launch_bwd_tile<4096>(p, s) : launch_bwd_tile<8192>(p, s);
  return hipSuccess;
}

}  // namespace

extern "C" {

int pcad_plan_create(pcad_plan **out, int64_t nseg, const int64_t *offsets, int64_t m,
                     unsigned flags) {
  if (!out || !offsets) return PCAD_E_NULLPTR;
  *out = nullptr;
  if (nseg < 1 || m < 1) return PCAD_E_INVALID_ARG;
  if (m > SEG_MAX_BINS || nseg > (1 << 24)) return PCAD_E_SIZE;
  if (flags & ~(unsigned)PCAD_PLAN_PER_SEGMENT) return PCAD_E_INVALID_ARG;
  if (offsets[0] != 0) return PCAD_E_INVALID_ARG;
  for (int64_t s = 0; s < nseg; ++s) {
    if (offsets[s + 1] < offsets[s]) return PCAD_E_INVALID_ARG;
    if (offsets[s + 1] - offsets[s] > 2147483647LL) return PCAD_E_SIZE;
  }
  if (offsets[nseg] > (1LL << 40)) return PCAD_E_SIZE;
  pcad_plan *p = new pcad_plan();
  p->S = nseg;
  p->m = m;
  p->flags = flags;
  p->tile = (int)knob_seg_tile();
  p->thf = knob_seg_threads(0);
  p->thb = knob_seg_threads(1);
  const int64_t SEG_T = p->tile;
  p->off.assign(offsets, offsets + nseg + 1);
  p->N = offsets[nseg];
  p->seg_item0.resize(nseg + 1);
  int64_t items = 0;
  for (int64_t s = 0; s < nseg; ++s) {
    p->seg_item0[s] = (int32_t)items;
    const int64_t st = offsets[s], en = offsets[s + 1];
    if (en > st) {
      items += (en - 1) / SEG_T - st / SEG_T + 1;
      p->nrows++;
    }
    if (items > 2147483647LL) {
      delete p;
      return PCAD_E_SIZE;
    }
  }
  p->seg_item0[nseg] = (int32_t)items;
  p->nitems = items;
  p->item_rec.resize(items > 0 ? items : 1);
  for (int64_t s = 0; s < nseg; ++s) {
    const int64_t st = offsets[s], en = offsets[s + 1];
    const int32_t i0 = p->seg_item0[s], nli = p->seg_item0[s + 1] - i0;
    for (int32_t li = 0; li < nli; ++li) {
      ItemRec &r = p->item_rec[i0 + li];
      r.wbase = (st / SEG_T + li) * (int64_t)SEG_T;
      r.start = st;
      r.lo = (int32_t)(std::max(st, r.wbase) - r.wbase);
      r.hi = (int32_t)(std::min(en, r.wbase + SEG_T) - r.wbase);
      r.s = (int32_t)s;
      r.li = li;
      r.nli = nli;
      r.len = (int32_t)(en - st);
    }
  }

  // workspace: control block, status words, merge keys, tables, plain-path scratch
  const int words = 4;  // linrec forward (2+2) and adjoint map (2+1) status words
  size_t o = kCtlBytes;
  p->ws_status = o;
  o = align256(o + (size_t)(items > 0 ? items : 1) * words * sizeof(uint64_t));
  p->ws_keys = o;
  o = align256(o + (size_t)nseg * m * sizeof(uint64_t));
  p->ws_tab = o;
  // the three tables, each starting on a 256-byte boundary (as bound)
  p->tab_off = align256(p->item_rec.size() * sizeof(ItemRec));
  p->tab_item0 = p->tab_off + align256((size_t)(nseg + 1) * 8);
  o = align256(o + p->tab_item0 + (size_t)(nseg + 1) * 4);
  p->ws_plain = o;
  size_t sv = 0;
  p->sv_carry = 0;
  sv = align256((size_t)(items > 0 ? items : 1) * 2 * sizeof(float));
  p->sv_plain = sv;
  if (flags & PCAD_PLAN_PER_SEGMENT) {
    // per-instance plain calls: one call's workspace (reused in order), the
    // summed output adjoint, and the per-instance scan prefixes and argk
    size_t wmax = 0, cmax = 0;
    for (int64_t s = 0; s < nseg; ++s) {
      const int64_t L = offsets[s + 1] - offsets[s];
      size_t w1 = 0, w2 = 0, s1 = 0;
      pcad_query(PCAD_SCAN, PCAD_LINREC, 1, L, 0, 0, &s1, &w1);
      pcad_query(PCAD_RBI, PCAD_MIN, 1, L, m, 0, nullptr, &w2);
      wmax = std::max(wmax, std::max(w1, w2));
      cmax += align256(s1);
    }
    p->plain_ws_bytes = wmax;
    o = align256(o + wmax);
    o = align256(o + (size_t)p->N * sizeof(float));  // y_bar_total
    sv = align256(sv + cmax);
  }
  p->ws_bytes = o;
  p->saved_bytes = sv;
  *out = p;
  return PCAD_OK;
}

int pcad_plan_query(const pcad_plan *p, size_t *saved_bytes, size_t *workspace_bytes,
                    int64_t *n_elements, int64_t *n_items) {
  if (!p) return PCAD_E_NULLPTR;
  if (saved_bytes) *saved_bytes = p->saved_bytes;
  if (workspace_bytes) *workspace_bytes = p->ws_bytes;
  if (n_elements) *n_elements = p->N;
  if (n_items) *n_items = p->nitems;
  return PCAD_OK;
}

int pcad_plan_bind(pcad_plan *p, const float *a, const float *b, const int32_t *idx, float *y,
                   float *h, int32_t *argk, const float *ybar, const float *hbar, float *abar,
                   float *bbar, void *saved, void *ws, size_t ws_bytes, void *stream) {
  if (!p) return PCAD_E_NULLPTR;
  if (!saved || !ws || !h || !argk || !hbar) return PCAD_E_NULLPTR;
  if (p->N > 0 && (!a || !b || !idx || !y || !ybar || !abar || !bbar)) return PCAD_E_NULLPTR;
  const void *al[] = {a, b, idx, y, h, argk, ybar, hbar, abar, bbar, saved};
  for (const void *q : al)
    if (q && ((uintptr_t)q & 15u)) return PCAD_E_MISALIGNED;
  if ((uintptr_t)ws & 255u) return PCAD_E_MISALIGNED;
  if (ws_bytes < p->ws_bytes) return PCAD_E_WORKSPACE;
  hipStream_t s = (hipStream_t)stream;
  for (int i = 0; i < 4; ++i)
    if (p->g[i]) {
      (void)hipGraphExecDestroy(p->g[i]);
      p->g[i] = nullptr;
    }
  p->bound = false;
  p->a = a; p->b = b; p->idx = idx; p->y = y; p->h = h; p->argk = argk;
  p->ybar = ybar; p->hbar = hbar; p->abar = abar; p->bbar = bbar;
  p->saved = static_cast<char *>(saved);
  p->ws = static_cast<char *>(ws);

  // device tables
  char *tab = p->ws + p->ws_tab;
  ItemRec *d_items = reinterpret_cast<ItemRec *>(tab);
  int64_t *d_off = reinterpret_cast<int64_t *>(tab + p->tab_off);
  int32_t *d_item0 = reinterpret_cast<int32_t *>(tab + p->tab_item0);
  int st = plan_hip(hipMemcpyAsync(d_items, p->item_rec.data(), p->item_rec.size() * sizeof(ItemRec),
                                   hipMemcpyHostToDevice, s));
  if (st == PCAD_OK)
    st = plan_hip(hipMemcpyAsync(d_off, p->off.data(), (p->S + 1) * 8, hipMemcpyHostToDevice, s));
  if (st == PCAD_OK)
    st = plan_hip(hipMemcpyAsync(d_item0, p->seg_item0.data(), (p->S + 1) * 4,
                                 hipMemcpyHostToDevice, s));
  if (st != PCAD_OK) return st;
  // merge keys start (and stay, between launches) at the neutral key
  uint64_t *keys = reinterpret_cast<uint64_t *>(p->ws + p->ws_keys);
  hipLaunchKernelGGL(k_fill_u64, dim3(1024), dim3(256), 0, s, keys, p->S * p->m, key_init<MIN>());
  if ((st = plan_hip(hipGetLastError())) != PCAD_OK) return st;
  if ((st = plan_hip(hipStreamSynchronize(s))) != PCAD_OK) return st;

  SegTables t{d_items, d_off, d_item0};
  Ctl *ctl = reinterpret_cast<Ctl *>(p->ws);
  uint64_t *status = reinterpret_cast<uint64_t *>(p->ws + p->ws_status);
  float *carry = reinterpret_cast<float *>(p->saved + p->sv_carry);
  p->fa = SegFwdArgs{t, p->nitems, p->N, (int)p->S, (int)p->m, (int)p->nrows, a, b, idx, y, h, argk, carry,
                     keys, ctl, status};
  p->ba = SegBwdArgs{t, p->nitems, p->N, (int)p->S, (int)p->m, (int)p->nrows, a, b, idx, y, argk,
                     ybar, hbar, abar, bbar, ctl, status};

  // one graph per phase: forward, adjoint, both
  if (!p->cap && (st = plan_hip(hipStreamCreateWithFlags(&p->cap, hipStreamNonBlocking))) != PCAD_OK)
    return st;
  for (int ph = 1; ph <= 3; ++ph) {
    hipGraph_t graph = nullptr;
    if ((st = plan_hip(hipStreamBeginCapture(p->cap, hipStreamCaptureModeThreadLocal))) != PCAD_OK)
      return st;
    hipError_t e = hipSuccess;
    if (ph & 1) e = launch_fwd_nodes(p, p->cap);
    if (e == hipSuccess && (ph & 2)) e = launch_bwd_nodes(p, p->cap);
    const hipError_t e2 = hipStreamEndCapture(p->cap, &graph);
    if (e != hipSuccess) return plan_hip(e);
    if ((st = plan_hip(e2)) != PCAD_OK) return st;
    st = plan_hip(hipGraphInstantiate(&p->g[ph], graph, nullptr, nullptr, 0));
    (void)hipGraphDestroy(graph);
    if (st != PCAD_OK) return st;
  }
  p->bound = true;
  return PCAD_OK;
}

int pcad_plan_run(pcad_plan *p, int phase, void *stream) {
  if (!p) return PCAD_E_NULLPTR;
  if (!p->bound) return PCAD_E_INVALID_ARG;
  if (phase < 1 || phase > 3) return PCAD_E_INVALID_ARG;
  return plan_hip(hipGraphLaunch(p->g[phase], (hipStream_t)stream));
}

int pcad_plan_run_per_segment(pcad_plan *p, int phase, void *stream) {
  if (!p) return PCAD_E_NULLPTR;
  if (!p->bound || !(p->flags & PCAD_PLAN_PER_SEGMENT)) return PCAD_E_INVALID_ARG;
  if (phase < 1 || phase > 3) return PCAD_E_INVALID_ARG;
  hipStream_t s = (hipStream_t)stream;
  void *wsp = p->ws + p->ws_plain;
  float *ytot = reinterpret_cast<float *>(p->ws + align256(p->ws_plain + p->plain_ws_bytes));
  char *svp = p->saved + p->sv_plain;
  size_t so = 0;
  for (int64_t s_ = 0; s_ < p->S; ++s_) {
    const int64_t o = p->off[s_], L = p->off[s_ + 1] - o;
    size_t s1 = 0;
    pcad_query(PCAD_SCAN, PCAD_LINREC, 1, L, 0, 0, &s1, nullptr);
    float *carry = reinterpret_cast<float *>(svp + so);
    so += align256(s1);
    int32_t *ak = p->argk + s_ * p->m;
    float *hh = p->h + s_ * p->m;
    if (phase & 1) {
      hipError_t e = scan_fwd_launch(PCAD_LINREC, 1, L, p->a + o, p->b + o, p->y + o, nullptr,
                                     carry, nullptr, false, wsp, s);
      if (e == hipSuccess)
        e = rbi_fwd_launch(PCAD_MIN, 1, L, p->m, p->idx + o, p->y + o, hh, ak, wsp, s);
      if (e != hipSuccess) return plan_hip(e);
    }
    if (phase & 2) {
      hipError_t e = hipSuccess;
      if (L > 0) e = hipMemcpyAsync(ytot + o, p->ybar + o, L * sizeof(float),
                                    hipMemcpyDeviceToDevice, s);
      if (e == hipSuccess)
        e = rbi_vjp_launch(PCAD_MIN, 1, L, p->m, p->idx + o, p->y + o, ak, p->hbar + s_ * p->m,
                           ytot + o, true, wsp, s);
      if (e == hipSuccess)
        e = scan_vjp_launch(PCAD_LINREC, 1, L, p->a + o, p->b + o, carry, nullptr, nullptr,
                            ytot + o, nullptr,
                            p->abar + o, p->bbar + o, false, wsp, s);
      if (e != hipSuccess) return plan_hip(e);
    }
  }
  return PCAD_OK;
}

void pcad_plan_destroy(pcad_plan *p) {
  if (!p) return;
  for (int i = 0; i < 4; ++i)
    if (p->g[i]) (void)hipGraphExecDestroy(p->g[i]);
  if (p->cap) (void)hipStreamDestroy(p->cap);
  delete p;
}

int pcad_plan_last_hip_error(void) { return g_plan_hip; }

}  // extern "C"
