// Inclusive scan (Section 5) and its adjoint (Section 5.2), single pass.
//
// Forward: every block takes the next tile id from a counter, scans its tile
// in registers (thread-serial over 4 elements, wave64 scan, cross-wave via
// LDS), publishes the tile aggregate, looks back over its predecessors'
// status words for its exclusive prefix, publishes its inclusive prefix and
// writes the outputs.  The exclusive prefix of every tile is also saved, so
// the adjoint can recompute forward prefixes inside a tile without storing y.
//
// Adjoint: tiles are taken in DESCENDING order.  A block loads x and ybar,
// recomputes the forward prefixes of its tile from the saved tile prefix,
// builds the adjoint maps h_i of adjoint.hpp, scans them right to left
// (thread, wave, block), looks back to the RIGHT for the incoming rho, and
// finishes with a thread-serial sweep that writes x_bar.  One kernel, where
// the paper's generated code uses two (Section 5.2, end).
#include "adjoint.hpp"
#include "internal.hpp"

namespace pcad {

// ---------------------------------------------------------------------------
// forward
// ---------------------------------------------------------------------------
struct ScanFwdArgs {
  const float *x0, *x1;
  float *y0, *y1;      // per-element outputs (y1: linrec A, optional)
  float *saved;        // exclusive prefix of every tile (N floats per tile)
  float *total;        // reduce mode: inclusive prefix of each row's last tile
  int64_t n;
  int tpr;             // tiles per row
  Ctl *ctl;
  uint64_t *status;
};

template <int OP, bool REDUCE>
__global__ __launch_bounds__(Shape<OP>::THREADS) void k_scan_fwd(ScanFwdArgs a) {
  using Op = FwdLB<OP>;
  using T = typename Op::T;
  using Io = IO<OP>;
  constexpr int EPL = Shape<OP>::EPL, K = Shape<OP>::K, TILE = Shape<OP>::TILE;
  constexpr int TH = Shape<OP>::THREADS, W = Shape<OP>::W;
  constexpr int NIN = Io::NIN, S = Io::S, N = Fwd<OP>::N;

  __shared__ T s_tot[K][W];
  __shared__ T s_pre[K][W];
  __shared__ T s_carry;
  __shared__ unsigned s_epoch;

  const int tid = threadIdx.x, lane = lane_id(), wave = tid / WAVE;
  if (tid == 0) s_epoch = ctl_load(&a.ctl->epoch);
  const TileInfo ti = tile_info(blockIdx.x, a.n, a.tpr, TILE);

  // load and thread-serial inclusive scan of each group
  T loc[K][EPL];
  T incl[K];
#pragma unroll
  for (int g = 0; g < K; ++g) {
    const int el = g * TH * EPL + tid * EPL;
    const int v = ti.valid - el;
    float4 in[NIN];
    const float *src[2] = {a.x0, a.x1};
#pragma unroll
    for (int s = 0; s < NIN; ++s)
      in[s] = load_group<S>(src[s], ti.base + el, v, ti.vec_ok, Io::fill(s));
    T acc = Io::elem(in, 0);
    loc[g][0] = acc;
#pragma unroll
    for (int j = 1; j < EPL; ++j) {
      acc = Op::comb(acc, Io::elem(in, j));
      loc[g][j] = acc;
    }
    incl[g] = wave_scan_fwd<Op>(acc);
    if (lane == WAVE - 1) s_tot[g][wave] = incl[g];
  }
  __syncthreads();
  const uint32_t tag = s_epoch + 1;

  // wave 0: block prefixes, publish, look back
  if (wave == 0) {
    const T tile_agg = wave0_block_prefix<Op, K, W, false>(s_tot, s_pre, Op::id());
    uint64_t *st = a.status + ti.tile * (Op::NA + Op::NP);
    T c = Op::id();
    if (ti.lt == 0) {
      if (lane == 0) publish<N>(st + Op::NA, tag, tile_agg);
    } else {
      if (lane == 0) publish<N>(st, tag, tile_agg);
      c = lookback<Op>(a.status, ti.tile, +1, ti.lt, tag, a.ctl);
      if (lane == 0) publish<N>(st + Op::NA, tag, Op::comb(c, tile_agg));
    }
    if (lane == 0) {
      s_carry = c;
      if (ti.lt == a.tpr - 1) ctl_row_done(a.ctl, gridDim.x / a.tpr, tag);
      if (a.saved) {
#pragma unroll
        for (int i = 0; i < N; ++i) a.saved[ti.tile * N + i] = c.f[i];
      }
      if (REDUCE && ti.lt == a.tpr - 1) {
        const T tot = Op::comb(c, tile_agg);
#pragma unroll
        for (int i = 0; i < N; ++i) a.total[ti.row * N + i] = tot.f[i];
      }
    }
  }
  if (REDUCE) return;
  __syncthreads();
  const T carry = s_carry;

#pragma unroll
  for (int g = 0; g < K; ++g) {
    T ex = shfl_up(incl[g], 1);
    if (lane == 0) ex = Op::id();
    const T full = Op::comb(Op::comb(carry, s_pre[g][wave]), ex);
    const int el = g * TH * EPL + tid * EPL;
    const int v = ti.valid - el;
    if (OP == MAT2) {
      const T o = Op::comb(full, loc[g][0]);
      store_group<4>(a.y0, ti.base + el, v, true, make_float4(o.f[0], o.f[1], o.f[2], o.f[3]));
    } else {
      float4 o0, o1;
#pragma unroll
      for (int j = 0; j < EPL; ++j) {
        const T o = Op::comb(full, loc[g][j]);
        if (OP == LINREC) {
          f4set(o0, j, o.f[1]);
          f4set(o1, j, o.f[0]);
        } else {
          f4set(o0, j, o.f[0]);
        }
      }
      store_group<1>(a.y0, ti.base + el, v, ti.vec_ok, o0);
      if (OP == LINREC && a.y1) store_group<1>(a.y1, ti.base + el, v, ti.vec_ok, o1);
    }
  }
}

// ---------------------------------------------------------------------------
// adjoint
// ---------------------------------------------------------------------------
struct ScanVjpArgs {
  const float *x0, *x1;
  const float *saved;
  const float *yb0, *yb1;
  float *xb0, *xb1;
  int64_t n;
  int tpr;
  int accumulate;
  Ctl *ctl;
  uint64_t *status;
};

template <int OP, bool ABAR>
__global__ __launch_bounds__(Shape<OP>::THREADS) void k_scan_vjp(ScanVjpArgs a) {
  using Op = FwdLB<OP>;
  using FT = typename Op::T;
  using A = Adj<OP, ABAR>;
  using M = typename A::M;
  using MT = typename M::T;
  using Io = IO<OP>;
  constexpr int EPL = Shape<OP>::EPL, K = Shape<OP>::K, TILE = Shape<OP>::TILE;
  constexpr int TH = Shape<OP>::THREADS, W = Shape<OP>::W;
  constexpr int NIN = Io::NIN, S = Io::S, N = Fwd<OP>::N;

  __shared__ FT s_ftot[K][W];
  __shared__ FT s_fpre[K][W];
  __shared__ MT s_mtot[K][W];
  __shared__ MT s_mpre[K][W];
  __shared__ MT s_carry;
  __shared__ unsigned s_epoch;

  const int tid = threadIdx.x, lane = lane_id(), wave = tid / WAVE;
  if (tid == 0) s_epoch = ctl_load(&a.ctl->epoch);
  // descending tile order: dispatch order runs right to left
  const TileInfo ti = tile_info(gridDim.x - 1 - blockIdx.x, a.n, a.tpr, TILE);

  // loads: x (forward inputs) and ybar
  float4 in[K][NIN];
  float4 yv[K][2];
#pragma unroll
  for (int g = 0; g < K; ++g) {
    const int el = g * TH * EPL + tid * EPL;
    const int v = ti.valid - el;
    const float *src[2] = {a.x0, a.x1};
#pragma unroll
    for (int s = 0; s < NIN; ++s)
      in[g][s] = load_group<S>(src[s], ti.base + el, v, ti.vec_ok, Io::fill(s));
    yv[g][0] = load_group<S>(a.yb0, ti.base + el, v, ti.vec_ok, make_float4(0, 0, 0, 0));
    if (ABAR) yv[g][1] = load_group<1>(a.yb1, ti.base + el, v, ti.vec_ok, make_float4(0, 0, 0, 0));
  }

  // forward prefixes: thread-local inclusive scan and wave scan
  FT loc[K][EPL];
  FT fincl[K];
  if (A::NEEDS_PREFIX) {
#pragma unroll
    for (int g = 0; g < K; ++g) {
      FT acc = Io::elem(in[g], 0);
      loc[g][0] = acc;
#pragma unroll
      for (int j = 1; j < EPL; ++j) {
        acc = Op::comb(acc, Io::elem(in[g], j));
        loc[g][j] = acc;
      }
      fincl[g] = wave_scan_fwd<Op>(acc);
      if (lane == WAVE - 1) s_ftot[g][wave] = fincl[g];
    }
  }
  // the forward prefix rs_{i-1} of slot j of group g, given the thread's
  // exclusive prefix
  auto prefix = [&](int g, int j, const FT &thr) -> FT {
    return j == 0 ? thr : Op::comb(thr, loc[g][j - 1]);
  };

  __syncthreads();
  FT thr_f[K];
  if (A::NEEDS_PREFIX) {
    if (wave == 0) {
      FT carry;
#pragma unroll
      for (int i = 0; i < N; ++i) carry.f[i] = a.saved[ti.tile * N + i];
      wave0_block_prefix<Op, K, W, false>(s_ftot, s_fpre, carry);
    }
    __syncthreads();
#pragma unroll
    for (int g = 0; g < K; ++g) {
      FT ex = shfl_up(fincl[g], 1);
      if (lane == 0) ex = Op::id();
      thr_f[g] = Op::comb(s_fpre[g][wave], ex);
    }
  }

  // adjoint maps: thread aggregate per group = h_0 o h_1 o ... o h_{EPL-1}
  MT mincl[K];
#pragma unroll
  for (int g = 0; g < K; ++g) {
    MT acc = M::id();
#pragma unroll
    for (int j = EPL - 1; j >= 0; --j) {
      float yb[4];
      if (S == 4) {
        yb[0] = yv[g][0].x; yb[1] = yv[g][0].y; yb[2] = yv[g][0].z; yb[3] = yv[g][0].w;
      } else {
        yb[0] = f4get(yv[g][0], j);
        yb[1] = ABAR ? f4get(yv[g][1], j) : 0.0f;
      }
      const bool first = ti.lt == 0 && g == 0 && tid == 0 && j == 0;
      const FT x = Io::elem(in[g], j);
      const FT p = A::NEEDS_PREFIX ? prefix(g, j, thr_f[g]) : Op::id();
      const MT h = A::make(p, x, yb, first);
      acc = (j == EPL - 1) ? h : M::comb(acc, h);
    }
    mincl[g] = wave_scan_rev<M>(acc);
    if (lane == 0) s_mtot[g][wave] = mincl[g];
  }
  __syncthreads();
  const uint32_t tag = s_epoch + 1;

  if (wave == 0) {
    const MT tile_agg = wave0_block_prefix<M, K, W, true>(s_mtot, s_mpre, M::id());
    uint64_t *st = a.status + ti.tile * (M::NA + M::NP);
    const int dist_max = a.tpr - 1 - ti.lt;
    typename M::P zero;
#pragma unroll
    for (int i = 0; i < M::NP; ++i) zero.f[i] = 0.0f;
    MT c = M::from_pre(zero);
    if (dist_max == 0) {
      if (lane == 0) publish<M::NP>(st + M::NA, tag, M::apply0(M::comb(c, tile_agg)));
    } else {
      if (lane == 0) publish<M::NA>(st, tag, tile_agg);
      c = lookback<M>(a.status, ti.tile, -1, dist_max, tag, a.ctl);
      if (lane == 0) publish<M::NP>(st + M::NA, tag, M::apply0(M::comb(c, tile_agg)));
    }
    if (lane == 0) {
      s_carry = c;
      if (ti.lt == 0) ctl_row_done(a.ctl, gridDim.x / a.tpr, tag);
    }
  }
  __syncthreads();
  const MT carry = s_carry;

  // thread-serial sweep, right to left
#pragma unroll
  for (int g = 0; g < K; ++g) {
    MT ex = shfl_down(mincl[g], 1);
    if (lane == WAVE - 1) ex = M::id();
    typename M::P rho = M::apply0(M::comb(M::comb(carry, s_mpre[g][wave]), ex));
    float4 o[2];
    o[0] = make_float4(0, 0, 0, 0);
    o[1] = make_float4(0, 0, 0, 0);
#pragma unroll
    for (int j = EPL - 1; j >= 0; --j) {
      float yb[4];
      if (S == 4) {
        yb[0] = yv[g][0].x; yb[1] = yv[g][0].y; yb[2] = yv[g][0].z; yb[3] = yv[g][0].w;
      } else {
        yb[0] = f4get(yv[g][0], j);
        yb[1] = ABAR ? f4get(yv[g][1], j) : 0.0f;
      }
      const bool first = ti.lt == 0 && g == 0 && tid == 0 && j == 0;
      const FT x = Io::elem(in[g], j);
      const FT p = A::NEEDS_PREFIX ? prefix(g, j, thr_f[g]) : Op::id();
      float xb[4];
      A::step(p, x, yb, first, rho, xb);
      if (S == 4) {
        o[0] = make_float4(xb[0], xb[1], xb[2], xb[3]);
      } else {
        f4set(o[0], j, xb[0]);
        if (A::NXB == 2) f4set(o[1], j, xb[1]);
      }
    }
    const int el = g * TH * EPL + tid * EPL;
    const int v = ti.valid - el;
    float *dst[2] = {a.xb0, a.xb1};
#pragma unroll
    for (int s = 0; s < A::NXB / (S == 4 ? 4 : 1); ++s) {
      float4 val = o[s];
      if (a.accumulate) {
        const float4 old = load_group<S>(dst[s], ti.base + el, v, ti.vec_ok, make_float4(0, 0, 0, 0));
        val.x += old.x; val.y += old.y; val.z += old.z; val.w += old.w;
      }
      store_group<S>(dst[s], ti.base + el, v, ti.vec_ok, val);
    }
  }
}

// ---------------------------------------------------------------------------
// host launchers
// ---------------------------------------------------------------------------
template <int OP>
static int tiles_per_row(int64_t n) {
  constexpr int TILE = Shape<OP>::TILE;
  return (int)((n + TILE - 1) / TILE);
}

int scan_tile_size(int op) {
  switch (op) {
  case ADD: return Shape<ADD>::TILE;
  case MUL: return Shape<MUL>::TILE;
  case MIN: return Shape<MIN>::TILE;
  case MAX: return Shape<MAX>::TILE;
  case LINREC: return Shape<LINREC>::TILE;
  case MAT2: return Shape<MAT2>::TILE;
  }
  return 0;
}

int scan_elem_floats(int op) { return op == LINREC ? 2 : (op == MAT2 ? 4 : 1); }

// status words per tile: forward (N + N); adjoint maps (NA + NP)
int scan_status_words(int op, bool abar) {
  switch (op) {
  case ADD: return 2;
  case MUL: case MIN: case MAX: return 3;
  case LINREC: return abar ? 5 : 4;
  case MAT2: return 12;
  }
  return 0;
}

template <int OP, bool REDUCE>
static hipError_t launch_fwd(const ScanFwdArgs &a, int64_t tiles, hipStream_t s) {
  hipLaunchKernelGGL((k_scan_fwd<OP, REDUCE>), dim3((unsigned)tiles), dim3(Shape<OP>::THREADS), 0, s, a);
  return hipGetLastError();
}

template <int OP, bool ABAR>
static hipError_t launch_vjp(const ScanVjpArgs &a, int64_t tiles, hipStream_t s) {
  hipLaunchKernelGGL((k_scan_vjp<OP, ABAR>), dim3((unsigned)tiles), dim3(Shape<OP>::THREADS), 0, s, a);
  return hipGetLastError();
}

hipError_t scan_fwd_launch(int op, int64_t batch, int64_t n, const float *x0, const float *x1,
                           float *y0, float *y1, float *saved, float *total, bool reduce,
                           void *ws, hipStream_t s) {
  const int tile = scan_tile_size(op);
  const int tpr = (int)((n + tile - 1) / tile);
  const int64_t tiles = batch * (int64_t)tpr;
  if (tiles == 0) return hipSuccess;
  ScanFwdArgs a;
  a.x0 = x0; a.x1 = x1; a.y0 = y0; a.y1 = y1; a.saved = saved; a.total = total;
  a.n = n; a.tpr = tpr;
  a.ctl = reinterpret_cast<Ctl *>(ws);
  a.status = reinterpret_cast<uint64_t *>(static_cast<char *>(ws) + kCtlBytes);
#define PCAD_FWD(OPV)                                                           \
  case OPV:                                                                     \
    return reduce ? launch_fwd<OPV, true>(a, tiles, s) : launch_fwd<OPV, false>(a, tiles, s);
  switch (op) {
    PCAD_FWD(ADD)
    PCAD_FWD(MUL)
    PCAD_FWD(MIN)
    PCAD_FWD(MAX)
    PCAD_FWD(LINREC)
    PCAD_FWD(MAT2)
  }
#undef PCAD_FWD
  return hipErrorInvalidValue;
}

hipError_t scan_vjp_launch(int op, int64_t batch, int64_t n, const float *x0, const float *x1,
                           const float *saved, const float *yb0, const float *yb1, float *xb0,
                           float *xb1, bool accumulate, void *ws, hipStream_t s) {
  const int tile = scan_tile_size(op);
  const int tpr = (int)((n + tile - 1) / tile);
  const int64_t tiles = batch * (int64_t)tpr;
  if (tiles == 0) return hipSuccess;
  ScanVjpArgs a;
  a.x0 = x0; a.x1 = x1; a.saved = saved; a.yb0 = yb0; a.yb1 = yb1; a.xb0 = xb0; a.xb1 = xb1;
  a.n = n; a.tpr = tpr; a.accumulate = accumulate ? 1 : 0;
  a.ctl = reinterpret_cast<Ctl *>(ws);
  a.status = reinterpret_cast<uint64_t *>(static_cast<char *>(ws) + kCtlBytes);
  switch (op) {
  case ADD: return launch_vjp<ADD, false>(a, tiles, s);
  case MUL: return launch_vjp<MUL, false>(a, tiles, s);
  case MIN: return launch_vjp<MIN, false>(a, tiles, s);
  case MAX: return launch_vjp<MAX, false>(a, tiles, s);
  case LINREC:
    return yb1 ? launch_vjp<LINREC, true>(a, tiles, s) : launch_vjp<LINREC, false>(a, tiles, s);
  case MAT2: return launch_vjp<MAT2, false>(a, tiles, s);
  }
  return hipErrorInvalidValue;
}

}  // namespace pcad
