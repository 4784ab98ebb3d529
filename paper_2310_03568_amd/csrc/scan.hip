// Inclusive scan (Section 5) and its adjoint (Section 5.2), single pass.
//
// Both kernels are persistent and software-pipelined.  The grid holds as many
// blocks as can be resident at once; block b owns tiles b, b+G, b+2G, ... of
// the scan order.  One iteration of a block scans its next tile in registers
// (thread-serial over 4 elements, wave64 scan, block prefix by wave 0) and
// publishes its aggregate, issuing the loads of a later tile a group at a
// time as the scan frees their registers; only then does it resolve the
// look-back of its pending tile (whose aggregate, and its predecessors',
// were published an iteration earlier, so one poll normally finds
// everything; the predecessor one round back is the block's own previous
// tile, whose prefix it keeps) and write that tile's outputs.  The memory
// pipe keeps streaming while a look-back waits, and a look-back reaches back
// at most one round of tiles.  (k_scan_vjp, kept for the 2x2 product's
// checkpoint form and the recurrence with the adjoint of its cumulative
// product, resolves its current tile's look-back before scanning the next
// tile, whose loads it issues first.)
//
// Forward: the exclusive prefix of every tile is saved, so the adjoint can
// recompute forward prefixes inside a tile without storing y.
//
// Adjoint: tiles in DESCENDING scan order.  A tile's first phase loads x and
// y_bar, recomputes the forward prefixes from the saved tile prefix, builds
// the adjoint maps h_i of adjoint.hpp and scans them right to left (thread,
// wave, block); after its look-back to the RIGHT, a thread-serial sweep writes
// x_bar.  One kernel, where the paper's generated code uses two (Section 5.2,
// end).
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
  int64_t ntiles;
  Ctl *ctl;
  uint64_t *status;
};

template <int OP, bool REDUCE, int TH_>
__global__ __launch_bounds__(TH_) void k_scan_fwd(ScanFwdArgs a) {
  using Op = FwdLB<OP>;
  using T = typename Op::T;
  using Io = IO<OP>;
  using Sh = ShapeT<OP, TH_>;
  constexpr int EPL = Sh::EPL, K = Sh::K, TILE = Sh::TILE;
  constexpr int TH = Sh::THREADS, W = Sh::W;
  constexpr int NIN = Io::NIN, S = Io::S, N = Fwd<OP>::N;
  constexpr bool LM = lane_major<OP, 0>();

  __shared__ T s_tot[K][W];
  __shared__ T s_pre[K][W];
  __shared__ T s_carry;
  __shared__ unsigned s_epoch;

  const int tid = threadIdx.x, lane = lane_id(), wave = tid / WAVE;
  const float *src[2] = {a.x0, a.x1};
  auto load_grp = [&](const TileInfo &ti, float4 (&buf)[K][NIN], int g) {
    const int el = group_el<LM, K, TH, EPL>(g, tid);
#pragma unroll
    for (int s = 0; s < NIN; ++s)
      buf[g][s] = load_group<S>(src[s], ti.base, el, ti.valid - el, ti.vec_ok, Io::fill(s));
  };
  auto load = [&](int64_t t, float4 (&buf)[K][NIN]) {
    const TileInfo ti = tile_info(t, a.n, a.tpr, TILE);
#pragma unroll
    for (int g = 0; g < K; ++g) load_grp(ti, buf, g);
  };

  if (tid == 0) s_epoch = ctl_load(&a.ctl->epoch);
  const int64_t G = gridDim.x;
  int64_t t = blockIdx.x;  // the tile whose outputs are pending
  float4 cur[K][NIN];
  load(t, cur);
  __syncthreads();
  const uint32_t tag = next_tag(s_epoch);

  // Scans the tile in `cur`: thread-serial inclusive values (lc), the
  // exclusive prefix of each thread's group inside the tile (thr), and, in
  // wave 0, the tile aggregate (ag), which is published (a row's first tile
  // publishes it as its inclusive prefix).  Group-major tiles: after(g) runs
  // once group g of `cur` has been read for the last time (its registers
  // may then receive the next tile's loads); lane-major tiles call it for
  // every group after the serial pass.
  auto phase1 = [&](int64_t tt, T (&thr)[K], T (&lc)[K][EPL], T &ag, auto &&after) {
    const TileInfo ti = tile_info(tt, a.n, a.tpr, TILE);
    if constexpr (LM) {
      // a thread's K groups are consecutive elements: one serial pass, one
      // wave scan, one block prefix
      T acc = Io::elem(cur[0], 0);
#pragma unroll
      for (int g = 0; g < K; ++g) {
#pragma unroll
        for (int j = 0; j < EPL; ++j) {
          if (g > 0 || j > 0) acc = Op::comb(acc, Io::elem(cur[g], j));
          lc[g][j] = acc;
        }
      }
#pragma unroll
      for (int g = 0; g < K; ++g) after(g);
      const T inc = wave_scan_fwd<Op>(acc);
      if (lane == WAVE - 1) s_tot[0][wave] = inc;
      __syncthreads();
      if (wave == 0) {
        ag = wave0_block_prefix<Op, 1, W, false>(s_tot, s_pre, Op::id());
        uint64_t *st = a.status + ti.tile * (Op::NA + Op::NP);
        if (lane == 0) publish<N>(ti.lt == 0 ? st + Op::NA : st, tag, ag);
      }
      __syncthreads();
      T ex = shift_up1(inc);
      if (lane == 0) ex = Op::id();
      const T tp = Op::comb(s_pre[0][wave], ex);
#pragma unroll
      for (int g = 0; g < K; ++g) thr[g] = tp;
      return;
    }
    T incl[K];
#pragma unroll
    for (int g = 0; g < K; ++g) {
      T acc = Io::elem(cur[g], 0);
      lc[g][0] = acc;
#pragma unroll
      for (int j = 1; j < EPL; ++j) {
        acc = Op::comb(acc, Io::elem(cur[g], j));
        lc[g][j] = acc;
      }
      after(g);
      incl[g] = wave_scan_fwd<Op>(acc);
      if (lane == WAVE - 1) s_tot[g][wave] = incl[g];
    }
    __syncthreads();
    if (wave == 0) {
      ag = wave0_block_prefix<Op, K, W, false>(s_tot, s_pre, Op::id());
      uint64_t *st = a.status + ti.tile * (Op::NA + Op::NP);
      if (lane == 0) publish<N>(ti.lt == 0 ? st + Op::NA : st, tag, ag);
    }
    __syncthreads();
#pragma unroll
    for (int g = 0; g < K; ++g) {
      T ex = shift_up1(incl[g]);
      if (lane == 0) ex = Op::id();
      thr[g] = Op::comb(s_pre[g][wave], ex);
    }
  };

  // The look-back of a tile runs one iteration after its aggregate was
  // published: in between, the block scans and publishes its next tile, so
  // the aggregates the look-back needs (the other blocks' tiles of the same
  // round) have long been published when it polls.
  T pthr[K], ploc[K][EPL];
  T pagg = Op::id();       // wave 0: aggregate of the pending tile
  T prev_incl = Op::id();  // wave 0: inclusive prefix of the block's previous tile
  int64_t tn = t + G;
  {
    // the next tile's loads go out a group at a time during the scan
    const bool has = tn < a.ntiles;
    const TileInfo tin = tile_info(has ? tn : t, a.n, a.tpr, TILE);
    phase1(t, pthr, ploc, pagg, [&](int g) {
      if (has) load_grp(tin, cur, g);
    });
  }
  for (;;) {
    const bool more = tn < a.ntiles;
    T nthr[K], nloc[K][EPL];
    T nagg = Op::id();
    if (more) {
      const bool has = tn + G < a.ntiles;
      const TileInfo tin = tile_info(has ? tn + G : tn, a.n, a.tpr, TILE);
      phase1(tn, nthr, nloc, nagg, [&](int g) {
        if (has) load_grp(tin, cur, g);
      });
    }

    const TileInfo ti = tile_info(t, a.n, a.tpr, TILE);
    if (wave == 0) {
      T c = Op::id();
      if (ti.lt > 0) {
        // predecessors at distances 1..G-1 belong to other blocks; the one at
        // distance G is this block's previous tile, whose prefix is known
        const int win = ti.lt < G ? ti.lt : (int)(G - 1);
        bool hit = false;
        if (win > 0) c = lookback<Op>(a.status, ti.tile, +1, win, tag, a.ctl, &hit);
        if (!hit) c = win > 0 ? Op::comb(prev_incl, c) : prev_incl;
        if (lane == 0)
          publish<N>(a.status + ti.tile * (Op::NA + Op::NP) + Op::NA, tag, Op::comb(c, pagg));
      }
      prev_incl = Op::comb(c, pagg);
      if (lane == 0) {
        s_carry = c;
        if (ti.lt == a.tpr - 1) ctl_row_done(a.ctl, (unsigned)(a.ntiles / a.tpr), tag);
        if (a.saved) {
#pragma unroll
          for (int i = 0; i < N; ++i) a.saved[ti.tile * N + i] = c.f[i];
        }
        if (REDUCE && ti.lt == a.tpr - 1) {
#pragma unroll
          for (int i = 0; i < N; ++i) a.total[ti.row * N + i] = prev_incl.f[i];
        }
      }
    }
    __syncthreads();

    if (!REDUCE) {
      const T carry = s_carry;
#pragma unroll
      for (int g = 0; g < K; ++g) {
        const T full = Op::comb(carry, pthr[g]);
        const int el = group_el<LM, K, TH, EPL>(g, tid);
        const int v = ti.valid - el;
        if constexpr (OP == MAT2) {
          const T o = Op::comb(full, ploc[g][0]);
          store_group<4>(a.y0, ti.base, el, v, true, make_float4(o.f[0], o.f[1], o.f[2], o.f[3]));
        } else {
          float4 o0, o1;
#pragma unroll
          for (int j = 0; j < EPL; ++j) {
            const T o = Op::comb(full, ploc[g][j]);
            if (OP == LINREC) {
              f4set(o0, j, o.f[1]);
              f4set(o1, j, o.f[0]);
            } else {
              f4set(o0, j, o.f[0]);
            }
          }
          store_group<1>(a.y0, ti.base, el, v, ti.vec_ok, o0);
          if (OP == LINREC && a.y1) store_group<1>(a.y1, ti.base, el, v, ti.vec_ok, o1);
        }
      }
    }
    if (!more) break;
    // s_carry is rewritten by wave 0 only after the barriers of the next
    // phase1, which every thread reaches after reading it above
    t = tn;
    tn = t + G;
#pragma unroll
    for (int g = 0; g < K; ++g) {
      pthr[g] = nthr[g];
#pragma unroll
      for (int j = 0; j < EPL; ++j) ploc[g][j] = nloc[g][j];
    }
    pagg = nagg;
  }
}

// ---------------------------------------------------------------------------
// adjoint
// ---------------------------------------------------------------------------
struct ScanVjpArgs {
  const float *x0, *x1;
  const float *saved;    // recompute: exclusive prefix of every tile
  const float *tp0, *tp1;  // checkpoint: the forward outputs (y; LINREC also A)
  const float *yb0, *yb1;
  float *xb0, *xb1;
  int64_t n;
  int tpr;
  int64_t ntiles;
  int accumulate;
  Ctl *ctl;
  uint64_t *status;
};

// CKPT: the forward prefix rs_{i-1} is read from the stored forward output
// (the tape) instead of being recomputed inside the tile from the saved tile
// prefix.  A linear recurrence with a tape never reads its offsets b.
template <int OP, bool ABAR, bool CKPT, int TH_>
__global__ __launch_bounds__(TH_) void k_scan_vjp(ScanVjpArgs a) {
  using Op = FwdLB<OP>;
  using FT = typename Op::T;
  using A = Adj<OP, ABAR>;
  using M = typename A::M;
  using MT = typename M::T;
  using Io = IO<OP>;
  using Sh = ShapeT<OP, TH_>;
  constexpr int EPL = Sh::EPL, K = Sh::K, TILE = Sh::TILE;
  constexpr int TH = Sh::THREADS, W = Sh::W;
  constexpr int NIN = Io::NIN, S = Io::S, N = Fwd<OP>::N;
  constexpr bool LM = lane_major<OP, 1>();
  constexpr bool RECOMP = A::NEEDS_PREFIX && !CKPT;
  constexpr bool TAPE = A::NEEDS_PREFIX && CKPT;
  // streams per group: x...; y_bar; [A_bar]; [tape y; [tape A]]
  constexpr int NX = (TAPE && OP == LINREC) ? 1 : NIN;
  constexpr int IYB = NX, IAB = NX + 1, IT = NX + 1 + (ABAR ? 1 : 0);
  constexpr int NT = TAPE ? ((OP == LINREC && ABAR) ? 2 : 1) : 0;
  constexpr int NB = IT + NT;
  constexpr int NTP = NT > 0 ? NT : 1;

  __shared__ FT s_ftot[RECOMP ? K : 1][W];
  __shared__ FT s_fpre[RECOMP ? K : 1][W];
  __shared__ MT s_mtot[K][W];
  __shared__ MT s_mpre[K][W];
  __shared__ MT s_carry;
  __shared__ unsigned s_epoch;

  const int tid = threadIdx.x, lane = lane_id(), wave = tid / WAVE;
  const float *src[2] = {a.x0, a.x1};
  const float *tp[2] = {a.tp0, a.tp1};
  // tape value before a row's first element: the neutral prefix component
  auto tape_id = [&](int s) -> float4 {
    const FT e = Op::id();
    if (OP == MAT2) return make_float4(e.f[0], e.f[1], e.f[2], e.f[3]);
    const float v = (OP == LINREC) ? (s == 0 ? e.f[1] : e.f[0]) : e.f[0];
    return make_float4(v, v, v, v);
  };
  // pv: for lane 0 only, the tape element just before the group (the other
  // lanes take it from their left neighbour)
  auto load = [&](int64_t t, float4 (&buf)[K][NB], float4 (&pv)[K][NTP]) {
    const TileInfo ti = tile_info(t, a.n, a.tpr, TILE);
#pragma unroll
    for (int g = 0; g < K; ++g) {
      const int el = group_el<LM, K, TH, EPL>(g, tid);
      const int v = ti.valid - el;
#pragma unroll
      for (int s = 0; s < NX; ++s)
        buf[g][s] = load_group<S, !LM>(src[s], ti.base, el, v, ti.vec_ok, Io::fill(s));
      buf[g][IYB] = load_group<S, !LM>(a.yb0, ti.base, el, v, ti.vec_ok, make_float4(0, 0, 0, 0));
      if (ABAR)
        buf[g][IAB] = load_group<1>(a.yb1, ti.base, el, v, ti.vec_ok, make_float4(0, 0, 0, 0));
#pragma unroll
      for (int s = 0; s < NT; ++s) {
        buf[g][IT + s] = load_group<S, !LM>(tp[s], ti.base, el, v, ti.vec_ok, tape_id(s));
        float4 q = tape_id(s);
        if (lane == 0 && v > 0 && !(ti.lt == 0 && el == 0)) {
          const int64_t e = ti.base + el - 1;
          if (S == 4) q = *reinterpret_cast<const float4 *>(tp[s] + e * 4);
          else q.x = tp[s][e];
        }
        pv[g][s] = q;
      }
    }
  };
  auto ybar_of = [&](const float4 (&buf)[K][NB], int g, int j, float *yb) {
    if (S == 4) {
      yb[0] = buf[g][IYB].x; yb[1] = buf[g][IYB].y; yb[2] = buf[g][IYB].z; yb[3] = buf[g][IYB].w;
    } else {
      yb[0] = f4get(buf[g][IYB], j);
      yb[1] = ABAR ? f4get(buf[g][IAB], j) : 0.0f;
    }
  };
  auto x_of = [&](const float4 (&buf)[K][NB], int g, int j) -> FT {
    float4 in[NIN];
#pragma unroll
    for (int s = 0; s < NIN; ++s) in[s] = s < NX ? buf[g][s] : Io::fill(s);
    return Io::elem(in, j);
  };

  if (tid == 0) s_epoch = ctl_load(&a.ctl->epoch);
  int64_t k = blockIdx.x;
  auto tile_of = [&](int64_t kk) { return a.ntiles - 1 - kk; };  // right to left
  float4 cur[K][NB];
  float4 cpv[K][NTP];
  load(tile_of(k), cur, cpv);
  __syncthreads();
  const uint32_t tag = next_tag(s_epoch);

  FT thr_f[K];   // recompute: forward prefix before each thread's group
  MT mincl[K];   // wave-inclusive (from the right) adjoint-map aggregates
  MT agg = M::id();
  // the forward prefixes rs_{i-1} of the EPL slots of group g, ascending
  auto prefixes = [&](int g, FT (&p)[EPL]) {
    if (TAPE) {
      if (S == 4 && LM) {
        // the element before group g: the same thread's group g-1, or for
        // g = 0 the left neighbour's last group (lane 0: loaded with pv)
        Vec<4> up;
        if (g > 0) {
          up = Vec<4>{{cur[g - 1][IT].x, cur[g - 1][IT].y, cur[g - 1][IT].z, cur[g - 1][IT].w}};
        } else {
          Vec<4> q = {{cur[K - 1][IT].x, cur[K - 1][IT].y, cur[K - 1][IT].z, cur[K - 1][IT].w}};
          up = shift_up1(q);
          if (lane == 0) up = Vec<4>{{cpv[0][0].x, cpv[0][0].y, cpv[0][0].z, cpv[0][0].w}};
        }
#pragma unroll
        for (int i = 0; i < N; ++i) p[0].f[i] = up.f[i];
      } else if (S == 4) {
        Vec<4> q = {{cur[g][IT].x, cur[g][IT].y, cur[g][IT].z, cur[g][IT].w}};
        Vec<4> up = shift_up1(q);
        if (lane == 0) up = Vec<4>{{cpv[g][0].x, cpv[g][0].y, cpv[g][0].z, cpv[g][0].w}};
#pragma unroll
        for (int i = 0; i < N; ++i) p[0].f[i] = up.f[i];
      } else {
        float prev[2][4];
#pragma unroll
        for (int s = 0; s < NT; ++s) {
          const float4 q = cur[g][IT + s];
          float w = dpp_f<kDppWaveShr1>(q.w);
          if (lane == 0) w = cpv[g][s].x;
          prev[s][0] = w; prev[s][1] = q.x; prev[s][2] = q.y; prev[s][3] = q.z;
        }
#pragma unroll
        for (int j = 0; j < EPL; ++j) {
          if (OP == LINREC) {
            p[j].f[0] = NT == 2 ? prev[NT - 1][j] : 1.0f;  // A_{i-1}: read only with A_bar
            p[j].f[1] = prev[0][j];
          } else {
            p[j].f[0] = prev[0][j];
          }
        }
      }
    } else {
      FT acc = thr_f[g];
#pragma unroll
      for (int j = 0; j < EPL; ++j) {
        p[j] = acc;
        if (RECOMP && j + 1 < EPL) acc = Op::comb(acc, x_of(cur, g, j));
      }
    }
  };

  auto phase1 = [&](int64_t kk) {
    const TileInfo ti = tile_info(tile_of(kk), a.n, a.tpr, TILE);
    if constexpr (LM) {
      // a thread's K groups are consecutive elements: one serial pass and
      // one wave scan each way
      if (RECOMP) {
        FT gagg[K];
#pragma unroll
        for (int g = 0; g < K; ++g) {
          FT e = x_of(cur, g, 0);
#pragma unroll
          for (int j = 1; j < EPL; ++j) e = Op::comb(e, x_of(cur, g, j));
          gagg[g] = e;
        }
        FT acc = gagg[0];
#pragma unroll
        for (int g = 1; g < K; ++g) acc = Op::comb(acc, gagg[g]);
        const FT fin = wave_scan_fwd<Op>(acc);
        if (lane == WAVE - 1) s_ftot[0][wave] = fin;
        __syncthreads();
        if (wave == 0) {
          FT c;
#pragma unroll
          for (int i = 0; i < N; ++i) c.f[i] = a.saved[ti.tile * N + i];
          wave0_block_prefix<Op, 1, W, false>(s_ftot, s_fpre, c);
        }
        __syncthreads();
        FT ex = shift_up1(fin);
        if (lane == 0) ex = Op::id();
        thr_f[0] = Op::comb(s_fpre[0][wave], ex);
#pragma unroll
        for (int g = 1; g < K; ++g) thr_f[g] = Op::comb(thr_f[g - 1], gagg[g - 1]);
      } else {
#pragma unroll
        for (int g = 0; g < K; ++g) thr_f[g] = Op::id();
      }
      MT acc = M::id();
#pragma unroll
      for (int g = K - 1; g >= 0; --g) {
        FT p[EPL];
        prefixes(g, p);
#pragma unroll
        for (int j = EPL - 1; j >= 0; --j) {
          float yb[4];
          ybar_of(cur, g, j, yb);
          const bool first = ti.lt == 0 && g == 0 && tid == 0 && j == 0;
          const MT h = A::make(p[j], x_of(cur, g, j), yb, first);
          acc = (g == K - 1 && j == EPL - 1) ? h : M::comb(acc, h);
        }
      }
      mincl[0] = wave_scan_rev<M>(acc);
      if (lane == 0) s_mtot[0][wave] = mincl[0];
      __syncthreads();
      if (wave == 0) {
        agg = wave0_block_prefix<M, 1, W, true>(s_mtot, s_mpre, M::id());
        uint64_t *st = a.status + ti.tile * (M::NA + M::NP);
        if (lane == 0) {
          if (ti.lt == a.tpr - 1) {
            typename M::P zero;
#pragma unroll
            for (int i = 0; i < M::NP; ++i) zero.f[i] = 0.0f;
            publish<M::NP>(st + M::NA, tag, M::apply0(M::comb(M::from_pre(zero), agg)));
          } else {
            publish<M::NA>(st, tag, agg);
          }
        }
      }
      return;
    }
    if (RECOMP) {
      FT fincl[K];
#pragma unroll
      for (int g = 0; g < K; ++g) {
        FT acc = x_of(cur, g, 0);
#pragma unroll
        for (int j = 1; j < EPL; ++j) acc = Op::comb(acc, x_of(cur, g, j));
        fincl[g] = wave_scan_fwd<Op>(acc);
        if (lane == WAVE - 1) s_ftot[g][wave] = fincl[g];
      }
      __syncthreads();
      if (wave == 0) {
        FT c;
#pragma unroll
        for (int i = 0; i < N; ++i) c.f[i] = a.saved[ti.tile * N + i];
        wave0_block_prefix<Op, K, W, false>(s_ftot, s_fpre, c);
      }
      __syncthreads();
#pragma unroll
      for (int g = 0; g < K; ++g) {
        FT ex = shift_up1(fincl[g]);
        if (lane == 0) ex = Op::id();
        thr_f[g] = Op::comb(s_fpre[g][wave], ex);
      }
    } else {
#pragma unroll
      for (int g = 0; g < K; ++g) thr_f[g] = Op::id();
    }
    // adjoint maps: thread aggregate per group = h_0 o h_1 o ... o h_{EPL-1}
#pragma unroll
    for (int g = 0; g < K; ++g) {
      FT p[EPL];
      prefixes(g, p);
      MT acc = M::id();
#pragma unroll
      for (int j = EPL - 1; j >= 0; --j) {
        float yb[4];
        ybar_of(cur, g, j, yb);
        const bool first = ti.lt == 0 && g == 0 && tid == 0 && j == 0;
        const MT h = A::make(p[j], x_of(cur, g, j), yb, first);
        acc = (j == EPL - 1) ? h : M::comb(acc, h);
      }
      mincl[g] = wave_scan_rev<M>(acc);
      if (lane == 0) s_mtot[g][wave] = mincl[g];
    }
    __syncthreads();
    if (wave == 0) {
      agg = wave0_block_prefix<M, K, W, true>(s_mtot, s_mpre, M::id());
      uint64_t *st = a.status + ti.tile * (M::NA + M::NP);
      if (lane == 0) {
        if (ti.lt == a.tpr - 1) {
          typename M::P zero;
#pragma unroll
          for (int i = 0; i < M::NP; ++i) zero.f[i] = 0.0f;
          publish<M::NP>(st + M::NA, tag, M::apply0(M::comb(M::from_pre(zero), agg)));
        } else {
          publish<M::NA>(st, tag, agg);
        }
      }
    }
  };

  phase1(k);
  for (;;) {
    const TileInfo ti = tile_info(tile_of(k), a.n, a.tpr, TILE);
    const int64_t kn = k + gridDim.x;
    const bool more = kn < a.ntiles;
    float4 nxt[K][NB];
    float4 npv[K][NTP];
    if (more) load(tile_of(kn), nxt, npv);

    if (wave == 0) {
      typename M::P zero;
#pragma unroll
      for (int i = 0; i < M::NP; ++i) zero.f[i] = 0.0f;
      MT c = M::from_pre(zero);
      const int dist_max = a.tpr - 1 - ti.lt;
      if (dist_max > 0) {
        c = lookback<M>(a.status, ti.tile, -1, dist_max, tag, a.ctl);
        if (lane == 0)
          publish<M::NP>(a.status + ti.tile * (M::NA + M::NP) + M::NA, tag,
                         M::apply0(M::comb(c, agg)));
      }
      if (lane == 0) {
        s_carry = c;
        if (ti.lt == 0) ctl_row_done(a.ctl, (unsigned)(a.ntiles / a.tpr), tag);
      }
    }
    __syncthreads();
    const MT carry = s_carry;

    // thread-serial sweep, right to left
    typename M::P rho_lm;
    float4 o_lm[LM ? K : 1];  // lane-major: a thread's groups are adjacent in
                              // memory; they are stored together after the sweep
    if constexpr (LM) {
      MT ex = shift_down1(mincl[0]);
      if (lane == WAVE - 1) ex = M::id();
      rho_lm = M::apply0(M::comb(M::comb(carry, s_mpre[0][wave]), ex));
    }
#pragma unroll
    for (int gi = 0; gi < K; ++gi) {
      // lane-major threads sweep their groups from the last one
      const int g = LM ? K - 1 - gi : gi;
      typename M::P rho;
      if constexpr (LM) {
        rho = rho_lm;
      } else {
        MT ex = shift_down1(mincl[g]);
        if (lane == WAVE - 1) ex = M::id();
        rho = M::apply0(M::comb(M::comb(carry, s_mpre[g][wave]), ex));
      }
      FT p[EPL];
      prefixes(g, p);
      float4 o[2];
      o[0] = make_float4(0, 0, 0, 0);
      o[1] = make_float4(0, 0, 0, 0);
#pragma unroll
      for (int j = EPL - 1; j >= 0; --j) {
        float yb[4];
        ybar_of(cur, g, j, yb);
        const bool first = ti.lt == 0 && g == 0 && tid == 0 && j == 0;
        float xb[4];
        A::step(p[j], x_of(cur, g, j), yb, first, rho, xb);
        if (S == 4) {
          o[0] = make_float4(xb[0], xb[1], xb[2], xb[3]);
        } else {
          f4set(o[0], j, xb[0]);
          if (A::NXB == 2) f4set(o[1], j, xb[1]);
        }
      }
      if constexpr (LM) {
        rho_lm = rho;
        o_lm[g] = o[0];
        continue;
      }
      const int el = group_el<LM, K, TH, EPL>(g, tid);
      const int v = ti.valid - el;
      float *dst[2] = {a.xb0, a.xb1};
#pragma unroll
      for (int s = 0; s < A::NXB / (S == 4 ? 4 : 1); ++s) {
        float4 val = o[s];
        if (a.accumulate) {
          const float4 old = load_group<S>(dst[s], ti.base, el, v, ti.vec_ok, make_float4(0, 0, 0, 0));
          val.x += old.x; val.y += old.y; val.z += old.z; val.w += old.w;
        }
        store_group<S>(dst[s], ti.base, el, v, ti.vec_ok, val);
      }
    }
    if constexpr (LM) {
      // back-to-back ordinary (not streaming) stores of the thread's
      // consecutive groups, so that L2 merges them into whole lines; the
      // streaming stores of one group per sweep step left half-written lines
      // (twice the output bytes in the write counter)
      static_assert(S == 4 && A::NXB == 4, "lane-major tiles hold 2x2 matrices");
#pragma unroll
      for (int g = 0; g < K; ++g) {
        const int el = group_el<LM, K, TH, EPL>(g, tid);
        if (el >= ti.valid) break;
        float4 *q = reinterpret_cast<float4 *>(a.xb0 + (ti.base + el) * 4);
        float4 val = o_lm[g];
        if (a.accumulate) {
          const float4 old = *q;
          val.x += old.x; val.y += old.y; val.z += old.z; val.w += old.w;
        }
        *q = val;
      }
    }
    if (!more) break;
    k = kn;
#pragma unroll
    for (int g = 0; g < K; ++g) {
#pragma unroll
      for (int s = 0; s < NB; ++s) cur[g][s] = nxt[g][s];
#pragma unroll
      for (int s = 0; s < NTP; ++s) cpv[g][s] = npv[g][s];
    }
    __syncthreads();  // LDS of the finished tile is rewritten below
    phase1(k);
  }
}

// The scan adjoint for group-major tiles (every operator but the 2x2
// product) with a delayed look-back, as in the forward: a tile's look-back
// runs one iteration after its map aggregate was published, once the block
// has scanned its next tile, so the aggregates it needs (the other blocks'
// tiles of the same round) have long been published when it polls, and the
// predecessor at distance G is this block's previous tile, whose inclusive
// prefix the block keeps: no persistent round waits on the publish-to-poll
// latency of the round before.  Three register buffers rotate (the loop is
// unrolled by three so that no register of a load in flight is copied): the
// tile being swept, the tile being scanned, and the tile whose loads go out
// a group at a time during that scan.  What a scanned tile leaves for its
// sweep (per thread: the forward prefixes and the wave-inclusive map
// aggregates; per wave: the block prefixes) waits in LDS, in two slots used
// by alternate tiles.  The per-tile arithmetic is that of k_scan_vjp.
template <int OP, bool ABAR, bool CKPT, int TH_>
__global__ __launch_bounds__(TH_) void k_scan_vjp_d(ScanVjpArgs a) {
  using Op = FwdLB<OP>;
  using FT = typename Op::T;
  using A = Adj<OP, ABAR>;
  using M = typename A::M;
  using MT = typename M::T;
  using Io = IO<OP>;
  using Sh = ShapeT<OP, TH_>;
  constexpr int EPL = Sh::EPL, K = Sh::K, TILE = Sh::TILE;
  constexpr int TH = Sh::THREADS, W = Sh::W;
  constexpr int NIN = Io::NIN, S = Io::S, N = Fwd<OP>::N, NA = M::NA;
  static_assert(!lane_major<OP, 1>() && IO<OP>::S == 1, "group-major tiles of scalar elements");
  constexpr bool LM = false;
  constexpr bool RECOMP = A::NEEDS_PREFIX && !CKPT;
  constexpr bool TAPE = A::NEEDS_PREFIX && CKPT;
  // streams per group: x...; y_bar; [A_bar]; [tape y; [tape A]]
  constexpr int NX = (TAPE && OP == LINREC) ? 1 : NIN;
  constexpr int IYB = NX, IAB = NX + 1, IT = NX + 1 + (ABAR ? 1 : 0);
  constexpr int NT = TAPE ? ((OP == LINREC && ABAR) ? 2 : 1) : 0;
  constexpr int NB = IT + NT;
  constexpr int NTP = NT > 0 ? NT : 1;
  using Buf = float4[K][NB];
  using PBuf = float4[K][NTP];

  __shared__ FT s_ftot[RECOMP ? K : 1][W];
  __shared__ FT s_fpre[RECOMP ? K : 1][W];
  __shared__ MT s_mtot[K][W];
  __shared__ MT s_mpre[2][K][W];
  // per-thread state of a scanned tile, component-major so that a wave's
  // accesses are consecutive words
  __shared__ float s_thr[2][RECOMP ? K * N : 1][TH];
  __shared__ float s_minc[2][K * NA][TH];
  __shared__ MT s_carry;
  __shared__ unsigned s_epoch;

  const int tid = threadIdx.x, lane = lane_id(), wave = tid / WAVE;
  const int64_t G = gridDim.x;
  const float *src[2] = {a.x0, a.x1};
  const float *tp[2] = {a.tp0, a.tp1};
  // tape value before a row's first element: the neutral prefix component
  auto tape_id = [&](int s) -> float4 {
    const FT e = Op::id();
    const float v = (OP == LINREC) ? (s == 0 ? e.f[1] : e.f[0]) : e.f[0];
    return make_float4(v, v, v, v);
  };
  // group g of tile ti; pv: for lane 0 only, the tape element just before
  // the group (the other lanes take it from their left neighbour)
  auto load_grp = [&](const TileInfo &ti, Buf &buf, PBuf &pv, int g) {
    const int el = group_el<LM, K, TH, EPL>(g, tid);
    const int v = ti.valid - el;
#pragma unroll
    for (int s = 0; s < NX; ++s)
      buf[g][s] = load_group<S>(src[s], ti.base, el, v, ti.vec_ok, Io::fill(s));
    buf[g][IYB] = load_group<S>(a.yb0, ti.base, el, v, ti.vec_ok, make_float4(0, 0, 0, 0));
    if (ABAR)
      buf[g][IAB] = load_group<1>(a.yb1, ti.base, el, v, ti.vec_ok, make_float4(0, 0, 0, 0));
#pragma unroll
    for (int s = 0; s < NT; ++s) {
      buf[g][IT + s] = load_group<S>(tp[s], ti.base, el, v, ti.vec_ok, tape_id(s));
      float4 q = tape_id(s);
      if (lane == 0 && v > 0 && !(ti.lt == 0 && el == 0)) q.x = tp[s][ti.base + el - 1];
      pv[g][s] = q;
    }
  };
  auto ybar_of = [&](const Buf &buf, int g, int j, float *yb) {
    yb[0] = f4get(buf[g][IYB], j);
    yb[1] = ABAR ? f4get(buf[g][IAB], j) : 0.0f;
  };
  auto x_of = [&](const Buf &buf, int g, int j) -> FT {
    float4 in[NIN];
#pragma unroll
    for (int s = 0; s < NIN; ++s) in[s] = s < NX ? buf[g][s] : Io::fill(s);
    return Io::elem(in, j);
  };
  // the forward prefixes rs_{i-1} of the EPL slots of group g, ascending;
  // thr: the forward prefix before the thread's group (recompute)
  auto prefixes = [&](const Buf &cur, const PBuf &cpv, const FT &thr, int g, FT (&p)[EPL]) {
    if (TAPE) {
      float prev[2][4];
#pragma unroll
      for (int s = 0; s < NT; ++s) {
        const float4 q = cur[g][IT + s];
        float w = dpp_f<kDppWaveShr1>(q.w);
        if (lane == 0) w = cpv[g][s].x;
        prev[s][0] = w; prev[s][1] = q.x; prev[s][2] = q.y; prev[s][3] = q.z;
      }
#pragma unroll
      for (int j = 0; j < EPL; ++j) {
        if (OP == LINREC) {
          p[j].f[0] = NT == 2 ? prev[NT - 1][j] : 1.0f;  // A_{i-1}: read only with A_bar
          p[j].f[1] = prev[0][j];
        } else {
          p[j].f[0] = prev[0][j];
        }
      }
    } else {
      FT acc = thr;
#pragma unroll
      for (int j = 0; j < EPL; ++j) {
        p[j] = acc;
        if (RECOMP && j + 1 < EPL) acc = Op::comb(acc, x_of(cur, g, j));
      }
    }
  };

  if (tid == 0) s_epoch = ctl_load(&a.ctl->epoch);
  int64_t k = blockIdx.x;
  uint32_t tag = 0;  // this launch's tag, set once the epoch has been read
  auto tile_of = [&](int64_t kk) { return a.ntiles - 1 - kk; };  // right to left

  // Scans tile kk (data in cur) up to the wave level: forward prefixes
  // (recompute) and the adjoint maps' wave scans, kept in LDS slot sl, and
  // the wave totals in s_mtot.  after(g) runs once group g's data has been
  // read for the last time before the sweep.  The block level follows in
  // `resolve`.
  auto phase1 = [&](int64_t kk, const Buf &cur, const PBuf &cpv, int sl, auto &&after) {
    const TileInfo ti = tile_info(tile_of(kk), a.n, a.tpr, TILE);
    FT thr[K];
    if (RECOMP) {
      FT fincl[K];
#pragma unroll
      for (int g = 0; g < K; ++g) {
        FT acc = x_of(cur, g, 0);
#pragma unroll
        for (int j = 1; j < EPL; ++j) acc = Op::comb(acc, x_of(cur, g, j));
        fincl[g] = wave_scan_fwd<Op>(acc);
        if (lane == WAVE - 1) s_ftot[g][wave] = fincl[g];
      }
      __syncthreads();
      if (wave == 0) {
        FT c;
#pragma unroll
        for (int i = 0; i < N; ++i) c.f[i] = a.saved[ti.tile * N + i];
        wave0_block_prefix<Op, K, W, false>(s_ftot, s_fpre, c);
      }
      __syncthreads();
#pragma unroll
      for (int g = 0; g < K; ++g) {
        FT ex = shift_up1(fincl[g]);
        if (lane == 0) ex = Op::id();
        thr[g] = Op::comb(s_fpre[g][wave], ex);
#pragma unroll
        for (int i = 0; i < N; ++i) s_thr[sl][g * N + i][tid] = thr[g].f[i];
      }
    } else {
#pragma unroll
      for (int g = 0; g < K; ++g) thr[g] = Op::id();
    }
    // adjoint maps: thread aggregate per group = h_0 o h_1 o ... o h_{EPL-1}
#pragma unroll
    for (int g = 0; g < K; ++g) {
      FT p[EPL];
      prefixes(cur, cpv, thr[g], g, p);
      MT acc = M::id();
#pragma unroll
      for (int j = EPL - 1; j >= 0; --j) {
        float yb[4];
        ybar_of(cur, g, j, yb);
        const bool first = ti.lt == 0 && g == 0 && tid == 0 && j == 0;
        const MT h = A::make(p[j], x_of(cur, g, j), yb, first);
        acc = (j == EPL - 1) ? h : M::comb(acc, h);
      }
      after(g);
      const MT mi = wave_scan_rev<M>(acc);
#pragma unroll
      for (int i = 0; i < NA; ++i) s_minc[sl][g * NA + i][tid] = mi.f[i];
      if (lane == 0) s_mtot[g][wave] = mi;
    }
  };

  // wave 0: the block prefix of scanned tile kk into slot sl, and the
  // publication of its aggregate (a row's last tile: its inclusive prefix)
  auto block_level = [&](int64_t kk, int sl) -> MT {
    const TileInfo ti = tile_info(tile_of(kk), a.n, a.tpr, TILE);
    const MT agg = wave0_block_prefix<M, K, W, true>(s_mtot, s_mpre[sl], M::id());
    uint64_t *st = a.status + ti.tile * (M::NA + M::NP);
    if (lane == 0) {
      if (ti.lt == a.tpr - 1) {
        typename M::P zero;
#pragma unroll
        for (int i = 0; i < M::NP; ++i) zero.f[i] = 0.0f;
        publish<M::NP>(st + M::NA, tag, M::apply0(M::comb(M::from_pre(zero), agg)));
      } else {
        publish<M::NA>(st, tag, agg);
      }
    }
    return agg;
  };

  MT prev_incl = M::id();  // wave 0: inclusive prefix of the block's previous tile
  // Wave 0: the block level of the scanned tile kp (if `scanned`), then the
  // look-back of the pending tile ks, whose inclusive prefix is published.
  auto resolve = [&](int64_t ks, const MT &agg_s, bool scanned, int64_t kp, MT &agg_p, int slp) {
    __syncthreads();
    if (wave == 0) {
      if (scanned) agg_p = block_level(kp, slp);
      const TileInfo ti = tile_info(tile_of(ks), a.n, a.tpr, TILE);
      typename M::P zero;
#pragma unroll
      for (int i = 0; i < M::NP; ++i) zero.f[i] = 0.0f;
      MT c = M::from_pre(zero);
      const int dist_max = a.tpr - 1 - ti.lt;
      if (dist_max > 0) {
        // successors at distances 1..G-1 belong to other blocks; the one at
        // distance G is this block's previous tile, in the same row
        const int win = dist_max < G ? dist_max : (int)(G - 1);
        bool hit = false;
        if (win > 0) c = lookback<M>(a.status, ti.tile, -1, win, tag, a.ctl, &hit);
        if (!hit) c = win > 0 ? M::comb(prev_incl, c) : prev_incl;
        if (lane == 0)
          publish<M::NP>(a.status + ti.tile * (M::NA + M::NP) + M::NA, tag,
                         M::apply0(M::comb(c, agg_s)));
      }
      prev_incl = M::from_pre(M::apply0(M::comb(c, agg_s)));
      if (lane == 0) {
        s_carry = c;
        if (ti.lt == 0) ctl_row_done(a.ctl, (unsigned)(a.ntiles / a.tpr), tag);
      }
    }
    __syncthreads();
  };

  // thread-serial sweep of tile ks (state in slot sl), right to left
  auto sweep = [&](int64_t ks, const Buf &cur, const PBuf &cpv, int sl) {
    const TileInfo ti = tile_info(tile_of(ks), a.n, a.tpr, TILE);
    const MT carry = s_carry;
#pragma unroll
    for (int g = 0; g < K; ++g) {
      MT mi;
#pragma unroll
      for (int i = 0; i < NA; ++i) mi.f[i] = s_minc[sl][g * NA + i][tid];
      FT thr = Op::id();
      if (RECOMP) {
#pragma unroll
        for (int i = 0; i < N; ++i) thr.f[i] = s_thr[sl][g * N + i][tid];
      }
      MT ex = shift_down1(mi);
      if (lane == WAVE - 1) ex = M::id();
      typename M::P rho = M::apply0(M::comb(M::comb(carry, s_mpre[sl][g][wave]), ex));
      FT p[EPL];
      prefixes(cur, cpv, thr, g, p);
      float4 o[2];
      o[0] = make_float4(0, 0, 0, 0);
      o[1] = make_float4(0, 0, 0, 0);
#pragma unroll
      for (int j = EPL - 1; j >= 0; --j) {
        float yb[4];
        ybar_of(cur, g, j, yb);
        const bool first = ti.lt == 0 && g == 0 && tid == 0 && j == 0;
        float xb[4];
        A::step(p[j], x_of(cur, g, j), yb, first, rho, xb);
        f4set(o[0], j, xb[0]);
        if (A::NXB == 2) f4set(o[1], j, xb[1]);
      }
      const int el = group_el<LM, K, TH, EPL>(g, tid);
      const int v = ti.valid - el;
      float *dst[2] = {a.xb0, a.xb1};
#pragma unroll
      for (int s = 0; s < A::NXB; ++s) {
        float4 val = o[s];
        if (a.accumulate) {
          const float4 old = load_group<S>(dst[s], ti.base, el, v, ti.vec_ok, make_float4(0, 0, 0, 0));
          val.x += old.x; val.y += old.y; val.z += old.z; val.w += old.w;
        }
        store_group<S>(dst[s], ti.base, el, v, ti.vec_ok, val);
      }
    }
  };

  Buf b0, b1, b2;
  PBuf p0, p1, p2;
  MT g0 = M::id(), g1 = M::id(), g2 = M::id();  // wave 0: map aggregates
  int sl = 0;  // LDS slot of the tile being swept
  {
    const TileInfo ti = tile_info(tile_of(k), a.n, a.tpr, TILE);
#pragma unroll
    for (int g = 0; g < K; ++g) load_grp(ti, b0, p0, g);
  }
  __syncthreads();
  tag = next_tag(s_epoch);
  {
    const bool has1 = k + G < a.ntiles;
    const TileInfo t1 = tile_info(tile_of(has1 ? k + G : k), a.n, a.tpr, TILE);
    phase1(k, b0, p0, 0, [&](int g) {
      if (has1) load_grp(t1, b1, p1, g);
    });
    // the first tile's block level; nothing is pending yet.  The barrier
    // after it keeps the next scan's wave totals out of s_mtot until wave 0
    // has read this tile's (a scan without a forward re-scan has no barrier
    // before it writes them).
    __syncthreads();
    if (wave == 0) g0 = block_level(k, 0);
    __syncthreads();
  }

  // S: tile k, scanned (state in slot sl); P: tile k+G, loaded (or
  // loading); L: free
  auto step = [&](Buf &bs, PBuf &ps, MT &gs, Buf &bp, PBuf &pp, MT &gp, Buf &bl,
                  PBuf &pl) -> bool {
    const bool scan = k + G < a.ntiles;
    if (scan) {
      const bool has2 = k + 2 * G < a.ntiles;
      const TileInfo t2 = tile_info(tile_of(has2 ? k + 2 * G : k), a.n, a.tpr, TILE);
      phase1(k + G, bp, pp, sl ^ 1, [&](int g) {
        if (has2) load_grp(t2, bl, pl, g);
      });
    }
    resolve(k, gs, scan, k + G, gp, sl ^ 1);
    sweep(k, bs, ps, sl);
    if (!scan) return false;
    k += G;
    sl ^= 1;
    return true;
  };
  for (;;) {
    if (!step(b0, p0, g0, b1, p1, g1, b2, p2)) break;
    if (!step(b1, p1, g1, b2, p2, g2, b0, p0)) break;
    if (!step(b2, p2, g2, b0, p0, g0, b1, p1)) break;
  }
}

// The 2x2-product scan adjoint (recompute form) with the delayed look-back
// of k_scan_vjp_d, on lane-major tiles: a thread's K groups are consecutive
// elements (one serial pass and one wave scan each way per thread), three
// register buffers rotate, and a scanned tile's state (per thread: the
// forward prefix before its first element and its wave-inclusive map
// aggregate; per wave: the block prefix) waits in two LDS slots.  The
// per-tile arithmetic is that of k_scan_vjp.
template <int TH_>
__global__ __launch_bounds__(TH_) void k_scan_vjp_m2d(ScanVjpArgs a) {
  constexpr int OP = MAT2;
  using Op = FwdLB<OP>;
  using FT = typename Op::T;
  using A = Adj<OP, false>;
  using M = typename A::M;
  using MT = typename M::T;
  using Sh = ShapeT<OP, TH_>;
  constexpr int K = Sh::K, TILE = Sh::TILE, TH = Sh::THREADS, W = Sh::W;
  constexpr int N = Fwd<OP>::N, NA = M::NA;
  static_assert(Sh::EPL == 1 && lane_major<OP, 1>(), "lane-major 2x2 tiles");
  struct Buf {
    float4 x[K], yb[K];
  };

  __shared__ FT s_ftot[W];
  __shared__ FT s_fpre[W];
  __shared__ MT s_mtot[W];
  __shared__ MT s_mpre[2][W];
  __shared__ float s_thr[2][N][TH];
  __shared__ float s_minc[2][NA][TH];
  __shared__ MT s_carry;
  __shared__ unsigned s_epoch;

  const int tid = threadIdx.x, lane = lane_id(), wave = tid / WAVE;
  const int64_t G = gridDim.x;
  // group g of tile ti: element tid*K + g (plain loads: the lanes stride
  // through lines that the next groups' loads read)
  auto load_grp = [&](const TileInfo &ti, Buf &b, int g) {
    const int el = group_el<true, K, TH, 1>(g, tid);
    const int v = ti.valid - el;
    b.x[g] = load_group<4, false>(a.x0, ti.base, el, v, true, make_float4(1, 0, 0, 1));
    b.yb[g] = load_group<4, false>(a.yb0, ti.base, el, v, true, make_float4(0, 0, 0, 0));
  };
  auto xg = [&](const Buf &b, int g) -> FT { return FT{{b.x[g].x, b.x[g].y, b.x[g].z, b.x[g].w}}; };
  auto ybg = [&](const Buf &b, int g, float *yb) {
    yb[0] = b.yb[g].x; yb[1] = b.yb[g].y; yb[2] = b.yb[g].z; yb[3] = b.yb[g].w;
  };

  if (tid == 0) s_epoch = ctl_load(&a.ctl->epoch);
  int64_t k = blockIdx.x;
  uint32_t tag = 0;
  auto tile_of = [&](int64_t kk) { return a.ntiles - 1 - kk; };  // right to left

  // scans tile kk up to the wave level, state into LDS slot sl
  auto phase1 = [&](int64_t kk, const Buf &cur, int sl, auto &&after) {
    const TileInfo ti = tile_info(tile_of(kk), a.n, a.tpr, TILE);
    FT acc = xg(cur, 0);
#pragma unroll
    for (int g = 1; g < K; ++g) acc = Op::comb(acc, xg(cur, g));
    const FT fin = wave_scan_fwd<Op>(acc);
    if (lane == WAVE - 1) s_ftot[wave] = fin;
    __syncthreads();
    if (wave == 0) {
      FT c;
#pragma unroll
      for (int i = 0; i < N; ++i) c.f[i] = a.saved[ti.tile * N + i];
      wave0_block_prefix<Op, 1, W, false>(reinterpret_cast<FT (*)[W]>(s_ftot),
                                          reinterpret_cast<FT (*)[W]>(s_fpre), c);
    }
    __syncthreads();
    FT thr[K];
    {
      FT ex = shift_up1(fin);
      if (lane == 0) ex = Op::id();
      thr[0] = Op::comb(s_fpre[wave], ex);
    }
#pragma unroll
    for (int i = 0; i < N; ++i) s_thr[sl][i][tid] = thr[0].f[i];
#pragma unroll
    for (int g = 1; g < K; ++g) thr[g] = Op::comb(thr[g - 1], xg(cur, g - 1));
    MT macc = M::id();
#pragma unroll
    for (int g = K - 1; g >= 0; --g) {
      float yb[4];
      ybg(cur, g, yb);
      const MT h = A::make(thr[g], xg(cur, g), yb, false);
      macc = (g == K - 1) ? h : M::comb(macc, h);
      after(g);
    }
    const MT mi = wave_scan_rev<M>(macc);
#pragma unroll
    for (int i = 0; i < NA; ++i) s_minc[sl][i][tid] = mi.f[i];
    if (lane == 0) s_mtot[wave] = mi;
  };

  auto block_level = [&](int64_t kk, int sl) -> MT {
    const TileInfo ti = tile_info(tile_of(kk), a.n, a.tpr, TILE);
    const MT agg = wave0_block_prefix<M, 1, W, true>(reinterpret_cast<MT (*)[W]>(s_mtot),
                                                     reinterpret_cast<MT (*)[W]>(s_mpre[sl]),
                                                     M::id());
    uint64_t *st = a.status + ti.tile * (M::NA + M::NP);
    if (lane == 0) {
      if (ti.lt == a.tpr - 1) {
        typename M::P zero;
#pragma unroll
        for (int i = 0; i < M::NP; ++i) zero.f[i] = 0.0f;
        publish<M::NP>(st + M::NA, tag, M::apply0(M::comb(M::from_pre(zero), agg)));
      } else {
        publish<M::NA>(st, tag, agg);
      }
    }
    return agg;
  };

  MT prev_incl = M::id();  // wave 0: inclusive prefix of the block's previous tile
  auto resolve = [&](int64_t ks, const MT &agg_s, bool scanned, int64_t kp, MT &agg_p, int slp) {
    __syncthreads();
    if (wave == 0) {
      if (scanned) agg_p = block_level(kp, slp);
      const TileInfo ti = tile_info(tile_of(ks), a.n, a.tpr, TILE);
      typename M::P zero;
#pragma unroll
      for (int i = 0; i < M::NP; ++i) zero.f[i] = 0.0f;
      MT c = M::from_pre(zero);
      const int dist_max = a.tpr - 1 - ti.lt;
      if (dist_max > 0) {
        const int win = dist_max < G ? dist_max : (int)(G - 1);
        bool hit = false;
        if (win > 0) c = lookback<M>(a.status, ti.tile, -1, win, tag, a.ctl, &hit);
        if (!hit) c = win > 0 ? M::comb(prev_incl, c) : prev_incl;
        if (lane == 0)
          publish<M::NP>(a.status + ti.tile * (M::NA + M::NP) + M::NA, tag,
                         M::apply0(M::comb(c, agg_s)));
      }
      prev_incl = M::from_pre(M::apply0(M::comb(c, agg_s)));
      if (lane == 0) {
        s_carry = c;
        if (ti.lt == 0) ctl_row_done(a.ctl, (unsigned)(a.ntiles / a.tpr), tag);
      }
    }
    __syncthreads();
  };

  // thread-serial sweep of tile ks from its last element; the thread's
  // elements are stored together afterwards with ordinary stores, which L2
  // merges into whole lines
  auto sweep = [&](int64_t ks, const Buf &cur, int sl) {
    const TileInfo ti = tile_info(tile_of(ks), a.n, a.tpr, TILE);
    MT mi;
#pragma unroll
    for (int i = 0; i < NA; ++i) mi.f[i] = s_minc[sl][i][tid];
    MT ex = shift_down1(mi);
    if (lane == WAVE - 1) ex = M::id();
    typename M::P rho = M::apply0(M::comb(M::comb(s_carry, s_mpre[sl][wave]), ex));
    FT thr[K];
#pragma unroll
    for (int i = 0; i < N; ++i) thr[0].f[i] = s_thr[sl][i][tid];
#pragma unroll
    for (int g = 1; g < K; ++g) thr[g] = Op::comb(thr[g - 1], xg(cur, g - 1));
    float4 o[K];
#pragma unroll
    for (int g = K - 1; g >= 0; --g) {
      float yb[4], xb[4];
      ybg(cur, g, yb);
      A::step(thr[g], xg(cur, g), yb, false, rho, xb);
      o[g] = make_float4(xb[0], xb[1], xb[2], xb[3]);
    }
#pragma unroll
    for (int g = 0; g < K; ++g) {
      const int el = group_el<true, K, TH, 1>(g, tid);
      if (el >= ti.valid) break;
      float4 *q = reinterpret_cast<float4 *>(a.xb0 + (ti.base + el) * 4);
      float4 val = o[g];
      if (a.accumulate) {
        const float4 old = *q;
        val.x += old.x; val.y += old.y; val.z += old.z; val.w += old.w;
      }
      *q = val;
    }
  };

  Buf b0, b1, b2;
  MT g0 = M::id(), g1 = M::id(), g2 = M::id();  // wave 0: map aggregates
  int sl = 0;
  {
    const TileInfo ti = tile_info(tile_of(k), a.n, a.tpr, TILE);
#pragma unroll
    for (int g = 0; g < K; ++g) load_grp(ti, b0, g);
  }
  __syncthreads();
  tag = next_tag(s_epoch);
  {
    const bool has1 = k + G < a.ntiles;
    const TileInfo t1 = tile_info(tile_of(has1 ? k + G : k), a.n, a.tpr, TILE);
    phase1(k, b0, 0, [&](int g) {
      if (has1) load_grp(t1, b1, g);
    });
    __syncthreads();
    if (wave == 0) g0 = block_level(k, 0);
    __syncthreads();  // s_mtot is rewritten by the next scan
  }
  auto step = [&](Buf &bs, MT &gs, Buf &bp, MT &gp, Buf &bl) -> bool {
    const bool scan = k + G < a.ntiles;
    if (scan) {
      const bool has2 = k + 2 * G < a.ntiles;
      const TileInfo t2 = tile_info(tile_of(has2 ? k + 2 * G : k), a.n, a.tpr, TILE);
      phase1(k + G, bp, sl ^ 1, [&](int g) {
        if (has2) load_grp(t2, bl, g);
      });
    }
    resolve(k, gs, scan, k + G, gp, sl ^ 1);
    sweep(k, bs, sl);
    if (!scan) return false;
    k += G;
    sl ^= 1;
    return true;
  };
  for (;;) {
    if (!step(b0, g0, b1, g1, b2)) break;
    if (!step(b1, g1, b2, g2, b0)) break;
    if (!step(b2, g2, b0, g0, b1)) break;
  }
}

// ---------------------------------------------------------------------------
// host launchers
// ---------------------------------------------------------------------------
int scan_tile_size(int op) {
  switch (op) {
  case ADD: return Shape<ADD>::TILE;
  case MUL: return Shape<MUL>::TILE;
  case MIN: return Shape<MIN>::TILE;
  case MAX: return Shape<MAX>::TILE;
  case SATADD: return Shape<SATADD>::TILE;
  case SUMPROD: return Shape<SUMPROD>::TILE;
  case LINREC: return Shape<LINREC>::TILE;
  case MAT2: return Shape<MAT2>::TILE;
  }
  return 0;
}

int scan_elem_floats(int op) { return (op == LINREC || op == SUMPROD) ? 2 : (op == MAT2 ? 4 : 1); }

// status words per tile: forward (N + N); adjoint maps (NA + NP)
int scan_status_words(int op, bool abar) {
  switch (op) {
  case ADD: return 2;
  case MUL: case MIN: case MAX: case SATADD: return 3;
  case LINREC: return abar ? 5 : 4;
  case MAT2: return 12;
  case SUMPROD: return 7;
  }
  return 0;
}

// Blocks that can be resident at once on the current device for a kernel.
// The persistent grids above rely on all of their blocks being co-resident:
// a block waits only on tiles of lower scan order, owned by resident blocks.
template <class F>
int64_t resident_blocks(F kernel, int threads) {
  int dev = 0, cus = 0, occ = 0;
  if (hipGetDevice(&dev) != hipSuccess) return 0;
  if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess) return 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&occ, kernel, threads, 0) != hipSuccess) return 0;
  return (int64_t)cus * (occ > 0 ? occ : 1);
}

template <int OP, bool REDUCE, int TH>
static hipError_t launch_fwd_t(const ScanFwdArgs &a, hipStream_t s) {
  static int64_t cap = 0;
  if (cap == 0) cap = resident_blocks(k_scan_fwd<OP, REDUCE, TH>, TH);
  if (cap == 0) return hipErrorInvalidDevice;
  const int64_t grid = a.ntiles < cap ? a.ntiles : cap;
  hipLaunchKernelGGL((k_scan_fwd<OP, REDUCE, TH>), dim3((unsigned)grid), dim3(TH), 0, s, a);
  return hipGetLastError();
}

// block size from the tuning knobs (the tile, and so every saved layout, is
// the same for every block size)
template <int OP, bool REDUCE>
static hipError_t launch_fwd(const ScanFwdArgs &a, hipStream_t s) {
  switch (knob_scan_threads(OP, 0)) {
  case 256: return launch_fwd_t<OP, REDUCE, 256>(a, s);
  case 512: return launch_fwd_t<OP, REDUCE, 512>(a, s);
  default: return launch_fwd_t<OP, REDUCE, 1024>(a, s);
  }
}

template <int OP, bool ABAR, bool CKPT, int TH>
static hipError_t launch_vjp_t(const ScanVjpArgs &a, hipStream_t s) {
  static int64_t cap = 0;
  // the delayed forms hold three tiles in registers: not for the 2x2
  // product's checkpoint form, nor for the recurrence with the adjoint of
  // its cumulative product, whose extra input streams would spill
  if constexpr (OP == MAT2 && !CKPT) {
    if (cap == 0) cap = resident_blocks(k_scan_vjp_m2d<TH>, TH);
    if (cap == 0) return hipErrorInvalidDevice;
    const int64_t grid = a.ntiles < cap ? a.ntiles : cap;
    hipLaunchKernelGGL((k_scan_vjp_m2d<TH>), dim3((unsigned)grid), dim3(TH), 0, s, a);
  } else if constexpr (lane_major<OP, 1>() || ABAR) {
    if (cap == 0) cap = resident_blocks(k_scan_vjp<OP, ABAR, CKPT, TH>, TH);
    if (cap == 0) return hipErrorInvalidDevice;
    const int64_t grid = a.ntiles < cap ? a.ntiles : cap;
    hipLaunchKernelGGL((k_scan_vjp<OP, ABAR, CKPT, TH>), dim3((unsigned)grid), dim3(TH), 0, s, a);
  } else {
    if (cap == 0) cap = resident_blocks(k_scan_vjp_d<OP, ABAR, CKPT, TH>, TH);
    if (cap == 0) return hipErrorInvalidDevice;
    const int64_t grid = a.ntiles < cap ? a.ntiles : cap;
    hipLaunchKernelGGL((k_scan_vjp_d<OP, ABAR, CKPT, TH>), dim3((unsigned)grid), dim3(TH), 0, s, a);
  }
  return hipGetLastError();
}

template <int OP, bool ABAR, bool CKPT>
static hipError_t launch_vjp(const ScanVjpArgs &a, hipStream_t s) {
  switch (knob_scan_threads(OP, 1)) {
  case 256: return launch_vjp_t<OP, ABAR, CKPT, 256>(a, s);
  case 1024: return launch_vjp_t<OP, ABAR, CKPT, 1024>(a, s);
  default: return launch_vjp_t<OP, ABAR, CKPT, 512>(a, s);
  }
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
  a.n = n; a.tpr = tpr; a.ntiles = tiles;
  a.ctl = reinterpret_cast<Ctl *>(ws);
  a.status = reinterpret_cast<uint64_t *>(static_cast<char *>(ws) + kCtlBytes);
#define PCAD_FWD(OPV)                                                           \
  case OPV:                                                                     \
    return reduce ? launch_fwd<OPV, true>(a, s) : launch_fwd<OPV, false>(a, s);
  switch (op) {
    PCAD_FWD(ADD)
    PCAD_FWD(MUL)
    PCAD_FWD(MIN)
    PCAD_FWD(MAX)
    PCAD_FWD(SATADD)
    PCAD_FWD(SUMPROD)
    PCAD_FWD(LINREC)
    PCAD_FWD(MAT2)
  }
#undef PCAD_FWD
  return hipErrorInvalidValue;
}

hipError_t scan_vjp_launch(int op, int64_t batch, int64_t n, const float *x0, const float *x1,
                           const float *saved, const float *tp0, const float *tp1,
                           const float *yb0, const float *yb1, float *xb0, float *xb1,
                           bool accumulate, void *ws, hipStream_t s) {
  const int tile = scan_tile_size(op);
  const int tpr = (int)((n + tile - 1) / tile);
  const int64_t tiles = batch * (int64_t)tpr;
  if (tiles == 0) return hipSuccess;
  ScanVjpArgs a;
  a.x0 = x0; a.x1 = x1; a.saved = saved; a.tp0 = tp0; a.tp1 = tp1;
  a.yb0 = yb0; a.yb1 = yb1; a.xb0 = xb0; a.xb1 = xb1;
  a.n = n; a.tpr = tpr; a.ntiles = tiles; a.accumulate = accumulate ? 1 : 0;
  a.ctl = reinterpret_cast<Ctl *>(ws);
  a.status = reinterpret_cast<uint64_t *>(static_cast<char *>(ws) + kCtlBytes);
  const bool ck = tp0 != nullptr;
  switch (op) {
  case ADD: return launch_vjp<ADD, false, false>(a, s);
  case MUL: return ck ? launch_vjp<MUL, false, true>(a, s) : launch_vjp<MUL, false, false>(a, s);
  case MIN: return ck ? launch_vjp<MIN, false, true>(a, s) : launch_vjp<MIN, false, false>(a, s);
  case MAX: return ck ? launch_vjp<MAX, false, true>(a, s) : launch_vjp<MAX, false, false>(a, s);
  case SATADD:
    return ck ? launch_vjp<SATADD, false, true>(a, s) : launch_vjp<SATADD, false, false>(a, s);
  case SUMPROD:  // recompute form only: the checkpoint form would need s as well
    return ck ? hipErrorInvalidValue : launch_vjp<SUMPROD, false, false>(a, s);
  case LINREC:
    if (yb1)
      return ck ? launch_vjp<LINREC, true, true>(a, s) : launch_vjp<LINREC, true, false>(a, s);
    return ck ? launch_vjp<LINREC, false, true>(a, s) : launch_vjp<LINREC, false, false>(a, s);
  case MAT2: return ck ? launch_vjp<MAT2, false, true>(a, s) : launch_vjp<MAT2, false, false>(a, s);
  }
  return hipErrorInvalidValue;
}

}  // namespace pcad
