// Device-side building blocks shared by the scan, reduce and reduce-by-index
// kernels: element types, the forward operators, the adjoint affine maps of
// the scan adjoint, wave64 scans, coalesced tile I/O, and the decoupled
// look-back protocol with epoch-tagged status words.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace pcad {

constexpr int BLOCK = 256;
constexpr int WAVE = 64;
constexpr int WAVES = BLOCK / WAVE;

// operator ids (same values as the public enum).  SUMPROD is Section 3.3's
// invertible operator sumOfProd (reduce, scan, reduce-by-index).
// SATADD is the saturated addition of the evaluation's operator figure.
enum { ADD = 0, MUL = 1, MIN = 2, MAX = 3, LINREC = 4, MAT2 = 5, SUMPROD = 6, SATADD = 7 };

// the saturation level of SATADD
constexpr float kSatCap = 1000000.0f;

template <int N>
struct Vec {
  float f[N];
};

// ---------------------------------------------------------------------------
// wave64 data movement (ds_bpermute through the LDS crossbar, no LDS storage)
// ---------------------------------------------------------------------------
__device__ __forceinline__ int lane_id() { return (int)__lane_id(); }

template <int N>
__device__ __forceinline__ Vec<N> shfl_up(const Vec<N> &v, int d) {
  Vec<N> r;
#pragma unroll
  for (int i = 0; i < N; ++i) r.f[i] = __shfl_up(v.f[i], d, WAVE);
  return r;
}

template <int N>
__device__ __forceinline__ Vec<N> shfl_down(const Vec<N> &v, int d) {
  Vec<N> r;
#pragma unroll
  for (int i = 0; i < N; ++i) r.f[i] = __shfl_down(v.f[i], d, WAVE);
  return r;
}

template <int N>
__device__ __forceinline__ Vec<N> readlane(const Vec<N> &v, int l) {
  Vec<N> r;
#pragma unroll
  for (int i = 0; i < N; ++i)
    r.f[i] = __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v.f[i]), l));
  return r;
}

// strong-zero product: 0 * anything = 0, so an overflowed partial product
// (inf) met by an exact zero does not turn into NaN.
__device__ __forceinline__ float mulz(float a, float b) {
  return (a == 0.0f || b == 0.0f) ? 0.0f : a * b;
}

// ---------------------------------------------------------------------------
// float += in LDS.  ds_add_f32 runs at a fixed low rate whatever the
// addresses, while a compare-and-swap runs at the full LDS rate when lanes
// hit different words; so one compare-and-swap is tried first and only the
// lanes that lost it (several lanes on one bin: skewed keys) fall back to
// ds_add_f32.  Either way v is added exactly once.
// ---------------------------------------------------------------------------
__device__ __forceinline__ void lds_add_f32(float *p, float v) {
  unsigned *u = reinterpret_cast<unsigned *>(p);
  unsigned old = __hip_atomic_load(u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
  if (!__hip_atomic_compare_exchange_strong(u, &old, __float_as_uint(__uint_as_float(old) + v),
                                            __ATOMIC_RELAXED, __ATOMIC_RELAXED,
                                            __HIP_MEMORY_SCOPE_WORKGROUP))
    atomicAdd(p, v);
}

// ---------------------------------------------------------------------------
// sumOfProd (Section 3.3) on lifted pairs (p, s):
//   (p1, s1) (.) (p2, s2) = (p1 + p2 + s1*s2, s1 + s2),  neutral (0, 0);
// an input a enters as (0, a).  A pair packs into one 64-bit word
// {s:32 | p:32} so that an update is one 64-bit compare-and-swap.
// ---------------------------------------------------------------------------
struct SP {
  float p, s;
};

__device__ __forceinline__ SP sp_comb(const SP &a, const SP &b) {
  return {a.p + b.p + a.s * b.s, a.s + b.s};
}

__device__ __forceinline__ uint64_t sp_pack(const SP &v) {
  return ((uint64_t)__float_as_uint(v.s) << 32) | __float_as_uint(v.p);
}

__device__ __forceinline__ SP sp_unpack(uint64_t w) {
  return {__uint_as_float((uint32_t)w), __uint_as_float((uint32_t)(w >> 32))};
}

// *w = *w (.) v, atomically; SCOPE: workgroup for LDS, agent for global
template <int SCOPE>
__device__ __forceinline__ void sp_atomic(uint64_t *w, const SP &v) {
  uint64_t old = __hip_atomic_load(w, __ATOMIC_RELAXED, SCOPE);
  for (;;) {
    const uint64_t nw = sp_pack(sp_comb(sp_unpack(old), v));
    if (__hip_atomic_compare_exchange_strong(w, &old, nw, __ATOMIC_RELAXED, __ATOMIC_RELAXED, SCOPE))
      return;
  }
}

// One wave's LDS update of table[bin] (.)= (0, x) for the lanes with ok.
// The lanes whose bin equals the first active lane's fold their elements
// with a butterfly first and make one update together (skewed keys would
// otherwise retry the same word 64 ways); must be called by all 64 lanes.
__device__ __forceinline__ void sp_wave_update(uint64_t *table, uint32_t bin, float x, bool ok) {
  const uint64_t act = __ballot(ok);
  if (act == 0) return;
  const int first = __builtin_ctzll(act);
  const uint32_t b0 = (uint32_t)__builtin_amdgcn_readlane((int)bin, first);
  const bool hot = ok && bin == b0;
  SP v = {0.0f, hot ? x : 0.0f};
#pragma unroll
  for (int d = 1; d < WAVE; d <<= 1) {
    const SP o = {__shfl_xor(v.p, d, WAVE), __shfl_xor(v.s, d, WAVE)};
    v = sp_comb(v, o);
  }
  if (lane_id() == first) sp_atomic<__HIP_MEMORY_SCOPE_WORKGROUP>(&table[b0], v);
  if (ok && !hot) sp_atomic<__HIP_MEMORY_SCOPE_WORKGROUP>(&table[bin], SP{0.0f, x});
}

// ---------------------------------------------------------------------------
// Lifted min/max as one 64-bit word, so "smallest value, then smallest
// index" is a single native 64-bit atomic min (or max with the index
// complemented): key = {ord(v):32 | index:32}.  ord is the order-preserving
// map float -> uint32 with -0.0 folded onto +0.0 (equal values tie).
// ---------------------------------------------------------------------------
__device__ __forceinline__ uint32_t ord_f32(float v) {
  uint32_t b = __float_as_uint(v == 0.0f ? 0.0f : v);
  return (b & 0x80000000u) ? ~b : (b | 0x80000000u);
}

// inverse of ord_f32 (returns +0.0 for a folded zero)
__device__ __forceinline__ float ord_inv(uint32_t o) {
  return __uint_as_float((o & 0x80000000u) ? (o & 0x7fffffffu) : ~o);
}

template <int OP>
__device__ __forceinline__ uint64_t key_of(float v, uint32_t i) {
  return OP == MIN ? (((uint64_t)ord_f32(v) << 32) | i)
                   : (((uint64_t)ord_f32(v) << 32) | (uint32_t)(~i));
}

template <int OP>
constexpr uint64_t key_init() {
  return OP == MIN ? ~0ull : 0ull;
}

// ---------------------------------------------------------------------------
// forward operators.  comb(earlier, later) in index order.
// ---------------------------------------------------------------------------
template <int OP>
struct Fwd;

template <>
struct Fwd<ADD> {
  static constexpr int N = 1;
  using T = Vec<1>;
  __device__ static T id() { return {{0.0f}}; }
  __device__ static T comb(const T &a, const T &b) { return {{a.f[0] + b.f[0]}}; }
};

template <>
struct Fwd<MUL> {
  static constexpr int N = 1;
  using T = Vec<1>;
  __device__ static T id() { return {{1.0f}}; }
  __device__ static T comb(const T &a, const T &b) { return {{mulz(a.f[0], b.f[0])}}; }
};

template <>
struct Fwd<MIN> {
  static constexpr int N = 1;
  using T = Vec<1>;
  __device__ static T id() { return {{__builtin_inff()}}; }
  // the earlier operand is kept on a tie (lowest index wins)
  __device__ static T comb(const T &a, const T &b) { return {{b.f[0] < a.f[0] ? b.f[0] : a.f[0]}}; }
};

template <>
struct Fwd<MAX> {
  static constexpr int N = 1;
  using T = Vec<1>;
  __device__ static T id() { return {{-__builtin_inff()}}; }
  __device__ static T comb(const T &a, const T &b) { return {{b.f[0] > a.f[0] ? b.f[0] : a.f[0]}}; }
};

// sumOfProd (Section 3.3) on lifted pairs (p, s); scans lift an input a to
// (0, a) and write p
template <>
struct Fwd<SUMPROD> {
  static constexpr int N = 2;
  using T = Vec<2>;
  __device__ static T id() { return {{0.0f, 0.0f}}; }
  __device__ static T comb(const T &a, const T &b) {
    return {{__builtin_fmaf(a.f[1], b.f[1], a.f[0] + b.f[0]), a.f[1] + b.f[1]}};
  }
};

// saturated addition: the sum, or the cap when the sum exceeds it
// (associative and commutative on values in [0, cap])
template <>
struct Fwd<SATADD> {
  static constexpr int N = 1;
  using T = Vec<1>;
  __device__ static T id() { return {{0.0f}}; }
  __device__ static T comb(const T &a, const T &b) {
    const float t = a.f[0] + b.f[0];
    return {{t > kSatCap ? kSatCap : t}};
  }
};

// linear-function composition, element (A = multiplier, B = offset):
// (A1,B1) then (A2,B2) = (A1*A2, A2*B1 + B2)
template <>
struct Fwd<LINREC> {
  static constexpr int N = 2;
  using T = Vec<2>;
  __device__ static T id() { return {{1.0f, 0.0f}}; }
  __device__ static T comb(const T &a, const T &b) {
    return {{a.f[0] * b.f[0], __builtin_fmaf(b.f[0], a.f[1], b.f[1])}};
  }
};

// 2x2 matrix product, row-major
template <>
struct Fwd<MAT2> {
  static constexpr int N = 4;
  using T = Vec<4>;
  __device__ static T id() { return {{1.0f, 0.0f, 0.0f, 1.0f}}; }
  __device__ static T comb(const T &p, const T &m) {
    return {{__builtin_fmaf(p.f[0], m.f[0], p.f[1] * m.f[2]),
             __builtin_fmaf(p.f[0], m.f[1], p.f[1] * m.f[3]),
             __builtin_fmaf(p.f[2], m.f[0], p.f[3] * m.f[2]),
             __builtin_fmaf(p.f[2], m.f[1], p.f[3] * m.f[3])}};
  }
};

// ---------------------------------------------------------------------------
// tile shapes.  A group is one 16-byte vector per input stream per lane:
// EPL elements.  A tile is K groups of THREADS lanes: element e of a tile
// lives in group e / (THREADS*EPL), lane (e % (THREADS*EPL)) / EPL, slot
// e % EPL.
// ---------------------------------------------------------------------------
// Scan tile shapes.  A tile holds PCAD_SCAN_TILE elements (a quarter of
// that for MAT2, whose elements are 16 bytes); the forward and the adjoint
// kernels may use different block sizes (DIR 0 / 1) over the same tiles, so
// the adjoint reads the forward's per-tile prefixes.  Build-time knobs for
// shape sweeps.
#ifndef PCAD_SCAN_TILE
#define PCAD_SCAN_TILE 8192
#endif
#ifndef PCAD_FWD_THREADS
#define PCAD_FWD_THREADS 1024
#endif
#ifndef PCAD_FWD_THREADS_WIDE  // LINREC and MAT2 (more state per element)
#define PCAD_FWD_THREADS_WIDE 512
#endif
#ifndef PCAD_VJP_THREADS
#define PCAD_VJP_THREADS 512
#endif

// a tile of the scan kernels split over TH_ threads
template <int OP, int TH_>
struct ShapeT {
  static constexpr int EPL = (OP == MAT2) ? 1 : 4;
  static constexpr int TILE = (OP == MAT2) ? PCAD_SCAN_TILE / 4 : PCAD_SCAN_TILE;
  static constexpr int THREADS = TH_;
  static constexpr int W = THREADS / WAVE;
  static constexpr int K = TILE / (THREADS * EPL);
  static_assert(K >= 1 && K * THREADS * EPL == TILE, "tile must be whole groups of the block");
};

// Element layout of a tile over the threads: group-major (group g of all
// threads, then group g+1) or lane-major (a thread's K groups are
// consecutive elements, so a tile needs one serial pass and one wave scan
// per thread instead of one per group).  Lane-major cuts the scan work
// where it dominates -- the adjoint of the 2x2 matrix product -- but its
// loads are strided by K groups, so it pays only with few groups per thread
// (1024-thread blocks); the forward kernels (DIR 0) stay group-major.
template <int OP, int DIR>
constexpr bool lane_major() {
  return DIR == 1 && OP == MAT2;
}

// first element of group g of thread tid within a tile
template <bool LM, int K, int TH, int EPL>
__device__ __forceinline__ int group_el(int g, int tid) {
  return LM ? (tid * K + g) * EPL : g * TH * EPL + tid * EPL;
}

template <int OP, int DIR = 0>
struct Shape {
  static constexpr int EPL = (OP == MAT2) ? 1 : 4;
  static constexpr int TILE = (OP == MAT2) ? PCAD_SCAN_TILE / 4 : PCAD_SCAN_TILE;
  static constexpr int THREADS =
      DIR == 1 ? PCAD_VJP_THREADS
               : ((OP == LINREC || OP == MAT2) ? PCAD_FWD_THREADS_WIDE : PCAD_FWD_THREADS);
  static constexpr int W = THREADS / WAVE;
  static constexpr int K = TILE / (THREADS * EPL);
  static_assert(K >= 1 && K * THREADS * EPL == TILE, "tile must be whole groups of the block");
};

// 16-byte load of data that a kernel reads once: the nontemporal hint
// streams it through the caches with early eviction.  A device copy
// measured 5.8 TB/s with the hint on both its loads and its stores and
// 5.2 TB/s with plain ones; the batched adjoint's traffic shape (4 read and
// 2 write streams in persistent 8192-element tiles) 5.7 against 5.4 TB/s
// with streaming stores only.
template <class V>
__device__ __forceinline__ V ld_stream(const void *p) {
  typedef int v4i __attribute__((ext_vector_type(4)));
  static_assert(sizeof(V) == 16, "16-byte vectors");
  return __builtin_bit_cast(V, __builtin_nontemporal_load(reinterpret_cast<const v4i *>(p)));
}

// 16-byte load of one group of one stream: element `el` (a lane's first)
// of the tile starting at element `base`.  `S` floats per element.  When the
// group is whole and the address 16-byte aligned, one dwordx4 load;
// otherwise element-wise loads of the valid part with `fill` elsewhere.
// The tile's base pointer is block-uniform and the lane offset 32-bit, so
// the address is a scalar base plus a vector offset.  NT: the nontemporal
// hint, for groups whose lines no other load instruction reads (off where
// lanes stride through lines that the next instructions read, as in
// lane-major tiles, whose fetched bytes grew 10% with it).
template <int S, bool NT = true>
__device__ __forceinline__ float4 load_group(const float *__restrict__ p, int64_t base, int el,
                                             int valid, bool vec_ok, float4 fill) {
  const float *__restrict__ q = p + base * S;
  const unsigned o = (unsigned)el * S;
  if (valid >= 4 / S && (S == 4 || vec_ok)) {
    return NT ? ld_stream<float4>(q + o) : *reinterpret_cast<const float4 *>(q + o);
  }
  float r[4] = {fill.x, fill.y, fill.z, fill.w};
  if (S == 4) {
    if (valid > 0) {
      float4 t = NT ? ld_stream<float4>(q + o) : *reinterpret_cast<const float4 *>(q + o);
      r[0] = t.x; r[1] = t.y; r[2] = t.z; r[3] = t.w;
    }
  } else {
#pragma unroll
    for (int j = 0; j < 4; ++j)
      if (j < valid) r[j] = q[o + j];
  }
  return make_float4(r[0], r[1], r[2], r[3]);
}

template <int S>
__device__ __forceinline__ void store_group(float *__restrict__ p, int64_t base, int el, int valid,
                                            bool vec_ok, float4 v) {
  float *__restrict__ q = p + base * S;
  const unsigned o = (unsigned)el * S;
  if (valid >= 4 / S && (S == 4 || vec_ok)) {
    // one 16-byte streaming store per lane: whole 64-byte lines per quad of
    // lanes, no partial-line writes
    typedef float v4f __attribute__((ext_vector_type(4)));
    v4f w = {v.x, v.y, v.z, v.w};
    __builtin_nontemporal_store(w, reinterpret_cast<v4f *>(q + o));
    return;
  }
  float r[4] = {v.x, v.y, v.z, v.w};
  if (S == 4) {
    if (valid > 0) {
#pragma unroll
      for (int j = 0; j < 4; ++j) q[o + j] = r[j];
    }
  } else {
#pragma unroll
    for (int j = 0; j < 4; ++j)
      if (j < valid) q[o + j] = r[j];
  }
}

__device__ __forceinline__ float f4get(const float4 &v, int j) {
  return j == 0 ? v.x : (j == 1 ? v.y : (j == 2 ? v.z : v.w));
}

__device__ __forceinline__ void f4set(float4 &v, int j, float x) {
  if (j == 0) v.x = x;
  else if (j == 1) v.y = x;
  else if (j == 2) v.z = x;
  else v.w = x;
}

// ---------------------------------------------------------------------------
// input / output streams per operator
// ---------------------------------------------------------------------------
template <int OP>
struct IO;

template <int OP>
struct IOScalar {
  static constexpr int NIN = 1, S = 1;
  using FT = typename Fwd<OP>::T;
  __device__ static float4 fill(int) {
    const float e = Fwd<OP>::id().f[0];
    return make_float4(e, e, e, e);
  }
  __device__ static FT elem(const float4 (&in)[NIN], int j) { return {{f4get(in[0], j)}}; }
};
template <>
struct IO<ADD> : IOScalar<ADD> {};
template <>
struct IO<MUL> : IOScalar<MUL> {};
template <>
struct IO<MIN> : IOScalar<MIN> {};
template <>
struct IO<MAX> : IOScalar<MAX> {};
template <>
struct IO<SATADD> : IOScalar<SATADD> {};

// sumOfProd: one scalar stream, each value lifted to (0, a)
template <>
struct IO<SUMPROD> {
  static constexpr int NIN = 1, S = 1;
  using FT = Fwd<SUMPROD>::T;
  __device__ static float4 fill(int) { return make_float4(0, 0, 0, 0); }
  __device__ static FT elem(const float4 (&in)[NIN], int j) { return {{0.0f, f4get(in[0], j)}}; }
};

template <>
struct IO<LINREC> {
  static constexpr int NIN = 2, S = 1;
  using FT = Fwd<LINREC>::T;
  __device__ static float4 fill(int s) {
    return s == 0 ? make_float4(1, 1, 1, 1) : make_float4(0, 0, 0, 0);
  }
  __device__ static FT elem(const float4 (&in)[NIN], int j) {
    return {{f4get(in[0], j), f4get(in[1], j)}};
  }
};

template <>
struct IO<MAT2> {
  static constexpr int NIN = 1, S = 4;
  using FT = Fwd<MAT2>::T;
  __device__ static float4 fill(int) { return make_float4(1, 0, 0, 1); }
  __device__ static FT elem(const float4 (&in)[NIN], int) {
    return {{in[0].x, in[0].y, in[0].z, in[0].w}};
  }
};

struct TileInfo {
  int64_t tile;   // global tile index
  int64_t row;
  int lt;         // tile index within the row
  int64_t base;   // global index of the tile's first element
  int valid;      // elements of the tile inside the row
  bool vec_ok;    // 16-byte aligned scalar streams
};

__device__ __forceinline__ TileInfo tile_info(int64_t tile, int64_t n, int tpr, int TILE) {
  TileInfo t;
  t.tile = tile;
  t.row = tile / tpr;
  t.lt = (int)(tile - t.row * tpr);
  const int64_t ts = (int64_t)t.lt * TILE;
  t.base = t.row * n + ts;
  const int64_t rem = n - ts;
  t.valid = (int)(rem < TILE ? rem : TILE);
  t.vec_ok = (t.base & 3) == 0;
  return t;
}

// ---------------------------------------------------------------------------
// wave64 inclusive scans.  Tr::comb(earlier, later).
//   forward: lower lanes are earlier;  reverse: higher lanes are earlier.
// ---------------------------------------------------------------------------
// ---------------------------------------------------------------------------
// Cross-lane steps through DPP (data-parallel primitives: the VALU reads a
// neighbour lane's register in the same instruction, no LDS round trip).
// Control codes of the GFX9 DPP encoding.
// ---------------------------------------------------------------------------
constexpr int kDppRowShl = 0x100;   // + n: lane i reads lane i+n of its row of 16
constexpr int kDppRowShr = 0x110;   // + n: lane i reads lane i-n of its row
constexpr int kDppWaveShl1 = 0x130; // lane i reads lane i+1 of the wave
constexpr int kDppWaveShr1 = 0x138; // lane i reads lane i-1 of the wave
constexpr int kDppBcast15 = 0x142;  // lane 15 of a row to the next row
constexpr int kDppBcast31 = 0x143;  // lane 31 to rows 2 and 3

template <int CTRL, int ROWS = 0xf>
__device__ __forceinline__ float dpp_f(float v) {
  // lanes without a source (or outside ROWS) keep their own value
  return __int_as_float(
      __builtin_amdgcn_update_dpp(__float_as_int(v), __float_as_int(v), CTRL, ROWS, 0xf, false));
}

template <int CTRL, int ROWS = 0xf, int N>
__device__ __forceinline__ Vec<N> dpp_v(const Vec<N> &v) {
  Vec<N> r;
#pragma unroll
  for (int i = 0; i < N; ++i) r.f[i] = dpp_f<CTRL, ROWS>(v.f[i]);
  return r;
}

// x = comb(neighbour, x) where `valid`, x unchanged elsewhere
template <class Tr, int CTRL, int ROWS = 0xf>
__device__ __forceinline__ typename Tr::T dpp_step(const typename Tr::T &x, bool valid) {
  const typename Tr::T o = dpp_v<CTRL, ROWS>(x);
  return valid ? Tr::comb(o, x) : x;
}

// lane i gets lane i-1's value (lane 0 keeps its own)
template <int N>
__device__ __forceinline__ Vec<N> shift_up1(const Vec<N> &v) {
  return dpp_v<kDppWaveShr1>(v);
}

// lane i gets lane i+1's value (lane 63 keeps its own)
template <int N>
__device__ __forceinline__ Vec<N> shift_down1(const Vec<N> &v) {
  return dpp_v<kDppWaveShl1>(v);
}

template <class Tr>
__device__ __forceinline__ typename Tr::T wave_scan_fwd(typename Tr::T x) {
  // rows of 16 lanes: shifts by 1, 2, 4, 8 inside a row, then the row
  // totals through the row broadcasts of lanes 15 and 31
  const int lane = lane_id();
  x = dpp_step<Tr, kDppRowShr + 1>(x, (lane & 15) >= 1);
  x = dpp_step<Tr, kDppRowShr + 2>(x, (lane & 15) >= 2);
  x = dpp_step<Tr, kDppRowShr + 4>(x, (lane & 15) >= 4);
  x = dpp_step<Tr, kDppRowShr + 8>(x, (lane & 15) >= 8);
  x = dpp_step<Tr, kDppBcast15, 0xa>(x, (lane & 16) != 0);
  x = dpp_step<Tr, kDppBcast31, 0xc>(x, lane >= 32);
  return x;
}

// Inclusive scan from the right: lane i gets x_63 (.) ... (.) x_i, the
// higher lanes being the earlier operands.
template <class Tr>
__device__ __forceinline__ typename Tr::T wave_scan_rev(typename Tr::T x) {
  using T = typename Tr::T;
  const int lane = lane_id();
  x = dpp_step<Tr, kDppRowShl + 1>(x, (lane & 15) + 1 < 16);
  x = dpp_step<Tr, kDppRowShl + 2>(x, (lane & 15) + 2 < 16);
  x = dpp_step<Tr, kDppRowShl + 4>(x, (lane & 15) + 4 < 16);
  x = dpp_step<Tr, kDppRowShl + 8>(x, (lane & 15) + 8 < 16);
  // lane 16r now holds the total of row r; rows take the later rows' totals
  const T t1 = readlane(x, 16), t2 = readlane(x, 32), t3 = readlane(x, 48);
  const T s2 = Tr::comb(t3, t2);
  const T s1 = Tr::comb(s2, t1);
  const int row = lane >> 4;
  if (row < 3) x = Tr::comb(row == 2 ? t3 : (row == 1 ? s2 : s1), x);
  return x;
}

// Run by wave 0 only.  s_tot[g][w] holds the total of (group g, wave w) of a
// tile; scan order is g-major, w-minor, or its reverse (REV).  Writes
// s_pre[g][w] = init (.) (exclusive scan-order prefix) and returns the tile
// total (in every lane of wave 0).  K*W <= 64.
template <class Tr, int K, int W, bool REV>
__device__ __forceinline__ typename Tr::T wave0_block_prefix(typename Tr::T (*s_tot)[W],
                                                             typename Tr::T (*s_pre)[W],
                                                             const typename Tr::T &init) {
  using T = typename Tr::T;
  constexpr int NI = K * W;
  static_assert(NI <= WAVE, "too many wave totals for one wave");
  const int lane = lane_id();
  const int idx = REV ? (NI - 1 - lane) : lane;
  T v = Tr::id();
  if (lane < NI) v = s_tot[idx / W][idx % W];
  const T inc = wave_scan_fwd<Tr>(v);
  T ex = shift_up1(inc);
  if (lane == 0) ex = Tr::id();
  if (lane < NI) s_pre[idx / W][idx % W] = Tr::comb(init, ex);
  return readlane(inc, NI - 1);
}

// ordered reduction where lane L+1 is EARLIER than lane L; the full result
// (lane 63 earliest ... lane 0 latest) lands in lane 0.
template <class Tr>
__device__ __forceinline__ typename Tr::T wave_reduce_desc(typename Tr::T x) {
#pragma unroll
  for (int d = 1; d < WAVE; d <<= 1) {
    typename Tr::T o = shfl_down(x, d);
    x = Tr::comb(o, x);
  }
  return x;
}

// ---------------------------------------------------------------------------
// Look-back status words.  Every 32-bit component of a published value is
// stored in its own 64-bit word {tag:32 | bits:32}; a word is valid for the
// current launch iff its tag equals the launch tag, so no reset pass, fence
// or flag/value ordering is needed: a reader spins until every word it needs
// carries the tag.  Aggregates and inclusive prefixes use separate words.
// ---------------------------------------------------------------------------
__device__ __forceinline__ void put_word(uint64_t *w, uint32_t tag, float v) {
  uint64_t u = ((uint64_t)tag << 32) | (uint64_t)__float_as_uint(v);
  __hip_atomic_store(w, u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

template <int N>
__device__ __forceinline__ void publish(uint64_t *w, uint32_t tag, const Vec<N> &v) {
#pragma unroll
  for (int i = 0; i < N; ++i) put_word(w + i, tag, v.f[i]);
}

__device__ __forceinline__ uint64_t load_word(const uint64_t *w) {
  return __hip_atomic_load(const_cast<uint64_t *>(w), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

template <int N>
__device__ __forceinline__ bool decode_words(const uint64_t (&u)[N], uint32_t tag, Vec<N> &v) {
  bool ok = true;
#pragma unroll
  for (int i = 0; i < N; ++i) {
    ok = ok && ((uint32_t)(u[i] >> 32) == tag);
    v.f[i] = __uint_as_float((uint32_t)u[i]);
  }
  return ok;
}

template <int N>
__device__ __forceinline__ bool read_words(const uint64_t *w, uint32_t tag, Vec<N> &v) {
  bool ok = true;
#pragma unroll
  for (int i = 0; i < N; ++i) {
    uint64_t u = __hip_atomic_load(const_cast<uint64_t *>(w + i), __ATOMIC_RELAXED,
                                   __HIP_MEMORY_SCOPE_AGENT);
    ok = ok && ((uint32_t)(u >> 32) == tag);
    v.f[i] = __uint_as_float((uint32_t)u);
  }
  return ok;
}

// Per-launch control block at the start of every workspace:
//   [0] rows finished in this launch, [1] launch epoch, [2] error word: the
//       tag of the last launch whose look-back wait timed out (0 = none),
//   [3] unused.
// The error word names its launch, so only the waits of that same launch give
// up early on it; a later launch (new tag) waits normally.  The host reads
// and clears it with pcad_ws_status.
// Tiles are taken in dispatch order (blockIdx), so no per-tile counter is
// needed.  The tile that comes last in scan order in a row has, once its
// look-back is done, seen every tile of its row publish (each publish
// happens after that block read the epoch); it then arrives at [0], and the
// last row to arrive resets [0] and advances the epoch for the next launch.
// Only the control block needs zero-initialisation; everything else in a
// workspace is validated by epoch tags.
struct Ctl {
  unsigned rows_done, epoch, err, pad;
};

constexpr int kSpinLimit = 1 << 20;

// The tag of the launch after the one with epoch e.  Tags stay in
// [1, 2^31): a zeroed word never matches, and neither does workspace data
// whose 8-byte words have an upper half >= 2^31 (the records and tables of
// the partitioned reduce-by-index).
__device__ __forceinline__ uint32_t next_tag(uint32_t e) { return e >= 0x7fffffffu ? 1u : e + 1u; }

__device__ __forceinline__ unsigned ctl_load(unsigned *p) {
  return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

__device__ __forceinline__ void ctl_error(Ctl *ctl, uint32_t tag) {
  __hip_atomic_store(&ctl->err, tag, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// whether a wait of the launch with this tag has already timed out
__device__ __forceinline__ bool ctl_failed(Ctl *ctl, uint32_t tag) {
  return __hip_atomic_load(&ctl->err, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) == tag;
}

// called once per row, by the row's last tile in scan order, after its
// look-back (or immediately for a single-tile row)
__device__ __forceinline__ void ctl_row_done(Ctl *ctl, unsigned nrows, uint32_t tag) {
  const unsigned d =
      __hip_atomic_fetch_add(&ctl->rows_done, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  if (d == nrows - 1) {
    __hip_atomic_store(&ctl->rows_done, 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    __hip_atomic_store(&ctl->epoch, tag, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  }
}

// predecessors polled per lane and round trip, by status-word count
template <int NW>
constexpr int lookback_q() {
  return NW <= 4 ? 4 : (NW <= 8 ? 2 : 1);
}

// Decoupled look-back, run by one whole wave.  The tile's predecessors in
// scan order sit at distances 1..dist_max; the predecessor at distance d has
// status index `tile - dir*d`.  Status block of tile t: NA aggregate words
// then NP prefix words at st + t*(NA+NP).  Lane L polls distances
// base + L*Q + 1 .. base + L*Q + Q, so one round trip covers 64*Q tiles.
// Returns (in every lane) the combination of all predecessors, earliest
// first, built from the nearest published inclusive prefix and the
// aggregates after it.  When no inclusive prefix lies within dist_max, the
// result is the combination of the dist_max aggregates and *hit (if given)
// is set false; the caller then supplies the prefix before the window.
// Every wait is bounded: after kSpinLimit polls, or as soon as any block of
// the same launch has flagged a timeout, the wave stops waiting (the result
// is then garbage and the error word tells the host).
template <class Tr>
__device__ typename Tr::T lookback(const uint64_t *st, int64_t tile, int dir, int dist_max,
                                   uint32_t tag, Ctl *ctl, bool *hit = nullptr) {
  using T = typename Tr::T;
  using P = typename Tr::P;
  constexpr int NA = Tr::NA, NP = Tr::NP, NW = NA + NP;
  constexpr int Q = lookback_q<NW>();
  const int lane = lane_id();
  T acc = Tr::id();
  bool have = false;
  for (int base = 0; base < dist_max; base += WAVE * Q) {
    T agg[Q];
    P pre[Q];
    int state[Q];  // 3: out of range, 2: prefix, 1: aggregate, 0: not yet
#pragma unroll
    for (int q = 0; q < Q; ++q) {
      agg[q] = Tr::id();
      state[q] = (base + lane * Q + q + 1 <= dist_max) ? 0 : 3;
    }
    int plane = WAVE, pq = Q;
    for (int spin = 0;; ++spin) {
      // one round trip per poll: every status word of every pending
      // position is requested before any of them is examined
      uint64_t wp[Q][NP], wa[Q][NA];
#pragma unroll
      for (int q = 0; q < Q; ++q) {
        if (state[q] < 2) {
          const uint64_t *w = st + (tile - (int64_t)dir * (base + lane * Q + q + 1)) * NW;
#pragma unroll
          for (int i = 0; i < NP; ++i) wp[q][i] = load_word(w + NA + i);
#pragma unroll
          for (int i = 0; i < NA; ++i) wa[q][i] = load_word(w + i);
        }
      }
#pragma unroll
      for (int q = 0; q < Q; ++q) {
        if (state[q] < 2) {
          if (decode_words<NP>(wp[q], tag, pre[q])) state[q] = 2;
          else if (decode_words<NA>(wa[q], tag, agg[q])) state[q] = 1;
        }
      }
      int myq = Q;
#pragma unroll
      for (int q = Q - 1; q >= 0; --q)
        if (state[q] == 2) myq = q;
      const uint64_t pm = __ballot(myq < Q);
      plane = pm ? (__ffsll((long long)pm) - 1) : WAVE;
      pq = plane < WAVE ? __shfl(myq, plane, WAVE) : Q;
      bool missing = false;
#pragma unroll
      for (int q = 0; q < Q; ++q) {
        const bool need = lane < plane || (lane == plane && q < pq);
        missing = missing || (need && state[q] == 0);
      }
      if (__ballot(missing) == 0) break;
      if ((spin & 255) == 255) {
        if (spin >= kSpinLimit) {
          ctl_error(ctl, tag);
          break;
        }
        if (ctl_failed(ctl, tag)) break;
      }
      __builtin_amdgcn_s_sleep(1);
    }
    // fold this lane's positions, farthest (earliest) first
    T v = Tr::id();
    if (lane <= plane) {
      const int top = (lane == plane) ? pq : Q - 1;
      bool started = false;
#pragma unroll
      for (int q = Q - 1; q >= 0; --q) {
        if (q > top) continue;
        const T x = (lane == plane && q == pq) ? Tr::from_pre(pre[q])
                                              : (state[q] == 1 ? agg[q] : Tr::id());
        v = started ? Tr::comb(v, x) : x;
        started = true;
      }
    }
    const T win = readlane(wave_reduce_desc<Tr>(v), 0);
    acc = have ? Tr::comb(win, acc) : win;
    have = true;
    if (plane < WAVE) {
      if (hit) *hit = true;
      return acc;
    }
  }
  if (hit) *hit = false;
  return acc;
}

}  // namespace pcad
