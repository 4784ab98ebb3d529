// Scan-adjoint algebra.
//
// The adjoint of an inclusive scan is the backward linear recurrence
//   lam_i = ybar_i + J_i^T lam_{i+1},   J_i = d(rs_i (.) x_{i+1}) / d rs_i
// (Section 5.1, end of the derivation).  We carry, instead of lam, the
// contribution handed to the left neighbour, rho_i = J_{i-1}^T lam_i, which
// depends only on position i (its prefix rs_{i-1}, element x_i and ybar_i):
//   rho_i = h_i(rho_{i+1}) with h_i(r) = J_{i-1}^T (ybar_i + r),
//   lam_i = ybar_i + rho_{i+1},
//   xbar_i = (d(rs_{i-1} (.) x_i) / d x_i)^T lam_i      (x_bar_0 = lam_0).
// The h_i are affine maps r -> o + W r; composing them is the
// linear-function-composition scan of the paper's rule figure, run right to
// left.  Jacobians with redundant block-diagonal structure (Section 5.3,
// RBDS) keep W small: a scalar for * min max and the linear recurrence,
// one 2x2 block for the 2x2 matrix product.
//
// Trait interface (all __device__):
//   T            map type (Vec<N>), P the vector type rho lives in
//   id()         identity map;  comb(earlier, later) = later o earlier,
//                "earlier" meaning further right (applied first)
//   from_pre(p)  the constant map r -> p;  apply0(t) = t(0)
//   NA, NP       status words of an aggregate map / of a vector
#pragma once

#include "device.hpp"

namespace pcad {

// traits of a forward operator as a look-back payload (prefix = element)
template <int OP>
struct FwdLB : Fwd<OP> {
  using T = typename Fwd<OP>::T;
  using P = T;
  static constexpr int NA = Fwd<OP>::N;
  static constexpr int NP = Fwd<OP>::N;
  __device__ static T from_pre(const P &p) { return p; }
  __device__ static P to_pre(const T &t) { return t; }
};

// + : W = 1, the map is r -> o + r
struct MapAdd {
  using T = Vec<1>;
  using P = Vec<1>;
  static constexpr int NA = 1, NP = 1;
  __device__ static T id() { return {{0.0f}}; }
  __device__ static T comb(const T &e, const T &l) { return {{l.f[0] + e.f[0]}}; }
  __device__ static T from_pre(const P &p) { return p; }
  __device__ static P apply0(const T &t) { return t; }
};

// scalar affine map (o, W): * min max and the linear recurrence without an
// adjoint of the cumulative product.  Strong zeros keep an exact 0 in W from
// meeting an overflowed partial (inf) as NaN.
// STRONG: products with an exact zero factor are exact zeros (the `*` and
// min/max selectors, whose adjoints may meet an overflowed partial product);
// the linear recurrence uses plain fused multiply-adds
template <bool STRONG>
struct MapScalT {
  using T = Vec<2>;  // o, W
  using P = Vec<1>;
  static constexpr int NA = 2, NP = 1;
  __device__ static T id() { return {{0.0f, 1.0f}}; }
  __device__ static T comb(const T &e, const T &l) {
    if (STRONG) return {{l.f[0] + mulz(l.f[1], e.f[0]), mulz(l.f[1], e.f[1])}};
    return {{__builtin_fmaf(l.f[1], e.f[0], l.f[0]), l.f[1] * e.f[1]}};
  }
  __device__ static T from_pre(const P &p) { return {{p.f[0], 0.0f}}; }
  __device__ static P apply0(const T &t) { return {{t.f[0]}}; }
};
using MapScal = MapScalT<true>;

// linear recurrence with an adjoint of the cumulative product: rho is the
// pair (rho_y, rho_A) and J_{i-1} = diag(a_i, a_i) (RBDS, q = 1, k = 2)
struct MapLin2 {
  using T = Vec<3>;  // o_y, o_A, W
  using P = Vec<2>;
  static constexpr int NA = 3, NP = 2;
  __device__ static T id() { return {{0.0f, 0.0f, 1.0f}}; }
  __device__ static T comb(const T &e, const T &l) {
    return {{__builtin_fmaf(l.f[2], e.f[0], l.f[0]), __builtin_fmaf(l.f[2], e.f[1], l.f[1]),
             l.f[2] * e.f[2]}};
  }
  __device__ static T from_pre(const P &p) { return {{p.f[0], p.f[1], 0.0f}}; }
  __device__ static P apply0(const T &t) { return {{t.f[0], t.f[1]}}; }
};

// 2x2 matrix product: rho is a 2x2 matrix and J_{i-1}^T acts as right
// multiplication by M_i^T (RBDS, q = 2, k = 2): r -> o + r W
struct MapMat {
  using T = Vec<8>;  // o[4], W[4], row-major
  using P = Vec<4>;
  static constexpr int NA = 8, NP = 4;
  __device__ static T id() { return {{0, 0, 0, 0, 1, 0, 0, 1}}; }
  // X (2x2) times Y (2x2), both row-major, from arrays
  __device__ static void mm(const float *x, const float *y, float *r) {
    r[0] = __builtin_fmaf(x[0], y[0], x[1] * y[2]);
    r[1] = __builtin_fmaf(x[0], y[1], x[1] * y[3]);
    r[2] = __builtin_fmaf(x[2], y[0], x[3] * y[2]);
    r[3] = __builtin_fmaf(x[2], y[1], x[3] * y[3]);
  }
  __device__ static T comb(const T &e, const T &l) {
    T r;
    float t[4];
    mm(e.f, l.f + 4, t);  // e.o * l.W
    r.f[0] = l.f[0] + t[0];
    r.f[1] = l.f[1] + t[1];
    r.f[2] = l.f[2] + t[2];
    r.f[3] = l.f[3] + t[3];
    mm(e.f + 4, l.f + 4, r.f + 4);  // e.W * l.W
    return r;
  }
  __device__ static T from_pre(const P &p) { return {{p.f[0], p.f[1], p.f[2], p.f[3], 0, 0, 0, 0}}; }
  __device__ static P apply0(const T &t) { return {{t.f[0], t.f[1], t.f[2], t.f[3]}}; }
};

// sumOfProd scans: rho is the pair (rho_p, rho_s) and J_{i-1}^T =
// [[1, 0], [a_i, 1]] acts on it; composed maps stay lower triangular,
// r -> o + W r with W = [[w0, 0], [w1, w2]] (constant maps have W = 0)
struct MapSP {
  using T = Vec<5>;  // o_p, o_s, w0, w1, w2
  using P = Vec<2>;
  static constexpr int NA = 5, NP = 2;
  __device__ static T id() { return {{0.0f, 0.0f, 1.0f, 0.0f, 1.0f}}; }
  __device__ static T comb(const T &e, const T &l) {
    // l o e: o = l.o + W_l e.o, W = W_l W_e
    return {{__builtin_fmaf(l.f[2], e.f[0], l.f[0]),
             __builtin_fmaf(l.f[3], e.f[0], __builtin_fmaf(l.f[4], e.f[1], l.f[1])),
             l.f[2] * e.f[2],
             __builtin_fmaf(l.f[3], e.f[2], l.f[4] * e.f[3]),
             l.f[4] * e.f[4]}};
  }
  __device__ static T from_pre(const P &p) { return {{p.f[0], p.f[1], 0.0f, 0.0f, 0.0f}}; }
  __device__ static P apply0(const T &t) { return {{t.f[0], t.f[1]}}; }
};

// ---------------------------------------------------------------------------
// Per-operator local rules.  `p` is rs_{i-1} (the forward exclusive prefix,
// the neutral element at a row start), `first` marks the row's first
// element, ybar holds the output adjoint of position i.
//   make(...)  the map h_i;   step(...) lam_i, xbar_i and rho_i from rho_{i+1}.
// ---------------------------------------------------------------------------
template <int OP, bool ABAR>
struct Adj;

template <bool ABAR>
struct Adj<ADD, ABAR> {
  using M = MapAdd;
  using FT = Fwd<ADD>::T;
  static constexpr bool NEEDS_PREFIX = false;
  static constexpr int NY = 1;   // adjoint floats per element
  static constexpr int NXB = 1;  // input-adjoint floats per element
  __device__ static M::T make(const FT &, const FT &, const float *yb, bool) { return {{yb[0]}}; }
  __device__ static void step(const FT &, const FT &, const float *yb, bool, M::P &rho,
                              float *xb) {
    const float lam = yb[0] + rho.f[0];
    xb[0] = lam;
    rho.f[0] = lam;
  }
};

template <bool ABAR>
struct Adj<MUL, ABAR> {
  using M = MapScal;
  using FT = Fwd<MUL>::T;
  static constexpr bool NEEDS_PREFIX = true;
  static constexpr int NY = 1, NXB = 1;
  // J_{i-1} = x_i, d/dx_i = rs_{i-1}; an exact zero prefix gives an exact 0
  __device__ static M::T make(const FT &, const FT &x, const float *yb, bool) {
    return {{mulz(x.f[0], yb[0]), x.f[0]}};
  }
  __device__ static void step(const FT &p, const FT &x, const float *yb, bool, M::P &rho,
                              float *xb) {
    const float lam = yb[0] + rho.f[0];
    xb[0] = mulz(p.f[0], lam);
    rho.f[0] = mulz(x.f[0], lam);
  }
};

// min/max: the accumulator is kept on a tie, so J_{i-1} = [rs_{i-1} <= x_i]
// (>= for max) and the element's partial is the complement; the row's first
// element always takes its own adjoint.
template <int OP, bool ABAR>
struct AdjMinMax {
  using M = MapScal;
  using FT = typename Fwd<OP>::T;
  static constexpr bool NEEDS_PREFIX = true;
  static constexpr int NY = 1, NXB = 1;
  __device__ static bool kept(const FT &p, const FT &x, bool first) {
    if (first) return false;
    return OP == MIN ? (p.f[0] <= x.f[0]) : (p.f[0] >= x.f[0]);
  }
  __device__ static typename M::T make(const FT &p, const FT &x, const float *yb, bool first) {
    const bool k = kept(p, x, first);
    return {{k ? yb[0] : 0.0f, k ? 1.0f : 0.0f}};
  }
  __device__ static void step(const FT &p, const FT &x, const float *yb, bool first,
                              typename M::P &rho, float *xb) {
    const float lam = yb[0] + rho.f[0];
    const bool k = kept(p, x, first);
    xb[0] = k ? 0.0f : lam;
    rho.f[0] = k ? lam : 0.0f;
  }
};
template <bool ABAR>
struct Adj<MIN, ABAR> : AdjMinMax<MIN, ABAR> {};
template <bool ABAR>
struct Adj<MAX, ABAR> : AdjMinMax<MAX, ABAR> {};

// saturated addition: both partials of rs_{i-1} (.) x_i are [rs_{i-1} + x_i
// <= cap] (0 on a saturated step), the same sum and test the forward made;
// the row's first element takes its own adjoint
template <bool ABAR>
struct Adj<SATADD, ABAR> {
  using M = MapScal;
  using FT = Fwd<SATADD>::T;
  static constexpr bool NEEDS_PREFIX = true;
  static constexpr int NY = 1, NXB = 1;
  __device__ static bool pass(const FT &p, const FT &x, bool first) {
    return first || !(p.f[0] + x.f[0] > kSatCap);
  }
  __device__ static M::T make(const FT &p, const FT &x, const float *yb, bool first) {
    const bool k = !first && pass(p, x, false);
    return {{k ? yb[0] : 0.0f, k ? 1.0f : 0.0f}};
  }
  __device__ static void step(const FT &p, const FT &x, const float *yb, bool first, M::P &rho,
                              float *xb) {
    const float lam = yb[0] + rho.f[0];
    const bool k = pass(p, x, first);
    xb[0] = k ? lam : 0.0f;
    rho.f[0] = (!first && k) ? lam : 0.0f;
  }
};

// sumOfProd scans: element x = (0, a_i), prefix p = (P_{i-1}, S_{i-1}); the
// output adjoint is (ybar_i, 0):
//   lam = ybar + rho,  a_bar = S_{i-1} lam_p + lam_s,  rho = (lam_p, a lam_p + lam_s)
template <bool ABAR>
struct Adj<SUMPROD, ABAR> {
  using M = MapSP;
  using FT = Fwd<SUMPROD>::T;
  static constexpr bool NEEDS_PREFIX = true;
  static constexpr int NY = 1, NXB = 1;
  __device__ static M::T make(const FT &, const FT &x, const float *yb, bool) {
    const float a = x.f[1];
    return {{yb[0], a * yb[0], 1.0f, a, 1.0f}};
  }
  __device__ static void step(const FT &p, const FT &x, const float *yb, bool, M::P &rho,
                              float *xb) {
    const float lp = yb[0] + rho.f[0], ls = rho.f[1];
    xb[0] = __builtin_fmaf(p.f[1], lp, ls);
    rho.f[0] = lp;
    rho.f[1] = __builtin_fmaf(x.f[1], lp, ls);
  }
};

// linear recurrence, element x = (a, b), prefix p = (A_{i-1}, y_{i-1});
// adjoint inputs (ybar_i[, Abar_i]); outputs (a_bar_i, b_bar_i):
//   b_bar = lam_y,  a_bar = lam_y*y_{i-1} + lam_A*A_{i-1},  rho = a*lam
template <>
struct Adj<LINREC, false> {
  using M = MapScalT<false>;
  using FT = Fwd<LINREC>::T;
  static constexpr bool NEEDS_PREFIX = true;
  static constexpr int NY = 1, NXB = 2;
  __device__ static M::T make(const FT &, const FT &x, const float *yb, bool) {
    return {{x.f[0] * yb[0], x.f[0]}};
  }
  __device__ static void step(const FT &p, const FT &x, const float *yb, bool, M::P &rho,
                              float *xb) {
    const float lam = yb[0] + rho.f[0];
    xb[0] = lam * p.f[1];
    xb[1] = lam;
    rho.f[0] = x.f[0] * lam;
  }
};

template <>
struct Adj<LINREC, true> {
  using M = MapLin2;
  using FT = Fwd<LINREC>::T;
  static constexpr bool NEEDS_PREFIX = true;
  static constexpr int NY = 2, NXB = 2;
  __device__ static M::T make(const FT &, const FT &x, const float *yb, bool) {
    return {{x.f[0] * yb[0], x.f[0] * yb[1], x.f[0]}};
  }
  __device__ static void step(const FT &p, const FT &x, const float *yb, bool, M::P &rho,
                              float *xb) {
    const float ly = yb[0] + rho.f[0];
    const float la = yb[1] + rho.f[1];
    xb[0] = __builtin_fmaf(ly, p.f[1], la * p.f[0]);
    xb[1] = ly;
    rho.f[0] = x.f[0] * ly;
    rho.f[1] = x.f[0] * la;
  }
};

// 2x2 matrix product P_i = P_{i-1} M_i:
//   lam = Pbar_i + rho,  Mbar_i = P_{i-1}^T lam,  rho_i = lam M_i^T
template <bool ABAR>
struct Adj<MAT2, ABAR> {
  using M = MapMat;
  using FT = Fwd<MAT2>::T;
  static constexpr bool NEEDS_PREFIX = true;
  static constexpr int NY = 4, NXB = 4;
  __device__ static void transpose(const float *m, float *t) {
    t[0] = m[0]; t[1] = m[2]; t[2] = m[1]; t[3] = m[3];
  }
  __device__ static M::T make(const FT &, const FT &x, const float *yb, bool) {
    M::T h;
    float mt[4];
    transpose(x.f, mt);
    MapMat::mm(yb, mt, h.f);
    h.f[4] = mt[0]; h.f[5] = mt[1]; h.f[6] = mt[2]; h.f[7] = mt[3];
    return h;
  }
  __device__ static void step(const FT &p, const FT &x, const float *yb, bool, M::P &rho,
                              float *xb) {
    float lam[4], pt[4], mt[4];
    for (int i = 0; i < 4; ++i) lam[i] = yb[i] + rho.f[i];
    transpose(p.f, pt);
    MapMat::mm(pt, lam, xb);
    transpose(x.f, mt);
    MapMat::mm(lam, mt, rho.f);
  }
};

}  // namespace pcad
