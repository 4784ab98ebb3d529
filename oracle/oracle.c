/*
 * Plain CPU oracle for reduce, inclusive scan and reduce-by-index, and their
 * reverse-mode adjoints (vector-Jacobian products).  TEST INFRASTRUCTURE ONLY:
 * only the test-suite, the smoke check and the CPU-baseline leg of the
 * benchmark may load this file.  It shares no code, header or table with the
 * GPU library.
 *
 * Precision: float64 throughout, single-threaded, no blocking, no
 * reassociation.  Inputs are the float32 arrays the GPU consumes, widened
 * exactly to float64 by the caller.
 *
 * Element types (d = number of float components per element):
 *   ADD, MUL, MIN, MAX : d = 1, a scalar.
 *   LINREC             : d = 2, (multiplier, offset).  The operator is
 *                        linear-function composition (Section 6.1, operator
 *                        figure): (A1,B1) (.) (a2,b2) = (A1*a2, a2*B1 + b2),
 *                        neutral (1,0).  A scan of (a_i,b_i) therefore yields
 *                        (A_i, y_i) with y_i = a_i*y_{i-1} + b_i, y_{-1}=0, and
 *                        A_i = a_0*...*a_i.
 *   MAT2               : d = 4, a row-major 2x2 matrix (a,b,c,d) =
 *                        [[a,b],[c,d]]; the operator is the matrix product
 *                        P (.) M = P x M (Section 6.1, operator figure),
 *                        neutral I.
 *   SATADD             : d = 1, saturated addition (the evaluation's operator
 *                        figure): acc (.) x = C if acc + x > C, else acc + x,
 *                        with C = 1e6 and neutral 0; its partials are 0 where
 *                        the sum saturates and 1 elsewhere.  Associative and
 *                        commutative on values in [0, C]; the derivative of a
 *                        fold depends on the bracketing where a bracket lands
 *                        exactly on C (a kink: a zero prefix meeting a
 *                        saturated suffix, or a partial sum equal to C), and
 *                        this oracle takes the sequential loop's.
 *   SUMPROD            : d = 2, the lifted pair (p, s) of the invertible
 *                        operator sumOfProd (Section 3.3):
 *                        (p1,s1) (.) (p2,s2) = (p1 + p2 + s1*s2, s1 + s2),
 *                        neutral (0,0).  A scalar input a enters as (0, a)
 *                        and the result is the p component, so a fold gives
 *                        p = sum over i<j of a_i*a_j and s = sum of a_i.
 *
 * Forward results are the plain definitions:
 *   reduce : the left fold x_0 (.) x_1 (.) ... (.) x_{n-1} (Section 3.1);
 *   scan   : rs_0 = x_0, rs_i = rs_{i-1} (.) x_i (Section 5.1, the
 *            sequential loop);
 *   RBI    : the sequential loop over i ascending that skips keys outside
 *            [0,m) and otherwise folds hist[k] = hist[k] (.) v_i, starting from
 *            the neutral element (Section 4, sequential semantics, and the
 *            rewrite to a neutral initial histogram).
 *
 * Adjoints are x_bar = J^T y_bar of those forward programs (Section 2.2,
 * the vjp interface, with the notation caveat that the product is really
 * y_bar * J).  They are computed by the hand-written reverse sweep of the
 * sequential loop (Section 5.1: unroll, apply the core rewrite rule of
 * Eq. (1) to each statement, roll back into a loop):
 *     lam = copy y_bar
 *     for i = n-1 .. 1:  x_bar[i]  = (d out/d x)^T   lam[i]
 *                        lam[i-1] += (d out/d acc)^T lam[i]
 *     x_bar[0] = lam[0]
 * where out = rs[i-1] (.) x[i].  The per-operator local partials are the
 * derivatives of the operator definitions; min/max keep the accumulator on a
 * tie, so the lowest index wins (Section 3.2, Min/Max, and Section 4.2).
 * Multiplication uses the plain partials (no division), so zeros are exact.
 *
 * Every floating output r also gets a companion c >= |r|: the same
 * multilinear expression evaluated on absolute values (|inputs|, |adjoints|,
 * |partials|), with the discrete decisions (which element wins a min/max)
 * taken from the real run.  This is the quantity of the standard forward
 * error bound |fl(r) - r| <= gamma_k * c.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

enum { OP_ADD = 0, OP_MUL = 1, OP_MIN = 2, OP_MAX = 3, OP_LINREC = 4, OP_MAT2 = 5, OP_SUMPROD = 6,
       OP_SATADD = 7 };

static const double SAT_CAP = 1e6;

int orc_dim(int op) { return (op == OP_LINREC || op == OP_SUMPROD) ? 2 : (op == OP_MAT2 ? 4 : 1); }

static int valid_op(int op) { return op >= OP_ADD && op <= OP_SATADD; }

/* neutral element e of the operator */
static void neutral(int op, double *e) {
  switch (op) {
  case OP_ADD: e[0] = 0.0; break;
  case OP_MUL: e[0] = 1.0; break;
  case OP_MIN: e[0] = INFINITY; break;
  case OP_MAX: e[0] = -INFINITY; break;
  case OP_LINREC: e[0] = 1.0; e[1] = 0.0; break;
  case OP_MAT2: e[0] = 1.0; e[1] = 0.0; e[2] = 0.0; e[3] = 1.0; break;
  case OP_SUMPROD: e[0] = 0.0; e[1] = 0.0; break;
  case OP_SATADD: e[0] = 0.0; break;
  }
}

/* out = acc (.) x.  For min/max the accumulator is kept on a tie. */
static void combine(int op, const double *acc, const double *x, double *out) {
  double t[4];
  switch (op) {
  case OP_ADD: out[0] = acc[0] + x[0]; break;
  case OP_MUL: out[0] = acc[0] * x[0]; break;
  case OP_MIN: out[0] = (acc[0] <= x[0]) ? acc[0] : x[0]; break;
  case OP_MAX: out[0] = (acc[0] >= x[0]) ? acc[0] : x[0]; break;
  case OP_LINREC:
    t[0] = acc[0] * x[0];
    t[1] = x[0] * acc[1] + x[1];
    out[0] = t[0]; out[1] = t[1];
    break;
  case OP_SATADD: out[0] = (acc[0] + x[0] > SAT_CAP) ? SAT_CAP : acc[0] + x[0]; break;
  case OP_SUMPROD:
    t[0] = acc[0] + x[0] + acc[1] * x[1];
    t[1] = acc[1] + x[1];
    out[0] = t[0]; out[1] = t[1];
    break;
  case OP_MAT2:
    t[0] = acc[0] * x[0] + acc[1] * x[2];
    t[1] = acc[0] * x[1] + acc[1] * x[3];
    t[2] = acc[2] * x[0] + acc[3] * x[2];
    t[3] = acc[2] * x[1] + acc[3] * x[3];
    memcpy(out, t, sizeof t);
    break;
  }
}

/* Companion of the combine: the same multilinear form on absolute values.
 * For min/max the companion is the absolute value of the selected operand. */
static void combine_abs(int op, const double *cacc, const double *cx,
                        const double *acc, const double *x, double *out) {
  switch (op) {
  case OP_MIN: out[0] = (acc[0] <= x[0]) ? cacc[0] : cx[0]; break;
  case OP_MAX: out[0] = (acc[0] >= x[0]) ? cacc[0] : cx[0]; break;
  case OP_MAT2: out[0] = out[1] = out[2] = out[3] = cacc[0] * cx[0]; break;
  case OP_SATADD: out[0] = (acc[0] + x[0] > SAT_CAP) ? SAT_CAP : cacc[0] + cx[0]; break;
  default: combine(op, cacc, cx, out); break;
  }
}

/*
 * Local partials of out = acc (.) x, as d x d matrices in row-major order,
 * row = output component, column = input component:
 *   JA[r][c] = d out_r / d acc_c,   JX[r][c] = d out_r / d x_c.
 */
static void partials(int op, const double *acc, const double *x, double *JA, double *JX) {
  int kept;
  switch (op) {
  case OP_ADD: JA[0] = 1.0; JX[0] = 1.0; break;
  case OP_MUL: JA[0] = x[0]; JX[0] = acc[0]; break;
  case OP_MIN:
    kept = acc[0] <= x[0];
    JA[0] = kept ? 1.0 : 0.0; JX[0] = kept ? 0.0 : 1.0;
    break;
  case OP_MAX:
    kept = acc[0] >= x[0];
    JA[0] = kept ? 1.0 : 0.0; JX[0] = kept ? 0.0 : 1.0;
    break;
  case OP_LINREC:
    /* out0 = A*a, out1 = a*B + b with acc = (A,B), x = (a,b) */
    JA[0] = x[0]; JA[1] = 0.0;
    JA[2] = 0.0;  JA[3] = x[0];
    JX[0] = acc[0]; JX[1] = 0.0;
    JX[2] = acc[1]; JX[3] = 1.0;
    break;
  case OP_SATADD:
    /* the saturated branch is a constant */
    JA[0] = JX[0] = (acc[0] + x[0] > SAT_CAP) ? 0.0 : 1.0;
    break;
  case OP_SUMPROD:
    /* out0 = P + p + S*s, out1 = S + s with acc = (P,S), x = (p,s) */
    JA[0] = 1.0; JA[1] = x[1];
    JA[2] = 0.0; JA[3] = 1.0;
    JX[0] = 1.0; JX[1] = acc[1];
    JX[2] = 0.0; JX[3] = 1.0;
    break;
  case OP_MAT2: {
    /* out[i][j] = sum_k P[i][k] M[k][j]; flat index 2*row + col */
    int i, j, p, q;
    for (i = 0; i < 16; ++i) { JA[i] = 0.0; JX[i] = 0.0; }
    for (i = 0; i < 2; ++i)
      for (j = 0; j < 2; ++j) {
        int r = 2 * i + j;
        for (p = 0; p < 2; ++p) { /* d out[i][j] / d P[i][p] = M[p][j] */
          JA[r * 4 + (2 * i + p)] = x[2 * p + j];
        }
        for (q = 0; q < 2; ++q) { /* d out[i][j] / d M[q][j] = P[i][q] */
          JX[r * 4 + (2 * q + j)] = acc[2 * i + q];
        }
      }
    break;
  }
  }
}

/* Companion partials: the same local derivatives evaluated on the companions
 * of the operands (|x| for inputs, the companion of the accumulator for
 * computed prefixes).  For min/max the 0/1 decision of the real run is used. */
static void partials_abs(int op, const double *acc, const double *x, const double *cacc,
                         const double *ax, double *JA, double *JX) {
  if (op == OP_MIN || op == OP_MAX || op == OP_SATADD) partials(op, acc, x, JA, JX);
  else partials(op, cacc, ax, JA, JX);
}

/* Companions of the 2x2 matrix product are norm-wise: every entry of a
 * product chain is bounded by the product of the factors' spectral norms,
 * and the rounding error of any bracketing by a small multiple of u times
 * that product.  (The entrywise |M_0||M_1|...|M_i| bound grows with the
 * spectral radius of |M| >= 1 even when the product is orthogonal, which
 * would make it useless for long chains.)  A MAT2 companion is stored as the
 * same scalar in all four entries. */
static double spec2(const double *m) {
  double f = m[0] * m[0] + m[1] * m[1] + m[2] * m[2] + m[3] * m[3];
  double det = m[0] * m[3] - m[1] * m[2];
  double disc = f * f - 4.0 * det * det;
  if (disc < 0.0) disc = 0.0;
  return sqrt(0.5 * (f + sqrt(disc)));
}

static double frob(const double *m) {
  return sqrt(m[0] * m[0] + m[1] * m[1] + m[2] * m[2] + m[3] * m[3]);
}

/* companion of one input element: |x|, or ||M||_2 broadcast for MAT2 */
static void elem_abs(int op, const double *x, double *ax) {
  if (op == OP_MAT2) {
    double s = spec2(x);
    ax[0] = ax[1] = ax[2] = ax[3] = s;
  } else {
    for (int t = 0; t < orc_dim(op); ++t) ax[t] = fabs(x[t]);
  }
}

/* companion of an output adjoint: |ybar|, or ||Ybar||_F broadcast for MAT2 */
static void adj_abs(int op, const double *y, double *ay) {
  if (op == OP_MAT2) {
    double s = frob(y);
    ay[0] = ay[1] = ay[2] = ay[3] = s;
  } else {
    for (int t = 0; t < orc_dim(op); ++t) ay[t] = fabs(y[t]);
  }
}

/* y += J^T v for a d x d matrix J */
static void add_JTv(int d, const double *J, const double *v, double *y) {
  for (int c = 0; c < d; ++c) {
    double s = 0.0;
    for (int r = 0; r < d; ++r) s += J[r * d + c] * v[r];
    y[c] += s;
  }
}

static void add_absJTv(int d, const double *J, const double *v, double *y) {
  for (int c = 0; c < d; ++c) {
    double s = 0.0;
    for (int r = 0; r < d; ++r) s += fabs(J[r * d + c]) * v[r];
    y[c] += s;
  }
}

/* companion of J^T v: entrywise |J|^T v, or for MAT2 the norm of the
 * linear map (the other factor's 2-norm) times the scalar companion v */
static void comp_JA(int op, const double *JA, const double *ax, const double *v, double *y) {
  if (op == OP_MAT2) {
    double t = ax[0] * v[0];
    y[0] += t; y[1] += t; y[2] += t; y[3] += t;
  } else {
    add_absJTv(orc_dim(op), JA, v, y);
  }
}

static void comp_JX(int op, const double *JX, const double *cacc, const double *v, double *y) {
  if (op == OP_MAT2) {
    double t = cacc[0] * v[0];
    y[0] += t; y[1] += t; y[2] += t; y[3] += t;
  } else {
    add_absJTv(orc_dim(op), JX, v, y);
  }
}

/* ------------------------------------------------------------------------ */
/* scan                                                                      */
/* ------------------------------------------------------------------------ */

/* Inclusive scan rs_0 = x_0, rs_i = rs_{i-1} (.) x_i.  c (may be NULL)
 * receives the companion.  Returns 0 on success. */
int orc_scan_fwd(int op, int64_t n, const double *x, double *rs, double *c) {
  if (!valid_op(op) || n < 0) return 1;
  const int d = orc_dim(op);
  for (int64_t i = 0; i < n; ++i) {
    if (i == 0) {
      memcpy(rs, x, sizeof(double) * d);
      if (c) elem_abs(op, x, c);
      continue;
    }
    double ax[4];
    elem_abs(op, x + i * d, ax);
    if (c) combine_abs(op, c + (i - 1) * d, ax, rs + (i - 1) * d, x + i * d, c + i * d);
    combine(op, rs + (i - 1) * d, x + i * d, rs + i * d);
  }
  return 0;
}

/* x_bar = J^T y_bar of the inclusive scan, by the reverse sweep of the
 * sequential loop.  cxbar (may be NULL) receives the companion, seeded with
 * cybar (non-negative, may be NULL to use |y_bar|).  Scratch is allocated
 * here (n*d*4 doubles). */
int orc_scan_vjp(int op, int64_t n, const double *x, const double *ybar, const double *cybar,
                 double *xbar, double *cxbar) {
  if (!valid_op(op) || n < 0) return 1;
  if (n == 0) return 0;
  const int d = orc_dim(op);
  double *rs = (double *)malloc(sizeof(double) * n * d);
  double *crs = (double *)malloc(sizeof(double) * n * d);
  double *lam = (double *)malloc(sizeof(double) * n * d);
  double *clam = (double *)malloc(sizeof(double) * n * d);
  if (!rs || !crs || !lam || !clam) { free(rs); free(crs); free(lam); free(clam); return 2; }
  orc_scan_fwd(op, n, x, rs, crs);
  for (int64_t i = 0; i < n * d; ++i) lam[i] = ybar[i];
  for (int64_t i = 0; i < n; ++i) {
    if (cybar) memcpy(clam + i * d, cybar + i * d, sizeof(double) * d);
    else adj_abs(op, ybar + i * d, clam + i * d);
  }
  double JA[16], JX[16], ax[4];
  for (int64_t i = n - 1; i >= 1; --i) {
    partials(op, rs + (i - 1) * d, x + i * d, JA, JX);
    for (int t = 0; t < d; ++t) xbar[i * d + t] = 0.0;
    add_JTv(d, JX, lam + i * d, xbar + i * d);
    add_JTv(d, JA, lam + i * d, lam + (i - 1) * d);
    elem_abs(op, x + i * d, ax);
    partials_abs(op, rs + (i - 1) * d, x + i * d, crs + (i - 1) * d, ax, JA, JX);
    if (cxbar) {
      for (int t = 0; t < d; ++t) cxbar[i * d + t] = 0.0;
      comp_JX(op, JX, crs + (i - 1) * d, clam + i * d, cxbar + i * d);
    }
    comp_JA(op, JA, ax, clam + i * d, clam + (i - 1) * d);
  }
  for (int t = 0; t < d; ++t) {
    xbar[t] = lam[t];
    if (cxbar) cxbar[t] = clam[t];
  }
  free(rs); free(crs); free(lam); free(clam);
  return 0;
}

/* ------------------------------------------------------------------------ */
/* reduce                                                                    */
/* ------------------------------------------------------------------------ */

/* Left fold.  For n = 0 the result is the neutral element.  Side outputs
 * (each may be NULL):
 *   k    : min/max -- smallest index attaining the extremum; n when empty.
 *   n0   : mul     -- number of exact zeros.
 *   ypos : mul     -- product of the non-zero elements (1 when none).
 * c (may be NULL) receives the companion of y. */
int orc_reduce_fwd(int op, int64_t n, const double *x, double *y, double *c, int64_t *k,
                   int64_t *n0, double *ypos) {
  if (!valid_op(op) || n < 0) return 1;
  const int d = orc_dim(op);
  double acc[4], cacc[4], nxt[4], cn[4], ax[4];
  int64_t win = n, zeros = 0;
  double prodnz = 1.0;
  neutral(op, acc);
  for (int t = 0; t < d; ++t) cacc[t] = fabs(acc[t]);
  for (int64_t i = 0; i < n; ++i) {
    const double *xi = x + i * d;
    if (op == OP_MUL) {
      if (xi[0] == 0.0) zeros++; else prodnz *= xi[0];
    }
    if (i == 0) {
      /* the first element always replaces the neutral (a real element beats
       * the sentinel of the lifted min/max) */
      memcpy(acc, xi, sizeof(double) * d);
      elem_abs(op, xi, cacc);
      win = 0;
      continue;
    }
    elem_abs(op, xi, ax);
    combine_abs(op, cacc, ax, acc, xi, cn);
    combine(op, acc, xi, nxt);
    if ((op == OP_MIN && xi[0] < acc[0]) || (op == OP_MAX && xi[0] > acc[0])) win = i;
    memcpy(acc, nxt, sizeof(double) * d);
    memcpy(cacc, cn, sizeof(double) * d);
  }
  memcpy(y, acc, sizeof(double) * d);
  if (c) memcpy(c, cacc, sizeof(double) * d);
  if (k) *k = (op == OP_MIN || op == OP_MAX) ? win : 0;
  if (n0) *n0 = zeros;
  if (ypos) *ypos = prodnz;
  return 0;
}

/* x_bar = J^T y_bar of the fold: the reverse sweep with an adjoint only on
 * the final accumulator. */
int orc_reduce_vjp(int op, int64_t n, const double *x, const double *ybar, double *xbar,
                   double *cxbar) {
  if (!valid_op(op) || n < 0) return 1;
  if (n == 0) return 0;
  const int d = orc_dim(op);
  double *rs = (double *)malloc(sizeof(double) * n * d);
  double *crs = (double *)malloc(sizeof(double) * n * d);
  if (!rs || !crs) { free(rs); free(crs); return 2; }
  orc_scan_fwd(op, n, x, rs, crs); /* the fold's intermediate accumulators */
  double lam[4], clam[4], nl[4], ncl[4], JA[16], JX[16], ax[4];
  for (int t = 0; t < d; ++t) lam[t] = ybar[t];
  adj_abs(op, ybar, clam);
  for (int64_t i = n - 1; i >= 1; --i) {
    partials(op, rs + (i - 1) * d, x + i * d, JA, JX);
    for (int t = 0; t < d; ++t) { xbar[i * d + t] = 0.0; nl[t] = 0.0; ncl[t] = 0.0; }
    add_JTv(d, JX, lam, xbar + i * d);
    add_JTv(d, JA, lam, nl);
    elem_abs(op, x + i * d, ax);
    partials_abs(op, rs + (i - 1) * d, x + i * d, crs + (i - 1) * d, ax, JA, JX);
    if (cxbar) {
      for (int t = 0; t < d; ++t) cxbar[i * d + t] = 0.0;
      comp_JX(op, JX, crs + (i - 1) * d, clam, cxbar + i * d);
    }
    comp_JA(op, JA, ax, clam, ncl);
    memcpy(lam, nl, sizeof lam);
    memcpy(clam, ncl, sizeof clam);
  }
  for (int t = 0; t < d; ++t) {
    xbar[t] = lam[t];
    if (cxbar) cxbar[t] = clam[t];
  }
  free(rs); free(crs);
  return 0;
}

/* ------------------------------------------------------------------------ */
/* reduce-by-index                                                           */
/* ------------------------------------------------------------------------ */

/* Sequential histogram.  Outputs (each may be NULL except hist):
 *   hist[m*d]  : per-bin fold, neutral when empty;
 *   chist[m*d] : companion;
 *   count[m]   : number of in-range elements per bin;
 *   argk[m]    : min/max -- smallest index attaining the bin's extremum,
 *                n for an empty bin;
 *   n0[m]      : number of exact zeros per bin (scalar ops);
 *   ypos[m]    : product of the non-zero elements per bin (1 when none). */
int orc_rbi_fwd(int op, int64_t n, int64_t m, const int32_t *idx, const double *v,
                double *hist, double *chist, int64_t *count, int64_t *argk, int64_t *n0,
                double *ypos) {
  if (!valid_op(op) || n < 0 || m < 0) return 1;
  const int d = orc_dim(op);
  int64_t *cnt = (int64_t *)calloc((size_t)(m > 0 ? m : 1), sizeof(int64_t));
  if (!cnt) return 2;
  double e[4];
  neutral(op, e);
  for (int64_t k = 0; k < m; ++k) {
    for (int t = 0; t < d; ++t) {
      hist[k * d + t] = e[t];
      if (chist) chist[k * d + t] = fabs(e[t]);
    }
    if (argk) argk[k] = n;
    if (n0) n0[k] = 0;
    if (ypos) ypos[k] = 1.0;
  }
  double nxt[4], cn[4], av[4];
  for (int64_t i = 0; i < n; ++i) {
    int64_t k = idx[i];
    if (k < 0 || k >= m) continue; /* out-of-bounds keys are ignored */
    const double *vi = v + i * d;
    if (op == OP_MUL) {
      if (n0 && vi[0] == 0.0) n0[k]++;
      if (ypos && vi[0] != 0.0) ypos[k] *= vi[0];
    }
    elem_abs(op, vi, av);
    if (cnt[k] == 0) {
      memcpy(hist + k * d, vi, sizeof(double) * d);
      if (chist) memcpy(chist + k * d, av, sizeof(double) * d);
      if (argk) argk[k] = i;
    } else {
      if (chist) {
        combine_abs(op, chist + k * d, av, hist + k * d, vi, cn);
        memcpy(chist + k * d, cn, sizeof(double) * d);
      }
      if (argk && ((op == OP_MIN && vi[0] < hist[k * d]) || (op == OP_MAX && vi[0] > hist[k * d])))
        argk[k] = i;
      combine(op, hist + k * d, vi, nxt);
      memcpy(hist + k * d, nxt, sizeof(double) * d);
    }
    cnt[k]++;
  }
  if (count) memcpy(count, cnt, sizeof(int64_t) * (size_t)m);
  free(cnt);
  return 0;
}

/* v_bar = J^T hist_bar of the sequential histogram: the reverse sweep of the
 * loop over i descending, one adjoint accumulator per bin.  Elements with an
 * out-of-range key get a zero adjoint. */
int orc_rbi_vjp(int op, int64_t n, int64_t m, const int32_t *idx, const double *v,
                const double *hbar, double *vbar, double *cvbar) {
  if (!valid_op(op) || n < 0 || m < 0) return 1;
  const int d = orc_dim(op);
  if (n == 0) return 0;
  double *before = (double *)malloc(sizeof(double) * n * d); /* bin state before element i */
  double *cbefore = (double *)malloc(sizeof(double) * n * d);
  double *cur = (double *)malloc(sizeof(double) * (size_t)(m > 0 ? m : 1) * d);
  double *ccur = (double *)malloc(sizeof(double) * (size_t)(m > 0 ? m : 1) * d);
  int64_t *cnt = (int64_t *)calloc((size_t)(m > 0 ? m : 1), sizeof(int64_t));
  unsigned char *first = (unsigned char *)calloc((size_t)n, 1);
  double *lam = (double *)malloc(sizeof(double) * (size_t)(m > 0 ? m : 1) * d);
  double *clam = (double *)malloc(sizeof(double) * (size_t)(m > 0 ? m : 1) * d);
  if (!before || !cbefore || !cur || !ccur || !cnt || !first || !lam || !clam) {
    free(before); free(cbefore); free(cur); free(ccur); free(cnt); free(first); free(lam);
    free(clam);
    return 2;
  }
  double av[4];
  /* primal re-execution, recording the bin state each element meets */
  for (int64_t i = 0; i < n; ++i) {
    int64_t k = idx[i];
    if (k < 0 || k >= m) continue;
    elem_abs(op, v + i * d, av);
    if (cnt[k] == 0) {
      first[i] = 1;
      memcpy(cur + k * d, v + i * d, sizeof(double) * d);
      memcpy(ccur + k * d, av, sizeof(double) * d);
    } else {
      memcpy(before + i * d, cur + k * d, sizeof(double) * d);
      memcpy(cbefore + i * d, ccur + k * d, sizeof(double) * d);
      double nxt[4], cn[4];
      combine_abs(op, ccur + k * d, av, cur + k * d, v + i * d, cn);
      combine(op, cur + k * d, v + i * d, nxt);
      memcpy(cur + k * d, nxt, sizeof(double) * d);
      memcpy(ccur + k * d, cn, sizeof(double) * d);
    }
    cnt[k]++;
  }
  for (int64_t k = 0; k < m * d; ++k) lam[k] = hbar[k];
  for (int64_t k = 0; k < m; ++k) adj_abs(op, hbar + k * d, clam + k * d);
  double JA[16], JX[16], nl[4], ncl[4];
  for (int64_t i = n - 1; i >= 0; --i) {
    int64_t k = idx[i];
    for (int t = 0; t < d; ++t) {
      vbar[i * d + t] = 0.0;
      if (cvbar) cvbar[i * d + t] = 0.0;
    }
    if (k < 0 || k >= m) continue;
    double *lk = lam + k * d, *clk = clam + k * d;
    if (first[i]) {
      for (int t = 0; t < d; ++t) {
        vbar[i * d + t] = lk[t];
        if (cvbar) cvbar[i * d + t] = clk[t];
      }
      continue;
    }
    partials(op, before + i * d, v + i * d, JA, JX);
    add_JTv(d, JX, lk, vbar + i * d);
    for (int t = 0; t < d; ++t) { nl[t] = 0.0; ncl[t] = 0.0; }
    add_JTv(d, JA, lk, nl);
    elem_abs(op, v + i * d, av);
    partials_abs(op, before + i * d, v + i * d, cbefore + i * d, av, JA, JX);
    if (cvbar) comp_JX(op, JX, cbefore + i * d, clk, cvbar + i * d);
    comp_JA(op, JA, av, clk, ncl);
    memcpy(lk, nl, sizeof(double) * d);
    memcpy(clk, ncl, sizeof(double) * d);
  }
  free(before); free(cbefore); free(cur); free(ccur); free(cnt); free(first); free(lam);
  free(clam);
  return 0;
}
