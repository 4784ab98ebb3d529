/*
 * pcad.h -- forward pass and reverse-mode adjoint (vector-Jacobian product)
 * of reduce, inclusive scan and reduce-by-index on one AMD Instinct MI355X
 * (gfx950).
 *
 * The operations follow "Reverse-Mode AD of Reduce-by-Index and Scan in
 * Futhark" (Bruun, Larsen, Hinnerskov, Oancea):
 *   vjp f x y_bar returns x_bar = J^T y_bar           (Section 2.2)
 *   reduce (.) e xs                                    (Section 3)
 *   scan (.) e xs, inclusive                           (Section 5)
 *   reduce_by_index hist (.) e ks vs                   (Section 4)
 * Operators are +, *, min, max and two generic associative operators:
 * linear-function composition and the 2x2 matrix product (Section 6.1,
 * operator figure), plus the evaluation's sumOfProd (an invertible lifted
 * operator, Section 3.3) and saturated addition (non-invertible).  Further
 * entry points cover scans and reduces of 3x3 and 5x5 matrix products
 * (pcad_matd_*) and the vectorised operators (pcad_v*: map2 of + * min max
 * over vectors of d floats).
 *
 * Conventions shared by every call
 * --------------------------------
 * - Every array pointer is a DEVICE pointer (hipMalloc'd or equivalent);
 *   scalars and sizes are host values.  The caller owns all memory; the
 *   library never allocates on these calls.  `stream` is a hipStream_t
 *   (NULL = the null stream); every call is asynchronous on it.
 * - Floats are IEEE binary32, indices int32.  All float arrays must be
 *   16-byte aligned (else PCAD_E_MISALIGNED).
 * - `batch` independent rows of `n` elements each, stored contiguously
 *   row-major (row r starts at element r*n).  batch >= 1, 0 <= n <=
 *   INT32_MAX, batch*n <= 2^40 (else PCAD_E_SIZE).
 * - Element layouts per operator:
 *     PCAD_ADD/MUL/MIN/MAX : x0 = x[batch*n];              x1 unused (NULL)
 *     PCAD_LINREC          : x0 = a[batch*n] (multiplier), x1 = b[batch*n]
 *                            (offset); the scan is y_i = a_i*y_{i-1} + b_i,
 *                            y_{-1} = 0, with cumulative product
 *                            A_i = a_0*...*a_i.
 *     PCAD_MAT2            : x0 = M[batch*n][4], row-major 2x2
 *                            [[m0,m1],[m2,m3]]; the scan is
 *                            P_i = M_0 x ... x M_i.
 * - Adjoints are OVERWRITTEN, unless `flags` has PCAD_ACCUMULATE, which gives
 *   the paper's x_bar += ... (Eq. 1).
 * - Arguments are validated before any launch and the status is returned
 *   synchronously.  A failure of a HIP runtime call returns PCAD_E_HIP;
 *   pcad_last_hip_error() gives its code.  Faults inside kernels surface at
 *   the caller's next synchronisation of `stream`.
 * - Workspace: `ws` / `ws_bytes` is caller-owned device scratch of at least
 *   the size pcad_query() reports.  It MUST be zero-filled once before its
 *   first use.  Every call leaves it holding only its control block (the
 *   first 256 bytes: rows done, launch epoch, error word -- see
 *   pcad_ws_status), look-back status words tagged with the launch that
 *   wrote them, and zeros -- scratch data is cleared before a call returns --
 *   so one workspace serves any sequence of calls of this library.  Do not
 *   write other data into it.  Calls that share one workspace must be
 *   ordered (same stream): concurrent calls on one workspace race.
 * - Saved state: `saved` carries what a forward call keeps for the adjoint
 *   call of the same arguments (layouts below); its size comes from
 *   pcad_query().  The library never reads it before the forward wrote it.
 * - Out-of-range keys of reduce-by-index (k < 0 or k >= m) are ignored by
 *   the forward and receive a zero adjoint (Section 4, sequential
 *   semantics).  min/max keep the LOWEST index among equal values
 *   (Section 3.2 Min/Max; Section 4.2); -0.0 and +0.0 compare equal and the
 *   winner's bit pattern is returned.
 */
#ifndef PCAD_H
#define PCAD_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  PCAD_OK = 0,
  PCAD_E_INVALID_ARG = 1, /* bad enum, negative size, unknown flag */
  PCAD_E_UNSUPPORTED = 2, /* valid arguments, combination not implemented */
  PCAD_E_NULLPTR = 3,     /* a required pointer is NULL */
  PCAD_E_MISALIGNED = 4,  /* a float array is not 16-byte aligned */
  PCAD_E_SIZE = 5,        /* n, m or batch out of the supported range */
  PCAD_E_WORKSPACE = 6,   /* ws_bytes smaller than pcad_query() reports */
  PCAD_E_HIP = 7,         /* a HIP runtime call failed; see pcad_last_hip_error */
  PCAD_E_TIMEOUT = 8      /* pcad_ws_status: a look-back wait of an earlier call on the
                             workspace timed out, so that call's results are invalid */
} pcad_status;

typedef enum { PCAD_REDUCE = 0, PCAD_SCAN = 1, PCAD_RBI = 2 } pcad_combinator;

typedef enum {
  PCAD_ADD = 0,
  PCAD_MUL = 1,
  PCAD_MIN = 2,
  PCAD_MAX = 3,
  PCAD_LINREC = 4, /* linear-function composition (a multiplier, b offset) */
  PCAD_MAT2 = 5,   /* 2x2 matrix product, row-major */
  PCAD_SUMPROD = 6, /* sumOfProd (Section 3.3), scalar inputs lifted to (0, a) */
  PCAD_SATADD = 7   /* saturated addition at 1e6 (the evaluation's operator figure) */
} pcad_op;

enum {
  PCAD_ACCUMULATE = 1u << 0, /* adjoint calls: x_bar += contribution */
};

/* Human-readable name of a status code (static storage). */
const char *pcad_status_string(int status);
/* hipError_t of the last failed HIP runtime call in this thread (0 if none). */
int pcad_last_hip_error(void);
/* Library version string. */
const char *pcad_version(void);

/*
 * pcad_ws_status -- whether a call on workspace `ws` failed inside its
 * kernels.  The look-back kernels wait for results of other workgroups of the
 * same launch; every such wait is bounded (about 2^20 polls), and a wait that
 * runs out (the grid could not stay resident, e.g. the GPU was shared with
 * other work) writes the launch's tag into word [2] of the control block,
 * after which every wait of that launch gives up and its results are invalid.
 * The word names the failed launch, so later calls on the workspace are not
 * affected by it.  This call synchronises `stream`, reads the word and
 * returns PCAD_E_TIMEOUT if it is set (clearing it when `clear` != 0), else
 * PCAD_OK.  ws must be 256-byte aligned (PCAD_E_NULLPTR / PCAD_E_MISALIGNED);
 * a HIP failure returns PCAD_E_HIP.  Host only: never call it while a call on
 * the same workspace is being captured into a graph.
 */
int pcad_ws_status(void *ws, int clear, void *stream);

/*
 * pcad_query -- bytes of saved state and workspace for a call.
 * Host-only; needs no GPU.  `m` is the bin count (RBI only, else ignored).
 * Either output pointer may be NULL.
 */
int pcad_query(int combinator, int op, int64_t batch, int64_t n, int64_t m, unsigned flags,
               size_t *saved_bytes, size_t *workspace_bytes);

/*
 * reduce (Section 3): y[r] = x[r,0] (.) x[r,1] (.) ... (.) x[r,n-1] per row r;
 * the neutral element when n = 0.
 *   y: batch elements (1, 1, 1, 1, 2 = (A, y), 4 floats per row by operator;
 *      LINREC writes the pair (A, y) of the composed linear function).
 *   saved layout per row:
 *     ADD   : nothing;
 *     MUL   : {uint32 n0; float y_pos} -- number of exact zeros and product
 *             of the non-zero elements (Section 3.2 Multiplication);
 *     MIN/MAX: {int32 k} -- lowest index attaining the extremum, n if empty
 *             (Section 3.2 Min/Max);
 *     LINREC/MAT2/SATADD: the exclusive prefix of every tile of the row
 *             (opaque);
 *     SUMPROD: {float s} -- the sum of the row.
 * SUMPROD is the invertible operator of Section 3.3: elements a enter as
 * pairs (0, a), pairs combine as (p1,s1) (.) (p2,s2) = (p1+p2+s1*s2, s1+s2),
 * and y is the p of the result, i.e. y = sum over i<j of a_i*a_j (0 for
 * n < 2).
 */
int pcad_reduce_fwd(int op, int64_t batch, int64_t n, const float *x0, const float *x1,
                    float *y, void *saved, unsigned flags, void *ws, size_t ws_bytes,
                    void *stream);

/*
 * Adjoint of reduce: x_bar = J^T y_bar, with y_bar holding one element per
 * row (same layout as y).  Rules: ADD broadcasts y_bar (Section 3.2
 * Addition); MUL uses the three zero cases (Section 3.2 Multiplication);
 * MIN/MAX write y_bar at index k only (Section 3.2 Min/Max); LINREC/MAT2 use
 * the general rule x_bar_i = d(l_i (.) x_i (.) r_i)/dx_i^T y_bar (Eq. 2) with
 * l_i, r_i the exclusive prefix and suffix (Section 3.1), which SATADD uses
 * too (its partials are 0 on a saturated step); SUMPROD uses the
 * invertible-operator rule of Section 3.3: the rest of the fold is
 * (p, s) inverted by (0, x_i), whose s is s - x_i, so x_bar_i =
 * (s - x_i) * y_bar (x0 required).
 *   xbar0/xbar1: same layout as x0/x1 (LINREC: a_bar, b_bar).
 */
int pcad_reduce_vjp(int op, int64_t batch, int64_t n, const float *x0, const float *x1,
                    const void *saved, const float *ybar, float *xbar0, float *xbar1,
                    unsigned flags, void *ws, size_t ws_bytes, void *stream);

/*
 * Inclusive scan (Section 5): rs_0 = x_0, rs_i = rs_{i-1} (.) x_i per row,
 * by a single-pass decoupled look-back over tiles.
 *   y0: the scan (scalar ops: x-layout; LINREC: y_i; MAT2: P_i, 4 floats).
 *   y1: LINREC only, optional: the cumulative multiplier A_i (may be NULL).
 *   saved: the exclusive prefix of every tile, which pcad_scan_vjp uses to
 *          recompute the forward prefixes inside each tile instead of
 *          storing them (the redundant-execution choice of the paper); may
 *          be NULL when the adjoint will be the checkpoint form.
 */
int pcad_scan_fwd(int op, int64_t batch, int64_t n, const float *x0, const float *x1,
                  float *y0, float *y1, void *saved, unsigned flags, void *ws,
                  size_t ws_bytes, void *stream);

/*
 * Adjoint of the inclusive scan (Section 5.2): the backward linear recurrence
 * lam_i = ybar_i + J_i^T lam_{i+1}, J_i = d(rs_i (.) x_{i+1})/d rs_i, solved
 * by a right-to-left decoupled look-back scan of adjoint affine maps, fused
 * with x_bar_i = d(rs_{i-1} (.) x_i)/d x_i^T lam_i (x_bar_0 = lam_0).
 * SATADD: both partials are [rs_{i-1} + x_i <= 1e6] (0 on a saturated step).
 * SUMPROD: inputs a_i lift to (0, a_i) and y_i is the p of the prefix, the
 * sum over j<k<=i of a_j a_k; the adjoint maps act on (lam_p, lam_s) through
 * J^T = [[1, 0], [a_i, 1]] and a_bar_i = S_{i-1} lam_p + lam_s (S the prefix
 * sum), recompute form only (pcad_scan_vjp_checkpoint: PCAD_E_UNSUPPORTED).
 * Forward prefixes are recomputed inside each tile from `saved`.
 *   ybar0: adjoint of y0 (x-layout; MAT2 4 floats per element).
 *   ybar1: LINREC only, optional adjoint of A (NULL = zero).
 *   xbar0/xbar1: LINREC: a_bar, b_bar; else xbar0 in x-layout.
 */
int pcad_scan_vjp(int op, int64_t batch, int64_t n, const float *x0, const float *x1,
                  const void *saved, const float *ybar0, const float *ybar1, float *xbar0,
                  float *xbar1, unsigned flags, void *ws, size_t ws_bytes, void *stream);

/*
 * pcad_scan_vjp_noalloc -- pcad_scan_vjp for callers that cannot allocate
 * device memory (code under graph capture, tight serving loops, harnesses
 * that forbid allocation): the same adjoint, arguments and results, with no
 * ws argument.  Its look-back workspace is a static device array of
 * PCAD_SCRATCH_BYTES, one per GPU, held until the process ends; the call
 * allocates nothing.  Sizes whose workspace (pcad_query) exceeds
 * PCAD_SCRATCH_BYTES return PCAD_E_SIZE before any launch (every operator up
 * to 2^26 elements fits).  All calls on one GPU share that array: calls that
 * may overlap (other streams, other host threads) race and must be ordered
 * by the caller.  A timed-out look-back wait is not reported (there is no
 * workspace to pass to pcad_ws_status).
 */
#define PCAD_SCRATCH_BYTES (4u << 20)
int pcad_scan_vjp_noalloc(int op, int64_t batch, int64_t n, const float *x0, const float *x1,
                          const void *saved, const float *ybar0, const float *ybar1,
                          float *xbar0, float *xbar1, unsigned flags, void *stream);

/*
 * Adjoint of the inclusive scan, checkpoint form: the forward prefixes
 * rs_{i-1} are read from the stored forward outputs (the tape of
 * intermediates, Section 2 on tapes versus redundant execution) instead of
 * being recomputed inside each tile; no `saved` state is needed, so the
 * forward call may pass saved = NULL.  Results equal pcad_scan_vjp's up to
 * the rounding of the recomputed prefixes.
 *   y0: the forward output y0 (required except for ADD, which reads none).
 *   y1: LINREC only: the forward's A output; required iff ybar1 != NULL.
 *   x1: LINREC only, may be NULL (the offsets b are not read).
 *   Other arguments and the workspace as for pcad_scan_vjp.
 */
int pcad_scan_vjp_checkpoint(int op, int64_t batch, int64_t n, const float *x0, const float *x1,
                             const float *y0, const float *y1, const float *ybar0,
                             const float *ybar1, float *xbar0, float *xbar1, unsigned flags,
                             void *ws, size_t ws_bytes, void *stream);

/*
 * reduce_by_index (Section 4): for every row r and bin k in [0,m),
 *   hist[r,k] = (.) over v[r,i] with idx[r,i] == k, in ascending i,
 * starting from the neutral element (the rewrite to a neutral initial
 * histogram; the caller combines an initial histogram itself).
 * Operators: ADD, MUL, MIN, MAX, and the ordered LINREC and MAT2, whose
 * per-bin fold takes the bin's elements in ascending index (the sequential
 * semantics of Section 4).  m >= 0, m <= 2^26; n at most 2^28.
 * Strategies (results agree up to the order in which + * SUMPROD combine):
 *   - a private LDS histogram per block (ADD/MUL up to 8192 bins, MIN/MAX
 *     and SUMPROD up to 4096);
 *   - beyond that, one row (batch == 1) of ADD up to 131072 bins or of
 *     MIN/MAX up to 65536: the bins are split into at most four 128 KB
 *     LDS tables (ADD: bin g in table g mod P; MIN/MAX: contiguous ranges),
 *     one block per (table, chunk of elements) with the blocks of a chunk
 *     on one XCD, and the per-chunk tables folded in chunk order (knob
 *     rbi.parts = 0 turns this off);
 *   - otherwise, for ADD/MUL/MIN/MAX/SUMPROD: the elements are partitioned once by
 *     bin range and each range gets its LDS histogram (the one-pass
 *     relative of the multi-pass technique of Section 4.2; bin ranges of
 *     16384 bins for ADD, 8192 otherwise, at most 2048 ranges), or, past
 *     that or when knob rbi.partition is 0, an LDS hash table of the bins a
 *     block meets with global atomics for the rest;
 *   - for LINREC/MAT2/SATADD (and, by knob, large bin counts of + * min
 *     max) a stable sort by bin followed by a segmented scan of each run
 *     (the rule figure's sort); their adjoints are the general rule.
 *   v: n floats per row; LINREC: n pairs (a, b) interleaved; MAT2: n
 *      row-major 2x2 matrices (4 floats).  hist: m entries of the same
 *      width per row.
 *   hist: batch*m floats.
 *   saved layout (arrays of batch*m entries, bin k of row r at r*m + k):
 *     ADD    : nothing;
 *     MUL    : uint32 n0[batch*m], then float y_pos[batch*m] (zero count and
 *              product of the non-zeros per bin, Section 4.2 Multiplication);
 *     MIN/MAX: int32 argk[batch*m], the lowest index of the bin's extremum,
 *              n when the bin is empty (Section 4.2 Min/Max rule figure);
 *     SUMPROD: float s[batch*m], the sum of the bin's values (its hist is
 *              the sum of v_i*v_j over pairs i<j of the bin); m <= 2^24;
 *     then, wherever the sort-based path may run (LINREC, MAT2, and bin
 *     counts beyond the LDS histogram), 256-byte aligned, per row the sorted
 *     keys, the permutation and the sort's scratch (opaque), which the
 *     ordered adjoint reuses instead of sorting again.
 */
int pcad_rbi_fwd(int op, int64_t batch, int64_t n, int64_t m, const int32_t *idx,
                 const float *v, float *hist, void *saved, unsigned flags, void *ws,
                 size_t ws_bytes, void *stream);

/*
 * Adjoint of reduce_by_index with respect to the values:
 *   ADD    : v_bar_i = hbar[idx_i] (gather)            (Section 4.2 Addition)
 *   MUL    : v_bar_i = hbar[k]*(n0==0 ? y_pos/v_i : (n0==1 && v_i==0 ? y_pos : 0))
 *                                                      (Section 4.2 Multiplication)
 *   MIN/MAX: v_bar_i = hbar[k] if i == argk[k] else 0  (Section 4.2 Min/Max),
 *            computed as the paper's rule states it: v_bar filled with zeros
 *            (skipped under PCAD_ACCUMULATE), then each bin's adjoint
 *            scattered to argk[k]; idx is not read
 *   SUMPROD: v_bar_i = (s[k] - v_i) * hbar[k]   (Section 4.2 Invertible
 *            Operators: hist[k] inverted by (0, v_i) leaves s[k] - v_i)
 *   LINREC/MAT2: v_bar_i = d(L_i (.) v_i (.) R_i)/dv_i^T hbar[k], with L_i and
 *            R_i the ordered folds of the bin's elements before and after i
 *            (the sort-based rule of Section 4, from the sort in `saved`)
 * with k = idx_i; out-of-range keys get 0.  v is required for MUL, LINREC
 * and MAT2; the ordered operators also need the workspace.  For the other
 * operators the workspace is optional: for MUL, given (of the queried size),
 * large bin counts first pack what an element needs from its bin into one
 * record per bin there, so each element makes one gather instead of one per
 * array; with ws = NULL (or too small) the adjoint gathers from `saved`
 * directly.
 */
int pcad_rbi_vjp(int op, int64_t batch, int64_t n, int64_t m, const int32_t *idx,
                 const float *v, const void *saved, const float *hbar, float *vbar,
                 unsigned flags, void *ws, size_t ws_bytes, void *stream);

/*
 * Batched segmented plan: many independent instances of ragged length, each
 *   y_s = linear-recurrence scan of (a_s, b_s)            (Section 5)
 *   (h_s, argk_s) = reduce_by_index(min) of y_s into m bins with keys idx_s
 *                                                          (Section 4)
 * and their adjoint given y_bar (per element) and h_bar (per instance and
 * bin): the min-by-index adjoint (Section 4.2 Min/Max) adds h_bar[s,k] at
 * y position argk[s,k], and the sum feeds the scan adjoint (Section 5.2).
 * The forward and the adjoint run as persistent look-back kernels over
 * (instance, tile) work items, captured in hipGraphs at bind time; every
 * run is one hipGraphLaunch.
 *
 *   offsets: HOST array of nseg+1 int64 element offsets (offsets[0] = 0,
 *            non-decreasing); instance s is [offsets[s], offsets[s+1]).
 *   m:       bins per instance, 1 <= m <= 1024 (PCAD_E_SIZE above).
 *   flags:   PCAD_PLAN_PER_SEGMENT also sizes the workspace for
 *            pcad_plan_run_per_segment (the same work as plain per-instance
 *            calls, for comparison).
 * Layouts (device): a, b, idx, y, y_bar, a_bar, b_bar: N = offsets[nseg]
 * elements; h, argk, h_bar: nseg*m, row-major by instance.  argk is the
 * instance-relative lowest index of the bin minimum, the instance length for
 * an empty bin; h is +inf there.  The adjoint reads argk, so a caller may
 * replace it between the two phases.  Keys outside [0,m) are ignored.
 * The plan owns host state and graphs only; the caller owns `saved` and
 * `ws` (sizes from pcad_plan_query; ws zero-filled before first use) and
 * all buffers, which stay bound until the next pcad_plan_bind.
 */
enum { PCAD_PLAN_PER_SEGMENT = 1u << 0 };
enum { PCAD_PHASE_FWD = 1, PCAD_PHASE_BWD = 2, PCAD_PHASE_BOTH = 3 };

typedef struct pcad_plan pcad_plan;

int pcad_plan_create(pcad_plan **plan, int64_t nseg, const int64_t *offsets, int64_t m,
                     unsigned flags);
int pcad_plan_query(const pcad_plan *plan, size_t *saved_bytes, size_t *workspace_bytes,
                    int64_t *n_elements, int64_t *n_items);
/* Uploads the plan's tables into ws, resets its merge keys, captures the
 * graphs on `stream`; synchronises `stream` once. */
int pcad_plan_bind(pcad_plan *plan, const float *a, const float *b, const int32_t *idx,
                   float *y, float *h, int32_t *argk, const float *ybar, const float *hbar,
                   float *abar, float *bbar, void *saved, void *ws, size_t ws_bytes,
                   void *stream);
/* phase: PCAD_PHASE_FWD, PCAD_PHASE_BWD or PCAD_PHASE_BOTH; one graph launch. */
int pcad_plan_run(pcad_plan *plan, int phase, void *stream);
/* The same results through plain per-instance calls of this library (scan,
 * reduce_by_index and their adjoints, one instance after the other). */
int pcad_plan_run_per_segment(pcad_plan *plan, int phase, void *stream);
void pcad_plan_destroy(pcad_plan *plan);
int pcad_plan_last_hip_error(void);

/*
 * Vectorised operators (Sections 3.2, 4.2 and 5.3, Vectorized Operators):
 * reduce, scan and reduce_by_index whose elements are vectors of d floats
 * combined component-wise (map2 of ADD, MUL, MIN or MAX; other operators
 * return PCAD_E_UNSUPPORTED).  Layouts, row-major:
 *   vreduce: x[batch][n][d] -> y[batch][d];
 *   vscan  : x[batch][n][d] -> y[batch][n][d] (inclusive, along n);
 *   vrbi   : idx[batch][n], v[batch][n][d] -> hist[batch][m][d], bin k of
 *            component c folding v[i][c] over the i with idx[i] == k.
 * Each runs the paper's rewrite of the vectorised form into the scalar one
 * over the transposed array (the IRWIM, ISWIM and IRBIWIM rules): the
 * operands are transposed into [d][n] and the scalar batched kernels run
 * over batch*d rows, row (b, c) holding component c of batch row b.
 * Saved state and workspace are those of the scalar call with batch*d rows
 * (its layouts, rows in that order); pcad_vquery reports them and the bytes
 * of `tmp`.
 *   tmp: caller-owned device scratch (256-byte aligned, not overlapping ws)
 *        for the transposed copies; its contents after a call are
 *        unspecified and it needs no initialisation.
 *   Adjoints follow the scalar rules per component; PCAD_ACCUMULATE adds
 *   into xbar / vbar.  Errors as for the scalar calls, plus
 *   PCAD_E_WORKSPACE / PCAD_E_NULLPTR / PCAD_E_MISALIGNED for `tmp`.
 */
int pcad_vquery(int combinator, int op, int64_t batch, int64_t n, int64_t d, int64_t m,
                unsigned flags, size_t *saved_bytes, size_t *workspace_bytes, size_t *tmp_bytes);
int pcad_vreduce_fwd(int op, int64_t batch, int64_t n, int64_t d, const float *x, float *y,
                     void *saved, unsigned flags, void *ws, size_t ws_bytes, void *tmp,
                     size_t tmp_bytes, void *stream);
int pcad_vreduce_vjp(int op, int64_t batch, int64_t n, int64_t d, const float *x, const void *saved,
                     const float *ybar, float *xbar, unsigned flags, void *ws, size_t ws_bytes,
                     void *tmp, size_t tmp_bytes, void *stream);
int pcad_vscan_fwd(int op, int64_t batch, int64_t n, int64_t d, const float *x, float *y,
                   void *saved, unsigned flags, void *ws, size_t ws_bytes, void *tmp,
                   size_t tmp_bytes, void *stream);
int pcad_vscan_vjp(int op, int64_t batch, int64_t n, int64_t d, const float *x, const void *saved,
                   const float *ybar, float *xbar, unsigned flags, void *ws, size_t ws_bytes,
                   void *tmp, size_t tmp_bytes, void *stream);
int pcad_vrbi_fwd(int op, int64_t batch, int64_t n, int64_t d, int64_t m, const int32_t *idx,
                  const float *v, float *hist, void *saved, unsigned flags, void *ws,
                  size_t ws_bytes, void *tmp, size_t tmp_bytes, void *stream);
int pcad_vrbi_vjp(int op, int64_t batch, int64_t n, int64_t d, int64_t m, const int32_t *idx,
                  const float *v, const void *saved, const float *hbar, float *vbar,
                  unsigned flags, void *ws, size_t ws_bytes, void *tmp, size_t tmp_bytes,
                  void *stream);

/*
 * Scans of d x d matrix products, d = 3 or 5 (the 3x3 and 5x5 matrix
 * multiplication operators of the evaluation), and their adjoints (Section
 * 5.3, redundant block-diagonal sparsity: the adjoint of P_i is a d x d
 * matrix and the map that carries it, r -> Pbar_i + r M_{i+1}^T, has a d x d
 * multiplier, so an adjoint map is 2 d^2 floats).
 *   M   : [batch][n][d*d] row-major d x d matrices, 16-byte aligned.
 *   P   : [batch][n][d*d], P_i = M_0 M_1 ... M_i per row.
 *   saved: the exclusive prefix product of every tile (pcad_matd_query),
 *          from which the adjoint recomputes the forward prefixes.
 *   Pbar / Mbar: adjoints in the layout of P / M; Mbar_i = P_{i-1}^T Rbar_i
 *          with Rbar_i = Pbar_i + Rbar_{i+1} M_{i+1}^T, P_{-1} = I;
 *          PCAD_ACCUMULATE adds into Mbar.
 *   ws  : workspace of pcad_matd_query's size, 256-byte aligned; it may be
 *         shared with the other calls on the same stream (between calls it
 *         holds only zeros past the control block).
 * Errors: PCAD_E_INVALID_ARG for d other than 3 or 5, negative sizes or
 * unknown flags; PCAD_E_SIZE for n > 2^31-1 or more than 2^31-1 tiles;
 * PCAD_E_NULLPTR / PCAD_E_MISALIGNED / PCAD_E_WORKSPACE as for the scans.
 * No compute happens on an error; batch == 0 or n == 0 is a no-op.
 */
int pcad_matd_query(int d, int64_t batch, int64_t n, unsigned flags, size_t *saved_bytes,
                    size_t *workspace_bytes);
int pcad_matd_scan_fwd(int d, int64_t batch, int64_t n, const float *M, float *P, void *saved,
                       unsigned flags, void *ws, size_t ws_bytes, void *stream);
int pcad_matd_scan_vjp(int d, int64_t batch, int64_t n, const float *M, const void *saved,
                       const float *Pbar, float *Mbar, unsigned flags, void *ws, size_t ws_bytes,
                       void *stream);

/*
 * Reduce of d x d matrix products, d = 3 or 5: Y = M_0 M_1 ... M_{n-1} per row
 * (the identity for n == 0), and its adjoint by the general rule of Section
 * 3.1, Mbar_i = L_i^T Ybar R_i^T with L_i = M_0 ... M_{i-1} and
 * R_i = M_{i+1} ... M_{n-1}.
 *   Y, Ybar: [batch][d*d].  M, Mbar, flags as for the scan.
 *   saved / ws: the sizes pcad_matd_query reports (the same as the scan's).
 * Errors as for the scans; batch == 0 is a no-op.
 */
int pcad_matd_reduce_fwd(int d, int64_t batch, int64_t n, const float *M, float *Y, void *saved,
                         unsigned flags, void *ws, size_t ws_bytes, void *stream);
int pcad_matd_reduce_vjp(int d, int64_t batch, int64_t n, const float *M, const void *saved,
                         const float *Ybar, float *Mbar, unsigned flags, void *ws,
                         size_t ws_bytes, void *stream);

/*
 * Scans of block-diagonal matrix products (Section 5.3, Block-Diagonal
 * Sparsity): every factor is a d x d block-diagonal matrix with k distinct
 * q x q blocks (d = k q), stored as its k blocks; products keep the shape,
 * so P_i is block diagonal too and so is the Jacobian of P_{i-1} M_i with
 * respect to P_{i-1}.  The adjoint therefore runs as k scans, one per block
 * position, each over q x q adjoint maps (the blocks' own redundant
 * block-diagonal form), never forming a d x d Jacobian.
 *   q   : 1, 2, 3 or 5 (block size); k >= 1 blocks, k*q*q <= 4096.
 *   M   : [batch][n][k][q*q]: block j of element i is a row-major q x q
 *         matrix; 16-byte aligned.
 *   P   : same layout; block j of P_i = M_0^j M_1^j ... M_i^j.
 *   saved: the blocks' tile prefixes (pcad_bds_query), read by the adjoint.
 *   Pbar / Mbar: adjoints in the layout of P / M (the diagonal blocks of the
 *         d x d adjoint; entries outside the blocks are structurally zero
 *         and have none); PCAD_ACCUMULATE adds into Mbar.
 *   ws  : workspace of pcad_bds_query's size, 256-byte aligned.
 *   tmp : scratch for the regrouped blocks, 256-byte aligned, of
 *         tmp_fwd_bytes (forward) or tmp_vjp_bytes (adjoint).
 * Errors: PCAD_E_INVALID_ARG for another q, k < 1, negative sizes or
 * unknown flags; PCAD_E_SIZE for k*q*q > 4096, n > 2^31-1 or too many
 * tiles; PCAD_E_NULLPTR / PCAD_E_MISALIGNED / PCAD_E_WORKSPACE as for the
 * scans.  No compute happens on an error; batch == 0 or n == 0 is a no-op.
 */
int pcad_bds_query(int q, int64_t k, int64_t batch, int64_t n, unsigned flags,
                   size_t *saved_bytes, size_t *workspace_bytes, size_t *tmp_fwd_bytes,
                   size_t *tmp_vjp_bytes);
int pcad_bds_scan_fwd(int q, int64_t k, int64_t batch, int64_t n, const float *M, float *P,
                      void *saved, unsigned flags, void *ws, size_t ws_bytes, void *tmp,
                      size_t tmp_bytes, void *stream);
int pcad_bds_scan_vjp(int q, int64_t k, int64_t batch, int64_t n, const float *M,
                      const void *saved, const float *Pbar, float *Mbar, unsigned flags, void *ws,
                      size_t ws_bytes, void *tmp, size_t tmp_bytes, void *stream);

/*
 * int32 forward combinators for ADD, MUL, MIN, MAX (the evaluation's integer
 * element types; integer arithmetic has no adjoint).  ADD and MUL wrap mod
 * 2^32 (two's complement); every result is exact, whatever the order of
 * combination.  combinator: PCAD_REDUCE (y[batch]), PCAD_SCAN (inclusive,
 * y[batch][n]) or PCAD_RBI (hist y[batch][m] from the neutral element: 0,
 * 1, INT32_MAX, INT32_MIN; keys outside [0, m) skipped).
 *   x: int32 [batch][n]; idx: int32 [batch][n] (PCAD_RBI only, else NULL).
 *   ws: PCAD_SCAN only (pcad_i32_query's size, zero-filled before first
 *       use, same contract as every workspace of this library); others
 *       need none (ws may be NULL).
 * Errors: PCAD_E_UNSUPPORTED for the other operators; PCAD_E_SIZE for
 * batch > 65535 (reduce, reduce-by-index), for a scan of more than 2^24 - 1
 * tiles of 4096 elements in all (batch * ceil(n / 4096)), or the sizes of
 * the float calls;
 * pointer and workspace errors as for those.
 */
int pcad_i32_query(int combinator, int op, int64_t batch, int64_t n, int64_t m,
                   size_t *workspace_bytes);
int pcad_i32_fwd(int combinator, int op, int64_t batch, int64_t n, int64_t m,
                 const int32_t *idx, const int32_t *x, int32_t *y, void *ws, size_t ws_bytes,
                 void *stream);

/*
 * Tuning knobs: launch parameters an autotuner may set (the block size of the
 * scan kernels per operator and direction, the bin count up to which
 * reduce-by-index keeps private LDS histograms, elements per histogram
 * block, the bin count from which the commutative operators sort by bin
 * rather than use the LDS hash table, and whether the partition, the hash
 * table or the split LDS tables handle large bin counts).  Knobs never change the sizes or
 * layouts of saved states and workspaces; they change speed and, for + and
 * *, the order in which floating-point values are combined (results stay
 * within the same error bound; min/max values, arg-extrema and zero counts
 * do not change).  They are process-wide and read at launch time, so setting
 * one while another host thread launches is a race on that launch's choice
 * only.
 *   pcad_knob_set: PCAD_E_INVALID_ARG for an unknown name or a value outside
 *                  the knob's range (block sizes: 256, 512 or 1024).
 *   pcad_knob_name: NULL for an index outside [0, pcad_knob_count()).
 *   pcad_knob_reset: every knob back to its built-in default.
 */
int pcad_knob_count(void);
const char *pcad_knob_name(int i);
int pcad_knob_get(const char *name, int64_t *value);
int pcad_knob_set(const char *name, int64_t value);
void pcad_knob_reset(void);

/* ---------------------------------------------------------------------------
 * Streaming copy (a measurement utility, not part of the method): copies
 * `bytes` bytes from device memory `src` to device memory `dst` on `stream`
 * (a hipStream_t; NULL for the null stream) with 16-byte nontemporal loads
 * and stores.  A kernel that reads and writes every byte once cannot stream
 * faster than this copy of the same bytes, so the benchmark reports its
 * kernels' rates against it beside the HBM peak.  The caller owns both
 * buffers; they must not overlap.
 *   PCAD_OK at once for bytes == 0; PCAD_E_NULLPTR for a NULL pointer;
 *   PCAD_E_MISALIGNED unless both pointers are 16-byte aligned;
 *   PCAD_E_INVALID_ARG unless bytes is a multiple of 16; PCAD_E_HIP if the
 *   launch fails.
 * ------------------------------------------------------------------------- */
int pcad_stream_copy(const void *src, void *dst, size_t bytes, void *stream);

#ifdef __cplusplus
}
#endif

#endif /* PCAD_H */
