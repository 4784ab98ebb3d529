// C-ABI entry points: argument validation (host only, before any launch),
// size queries, dispatch to the kernels.  See include/pcad.h.
#include <stdint.h>
#include <string.h>

#include <mutex>

#include "../../include/pcad.h"
#include "internal.hpp"

namespace pcad {

thread_local int g_last_hip = 0;

// records a failed HIP call for pcad_last_hip_error
int hip_status(hipError_t e) {
  if (e == hipSuccess) return PCAD_OK;
  g_last_hip = (int)e;
  return PCAD_E_HIP;
}

}  // namespace pcad

using namespace pcad;

namespace {

constexpr int64_t kMaxN = 2147483647LL;
constexpr int64_t kMaxTotal = 1LL << 40;
constexpr int64_t kMaxBins = 1LL << 26;
constexpr int64_t kMaxBinsSumProd = 1LL << 24;  // LDS histogram or at most 2048 bin ranges
constexpr unsigned kKnownFlags = PCAD_ACCUMULATE;


bool aligned16(const void *p) { return ((uintptr_t)p & 15u) == 0; }

int check_common(int op, int64_t batch, int64_t n, unsigned flags) {
  if (op < PCAD_ADD || op > PCAD_SATADD) return PCAD_E_INVALID_ARG;
  if (flags & ~kKnownFlags) return PCAD_E_INVALID_ARG;
  if (batch < 0 || n < 0) return PCAD_E_INVALID_ARG;
  if (n > kMaxN) return PCAD_E_SIZE;
  if (batch > 0 && n > 0 && batch > kMaxTotal / n) return PCAD_E_SIZE;
  return PCAD_OK;
}

// a required float array: non-null and 16-byte aligned
int need(const void *p) {
  if (!p) return PCAD_E_NULLPTR;
  if (!aligned16(p)) return PCAD_E_MISALIGNED;
  return PCAD_OK;
}

// an optional float array: null or 16-byte aligned
int opt(const void *p) { return (p && !aligned16(p)) ? PCAD_E_MISALIGNED : PCAD_OK; }

#define PCAD_TRY(expr)          \
  do {                          \
    const int _st = (expr);     \
    if (_st != PCAD_OK) return _st; \
  } while (0)

int64_t scan_tiles(int op, int64_t batch, int64_t n) {
  const int t = scan_tile_size(op);
  return batch * ((n + t - 1) / t);
}

size_t scan_saved(int op, int64_t batch, int64_t n) {
  return (size_t)scan_tiles(op, batch, n) * scan_elem_floats(op) * sizeof(float);
}

size_t scan_ws(int op, int64_t batch, int64_t n) {
  const int fw = 2 * scan_elem_floats(op);
  const int bw = scan_status_words(op, true);
  const int w = fw > bw ? fw : bw;
  return kCtlBytes + (size_t)scan_tiles(op, batch, n) * w * sizeof(uint64_t);
}

size_t reduce_saved(int op, int64_t batch, int64_t n) {
  switch (op) {
  case PCAD_ADD: return 0;
  case PCAD_MUL: return (size_t)batch * 8;
  case PCAD_MIN:
  case PCAD_MAX:
  case PCAD_SUMPROD: return (size_t)batch * 4;
  default: return scan_saved(op, batch, n);
  }
}

int query(int comb, int op, int64_t batch, int64_t n, int64_t m, size_t *saved, size_t *ws) {
  size_t s = 0, w = 0;
  switch (comb) {
  case PCAD_REDUCE:
    s = reduce_saved(op, batch, n);
    w = reduce_ws_bytes(op, batch, n);
    break;
  case PCAD_SCAN:
    s = scan_saved(op, batch, n);
    w = scan_ws(op, batch, n);
    break;
  case PCAD_RBI:
    if (m < 0) return PCAD_E_INVALID_ARG;
    if (m > (op == PCAD_SUMPROD ? kMaxBinsSumProd : kMaxBins)) return PCAD_E_SIZE;
    if (!sort_supported(n)) return PCAD_E_SIZE;
    s = rbi_saved_bytes(op, batch, n, m);
    w = rbi_ws_bytes(op, batch, n, m);
    break;
  default: return PCAD_E_INVALID_ARG;
  }
  if (saved) *saved = s;
  if (ws) *ws = w;
  return PCAD_OK;
}

int check_ws(int comb, int op, int64_t batch, int64_t n, int64_t m, const void *ws,
             size_t ws_bytes) {
  size_t need_ws = 0;
  PCAD_TRY(query(comb, op, batch, n, m, nullptr, &need_ws));
  if (ws_bytes < need_ws) return PCAD_E_WORKSPACE;
  if (need_ws > 0 && !ws) return PCAD_E_NULLPTR;
  if (ws && ((uintptr_t)ws & 255u)) return PCAD_E_MISALIGNED;
  return PCAD_OK;
}

int check_saved(int comb, int op, int64_t batch, int64_t n, int64_t m, const void *saved) {
  size_t s = 0;
  PCAD_TRY(query(comb, op, batch, n, m, &s, nullptr));
  if (s > 0 && !saved) return PCAD_E_NULLPTR;
  if (saved && !aligned16(saved)) return PCAD_E_MISALIGNED;
  return PCAD_OK;
}

// vectorised calls: + * min max over vectors of d floats; the scalar
// batched call they run has batch*d rows
int check_vec(int comb, int op, int64_t batch, int64_t n, int64_t d, int64_t m, unsigned flags) {
  if (op < PCAD_ADD || op > PCAD_SATADD) return PCAD_E_INVALID_ARG;
  if (op > PCAD_MAX) return PCAD_E_UNSUPPORTED;
  if (comb < PCAD_REDUCE || comb > PCAD_RBI) return PCAD_E_INVALID_ARG;
  if (d < 1 || batch < 0 || n < 0 || m < 0) return PCAD_E_INVALID_ARG;
  if (batch > 0 && d > kMaxTotal / batch) return PCAD_E_SIZE;
  PCAD_TRY(check_common(op, batch * d, n, flags));
  if (comb == PCAD_RBI && batch > 0 && m > kMaxTotal / (batch * d)) return PCAD_E_SIZE;
  return PCAD_OK;
}

int vquery(int comb, int op, int64_t batch, int64_t n, int64_t d, int64_t m, size_t *saved,
           size_t *ws, size_t *tmp) {
  PCAD_TRY(query(comb, op, batch * d, n, m, saved, ws));
  if (tmp) *tmp = vec_tmp_bytes(comb, batch, n, d, m);
  return PCAD_OK;
}

int check_tmp(int comb, int64_t batch, int64_t n, int64_t d, int64_t m, const void *tmp,
              size_t tmp_bytes) {
  const size_t need_tmp = vec_tmp_bytes(comb, batch, n, d, m);
  if (tmp_bytes < need_tmp) return PCAD_E_WORKSPACE;
  if (need_tmp > 0 && !tmp) return PCAD_E_NULLPTR;
  if (tmp && ((uintptr_t)tmp & 255u)) return PCAD_E_MISALIGNED;
  return PCAD_OK;
}

}  // namespace

extern "C" {

const char *pcad_status_string(int status) {
  switch (status) {
  case PCAD_OK: return "ok";
  case PCAD_E_INVALID_ARG: return "invalid argument";
  case PCAD_E_UNSUPPORTED: return "unsupported combination";
  case PCAD_E_NULLPTR: return "null pointer";
  case PCAD_E_MISALIGNED: return "pointer not 16-byte aligned";
  case PCAD_E_SIZE: return "size out of range";
  case PCAD_E_WORKSPACE: return "workspace too small";
  case PCAD_E_HIP: return "HIP runtime error";
  case PCAD_E_TIMEOUT: return "a look-back wait timed out: the results of that launch are invalid";
  }
  return "unknown status";
}

int pcad_last_hip_error(void) { return g_last_hip; }

int pcad_ws_status(void *ws, int clear, void *stream) {
  if (!ws) return PCAD_E_NULLPTR;
  if ((uintptr_t)ws & 255u) return PCAD_E_MISALIGNED;
  hipStream_t s = (hipStream_t)stream;
  uint32_t *err = reinterpret_cast<uint32_t *>(static_cast<char *>(ws) + 8);
  uint32_t word = 0;
  PCAD_TRY(hip_status(hipMemcpyAsync(&word, err, sizeof word, hipMemcpyDeviceToHost, s)));
  PCAD_TRY(hip_status(hipStreamSynchronize(s)));
  if (word == 0) return PCAD_OK;
  if (clear) {
    const uint32_t zero = 0;
    PCAD_TRY(hip_status(hipMemcpyAsync(err, &zero, sizeof zero, hipMemcpyHostToDevice, s)));
    PCAD_TRY(hip_status(hipStreamSynchronize(s)));
  }
  return PCAD_E_TIMEOUT;
}

const char *pcad_version(void) { return "pcad 0.1 gfx950"; }

int pcad_query(int combinator, int op, int64_t batch, int64_t n, int64_t m, unsigned flags,
               size_t *saved_bytes, size_t *workspace_bytes) {
  PCAD_TRY(check_common(op, batch, n, flags));
  return query(combinator, op, batch, n, m, saved_bytes, workspace_bytes);
}

int pcad_reduce_fwd(int op, int64_t batch, int64_t n, const float *x0, const float *x1, float *y,
                    void *saved, unsigned flags, void *ws, size_t ws_bytes, void *stream) {
  PCAD_TRY(check_common(op, batch, n, flags));
  if (batch == 0) return PCAD_OK;
  if (n > 0) {
    PCAD_TRY(need(x0));
    if (op == PCAD_LINREC) PCAD_TRY(need(x1));
  }
  PCAD_TRY(need(y));
  PCAD_TRY(check_saved(PCAD_REDUCE, op, batch, n, 0, saved));
  PCAD_TRY(check_ws(PCAD_REDUCE, op, batch, n, 0, ws, ws_bytes));
  return hip_status(reduce_fwd_launch(op, batch, n, x0, x1, y, saved, ws, (hipStream_t)stream));
}

int pcad_reduce_vjp(int op, int64_t batch, int64_t n, const float *x0, const float *x1,
                    const void *saved, const float *ybar, float *xbar0, float *xbar1,
                    unsigned flags, void *ws, size_t ws_bytes, void *stream) {
  PCAD_TRY(check_common(op, batch, n, flags));
  if (batch == 0 || n == 0) return PCAD_OK;
  if (op != PCAD_ADD) PCAD_TRY(need(x0));
  if (op == PCAD_LINREC) PCAD_TRY(need(x1));
  PCAD_TRY(need(ybar));
  PCAD_TRY(need(xbar0));
  if (op == PCAD_LINREC) PCAD_TRY(need(xbar1));
  PCAD_TRY(check_saved(PCAD_REDUCE, op, batch, n, 0, saved));
  PCAD_TRY(check_ws(PCAD_REDUCE, op, batch, n, 0, ws, ws_bytes));
  return hip_status(reduce_vjp_launch(op, batch, n, x0, x1, saved, ybar, xbar0, xbar1,
                                      (flags & PCAD_ACCUMULATE) != 0, ws, (hipStream_t)stream));
}

int pcad_scan_fwd(int op, int64_t batch, int64_t n, const float *x0, const float *x1, float *y0,
                  float *y1, void *saved, unsigned flags, void *ws, size_t ws_bytes,
                  void *stream) {
  PCAD_TRY(check_common(op, batch, n, flags));
  if (batch == 0 || n == 0) return PCAD_OK;
  if (scan_tiles(op, batch, n) > 2147483647LL) return PCAD_E_SIZE;
  PCAD_TRY(need(x0));
  if (op == PCAD_LINREC) PCAD_TRY(need(x1));
  PCAD_TRY(need(y0));
  PCAD_TRY(opt(y1));
  if (op != PCAD_LINREC && y1) return PCAD_E_INVALID_ARG;
  PCAD_TRY(opt(saved));  // NULL: no tile prefixes kept (checkpoint adjoint)
  PCAD_TRY(check_ws(PCAD_SCAN, op, batch, n, 0, ws, ws_bytes));
  return hip_status(scan_fwd_launch(op, batch, n, x0, x1, y0, y1, static_cast<float *>(saved),
                                    nullptr, false, ws, (hipStream_t)stream));
}

int pcad_scan_vjp(int op, int64_t batch, int64_t n, const float *x0, const float *x1,
                  const void *saved, const float *ybar0, const float *ybar1, float *xbar0,
                  float *xbar1, unsigned flags, void *ws, size_t ws_bytes, void *stream) {
  PCAD_TRY(check_common(op, batch, n, flags));
  if (batch == 0 || n == 0) return PCAD_OK;
  if (scan_tiles(op, batch, n) > 2147483647LL) return PCAD_E_SIZE;
  PCAD_TRY(need(x0));
  if (op == PCAD_LINREC) PCAD_TRY(need(x1));
  PCAD_TRY(need(ybar0));
  PCAD_TRY(opt(ybar1));
  if (op != PCAD_LINREC && ybar1) return PCAD_E_INVALID_ARG;
  PCAD_TRY(need(xbar0));
  if (op == PCAD_LINREC) PCAD_TRY(need(xbar1));
  PCAD_TRY(check_saved(PCAD_SCAN, op, batch, n, 0, saved));
  PCAD_TRY(check_ws(PCAD_SCAN, op, batch, n, 0, ws, ws_bytes));
  return hip_status(scan_vjp_launch(op, batch, n, x0, x1, static_cast<const float *>(saved),
                                    nullptr, nullptr, ybar0, ybar1, xbar0, xbar1,
                                    (flags & PCAD_ACCUMULATE) != 0, ws, (hipStream_t)stream));
}

// ---------------------------------------------------------------------------
// pcad_scan_vjp_noalloc: pcad_scan_vjp with its look-back workspace in a
// file-scope device array (one copy per GPU) instead of a caller's buffer.
// Device variables without an initialiser start zeroed, which is the state
// the control block needs before its first launch; every launch leaves the
// block ready for the next (the epoch advances, the finished-row count
// returns to 0), and the status words are validated by the launch tag, so
// nothing is cleared between calls.
// ---------------------------------------------------------------------------
static __device__ __align__(256) unsigned char scratch[PCAD_SCRATCH_BYTES];

namespace {

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void *g_scratch_dev[kMaxDevices];  // device address of `scratch` on each GPU

// the device address of the current GPU's copy of `scratch`, looked up once
// per GPU (the host-side name is only a stand-in for it)
int scratch_address(void **out) {
  int dev = 0;
  PCAD_TRY(hip_status(hipGetDevice(&dev)));
  if (dev < 0 || dev >= kMaxDevices) return PCAD_E_UNSUPPORTED;
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_dev[dev]) {
    void *p = nullptr;
    PCAD_TRY(hip_status(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch))));
    if (!p) return PCAD_E_HIP;
    g_scratch_dev[dev] = p;
  }
  *out = g_scratch_dev[dev];
  return PCAD_OK;
}

}  // namespace

int pcad_scan_vjp_noalloc(int op, int64_t batch, int64_t n, const float *x0, const float *x1,
                          const void *saved, const float *ybar0, const float *ybar1,
                          float *xbar0, float *xbar1, unsigned flags, void *stream) {
  PCAD_TRY(check_common(op, batch, n, flags));
  if (batch == 0 || n == 0) return PCAD_OK;
  if (scan_tiles(op, batch, n) > 2147483647LL) return PCAD_E_SIZE;
  if (scan_ws(op, batch, n) > (size_t)PCAD_SCRATCH_BYTES) return PCAD_E_SIZE;
  PCAD_TRY(need(x0));
  if (op == PCAD_LINREC) PCAD_TRY(need(x1));
  PCAD_TRY(need(ybar0));
  PCAD_TRY(opt(ybar1));
  if (op != PCAD_LINREC && ybar1) return PCAD_E_INVALID_ARG;
  PCAD_TRY(need(xbar0));
  if (op == PCAD_LINREC) PCAD_TRY(need(xbar1));
  PCAD_TRY(check_saved(PCAD_SCAN, op, batch, n, 0, saved));
  void *ws = nullptr;
  PCAD_TRY(scratch_address(&ws));
  return hip_status(scan_vjp_launch(op, batch, n, x0, x1, static_cast<const float *>(saved),
                                    nullptr, nullptr, ybar0, ybar1, xbar0, xbar1,
                                    (flags & PCAD_ACCUMULATE) != 0, ws, (hipStream_t)stream));
}

int pcad_scan_vjp_checkpoint(int op, int64_t batch, int64_t n, const float *x0, const float *x1,
                             const float *y0, const float *y1, const float *ybar0,
                             const float *ybar1, float *xbar0, float *xbar1, unsigned flags,
                             void *ws, size_t ws_bytes, void *stream) {
  PCAD_TRY(check_common(op, batch, n, flags));
  if (op == PCAD_SUMPROD) return PCAD_E_UNSUPPORTED;  // needs the s of every prefix
  if (batch == 0 || n == 0) return PCAD_OK;
  if (scan_tiles(op, batch, n) > 2147483647LL) return PCAD_E_SIZE;
  PCAD_TRY(need(x0));
  PCAD_TRY(opt(x1));
  if (op != PCAD_LINREC && x1) return PCAD_E_INVALID_ARG;
  if (op != PCAD_ADD) PCAD_TRY(need(y0));
  else PCAD_TRY(opt(y0));
  PCAD_TRY(opt(y1));
  PCAD_TRY(need(ybar0));
  PCAD_TRY(opt(ybar1));
  if (op != PCAD_LINREC && (ybar1 || y1)) return PCAD_E_INVALID_ARG;
  if (ybar1 && !y1) return PCAD_E_NULLPTR;  // A_bar needs the A tape
  PCAD_TRY(need(xbar0));
  if (op == PCAD_LINREC) PCAD_TRY(need(xbar1));
  PCAD_TRY(check_ws(PCAD_SCAN, op, batch, n, 0, ws, ws_bytes));
  // ADD reads no prefix: its adjoint is the recompute form with nothing to recompute
  const float *tp0 = op == PCAD_ADD ? nullptr : y0;
  return hip_status(scan_vjp_launch(op, batch, n, x0, x1, nullptr, tp0, ybar1 ? y1 : nullptr,
                                    ybar0, ybar1, xbar0, xbar1,
                                    (flags & PCAD_ACCUMULATE) != 0, ws, (hipStream_t)stream));
}

int pcad_rbi_fwd(int op, int64_t batch, int64_t n, int64_t m, const int32_t *idx, const float *v,
                 float *hist, void *saved, unsigned flags, void *ws, size_t ws_bytes,
                 void *stream) {
  PCAD_TRY(check_common(op, batch, n, flags));
  if (m < 0) return PCAD_E_INVALID_ARG;
  if (m > (op == PCAD_SUMPROD ? kMaxBinsSumProd : kMaxBins)) return PCAD_E_SIZE;
  if (batch == 0 || m == 0) return PCAD_OK;
  if (n > 0) {
    PCAD_TRY(need(idx));
    PCAD_TRY(need(v));
  }
  PCAD_TRY(need(hist));
  PCAD_TRY(check_saved(PCAD_RBI, op, batch, n, m, saved));
  PCAD_TRY(check_ws(PCAD_RBI, op, batch, n, m, ws, ws_bytes));
  return hip_status(rbi_fwd_launch(op, batch, n, m, idx, v, hist, saved, ws, (hipStream_t)stream));
}

int pcad_rbi_vjp(int op, int64_t batch, int64_t n, int64_t m, const int32_t *idx, const float *v,
                 const void *saved, const float *hbar, float *vbar, unsigned flags, void *ws,
                 size_t ws_bytes, void *stream) {
  PCAD_TRY(check_common(op, batch, n, flags));
  if (m < 0) return PCAD_E_INVALID_ARG;
  if (m > (op == PCAD_SUMPROD ? kMaxBinsSumProd : kMaxBins)) return PCAD_E_SIZE;
  if (batch == 0 || n == 0) return PCAD_OK;
  PCAD_TRY(need(idx));
  // the general rule (ordered operators, saturated addition) reads the values
  // and the sort's status words in the workspace
  const bool ordered = op == PCAD_LINREC || op == PCAD_MAT2 || op == PCAD_SATADD;
  if (op == PCAD_MUL || op == PCAD_SUMPROD || ordered) PCAD_TRY(need(v));
  if (m > 0) PCAD_TRY(need(hbar));
  PCAD_TRY(need(vbar));
  PCAD_TRY(check_saved(PCAD_RBI, op, batch, n, m, saved));
  if (ordered) {
    PCAD_TRY(check_ws(PCAD_RBI, op, batch, n, m, ws, ws_bytes));
  } else if (ws != nullptr && check_ws(PCAD_RBI, op, batch, n, m, ws, ws_bytes) != PCAD_OK) {
    // optional for + * min max: without a (sufficient) workspace the
    // adjoint gathers from the saved arrays directly
    ws = nullptr;
  }
  return hip_status(rbi_vjp_launch(op, batch, n, m, idx, v, saved, hbar, vbar,
                                   (flags & PCAD_ACCUMULATE) != 0, ws, (hipStream_t)stream));
}

}  // extern "C"

extern "C" {

int pcad_vquery(int combinator, int op, int64_t batch, int64_t n, int64_t d, int64_t m,
                unsigned flags, size_t *saved_bytes, size_t *workspace_bytes, size_t *tmp_bytes) {
  PCAD_TRY(check_vec(combinator, op, batch, n, d, m, flags));
  return vquery(combinator, op, batch, n, d, m, saved_bytes, workspace_bytes, tmp_bytes);
}

int pcad_vreduce_fwd(int op, int64_t batch, int64_t n, int64_t d, const float *x, float *y,
                     void *saved, unsigned flags, void *ws, size_t ws_bytes, void *tmp,
                     size_t tmp_bytes, void *stream) {
  PCAD_TRY(check_vec(PCAD_REDUCE, op, batch, n, d, 0, flags));
  if (batch == 0) return PCAD_OK;
  if (n > 0) PCAD_TRY(need(x));
  PCAD_TRY(need(y));
  PCAD_TRY(check_saved(PCAD_REDUCE, op, batch * d, n, 0, saved));
  PCAD_TRY(check_ws(PCAD_REDUCE, op, batch * d, n, 0, ws, ws_bytes));
  PCAD_TRY(check_tmp(PCAD_REDUCE, batch, n, d, 0, tmp, tmp_bytes));
  return hip_status(vreduce_fwd_launch(op, batch, n, d, x, y, saved, ws, tmp, (hipStream_t)stream));
}

int pcad_vreduce_vjp(int op, int64_t batch, int64_t n, int64_t d, const float *x, const void *saved,
                     const float *ybar, float *xbar, unsigned flags, void *ws, size_t ws_bytes,
                     void *tmp, size_t tmp_bytes, void *stream) {
  PCAD_TRY(check_vec(PCAD_REDUCE, op, batch, n, d, 0, flags));
  if (batch == 0 || n == 0) return PCAD_OK;
  if (op != PCAD_ADD) PCAD_TRY(need(x));
  PCAD_TRY(need(ybar));
  PCAD_TRY(need(xbar));
  PCAD_TRY(check_saved(PCAD_REDUCE, op, batch * d, n, 0, saved));
  PCAD_TRY(check_ws(PCAD_REDUCE, op, batch * d, n, 0, ws, ws_bytes));
  PCAD_TRY(check_tmp(PCAD_REDUCE, batch, n, d, 0, tmp, tmp_bytes));
  return hip_status(vreduce_vjp_launch(op, batch, n, d, x, saved, ybar, xbar,
                                       (flags & PCAD_ACCUMULATE) != 0, ws, tmp, (hipStream_t)stream));
}

int pcad_vscan_fwd(int op, int64_t batch, int64_t n, int64_t d, const float *x, float *y,
                   void *saved, unsigned flags, void *ws, size_t ws_bytes, void *tmp,
                   size_t tmp_bytes, void *stream) {
  PCAD_TRY(check_vec(PCAD_SCAN, op, batch, n, d, 0, flags));
  if (batch == 0 || n == 0) return PCAD_OK;
  if (scan_tiles(op, batch * d, n) > 2147483647LL) return PCAD_E_SIZE;
  PCAD_TRY(need(x));
  PCAD_TRY(need(y));
  PCAD_TRY(check_saved(PCAD_SCAN, op, batch * d, n, 0, saved));
  PCAD_TRY(check_ws(PCAD_SCAN, op, batch * d, n, 0, ws, ws_bytes));
  PCAD_TRY(check_tmp(PCAD_SCAN, batch, n, d, 0, tmp, tmp_bytes));
  return hip_status(vscan_fwd_launch(op, batch, n, d, x, y, saved, ws, tmp, (hipStream_t)stream));
}

int pcad_vscan_vjp(int op, int64_t batch, int64_t n, int64_t d, const float *x, const void *saved,
                   const float *ybar, float *xbar, unsigned flags, void *ws, size_t ws_bytes,
                   void *tmp, size_t tmp_bytes, void *stream) {
  PCAD_TRY(check_vec(PCAD_SCAN, op, batch, n, d, 0, flags));
  if (batch == 0 || n == 0) return PCAD_OK;
  if (scan_tiles(op, batch * d, n) > 2147483647LL) return PCAD_E_SIZE;
  PCAD_TRY(need(x));
  PCAD_TRY(need(ybar));
  PCAD_TRY(need(xbar));
  PCAD_TRY(check_saved(PCAD_SCAN, op, batch * d, n, 0, saved));
  PCAD_TRY(check_ws(PCAD_SCAN, op, batch * d, n, 0, ws, ws_bytes));
  PCAD_TRY(check_tmp(PCAD_SCAN, batch, n, d, 0, tmp, tmp_bytes));
  return hip_status(vscan_vjp_launch(op, batch, n, d, x, saved, ybar, xbar,
                                     (flags & PCAD_ACCUMULATE) != 0, ws, tmp, (hipStream_t)stream));
}

int pcad_vrbi_fwd(int op, int64_t batch, int64_t n, int64_t d, int64_t m, const int32_t *idx,
                  const float *v, float *hist, void *saved, unsigned flags, void *ws,
                  size_t ws_bytes, void *tmp, size_t tmp_bytes, void *stream) {
  PCAD_TRY(check_vec(PCAD_RBI, op, batch, n, d, m, flags));
  if (m > kMaxBins) return PCAD_E_SIZE;
  if (batch == 0 || m == 0) return PCAD_OK;
  if (n > 0) {
    PCAD_TRY(need(idx));
    PCAD_TRY(need(v));
  }
  PCAD_TRY(need(hist));
  PCAD_TRY(check_saved(PCAD_RBI, op, batch * d, n, m, saved));
  PCAD_TRY(check_ws(PCAD_RBI, op, batch * d, n, m, ws, ws_bytes));
  PCAD_TRY(check_tmp(PCAD_RBI, batch, n, d, m, tmp, tmp_bytes));
  return hip_status(vrbi_fwd_launch(op, batch, n, d, m, idx, v, hist, saved, ws, tmp,
                                    (hipStream_t)stream));
}

int pcad_vrbi_vjp(int op, int64_t batch, int64_t n, int64_t d, int64_t m, const int32_t *idx,
                  const float *v, const void *saved, const float *hbar, float *vbar,
                  unsigned flags, void *ws, size_t ws_bytes, void *tmp, size_t tmp_bytes,
                  void *stream) {
  PCAD_TRY(check_vec(PCAD_RBI, op, batch, n, d, m, flags));
  if (m > kMaxBins) return PCAD_E_SIZE;
  if (batch == 0 || n == 0) return PCAD_OK;
  PCAD_TRY(need(idx));
  if (op == PCAD_MUL) PCAD_TRY(need(v));
  if (m > 0) PCAD_TRY(need(hbar));
  PCAD_TRY(need(vbar));
  PCAD_TRY(check_saved(PCAD_RBI, op, batch * d, n, m, saved));
  PCAD_TRY(check_ws(PCAD_RBI, op, batch * d, n, m, ws, ws_bytes));
  PCAD_TRY(check_tmp(PCAD_RBI, batch, n, d, m, tmp, tmp_bytes));
  return hip_status(vrbi_vjp_launch(op, batch, n, d, m, idx, v, saved, hbar, vbar,
                                    (flags & PCAD_ACCUMULATE) != 0, ws, tmp, (hipStream_t)stream));
}

}  // extern "C"

namespace {

int check_matd(int d, int64_t batch, int64_t n, unsigned flags) {
  if (d != 3 && d != 5) return PCAD_E_INVALID_ARG;
  if (flags & ~kKnownFlags) return PCAD_E_INVALID_ARG;
  if (batch < 0 || n < 0) return PCAD_E_INVALID_ARG;
  if (n > kMaxN) return PCAD_E_SIZE;
  if (batch > 0 && n > 0 && batch > kMaxTotal / n) return PCAD_E_SIZE;
  if (matd_tiles(d, batch, n) > 2147483647LL) return PCAD_E_SIZE;
  return PCAD_OK;
}

int check_matd_ws(int d, int64_t batch, int64_t n, const void *ws, size_t ws_bytes) {
  if (ws_bytes < matd_ws_bytes(d, batch, n)) return PCAD_E_WORKSPACE;
  if (!ws) return PCAD_E_NULLPTR;
  if ((uintptr_t)ws & 255u) return PCAD_E_MISALIGNED;
  return PCAD_OK;
}

}  // namespace

extern "C" {

int pcad_matd_query(int d, int64_t batch, int64_t n, unsigned flags, size_t *saved_bytes,
                    size_t *workspace_bytes) {
  PCAD_TRY(check_matd(d, batch, n, flags));
  if (saved_bytes) *saved_bytes = matd_saved_bytes(d, batch, n);
  if (workspace_bytes) *workspace_bytes = matd_ws_bytes(d, batch, n);
  return PCAD_OK;
}

int pcad_matd_scan_fwd(int d, int64_t batch, int64_t n, const float *M, float *P, void *saved,
                       unsigned flags, void *ws, size_t ws_bytes, void *stream) {
  PCAD_TRY(check_matd(d, batch, n, flags));
  if (batch == 0 || n == 0) return PCAD_OK;
  PCAD_TRY(need(M));
  PCAD_TRY(need(P));
  PCAD_TRY(need(saved));
  PCAD_TRY(check_matd_ws(d, batch, n, ws, ws_bytes));
  return hip_status(matd_fwd_launch(d, batch, n, M, P, static_cast<float *>(saved), ws,
                                    (hipStream_t)stream));
}

int pcad_matd_scan_vjp(int d, int64_t batch, int64_t n, const float *M, const void *saved,
                       const float *Pbar, float *Mbar, unsigned flags, void *ws, size_t ws_bytes,
                       void *stream) {
  PCAD_TRY(check_matd(d, batch, n, flags));
  if (batch == 0 || n == 0) return PCAD_OK;
  PCAD_TRY(need(M));
  PCAD_TRY(need(saved));
  PCAD_TRY(need(Pbar));
  PCAD_TRY(need(Mbar));
  PCAD_TRY(check_matd_ws(d, batch, n, ws, ws_bytes));
  return hip_status(matd_vjp_launch(d, batch, n, M, static_cast<const float *>(saved), Pbar, Mbar,
                                    (flags & PCAD_ACCUMULATE) != 0, ws, (hipStream_t)stream));
}

int pcad_matd_reduce_fwd(int d, int64_t batch, int64_t n, const float *M, float *Y, void *saved,
                         unsigned flags, void *ws, size_t ws_bytes, void *stream) {
  PCAD_TRY(check_matd(d, batch, n, flags));
  if (batch == 0) return PCAD_OK;
  PCAD_TRY(need(Y));
  if (n > 0) {
    PCAD_TRY(need(M));
    PCAD_TRY(need(saved));
    PCAD_TRY(check_matd_ws(d, batch, n, ws, ws_bytes));
  }
  return hip_status(matd_reduce_fwd_launch(d, batch, n, M, Y, static_cast<float *>(saved), ws,
                                           (hipStream_t)stream));
}

int pcad_matd_reduce_vjp(int d, int64_t batch, int64_t n, const float *M, const void *saved,
                         const float *Ybar, float *Mbar, unsigned flags, void *ws,
                         size_t ws_bytes, void *stream) {
  PCAD_TRY(check_matd(d, batch, n, flags));
  if (batch == 0 || n == 0) return PCAD_OK;
  PCAD_TRY(need(M));
  PCAD_TRY(need(saved));
  PCAD_TRY(need(Ybar));
  PCAD_TRY(need(Mbar));
  PCAD_TRY(check_matd_ws(d, batch, n, ws, ws_bytes));
  return hip_status(matd_reduce_vjp_launch(d, batch, n, M, static_cast<const float *>(saved),
                                           Ybar, Mbar, (flags & PCAD_ACCUMULATE) != 0, ws,
                                           (hipStream_t)stream));
}

namespace {

int check_i32(int comb, int op, int64_t batch, int64_t n, int64_t m) {
  if (comb < PCAD_REDUCE || comb > PCAD_RBI) return PCAD_E_INVALID_ARG;
  if (op < PCAD_ADD || op > PCAD_SATADD) return PCAD_E_INVALID_ARG;
  if (op > PCAD_MAX) return PCAD_E_UNSUPPORTED;
  PCAD_TRY(check_common(op, batch, n, 0));
  if (comb != PCAD_SCAN && batch > 65535) return PCAD_E_SIZE;
  // the scan launches one 256-thread block per tile and per row; a grid
  // dimension holds fewer than 2^32 threads
  if (comb == PCAD_SCAN && n > 0 && i32_scan_tiles(batch, n) > kI32MaxScanTiles) return PCAD_E_SIZE;
  if (comb == PCAD_RBI) {
    if (m < 0) return PCAD_E_INVALID_ARG;
    if (m > kMaxBins) return PCAD_E_SIZE;
  }
  return PCAD_OK;
}

}  // namespace

int pcad_i32_query(int combinator, int op, int64_t batch, int64_t n, int64_t m,
                   size_t *workspace_bytes) {
  PCAD_TRY(check_i32(combinator, op, batch, n, m));
  if (workspace_bytes) *workspace_bytes = i32_ws_bytes(combinator, batch, n);
  return PCAD_OK;
}

int pcad_i32_fwd(int combinator, int op, int64_t batch, int64_t n, int64_t m,
                 const int32_t *idx, const int32_t *x, int32_t *y, void *ws, size_t ws_bytes,
                 void *stream) {
  PCAD_TRY(check_i32(combinator, op, batch, n, m));
  if (batch == 0) return PCAD_OK;
  if (combinator == PCAD_SCAN && n == 0) return PCAD_OK;
  if (combinator == PCAD_RBI && m == 0) return PCAD_OK;
  if (n > 0) PCAD_TRY(need(x));
  if (combinator == PCAD_RBI && n > 0) PCAD_TRY(need(idx));
  PCAD_TRY(need(y));
  const size_t need_ws = i32_ws_bytes(combinator, batch, n);
  if (need_ws > 0) {
    if (ws_bytes < need_ws) return PCAD_E_WORKSPACE;
    if (!ws) return PCAD_E_NULLPTR;
    if ((uintptr_t)ws & 255u) return PCAD_E_MISALIGNED;
  }
  return hip_status(i32_fwd_launch(combinator, op, batch, n, m, idx, x, y, ws,
                                   (hipStream_t)stream));
}

}  // extern "C"

// ---------------------------------------------------------------------------
// block-diagonal matrix-product scans (k blocks of q x q)
// ---------------------------------------------------------------------------
namespace {

int check_bds(int q, int64_t k, int64_t batch, int64_t n, unsigned flags) {
  if (flags & ~kKnownFlags) return PCAD_E_INVALID_ARG;
  if (k < 1 || batch < 0 || n < 0) return PCAD_E_INVALID_ARG;
  if (q != 1 && q != 2 && q != 3 && q != 5) return PCAD_E_INVALID_ARG;
  if (!bds_supported(q, k)) return PCAD_E_SIZE;
  if (n > kMaxN) return PCAD_E_SIZE;
  if (batch > 0 && n > 0 && batch > kMaxTotal / n / k) return PCAD_E_SIZE;
  const int64_t rows = batch * k;
  if (q >= 3) {
    if (matd_tiles(q, rows, n) > 2147483647LL) return PCAD_E_SIZE;
  } else if (scan_tiles(q == 1 ? PCAD_MUL : PCAD_MAT2, rows, n) > 2147483647LL) {
    return PCAD_E_SIZE;
  }
  return PCAD_OK;
}

void bds_sizes(int q, int64_t k, int64_t batch, int64_t n, size_t *saved, size_t *ws) {
  const int64_t rows = batch * k;
  if (q >= 3) {
    *saved = matd_saved_bytes(q, rows, n);
    *ws = matd_ws_bytes(q, rows, n);
  } else {
    const int op = q == 1 ? PCAD_MUL : PCAD_MAT2;
    *saved = scan_saved(op, rows, n);
    *ws = scan_ws(op, rows, n);
  }
}

int check_bds_bufs(int q, int64_t k, int64_t batch, int64_t n, int dir, const void *saved,
                   const void *ws, size_t ws_bytes, const void *tmp, size_t tmp_bytes) {
  size_t sv = 0, w = 0;
  bds_sizes(q, k, batch, n, &sv, &w);
  if (sv > 0) PCAD_TRY(need(saved));
  if (ws_bytes < w) return PCAD_E_WORKSPACE;
  if (!ws) return PCAD_E_NULLPTR;
  if ((uintptr_t)ws & 255u) return PCAD_E_MISALIGNED;
  if (tmp_bytes < bds_tmp_bytes(dir, q, k, batch, n)) return PCAD_E_WORKSPACE;
  if (!tmp) return PCAD_E_NULLPTR;
  if ((uintptr_t)tmp & 255u) return PCAD_E_MISALIGNED;
  return PCAD_OK;
}

}  // namespace

extern "C" {

int pcad_bds_query(int q, int64_t k, int64_t batch, int64_t n, unsigned flags,
                   size_t *saved_bytes, size_t *workspace_bytes, size_t *tmp_fwd_bytes,
                   size_t *tmp_vjp_bytes) {
  PCAD_TRY(check_bds(q, k, batch, n, flags));
  size_t sv = 0, w = 0;
  bds_sizes(q, k, batch, n, &sv, &w);
  if (saved_bytes) *saved_bytes = sv;
  if (workspace_bytes) *workspace_bytes = w;
  if (tmp_fwd_bytes) *tmp_fwd_bytes = bds_tmp_bytes(0, q, k, batch, n);
  if (tmp_vjp_bytes) *tmp_vjp_bytes = bds_tmp_bytes(1, q, k, batch, n);
  return PCAD_OK;
}

int pcad_bds_scan_fwd(int q, int64_t k, int64_t batch, int64_t n, const float *M, float *P,
                      void *saved, unsigned flags, void *ws, size_t ws_bytes, void *tmp,
                      size_t tmp_bytes, void *stream) {
  PCAD_TRY(check_bds(q, k, batch, n, flags));
  if (batch == 0 || n == 0) return PCAD_OK;
  PCAD_TRY(need(M));
  PCAD_TRY(need(P));
  PCAD_TRY(check_bds_bufs(q, k, batch, n, 0, saved, ws, ws_bytes, tmp, tmp_bytes));
  return hip_status(bds_fwd_launch(q, k, batch, n, M, P, saved, ws, tmp, (hipStream_t)stream));
}

int pcad_bds_scan_vjp(int q, int64_t k, int64_t batch, int64_t n, const float *M,
                      const void *saved, const float *Pbar, float *Mbar, unsigned flags, void *ws,
                      size_t ws_bytes, void *tmp, size_t tmp_bytes, void *stream) {
  PCAD_TRY(check_bds(q, k, batch, n, flags));
  if (batch == 0 || n == 0) return PCAD_OK;
  PCAD_TRY(need(M));
  PCAD_TRY(need(Pbar));
  PCAD_TRY(need(Mbar));
  PCAD_TRY(check_bds_bufs(q, k, batch, n, 1, saved, ws, ws_bytes, tmp, tmp_bytes));
  return hip_status(bds_vjp_launch(q, k, batch, n, M, saved, Pbar, Mbar,
                                   (flags & PCAD_ACCUMULATE) != 0, ws, tmp, (hipStream_t)stream));
}

}  // extern "C"
