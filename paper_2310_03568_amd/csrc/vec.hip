// Vectorised operators (Sections 3.2, 4.2 and 5.3, Vectorized Operators):
// reduce, scan and reduce_by_index whose elements are vectors of d floats
// combined component-wise (map2 of + * min max).  The paper rewrites them
// into the scalar combinators over the transposed array (the IRWIM, ISWIM
// and IRBIWIM rules) and differentiates the result; that is what runs here:
// an LDS-tiled transpose of every [n][d] operand into [d][n], the scalar
// batched kernels over batch*d rows, and a transpose back where a result is
// laid out by element.  Reduce-by-index shares one key array among the d
// columns, so the keys are repeated per column for the batched kernels.
//
// The transposed copies live in a caller-provided scratch buffer of their
// own (`tmp`), not in the workspace, whose words the look-back protocol
// reads as status words.
#include "device.hpp"
#include "internal.hpp"

namespace pcad {
namespace {

constexpr int TR_TH = 256;
constexpr int TR_ELEMS = 4096;  // elements per tile

// out[b][c][r] = in[b][r][c] (or +=) for a batch of rows x cols matrices.
// A tile is R x C elements (R*C = 4096, both powers of two), shaped so that
// both the reads (along c) and the writes (along r) are contiguous runs:
// C covers all of a narrow matrix's columns, R all of a short one's rows.
__global__ __launch_bounds__(TR_TH) void k_transpose(const float *in, float *out, int64_t rows,
                                                     int64_t cols, int lr, int lc,
                                                     int64_t tiles_r, int64_t tiles_c,
                                                     int64_t nbatch, int accumulate) {
  extern __shared__ float s_t[];  // R x (C + 1)
  const int R = 1 << lr, C = 1 << lc;
  const int64_t per = tiles_r * tiles_c;
  for (int64_t id = blockIdx.x; id < per * nbatch; id += gridDim.x) {
    const int64_t b = id / per, rem = id - b * per;
    const int64_t r0 = (rem / tiles_c) << lr, c0 = (rem % tiles_c) << lc;
    const float *ib = in + b * rows * cols;
    float *ob = out + b * rows * cols;
    for (int f = threadIdx.x; f < TR_ELEMS; f += TR_TH) {
      const int r = f >> lc, c = f & (C - 1);
      const int64_t gr = r0 + r, gc = c0 + c;
      if (gr < rows && gc < cols) s_t[r * (C + 1) + c] = ib[gr * cols + gc];
    }
    __syncthreads();
    for (int f = threadIdx.x; f < TR_ELEMS; f += TR_TH) {
      const int c = f >> lr, r = f & (R - 1);
      const int64_t gr = r0 + r, gc = c0 + c;
      if (gr < rows && gc < cols) {
        const float v = s_t[r * (C + 1) + c];
        float *o = ob + gc * rows + gr;
        *o = accumulate ? *o + v : v;
      }
    }
    __syncthreads();
  }
}

// out[b][c][i] = idx[b][i] for c < d
__global__ __launch_bounds__(256) void k_repeat_keys(const int32_t *idx, int32_t *out,
                                                    int64_t batch, int64_t n, int64_t d) {
  const int64_t total = batch * d * n;
  for (int64_t t = (int64_t)blockIdx.x * 256 + threadIdx.x; t < total;
       t += (int64_t)gridDim.x * 256) {
    const int64_t i = t % n, bc = t / n, b = bc / d;
    out[t] = idx[b * n + i];
  }
}

int ceil_log2(int64_t x) {
  int l = 0;
  while (((int64_t)1 << l) < x) ++l;
  return l;
}

int64_t grid_for(int64_t work) {
  int64_t g = work;
  if (g > 65535) g = 65535;
  if (g < 1) g = 1;
  return g;
}

size_t al256(size_t x) { return (x + 255) / 256 * 256; }

}  // namespace

hipError_t transpose_launch(const float *in, float *out, int64_t batch, int64_t rows, int64_t cols,
                            bool accumulate, hipStream_t s) {
  if (batch == 0 || rows == 0 || cols == 0) return hipSuccess;
  int lc, lr;
  if (cols < 64) {
    lc = ceil_log2(cols);
    lr = 12 - lc;
  } else if (rows < 64) {
    lr = ceil_log2(rows);
    lc = 12 - lr;
  } else {
    lr = lc = 6;
  }
  const int64_t tr = (rows + ((int64_t)1 << lr) - 1) >> lr;
  const int64_t tc = (cols + ((int64_t)1 << lc) - 1) >> lc;
  const size_t shm = (size_t)(((int64_t)1 << lr) * (((int64_t)1 << lc) + 1)) * sizeof(float);
  hipLaunchKernelGGL(k_transpose, dim3((unsigned)grid_for(tr * tc * batch)), dim3(TR_TH), shm, s,
                     in, out, rows, cols, lr, lc, tr, tc, batch, accumulate ? 1 : 0);
  return hipGetLastError();
}

// scratch (`tmp`) per combinator and direction, in bytes
size_t vec_tmp_bytes(int comb, int64_t batch, int64_t n, int64_t d, int64_t m) {
  const size_t col = al256((size_t)(batch * d * n) * 4);  // one [batch][d][n] array
  switch (comb) {
  case 0: return 2 * col;                                  // xT, x_barT
  case 1: return 3 * col;                                  // xT, yT / y_barT, x_barT
  case 2: return 3 * col + al256((size_t)(batch * d * m) * 4);  // vT, keys, v_barT, histT
  }
  return 0;
}

hipError_t vreduce_fwd_launch(int op, int64_t batch, int64_t n, int64_t d, const float *x,
                              float *y, void *saved, void *ws, void *tmp, hipStream_t s) {
  float *xt = static_cast<float *>(tmp);
  hipError_t e = transpose_launch(x, xt, batch, n, d, false, s);
  if (e != hipSuccess) return e;
  return reduce_fwd_launch(op, batch * d, n, xt, nullptr, y, saved, ws, s);
}

hipError_t vreduce_vjp_launch(int op, int64_t batch, int64_t n, int64_t d, const float *x,
                              const void *saved, const float *ybar, float *xbar, bool accumulate,
                              void *ws, void *tmp, hipStream_t s) {
  const size_t col = al256((size_t)(batch * d * n) * 4);
  float *xt = static_cast<float *>(tmp);
  float *gt = reinterpret_cast<float *>(static_cast<char *>(tmp) + col);
  hipError_t e = hipSuccess;
  if (op != ADD) e = transpose_launch(x, xt, batch, n, d, false, s);
  if (e != hipSuccess) return e;
  e = reduce_vjp_launch(op, batch * d, n, xt, nullptr, saved, ybar, gt, nullptr, false, ws, s);
  if (e != hipSuccess) return e;
  return transpose_launch(gt, xbar, batch, d, n, accumulate, s);
}

hipError_t vscan_fwd_launch(int op, int64_t batch, int64_t n, int64_t d, const float *x, float *y,
                            void *saved, void *ws, void *tmp, hipStream_t s) {
  const size_t col = al256((size_t)(batch * d * n) * 4);
  float *xt = static_cast<float *>(tmp);
  float *yt = reinterpret_cast<float *>(static_cast<char *>(tmp) + col);
  hipError_t e = transpose_launch(x, xt, batch, n, d, false, s);
  if (e != hipSuccess) return e;
  e = scan_fwd_launch(op, batch * d, n, xt, nullptr, yt, nullptr, static_cast<float *>(saved),
                      nullptr, false, ws, s);
  if (e != hipSuccess) return e;
  return transpose_launch(yt, y, batch, d, n, false, s);
}

hipError_t vscan_vjp_launch(int op, int64_t batch, int64_t n, int64_t d, const float *x,
                            const void *saved, const float *ybar, float *xbar, bool accumulate,
                            void *ws, void *tmp, hipStream_t s) {
  const size_t col = al256((size_t)(batch * d * n) * 4);
  char *t = static_cast<char *>(tmp);
  float *xt = reinterpret_cast<float *>(t);
  float *ybt = reinterpret_cast<float *>(t + col);
  float *gt = reinterpret_cast<float *>(t + 2 * col);
  hipError_t e = transpose_launch(x, xt, batch, n, d, false, s);
  if (e != hipSuccess) return e;
  e = transpose_launch(ybar, ybt, batch, n, d, false, s);
  if (e != hipSuccess) return e;
  e = scan_vjp_launch(op, batch * d, n, xt, nullptr, static_cast<const float *>(saved), nullptr,
                      nullptr, ybt, nullptr, gt, nullptr, false, ws, s);
  if (e != hipSuccess) return e;
  return transpose_launch(gt, xbar, batch, d, n, accumulate, s);
}

hipError_t vrbi_fwd_launch(int op, int64_t batch, int64_t n, int64_t d, int64_t m,
                           const int32_t *idx, const float *v, float *hist, void *saved, void *ws,
                           void *tmp, hipStream_t s) {
  const size_t col = al256((size_t)(batch * d * n) * 4);
  char *t = static_cast<char *>(tmp);
  float *vt = reinterpret_cast<float *>(t);
  int32_t *keys = reinterpret_cast<int32_t *>(t + col);
  float *ht = reinterpret_cast<float *>(t + 3 * col);
  hipError_t e = transpose_launch(v, vt, batch, n, d, false, s);
  if (e != hipSuccess) return e;
  if (n > 0)
    hipLaunchKernelGGL(k_repeat_keys, dim3((unsigned)grid_for((batch * d * n + 255) / 256)),
                       dim3(256), 0, s, idx, keys, batch, n, d);
  e = rbi_fwd_launch(op, batch * d, n, m, keys, vt, ht, saved, ws, s);
  if (e != hipSuccess) return e;
  return transpose_launch(ht, hist, batch, d, m, false, s);
}

hipError_t vrbi_vjp_launch(int op, int64_t batch, int64_t n, int64_t d, int64_t m,
                           const int32_t *idx, const float *v, const void *saved,
                           const float *hbar, float *vbar, bool accumulate, void *ws, void *tmp,
                           hipStream_t s) {
  const size_t col = al256((size_t)(batch * d * n) * 4);
  char *t = static_cast<char *>(tmp);
  float *vt = reinterpret_cast<float *>(t);
  int32_t *keys = reinterpret_cast<int32_t *>(t + col);
  float *gt = reinterpret_cast<float *>(t + 2 * col);
  float *hbt = reinterpret_cast<float *>(t + 3 * col);
  hipError_t e = hipSuccess;
  if (op == MUL) e = transpose_launch(v, vt, batch, n, d, false, s);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_repeat_keys, dim3((unsigned)grid_for((batch * d * n + 255) / 256)), dim3(256),
                     0, s, idx, keys, batch, n, d);
  e = transpose_launch(hbar, hbt, batch, m, d, false, s);
  if (e != hipSuccess) return e;
  e = rbi_vjp_launch(op, batch * d, n, m, keys, vt, saved, hbt, gt, false, ws, s);
  if (e != hipSuccess) return e;
  return transpose_launch(gt, vbar, batch, d, n, accumulate, s);
}

}  // namespace pcad
