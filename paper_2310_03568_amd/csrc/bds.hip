// Block-diagonal sparsity (Section 5.3, Block-Diagonal Sparsity): the scan
// of d x d matrix products whose factors are block diagonal with k distinct
// q x q blocks (d = k q).  Products keep that shape, and the Jacobian of
// rs_i (.) a_{i+1} with respect to rs_i is block diagonal too, so the
// adjoint needs no d x d Jacobian: it is k independent scans, one per block
// position, each over (alpha^q, alpha^{q x q}) adjoint maps.  Here the k
// block scans run as one batched scan of batch*k rows: the blocks are
// regrouped from [batch][n][k][q*q] into [batch][k][n][q*q] (an LDS-staged
// regrouping, coalesced both ways), the batched kernels of the q x q
// operator run (q = 1: the scalar product; 2: the 2 x 2 product; 3, 5: the
// d x d product kernels), and the results are regrouped back.  Each block
// scan's own adjoint maps are the redundant form (RBDS) of its operator.
//
// The regrouped copies live in a caller-provided scratch buffer (`tmp`),
// not in the workspace, whose words the look-back protocol reads.
#include "../../include/pcad.h"
#include "device.hpp"
#include "internal.hpp"

namespace pcad {
namespace {

constexpr int BT_TH = 256;
constexpr int BT_FLOATS = 4096;  // floats of a staged tile (16 KB of LDS)

// DIR 0: out[b][c][r][u] = in[b][r][c][u]; DIR 1: the inverse (accumulating
// into out if asked).  A tile is T consecutive r (all k blocks of each), so
// the [r][c][u] side is one contiguous run and the [c][r][u] side k runs.
template <int U, int DIR>
__global__ __launch_bounds__(BT_TH) void k_bds_regroup(const float *__restrict__ in,
                                                       float *__restrict__ out, int64_t batch,
                                                       int64_t n, int k, int T, int accumulate) {
  __shared__ float s[BT_FLOATS];
  const int kU = k * U;
  const int64_t tiles = (n + T - 1) / T;
  for (int64_t id = blockIdx.x; id < tiles * batch; id += gridDim.x) {
    const int64_t b = id / tiles, r0 = (id - b * tiles) * T;
    const int rows = (int)(n - r0 < T ? n - r0 : T);
    const int cnt = rows * kU;
    const int64_t row_major = (b * n + r0) * kU;  // [b][r0][0][0]
    if (DIR == 0) {
      for (int f = threadIdx.x; f < cnt; f += BT_TH) s[f] = in[row_major + f];
    } else {
      for (int f = threadIdx.x; f < cnt; f += BT_TH) {
        const int c = f / (rows * U), rem = f - c * (rows * U);
        const int r = rem / U, u = rem - r * U;
        s[r * kU + c * U + u] = in[((b * k + c) * n + r0) * U + rem];
      }
    }
    __syncthreads();
    if (DIR == 0) {
      for (int f = threadIdx.x; f < cnt; f += BT_TH) {
        const int c = f / (rows * U), rem = f - c * (rows * U);
        const int r = rem / U, u = rem - r * U;
        out[((b * k + c) * n + r0) * U + rem] = s[r * kU + c * U + u];
      }
    } else {
      for (int f = threadIdx.x; f < cnt; f += BT_TH) {
        const float v = s[f];
        float *o = out + row_major + f;
        *o = accumulate ? *o + v : v;
      }
    }
    __syncthreads();
  }
}

template <int U>
hipError_t regroup_u(const float *in, float *out, int64_t batch, int64_t n, int k, int dir,
                     bool accumulate, hipStream_t s) {
  const int T = BT_FLOATS / (k * U);
  const int64_t work = batch * ((n + T - 1) / T);
  const unsigned grid = (unsigned)(work < 65535 ? work : 65535);
  if (dir == 0)
    hipLaunchKernelGGL((k_bds_regroup<U, 0>), dim3(grid), dim3(BT_TH), 0, s, in, out, batch, n, k,
                       T, accumulate ? 1 : 0);
  else
    hipLaunchKernelGGL((k_bds_regroup<U, 1>), dim3(grid), dim3(BT_TH), 0, s, in, out, batch, n, k,
                       T, accumulate ? 1 : 0);
  return hipGetLastError();
}

hipError_t regroup(int q, const float *in, float *out, int64_t batch, int64_t n, int k, int dir,
                   bool accumulate, hipStream_t s) {
  if (batch == 0 || n == 0) return hipSuccess;
  switch (q) {
  case 1: return regroup_u<1>(in, out, batch, n, k, dir, accumulate, s);
  case 2: return regroup_u<4>(in, out, batch, n, k, dir, accumulate, s);
  case 3: return regroup_u<9>(in, out, batch, n, k, dir, accumulate, s);
  case 5: return regroup_u<25>(in, out, batch, n, k, dir, accumulate, s);
  }
  return hipErrorInvalidValue;
}

size_t al256(size_t x) { return (x + 255) / 256 * 256; }

}  // namespace

bool bds_supported(int q, int64_t k) {
  return (q == 1 || q == 2 || q == 3 || q == 5) && k >= 1 && k * q * q <= kBdsMaxBlockFloats;
}

size_t bds_tmp_bytes(int comb_dir, int q, int64_t k, int64_t batch, int64_t n) {
  const size_t col = al256((size_t)(batch * k * n) * q * q * 4);
  return comb_dir == 0 ? 2 * col : 3 * col;
}

hipError_t bds_fwd_launch(int q, int64_t k, int64_t batch, int64_t n, const float *M, float *P,
                          void *saved, void *ws, void *tmp, hipStream_t s) {
  const size_t col = al256((size_t)(batch * k * n) * q * q * 4);
  float *mt = static_cast<float *>(tmp);
  float *pt = reinterpret_cast<float *>(static_cast<char *>(tmp) + col);
  hipError_t e = regroup(q, M, mt, batch, n, (int)k, 0, false, s);
  if (e != hipSuccess) return e;
  float *sv = static_cast<float *>(saved);
  if (q == 1) e = scan_fwd_launch(MUL, batch * k, n, mt, nullptr, pt, nullptr, sv, nullptr, false, ws, s);
  else if (q == 2) e = scan_fwd_launch(MAT2, batch * k, n, mt, nullptr, pt, nullptr, sv, nullptr, false, ws, s);
  else e = matd_fwd_launch(q, batch * k, n, mt, pt, sv, ws, s);
  if (e != hipSuccess) return e;
  return regroup(q, pt, P, batch, n, (int)k, 1, false, s);
}

hipError_t bds_vjp_launch(int q, int64_t k, int64_t batch, int64_t n, const float *M,
                          const void *saved, const float *Pbar, float *Mbar, bool accumulate,
                          void *ws, void *tmp, hipStream_t s) {
  const size_t col = al256((size_t)(batch * k * n) * q * q * 4);
  char *t = static_cast<char *>(tmp);
  float *mt = reinterpret_cast<float *>(t);
  float *pbt = reinterpret_cast<float *>(t + col);
  float *gt = reinterpret_cast<float *>(t + 2 * col);
  hipError_t e = regroup(q, M, mt, batch, n, (int)k, 0, false, s);
  if (e == hipSuccess) e = regroup(q, Pbar, pbt, batch, n, (int)k, 0, false, s);
  if (e != hipSuccess) return e;
  const float *sv = static_cast<const float *>(saved);
  if (q == 1)
    e = scan_vjp_launch(MUL, batch * k, n, mt, nullptr, sv, nullptr, nullptr, pbt, nullptr, gt,
                        nullptr, false, ws, s);
  else if (q == 2)
    e = scan_vjp_launch(MAT2, batch * k, n, mt, nullptr, sv, nullptr, nullptr, pbt, nullptr, gt,
                        nullptr, false, ws, s);
  else
    e = matd_vjp_launch(q, batch * k, n, mt, sv, pbt, gt, false, ws, s);
  if (e != hipSuccess) return e;
  return regroup(q, gt, Mbar, batch, n, (int)k, 1, accumulate, s);
}

}  // namespace pcad
