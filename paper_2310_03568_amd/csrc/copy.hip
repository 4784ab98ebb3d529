// Streaming device copy: the reference rate for bandwidth fractions.  A
// kernel that reads and writes each byte once cannot stream faster than a
// copy of the same bytes, so the benchmark prices its kernels against this
// copy as well as against the HBM peak.  Loads and stores carry the
// nontemporal hint, as the library's streaming kernels do (a copy with
// plain accesses measured about 10% slower).
#include "../../include/pcad.h"
#include "device.hpp"
#include "internal.hpp"

namespace pcad {
namespace {

constexpr int COPY_TH = 256;

__global__ __launch_bounds__(COPY_TH) void k_copy_stream(const int4 *__restrict__ src,
                                                         int4 *__restrict__ dst, int64_t n16) {
  typedef int v4i __attribute__((ext_vector_type(4)));
  for (int64_t i = (int64_t)blockIdx.x * COPY_TH + threadIdx.x; i < n16;
       i += (int64_t)gridDim.x * COPY_TH) {
    const v4i v = __builtin_bit_cast(v4i, ld_stream<int4>(src + i));
    __builtin_nontemporal_store(v, reinterpret_cast<v4i *>(dst + i));
  }
}

}  // namespace
}  // namespace pcad

using namespace pcad;

extern "C" int pcad_stream_copy(const void *src, void *dst, size_t bytes, void *stream) {
  if (bytes == 0) return PCAD_OK;
  if (!src || !dst) return PCAD_E_NULLPTR;
  if ((reinterpret_cast<uintptr_t>(src) | reinterpret_cast<uintptr_t>(dst)) & 15)
    return PCAD_E_MISALIGNED;
  if (bytes & 15) return PCAD_E_INVALID_ARG;
  int dev = 0, cus = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e == hipSuccess) e = hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
  if (e != hipSuccess) return hip_status(e);
  const int64_t n16 = (int64_t)(bytes / 16);
  int64_t grid = (int64_t)cus * 16;
  const int64_t need = (n16 + COPY_TH - 1) / COPY_TH;
  if (grid > need) grid = need;
  hipLaunchKernelGGL(k_copy_stream, dim3((unsigned)grid), dim3(COPY_TH), 0,
                     static_cast<hipStream_t>(stream), static_cast<const int4 *>(src),
                     static_cast<int4 *>(dst), n16);
  return hip_status(hipGetLastError());
}
