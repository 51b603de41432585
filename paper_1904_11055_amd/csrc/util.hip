// Small utility kernels.
#include "kernels.h"

namespace ps {

// Fills n_words 32-bit words with value (a kernel rather than hipMemsetAsync so
// that the work stays an ordinary kernel node when a caller captures the stream).
__global__ void fill_u32(unsigned* __restrict__ dst, unsigned value, size_t n) {
  size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x;
  const size_t stride = (size_t)gridDim.x * blockDim.x;
  for (; i < n; i += stride) dst[i] = value;
}

hipError_t launch_fill_u32(void* dst, unsigned value, size_t n_words, hipStream_t st) {
  if (n_words == 0) return hipSuccess;
  size_t blocks = (n_words + 255) / 256;
  if (blocks > 65536) blocks = 65536;
  hipLaunchKernelGGL(fill_u32, dim3((unsigned)blocks), dim3(256), 0, st, (unsigned*)dst, value, n_words);
  return hipGetLastError();
}

}  // namespace ps
