// Small utility kernels, and the library's static device scratch.
#include <mutex>

#include "kernels.h"

namespace ps {

// Workspace of polyspec_forward_static (for callers that cannot allocate): a
// file-scope device array, one copy per GPU, held until the process ends.  Host code
// never passes this name to a kernel (on the host it is only a stand-in); it uses
// the device address that static_scratch_address() looks up once per device.
static __device__ __align__(256) unsigned char scratch[kStaticScratchBytes];

hipError_t static_scratch_address(int device, void** ptr) {
  static std::mutex mu;
  static void* addr[kMaxDevices] = {};
  if (device < 0 || device >= kMaxDevices) return hipErrorInvalidDevice;
  std::lock_guard<std::mutex> lock(mu);
  if (addr[device] == nullptr) {
    int cur = -1;
    hipError_t e = hipGetDevice(&cur);
    if (e != hipSuccess) return e;
    if (cur != device) return hipErrorInvalidDevice;   // the lookup runs with `device` current
    void* a = nullptr;
    e = hipGetSymbolAddress(&a, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    addr[device] = a;
  }
  *ptr = addr[device];
  return hipSuccess;
}

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

// Partial maxima of |x| over each field z of length G (float bits), spread over
// spread words per field; reduce_absmax then takes the maximum of each field's words.
__global__ void fields_absmax(const float* __restrict__ x, long long G, unsigned* __restrict__ part, int spread) {
  const int z = blockIdx.y;
  const float* f = x + (size_t)z * G;
  float m = 0.f;
  for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < G; i += (long long)gridDim.x * blockDim.x)
    m = fmaxf(m, fabsf(f[i]));
  for (int off = 32; off > 0; off >>= 1) m = fmaxf(m, __shfl_xor(m, off));
  if ((threadIdx.x & 63) == 0) atomicMax(part + (size_t)z * spread + (blockIdx.x % spread), __float_as_uint(m));
}

hipError_t launch_fields_absmax(const float* x, long long G, int nz, unsigned* part, int spread, hipStream_t st) {
  hipLaunchKernelGGL(fields_absmax, dim3(1024, nz), dim3(256), 0, st, x, G, part, spread);
  return hipGetLastError();
}

}  // namespace ps
