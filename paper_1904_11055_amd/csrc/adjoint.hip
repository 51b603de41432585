// Adjoint weights and the precision dispatch of the adjoint products (adjoint.h).
// The kernels of each precision are instantiated in adjoint_fp32/bf16/fp16.hip.
#include "adjoint.h"

namespace ps {

template <int PREC>
hipError_t launch_adjoint_gemm_prec(const float*, const uint4*, const int*, const unsigned*, const unsigned long long*,
                                    int, long long, float*, cplx<float>*, const cplx<float>*, Geom, int, hipStream_t);
template <int PREC>
hipError_t launch_adjoint4_gemm_prec(const float*, const uint4*, const int*, const unsigned*, const unsigned long long*,
                                     int, long long, float*, cplx<float>*, const cplx<float>*, Geom, int, hipStream_t);
extern template hipError_t launch_adjoint_gemm_prec<kFP32>(const float*, const uint4*, const int*, const unsigned*,
                                                           const unsigned long long*, int, long long, float*,
                                                           cplx<float>*, const cplx<float>*, Geom, int, hipStream_t);
extern template hipError_t launch_adjoint_gemm_prec<kBF16>(const float*, const uint4*, const int*, const unsigned*,
                                                           const unsigned long long*, int, long long, float*,
                                                           cplx<float>*, const cplx<float>*, Geom, int, hipStream_t);
extern template hipError_t launch_adjoint_gemm_prec<kFP16>(const float*, const uint4*, const int*, const unsigned*,
                                                           const unsigned long long*, int, long long, float*,
                                                           cplx<float>*, const cplx<float>*, Geom, int, hipStream_t);
extern template hipError_t launch_adjoint4_gemm_prec<kFP32>(const float*, const uint4*, const int*, const unsigned*,
                                                            const unsigned long long*, int, long long, float*,
                                                            cplx<float>*, const cplx<float>*, Geom, int, hipStream_t);
extern template hipError_t launch_adjoint4_gemm_prec<kBF16>(const float*, const uint4*, const int*, const unsigned*,
                                                            const unsigned long long*, int, long long, float*,
                                                            cplx<float>*, const cplx<float>*, Geom, int, hipStream_t);
extern template hipError_t launch_adjoint4_gemm_prec<kFP16>(const float*, const uint4*, const int*, const unsigned*,
                                                            const unsigned long long*, int, long long, float*,
                                                            cplx<float>*, const cplx<float>*, Geom, int, hipStream_t);

// dL/dB_t f / (N^3 n_t) times the number of times m occurs in t = sort(shells), or 0
// when t does not close.
template <int ORDER>
__device__ __forceinline__ double adj_weight(const double* __restrict__ grad, const double* __restrict__ fnorm,
                                             const int* __restrict__ lookup, int n_shells, int n_closing, int b,
                                             int m, const int (&rest)[ORDER - 1]) {
  int t[ORDER];
  t[0] = m;
#pragma unroll
  for (int j = 1; j < ORDER; ++j) t[j] = rest[j - 1];
#pragma unroll
  for (int a = 0; a < ORDER - 1; ++a)
#pragma unroll
    for (int c = 0; c < ORDER - 1 - a; ++c)
      if (t[c] > t[c + 1]) { const int x = t[c]; t[c] = t[c + 1]; t[c + 1] = x; }
  size_t key = 0;
#pragma unroll
  for (int j = 0; j < ORDER; ++j) key = key * n_shells + t[j];
  const int id = lookup[key];
  if (id < 0) return 0.0;
  int mult = 0;
#pragma unroll
  for (int j = 0; j < ORDER; ++j) mult += t[j] == m;
  return (double)mult * grad[(size_t)b * n_closing + id] * fnorm[id];
}

// Power-of-two exponent that the FP16 path folds into the weight of (m, rest): the
// row's scale e_m, the inverse of the rest's field scales, and for order 4 the 2^7
// that brings the triple products into range.
template <int ORDER>
__device__ __forceinline__ int adj_weight_exp(const unsigned* absmax, int b, int n_shells, const int (&rest)[ORDER - 1]) {
  int ex = ORDER == 4 ? kTripleShift : 0;
#pragma unroll
  for (int j = 0; j < ORDER - 1; ++j) ex -= shell_scale_exp(absmax, b * n_shells + rest[j]);
  return ex;
}

// FP16 only: rowmax[b][m] = max over the rests of |W[m][rest]| times the rest's scale
// factor (float64 bits; non-negative doubles order like their bit patterns).
// Order 3: grid (n_shells: v, batch), threads m; the rests (u <= v) of one v.
__global__ void adjoint_rowmax(const double* __restrict__ grad, const double* __restrict__ fnorm,
                               const int* __restrict__ lookup, int n_shells, int n_closing,
                               const unsigned* __restrict__ absmax, unsigned long long* __restrict__ rowmax) {
  const int m = threadIdx.x, v = blockIdx.x, b = blockIdx.y;
  if (m >= n_shells) return;
  double mx = 0.0;
  for (int u = 0; u <= v; ++u) {
    const int rest[2] = {u, v};
    const double w = adj_weight<3>(grad, fnorm, lookup, n_shells, n_closing, b, m, rest);
    if (w != 0.0) mx = fmax(mx, fabs(ldexp(w, adj_weight_exp<3>(absmax, b, n_shells, rest))));
  }
  if (mx > 0.0) atomicMax(rowmax + b * 64 + m, (unsigned long long)__double_as_longlong(mx));
}

// Order 4: grid (items (w, v <= w), batch), threads m; the rests (u <= v, v, w) of one item.
__global__ void adjoint4_rowmax(const double* __restrict__ grad, const double* __restrict__ fnorm,
                                const int* __restrict__ lookup, int n_shells, int n_closing,
                                const unsigned* __restrict__ absmax, unsigned long long* __restrict__ rowmax) {
  const int m = threadIdx.x, it = blockIdx.x, b = blockIdx.y;
  if (m >= n_shells) return;
  int w = 0;
  while ((w + 1) * (w + 2) / 2 <= it) ++w;
  const int v = it - w * (w + 1) / 2;
  double mx = 0.0;
  for (int u = 0; u <= v; ++u) {
    const int rest[3] = {u, v, w};
    const double x = adj_weight<4>(grad, fnorm, lookup, n_shells, n_closing, b, m, rest);
    if (x != 0.0) mx = fmax(mx, fabs(ldexp(x, adj_weight_exp<4>(absmax, b, n_shells, rest))));
  }
  if (mx > 0.0) atomicMax(rowmax + b * 64 + m, (unsigned long long)__double_as_longlong(mx));
}

// Writes one weight into its operand word: lane `ln`, element r of the hi and lo
// 16-byte words at base[ln] and base[64 + ln] (float32: values 0..3 / 4..7).
__device__ __forceinline__ void adj_store_weight(uint4* base, int ln, int r, double w, int prec) {
  if (prec == kFP32) {
    float* dst = reinterpret_cast<float*>(&base[(r < 4 ? 0 : 64) + ln]);
    dst[r & 3] = (float)w;
  } else if (prec == kBF16) {
    const float x = (float)w;
    const unsigned bits = __float_as_uint(x);
    const float h = __uint_as_float(bits & 0xffff0000u);
    reinterpret_cast<unsigned short*>(&base[ln])[r] = (unsigned short)(bits >> 16);
    reinterpret_cast<unsigned short*>(&base[64 + ln])[r] = __builtin_bit_cast(unsigned short, (__bf16)(x - h));
  } else {
    const float x = (float)w;
    const _Float16 h = (_Float16)x;
    reinterpret_cast<unsigned short*>(&base[ln])[r] = __builtin_bit_cast(unsigned short, h);
    reinterpret_cast<unsigned short*>(&base[64 + ln])[r] = __builtin_bit_cast(unsigned short, (_Float16)(x - (float)h));
  }
}

// Order 3: W in operand order, [b][v][uc][mb][hi, lo][lane]: lane l holds W[m][(u, v)]
// for m = 32 mb + l % 32 and u = 16 uc + 8 (l / 32) + r, r = 0..7 (zero when u > v).
// FP16: scaled by 2^(e_m - sigma_u - sigma_v).  grid (64: u, n_shells: v, batch), threads m.
__global__ void adjoint_weights(const double* __restrict__ grad, const double* __restrict__ fnorm,
                                const int* __restrict__ lookup, int n_shells, int n_closing, int prec,
                                const unsigned* __restrict__ absmax, const unsigned long long* __restrict__ rowmax,
                                uint4* __restrict__ W) {
  const int m = threadIdx.x, u = blockIdx.x, v = blockIdx.y, b = blockIdx.z;
  double w = 0.0;
  if (m < n_shells && u < n_shells && u <= v) {
    const int rest[2] = {u, v};
    w = adj_weight<3>(grad, fnorm, lookup, n_shells, n_closing, b, m, rest);
    if (prec == kFP16 && w != 0.0)
      w = ldexp(w, adj_row_exp(rowmax, b * 64 + m) + adj_weight_exp<3>(absmax, b, n_shells, rest));
  }
  const int uc = u >> 4, q = u & 15, hh = q >> 3, r = q & 7;
  const int ln = 32 * hh + (m & 31), mb = m >> 5;
  uint4* base = W + ((((size_t)b * n_shells + v) * 4 + uc) * kAdjMaxMb + mb) * 2 * 64;
  adj_store_weight(base, ln, r, w, prec);
}

// Order 4: W4[b][item (w, v <= w)][uc][mb][hi, lo][lane] (NC chunks of u, NC / 2 blocks
// of m: adj4_chunks): lane l holds row m = 32 mb + l % 32 and u = 16 uc + 8 (l / 32) + r
// (zero when u > v).  FP16: scaled by 2^(e_m + 7 - sigma_u - sigma_v - sigma_w).
// grid (16 NC: u, items, batch), threads m (16 NC).
__global__ void adjoint4_weights(const double* __restrict__ grad, const double* __restrict__ fnorm,
                                 const int* __restrict__ lookup, int n_shells, int n_closing, int prec,
                                 const unsigned* __restrict__ absmax, const unsigned long long* __restrict__ rowmax,
                                 uint4* __restrict__ W) {
  const int m = threadIdx.x, u = blockIdx.x, it = blockIdx.y, b = blockIdx.z;
  int w = 0;
  while ((w + 1) * (w + 2) / 2 <= it) ++w;
  const int v = it - w * (w + 1) / 2;
  double val = 0.0;
  if (m < n_shells && u < n_shells && u <= v) {
    const int rest[3] = {u, v, w};
    val = adj_weight<4>(grad, fnorm, lookup, n_shells, n_closing, b, m, rest);
    if (prec == kFP16 && val != 0.0)
      val = ldexp(val, adj_row_exp(rowmax, b * 64 + m) + adj_weight_exp<4>(absmax, b, n_shells, rest));
  }
  const int n_items = n_shells * (n_shells + 1) / 2;
  const int nc = adj4_chunks(n_shells), nm = nc / 2;
  const int uc = u >> 4, q = u & 15, hh = q >> 3, r = q & 7;
  const int ln = 32 * hh + (m & 31), mb = m >> 5;
  uint4* base = W + ((((size_t)b * n_items + it) * nc + uc) * nm + mb) * 2 * 64;
  adj_store_weight(base, ln, r, val, prec);
}

// ---------------------------------------------------------------------------
// launchers
// ---------------------------------------------------------------------------
hipError_t launch_adjoint_weights(const double* grad, const double* fnorm, const int* lookup, int n_shells,
                                  int n_closing, int prec, const unsigned* absmax, unsigned long long* rowmax,
                                  uint4* W, int batch, hipStream_t st) {
  if (n_shells > 64) return hipErrorInvalidValue;
  if (prec == kFP16) {
    hipError_t e = launch_fill_u32(rowmax, 0u, (size_t)batch * 64 * 2, st);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(adjoint_rowmax, dim3(n_shells, batch), dim3(64), 0, st, grad, fnorm, lookup, n_shells,
                       n_closing, absmax, rowmax);
  }
  hipLaunchKernelGGL(adjoint_weights, dim3(64, n_shells, batch), dim3(64), 0, st, grad, fnorm, lookup, n_shells,
                     n_closing, prec, absmax, rowmax, W);
  return hipGetLastError();
}

hipError_t launch_adjoint4_weights(const double* grad, const double* fnorm, const int* lookup, int n_shells,
                                   int n_closing, int prec, const unsigned* absmax, unsigned long long* rowmax,
                                   uint4* W, int batch, hipStream_t st) {
  if (n_shells > kAdj4MaxShells) return hipErrorInvalidValue;
  const int n_items = n_shells * (n_shells + 1) / 2;
  const int nu = 16 * adj4_chunks(n_shells);   // values of u (and of m) the operand words cover
  if (prec == kFP16) {
    hipError_t e = launch_fill_u32(rowmax, 0u, (size_t)batch * 64 * 2, st);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(adjoint4_rowmax, dim3(n_items, batch), dim3(nu), 0, st, grad, fnorm, lookup, n_shells,
                       n_closing, absmax, rowmax);
  }
  hipLaunchKernelGGL(adjoint4_weights, dim3(nu, n_items, batch), dim3(nu), 0, st, grad, fnorm, lookup, n_shells,
                     n_closing, prec, absmax, rowmax, W);
  return hipGetLastError();
}

hipError_t launch_adjoint_gemm(int prec, const float* D, const uint4* W, const int* vmask, const unsigned* absmax,
                               const unsigned long long* rowmax, int n_shells, long long G, float* A,
                               cplx<float>* H2, const cplx<float>* tw, Geom g, int batch, hipStream_t st) {
  const bool fused = adjoint_fuses_rows(g.N);
  if (fused == (H2 == nullptr) || fused == (A != nullptr) || n_shells > 64 || G % kAdjPts != 0)
    return hipErrorInvalidValue;
  if (prec == kFP32) return launch_adjoint_gemm_prec<kFP32>(D, W, vmask, absmax, rowmax, n_shells, G, A, H2, tw, g, batch, st);
  if (prec == kBF16) return launch_adjoint_gemm_prec<kBF16>(D, W, vmask, absmax, rowmax, n_shells, G, A, H2, tw, g, batch, st);
  return launch_adjoint_gemm_prec<kFP16>(D, W, vmask, absmax, rowmax, n_shells, G, A, H2, tw, g, batch, st);
}

hipError_t launch_adjoint4_gemm(int prec, const float* D, const uint4* W, const int* imask, const unsigned* absmax,
                                const unsigned long long* rowmax, int n_shells, long long G, float* A,
                                cplx<float>* H2, const cplx<float>* tw, Geom g, int batch, hipStream_t st) {
  const bool fused = adjoint_fuses_rows(g.N);
  if (fused == (H2 == nullptr) || fused == (A != nullptr) || n_shells > kAdj4MaxShells || G % kAdjPts != 0)
    return hipErrorInvalidValue;
  if (prec == kFP32) return launch_adjoint4_gemm_prec<kFP32>(D, W, imask, absmax, rowmax, n_shells, G, A, H2, tw, g, batch, st);
  if (prec == kBF16) return launch_adjoint4_gemm_prec<kBF16>(D, W, imask, absmax, rowmax, n_shells, G, A, H2, tw, g, batch, st);
  return launch_adjoint4_gemm_prec<kFP16>(D, W, imask, absmax, rowmax, n_shells, G, A, H2, tw, g, batch, st);
}

}  // namespace ps
