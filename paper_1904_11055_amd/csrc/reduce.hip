// Float64 reductions over grid chunks, the tuple gather and normalisation, and the
// plan-time polygon counts.
#include "mfma_ops.h"

namespace ps {

// level 1: tmp[b][grp][e] = sum_{c in grp} part[b][c][e], or += when accumulating
// over the slabs of a streamed contraction.  With `closing_of_entry` (streamed plans
// whose operands were scaled by the slab's own maxima) the sum of an entry is unscaled
// here, with the exponents of the closing tuple it holds; entries holding no closing
// tuple are left at zero.
__global__ void reduce_chunks_f32(const float* __restrict__ part, double* __restrict__ tmp, int n_chunks,
                                  int chunks_per_group, int n_groups, long long n_ent, int accumulate,
                                  const int* __restrict__ closing_of_entry, const int* __restrict__ bins, int order,
                                  const unsigned* __restrict__ absmax, int n_shells, int prec) {
  const long long e = blockIdx.x * (long long)blockDim.x + threadIdx.x;
  const int grp = blockIdx.y;
  const int b = blockIdx.z;
  if (e >= n_ent) return;
  const int c0 = grp * chunks_per_group;
  const int c1 = min(n_chunks, c0 + chunks_per_group);
  const float* src = part + (size_t)b * n_chunks * n_ent;
  double s = 0.0;
  for (int c = c0; c < c1; ++c) s += (double)src[(size_t)c * n_ent + e];
  if (closing_of_entry != nullptr) {
    const int t = closing_of_entry[e];
    s = t < 0 ? 0.0 : ldexp(s, tuple_unscale_exp(absmax, b, n_shells, bins, t, order, prec));
  }
  double& dst = tmp[((size_t)b * n_groups + grp) * n_ent + e];
  dst = accumulate ? dst + s : s;
}

__global__ void reduce_chunks_f64(const double* __restrict__ part, double* __restrict__ tmp, int n_chunks,
                                  int chunks_per_group, int n_groups, long long n_ent) {
  const long long e = blockIdx.x * (long long)blockDim.x + threadIdx.x;
  const int grp = blockIdx.y;
  const int b = blockIdx.z;
  if (e >= n_ent) return;
  const int c0 = grp * chunks_per_group;
  const int c1 = min(n_chunks, c0 + chunks_per_group);
  const double* src = part + (size_t)b * n_chunks * n_ent;
  double s = 0.0;
  for (int c = c0; c < c1; ++c) s += src[(size_t)c * n_ent + e];
  tmp[((size_t)b * n_groups + grp) * n_ent + e] = s;
}

// S_t and B_t for every closing tuple: S = sum over groups of tmp at the tuple's
// tile entry, scaled back for FP16; B = S * fnorm (fnorm = f / (N^3 n_t)).
__global__ void gather_normalize(const double* __restrict__ tmp, int n_groups, long long n_ent,
                                 const int* __restrict__ ent_idx, const int* __restrict__ bins, int order,
                                 const double* __restrict__ fnorm, int n_closing, const unsigned* absmax,
                                 int n_shells, int prec, double* __restrict__ out, double* __restrict__ raw,
                                 int* __restrict__ nonfinite) {
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  const int b = blockIdx.y;
  if (t >= n_closing) return;
  const long long e = ent_idx[t];
  const double* src = tmp + (size_t)b * n_groups * n_ent;
  double s = 0.0;
  for (int grp = 0; grp < n_groups; ++grp) s += src[(size_t)grp * n_ent + e];
  // the scaling of the contraction's operands (absmax is null when the reduction has
  // already removed it)
  if (absmax != nullptr && (prec == kFP16 || order >= 5))
    s = ldexp(s, tuple_unscale_exp(absmax, b, n_shells, bins, t, order, prec));
  const double B = s * fnorm[t];
  out[(size_t)b * n_closing + t] = B;
  if (raw != nullptr) raw[(size_t)b * n_closing + t] = s;
  if (nonfinite != nullptr && !isfinite(B)) atomicOr(nonfinite, 1);
}

// ---------------------------------------------------------------------------
// Plan-time polygon counts in float64 over the symmetry wedge.
// C_t = sum_x prod_j c_{t_j}[x] = sum_{x in wedge} w(x) prod_j c_{t_j}[x], where
// the wedge 0 <= x0 <= x1 <= x2 <= N/2 holds one point of every orbit of the 48
// signed axis permutations (every unit-shell field is invariant under them) and
// w(x) is the orbit size.
// ---------------------------------------------------------------------------
constexpr int kCntThreads = 256;
constexpr int kCntTuples = 4;     // candidate tuples per thread
constexpr int kCntStage = 32;     // wedge points per LDS stage

// Error-free sum of two doubles: s + e == a + b exactly.
__device__ __forceinline__ void two_sum(double a, double b, double& s, double& e) {
  s = a + b;
  const double bb = s - a;
  e = (a - (s - bb)) + (b - bb);
}

// Partials are (hi, lo) pairs: the sum of each thread's terms carried with the
// rounding errors of every addition, so that counts near 10^12 (C_t near 10^20)
// still round to the right integer.
template <int ORDER>
__global__ __launch_bounds__(kCntThreads) void counts_wedge(const double* __restrict__ cw, long long nwedge,
                                                            const unsigned char* __restrict__ wmult,
                                                            const int* __restrict__ cand, int n_cand,
                                                            int n_shells, int stages_per_chunk,
                                                            double2* __restrict__ part) {
  extern __shared__ double sc[];  // [n_shells][kCntStage] + weights[kCntStage]
  double* sw = sc + (size_t)n_shells * kCntStage;
  const int chunk = blockIdx.x;
  const int tgrp = blockIdx.y;
  int sh[kCntTuples][ORDER];
  bool ok[kCntTuples];
#pragma unroll
  for (int u = 0; u < kCntTuples; ++u) {
    const int t = (tgrp * kCntTuples + u) * kCntThreads + threadIdx.x;
    ok[u] = t < n_cand;
#pragma unroll
    for (int j = 0; j < ORDER; ++j) sh[u][j] = ok[u] ? cand[t * ORDER + j] : 0;
  }
  double hi[kCntTuples] = {}, lo[kCntTuples] = {};
  const long long p0 = (long long)chunk * stages_per_chunk * kCntStage;
  for (int st = 0; st < stages_per_chunk; ++st) {
    const long long base = p0 + (long long)st * kCntStage;
    if (base >= nwedge) break;
    __syncthreads();
    for (int i = threadIdx.x; i < n_shells * kCntStage; i += kCntThreads) {
      const int s = i / kCntStage, q = i % kCntStage;
      const long long x = base + q;
      sc[i] = x < nwedge ? cw[(size_t)s * nwedge + x] : 0.0;
    }
    for (int q = threadIdx.x; q < kCntStage; q += kCntThreads)
      sw[q] = (base + q) < nwedge ? (double)wmult[base + q] : 0.0;
    __syncthreads();
    for (int q = 0; q < kCntStage; ++q) {
      const double w = sw[q];
#pragma unroll
      for (int u = 0; u < kCntTuples; ++u) {
        double v = w;
#pragma unroll
        for (int j = 0; j < ORDER; ++j) v *= sc[sh[u][j] * kCntStage + q];
        double s, e;
        two_sum(hi[u], v, s, e);
        hi[u] = s;
        lo[u] += e;
      }
    }
  }
#pragma unroll
  for (int u = 0; u < kCntTuples; ++u) {
    const int t = (tgrp * kCntTuples + u) * kCntThreads + threadIdx.x;
    if (ok[u]) part[(size_t)chunk * n_cand + t] = make_double2(hi[u], lo[u]);
  }
}

// tmp[grp][e] = sum of part[c][e] over the chunks c of group grp, as (hi, lo) pairs.
__global__ void reduce_chunks_dd(const double2* __restrict__ part, double2* __restrict__ tmp, int n_chunks,
                                 int chunks_per_group, long long n_ent) {
  const long long e = blockIdx.x * (long long)blockDim.x + threadIdx.x;
  const int grp = blockIdx.y;
  if (e >= n_ent) return;
  const int c0 = grp * chunks_per_group;
  const int c1 = min(n_chunks, c0 + chunks_per_group);
  double hi = 0.0, lo = 0.0;
  for (int c = c0; c < c1; ++c) {
    const double2 v = part[(size_t)c * n_ent + e];
    double s, err;
    two_sum(hi, v.x, s, err);
    hi = s;
    lo += err + v.y;
  }
  tmp[(size_t)grp * n_ent + e] = make_double2(hi, lo);
}

hipError_t launch_reduce_f32(const float* part, double* tmp, int n_chunks, int cpg, int n_groups, long long n_ent,
                             bool accumulate, const int* closing_of_entry, const int* bins, int order,
                             const unsigned* absmax, int n_shells, int prec, int batch, hipStream_t st) {
  dim3 grid((unsigned)((n_ent + 255) / 256), n_groups, batch);
  hipLaunchKernelGGL(reduce_chunks_f32, grid, dim3(256), 0, st, part, tmp, n_chunks, cpg, n_groups, n_ent,
                     accumulate ? 1 : 0, closing_of_entry, bins, order, absmax, n_shells, prec);
  return hipGetLastError();
}

hipError_t launch_reduce_f64(const double* part, double* tmp, int n_chunks, int cpg, int n_groups, long long n_ent,
                             int batch, hipStream_t st) {
  dim3 grid((unsigned)((n_ent + 255) / 256), n_groups, batch);
  hipLaunchKernelGGL(reduce_chunks_f64, grid, dim3(256), 0, st, part, tmp, n_chunks, cpg, n_groups, n_ent);
  return hipGetLastError();
}

hipError_t launch_gather(const double* tmp, int n_groups, long long n_ent, const int* ent_idx, const int* bins,
                         int order, const double* fnorm, int n_closing, const unsigned* absmax, int n_shells,
                         int prec, double* out, double* raw, int* nonfinite, int batch, hipStream_t st) {
  dim3 grid((n_closing + 255) / 256, batch);
  hipLaunchKernelGGL(gather_normalize, grid, dim3(256), 0, st, tmp, n_groups, n_ent, ent_idx, bins, order, fnorm,
                     n_closing, absmax, n_shells, prec, out, raw, nonfinite);
  return hipGetLastError();
}

hipError_t launch_counts_wedge(int order, const double* cw, long long nwedge, const unsigned char* wmult,
                               const int* cand, int n_cand, int n_shells, int stages_per_chunk, int n_chunks,
                               double2* part, hipStream_t st) {
  const int per_grp = kCntThreads * kCntTuples;
  dim3 grid(n_chunks, (n_cand + per_grp - 1) / per_grp);
  const size_t shm = ((size_t)n_shells * kCntStage + kCntStage) * sizeof(double);
  if (order == 2)
    hipLaunchKernelGGL(counts_wedge<2>, grid, dim3(kCntThreads), shm, st, cw, nwedge, wmult, cand, n_cand, n_shells,
                       stages_per_chunk, part);
  else if (order == 3)
    hipLaunchKernelGGL(counts_wedge<3>, grid, dim3(kCntThreads), shm, st, cw, nwedge, wmult, cand, n_cand, n_shells,
                       stages_per_chunk, part);
  else if (order == 4)
    hipLaunchKernelGGL(counts_wedge<4>, grid, dim3(kCntThreads), shm, st, cw, nwedge, wmult, cand, n_cand, n_shells,
                       stages_per_chunk, part);
  else if (order == 5)
    hipLaunchKernelGGL(counts_wedge<5>, grid, dim3(kCntThreads), shm, st, cw, nwedge, wmult, cand, n_cand, n_shells,
                       stages_per_chunk, part);
  else if (order == 6)
    hipLaunchKernelGGL(counts_wedge<6>, grid, dim3(kCntThreads), shm, st, cw, nwedge, wmult, cand, n_cand, n_shells,
                       stages_per_chunk, part);
  else
    return hipErrorInvalidValue;
  return hipGetLastError();
}

hipError_t launch_reduce_dd(const double2* part, double2* tmp, int n_chunks, int cpg, int n_groups, long long n_ent,
                            hipStream_t st) {
  dim3 grid((unsigned)((n_ent + 255) / 256), n_groups);
  hipLaunchKernelGGL(reduce_chunks_dd, grid, dim3(256), 0, st, part, tmp, n_chunks, cpg, n_ent);
  return hipGetLastError();
}

}  // namespace ps
