// Product-sum contraction of shell fields on the matrix cores (gfx950).
//
// S_t = sum_x prod_j d_{t_j}[x] for sorted tuples t (the grid sum of products of
// the shell fields I_k, Sec. 2 and Appendix A) is evaluated as a batch of small
// GEMMs whose reduction dimension is the grid:
//   n = 3:  S[(i,j), k] = sum_x (d_i d_j)[x] d_k[x]     rows: pairs, cols: shells
//   n = 4:  S[(i,j), (k,l)] = sum_x (d_i d_j)[x] (d_k d_l)[x]
//   n = 2:  S[i, k] = sum_x d_i[x] d_k[x]
// Pair products are formed in registers from an LDS-staged slice of the fields
// and never stored.  Only 16x16 output tiles that hold a candidate tuple run.
//
// One workgroup (8 waves) owns a contiguous chunk of grid points and every tile;
// each wave owns up to kSlots tiles whose accumulators stay in registers for the
// whole chunk.  The chunk's float32 partial sums go to memory and are summed over
// chunks in float64, in a fixed order (bitwise reproducible).
//
// Arithmetic per 16x16 tile and 32 grid points:
//   FP32        eight v_mfma_f32_16x16x4_f32 on the float32 values,
//   SPLIT_BF16  x = hi + lo (bf16 each), hi*hi + hi*lo + lo*hi with three
//               v_mfma_f32_16x16x32_bf16, float32 accumulation,
//   SPLIT_FP16  the same with f16 after a power-of-two scaling of every shell.
#include "common.h"
#include "kernels.h"

namespace ps {

typedef __attribute__((__vector_size__(8 * sizeof(__bf16)))) __bf16 bf16x8;
typedef __attribute__((__vector_size__(8 * sizeof(_Float16)))) _Float16 f16x8;
typedef __attribute__((__vector_size__(4 * sizeof(float)))) float f32x4;

enum { kFP32 = 0, kBF16 = 1, kFP16 = 2 };

constexpr int kCtrWaves = 8;
constexpr int kCtrThreads = 64 * kCtrWaves;
constexpr int kSlots = 32;       // tiles per wave
constexpr int kKStep = 32;       // grid points per LDS stage
constexpr int kRowStride = 36;   // floats per staged field row (32 + 4 pad)
constexpr int kMaxBlk = 4;       // shell blocks of 16 (n_shells <= 64)
constexpr int kFp16Top = 14;     // |scaled shell value| < 2^15
constexpr int kPairShift = 15;   // pair products are scaled down by 2^15 in FP16 mode

template <int PREC>
struct Operand;
template <>
struct Operand<kFP32> {
  float v[8];
};
template <>
struct Operand<kBF16> {
  bf16x8 hi, lo;
};
template <>
struct Operand<kFP16> {
  f16x8 hi, lo;
};

template <int PREC>
__device__ __forceinline__ Operand<PREC> make_operand(const float (&x)[8], float scale) {
  Operand<PREC> o;
  if constexpr (PREC == kFP32) {
#pragma unroll
    for (int r = 0; r < 8; ++r) o.v[r] = x[r];
  } else if constexpr (PREC == kBF16) {
#pragma unroll
    for (int r = 0; r < 8; ++r) {
      const unsigned bits = __float_as_uint(x[r]);
      const float h = __uint_as_float(bits & 0xffff0000u);  // truncation: exact bf16
      o.hi[r] = __builtin_bit_cast(__bf16, (unsigned short)(bits >> 16));
      o.lo[r] = (__bf16)(x[r] - h);                          // exact residual, rounded once
    }
  } else {
#pragma unroll
    for (int r = 0; r < 8; ++r) {
      const float y = x[r] * scale;
      const _Float16 h = (_Float16)y;
      o.hi[r] = h;
      o.lo[r] = (_Float16)(y - (float)h);
    }
  }
  return o;
}

template <int PREC>
__device__ __forceinline__ void mma(f32x4& acc, const Operand<PREC>& a, const Operand<PREC>& b) {
  if constexpr (PREC == kFP32) {
#pragma unroll
    for (int r = 0; r < 8; ++r) acc = __builtin_amdgcn_mfma_f32_16x16x4f32(a.v[r], b.v[r], acc, 0, 0, 0);
  } else if constexpr (PREC == kBF16) {
    acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a.hi, b.hi, acc, 0, 0, 0);
    acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a.hi, b.lo, acc, 0, 0, 0);
    acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a.lo, b.hi, acc, 0, 0, 0);
  } else {
    acc = __builtin_amdgcn_mfma_f32_16x16x32_f16(a.hi, b.hi, acc, 0, 0, 0);
    acc = __builtin_amdgcn_mfma_f32_16x16x32_f16(a.hi, b.lo, acc, 0, 0, 0);
    acc = __builtin_amdgcn_mfma_f32_16x16x32_f16(a.lo, b.hi, acc, 0, 0, 0);
  }
}

// Lane l of a 16x16x32 operand holds row (l % 16) at grid points 8 (l / 16) .. +7
// of the current 32-point stage (the same K mapping for both operands).
__device__ __forceinline__ void load_row8(const float* lds_row, int g, float (&x)[8]) {
  const float4 a = *reinterpret_cast<const float4*>(lds_row + 8 * g);
  const float4 b = *reinterpret_cast<const float4*>(lds_row + 8 * g + 4);
  x[0] = a.x; x[1] = a.y; x[2] = a.z; x[3] = a.w;
  x[4] = b.x; x[5] = b.y; x[6] = b.z; x[7] = b.w;
}

// Slot word: bits 0..11 A block, 12..23 B block, bit 24 "form A" (A block differs
// from the previous valid slot's), bit 31 set = empty slot.
struct SlotWord {
  int w;
  __device__ __forceinline__ bool empty() const { return w < 0; }
  __device__ __forceinline__ int ablk() const { return w & 0xfff; }
  __device__ __forceinline__ int bblk() const { return (w >> 12) & 0xfff; }
  __device__ __forceinline__ bool form() const { return (w >> 24) & 1; }
};


__device__ __forceinline__ int fp16_shell_exp(const unsigned* absmax, int idx) {
  const float m = __uint_as_float(absmax[idx]);
  if (!(m > 0.f)) return 0;
  return kFp16Top - ilogbf(m);
}

// ORDER 2: A = shell block, B = shell block;  ORDER 3: A = pair block, B = shell
// block;  ORDER 4: A = pair block, B = pair block.
template <int PREC, int ORDER>
__global__ __launch_bounds__(kCtrThreads, 1) void contract_tiles(CtrParams p) {
  __shared__ __attribute__((aligned(16))) float stage[2][(kMaxBlk * 16 + 1) * kRowStride];
  __shared__ int lds_pairs[2080 + 16];
  __shared__ float lds_scale[kMaxBlk * 16 + 1];

  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int g = lane >> 4;   // which 8-point group of the stage
  const int row = lane & 15;
  const int chunk = blockIdx.x;
  const int group = blockIdx.y;
  const int b = blockIdx.z;
  const int nrows = p.n_blk * 16;   // staged shell rows (zero beyond n_shells)
  const int zrow = nrows;           // all-zero row used by padded pairs

  if (ORDER >= 3) {
    for (int i = tid; i < p.n_pairs_padded; i += kCtrThreads) lds_pairs[i] = p.pair_uv[i];
  }
  if (PREC == kFP16) {
    for (int i = tid; i <= nrows; i += kCtrThreads) {
      float sc = 0.f;
      if (i < p.n_shells) sc = ldexpf(1.0f, fp16_shell_exp(p.absmax, b * p.n_shells + i));
      lds_scale[i] = sc;
    }
  }
  // zero rows (padding shells and the zero row) of both stage buffers
  for (int i = tid; i < 2 * (nrows + 1) * kRowStride; i += kCtrThreads) {
    const int buf = i / ((nrows + 1) * kRowStride);
    const int rr = (i / kRowStride) % (nrows + 1);
    if (rr >= p.n_shells) stage[buf][i % ((nrows + 1) * kRowStride)] = 0.f;
  }

  SlotWord sw[kSlots];
  const int* my_slots = p.slots + ((size_t)group * kCtrWaves + wave) * kSlots;
#pragma unroll
  for (int s = 0; s < kSlots; ++s) sw[s].w = __builtin_amdgcn_readfirstlane(my_slots[s]);

  f32x4 acc[kSlots];
#pragma unroll
  for (int s = 0; s < kSlots; ++s) acc[s] = f32x4{0.f, 0.f, 0.f, 0.f};

  // global -> LDS staging: thread t moves float4 #t of the (n_shells x 32) slice
  const float* Db = p.D + (size_t)b * p.n_shells * p.G;
  const long long x_base = (long long)chunk * p.ksteps * kKStep;
  const int st_row = tid >> 3, st_col = (tid & 7) * 4;
  const bool st_active = st_row < p.n_shells;
  float4 pre = make_float4(0.f, 0.f, 0.f, 0.f);
  if (st_active) pre = *reinterpret_cast<const float4*>(Db + (size_t)st_row * p.G + x_base + st_col);
  __syncthreads();
  if (st_active) *reinterpret_cast<float4*>(&stage[0][st_row * kRowStride + st_col]) = pre;
  __syncthreads();

  for (int ks = 0; ks < p.ksteps; ++ks) {
    const int cur = ks & 1;
    if (ks + 1 < p.ksteps && st_active)
      pre = *reinterpret_cast<const float4*>(Db + (size_t)st_row * p.G + x_base + (ks + 1) * kKStep + st_col);
    const float* S = stage[cur];

    // shell-block operands used as B (ORDER 2, 3) or A (ORDER 2)
    Operand<PREC> sb[kMaxBlk];
    if (ORDER <= 3) {
#pragma unroll
      for (int kb = 0; kb < kMaxBlk; ++kb) {
        if (kb < p.n_blk) {
          float x[8];
          load_row8(S + (kb * 16 + row) * kRowStride, g, x);
          sb[kb] = make_operand<PREC>(x, PREC == kFP16 ? lds_scale[kb * 16 + row] : 1.f);
        }
      }
    }

    Operand<PREC> A;
#pragma unroll
    for (int s = 0; s < kSlots; ++s) {
      if (sw[s].empty()) continue;
      if (ORDER == 2) {
        const int ab = sw[s].ablk(), bb = sw[s].bblk();
        Operand<PREC> a2, b2;
        switch (ab) {
          case 0: a2 = sb[0]; break;
          case 1: a2 = sb[1]; break;
          case 2: a2 = sb[2]; break;
          default: a2 = sb[3]; break;
        }
        switch (bb) {
          case 0: b2 = sb[0]; break;
          case 1: b2 = sb[1]; break;
          case 2: b2 = sb[2]; break;
          default: b2 = sb[3]; break;
        }
        mma<PREC>(acc[s], a2, b2);
        continue;
      }
      if (sw[s].form()) {
        const int uv = lds_pairs[sw[s].ablk() * 16 + row];
        const int u = uv & 0xffff, v = uv >> 16;
        float x[8], y[8];
        load_row8(S + u * kRowStride, g, x);
        load_row8(S + v * kRowStride, g, y);
#pragma unroll
        for (int r = 0; r < 8; ++r) x[r] *= y[r];
        float sc = 1.f;
        if (PREC == kFP16) sc = lds_scale[u] * lds_scale[v] * (1.0f / (float)(1 << kPairShift));
        A = make_operand<PREC>(x, sc);
      }
      if (ORDER == 3) {
        switch (sw[s].bblk()) {
          case 0: mma<PREC>(acc[s], A, sb[0]); break;
          case 1: mma<PREC>(acc[s], A, sb[1]); break;
          case 2: mma<PREC>(acc[s], A, sb[2]); break;
          default: mma<PREC>(acc[s], A, sb[3]); break;
        }
      } else {  // ORDER 4: B is a pair block too
        const int uv = lds_pairs[sw[s].bblk() * 16 + row];
        const int u = uv & 0xffff, v = uv >> 16;
        float x[8], y[8];
        load_row8(S + u * kRowStride, g, x);
        load_row8(S + v * kRowStride, g, y);
#pragma unroll
        for (int r = 0; r < 8; ++r) x[r] *= y[r];
        float sc = 1.f;
        if (PREC == kFP16) sc = lds_scale[u] * lds_scale[v] * (1.0f / (float)(1 << kPairShift));
        const Operand<PREC> Bp = make_operand<PREC>(x, sc);
        mma<PREC>(acc[s], A, Bp);
      }
    }
    if (ks + 1 < p.ksteps && st_active)
      *reinterpret_cast<float4*>(&stage[cur ^ 1][st_row * kRowStride + st_col]) = pre;
    __syncthreads();
  }

  // dump accumulators: tile t, lane l, register r -> partials[..][t][4 l + r]
  const int* my_tiles = p.slot_tile + ((size_t)group * kCtrWaves + wave) * kSlots;
  float* out = p.partials + ((size_t)b * p.n_chunks + chunk) * (size_t)p.n_tiles * 256;
#pragma unroll
  for (int s = 0; s < kSlots; ++s) {
    if (sw[s].empty()) continue;
    const int t = my_tiles[s];
    *reinterpret_cast<f32x4*>(out + (size_t)t * 256 + 4 * lane) = acc[s];
  }
}

// Sum float32 partials over chunk ranges in float64, fixed order.
// level 1: tmp[b][grp][e] = sum_{c in grp} part[b][c][e]
__global__ void reduce_chunks_f32(const float* __restrict__ part, double* __restrict__ tmp, int n_chunks,
                                  int chunks_per_group, int n_groups, long long n_ent) {
  const long long e = blockIdx.x * (long long)blockDim.x + threadIdx.x;
  const int grp = blockIdx.y;
  const int b = blockIdx.z;
  if (e >= n_ent) return;
  const int c0 = grp * chunks_per_group;
  const int c1 = min(n_chunks, c0 + chunks_per_group);
  const float* src = part + (size_t)b * n_chunks * n_ent;
  double s = 0.0;
  for (int c = c0; c < c1; ++c) s += (double)src[(size_t)c * n_ent + e];
  tmp[((size_t)b * n_groups + grp) * n_ent + e] = s;
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
  if (prec == kFP16) {
    int ex = 0;
    for (int j = 0; j < order; ++j) ex += fp16_shell_exp(absmax, b * n_shells + bins[t * order + j]);
    if (order == 3) ex -= kPairShift;
    if (order == 4) ex -= 2 * kPairShift;
    s = ldexp(s, -ex);
  }
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

template <int ORDER>
__global__ __launch_bounds__(kCntThreads) void counts_wedge(const double* __restrict__ cw, long long nwedge,
                                                            const unsigned char* __restrict__ wmult,
                                                            const int* __restrict__ cand, int n_cand,
                                                            int n_shells, int stages_per_chunk,
                                                            double* __restrict__ part) {
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
  double acc[kCntTuples] = {};
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
        acc[u] += v;
      }
    }
  }
#pragma unroll
  for (int u = 0; u < kCntTuples; ++u) {
    const int t = (tgrp * kCntTuples + u) * kCntThreads + threadIdx.x;
    if (ok[u]) part[(size_t)chunk * n_cand + t] = acc[u];
  }
}

// ---------------------------------------------------------------------------
// Adjoint (order 3).  W[b][m][pair] = mult * dL/dB_t * fnorm_t with t = sort(m, u, v)
// and mult the number of times m occurs in t; then a_m[x] = sum_pairs W[m][pair]
// (d_u d_v)[x] on the matrix cores.
// ---------------------------------------------------------------------------
__global__ void adjoint_weights(const double* __restrict__ grad, const double* __restrict__ fnorm,
                                const int* __restrict__ lookup /*[nb^3] closing index or -1*/,
                                const int* __restrict__ pair_uv, int n_pairs, int n_pairs_padded,
                                int n_shells, int n_closing, float* __restrict__ W) {
  const int pidx = blockIdx.x * blockDim.x + threadIdx.x;
  const int m = blockIdx.y;
  const int b = blockIdx.z;
  if (pidx >= n_pairs_padded) return;
  float w = 0.f;
  if (pidx < n_pairs) {
    const int uv = pair_uv[pidx];
    int t0 = m, t1 = uv & 0xffff, t2 = uv >> 16;
    // sort three values
    if (t0 > t1) { int tmp = t0; t0 = t1; t1 = tmp; }
    if (t1 > t2) { int tmp = t1; t1 = t2; t2 = tmp; }
    if (t0 > t1) { int tmp = t0; t0 = t1; t1 = tmp; }
    const int id = lookup[(t0 * n_shells + t1) * n_shells + t2];
    if (id >= 0) {
      const int mult = (t0 == m) + (t1 == m) + (t2 == m);
      w = (float)((double)mult * grad[(size_t)b * n_closing + id] * fnorm[id]);
    }
  }
  W[((size_t)b * n_shells + m) * n_pairs_padded + pidx] = w;
}

// a[b][m][x]: one workgroup = 8 waves = 128 grid points (each wave 16 points) and
// all shells m (blocks of 16).  Reduction over pairs in chunks of 32.
constexpr int kAdjWaves = 8;
constexpr int kAdjPts = 16 * kAdjWaves;
constexpr int kAdjStride = kAdjPts + 4;

template <int PREC>
__global__ __launch_bounds__(64 * kAdjWaves, 1) void adjoint_gemm(const float* __restrict__ D,
                                                                  const float* __restrict__ W,
                                                                  const unsigned char* __restrict__ wmask,
                                                                  const int* __restrict__ pair_uv,
                                                                  int n_pairs_padded, int n_shells, int n_blk,
                                                                  long long G, float* __restrict__ A) {
  __shared__ __attribute__((aligned(16))) float fld[(kMaxBlk * 16 + 1) * kAdjStride];
  __shared__ __attribute__((aligned(16))) float wch[kMaxBlk * 16][32 + 4];
  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const int wave = tid >> 6;
  const int g = lane >> 4, col = lane & 15;
  const int b = blockIdx.y;
  const long long x0 = (long long)blockIdx.x * kAdjPts;
  const int zrow = n_blk * 16;
  const float* Db = D + (size_t)b * n_shells * G;
  for (int i = tid; i < (zrow + 1) * kAdjPts; i += 64 * kAdjWaves) {
    const int s = i / kAdjPts, q = i % kAdjPts;
    fld[s * kAdjStride + q] = (s < n_shells) ? Db[(size_t)s * G + x0 + q] : 0.f;
  }
  f32x4 acc[kMaxBlk];
#pragma unroll
  for (int mb = 0; mb < kMaxBlk; ++mb) acc[mb] = f32x4{0.f, 0.f, 0.f, 0.f};
  const float* Wb = W + (size_t)b * n_shells * n_pairs_padded;
  const int n_kc = n_pairs_padded / 32;
  const int my_pt = wave * 16 + col;  // this lane's grid point (B column)
  for (int kc = 0; kc < n_kc; ++kc) {
    __syncthreads();
    for (int i = tid; i < zrow * 32; i += 64 * kAdjWaves) {
      const int m = i / 32, q = i % 32;
      wch[m][q] = (m < n_shells) ? Wb[(size_t)m * n_pairs_padded + kc * 32 + q] : 0.f;
    }
    __syncthreads();
    bool any = false;
#pragma unroll
    for (int mb = 0; mb < kMaxBlk; ++mb) any |= (mb < n_blk) && wmask[kc * kMaxBlk + mb];
    if (!any) continue;
    // B operand: pair products of pairs kc*32 + 8g + r at this lane's point
    float x[8];
#pragma unroll
    for (int r = 0; r < 8; ++r) {
      const int uv = pair_uv[kc * 32 + 8 * g + r];
      const int u = uv & 0xffff, v = uv >> 16;
      x[r] = fld[u * kAdjStride + my_pt] * fld[v * kAdjStride + my_pt];
    }
    const Operand<PREC> Bop = make_operand<PREC>(x, 1.f);
#pragma unroll
    for (int mb = 0; mb < kMaxBlk; ++mb) {
      if (mb >= n_blk || !wmask[kc * kMaxBlk + mb]) continue;
      float w8[8];
      load_row8(&wch[mb * 16 + col][0], g, w8);
      const Operand<PREC> Aop = make_operand<PREC>(w8, 1.f);
      mma<PREC>(acc[mb], Aop, Bop);
    }
  }
  // acc[mb]: lane l, reg r -> row m = 16 mb + 4 (l / 16) + r, column = point l % 16
  float* Ab = A + (size_t)b * n_shells * G;
#pragma unroll
  for (int mb = 0; mb < kMaxBlk; ++mb) {
    if (mb >= n_blk) continue;
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int m = mb * 16 + 4 * g + r;
      if (m < n_shells) Ab[(size_t)m * G + x0 + wave * 16 + col] = acc[mb][r];
    }
  }
}

// ---------------------------------------------------------------------------
// launchers
// ---------------------------------------------------------------------------
hipError_t launch_contract(int prec, int order, const CtrParams& p, int n_groups, int batch, hipStream_t st) {
  dim3 grid(p.n_chunks, n_groups, batch);
#define L(P, O) hipLaunchKernelGGL((contract_tiles<P, O>), grid, dim3(kCtrThreads), 0, st, p)
  if (order == 2) {
    if (prec == kFP32) L(kFP32, 2); else if (prec == kBF16) L(kBF16, 2); else L(kFP16, 2);
  } else if (order == 3) {
    if (prec == kFP32) L(kFP32, 3); else if (prec == kBF16) L(kBF16, 3); else L(kFP16, 3);
  } else {
    if (prec == kFP32) L(kFP32, 4); else if (prec == kBF16) L(kBF16, 4); else L(kFP16, 4);
  }
#undef L
  return hipGetLastError();
}

hipError_t launch_reduce_f32(const float* part, double* tmp, int n_chunks, int cpg, int n_groups, long long n_ent,
                             int batch, hipStream_t st) {
  dim3 grid((unsigned)((n_ent + 255) / 256), n_groups, batch);
  hipLaunchKernelGGL(reduce_chunks_f32, grid, dim3(256), 0, st, part, tmp, n_chunks, cpg, n_groups, n_ent);
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
                               double* part, hipStream_t st) {
  const int per_grp = kCntThreads * kCntTuples;
  dim3 grid(n_chunks, (n_cand + per_grp - 1) / per_grp);
  const size_t shm = ((size_t)n_shells * kCntStage + kCntStage) * sizeof(double);
  if (order == 2)
    hipLaunchKernelGGL(counts_wedge<2>, grid, dim3(kCntThreads), shm, st, cw, nwedge, wmult, cand, n_cand, n_shells,
                       stages_per_chunk, part);
  else if (order == 3)
    hipLaunchKernelGGL(counts_wedge<3>, grid, dim3(kCntThreads), shm, st, cw, nwedge, wmult, cand, n_cand, n_shells,
                       stages_per_chunk, part);
  else
    hipLaunchKernelGGL(counts_wedge<4>, grid, dim3(kCntThreads), shm, st, cw, nwedge, wmult, cand, n_cand, n_shells,
                       stages_per_chunk, part);
  return hipGetLastError();
}

hipError_t launch_adjoint_weights(const double* grad, const double* fnorm, const int* lookup, const int* pair_uv,
                                  int n_pairs, int n_pairs_padded, int n_shells, int n_closing, float* W, int batch,
                                  hipStream_t st) {
  dim3 grid((n_pairs_padded + 255) / 256, n_shells, batch);
  hipLaunchKernelGGL(adjoint_weights, grid, dim3(256), 0, st, grad, fnorm, lookup, pair_uv, n_pairs, n_pairs_padded,
                     n_shells, n_closing, W);
  return hipGetLastError();
}

hipError_t launch_adjoint_gemm(int prec, const float* D, const float* W, const unsigned char* wmask,
                               const int* pair_uv, int n_pairs_padded, int n_shells, int n_blk, long long G,
                               float* A, int batch, hipStream_t st) {
  dim3 grid((unsigned)(G / kAdjPts), batch);
  if (prec == kFP32)
    hipLaunchKernelGGL(adjoint_gemm<kFP32>, grid, dim3(64 * kAdjWaves), 0, st, D, W, wmask, pair_uv, n_pairs_padded,
                       n_shells, n_blk, G, A);
  else
    hipLaunchKernelGGL(adjoint_gemm<kBF16>, grid, dim3(64 * kAdjWaves), 0, st, D, W, wmask, pair_uv, n_pairs_padded,
                       n_shells, n_blk, G, A);
  return hipGetLastError();
}

}  // namespace ps
