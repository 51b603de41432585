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
#include <utility>

#include "common.h"
#include "fft_core.h"
#include "kernels.h"

namespace ps {

// Calls f(std::integral_constant<int, i>) for i = 0 .. N-1: loop bodies with
// compile-time indices (static register arrays) without relying on unrolling.
template <typename F, int... I>
__device__ __forceinline__ void static_for_impl(F&& f, std::integer_sequence<int, I...>) {
  (f(std::integral_constant<int, I>{}), ...);
}
template <int N, typename F>
__device__ __forceinline__ void static_for(F&& f) {
  static_for_impl(f, std::make_integer_sequence<int, N>{});
}

typedef __attribute__((__vector_size__(8 * sizeof(__bf16)))) __bf16 bf16x8;
typedef __attribute__((__vector_size__(8 * sizeof(_Float16)))) _Float16 f16x8;
typedef __attribute__((__vector_size__(4 * sizeof(float)))) float f32x4;

enum { kFP32 = 0, kBF16 = 1, kFP16 = 2 };

constexpr int kCtrWaves = 16;
constexpr int kCtrThreads = 64 * kCtrWaves;
constexpr int kSlots = 14;       // tiles per wave (order 3)
constexpr int kSlots4 = 10;      // tiles per wave (order 4: B rows formed too)
constexpr int kSlots56 = 8;      // tiles per wave (order 5: triple rows formed)
constexpr int kSlots6 = 7;       // tiles per wave (order 6: triples on both sides; 8 would spill)
constexpr int kSlotsMax = 16;    // stride of the per-wave slot tables
constexpr int kKStep = 64;       // grid points per LDS stage (two MFMA K-steps)
constexpr int kRowStride = 68;   // floats per staged field row (64 + 4 pad)
constexpr int kMaxBlk = 4;       // shell blocks of 16 (n_shells <= 64)
constexpr int kFp16Top = 6;      // |scaled shell value| < 2^7, so pair products stay below 2^14
constexpr int kTripleShift = 7;  // FP16: triple products (< 2^21) are scaled by 2^-7 into range

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



__device__ __forceinline__ int shell_scale_exp(const unsigned* absmax, int idx) {
  const float m = __uint_as_float(absmax[idx]);
  if (!(m > 0.f)) return 0;
  return kFp16Top - ilogbf(m);
}

// Operands in LDS: for each 16-row block, lane l's eight values (rows l % 16,
// points 8 (l / 16) .. +7) as two 16-byte halves -- hi / lo for the split
// precisions, values 0..3 / 4..7 for float32 -- stored in separate arrays so
// consecutive lanes read consecutive 16-byte words.
template <int PREC>
__device__ __forceinline__ Operand<PREC> op_from_words(uint4 h, uint4 l) {
  Operand<PREC> o;
  if constexpr (PREC == kFP32) {
    o.v[0] = __uint_as_float(h.x); o.v[1] = __uint_as_float(h.y);
    o.v[2] = __uint_as_float(h.z); o.v[3] = __uint_as_float(h.w);
    o.v[4] = __uint_as_float(l.x); o.v[5] = __uint_as_float(l.y);
    o.v[6] = __uint_as_float(l.z); o.v[7] = __uint_as_float(l.w);
  } else if constexpr (PREC == kBF16) {
    o.hi = __builtin_bit_cast(bf16x8, h);
    o.lo = __builtin_bit_cast(bf16x8, l);
  } else {
    o.hi = __builtin_bit_cast(f16x8, h);
    o.lo = __builtin_bit_cast(f16x8, l);
  }
  return o;
}

// Split four consecutive values of one operand lane into 8-byte hi and lo words.
template <int PREC>
__device__ __forceinline__ void split4(float4 v, float scale, uint2& hi, uint2& lo) {
  if constexpr (PREC == kBF16) {
    const unsigned b0 = __float_as_uint(v.x), b1 = __float_as_uint(v.y);
    const unsigned b2 = __float_as_uint(v.z), b3 = __float_as_uint(v.w);
    hi.x = (b0 >> 16) | (b1 & 0xffff0000u);
    hi.y = (b2 >> 16) | (b3 & 0xffff0000u);
    const __bf16 l0 = (__bf16)(v.x - __uint_as_float(b0 & 0xffff0000u));
    const __bf16 l1 = (__bf16)(v.y - __uint_as_float(b1 & 0xffff0000u));
    const __bf16 l2 = (__bf16)(v.z - __uint_as_float(b2 & 0xffff0000u));
    const __bf16 l3 = (__bf16)(v.w - __uint_as_float(b3 & 0xffff0000u));
    lo.x = (unsigned)__builtin_bit_cast(unsigned short, l0) | ((unsigned)__builtin_bit_cast(unsigned short, l1) << 16);
    lo.y = (unsigned)__builtin_bit_cast(unsigned short, l2) | ((unsigned)__builtin_bit_cast(unsigned short, l3) << 16);
  } else {
    const float y[4] = {v.x * scale, v.y * scale, v.z * scale, v.w * scale};
    unsigned short hs[4], ls[4];
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const _Float16 h = (_Float16)y[r];
      hs[r] = __builtin_bit_cast(unsigned short, h);
      ls[r] = __builtin_bit_cast(unsigned short, (_Float16)(y[r] - (float)h));
    }
    hi.x = hs[0] | ((unsigned)hs[1] << 16);
    hi.y = hs[2] | ((unsigned)hs[3] << 16);
    lo.x = ls[0] | ((unsigned)ls[1] << 16);
    lo.y = ls[2] | ((unsigned)ls[3] << 16);
  }
}

template <int PREC>
__device__ __forceinline__ Operand<PREC> form_pair(const float* S, int uv, int g) {
  const int u = uv & 0xff, v = (uv >> 8) & 0xff;
  float x[8], y[8];
  load_row8(S + u * kRowStride, g, x);
  load_row8(S + v * kRowStride, g, y);
#pragma unroll
  for (int r = 0; r < 8; ++r) x[r] *= y[r];
  return make_operand<PREC>(x, 1.f);
}

// Product of NF staged shell rows (shell indices in the bytes of w), split for the
// matrix cores.  In FP16 a triple of scaled values can reach 2^21, beyond the
// format's range, so it enters the split scaled by 2^-kTripleShift (removed in FP64
// with the other scale factors).
template <int PREC, int NF>
__device__ __forceinline__ Operand<PREC> form_rows(const float* S, int w, int g) {
  float x[8], y[8];
  load_row8(S + (w & 0xff) * kRowStride, g, x);
#pragma unroll
  for (int f = 1; f < NF; ++f) {
    load_row8(S + ((w >> (8 * f)) & 0xff) * kRowStride, g, y);
#pragma unroll
    for (int r = 0; r < 8; ++r) x[r] *= y[r];
  }
  return make_operand<PREC>(x, NF == 3 ? 1.0f / (1 << kTripleShift) : 1.0f);
}

// FP16 pair product straight from the split operand words of its two shell rows,
// with packed half-precision error-free products: p_hi = fl(u_hi v_hi), its rounding
// error e = u_hi v_hi - p_hi exactly (one fused multiply-add), and
// p_lo = fl(u_hi v_lo + u_lo v_hi + e).  The dropped u_lo v_lo and the rounding of
// p_lo are both about 2^-22 of the product.  Row r of shell block kb at point group
// g sits at word [kb][16 g + r % 16] of the operand arrays.
typedef __attribute__((__vector_size__(2 * sizeof(_Float16)))) _Float16 f16x2;
__device__ __forceinline__ Operand<kFP16> form_pair_f16(const uint4 (*hi)[64], const uint4 (*lo)[64], int uv,
                                                        int lane) {
  const int u = uv & 0xff, v = (uv >> 8) & 0xff;
  const int iu = (lane & 0x30) | (u & 15), iv = (lane & 0x30) | (v & 15);
  const f16x8 uh = __builtin_bit_cast(f16x8, hi[u >> 4][iu]);
  const f16x8 ul = __builtin_bit_cast(f16x8, lo[u >> 4][iu]);
  const f16x8 vh = __builtin_bit_cast(f16x8, hi[v >> 4][iv]);
  const f16x8 vl = __builtin_bit_cast(f16x8, lo[v >> 4][iv]);
  Operand<kFP16> o;
  o.hi = uh * vh;
  const f16x8 e = __builtin_elementwise_fma(uh, vh, -o.hi);
  o.lo = __builtin_elementwise_fma(uh, vl, __builtin_elementwise_fma(ul, vh, e));
  return o;
}

// ORDER 2: A = shell block, B = shell block;  ORDER 3: A = pair block, B = shell
// block;  ORDER 4: A = pair block, B = pair block;  ORDER 5: A = pair block, B =
// triple block;  ORDER 6: A = triple block, B = triple block.
//
// A stage holds 64 grid points (two MFMA K-steps of 32).  16 waves share one stage;
// each wave owns up to slots_for<ORDER>() tiles.
template <int ORDER>
constexpr int slots_for() { return ORDER == 2 ? 4 : ORDER == 3 ? kSlots : ORDER == 4 ? kSlots4 : ORDER == 5 ? kSlots56 : kSlots6; }

template <int PREC, int ORDER>
__global__ __launch_bounds__(kCtrThreads, 1) void contract_tiles(CtrParams p) {
  // FP16 up to order 4 forms pair products from the operand words alone; the other
  // precisions, and every precision at orders 5 and 6, form their row products from
  // float32 rows staged in `stage`
  constexpr bool kFloatStage = PREC != kFP16 || ORDER >= 5;
  // FP16 needs the per-shell power-of-two scaling for its range; at orders 5 and 6 every
  // precision takes it, since unscaled products of five or six shell values summed over
  // the grid overflow float32 (they reach 1e45 at 256^3)
  constexpr bool kScaled = PREC == kFP16 || ORDER >= 5;
  constexpr int kStageFloats = kFloatStage ? (kMaxBlk * 16 + 1) * kRowStride : 4;
  __shared__ __attribute__((aligned(16))) float stage[2][kStageFloats];
  // [buffer][K-step][shell block][lane]; block kMaxBlk stays zero (padding pairs)
  __shared__ uint4 opHi[2][2][kMaxBlk + 1][64];
  __shared__ uint4 opLo[2][2][kMaxBlk + 1][64];
  __shared__ float lds_scale[kMaxBlk * 16 + 1];

  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int g = lane >> 4;   // which 8-point group of a K-step
  const int row = lane & 15;
  const int chunk = blockIdx.x;
  const int group = blockIdx.y;
  const int b = blockIdx.z;
  const int nrows = p.n_blk * 16;   // staged shell rows (zero beyond n_shells); row nrows is all zero

  for (int i = tid; i <= nrows; i += kCtrThreads) {
    float sc = 1.f;
    if (kScaled) sc = i < p.n_shells ? ldexpf(1.0f, shell_scale_exp(p.absmax, b * p.n_shells + i)) : 0.f;
    lds_scale[i] = sc;
  }
  if constexpr (kFloatStage) {
    for (int i = tid; i < 2 * (nrows + 1) * kRowStride; i += kCtrThreads) {
      const int buf = i / ((nrows + 1) * kRowStride);
      const int rr = (i / kRowStride) % (nrows + 1);
      if (rr >= p.n_shells) stage[buf][i % ((nrows + 1) * kRowStride)] = 0.f;
    }
  }
  for (int i = tid; ORDER <= 4 && i < 4 * (kMaxBlk + 1) * 64; i += kCtrThreads) {
    const int bh = i / ((kMaxBlk + 1) * 64), kb = (i / 64) % (kMaxBlk + 1), ln = i % 64;
    if (kb * 16 + (ln & 15) >= p.n_shells) {
      opHi[bh >> 1][bh & 1][kb][ln] = make_uint4(0, 0, 0, 0);
      opLo[bh >> 1][bh & 1][kb][ln] = make_uint4(0, 0, 0, 0);
    }
  }

  constexpr int NS = slots_for<ORDER>();
  f32x4 acc[NS];
#pragma unroll
  for (int s = 0; s < NS; ++s) acc[s] = f32x4{0.f, 0.f, 0.f, 0.f};

  // global -> LDS staging: thread t moves float4 #t of the (n_shells x 64) slice and
  // also writes it, split, into the operand arrays of its shell block and K-step
  const float* Db = p.D + (size_t)b * p.n_shells * p.G;
  const long long x_base = (long long)chunk * p.ksteps * kKStep;
  const int st_row = tid >> 4, st_col = (tid & 15) * 4;
  const bool st_active = st_row < p.n_shells;
  const int st_kb = st_row >> 4;
  const int st_h = st_col >> 5;                                  // K-step of the stage
  const int st_lane = (((st_col & 31) >> 3) << 4) | (st_row & 15);
  const int st_half = (st_col >> 2) & 1;
  auto stage_store = [&](int buf, float4 v) {
    if (kScaled) {  // every operand works on the power-of-two scaled values
      const float sc = lds_scale[st_row];
      v = make_float4(v.x * sc, v.y * sc, v.z * sc, v.w * sc);
    }
    if constexpr (kFloatStage) *reinterpret_cast<float4*>(&stage[buf][st_row * kRowStride + st_col]) = v;
    if constexpr (ORDER >= 5) {
      // every operand is formed from the float rows
    } else if constexpr (PREC == kFP32) {
      const uint4 w = make_uint4(__float_as_uint(v.x), __float_as_uint(v.y), __float_as_uint(v.z),
                                 __float_as_uint(v.w));
      if (st_half) opLo[buf][st_h][st_kb][st_lane] = w; else opHi[buf][st_h][st_kb][st_lane] = w;
    } else {
      uint2 hi, lo;
      split4<PREC>(v, 1.f, hi, lo);
      reinterpret_cast<uint2*>(&opHi[buf][st_h][st_kb][st_lane])[st_half] = hi;
      reinterpret_cast<uint2*>(&opLo[buf][st_h][st_kb][st_lane])[st_half] = lo;
    }
  };
  float4 pre = make_float4(0.f, 0.f, 0.f, 0.f);
  if (st_active) pre = *reinterpret_cast<const float4*>(Db + (size_t)st_row * p.G + x_base + st_col);
  __syncthreads();
  if (st_active) stage_store(0, pre);
  __syncthreads();

  // Slot state for the whole chunk.  Uniform byte per slot (4 slots per word, in
  // SGPRs): bits 0-1 B shell block, 2-3 A shell block (order 2), 4 = form A here,
  // 7 = empty.  Per-lane shells of the lane's pair rows: order 3 packs (u, v) of
  // two slots per word, order 4 packs (u_A, v_A, u_B, v_B) of one slot per word;
  // orders 5 and 6 use two words per slot, the A row's shells then the B row's.
  constexpr int NLW = ORDER == 4 ? NS : ORDER >= 5 ? 2 * NS : (NS + 1) / 2;
  const int* uni = p.slot_uni + ((size_t)group * kCtrWaves + wave) * (kSlotsMax / 4);
  int un[(NS + 3) / 4];
#pragma unroll
  for (int i = 0; i < (NS + 3) / 4; ++i) un[i] = __builtin_amdgcn_readfirstlane(uni[i]);
  int lv[NLW];
  if (ORDER >= 3) {
    const int* lw = p.slot_lane + (((size_t)group * kCtrWaves + wave) * 16 + row) * kSlotsMax;
#pragma unroll
    for (int i = 0; i < NLW; ++i) lv[i] = lw[i];
  }
  for (int ks = 0; ks < p.ksteps; ++ks) {
    const int cur = ks & 1;
    if (ks + 1 < p.ksteps && st_active)
      pre = *reinterpret_cast<const float4*>(Db + (size_t)st_row * p.G + x_base + (ks + 1) * kKStep + st_col);
    const float* S = stage[cur];
#pragma unroll
    for (int h = 0; h < 2; ++h) {
      Operand<PREC> A;
#pragma unroll
      for (int s = 0; s < NS; ++s) {
        const int info = (un[s / 4] >> (8 * (s % 4))) & 0xff;
        if (info & 0x80) break;
        if constexpr (ORDER >= 5) {
          if (info & 0x10) A = form_rows<PREC, ORDER == 6 ? 3 : 2>(S + 32 * h, lv[2 * s], g);
          const Operand<PREC> Bop = form_rows<PREC, 3>(S + 32 * h, lv[2 * s + 1], g);
          mma<PREC>(acc[s], A, Bop);
          continue;
        }
        if (ORDER == 2) {
          const int ab = (info >> 2) & 3;
          A = op_from_words<PREC>(opHi[cur][h][ab][lane], opLo[cur][h][ab][lane]);
        } else if (info & 0x10) {
          const int uv = ORDER == 3 ? (lv[s / 2] >> (16 * (s % 2))) & 0xffff : lv[s] & 0xffff;
          if constexpr (PREC == kFP16) A = form_pair_f16(opHi[cur][h], opLo[cur][h], uv, lane);
          else A = form_pair<PREC>(S + 32 * h, uv, g);
        }
        Operand<PREC> Bop;
        if (ORDER == 4) {
          if constexpr (PREC == kFP16) Bop = form_pair_f16(opHi[cur][h], opLo[cur][h], (lv[s] >> 16) & 0xffff, lane);
          else Bop = form_pair<PREC>(S + 32 * h, (lv[s] >> 16) & 0xffff, g);
        } else {
          const int bb = info & 3;
          Bop = op_from_words<PREC>(opHi[cur][h][bb][lane], opLo[cur][h][bb][lane]);
        }
        mma<PREC>(acc[s], A, Bop);
      }
    }
    if (ks + 1 < p.ksteps && st_active) stage_store(cur ^ 1, pre);
    __syncthreads();
  }

  // dump accumulators: tile t, lane l, register r -> partials[..][t][4 l + r]
  const int* my_tiles = p.slot_tile + ((size_t)group * kCtrWaves + wave) * kSlotsMax;
  float* out = p.partials + ((size_t)b * p.n_chunks + chunk) * (size_t)p.n_tiles * 256;
#pragma unroll
  for (int s = 0; s < NS; ++s) {
    if ((un[s / 4] >> (8 * (s % 4))) & 0x80) break;
    const int t = my_tiles[s];
    *reinterpret_cast<f32x4*>(out + (size_t)t * 256 + 4 * lane) = acc[s];
  }
}

// ---------------------------------------------------------------------------
// Order 3, pair blocks aligned to shell blocks (FP16 split).
//   S[(i, j), k] = sum_x d_i d_j d_k  for i in shell block ib, one shell j, k in block kb.
// For j in the first two shell blocks the A operand of tile (ib, j, kb) is the
// shell-block operand of ib times the row of shell j (the same for all 16 rows); for
// j in the last two, where fewer blocks kb >= jb than ib <= jb exist, the B operand
// of kb is scaled by d_j instead.  Either way every operand of a 32-point step comes
// from the four shell-block operands held in registers plus two LDS reads per j (all
// 16 rows of a point group read one word).  Wave w owns j = w + 8 q and the
// tiles (ib <= jb = q / 2, kb >= jb), one static accumulator each; a per-wave mask
// says which of them hold a candidate tuple.  Rows i > j of the diagonal block are
// computed and never read.
// ---------------------------------------------------------------------------
constexpr int kJThreads = 64 * kJWaves;
static_assert(jslot(7, 3, 3) + 1 == kJSlots, "slot numbering");
static_assert(kSlots == kSlotsHost && kSlots4 == kSlots4Host && kSlots56 == kSlots56Host && kSlots6 == kSlots6Host &&
                  kSlotsMax == kSlotsMaxHost && 2 * kSlots56 <= kSlotsMax && kMaxBlk == kMaxBlkHost &&
                  kCtrWaves == kCtrWavesHost,
              "host and device tile tables agree");

__device__ __forceinline__ Operand<kFP16> pair_f16(const Operand<kFP16>& a, const Operand<kFP16>& b) {
  Operand<kFP16> o;
  o.hi = a.hi * b.hi;
  const f16x8 e = __builtin_elementwise_fma(a.hi, b.hi, -o.hi);
  o.lo = __builtin_elementwise_fma(a.hi, b.lo, __builtin_elementwise_fma(a.lo, b.hi, e));
  return o;
}

template <int PREC>
__global__ __launch_bounds__(kJThreads, 1) void contract_j3(CtrJParams p) {
  static_assert(PREC == kFP16, "shell-block aligned contraction is implemented for the FP16 split");
  __shared__ uint4 opHi[2][2][kMaxBlk][64];   // [buffer][K-step][shell block][lane]
  __shared__ uint4 opLo[2][2][kMaxBlk][64];
  __shared__ float lds_scale[kMaxBlk * 16];

  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int chunk = blockIdx.x;
  const int b = blockIdx.z;

  for (int i = tid; i < kMaxBlk * 16; i += kJThreads)
    lds_scale[i] = i < p.n_shells ? ldexpf(1.0f, shell_scale_exp(p.absmax, b * p.n_shells + i)) : 0.f;
  for (int i = tid; i < 4 * kMaxBlk * 64; i += kJThreads) {
    const int bh = i / (kMaxBlk * 64), kb = (i / 64) % kMaxBlk, ln = i % 64;
    if (kb * 16 + (ln & 15) >= p.n_shells) {
      opHi[bh >> 1][bh & 1][kb][ln] = make_uint4(0, 0, 0, 0);
      opLo[bh >> 1][bh & 1][kb][ln] = make_uint4(0, 0, 0, 0);
    }
  }
  __syncthreads();

  // staging: float4 #f of the (64 shells x 64 points) slice, f = tid and tid + kJThreads
  const float* Db = p.D + (size_t)b * p.n_shells * p.G;
  const long long x_base = (long long)chunk * p.ksteps * kKStep;
  constexpr int kF4 = 64 * kKStep / 4 / kJThreads;   // float4 per thread per stage
  int st_row[kF4], st_col[kF4];
#pragma unroll
  for (int f = 0; f < kF4; ++f) {
    const int idx = tid + f * kJThreads;
    st_row[f] = idx >> 4;
    st_col[f] = (idx & 15) * 4;
  }
  auto stage_store = [&](int buf, int f, float4 v) {
    const int row = st_row[f], col = st_col[f];
    const float sc = lds_scale[row];
    v = make_float4(v.x * sc, v.y * sc, v.z * sc, v.w * sc);
    uint2 hi, lo;
    split4<PREC>(v, 1.f, hi, lo);
    const int h = col >> 5, kb = row >> 4, ln = (((col & 31) >> 3) << 4) | (row & 15), half = (col >> 2) & 1;
    reinterpret_cast<uint2*>(&opHi[buf][h][kb][ln])[half] = hi;
    reinterpret_cast<uint2*>(&opLo[buf][h][kb][ln])[half] = lo;
  };
  float4 pre[kF4];
#pragma unroll
  for (int f = 0; f < kF4; ++f) {
    pre[f] = make_float4(0.f, 0.f, 0.f, 0.f);
    if (st_row[f] < p.n_shells)
      pre[f] = *reinterpret_cast<const float4*>(Db + (size_t)st_row[f] * p.G + x_base + st_col[f]);
  }
#pragma unroll
  for (int f = 0; f < kF4; ++f)
    if (st_row[f] < p.n_shells) stage_store(0, f, pre[f]);
  __syncthreads();

  const unsigned m0 = __builtin_amdgcn_readfirstlane(p.slot_mask[2 * wave]);
  const unsigned m1 = __builtin_amdgcn_readfirstlane(p.slot_mask[2 * wave + 1]);
  f32x4 acc[kJSlots];
#pragma unroll
  for (int s = 0; s < kJSlots; ++s) acc[s] = f32x4{0.f, 0.f, 0.f, 0.f};

  for (int ks = 0; ks < p.ksteps; ++ks) {
    const int cur = ks & 1;
    if (ks + 1 < p.ksteps) {
#pragma unroll
      for (int f = 0; f < kF4; ++f)
        if (st_row[f] < p.n_shells)
          pre[f] = *reinterpret_cast<const float4*>(Db + (size_t)st_row[f] * p.G + x_base + (ks + 1) * kKStep +
                                                    st_col[f]);
    }
#pragma unroll
    for (int h = 0; h < 2; ++h) {
    // the slot masks are re-read from SGPRs every half step (scalar bit tests) instead
    // of being kept as 40 precomputed lane masks, which would not fit in the SGPRs: with
    // one re-read per step the compiler still kept the 40 conditions of both halves and
    // spilled them into VGPR lanes (51.0 -> 47.5 ms for the 512^3 contraction)
    unsigned mm0 = m0, mm1 = m1;
    asm volatile("" : "+s"(mm0), "+s"(mm1));
    mm0 = __builtin_amdgcn_readfirstlane(mm0);
    mm1 = __builtin_amdgcn_readfirstlane(mm1);
    auto active = [&](int s) { return ((s < 32 ? mm0 >> s : mm1 >> (s - 32)) & 1u) != 0; };
      Operand<PREC> Bop[kMaxBlk];
#pragma unroll
      for (int kb = 0; kb < kMaxBlk; ++kb) Bop[kb] = op_from_words<PREC>(opHi[cur][h][kb][lane], opLo[cur][h][kb][lane]);
      static_for<8>([&](auto qc) {
        constexpr int q = decltype(qc)::value;
        constexpr int jb = q / 2;
        const int j = wave + kJWaves * q;
        if (j >= p.n_shells) return;
        const int rj = (lane & 0x30) | (j & 15);
        const Operand<PREC> dj = op_from_words<PREC>(opHi[cur][h][jb][rj], opLo[cur][h][jb][rj]);
        if constexpr (jb <= 1) {
          // few blocks ib <= jb: scale the A side, A = (d_i d_j) rows
          static_for<jb + 1>([&](auto ibc) {
            constexpr int ib = decltype(ibc)::value;
            bool any = false;
            static_for<kMaxBlk - jb>([&](auto kc) { any = any || active(jslot(q, ib, jb + decltype(kc)::value)); });
            if (!any) return;
            const Operand<PREC> A = pair_f16(Bop[ib], dj);
            static_for<kMaxBlk - jb>([&](auto kc) {
              constexpr int kb = jb + decltype(kc)::value;
              if (active(jslot(q, ib, kb))) mma<PREC>(acc[jslot(q, ib, kb)], A, Bop[kb]);
            });
          });
        } else {
          // few blocks kb >= jb: scale the B side, B = (d_j d_k) columns; same sums
          static_for<kMaxBlk - jb>([&](auto kc) {
            constexpr int kb = jb + decltype(kc)::value;
            bool any = false;
            static_for<jb + 1>([&](auto ibc) { any = any || active(jslot(q, decltype(ibc)::value, kb)); });
            if (!any) return;
            const Operand<PREC> Bs = pair_f16(Bop[kb], dj);
            static_for<jb + 1>([&](auto ibc) {
              constexpr int ib = decltype(ibc)::value;
              if (active(jslot(q, ib, kb))) mma<PREC>(acc[jslot(q, ib, kb)], Bop[ib], Bs);
            });
          });
        }
      });
    }
    if (ks + 1 < p.ksteps) {
#pragma unroll
      for (int f = 0; f < kF4; ++f)
        if (st_row[f] < p.n_shells) stage_store(cur ^ 1, f, pre[f]);
    }
    __syncthreads();
  }

  auto active = [&](int s) { return ((s < 32 ? m0 >> s : m1 >> (s - 32)) & 1u) != 0; };
  const int* my_tiles = p.tile_of_slot + wave * kJSlots;
  float* out = p.partials + ((size_t)b * p.n_chunks + chunk) * (size_t)p.n_tiles * 256;
#pragma unroll
  for (int s = 0; s < kJSlots; ++s) {
    if (!active(s)) continue;
    *reinterpret_cast<f32x4*>(out + (size_t)my_tiles[s] * 256 + 4 * lane) = acc[s];
  }
}

// Power of two that undoes the operand scaling of the contraction for closing tuple t
// of field b: the shells' scales, and for FP16 at orders 5 and 6 the extra 2^-7 of
// every triple operand.
__device__ __forceinline__ int tuple_unscale_exp(const unsigned* absmax, int b, int n_shells, const int* bins,
                                                 int t, int order, int prec) {
  int ex = 0;
  for (int j = 0; j < order; ++j) ex += shell_scale_exp(absmax, b * n_shells + bins[t * order + j]);
  const int triples = prec != kFP16 ? 0 : order == 5 ? 1 : order == 6 ? 2 : 0;
  return triples * kTripleShift - ex;
}

// Sum float32 partials over chunk ranges in float64, fixed order.
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

// ---------------------------------------------------------------------------
// Adjoint (order 3).  W[b][m][pair] = mult * dL/dB_t * fnorm_t with t = sort(m, u, v)
// and mult the number of times m occurs in t; then a_m[x] = sum_pairs W[m][pair]
// (d_u d_v)[x] on the matrix cores with v_mfma_f32_32x32x16 (32 shells m x 32 grid
// points per tile, 16 pairs per step).  W is written straight into operand order:
// for pair chunk kc (16 pairs) and shell block mb (32 shells), lane l holds row
// m = 32 mb + l % 32 and pairs 16 kc + 8 (l / 32) + r, r = 0..7, as two 16-byte
// words (hi / lo, or values 0..3 / 4..7 in float32).
// ---------------------------------------------------------------------------
typedef __attribute__((__vector_size__(16 * sizeof(float)))) float f32x16;
constexpr int kAdjMaxMb = 2;   // shell blocks of 32 (n_shells <= 64)

// W in operand order for the v-major adjoint below: for each v, shell chunk uc of u
// (16 shells) and shell block mb of m (32 shells), lane l holds W[m][(u, v)] for
// m = 32 mb + l % 32 and u = 16 uc + 8 (l / 32) + r (r = 0..7; zero when u > v),
// as two 16-byte words (hi / lo bf16, or values 0..3 / 4..7 in float32).
// Layout [b][v][uc][mb][hi, lo][lane].
__global__ void adjoint_weights(const double* __restrict__ grad, const double* __restrict__ fnorm,
                                const int* __restrict__ lookup /*[nb^3] closing index or -1*/, int n_shells,
                                int n_closing, int prec, uint4* __restrict__ W) {
  const int m = threadIdx.x;            // 0..63
  const int u = blockIdx.x;             // 0..63
  const int v = blockIdx.y;             // 0..n_shells-1
  const int b = blockIdx.z;
  float w = 0.f;
  if (m < n_shells && u < n_shells && u <= v) {
    int t0 = m, t1 = u, t2 = v;
    if (t0 > t1) { int tmp = t0; t0 = t1; t1 = tmp; }
    if (t1 > t2) { int tmp = t1; t1 = t2; t2 = tmp; }
    if (t0 > t1) { int tmp = t0; t0 = t1; t1 = tmp; }
    const int id = lookup[(t0 * n_shells + t1) * n_shells + t2];
    if (id >= 0) {
      const int mult = (t0 == m) + (t1 == m) + (t2 == m);
      w = (float)((double)mult * grad[(size_t)b * n_closing + id] * fnorm[id]);
    }
  }
  const int uc = u >> 4, q = u & 15, hh = q >> 3, r = q & 7;
  const int lane = 32 * hh + (m & 31), mb = m >> 5;
  uint4* base = W + ((((size_t)b * n_shells + v) * 4 + uc) * kAdjMaxMb + mb) * 2 * 64;
  if (prec == kFP32) {
    float* dst = reinterpret_cast<float*>(&base[(r < 4 ? 0 : 64) + lane]);
    dst[r & 3] = w;
  } else {
    const unsigned bits = __float_as_uint(w);
    const float h = __uint_as_float(bits & 0xffff0000u);
    reinterpret_cast<unsigned short*>(&base[lane])[r] = (unsigned short)(bits >> 16);
    reinterpret_cast<unsigned short*>(&base[64 + lane])[r] = __builtin_bit_cast(unsigned short, (__bf16)(w - h));
  }
}

template <int PREC>
__device__ __forceinline__ void mma32(f32x16& acc, const Operand<PREC>& a, const Operand<PREC>& b) {
  if constexpr (PREC == kFP32) {
    // 32x32x2 float32: eight steps; lane l holds K index l / 32 of each
#pragma unroll
    for (int r = 0; r < 8; ++r) acc = __builtin_amdgcn_mfma_f32_32x32x2f32(a.v[r], b.v[r], acc, 0, 0, 0);
  } else {
    acc = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a.hi, b.hi, acc, 0, 0, 0);
    acc = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a.hi, b.lo, acc, 0, 0, 0);
    acc = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a.lo, b.hi, acc, 0, 0, 0);
  }
}

// As mma32, into a fresh accumulator (C = 0).
template <int PREC>
__device__ __forceinline__ void mma32_first(f32x16& acc, const Operand<PREC>& a, const Operand<PREC>& b) {
  const f32x16 z = {0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f};
  if constexpr (PREC == kFP32) {
    acc = __builtin_amdgcn_mfma_f32_32x32x2f32(a.v[0], b.v[0], z, 0, 0, 0);
#pragma unroll
    for (int r = 1; r < 8; ++r) acc = __builtin_amdgcn_mfma_f32_32x32x2f32(a.v[r], b.v[r], acc, 0, 0, 0);
  } else {
    acc = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a.hi, b.hi, z, 0, 0, 0);
    acc = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a.hi, b.lo, acc, 0, 0, 0);
    acc = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a.lo, b.hi, acc, 0, 0, 0);
  }
}

template <int PREC>
__device__ __forceinline__ float operand_value(const Operand<PREC>& o, int r) {
  if constexpr (PREC == kFP32) return o.v[r];
  else return (float)o.hi[r] + (float)o.lo[r];
}

// a_m[x] = sum_v d_v[x] Y_v[m][x],  Y_v[m][x] = sum_{u <= v} W[m][(u, v)] d_u[x].
// A workgroup of 8 waves owns 512 grid points, each wave two 32-point column blocks,
// and every shell m.  The B operands (the fields d_u at the wave's points, 4 chunks
// of 16 shells per column block) are loaded once from HBM straight into registers;
// d_v is read back from them.  The weight operands of kAdjVG values of v at a time
// are staged in LDS, double buffered: while one stage is in use the next one is
// copied in, a piece per v, with one barrier per stage.  Each weight block read
// from LDS feeds both column blocks (two independent MFMA chains).
constexpr int kAdjWaves = 8;
constexpr int kAdjPB = 2;                                   // 32-point column blocks per wave
constexpr int kAdjThreads = 64 * kAdjWaves;
constexpr int kAdjPts = 32 * kAdjPB * kAdjWaves;
constexpr int kAdjVG = 4;
constexpr int kAdjWPerV = 4 * kAdjMaxMb * 2 * 64;           // uint4 words of W per v
constexpr int kAdjStageWords = kAdjVG * kAdjWPerV;
constexpr int kAdjPiece = kAdjWPerV / kAdjThreads;          // words per thread per v step
static_assert(kAdjPiece * kAdjThreads == kAdjWPerV, "a stage is copied in kAdjVG equal pieces");

// Fused epilogue (NF = N <= 512): the workgroup's 512 points are 512 / N whole rows
// of x2, so the adjoint fields a_m of those rows are transformed to the half spectrum
// q2 = 0..Kc right here (two rows m per complex FFT, the same real-to-complex pass as
// the backward's first transform) and written to H2; the fields themselves never
// reach HBM.  NF = 0 writes a_m to A for a separate transform (N = 1024).
template <int NF>
constexpr int adj_pencils() { return NF ? 32 * (kAdjPts / NF) : 0; }
template <int NF>
constexpr size_t adj_lds_bytes() {
  const size_t stage = (size_t)2 * kAdjStageWords * sizeof(uint4);
  if constexpr (NF == 0) {
    return stage;
  } else {
    const size_t fft = ((size_t)adj_pencils<NF>() * pencil_stride<NF>() + stage_tw_size<NF>()) * sizeof(cplx<float>);
    return fft > stage ? fft : stage;
  }
}

// Writes the accumulated adjoint fields: acc[pb][mb] of lane l, register i is row
// m = 32 mb + 8 (i / 4) + 4 (l / 32) + i % 4 at point l % 32 of column block pb.
template <int NF>
__device__ __forceinline__ void adjoint_epilogue(const f32x16 (&acc)[kAdjPB][kAdjMaxMb], unsigned char* lds, int lane,
                                                 int wave, int hh, int col, int b, long long xw, int n_shells,
                                                 long long G, float* __restrict__ A, cplx<float>* __restrict__ H2,
                                                 const cplx<float>* __restrict__ tw, const Geom& g) {
  if constexpr (NF == 0) {
    float* Ab = A + (size_t)b * n_shells * G + xw;
#pragma unroll
    for (int pb = 0; pb < kAdjPB; ++pb) {
#pragma unroll
      for (int mb = 0; mb < kAdjMaxMb; ++mb) {
#pragma unroll
        for (int i = 0; i < 16; ++i) {
          const int m = mb * 32 + 8 * (i / 4) + 4 * hh + (i % 4);
          if (m < n_shells) Ab[(size_t)m * G + 32 * pb] = acc[pb][mb][i];
        }
      }
    }
  } else {
    constexpr int P = adj_pencils<NF>();          // pencil rho * 32 + m / 2 holds rows m, m + 1 of x2-row rho
    constexpr int NS = pencil_stride<NF>();
    cplx<float>* buf = reinterpret_cast<cplx<float>*>(lds);
    cplx<float>* stw = buf + P * NS;
    __syncthreads();                              // every wave is done with the weight stages
#pragma unroll
    for (int pb = 0; pb < kAdjPB; ++pb) {
      const int x = wave * 32 * kAdjPB + 32 * pb + col;   // point within the workgroup
      const int rho = x / NF, x2 = x % NF;
#pragma unroll
      for (int mb = 0; mb < kAdjMaxMb; ++mb) {
#pragma unroll
        for (int i = 0; i < 16; ++i) {
          const int m = mb * 32 + 8 * (i / 4) + 4 * hh + (i % 4);
          float* slot = reinterpret_cast<float*>(&buf[(rho * 32 + (m >> 1)) * NS + pad8(x2)]);
          slot[m & 1] = acc[pb][mb][i];
        }
      }
    }
    build_stage_twiddles<float, NF, kAdjThreads>(stw, tw);
    __syncthreads();
    fft_block<float, NF, P, NS, -1, kAdjThreads>(buf, stw);
    // half spectrum of each real row: A = (Z[c] + conj Z[-c]) / 2 (row m), B = (Z[c] - conj Z[-c]) / 2i (row m + 1)
    const long long row0 = (long long)blockIdx.x * (kAdjPts / NF);
    for (int u = threadIdx.x; u < 2 * P * g.B2; u += kAdjThreads) {
      const int r = u / g.B2, c = u % g.B2;
      const int pen = r >> 1;
      const int m = 2 * (pen & 31) + (r & 1), rho = pen >> 5;
      if (m >= n_shells) continue;
      const cplx<float> Zp = buf[pen * NS + pad8(c)];
      const cplx<float> Zm = buf[pen * NS + pad8((NF - c) & (NF - 1))];
      cplx<float> v;
      if ((r & 1) == 0) v = cplx<float>{0.5f * (Zp.re + Zm.re), 0.5f * (Zp.im - Zm.im)};
      else v = cplx<float>{0.5f * (Zp.im + Zm.im), 0.5f * (Zm.re - Zp.re)};
      H2[((size_t)(b * n_shells + m) * (G / NF) + row0 + rho) * g.B2 + c] = v;   // G / NF rows per field
    }
  }
}

template <int PREC, int NF>
__global__ __launch_bounds__(kAdjThreads, 1) void adjoint_gemm(const float* __restrict__ D,
                                                             const uint4* __restrict__ W,
                                                             const int* __restrict__ vmask, int n_shells,
                                                             long long G, float* __restrict__ A,
                                                             cplx<float>* __restrict__ H2,
                                                             const cplx<float>* __restrict__ tw, Geom g) {
  __shared__ __attribute__((aligned(16))) unsigned char lds[adj_lds_bytes<NF>()];
  auto wst = reinterpret_cast<uint4(*)[kAdjStageWords]>(lds);
  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const int wave = tid >> 6;
  const int hh = lane >> 5, col = lane & 31;
  const int b = blockIdx.y;
  const long long xw = (long long)blockIdx.x * kAdjPts + wave * 32 * kAdjPB + col;
  const float* Db = D + (size_t)b * n_shells * G;

  // B operands: lane (hh, col) holds shells 16 uc + 8 hh + r at point col of block pb
  Operand<PREC> Bu[kAdjPB][4];
#pragma unroll
  for (int pb = 0; pb < kAdjPB; ++pb) {
#pragma unroll
    for (int uc = 0; uc < 4; ++uc) {
      float x[8];
#pragma unroll
      for (int r = 0; r < 8; ++r) {
        const int sh = 16 * uc + 8 * hh + r;
        x[r] = sh < n_shells ? Db[(size_t)sh * G + xw + 32 * pb] : 0.f;
      }
      Bu[pb][uc] = make_operand<PREC>(x, 1.f);
    }
  }

  const uint4* Wb = W + (size_t)b * n_shells * kAdjWPerV;
  const int n_stages = (n_shells + kAdjVG - 1) / kAdjVG;
  uint4 wp[kAdjPiece];
  // piece q of stage s: words (q kAdjPiece + k) kAdjThreads + tid of the stage
  auto w_load = [&](int s, int q) {
#pragma unroll
    for (int k = 0; k < kAdjPiece; ++k) {
      const int i = (q * kAdjPiece + k) * kAdjThreads + tid;
      const int v = s * kAdjVG + i / kAdjWPerV;
      wp[k] = v < n_shells ? Wb[(size_t)s * kAdjStageWords + i] : make_uint4(0, 0, 0, 0);
    }
  };
  auto w_store = [&](int buf, int q) {
#pragma unroll
    for (int k = 0; k < kAdjPiece; ++k) wst[buf][(q * kAdjPiece + k) * kAdjThreads + tid] = wp[k];
  };
  for (int q = 0; q < kAdjVG; ++q) {
    w_load(0, q);
    w_store(0, q);
  }
  __syncthreads();

  f32x16 acc[kAdjPB][kAdjMaxMb];
#pragma unroll
  for (int pb = 0; pb < kAdjPB; ++pb)
#pragma unroll
    for (int mb = 0; mb < kAdjMaxMb; ++mb)
#pragma unroll
      for (int i = 0; i < 16; ++i) acc[pb][mb][i] = 0.f;

#pragma unroll
  for (int vc = 0; vc < 4; ++vc) {            // fully unrolled: register indices stay static
    if (16 * vc >= n_shells) break;
#pragma unroll
    for (int vv = 0; vv < 16; ++vv) {
      const int v = 16 * vc + vv;
      if (v >= n_shells) break;
      const int st = v / kAdjVG, vi = v % kAdjVG;
      const bool more = st + 1 < n_stages;
      if (more) {                 // copy the next stage in, one piece per v
        if (vi > 0) w_store((st + 1) & 1, vi - 1);
        w_load(st + 1, vi);
      }
      const int mask = __builtin_amdgcn_readfirstlane(vmask[v]);   // bit 2 uc + mb
      const uint4* wv = wst[st & 1] + vi * kAdjWPerV;
      // d_v at this lane's points: element vv % 8 of chunk vc, held by the half vv / 8
      float dv[kAdjPB];
#pragma unroll
      for (int pb = 0; pb < kAdjPB; ++pb) {
        const float own = operand_value<PREC>(Bu[pb][vc], vv % 8);
        const float other = __shfl_xor(own, 32);
        dv[pb] = (hh == vv / 8) ? own : other;
      }
#pragma unroll
      for (int mb = 0; mb < kAdjMaxMb; ++mb) {
        if (!(mask & (0x55 << mb))) continue;   // no weight in this shell block of m
        Operand<PREC> Wop[4];
#pragma unroll
        for (int uc = 0; uc <= vc; ++uc) {
          const uint4* blk = wv + (uc * kAdjMaxMb + mb) * 2 * 64;
          Wop[uc] = op_from_words<PREC>(blk[lane], blk[64 + lane]);
        }
        f32x16 Y[kAdjPB];
#pragma unroll
        for (int uc = 0; uc <= vc; ++uc) {
#pragma unroll
          for (int pb = 0; pb < kAdjPB; ++pb) {
            if (uc == 0) mma32_first<PREC>(Y[pb], Wop[uc], Bu[pb][uc]);
            else mma32<PREC>(Y[pb], Wop[uc], Bu[pb][uc]);
          }
        }
#pragma unroll
        for (int pb = 0; pb < kAdjPB; ++pb)
#pragma unroll
          for (int i = 0; i < 16; ++i) acc[pb][mb][i] += dv[pb] * Y[pb][i];
      }
      if (more && (vi == kAdjVG - 1)) {
        w_store((st + 1) & 1, kAdjVG - 1);
        __syncthreads();          // the next stage is complete; this one is free
      }
    }
  }
  adjoint_epilogue<NF>(acc, lds, lane, wave, hh, col, b, xw, n_shells, G, A, H2, tw, g);
}

// ---------------------------------------------------------------------------
// Adjoint, order 4 (at most 32 shells).  With the closing 4-tuples t and their
// weights w_t = dL/dB_t f / (N^3 n_t),
//   a_m[x] = sum over sorted (u <= v <= w) of W4[m][(u, v, w)] d_u d_v d_w,
// W4[m][(u, v, w)] = (times m occurs in t) w_t for t = sort(m, u, v, w).  Grouped by
// the largest shell w and then v, the kernel forms Y_(v,w) = W4_(v,w) D_w on the
// matrix cores, D_w the fields d_u d_w of the lane's points, and adds d_v Y_(v,w).
// ---------------------------------------------------------------------------
// W4 in operand order: item it = w (w + 1) / 2 + v, 16-shell chunk uc of u, lane l holds
// row m = l % 32 and u = 16 uc + 8 (l / 32) + r (r = 0..7; zero when u > v), as two
// 16-byte words (hi / lo bf16, or values 0..3 / 4..7 in float32).
__global__ void adjoint4_weights(const double* __restrict__ grad, const double* __restrict__ fnorm,
                                 const int* __restrict__ lookup /*[nb^4] closing index or -1*/, int n_shells,
                                 int n_closing, int prec, uint4* __restrict__ W) {
  const int m = threadIdx.x;            // 0..31
  const int u = blockIdx.x;             // 0..31
  const int it = blockIdx.y;            // item (w, v)
  const int b = blockIdx.z;
  int w = 0;
  while ((w + 1) * (w + 2) / 2 <= it) ++w;
  const int v = it - w * (w + 1) / 2;
  float val = 0.f;
  if (m < n_shells && u < n_shells && u <= v) {
    int t[4] = {m, u, v, w};
#pragma unroll
    for (int a = 0; a < 3; ++a)
#pragma unroll
      for (int c = 0; c < 3 - a; ++c)
        if (t[c] > t[c + 1]) { const int x = t[c]; t[c] = t[c + 1]; t[c + 1] = x; }
    const int id = lookup[(((size_t)t[0] * n_shells + t[1]) * n_shells + t[2]) * n_shells + t[3]];
    if (id >= 0) {
      const int mult = (t[0] == m) + (t[1] == m) + (t[2] == m) + (t[3] == m);
      val = (float)((double)mult * grad[(size_t)b * n_closing + id] * fnorm[id]);
    }
  }
  const int n_items = n_shells * (n_shells + 1) / 2;
  const int uc = u >> 4, q = u & 15, hh = q >> 3, r = q & 7;
  const int lane = 32 * hh + m;
  uint4* base = W + (((size_t)b * n_items + it) * 2 + uc) * 2 * 64;
  if (prec == kFP32) {
    float* dst = reinterpret_cast<float*>(&base[(r < 4 ? 0 : 64) + lane]);
    dst[r & 3] = val;
  } else {
    const unsigned bits = __float_as_uint(val);
    const float h = __uint_as_float(bits & 0xffff0000u);
    reinterpret_cast<unsigned short*>(&base[lane])[r] = (unsigned short)(bits >> 16);
    reinterpret_cast<unsigned short*>(&base[64 + lane])[r] = __builtin_bit_cast(unsigned short, (__bf16)(val - h));
  }
}

template <int NF>
constexpr size_t adj4_lds_bytes() {
  const size_t stage = (size_t)kAdj4MaxShells * kAdj4WordsPerItem * sizeof(uint4);   // the items of one w
  if constexpr (NF == 0) {
    return stage;
  } else {
    const size_t fft = ((size_t)adj_pencils<NF>() * pencil_stride<NF>() + stage_tw_size<NF>()) * sizeof(cplx<float>);
    return fft > stage ? fft : stage;
  }
}

// A workgroup of 8 waves owns 512 grid points (64 per wave, two column blocks) and
// all shells m < 32.  For each w the weights of the items (w, v <= w) are staged in
// LDS and the fields of the lane's points, scaled by d_w, become the B operands.
template <int PREC, int NF>
__global__ __launch_bounds__(kAdjThreads, 1) void adjoint4_gemm(const float* __restrict__ D,
                                                              const uint4* __restrict__ W,
                                                              const int* __restrict__ imask, int n_shells,
                                                              long long G, float* __restrict__ A,
                                                              cplx<float>* __restrict__ H2,
                                                              const cplx<float>* __restrict__ tw, Geom g) {
  __shared__ __attribute__((aligned(16))) unsigned char lds[adj4_lds_bytes<NF>()];
  uint4* wst = reinterpret_cast<uint4*>(lds);
  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const int wave = tid >> 6;
  const int hh = lane >> 5, col = lane & 31;
  const int b = blockIdx.y;
  const long long xw = (long long)blockIdx.x * kAdjPts + wave * 32 * kAdjPB + col;
  const float* Db = D + (size_t)b * n_shells * G;
  const int n_items = n_shells * (n_shells + 1) / 2;
  const uint4* Wb = W + (size_t)b * n_items * kAdj4WordsPerItem;

  // fields at the lane's points: F[pb][uc][r] = d_u, u = 16 uc + 8 hh + r
  float F[kAdjPB][2][8];
#pragma unroll
  for (int pb = 0; pb < kAdjPB; ++pb)
#pragma unroll
    for (int uc = 0; uc < 2; ++uc)
#pragma unroll
      for (int r = 0; r < 8; ++r) {
        const int sh = 16 * uc + 8 * hh + r;
        F[pb][uc][r] = sh < n_shells ? Db[(size_t)sh * G + xw + 32 * pb] : 0.f;
      }
  f32x16 acc[kAdjPB][kAdjMaxMb];
#pragma unroll
  for (int pb = 0; pb < kAdjPB; ++pb)
#pragma unroll
    for (int mb = 0; mb < kAdjMaxMb; ++mb)
#pragma unroll
      for (int i = 0; i < 16; ++i) acc[pb][mb][i] = 0.f;

  for (int w = 0; w < n_shells; ++w) {
    const int it0 = w * (w + 1) / 2;
    __syncthreads();                              // the previous w's stage is consumed
    for (int i = tid; i < (w + 1) * kAdj4WordsPerItem; i += kAdjThreads) wst[i] = Wb[(size_t)it0 * kAdj4WordsPerItem + i];
    float dw[kAdjPB];
#pragma unroll
    for (int pb = 0; pb < kAdjPB; ++pb) dw[pb] = Db[(size_t)w * G + xw + 32 * pb];
    Operand<PREC> Bu[kAdjPB][2];
#pragma unroll
    for (int pb = 0; pb < kAdjPB; ++pb)
#pragma unroll
      for (int uc = 0; uc < 2; ++uc) {
        float x[8];
#pragma unroll
        for (int r = 0; r < 8; ++r) x[r] = F[pb][uc][r] * dw[pb];
        Bu[pb][uc] = make_operand<PREC>(x, 1.f);
      }
    const int my_mask = lane <= w ? imask[it0 + lane] : 0;   // items (w, v = lane)
    __syncthreads();
#pragma unroll
    for (int vc = 0; vc < 2; ++vc) {
#pragma unroll
      for (int vv = 0; vv < 16; ++vv) {
        const int v = 16 * vc + vv;
        if (v > w) break;
        const int mask = __builtin_amdgcn_readlane(my_mask, v);   // bit uc
        if (!mask) continue;
        const uint4* wv = wst + v * kAdj4WordsPerItem;
        float dv[kAdjPB];
#pragma unroll
        for (int pb = 0; pb < kAdjPB; ++pb) {
          const unsigned own = __float_as_uint(F[pb][vc][vv % 8]);
          const auto sw = __builtin_amdgcn_permlane32_swap(own, own, false, false);
          dv[pb] = __uint_as_float(vv / 8 == 0 ? sw[0] : sw[1]);
        }
        Operand<PREC> Wop[2];
#pragma unroll
        for (int uc = 0; uc <= vc; ++uc) Wop[uc] = op_from_words<PREC>(wv[uc * 128 + lane], wv[uc * 128 + 64 + lane]);
        f32x16 Y[kAdjPB];
#pragma unroll
        for (int uc = 0; uc <= vc; ++uc) {
#pragma unroll
          for (int pb = 0; pb < kAdjPB; ++pb) {
            if (uc == 0) mma32_first<PREC>(Y[pb], Wop[uc], Bu[pb][uc]);
            else mma32<PREC>(Y[pb], Wop[uc], Bu[pb][uc]);
          }
        }
#pragma unroll
        for (int pb = 0; pb < kAdjPB; ++pb)
#pragma unroll
          for (int i = 0; i < 16; ++i) acc[pb][0][i] += dv[pb] * Y[pb][i];
      }
    }
  }
  __syncthreads();
  adjoint_epilogue<NF>(acc, lds, lane, wave, hh, col, b, xw, n_shells, G, A, H2, tw, g);
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
  } else if (order == 4) {
    if (prec == kFP32) L(kFP32, 4); else if (prec == kBF16) L(kBF16, 4); else L(kFP16, 4);
  } else if (order == 5) {
    if (prec == kFP32) L(kFP32, 5); else if (prec == kBF16) L(kBF16, 5); else L(kFP16, 5);
  } else if (order == 6) {
    if (prec == kFP32) L(kFP32, 6); else if (prec == kBF16) L(kBF16, 6); else L(kFP16, 6);
  } else {
    return hipErrorInvalidValue;
  }
#undef L
  return hipGetLastError();
}

hipError_t launch_contract_j3(int prec, const CtrJParams& p, int batch, hipStream_t st) {
  if (prec != kFP16) return hipErrorInvalidValue;
  dim3 grid(p.n_chunks, 1, batch);
  hipLaunchKernelGGL(contract_j3<kFP16>, grid, dim3(kJThreads), 0, st, p);
  return hipGetLastError();
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

hipError_t launch_adjoint_weights(const double* grad, const double* fnorm, const int* lookup, int n_shells,
                                  int n_closing, int prec, uint4* W, int batch, hipStream_t st) {
  dim3 grid(64, n_shells, batch);
  hipLaunchKernelGGL(adjoint_weights, grid, dim3(64), 0, st, grad, fnorm, lookup, n_shells, n_closing, prec, W);
  return hipGetLastError();
}

hipError_t launch_adjoint4_weights(const double* grad, const double* fnorm, const int* lookup, int n_shells,
                                   int n_closing, int prec, uint4* W, int batch, hipStream_t st) {
  if (n_shells > kAdj4MaxShells) return hipErrorInvalidValue;
  dim3 grid(32, n_shells * (n_shells + 1) / 2, batch);
  hipLaunchKernelGGL(adjoint4_weights, grid, dim3(32), 0, st, grad, fnorm, lookup, n_shells, n_closing, prec, W);
  return hipGetLastError();
}

hipError_t launch_adjoint4_gemm(int prec, const float* D, const uint4* W, const int* imask, int n_shells, long long G,
                                float* A, cplx<float>* H2, const cplx<float>* tw, Geom g, int batch, hipStream_t st) {
  if (n_shells > kAdj4MaxShells) return hipErrorInvalidValue;
  dim3 grid((unsigned)(G / kAdjPts), batch);
  const bool fused = adjoint_fuses_rows(g.N);
  if (fused == (H2 == nullptr) || fused == (A != nullptr)) return hipErrorInvalidValue;
#define L(P, NF) hipLaunchKernelGGL((adjoint4_gemm<P, NF>), grid, dim3(kAdjThreads), 0, st, D, W, imask, n_shells, G, A, H2, tw, g)
#define BY_N(P)                                  \
  switch (g.N) {                                 \
    case 32: L(P, 32); break;                    \
    case 64: L(P, 64); break;                    \
    case 128: L(P, 128); break;                  \
    case 256: L(P, 256); break;                  \
    case 512: L(P, 512); break;                  \
    default: L(P, 0); break;                     \
  }
  if (prec == kFP32) {
    BY_N(kFP32)
  } else {
    BY_N(kBF16)
  }
#undef BY_N
#undef L
  return hipGetLastError();
}

hipError_t launch_adjoint_gemm(int prec, const float* D, const uint4* W, const int* vmask, int n_shells, long long G,
                               float* A, cplx<float>* H2, const cplx<float>* tw, Geom g, int batch, hipStream_t st) {
  dim3 grid((unsigned)(G / kAdjPts), batch);
  const bool fused = adjoint_fuses_rows(g.N);
  if (fused == (H2 == nullptr) || fused == (A != nullptr)) return hipErrorInvalidValue;
#define L(P, NF) hipLaunchKernelGGL((adjoint_gemm<P, NF>), grid, dim3(kAdjThreads), 0, st, D, W, vmask, n_shells, G, A, H2, tw, g)
#define BY_N(P)                                  \
  switch (g.N) {                                 \
    case 32: L(P, 32); break;                    \
    case 64: L(P, 64); break;                    \
    case 128: L(P, 128); break;                  \
    case 256: L(P, 256); break;                  \
    case 512: L(P, 512); break;                  \
    default: L(P, 0); break;                     \
  }
  if (prec == kFP32) {
    BY_N(kFP32)
  } else {
    BY_N(kBF16)
  }
#undef BY_N
#undef L
  return hipGetLastError();
}

}  // namespace ps
