// Device helpers shared by the matrix-core kernels (gfx950, wave64): operand
// types of the three precisions, the hi/lo splits, MFMA wrappers and the
// row-product formation from staged shell fields.
#pragma once

#include <utility>

#include "common.h"
#include "kernels.h"

namespace ps {

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
typedef __attribute__((__vector_size__(4 * sizeof(unsigned)))) unsigned u32x4;

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



// LDS word of operand lane ln = 16 g + r (point group g, row r) in the staged operand
// arrays: the rows of group g are rotated by 4 g words.  An MFMA operand read (every
// lane its own word) still reads each group's 256 bytes, while the four groups of one
// row (the broadcast read of one shell, and the staging writes of four consecutive
// rows) land in different LDS banks instead of 256 bytes apart.
__device__ __forceinline__ int op_slot(int ln) { return (ln & 0x30) | ((ln + ((ln >> 4) << 2)) & 15); }

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
  const int iu = op_slot((lane & 0x30) | (u & 15)), iv = op_slot((lane & 0x30) | (v & 15));
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

__device__ __forceinline__ Operand<kFP16> pair_f16(const Operand<kFP16>& a, const Operand<kFP16>& b) {
  Operand<kFP16> o;
  o.hi = a.hi * b.hi;
  const f16x8 e = __builtin_elementwise_fma(a.hi, b.hi, -o.hi);
  o.lo = __builtin_elementwise_fma(a.hi, b.lo, __builtin_elementwise_fma(a.lo, b.hi, e));
  return o;
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


typedef __attribute__((__vector_size__(16 * sizeof(float)))) float f32x16;

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


}  // namespace ps
