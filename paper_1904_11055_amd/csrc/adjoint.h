// Adjoint product of the estimator (not in the paper: the gradient extension).
//
// Order 3: a_m[x] = sum_{u <= v} W[m][(u, v)] d_u[x] d_v[x] with
// W[m][(u, v)] = (times m occurs in t) dL/dB_t f / (N^3 n_t), t = sort(m, u, v),
// summed over the closing triplets t (dS_t / d d_m is the product of the other two
// fields, once per position of m in t).
// Order 4: a_m[x] = sum_{u <= v <= w} W4[m][(u, v, w)] d_u[x] d_v[x] d_w[x], likewise.
//
// Both are one matrix product per workgroup: rows m (32 per block), columns the grid
// points, and the reduction over the row products of the other fields.  A reduction
// step is a 16-shell chunk uc of u with the rest fixed (v, or the item (v, w)): the
// B operand is the 16 fields d_u at the wave's 32 points times the scalar field
// d_v (d_v d_w) at each point, formed on the VALU from fields held in registers, and
// the A operand is the matching weight block from LDS.  The products go straight
// into the output accumulators, so nothing on the VALU waits for a matrix result.
//
// Precisions: FP32 (v_mfma_f32_32x32x2_f32 on the float32 products), SPLIT_BF16
// (products formed in float32, split hi + lo, hh + hl + lh with
// v_mfma_f32_32x32x16_bf16), SPLIT_FP16 (v_mfma_f32_32x32x16_f16; the fields carry
// the forward's per-shell power-of-two scale and the pair products are formed from
// their split halves with error-free half-precision products; each weight row m
// carries its own power of two so that its largest magnitude lies in [2^14, 2^15),
// and the epilogue removes it exactly).
#pragma once

#include "fft_core.h"
#include "mfma_ops.h"

namespace ps {

constexpr int kAdjMaxMb = 2;      // 32-row blocks of m (n_shells <= 64)
constexpr int kAdjRowTop = 14;    // FP16: largest |W'| of a row in [2^14, 2^15)
constexpr int kAdjWaves = 8;
constexpr int kAdjPB = 2;                                   // 32-point column blocks per wave
constexpr int kAdjThreads = 64 * kAdjWaves;
constexpr int kAdjPts = 32 * kAdjPB * kAdjWaves;
constexpr int kAdjVG = 4;
constexpr int kAdjWPerV = 4 * kAdjMaxMb * 2 * 64;           // uint4 words of W per v
constexpr int kAdjStageWords = kAdjVG * kAdjWPerV;
constexpr int kAdjPiece = kAdjWPerV / kAdjThreads;          // words per thread per v step
static_assert(kAdjPiece * kAdjThreads == kAdjWPerV, "a stage is copied in kAdjVG equal pieces");
static_assert(kAdjPtsHost == kAdjPts, "host and device agree on the adjoint's points per workgroup");

// Exponent of the power of two carried by weight row (b, m) in FP16 (0 for an empty row).
__device__ __forceinline__ int adj_row_exp(const unsigned long long* rowmax, int idx) {
  const double m = __longlong_as_double((long long)rowmax[idx]);
  if (!(m > 0.0)) return 0;
  return kAdjRowTop - ilogb(m);
}

template <int NF>
constexpr int adj_pencils() { return NF ? 32 * (kAdjPts / NF) : 0; }
template <int NF>
constexpr size_t adj_fft_lds_bytes() {
  return NF ? ((size_t)adj_pencils<NF>() * pencil_stride<NF>() + stage_tw_size<NF>()) * sizeof(cplx<float>) : 0;
}
template <int NF>
constexpr size_t adj_lds_bytes() {
  const size_t stage = (size_t)2 * kAdjStageWords * sizeof(uint4);
  return adj_fft_lds_bytes<NF>() > stage ? adj_fft_lds_bytes<NF>() : stage;
}
// Order 4 with NC chunks of 16 shells (2: up to 32 shells, one 32-row block of m; 4: up
// to 64, two blocks): items (w, v) per LDS stage, operand words per stage and per thread.
template <int NC>
constexpr int adj4_stage_items() { return NC == 2 ? 8 : 2; }
template <int NC>
constexpr int adj4_stage_words() { return adj4_stage_items<NC>() * adj4_words_per_item(16 * NC); }
template <int NC>
constexpr int adj4_piece() { return adj4_stage_words<NC>() / kAdjThreads; }
static_assert(adj4_piece<2>() * kAdjThreads == adj4_stage_words<2>() &&
                  adj4_piece<4>() * kAdjThreads == adj4_stage_words<4>(),
              "an order-4 stage is copied in equal pieces");
template <int NF, int NC>
constexpr size_t adj4_lds_bytes() {
  const size_t stage = (size_t)2 * adj4_stage_words<NC>() * sizeof(uint4);   // double buffered
  return adj_fft_lds_bytes<NF>() > stage ? adj_fft_lds_bytes<NF>() : stage;
}

// Writes the accumulated adjoint fields: acc[pb][mb] of lane l, register i is row
// m = 32 mb + 8 (i / 4) + 4 (l / 32) + i % 4 at point l % 32 of column block pb.
// Fused form (NF = N <= 512): the workgroup's 512 points are 512 / N whole rows of x2,
// so the rows are transformed to the half spectrum q2 = 0..Kc right here (two rows m
// per complex FFT, the same real-to-complex pass as the backward's first transform)
// and written to H2; the fields never reach HBM.  NF = 0 writes a_m to A.
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
      H2[((size_t)(b * n_shells + m) * (G / NF) + row0 + rho) * g.H2s + c] = v;   // G / NF rows per field
    }
  }
}

// The fields of the lane's points: shells u = 16 uc + 8 hh + r, r = 0..7, of column
// block pb, as float32 (F, for the FP32 and BF16 paths) or as FP16 split operands of
// the scaled values (H, for the FP16 path).
template <int PREC, int NC>
struct AdjFields {
  float F[kAdjPB][NC][8];
};
template <int NC>
struct AdjFields<kFP16, NC> {
  Operand<kFP16> H[kAdjPB][NC];
};

template <int PREC, int NC>
__device__ __forceinline__ void adj_load_fields(AdjFields<PREC, NC>& f, const float* __restrict__ Db, long long G,
                                                long long xw, int hh, int n_shells, const unsigned* absmax,
                                                int b) {
#pragma unroll
  for (int pb = 0; pb < kAdjPB; ++pb) {
#pragma unroll
    for (int uc = 0; uc < NC; ++uc) {
      float x[8];
#pragma unroll
      for (int r = 0; r < 8; ++r) {
        const int sh = 16 * uc + 8 * hh + r;
        x[r] = sh < n_shells ? Db[(size_t)sh * G + xw + 32 * pb] : 0.f;
      }
      if constexpr (PREC == kFP16) {
#pragma unroll
        for (int r = 0; r < 8; ++r) {
          const int sh = 16 * uc + 8 * hh + r;
          if (sh < n_shells) x[r] = ldexpf(x[r], shell_scale_exp(absmax, b * n_shells + sh));
        }
        f.H[pb][uc] = make_operand<kFP16>(x, 1.f);
      } else {
#pragma unroll
        for (int r = 0; r < 8; ++r) f.F[pb][uc][r] = x[r];
      }
    }
  }
}

// The scalar field s at this lane's point of column block pb, for the shell v = 16 vc
// + vv held in register vv % 8 of the lanes of half vv / 8 (one permlane32 swap
// brings the other half's value).  FP16: s holds (hi, lo) of the scaled value as the
// halves of one 32-bit word.
template <int PREC, int NC, int VC, int VV>
__device__ __forceinline__ unsigned adj_scalar(const AdjFields<PREC, NC>& f, int pb) {
  unsigned own;
  if constexpr (PREC == kFP16) {
    // the elements are copied out before the bit cast: the cast applied directly to a
    // vector subscript compiles to element 0 whatever the index (hipcc, gfx950)
    const _Float16 eh = f.H[pb][VC].hi[VV % 8];
    const _Float16 el = f.H[pb][VC].lo[VV % 8];
    own = (unsigned)__builtin_bit_cast(unsigned short, eh) | ((unsigned)__builtin_bit_cast(unsigned short, el) << 16);
  } else {
    own = __float_as_uint(f.F[pb][VC][VV % 8]);
  }
  const auto sw = __builtin_amdgcn_permlane32_swap(own, own, false, false);
  return VV / 8 == 0 ? sw[0] : sw[1];
}

// B operand: fields of chunk uc at this lane's points times the scalar s (bits from
// adj_scalar, or an FP16 split pair already scaled).
template <int PREC, int NC>
__device__ __forceinline__ Operand<PREC> adj_pair_operand(const AdjFields<PREC, NC>& f, int pb, int uc, unsigned s) {
  if constexpr (PREC == kFP16) {
    Operand<kFP16> sv;
    const _Float16 sh = __builtin_bit_cast(_Float16, (unsigned short)(s & 0xffffu));
    const _Float16 sl = __builtin_bit_cast(_Float16, (unsigned short)(s >> 16));
#pragma unroll
    for (int r = 0; r < 8; ++r) {
      sv.hi[r] = sh;
      sv.lo[r] = sl;
    }
    return pair_f16(f.H[pb][uc], sv);
  } else {
    const float sf = __uint_as_float(s);
    float x[8];
#pragma unroll
    for (int r = 0; r < 8; ++r) x[r] = f.F[pb][uc][r] * sf;
    return make_operand<PREC>(x, 1.f);
  }
}

// Product of two scalar fields as an FP16 split pair (error-free product of the split
// halves) times 2^-shift, packed like adj_scalar's words.
__device__ __forceinline__ unsigned f16_scalar_product(unsigned a, unsigned b, int shift) {
  const _Float16 ah = __builtin_bit_cast(_Float16, (unsigned short)(a & 0xffffu));
  const _Float16 al = __builtin_bit_cast(_Float16, (unsigned short)(a >> 16));
  const _Float16 bh = __builtin_bit_cast(_Float16, (unsigned short)(b & 0xffffu));
  const _Float16 bl = __builtin_bit_cast(_Float16, (unsigned short)(b >> 16));
  const _Float16 sc = (_Float16)ldexpf(1.0f, -shift);
  _Float16 ph = ah * bh;
  const _Float16 e = __builtin_fmaf16(ah, bh, -ph);
  _Float16 pl = __builtin_fmaf16(ah, bl, __builtin_fmaf16(al, bh, e));
  ph = ph * sc;   // a power of two: exact while in the normal range
  pl = pl * sc;
  return (unsigned)__builtin_bit_cast(unsigned short, ph) | ((unsigned)__builtin_bit_cast(unsigned short, pl) << 16);
}

template <int PREC>
__device__ __forceinline__ void adj_mma(f32x16& acc, const Operand<PREC>& a, const Operand<PREC>& b) {
  if constexpr (PREC == kFP16) {
    acc = __builtin_amdgcn_mfma_f32_32x32x16_f16(a.hi, b.hi, acc, 0, 0, 0);
    acc = __builtin_amdgcn_mfma_f32_32x32x16_f16(a.hi, b.lo, acc, 0, 0, 0);
    acc = __builtin_amdgcn_mfma_f32_32x32x16_f16(a.lo, b.hi, acc, 0, 0, 0);
  } else {
    mma32<PREC>(acc, a, b);
  }
}

// As adj_mma, into a fresh accumulator (C = 0).
template <int PREC>
__device__ __forceinline__ void adj_mma_first(f32x16& acc, const Operand<PREC>& a, const Operand<PREC>& b) {
  if constexpr (PREC == kFP16) {
    const f32x16 z = {0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f};
    acc = __builtin_amdgcn_mfma_f32_32x32x16_f16(a.hi, b.hi, z, 0, 0, 0);
    acc = __builtin_amdgcn_mfma_f32_32x32x16_f16(a.hi, b.lo, acc, 0, 0, 0);
    acc = __builtin_amdgcn_mfma_f32_32x32x16_f16(a.lo, b.hi, acc, 0, 0, 0);
  } else {
    mma32_first<PREC>(acc, a, b);
  }
}

// FP16: multiply every accumulated row by 2^-e_m (the weight row's scale).
template <int PREC>
__device__ __forceinline__ void adj_unscale(f32x16 (&acc)[kAdjPB][kAdjMaxMb], const unsigned long long* rowmax,
                                            int b, int hh) {
  if constexpr (PREC == kFP16) {
#pragma unroll
    for (int mb = 0; mb < kAdjMaxMb; ++mb) {
#pragma unroll
      for (int i = 0; i < 16; ++i) {
        const int m = mb * 32 + 8 * (i / 4) + 4 * hh + (i % 4);
        const int e = adj_row_exp(rowmax, b * 64 + m);
#pragma unroll
        for (int pb = 0; pb < kAdjPB; ++pb) acc[pb][mb][i] = ldexpf(acc[pb][mb][i], -e);
      }
    }
  }
}

// One partner v of the order-3 adjoint: Y[mb] = sum over the chunks uc <= VC of the
// weight block (uc, mb) times the field operands, for the first NM m-blocks, then
// a_m += d_v Y[mb].  Straight-line code, so that the multiply-adds of one m-block are
// scheduled under the products of the next.
template <int PREC, int NM, int VC>
__device__ __forceinline__ void adj_partner(f32x16 (&acc)[kAdjPB][kAdjMaxMb], const float (&dv)[kAdjPB],
                                            const uint4* wv, const Operand<PREC> (&fop)[kAdjPB][4], int lane) {
  f32x16 Y[NM][kAdjPB];
  static_for<NM>([&](auto mbc) {
    constexpr int mb = decltype(mbc)::value;
    static_for<VC + 1>([&](auto ucc) {
      constexpr int uc = decltype(ucc)::value;
      const uint4* blk = wv + (uc * kAdjMaxMb + mb) * 2 * 64;
      const Operand<PREC> Wop = op_from_words<PREC>(blk[lane], blk[64 + lane]);
#pragma unroll
      for (int pb = 0; pb < kAdjPB; ++pb) {
        if constexpr (uc == 0) adj_mma_first<PREC>(Y[mb][pb], Wop, fop[pb][uc]);
        else adj_mma<PREC>(Y[mb][pb], Wop, fop[pb][uc]);
      }
    });
  });
#pragma unroll
  for (int mb = 0; mb < NM; ++mb)
#pragma unroll
    for (int pb = 0; pb < kAdjPB; ++pb)
#pragma unroll
      for (int i = 0; i < 16; ++i) acc[pb][mb][i] = fmaf(dv[pb], Y[mb][pb][i], acc[pb][mb][i]);
}

// Order 3.  A workgroup of 8 waves owns 512 grid points (each wave two 32-point
// column blocks) and every m.  For each partner v and 32-row block mb of m,
// Y = sum over the chunks uc <= v / 16 of W_v[uc, mb] d_u runs on the matrix cores with
// the register-held field operands as B, and a_m += d_v Y is one float32 multiply-add
// per accumulator element (forming d_u d_v for every chunk on the VALU instead, and
// accumulating on the matrix cores directly, measured slower).  The weight operands of
// kAdjVG values of v at a time are staged in LDS, double buffered: while one stage is in
// use the next one is copied in, a piece per v, with one barrier per stage.  Each weight
// block read from LDS feeds both column blocks.  Values of v, and (v, mb) blocks,
// without any weight (vmask: bit 2 uc + mb) are skipped.
// MBN: 32-row blocks of m that can hold a weight (1 when n_shells <= 32, else 2).
template <int PREC, int NF, int MBN>
__global__ __launch_bounds__(kAdjThreads, 1) void adjoint_gemm(const float* __restrict__ D,
                                                             const uint4* __restrict__ W,
                                                             const int* __restrict__ vmask,
                                                             const unsigned* __restrict__ absmax,
                                                             const unsigned long long* __restrict__ rowmax,
                                                             int n_shells, long long G, float* __restrict__ A,
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

  AdjFields<PREC, 4> f;
  adj_load_fields<PREC, 4>(f, Db, G, xw, hh, n_shells, absmax, b);
  // the fields as B operands (FP16: the split operands themselves)
  Operand<PREC> fop[kAdjPB][4];
#pragma unroll
  for (int pb = 0; pb < kAdjPB; ++pb)
#pragma unroll
    for (int uc = 0; uc < 4; ++uc) {
      if constexpr (PREC == kFP16) fop[pb][uc] = f.H[pb][uc];
      else fop[pb][uc] = make_operand<PREC>(f.F[pb][uc], 1.f);
    }

  // the weight-block masks of every v, one per lane (bit 2 uc + mb)
  const int vml = lane < n_shells ? vmask[lane] : 0;

  const uint4* Wb = W + (size_t)b * n_shells * kAdjWPerV;
  const int n_stages = (n_shells + kAdjVG - 1) / kAdjVG;
  u32x4 wp[kAdjPiece];   // a native vector: an array of uint4 here ends up in scratch memory
  // piece q of stage s: words (q kAdjPiece + k) kAdjThreads + tid of the stage.  Words of
  // v >= n_shells (a last, partial stage) are never read from LDS, so their loads only
  // need to stay in bounds: they reread the batch's first words.  No branch around the
  // load: a guarded load makes the compiler wait for it on the spot.
  auto w_load = [&](int s, int q) {
#pragma unroll
    for (int k = 0; k < kAdjPiece; ++k) {
      const int i = (q * kAdjPiece + k) * kAdjThreads + tid;
      const int v = s * kAdjVG + i / kAdjWPerV;
      wp[k] = *reinterpret_cast<const u32x4*>(Wb + (v < n_shells ? (size_t)s * kAdjStageWords + i : (size_t)i));
    }
  };
  auto w_store = [&](int buf, int q) {
#pragma unroll
    for (int k = 0; k < kAdjPiece; ++k) *reinterpret_cast<u32x4*>(&wst[buf][(q * kAdjPiece + k) * kAdjThreads + tid]) = wp[k];
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

  static_for<4>([&](auto vcc) {            // static v: register indices stay compile-time
    constexpr int vc = decltype(vcc)::value;
    if (16 * vc >= n_shells) return;
    static_for<16>([&](auto vvc) {
      constexpr int vv = decltype(vvc)::value;
      const int v = 16 * vc + vv;
      if (v >= n_shells) return;
      const int st = v / kAdjVG, vi = v % kAdjVG;
      const bool more = st + 1 < n_stages;
      if (more) {                 // copy the next stage in, one piece per v
        if (vi > 0) w_store((st + 1) & 1, vi - 1);
        w_load(st + 1, vi);
      }
      const int mask = __builtin_amdgcn_readlane(vml, v);
      if (mask != 0) {
        const uint4* wv = wst[st & 1] + vi * kAdjWPerV;
        // d_v at the lane's points as float32 (FP16: the scaled value)
        float dv[kAdjPB];
#pragma unroll
        for (int pb = 0; pb < kAdjPB; ++pb) {
          const unsigned w = adj_scalar<PREC, 4, vc, vv>(f, pb);
          if constexpr (PREC == kFP16)
            dv[pb] = (float)__builtin_bit_cast(_Float16, (unsigned short)(w & 0xffffu)) +
                     (float)__builtin_bit_cast(_Float16, (unsigned short)(w >> 16));
          else
            dv[pb] = __uint_as_float(w);
        }
        if constexpr (PREC != kFP16 && vc > 0) {
          adj_partner<PREC, MBN, vc>(acc, dv, wv, fop, lane);   // every block, straight-line
        } else {
          // blocks (uc, mb) without a weight skipped (v < 16: one chunk, and m-block 1
          // rarely holds a weight; FP16: the straight-line form spills registers)
#pragma unroll
          for (int mb = 0; mb < MBN; ++mb) {
            if (!(mask & (0x55 << mb))) continue;   // no weight in this block of m
            f32x16 Y[kAdjPB];
            static_for<vc + 1>([&](auto ucc) {
              constexpr int uc = decltype(ucc)::value;
              const bool on = (mask >> (2 * uc + mb)) & 1;   // a weight in block (uc, mb)
              if (on) {
                const uint4* blk = wv + (uc * kAdjMaxMb + mb) * 2 * 64;
                const Operand<PREC> Wop = op_from_words<PREC>(blk[lane], blk[64 + lane]);
#pragma unroll
                for (int pb = 0; pb < kAdjPB; ++pb) {
                  if constexpr (uc == 0) adj_mma_first<PREC>(Y[pb], Wop, fop[pb][uc]);
                  else adj_mma<PREC>(Y[pb], Wop, fop[pb][uc]);
                }
              } else if constexpr (uc == 0) {
#pragma unroll
                for (int pb = 0; pb < kAdjPB; ++pb)
#pragma unroll
                  for (int i = 0; i < 16; ++i) Y[pb][i] = 0.f;
              }
            });
#pragma unroll
            for (int pb = 0; pb < kAdjPB; ++pb)
#pragma unroll
              for (int i = 0; i < 16; ++i) acc[pb][mb][i] = fmaf(dv[pb], Y[pb][i], acc[pb][mb][i]);
          }
        }
      }
      if (more && (vi == kAdjVG - 1)) {
        w_store((st + 1) & 1, kAdjVG - 1);
        __syncthreads();          // the next stage is complete; this one is free
      }
    });
  });
  adj_unscale<PREC>(acc, rowmax, b, hh);
  adjoint_epilogue<NF>(acc, lds, lane, wave, hh, col, b, xw, n_shells, G, A, H2, tw, g);
}

// Order 4 (NC = 2: at most 32 shells, one 32-row block of m; NC = 4: at most 64 shells,
// two blocks).  Items (w, v <= w) in order of w; for each item and block of m,
// Y = sum over the chunks uc <= v / 16 of W4_(v,w) d_u runs on the matrix
// cores with the fields themselves as the B operand, and a_m += d_v d_w Y on the VALU,
// one float32 multiply-add per accumulator element (FP16: the scaled scalar times 2^-7,
// the shift that the weights' row exponents carry).  Forming d_u d_v d_w for every item
// and chunk instead cost more VALU instructions than the MFMAs could hide.  The weights
// pass through LDS in stages of adj4_stage_items items of one w (8 for NC = 2, 2 for 4),
// double buffered: the next stage is loaded into registers while one is in use, then
// stored, with one barrier per stage.  d_w and the item masks of the next w are likewise
// loaded a w ahead.
template <int PREC, int NF, int NC>
__global__ __launch_bounds__(kAdjThreads, 1) void adjoint4_gemm(const float* __restrict__ D,
                                                              const uint4* __restrict__ W,
                                                              const int* __restrict__ imask,
                                                              const unsigned* __restrict__ absmax,
                                                              const unsigned long long* __restrict__ rowmax,
                                                              int n_shells, long long G, float* __restrict__ A,
                                                              cplx<float>* __restrict__ H2,
                                                              const cplx<float>* __restrict__ tw, Geom g) {
  constexpr int MB = NC / 2;                               // 32-row blocks of m
  constexpr int WPI = adj4_words_per_item(16 * NC);       // operand words per item
  constexpr int SI = adj4_stage_items<NC>();
  constexpr int SW = adj4_stage_words<NC>();
  constexpr int PIECE = adj4_piece<NC>();
  __shared__ __attribute__((aligned(16))) unsigned char lds[adj4_lds_bytes<NF, NC>()];
  auto wst = reinterpret_cast<uint4(*)[SW]>(lds);
  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const int wave = tid >> 6;
  const int hh = lane >> 5, col = lane & 31;
  const int b = blockIdx.y;
  const long long xw = (long long)blockIdx.x * kAdjPts + wave * 32 * kAdjPB + col;
  const float* Db = D + (size_t)b * n_shells * G;
  const int n_items = n_shells * (n_shells + 1) / 2;
  const uint4* Wb = W + (size_t)b * n_items * WPI;
  const int* Ib = imask;   // one mask per item, shared by the batch

  AdjFields<PREC, NC> f;
  adj_load_fields<PREC, NC>(f, Db, G, xw, hh, n_shells, absmax, b);
  // the fields as B operands (FP16: the split operands themselves)
  Operand<PREC> fop[kAdjPB][NC];
#pragma unroll
  for (int pb = 0; pb < kAdjPB; ++pb)
#pragma unroll
    for (int uc = 0; uc < NC; ++uc) {
      if constexpr (PREC == kFP16) fop[pb][uc] = f.H[pb][uc];
      else fop[pb][uc] = make_operand<PREC>(f.F[pb][uc], 1.f);
    }
  f32x16 acc[kAdjPB][kAdjMaxMb];
#pragma unroll
  for (int pb = 0; pb < kAdjPB; ++pb)
#pragma unroll
    for (int mb = 0; mb < kAdjMaxMb; ++mb)
#pragma unroll
      for (int i = 0; i < 16; ++i) acc[pb][mb][i] = 0.f;

  // stage (w, c): items w (w + 1) / 2 + SI c + k, k < SI.  Items past w are never read
  // from LDS; their loads only stay in bounds (they reread the first item).
  u32x4 wp[PIECE];
  auto s_load = [&](int w, int c) {
    const size_t base = (size_t)(w * (w + 1) / 2 + SI * c) * WPI;
#pragma unroll
    for (int k = 0; k < PIECE; ++k) {
      const int i = k * kAdjThreads + tid;
      const bool real = SI * c + i / WPI <= w;
      wp[k] = *reinterpret_cast<const u32x4*>(Wb + (real ? base + i : (size_t)(i % WPI)));
    }
  };
  auto s_store = [&](int buf) {
#pragma unroll
    for (int k = 0; k < PIECE; ++k) *reinterpret_cast<u32x4*>(&wst[buf][k * kAdjThreads + tid]) = wp[k];
  };
  s_load(0, 0);
  s_store(0);
  // d_w at the lane's points and the masks of the items (w, v = lane), a w ahead
  float dw_next[kAdjPB];
#pragma unroll
  for (int pb = 0; pb < kAdjPB; ++pb) dw_next[pb] = Db[xw + 32 * pb];
  int mask_next = lane == 0 ? Ib[0] : 0;
  __syncthreads();

  int buf = 0;
  for (int w = 0; w < n_shells; ++w) {
    float dw[kAdjPB];   // FP16: d_w scaled like the register fields, times 2^-7
#pragma unroll
    for (int pb = 0; pb < kAdjPB; ++pb) {
      if constexpr (PREC == kFP16) dw[pb] = ldexpf(dw_next[pb], shell_scale_exp(absmax, b * n_shells + w) - kTripleShift);
      else dw[pb] = dw_next[pb];
    }
    const int my_mask = mask_next;
    if (w + 1 < n_shells) {
#pragma unroll
      for (int pb = 0; pb < kAdjPB; ++pb) dw_next[pb] = Db[(size_t)(w + 1) * G + xw + 32 * pb];
      const int it1 = (w + 1) * (w + 2) / 2;
      mask_next = lane <= w + 1 ? Ib[it1 + lane] : 0;
    }
    static_for<16 * NC / SI>([&](auto cc) {
      constexpr int c = decltype(cc)::value;
      if (SI * c > w) return;
      int nw = w, nc = c + 1;                       // the stage after this one
      if (SI * nc > w) {
        nw = w + 1;
        nc = 0;
      }
      const bool more = nw < n_shells;
      if (more) s_load(nw, nc);
      static_for<SI>([&](auto kc) {
        constexpr int k = decltype(kc)::value;
        constexpr int v = SI * c + k;
        constexpr int vc = v / 16, vv = v % 16;
        if (v > w) return;
        const int mask = __builtin_amdgcn_readlane(my_mask, v);   // bit 2 uc + mb
        if (!mask) return;
        const uint4* wv = wst[buf] + k * WPI;
        if constexpr (MB == 1) {
          // one block of m: the chain, then the scalar and the multiply-adds
          f32x16 Y[kAdjPB];
          static_for<vc + 1>([&](auto ucc) {
            constexpr int uc = decltype(ucc)::value;   // no branch per chunk (zero weights where empty)
            const Operand<PREC> Wop = op_from_words<PREC>(wv[uc * 128 + lane], wv[uc * 128 + 64 + lane]);
#pragma unroll
            for (int pb = 0; pb < kAdjPB; ++pb) {
              if constexpr (uc == 0) adj_mma_first<PREC>(Y[pb], Wop, fop[pb][uc]);
              else adj_mma<PREC>(Y[pb], Wop, fop[pb][uc]);
            }
          });
#pragma unroll
          for (int pb = 0; pb < kAdjPB; ++pb) {
            const unsigned dv = adj_scalar<PREC, NC, vc, vv>(f, pb);
            float sv;
            if constexpr (PREC == kFP16)
              sv = (float)__builtin_bit_cast(_Float16, (unsigned short)(dv & 0xffffu)) +
                   (float)__builtin_bit_cast(_Float16, (unsigned short)(dv >> 16));
            else
              sv = __uint_as_float(dv);
            const float sc = sv * dw[pb];
#pragma unroll
            for (int i = 0; i < 16; ++i) acc[pb][0][i] = fmaf(sc, Y[pb][i], acc[pb][0][i]);
          }
        } else {
          float sc[kAdjPB];
#pragma unroll
          for (int pb = 0; pb < kAdjPB; ++pb) {
            const unsigned dv = adj_scalar<PREC, NC, vc, vv>(f, pb);
            float sv;
            if constexpr (PREC == kFP16)
              sv = (float)__builtin_bit_cast(_Float16, (unsigned short)(dv & 0xffffu)) +
                   (float)__builtin_bit_cast(_Float16, (unsigned short)(dv >> 16));
            else
              sv = __uint_as_float(dv);
            sc[pb] = sv * dw[pb];
          }
#pragma unroll
          for (int mb = 0; mb < MB; ++mb) {
            if (!(mask & (0x55 << mb))) continue;   // no weight in this block of m
            f32x16 Y[kAdjPB];
            static_for<vc + 1>([&](auto ucc) {
              constexpr int uc = decltype(ucc)::value;
              const uint4* wb = wv + (uc * MB + mb) * 128;
              const Operand<PREC> Wop = op_from_words<PREC>(wb[lane], wb[64 + lane]);
#pragma unroll
              for (int pb = 0; pb < kAdjPB; ++pb) {
                if constexpr (uc == 0) adj_mma_first<PREC>(Y[pb], Wop, fop[pb][uc]);
                else adj_mma<PREC>(Y[pb], Wop, fop[pb][uc]);
              }
            });
#pragma unroll
            for (int pb = 0; pb < kAdjPB; ++pb)
#pragma unroll
              for (int i = 0; i < 16; ++i) acc[pb][mb][i] = fmaf(sc[pb], Y[pb][i], acc[pb][mb][i]);
          }
        }
      });
      if (more) s_store(buf ^ 1);
      __syncthreads();                              // the next stage is complete; this one is free
      buf ^= 1;
    });
  }
  adj_unscale<PREC>(acc, rowmax, b, hh);
  adjoint_epilogue<NF>(acc, lds, lane, wave, hh, col, b, xw, n_shells, G, A, H2, tw, g);
}

template <int PREC>
hipError_t launch_adjoint_gemm_prec(const float* D, const uint4* W, const int* vmask, const unsigned* absmax,
                                    const unsigned long long* rowmax, int n_shells, long long G, float* A,
                                    cplx<float>* H2, const cplx<float>* tw, Geom g, int batch, hipStream_t st) {
  dim3 grid((unsigned)(G / kAdjPts), batch);
#define L2(NF, MBN) hipLaunchKernelGGL((adjoint_gemm<PREC, NF, MBN>), grid, dim3(kAdjThreads), 0, st, D, W, vmask, \
                                       absmax, rowmax, n_shells, G, A, H2, tw, g)
#define L(NF) do { if (n_shells > 32) L2(NF, 2); else L2(NF, 1); } while (0)
  switch (g.N) {
    case 32: L(32); break;
    case 64: L(64); break;
    case 128: L(128); break;
    case 256: L(256); break;
    case 512: L(512); break;
    default: L(0); break;
  }
#undef L
#undef L2
  return hipGetLastError();
}

template <int PREC>
hipError_t launch_adjoint4_gemm_prec(const float* D, const uint4* W, const int* imask, const unsigned* absmax,
                                     const unsigned long long* rowmax, int n_shells, long long G, float* A,
                                     cplx<float>* H2, const cplx<float>* tw, Geom g, int batch, hipStream_t st) {
  dim3 grid((unsigned)(G / kAdjPts), batch);
#define L4(NF, NC) hipLaunchKernelGGL((adjoint4_gemm<PREC, NF, NC>), grid, dim3(kAdjThreads), 0, st, D, W, imask, \
                                      absmax, rowmax, n_shells, G, A, H2, tw, g)
#define L(NF)                      \
  do {                             \
    if (n_shells <= 32) L4(NF, 2); \
    else L4(NF, 4);                \
  } while (0)
  switch (g.N) {
    case 32: L(32); break;
    case 64: L(64); break;
    case 128: L(128); break;
    case 256: L(256); break;
    case 512: L(512); break;
    default: L(0); break;
  }
#undef L
#undef L4
  return hipGetLastError();
}

}  // namespace ps
