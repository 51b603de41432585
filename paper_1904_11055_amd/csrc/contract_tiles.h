// Tile contraction kernel template (orders 2 to 6); instantiated by
// contract_tiles_lo.hip and contract_tiles_hi.hip.
#pragma once

#include "mfma_ops.h"

namespace ps {

template <int ORDER>
constexpr int slots_for() { return ORDER == 2 ? 4 : ORDER == 3 ? kSlots : ORDER == 4 ? kSlots4 : ORDER == 5 ? kSlots56 : kSlots6; }

constexpr int kMaxPairBlocks = kMaxPairBlocksHost;

// MB: shell blocks of 16 staged per K-step (4: up to 64 shells; 8: up to 128, orders 2 to 4).
// PLDS (order 4, FP16): at the start of each K-step every pair block's operands (both
// 32-point halves) are formed once, by the waves in turn, into LDS, and each slot reads
// its A and B operands from there; otherwise each slot forms them itself from the staged
// shell words, which costs more VALU instructions than its three MFMAs can hide.
template <int PREC, int ORDER, int MB, bool PLDS = false>
__global__ __launch_bounds__(kCtrThreads, 1) void contract_tiles(CtrParams p) {
  static_assert(!PLDS || (ORDER == 4 && PREC == kFP16), "shared pair operands: order 4, split FP16");
  // FP16 up to order 4 forms pair products from the operand words alone; the other
  // precisions, and every precision at orders 5 and 6, form their row products from
  // float32 rows staged in `stage`
  constexpr bool kFloatStage = PREC != kFP16 || ORDER >= 5;
  // FP16 needs the per-shell power-of-two scaling for its range; at orders 5 and 6 every
  // precision takes it, since unscaled products of five or six shell values summed over
  // the grid overflow float32 (they reach 1e45 at 256^3)
  constexpr bool kScaled = PREC == kFP16 || ORDER >= 5;
  constexpr int kStageFloats = kFloatStage ? (MB * 16 + 1) * kRowStride : 4;
  __shared__ __attribute__((aligned(16))) float stage[2][kStageFloats];
  // [buffer][K-step][shell block][lane]; block MB stays zero (padding pairs)
  __shared__ uint4 opHi[2][2][MB + 1][64];
  __shared__ uint4 opLo[2][2][MB + 1][64];
  __shared__ float lds_scale[MB * 16 + 1];
  // [32-point half][pair block][hi, lo][lane]
  __shared__ uint4 pairOp[PLDS ? 2 * kMaxPairBlocks * 2 * 64 : 1];

  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const int my_slot = op_slot(lane);
  auto pair_word = [&](int h, int pb, int part) -> uint4& { return pairOp[((h * kMaxPairBlocks + pb) * 2 + part) * 64 + lane]; };
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
  for (int i = tid; ORDER <= 4 && i < 4 * (MB + 1) * 64; i += kCtrThreads) {
    const int bh = i / ((MB + 1) * 64), kb = (i / 64) % (MB + 1), ln = i % 64;
    if (kb * 16 + (ln & 15) >= p.n_shells) {
      opHi[bh >> 1][bh & 1][kb][op_slot(ln)] = make_uint4(0, 0, 0, 0);
      opLo[bh >> 1][bh & 1][kb][op_slot(ln)] = make_uint4(0, 0, 0, 0);
    }
  }

  constexpr int NS = slots_for<ORDER>();
  f32x4 acc[NS];
#pragma unroll
  for (int s = 0; s < NS; ++s) acc[s] = f32x4{0.f, 0.f, 0.f, 0.f};

  // global -> LDS staging: thread t moves float4 #(t + 1024 q), q < SP, of the
  // (staged rows x 64) slice and also writes it, split, into the operand arrays of its
  // shell block and K-step
  constexpr int SP = MB / 4;
  const float* Db = p.D + (size_t)b * p.n_shells * p.G;
  const long long x_base = (long long)chunk * p.ksteps * kKStep;
  int st_row[SP], st_col[SP];
#pragma unroll
  for (int q = 0; q < SP; ++q) {
    st_row[q] = (tid + q * kCtrThreads) >> 4;
    st_col[q] = (tid & 15) * 4;
  }
  auto stage_store = [&](int buf, int q, float4 v) {
    const int row = st_row[q], col = st_col[q];
    const int kb = row >> 4, h = col >> 5, half = (col >> 2) & 1;
    const int ln = op_slot((((col & 31) >> 3) << 4) | (row & 15));
    if (kScaled) {  // every operand works on the power-of-two scaled values
      const float sc = lds_scale[row];
      v = make_float4(v.x * sc, v.y * sc, v.z * sc, v.w * sc);
    }
    if constexpr (kFloatStage) *reinterpret_cast<float4*>(&stage[buf][row * kRowStride + col]) = v;
    if constexpr (ORDER >= 5) {
      // every operand is formed from the float rows
    } else if constexpr (PREC == kFP32) {
      const uint4 w = make_uint4(__float_as_uint(v.x), __float_as_uint(v.y), __float_as_uint(v.z),
                                 __float_as_uint(v.w));
      if (half) opLo[buf][h][kb][ln] = w; else opHi[buf][h][kb][ln] = w;
    } else {
      uint2 hi, lo;
      split4<PREC>(v, 1.f, hi, lo);
      reinterpret_cast<uint2*>(&opHi[buf][h][kb][ln])[half] = hi;
      reinterpret_cast<uint2*>(&opLo[buf][h][kb][ln])[half] = lo;
    }
  };
  float4 pre[SP];
#pragma unroll
  for (int q = 0; q < SP; ++q) {
    pre[q] = make_float4(0.f, 0.f, 0.f, 0.f);
    if (st_row[q] < p.n_shells) pre[q] = *reinterpret_cast<const float4*>(Db + (size_t)st_row[q] * p.G + x_base + st_col[q]);
  }
  __syncthreads();
#pragma unroll
  for (int q = 0; q < SP; ++q)
    if (st_row[q] < p.n_shells) stage_store(0, q, pre[q]);
  __syncthreads();

  // Slot state for the whole chunk.  Uniform byte per slot (4 slots per word, in
  // SGPRs): bits 0-2 B shell block, 3-5 A shell block (order 2), 6 = form A here,
  // 7 = empty.  Per-lane shells of the lane's pair rows: order 3 packs (u, v) of
  // two slots per word, order 4 packs (u_A, v_A, u_B, v_B) of one slot per word;
  // orders 5 and 6 use two words per slot, the A row's shells then the B row's.
  constexpr int NLW = ORDER == 4 ? NS : ORDER >= 5 ? 2 * NS : (NS + 1) / 2;
  const int* uni = p.slot_uni + ((size_t)group * kCtrWaves + wave) * (kSlotsMax / 4);
  int un[(NS + 3) / 4];
#pragma unroll
  for (int i = 0; i < (NS + 3) / 4; ++i) un[i] = __builtin_amdgcn_readfirstlane(uni[i]);
  int lv[NLW];
  if (ORDER >= 3 && !PLDS) {
    const int* lw = p.slot_lane + (((size_t)group * kCtrWaves + wave) * 16 + row) * kSlotsMax;
#pragma unroll
    for (int i = 0; i < NLW; ++i) lv[i] = lw[i];
  }
  // PLDS: the slots' pair blocks (uniform) and the pairs this lane forms each K-step
  constexpr int kForm = PLDS ? (2 * kMaxPairBlocks + kCtrWaves - 1) / kCtrWaves : 1;
  // pair blocks formed per K-step: all of the plan's, or the tile group's own
  const int n_local = PLDS ? (p.grp_nblk ? p.grp_nblk[group] : p.n_pair_blocks) : 0;
  int blk[PLDS ? NS : 1];
  int fuv[kForm];
  if constexpr (PLDS) {
    const int* bw = p.slot_blk + ((size_t)group * kCtrWaves + wave) * kSlotsMax;
#pragma unroll
    for (int s = 0; s < NS; ++s) blk[s] = __builtin_amdgcn_readfirstlane(bw[s]);
#pragma unroll
    for (int f = 0; f < kForm; ++f) {
      const int t = wave + f * kCtrWaves;           // (pair block t / 2, half t % 2)
      int gb = t >> 1;                              // the block's global id
      if (p.grp_blk) gb = t < 2 * n_local ? p.grp_blk[group * kMaxPairBlocks + (t >> 1)] : 0;
      const int w = t < 2 * n_local ? p.pair_uv[16 * gb + row] : 0;
      fuv[f] = (w & 0xff) | (((w >> 16) & 0xff) << 8);
    }
  }
  for (int ks = 0; ks < p.ksteps; ++ks) {
    const int cur = ks & 1;
    if (ks + 1 < p.ksteps) {
#pragma unroll
      for (int q = 0; q < SP; ++q)
        if (st_row[q] < p.n_shells)
          pre[q] = *reinterpret_cast<const float4*>(Db + (size_t)st_row[q] * p.G + x_base + (ks + 1) * kKStep + st_col[q]);
    }
    const float* S = stage[cur];
    if constexpr (PLDS) {
#pragma unroll
      for (int f = 0; f < kForm; ++f) {
        const int t = wave + f * kCtrWaves;
        if (t < 2 * n_local) {
          const Operand<kFP16> o = form_pair_f16(opHi[cur][t & 1], opLo[cur][t & 1], fuv[f], lane);
          pair_word(t & 1, t >> 1, 0) = __builtin_bit_cast(uint4, o.hi);
          pair_word(t & 1, t >> 1, 1) = __builtin_bit_cast(uint4, o.lo);
        }
      }
      __syncthreads();                              // every pair operand of the K-step is in LDS
    }
#pragma unroll
    for (int h = 0; h < 2; ++h) {
      Operand<PREC> A;
#pragma unroll
      for (int s = 0; s < NS; ++s) {
        const int info = (un[s / 4] >> (8 * (s % 4))) & 0xff;
        if (info & 0x80) break;
        if constexpr (PLDS) {
          if (info & 0x40) {
            const int a = blk[s] & 0xffff;
            A = op_from_words<PREC>(pair_word(h, a, 0), pair_word(h, a, 1));
          }
          const int bb = blk[s] >> 16;
          const Operand<PREC> Bp = op_from_words<PREC>(pair_word(h, bb, 0), pair_word(h, bb, 1));
          mma<PREC>(acc[s], A, Bp);
          continue;
        }
        if constexpr (ORDER >= 5) {
          if (info & 0x40) A = form_rows<PREC, ORDER == 6 ? 3 : 2>(S + 32 * h, lv[2 * s], g);
          const Operand<PREC> Bop = form_rows<PREC, 3>(S + 32 * h, lv[2 * s + 1], g);
          mma<PREC>(acc[s], A, Bop);
          continue;
        }
        if (ORDER == 2) {
          const int ab = (info >> 3) & 7;
          A = op_from_words<PREC>(opHi[cur][h][ab][my_slot], opLo[cur][h][ab][my_slot]);
        } else if (info & 0x40) {
          const int uv = ORDER == 3 ? (lv[s / 2] >> (16 * (s % 2))) & 0xffff : lv[s] & 0xffff;
          if constexpr (PREC == kFP16) A = form_pair_f16(opHi[cur][h], opLo[cur][h], uv, lane);
          else A = form_pair<PREC>(S + 32 * h, uv, g);
        }
        Operand<PREC> Bop;
        if (ORDER == 4) {
          if constexpr (PREC == kFP16) Bop = form_pair_f16(opHi[cur][h], opLo[cur][h], (lv[s] >> 16) & 0xffff, lane);
          else Bop = form_pair<PREC>(S + 32 * h, (lv[s] >> 16) & 0xffff, g);
        } else {
          const int bb = info & 7;
          Bop = op_from_words<PREC>(opHi[cur][h][bb][my_slot], opLo[cur][h][bb][my_slot]);
        }
        mma<PREC>(acc[s], A, Bop);
      }
    }
    if (ks + 1 < p.ksteps) {
#pragma unroll
      for (int q = 0; q < SP; ++q)
        if (st_row[q] < p.n_shells) stage_store(cur ^ 1, q, pre[q]);
    }
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

}  // namespace ps
