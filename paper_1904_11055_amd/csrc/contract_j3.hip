#include "mfma_ops.h"

namespace ps {

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


template <int PREC>
__global__ __launch_bounds__(kJThreads, 1) void contract_j3(CtrJParams p) {
  static_assert(PREC == kFP16, "shell-block aligned contraction is implemented for the FP16 split");
  __shared__ uint4 opHi[2][2][kMaxBlk][64];   // [buffer][K-step][shell block][lane]
  __shared__ uint4 opLo[2][2][kMaxBlk][64];
  __shared__ float lds_scale[kMaxBlk * 16];

  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const int my_slot = op_slot(lane);
  const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int chunk = blockIdx.x;
  const int b = blockIdx.z;

  for (int i = tid; i < kMaxBlk * 16; i += kJThreads)
    lds_scale[i] = i < p.n_shells ? ldexpf(1.0f, shell_scale_exp(p.absmax, b * p.n_shells + i)) : 0.f;
  for (int i = tid; i < 4 * kMaxBlk * 64; i += kJThreads) {
    const int bh = i / (kMaxBlk * 64), kb = (i / 64) % kMaxBlk, ln = i % 64;
    if (kb * 16 + (ln & 15) >= p.n_shells) {
      opHi[bh >> 1][bh & 1][kb][op_slot(ln)] = make_uint4(0, 0, 0, 0);
      opLo[bh >> 1][bh & 1][kb][op_slot(ln)] = make_uint4(0, 0, 0, 0);
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
    const int h = col >> 5, kb = row >> 4, ln = op_slot((((col & 31) >> 3) << 4) | (row & 15)), half = (col >> 2) & 1;
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
      for (int kb = 0; kb < kMaxBlk; ++kb) Bop[kb] = op_from_words<PREC>(opHi[cur][h][kb][my_slot], opLo[cur][h][kb][my_slot]);
      static_for<8>([&](auto qc) {
        constexpr int q = decltype(qc)::value;
        constexpr int jb = q / 2;
        const int j = wave + kJWaves * q;
        if (j >= p.n_shells) return;
        const int rj = op_slot((lane & 0x30) | (j & 15));
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

hipError_t launch_contract_j3(int prec, const CtrJParams& p, int batch, hipStream_t st) {
  if (prec != kFP16) return hipErrorInvalidValue;
  dim3 grid(p.n_chunks, 1, batch);
  hipLaunchKernelGGL(contract_j3<kFP16>, grid, dim3(kJThreads), 0, st, p);
  return hipGetLastError();
}

}  // namespace ps
