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
// One workgroup (16 waves) owns a contiguous chunk of grid points and every tile;
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
#include "contract_tiles.h"

namespace ps {

// Orders 2 to 4 here; orders 5 and 6 in contract_tiles_hi.hip (launch_contract_hi).
hipError_t launch_contract_hi(int prec, int order, const CtrParams& p, int n_groups, int batch, hipStream_t st);

hipError_t launch_contract(int prec, int order, const CtrParams& p, int n_groups, int batch, hipStream_t st) {
  if (order >= 5) return launch_contract_hi(prec, order, p, n_groups, batch, st);
  if (p.n_blk > 8) return hipErrorInvalidValue;
  dim3 grid(p.n_chunks, n_groups, batch);
  // 4 staged shell blocks (up to 64 shells) keep the LDS small enough for two
  // workgroups per CU; 8 blocks take up to 128 shells
#define L(P, O, MB) hipLaunchKernelGGL((contract_tiles<P, O, MB>), grid, dim3(kCtrThreads), 0, st, p)
#define BY_MB(P, O) do { if (p.n_blk <= 4) L(P, O, 4); else L(P, O, 8); } while (0)
#define BY_PREC(O) do { if (prec == kFP32) BY_MB(kFP32, O); else if (prec == kBF16) BY_MB(kBF16, O); else BY_MB(kFP16, O); } while (0)
  if (order == 2) BY_PREC(2);
  else if (order == 3) BY_PREC(3);
  else if (order == 4 && prec == kFP16 && p.n_pair_blocks > 0) {
    if (p.n_pair_blocks > kMaxPairBlocksHost || p.n_blk > 4) return hipErrorInvalidValue;
    hipLaunchKernelGGL((contract_tiles<kFP16, 4, 4, true>), grid, dim3(kCtrThreads), 0, st, p);
  } else if (order == 4) BY_PREC(4);
  else return hipErrorInvalidValue;
#undef BY_PREC
#undef BY_MB
#undef L
  return hipGetLastError();
}

}  // namespace ps
