// Tile contraction, orders 5 (pair x triple) and 6 (triple x triple).
#include "contract_tiles.h"

namespace ps {

hipError_t launch_contract_hi(int prec, int order, const CtrParams& p, int n_groups, int batch, hipStream_t st) {
  dim3 grid(p.n_chunks, n_groups, batch);
  if (p.n_blk > 4) return hipErrorInvalidValue;   // orders 5 and 6 hold at most 32 shells
#define L(P, O) hipLaunchKernelGGL((contract_tiles<P, O, 4>), grid, dim3(kCtrThreads), 0, st, p)
  if (order == 5) {
    if (prec == kFP32) L(kFP32, 5); else if (prec == kBF16) L(kBF16, 5); else L(kFP16, 5);
  } else if (order == 6) {
    if (prec == kFP32) L(kFP32, 6); else if (prec == kBF16) L(kBF16, 6); else L(kFP16, 6);
  } else {
    return hipErrorInvalidValue;
  }
#undef L
  return hipGetLastError();
}

}  // namespace ps
