// Adjoint products (orders 3 and 4) instantiated for one precision; see adjoint.h.
#include "adjoint.h"

namespace ps {

template hipError_t launch_adjoint_gemm_prec<kFP16>(const float*, const uint4*, const int*, const unsigned*,
                                                 const unsigned long long*, int, long long, float*, cplx<float>*,
                                                 const cplx<float>*, Geom, int, hipStream_t);
template hipError_t launch_adjoint4_gemm_prec<kFP16>(const float*, const uint4*, const int*, const unsigned*,
                                                  const unsigned long long*, int, long long, float*, cplx<float>*,
                                                  const cplx<float>*, Geom, int, hipStream_t);

}  // namespace ps
