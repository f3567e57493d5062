// One (operator, precision) pair of the per-operator kernels: the stencil
// kernel and, for working-precision storage, the single-workgroup solve.  The
// build compiles this file once per pair with JFNK_OP (operator type),
// JFNK_T (arithmetic type), JFNK_VT (storage type of the tangent) and
// JFNK_FUSED (1: also the single-workgroup solve) defined.
#include "launch_stencil.hpp"

namespace jfnk {

template hipError_t launch_stencil_p<JFNK_OP, JFNK_T, JFNK_VT>(int, int, bool, bool, const StencilArgs<JFNK_T, JFNK_VT>&,
                                                               const Coefs&, int, hipStream_t, int*);
#if JFNK_FUSED
template hipError_t launch_fused_p<JFNK_OP, JFNK_T>(const FusedArgs<JFNK_T>&, size_t, hipStream_t);
#endif

}  // namespace jfnk
