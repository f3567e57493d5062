// FP16-storage instantiation: FP32 arithmetic, Krylov basis and JVP tangent in FP16.
#include "launch_impl.hpp"

namespace jfnk {

JFNK_INSTANTIATE(float, __half)

}  // namespace jfnk
