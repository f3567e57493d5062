// FP32 instantiation of the JFNK kernels and launchers.
#include "launch_impl.hpp"

namespace jfnk {

JFNK_INSTANTIATE(float, float)
JFNK_INSTANTIATE_SCALAR(float)

}  // namespace jfnk
