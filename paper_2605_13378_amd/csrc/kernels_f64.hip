// FP64 instantiation of the JFNK kernels and launchers.
#include "launch_impl.hpp"

namespace jfnk {

JFNK_INSTANTIATE(double, double)
JFNK_INSTANTIATE_SCALAR(double)

hipError_t launch_ctl_begin(Ctl* c, double tol, double brk_tol, int m, hipStream_t s) {
  JFNK_LAUNCH(ctl_begin_kernel<0>, dim3(1), dim3(64), s, c, tol, brk_tol, m);
  return hipGetLastError();
}

hipError_t launch_fp16_tangent(long long n, const float* v, __half* out, const double* vn2, double* inv_sigma,
                               int grid, hipStream_t s) {
  JFNK_LAUNCH(fp16_tangent_kernel<0>, dim3(grid), dim3(kStreamThreads), s, n, v, out, vn2, inv_sigma);
  return hipGetLastError();
}

hipError_t launch_cycle_begin(Ctl* c, Partials in, int m, long long n, int fp16, hipStream_t s) {
  JFNK_LAUNCH(cycle_begin_kernel<0>, dim3(1), dim3(kStreamThreads), s, c, in, m, n, fp16);
  return hipGetLastError();
}

hipError_t launch_publish_ctl(const Ctl* c, int* dst, int words, int* seq_dst, int seq, hipStream_t s) {
  JFNK_LAUNCH(publish_ctl_kernel<0>, dim3(1), dim3(64), s, c, dst, words, seq_dst, seq);
  return hipGetLastError();
}

hipError_t launch_finish_sums(Partials in, int nr, double* out0, double* out1, hipStream_t s) {
  JFNK_LAUNCH(finish_sums_kernel<0>, dim3(1), dim3(kStreamThreads), s, in, nr, out0, out1);
  return hipGetLastError();
}

}  // namespace jfnk
