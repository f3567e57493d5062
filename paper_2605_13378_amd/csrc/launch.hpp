// Host-side launchers for the JFNK kernels.  Declarations only; the
// definitions live in launch_impl.hpp and are instantiated once per
// precision (kernels_f64.hip, kernels_f32.hip, kernels_f16.hip) so the
// translation units compile in parallel.
#pragma once

#include <hip/hip_runtime.h>

#include "common.hpp"
#include "krylov.hpp"
#include "problems.hpp"
#include "stencil.hpp"

namespace jfnk {

enum ProblemKind { kBurgers1D = 0, kBurgers2D = 1, kGrayScott = 2, kKerr = 3 };

// Elements per thread of the stencil kernel's vector path (16-byte accesses).
template <class T>
constexpr int stencil_vec(int pid) {
  return pid == kKerr ? (int)(8 / sizeof(T)) : (int)(16 / sizeof(T));
}
// Elements per thread of the streaming Krylov kernels.
template <class T>
constexpr int krylov_vec() {
  return (int)(16 / sizeof(T));
}

constexpr int kStencilRY = 4;       // rows per thread (2D problems)
constexpr int kStencilThreads = 256;
constexpr int kKrylovThreads = 512;
constexpr int kStreamThreads = 256;

// Launch shape of the stencil kernel for an nx-by-ny grid.
inline void stencil_shape(int pid, int nx, int ny, int vec, dim3& grid, dim3& block) {
  const bool dim2 = pid != kBurgers1D;
  const int tcols = (nx + vec - 1) / vec;
  int tx = ((tcols + kWave - 1) / kWave) * kWave;
  if (tx > kStencilThreads) tx = kStencilThreads;
  const int ty = dim2 ? kStencilThreads / tx : 1;
  block = dim3(tx, ty, 1);
  grid = dim3((tcols + tx - 1) / tx, dim2 ? (ny + ty * kStencilRY - 1) / (ty * kStencilRY) : 1, 1);
}

// Launches the stencil kernel; *nblocks (nullable) receives its block count
// (the number of partial rows it writes when reducing).
template <class T, class VT>
hipError_t launch_stencil(int pid, int op, bool withf, bool vectorized, const StencilArgs<T, VT>& a,
                          const Coefs& c, hipStream_t s, int* nblocks = nullptr);

template <class T, class VT>
hipError_t launch_cgs(int mode, const KArgs<T, VT>& a, int grid, hipStream_t s);

template <class T, class VT>
hipError_t launch_init(const InitArgs<T, VT>& a, int grid, hipStream_t s);

template <class T, class VT>
hipError_t launch_vy(const VyArgs<T, VT>& a, int m, int grid, hipStream_t s);

template <class T>
hipError_t launch_trial(long long n, const double* x64, const T* dx, double alpha, double* x64t, T* xw, int grid,
                        hipStream_t s);

template <class T>
hipError_t launch_cast(long long n, const double* src, T* dst, int grid, hipStream_t s);

template <class T>
hipError_t launch_norm2(long long n, const T* p, double* part, int grid, hipStream_t s);

template <class T>
hipError_t launch_fill_zero(long long n, T* p, int grid, hipStream_t s);

hipError_t launch_ctl_begin(Ctl* c, double tol, double brk_tol, int m, hipStream_t s);
hipError_t launch_cycle_begin(Ctl* c, Partials in, int m, hipStream_t s);
hipError_t launch_finish_sums(Partials in, int nr, double* out0, double* out1, hipStream_t s);

}  // namespace jfnk
