// Host-side launchers for the JFNK kernels.  Declarations only; the
// definitions live in launch_impl.hpp and are instantiated once per
// precision (kernels_f64.hip, kernels_f32.hip, kernels_f16.hip) so the
// translation units compile in parallel.
#pragma once

#include <hip/hip_ext.h>
#include <hip/hip_runtime.h>

#include "common.hpp"
#include "krylov.hpp"
#include "problems.hpp"
#include "stencil.hpp"

namespace jfnk {

enum ProblemKind { kBurgers1D = 0, kBurgers2D = 1, kGrayScott = 2, kKerr = 3 };

// Kernel timing: when the host driver sets g_timing around one launch, the
// launch goes through hipExtLaunchKernelGGL with start/stop events attached
// to the dispatch itself, so the events measure the kernel's execution
// rather than launch-to-completion on the stream.
struct KernelTiming {
  hipEvent_t start = nullptr;
  hipEvent_t stop = nullptr;
};
extern thread_local KernelTiming* g_timing;

#define JFNK_LAUNCH(kernel, grid, block, stream, ...)                                                     \
  do {                                                                                                    \
    if (::jfnk::g_timing != nullptr)                                                                      \
      hipExtLaunchKernelGGL(kernel, grid, block, 0, stream, ::jfnk::g_timing->start, ::jfnk::g_timing->stop, \
                            0, __VA_ARGS__);                                                              \
    else                                                                                                  \
      hipLaunchKernelGGL(kernel, grid, block, 0, stream, __VA_ARGS__);                                    \
  } while (0)

// Elements per thread of the stencil kernel's vector path (16-byte accesses).
template <class T>
constexpr int stencil_vec(int pid) {
  return pid == kKerr ? (int)(8 / sizeof(T)) : (int)(16 / sizeof(T));
}
// Elements per thread of the streaming Krylov kernels (16-byte accesses; the
// FP64 passes over 17..32 basis vectors use 8-byte accesses so that the
// register-resident basis chunk fits without spilling).
template <class T>
constexpr int krylov_vec() {
  return (int)(16 / sizeof(T));
}
template <class T, int KMAX>
constexpr int cgs_vec() {
  return (sizeof(T) == 8 && KMAX > 16) ? 1 : (int)(16 / sizeof(T));
}

constexpr int kStencilRY = 4;       // rows per thread (2D problems)
constexpr int kStencilThreads = 256;
constexpr int kKrylovThreads = 512;
constexpr int kStreamThreads = 256;

// Block shape and tile count of the stencil kernel for an nx-by-ny grid:
// blocks of 256 threads, blockDim.x a multiple of 64 covering up to 256 * vec
// columns; a tile is blockDim.x * vec columns by blockDim.y * kStencilRY rows.
inline void stencil_shape(int pid, int nx, int ny, int vec, dim3& block, int& ntiles) {
  const bool dim2 = pid != kBurgers1D;
  const int tcols = (nx + vec - 1) / vec;
  int tx = ((tcols + kWave - 1) / kWave) * kWave;
  if (tx > kStencilThreads) tx = kStencilThreads;
  const int ty = dim2 ? kStencilThreads / tx : 1;
  block = dim3(tx, ty, 1);
  const int tiles_x = (tcols + tx - 1) / tx;
  const int tiles_y = dim2 ? (ny + ty * kStencilRY - 1) / (ty * kStencilRY) : 1;
  ntiles = tiles_x * tiles_y;
}

// Blocks of a persistent stencil launch with at most `cap` blocks.
inline int stencil_blocks(int pid, int nx, int ny, int vec, int cap) {
  dim3 b;
  int nt = 0;
  stencil_shape(pid, nx, ny, vec, b, nt);
  return nt < cap ? nt : cap;
}

// Launches the stencil kernel on at most `cap` blocks; *nblocks (nullable)
// receives the block count (the number of partial rows it writes).  In
// Arnoldi mode with a.Vb set, the first CGS projection on a.K basis vectors
// is fused in.
template <class T, class VT>
hipError_t launch_stencil(int pid, int op, bool withf, bool vectorized, const StencilArgs<T, VT>& a,
                          const Coefs& c, int cap, hipStream_t s, int* nblocks = nullptr);

template <class T, class VT>
hipError_t launch_cgs(int mode, const KArgs<T, VT>& a, int grid, hipStream_t s);

template <class T, class VT>
hipError_t launch_init(const InitArgs<T, VT>& a, int grid, hipStream_t s);

template <class T, class VT>
hipError_t launch_vy(const VyArgs<T, VT>& a, int m, int grid, hipStream_t s);

template <class T, class VT>
hipError_t launch_store_basis0(long long n, const T* r, VT* V0, const Ctl* c, int grid, hipStream_t s);

template <class T>
hipError_t launch_trial(long long n, const double* x64, const T* dx, double alpha, double* x64t, T* xw, int grid,
                        hipStream_t s);

template <class T>
hipError_t launch_cast(long long n, const double* src, T* dst, int grid, hipStream_t s);

template <class T>
hipError_t launch_norm2(long long n, const T* p, PartSink part, int grid, hipStream_t s);

template <class T>
hipError_t launch_fill_zero(long long n, T* p, int grid, hipStream_t s);

hipError_t launch_ctl_begin(Ctl* c, double tol, double brk_tol, int m, hipStream_t s);
hipError_t launch_cycle_begin(Ctl* c, Partials in, int m, long long n, int fp16, hipStream_t s);
hipError_t launch_finish_sums(Partials in, int nr, double* out0, double* out1, hipStream_t s);

}  // namespace jfnk
