// Host-side launchers for the JFNK kernels.  Declarations only; the
// definitions live in launch_impl.hpp and are instantiated once per
// precision (kernels_f64.hip, kernels_f32.hip, kernels_f16.hip) so the
// translation units compile in parallel.
#pragma once

#include <hip/hip_ext.h>
#include <hip/hip_runtime.h>

#include "bicgstab.hpp"
#include "cg.hpp"
#include "common.hpp"
#include "fused.hpp"
#include "krylov.hpp"
#include "problems.hpp"
#include "stencil.hpp"

namespace jfnk {

// Problem kinds: the public ids, plus kSuOlsonPY for the Su-Olson problem in
// its periodic-row configuration (public id 5 with p[1] = 1).
enum ProblemKind {
  kBurgers1D = 0, kBurgers2D = 1, kGrayScott = 2, kKerr = 3, kRD2D = 4, kSuOlson = 5, kMaxwell = 6, kSuOlsonPY = 7
};

// Kernel timing: when the host driver sets g_timing around one launch, the
// launch goes through hipExtLaunchKernelGGL with start/stop events attached
// to the dispatch itself, so the events measure the kernel's execution
// rather than launch-to-completion on the stream.
struct KernelTiming {
  hipEvent_t start = nullptr;
  hipEvent_t stop = nullptr;
};
extern thread_local KernelTiming* g_timing;

#define JFNK_LAUNCH_SHM(kernel, grid, block, shm, stream, ...)                                            \
  do {                                                                                                    \
    if (::jfnk::g_timing != nullptr)                                                                      \
      hipExtLaunchKernelGGL(kernel, grid, block, shm, stream, ::jfnk::g_timing->start,                    \
                            ::jfnk::g_timing->stop, 0, __VA_ARGS__);                                      \
    else                                                                                                  \
      hipLaunchKernelGGL(kernel, grid, block, shm, stream, __VA_ARGS__);                                  \
  } while (0)

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
  // 8-byte accesses for the interleaved Kerr pairs and the four-plane Maxwell
  // field (whose corner halos would not fit the registers at 16 bytes)
  return (pid == kKerr || pid == kMaxwell) ? (int)(8 / sizeof(T)) : (int)(16 / sizeof(T));
}
// Elements per thread of the streaming Krylov kernels (16-byte accesses; the
// FP64 passes over 17..32 basis vectors use 8-byte accesses so that the
// register-resident basis chunk fits without spilling).
template <class T>
constexpr int krylov_vec() {
  return (int)(16 / sizeof(T));
}
// Elements per thread of the Krylov passes: 16-byte loads of the basis (FP16
// storage: eight elements), one FP64 element when 32 vectors would not fit
// the registers at two.
template <class T, class VT, int KMAX>
constexpr int cgs_vec() {
  return sizeof(VT) == 2 ? 8 : ((sizeof(T) == 8 && KMAX > 16) ? 1 : (int)(16 / sizeof(T)));
}

constexpr int kStencilThreads = 256;
constexpr int kKrylovThreads = 512;
constexpr int kStreamThreads = 256;

// Launch plan of the stencil kernel for an nx-by-ny grid.  2D problems use
// blocks of one wavefront across (64 lanes x VEC columns) by 4 wavefronts
// down, each thread owning RY consecutive rows; a tile is 64 * VEC columns
// by 4 * RY rows.  1D problems use one row of up to 256 lanes.  RY is 2
// unless that gives more tiles than the block cap, then 4 (the vector path
// only); the grid is min(tiles, cap) and each block walks a contiguous range
// of tiles.  Measured on MI355X: one-wavefront-wide blocks with one tile
// each stream 1.3-1.4x faster than 256-lane-wide row blocks, and a kernel
// that writes per-block partial sums keeps its grid at or below 512-1024
// blocks so that the consumer's prologue reduction stays within one memory
// round trip.
struct StencilPlan {
  dim3 block;
  int ry = 2;
  int ntiles = 0;
  int grid = 0;
};

inline int stencil_tiles(int pid, int nx, int ny, int vec, int ry, dim3& block) {
  const int tcols = (nx + vec - 1) / vec;
  if (pid == kBurgers1D) {
    int tx = ((tcols + kWave - 1) / kWave) * kWave;
    if (tx > kStencilThreads) tx = kStencilThreads;
    block = dim3(tx, 1, 1);
    return (tcols + tx - 1) / tx;
  }
  block = dim3(kWave, kStencilThreads / kWave, 1);
  const int tiles_x = (tcols + kWave - 1) / kWave;
  const int band = (int)block.y * ry;
  return tiles_x * ((ny + band - 1) / band);
}

constexpr int kStencilUncapped = 1 << 29;  // caps at or above this: one tile per block
constexpr int kStencilRY1Tiles = 1 << 30;  // RY = 1 for uncapped 2D launches with this many tiles (off)

inline StencilPlan stencil_plan(int pid, int nx, int ny, int vec, int cap) {
  StencilPlan p;
  p.ry = 2;
  p.ntiles = stencil_tiles(pid, nx, ny, vec, 2, p.block);
  if (pid != kBurgers1D && vec > 1 && p.ntiles > cap) {
    p.ry = 4;
    p.ntiles = stencil_tiles(pid, nx, ny, vec, 4, p.block);
  } else if (pid != kBurgers1D && vec > 1 && cap >= kStencilUncapped) {
    // large grids without partial sums could take one row per thread; kept
    // off: a batch-averaged probe favoured it at 2048^2 (19.0 vs 19.9 us), the
    // per-dispatch timing of the benchmark did not (19.0 vs 18.5 us)
    dim3 b1;
    const int t1 = stencil_tiles(pid, nx, ny, vec, 1, b1);
    if (t1 >= kStencilRY1Tiles) {
      p.ry = 1;
      p.ntiles = t1;
      p.block = b1;
    }
  }
  p.grid = p.ntiles < cap ? p.ntiles : cap;
  if (p.grid < 1) p.grid = 1;
  return p;
}

// Blocks of a stencil launch with at most `cap` blocks.
inline int stencil_blocks(int pid, int nx, int ny, int vec, int cap) { return stencil_plan(pid, nx, ny, vec, cap).grid; }

// Per-operator launchers (launch_stencil.hpp), each (operator, precision)
// pair instantiated in its own translation unit.
template <class P, class T, class VT>
hipError_t launch_stencil_p(int pid, int op, bool withf, bool vectorized, const StencilArgs<T, VT>& a, const Coefs& c,
                            int cap, hipStream_t s, int* nblocks);
template <class P, class T>
hipError_t launch_fused_p(const FusedArgs<T>& a, size_t lds, hipStream_t s);

// Launches the stencil kernel on at most `cap` blocks; *nblocks (nullable)
// receives the block count (the number of partial rows it writes).  In
// Arnoldi mode with a.Vb set, the first CGS projection on a.K basis vectors
// is fused in.
template <class T, class VT>
hipError_t launch_stencil(int pid, int op, bool withf, bool vectorized, const StencilArgs<T, VT>& a,
                          const Coefs& c, int cap, hipStream_t s, int* nblocks = nullptr);

// z = M^{-1} z in place for the problem's diagonal preconditioner, frozen at
// x (problems that define one only; others return hipErrorInvalidValue).
template <class T>
hipError_t launch_cslp_apply(int pid, const T* x, T* z, int nx, int ny, const Coefs& c, int grid, hipStream_t s);
template <class T, class VT>
hipError_t launch_cgs(int mode, const KArgs<T, VT>& a, int grid, hipStream_t s);

// Update pass of the delayed-second-pass Arnoldi step (K = j + 1).
template <class T, class VT>
hipError_t launch_dcgs(const KArgs<T, VT>& a, int grid, hipStream_t s);

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

// Whole Newton-GMRES solve in one workgroup with `lds` bytes of LDS
// (fused_lds_bytes<T>(n, m)); problem kinds as in launch_stencil.
template <class T>
hipError_t launch_fused_solve(int pid, const FusedArgs<T>& a, size_t lds, hipStream_t s);

// BiCGSTAB streaming kernels (bicgstab.hpp) on `grid` blocks of
// kStreamThreads; `tol` is read by the p kernel only.
enum { BI_INIT = 0, BI_P = 1, BI_S = 2, BI_XR = 3 };
template <class T>
hipError_t launch_bi(int kind, const BiArgs<T>& a, double tol, int grid, hipStream_t s);

// CG streaming kernels (cg.hpp) on `grid` blocks of kStreamThreads.
enum { CG_INIT = 0, CG_P = 1, CG_XR = 2 };
template <class T>
hipError_t launch_cg(int kind, const CgArgs<T>& a, double tol, int grid, hipStream_t s);

hipError_t launch_ctl_begin(Ctl* c, double tol, double brk_tol, int m, hipStream_t s);
// out = half(v sigma), sigma = fp16_scale(sqrt(*vn2)), *inv_sigma = 1 / sigma.
hipError_t launch_fp16_tangent(long long n, const float* v, __half* out, const double* vn2, double* inv_sigma,
                               int grid, hipStream_t s);
hipError_t launch_cycle_begin(Ctl* c, Partials in, int m, long long n, int fp16, hipStream_t s);
hipError_t launch_finish_sums(Partials in, int nr, double* out0, double* out1, hipStream_t s);
// Copies the first `words` 32-bit words of the control block to mapped host
// memory `dst`, then writes `seq` to the mapped word `seq_dst`.
hipError_t launch_publish_ctl(const Ctl* c, int* dst, int words, int* seq_dst, int seq, hipStream_t s);

}  // namespace jfnk
