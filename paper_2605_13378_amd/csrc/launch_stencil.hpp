// Launchers of the kernels that are instantiated per operator type P: the
// stencil kernel (residual, AD and FD JVPs, with its launch plan) and the
// single-workgroup solve.  Each (operator, precision) pair is its own
// translation unit (stencil_inst.hip, compiled once per pair) so that the
// build compiles them in parallel.
#pragma once

#include "launch.hpp"

namespace jfnk {

template <class P, class T, class VT, int VEC, int RY, int OP>
static hipError_t stencil_kdot(const StencilArgs<T, VT>& a, const Coefs& c, dim3 grid, dim3 block, hipStream_t s) {
  if constexpr (RY == 1) {
    // RY = 1 plans only uncapped launches, which carry no fused projection
    if (a.Vb != nullptr) return hipErrorInvalidValue;
    JFNK_LAUNCH((stencil_kernel<P, T, VT, VEC, RY, OP, false, 0>), grid, block, s, a, c);
  } else {
    if (a.Vb == nullptr) {
      if (a.ctl != nullptr) return hipErrorInvalidValue;  // Arnoldi mode always fuses the projection
      JFNK_LAUNCH((stencil_kernel<P, T, VT, VEC, RY, OP, false, 0>), grid, block, s, a, c);
    }
    else if (a.K <= 4)
      JFNK_LAUNCH((stencil_kernel<P, T, VT, VEC, RY, OP, false, 4>), grid, block, s, a, c);
    else if (a.K <= 8)
      JFNK_LAUNCH((stencil_kernel<P, T, VT, VEC, RY, OP, false, 8>), grid, block, s, a, c);
    else if (a.K <= 16)
      JFNK_LAUNCH((stencil_kernel<P, T, VT, VEC, RY, OP, false, 16>), grid, block, s, a, c);
    else
      JFNK_LAUNCH((stencil_kernel<P, T, VT, VEC, RY, OP, false, 32>), grid, block, s, a, c);
  }
  return hipGetLastError();
}

template <class P, class T, class VT, int VEC, int RY>
static hipError_t stencil_by_op(int op, bool withf, const StencilArgs<T, VT>& a, const Coefs& c, dim3 grid,
                                dim3 block, hipStream_t s) {
  if (op == OP_RES) {
    if constexpr (std::is_same<T, VT>::value) {
      JFNK_LAUNCH((stencil_kernel<P, T, VT, VEC, RY, OP_RES, false, 0>), grid, block, s, a, c);
      return hipGetLastError();
    } else {
      return hipErrorInvalidValue;
    }
  }
  if (op == OP_AD) {
    if (withf) {
      JFNK_LAUNCH((stencil_kernel<P, T, VT, VEC, RY, OP_AD, true, 0>), grid, block, s, a, c);
      return hipGetLastError();
    }
    return stencil_kdot<P, T, VT, VEC, RY, OP_AD>(a, c, grid, block, s);
  }
  return stencil_kdot<P, T, VT, VEC, RY, OP_FD>(a, c, grid, block, s);
}

template <class P, class T, class VT>
hipError_t launch_stencil_p(int pid, int op, bool withf, bool vectorized, const StencilArgs<T, VT>& a, const Coefs& c,
                            int cap, hipStream_t s, int* nblocks) {
  constexpr int V = (P::kInterleaved || P::kCorners) ? (int)(8 / sizeof(T)) : (int)(16 / sizeof(T));
  const int vec = vectorized ? V : 1;
  const StencilPlan p = stencil_plan(pid, a.nx, a.ny, vec, cap);
  if (nblocks) *nblocks = p.grid;
  const dim3 grid(p.grid, 1, 1);
  if (!vectorized) return stencil_by_op<P, T, VT, 1, 2>(op, withf, a, c, grid, p.block, s);
  if constexpr (P::kDim2) {
    if (p.ry == 4) return stencil_by_op<P, T, VT, V, 4>(op, withf, a, c, grid, p.block, s);
    if (p.ry == 1) return stencil_by_op<P, T, VT, V, 1>(op, withf, a, c, grid, p.block, s);
  }
  return stencil_by_op<P, T, VT, V, 2>(op, withf, a, c, grid, p.block, s);
}

template <class P, class T>
hipError_t launch_fused_p(const FusedArgs<T>& a, size_t lds, hipStream_t s) {
  const auto k = fused_solve_kernel<P, T>;
  hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void*>(k), hipFuncAttributeMaxDynamicSharedMemorySize,
                                     (int)lds);
  if (e != hipSuccess) return e;
  JFNK_LAUNCH_SHM(k, dim3(1), dim3(kFusedThreads), lds, s, a);
  return hipGetLastError();
}

}  // namespace jfnk
