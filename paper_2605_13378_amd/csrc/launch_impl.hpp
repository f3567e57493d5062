// Definitions of the launchers declared in launch.hpp (included by the
// per-precision translation units only).
#pragma once

#include "launch.hpp"

namespace jfnk {

template <class T, class VT>
hipError_t launch_stencil(int pid, int op, bool withf, bool vectorized, const StencilArgs<T, VT>& a,
                          const Coefs& c, int cap, hipStream_t s, int* nblocks) {
  switch (pid) {
    case kBurgers1D:
      return launch_stencil_p<Burgers1DOp, T, VT>(pid, op, withf, vectorized, a, c, cap, s, nblocks);
    case kBurgers2D:
      return launch_stencil_p<Burgers2DOp, T, VT>(pid, op, withf, vectorized, a, c, cap, s, nblocks);
    case kGrayScott:
      return launch_stencil_p<GrayScottOp, T, VT>(pid, op, withf, vectorized, a, c, cap, s, nblocks);
    case kKerr:
      if (a.precond && op != OP_RES)
        return launch_stencil_p<KerrCslpOp, T, VT>(pid, op, withf, vectorized, a, c, cap, s, nblocks);
      return launch_stencil_p<KerrOp, T, VT>(pid, op, withf, vectorized, a, c, cap, s, nblocks);
    case kRD2D:
      return launch_stencil_p<RD2DOp, T, VT>(pid, op, withf, vectorized, a, c, cap, s, nblocks);
    case kSuOlson:
      return launch_stencil_p<SuOlsonOp, T, VT>(pid, op, withf, vectorized, a, c, cap, s, nblocks);
    case kSuOlsonPY:
      return launch_stencil_p<SuOlsonPYOp, T, VT>(pid, op, withf, vectorized, a, c, cap, s, nblocks);
    case kMaxwell:
      if (a.precond && op != OP_RES)
        return launch_stencil_p<MaxwellTECslpOp, T, VT>(pid, op, withf, vectorized, a, c, cap, s, nblocks);
      return launch_stencil_p<MaxwellTEOp, T, VT>(pid, op, withf, vectorized, a, c, cap, s, nblocks);
    default:
      return hipErrorInvalidValue;
  }
}

template <class T>
hipError_t launch_cslp_apply(int pid, const T* x, T* z, int nx, int ny, const Coefs& c, int grid, hipStream_t s) {
  if (pid == kMaxwell)
    JFNK_LAUNCH((cslp_apply_kernel<MaxwellTEOp, T>), dim3(grid), dim3(kStreamThreads), s, x, z, nx, ny,
                (long long)nx * ny, c);
  else if (pid == kKerr)
    JFNK_LAUNCH((cslp_apply_kernel<KerrOp, T>), dim3(grid), dim3(kStreamThreads), s, x, z, nx, ny,
                (long long)nx * ny, c);
  else
    return hipErrorInvalidValue;
  return hipGetLastError();
}

template <class T, class VT, int KMAX, bool NT>
static hipError_t cgs_by_mode(int mode, const KArgs<T, VT>& a, int grid, hipStream_t s) {
  constexpr int VEC = cgs_vec<T, VT, KMAX>();
  const dim3 g(grid), b(kKrylovThreads);
  if (mode == PASS_A)
    JFNK_LAUNCH((cgs_kernel<T, VT, KMAX, VEC, PASS_A, NT>), g, b, s, a);
  else if (mode == PASS_B)
    JFNK_LAUNCH((cgs_kernel<T, VT, KMAX, VEC, PASS_B, NT>), g, b, s, a);
  else
    JFNK_LAUNCH((cgs_kernel<T, VT, KMAX, VEC, PASS_C, NT>), g, b, s, a);
  return hipGetLastError();
}

template <class T, class VT, bool NT>
static hipError_t launch_cgs_nt(int mode, const KArgs<T, VT>& a, int grid, hipStream_t s) {
  if (a.K <= 4) return cgs_by_mode<T, VT, 4, NT>(mode, a, grid, s);
  if (a.K <= 8) return cgs_by_mode<T, VT, 8, NT>(mode, a, grid, s);
  if (a.K <= 16) return cgs_by_mode<T, VT, 16, NT>(mode, a, grid, s);
  return cgs_by_mode<T, VT, 32, NT>(mode, a, grid, s);
}

template <class T, class VT>
hipError_t launch_cgs(int mode, const KArgs<T, VT>& a, int grid, hipStream_t s) {
  return a.nt ? launch_cgs_nt<T, VT, true>(mode, a, grid, s) : launch_cgs_nt<T, VT, false>(mode, a, grid, s);
}

template <class T, class VT, bool NT>
static hipError_t launch_dcgs_nt(const KArgs<T, VT>& a, int grid, hipStream_t s) {
  const dim3 b(kKrylovThreads);
  if (a.K <= 4)
    JFNK_LAUNCH((dcgs_kernel<T, VT, 4, cgs_vec<T, VT, 4>(), NT>), dim3(grid), b, s, a);
  else if (a.K <= 8)
    JFNK_LAUNCH((dcgs_kernel<T, VT, 8, cgs_vec<T, VT, 8>(), NT>), dim3(grid), b, s, a);
  else if (a.K <= 16)
    JFNK_LAUNCH((dcgs_kernel<T, VT, 16, cgs_vec<T, VT, 16>(), NT>), dim3(grid), b, s, a);
  else
    JFNK_LAUNCH((dcgs_kernel<T, VT, 32, cgs_vec<T, VT, 32>(), NT>), dim3(grid), b, s, a);
  return hipGetLastError();
}

template <class T, class VT>
hipError_t launch_dcgs(const KArgs<T, VT>& a, int grid, hipStream_t s) {
  return a.nt ? launch_dcgs_nt<T, VT, true>(a, grid, s) : launch_dcgs_nt<T, VT, false>(a, grid, s);
}

template <class T, class VT>
hipError_t launch_init(const InitArgs<T, VT>& a, int grid, hipStream_t s) {
  constexpr int VEC = krylov_vec<T>();
  JFNK_LAUNCH((init_cycle_kernel<T, VT, VEC>), dim3(grid), dim3(kStreamThreads), s, a);
  return hipGetLastError();
}

template <class T, class VT, bool NT>
static hipError_t launch_vy_nt(const VyArgs<T, VT>& a, int m, int grid, hipStream_t s) {
  constexpr int VEC = sizeof(VT) == 2 ? 8 : krylov_vec<T>();  // 16-byte basis loads
  const dim3 g(grid), b(kKrylovThreads);
  if (m <= 8)
    JFNK_LAUNCH((vy_kernel<T, VT, 8, VEC, NT>), g, b, s, a);
  else if (m <= 16)
    JFNK_LAUNCH((vy_kernel<T, VT, 16, VEC, NT>), g, b, s, a);
  else
    JFNK_LAUNCH((vy_kernel<T, VT, 32, VEC, NT>), g, b, s, a);
  return hipGetLastError();
}

template <class T, class VT>
hipError_t launch_vy(const VyArgs<T, VT>& a, int m, int grid, hipStream_t s) {
  return a.nt ? launch_vy_nt<T, VT, true>(a, m, grid, s) : launch_vy_nt<T, VT, false>(a, m, grid, s);
}

template <class T, class VT>
hipError_t launch_store_basis0(long long n, const T* r, VT* V0, const Ctl* c, int grid, hipStream_t s) {
  constexpr int VEC = krylov_vec<T>();
  JFNK_LAUNCH((store_basis0_kernel<T, VT, VEC>), dim3(grid), dim3(kStreamThreads), s, n, r, V0, c);
  return hipGetLastError();
}

template <class T>
hipError_t launch_trial(long long n, const double* x64, const T* dx, double alpha, double* x64t, T* xw, int grid,
                        hipStream_t s) {
  JFNK_LAUNCH((newton_trial_kernel<T, 2>), dim3(grid), dim3(kStreamThreads), s, n, x64, dx, alpha, x64t,
                     xw);
  return hipGetLastError();
}

template <class T>
hipError_t launch_cast(long long n, const double* src, T* dst, int grid, hipStream_t s) {
  JFNK_LAUNCH((cast_kernel<T, 2>), dim3(grid), dim3(kStreamThreads), s, n, src, dst);
  return hipGetLastError();
}

template <class T>
hipError_t launch_norm2(long long n, const T* p, PartSink part, int grid, hipStream_t s) {
  JFNK_LAUNCH((norm2_kernel<T>), dim3(grid), dim3(kStreamThreads), s, n, p, part);
  return hipGetLastError();
}

template <class T>
hipError_t launch_fill_zero(long long n, T* p, int grid, hipStream_t s) {
  JFNK_LAUNCH((fill_zero_kernel<T>), dim3(grid), dim3(kStreamThreads), s, n, p);
  return hipGetLastError();
}

template <class T>
hipError_t launch_bi(int kind, const BiArgs<T>& a, double tol, int grid, hipStream_t s) {
  constexpr int VEC = krylov_vec<T>();
  const dim3 g(grid), b(kStreamThreads);
  switch (kind) {
    case BI_INIT:
      JFNK_LAUNCH((bi_init_kernel<T, VEC>), g, b, s, a);
      break;
    case BI_P:
      JFNK_LAUNCH((bi_p_kernel<T, VEC>), g, b, s, a, tol);
      break;
    case BI_S:
      JFNK_LAUNCH((bi_s_kernel<T, VEC>), g, b, s, a);
      break;
    case BI_XR:
      JFNK_LAUNCH((bi_xr_kernel<T, VEC>), g, b, s, a);
      break;
    default:
      return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

template <class T>
hipError_t launch_cg(int kind, const CgArgs<T>& a, double tol, int grid, hipStream_t s) {
  constexpr int VEC = krylov_vec<T>();
  const dim3 g(grid), b(kStreamThreads);
  switch (kind) {
    case CG_INIT:
      JFNK_LAUNCH((cg_init_kernel<T, VEC>), g, b, s, a);
      break;
    case CG_P:
      JFNK_LAUNCH((cg_p_kernel<T, VEC>), g, b, s, a, tol);
      break;
    case CG_XR:
      JFNK_LAUNCH((cg_xr_kernel<T, VEC>), g, b, s, a);
      break;
    default:
      return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

template <class T>
hipError_t launch_fused_solve(int pid, const FusedArgs<T>& a, size_t lds, hipStream_t s) {
  switch (pid) {
    case kBurgers1D:
      return launch_fused_p<Burgers1DOp, T>(a, lds, s);
    case kBurgers2D:
      return launch_fused_p<Burgers2DOp, T>(a, lds, s);
    case kGrayScott:
      return launch_fused_p<GrayScottOp, T>(a, lds, s);
    case kKerr:
      return launch_fused_p<KerrOp, T>(a, lds, s);
    case kRD2D:
      return launch_fused_p<RD2DOp, T>(a, lds, s);
    case kSuOlson:
      return launch_fused_p<SuOlsonOp, T>(a, lds, s);
    case kSuOlsonPY:
      return launch_fused_p<SuOlsonPYOp, T>(a, lds, s);
    case kMaxwell:
      return launch_fused_p<MaxwellTEOp, T>(a, lds, s);
    default:
      return hipErrorInvalidValue;
  }
}

#define JFNK_INSTANTIATE(T, VT)                                                                                  \
  template hipError_t launch_stencil<T, VT>(int, int, bool, bool, const StencilArgs<T, VT>&, const Coefs&, int, \
                                            hipStream_t, int*);                                                 \
  template hipError_t launch_cgs<T, VT>(int, const KArgs<T, VT>&, int, hipStream_t);                            \
  template hipError_t launch_init<T, VT>(const InitArgs<T, VT>&, int, hipStream_t);                             \
  template hipError_t launch_dcgs<T, VT>(const KArgs<T, VT>&, int, hipStream_t);                                \
  template hipError_t launch_vy<T, VT>(const VyArgs<T, VT>&, int, int, hipStream_t);                            \
  template hipError_t launch_store_basis0<T, VT>(long long, const T*, VT*, const Ctl*, int, hipStream_t);

#define JFNK_INSTANTIATE_SCALAR(T)                                                                               \
  template hipError_t launch_trial<T>(long long, const double*, const T*, double, double*, T*, int, hipStream_t);\
  template hipError_t launch_cast<T>(long long, const double*, T*, int, hipStream_t);                           \
  template hipError_t launch_norm2<T>(long long, const T*, PartSink, int, hipStream_t);                         \
  template hipError_t launch_fill_zero<T>(long long, T*, int, hipStream_t);                                     \
  template hipError_t launch_cslp_apply<T>(int, const T*, T*, int, int, const Coefs&, int, hipStream_t);        \
  template hipError_t launch_fused_solve<T>(int, const FusedArgs<T>&, size_t, hipStream_t);                 \
  template hipError_t launch_bi<T>(int, const BiArgs<T>&, double, int, hipStream_t);                        \
  template hipError_t launch_cg<T>(int, const CgArgs<T>&, double, int, hipStream_t);

}  // namespace jfnk
