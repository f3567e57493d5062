// Whole Newton-GMRES solve of a small problem in one workgroup.
//
// For problems whose vectors all fit in the 160 KB of LDS of one compute unit
// (about 490 unknowns in FP64, 950 in FP32 with GMRES(30)), launch latency
// and host round trips dominate the multi-kernel path: every Arnoldi step
// there costs three kernel launches, and every restart cycle and residual a
// host synchronization.  This kernel runs the same algorithm (paper,
// Section 2: Newton with backtracking line search around restarted GMRES(m)
// with classical Gram-Schmidt applied twice and Givens rotations in FP64)
// from one launch: the state, the Krylov basis and the Hessenberg matrix
// live in LDS, every phase is a block-wide loop separated by barriers, and
// the scalar decisions (Givens rotations, convergence and line-search tests)
// are taken by one thread and published through LDS.  Global memory is
// touched only to read the constant part b and the start iterate, and to
// write the result, the optional iterate history and the info record.
//
// The control flow is uniform across the block: every loop bound and every
// branch depends only on values all threads read from LDS after a barrier.
// Every loop is bounded by the iteration caps, so the kernel always ends.
#pragma once

#include "common.hpp"
#include "problems.hpp"
#include "stencil.hpp"

namespace jfnk {

// eight wavefronts: the dot products over the basis split each vector over
// twice the lanes of four (measured 2% lower solve latency at 1D Burgers
// N = 256 FP64; sixteen wavefronts were 25% slower)
constexpr int kFusedThreads = 512;
constexpr int kFusedMaxIters = 64;

struct FusedOpts {
  int m, max_restarts, max_newton, ls_max;
  double tol_k, tol_n, ls_c, fd_eps, brk, root_eps;
  int mode;      // 0 AD, 1 FD
  int eps_rule;  // 0 sqrt(eps_m) max(1, ||x||), 1 sqrt(eps_m) (1 + ||x||) / ||v||
};

// Result record (the fields of the ABI's info struct that a Newton solve fills).
struct FusedInfo {
  int status;  // 0 converged, 4 non-finite, 6 iteration cap
  int converged, newton_iters, krylov_iters, restarts, ls_backtracks, ls_failures;
  int lin_iters[kFusedMaxIters];
  double rel_res[kFusedMaxIters + 1];
  double alpha[kFusedMaxIters];
  double f0_norm;
};

template <class T>
struct FusedArgs {
  int nx, ny;
  int cells;  // nx * ny
  int n;      // unknowns
  double alpha, cN, beta;
  Coefs coefs;
  const T* b;        // constant part (nullable: zero)
  double* x;         // FP64 iterate, in and out
  double* history;   // nullable: iterate k at history + k * n
  FusedOpts o;
  FusedInfo* info;
};

// Row stride of the basis in LDS: a multiple of 32 elements plus 8, so that
// lane groups of a wavefront reading consecutive elements of different
// vectors start on different banks (8 banks apart for 4-byte elements, 16
// for 8-byte ones).
__host__ __device__ constexpr int fused_ldv(long long n) { return (int)((n + 31) / 32 * 32 + 8); }

// LDS bytes of the kernel for n unknowns and restart length m: FP64 master
// and trial iterates, the Hessenberg/rotation arrays and scalars in FP64; the
// working copies, F, trial F, w, dx, b and the m + 1 basis vectors in T.
template <class T>
constexpr size_t fused_lds_bytes(long long n, int m) {
  const size_t dbl = (size_t)2 * n + (size_t)(m + 1) * m + 4 * (size_t)m + 1 + 64 + kMaxCols;
  const size_t wt = (sizeof(T) == 8 ? 5 : 7) * (size_t)n + (size_t)(m + 1) * fused_ldv(n);
  return dbl * 8 + wt * sizeof(T);
}

namespace fused {

enum { S_SUM0 = 0, S_SUM1 = 1, S_EST = 2, S_FLAG = 3, S_RED = 8 };  // scalar slots (S_RED.. per-wave partials)

// Block-wide FP64 sums of a and b; every thread returns the same totals.
__device__ __forceinline__ void block_sum2(double a, double b, double* sc, double& ta, double& tb) {
  const int lane = threadIdx.x & (kWave - 1);
  const int wid = threadIdx.x / kWave;
  constexpr int nw = kFusedThreads / kWave;
  a = wave_sum(a);
  b = wave_sum(b);
  __syncthreads();
  if (lane == 0) {
    sc[S_RED + wid] = a;
    sc[S_RED + nw + wid] = b;
  }
  __syncthreads();
  ta = 0.0;
  tb = 0.0;
#pragma unroll
  for (int w = 0; w < nw; ++w) {
    ta += sc[S_RED + w];
    tb += sc[S_RED + nw + w];
  }
}

// out[i] = V_i . w for i < K (FP64 accumulation): G lanes of one wavefront
// per vector (G a power of two, G * K <= threads), each with four partial
// sums, then a reduction inside each lane group (group_sum).  Vector i starts at V + i * ldv; the padded stride puts
// the lane groups of one wavefront on different LDS banks.  Barriers on
// entry (earlier readers of `out`) and exit.
template <class T>
__device__ __forceinline__ void block_dots(const T* V, int n, int ldv, int K, const T* w, double* out) {
  int G = kWave;
  while (G > 1 && G * K > kFusedThreads) G >>= 1;
  const int i = threadIdx.x / G;
  const int g = threadIdx.x % G;
  double s = 0.0;
  if (i < K) {
    // four partial sums: a dependency chain a quarter as long
    const T* v = V + (size_t)i * ldv;
    double s1 = 0.0, s2 = 0.0, s3 = 0.0;
    int e = g;
    for (; e + 3 * G < n; e += 4 * G) {
      s += (double)v[e] * (double)w[e];
      s1 += (double)v[e + G] * (double)w[e + G];
      s2 += (double)v[e + 2 * G] * (double)w[e + 2 * G];
      s3 += (double)v[e + 3 * G] * (double)w[e + 3 * G];
    }
    for (; e < n; e += G) s += (double)v[e] * (double)w[e];
    s = (s + s1) + (s2 + s3);
  }
  s = group_sum_rt(s, G);
  __syncthreads();
  if (i < K && g == 0) out[i] = s;
  __syncthreads();
}

// w_e - sum_i h_i V_i[e] over i < K, as two interleaved chains of
// products (half the dependency length), subtracted at the end.
template <class T>
__device__ __forceinline__ T cgs_update(T we, const double* hv, const T* V, int ldv, int K, int e) {
  T a = we, b = T(0);
  int i = 0;
  for (; i + 1 < K; i += 2) {
    a = a - T(hv[i]) * V[(size_t)i * ldv + e];
    b = b + T(hv[i + 1]) * V[(size_t)(i + 1) * ldv + e];
  }
  if (i < K) a = a - T(hv[i]) * V[(size_t)i * ldv + e];
  return a - b;
}

// One Hillis-Steele step of the Givens scan inside rows of 16 lanes: lane l
// composes its map with that of lane l - D (DPP row shift, no LDS round
// trip) when take is set, the composition order being the scan's.
template <int D>
__device__ __forceinline__ void affine_scan_step(double& A, double& B, bool take) {
  const double Ap = dpp_f64<0x110 + D>(A), Bp = dpp_f64<0x110 + D>(B);  // row_shr:D
  if (take) {
    B = A * Bp + B;
    A = A * Ap;
  }
}

template <class P, class T>
__device__ __forceinline__ int at(int f, int c, int cells) {
  return P::kInterleaved ? 2 * c + f : f * cells + c;
}

template <class P, class T>
__device__ __forceinline__ void gather(const T* a, int c, int nx, int ny, int cells, Nbr<T> (&o)[P::NF]) {
  const int i = P::kDim2 ? c % nx : c;
  const int j = P::kDim2 ? c / nx : 0;
  const int il = wrap_idx<P::kPeriodic>(i - 1, nx);
  const int ir = wrap_idx<P::kPeriodic>(i + 1, nx);
  const int cl = j * nx + il, cr = j * nx + ir;
  int cd = c, cu = c;
  if constexpr (P::kDim2) {
    cd = wrap_idx<periodic_rows<P>::value>(j - 1, ny) * nx + i;
    cu = wrap_idx<periodic_rows<P>::value>(j + 1, ny) * nx + i;
  }
#pragma unroll
  for (int f = 0; f < P::NF; ++f) {
    o[f].c = a[at<P, T>(f, c, cells)];
    o[f].l = a[at<P, T>(f, cl, cells)];
    o[f].r = a[at<P, T>(f, cr, cells)];
    o[f].d = a[at<P, T>(f, cd, cells)];
    o[f].u = a[at<P, T>(f, cu, cells)];
  }
  if constexpr (P::kCorners) {
    const int jd = cd / nx, ju = cu / nx;
#pragma unroll
    for (int f = 0; f < P::NF; ++f) {
      o[f].dl = a[at<P, T>(f, jd * nx + il, cells)];
      o[f].dr = a[at<P, T>(f, jd * nx + ir, cells)];
      o[f].ul = a[at<P, T>(f, ju * nx + il, cells)];
      o[f].ur = a[at<P, T>(f, ju * nx + ir, cells)];
    }
  }
}

// out = F(x) (OP_RES), J(x) v (OP_AD) or (F(x + eps v) - F(x)) / eps (OP_FD),
// with the same pointwise expressions as the streaming stencil kernel.
// Returns sum(out^2) and sum(x^2) (FP64) to every thread.
template <class P, class T, int OP>
__device__ void eval(const typename P::template K<T>& k, const FusedArgs<T>& a, const T* x, const T* v, const T* bl,
                     T* out, T eps_s, T eps_t, double* sc, double& on2, double& xn2) {
  const T alpha = T(a.alpha), cN = T(a.cN), beta = T(a.beta);
  double so = 0.0, sx = 0.0;
  for (int c = threadIdx.x; c < a.cells; c += kFusedThreads) {
    Nbr<T> xn[P::NF];
    gather<P, T>(x, c, a.nx, a.ny, a.cells, xn);
    const int i = P::kDim2 ? c % a.nx : c;
    const int j = P::kDim2 ? c / a.nx : 0;
    const bool bnd = P::boundary(i, j, a.nx, a.ny);
    T o[P::NF];
    if constexpr (OP == OP_RES) {
      T nv[P::NF];
      P::template N<T, T>(k, xn, nv);
#pragma unroll
      for (int f = 0; f < P::NF; ++f) {
        const T bv = bl ? bl[at<P, T>(f, c, a.cells)] : T(0);
        o[f] = bnd ? xn[f].c : (alpha * xn[f].c + cN * nv[f]) + beta * bv;
      }
    } else if constexpr (OP == OP_AD) {
      Nbr<T> vn[P::NF];
      gather<P, T>(v, c, a.nx, a.ny, a.cells, vn);
      Nbr<dual<T>> dn[P::NF];
#pragma unroll
      for (int f = 0; f < P::NF; ++f) nbr_dual<P, T>(xn[f], vn[f], dn[f]);
      dual<T> nv[P::NF];
      P::template N<T, dual<T>>(k, dn, nv);
#pragma unroll
      for (int f = 0; f < P::NF; ++f) o[f] = bnd ? vn[f].c : alpha * vn[f].c + cN * nv[f].t;
    } else {
      Nbr<T> vn[P::NF];
      gather<P, T>(v, c, a.nx, a.ny, a.cells, vn);
      Nbr<T> yn[P::NF];
#pragma unroll
      for (int f = 0; f < P::NF; ++f) nbr_axpy<P, T>(xn[f], eps_s, vn[f], yn[f]);
      T n0[P::NF], n1[P::NF];
      P::template N<T, T>(k, xn, n0);
      P::template N<T, T>(k, yn, n1);
#pragma unroll
      for (int f = 0; f < P::NF; ++f) {
        const T bv = bl ? bl[at<P, T>(f, c, a.cells)] : T(0);
        const T f0 = bnd ? xn[f].c : (alpha * xn[f].c + cN * n0[f]) + beta * bv;
        const T f1 = bnd ? yn[f].c : (alpha * yn[f].c + cN * n1[f]) + beta * bv;
        o[f] = (f1 - f0) / eps_t;
      }
    }
#pragma unroll
    for (int f = 0; f < P::NF; ++f) {
      out[at<P, T>(f, c, a.cells)] = o[f];
      so += (double)o[f] * (double)o[f];
      sx += (double)xn[f].c * (double)xn[f].c;
    }
  }
  block_sum2(so, sx, sc, on2, xn2);
}

}  // namespace fused

template <class P, class T>
__global__ void __launch_bounds__(kFusedThreads) fused_solve_kernel(const FusedArgs<T> a) {
  using namespace fused;
  extern __shared__ double smem[];
  const int n = a.n;
  const int m = a.o.m;
  const int tid = threadIdx.x;
  constexpr bool f64 = sizeof(T) == 8;
  const auto kc = P::template make<T>(a.coefs);
  FusedInfo* info = a.info;

  // ---- LDS carve-up: FP64 arrays first, then the working-precision ones ----
  double* x64 = smem;
  double* x64t = x64 + n;
  double* H = x64t + n;                 // (m + 1) x m, column-major, ld = m + 1
  double* g = H + (size_t)(m + 1) * m;  // m + 1
  double* cs = g + (m + 1);
  double* sn = cs + m;
  double* yv = sn + m;
  double* hv = yv + m;                  // projections of the current column
  double* sc = hv + kMaxCols;           // scalars and reduction scratch
  T* tbase = reinterpret_cast<T*>(sc + 64);
  T* xw;
  T* xwt;
  T* rest;
  if constexpr (f64) {
    xw = reinterpret_cast<T*>(x64);
    xwt = reinterpret_cast<T*>(x64t);
    rest = tbase;
  } else {
    xw = tbase;
    xwt = tbase + n;
    rest = tbase + 2 * n;
  }
  T* F = rest;
  T* Ft = F + n;
  T* w = Ft + n;
  T* dx = w + n;
  T* bl = dx + n;
  T* V = bl + n;  // m + 1 vectors of n, stride ldv
  const int ldv = fused_ldv(n);

  for (int e = tid; e < n; e += kFusedThreads) {
    const double xv = a.x[e];
    x64[e] = xv;
    if constexpr (!f64) xw[e] = T(xv);
    bl[e] = a.b ? a.b[e] : T(0);
    if (a.history) a.history[e] = xv;
  }
  __syncthreads();

  double fk2 = 0.0, xn2 = 0.0, dummy = 0.0;
  eval<P, T, OP_RES>(kc, a, xw, nullptr, bl, F, T(0), T(1), sc, fk2, xn2);
  const double n0 = sqrt(fk2);
  double fk = n0;
  int k = 0, status = 6, converged = 0;
  int kry = 0, rst = 0, lsb = 0, lsf = 0;

  // w = J(x) v (AD, or FD with the step of the chosen rule; vn = ||v||)
  auto jvp = [&](const T* v, double vn, double& jn2) {
    if (a.o.mode == 0) {
      eval<P, T, OP_AD>(kc, a, xw, v, bl, w, T(0), T(1), sc, jn2, dummy);
    } else {
      const double xn = sqrt(xn2);
      double eps = a.o.fd_eps;
      if (!(eps > 0.0))
        eps = a.o.eps_rule == 0 ? a.o.root_eps * (xn > 1.0 ? xn : 1.0) : a.o.root_eps * (1.0 + xn) / vn;
      eval<P, T, OP_FD>(kc, a, xw, v, bl, w, T(eps), T(eps), sc, jn2, dummy);
    }
  };

  for (;;) {
    if (!isfinite(fk)) {
      status = 4;
      break;
    }
    const double rho = n0 > 0.0 ? fk / n0 : 0.0;
    if (tid == 0) info->rel_res[k] = rho;
    if (rho < a.o.tol_n) {
      status = 0;
      converged = 1;
      break;
    }
    if (k == a.o.max_newton) {
      status = 6;
      break;
    }

    // ---- GMRES(m) on J dx = -F from dx = 0 ----
    int iters = 0, cycles = 0;
    bool nonfinite = false;
    for (int e = tid; e < n; e += kFusedThreads) dx[e] = T(0);
    __syncthreads();
    const double bnorm = fk;  // ||-F||
    if (bnorm > 0.0) {
      const double target = a.o.tol_k * bnorm;
      for (int cycle = 0;; ++cycle) {
        double jn2 = 0.0;
        if (cycle > 0) {
          double dn2 = 0.0, d0 = 0.0;
          double sd = 0.0;
          for (int e = tid; e < n; e += kFusedThreads) sd += (double)dx[e] * (double)dx[e];
          block_sum2(sd, 0.0, sc, dn2, d0);
          jvp(dx, sqrt(dn2), jn2);
        }
        double sr = 0.0;
        for (int e = tid; e < n; e += kFusedThreads) {
          const T r = cycle == 0 ? -F[e] : -F[e] - w[e];
          w[e] = r;
          sr += (double)r * (double)r;
        }
        double beta2 = 0.0;
        block_sum2(sr, 0.0, sc, beta2, dummy);
        const double beta = sqrt(beta2);
        if (!isfinite(beta)) {
          nonfinite = true;
          break;
        }
        if (beta <= target) break;
        if (cycle == a.o.max_restarts) break;
        cycles += 1;
        for (int e = tid; e < n; e += kFusedThreads) V[e] = T((double)w[e] / beta);
        if (tid == 0) {
          g[0] = beta;
          for (int i = 1; i <= m; ++i) g[i] = 0.0;
        }
        __syncthreads();
        int kk = 0;
        for (int j = 0; j < m; ++j) {
          const int K = j + 1;
          jvp(V + (size_t)j * ldv, 1.0, jn2);
          // classical Gram-Schmidt, first pass: h = V^T w, w -= V h
          block_dots<T>(V, n, ldv, K, w, hv);
          for (int e = tid; e < n; e += kFusedThreads) w[e] = cgs_update<T>(w[e], hv, V, ldv, K, e);
          if (tid < K) H[tid + (size_t)j * (m + 1)] = hv[tid];
          __syncthreads();
          // second pass: h2 = V^T w, w -= V h2, ||w||^2
          block_dots<T>(V, n, ldv, K, w, hv);
          double sw = 0.0;
          for (int e = tid; e < n; e += kFusedThreads) {
            const T acc = cgs_update<T>(w[e], hv, V, ldv, K, e);
            w[e] = acc;
            sw += (double)acc * (double)acc;
          }
          if (tid < K) H[tid + (size_t)j * (m + 1)] += hv[tid];
          double wn2 = 0.0;
          block_sum2(sw, 0.0, sc, wn2, dummy);
          const double wn = sqrt(wn2);
          // the next basis vector, written by the other wavefronts while
          // wavefront 0 rotates the column (left unused if the cycle stops
          // at this step)
          if (tid >= kWave)
            for (int e = tid - kWave; e < n; e += kFusedThreads - kWave) V[(size_t)K * ldv + e] = T((double)w[e] / wn);
          // Givens rotations of column j on wavefront 0: lane i holds entry i
          // of the column and rotation i (all read at once).  Rotation i maps
          // the entry carried down the column, cur_i, to
          // cur_{i+1} = -s_i cur_i + c_i h_{i+1}, an affine map; a scan of
          // their compositions across the lanes (log2 j steps) gives every
          // lane its cur_i at once, and lane i forms its rotated entry
          // c_i cur_i + s_i h_{i+1}.  Stop tests published in LDS.
          if (tid < kWave) {
            double* __restrict__ col = H + (size_t)j * (m + 1);
            const double hl = tid < K ? col[tid] : 0.0;
            const double cl = tid < j ? cs[tid] : 0.0;
            const double sl = tid < j ? sn[tid] : 0.0;
            const bool ok = isfinite(wn) && __any(tid < K && !isfinite(hl)) == 0;
            if (ok) {
              const double h0 = lane_f64(hl, 0);
              const double hnext = dpp_f64<0x130>(hl);  // wave_shl:1: h_{i+1} on lane i
              // f_i(x) = A x + B on lanes i < j, the identity above; the
              // scan runs within rows of 16 lanes (shifts 1, 2, 4, 8), then
              // row 1 composes with row 0's total, lane 15's (row_bcast:15):
              // j <= 31, so lanes 32-63 are never read
              double A = tid < j ? -sl : 1.0;
              double B = tid < j ? cl * hnext : 0.0;
              const int r = tid & 15;
              if (j > 1) affine_scan_step<1>(A, B, r >= 1);
              if (j > 2) affine_scan_step<2>(A, B, r >= 2);
              if (j > 4) affine_scan_step<4>(A, B, r >= 4);
              if (j > 8) affine_scan_step<8>(A, B, r >= 8);
              if (j > 16) {
                const double Ap = dpp_f64<0x142>(A), Bp = dpp_f64<0x142>(B);
                if (tid >= 16 && tid < 32) {
                  B = A * Bp + B;
                  A = A * Ap;
                }
              }
              // lane i: f_i o ... o f_0; cur_i from lane i - 1's composition
              // (wave_shr:1)
              const double Ap = dpp_f64<0x138>(A), Bp = dpp_f64<0x138>(B);
              const double cur_i = tid == 0 ? h0 : Ap * h0 + Bp;
              if (tid < j) col[tid] = cl * cur_i + sl * hnext;
              const double cur = j == 0 ? h0 : lane_f64(A, j - 1) * h0 + lane_f64(B, j - 1);
              if (tid == 0) {
                const double ha = cur, hb = wn;
                double c = 1.0, s = 0.0;
                if (hb != 0.0) {
                  const double r = hypot(ha, hb);
                  c = ha / r;
                  s = hb / r;
                }
                cs[j] = c;
                sn[j] = s;
                col[j] = c * ha + s * hb;
                col[j + 1] = 0.0;
                g[j + 1] = -s * g[j];
                g[j] = c * g[j];
                sc[S_EST] = fabs(g[j + 1]);
              }
            } else if (tid == 0) {
              col[K] = wn;
            }
            if (tid == 0) sc[S_FLAG] = ok ? 0.0 : 1.0;
          }
          __syncthreads();
          if (sc[S_FLAG] != 0.0) {
            nonfinite = true;
            break;
          }
          kk = K;
          iters += 1;
          if (sc[S_EST] <= target) break;
          if (wn <= a.o.brk * sqrt(jn2)) break;
        }
        if (nonfinite) break;
        // y = R^{-1} g (back substitution by columns on wavefront 0: lane l
        // keeps row l's partial sum; each y_i, once divided out, is removed
        // from the rows above it in one step), dx += V y
        if (tid < kWave) {
          double t = tid < kk ? g[tid] : 0.0;
          for (int i = kk - 1; i >= 0; --i) {
            const double yi = lane_f64(t, i) / H[i + (size_t)i * (m + 1)];
            if (tid == i) yv[i] = yi;
            if (tid < i) t -= H[tid + (size_t)i * (m + 1)] * yi;
          }
        }
        __syncthreads();
        for (int e = tid; e < n; e += kFusedThreads) {
          T acc = dx[e];
          for (int i = 0; i < kk; ++i) acc = acc + T(yv[i]) * V[(size_t)i * ldv + e];
          dx[e] = acc;
        }
        __syncthreads();
      }
    }
    kry += iters;
    rst += cycles;
    if (tid == 0) info->lin_iters[k] = iters;
    if (nonfinite) {
      status = 4;
      break;
    }

    // ---- backtracking line search on the FP64 merit norm ----
    double alpha = 1.0, ft = 0.0, xt2 = 0.0;
    bool accepted = false;
    for (int t = 0; t <= a.o.ls_max; ++t) {
      for (int e = tid; e < n; e += kFusedThreads) {
        const double xv = x64[e] + alpha * (double)dx[e];
        x64t[e] = xv;
        if constexpr (!f64) xwt[e] = T(xv);
      }
      __syncthreads();
      double ft2 = 0.0;
      eval<P, T, OP_RES>(kc, a, xwt, nullptr, bl, Ft, T(0), T(1), sc, ft2, xt2);
      ft = sqrt(ft2);
      if (isfinite(ft) && ft <= (1.0 - a.o.ls_c * alpha) * fk) {
        accepted = true;
        break;
      }
      if (t < a.o.ls_max) {
        alpha *= 0.5;
        lsb += 1;
      }
    }
    if (!accepted) lsf += 1;
    if (tid == 0) info->alpha[k] = alpha;
    {
      double* t64 = x64; x64 = x64t; x64t = t64;
      T* tw = xw; xw = xwt; xwt = tw;
      T* tf = F; F = Ft; Ft = tf;
    }
    fk = ft;
    xn2 = xt2;
    k += 1;
    if (a.history)
      for (int e = tid; e < n; e += kFusedThreads) a.history[(size_t)k * n + e] = x64[e];
    __syncthreads();
  }

  for (int e = tid; e < n; e += kFusedThreads) a.x[e] = x64[e];
  if (tid == 0) {
    info->status = status;
    info->converged = converged;
    info->newton_iters = k;
    info->krylov_iters = kry;
    info->restarts = rst;
    info->ls_backtracks = lsb;
    info->ls_failures = lsf;
    info->f0_norm = n0;
  }
}

}  // namespace jfnk
