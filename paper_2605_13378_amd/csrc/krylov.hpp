// Krylov kernels of restarted GMRES(m) with CGS2 Arnoldi (paper, Section 2:
// GMRES minimizes the residual over the Krylov space and is restarted).
//
// One Arnoldi step j (K = j + 1 basis vectors V_0..V_j, w = J v_j) is three
// streaming passes, each a single read of the basis:
//   pass A:  h  = V^T w,  ||w||^2                        (CGS, first projection)
//   pass B:  w -= V h;   h2 = V^T w                      (update fused with the second projection)
//   pass C:  w -= V h2;  ||w||^2;  V_{j+1} <- w          (update fused with the norm)
// Each pass writes one row of FP64 partial sums per block; the next kernel
// adds them in its prologue (pass B the h of pass A, pass C the h2 of pass B,
// and the JVP of step j+1 -- or the V y kernel at the end of a cycle -- the
// ||w||^2 of pass C, after which it applies the previous Givens rotations to
// the new Hessenberg column, forms the new rotation and updates g, in FP64).
// The basis is stored unnormalized: V_i holds a multiple of v_i and
// Ctl::scale[i] = 1 / ||V_i|| is folded into the coefficients instead of a
// separate normalization pass.  Coefficients and stop flags live in the
// device control block, so a cycle runs without host round trips.
//
// Threads hold VEC consecutive elements of w and of every basis vector in
// registers, so each element of V is loaded once per pass and the update and
// the dot products share that load.  All vectors here are solver-internal,
// padded with zeros to a multiple of 256 elements and 256-byte aligned.
#pragma once

#include "common.hpp"

namespace jfnk {

enum { PASS_A = 0, PASS_B = 1, PASS_C = 2 };

// ---------------------------------------------------------------------------
// Givens update of Hessenberg column j (FP64), in the prologue of the kernel
// that follows the pass which produced the column's last sums.  The first
// wavefront of every block does it: the lanes check and prepare the
// column's entries in parallel, one lane runs the rotation chain, and block 0
// commits the result to Ctl.
// ---------------------------------------------------------------------------
struct GivensOut {
  double c, s, gr, gp1, est, wn;
  double vs;  // scale of the stored V_{j+1}: 1 / (||w|| * storage scale)
  int done;
};

// Inputs of one column update, gathered into LDS by all threads at once.
struct GivensIn {
  double h[kMaxM + 1];  // hA + hB
  double cs[kMaxM];
  double sn[kMaxM];
  double gp, tol_abs, brk_tol, jvn2, sig;
};

__device__ inline void givens_gather(const Ctl* __restrict__ ctl, int j, GivensIn& in) {
  const int tid = threadIdx.y * blockDim.x + threadIdx.x;
  if (tid <= j) in.h[tid] = ctl->hA[tid] + ctl->hB[tid];
  if (tid < j) {
    in.cs[tid] = ctl->cs[tid];
    in.sn[tid] = ctl->sn[tid];
  }
  if (tid == 0) {
    in.gp = ctl->gp[j];
    in.tol_abs = ctl->tol_abs;
    in.brk_tol = ctl->brk_tol;
    in.jvn2 = ctl->jvn2;
    in.sig = ctl->vsig[j + 1];
  }
}

// Column j = (in.h[0..j], sqrt(wn2)) rotated by G_0..G_{j-1}, the new rotation
// G_j and the g update, written to `col` (LDS, j + 2 entries) and `out` (LDS).
// Called by the threads of the first wavefront (tid < 64); `any_bad` is their
// vote on a non-finite entry of in.h.  The rotated entry is carried in a
// register from one rotation to the next, with the rotation inputs read from
// LDS four at a time ahead of the arithmetic, so the chain costs FP64
// latency only (a column kept in LDS costs an LDS round trip per rotation).
__device__ inline void givens_column(const GivensIn& in, int j, double wn2, bool any_bad, double* col,
                                     GivensOut& out) {
  if (threadIdx.x != 0 || threadIdx.y != 0) return;
  GivensOut o;
  o.wn = sqrt(wn2);
  o.vs = 1.0 / (o.wn * in.sig);
  double a = in.h[0];
  for (int i0 = 0; i0 < j; i0 += 4) {
    double hb[4], cb[4], sb[4];
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const int i = i0 + u < kMaxM ? i0 + u : kMaxM - 1;  // in bounds; slots past j unused
      hb[u] = in.h[i + 1];
      cb[u] = in.cs[i];
      sb[u] = in.sn[i];
    }
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      if (i0 + u < j) {
        const double b = hb[u];
        col[i0 + u] = cb[u] * a + sb[u] * b;
        a = -sb[u] * a + cb[u] * b;
      }
    }
  }
  o.c = 1.0;
  o.s = 0.0;
  if (o.wn != 0.0) {
    const double r = hypot(a, o.wn);
    o.c = a / r;
    o.s = o.wn / r;
  }
  col[j] = o.c * a + o.s * o.wn;
  col[j + 1] = 0.0;
  o.gr = o.c * in.gp;
  o.gp1 = -o.s * in.gp;
  o.est = fabs(o.gp1);
  const bool finite = !any_bad && isfinite(o.wn) && isfinite(a) && isfinite(o.est);
  o.done = kRunning;
  if (!finite)
    o.done = kNonfinite;
  else if (o.est <= in.tol_abs)
    o.done = kConverged;
  else if (o.wn <= in.brk_tol * sqrt(in.jvn2))
    o.done = kBreakdown;
  out = o;
}

// Block 0's commit of column j, after a barrier: the rotated column to H and
// the unrotated one (`ucol`, j + 2 entries in LDS) to Hu by the lanes of the
// first wavefront, the scalars by lane 0.
__device__ inline void givens_commit(Ctl* __restrict__ ctl, int j, const GivensOut& o, const double* col,
                                     const double* ucol, int* host_flags) {
  const int tid = threadIdx.y * blockDim.x + threadIdx.x;
  const int ld = kMaxM + 1;
  if (tid <= j + 1) {
    ctl->H[j * ld + tid] = col[tid];
    ctl->Hu[j * ld + tid] = ucol[tid];
  }
  if (tid == 0) {
    ctl->cs[j] = o.c;
    ctl->sn[j] = o.s;
    ctl->gr[j] = o.gr;
    ctl->gp[j + 1] = o.gp1;
    ctl->res_est = o.est;
    ctl->scale[j + 1] = o.vs;
    ctl->done_col[j + 1] = o.done;
    if (host_flags) host_flags[j] = o.done;
  }
}

// Prologue of the kernel that follows pass C of step j (the JVP of step j+1
// or the V y update): reduce ||w||^2 and update column j.  Every thread of
// every block gets the same outcome; `col` (LDS, kMaxM + 1 doubles) receives
// the rotated column.
__device__ inline GivensOut finish_column(Ctl* __restrict__ ctl, int j, const Partials& pc, int* host_flags,
                                          double* col) {
  __shared__ double tot[1];
  __shared__ GivensIn in;
  __shared__ GivensOut out;
  __shared__ double ucol[kMaxM + 2];
  givens_gather(ctl, j, in);
  reduce_partials(pc, 1, tot);  // ends with a barrier: `in` is complete too
  const int tid = threadIdx.y * blockDim.x + threadIdx.x;
  if (tid < kWave) {
    const bool any_bad = __any(tid <= j && !isfinite(in.h[tid])) != 0;
    if (tid <= j) ucol[tid] = in.h[tid];
    givens_column(in, j, tot[0], any_bad, col, out);  // lane 0 only
    if (tid == 0) ucol[j + 1] = out.wn;
  }
  __syncthreads();
  if (blockIdx.x == 0 && blockIdx.y == 0) givens_commit(ctl, j, out, col, ucol, host_flags);
  return out;
}

// Inputs of the completion of column c in the delayed form, fetched into
// registers before a kernel's main loads (lagged_prefetch) so that their
// round trips overlap those loads.
struct LaggedPrefetch {
  PartialFetch pf;
  double h, cs, sn;
  double gp, tol_abs, brk_tol, jvn2, sig;  // thread 0's scalars of the column update
};

// All of these are vector loads issued before the kernel's main loads: a
// control-block read issued after them would wait for them to complete.
template <bool HALF = false>
__device__ __forceinline__ void lagged_prefetch(const Ctl* __restrict__ ctl, int c, const Partials& pd,
                                                LaggedPrefetch& lp) {
  const int tid = threadIdx.y * blockDim.x + threadIdx.x;
  const int ld = kMaxM + 1;
  partials_fetch(pd, c + 2, lp.pf);
  lp.h = tid <= c ? ctl->Hp[c * ld + tid] : 0.0;
  lp.cs = tid < c ? ctl->cs[tid] : 0.0;
  lp.sn = tid < c ? ctl->sn[tid] : 0.0;
  if (tid == 0) {
    lp.gp = ctl->gp[c];
    lp.tol_abs = ctl->tol_abs;
    lp.brk_tol = ctl->brk_tol;
    lp.jvn2 = ctl->jvn2c[c];
    lp.sig = HALF ? ctl->vsig[c + 1] : 1.0;
  }
}

// Delayed second pass (the alternative Arnoldi form): column c is completed
// by the kernel after the update pass of step c, from that pass's partial
// sums pd = [v_0..v_c . u, u . u] of the pending vector u (once projected):
// a = V^T u, beta = sqrt(u.u - a.a), column = (first projection + a, beta),
// then the Givens update as for CGS2.  Block 0 commits the unrotated column,
// the rotation, a / beta and 1 / (beta sigma) (the tangent scale of step
// c + 1; sigma = vsig[c + 1] is the FP16 storage scale of u, 1 otherwise).
template <bool HALF>
__device__ __forceinline__ GivensOut finish_column_lagged_from(Ctl* __restrict__ ctl, int c, const Partials& pd,
                                                               int* host_flags, double* col, const LaggedPrefetch& lp) {
  __shared__ double tot[kMaxM + 2];
  __shared__ GivensIn in;
  __shared__ GivensOut out;
  __shared__ double ucol[kMaxM + 2];
  __shared__ double s_beta;
  const int tid = threadIdx.y * blockDim.x + threadIdx.x;
  // the first projection comes from Hp, which no block of this kernel
  // writes; block 0 commits the completed column to Hu, which no block of
  // this kernel reads
  if (tid <= c) in.h[tid] = lp.h;
  if (tid < c) {
    in.cs[tid] = lp.cs;
    in.sn[tid] = lp.sn;
  }
  if (tid == 0) {
    in.gp = lp.gp;
    in.tol_abs = lp.tol_abs;
    in.brk_tol = lp.brk_tol;
    in.jvn2 = lp.jvn2;
    in.sig = lp.sig;
  }
  __shared__ double s_b2;
  __shared__ int s_bad;
  partials_reduce(pd, c + 2, lp.pf, tot);  // ends with a barrier: `in` is complete too
  if (tid < kWave) {
    // the second-pass coefficients a_i = tot[i] (lane i), ||a||^2 over the wavefront
    const double ai = tid <= c ? tot[tid] : 0.0;
    const double aa = wave_sum(ai * ai);
    const double uu = tot[c + 1];
    const double b2 = uu - aa;
    bool bad = false;
    if (tid <= c) {
      const double h = in.h[tid] + ai;
      in.h[tid] = h;
      ucol[tid] = h;
      bad = !isfinite(h);
    }
    const bool any_bad = __any(bad) != 0;
    if (tid == 0) {
      s_b2 = b2 > 0.0 ? b2 : 0.0;
      s_bad = (any_bad || !isfinite(uu)) ? 1 : 0;
      s_beta = b2 > 0.0 ? sqrt(b2) : 0.0;
      ucol[c + 1] = s_beta;
    }
  }
  __syncthreads();
  givens_column(in, c, s_b2, s_bad != 0, col, out);  // its norm is sqrt(b2) = beta; lane 0 only
  __syncthreads();
  if (blockIdx.x == 0 && blockIdx.y == 0) {
    givens_commit(ctl, c, out, col, ucol, host_flags);
    if (tid <= c) ctl->ahat[tid] = tot[tid] / s_beta;
    if (tid == 0) ctl->tscale[c + 1] = out.vs;
  }
  return out;
}

// The same, fetching its own inputs.
template <bool HALF>
__device__ inline GivensOut finish_column_lagged(Ctl* __restrict__ ctl, int c, const Partials& pd, int* host_flags,
                                                 double* col) {
  LaggedPrefetch lp;
  lagged_prefetch<HALF>(ctl, c, pd, lp);
  return finish_column_lagged_from<HALF>(ctl, c, pd, host_flags, col, lp);
}

// ---------------------------------------------------------------------------
// CGS passes
// ---------------------------------------------------------------------------
template <class T, class VT>
struct KArgs {
  long long n;        // padded length
  const VT* V;        // basis, vector i at V + i * vstride
  long long vstride;
  T* w;               // working vector
  VT* wout;           // pass C destination (V_{j+1})
  int K;              // basis vectors in use (j + 1)
  Ctl* ctl;
  Partials in;        // partials of the previous pass (B: pass A's, C: pass B's)
  PartSink out;       // this pass's partial sums
  int nt;             // 1: basis read with the non-temporal hint
};

// One thread's chunks of the K basis vectors (VEC consecutive elements of
// each), held in registers in the working precision T.  FP16 storage keeps
// them as loaded, two elements to a 32-bit register, and converts an element
// where it is used: twice the elements per load for the same registers.
// Chunks k >= K are never loaded and stay zero, so the arithmetic runs over
// all KMAX slots without per-slot conditions (a zero coefficient times a zero
// element leaves every sum unchanged, exactly).
// NT: basis read with the non-temporal hint (a template parameter: a
// run-time choice between two load sequences costs the register-resident
// basis chunk its registers).
template <class T, class VT, int KMAX, int VEC>
struct Chunks {
  T v[KMAX][VEC];
  __device__ __forceinline__ void zero() {
#pragma unroll
    for (int k = 0; k < KMAX; ++k)
#pragma unroll
      for (int e = 0; e < VEC; ++e) v[k][e] = T(0);
  }
  template <bool NT>
  __device__ __forceinline__ void load(const VT* p, int k) {
    VT t[VEC];
    if constexpr (NT)
      load_vec_nt<VT, VEC>(p, t);
    else
      load_vec<VT, VEC>(p, t);
#pragma unroll
    for (int e = 0; e < VEC; ++e) v[k][e] = to_c<T>(t[e]);
  }
  __device__ __forceinline__ T get(int k, int e) const { return v[k][e]; }
};

template <int KMAX, int VEC>
struct Chunks<float, __half, KMAX, VEC> {
  static_assert(VEC % 2 == 0, "FP16 chunks hold element pairs");
  unsigned int v[KMAX][VEC / 2];
  __device__ __forceinline__ void zero() {
#pragma unroll
    for (int k = 0; k < KMAX; ++k)
#pragma unroll
      for (int e = 0; e < VEC / 2; ++e) v[k][e] = 0u;
  }
  template <bool NT>
  __device__ __forceinline__ void load(const __half* p, int k) {
    if constexpr (NT)
      load_vec_nt<unsigned int, VEC / 2>(reinterpret_cast<const unsigned int*>(p), v[k]);
    else
      load_vec<unsigned int, VEC / 2>(reinterpret_cast<const unsigned int*>(p), v[k]);
  }
  __device__ __forceinline__ float get(int k, int e) const {
    const unsigned int u = v[k][e >> 1];
    const unsigned short h = (unsigned short)((e & 1) ? (u >> 16) : (u & 0xffffu));
    return __half2float(__ushort_as_half(h));
  }
};

// Loads w and the K basis chunks at element i.
template <class T, class VT, int KMAX, int VEC, bool NT>
__device__ __forceinline__ void cgs_load(const KArgs<T, VT>& a, long long i, int K, T (&w)[VEC],
                                         Chunks<T, VT, KMAX, VEC>& vv) {
  load_vec<T, VEC>(a.w + i, w);
#pragma unroll
  for (int k = 0; k < KMAX; ++k)
    if (k < K) vv.template load<NT>(a.V + k * a.vstride + i, k);
}

// Dot product of one thread's VEC-element chunks, returned in FP64 for the
// FP64 accumulation across chunks.  FP64 arithmetic: exact products summed in
// FP64.  FP32 arithmetic: the VEC products are summed in FP32 first (one
// conversion per chunk instead of one per element); the chunk sum carries a
// relative error of a few 2^-24, which stays far below the FP32 rounding of
// the vectors themselves, also for the small second-pass projections.
template <class T, int VEC>
__device__ __forceinline__ double group_dot(const T (&a)[VEC], const T (&b)[VEC]) {
  if constexpr (sizeof(T) == 4) {
    T p = a[0] * b[0];
#pragma unroll
    for (int e = 1; e < VEC; ++e) p = fmaf(a[e], b[e], p);
    return (double)p;
  } else {
    double p = 0.0;
#pragma unroll
    for (int e = 0; e < VEC; ++e) p += (double)a[e] * (double)b[e];
    return p;
  }
}

// The same with basis chunk k as the first operand.
template <class T, class VT, int KMAX, int VEC>
__device__ __forceinline__ double group_dot(const Chunks<T, VT, KMAX, VEC>& a, int k, const T (&b)[VEC]) {
  if constexpr (sizeof(T) == 4) {
    T p = a.get(k, 0) * b[0];
#pragma unroll
    for (int e = 1; e < VEC; ++e) p = fmaf(a.get(k, e), b[e], p);
    return (double)p;
  } else {
    double p = 0.0;
#pragma unroll
    for (int e = 0; e < VEC; ++e) p += (double)a.get(k, e) * (double)b[e];
    return p;
  }
}

template <class T, class VT, int KMAX, int VEC, int MODE, bool NT>
__global__ void __launch_bounds__(512) cgs_kernel(const KArgs<T, VT> a) {
  Ctl* ctl = a.ctl;
  const int K = a.K;
  const long long step = (long long)gridDim.x * blockDim.x * VEC;
  long long i = ((long long)blockIdx.x * blockDim.x + threadIdx.x) * VEC;
  // the first chunk's loads go out before the stop check and the coefficient
  // reduction (in-bounds either way; unused if the cycle has stopped)
  T w[VEC];
  Chunks<T, VT, KMAX, VEC> vv;
  vv.zero();
  if (i < a.n) cgs_load<T, VT, KMAX, VEC, NT>(a, i, K, w, vv);
  if (ctl->done_col[K - 1] != kRunning) return;  // state after the Givens update of column K-2

  __shared__ double tot[KMAX + 1];
  __shared__ double s_sig;
  T coef[KMAX];
  T sig = T(1);
  if constexpr (MODE != PASS_A) {
    // projections of the previous pass on the stored vectors (+ ||J v_j||^2
    // from pass A; + ||w||^2 from pass B when the basis is stored in FP16)
    reduce_partials(a.in, (MODE == PASS_B || is_half<VT>()) ? K + 1 : K, tot);
#pragma unroll
    for (int k = 0; k < KMAX; ++k) coef[k] = uniform(k < K ? T(tot[k] * ctl->scale[k] * ctl->scale[k]) : T(0));
    if (blockIdx.x == 0 && threadIdx.x < K) {
      const double h = tot[threadIdx.x] * ctl->scale[threadIdx.x];
      if (MODE == PASS_B)
        ctl->hA[threadIdx.x] = h;
      else
        ctl->hB[threadIdx.x] = h;
    }
    if (MODE == PASS_B && blockIdx.x == 0 && threadIdx.x == 0) ctl->jvn2 = tot[K];
    if constexpr (MODE == PASS_C) {
      if (threadIdx.x == 0) {
        double sg = 1.0;
        if constexpr (is_half<VT>()) {
          // ||w_C||^2 = ||w_B||^2 - ||h2||^2 (orthogonal projection), to pick
          // the power-of-two storage scale before w_C is written
          double p2 = 0.0;
          for (int k = 0; k < K; ++k) {
            const double h = tot[k] * ctl->scale[k];
            p2 += h * h;
          }
          const double wb2 = tot[K];
          const double wc2 = wb2 - p2;
          sg = fp16_scale(sqrt(wc2 > 1e-6 * wb2 ? wc2 : 1e-6 * wb2), a.n);
        }
        s_sig = sg;
        if (blockIdx.x == 0) ctl->vsig[K] = sg;
      }
      __syncthreads();
      sig = T(s_sig);
    }
  }
  double acc[KMAX + 1];
#pragma unroll
  for (int k = 0; k <= KMAX; ++k) acc[k] = 0.0;

  for (; i < a.n; i += step) {
    if constexpr (MODE == PASS_A) {
#pragma unroll
      for (int kb = 0; kb < KMAX; kb += 4)
        if (kb < K)
#pragma unroll
          for (int u = 0; u < 4 && kb + u < KMAX; ++u) acc[kb + u] += group_dot(vv, kb + u, w);
#pragma unroll
      for (int e = 0; e < VEC; ++e) acc[KMAX] += (double)w[e] * (double)w[e];
    } else {
      T wn[VEC];
#pragma unroll
      for (int e = 0; e < VEC; ++e) {
        T x = w[e];
#pragma unroll
        for (int k = 0; k < KMAX; ++k) x = x - coef[k] * vv.get(k, e);
        wn[e] = x;
      }
      if constexpr (MODE == PASS_B) {
        // groups of four slots behind one uniform branch; chunks k >= K in a
        // partly used group are zero and add exactly 0
#pragma unroll
        for (int kb = 0; kb < KMAX; kb += 4)
          if (kb < K)
#pragma unroll
            for (int u = 0; u < 4 && kb + u < KMAX; ++u) acc[kb + u] += group_dot(vv, kb + u, wn);
        if constexpr (is_half<VT>()) {
#pragma unroll
          for (int e = 0; e < VEC; ++e) acc[KMAX] += (double)wn[e] * (double)wn[e];
        }
        store_vec<T, VEC>(a.w + i, wn);
      } else {
#pragma unroll
        for (int e = 0; e < VEC; ++e) acc[0] += (double)wn[e] * (double)wn[e];
        VT o[VEC];
#pragma unroll
        for (int e = 0; e < VEC; ++e) o[e] = to_s<VT>(is_half<VT>() ? wn[e] * sig : wn[e]);
        store_vec<VT, VEC>(a.wout + i, o);
      }
    }
    if (i + step < a.n) cgs_load<T, VT, KMAX, VEC, NT>(a, i + step, K, w, vv);
  }

  int nr = MODE == PASS_C ? 1 : K;
  if constexpr (MODE == PASS_A || (MODE == PASS_B && is_half<VT>())) {
    // move ||w||^2 next to the K dot products (static indices keep acc in registers)
#pragma unroll
    for (int k = 0; k < KMAX; ++k)
      if (k == K) acc[k] = acc[KMAX];
    nr = K + 1;
  }
  __shared__ double lds[(KMAX + 1) * 8];
  block_partials<KMAX + 1>(acc, nr, a.out.part, a.out.ld, lds);
}

// Update pass of the delayed-second-pass Arnoldi step j (K = j + 1 slots:
// final V_0..V_{j-1} and the pending U_j, the JVP tangent of step j, with
// w = J (tscale_j U_j) from the Arnoldi JVP).  With a^ the second-pass
// coefficients of U_j and H the completed columns 0..j-1, every block forms in
// FP64 from the JVP's partial sums P = [V_0..V_j . w, w . w]:
//   b_i = P_i (i < j), d = tscale_j P_j, gamma = d - a^.b,
//   h_i = b_i - (H a^)_i, h_j = gamma - (H a^)_j        (first projection of J v_j)
// and streams
//   V_j     <- tscale_j U_j - sum_i a^_i V_i           (v_j, unit norm)
//   U_{j+1} <- w - sum_i ((H a^)_i + h_i - gamma a^_i) V_i - gamma tscale_j U_j
// with partial sums [v_0..v_j . U_{j+1}, ||U_{j+1}||^2] for the next column's
// completion.  Block 0 commits h to the unrotated Hessenberg, scale_j and
// ||w||^2.  One read of the basis per step, where CGS2 takes two.
//
// FP16 storage: both written vectors are stored times a scale fixed before
// the stream starts, sigma_v = fp16_scale(1) for the unit v_j (scale_j =
// 1 / sigma_v; at j = 0 sigma_v = 1 / tscale_0, which leaves the stored V_0
// as it is) and sigma_u = fp16_scale(||U_{j+1}||) from the orthogonal
// projection identity ||U_{j+1}||^2 ~ ||w||^2 - ||h||^2 (vsig[j + 1], folded
// into the next tangent scale by the completion).  The sums for the
// completion are taken over the rounded stored values, so the second pass
// projects what the basis actually holds.
template <class T, class VT, int KMAX, int VEC, bool NT>
__global__ void __launch_bounds__(512) dcgs_kernel(const KArgs<T, VT> a) {
  Ctl* ctl = a.ctl;
  const int K = a.K;
  const int j = K - 1;
  const long long step = (long long)gridDim.x * blockDim.x * VEC;
  long long i = ((long long)blockIdx.x * blockDim.x + threadIdx.x) * VEC;
  const int state = ctl->done_col[j];  // state after column j-1, tested once the loads below are out

  // The prologue's loads (partial sums, control-block inputs) go out first,
  // then the first basis chunk, whose round trip then overlaps the prologue's
  // arithmetic (vector loads complete in order: the prologue waits only for
  // its own, older loads).  If the cycle has stopped the loads are unused.
  PartialFetch pf;
  partials_fetch(a.in, K + 1, pf);
  __shared__ double tot[KMAX + 1];
  __shared__ double sh_ah[KMAX], sh_sc[KMAX], sh_b[KMAX], sh_ha[KMAX + 1];
  __shared__ double sh_cv[KMAX], sh_cw[KMAX];
  __shared__ double sh_hu[KMAX * KMAX];  // completed columns 0..j-1, rows 0..j (stride j + 1)
  __shared__ double sh_ts;
  __shared__ double sh_sv, sh_su;  // FP16 storage scales of v_j and U_{j+1}
  const int tid = threadIdx.x;
  const int ld = kMaxM + 1;
  // control-block inputs loaded into registers by all threads at once (at
  // most two completed-column entries each: j (j + 1) <= 992 < 2 * 512) and
  // staged into LDS only after the basis loads have gone out: an LDS store
  // waits for its load, and the basis loads would queue behind that wait
  const int nhu = j * (j + 1);
  const int i0 = tid, i1 = tid + blockDim.x;
  double hu0 = 0.0, hu1 = 0.0, ah = 0.0, sc = 0.0, ts = 0.0;
  if (i0 < nhu) hu0 = ctl->Hu[(i0 / (j + 1)) * ld + i0 % (j + 1)];
  if (i1 < nhu) hu1 = ctl->Hu[(i1 / (j + 1)) * ld + i1 % (j + 1)];
  if (tid < j) {
    ah = ctl->ahat[tid];
    sc = ctl->scale[tid];
  }
  if (tid == 0) ts = ctl->tscale[j];
  T w[VEC];
  Chunks<T, VT, KMAX, VEC> vv;
  vv.zero();
  if (i < a.n) cgs_load<T, VT, KMAX, VEC, NT>(a, i, K, w, vv);
  if (state != kRunning) return;
  if (i0 < nhu) sh_hu[i0] = hu0;
  if (i1 < nhu) sh_hu[i1] = hu1;
  if (tid < j) {
    sh_ah[tid] = ah;
    sh_sc[tid] = sc;
  }
  if (tid == 0) sh_ts = ts;
  partials_reduce(a.in, K + 1, pf, tot);  // ends with a barrier
  if (tid < j) sh_b[tid] = tot[tid] * sh_sc[tid];
  {
    // (H a^)_i over the completed columns 0..j-1 (row j only has column
    // j-1): row i by 16 lanes (32 rows x 16 lanes = the 512 threads), each
    // summing every 16th column, then a 16-lane sum
    const int r = tid >> 4, g = tid & 15;
    double s = 0.0;
    if (r <= j)
      for (int l = g; l < j; l += 16) s += sh_hu[l * (j + 1) + r] * sh_ah[l];
    s = group_sum<16>(s);
    if (r <= j && g == 0) sh_ha[r] = s;
  }
  __syncthreads();
  if (tid < kWave) {
    // the coefficients, lane l for vector l (j < 64), sums across the wavefront
    const int l = tid;
    const double ts = sh_ts;
    const double ahl = l < j ? sh_ah[l] : 0.0;
    const double bl = l < j ? sh_b[l] : 0.0;
    const double gamma = ts * tot[j] - wave_sum(ahl * bl);
    double hl = 0.0;
    if (l < j) {
      hl = bl - sh_ha[l];
      sh_cv[l] = -ahl * sh_sc[l];
      sh_cw[l] = (sh_ha[l] + hl - gamma * ahl) * sh_sc[l];
    } else if (l == j) {
      hl = gamma - sh_ha[j];
      sh_cv[j] = ts;
      sh_cw[j] = gamma * ts;
    }
    if (blockIdx.x == 0 && l <= j) ctl->Hp[j * ld + l] = hl;
    double sv = 1.0, su = 1.0;
    if constexpr (is_half<VT>()) {
      const double hh = wave_sum(hl * hl);
      const double ww = tot[K];
      const double uu = ww - hh;
      // v_0 = tscale_0 U_0 is U_0 itself: stored with the inverse scale, the
      // rewrite returns its FP16 values unchanged instead of rounding again
      sv = j == 0 ? 1.0 / ts : fp16_scale(1.0, a.n);
      su = fp16_scale(sqrt(uu > 1e-6 * ww ? uu : 1e-6 * ww), a.n);
    }
    if (l == 0) {
      sh_sv = sv;
      sh_su = su;
      if (blockIdx.x == 0) {
        ctl->scale[j] = 1.0 / sv;
        ctl->vsig[j + 1] = su;
        ctl->jvn2c[j] = tot[K];
      }
    }
  }
  __syncthreads();
  T cv[KMAX], cw[KMAX];
#pragma unroll
  for (int k = 0; k < KMAX; ++k) {
    cv[k] = uniform(k < K ? T(sh_cv[k]) : T(0));
    cw[k] = uniform(k < K ? T(sh_cw[k]) : T(0));
  }
  double acc[KMAX + 1];
#pragma unroll
  for (int k = 0; k <= KMAX; ++k) acc[k] = 0.0;
  double accv = 0.0;
  VT* vj_out = a.wout - a.vstride;  // slot j (wout is slot j + 1)
  if constexpr (is_half<VT>()) {
    // FP16 storage: both vectors are rounded to their scaled FP16 values as
    // they are formed, and the sums are taken over those stored values with
    // packed FP16 dot products (the products of two FP16 numbers are exact in
    // FP32, the chunk sums carry a few 2^-24) -- the basis chunks are used in
    // their packed form, with no second conversion
    const float sv = (float)sh_sv, su = (float)sh_su;
    for (; i < a.n; i += step) {
      // vector by vector, so that each converted element is used at once
      float x[VEC], y[VEC];
#pragma unroll
      for (int e = 0; e < VEC; ++e) {
        x[e] = 0.0f;
        y[e] = w[e];
      }
#pragma unroll
      for (int k = 0; k < KMAX; ++k)
#pragma unroll
        for (int e = 0; e < VEC; ++e) {
          x[e] = fma_mix_half(cv[k], vv.v[k][e >> 1], e & 1, x[e]);
          y[e] = y[e] - cw[k] * vv.get(k, e);
        }
      unsigned int p1[VEC / 2], p2[VEC / 2];
#pragma unroll
      for (int e = 0; e < VEC; e += 2) {
        p1[e / 2] = pack_half2(x[e] * sv, x[e + 1] * sv);
        p2[e / 2] = pack_half2(y[e] * su, y[e + 1] * su);
      }
#pragma unroll
      for (int kb = 0; kb < KMAX; kb += 4)
        if (kb < K)
#pragma unroll
          for (int u = 0; u < 4 && kb + u < KMAX; ++u) acc[kb + u] += dot_half2<VEC / 2>(vv.v[kb + u], p2);
      accv += dot_half2<VEC / 2>(p1, p2);
      acc[KMAX] += dot_half2<VEC / 2>(p2, p2);
      store_vec<unsigned int, VEC / 2>(reinterpret_cast<unsigned int*>(vj_out + i), p1);
      store_vec<unsigned int, VEC / 2>(reinterpret_cast<unsigned int*>(a.wout + i), p2);
      if (i + step < a.n) cgs_load<T, VT, KMAX, VEC, NT>(a, i + step, K, w, vv);
    }
    // back to unscaled sums: V_i = v_i / scale_i (i < j), the stored v_j and
    // U_{j+1} carry sigma_v and sigma_u (powers of two, exact, except for
    // v_0's scale: one FP64 rounding)
    const double isu = 1.0 / sh_su;
#pragma unroll
    for (int k = 0; k < KMAX; ++k)
      if (k < j) acc[k] *= sh_sc[k] * isu;
    accv *= isu / sh_sv;
    acc[KMAX] *= isu * isu;
  } else {
    for (; i < a.n; i += step) {
      T vn[VEC], wn[VEC];
#pragma unroll
      for (int e = 0; e < VEC; ++e) {
        T x = T(0);
        T y = w[e];
#pragma unroll
        for (int k = 0; k < KMAX; ++k) {
          const T v = vv.get(k, e);
          x = x + cv[k] * v;
          y = y - cw[k] * v;
        }
        vn[e] = x;
        wn[e] = y;
      }
      // groups of four slots behind one uniform branch; slot j's product (with
      // U_j) is replaced by the one with the new v_j below
#pragma unroll
      for (int kb = 0; kb < KMAX; kb += 4)
        if (kb < K)
#pragma unroll
          for (int u = 0; u < 4 && kb + u < KMAX; ++u) acc[kb + u] += group_dot(vv, kb + u, wn);
      accv += group_dot<T, VEC>(vn, wn);
#pragma unroll
      for (int e = 0; e < VEC; ++e) acc[KMAX] += (double)wn[e] * (double)wn[e];
      store_vec<VT, VEC>(vj_out + i, vn);
      store_vec<VT, VEC>(a.wout + i, wn);
      if (i + step < a.n) cgs_load<T, VT, KMAX, VEC, NT>(a, i + step, K, w, vv);
    }
  }
  // [v_0..v_{j-1} . U_{j+1}, v_j . U_{j+1}, ||U_{j+1}||^2] (static indices keep acc in registers)
#pragma unroll
  for (int k = 0; k < KMAX; ++k) {
    if (k == j) acc[k] = accv;
    if (k == K) acc[k] = acc[KMAX];
  }
  __shared__ double lds[(KMAX + 1) * 8];
  block_partials<KMAX + 1>(acc, K + 1, a.out.part, a.out.ld, lds);
}

// Start of a restart cycle: V_0 = sign * R - w (w nullable) and its partial
// norms; cycle_begin_kernel then fixes beta, g, scale[0] and the flags.
template <class T, class VT>
struct InitArgs {
  long long n;
  const T* R;
  double sign;
  const T* w;   // nullable
  VT* V0;
  PartSink out;
  T* tmp;       // FP16 storage: r is written here in the working precision
};

template <class T, class VT, int VEC>
__global__ void __launch_bounds__(256) init_cycle_kernel(const InitArgs<T, VT> a) {
  double acc[1] = {0.0};
  const T sg = T(a.sign);
  const long long step = (long long)gridDim.x * blockDim.x * VEC;
  for (long long i = ((long long)blockIdx.x * blockDim.x + threadIdx.x) * VEC; i < a.n; i += step) {
    T r[VEC];
    load_vec<T, VEC>(a.R + i, r);
    if (a.w != nullptr) {
      T w[VEC];
      load_vec<T, VEC>(a.w + i, w);
#pragma unroll
      for (int e = 0; e < VEC; ++e) r[e] = sg * r[e] - w[e];
    } else {
#pragma unroll
      for (int e = 0; e < VEC; ++e) r[e] = sg * r[e];
    }
#pragma unroll
    for (int e = 0; e < VEC; ++e) acc[0] += (double)r[e] * (double)r[e];
    if constexpr (is_half<VT>()) {
      store_vec<T, VEC>(a.tmp + i, r);
    } else {
      store_vec<VT, VEC>(a.V0 + i, r);
    }
  }
  __shared__ double lds[4];
  block_partials<1>(acc, 1, a.out.part, a.out.ld, lds);
}

// One block: beta = ||V_0||; the first cycle of a solve also fixes ||rhs||.
template <int kUnused = 0>
__global__ void __launch_bounds__(256) cycle_begin_kernel(Ctl* ctl, Partials in, int m, long long n, int fp16) {
  __shared__ double tot[1];
  reduce_partials(in, 1, tot);
  if (threadIdx.x == 0) {
    const double beta = sqrt(tot[0]);
    const double sig = fp16 ? fp16_scale(beta, n) : 1.0;
    ctl->vsig[0] = sig;
    if (ctl->first) {
      ctl->bnorm = beta;
      ctl->tol_abs = ctl->tol * beta;
      ctl->first = 0;
    }
    ctl->beta = beta;
    ctl->res_est = beta;
    ctl->gp[0] = beta;
    ctl->scale[0] = 1.0 / (beta * sig);
    ctl->k = 0;
    ctl->tscale[0] = ctl->scale[0];
    ctl->done_col[0] = !isfinite(beta) ? kNonfinite : (beta <= ctl->tol_abs ? kConverged : kRunning);
  }
  if (threadIdx.x >= 1 && threadIdx.x <= m) ctl->done_col[threadIdx.x] = kRunning;
}

// FP16 storage of a caller's tangent (standalone JVP of an FP16S solver):
// sigma = fp16_scale(||v||) from the FP64 norm at *vn2, out = half(v sigma)
// (n entries, any alignment) and *inv_sigma = 1 / sigma, the scale the JVP
// folds back in.
template <int kUnused = 0>
__global__ void __launch_bounds__(256) fp16_tangent_kernel(long long n, const float* __restrict__ v,
                                                           __half* __restrict__ out, const double* vn2,
                                                           double* inv_sigma) {
  const double sig = fp16_scale(sqrt(*vn2), n);
  const float sf = (float)sig;
  const long long step = (long long)gridDim.x * blockDim.x;
  for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += step)
    out[i] = __float2half_rn(v[i] * sf);
  if (blockIdx.x == 0 && threadIdx.x == 0) *inv_sigma = 1.0 / sig;
}

// FP16 storage of the first basis vector: V_0 = half(r * vsig[0]).
template <class T, class VT, int VEC>
__global__ void __launch_bounds__(256) store_basis0_kernel(long long n, const T* __restrict__ r, VT* __restrict__ V0,
                                                          const Ctl* ctl) {
  const T sig = T(ctl->vsig[0]);
  const long long step = (long long)gridDim.x * blockDim.x * VEC;
  for (long long i = ((long long)blockIdx.x * blockDim.x + threadIdx.x) * VEC; i < n; i += step) {
    T x[VEC];
    load_vec<T, VEC>(r + i, x);
    VT o[VEC];
#pragma unroll
    for (int e = 0; e < VEC; ++e) o[e] = to_s<VT>(x[e] * sig);
    store_vec<VT, VEC>(V0 + i, o);
  }
}

// End of a cycle: finish the pending Givens column (if the last enqueued step
// ran), y = R^{-1} g by back substitution (FP64, every block alike), then
// dx = [dx] + sum_i y_i scale_i V_i with its partial norms.
template <class T, class VT>
struct VyArgs {
  long long n;
  const VT* V;
  long long vstride;
  T* dx;
  int first;    // 1: dx = V y (dx not read)
  int jmax;     // last Arnoldi step enqueued in this cycle (-1: none)
  Ctl* ctl;
  Partials pc;  // partial norms of the last pass C (delayed form: of the last update pass)
  PartSink out;  // partial sums of ||dx||^2
  int* host_flags;
  int lagged;    // 1: the basis comes from the delayed-second-pass Arnoldi steps
  int nt;        // 1: basis read with the non-temporal hint
};

template <class T, class VT, int KMAX, int VEC, bool NT>
__global__ void __launch_bounds__(512) vy_kernel(const VyArgs<T, VT> a) {
  Ctl* ctl = a.ctl;
  __shared__ double y[kMaxM];
  __shared__ double lastcol[kMaxM + 1];
  __shared__ double lastgr;
  __shared__ int flags[kMaxM + 1];
  __shared__ double R[kMaxM * kMaxM];  // columns l < k of the rotated H (rows i <= l), column-major
  __shared__ double gr[kMaxM];
  __shared__ int s_k;
  const int tid = threadIdx.x;
  const int nt = blockDim.x;
  // stop flags of the cycle, read by all threads at once
  if (a.jmax >= 0 && tid <= a.jmax) flags[tid] = ctl->done_col[tid];
  __syncthreads();
  // columns completed: stop at the first column whose Givens update ended the cycle
  if (tid == 0) {
    int kk = 0;
    if (a.jmax >= 0 && flags[0] == kRunning) {
      kk = a.jmax + 1;
      for (int c = 0; c < a.jmax; ++c)
        if (flags[c + 1] != kRunning) {
          kk = c + 1;
          break;
        }
    }
    s_k = kk;
  }
  __syncthreads();
  const int k = s_k;
  const bool pending = a.jmax >= 0 && k == a.jmax + 1;
  __shared__ int lastdone;
  if (pending) {
    const GivensOut g = a.lagged ? finish_column_lagged<is_half<VT>()>(ctl, a.jmax, a.pc, a.host_flags, lastcol)
                                 : finish_column(ctl, a.jmax, a.pc, a.host_flags, lastcol);
    if (tid == 0) {
      lastgr = g.gr;
      lastdone = g.done;
    }
  }
  // block 0 may just have written column k-1 of H: every block uses the
  // column it computed itself for that one; the others are staged in LDS
  const int ld = kMaxM + 1;
  const int kc = pending ? k - 1 : k;  // columns read from the control block
  for (int idx = tid; idx < kc * kMaxM; idx += nt) {
    const int l = idx / kMaxM, i = idx % kMaxM;
    if (i <= l) R[l * kMaxM + i] = ctl->H[l * ld + i];
  }
  if (tid < k) gr[tid] = (pending && tid == k - 1) ? 0.0 : ctl->gr[tid];
  __syncthreads();
  // y = R^{-1} g by columns on the first wavefront: lane i keeps row i's
  // partial sum, and each y_l, once divided out, is taken out of the rows
  // above it in one step (k dependent steps, not k^2 / 2)
  if (tid < kWave) {
    double t = tid < k ? ((pending && tid == k - 1) ? lastgr : gr[tid]) : 0.0;
    for (int l = k - 1; l >= 0; --l) {
      const bool last = pending && l == k - 1;  // the column this kernel completed itself
      const double yl = lane_f64(t, l) / (last ? lastcol[l] : R[l * kMaxM + l]);
      if (tid == l) y[l] = yl;
      if (tid < l) t -= (last ? lastcol[tid] : R[l * kMaxM + tid]) * yl;
    }
    if (tid == 0 && blockIdx.x == 0) {
      ctl->k = k;
      ctl->k_last = k;
      ctl->k_last_state = k == 0 ? kRunning : (pending ? lastdone : flags[k]);
    }
  }
  __syncthreads();
  T coef[KMAX];
#pragma unroll
  for (int c = 0; c < KMAX; ++c) coef[c] = uniform(c < k ? T(y[c] * ctl->scale[c]) : T(0));
  double acc[1] = {0.0};
  const long long step = (long long)gridDim.x * blockDim.x * VEC;
  for (long long i = ((long long)blockIdx.x * blockDim.x + threadIdx.x) * VEC; i < a.n; i += step) {
    T d[VEC];
    if (a.first) {
#pragma unroll
      for (int e = 0; e < VEC; ++e) d[e] = T(0);
    } else {
      load_vec<T, VEC>(a.dx + i, d);
    }
    Chunks<T, VT, KMAX, VEC> t;
    t.zero();
#pragma unroll
    for (int c = 0; c < KMAX; ++c)
      if (c < k) t.template load<NT>(a.V + c * a.vstride + i, c);
#pragma unroll
    for (int c = 0; c < KMAX; ++c)
#pragma unroll
      for (int e = 0; e < VEC; ++e) d[e] = d[e] + coef[c] * t.get(c, e);
#pragma unroll
    for (int e = 0; e < VEC; ++e) acc[0] += (double)d[e] * (double)d[e];
    store_vec<T, VEC>(a.dx + i, d);
  }
  __shared__ double lds[8];
  block_partials<1>(acc, 1, a.out.part, a.out.ld, lds);
}

// One block: write column sums of earlier partial rows to device scalars.
template <int kUnused = 0>
__global__ void __launch_bounds__(256) finish_sums_kernel(Partials in, int nr, double* out0, double* out1) {
  __shared__ double tot[2];
  reduce_partials(in, nr, tot);
  if (threadIdx.x == 0) {
    *out0 = tot[0];
    if (nr > 1 && out1) *out1 = tot[1];
  }
}

// Newton trial point: x64t = x64 + alpha dx (FP64 accumulation of the update),
// xw = working-precision copy (nullable when the working precision is FP64).
template <class T, int VEC>
__global__ void __launch_bounds__(256) newton_trial_kernel(long long n, const double* __restrict__ x64,
                                                           const T* __restrict__ dx, double alpha,
                                                           double* __restrict__ x64t, T* __restrict__ xw) {
  const long long step = (long long)gridDim.x * blockDim.x * VEC;
  for (long long i = ((long long)blockIdx.x * blockDim.x + threadIdx.x) * VEC; i < n; i += step) {
    double x[VEC];
    T d[VEC];
    load_vec<double, VEC>(x64 + i, x);
    load_vec<T, VEC>(dx + i, d);
    T o[VEC];
#pragma unroll
    for (int e = 0; e < VEC; ++e) {
      x[e] = x[e] + alpha * (double)d[e];
      o[e] = T(x[e]);
    }
    store_vec<double, VEC>(x64t + i, x);
    if (xw != nullptr) store_vec<T, VEC>(xw + i, o);
  }
}

// Working-precision copy of an FP64 vector.
template <class T, int VEC>
__global__ void __launch_bounds__(256) cast_kernel(long long n, const double* __restrict__ src, T* __restrict__ dst) {
  const long long step = (long long)gridDim.x * blockDim.x * VEC;
  for (long long i = ((long long)blockIdx.x * blockDim.x + threadIdx.x) * VEC; i < n; i += step) {
    double x[VEC];
    load_vec<double, VEC>(src + i, x);
    T o[VEC];
#pragma unroll
    for (int e = 0; e < VEC; ++e) o[e] = T(x[e]);
    store_vec<T, VEC>(dst + i, o);
  }
}

// Partial sums of p^2 over an arbitrary (possibly unaligned) vector.
template <class T>
__global__ void __launch_bounds__(256) norm2_kernel(long long n, const T* __restrict__ p, PartSink out) {
  double acc[1] = {0.0};
  const long long step = (long long)gridDim.x * blockDim.x;
  for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += step) {
    const double v = (double)p[i];
    acc[0] += v * v;
  }
  __shared__ double lds[4];
  block_partials<1>(acc, 1, out.part, out.ld, lds);
}

// Zero fill (used instead of memset so every step is a plain kernel).
template <class T>
__global__ void __launch_bounds__(256) fill_zero_kernel(long long n, T* __restrict__ p) {
  const long long step = (long long)gridDim.x * blockDim.x;
  for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += step) p[i] = T(0);
}

// Begin a GMRES solve: reset the control flags on the device.
template <int kUnused = 0>
__global__ void ctl_begin_kernel(Ctl* c, double tol, double brk_tol, int m) {
  if (threadIdx.x == 0 && blockIdx.x == 0) {
    c->k = 0;
    c->m = m;
    c->first = 1;
    c->tol = tol;
    c->brk_tol = brk_tol;
    c->tol_abs = 0.0;
    c->bnorm = 0.0;
  }
}

// Publish the control block's head (the scalars the host driver reads between
// kernels: counts, stop states, norms; `words` 32-bit words) to mapped host
// memory, then set the sequence word there to `seq`.  The host waits by
// spinning on that word instead of a stream synchronization plus a copy; the
// kernel runs after everything before it on the stream, so the head is
// final.  One wavefront, vector stores only.
template <int kUnused = 0>
__global__ void __launch_bounds__(64) publish_ctl_kernel(const Ctl* __restrict__ c, int* __restrict__ dst, int words,
                                                         int* __restrict__ seq_dst, int seq) {
  const int* src = reinterpret_cast<const int*>(c);
  for (int i = threadIdx.x; i < words; i += blockDim.x) dst[i] = src[i];
  __threadfence_system();
  __syncthreads();
  if (threadIdx.x == 0) {
    __threadfence_system();
    *reinterpret_cast<volatile int*>(seq_dst) = seq;
  }
}

}  // namespace jfnk
