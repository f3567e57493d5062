// Streaming kernels of conjugate gradients (paper, Section 2: Hestenes and
// Stiefel's method for symmetric positive-definite systems; the paper runs it
// on the reaction-diffusion problem, whose linearization is SPD).
//
// One iteration i is three kernels, the Jacobian-vector product done by the
// stencil kernel with its fused-projection slot taking (p, J p):
//   p kernel : checks of iteration i-1 (||r||), beta = (r, r)_i / (r, r)_{i-1},
//              p = r + beta p                             [+ ||p||^2]
//   JVP      : q = J p                                    [+ (p, q)]
//   xr kernel: (p, q) <= 0 -> breakdown; alpha = (r, r) / (p, q);
//              x += alpha p; r -= alpha q                 [+ (r, r)]
// The partial-sum and control conventions are those of the BiCGSTAB kernels:
// FP64 sums reduced by the consumer, scalars formed by every block alike and
// recorded by block 0 in fields no block of the same launch reads ((r, r)
// alternates between two slots by iteration parity), stopped states carried
// forward by kernels queued after the stop.
#pragma once

#include "common.hpp"

namespace jfnk {

struct CgCtl {
  int state_p;    // after the p kernel's checks (read by the JVP and the xr kernel)
  int state_x;    // after the xr kernel (read by the next p kernel)
  int iters;      // completed iterations
  int pad0;
  double bnorm;   // ||rhs||
  double target;  // tol * ||rhs||
  double res;     // latest ||r||
  double rr[2];   // (r, r) at the start of iteration i in slot i & 1
};

template <class T>
struct CgArgs {
  long long n;        // padded length (solver-internal, zero-padded vectors)
  int it;             // iteration, 1-based
  int check_only;     // p kernel after the last iteration: checks only
  CgCtl* c;
  const T* R;         // init: right-hand side (times sign)
  double sign;
  T* r;
  T* p;
  T* q;               // J p
  T* x;
  Partials in;        // partial sums read in the prologue
  PartSink out;
  int* host_flags;    // p kernel: state after its checks, at host_flags[flag_slot]
  int flag_slot;
};

// r = sign R, x = 0; partials of (r, r).
template <class T, int VEC>
__global__ void __launch_bounds__(256) cg_init_kernel(const CgArgs<T> a) {
  double acc[1] = {0.0};
  const T sg = T(a.sign);
  const long long step = (long long)gridDim.x * blockDim.x * VEC;
  for (long long i = ((long long)blockIdx.x * blockDim.x + threadIdx.x) * VEC; i < a.n; i += step) {
    T r[VEC], z[VEC];
    load_vec<T, VEC>(a.R + i, r);
#pragma unroll
    for (int e = 0; e < VEC; ++e) {
      r[e] = sg * r[e];
      z[e] = T(0);
      acc[0] += (double)r[e] * (double)r[e];
    }
    store_vec<T, VEC>(a.r + i, r);
    store_vec<T, VEC>(a.x + i, z);
  }
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    a.c->state_x = kRunning;
    a.c->iters = 0;
    a.c->res = 0.0;
  }
  __shared__ double lds[4];
  block_partials<1>(acc, 1, a.out.part, a.out.ld, lds);
}

template <class T, int VEC>
__global__ void __launch_bounds__(256) cg_p_kernel(const CgArgs<T> a, double tol) {
  CgCtl* c = a.c;
  const int tid = threadIdx.x;
  const bool lead = blockIdx.x == 0 && tid == 0;
  const int st_in = c->state_x;
  if (st_in != kRunning) {
    if (lead) {
      c->state_p = st_in;
      if (a.host_flags) a.host_flags[a.flag_slot] = st_in;
    }
    return;
  }
  __shared__ double tot[1];
  __shared__ int s_state;
  __shared__ double s_beta;
  reduce_partials(a.in, 1, tot);
  if (tid == 0) {
    const double rr = tot[0];
    const double rn = sqrt(rr);
    int st = kRunning;
    double target;
    if (a.it == 1) {
      target = tol * rn;
      if (!isfinite(rn))
        st = kNonfinite;
      else if (rn == 0.0)
        st = kConverged;
    } else {
      target = c->target;
      if (!isfinite(rn))
        st = kNonfinite;
      else if (rn <= target)
        st = kConverged;
    }
    s_state = st;
    s_beta = a.it > 1 ? rr / c->rr[(a.it - 1) & 1] : 0.0;
    if (blockIdx.x == 0) {
      if (a.it == 1) {
        c->bnorm = rn;
        c->target = target;
      }
      c->res = rn;
      c->rr[a.it & 1] = rr;
      c->state_p = st;
      if (a.host_flags) a.host_flags[a.flag_slot] = st;
    }
  }
  __syncthreads();
  if (s_state != kRunning || a.check_only) return;
  const bool first = a.it == 1;
  const T beta = T(s_beta);
  double acc[1] = {0.0};
  const long long step = (long long)gridDim.x * blockDim.x * VEC;
  for (long long i = ((long long)blockIdx.x * blockDim.x + tid) * VEC; i < a.n; i += step) {
    T r[VEC], p[VEC];
    load_vec<T, VEC>(a.r + i, r);
    if (first) {
#pragma unroll
      for (int e = 0; e < VEC; ++e) p[e] = r[e];
    } else {
      load_vec<T, VEC>(a.p + i, p);
#pragma unroll
      for (int e = 0; e < VEC; ++e) p[e] = r[e] + beta * p[e];
    }
#pragma unroll
    for (int e = 0; e < VEC; ++e) acc[0] += (double)p[e] * (double)p[e];
    store_vec<T, VEC>(a.p + i, p);
  }
  __shared__ double lds[4];
  block_partials<1>(acc, 1, a.out.part, a.out.ld, lds);
}

template <class T, int VEC>
__global__ void __launch_bounds__(256) cg_xr_kernel(const CgArgs<T> a) {
  CgCtl* c = a.c;
  const int tid = threadIdx.x;
  const bool lead = blockIdx.x == 0 && tid == 0;
  const int st_in = c->state_p;
  if (st_in != kRunning) {
    if (lead) c->state_x = st_in;
    return;
  }
  __shared__ double tot[1];
  __shared__ int s_state;
  __shared__ double s_alpha;
  reduce_partials(a.in, 1, tot);
  if (tid == 0) {
    const double pq = tot[0];
    int st = kRunning;
    double al = 0.0;
    if (!isfinite(pq))
      st = kNonfinite;
    else if (pq <= 0.0)
      st = kBreakdown;
    else
      al = c->rr[a.it & 1] / pq;
    s_state = st;
    s_alpha = al;
    if (blockIdx.x == 0) {
      c->state_x = st;
      if (st == kRunning) c->iters = a.it;
    }
  }
  __syncthreads();
  if (s_state != kRunning) return;
  const T al = T(s_alpha);
  double acc[1] = {0.0};
  const long long step = (long long)gridDim.x * blockDim.x * VEC;
  for (long long i = ((long long)blockIdx.x * blockDim.x + tid) * VEC; i < a.n; i += step) {
    T x[VEC], p[VEC], r[VEC], q[VEC];
    load_vec<T, VEC>(a.x + i, x);
    load_vec<T, VEC>(a.p + i, p);
    load_vec<T, VEC>(a.r + i, r);
    load_vec<T, VEC>(a.q + i, q);
#pragma unroll
    for (int e = 0; e < VEC; ++e) {
      x[e] = x[e] + al * p[e];
      r[e] = r[e] - al * q[e];
      acc[0] += (double)r[e] * (double)r[e];
    }
    store_vec<T, VEC>(a.x + i, x);
    store_vec<T, VEC>(a.r + i, r);
  }
  __shared__ double lds[4];
  block_partials<1>(acc, 1, a.out.part, a.out.ld, lds);
}

}  // namespace jfnk
