// Streaming kernels of BiCGSTAB (paper, Section 2: van der Vorst's
// stabilized bi-conjugate gradient method, the short-recurrence alternative
// to GMRES for nonsymmetric Jacobians; Section 3.3: the same iteration cap
// as the GMRES restart cap).
//
// One iteration i is five kernels, with the two Jacobian-vector products
// done by the stencil kernel (first CGS projection slot reused for one dot
// product):
//   p kernel : checks of iteration i-1 (||r||, omega), rho = (r^, r),
//              beta = (rho / rho_prev) (alpha / omega),
//              p = r + beta (p - omega v)                   [+ ||p||^2]
//   JVP      : v = J p                                      [+ (r^, v)]
//   s kernel : alpha = rho / (r^, v);  s = r - alpha v     [+ ||s||^2]
//   JVP      : t = J s, skipped once ||s|| meets the target [+ (s, t), ||t||^2]
//   xr kernel: half-step stop (x += alpha p) or
//              omega = (t, s) / (t, t); x += alpha p + omega s;
//              r = s - omega t                              [+ (r^, r), ||r||^2]
// Every bracketed sum is a row of FP64 partials per block that the next
// consumer adds in its prologue, as in the GMRES kernels: no grid-wide
// fences or atomics, results independent of timing.  The scalars of the
// recurrence are formed in FP64 by every block alike; block 0 records them
// in BiCtl for later kernels.  Each kernel writes only BiCtl fields that no
// block of the same launch reads (rho alternates between two slots by
// iteration parity, and each stage has its own state field), and a kernel
// that finds the solve stopped carries the state forward before leaving, so
// kernels enqueued after the stop all exit at once.
#pragma once

#include "common.hpp"

namespace jfnk {

struct BiCtl {
  int state_p;    // after the p kernel's checks (read by the JVP of p, the s kernel)
  int state_s;    // after the s kernel (read by the JVP of s, the xr kernel)
  int state_x;    // after the xr kernel (read by the next p kernel)
  int iters;      // completed iterations (a half-step stop counts its iteration)
  double bnorm;   // ||rhs||
  double target;  // tol * ||rhs||
  double res;     // latest ||r|| (or ||s|| at a half-step stop)
  double rho[2];  // (r^, r) of iteration i in slot i & 1
  double alpha;
  double omega;
};

template <class T>
struct BiArgs {
  long long n;        // padded length (all vectors solver-internal, zero padded)
  int it;             // iteration, 1-based
  int check_only;     // p kernel after the last iteration: checks only
  BiCtl* c;
  const T* R;         // init: right-hand side (times sign)
  double sign;
  T* rh;              // shadow residual r^ = r_0
  T* r;
  T* p;
  T* v;               // J p
  T* s;
  T* t;               // J s
  T* x;
  Partials in;        // partial sums read in the prologue
  Partials in2;       // xr kernel: partials of the JVP of s
  PartSink out;
  int* host_flags;    // p kernel: state after its checks, at host_flags[flag_slot]
  int flag_slot;
};

// r = r^ = sign R, x = 0; partials [(r^, r), ||r||^2] (equal here).
template <class T, int VEC>
__global__ void __launch_bounds__(256) bi_init_kernel(const BiArgs<T> a) {
  double acc[2] = {0.0, 0.0};
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
    store_vec<T, VEC>(a.rh + i, r);
    store_vec<T, VEC>(a.x + i, z);
  }
  acc[1] = acc[0];
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    BiCtl* c = a.c;
    c->state_x = kRunning;
    c->iters = 0;
    c->res = 0.0;
    c->alpha = 1.0;
    c->omega = 1.0;
  }
  __shared__ double lds[2 * 4];
  block_partials<2>(acc, 2, a.out.part, a.out.ld, lds);
}

struct BiPScalars {
  int state;
  double rho, beta, res, bnorm, target;
};

// The checks that end iteration it-1 and the scalars of iteration it, from
// the partial sums [(r^, r), ||r||^2] of the previous xr (or init) kernel.
__device__ inline BiPScalars bi_p_scalars(const BiCtl* c, int it, int check_only, double rr_hat, double rr,
                                          double tol) {
  BiPScalars o{kRunning, 0.0, 0.0, 0.0, 0.0, 0.0};
  const double rn = sqrt(rr);
  o.res = rn;
  if (it == 1) {
    o.bnorm = rn;
    o.target = tol * rn;
    if (!isfinite(rn)) {
      o.state = kNonfinite;
      return o;
    }
    if (rn == 0.0) {
      o.state = kConverged;
      return o;
    }
  } else {
    o.bnorm = c->bnorm;
    o.target = c->target;
    if (!isfinite(rn)) {
      o.state = kNonfinite;
      return o;
    }
    if (rn <= o.target) {
      o.state = kConverged;
      return o;
    }
    if (c->omega == 0.0) {
      o.state = kBreakdown;
      return o;
    }
  }
  if (check_only) return o;
  o.rho = rr_hat;
  if (!isfinite(o.rho)) {
    o.state = kNonfinite;
    return o;
  }
  if (o.rho == 0.0) {
    o.state = kBreakdown;
    return o;
  }
  if (it > 1) o.beta = (o.rho / c->rho[(it - 1) & 1]) * (c->alpha / c->omega);
  return o;
}

template <class T, int VEC>
__global__ void __launch_bounds__(256) bi_p_kernel(const BiArgs<T> a, double tol) {
  BiCtl* c = a.c;
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
  __shared__ double tot[2];
  __shared__ BiPScalars sc;
  reduce_partials(a.in, 2, tot);
  if (tid == 0) {
    sc = bi_p_scalars(c, a.it, a.check_only, tot[0], tot[1], tol);
    if (blockIdx.x == 0) {
      if (a.it == 1) {
        c->bnorm = sc.bnorm;
        c->target = sc.target;
      }
      c->res = sc.res;
      c->rho[a.it & 1] = sc.rho;
      c->state_p = sc.state;
      if (a.host_flags) a.host_flags[a.flag_slot] = sc.state;
    }
  }
  __syncthreads();
  if (sc.state != kRunning || a.check_only) return;
  const bool first = a.it == 1;
  const T beta = T(sc.beta);
  const T om = T(c->omega);
  double acc[1] = {0.0};
  const long long step = (long long)gridDim.x * blockDim.x * VEC;
  for (long long i = ((long long)blockIdx.x * blockDim.x + tid) * VEC; i < a.n; i += step) {
    T r[VEC], p[VEC];
    load_vec<T, VEC>(a.r + i, r);
    if (first) {
#pragma unroll
      for (int e = 0; e < VEC; ++e) p[e] = r[e];
    } else {
      T v[VEC];
      load_vec<T, VEC>(a.p + i, p);
      load_vec<T, VEC>(a.v + i, v);
#pragma unroll
      for (int e = 0; e < VEC; ++e) p[e] = r[e] + beta * (p[e] - om * v[e]);
    }
#pragma unroll
    for (int e = 0; e < VEC; ++e) acc[0] += (double)p[e] * (double)p[e];
    store_vec<T, VEC>(a.p + i, p);
  }
  __shared__ double lds[4];
  block_partials<1>(acc, 1, a.out.part, a.out.ld, lds);
}

// alpha = rho / (r^, v); s = r - alpha v with partial sums of ||s||^2.
template <class T, int VEC>
__global__ void __launch_bounds__(256) bi_s_kernel(const BiArgs<T> a) {
  BiCtl* c = a.c;
  const int tid = threadIdx.x;
  const bool lead = blockIdx.x == 0 && tid == 0;
  const int st_in = c->state_p;
  if (st_in != kRunning) {
    if (lead) c->state_s = st_in;
    return;
  }
  __shared__ double tot[1];
  __shared__ int s_state;
  __shared__ double s_alpha;
  reduce_partials(a.in, 1, tot);
  if (tid == 0) {
    const double r0v = tot[0];
    int st = kRunning;
    double al = 0.0;
    if (!isfinite(r0v))
      st = kNonfinite;
    else if (r0v == 0.0)
      st = kBreakdown;
    else
      al = c->rho[a.it & 1] / r0v;
    s_state = st;
    s_alpha = al;
    if (blockIdx.x == 0) {
      c->state_s = st;
      if (st == kRunning) c->alpha = al;
    }
  }
  __syncthreads();
  if (s_state != kRunning) return;
  const T al = T(s_alpha);
  double acc[1] = {0.0};
  const long long step = (long long)gridDim.x * blockDim.x * VEC;
  for (long long i = ((long long)blockIdx.x * blockDim.x + tid) * VEC; i < a.n; i += step) {
    T r[VEC], v[VEC], s[VEC];
    load_vec<T, VEC>(a.r + i, r);
    load_vec<T, VEC>(a.v + i, v);
#pragma unroll
    for (int e = 0; e < VEC; ++e) {
      s[e] = r[e] - al * v[e];
      acc[0] += (double)s[e] * (double)s[e];
    }
    store_vec<T, VEC>(a.s + i, s);
  }
  __shared__ double lds[4];
  block_partials<1>(acc, 1, a.out.part, a.out.ld, lds);
}

// Half-step stop, or omega and the x / r updates with partial sums
// [(r^, r), ||r||^2] for the next p kernel.
template <class T, int VEC>
__global__ void __launch_bounds__(256) bi_xr_kernel(const BiArgs<T> a) {
  BiCtl* c = a.c;
  const int tid = threadIdx.x;
  const bool lead = blockIdx.x == 0 && tid == 0;
  const int st_in = c->state_s;
  if (st_in != kRunning) {
    if (lead) c->state_x = st_in;
    return;
  }
  __shared__ double tot[1];
  __shared__ double tot2[2];
  __shared__ int s_state;
  __shared__ int s_half;
  __shared__ double s_omega;
  reduce_partials(a.in, 1, tot);
  if (tid == 0) {
    const double sn = sqrt(tot[0]);
    s_half = 0;
    s_state = kRunning;
    if (!isfinite(sn))
      s_state = kNonfinite;
    else if (sn <= c->target)
      s_half = 1;
  }
  __syncthreads();
  const bool half = s_half != 0;
  if (s_state == kRunning && !half) {
    // the JVP of s ran: its partial sums hold (s, t) and ||t||^2
    reduce_partials(a.in2, 2, tot2);
    if (tid == 0) {
      const double ts = tot2[0], tt = tot2[1];
      if (!(isfinite(ts) && isfinite(tt)))
        s_state = kNonfinite;
      else if (tt == 0.0)
        s_state = kBreakdown;
      else
        s_omega = ts / tt;
    }
    __syncthreads();
  }
  const int st = s_state;
  if (lead) {
    c->state_x = half ? kConverged : st;
    if (st == kRunning) c->iters = a.it;
    if (half) c->res = sqrt(tot[0]);
    if (st == kRunning && !half) c->omega = s_omega;
  }
  if (st != kRunning) return;
  const T al = T(c->alpha);
  const T om = half ? T(0) : T(s_omega);
  double acc[2] = {0.0, 0.0};
  const long long step = (long long)gridDim.x * blockDim.x * VEC;
  for (long long i = ((long long)blockIdx.x * blockDim.x + tid) * VEC; i < a.n; i += step) {
    T x[VEC], p[VEC];
    load_vec<T, VEC>(a.x + i, x);
    load_vec<T, VEC>(a.p + i, p);
    if (half) {
#pragma unroll
      for (int e = 0; e < VEC; ++e) x[e] = x[e] + al * p[e];
    } else {
      T s[VEC], t[VEC], rh[VEC], r[VEC];
      load_vec<T, VEC>(a.s + i, s);
      load_vec<T, VEC>(a.t + i, t);
      load_vec<T, VEC>(a.rh + i, rh);
#pragma unroll
      for (int e = 0; e < VEC; ++e) {
        x[e] = x[e] + al * p[e] + om * s[e];
        r[e] = s[e] - om * t[e];
        acc[0] += (double)rh[e] * (double)r[e];
        acc[1] += (double)r[e] * (double)r[e];
      }
      store_vec<T, VEC>(a.r + i, r);
    }
    store_vec<T, VEC>(a.x + i, x);
  }
  if (!half) {
    __shared__ double lds[2 * 4];
    block_partials<2>(acc, 2, a.out.part, a.out.ld, lds);
  }
}

}  // namespace jfnk
