// Pointwise spatial operators N of the benchmark problems, written once over
// a scalar type S (T for the residual and FD, dual<T> for the AD JVP).
//
// Discretization (paper, Section 3.2 and Appendix A): second-order central
// differences on a 5-point stencil, D_x f = (f_{i+1} - f_{i-1}) / (2 hx),
// D_xx f = (f_{i+1} - 2 f_i + f_{i-1}) / hx^2.  Each operator receives the
// centre value and its four neighbours of every field (Nbr) and returns N per
// field; the kernel forms alpha x + cN N(x) + beta b around it.
//
//   Burgers 1D:   N = u D_x u - nu D_xx u
//   Burgers 2D:   N = (u D_x + v D_y) U - nu Lap U            (Appendix A.1)
//   Gray-Scott:   N = (-D Lap u - u^2 v + (F+k) u, -Dv Lap v + u^2 v - F (1-v))
//   Kerr:         N = -Lap E - k0^2 (eps_L + chi3 |E|^2) E on (re, im),
//                 |E|^2 = re^2 + im^2; PEC boundary nodes are identity rows.
//   RD:           N = -D Lap u + u^3                    (Appendix A.3)
//                 homogeneous Dirichlet boundary nodes are identity rows.
//   Su-Olson:     N = (-(1/3) Lap U + (U - V), -xi (U - V))  (Appendix A.2)
//                 Dirichlet boundary nodes are identity rows.
//   Maxwell TE:   N = curl curl E - omega^2 eps(E) E on (Re Ex, Im Ex, Re Ey, Im Ey)
//                 (Appendix A.4), eps = (1 - i loss)(1 + chi |E|), the mixed
//                 derivative D_x D_y from the diagonal neighbours; PEC nodes held.
#pragma once

#include "common.hpp"

namespace jfnk {

template <class S>
struct Nbr {
  S c, l, r, d, u;     // centre, x-1, x+1, y-1, y+1
  S dl, dr, ul, ur;    // (x-1, y-1), (x+1, y-1), (x-1, y+1), (x+1, y+1): operators with kCorners only
};

// Dual-number neighbourhood (value x, tangent v) and the FD trial point x + e v.
template <class P, class T>
__device__ __forceinline__ void nbr_dual(const Nbr<T>& x, const Nbr<T>& v, Nbr<dual<T>>& o) {
  o.c = {x.c, v.c};
  o.l = {x.l, v.l};
  o.r = {x.r, v.r};
  o.d = {x.d, v.d};
  o.u = {x.u, v.u};
  if constexpr (P::kCorners) {
    o.dl = {x.dl, v.dl};
    o.dr = {x.dr, v.dr};
    o.ul = {x.ul, v.ul};
    o.ur = {x.ur, v.ur};
  }
}

template <class P, class T>
__device__ __forceinline__ void nbr_axpy(const Nbr<T>& x, T e, const Nbr<T>& v, Nbr<T>& o) {
  o.c = x.c + e * v.c;
  o.l = x.l + e * v.l;
  o.r = x.r + e * v.r;
  o.d = x.d + e * v.d;
  o.u = x.u + e * v.u;
  if constexpr (P::kCorners) {
    o.dl = x.dl + e * v.dl;
    o.dr = x.dr + e * v.dr;
    o.ul = x.ul + e * v.ul;
    o.ur = x.ur + e * v.ur;
  }
}

// |E| = sqrt(s) with the AD guard of the Maxwell-Kerr permittivity: the
// tangent of |E| is 0 where s = 0 (sqrt is not differentiable there).
template <class T>
__device__ __forceinline__ T guarded_norm(T s) {
  return sqrt(s);
}
template <class T>
__device__ __forceinline__ dual<T> guarded_norm(dual<T> s) {
  const T v = sqrt(s.v);
  return {v, v > T(0) ? s.t / (T(2) * v) : T(0)};
}

// Host-filled coefficient block (double); kernels convert to T.
struct Coefs {
  double c[12];
};

struct Burgers1DOp {
  static constexpr int NF = 1;
  static constexpr bool kDim2 = false;
  static constexpr bool kPeriodic = true;
  static constexpr bool kInterleaved = false;
  static constexpr bool kCorners = false;
  // c: 0 = 1/(2h), 1 = nu/h^2
  template <class T>
  struct K {
    T i2h, nuh2;
  };
  template <class T>
  __host__ __device__ static K<T> make(const Coefs& c) {
    return {T(c.c[0]), T(c.c[1])};
  }
  template <class T, class S>
  __device__ __forceinline__ static void N(const K<T>& k, const Nbr<S> (&f)[1], S (&out)[1]) {
    const Nbr<S>& q = f[0];
    const S dx = (q.r - q.l) * k.i2h;
    const S dxx = (q.r - T(2) * q.c) + q.l;
    out[0] = q.c * dx - k.nuh2 * dxx;
  }
  __device__ __forceinline__ static bool boundary(int, int, int, int) { return false; }
};

struct Burgers2DOp {
  static constexpr int NF = 2;
  static constexpr bool kDim2 = true;
  static constexpr bool kPeriodic = true;
  static constexpr bool kInterleaved = false;
  static constexpr bool kCorners = false;
  // c: 0 = 1/(2hx), 1 = 1/(2hy), 2 = nu/hx^2, 3 = nu/hy^2
  template <class T>
  struct K {
    T i2hx, i2hy, nux, nuy;
  };
  template <class T>
  __host__ __device__ static K<T> make(const Coefs& c) {
    return {T(c.c[0]), T(c.c[1]), T(c.c[2]), T(c.c[3])};
  }
  template <class T, class S>
  __device__ __forceinline__ static void N(const K<T>& k, const Nbr<S> (&f)[2], S (&out)[2]) {
    const S u = f[0].c;
    const S v = f[1].c;
#pragma unroll
    for (int q = 0; q < 2; ++q) {
      const Nbr<S>& a = f[q];
      const S dx = (a.r - a.l) * k.i2hx;
      const S dy = (a.u - a.d) * k.i2hy;
      const S lx = (a.r - T(2) * a.c) + a.l;
      const S ly = (a.u - T(2) * a.c) + a.d;
      out[q] = (u * dx + v * dy) - (k.nux * lx + k.nuy * ly);
    }
  }
  __device__ __forceinline__ static bool boundary(int, int, int, int) { return false; }
};

struct GrayScottOp {
  static constexpr int NF = 2;
  static constexpr bool kDim2 = true;
  static constexpr bool kPeriodic = true;
  static constexpr bool kInterleaved = false;
  static constexpr bool kCorners = false;
  // c: 0 = D/hx^2, 1 = D/hy^2, 2 = Dv/hx^2, 3 = Dv/hy^2, 4 = F + k, 5 = F
  template <class T>
  struct K {
    T dux, duy, dvx, dvy, fk, feed;
  };
  template <class T>
  __host__ __device__ static K<T> make(const Coefs& c) {
    return {T(c.c[0]), T(c.c[1]), T(c.c[2]), T(c.c[3]), T(c.c[4]), T(c.c[5])};
  }
  template <class T, class S>
  __device__ __forceinline__ static void N(const K<T>& k, const Nbr<S> (&f)[2], S (&out)[2]) {
    const Nbr<S>& u = f[0];
    const Nbr<S>& v = f[1];
    const S lu = k.dux * ((u.r - T(2) * u.c) + u.l) + k.duy * ((u.u - T(2) * u.c) + u.d);
    const S lv = k.dvx * ((v.r - T(2) * v.c) + v.l) + k.dvy * ((v.u - T(2) * v.c) + v.d);
    const S uuv = (u.c * u.c) * v.c;
    out[0] = (k.fk * u.c - uuv) - lu;
    out[1] = (uuv - k.feed * (T(1) - v.c)) - lv;
  }
  __device__ __forceinline__ static bool boundary(int, int, int, int) { return false; }
};

struct KerrOp {
  static constexpr int NF = 2;  // real and imaginary parts, interleaved in memory
  static constexpr bool kDim2 = true;
  static constexpr bool kPeriodic = false;
  static constexpr bool kInterleaved = true;
  static constexpr bool kCorners = false;
  // c: 0 = 1/hx^2, 1 = 1/hy^2, 2 = k0^2, 3 = eps_re, 4 = eps_im, 5 = chi3
  template <class T>
  struct K {
    T ihx2, ihy2, k2, er, ei, chi;
  };
  template <class T>
  __host__ __device__ static K<T> make(const Coefs& c) {
    return {T(c.c[0]), T(c.c[1]), T(c.c[2]), T(c.c[3]), T(c.c[4]), T(c.c[5])};
  }
  template <class T, class S>
  __device__ __forceinline__ static void N(const K<T>& k, const Nbr<S> (&f)[2], S (&out)[2]) {
    const Nbr<S>& re = f[0];
    const Nbr<S>& im = f[1];
    const S lre = k.ihx2 * ((re.r - T(2) * re.c) + re.l) + k.ihy2 * ((re.u - T(2) * re.c) + re.d);
    const S lim = k.ihx2 * ((im.r - T(2) * im.c) + im.l) + k.ihy2 * ((im.u - T(2) * im.c) + im.d);
    const S a = k.er + k.chi * (re.c * re.c + im.c * im.c);
    out[0] = -lre - k.k2 * (a * re.c - k.ei * im.c);
    out[1] = -lim - k.k2 * (a * im.c + k.ei * re.c);
  }
  __device__ __forceinline__ static bool boundary(int i, int j, int nx, int ny) {
    return i == 0 || j == 0 || i == nx - 1 || j == ny - 1;
  }
  // The complex shifted-Laplacian preconditioner of Appendix A.4 on this
  // scalar operator, frozen at the state x of an interior node: v's pair
  // (Re, Im) is divided, as a complex number, by
  // M = 2/hx^2 + 2/hy^2 - k0^2 eps(E) (1 - 0.5 i), eps(E) = eps_L + chi3 |E|^2
  // (the diagonal of -Lap and the damped permittivity of the TE form).
  template <class T>
  __device__ __forceinline__ static void cslp_inv(const K<T>& k, const T (&x)[2], T (&v)[2]) {
    const T a = k.er + k.chi * (x[0] * x[0] + x[1] * x[1]);
    // k0^2 eps (1 - 0.5 i) = k2 ((a + ei/2) + (ei - a/2) i)
    const T mr = T(2) * (k.ihx2 + k.ihy2) - k.k2 * (a + T(0.5) * k.ei);
    const T mi = -(k.k2 * (k.ei - T(0.5) * a));
    const T d = T(1) / (mr * mr + mi * mi);
    const T v0 = v[0], v1 = v[1];
    v[0] = (v0 * mr + v1 * mi) * d;
    v[1] = (v1 * mr - v0 * mi) * d;
  }
};

// The Helmholtz-Kerr operator with the CSLP preconditioner applied to every
// JVP tangent (right preconditioning), as MaxwellTECslpOp.
struct KerrCslpOp : KerrOp {
  static constexpr bool kPrecondTangent = true;
};

struct RD2DOp {
  static constexpr int NF = 1;
  static constexpr bool kDim2 = true;
  static constexpr bool kPeriodic = false;
  static constexpr bool kInterleaved = false;
  static constexpr bool kCorners = false;
  // c: 0 = D/hx^2, 1 = D/hy^2
  template <class T>
  struct K {
    T dx, dy;
  };
  template <class T>
  __host__ __device__ static K<T> make(const Coefs& c) {
    return {T(c.c[0]), T(c.c[1])};
  }
  template <class T, class S>
  __device__ __forceinline__ static void N(const K<T>& k, const Nbr<S> (&f)[1], S (&out)[1]) {
    const Nbr<S>& u = f[0];
    const S lu = k.dx * ((u.r - T(2) * u.c) + u.l) + k.dy * ((u.u - T(2) * u.c) + u.d);
    out[0] = (u.c * u.c) * u.c - lu;
  }
  __device__ __forceinline__ static bool boundary(int i, int j, int nx, int ny) {
    return i == 0 || j == 0 || i == nx - 1 || j == ny - 1;
  }
};

struct SuOlsonOp {
  static constexpr int NF = 2;
  static constexpr bool kDim2 = true;
  static constexpr bool kPeriodic = false;
  static constexpr bool kInterleaved = false;
  static constexpr bool kCorners = false;
  // c: 0 = 1/(3 hx^2), 1 = 1/(3 hy^2), 2 = xi
  template <class T>
  struct K {
    T dx, dy, xi;
  };
  template <class T>
  __host__ __device__ static K<T> make(const Coefs& c) {
    return {T(c.c[0]), T(c.c[1]), T(c.c[2])};
  }
  template <class T, class S>
  __device__ __forceinline__ static void N(const K<T>& k, const Nbr<S> (&f)[2], S (&out)[2]) {
    const Nbr<S>& u = f[0];
    const S d = u.c - f[1].c;
    const S lu = k.dx * ((u.r - T(2) * u.c) + u.l) + k.dy * ((u.u - T(2) * u.c) + u.d);
    out[0] = d - lu;
    out[1] = -(k.xi * d);
  }
  __device__ __forceinline__ static bool boundary(int i, int j, int nx, int ny) {
    return i == 0 || j == 0 || i == nx - 1 || j == ny - 1;
  }
};

// Su-Olson's classic 1D-profile configuration (Appendix A.2): the rows wrap
// (periodic in y) and only the first and last columns are Dirichlet nodes.
struct SuOlsonPYOp : SuOlsonOp {
  static constexpr bool kPeriodicRows = true;
  __device__ __forceinline__ static bool boundary(int i, int, int nx, int) { return i == 0 || i == nx - 1; }
};

struct MaxwellTEOp {
  static constexpr int NF = 4;  // planes Re Ex, Im Ex, Re Ey, Im Ey
  static constexpr bool kDim2 = true;
  static constexpr bool kPeriodic = false;
  static constexpr bool kInterleaved = false;
  static constexpr bool kCorners = true;
  // c: 0 = 1/hx^2, 1 = 1/hy^2, 2 = 1/(4 hx hy), 3 = omega^2, 4 = loss, 5 = chi
  template <class T>
  struct K {
    T ixx, iyy, ixy, w2, loss, chi;
  };
  template <class T>
  __host__ __device__ static K<T> make(const Coefs& c) {
    return {T(c.c[0]), T(c.c[1]), T(c.c[2]), T(c.c[3]), T(c.c[4]), T(c.c[5])};
  }
  template <class T, class S>
  __device__ __forceinline__ static S dxdy(const K<T>& k, const Nbr<S>& q) {
    return k.ixy * ((q.ur - q.ul) - (q.dr - q.dl));
  }
  template <class T, class S>
  __device__ __forceinline__ static void N(const K<T>& k, const Nbr<S> (&f)[4], S (&out)[4]) {
    const S xr = f[0].c, xi = f[1].c, yr = f[2].c, yi = f[3].c;
    const S m = T(1) + k.chi * guarded_norm(((xr * xr + xi * xi) + yr * yr) + yi * yi);
    const S dyy0 = k.iyy * ((f[0].u - T(2) * xr) + f[0].d);
    const S dyy1 = k.iyy * ((f[1].u - T(2) * xi) + f[1].d);
    const S dxx2 = k.ixx * ((f[2].r - T(2) * yr) + f[2].l);
    const S dxx3 = k.ixx * ((f[3].r - T(2) * yi) + f[3].l);
    out[0] = (dxdy(k, f[2]) - dyy0) - k.w2 * (m * (xr + k.loss * xi));
    out[1] = (dxdy(k, f[3]) - dyy1) - k.w2 * (m * (xi - k.loss * xr));
    out[2] = (dxdy(k, f[0]) - dxx2) - k.w2 * (m * (yr + k.loss * yi));
    out[3] = (dxdy(k, f[1]) - dxx3) - k.w2 * (m * (yi - k.loss * yr));
  }
  __device__ __forceinline__ static bool boundary(int i, int j, int nx, int ny) {
    return i == 0 || j == 0 || i == nx - 1 || j == ny - 1;
  }
  // Block-diagonal complex shifted-Laplacian preconditioner (Appendix A.4),
  // frozen at the state x of an interior node: v's Ex pair (Re, Im) is
  // divided, as a complex number, by M_xx = 2/hy^2 - omega^2 eps_p and its
  // Ey pair by M_yy = 2/hx^2 - omega^2 eps_p, with the damped permittivity
  // eps_p = (1 - loss i)(1 + chi |E|)(1 - 0.5 i).  (Boundary nodes: identity,
  // left to the caller.)
  template <class T>
  __device__ __forceinline__ static void cslp_inv(const K<T>& k, const T (&x)[4], T (&v)[4]) {
    const T m = T(1) + k.chi * sqrt(((x[0] * x[0] + x[1] * x[1]) + x[2] * x[2]) + x[3] * x[3]);
    // omega^2 eps_p = w2 m ((1 - loss/2) - (loss + 1/2) i)
    const T pr = k.w2 * m * (T(1) - T(0.5) * k.loss);
    const T pi = -(k.w2 * m * (k.loss + T(0.5)));
    const T mi = -pi;                       // Im M_xx = Im M_yy
    const T mxr = T(2) * k.iyy - pr;        // Re M_xx
    const T myr = T(2) * k.ixx - pr;        // Re M_yy
    const T dx = T(1) / (mxr * mxr + mi * mi);
    const T dy = T(1) / (myr * myr + mi * mi);
    const T a0 = v[0], a1 = v[1], b0 = v[2], b1 = v[3];
    v[0] = (a0 * mxr + a1 * mi) * dx;
    v[1] = (a1 * mxr - a0 * mi) * dx;
    v[2] = (b0 * myr + b1 * mi) * dy;
    v[3] = (b1 * myr - b0 * mi) * dy;
  }
};

// The Maxwell-Kerr operator with the CSLP preconditioner applied to every
// JVP tangent (right preconditioning): a type of its own, so that the
// unpreconditioned kernels are compiled without the extra code.
struct MaxwellTECslpOp : MaxwellTEOp {
  static constexpr bool kPrecondTangent = true;
};

// Row (y) periodicity: P::kPeriodicRows where an operator sets it, else the
// operator's kPeriodic (which always governs the columns).
template <class P, class = void>
struct periodic_rows {
  static constexpr bool value = P::kPeriodic;
};
template <class P>
struct periodic_rows<P, decltype((void)P::kPeriodicRows)> {
  static constexpr bool value = P::kPeriodicRows;
};

// Operators whose JVP tangent is preconditioned (P::kPrecondTangent).
template <class P, class = void>
struct precond_tangent {
  static constexpr bool value = false;
};
template <class P>
struct precond_tangent<P, decltype((void)P::kPrecondTangent)> {
  static constexpr bool value = P::kPrecondTangent;
};

}  // namespace jfnk
