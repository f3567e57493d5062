// Fused stencil kernel: residual, AD JVP and FD JVP in one template.
//
//   OP_RES: out = alpha x + cN N(x) + beta b                 (residual F(x))
//   OP_AD : out = alpha v + cN [N'(x) v]   (+ out2 = F(x))   (AD JVP, dual numbers)
//   OP_FD : out = (F(x + eps v) - F(x)) / eps                (FD JVP, both in registers)
//
// Paper, Section 2: the AD JVP returns F(x) and J(x) v from one evaluation of
// the residual on dual numbers; the FD JVP evaluates the same residual twice
// and differences.  Here both live in a single pass over HBM: each thread
// owns VEC consecutive columns of RY consecutive rows, loads rows
// r0-1 .. r0+RY (periodic wrap, or clamp for PEC) of x (and v) once with
// 8/16-byte accesses, gets its left/right neighbours from the adjacent lane
// by cross-lane shuffle (global load only at wavefront and grid edges), and
// writes out with vector stores.  The tangent is carried in the same
// registers as the value (dual<T>), so the AD JVP costs one read of x and v
// and one write of Jv: three vectors of HBM traffic.
//
// Layout: SoA planes (field f at f * plane), row-major rows of nx elements;
// Kerr: interleaved (re, im) pairs.  Any nx, ny; the vector path needs nx a
// multiple of VEC and 16-byte aligned pointers (the host picks VEC = 1
// otherwise).  Optional FP64 reductions of sum(out^2) and sum(x^2) (residual
// norm and state norm for the FD step) go through grid_reduce.
#pragma once

#include "common.hpp"
#include "krylov.hpp"
#include "problems.hpp"

namespace jfnk {

enum { OP_RES = 0, OP_AD = 1, OP_FD = 2 };

template <class T, class VT>
struct StencilArgs {
  int nx, ny;
  long long plane;     // nx * ny
  const T* x;          // linearization point / state
  const VT* v;         // direction (stored; true v = vscale * v)
  const T* b;          // pointwise term multiplied by beta (nullable -> 0)
  T* out;              // F (RES) or Jv
  T* out2;             // F (AD with F output), nullable
  double alpha, cN, beta;
  const double* vscale;  // device scalar, nullable -> 1
  EpsSpec eps;
  // Arnoldi JVP of step arn_j (ctl non-null, with the fused projection: Vb
  // set): finishes the Givens update of column arn_j - 1 from pass C's
  // partials `pc`, stops early once the cycle is done, and takes the basis
  // scale from that update.
  Ctl* ctl;
  int arn_j;
  int lagged;            // delayed-second-pass Arnoldi: pc holds the update pass's sums
  Partials pc;
  int* host_flags;
  PartSink part_out;     // RES: partial sums of sum(out^2) and sum(x^2)
  int nred;              // 0, 1 or 2 reductions
  // Arnoldi JVP with the first CGS projection fused in (KDOT > 0):
  // partial sums of V_k . Jv for k < K and of ||Jv||^2 go to dots_out.
  const VT* Vb;          // basis, vector k at Vb + k * vstride
  long long vstride;
  int K;
  int nt_basis;          // 1: basis rows read with the non-temporal hint
  PartSink dots_out;
  // BiCGSTAB JVPs (gate non-null): leave at once when *gate is not
  // kRunning, or, with gate_parts rows, when the square root of their
  // column-0 sum is not above *gate_tol (the half-step stop test).
  const int* gate;
  Partials gate_parts;
  const double* gate_tol;
  // Right preconditioning (problems with a diagonal preconditioner only):
  // the JVP is applied to M^{-1} v, M frozen at x; the launcher picks the
  // operator type that applies it.
  int precond;
};

template <bool PERIODIC>
__device__ __forceinline__ int wrap_idx(int i, int n) {
  if (PERIODIC) {
    i %= n;
    return i < 0 ? i + n : i;
  }
  return i < 0 ? 0 : (i >= n ? n - 1 : i);
}

template <class P, class S, int VEC>
__device__ __forceinline__ void load_nodes(const S* __restrict__ base, long long plane, int nx, int r, int c,
                                           S (&out)[P::NF][VEC]) {
  if constexpr (P::kInterleaved) {
    S tmp[2 * VEC];
    load_vec<S, 2 * VEC>(base + 2 * ((long long)r * nx + c), tmp);
#pragma unroll
    for (int e = 0; e < VEC; ++e) {
      out[0][e] = tmp[2 * e];
      out[1][e] = tmp[2 * e + 1];
    }
  } else {
#pragma unroll
    for (int f = 0; f < P::NF; ++f) load_vec<S, VEC>(base + f * plane + (long long)r * nx + c, out[f]);
  }
}

// load_nodes with the non-temporal hint (basis rows read once per pass)
template <class P, class S, int VEC>
__device__ __forceinline__ void load_nodes_nt(const S* __restrict__ base, long long plane, int nx, int r, int c,
                                              S (&out)[P::NF][VEC]) {
  if constexpr (P::kInterleaved) {
    S tmp[2 * VEC];
    load_vec_nt<S, 2 * VEC>(base + 2 * ((long long)r * nx + c), tmp);
#pragma unroll
    for (int e = 0; e < VEC; ++e) {
      out[0][e] = tmp[2 * e];
      out[1][e] = tmp[2 * e + 1];
    }
  } else {
#pragma unroll
    for (int f = 0; f < P::NF; ++f) load_vec_nt<S, VEC>(base + f * plane + (long long)r * nx + c, out[f]);
  }
}

// The pointwise term b of the RC centre rows starting at r0 (zero when not used).
template <class P, class T, int VEC, int RC>
__device__ __forceinline__ void load_b_rows(const T* __restrict__ b, long long plane, int nx, int ny, int r0, int cc,
                                            bool use, T (&bv)[RC][P::NF][VEC]) {
#pragma unroll
  for (int tt = 0; tt < RC; ++tt) {
    T t[P::NF][VEC];
#pragma unroll
    for (int f = 0; f < P::NF; ++f)
#pragma unroll
      for (int e = 0; e < VEC; ++e) t[f][e] = T(0);
    if (use) {
      const int r = r0 + tt;
      load_nodes<P, T, VEC>(b, plane, nx, P::kDim2 ? (r < ny ? r : 0) : 0, cc, t);
    }
#pragma unroll
    for (int f = 0; f < P::NF; ++f)
#pragma unroll
      for (int e = 0; e < VEC; ++e) bv[tt][f][e] = t[f][e];
  }
}

template <class P, class S>
__device__ __forceinline__ S load_node(const S* __restrict__ base, long long plane, int nx, int r, int c, int f) {
  if constexpr (P::kInterleaved) return base[2 * ((long long)r * nx + c) + f];
  return base[f * plane + (long long)r * nx + c];
}

template <class P, class S, int VEC, bool NT = false>
__device__ __forceinline__ void store_nodes(S* __restrict__ base, long long plane, int nx, int r, int c,
                                            const S (&in)[P::NF][VEC]) {
  if constexpr (P::kInterleaved) {
    S tmp[2 * VEC];
#pragma unroll
    for (int e = 0; e < VEC; ++e) {
      tmp[2 * e] = in[0][e];
      tmp[2 * e + 1] = in[1][e];
    }
    if constexpr (NT)
      store_vec_nt<S, 2 * VEC>(base + 2 * ((long long)r * nx + c), tmp);
    else
      store_vec<S, 2 * VEC>(base + 2 * ((long long)r * nx + c), tmp);
  } else {
#pragma unroll
    for (int f = 0; f < P::NF; ++f) {
      if constexpr (NT)
        store_vec_nt<S, VEC>(base + f * plane + (long long)r * nx + c, in[f]);
      else
        store_vec<S, VEC>(base + f * plane + (long long)r * nx + c, in[f]);
    }
  }
}

// Rows [r0-1, r0+RY] (2D) or the single row (1D) of one array for one thread,
// plus the left/right halo of every centre row.
template <class P, class T, int VEC, int RY>
struct Tile {
  static constexpr int NR = P::kDim2 ? RY + 2 : 1;
  static constexpr int RC = P::kDim2 ? RY : 1;
  // rows with left/right halo words: the centre rows, or every loaded row
  // when the operator reaches the diagonal neighbours
  static constexpr int RH = P::kCorners ? NR : RC;
  T a[P::NF][NR][VEC];
  T lh[P::NF][RH];
  T rh[P::NF][RH];

  // loaded row of halo row hh, and halo row of loaded row t
  static __device__ __forceinline__ int halo_row(int hh) { return P::kCorners ? hh : (P::kDim2 ? hh + 1 : 0); }

  // Issue the loads: rows r0-1 .. r0+RY, and the left/right halo words of
  // lanes at a wavefront or grid edge (the rest come from exchange()).
  template <class S>
  __device__ __forceinline__ void load(const S* __restrict__ base, long long plane, int nx, int ny, int r0,
                                       int col0, int cc, int lane) {
#pragma unroll
    for (int t = 0; t < NR; ++t) {
      const int r = P::kDim2 ? wrap_idx<periodic_rows<P>::value>(r0 - 1 + t, ny) : 0;
      S tmp[P::NF][VEC];
      load_nodes<P, S, VEC>(base, plane, nx, r, cc, tmp);
#pragma unroll
      for (int f = 0; f < P::NF; ++f)
#pragma unroll
        for (int e = 0; e < VEC; ++e) a[f][t][e] = to_c<T>(tmp[f][e]);
    }
    const int cl = wrap_idx<P::kPeriodic>(col0 - 1, nx);
    const int cr = wrap_idx<P::kPeriodic>(col0 + VEC, nx);
    const bool need_l = (lane == 0) || (col0 == 0);
    const bool need_r = (lane == kWave - 1) || (col0 + VEC >= nx);
#pragma unroll
    for (int hh = 0; hh < RH; ++hh) {
      const int r = P::kDim2 ? wrap_idx<periodic_rows<P>::value>(r0 - 1 + halo_row(hh), ny) : 0;
#pragma unroll
      for (int f = 0; f < P::NF; ++f) {
        lh[f][hh] = need_l ? to_c<T>(load_node<P, S>(base, plane, nx, r, cl, f)) : T(0);
        rh[f][hh] = need_r ? to_c<T>(load_node<P, S>(base, plane, nx, r, cr, f)) : T(0);
      }
    }
  }

  // Left/right neighbours of the other lanes from the adjacent lane.
  __device__ __forceinline__ void exchange(int col0, int nx, int lane) {
    const bool need_l = (lane == 0) || (col0 == 0);
    const bool need_r = (lane == kWave - 1) || (col0 + VEC >= nx);
#pragma unroll
    for (int hh = 0; hh < RH; ++hh) {
      const int t = halo_row(hh);
#pragma unroll
      for (int f = 0; f < P::NF; ++f) {
        const T lv = __shfl_up(a[f][t][VEC - 1], 1, kWave);
        const T rv = __shfl_down(a[f][t][0], 1, kWave);
        if (!need_l) lh[f][hh] = lv;
        if (!need_r) rh[f][hh] = rv;
      }
    }
  }

  __device__ __forceinline__ void scale_by(T s) {
#pragma unroll
    for (int f = 0; f < P::NF; ++f) {
#pragma unroll
      for (int t = 0; t < NR; ++t)
#pragma unroll
        for (int e = 0; e < VEC; ++e) a[f][t][e] *= s;
#pragma unroll
      for (int hh = 0; hh < RH; ++hh) {
        lh[f][hh] *= s;
        rh[f][hh] *= s;
      }
    }
  }

  __device__ __forceinline__ void nbr(int tt, int e, Nbr<T> (&o)[P::NF]) const {
    const int t = P::kDim2 ? tt + 1 : 0;
    const int hc = P::kCorners ? t : tt;  // halo row of loaded row t
#pragma unroll
    for (int f = 0; f < P::NF; ++f) {
      o[f].c = a[f][t][e];
      o[f].l = e > 0 ? a[f][t][e - 1] : lh[f][hc];
      o[f].r = e < VEC - 1 ? a[f][t][e + 1] : rh[f][hc];
      o[f].d = P::kDim2 ? a[f][t - 1][e] : a[f][t][e];
      o[f].u = P::kDim2 ? a[f][t + 1][e] : a[f][t][e];
      if constexpr (P::kCorners) {
        o[f].dl = e > 0 ? a[f][t - 1][e - 1] : lh[f][t - 1];
        o[f].dr = e < VEC - 1 ? a[f][t - 1][e + 1] : rh[f][t - 1];
        o[f].ul = e > 0 ? a[f][t + 1][e - 1] : lh[f][t + 1];
        o[f].ur = e < VEC - 1 ? a[f][t + 1][e + 1] : rh[f][t + 1];
      }
    }
  }
};

// Right preconditioning of a loaded tangent tile: every value, halo words
// included, becomes M^{-1} v at its node, with M frozen at the state values
// loaded at the same place (identity on boundary nodes).  Row and column of
// each word are those its load used (clamped at the non-periodic edges).
template <class P, class T, int VEC, int RY, class KT>
__device__ __forceinline__ void precondition_tile(const KT& k, const Tile<P, T, VEC, RY>& X, Tile<P, T, VEC, RY>& V,
                                                  int col0, int r0, int nx, int ny) {
  using TileT = Tile<P, T, VEC, RY>;
  constexpr int NF = P::NF;
  auto node = [&](int c, int r, auto get_x, auto get_v, auto set_v) {
    if (P::boundary(c, r, nx, ny)) return;
    T xv[NF], vv[NF];
#pragma unroll
    for (int f = 0; f < NF; ++f) {
      xv[f] = get_x(f);
      vv[f] = get_v(f);
    }
    P::template cslp_inv<T>(k, xv, vv);
#pragma unroll
    for (int f = 0; f < NF; ++f) set_v(f, vv[f]);
  };
#pragma unroll
  for (int t = 0; t < TileT::NR; ++t) {
    const int r = P::kDim2 ? wrap_idx<periodic_rows<P>::value>(r0 - 1 + t, ny) : 0;
#pragma unroll
    for (int e = 0; e < VEC; ++e)
      node(col0 + e, r, [&](int f) { return X.a[f][t][e]; }, [&](int f) { return V.a[f][t][e]; },
           [&](int f, T y) { V.a[f][t][e] = y; });
  }
  const int cl = wrap_idx<P::kPeriodic>(col0 - 1, nx);
  const int cr = wrap_idx<P::kPeriodic>(col0 + VEC, nx);
#pragma unroll
  for (int hh = 0; hh < TileT::RH; ++hh) {
    const int r = P::kDim2 ? wrap_idx<periodic_rows<P>::value>(r0 - 1 + TileT::halo_row(hh), ny) : 0;
    node(cl, r, [&](int f) { return X.lh[f][hh]; }, [&](int f) { return V.lh[f][hh]; },
         [&](int f, T y) { V.lh[f][hh] = y; });
    node(cr, r, [&](int f) { return X.rh[f][hh]; }, [&](int f) { return V.rh[f][hh]; },
         [&](int f, T y) { V.rh[f][hh] = y; });
  }
}

// dx = M^{-1} z in place (the update of right-preconditioned GMRES), one
// node per thread, grid-stride; SoA planes or interleaved pairs, as the
// operator stores them.
template <class P, class T>
__global__ void __launch_bounds__(256) cslp_apply_kernel(const T* __restrict__ x, T* __restrict__ z, int nx, int ny,
                                                          long long plane, const Coefs coefs) {
  const auto k = P::template make<T>(coefs);
  const long long step = (long long)gridDim.x * blockDim.x;
  for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < plane; i += step) {
    const int c = (int)(i % nx);
    const int r = (int)(i / nx);
    if (P::boundary(c, r, nx, ny)) continue;
    T xv[P::NF], vv[P::NF];
#pragma unroll
    for (int f = 0; f < P::NF; ++f) {
      const long long o = P::kInterleaved ? P::NF * i + f : f * plane + i;
      xv[f] = x[o];
      vv[f] = z[o];
    }
    P::template cslp_inv<T>(k, xv, vv);
#pragma unroll
    for (int f = 0; f < P::NF; ++f) z[P::kInterleaved ? P::NF * i + f : f * plane + i] = vv[f];
  }
}

// First CGS projection of an Arnoldi JVP's outputs on the stored basis:
// Loads the rows `rows` (column cc) of basis vectors q0 .. q0+G-1 into vq;
// slots at or beyond K reload vector K-1 (their products are discarded).
template <class P, class T, class VT, int VEC, int R, int G>
__device__ __forceinline__ void project_load(const StencilArgs<T, VT>& a, int nx, int cc, const int (&rows)[R],
                                             int q0, VT (&vq)[G][R][P::NF][VEC]) {
  if (a.nt_basis) {
#pragma unroll
    for (int u = 0; u < G; ++u) {
      const int q = q0 + u < a.K ? q0 + u : a.K - 1;
#pragma unroll
      for (int tt = 0; tt < R; ++tt) load_nodes_nt<P, VT, VEC>(a.Vb + q * a.vstride, a.plane, nx, rows[tt], cc, vq[u][tt]);
    }
  } else {
#pragma unroll
    for (int u = 0; u < G; ++u) {
      const int q = q0 + u < a.K ? q0 + u : a.K - 1;
#pragma unroll
      for (int tt = 0; tt < R; ++tt) load_nodes<P, VT, VEC>(a.Vb + q * a.vstride, a.plane, nx, rows[tt], cc, vq[u][tt]);
    }
  }
}

// acc[q0 + u] += V_{q0+u} . o for the G loaded vectors (u with q0 + u < K).
template <class P, class T, class VT, int VEC, int R, int G, int KDOT>
__device__ __forceinline__ void project_accumulate(const StencilArgs<T, VT>& a, int q0,
                                                   const VT (&vq)[G][R][P::NF][VEC], const T (&o)[R][P::NF][VEC],
                                                   double (&acc)[KDOT + 1]) {
  constexpr int NF = P::NF;
#pragma unroll
  for (int u = 0; u < G; ++u) {
    double sum;
    if constexpr (sizeof(T) == 4) {
      // FP32 sum over the thread's chunk, FP64 across chunks (as in the update pass)
      T p = T(0);
#pragma unroll
      for (int tt = 0; tt < R; ++tt)
#pragma unroll
        for (int f = 0; f < NF; ++f)
#pragma unroll
          for (int e = 0; e < VEC; ++e) p = fmaf(to_c<T>(vq[u][tt][f][e]), o[tt][f][e], p);
      sum = (double)p;
    } else {
      sum = 0.0;
#pragma unroll
      for (int tt = 0; tt < R; ++tt)
#pragma unroll
        for (int f = 0; f < NF; ++f)
#pragma unroll
          for (int e = 0; e < VEC; ++e) sum += (double)to_c<T>(vq[u][tt][f][e]) * (double)o[tt][f][e];
    }
    if (q0 + u < KDOT) acc[q0 + u] += q0 + u < a.K ? sum : 0.0;
  }
}

// acc[q] += V_q . o over the R rows `rows` (column cc) of this thread, for
// q < a.K, starting at vector Q0.  The rows of G basis vectors are loaded
// together before any is used (G chosen for about 256 bytes in flight per
// lane; a load-use pair per vector and row would leave the pass waiting on one
// memory round trip after another).
template <class P, class T, class VT, int VEC, int R, int G, int KDOT, int Q0 = 0>
__device__ __forceinline__ void project_rows(const StencilArgs<T, VT>& a, int nx, int cc, const int (&rows)[R],
                                             const T (&o)[R][P::NF][VEC], double (&acc)[KDOT + 1]) {
#pragma unroll
  for (int qb = Q0; qb < KDOT; qb += G) {
    if (qb < a.K) {
      VT vq[G][R][P::NF][VEC];
      project_load<P, T, VT, VEC, R, G>(a, nx, cc, rows, qb, vq);
      project_accumulate<P, T, VT, VEC, R, G, KDOT>(a, qb, vq, o, acc);
    }
  }
}

// Persistent launch: the grid holds at most a bounded number of blocks and
// each block walks a contiguous range of tiles (vertically adjacent row
// bands, so the halo rows of one tile are still in cache for the next).  A
// tile is blockDim.x * VEC columns by blockDim.y * RY rows.
template <class P, class T, class VT, int VEC, int RY, int OP, bool WITHF, int KDOT>
__global__ void __launch_bounds__(256)
stencil_kernel(const StencilArgs<T, VT> a, const Coefs coefs) {
  constexpr int NF = P::NF;
  constexpr int RC = P::kDim2 ? RY : 1;
  const auto k = P::template make<T>(coefs);
  const int nx = a.nx, ny = a.ny;
  const int lane = threadIdx.x & (kWave - 1);
  const T alpha = T(a.alpha), cN = T(a.cN), beta = T(a.beta);

  // this block's tiles
  const int tcols = (nx + VEC - 1) / VEC;
  const int tiles_x = (tcols + blockDim.x - 1) / blockDim.x;
  const int band = P::kDim2 ? blockDim.y * RY : 1;
  const int tiles_y = P::kDim2 ? (ny + band - 1) / band : 1;
  const int ntiles = tiles_x * tiles_y;
  const int per = (ntiles + gridDim.x - 1) / gridDim.x;
  const int t_begin = blockIdx.x * per;
  const int t_end = min(ntiles, t_begin + per);

  auto tile_origin = [&](int t, int& col0, int& r0) {
    const int tx = t % tiles_x;
    const int ty = t / tiles_x;
    col0 = (tx * blockDim.x + threadIdx.x) * VEC;
    r0 = P::kDim2 ? (ty * blockDim.y + threadIdx.y) * RY : 0;
  };

  Tile<P, T, VEC, RY> X;
  Tile<P, T, VEC, RY> Vt;
  int col0 = 0, r0 = 0;
  // the pointwise term b of the centre rows (zero when absent), loaded with
  // the tile so that its latency overlaps the exchange; the AD tangent alone
  // does not involve it
  constexpr bool kNeedB = OP != OP_AD || WITHF;
  // early only while the rows fit 64 bytes per lane (operators with four
  // fields and corner halos load them row by row, as their registers are full)
  constexpr bool kEarlyB = RC * NF * VEC * (int)sizeof(T) <= 64;
  T bval[kEarlyB ? RC : 1][NF][VEC];
  const bool use_b = kNeedB && a.b != nullptr;
  // Arnoldi JVP: the projection on the basis covers all of the thread's rows
  // at once when their outputs fit 64 bytes per lane (kept in po), else it
  // runs row by row; kProjGroup basis vectors' loads go out together
  constexpr bool kProjAll = RC * NF * VEC * (int)sizeof(T) <= 64;
  constexpr int PR = kProjAll ? RC : 1;
  constexpr int kProjBytes = PR * NF * VEC * (int)sizeof(VT);
  constexpr int kProjGroup0 = 256 / kProjBytes < 1 ? 1 : (256 / kProjBytes > 8 ? 8 : 256 / kProjBytes);
  constexpr int kProjGroup = KDOT > 0 && kProjGroup0 > KDOT ? KDOT : kProjGroup0;
  T po[KDOT > 0 ? PR : 1][NF][VEC];
  int prow[KDOT > 0 ? PR : 1];
  // the first tile's first group of basis rows is loaded right after the
  // tile (it needs only the tile's position), so that its round trip
  // overlaps the stencil arithmetic instead of following it; while all rows
  // are projected at once and the group fits 64 registers per lane
  // (FP16 basis values take a register each: the group is cut to fit)
  constexpr int kPreVecRegs = PR * NF * VEC * ((int)sizeof(VT) >= 4 ? (int)sizeof(VT) / 4 : 1);
  constexpr int kPreGroup = 64 / kPreVecRegs < kProjGroup ? 64 / kPreVecRegs : kProjGroup;
  constexpr bool kPre = OP != OP_RES && KDOT > 0 && KDOT <= 16 && kProjAll && kPreGroup >= 1;
  VT vpre[kPre ? kPreGroup : 1][kPre ? PR : 1][NF][VEC];
  // Arnoldi JVP of the delayed form: the loads of the column completion in
  // the prologue go out first, then the first tile's (in-bounds either way;
  // unused if the cycle has stopped), so that the two sets of round trips
  // overlap (vector loads complete in order: issued after the tile, the
  // prologue's loads would wait for all of it).
  // The stop state and the first step's tangent scale are read here too: a
  // control-block read issued after the tile's loads would wait for them.
  LaggedPrefetch lpf;
  [[maybe_unused]] int prev_state = kRunning;
  [[maybe_unused]] double vscale0 = 1.0;
  if constexpr (OP != OP_RES && KDOT > 0) {
    if (a.ctl != nullptr) {
      const int j = a.arn_j;
      prev_state = a.ctl->done_col[j > 0 ? j - 1 : 0];
      if (j == 0) vscale0 = a.ctl->scale[0];
      if (a.lagged && j > 0) lagged_prefetch<is_half<VT>()>(a.ctl, j - 1, a.pc, lpf);
    }
  }
  if (t_begin < t_end) {
    tile_origin(t_begin, col0, r0);
    const int cc = col0 < nx ? col0 : 0;
    X.load(a.x, a.plane, nx, ny, r0, col0, cc, lane);
    if constexpr (OP != OP_RES) Vt.load(a.v, a.plane, nx, ny, r0, col0, cc, lane);
    if constexpr (kEarlyB) load_b_rows<P, T, VEC, RC>(a.b, a.plane, nx, ny, r0, cc, use_b, bval);
    if constexpr (kPre) {
      if (a.Vb != nullptr) {
        int rows[PR];
#pragma unroll
        for (int tt = 0; tt < PR; ++tt) {
          const int r = r0 + tt;
          rows[tt] = P::kDim2 ? (r < ny ? r : 0) : 0;
        }
        project_load<P, T, VT, VEC, PR, kPreGroup>(a, nx, cc, rows, 0, vpre);
      }
    }
  }

  // Arnoldi mode (only instances with the fused projection, KDOT > 0): leave
  // at once if the cycle has already stopped
  if constexpr (OP != OP_RES && KDOT > 0) {
    if (a.ctl != nullptr) {
      const int j = a.arn_j;
      const int prev = prev_state;
      if (prev != kRunning) {
        // carry the state forward so that the flags stay monotone (later
        // kernels only look at the state after their own column)
        if (j > 0 && blockIdx.x == 0 && threadIdx.x == 0 && threadIdx.y == 0) {
          a.ctl->done_col[j] = prev;
          if (a.host_flags) a.host_flags[j - 1] = prev;
        }
        return;
      }
    }
  }

  if constexpr (OP != OP_RES) {
    if (a.gate != nullptr) {
      if (*a.gate != kRunning) return;
      if (a.gate_parts.nb > 0) {
        __shared__ double gsum[1];
        reduce_partials(a.gate_parts, 1, gsum);
        if (!(sqrt(gsum[0]) > *a.gate_tol)) return;  // uniform across the block
      }
    }
  }

  double vscale = 1.0;
  if constexpr (OP != OP_RES) {
    bool arnoldi = false;
    if constexpr (KDOT > 0) {
      if (a.ctl != nullptr) {
        arnoldi = true;
        const int j = a.arn_j;
        if (j == 0) {
          vscale = vscale0;
        } else {
          __shared__ double gcol[kMaxM + 1];
          const GivensOut g = a.lagged ? finish_column_lagged_from<is_half<VT>()>(a.ctl, j - 1, a.pc, a.host_flags,
                                                                                  gcol, lpf)
                                       : finish_column(a.ctl, j - 1, a.pc, a.host_flags, gcol);
          if (g.done != kRunning) return;  // uniform: every block computed the same update
          vscale = g.vs;
        }
      }
    }
    if (!arnoldi && a.vscale != nullptr) vscale = *a.vscale;
  }
  double eps = 0.0;
  T eps_s = T(0);
  if constexpr (OP == OP_FD) {
    double vn2 = -1.0;
    if (a.eps.vparts.nb > 0) {
      __shared__ double tot[1];
      reduce_partials(a.eps.vparts, 1, tot);
      vn2 = tot[0];
    }
    eps = fd_eps(a.eps, vn2);
    eps_s = T(eps * vscale);
  }
  // the quotient by eps as a product with its reciprocal (formed once, in
  // FP64): within one rounding of the division, far inside the FD JVP's
  // rounding bound of a few u S / eps
  const T inv_eps = T(OP == OP_FD ? 1.0 / eps : 0.0);
  const T vs_t = T(vscale);

  constexpr int NACC = OP == OP_RES ? 2 : (KDOT > 0 ? KDOT + 1 : 1);
  double acc[NACC];
#pragma unroll
  for (int q = 0; q < NACC; ++q) acc[q] = 0.0;


  // one tile whose loads have been issued (X, Vt at col0, r0)
  auto process = [&](bool pre) {
    const bool colok = col0 < nx;
    const int cc = colok ? col0 : 0;
    const int pcc = cc;
    X.exchange(col0, nx, lane);
    if constexpr (OP != OP_RES) {
      Vt.exchange(col0, nx, lane);
      if constexpr (OP == OP_AD) {
        if (vscale != 1.0) Vt.scale_by(vs_t);
      }
      if constexpr (precond_tangent<P>::value) precondition_tile<P, T, VEC, RY>(k, X, Vt, col0, r0, nx, ny);
    }

#pragma unroll
    for (int tt = 0; tt < RC; ++tt) {
      const int r = r0 + tt;
      const bool ok = colok && (!P::kDim2 || r < ny);
      const int rr = P::kDim2 ? (r < ny ? r : 0) : 0;
      T brow[NF][VEC];
      if constexpr (kEarlyB) {
#pragma unroll
        for (int f = 0; f < NF; ++f)
#pragma unroll
          for (int e = 0; e < VEC; ++e) brow[f][e] = bval[tt][f][e];
      } else {
#pragma unroll
        for (int f = 0; f < NF; ++f)
#pragma unroll
          for (int e = 0; e < VEC; ++e) brow[f][e] = T(0);
        if (use_b) load_nodes<P, T, VEC>(a.b, a.plane, nx, rr, cc, brow);
      }
      T o[NF][VEC];
      T o2[NF][VEC];
#pragma unroll
      for (int e = 0; e < VEC; ++e) {
        Nbr<T> xn[NF];
        X.nbr(tt, e, xn);
        const bool bnd = P::boundary(col0 + e, rr, nx, ny);
        if constexpr (OP == OP_RES) {
          T n[NF];
          P::template N<T, T>(k, xn, n);
#pragma unroll
          for (int f = 0; f < NF; ++f)
            o[f][e] = bnd ? xn[f].c : (alpha * xn[f].c + cN * n[f]) + beta * brow[f][e];
        } else if constexpr (OP == OP_AD) {
          Nbr<T> vn[NF];
          Vt.nbr(tt, e, vn);
          Nbr<dual<T>> dn[NF];
#pragma unroll
          for (int f = 0; f < NF; ++f) nbr_dual<P, T>(xn[f], vn[f], dn[f]);
          dual<T> n[NF];
          P::template N<T, dual<T>>(k, dn, n);
#pragma unroll
          for (int f = 0; f < NF; ++f) {
            o[f][e] = bnd ? vn[f].c : alpha * vn[f].c + cN * n[f].t;
            o2[f][e] = bnd ? xn[f].c : (alpha * xn[f].c + cN * n[f].v) + beta * brow[f][e];
          }
        } else {
          Nbr<T> vn[NF];
          Vt.nbr(tt, e, vn);
          Nbr<T> yn[NF];
#pragma unroll
          for (int f = 0; f < NF; ++f) nbr_axpy<P, T>(xn[f], eps_s, vn[f], yn[f]);
          T n0[NF], n1[NF];
          P::template N<T, T>(k, xn, n0);
          P::template N<T, T>(k, yn, n1);
#pragma unroll
          for (int f = 0; f < NF; ++f) {
            const T f0 = bnd ? xn[f].c : (alpha * xn[f].c + cN * n0[f]) + beta * brow[f][e];
            const T f1 = bnd ? yn[f].c : (alpha * yn[f].c + cN * n1[f]) + beta * brow[f][e];
            o[f][e] = (f1 - f0) * inv_eps;
          }
        }
      }
      if (ok) {
        // a standalone JVP's output streams to memory (measured 7-8% faster at
        // 25 MB per call); the Arnoldi JVP's output is read back by the next
        // pass at once and the residual's soon after, so those stay cached
        constexpr bool kNT = OP != OP_RES && KDOT == 0;
        store_nodes<P, T, VEC, kNT>(a.out, a.plane, nx, rr, cc, o);
        if constexpr (OP == OP_AD && WITHF) store_nodes<P, T, VEC, kNT>(a.out2, a.plane, nx, rr, cc, o2);
        if constexpr (OP == OP_RES) {
          const int t2 = P::kDim2 ? tt + 1 : 0;
#pragma unroll
          for (int f = 0; f < NF; ++f)
#pragma unroll
            for (int e = 0; e < VEC; ++e) {
              acc[0] += (double)o[f][e] * (double)o[f][e];
              acc[1] += (double)X.a[f][t2][e] * (double)X.a[f][t2][e];
            }
        }
        if constexpr (OP != OP_RES && KDOT > 0) {
#pragma unroll
          for (int f = 0; f < NF; ++f)
#pragma unroll
            for (int e = 0; e < VEC; ++e) acc[KDOT] += (double)o[f][e] * (double)o[f][e];
        }
      }
      if constexpr (OP != OP_RES && KDOT > 0) {
        // keep the row (zero outside the grid) for the projection
        const int pt = kProjAll ? tt : 0;
        prow[pt] = rr;
#pragma unroll
        for (int f = 0; f < NF; ++f)
#pragma unroll
          for (int e = 0; e < VEC; ++e) po[pt][f][e] = ok ? o[f][e] : T(0);
        if constexpr (!kProjAll) project_rows<P, T, VT, VEC, 1, kProjGroup, KDOT>(a, nx, cc, prow, po, acc);
      }
    }
    if constexpr (OP != OP_RES && KDOT > 0 && kProjAll) {
      if constexpr (kPre) {
        if (pre) {
          project_accumulate<P, T, VT, VEC, RC, kPreGroup, KDOT>(a, 0, vpre, po, acc);
          project_rows<P, T, VT, VEC, RC, kProjGroup, KDOT, kPreGroup>(a, nx, pcc, prow, po, acc);
          return;
        }
      }
      project_rows<P, T, VT, VEC, RC, kProjGroup, KDOT>(a, nx, pcc, prow, po, acc);
    }
  };

  if (t_begin < t_end) process(true);
  for (int t = t_begin + 1; t < t_end; ++t) {
    tile_origin(t, col0, r0);
    const int cc = col0 < nx ? col0 : 0;
    X.load(a.x, a.plane, nx, ny, r0, col0, cc, lane);
    if constexpr (OP != OP_RES) Vt.load(a.v, a.plane, nx, ny, r0, col0, cc, lane);
    if constexpr (kEarlyB) load_b_rows<P, T, VEC, RC>(a.b, a.plane, nx, ny, r0, cc, use_b, bval);
    process(false);
  }

  if constexpr (OP == OP_RES) {
    if (a.nred > 0) {
      __shared__ double lds[2 * 4];
      block_partials<2>(acc, a.nred, a.part_out.part, a.part_out.ld, lds);
    }
  } else if constexpr (KDOT > 0) {
    // ||Jv||^2 next to the K projections (static indices keep acc in registers)
#pragma unroll
    for (int q = 0; q < KDOT; ++q)
      if (q == a.K) acc[q] = acc[KDOT];
    __shared__ double lds[(KDOT + 1) * 4];
    block_partials<KDOT + 1>(acc, a.K + 1, a.dots_out.part, a.dots_out.ld, lds);
  }
}

}  // namespace jfnk
