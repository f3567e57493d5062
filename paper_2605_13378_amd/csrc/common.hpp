// Device-side building blocks shared by the JFNK kernels (gfx950, wave64).
//
//  * dual<T>: value + tangent pair; arithmetic applies the sum and product
//    rules, so a residual written once over a scalar type S yields F(x) for
//    S = T and (F(x), J(x) v) for S = dual<T> (forward-mode AD JVP).
//  * vec<T, N>: aligned vector of N elements for 8/16-byte global accesses.
//  * wave_sum / block_partials / reduce_partials: deterministic reductions in
//    FP64.  A block sums its wavefronts in fixed order and writes one row of
//    partials; the next kernel adds the rows in fixed order.
//  * Ctl: the GMRES control block that lives in device memory, so Arnoldi
//    kernels read their coefficients and flags without any host round trip.
#pragma once

#include <hip/hip_runtime.h>
#include <hip/hip_fp16.h>
#include <stdint.h>

namespace jfnk {

constexpr int kMaxM = 32;     // largest GMRES restart length
constexpr int kWave = 64;     // CDNA wavefront width

// ---------------------------------------------------------------------------
// dual numbers
// ---------------------------------------------------------------------------
template <class T>
struct dual {
  T v, t;
};

template <class T> __device__ __forceinline__ dual<T> operator+(dual<T> a, dual<T> b) { return {a.v + b.v, a.t + b.t}; }
template <class T> __device__ __forceinline__ dual<T> operator-(dual<T> a, dual<T> b) { return {a.v - b.v, a.t - b.t}; }
template <class T> __device__ __forceinline__ dual<T> operator-(dual<T> a) { return {-a.v, -a.t}; }
template <class T> __device__ __forceinline__ dual<T> operator*(dual<T> a, dual<T> b) { return {a.v * b.v, a.v * b.t + a.t * b.v}; }
template <class T> __device__ __forceinline__ dual<T> operator*(T c, dual<T> a) { return {c * a.v, c * a.t}; }
template <class T> __device__ __forceinline__ dual<T> operator*(dual<T> a, T c) { return {a.v * c, a.t * c}; }
template <class T> __device__ __forceinline__ dual<T> operator+(dual<T> a, T c) { return {a.v + c, a.t}; }
template <class T> __device__ __forceinline__ dual<T> operator+(T c, dual<T> a) { return {c + a.v, a.t}; }
template <class T> __device__ __forceinline__ dual<T> operator-(dual<T> a, T c) { return {a.v - c, a.t}; }
template <class T> __device__ __forceinline__ dual<T> operator-(T c, dual<T> a) { return {c - a.v, -a.t}; }

// ---------------------------------------------------------------------------
// vector memory access
// ---------------------------------------------------------------------------
template <class T, int N>
struct alignas(sizeof(T) * N) vec {
  T a[N];
};

template <class T, int N>
__device__ __forceinline__ void load_vec(const T* __restrict__ p, T (&out)[N]) {
  const vec<T, N> t = *reinterpret_cast<const vec<T, N>*>(p);
#pragma unroll
  for (int e = 0; e < N; ++e) out[e] = t.a[e];
}

template <class T, int N>
__device__ __forceinline__ void store_vec(T* __restrict__ p, const T (&in)[N]) {
  vec<T, N> t;
#pragma unroll
  for (int e = 0; e < N; ++e) t.a[e] = in[e];
  *reinterpret_cast<vec<T, N>*>(p) = t;
}

// Load with a non-temporal hint, for streams read once per pass (the Krylov
// basis): on MI355X such loads stream from HBM without being kept in the
// last-level cache, where a basis larger than that cache would only evict
// the small vectors that are reused (multi-stream read microbenchmark, 16
// streams of 8 MB: 5.3 TB/s with ordinary loads, 5.9 TB/s with the hint).
template <class T, int N>
__device__ __forceinline__ void load_vec_nt(const T* __restrict__ p, T (&out)[N]) {
  constexpr int B = (int)sizeof(T) * N;
  static_assert(B == 2 || B == 4 || B == 8 || B == 16, "vector access of 2, 4, 8 or 16 bytes");
  vec<T, N> t;
  if constexpr (B == 2) {
    const unsigned short u = __builtin_nontemporal_load(reinterpret_cast<const unsigned short*>(p));
    __builtin_memcpy(&t, &u, B);
  } else if constexpr (B == 4) {
    const unsigned int u = __builtin_nontemporal_load(reinterpret_cast<const unsigned int*>(p));
    __builtin_memcpy(&t, &u, B);
  } else {
    typedef unsigned int uv __attribute__((ext_vector_type(B / 4)));
    const uv u = __builtin_nontemporal_load(reinterpret_cast<const uv*>(p));
    __builtin_memcpy(&t, &u, B);
  }
#pragma unroll
  for (int e = 0; e < N; ++e) out[e] = t.a[e];
}

// The same with a non-temporal hint: for outputs that no kernel of the same
// sequence reads back right away, so they stream to memory instead of
// displacing cached inputs.
template <class T, int N>
__device__ __forceinline__ void store_vec_nt(T* __restrict__ p, const T (&in)[N]) {
  if constexpr (N == 1) {
    __builtin_nontemporal_store(in[0], p);
  } else {
    typedef T vt __attribute__((ext_vector_type(N)));
    vt t;
#pragma unroll
    for (int e = 0; e < N; ++e) t[e] = in[e];
    __builtin_nontemporal_store(t, reinterpret_cast<vt*>(p));
  }
}

// storage <-> compute conversions (FP16 storage carries a power-of-two scale
// applied by the caller)
template <class C, class S> __device__ __forceinline__ C to_c(S x) { return static_cast<C>(x); }
template <> __device__ __forceinline__ float to_c<float, __half>(__half x) { return __half2float(x); }
template <class S, class C> __device__ __forceinline__ S to_s(C x) { return static_cast<S>(x); }
template <> __device__ __forceinline__ __half to_s<__half, float>(float x) { return __float2half_rn(x); }

// Two FP32 values rounded to FP16 (nearest even), packed low then high.
__device__ __forceinline__ unsigned int pack_half2(float lo, float hi) {
  return (unsigned int)__half_as_ushort(__float2half_rn(lo)) |
         ((unsigned int)__half_as_ushort(__float2half_rn(hi)) << 16);
}

// Dot product of N packed FP16 pairs, accumulated in FP32 (the products are
// exact), returned in FP64.
template <int N>
__device__ __forceinline__ double dot_half2(const unsigned int (&a)[N], const unsigned int (&b)[N]) {
  typedef _Float16 h2 __attribute__((ext_vector_type(2)));
  float p = 0.0f;
#pragma unroll
  for (int q = 0; q < N; ++q) p = __builtin_amdgcn_fdot2(__builtin_bit_cast(h2, a[q]), __builtin_bit_cast(h2, b[q]), p, false);
  return (double)p;
}

// a * (FP16 element `hi` of the packed pair h2, widened) + c in one fused
// operation.  The compiler forms this instruction itself for a widened FP16
// operand with a single use; written out where one element feeds two sums,
// which the compiler would otherwise serve from a register per widened
// element.  `hi` must be a compile-time constant.
__device__ __forceinline__ float fma_mix_half(float a, unsigned int h2, int hi, float c) {
  float d;
  if (hi)
    asm("v_fma_mix_f32 %0, %1, %2, %3 op_sel:[0,1,0] op_sel_hi:[0,1,0]" : "=v"(d) : "s"(a), "v"(h2), "v"(c));
  else
    asm("v_fma_mix_f32 %0, %1, %2, %3 op_sel_hi:[0,1,0]" : "=v"(d) : "s"(a), "v"(h2), "v"(c));
  return d;
}

template <class VT> constexpr bool is_half() { return false; }
template <> constexpr bool is_half<__half>() { return true; }

// Power-of-two storage scale for an FP16 basis vector of n entries and 2-norm
// `norm`: typical entries |w_i| ~ norm / sqrt(n) are mapped near 1, far from
// FP16's overflow (65504) and subnormal (6.1e-5) limits.
__device__ __forceinline__ double fp16_scale(double norm, long long n) {
  if (!(norm > 0.0) || !isfinite(norm)) return 1.0;
  const double typical = norm / sqrt((double)n);
  return exp2(-rint(log2(typical)));
}

// Wave-uniform values moved to scalar registers (the coefficients of the
// Krylov updates), freeing vector registers for the register-resident basis.
__device__ __forceinline__ float uniform(float x) {
  return __int_as_float(__builtin_amdgcn_readfirstlane(__float_as_int(x)));
}
__device__ __forceinline__ double uniform(double x) {
  const long long u = __double_as_longlong(x);
  const int lo = __builtin_amdgcn_readfirstlane((int)(u & 0xffffffffLL));
  const int hi = __builtin_amdgcn_readfirstlane((int)(u >> 32));
  return __longlong_as_double(((long long)hi << 32) | (long long)(unsigned)lo);
}

// ---------------------------------------------------------------------------
// reductions
// ---------------------------------------------------------------------------
// Cross-lane moves of an FP64 value by DPP (data-parallel primitives: the
// lane exchange happens inside a VALU instruction, no LDS round trip), as
// two 32-bit halves.  CTRL is the DPP control word: quad_perm [1,0,3,2] =
// 0xB1, [2,3,0,1] = 0x4E, row_half_mirror = 0x141, row_mirror = 0x140.
template <int CTRL>
__device__ __forceinline__ double dpp_f64(double v) {
  const long long u = __double_as_longlong(v);
  const int lo = __builtin_amdgcn_update_dpp(0, (int)(u & 0xffffffffLL), CTRL, 0xF, 0xF, false);
  const int hi = __builtin_amdgcn_update_dpp(0, (int)(u >> 32), CTRL, 0xF, 0xF, false);
  return __longlong_as_double(((long long)hi << 32) | (long long)(unsigned)lo);
}

// v + (v of the lane 16 or 32 away across rows): gfx950's permlane swaps
// exchange odd and even rows (16) or the two wavefront halves (32) between
// two registers; swapping a value with itself leaves (own, partner) in the
// pair, so both partners form the same sum.
template <int D>
__device__ __forceinline__ double swap_add_f64(double v) {
  const long long u = __double_as_longlong(v);
  const unsigned lo = (unsigned)(u & 0xffffffffLL), hi = (unsigned)(u >> 32);
  unsigned l0, l1, h0, h1;
  if constexpr (D == 16) {
    const auto a = __builtin_amdgcn_permlane16_swap(lo, lo, false, false);
    const auto b = __builtin_amdgcn_permlane16_swap(hi, hi, false, false);
    l0 = a[0]; l1 = a[1]; h0 = b[0]; h1 = b[1];
  } else {
    const auto a = __builtin_amdgcn_permlane32_swap(lo, lo, false, false);
    const auto b = __builtin_amdgcn_permlane32_swap(hi, hi, false, false);
    l0 = a[0]; l1 = a[1]; h0 = b[0]; h1 = b[1];
  }
  return __longlong_as_double(((long long)h0 << 32) | (long long)l0) +
         __longlong_as_double(((long long)h1 << 32) | (long long)l1);
}

// Sum over aligned groups of G consecutive lanes (G a power of two up to 64);
// every lane of a group returns its group's sum.  Within a row of 16 lanes
// the partners come from DPP moves (pairs, quads, half rows, rows, each step
// combining two halves whose lanes already agree), across rows from the
// permlane swaps: register-to-register exchanges, no LDS round trip.  Fixed
// order: the result does not depend on timing.
template <int G>
__device__ __forceinline__ double group_sum(double v) {
  if constexpr (G >= 2) v += dpp_f64<0xB1>(v);
  if constexpr (G >= 4) v += dpp_f64<0x4E>(v);
  if constexpr (G >= 8) v += dpp_f64<0x141>(v);
  if constexpr (G >= 16) v += dpp_f64<0x140>(v);
  if constexpr (G >= 32) v = swap_add_f64<16>(v);
  if constexpr (G >= 64) v = swap_add_f64<32>(v);
  return v;
}

__device__ __forceinline__ double wave_sum(double v) { return group_sum<kWave>(v); }

// One halving step of a transposed wavefront sum: the lanes whose bit D of
// the lane id is 0 keep the lower half of the M values (x = v[i], i < M/2),
// the others the upper half (y = v[i + M/2]), each adding its partner's
// copy of the half it keeps.  D = 32 and 16 use the permlane swaps, which
// exchange x of one side for y of the other, so vdst + vsrc after the swap
// is the kept half's pair sum on either side; smaller D use DPP moves of the
// half the lane gives away.
template <int D>
__device__ __forceinline__ double halve_step(double x, double y, int lane) {
  if constexpr (D == 32 || D == 16) {
    const long long ux = __double_as_longlong(x), uy = __double_as_longlong(y);
    const unsigned xl = (unsigned)(ux & 0xffffffffLL), xh = (unsigned)(ux >> 32);
    const unsigned yl = (unsigned)(uy & 0xffffffffLL), yh = (unsigned)(uy >> 32);
    unsigned l0, l1, h0, h1;
    if constexpr (D == 32) {
      const auto a = __builtin_amdgcn_permlane32_swap(xl, yl, false, false);
      const auto b = __builtin_amdgcn_permlane32_swap(xh, yh, false, false);
      l0 = a[0]; l1 = a[1]; h0 = b[0]; h1 = b[1];
    } else {
      const auto a = __builtin_amdgcn_permlane16_swap(xl, yl, false, false);
      const auto b = __builtin_amdgcn_permlane16_swap(xh, yh, false, false);
      l0 = a[0]; l1 = a[1]; h0 = b[0]; h1 = b[1];
    }
    return __longlong_as_double(((long long)h0 << 32) | (long long)l0) +
           __longlong_as_double(((long long)h1 << 32) | (long long)l1);
  } else {
    // partners: D = 8 row mirror (i <-> 15 - i), 4 half-row mirror (i <-> 7 - i),
    // 2 and 1 lane xor within a quad; the partner's bit D is the opposite one
    constexpr int CTRL = D == 8 ? 0x140 : (D == 4 ? 0x141 : (D == 2 ? 0x4E : 0xB1));
    const bool low = (lane & D) == 0;
    const double give = low ? y : x;
    const double keep = low ? x : y;
    return keep + dpp_f64<CTRL>(give);
  }
}

// Lane i's copy of a 64-bit value (i uniform across the wavefront; every
// lane active).
__device__ __forceinline__ double lane_f64(double v, int i) {
  const long long u = __double_as_longlong(v);
  const unsigned lo = (unsigned)__builtin_amdgcn_readlane((int)(u & 0xffffffffLL), i);
  const unsigned hi = (unsigned)__builtin_amdgcn_readlane((int)(u >> 32), i);
  return __longlong_as_double((long long)(((unsigned long long)hi << 32) | lo));
}

// Sums of M values (a power of two, at most 32) over the 64 lanes of a
// wavefront, transposed: lane l returns the sum of value l >> (6 - log2 M).
// log2 M halving steps (M - 1 exchanges in all) and plain pair sums for the
// remaining lane bits, where M separate wavefront sums would take 6 M.
template <int M>
__device__ __forceinline__ double wave_sum_transposed(const double (&v)[M], int lane) {
  static_assert(M >= 1 && M <= 32 && (M & (M - 1)) == 0, "M: a power of two up to 32");
  double a[M];
#pragma unroll
  for (int i = 0; i < M; ++i) a[i] = v[i];
  int m = M;
  // halving on lane bits 5, 4, 3, ... (D = 32, 16, 8, ...) while values remain
#pragma unroll
  for (int s = 0; s < 6; ++s) {
    const int D = 32 >> s;
    if (m > 1) {
#pragma unroll
      for (int i = 0; i < M / 2; ++i) {
        if (i < m / 2) {
          switch (D) {
            case 32: a[i] = halve_step<32>(a[i], a[i + m / 2], lane); break;
            case 16: a[i] = halve_step<16>(a[i], a[i + m / 2], lane); break;
            case 8: a[i] = halve_step<8>(a[i], a[i + m / 2], lane); break;
            case 4: a[i] = halve_step<4>(a[i], a[i + m / 2], lane); break;
            case 2: a[i] = halve_step<2>(a[i], a[i + m / 2], lane); break;
            default: a[i] = halve_step<1>(a[i], a[i + m / 2], lane); break;
          }
        }
      }
      m /= 2;
    } else {
      // one value left: a plain pair sum over this lane bit
      switch (D) {
        case 32: a[0] = swap_add_f64<32>(a[0]); break;
        case 16: a[0] = swap_add_f64<16>(a[0]); break;
        case 8: a[0] += dpp_f64<0x140>(a[0]); break;
        case 4: a[0] += dpp_f64<0x141>(a[0]); break;
        case 2: a[0] += dpp_f64<0x4E>(a[0]); break;
        default: a[0] += dpp_f64<0xB1>(a[0]); break;
      }
    }
  }
  return a[0];
}

// group_sum for a group size known only at run time (uniform across the wavefront).
__device__ __forceinline__ double group_sum_rt(double v, int G) {
  switch (G) {
    case 64: return group_sum<64>(v);
    case 32: return group_sum<32>(v);
    case 16: return group_sum<16>(v);
    case 8: return group_sum<8>(v);
    case 4: return group_sum<4>(v);
    case 2: return group_sum<2>(v);
    default: return v;
  }
}

// Block partial sums.  A reducing kernel writes one FP64 partial sum per
// block and column; the next kernel in stream order adds them in its
// prologue (reduce_partials), every block alike and in the same order.  The
// kernel boundary makes the sums visible, so no kernel needs a grid-wide
// fence or atomic (on gfx950 a device-scope fence writes back and
// invalidates the whole L2), and results depend only on the launch shape,
// never on timing.  Storage is column-major: column c of block b at
// part[c * ld + b], so the lanes summing one column read consecutive words.
constexpr int kMaxCols = kMaxM + 1;

struct Partials {
  const double* part;
  int nb;  // rows (blocks of the producer); 0 = none
  int ld;  // column stride
};

// Destination of a producer's partial sums.
struct PartSink {
  double* part;
  int ld;
};

// Write this block's sums of acc[k], k < nr, to column k, row blockIdx.
// `lds` must hold NR * (threads / 64) doubles.  All threads must call it.
template <int NR>
__device__ __forceinline__ void block_partials(double (&acc)[NR], int nr, double* __restrict__ part, int ld,
                                               double* lds) {
  const int nthreads = blockDim.x * blockDim.y;
  const int tid = threadIdx.y * blockDim.x + threadIdx.x;
  const int lane = tid & (kWave - 1);
  const int wid = tid / kWave;
  const int nw = nthreads / kWave;
  const int bid = blockIdx.y * gridDim.x + blockIdx.x;
  // the first M values (M = NR rounded up to a power of two, at most 32) in
  // one transposed wavefront sum, any further ones one by one
  constexpr int M = NR <= 1 ? 1 : (NR <= 2 ? 2 : (NR <= 4 ? 4 : (NR <= 8 ? 8 : (NR <= 16 ? 16 : 32))));
  constexpr int SH = M == 1 ? 6 : (M == 2 ? 5 : (M == 4 ? 4 : (M == 8 ? 3 : (M == 16 ? 2 : 1))));
  double v[M];
#pragma unroll
  for (int k = 0; k < M; ++k) v[k] = k < NR ? acc[k < NR ? k : 0] : 0.0;
  const double t = wave_sum_transposed<M>(v, lane);
  const int c = lane >> SH;
  if ((lane & ((1 << SH) - 1)) == 0 && c < nr) lds[c * nw + wid] = t;
#pragma unroll
  for (int k = M; k < NR; ++k) {
    if (k < nr) {
      const double s = wave_sum(acc[k]);
      if (lane == 0) lds[k * nw + wid] = s;
    }
  }
  __syncthreads();
  if (tid < nr) {
    double s = 0.0;
    for (int w = 0; w < nw; ++w) s += lds[tid * nw + w];
    part[(size_t)tid * ld + bid] = s;
  }
}

// Column sums of the first nb rows for columns k < nr into `tot` (LDS),
// visible to the whole block on return, in two phases: partials_fetch issues
// each lane's first 16 loads into registers (a kernel can do this before its
// main loads, so that the round trips overlap), partials_reduce adds them,
// loads and adds any further rows, reduces within the lane groups and writes
// `tot`.  G lanes share a column (G a power of two, G * nr <= threads).
struct PartialFetch {
  static constexpr int CH = 16;
  double v[CH];
};

__device__ __forceinline__ int partials_group(int nr) {
  const int nthreads = blockDim.x * blockDim.y;
  int G = kWave;
  while (G > 1 && G * nr > nthreads) G >>= 1;
  return G;
}

__device__ __forceinline__ void partials_fetch(const Partials& p, int nr, PartialFetch& f) {
  constexpr int CH = PartialFetch::CH;
  const int tid = threadIdx.y * blockDim.x + threadIdx.x;
  const int G = partials_group(nr);
  const int col = tid / G;
  const int g = tid % G;
  if (col < nr) {
    const double* __restrict__ q = p.part + (size_t)col * p.ld;
#pragma unroll
    for (int r = 0; r < CH; ++r) {
      const int b = g + r * G;
      f.v[r] = b < p.nb ? q[b] : 0.0;
    }
  } else {
#pragma unroll
    for (int r = 0; r < CH; ++r) f.v[r] = 0.0;
  }
}

__device__ __forceinline__ void partials_reduce(const Partials& p, int nr, const PartialFetch& f, double* tot) {
  constexpr int CH = PartialFetch::CH;
  const int tid = threadIdx.y * blockDim.x + threadIdx.x;
  const int G = partials_group(nr);
  const int col = tid / G;
  const int g = tid % G;
  double s = 0.0;
#pragma unroll
  for (int r = 0; r < CH; ++r) s += f.v[r];
  if (col < nr) {
    const double* __restrict__ q = p.part + (size_t)col * p.ld;
    for (int b0 = g + G * CH; b0 < p.nb; b0 += G * CH) {
      double v[CH];
#pragma unroll
      for (int r = 0; r < CH; ++r) {
        const int b = b0 + r * G;
        v[r] = b < p.nb ? q[b] : 0.0;
      }
#pragma unroll
      for (int r = 0; r < CH; ++r) s += v[r];
    }
  }
  s = group_sum_rt(s, G);
  if (col < nr && g == 0) tot[col] = s;
  __syncthreads();
}

__device__ __forceinline__ void reduce_partials(const Partials& p, int nr, double* tot) {
  PartialFetch f;
  partials_fetch(p, nr, f);
  partials_reduce(p, nr, f, tot);
}

// ---------------------------------------------------------------------------
// GMRES / Newton control block (device resident)
// ---------------------------------------------------------------------------
enum : int {
  kRunning = 0,
  kConverged = 1,   // residual (true or estimated) below tolerance
  kBreakdown = 2,   // happy breakdown: ||w|| tiny against ||J v_j||
  kNonfinite = 3,   // NaN/Inf met
};

// Every field is written by exactly one kind of kernel and only read by
// later kernels in stream order: no kernel reads a field that another block
// of the same kernel may write.  done_col[0] is the state after the cycle
// start, done_col[c + 1] the state after the Givens rotation of column c.
struct Ctl {
  int k;             // Arnoldi columns completed in the current cycle (written by the V y kernel)
  int m;             // restart length of the current solve
  int first;         // 1 until the first cycle start has fixed ||rhs||
  int k_last;        // k of the last V y update (kept across the next cycle start)
  int k_last_state;  // stop state after that update's last column (kRunning if k_last == 0)
  int pad0;
  int done_col[kMaxM + 2];
  double bnorm;      // ||rhs||
  double tol;        // relative Krylov tolerance
  double tol_abs;    // tol * bnorm
  double brk_tol;    // happy-breakdown threshold (relative to ||J v_j||)
  double beta;       // ||r|| at the start of the current cycle
  double res_est;    // latest Givens residual estimate |g_{k}|
  double jvn2;       // ||J v_j||^2 of the current step (pass A, written by pass B)
  double fnorm2;     // ||F||^2 of the latest residual evaluation
  double xnorm2;     // ||x||^2 of the latest residual evaluation (must follow fnorm2)
  double dxnorm2;    // 1 / (FP16 storage scale) of a standalone JVP tangent (FP16S solvers)
  double aux2;       // ||v||^2 for standalone FD JVP calls
  double gp[kMaxM + 1];              // g entry j before rotation j (gp[0] = beta)
  double gr[kMaxM];                  // g entry j after rotation j
  double cs[kMaxM];
  double sn[kMaxM];
  double hA[kMaxM + 1];              // first CGS projection of the current column
  double hB[kMaxM + 1];              // second CGS projection of the current column
  double scale[kMaxM + 1];           // stored V_i = v_i / scale_i  (true v_i = scale_i * V_i)
  double vsig[kMaxM + 1];            // FP16 storage: V_i holds w_i * vsig_i (a power of two)
  double H[(kMaxM + 1) * kMaxM];     // rotated Hessenberg, column-major, ld = kMaxM + 1
  // Arnoldi with the second Gram-Schmidt pass delayed one step (krylov.hpp):
  double Hu[(kMaxM + 1) * kMaxM];    // unrotated Hessenberg, completed columns (written by the column's completion;
                                     // read by the DCGS2 update pass and by jfnk_gmres_hessenberg)
  double Hp[(kMaxM + 1) * kMaxM];    // first projections of each column (written by the update pass, read by the completion)
  double tscale[kMaxM + 1];          // scale of the JVP tangent of step j: J (tscale_j U_j)
  double ahat[kMaxM + 1];            // second-pass coefficients of the pending vector over its norm
  double jvn2c[kMaxM + 1];           // ||J u^_j||^2 of step j (breakdown test of column j)
};

// FD step parameters (evaluated on the device from device-resident norms).
struct EpsSpec {
  double fixed;              // > 0: use as eps
  double root_eps;           // sqrt(eps_mach)
  int rule;                  // 0 paper, 1 normalized
  const double* xnorm2;      // ||x||^2 (device)
  const double* vnorm2;      // ||v_true||^2 (device); null: ||v|| = 1 (or vparts)
  Partials vparts;           // ||v_true||^2 as partial rows of an earlier kernel (nb > 0)
};

// `vn2` is ||v||^2 when the caller already reduced it (negative: not known).
__device__ __forceinline__ double fd_eps(const EpsSpec& e, double vn2) {
  if (e.fixed > 0.0) return e.fixed;
  const double xn = sqrt(*e.xnorm2);
  if (e.rule == 0) return e.root_eps * fmax(1.0, xn);
  const double vn = vn2 >= 0.0 ? sqrt(vn2) : (e.vnorm2 ? sqrt(*e.vnorm2) : 1.0);
  return e.root_eps * (1.0 + xn) / vn;
}

}  // namespace jfnk
