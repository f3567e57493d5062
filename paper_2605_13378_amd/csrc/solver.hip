// Host side of the JFNK library: solver handle, workspace, the GMRES and
// Newton drivers and the C ABI of include/jfnk.h.
//
// The drivers only enqueue kernels and read back a few scalars:
//  * GMRES: one synchronization per restart cycle (true residual at the cycle
//    start, Arnoldi step count at its end).  Inside a cycle the Arnoldi steps
//    are enqueued back to back; every kernel reads its coefficients and the
//    stop flag from the device control block, and the host looks at the flag
//    of step j-1 (written by that step's last block into mapped host memory)
//    while step j is already queued, so the GPU never waits for the host.
//  * Newton: one synchronization per residual evaluation (the FP64 merit norm
//    decides the line search on the host).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <chrono>
#include <cmath>
#include <cstddef>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <string>
#include <type_traits>
#include <vector>

#include "jfnk.h"
#include "launch.hpp"

using namespace jfnk;

namespace jfnk {
thread_local KernelTiming* g_timing = nullptr;
}

namespace {

constexpr int kNumProf = 13;
enum ProfKernel {
  PK_RES = 0, PK_AD = 1, PK_FD = 2, PK_A = 3, PK_B = 4, PK_C = 5, PK_VY = 6, PK_INIT = 7, PK_TRIAL = 8, PK_FUSED = 9,
  PK_BI = 10, PK_CG = 11, PK_D = 12
};

struct ProfRec {
  int kid;
  double bytes;
  hipEvent_t a, b;
  int step;  // Arnoldi step index (-1 outside a cycle)
};

double eps_mach(int prec) { return prec == JFNK_F64 ? std::ldexp(1.0, -52) : std::ldexp(1.0, -23); }

long long round_up(long long v, long long q) { return (v + q - 1) / q * q; }

// Padding between consecutive basis vectors (elements): keeps the K streams of
// an Arnoldi pass off a power-of-two stride (a 2^21-element vector would put
// element i of every basis vector on the same memory channel).  Measured on
// the Gray-Scott 1024^2 FP32 solve: no pad 346, 256 351, 1056 355.6, 2080 353,
// 4160 351 solves/s.
constexpr long long kBasisPad = 1056;

// Basis passes read with the non-temporal hint once their working set
// exceeds this many bytes (1.5 times the 256 MB last-level cache).  Below it
// the basis of a restart cycle stays largely cache-resident from one pass to
// the next and ordinary loads win; above it a cyclic sweep would only evict
// the reused vectors.  Measured per Arnoldi step (Gray-Scott, DCGS2): 2048^2
// FP32 from j = 8 (~400 MB) on 8-14% faster, 1024^2 FP64 faster from j = 20
// and slower below j = 16 (~340 MB), 1024^2 FP32 slower at every step.
constexpr double kNtBasisBytes = 384.0 * (1 << 20);

}  // namespace

struct jfnk_solver {
  jfnk_problem prob{};
  int prec = 0;
  int m = 0;
  hipStream_t stream = nullptr;
  int pid = 0;
  long long n = 0;
  long long npad = 0;
  long long vstride = 0;   // elements between consecutive basis vectors (npad + kBasisPad)
  Coefs coefs{};
  double alpha = 1.0, cN = 0.0, beta = -1.0;
  int cu = 256;
  size_t tsize = 8;
  size_t vsize = 8;
  void* V = nullptr;
  void* w = nullptr;
  void* R = nullptr;
  void* dx = nullptr;
  void* F = nullptr;
  void* Ft = nullptr;
  void* xw = nullptr;
  void* xwt = nullptr;
  void* b = nullptr;
  double* x64 = nullptr;
  double* x64t = nullptr;
  double* tmp64 = nullptr;
  // partial-sum rows: 0 pass A, 1 pass B, 2 pass C, 3 cycle start, 4 V y, 5 residual / norms
  double* parts = nullptr;
  size_t part_rows = 0;
  Ctl* ctl = nullptr;
  Ctl* hctl = nullptr;     // pinned host mirror of the control block header (+ one whole-block copy)
  int* hflags = nullptr;   // pinned, mapped: per-step stop flags written by the device
  int* dflags = nullptr;   // device view of hflags
  int* hpub = nullptr;     // pinned, mapped: the control block's head published by the device, then its sequence word
  int* dpub = nullptr;     // device view of hpub
  int pub_seq = 0;         // last sequence number asked for
  size_t lds_max = 0;           // LDS bytes one workgroup may use
  FusedInfo* dinfo = nullptr;   // single-workgroup solve record (device)
  FusedInfo* hinfo = nullptr;   // pinned host copy
  BiCtl* dbi = nullptr;         // BiCGSTAB scalars (device)
  BiCtl* hbi = nullptr;         // pinned host copy
  CgCtl* dcg = nullptr;         // CG scalars (device)
  CgCtl* hcg = nullptr;         // pinned host copy
  bool has_prev = false;
  int orth = 0;                 // Gram-Schmidt form of jfnk_gmres calls (jfnk_orth)
  int precond = 0;              // preconditioner of jfnk_gmres calls (jfnk_precond)
  std::string err;
  bool prof = false;
  int cur_step = -1;
  // MULTI_KERNEL_GRAPH engine: the Arnoldi steps and V y update of a restart
  // cycle, captured once per launch configuration and replayed
  struct CycleGraph {
    long long key[8];
    hipGraphExec_t exec;
  };
  bool graph = false;  // the current solve replays captured cycles
  std::vector<CycleGraph> graphs;
  std::vector<ProfRec> recs;
  std::vector<hipEvent_t> pool;
  long long p_count[kNumProf] = {};
  double p_ms[kNumProf] = {};
  double p_bytes[kNumProf] = {};
};

#define JFNK_HIP(s, ...)                                                   \
  do {                                                                     \
    hipError_t e_ = (__VA_ARGS__);                                         \
    if (e_ != hipSuccess) {                                                \
      (s)->err = std::string(#__VA_ARGS__) + ": " + hipGetErrorString(e_); \
      return JFNK_ERR_HIP;                                                 \
    }                                                                      \
  } while (0)

#define JFNK_TRY(...)                   \
  do {                                  \
    jfnk_status st_ = (__VA_ARGS__);    \
    if (st_ != JFNK_OK) return st_;     \
  } while (0)

namespace {

// ---------------------------------------------------------------------------
// profiling with HIP events on the solver's stream
// ---------------------------------------------------------------------------
hipEvent_t pool_get(jfnk_solver* s) {
  if (!s->pool.empty()) {
    hipEvent_t e = s->pool.back();
    s->pool.pop_back();
    return e;
  }
  hipEvent_t e = nullptr;
  if (hipEventCreate(&e) != hipSuccess) return nullptr;
  return e;
}

// Times the single kernel launched while it is alive (see g_timing).
struct ProfScope {
  jfnk_solver* s;
  int kid;
  double bytes;
  KernelTiming t;
  ProfScope(jfnk_solver* s_, int kid_, double bytes_) : s(s_), kid(kid_), bytes(bytes_) {
    if (s->prof) {
      t.start = pool_get(s);
      t.stop = pool_get(s);
      if (t.start && t.stop) g_timing = &t;
    }
  }
  ~ProfScope() {
    if (g_timing == &t) {
      g_timing = nullptr;
      s->recs.push_back({kid, bytes, t.start, t.stop, s->cur_step});
    } else {
      if (t.start) s->pool.push_back(t.start);
      if (t.stop) s->pool.push_back(t.stop);
    }
  }
};

// Fold completed event pairs into the per-kernel totals.  Launches of Arnoldi
// steps at or beyond `steps_done` early-exited (the cycle had already stopped)
// and are not counted.
void prof_harvest(jfnk_solver* s, int steps_done) {
  for (const ProfRec& r : s->recs) {
    float ms = 0.f;
    const bool skipped = r.step >= 0 && r.step >= steps_done;
    if (!skipped && hipEventElapsedTime(&ms, r.a, r.b) == hipSuccess) {
      s->p_count[r.kid] += 1;
      s->p_ms[r.kid] += ms;
      s->p_bytes[r.kid] += r.bytes;
    }
    s->pool.push_back(r.a);
    s->pool.push_back(r.b);
  }
  s->recs.clear();
}

// Bring the control block's head (the fields up to gp) to s->hctl once all
// queued work has run.  Normally a one-wavefront kernel writes it to mapped
// host memory and then a sequence word, and the host spins on that word (a
// stream synchronization's wake-up and a copy cost more); with kernel timing
// on, or if the stream drains without the word appearing, a copy and a
// stream synchronization instead.
constexpr int kPubWords = (int)(offsetof(Ctl, gp) / sizeof(int));
static_assert(offsetof(Ctl, gp) % sizeof(int) == 0, "control block head must be whole words");

jfnk_status sync_read_ctl(jfnk_solver* s) {
  if (!s->prof && s->hpub != nullptr) {
    const int seq = ++s->pub_seq;
    JFNK_HIP(s, launch_publish_ctl(s->ctl, s->dpub, kPubWords, s->dpub + kPubWords, seq, s->stream));
    volatile int* word = s->hpub + kPubWords;
    bool seen = false;
    for (unsigned it = 1;; ++it) {
      if (*word == seq) {
        seen = true;
        break;
      }
      if ((it & 1023u) == 0) {
        const hipError_t q = hipStreamQuery(s->stream);
        if (q == hipSuccess) {
          seen = *word == seq;
          break;
        }
        if (q != hipErrorNotReady) JFNK_HIP(s, q);
      }
      __builtin_ia32_pause();
    }
    if (seen) {
      std::atomic_thread_fence(std::memory_order_acquire);
      std::memcpy(static_cast<void*>(s->hctl), const_cast<const int*>(static_cast<volatile int*>(s->hpub)),
                  offsetof(Ctl, gp));
      return JFNK_OK;
    }
  }
  JFNK_HIP(s, hipMemcpyAsync(s->hctl, s->ctl, offsetof(Ctl, gp), hipMemcpyDeviceToHost, s->stream));
  JFNK_HIP(s, hipStreamSynchronize(s->stream));
  return JFNK_OK;
}

int krylov_grid(const jfnk_solver* s, int vec) {
  const long long need = (s->npad + (long long)kKrylovThreads * vec - 1) / ((long long)kKrylovThreads * vec);
  return (int)std::max<long long>(1, std::min<long long>(need, s->cu));
}

int stream_grid(const jfnk_solver* s, int vec) {
  const long long need = (s->npad + (long long)kStreamThreads * vec - 1) / ((long long)kStreamThreads * vec);
  return (int)std::max<long long>(1, std::min<long long>(need, 4LL * s->cu));
}

// Block caps of stencil launches: a launch that writes per-block partial sums
// (residual norms) stays within the partial-sum rows; the Arnoldi JVP, whose
// partials carry up to 33 columns, within 2 blocks per compute unit; launches
// without partial sums take one tile per block.
int stencil_cap(const jfnk_solver* s) { return 4 * s->cu; }
int arnoldi_cap(const jfnk_solver* s) { return 2 * s->cu; }
constexpr int kNoCap = 1 << 30;

bool aligned(const void* p, size_t a) { return p == nullptr || (reinterpret_cast<uintptr_t>(p) % a) == 0; }

EpsSpec eps_spec(const jfnk_solver* s, double fixed, int rule, const double* vnorm2) {
  EpsSpec e{};
  e.fixed = fixed;
  e.root_eps = std::sqrt(eps_mach(s->prec));
  e.rule = rule;
  e.xnorm2 = &s->ctl->xnorm2;
  e.vnorm2 = rule == JFNK_EPS_NORMALIZED ? vnorm2 : nullptr;
  return e;
}

// First Arnoldi step after which the host keeps one step queued ahead
// instead of two (measured at Gray-Scott 1024^2 FP32: 438 against 432
// solves/s; one step ahead from the start, 436: the first steps are too
// short to cover the host's launches).
constexpr int kOneAheadFrom = 8;

// Spin until the device has written a step's stop flag into mapped host
// memory (the host resets it to -1 before launching the writer).  Returns
// false if the stream went idle without writing it or reported an error; the
// caller then stops the cycle and its next synchronization reads the device
// state (and reports any error).
bool wait_flag(jfnk_solver* s, volatile int* flags, int c) {
  for (unsigned it = 1;; ++it) {
    if (flags[c] != -1) return true;
    if ((it & 1023u) == 0) {
      const hipError_t q = hipStreamQuery(s->stream);
      if (q == hipSuccess) return flags[c] != -1;
      if (q != hipErrorNotReady) return false;
    }
    __builtin_ia32_pause();
  }
}

// ---------------------------------------------------------------------------
// precision-generic drivers
// ---------------------------------------------------------------------------
template <class T, class VT>
struct Impl {
  static constexpr int KVEC = krylov_vec<T>();

  // Grid of the CGS passes over K basis vectors: two 512-thread blocks per
  // compute unit while the pass's registers leave room for them (up to 16
  // vectors: ~120 VGPRs), one block otherwise (measured on MI355X: 512 blocks
  // run passes B and C 4-10% faster at K = 12, 256 blocks 20% faster at
  // K = 24).  Consumers of a pass's partial sums use the same grid.
  static int cgs_grid(const jfnk_solver* s, int K) {
    const int kmax = K <= 4 ? 4 : (K <= 8 ? 8 : (K <= 16 ? 16 : 32));
    const int vec = sizeof(VT) == 2 ? 8 : ((sizeof(T) == 8 && kmax > 16) ? 1 : (int)(16 / sizeof(T)));
    const bool two = kmax <= 16;
    const long long need = (s->npad + (long long)kKrylovThreads * vec - 1) / ((long long)kKrylovThreads * vec);
    return (int)std::max<long long>(1, std::min<long long>(need, (two ? 2LL : 1LL) * s->cu));
  }

  // Grid of the DCGS2 update pass (and the row count of its partial sums,
  // which the next Arnoldi JVP and the V y kernel reduce).
  static int dcgs_grid(const jfnk_solver* s, int K) { return cgs_grid(s, K <= 16 ? 32 : K); }

  static double* part(jfnk_solver* s, int region) { return s->parts + (size_t)region * s->part_rows * kMaxCols; }
  static PartSink sink(jfnk_solver* s, int region) { return PartSink{part(s, region), (int)s->part_rows}; }
  static Partials parts(jfnk_solver* s, int region, int nb) { return Partials{part(s, region), nb, (int)s->part_rows}; }

  // Residual F = alpha x + cN N(x) + beta b; optional norms into ctl.
  static jfnk_status residual(jfnk_solver* s, const T* x, T* F, bool norms) {
    StencilArgs<T, T> a{};
    a.nx = s->prob.nx;
    a.ny = s->prob.ny;
    a.plane = (long long)s->prob.nx * s->prob.ny;
    a.x = x;
    a.b = static_cast<const T*>(s->b);
    a.out = F;
    a.alpha = s->alpha;
    a.cN = s->cN;
    a.beta = s->beta;
    a.part_out = sink(s, 5);
    a.nred = norms ? 2 : 0;
    const int vec = stencil_vec<T>(s->pid);
    const bool vz = (s->prob.nx % vec == 0) && aligned(x, 16) && aligned(F, 16) && aligned(s->b, 16);
    int nb = 0;
    {
      ProfScope ps(s, PK_RES, 3.0 * s->n * sizeof(T));
      JFNK_HIP(s, launch_stencil<T, T>(s->pid, OP_RES, false, vz, a, s->coefs, norms ? stencil_cap(s) : kNoCap,
                                        s->stream, &nb));
    }
    if (norms) JFNK_HIP(s, launch_finish_sums(parts(s, 5, nb), 2, &s->ctl->fnorm2, &s->ctl->xnorm2, s->stream));
    return JFNK_OK;
  }

  // Jv = J(x) v (AD or FD), optional F(x) for AD; v is of type W (T or VT).
  // Arnoldi mode (arn_j >= 0): v is basis vector arn_j, its scale and the
  // pending Givens column come from the device control block, and the first
  // CGS projection on V_0..V_arn_j is fused in (partial sums into region 0;
  // *nb_out receives their row count).
  template <class W>
  static jfnk_status jvp(jfnk_solver* s, const T* x, const W* v, const double* vscale, T* Jv, T* Fout, int mode,
                         const EpsSpec& eps, int arn_j = -1, int* nb_out = nullptr, bool lagged = false,
                         bool pre = false) {
    StencilArgs<T, W> a{};
    a.nx = s->prob.nx;
    a.ny = s->prob.ny;
    a.plane = (long long)s->prob.nx * s->prob.ny;
    a.x = x;
    a.v = v;
    // the AD tangent does not involve b; F(x) and the FD difference do
    a.b = (mode == JFNK_JVP_AD && Fout == nullptr) ? nullptr : static_cast<const T*>(s->b);
    a.out = Jv;
    a.out2 = Fout;
    a.alpha = s->alpha;
    a.cN = s->cN;
    a.beta = s->beta;
    a.vscale = vscale;
    a.eps = eps;
    a.precond = pre ? 1 : 0;
    if (arn_j >= 0) {
      a.ctl = s->ctl;
      a.arn_j = arn_j;
      a.lagged = lagged ? 1 : 0;
      // the sums that complete column arn_j - 1: pass C's (CGS2) or the update pass's (DCGS2)
      a.pc = lagged ? parts(s, 1, dcgs_grid(s, arn_j > 0 ? arn_j : 1)) : parts(s, 2, cgs_grid(s, arn_j > 0 ? arn_j : 1));
      a.host_flags = s->dflags;
      a.Vb = reinterpret_cast<const W*>(basis(s, 0));
      a.vstride = s->vstride;
      a.K = arn_j + 1;
      a.dots_out = sink(s, 0);
      a.nt_basis = (double)(arn_j + 4) * s->n * sizeof(W) > kNtBasisBytes ? 1 : 0;
    }
    const int vec = stencil_vec<T>(s->pid);
    const bool vz = (s->prob.nx % vec == 0) && aligned(x, 16) && aligned(v, vec * sizeof(W)) && aligned(Jv, 16) &&
                    aligned(Fout, 16) && aligned(a.b, 16);
    const int op = mode == JFNK_JVP_AD ? OP_AD : OP_FD;
    // algorithmic bytes: x, v (b for F / FD), Jv (F); fused: x, V_0..V_j, Jv
    double bytes = (mode == JFNK_JVP_AD ? 2.0 + (Fout ? 2.0 : 0.0) : 3.0) * s->n * sizeof(T) + (double)s->n * sizeof(W);
    if (arn_j >= 0) bytes += (double)arn_j * s->n * sizeof(W);
    ProfScope ps(s, mode == JFNK_JVP_AD ? PK_AD : PK_FD, bytes);
    const int cap = arn_j >= 0 ? arnoldi_cap(s) : kNoCap;
    JFNK_HIP(s, launch_stencil<T, W>(s->pid, op, Fout != nullptr, vz, a, s->coefs, cap, s->stream, nb_out));
    return JFNK_OK;
  }

  struct GOut {
    bool converged = false, nonfinite = false;
    // the Newton trial point x + dx and its residual norms were queued
    // before the solve's last synchronization and read back with it
    bool trial_done = false;
    int iters = 0, cycles = 0;
    double bnorm = 0.0, true_res = 0.0;
  };

  // Newton trial point x64t = x64 + alpha dx (and its working copy), then its
  // residual Ft with the norms ||Ft||^2, ||xt||^2 into the control block.
  static jfnk_status queue_trial(jfnk_solver* s, double alpha, int sgrid) {
    constexpr bool f64 = std::is_same<T, double>::value;
    {
      ProfScope ps(s, PK_TRIAL, (double)s->n * (16.0 + sizeof(T) + (f64 ? 0.0 : sizeof(T))));
      JFNK_HIP(s, launch_trial<T>(s->npad, s->x64, static_cast<const T*>(s->dx), alpha, s->x64t,
                                  f64 ? nullptr : static_cast<T*>(s->xwt), sgrid, s->stream));
    }
    const T* xt = f64 ? reinterpret_cast<const T*>(s->x64t) : static_cast<const T*>(s->xwt);
    JFNK_TRY(residual(s, xt, static_cast<T*>(s->Ft), true));
    return JFNK_OK;
  }

  static VT* basis(jfnk_solver* s, int i) { return static_cast<VT*>(s->V) + (long long)i * s->vstride; }

  // Arnoldi step j of a cycle: the JVP of basis vector j with the first
  // projection fused in, then the Gram-Schmidt pass(es).
  static jfnk_status arnoldi_step(jfnk_solver* s, const T* x, int j, int mode, const EpsSpec& eps_arnoldi,
                                  bool lagged, bool pre) {
    T* w = static_cast<T*>(s->w);
    s->cur_step = j;
    const int K = j + 1;
    int nb_jvp = 0;  // the JVP carries the first projection (pass A)
    JFNK_TRY(jvp<VT>(s, x, basis(s, j), nullptr, w, nullptr, mode, eps_arnoldi, j, &nb_jvp, lagged, pre));
    KArgs<T, VT> ka{s->npad, basis(s, 0), s->vstride, w, basis(s, K), K, s->ctl, parts(s, 0, nb_jvp), sink(s, 1),
                    (double)(K + 3) * s->n * sizeof(VT) > kNtBasisBytes ? 1 : 0};
    if (lagged) {
      // one update pass: v_j completed, the next vector projected once
      ProfScope ps(s, PK_D, (double)s->n * ((K + 2) * sizeof(VT) + sizeof(T)));
      JFNK_HIP(s, launch_dcgs<T, VT>(ka, dcgs_grid(s, K), s->stream));
    } else {
      {
        ProfScope ps(s, PK_B, (double)s->n * (K * sizeof(VT) + 2 * sizeof(T)));
        JFNK_HIP(s, launch_cgs<T, VT>(PASS_B, ka, cgs_grid(s, K), s->stream));
      }
      ka.in = parts(s, 1, cgs_grid(s, K));
      ka.out = sink(s, 2);
      ProfScope ps(s, PK_C, (double)s->n * (K * sizeof(VT) + sizeof(T) + sizeof(VT)));
      JFNK_HIP(s, launch_cgs<T, VT>(PASS_C, ka, cgs_grid(s, K), s->stream));
    }
    return JFNK_OK;
  }

  // End of a cycle whose last enqueued step is jmax: the V y update.
  static jfnk_status cycle_end(jfnk_solver* s, int jmax, int first, int m, bool lagged, int kgrid) {
    VyArgs<T, VT> va{s->npad, basis(s, 0), s->vstride, static_cast<T*>(s->dx), first, jmax, s->ctl,
                     lagged ? parts(s, 1, dcgs_grid(s, jmax >= 0 ? jmax + 1 : 1))
                            : parts(s, 2, cgs_grid(s, jmax >= 0 ? jmax + 1 : 1)),
                     sink(s, 4), s->dflags,
                     lagged ? 1 : 0, (double)(jmax + 3) * s->n * sizeof(VT) > kNtBasisBytes ? 1 : 0};
    ProfScope ps(s, PK_VY, 0.0);  // bytes filled in once k is known
    JFNK_HIP(s, launch_vy<T, VT>(va, m, kgrid, s->stream));
    return JFNK_OK;
  }

  // The captured graph of one cycle's m Arnoldi steps and V y update for
  // this launch configuration (every kernel argument is fixed by it: the
  // solver's buffers, m, the JVP kind and step rule, the Gram-Schmidt form,
  // the preconditioner and whether dx is overwritten or accumulated),
  // captured on the first use and kept until the solver is destroyed.
  static jfnk_status cycle_graph(jfnk_solver* s, const T* x, int m, int mode, const EpsSpec& eps, bool lagged,
                                 bool pre, int first, int kgrid, hipGraphExec_t* out) {
    long long fe = 0;
    std::memcpy(&fe, &eps.fixed, sizeof(fe));
    const long long key[8] = {(long long)(uintptr_t)x, m, mode, fe, eps.rule, lagged ? 1 : 0, pre ? 1 : 0, first};
    for (const auto& g : s->graphs)
      if (std::equal(key, key + 8, g.key)) {
        *out = g.exec;
        return JFNK_OK;
      }
    JFNK_HIP(s, hipStreamBeginCapture(s->stream, hipStreamCaptureModeThreadLocal));
    jfnk_status st = JFNK_OK;
    for (int j = 0; j < m && st == JFNK_OK; ++j) st = arnoldi_step(s, x, j, mode, eps, lagged, pre);
    s->cur_step = -1;
    if (st == JFNK_OK) st = cycle_end(s, m - 1, first, m, lagged, kgrid);
    hipGraph_t g = nullptr;
    const hipError_t ec = hipStreamEndCapture(s->stream, &g);  // ends the capture on every path
    if (st != JFNK_OK) {
      if (g) (void)hipGraphDestroy(g);
      return st;
    }
    if (ec != hipSuccess) {
      s->err = std::string("hipStreamEndCapture: ") + hipGetErrorString(ec);
      return JFNK_ERR_HIP;
    }
    hipGraphExec_t exec = nullptr;
    const hipError_t ei = hipGraphInstantiate(&exec, g, nullptr, nullptr, 0);
    (void)hipGraphDestroy(g);
    if (ei != hipSuccess) {
      s->err = std::string("hipGraphInstantiate: ") + hipGetErrorString(ei);
      return JFNK_ERR_HIP;
    }
    jfnk_solver::CycleGraph cg{};
    std::copy(key, key + 8, cg.key);
    cg.exec = exec;
    s->graphs.push_back(cg);
    *out = exec;
    return JFNK_OK;
  }

  // Restarted GMRES(m) on J(x) dx = sign * R (R internal, padded), dx internal.
  // With `pre` (right preconditioning by the problem's diagonal M, frozen at
  // x) every JVP of the solve is applied to M^{-1} times its vector, so the
  // iterate z and the basis live in the preconditioned space and the
  // residual, its norm and the stopping tests are those of J dx = sign * R;
  // dx = M^{-1} z at the end.
  // spec_trial (Newton, AD JVP, no preconditioner): the second cycle's start,
  // where a solve that converged in one cycle ends, also queues the Newton
  // trial point with alpha = 1 and its residual, so that one synchronization
  // reads back both (go.trial_done); if the solve goes on they are discarded
  // (scratch vectors and residual norms only: no kernel of the solve reads
  // them, which is why the FD JVP, whose step reads ||x||, is left out).
  static jfnk_status gmres(jfnk_solver* s, const T* x, const T* R, double sign, int m, double tol, int max_restarts,
                           int mode, double fixed_eps, int eps_rule, double brk, GOut& go, bool lagged = false,
                           bool pre = false, bool spec_trial = false) {
    go = GOut{};
    T* dxi = static_cast<T*>(s->dx);
    T* w = static_cast<T*>(s->w);
    // captured cycles need a stream of their own (the null stream cannot be
    // captured) and no per-kernel timing events
    const bool use_graph = s->graph && s->stream != nullptr && !s->prof;
    const int kgrid = krylov_grid(s, KVEC);
    const int sgrid = stream_grid(s, KVEC);
    const EpsSpec eps_arnoldi = eps_spec(s, fixed_eps, eps_rule, nullptr);  // ||v_j|| = 1
    EpsSpec eps_restart = eps_spec(s, fixed_eps, eps_rule, nullptr);        // v = dx
    if (eps_rule == JFNK_EPS_NORMALIZED) eps_restart.vparts = parts(s, 4, kgrid);
    volatile int* flags = reinterpret_cast<volatile int*>(s->hflags);
    JFNK_HIP(s, launch_ctl_begin(s->ctl, tol, brk, m, s->stream));
    bool updated = false;
    // The V y update that ends a cycle is read back together with the next
    // cycle's start (one synchronization per cycle): its k and stop state sit
    // in fields the cycle start leaves alone.
    bool pending_vy = false;
    int spec_cycle = -1, last_cycle = 0;
    for (int cycle = 0;; ++cycle) {
      last_cycle = cycle;
      const T* wr = nullptr;
      s->cur_step = -1;
      if (cycle > 0) {
        JFNK_TRY(jvp<T>(s, x, dxi, nullptr, w, nullptr, mode, eps_restart, -1, nullptr, false, pre));
        wr = w;
      }
      {
        InitArgs<T, VT> ia{s->npad, R, sign, wr, basis(s, 0), sink(s, 3), w};
        ProfScope ps(s, PK_INIT, (double)s->n * ((wr ? 2.0 : 1.0) * sizeof(T) + sizeof(VT)));
        JFNK_HIP(s, launch_init<T, VT>(ia, sgrid, s->stream));
      }
      constexpr bool fp16 = !std::is_same<T, VT>::value;
      JFNK_HIP(s, launch_cycle_begin(s->ctl, parts(s, 3, sgrid), m, s->n, fp16 ? 1 : 0, s->stream));
      if (fp16) JFNK_HIP(s, launch_store_basis0<T, VT>(s->npad, w, basis(s, 0), s->ctl, sgrid, s->stream));
      if (spec_trial && !pre && cycle == 1) {
        JFNK_TRY(queue_trial(s, 1.0, sgrid));
        spec_cycle = cycle;
      }
      // The first cycle's start is not read back: its Arnoldi steps are
      // queued at once, and if the start already stopped the cycle (a zero
      // or non-finite right-hand side) they leave at once on the device and
      // the V y update writes dx = 0 with k = 0; the next cycle's start
      // reads both back (one synchronization fewer per solve).
      if (cycle > 0 || max_restarts == 0) {
        JFNK_TRY(sync_read_ctl(s));
        if (pending_vy) {
          pending_vy = false;
          const int k = s->hctl->k_last;
          if (s->prof) {
            for (ProfRec& r : s->recs)
              if (r.kid == PK_VY) r.bytes = (double)s->n * (k * sizeof(VT) + (cycle == 1 ? 1.0 : 2.0) * sizeof(T));
            prof_harvest(s, k);
          }
          go.iters += k;
          if (k == 0) go.cycles -= 1;  // the cycle stopped at its start: not a cycle run
          if (k > 0 && s->hctl->k_last_state == kNonfinite) {
            go.nonfinite = true;
            break;
          }
        } else if (s->prof) {
          prof_harvest(s, 0);
        }
        if (cycle <= 1) go.bnorm = s->hctl->bnorm;  // written by the first cycle's start only
        go.true_res = s->hctl->beta;
        const int d0 = s->hctl->done_col[0];
        if (d0 == kNonfinite) {
          go.nonfinite = true;
          break;
        }
        if (d0 == kConverged) {
          go.converged = true;
          break;
        }
        if (cycle == max_restarts) break;
      }
      go.cycles += 1;
      // Arnoldi steps back to back; the Givens update of column j runs in the
      // prologue of step j+1's JVP and reports its stop flag to mapped host
      // memory.  After enqueueing step j the host waits until step j-1's JVP
      // has published column j-2's flag (two steps queued ahead), and from
      // step kOneAheadFrom on, when a step's kernels outlast the host's
      // launches, until step j's own JVP has published column j-1's (one
      // step ahead): at most one or two enqueued steps are skipped after
      // the stop, and no marker is placed in the stream between steps.  The
      // delayed-second-pass form runs two kernels per step (JVP with the
      // first projection and the completion of column j-1 in its prologue,
      // then one update pass) with the same flag protocol.
      if (use_graph) {
        // the whole cycle from its captured graph: every step is launched;
        // steps after the one that stopped the cycle find the stop state in
        // the control block and leave at once (as the up to two steps the
        // direct path queues ahead do)
        hipGraphExec_t ge = nullptr;
        JFNK_TRY(cycle_graph(s, x, m, mode, eps_arnoldi, lagged, pre, updated ? 0 : 1, kgrid, &ge));
        JFNK_HIP(s, hipGraphLaunch(ge, s->stream));
        updated = true;
        pending_vy = true;
        continue;
      }
      int jmax = -1;
      for (int j = 0; j < m; ++j) {
        if (j >= 1) flags[j - 1] = -1;
        JFNK_TRY(arnoldi_step(s, x, j, mode, eps_arnoldi, lagged, pre));
        jmax = j;
        const int lag = j >= kOneAheadFrom ? 1 : 2;
        if (j >= lag && (!wait_flag(s, flags, j - lag) || flags[j - lag] != kRunning)) break;
      }
      s->cur_step = -1;
      flags[jmax] = -1;
      JFNK_TRY(cycle_end(s, jmax, updated ? 0 : 1, m, lagged, kgrid));
      updated = true;
      pending_vy = true;
    }
    go.trial_done = spec_cycle >= 0 && spec_cycle == last_cycle;
    if (!updated) JFNK_HIP(s, launch_fill_zero<T>(s->npad, dxi, sgrid, s->stream));
    if (pre && updated)
      JFNK_HIP(s, launch_cslp_apply<T>(s->pid, x, dxi, s->prob.nx, s->prob.ny, s->coefs, sgrid, s->stream));
    return JFNK_OK;
  }

  // Jacobian-vector product of a BiCGSTAB iteration: Jv = J(x) v with the
  // partial sums of (dotv, Jv) and ||Jv||^2 into region `region` (the fused
  // projection slot of the Arnoldi JVP with one vector); skipped on the
  // device once the solve has stopped (see StencilArgs::gate).
  static jfnk_status jvp_bi(jfnk_solver* s, const T* x, const T* v, T* Jv, int mode, const EpsSpec& eps,
                            const T* dotv, int region, const int* gate, Partials gate_parts, const double* gate_tol,
                            int* nb_out) {
    StencilArgs<T, T> a{};
    a.nx = s->prob.nx;
    a.ny = s->prob.ny;
    a.plane = (long long)s->prob.nx * s->prob.ny;
    a.x = x;
    a.v = v;
    a.b = mode == JFNK_JVP_AD ? nullptr : static_cast<const T*>(s->b);
    a.out = Jv;
    a.alpha = s->alpha;
    a.cN = s->cN;
    a.beta = s->beta;
    a.eps = eps;
    a.Vb = dotv;
    a.vstride = s->vstride;
    a.K = 1;
    a.dots_out = sink(s, region);
    a.gate = gate;
    a.gate_parts = gate_parts;
    a.gate_tol = gate_tol;
    const int vec = stencil_vec<T>(s->pid);
    const bool vz = (s->prob.nx % vec == 0) && aligned(x, 16) && aligned(v, 16) && aligned(Jv, 16) &&
                    aligned(a.b, 16) && aligned(dotv, 16);
    const int op = mode == JFNK_JVP_AD ? OP_AD : OP_FD;
    // algorithmic bytes: x, v, Jv (+ b for FD) and the dot vector unless it is v itself
    const double bytes = ((mode == JFNK_JVP_AD ? 3.0 : 4.0) + (dotv == v ? 0.0 : 1.0)) * s->n * sizeof(T);
    ProfScope ps(s, mode == JFNK_JVP_AD ? PK_AD : PK_FD, bytes);
    JFNK_HIP(s, launch_stencil<T, T>(s->pid, op, false, vz, a, s->coefs, arnoldi_cap(s), s->stream, nb_out));
    return JFNK_OK;
  }

  struct BOut {
    bool converged = false, nonfinite = false, breakdown = false;
    int iters = 0;
    double bnorm = 0.0, res = 0.0;
  };

  // BiCGSTAB on J(x) dx = sign * R (R internal, padded) from dx = 0, dx
  // internal.  r^, r, p, v, s, t occupy basis slots 0..5 (working precision;
  // callers check that the basis has them).  Iterations are enqueued back to
  // back; the p kernel of iteration i publishes the state after iteration
  // i-1 to mapped host memory, and after enqueueing iteration i the host
  // waits for iteration i-1's flag, so at most two enqueued iterations run
  // empty after the stop.  A last p kernel in check-only mode settles the
  // state after the final iteration.
  static jfnk_status bicgstab(jfnk_solver* s, const T* x, const T* R, double sign, double tol, int maxiter,
                              int mode, double fixed_eps, int eps_rule, BOut& bo) {
    static_assert(std::is_same<T, VT>::value, "BiCGSTAB keeps its vectors in the working precision");
    bo = BOut{};
    T* rh = basis(s, 0);
    T* r = basis(s, 1);
    T* p = basis(s, 2);
    T* v = basis(s, 3);
    T* sv = basis(s, 4);
    T* t = basis(s, 5);
    const int sgrid = stream_grid(s, KVEC);
    BiArgs<T> a{};
    a.n = s->npad;
    a.c = s->dbi;
    a.R = R;
    a.sign = sign;
    a.rh = rh;
    a.r = r;
    a.p = p;
    a.v = v;
    a.s = sv;
    a.t = t;
    a.x = static_cast<T*>(s->dx);
    a.host_flags = s->dflags;
    EpsSpec eps_p = eps_spec(s, fixed_eps, eps_rule, nullptr);
    EpsSpec eps_s = eps_p;
    if (eps_rule == JFNK_EPS_NORMALIZED) {
      eps_p.vparts = parts(s, 1, sgrid);  // ||p||^2 from the p kernel
      eps_s.vparts = parts(s, 3, sgrid);  // ||s||^2 from the s kernel
    }
    const double vec_bytes = (double)s->n * sizeof(T);
    // partial-sum regions: 0 xr / init, 1 p, 2 JVP of p, 3 s, 4 JVP of s
    s->cur_step = -1;
    a.out = sink(s, 0);
    {
      ProfScope ps(s, PK_BI, 4.0 * vec_bytes);
      JFNK_HIP(s, launch_bi<T>(BI_INIT, a, tol, sgrid, s->stream));
    }
    volatile int* flags = reinterpret_cast<volatile int*>(s->hflags);
    constexpr int kRing = kMaxM + 1;
    int last = 0;
    for (int it = 1; it <= maxiter; ++it) {
      s->cur_step = it - 1;
      a.it = it;
      a.check_only = 0;
      a.flag_slot = it % kRing;
      flags[a.flag_slot] = -1;
      a.in = parts(s, 0, sgrid);
      a.out = sink(s, 1);
      {
        ProfScope ps(s, PK_BI, (it == 1 ? 2.0 : 4.0) * vec_bytes);
        JFNK_HIP(s, launch_bi<T>(BI_P, a, tol, sgrid, s->stream));
      }
      int nb_v = 0;
      JFNK_TRY(jvp_bi(s, x, p, v, mode, eps_p, rh, 2, &s->dbi->state_p, Partials{nullptr, 0, 0}, nullptr, &nb_v));
      a.in = parts(s, 2, nb_v);
      a.out = sink(s, 3);
      {
        ProfScope ps(s, PK_BI, 3.0 * vec_bytes);
        JFNK_HIP(s, launch_bi<T>(BI_S, a, tol, sgrid, s->stream));
      }
      int nb_t = 0;
      JFNK_TRY(jvp_bi(s, x, sv, t, mode, eps_s, sv, 4, &s->dbi->state_s, parts(s, 3, sgrid), &s->dbi->target,
                      &nb_t));
      a.in = parts(s, 3, sgrid);
      a.in2 = parts(s, 4, nb_t);
      a.out = sink(s, 0);
      {
        ProfScope ps(s, PK_BI, 7.0 * vec_bytes);
        JFNK_HIP(s, launch_bi<T>(BI_XR, a, tol, sgrid, s->stream));
      }
      last = it;
      if (it >= 2) {
        const int ps = (it - 1) % kRing;
        if (!wait_flag(s, flags, ps) || flags[ps] != kRunning) break;
      }
    }
    s->cur_step = -1;
    a.it = last + 1;
    a.check_only = 1;
    a.flag_slot = (last + 1) % kRing;
    a.in = parts(s, 0, sgrid);
    JFNK_HIP(s, launch_bi<T>(BI_P, a, tol, sgrid, s->stream));
    JFNK_HIP(s, hipMemcpyAsync(s->hbi, s->dbi, sizeof(BiCtl), hipMemcpyDeviceToHost, s->stream));
    JFNK_HIP(s, hipStreamSynchronize(s->stream));
    const BiCtl& h = *s->hbi;
    if (s->prof) prof_harvest(s, h.iters + 1);
    bo.iters = h.iters;
    bo.bnorm = h.bnorm;
    bo.res = h.res;
    bo.converged = h.state_p == kConverged;
    bo.nonfinite = h.state_p == kNonfinite;
    bo.breakdown = h.state_p == kBreakdown;
    return JFNK_OK;
  }

  // Conjugate gradients on J(x) dx = sign * R (R internal, padded) from
  // dx = 0, dx internal; r, p, q = J p occupy basis slots 0..2.  The host
  // loop and the flag protocol are those of bicgstab() with three kernels per
  // iteration.
  static jfnk_status cg(jfnk_solver* s, const T* x, const T* R, double sign, double tol, int maxiter, int mode,
                        double fixed_eps, int eps_rule, BOut& bo) {
    static_assert(std::is_same<T, VT>::value, "CG keeps its vectors in the working precision");
    bo = BOut{};
    T* r = basis(s, 0);
    T* p = basis(s, 1);
    T* q = basis(s, 2);
    const int sgrid = stream_grid(s, KVEC);
    CgArgs<T> a{};
    a.n = s->npad;
    a.c = s->dcg;
    a.R = R;
    a.sign = sign;
    a.r = r;
    a.p = p;
    a.q = q;
    a.x = static_cast<T*>(s->dx);
    a.host_flags = s->dflags;
    EpsSpec eps_p = eps_spec(s, fixed_eps, eps_rule, nullptr);
    if (eps_rule == JFNK_EPS_NORMALIZED) eps_p.vparts = parts(s, 1, sgrid);  // ||p||^2 from the p kernel
    const double vec_bytes = (double)s->n * sizeof(T);
    // partial-sum regions: 0 xr / init, 1 p, 2 JVP
    s->cur_step = -1;
    a.out = sink(s, 0);
    {
      ProfScope ps(s, PK_CG, 3.0 * vec_bytes);
      JFNK_HIP(s, launch_cg<T>(CG_INIT, a, tol, sgrid, s->stream));
    }
    volatile int* flags = reinterpret_cast<volatile int*>(s->hflags);
    constexpr int kRing = kMaxM + 1;
    int last = 0;
    for (int it = 1; it <= maxiter; ++it) {
      s->cur_step = it - 1;
      a.it = it;
      a.check_only = 0;
      a.flag_slot = it % kRing;
      flags[a.flag_slot] = -1;
      a.in = parts(s, 0, sgrid);
      a.out = sink(s, 1);
      {
        ProfScope ps(s, PK_CG, (it == 1 ? 2.0 : 3.0) * vec_bytes);
        JFNK_HIP(s, launch_cg<T>(CG_P, a, tol, sgrid, s->stream));
      }
      int nb_q = 0;
      JFNK_TRY(jvp_bi(s, x, p, q, mode, eps_p, p, 2, &s->dcg->state_p, Partials{nullptr, 0, 0}, nullptr, &nb_q));
      a.in = parts(s, 2, nb_q);
      a.out = sink(s, 0);
      {
        ProfScope ps(s, PK_CG, 6.0 * vec_bytes);
        JFNK_HIP(s, launch_cg<T>(CG_XR, a, tol, sgrid, s->stream));
      }
      last = it;
      if (it >= 2) {
        const int ps = (it - 1) % kRing;
        if (!wait_flag(s, flags, ps) || flags[ps] != kRunning) break;
      }
    }
    s->cur_step = -1;
    a.it = last + 1;
    a.check_only = 1;
    a.flag_slot = (last + 1) % kRing;
    a.in = parts(s, 0, sgrid);
    JFNK_HIP(s, launch_cg<T>(CG_P, a, tol, sgrid, s->stream));
    JFNK_HIP(s, hipMemcpyAsync(s->hcg, s->dcg, sizeof(CgCtl), hipMemcpyDeviceToHost, s->stream));
    JFNK_HIP(s, hipStreamSynchronize(s->stream));
    const CgCtl& h = *s->hcg;
    if (s->prof) prof_harvest(s, h.iters + 1);
    bo.iters = h.iters;
    bo.bnorm = h.bnorm;
    bo.res = h.res;
    bo.converged = h.state_p == kConverged;
    bo.nonfinite = h.state_p == kNonfinite;
    bo.breakdown = h.state_p == kBreakdown;
    return JFNK_OK;
  }

  // The whole solve in one workgroup (small problems, FP64/FP32).
  static bool fused_fits(const jfnk_solver* s, int m) {
    return std::is_same<T, VT>::value && fused_lds_bytes<T>(s->n, m) <= s->lds_max;
  }

  static jfnk_status newton_fused(jfnk_solver* s, double* x_user, const jfnk_options& o, jfnk_info* info) {
    FusedArgs<T> a{};
    a.nx = s->prob.nx;
    a.ny = s->prob.ny;
    a.cells = s->prob.nx * s->prob.ny;
    a.n = (int)s->n;
    a.alpha = s->alpha;
    a.cN = s->cN;
    a.beta = s->beta;
    a.coefs = s->coefs;
    a.b = static_cast<const T*>(s->b);
    a.x = x_user;
    a.history = o.history;
    a.o.m = o.m;
    a.o.max_restarts = o.max_restarts;
    a.o.max_newton = o.max_newton;
    a.o.ls_max = o.ls_max_backtracks;
    a.o.tol_k = o.tol_krylov;
    a.o.tol_n = o.tol_newton;
    a.o.ls_c = o.ls_c;
    a.o.fd_eps = o.fd_eps;
    a.o.brk = o.breakdown_tol;
    a.o.root_eps = std::sqrt(eps_mach(s->prec));
    a.o.mode = o.mode;
    a.o.eps_rule = o.eps_rule;
    a.info = s->dinfo;
    {
      ProfScope ps(s, PK_FUSED, 0.0);
      JFNK_HIP(s, launch_fused_solve<T>(s->pid, a, fused_lds_bytes<T>(s->n, o.m), s->stream));
    }
    JFNK_HIP(s, hipMemcpyAsync(s->hinfo, s->dinfo, sizeof(FusedInfo), hipMemcpyDeviceToHost, s->stream));
    JFNK_HIP(s, hipStreamSynchronize(s->stream));
    if (s->prof) prof_harvest(s, 0);
    const FusedInfo& h = *s->hinfo;
    const int k = std::min(std::max(h.newton_iters, 0), JFNK_MAX_ITERS);
    info->converged = h.converged;
    info->newton_iters = k;
    info->krylov_iters = h.krylov_iters;
    info->restarts = h.restarts;
    info->ls_backtracks = h.ls_backtracks;
    info->ls_failures = h.ls_failures;
    info->f0_norm = h.f0_norm;
    for (int i = 0; i < k; ++i) {
      info->lin_iters[i] = h.lin_iters[i];
      info->alpha[i] = h.alpha[i];
    }
    for (int i = 0; i <= k; ++i) info->rel_res[i] = h.rel_res[i];
    if (h.status == 0) return JFNK_OK;
    if (h.status == 4) return JFNK_ERR_NONFINITE;
    return JFNK_ERR_NOT_CONVERGED;
  }

  static jfnk_status newton(jfnk_solver* s, double* x_user, const jfnk_options& o, jfnk_info* info) {
    if (o.engine == JFNK_ENGINE_SINGLE_WORKGROUP && o.krylov != JFNK_KRYLOV_GMRES) {
      s->err = "the single-workgroup engine runs GMRES only";
      return JFNK_ERR_ARG;
    }
    if (o.engine == JFNK_ENGINE_SINGLE_WORKGROUP && !fused_fits(s, o.m)) {
      s->err = "the single-workgroup engine needs FP64 or FP32 and a problem that fits in LDS";
      return JFNK_ERR_ARG;
    }
    if (o.krylov == JFNK_KRYLOV_GMRES &&
        (o.engine == JFNK_ENGINE_AUTO || o.engine == JFNK_ENGINE_SINGLE_WORKGROUP) &&
        o.precond == JFNK_PRECOND_NONE && fused_fits(s, o.m))
      return newton_fused(s, x_user, o, info);
    const long long n = s->n;
    const bool f64 = std::is_same<T, double>::value;
    const int sgrid = stream_grid(s, 2);
    JFNK_HIP(s, hipMemcpyAsync(s->x64, x_user, n * sizeof(double), hipMemcpyDeviceToDevice, s->stream));
    auto cur_x = [&]() -> T* { return f64 ? reinterpret_cast<T*>(s->x64) : static_cast<T*>(s->xw); };
    if (!f64) JFNK_HIP(s, launch_cast<T>(s->npad, s->x64, static_cast<T*>(s->xw), sgrid, s->stream));
    if (o.history) JFNK_HIP(s, hipMemcpyAsync(o.history, s->x64, n * sizeof(double), hipMemcpyDeviceToDevice, s->stream));
    JFNK_TRY(residual(s, cur_x(), static_cast<T*>(s->F), true));
    JFNK_TRY(sync_read_ctl(s));
    if (s->prof) prof_harvest(s, 0);
    const double n0 = std::sqrt(s->hctl->fnorm2);
    double fk = n0;
    info->f0_norm = n0;
    int k = 0;
    jfnk_status result = JFNK_ERR_NOT_CONVERGED;
    while (true) {
      if (!std::isfinite(fk)) {
        result = JFNK_ERR_NONFINITE;
        break;
      }
      const double rho = n0 > 0.0 ? fk / n0 : 0.0;
      info->rel_res[k] = rho;
      if (rho < o.tol_newton) {
        result = JFNK_OK;
        info->converged = 1;
        break;
      }
      if (k == o.max_newton) {
        result = JFNK_ERR_NOT_CONVERGED;
        break;
      }
      GOut go;
      if (o.krylov == JFNK_KRYLOV_BICGSTAB || o.krylov == JFNK_KRYLOV_CG) {
        if constexpr (std::is_same<T, VT>::value) {
          BOut bo;
          if (o.krylov == JFNK_KRYLOV_BICGSTAB)
            JFNK_TRY(bicgstab(s, cur_x(), static_cast<const T*>(s->F), -1.0, o.tol_krylov, o.max_restarts, o.mode,
                              o.fd_eps, o.eps_rule, bo));
          else
            JFNK_TRY(cg(s, cur_x(), static_cast<const T*>(s->F), -1.0, o.tol_krylov, o.max_restarts, o.mode,
                        o.fd_eps, o.eps_rule, bo));
          go.iters = bo.iters;
          go.nonfinite = bo.nonfinite;
        }
      } else {
        JFNK_TRY(gmres(s, cur_x(), static_cast<const T*>(s->F), -1.0, o.m, o.tol_krylov, o.max_restarts, o.mode,
                       o.fd_eps, o.eps_rule, o.breakdown_tol, go, o.orth == JFNK_ORTH_DCGS2,
                       o.precond == JFNK_PRECOND_CSLP, o.mode == JFNK_JVP_AD));
      }
      info->krylov_iters += go.iters;
      info->restarts += go.cycles;
      info->lin_iters[k] = go.iters;
      if (go.nonfinite) {
        result = JFNK_ERR_NONFINITE;
        break;
      }
      double alpha = 1.0;
      double ft = 0.0;
      bool accepted = false;
      for (int t = 0; t <= o.ls_max_backtracks; ++t) {
        // the full step's trial may have been read back with the linear solve
        if (t > 0 || !go.trial_done) {
          JFNK_TRY(queue_trial(s, alpha, sgrid));
          JFNK_TRY(sync_read_ctl(s));
          if (s->prof) prof_harvest(s, 0);
        }
        ft = std::sqrt(s->hctl->fnorm2);
        if (std::isfinite(ft) && ft <= (1.0 - o.ls_c * alpha) * fk) {
          accepted = true;
          break;
        }
        if (t < o.ls_max_backtracks) {
          alpha *= 0.5;
          info->ls_backtracks += 1;
        }
      }
      if (!accepted) info->ls_failures += 1;
      info->alpha[k] = alpha;
      std::swap(s->x64, s->x64t);
      std::swap(s->xw, s->xwt);
      std::swap(s->F, s->Ft);
      fk = ft;
      k += 1;
      info->newton_iters = k;
      if (o.history)
        JFNK_HIP(s, hipMemcpyAsync(o.history + (long long)k * n, s->x64, n * sizeof(double),
                                   hipMemcpyDeviceToDevice, s->stream));
    }
    JFNK_HIP(s, hipMemcpyAsync(x_user, s->x64, n * sizeof(double), hipMemcpyDeviceToDevice, s->stream));
    JFNK_HIP(s, hipStreamSynchronize(s->stream));
    return result;
  }
};

// ---------------------------------------------------------------------------
// problem set-up
// ---------------------------------------------------------------------------
jfnk_status fill_problem(jfnk_solver* s) {
  const jfnk_problem& p = s->prob;
  Coefs& c = s->coefs;
  std::memset(&c, 0, sizeof(c));
  switch (p.id) {
    case JFNK_BURGERS1D:
      c.c[0] = 1.0 / (2.0 * p.hx);
      c.c[1] = p.p[0] / (p.hx * p.hx);
      break;
    case JFNK_BURGERS2D:
      c.c[0] = 1.0 / (2.0 * p.hx);
      c.c[1] = 1.0 / (2.0 * p.hy);
      c.c[2] = p.p[0] / (p.hx * p.hx);
      c.c[3] = p.p[0] / (p.hy * p.hy);
      break;
    case JFNK_GRAYSCOTT2D:
      c.c[0] = p.p[0] / (p.hx * p.hx);
      c.c[1] = p.p[0] / (p.hy * p.hy);
      c.c[2] = p.p[1] / (p.hx * p.hx);
      c.c[3] = p.p[1] / (p.hy * p.hy);
      c.c[4] = p.p[2] + p.p[3];
      c.c[5] = p.p[2];
      break;
    case JFNK_RD2D:
      c.c[0] = p.p[0] / (p.hx * p.hx);
      c.c[1] = p.p[0] / (p.hy * p.hy);
      break;
    case JFNK_SUOLSON2D:
      c.c[0] = 1.0 / (3.0 * p.hx * p.hx);
      c.c[1] = 1.0 / (3.0 * p.hy * p.hy);
      c.c[2] = p.p[0];
      break;
    case JFNK_MAXWELL2D:
      c.c[0] = 1.0 / (p.hx * p.hx);
      c.c[1] = 1.0 / (p.hy * p.hy);
      c.c[2] = 1.0 / (4.0 * p.hx * p.hy);
      c.c[3] = p.p[0] * p.p[0];
      c.c[4] = p.p[1];
      c.c[5] = p.p[2];
      break;
    case JFNK_KERR2D:
      c.c[0] = 1.0 / (p.hx * p.hx);
      c.c[1] = 1.0 / (p.hy * p.hy);
      c.c[2] = p.p[0] * p.p[0];
      c.c[3] = p.p[1];
      c.c[4] = p.p[2];
      c.c[5] = p.p[3];
      break;
    default:
      s->err = "unknown problem id";
      return JFNK_ERR_ARG;
  }
  if (p.id == JFNK_KERR2D || p.id == JFNK_MAXWELL2D) {
    s->alpha = 0.0;
    s->cN = 1.0;
    s->beta = -1.0;
  } else {
    s->alpha = 1.0;
    s->cN = p.theta * p.dt;
    s->beta = -1.0;
  }
  return JFNK_OK;
}

bool problem_valid(const jfnk_problem* p, std::string* why) {
  if (p == nullptr) {
    if (why) *why = "null problem";
    return false;
  }
  if (p->id < JFNK_BURGERS1D || p->id > JFNK_MAXWELL2D) {
    if (why) *why = "unknown problem id";
    return false;
  }
  if (p->nx < 3 || (p->id == JFNK_BURGERS1D ? p->ny != 1 : p->ny < 3)) {
    if (why) *why = "grid too small (nx >= 3; ny = 1 for 1D, ny >= 3 for 2D)";
    return false;
  }
  if ((long long)p->nx * p->ny > (1LL << 30)) {
    if (why) *why = "grid too large";
    return false;
  }
  if (!(p->hx > 0.0) || (p->id != JFNK_BURGERS1D && !(p->hy > 0.0))) {
    if (why) *why = "grid spacing must be positive";
    return false;
  }
  if (p->id != JFNK_KERR2D && p->id != JFNK_MAXWELL2D && (!(p->dt > 0.0) || !(p->theta > 0.0) || p->theta > 1.0)) {
    if (why) *why = "time-dependent problems need dt > 0 and 0 < theta <= 1";
    return false;
  }
  if (p->id == JFNK_SUOLSON2D && p->p[1] != 0.0 && p->p[1] != 1.0) {
    if (why) *why = "Su-Olson p[1] (periodic rows) must be 0 or 1";
    return false;
  }
  return true;
}

// Kernel dispatch kind of a problem: its public id, except the Su-Olson
// problem in its periodic-row configuration.
int problem_kind(const jfnk_problem* p) {
  if (p->id == JFNK_SUOLSON2D && p->p[1] == 1.0) return kSuOlsonPY;
  return p->id;
}

long long problem_n(const jfnk_problem* p) {
  const long long cells = (long long)p->nx * p->ny;
  if (p->id == JFNK_MAXWELL2D) return 4 * cells;
  return (p->id == JFNK_BURGERS1D || p->id == JFNK_RD2D) ? cells : 2 * cells;
}

// Upper bound on the blocks of any reducing launch: persistent stencil
// launches take at most 4 * cu blocks, Krylov launches at most cu, streaming
// ones at most 4 * cu.
size_t max_blocks(const jfnk_problem*, int cu) { return (size_t)4 * cu + 1; }

size_t elem_size(int prec) { return prec == JFNK_F64 ? 8 : 4; }
size_t basis_elem_size(int prec) { return prec == JFNK_F64 ? 8 : (prec == JFNK_F32 ? 4 : 2); }

size_t footprint(const jfnk_problem* p, int prec, int m, int cu) {
  const long long npad = round_up(problem_n(p), 256);
  const size_t t = elem_size(prec);
  size_t bytes = 0;
  bytes += (size_t)(m + 1) * (npad + kBasisPad) * basis_elem_size(prec);  // basis
  bytes += 8 * (size_t)npad * t;                            // w R dx F Ft xw xwt b
  bytes += 3 * (size_t)npad * 8;                            // x64 x64t tmp64
  bytes += 6 * max_blocks(p, cu) * kMaxCols * 8;            // partial sums
  bytes += sizeof(Ctl) + sizeof(FusedInfo) + sizeof(BiCtl) + sizeof(CgCtl);
  return bytes;
}

template <class T>
jfnk_status malloc_dev(jfnk_solver* s, T** p, size_t bytes) {
  void* q = nullptr;
  if (hipMalloc(&q, bytes) != hipSuccess) {
    s->err = "hipMalloc of " + std::to_string(bytes) + " bytes failed";
    return JFNK_ERR_OOM;
  }
  *p = static_cast<T*>(q);
  // zeroed on the solver's stream (jfnk_create synchronizes it before
  // returning): a synchronous memset would be a null-stream operation, which
  // invalidates a graph another thread is capturing at the same time
  if (hipMemsetAsync(q, 0, bytes, s->stream) != hipSuccess) {
    s->err = "hipMemsetAsync failed";
    return JFNK_ERR_HIP;
  }
  return JFNK_OK;
}

void release(jfnk_solver* s) {
  for (auto& g : s->graphs) (void)hipGraphExecDestroy(g.exec);
  s->graphs.clear();
  void* bufs[] = {s->V, s->w, s->R, s->dx, s->F, s->Ft, s->xw, s->xwt, s->b, s->x64, s->x64t, s->tmp64,
                  s->parts, s->ctl};
  for (void* p : bufs)
    if (p) (void)hipFree(p);
  if (s->hctl) (void)hipHostFree(s->hctl);
  if (s->hflags) (void)hipHostFree(s->hflags);
  if (s->hpub) (void)hipHostFree(s->hpub);
  if (s->dinfo) (void)hipFree(s->dinfo);
  if (s->hinfo) (void)hipHostFree(s->hinfo);
  if (s->dbi) (void)hipFree(s->dbi);
  if (s->hbi) (void)hipHostFree(s->hbi);
  if (s->dcg) (void)hipFree(s->dcg);
  if (s->hcg) (void)hipHostFree(s->hcg);
  for (hipEvent_t e : s->pool)
    if (e) (void)hipEventDestroy(e);
  for (ProfRec& r : s->recs) {
    (void)hipEventDestroy(r.a);
    (void)hipEventDestroy(r.b);
  }
}

// Last error of the calls that take no handle (jfnk_create,
// jfnk_newton_solve_noalloc), per thread; a fixed buffer, so that recording
// an error allocates nothing.
thread_local char g_free_error[256] = "";

void set_free_error(const char* msg) {
  std::snprintf(g_free_error, sizeof(g_free_error), "%s", msg);
}

}  // namespace

namespace {
// ||p||^2 of a caller vector into a device scalar (stream-ordered).
template <class T>
jfnk_status device_norm2(jfnk_solver* s, const T* p, double* out) {
  double* part = s->parts + 5 * s->part_rows * kMaxCols;
  const int g = stream_grid(s, 1);
  JFNK_HIP(s, launch_norm2<T>(s->n, p, PartSink{part, (int)s->part_rows}, g, s->stream));
  JFNK_HIP(s, launch_finish_sums(Partials{part, g, (int)s->part_rows}, 1, out, nullptr, s->stream));
  return JFNK_OK;
}

// Standalone JVP of an FP16S solver: the tangent is stored in FP16 with a
// power-of-two scale first (basis slot 0 holds it), as Krylov vectors are,
// and the JVP reads it from there.
jfnk_status jvp_api_f16s(jfnk_solver* s, const float* x, const float* v, float* Jv, float* F, int mode, double eps,
                         int rule) {
  EpsSpec e = eps_spec(s, eps, rule, &s->ctl->aux2);
  JFNK_TRY(device_norm2<float>(s, v, &s->ctl->aux2));
  if (mode == JFNK_JVP_FD && !(eps > 0.0)) JFNK_TRY(device_norm2<float>(s, x, &s->ctl->xnorm2));
  __half* vh = static_cast<__half*>(s->V);
  JFNK_HIP(s, launch_fp16_tangent(s->n, v, vh, &s->ctl->aux2, &s->ctl->dxnorm2, stream_grid(s, 1), s->stream));
  return Impl<float, __half>::template jvp<__half>(s, x, vh, &s->ctl->dxnorm2, Jv, mode == JFNK_JVP_AD ? F : nullptr,
                                                   mode, e);
}

template <class T>
jfnk_status jvp_api(jfnk_solver* s, const T* x, const T* v, T* Jv, T* F, int mode, double eps, int rule) {
  EpsSpec e = eps_spec(s, eps, rule, &s->ctl->aux2);
  if (mode == JFNK_JVP_FD && !(eps > 0.0)) {
    JFNK_TRY(device_norm2<T>(s, x, &s->ctl->xnorm2));
    if (rule == JFNK_EPS_NORMALIZED) JFNK_TRY(device_norm2<T>(s, v, &s->ctl->aux2));
  }
  return Impl<T, T>::template jvp<T>(s, x, v, nullptr, Jv, mode == JFNK_JVP_AD ? F : nullptr, mode, e);
}

template <class T, class VT>
jfnk_status gmres_api(jfnk_solver* s, const T* x, const T* rhs, T* dx, int m, double tol, int max_restarts, int mode,
                      double eps, int rule, jfnk_info* info) {
  const long long n = s->n;
  JFNK_HIP(s, hipMemcpyAsync(s->R, rhs, n * sizeof(T), hipMemcpyDeviceToDevice, s->stream));
  if (mode == JFNK_JVP_FD && !(eps > 0.0)) JFNK_TRY(device_norm2<T>(s, x, &s->ctl->xnorm2));
  const double brk = s->prec == JFNK_F64 ? 1e-14 : 1e-6;
  typename Impl<T, VT>::GOut go;
  JFNK_TRY(Impl<T, VT>::gmres(s, x, static_cast<const T*>(s->R), 1.0, m, tol, max_restarts, mode, eps, rule, brk, go,
                              s->orth == JFNK_ORTH_DCGS2, s->precond == JFNK_PRECOND_CSLP));
  JFNK_HIP(s, hipMemcpyAsync(dx, s->dx, n * sizeof(T), hipMemcpyDeviceToDevice, s->stream));
  JFNK_HIP(s, hipStreamSynchronize(s->stream));
  if (info) {
    info->converged = go.converged ? 1 : 0;
    info->krylov_iters = go.iters;
    info->restarts = go.cycles;
    info->final_res = go.true_res;
    info->f0_norm = go.bnorm;
    info->status = go.nonfinite ? JFNK_ERR_NONFINITE : JFNK_OK;
  }
  return go.nonfinite ? JFNK_ERR_NONFINITE : JFNK_OK;
}
template <class T>
jfnk_status short_recurrence_api(jfnk_solver* s, int krylov, const T* x, const T* rhs, T* dx, double tol,
                                 int max_iters, int mode, double eps, int rule, jfnk_info* info) {
  const long long n = s->n;
  JFNK_HIP(s, hipMemcpyAsync(s->R, rhs, n * sizeof(T), hipMemcpyDeviceToDevice, s->stream));
  if (mode == JFNK_JVP_FD && !(eps > 0.0)) JFNK_TRY(device_norm2<T>(s, x, &s->ctl->xnorm2));
  typename Impl<T, T>::BOut bo;
  if (krylov == JFNK_KRYLOV_CG)
    JFNK_TRY(Impl<T, T>::cg(s, x, static_cast<const T*>(s->R), 1.0, tol, max_iters, mode, eps, rule, bo));
  else
    JFNK_TRY(Impl<T, T>::bicgstab(s, x, static_cast<const T*>(s->R), 1.0, tol, max_iters, mode, eps, rule, bo));
  JFNK_HIP(s, hipMemcpyAsync(dx, s->dx, n * sizeof(T), hipMemcpyDeviceToDevice, s->stream));
  JFNK_HIP(s, hipStreamSynchronize(s->stream));
  const jfnk_status st = bo.nonfinite ? JFNK_ERR_NONFINITE : (bo.breakdown ? JFNK_ERR_BREAKDOWN : JFNK_OK);
  if (info) {
    info->converged = bo.converged ? 1 : 0;
    info->krylov_iters = bo.iters;
    info->final_res = bo.res;
    info->f0_norm = bo.bnorm;
    info->status = st;
  }
  return st;
}

// The CSLP preconditioner: the Maxwell-Kerr problem and the Helmholtz-Kerr
// workload (the same construction on the scalar operator), with GMRES on the
// multi-kernel engine; the FD JVP takes the paper's step rule (the
// normalized rule would need the norm of M^{-1} v).
bool precond_ok(const jfnk_solver* s, int precond, int krylov, int engine, int mode, int eps_rule, double fd_eps,
                std::string* why) {
  if (precond == JFNK_PRECOND_NONE) return true;
  if (precond != JFNK_PRECOND_CSLP) {
    *why = "unknown preconditioner";
    return false;
  }
  if (s->pid != kMaxwell && s->pid != kKerr) {
    *why = "the CSLP preconditioner is defined for the Maxwell-Kerr and Helmholtz-Kerr problems only";
    return false;
  }
  if (krylov != JFNK_KRYLOV_GMRES || engine == JFNK_ENGINE_SINGLE_WORKGROUP) {
    *why = "the CSLP preconditioner runs with GMRES on the multi-kernel engine";
    return false;
  }
  if (mode == JFNK_JVP_FD && eps_rule == JFNK_EPS_NORMALIZED && !(fd_eps > 0.0)) {
    *why = "the CSLP preconditioner takes the paper's FD step rule (or a fixed step)";
    return false;
  }
  return true;
}

// BiCGSTAB keeps r^, r, p, v, s, t in the first six basis slots, CG r, p,
// J p in the first three.
bool short_recurrence_fits(const jfnk_solver* s, int krylov, std::string* why) {
  const char* name = krylov == JFNK_KRYLOV_CG ? "CG" : "BiCGSTAB";
  if (s->prec == JFNK_F16S) {
    *why = std::string(name) + " runs in FP64 or FP32 (FP16 storage applies to the GMRES basis only)";
    return false;
  }
  const int need = krylov == JFNK_KRYLOV_CG ? 2 : 5;
  if (s->m < need) {
    *why = std::string(name) + " needs a solver created with m >= " + std::to_string(need) + " (" +
           std::to_string(need + 1) + " work vectors)";
    return false;
  }
  return true;
}
}  // namespace

namespace {
jfnk_status short_recurrence_entry(jfnk_solver* s, int krylov, const void* x, const void* rhs, void* dx,
                                   double tol, int max_iters, int mode, double eps, int eps_rule, jfnk_info* info) {
  if (!s || !x || !rhs || !dx) return JFNK_ERR_ARG;
  if (max_iters < 0 || !(tol >= 0.0)) {
    s->err = "max_iters >= 0 and tol >= 0 are required";
    return JFNK_ERR_ARG;
  }
  if ((mode != JFNK_JVP_AD && mode != JFNK_JVP_FD) || (eps_rule != JFNK_EPS_PAPER && eps_rule != JFNK_EPS_NORMALIZED))
    return JFNK_ERR_ARG;
  if (!s->has_prev) {
    s->err = "jfnk_set_previous must be called first";
    return JFNK_ERR_ARG;
  }
  if (!short_recurrence_fits(s, krylov, &s->err)) return JFNK_ERR_ARG;
  if (info) std::memset(info, 0, sizeof(*info));
  const auto t0 = std::chrono::steady_clock::now();
  jfnk_status st;
  if (s->prec == JFNK_F64)
    st = short_recurrence_api<double>(s, krylov, (const double*)x, (const double*)rhs, (double*)dx, tol, max_iters,
                                      mode, eps, eps_rule, info);
  else
    st = short_recurrence_api<float>(s, krylov, (const float*)x, (const float*)rhs, (float*)dx, tol, max_iters,
                                     mode, eps, eps_rule, info);
  if (info) info->seconds = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
  return st;
}
}  // namespace

// ===========================================================================
// C ABI
// ===========================================================================
extern "C" {

size_t jfnk_problem_size(const jfnk_problem* problem) {
  if (!problem_valid(problem, nullptr)) return 0;
  return (size_t)problem_n(problem);
}

size_t jfnk_footprint_bytes(const jfnk_problem* problem, int precision, int m) {
  if (!problem_valid(problem, nullptr) || m < 1 || m > kMaxM) return 0;
  if (precision < JFNK_F64 || precision > JFNK_F16S) return 0;
  return footprint(problem, precision, m, 256);
}

void jfnk_default_options(int precision, jfnk_options* o) {
  if (!o) return;
  std::memset(o, 0, sizeof(*o));
  o->m = 30;
  o->max_restarts = 100;
  o->max_newton = 15;
  o->ls_max_backtracks = 10;
  o->ls_c = 1e-4;
  o->mode = JFNK_JVP_AD;
  o->eps_rule = JFNK_EPS_PAPER;
  o->engine = JFNK_ENGINE_AUTO;
  o->orth = JFNK_ORTH_DCGS2;
  if (precision == JFNK_F64) {
    o->tol_newton = 1e-6;
    o->tol_krylov = 1e-8;
    o->breakdown_tol = 1e-14;
  } else {
    o->tol_newton = 1e-4;
    o->tol_krylov = 1e-6;
    o->breakdown_tol = 1e-6;
  }
}

const char* jfnk_status_string(int status) {
  switch (status) {
    case JFNK_OK: return "ok";
    case JFNK_ERR_ARG: return "invalid argument";
    case JFNK_ERR_OOM: return "out of device memory";
    case JFNK_ERR_HIP: return "HIP runtime error";
    case JFNK_ERR_NONFINITE: return "non-finite value";
    case JFNK_ERR_BREAKDOWN: return "Krylov breakdown";
    case JFNK_ERR_NOT_CONVERGED: return "not converged";
    default: return "unknown status";
  }
}

const char* jfnk_last_error(const jfnk_solver* s) {
  if (!s) return g_free_error;
  return s->err.c_str();
}

jfnk_status jfnk_create(const jfnk_problem* problem, int precision, int m, void* hip_stream, jfnk_solver** out) {
  if (!out) return JFNK_ERR_ARG;
  *out = nullptr;
  std::string why;
  if (!problem_valid(problem, &why)) {
    set_free_error(why.c_str());
    return JFNK_ERR_ARG;
  }
  if (precision != JFNK_F64 && precision != JFNK_F32 && precision != JFNK_F16S) {
    set_free_error("unknown precision");
    return JFNK_ERR_ARG;
  }
  if (m < 1 || m > kMaxM) {
    set_free_error("m must be in 1..32");
    return JFNK_ERR_ARG;
  }
  jfnk_solver* s = new jfnk_solver();
  s->prob = *problem;
  s->prec = precision;
  s->m = m;
  s->stream = static_cast<hipStream_t>(hip_stream);
  s->pid = problem_kind(problem);
  s->n = problem_n(problem);
  s->npad = round_up(s->n, 256);
  s->vstride = s->npad + kBasisPad;
  s->tsize = elem_size(precision);
  s->vsize = basis_elem_size(precision);
  s->orth = JFNK_ORTH_DCGS2;
  int dev = 0;
  hipDeviceProp_t prop{};
  if (hipGetDevice(&dev) == hipSuccess && hipGetDeviceProperties(&prop, dev) == hipSuccess &&
      prop.multiProcessorCount > 0)
    s->cu = prop.multiProcessorCount;
  {
    int lds = 0;
    if (hipDeviceGetAttribute(&lds, hipDeviceAttributeMaxSharedMemoryPerBlock, dev) == hipSuccess && lds > 0)
      s->lds_max = (size_t)lds;
  }
  jfnk_status st = fill_problem(s);
  const size_t vec_bytes = (size_t)s->npad * s->tsize;
  if (st == JFNK_OK) st = malloc_dev(s, &s->V, (size_t)(m + 1) * s->vstride * s->vsize);
  void** tv[] = {&s->w, &s->R, &s->dx, &s->F, &s->Ft, &s->xw, &s->xwt, &s->b};
  for (void** p : tv)
    if (st == JFNK_OK) st = malloc_dev(s, p, vec_bytes);
  if (st == JFNK_OK) st = malloc_dev(s, &s->x64, (size_t)s->npad * 8);
  if (st == JFNK_OK) st = malloc_dev(s, &s->x64t, (size_t)s->npad * 8);
  if (st == JFNK_OK) st = malloc_dev(s, &s->tmp64, (size_t)s->npad * 8);
  s->part_rows = max_blocks(problem, s->cu);
  if (st == JFNK_OK) st = malloc_dev(s, &s->parts, 6 * s->part_rows * kMaxCols * sizeof(double));
  if (st == JFNK_OK) st = malloc_dev(s, &s->ctl, sizeof(Ctl));
  if (st == JFNK_OK) st = malloc_dev(s, &s->dinfo, sizeof(FusedInfo));
  if (st == JFNK_OK) st = malloc_dev(s, &s->dbi, sizeof(BiCtl));
  if (st == JFNK_OK) st = malloc_dev(s, &s->dcg, sizeof(CgCtl));
  if (st == JFNK_OK) {
    void* h = nullptr;
    if (hipHostMalloc(&h, sizeof(CgCtl), hipHostMallocDefault) != hipSuccess) {
      s->err = "hipHostMalloc (CG scalars) failed";
      st = JFNK_ERR_OOM;
    } else {
      s->hcg = static_cast<CgCtl*>(h);
    }
  }
  if (st == JFNK_OK) {
    void* h = nullptr;
    if (hipHostMalloc(&h, sizeof(BiCtl), hipHostMallocDefault) != hipSuccess) {
      s->err = "hipHostMalloc (BiCGSTAB scalars) failed";
      st = JFNK_ERR_OOM;
    } else {
      s->hbi = static_cast<BiCtl*>(h);
    }
  }
  if (st == JFNK_OK) {
    void* h = nullptr;
    if (hipHostMalloc(&h, sizeof(FusedInfo), hipHostMallocDefault) != hipSuccess) {
      s->err = "hipHostMalloc (info) failed";
      st = JFNK_ERR_OOM;
    } else {
      s->hinfo = static_cast<FusedInfo*>(h);
    }
  }
  if (st == JFNK_OK) {
    void* h = nullptr;
    // two control blocks: the head mirror, then a whole-block copy for jfnk_gmres_hessenberg
    if (hipHostMalloc(&h, 2 * sizeof(Ctl), hipHostMallocDefault) != hipSuccess) {
      s->err = "hipHostMalloc failed";
      st = JFNK_ERR_OOM;
    } else {
      s->hctl = static_cast<Ctl*>(h);
      std::memset(s->hctl, 0, 2 * sizeof(Ctl));
    }
  }
  if (st == JFNK_OK) {
    void* h = nullptr;
    if (hipHostMalloc(&h, sizeof(int) * (kMaxM + 1), hipHostMallocMapped | hipHostMallocCoherent) != hipSuccess) {
      s->err = "hipHostMalloc (flags) failed";
      st = JFNK_ERR_OOM;
    } else {
      s->hflags = static_cast<int*>(h);
      void* d = nullptr;
      if (hipHostGetDevicePointer(&d, h, 0) != hipSuccess) {
        s->err = "hipHostGetDevicePointer failed";
        st = JFNK_ERR_HIP;
      }
      s->dflags = static_cast<int*>(d);
    }
  }
  if (st == JFNK_OK) {
    void* h = nullptr;
    if (hipHostMalloc(&h, sizeof(int) * (kPubWords + 1), hipHostMallocMapped | hipHostMallocCoherent) != hipSuccess) {
      s->err = "hipHostMalloc (published control block) failed";
      st = JFNK_ERR_OOM;
    } else {
      s->hpub = static_cast<int*>(h);
      std::memset(h, 0, sizeof(int) * (kPubWords + 1));
      void* d = nullptr;
      if (hipHostGetDevicePointer(&d, h, 0) != hipSuccess) {
        s->err = "hipHostGetDevicePointer failed";
        st = JFNK_ERR_HIP;
      }
      s->dpub = static_cast<int*>(d);
    }
  }
  if (st == JFNK_OK && hipStreamSynchronize(s->stream) != hipSuccess) {
    s->err = "stream synchronize after set-up failed";
    st = JFNK_ERR_HIP;
  }
  if (st != JFNK_OK) {
    set_free_error(s->err.c_str());
    release(s);
    delete s;
    return st;
  }
  *out = s;
  return JFNK_OK;
}

jfnk_status jfnk_set_orthogonalization(jfnk_solver* s, int orth) {
  if (!s) return JFNK_ERR_ARG;
  if (orth != JFNK_ORTH_CGS2 && orth != JFNK_ORTH_DCGS2) {
    s->err = "unknown Gram-Schmidt form";
    return JFNK_ERR_ARG;
  }
  s->orth = orth;
  return JFNK_OK;
}

jfnk_status jfnk_set_preconditioner(jfnk_solver* s, int precond) {
  if (!s) return JFNK_ERR_ARG;
  if (precond != JFNK_PRECOND_NONE &&
      !precond_ok(s, precond, JFNK_KRYLOV_GMRES, JFNK_ENGINE_MULTI_KERNEL, JFNK_JVP_AD, JFNK_EPS_PAPER, 0.0, &s->err))
    return JFNK_ERR_ARG;
  s->precond = precond;
  return JFNK_OK;
}

jfnk_status jfnk_set_stream(jfnk_solver* s, void* hip_stream) {
  if (!s) return JFNK_ERR_ARG;
  s->stream = static_cast<hipStream_t>(hip_stream);
  return JFNK_OK;
}

jfnk_status jfnk_destroy(jfnk_solver* s) {
  if (!s) return JFNK_ERR_ARG;
  if (s->stream) (void)hipStreamSynchronize(s->stream);
  release(s);
  delete s;
  return JFNK_OK;
}

jfnk_status jfnk_set_previous(jfnk_solver* s, const double* x_prev, const double* source) {
  if (!s) return JFNK_ERR_ARG;
  const jfnk_problem& p = s->prob;
  const long long n = s->n;
  const int sgrid = stream_grid(s, 2);
  if (p.id == JFNK_KERR2D || p.id == JFNK_MAXWELL2D) {
    // b = f (the source), cast to the working precision
    if (source == nullptr) {
      if (s->prec == JFNK_F64)
        JFNK_HIP(s, launch_fill_zero<double>(s->npad, static_cast<double*>(s->b), sgrid, s->stream));
      else
        JFNK_HIP(s, launch_fill_zero<float>(s->npad, static_cast<float*>(s->b), sgrid, s->stream));
    } else if (s->prec == JFNK_F64) {
      JFNK_HIP(s, hipMemcpyAsync(s->b, source, n * 8, hipMemcpyDeviceToDevice, s->stream));
    } else {
      JFNK_HIP(s, hipMemcpyAsync(s->tmp64, source, n * 8, hipMemcpyDeviceToDevice, s->stream));
      JFNK_HIP(s, launch_cast<float>(s->npad, s->tmp64, static_cast<float*>(s->b), sgrid, s->stream));
    }
    s->has_prev = true;
    return JFNK_OK;
  }
  if (x_prev == nullptr) {
    s->err = "x_prev is required for time-dependent problems";
    return JFNK_ERR_ARG;
  }
  // b = x^n - (1 - theta) dt N(x^n) + dt s, evaluated in FP64
  StencilArgs<double, double> a{};
  a.nx = p.nx;
  a.ny = p.ny;
  a.plane = (long long)p.nx * p.ny;
  a.x = x_prev;
  a.b = source;
  a.alpha = 1.0;
  a.cN = -(1.0 - p.theta) * p.dt;
  a.beta = p.dt;
  a.nred = 0;
  double* dst = s->prec == JFNK_F64 ? static_cast<double*>(s->b) : s->tmp64;
  a.out = dst;
  const int vec = stencil_vec<double>(s->pid);
  const bool vz = (p.nx % vec == 0) && aligned(x_prev, 16) && aligned(source, 16);
  JFNK_HIP(s, launch_stencil<double, double>(s->pid, OP_RES, false, vz, a, s->coefs, kNoCap, s->stream));
  if (s->prec != JFNK_F64)
    JFNK_HIP(s, launch_cast<float>(s->npad, s->tmp64, static_cast<float*>(s->b), sgrid, s->stream));
  s->has_prev = true;
  return JFNK_OK;
}

jfnk_status jfnk_residual(jfnk_solver* s, const void* x, void* F) {
  if (!s || !x || !F) return JFNK_ERR_ARG;
  if (!s->has_prev) {
    s->err = "jfnk_set_previous must be called first";
    return JFNK_ERR_ARG;
  }
  if (s->prec == JFNK_F64) return Impl<double, double>::residual(s, (const double*)x, (double*)F, false);
  return Impl<float, float>::residual(s, (const float*)x, (float*)F, false);
}


jfnk_status jfnk_jvp(jfnk_solver* s, const void* x, const void* v, void* Jv, void* F_or_null, int mode, double eps,
                     int eps_rule) {
  if (!s || !x || !v || !Jv) return JFNK_ERR_ARG;
  if (mode != JFNK_JVP_AD && mode != JFNK_JVP_FD) return JFNK_ERR_ARG;
  if (eps_rule != JFNK_EPS_PAPER && eps_rule != JFNK_EPS_NORMALIZED) return JFNK_ERR_ARG;
  if (!s->has_prev) {
    s->err = "jfnk_set_previous must be called first";
    return JFNK_ERR_ARG;
  }
  if (s->prec == JFNK_F64)
    return jvp_api<double>(s, (const double*)x, (const double*)v, (double*)Jv, (double*)F_or_null, mode, eps,
                           eps_rule);
  if (s->prec == JFNK_F16S)
    return jvp_api_f16s(s, (const float*)x, (const float*)v, (float*)Jv, (float*)F_or_null, mode, eps, eps_rule);
  return jvp_api<float>(s, (const float*)x, (const float*)v, (float*)Jv, (float*)F_or_null, mode, eps, eps_rule);
}

jfnk_status jfnk_gmres(jfnk_solver* s, const void* x, const void* rhs, void* dx, int m, double tol, int max_restarts,
                       int mode, double eps, int eps_rule, jfnk_info* info) {
  if (!s || !x || !rhs || !dx) return JFNK_ERR_ARG;
  if (m < 1 || m > s->m || max_restarts < 0 || !(tol >= 0.0)) {
    s->err = "m must be in 1..(solver m), max_restarts >= 0, tol >= 0";
    return JFNK_ERR_ARG;
  }
  if (mode != JFNK_JVP_AD && mode != JFNK_JVP_FD) return JFNK_ERR_ARG;
  if (!s->has_prev) {
    s->err = "jfnk_set_previous must be called first";
    return JFNK_ERR_ARG;
  }
  if (!precond_ok(s, s->precond, JFNK_KRYLOV_GMRES, JFNK_ENGINE_MULTI_KERNEL, mode, eps_rule, eps, &s->err))
    return JFNK_ERR_ARG;
  if (info) std::memset(info, 0, sizeof(*info));
  const auto t0 = std::chrono::steady_clock::now();
  jfnk_status st;
  if (s->prec == JFNK_F64)
    st = gmres_api<double, double>(s, (const double*)x, (const double*)rhs, (double*)dx, m, tol, max_restarts, mode,
                                   eps, eps_rule, info);
  else if (s->prec == JFNK_F32)
    st = gmres_api<float, float>(s, (const float*)x, (const float*)rhs, (float*)dx, m, tol, max_restarts, mode, eps,
                                 eps_rule, info);
  else
    st = gmres_api<float, __half>(s, (const float*)x, (const float*)rhs, (float*)dx, m, tol, max_restarts, mode, eps,
                                  eps_rule, info);
  if (info) info->seconds = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
  return st;
}

jfnk_status jfnk_gmres_hessenberg(jfnk_solver* s, double* H, int ldh, int* k_out) {
  if (!s || !k_out) return JFNK_ERR_ARG;
  Ctl* c = s->hctl + 1;  // host scratch behind the head mirror
  JFNK_HIP(s, hipMemcpyAsync(c, s->ctl, sizeof(Ctl), hipMemcpyDeviceToHost, s->stream));
  JFNK_HIP(s, hipStreamSynchronize(s->stream));
  const int k = c->k_last;
  *k_out = k;
  if (k == 0) return JFNK_OK;
  if (!H || ldh < k + 1) {
    s->err = "H must hold (k + 1) x k doubles with ldh >= k + 1";
    return JFNK_ERR_ARG;
  }
  const int ld = kMaxM + 1;
  for (int l = 0; l < k; ++l)
    for (int i = 0; i <= k; ++i) H[(size_t)l * ldh + i] = i <= l + 1 ? c->Hu[l * ld + i] : 0.0;
  return JFNK_OK;
}

jfnk_status jfnk_bicgstab(jfnk_solver* s, const void* x, const void* rhs, void* dx, double tol, int max_iters,
                          int mode, double eps, int eps_rule, jfnk_info* info) {
  return short_recurrence_entry(s, JFNK_KRYLOV_BICGSTAB, x, rhs, dx, tol, max_iters, mode, eps, eps_rule, info);
}

jfnk_status jfnk_cg(jfnk_solver* s, const void* x, const void* rhs, void* dx, double tol, int max_iters, int mode,
                    double eps, int eps_rule, jfnk_info* info) {
  return short_recurrence_entry(s, JFNK_KRYLOV_CG, x, rhs, dx, tol, max_iters, mode, eps, eps_rule, info);
}

jfnk_status jfnk_newton_solve(jfnk_solver* s, double* x_inout, const jfnk_options* opts, jfnk_info* info) {
  if (!s || !x_inout || !opts || !info) return JFNK_ERR_ARG;
  const jfnk_options& o = *opts;
  if (o.m < 1 || o.m > s->m || o.max_newton < 0 || o.max_newton > JFNK_MAX_ITERS || o.max_restarts < 0 ||
      o.ls_max_backtracks < 0 || (o.mode != JFNK_JVP_AD && o.mode != JFNK_JVP_FD) ||
      (o.eps_rule != JFNK_EPS_PAPER && o.eps_rule != JFNK_EPS_NORMALIZED) || !(o.tol_krylov >= 0.0) ||
      o.engine < JFNK_ENGINE_AUTO || o.engine > JFNK_ENGINE_MULTI_KERNEL_GRAPH ||
      o.krylov < JFNK_KRYLOV_GMRES || o.krylov > JFNK_KRYLOV_CG || o.orth < JFNK_ORTH_CGS2 ||
      o.orth > JFNK_ORTH_DCGS2) {
    s->err = "invalid options";
    return JFNK_ERR_ARG;
  }
  if (o.engine == JFNK_ENGINE_MULTI_KERNEL_GRAPH && o.krylov != JFNK_KRYLOV_GMRES) {
    s->err = "the graph engine replays GMRES cycles (BiCGSTAB and CG run on the multi-kernel engine)";
    return JFNK_ERR_ARG;
  }
  if (o.krylov != JFNK_KRYLOV_GMRES && !short_recurrence_fits(s, o.krylov, &s->err)) return JFNK_ERR_ARG;
  if (!precond_ok(s, o.precond, o.krylov, o.engine, o.mode, o.eps_rule, o.fd_eps, &s->err)) return JFNK_ERR_ARG;
  if (!s->has_prev) {
    s->err = "jfnk_set_previous must be called first";
    return JFNK_ERR_ARG;
  }
  std::memset(info, 0, sizeof(*info));
  const auto t0 = std::chrono::steady_clock::now();
  jfnk_status st;
  s->graph = o.engine == JFNK_ENGINE_MULTI_KERNEL_GRAPH;
  if (s->prec == JFNK_F64)
    st = Impl<double, double>::newton(s, x_inout, o, info);
  else if (s->prec == JFNK_F32)
    st = Impl<float, float>::newton(s, x_inout, o, info);
  else
    st = Impl<float, __half>::newton(s, x_inout, o, info);
  s->graph = false;
  info->status = st;
  info->seconds = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
  return st;
}

}  // extern "C"

// ---------------------------------------------------------------------------
// Newton solve without allocation (single-workgroup engine)
// ---------------------------------------------------------------------------
namespace {

// Device workspace of jfnk_newton_solve_noalloc: the solve record, then the
// constant part in FP64 and in the working precision, for at most
// kNoAllocMaxN unknowns.  One copy per GPU, held until the process ends;
// every call on a GPU shares it.
constexpr long long kNoAllocMaxN = 4096;
constexpr size_t kNoAllocInfoBytes = 4096;
constexpr size_t kNoAllocScratchBytes = kNoAllocInfoBytes + 2 * (size_t)kNoAllocMaxN * sizeof(double);
static_assert(sizeof(FusedInfo) <= kNoAllocInfoBytes, "solve record must fit its slot");

static __device__ __align__(256) unsigned char scratch[kNoAllocScratchBytes];

// Per device: the address of `scratch` (from hipGetSymbolAddress; the array's
// name is not a device address in host code), its compute units and LDS size.
constexpr int kNoAllocMaxDevices = 64;
struct NoAllocDevice {
  unsigned char* ptr = nullptr;
  int cu = 0;
  size_t lds = 0;
};
NoAllocDevice g_noalloc_dev[kNoAllocMaxDevices];
std::mutex g_noalloc_mu;

// Set-up on the first call on a device, with that device current.
bool noalloc_device(NoAllocDevice* out) {
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= kNoAllocMaxDevices) {
    set_free_error("no current HIP device (or device index above 63)");
    return false;
  }
  std::lock_guard<std::mutex> lock(g_noalloc_mu);
  NoAllocDevice& d = g_noalloc_dev[dev];
  if (d.ptr == nullptr) {
    void* ptr = nullptr;
    const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    if (e != hipSuccess || ptr == nullptr) {
      set_free_error("hipGetSymbolAddress of the static workspace failed");
      return false;
    }
    int cu = 0, lds = 0;
    if (hipDeviceGetAttribute(&cu, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || cu <= 0 ||
        hipDeviceGetAttribute(&lds, hipDeviceAttributeMaxSharedMemoryPerBlock, dev) != hipSuccess || lds <= 0) {
      set_free_error("device attribute query failed");
      return false;
    }
    d.cu = cu;
    d.lds = (size_t)lds;
    d.ptr = static_cast<unsigned char*>(ptr);
  }
  *out = d;
  return true;
}

}  // namespace

extern "C" {

jfnk_status jfnk_newton_solve_noalloc(const jfnk_problem* problem, int precision, const double* x_prev,
                                      const double* source, double* x_inout, const jfnk_options* opts,
                                      jfnk_info* info, void* hip_stream) {
  if (!problem || !x_inout || !opts || !info) {
    set_free_error("problem, x_inout, opts and info are required");
    return JFNK_ERR_ARG;
  }
  std::string why;
  if (!problem_valid(problem, &why)) {
    set_free_error(why.c_str());
    return JFNK_ERR_ARG;
  }
  if (precision != JFNK_F64 && precision != JFNK_F32) {
    set_free_error("the allocation-free solve runs in FP64 or FP32");
    return JFNK_ERR_ARG;
  }
  const jfnk_options& o = *opts;
  if (o.m < 1 || o.m > kMaxM || o.max_newton < 0 || o.max_newton > JFNK_MAX_ITERS || o.max_restarts < 0 ||
      o.ls_max_backtracks < 0 || (o.mode != JFNK_JVP_AD && o.mode != JFNK_JVP_FD) ||
      (o.eps_rule != JFNK_EPS_PAPER && o.eps_rule != JFNK_EPS_NORMALIZED) || !(o.tol_krylov >= 0.0)) {
    set_free_error("invalid options");
    return JFNK_ERR_ARG;
  }
  if (o.krylov != JFNK_KRYLOV_GMRES || o.engine == JFNK_ENGINE_MULTI_KERNEL ||
      o.engine == JFNK_ENGINE_MULTI_KERNEL_GRAPH || o.precond != JFNK_PRECOND_NONE) {
    set_free_error("the allocation-free solve runs GMRES on the single-workgroup engine, unpreconditioned");
    return JFNK_ERR_ARG;
  }
  const long long n = problem_n(problem);
  if (n > kNoAllocMaxN) {
    set_free_error("problem exceeds the 4096 unknowns of the allocation-free solve's static workspace");
    return JFNK_ERR_ARG;
  }
  const bool bvp = problem->id == JFNK_KERR2D || problem->id == JFNK_MAXWELL2D;
  if (!bvp && x_prev == nullptr) {
    set_free_error("x_prev is required for time-dependent problems");
    return JFNK_ERR_ARG;
  }
  NoAllocDevice d;
  if (!noalloc_device(&d)) return JFNK_ERR_HIP;
  const size_t need = precision == JFNK_F64 ? fused_lds_bytes<double>(n, o.m) : fused_lds_bytes<float>(n, o.m);
  if (need > d.lds) {
    set_free_error("problem does not fit the single-workgroup engine's LDS");
    return JFNK_ERR_ARG;
  }
  // a handle on the stack whose workspace pointers point into the static
  // array (constant part in FP64, then in the working precision; the solve
  // record, fully written by the solve kernel before the host reads it)
  FusedInfo hrec{};
  jfnk_solver loc;
  loc.prob = *problem;
  loc.prec = precision;
  loc.m = o.m;
  loc.stream = static_cast<hipStream_t>(hip_stream);
  loc.pid = problem_kind(problem);
  loc.n = n;
  loc.npad = round_up(n, 256);
  loc.vstride = loc.npad;
  loc.tsize = elem_size(precision);
  loc.vsize = loc.tsize;
  loc.cu = d.cu;
  loc.lds_max = d.lds;
  loc.dinfo = reinterpret_cast<FusedInfo*>(d.ptr);
  loc.hinfo = &hrec;
  loc.tmp64 = reinterpret_cast<double*>(d.ptr + kNoAllocInfoBytes);
  loc.b = d.ptr + kNoAllocInfoBytes + (size_t)kNoAllocMaxN * sizeof(double);
  jfnk_status st = fill_problem(&loc);
  if (st == JFNK_OK) st = jfnk_set_previous(&loc, x_prev, source);
  if (st == JFNK_OK) {
    std::memset(info, 0, sizeof(*info));
    const auto t0 = std::chrono::steady_clock::now();
    if (precision == JFNK_F64)
      st = Impl<double, double>::newton_fused(&loc, x_inout, o, info);
    else
      st = Impl<float, float>::newton_fused(&loc, x_inout, o, info);
    info->status = st;
    info->seconds = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
  }
  if (st != JFNK_OK && st != JFNK_ERR_NOT_CONVERGED && st != JFNK_ERR_NONFINITE) set_free_error(loc.err.c_str());
  return st;
}

jfnk_status jfnk_profile_enable(jfnk_solver* s, int on) {
  if (!s) return JFNK_ERR_ARG;
  if (!on && s->prof) {
    JFNK_HIP(s, hipStreamSynchronize(s->stream));
    prof_harvest(s, 1 << 30);
  }
  s->prof = on != 0;
  return JFNK_OK;
}

jfnk_status jfnk_profile_read(jfnk_solver* s, int kernel, long long* launches, double* total_ms, double* bytes) {
  if (!s || kernel < 0 || kernel >= kNumProf) return JFNK_ERR_ARG;
  JFNK_HIP(s, hipStreamSynchronize(s->stream));
  prof_harvest(s, 1 << 30);
  if (launches) *launches = s->p_count[kernel];
  if (total_ms) *total_ms = s->p_ms[kernel];
  if (bytes) *bytes = s->p_bytes[kernel];
  return JFNK_OK;
}

jfnk_status jfnk_profile_reset(jfnk_solver* s) {
  if (!s) return JFNK_ERR_ARG;
  JFNK_HIP(s, hipStreamSynchronize(s->stream));
  prof_harvest(s, 1 << 30);
  for (int i = 0; i < kNumProf; ++i) {
    s->p_count[i] = 0;
    s->p_ms[i] = 0.0;
    s->p_bytes[i] = 0.0;
  }
  return JFNK_OK;
}

int jfnk_cycle_graphs(const jfnk_solver* s) { return s ? (int)s->graphs.size() : -1; }

jfnk_status jfnk_frequency_sweep(const jfnk_problem* problems, const double* const* sources, int count,
                                 int precision, const jfnk_options* opts, void* hip_stream, double* fields,
                                 jfnk_info* infos, int* run_failed) {
  if (!problems || count < 1 || !opts || !fields || !run_failed) {
    set_free_error("jfnk_frequency_sweep: null argument or count < 1");
    return JFNK_ERR_ARG;
  }
  const size_t n = jfnk_problem_size(&problems[0]);
  for (int i = 0; i < count; ++i)
    if (n == 0 || jfnk_problem_size(&problems[i]) != n) {
      set_free_error("jfnk_frequency_sweep: the problems differ in size or are invalid");
      return JFNK_ERR_ARG;
    }
  hipStream_t st = static_cast<hipStream_t>(hip_stream);
  const size_t vb = n * sizeof(double);
  double* d_x = nullptr;
  double* d_src = nullptr;
  if (hipMalloc(&d_x, vb) != hipSuccess || hipMalloc(&d_src, vb) != hipSuccess) {
    if (d_x) (void)hipFree(d_x);
    set_free_error("jfnk_frequency_sweep: device allocation failed");
    return JFNK_ERR_OOM;
  }
  const std::vector<double> zeros(n, 0.0);
  jfnk_status out = JFNK_OK;
  int failed = 0;
  bool have_prev = false;  // d_x holds the previous frequency's converged field
  for (int i = 0; i < count && out == JFNK_OK; ++i) {
    jfnk_solver* s = nullptr;
    jfnk_status rc = jfnk_create(&problems[i], precision, opts->m, hip_stream, &s);
    if (rc != JFNK_OK) {
      out = rc;
      break;
    }
    const double* src = (sources && sources[i]) ? sources[i] : nullptr;
    if (src && hipMemcpyAsync(d_src, src, vb, hipMemcpyHostToDevice, st) != hipSuccess) rc = JFNK_ERR_HIP;
    if (rc == JFNK_OK) rc = jfnk_set_previous(s, nullptr, src ? d_src : nullptr);
    if (rc == JFNK_OK && !have_prev &&
        hipMemcpyAsync(d_x, zeros.data(), vb, hipMemcpyHostToDevice, st) != hipSuccess)
      rc = JFNK_ERR_HIP;
    jfnk_info info{};
    if (rc == JFNK_OK) {
      rc = jfnk_newton_solve(s, d_x, opts, &info);
      const bool ran = rc == JFNK_OK || rc == JFNK_ERR_NOT_CONVERGED || rc == JFNK_ERR_NONFINITE ||
                       rc == JFNK_ERR_BREAKDOWN;
      if (ran) {
        if (hipMemcpyAsync(fields + (size_t)i * n, d_x, vb, hipMemcpyDeviceToHost, st) != hipSuccess ||
            hipStreamSynchronize(st) != hipSuccess) {
          rc = JFNK_ERR_HIP;
        } else {
          if (infos) infos[i] = info;
          const bool conv = rc == JFNK_OK && info.converged;
          failed += conv ? 0 : 1;
          have_prev = conv;
          rc = JFNK_OK;
        }
      }
    }
    if (rc != JFNK_OK) {
      set_free_error(jfnk_last_error(s));
      out = rc;
    }
    (void)jfnk_destroy(s);
  }
  (void)hipFree(d_x);
  (void)hipFree(d_src);
  if (out == JFNK_OK) *run_failed = 5 * failed > count ? 1 : 0;  // more than 20% of the frequencies
  return out;
}

}  // extern "C"
