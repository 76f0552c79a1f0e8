// extern "C" entry points and the host-side sequencing of the rounding.
//
// Each device entry point is written once as an `exec` routine over an Arena;
// run with a null base it only measures, which is how the *_workspace queries
// compute sizes, so queries and runs cannot disagree about the layout.
//
// Path of tt_round_rand (Algorithm 5; Algorithm 7 for tt_sum_round):
//   1. sketch cores (Definition 3.1) drawn on the device into the workspace
//   2. W chain (Algorithm 3), right to left, one MFMA GEMM pair per core
//   3. left-to-right sweep: Y_n = Z_n W_n, thin QR, M_n = Q^T Z_n,
//      next core M_n H(Y_{n+1}) (per summand for sums)
//   4. right-to-left truncation when an output rank is below the sketch rank
#include <algorithm>
#include <cmath>
#include <cstdlib>
#include <cstring>

#include "tt_internal.h"

namespace ttr {

thread_local bool g_spec_off = false;

static thread_local std::string g_err = "no error";

void set_error(const std::string &msg) { g_err = msg; }
int fail(int status, const std::string &msg) {
  g_err = msg;
  return status;
}

// ---------------------------------------------------------------- validation

int check_shape(int32_t N, const int64_t *dims, const int64_t *ranks, const char *what) {
  if (N < 1 || N > TT_MAX_ORDER)
    return fail(TT_EINVAL, std::string(what) + ": order N out of range");
  if (!dims || !ranks) return fail(TT_EINVAL, std::string(what) + ": null dims/ranks");
  if (ranks[0] != 1 || ranks[N] != 1)
    return fail(TT_EINVAL, std::string(what) + ": ranks[0] and ranks[N] must be 1");
  for (int n = 0; n < N; ++n) {
    if (dims[n] < 1) return fail(TT_EINVAL, std::string(what) + ": dims must be >= 1");
    if (ranks[n + 1] < 1) return fail(TT_EINVAL, std::string(what) + ": ranks must be >= 1");
    if (dims[n] > (int64_t(1) << 31) || ranks[n + 1] > (int64_t(1) << 20))
      return fail(TT_EINVAL, std::string(what) + ": dimension too large");
  }
  return TT_OK;
}

int check_ptrs(int32_t N, const void *const *p, const char *what) {
  if (!p) return fail(TT_EINVAL, std::string(what) + ": null pointer array");
  for (int n = 0; n < N; ++n)
    if (!p[n]) return fail(TT_EINVAL, std::string(what) + ": null core pointer");
  return TT_OK;
}

void plan_ranks(int N, const int64_t *dims, const int64_t *R, int64_t target, int64_t over,
                std::vector<int64_t> &ell, std::vector<int64_t> &out) {
  const int64_t lreq = target + over;
  std::vector<int64_t> u(N + 1, 1);
  for (int n = N - 1; n >= 1; --n) u[n] = std::min<int64_t>(lreq, dims[n] * u[n + 1]);
  ell.assign(N + 1, 1);
  for (int n = 1; n < N; ++n)
    ell[n] = std::min({lreq, ell[n - 1] * dims[n - 1], u[n], R[n]});
  out.assign(N + 1, 1);
  for (int n = 1; n < N; ++n) out[n] = std::min(target, ell[n]);
}

int prec_cfg(int32_t prec, Prec &p) {
  switch (prec) {
    case TT_PREC_F64:
      p = Prec{DType::F64, DType::F64, DType::F64, false};
      return TT_OK;
    case TT_PREC_F32:
      p = Prec{DType::F32, DType::F32, DType::F32, true};
      return TT_OK;
    case TT_PREC_MIXED_BF16:
      p = Prec{DType::F32, DType::BF16, DType::BF16, true};
      return TT_OK;
    default:
      return fail(TT_EINVAL, "unknown prec");
  }
}

int check_dtype(int32_t dtype, const Prec &p) {
  if (dtype == TT_BF16) return fail(TT_EUNSUPPORTED, "BF16 storage of TT cores is not supported");
  if (dtype != TT_F64 && dtype != TT_F32) return fail(TT_EINVAL, "unknown dtype");
  if (dtype != (int32_t)p.store)
    return fail(TT_EINVAL, p.store == DType::F64 ? "TT_PREC_F64 needs TT_F64 storage"
                                                 : "TT_PREC_F32 and TT_PREC_MIXED_BF16 need "
                                                   "TT_F32 storage");
  return TT_OK;
}

size_t dtype_bytes(DType t) { return t == DType::F64 ? 8 : (t == DType::F32 ? 4 : 2); }

// W-chain levels: fused kernel where it fits (0) or always two products (1)
static int g_wchain_mode = 0;

void read_env() {
  const char *w = std::getenv("TT_WCHAIN");
  g_wchain_mode = (w && !std::strcmp(w, "gemm")) ? 1 : 0;
  const char *gm = std::getenv("TT_GRAM");
  gram_set_mode((gm && !std::strcmp(gm, "gemm")) ? 1 : 0);
  const char *q = std::getenv("TT_QR");
  if (!q) qr_set_mode(0);
  else if (!std::strcmp(q, "householder")) qr_set_mode(1);
  else if (!std::strcmp(q, "cholqr2")) qr_set_mode(2);
  else qr_set_mode(0);
  const char *e = std::getenv("TT_EIG");
  eig_set_mode((e && !std::strcmp(e, "jacobi")) ? 1 : 0);
}

// ---------------------------------------------------------------- context

struct Ctx {
  bool dry = true;
  Arena arena;
  hipStream_t s = nullptr;
  size_t partial_need = 0;  // bytes of split-K partials
  void *partial = nullptr;
  size_t partial_cap = 0;   // bytes
  size_t peak = 0;          // largest arena offset of nested, rolled-back regions
};

// Opt-in launch timer (tt_timing_start / tt_timing_stop).
struct Timer {
  int site = -1;
  std::vector<hipEvent_t> ev;  // 2 per timed product
  std::vector<int> reps;       // launches between each pair
  size_t used = 0;
};
constexpr int kTimingRepeats = 8;
Timer g_timer;

// run(): the launches of one product; timed when the recorder is armed for
// its site.  Back-to-back repeats of the same product amortise the event
// overhead; only products that overwrite their output can be repeated.
template <class Run>
int timed_launch(Ctx &c, int site, bool repeatable, Run run) {
  const bool timed = site >= 0 && site == g_timer.site && g_timer.used + 2 <= g_timer.ev.size();
  if (!timed) return run();
  const int reps = repeatable ? kTimingRepeats : 1;
  TTR_HIP(hipEventRecord(g_timer.ev[g_timer.used], c.s));
  for (int r = 0; r < reps; ++r) TTR_TRY(run());
  TTR_HIP(hipEventRecord(g_timer.ev[g_timer.used + 1], c.s));
  g_timer.reps.push_back(reps);
  g_timer.used += 2;
  return TT_OK;
}

int gemm(Ctx &c, GemmX g, int site = -1) {
  const int sp = (g.batch > 1) ? 1 : gemm_pick_splits(g.M, g.N, g.K, g.math);
  const size_t need = sp > 1 ? (size_t)sp * g.M * g.N * gemm_acc_bytes(g.math) : 0;
  c.partial_need = std::max(c.partial_need, need);
  if (c.dry) return TT_OK;
  if (need > c.partial_cap) return fail(TT_EINVAL, "internal: split-K buffer too small");
  g.splits = sp;
  g.partial = c.partial;
  return timed_launch(c, site, g.beta == 0.0, [&] { return gemmx_run(g, c.s); });
}
template <typename T>
int gemm(Ctx &c, const Gemm<T> &g, int site = -1) {
  return gemm(c, g.x(), site);
}

int make_problem(Problem &P, int s, int N, const int64_t *dims, const int64_t *ranks,
                 int64_t target, int64_t over, const double *coeffs) {
  if (s < 1) return fail(TT_EINVAL, "need at least one summand");
  if (target < 1) return fail(TT_EINVAL, "target_rank must be >= 1");
  if (over < 0) return fail(TT_EINVAL, "oversample must be >= 0");
  P.N = N;
  P.s = s;
  P.dims.assign(dims, dims + N);
  P.R.resize(s);
  P.Rsum.assign(N + 1, 0);
  for (int j = 0; j < s; ++j) {
    TTR_TRY(check_shape(N, dims, ranks + (size_t)j * (N + 1), "input TT"));
    P.R[j].assign(ranks + (size_t)j * (N + 1), ranks + (size_t)(j + 1) * (N + 1));
    for (int n = 0; n <= N; ++n) P.Rsum[n] += P.R[j][n];
  }
  P.Rsum[0] = P.Rsum[N] = 1;
  plan_ranks(N, dims, P.Rsum.data(), target, over, P.ell, P.out);
  P.coeffs.assign(s, 1.0);
  if (coeffs)
    for (int j = 0; j < s; ++j) P.coeffs[j] = coeffs[j];
  P.truncate = false;
  P.max_ell = 1;
  for (int n = 0; n <= N; ++n) {
    if (P.out[n] < P.ell[n]) P.truncate = true;
    P.max_ell = std::max(P.max_ell, P.ell[n]);
  }
  if (N > 1 && P.max_ell > TT_MAX_SKETCH_RANK)
    return fail(TT_EUNSUPPORTED, "sketch rank above TT_MAX_SKETCH_RANK");
  return TT_OK;
}

namespace {

// ---------------------------------------------------------------- W chain
// Partial contractions of s TTs Y^(j) (cores Y[j*N + n], ranks R[j]) with one
// sketch TT (cores Sk, ranks L): W^(j)_n = H(Y^(j)_{n+1:N}) H(Sk_{n+1:N})^T for
// n = 1..N-1, written into the stacked W[n] (rows of summand j start at
// sum_{i<j} R[i][n], leading dimension L[n]).  Level by level (all summands of
// level n before level n-1), so that with `renorm` every level is scaled by
// one power of two common to all summands.
template <typename T>
int wchain(Ctx &c, const Prec &p, bool renorm, int N, const int64_t *dims, int s,
           const int64_t *const *R, const T *const *Y, const int64_t *L,
           const void *const *Sk, T *const *W, double *factors = nullptr) {
  int64_t zmax = 0;
  for (int j = 0; j < s; ++j)
    for (int n = 2; n <= N - 1; ++n) zmax = std::max(zmax, R[j][n - 1] * dims[n - 1] * L[n]);
  T *zc = c.arena.take<T>((size_t)zmax);
  auto wrow = [&](int j, int n) {  // first row of summand j in the stacked W[n]
    int64_t off = 0;
    for (int i = 0; i < j; ++i) off += R[i][n];
    return W[n] ? W[n] + off * L[n] : nullptr;
  };
  auto rows = [&](int n) {
    int64_t r = 0;
    for (int j = 0; j < s; ++j) r += R[j][n];
    return r;
  };
  // W_{n-1} (or W_{N-1} from the last core) = H(A) H(Sk_n)^T, A: M x K rows
  auto sk_product = [&](const T *A, int64_t M, int64_t K, int core, T *C, int64_t ncols) {
    GemmX g;
    g.A = A;
    g.lda = K;
    g.a_kc = true;
    g.ta = p.store;
    g.B = Sk[core];
    g.ldb = K;
    g.b_kc = true;
    g.tb = p.sk;
    g.C = C;
    g.ldc = ncols;
    g.tc = p.store;
    g.M = M;
    g.N = ncols;
    g.K = K;
    g.math = p.wmath;
    return gemm(c, g, TT_SITE_WCHAIN_W);
  };
  for (int j = 0; j < s; ++j)
    TTR_TRY(sk_product(Y[(size_t)j * N + N - 1], R[j][N - 1], dims[N - 1], N - 1,
                       wrow(j, N - 1), L[N - 1]));
  if (renorm && !c.dry)
    TTR_TRY(scale_pow2<T>(W[N - 1], rows(N - 1) * L[N - 1], c.s,
                          factors ? factors + N - 1 : nullptr));
  for (int n = N - 1; n >= 2; --n) {
    const int64_t I = dims[n - 1];
    // W_{n-1} = H(V(Y_n) W_n) H(Sk_n)^T for every summand in one kernel
    WFuse f;
    f.Sk = Sk[n - 1];
    f.t = DTypeOf<T>::value;
    f.math = p.wmath;
    f.sk = p.sk;
    f.I = I;
    f.L1 = L[n];
    f.L0 = L[n - 1];
    for (int j = 0; j < s; ++j) {
      WFuseItem it;
      it.Y = Y[(size_t)j * N + n - 1];
      it.W = wrow(j, n);
      it.C = wrow(j, n - 1);
      it.R0 = R[j][n - 1];
      it.R1 = R[j][n];
      f.items.push_back(it);
    }
    // the dry pass sizes the split buffer for both forms (the cores'
    // alignment, which the fused kernel needs, is known only at run time)
    const bool fusable = g_wchain_mode == 0 && wfuse_supported(f);
    bool fused = false;
    if (fusable) {
      const size_t need = (size_t)wfuse_partial_elems(f) * sizeof(T);
      c.partial_need = std::max(c.partial_need, need);
      if (!c.dry && wfuse_aligned(f)) {
        if (need > c.partial_cap) return fail(TT_EINVAL, "internal: split buffer too small");
        TTR_TRY(timed_launch(c, TT_SITE_WCHAIN_FUSED, true,
                             [&] { return wfuse_run(f, c.partial, c.partial_cap, c.s); }));
        TTR_TRY(wfuse_sum(f, c.partial, c.s));
        fused = true;
      }
    }
    for (int j = 0; j < s && !fused; ++j) {
      GemmX g;  // V(Z_n) = V(Y_n) W_n
      g.A = Y[(size_t)j * N + n - 1];
      g.lda = R[j][n];
      g.a_kc = true;
      g.ta = p.store;
      g.B = wrow(j, n);
      g.ldb = L[n];
      g.b_kc = false;
      g.tb = p.store;
      g.C = zc;
      g.ldc = L[n];
      g.tc = p.store;
      g.M = R[j][n - 1] * I;
      g.N = L[n];
      g.K = R[j][n];
      g.math = p.wmath;
      TTR_TRY(gemm(c, g, TT_SITE_WCHAIN_Z));
      TTR_TRY(sk_product(zc, R[j][n - 1], I * L[n], n - 1, wrow(j, n - 1), L[n - 1]));
    }
    if (renorm && !c.dry)
      TTR_TRY(scale_pow2<T>(W[n - 1], rows(n - 1) * L[n - 1], c.s,
                            factors ? factors + n - 1 : nullptr));
  }
  return TT_OK;
}

// ---------------------------------------------------------------- rounding
// Speculative form: copies `count` device flag words back (waits for the
// stream).
int read_flags(Ctx &c, const int *d, int count, std::vector<int> &h) {
  h.assign((size_t)count, 0);
  TTR_HIP(hipMemcpyAsync(h.data(), d, sizeof(int) * (size_t)count, hipMemcpyDeviceToHost, c.s));
  TTR_HIP(hipStreamSynchronize(c.s));
  return TT_OK;
}
// The per-site timer records the first run of a phase only, not its redo.
struct TimerPause {
  int site = g_timer.site;
  TimerPause() { g_timer.site = -1; }
  ~TimerPause() { g_timer.site = site; }
};

// Kept eigenvalues of a truncation Gram below this fraction of the largest
// (singular values below 1e-2 of the largest) take the second pass of
// trunc_refine.hip; above it the first pass resolves the kept directions and
// the new core rows to about 1e-12 (FP64).
constexpr double kTruncRefineTau = 1e-4;

// Y: s summands, cores Y[j*N + n].  Sk: sketch cores (p.sk storage).
// out: output cores.
template <typename T>
int round_exec(Ctx &c, const Problem &P, const Prec &p, const T *const *Y,
               const void *const *Sk, T *const *out, T *const *W_given = nullptr) {
  const int N = P.N, s = P.s;
  const int64_t *dims = P.dims.data();
  const std::vector<int64_t> &L = P.ell;
  const std::vector<int64_t> &Rs = P.Rsum;

  // ---- W chains: stacked W_n = [W^(1)_n; ...; W^(s)_n], (sum_j R^(j)_n) x l_n
  // (or the sketch matrices of Algorithm 4 when given: Y_n = Z_n W_n alike)
  std::vector<T *> W(N, nullptr);
  if (W_given) {
    for (int n = 1; n <= N - 1; ++n) W[n] = W_given[n];
  } else {
    for (int n = 1; n <= N - 1; ++n) W[n] = c.arena.take<T>((size_t)(Rs[n] * L[n]));
    std::vector<const int64_t *> Rj(s);
    for (int j = 0; j < s; ++j) Rj[j] = P.R[j].data();
    TTR_TRY(wchain<T>(c, p, p.renorm, N, dims, s, Rj.data(), Y, L.data(), Sk, W.data()));
  }

  // ---- buffers of the sweep
  int64_t ys_max = 1, x_max = 1, m_max = 1;
  for (int n = 1; n <= N - 1; ++n) {
    ys_max = std::max(ys_max, L[n - 1] * dims[n - 1] * L[n]);
    m_max = std::max(m_max, L[n] * Rs[n]);
    if (n + 1 <= N - 1) x_max = std::max(x_max, L[n] * dims[n] * Rs[n + 1]);
  }
  T *ys = c.arena.take<T>((size_t)ys_max);
  T *mbuf = c.arena.take<T>((size_t)m_max);
  T *xb[2] = {c.arena.take<T>((size_t)x_max), c.arena.take<T>((size_t)x_max)};
  const bool plain_first = (s == 1 && P.coeffs[0] == 1.0);
  T *x1 = plain_first ? nullptr : c.arena.take<T>((size_t)(dims[0] * Rs[1]));
  QrScratch qs;
  const int64_t lm = P.max_ell;
  qs.gram = c.arena.take<double>((size_t)std::max(lm * lm, 2 * lm));
  qs.rinv = c.arena.take<double>((size_t)std::max(lm * lm, 2 * lm));
  if (sizeof(T) == 4) qs.rinv_f = c.arena.take<float>((size_t)(lm * lm));
  qs.q1 = c.arena.take<T>((size_t)ys_max);
  qs.flag = c.arena.take<int>(4);
  // speculative form: QR flag of core n at sflags[4 n], truncation control of
  // bond n at sflags[4 (N + 1) + 4 n], cleared first (the form is never
  // captured into a graph)
  int *sflags = c.arena.take<int>((size_t)8 * (N + 1));
  int *const qflag = qs.flag;
  // sflags[0]: the speculative sweep's go word (1, cleared on a breakdown,
  // after which its launches return at once)
  int *const go = sflags;
  if (P.spec && !c.dry) {
    TTR_HIP(hipMemsetAsync(sflags, 0, sizeof(int) * 8 * (size_t)(N + 1), c.s));
    TTR_HIP(hipMemsetD32Async(reinterpret_cast<hipDeviceptr_t>(go), 1, 1, c.s));
  }
  // the QR's own split-K Gram (FP64 accumulator) uses the shared partial buffer
  for (int n = 1; n <= N - 1; ++n) {
    const size_t need = qr_partial_elems(L[n - 1] * dims[n - 1], L[n]) * sizeof(double);
    c.partial_need = std::max(c.partial_need, need);
  }
  // sweep output: straight into `out` unless a truncation follows
  std::vector<T *> xs(N + 1, nullptr);
  for (int n = 1; n <= N; ++n)
    xs[n] = P.truncate ? c.arena.take<T>((size_t)(L[n - 1] * dims[n - 1] * L[n])) : out[n - 1];
  // truncation scratch
  double *gbuf = nullptr, *lam = nullptr, *U = nullptr, *tails = nullptr;
  int *eflag = nullptr;
  double *escr = nullptr;
  T *Pf = nullptr, *Sf = nullptr, *tb[2] = {nullptr, nullptr};
  // second pass for kept directions far below the largest (its contractions
  // in FP64 arithmetic whatever the storage)
  const bool refine = P.truncate;
  int *ctl = nullptr, *nmask = nullptr;
  double *U1 = nullptr, *G2 = nullptr, *rscr = nullptr, *cscr = nullptr, *lamc = nullptr;
  T *Ff = nullptr, *Bb = nullptr;
  if (refine) {
    int64_t cmax = 1;
    for (int n = 2; n <= N; ++n) cmax = std::max(cmax, dims[n - 1] * P.out[n]);
    ctl = c.arena.take<int>(4);
    nmask = c.arena.take<int>((size_t)lm);
    U1 = c.arena.take<double>((size_t)(lm * lm));
    G2 = c.arena.take<double>((size_t)(lm * lm));
    rscr = c.arena.take<double>(trunc_refine_scratch(lm, lm));
    Ff = c.arena.take<T>((size_t)(lm * lm));
    Bb = c.arena.take<T>((size_t)(lm * cmax));
    cscr = c.arena.take<double>(trunc_complete_scratch(lm, cmax));
    lamc = c.arena.take<double>((size_t)lm);
  }
  if (P.truncate) {
    gbuf = c.arena.take<double>((size_t)(lm * lm));
    lam = c.arena.take<double>((size_t)lm);
    U = c.arena.take<double>((size_t)(lm * lm));
    tails = c.arena.take<double>((size_t)(N + 1));
    eflag = c.arena.take<int>(4);
    escr = c.arena.take<double>(eig_trunc_scratch(lm, lm));
    Pf = c.arena.take<T>((size_t)(lm * lm));
    Sf = c.arena.take<T>((size_t)(lm * lm));
    int64_t tmax = 1;
    for (int n = 2; n <= N - 1; ++n) tmax = std::max(tmax, L[n - 1] * dims[n - 1] * P.out[n]);
    tb[0] = c.arena.take<T>((size_t)tmax);
    tb[1] = c.arena.take<T>((size_t)tmax);
  }
  // ---- first core: X_1 = [c_1 Y^(1)_1 ... c_s Y^(s)_1]
  const T *cur = nullptr;
  if (plain_first) {
    cur = Y[0];
  } else {
    int64_t off = 0;
    for (int j = 0; j < s; ++j) {
      const int64_t rj = P.R[j][1];
      if (!c.dry)
        TTR_TRY(copy2d<T>(x1 + off, Rs[1], Y[(size_t)j * N], rj, dims[0], rj, P.coeffs[j], 0.0,
                          c.s));
      off += rj;
    }
    cur = x1;
  }

  // ---- left-to-right sweep; spec: the speculative form (Problem::spec)
  const T *const first = cur;
  auto sweep = [&](bool spec) -> int {
  const T *cur = first;
  qs.speculative = spec;
  qs.go = spec ? go : nullptr;
  for (int n = 1; n <= N - 1; ++n) {
    const int64_t m = L[n - 1] * dims[n - 1];
    Gemm<T> g;  // Y_n = Z_n W_n
    g.A = cur;
    g.lda = Rs[n];
    g.a_kc = true;
    g.B = W[n];
    g.ldb = L[n];
    g.b_kc = false;
    g.C = ys;
    g.ldc = L[n];
    g.M = m;
    g.N = L[n];
    g.K = Rs[n];
    GemmX gx = g.x();
    gx.gate = qs.go;
    TTR_TRY(gemm(c, gx, TT_SITE_SWEEP_Y));
    qs.partial = c.partial;
    qs.flag = spec ? sflags + 4 * n : qflag;
    if (!c.dry) TTR_TRY(qr_thin<T>(ys, xs[n], m, L[n], qs, c.s));
    Gemm<T> h;  // M_n = Q^T Z_n
    h.A = xs[n];
    h.lda = L[n];
    h.a_kc = false;
    h.B = cur;
    h.ldb = Rs[n];
    h.b_kc = false;
    h.C = mbuf;
    h.ldc = Rs[n];
    h.M = L[n];
    h.N = Rs[n];
    h.K = m;
    GemmX hx = h.x();
    hx.gate = qs.go;
    TTR_TRY(gemm(c, hx, TT_SITE_SWEEP_M));
    // next core
    const int64_t I1 = dims[n];
    const bool last = (n + 1 == N);
    T *dst = last ? xs[N] : xb[n & 1];
    if (s > 1 && !last) {
      // all summands' slice-wise products in one launch when they fit
      std::vector<SumNextEntry> se((size_t)s);
      int64_t om = 0, on = 0;
      for (int j = 0; j < s; ++j) {
        se[j].Y = Y[(size_t)j * N + n];
        se[j].offm = om;
        se[j].offn = on;
        se[j].rj = (int32_t)P.R[j][n];
        se[j].rj1 = (int32_t)P.R[j][n + 1];
        om += P.R[j][n];
        on += P.R[j][n + 1];
      }
      if (sum_next_fits(sizeof(T), L[n], I1, se.data(), s)) {
        if (!c.dry)
          TTR_TRY(timed_launch(c, TT_SITE_SWEEP_NEXT, true, [&] {
            return sum_next_run<T>(mbuf, Rs[n], dst, L[n], I1, Rs[n + 1], se.data(), s, qs.go,
                                   c.s);
          }));
        cur = dst;
        continue;
      }
    }
    int64_t offm = 0, offn = 0;
    for (int j = 0; j < s; ++j) {
      const T *Yj = Y[(size_t)j * N + n];
      const int64_t rj = P.R[j][n], rj1 = P.R[j][n + 1];
      Gemm<T> k;
      k.A = mbuf + offm;  // columns offm.. of M_n
      k.lda = Rs[n];
      k.a_kc = true;
      k.M = L[n];
      k.K = rj;
      if (s == 1 || last) {
        // H(X_{n+1}) (+)= M^(j) H(Y^(j)_{n+1})
        k.B = Yj;
        k.ldb = I1 * rj1;
        k.b_kc = false;
        k.C = dst;
        k.ldc = I1 * rj1;
        k.N = I1 * rj1;
        k.beta = (last && j > 0) ? T(1) : T(0);
      } else {
        // slice-wise: X_{n+1}(:, i, offn + r) = (M^(j) Y^(j)_{n+1}(:, i, :))(:, r)
        k.B = Yj;
        k.ldb = I1 * rj1;
        k.b_kc = false;
        k.C = dst + offn;
        k.ldc = I1 * Rs[n + 1];
        k.N = rj1;
        k.batch = I1;
        k.sB = rj1;
        k.sC = Rs[n + 1];
      }
      GemmX kx = k.x();
      kx.gate = qs.go;
      TTR_TRY(gemm(c, kx, TT_SITE_SWEEP_NEXT));
      offm += rj;
      offn += rj1;
    }
    cur = dst;
  }
  return TT_OK;
  };
  // A speculative sweep whose flags show a breakdown is redone guarded (the W
  // chain is kept), and the truncation then runs guarded too: an input that
  // needed the thin QR's rescue usually needs the truncation's second pass.
  // With a truncation following, the flags are read back after its first
  // bond, so that one synchronisation covers both.
  TTR_TRY(sweep(P.spec));
  std::vector<int> hf;
  auto sweep_bad = [&]() {
    bool bad = false;
    for (int n = 1; n <= N - 1; ++n) bad = bad || hf[(size_t)4 * n] != 0;
    return bad;
  };
  if (P.spec && !c.dry && !P.truncate) {
    TTR_TRY(read_flags(c, sflags, 4 * (N + 1), hf));
    if (sweep_bad()) {
      TimerPause tp;
      TTR_TRY(sweep(false));
    }
  }

  if (P.ranks_out)
    for (int n = 0; n <= N; ++n) P.ranks_out[n] = P.truncate ? P.out[n] : L[n];
  if (!P.truncate) return TT_OK;

  // ---- right-to-left truncation of the left-orthogonal result (to the
  // plan's ranks, or with eps_mode to the smallest ranks meeting the eps rule
  // of Algorithm 2: eps = eps0 ||X|| / sqrt(N-1), ||X|| = ||X_N||_F since
  // cores 1..N-1 are left-orthogonal; the rank of each bond is read back)
  double *dnorm = nullptr;
  int *dk = nullptr;
  if (P.eps_mode) {
    dnorm = c.arena.take<double>(1);
    dk = c.arena.take<int>((size_t)N + 1);
    if (!c.dry) TTR_TRY(frob_norm<T>(xs[N], L[N - 1] * dims[N - 1], dnorm, c.s));
  }
  // the sweep's output xs stays intact: a speculative truncation whose
  // controls show that a bond needed the second pass is redone guarded.
  // truncate(spec, hi, lo) runs bonds hi down to lo, from the start when
  // hi = N.
  const T *hsrc = xs[N];
  int64_t rr = 1;  // right rank of the current core
  auto truncate = [&](bool spec, int n_hi, int n_lo) -> int {
  if (n_hi == N) {
    hsrc = xs[N];
    rr = 1;
  }
  for (int n = n_hi; n >= n_lo; --n) {
    const int64_t lr = L[n - 1], kcap = P.out[n - 1], cols = dims[n - 1] * rr;
    const int64_t keig = P.eps_mode ? lr : kcap;
    if (gram_supported(lr, cols))  // both forms size the split buffer
      c.partial_need = std::max(c.partial_need, gram_partial_elems(lr, cols) * sizeof(double));
    if (gram_enabled(lr, cols)) {
      // G = H H^T: the panel H^T is stored transposed (rows of H)
      if (!c.dry)
        TTR_TRY(timed_launch(c, TT_SITE_TRUNC, true, [&] {
          return gram_run(hsrc, p.store, true, cols, lr, cols, gbuf, lr, c.partial, c.partial_cap,
                          c.s);
        }));
    } else {
    GemmX g;  // G = H H^T, FP64 arithmetic and result whatever the storage
    g.A = hsrc;
    g.lda = cols;
    g.a_kc = true;
    g.ta = p.store;
    g.B = hsrc;
    g.ldb = cols;
    g.b_kc = true;
    g.tb = p.store;
    g.C = gbuf;
    g.ldc = lr;
    g.tc = DType::F64;
    g.M = lr;
    g.N = lr;
    g.K = cols;
    g.math = DType::F64;
    TTR_TRY(gemm(c, g, TT_SITE_TRUNC));
    }
    // (speculative: the bond's own control word, read back by the caller)
    int *ctl_b = spec ? sflags + 4 * (N + 1) + 4 * n : ctl;
    if (!c.dry)
      TTR_TRY(eig_trunc<T>(gbuf, lr, keig, lam, U, Pf, Sf, tails + n - 1, eflag, escr, c.s,
                           refine ? ctl_b : nullptr, refine ? kTruncRefineTau : 0.0, U1));
    // second pass's contractions (only when ctl[0] = 1, decided on the device)
    auto refine_contractions = [&]() -> int {
      GemmX b;  // B = U1^T H(X_n)
      b.A = U1;
      b.lda = lr;
      b.a_kc = false;
      b.ta = DType::F64;
      b.B = hsrc;
      b.ldb = cols;
      b.b_kc = false;
      b.tb = p.store;
      b.C = Bb;
      b.ldc = cols;
      b.tc = p.store;
      b.M = lr;
      b.N = cols;
      b.K = lr;
      b.math = DType::F64;
      b.gate = ctl;
      TTR_TRY(gemm(c, b, TT_SITE_TRUNC));
      if (gram_enabled(lr, cols)) {  // G2 = B B^T
        if (!c.dry)
          TTR_TRY(gram_run(Bb, p.store, true, cols, lr, cols, G2, lr, c.partial, c.partial_cap,
                           c.s, ctl));
        return TT_OK;
      }
      GemmX g;
      g.A = Bb;
      g.lda = cols;
      g.a_kc = true;
      g.ta = p.store;
      g.B = Bb;
      g.ldb = cols;
      g.b_kc = true;
      g.tb = p.store;
      g.C = G2;
      g.ldc = lr;
      g.tc = DType::F64;
      g.M = lr;
      g.N = lr;
      g.K = cols;
      g.math = DType::F64;
      g.gate = ctl;
      return gemm(c, g, TT_SITE_TRUNC);
    };
    int64_t k = kcap;
    if (P.eps_mode) {
      // the rank from the eps rule; with weak directions present their
      // eigenvalues come from the second pass (the first resolves them only
      // to about u lambda_1)
      const double *lsel = lam;
      if (refine) {
        TTR_TRY(refine_contractions());
        if (!c.dry) TTR_TRY(trunc_refine_eps<T>(G2, U1, lr, ctl, nmask, rscr, lam, lamc, c.s));
        lsel = lamc;
      }
      if (!c.dry) {
        TTR_TRY(select_rank(lsel, (int)lr, dnorm, P.eps0, N, (int)kcap, dk + n - 1,
                            tails + n - 1, c.s));
        int hk = 0;
        TTR_HIP(hipMemcpyAsync(&hk, dk + n - 1, sizeof(int), hipMemcpyDeviceToHost, c.s));
        TTR_HIP(hipStreamSynchronize(c.s));
        if (hk < 1 || hk > kcap) return fail(TT_ENUMERIC, "tolerance rounding: invalid rank");
        k = hk;
        if (k < keig) {  // first-pass factors of the chosen rank (tail kept from the rule)
          TTR_TRY(trunc_factors<T>(lam, U, lr, k, Pf, Sf, escr, c.s));
          if (refine) TTR_TRY(trunc_refine_setk(ctl, k, c.s));
        }
        if (refine) TTR_TRY(trunc_refine_final<T>(G2, U1, lr, k, ctl, nmask, rscr, Ff, Pf, c.s));
      }
    }
    if (P.ranks_out) P.ranks_out[n - 1] = k;
    const bool guarded = refine && !spec;  // the second pass's launches are enqueued
    if (guarded && !P.eps_mode) {
      TTR_TRY(refine_contractions());
      if (!c.dry) TTR_TRY(trunc_refine_solve<T>(G2, U1, lr, k, ctl, nmask, rscr, Ff, Pf, c.s));
    }
    // new core: H(X_n) <- s^-1 U^T H(X_n) (first pass), or F B when the
    // second pass ran (operands chosen on the device, one launch)
    Gemm<T> h;
    h.A = Sf;
    h.lda = lr;
    h.a_kc = true;
    h.B = hsrc;
    h.ldb = cols;
    h.b_kc = false;
    h.C = out[n - 1];
    h.ldc = cols;
    h.M = k;
    h.N = cols;
    h.K = lr;
    GemmX hx = h.x();
    if (guarded) {
      hx.sel = ctl;
      hx.A2 = Ff;
      hx.B2 = Bb;
    }
    TTR_TRY(gemm(c, hx, TT_SITE_TRUNC));
    // orthonormal rows in place of directions with no information left
    if (guarded && !c.dry)
      TTR_TRY(trunc_refine_complete<T>(out[n - 1], k, cols, ctl, nmask, cscr, c.s));
    Gemm<T> p;  // X_{n-1} <- X_{n-1} x_3 (U s)
    const int64_t rows = L[n - 2] * dims[n - 2];
    p.A = xs[n - 1];
    p.lda = lr;
    p.a_kc = true;
    p.B = Pf;
    p.ldb = k;
    p.b_kc = false;
    T *dst = (n - 1 == 1) ? out[0] : tb[n & 1];
    p.C = dst;
    p.ldc = k;
    p.M = rows;
    p.N = k;
    p.K = lr;
    TTR_TRY(gemm(c, p, TT_SITE_TRUNC));
    hsrc = dst;
    rr = k;
  }
  return TT_OK;
  };
  if (!P.spec || c.dry) return truncate(P.spec, N, 2);
  // speculative: the first bond, then one read-back of the sweep's flags and
  // that bond's control; a bond that needs the second pass makes the whole
  // truncation run guarded
  TTR_TRY(truncate(true, N, N));
  TTR_TRY(read_flags(c, sflags, 8 * (N + 1), hf));
  if (sweep_bad()) {
    TimerPause tp;
    TTR_TRY(sweep(false));
    return truncate(false, N, 2);
  }
  if (hf[(size_t)4 * (N + 1) + 4 * N] != 0) {
    TimerPause tp;
    return truncate(false, N, 2);
  }
  TTR_TRY(truncate(true, N - 1, 2));
  TTR_TRY(read_flags(c, sflags + 4 * (N + 1), 4 * (N + 1), hf));
  bool bad = false;
  for (int n = 2; n <= N; ++n) bad = bad || hf[(size_t)4 * n] != 0;
  if (bad) {
    TimerPause tp;
    TTR_TRY(truncate(false, N, 2));
  }
  return TT_OK;
}

// ---------------------------------------------------------------- adjoint
// Reverse mode of Randomize-then-Orthogonalize without truncation (single
// TT, sketch fixed).  The forward pass is recomputed first (W chain,
// including its power-of-two factors in the FP32 mode, and the sweep, whose
// current cores Z_n, factors Q_n, M_n and R_n^{-1} stay in the workspace).
// Then, with dX~_N = the cotangent of the last output core and n = N-1..1:
//   dM_n = dH(X~_{n+1}) H(Y_{n+1})^T          dH(Y_{n+1})  = M_n^T dH(X~_{n+1})
//   dQ   = dO_n + Z_n dM_n^T                   dZ_n         = Q_n dM_n
//   dY_n = (dQ + Q_n copyltu(-dQ^T Q_n)) R_n^{-T}     (QR adjoint, R unused)
//   dZ_n += dY_n W_n^T                         dW_n         = Z_n^T dY_n
// and dX~_n = dZ_n (dY_1 = dZ_1).  R_n = Q_n^T Y_n is formed from the Q_n the
// sweep produced (whichever QR path produced it) and inverted by back
// substitution.  Finally the W chain in reverse, n = 1..N-2:
//   dZc = f_n dW_n H(S_{n+1}),  dV(Y_{n+1}) += dV(Zc) W_{n+1}^T,
//   dW_{n+1} += V(Y_{n+1})^T dV(Zc),   and dH(Y_N) += f_{N-1} dW_{N-1} H(S_N)
// (f_n: the power-of-two factor applied to W_n, 1 in FP64).
template <typename T>
int backward_exec(Ctx &c, const Problem &P, const Prec &p, const T *const *Y,
                  const void *const *Sk, const T *const *gout, T *const *gin) {
  const int N = P.N;
  const int64_t *dims = P.dims.data();
  const std::vector<int64_t> &L = P.ell;
  const std::vector<int64_t> &R = P.R[0];
  // ---- forward recomputation
  std::vector<T *> W(N, nullptr);
  for (int n = 1; n <= N - 1; ++n) W[n] = c.arena.take<T>((size_t)(R[n] * L[n]));
  double *fac = c.arena.take<double>((size_t)N + 1);
  {
    const int64_t *Rp = R.data();
    TTR_TRY(wchain<T>(c, p, p.renorm, N, dims, 1, &Rp, Y, L.data(), Sk, W.data(), fac));
  }
  std::vector<T *> xt(N + 1, nullptr), q(N, nullptr), mm(N, nullptr);
  std::vector<double *> rinv(N, nullptr);
  std::vector<float *> rinvf(N, nullptr);
  int64_t m_max = 1, x_max = 1, l_max = 1, r_max = 1;
  for (int n = 1; n <= N; ++n) {
    x_max = std::max(x_max, L[n - 1] * dims[n - 1] * R[n]);
    l_max = std::max(l_max, L[n]);
    r_max = std::max(r_max, R[n]);
    if (n <= N - 1) m_max = std::max(m_max, L[n - 1] * dims[n - 1]);
  }
  xt[1] = const_cast<T *>(Y[0]);
  for (int n = 2; n <= N; ++n) xt[n] = c.arena.take<T>((size_t)(L[n - 1] * dims[n - 1] * R[n]));
  for (int n = 1; n <= N - 1; ++n) {
    q[n] = c.arena.take<T>((size_t)(L[n - 1] * dims[n - 1] * L[n]));
    mm[n] = c.arena.take<T>((size_t)(L[n] * R[n]));
    rinv[n] = c.arena.take<double>((size_t)(L[n] * L[n]));
    if (sizeof(T) == 4) rinvf[n] = c.arena.take<float>((size_t)(L[n] * L[n]));
  }
  T *ys = c.arena.take<T>((size_t)(m_max * l_max));
  double *gram = c.arena.take<double>((size_t)(l_max * l_max));
  int *cflag = c.arena.take<int>(4);
  QrScratch qs;
  qs.gram = c.arena.take<double>((size_t)std::max(l_max * l_max, 2 * l_max));
  qs.rinv = c.arena.take<double>((size_t)std::max(l_max * l_max, 2 * l_max));
  if (sizeof(T) == 4) qs.rinv_f = c.arena.take<float>((size_t)(l_max * l_max));
  qs.q1 = c.arena.take<T>((size_t)(m_max * l_max));
  qs.flag = c.arena.take<int>(4);
  for (int n = 1; n <= N - 1; ++n) {
    const int64_t m = L[n - 1] * dims[n - 1];
    Gemm<T> g;  // Y_n = Z_n W_n
    g.A = xt[n];
    g.lda = R[n];
    g.a_kc = true;
    g.B = W[n];
    g.ldb = L[n];
    g.b_kc = false;
    g.C = ys;
    g.ldc = L[n];
    g.M = m;
    g.N = L[n];
    g.K = R[n];
    TTR_TRY(gemm(c, g));
    c.partial_need = std::max(c.partial_need, qr_partial_elems(m, L[n]) * sizeof(double));
    if (!c.dry) {
      qs.partial = c.partial;
      TTR_TRY(qr_thin<T>(ys, q[n], m, L[n], qs, c.s));
    }
    GemmX gr;  // R_n = Q_n^T Y_n (FP64): the factor of the Q the sweep produced
    gr.A = q[n];
    gr.lda = L[n];
    gr.a_kc = false;
    gr.ta = p.store;
    gr.B = ys;
    gr.ldb = L[n];
    gr.b_kc = false;
    gr.tb = p.store;
    gr.C = gram;
    gr.ldc = L[n];
    gr.tc = DType::F64;
    gr.M = L[n];
    gr.N = L[n];
    gr.K = m;
    gr.math = DType::F64;
    TTR_TRY(gemm(c, gr));
    if (!c.dry) TTR_TRY(tri_inv_upper(gram, L[n], rinv[n], rinvf[n], cflag, n == 1, c.s));
    Gemm<T> h;  // M_n = Q^T Z_n
    h.A = q[n];
    h.lda = L[n];
    h.a_kc = false;
    h.B = xt[n];
    h.ldb = R[n];
    h.b_kc = false;
    h.C = mm[n];
    h.ldc = R[n];
    h.M = L[n];
    h.N = R[n];
    h.K = m;
    TTR_TRY(gemm(c, h));
    const int64_t cols = dims[n] * R[n + 1];
    Gemm<T> k;  // H(X~_{n+1}) = M_n H(Y_{n+1})
    k.A = mm[n];
    k.lda = R[n];
    k.a_kc = true;
    k.B = Y[n];
    k.ldb = cols;
    k.b_kc = false;
    k.C = xt[n + 1];
    k.ldc = cols;
    k.M = L[n];
    k.N = cols;
    k.K = R[n];
    TTR_TRY(gemm(c, k));
  }
  // ---- reverse sweep
  T *dxb[2] = {c.arena.take<T>((size_t)x_max), c.arena.take<T>((size_t)x_max)};
  T *dM = c.arena.take<T>((size_t)(l_max * r_max));
  T *dQ = c.arena.take<T>((size_t)(m_max * l_max));
  T *dYs = c.arena.take<T>((size_t)(m_max * l_max));
  T *Mq = c.arena.take<T>((size_t)(l_max * l_max));
  T *Cq = c.arena.take<T>((size_t)(l_max * l_max));
  std::vector<T *> dW(N, nullptr);
  for (int n = 1; n <= N - 1; ++n) dW[n] = c.arena.take<T>((size_t)(R[n] * L[n]));
  const T *dX = gout[N - 1];
  for (int n = N - 1; n >= 1; --n) {
    const int64_t m = L[n - 1] * dims[n - 1], cols = dims[n] * R[n + 1];
    const int64_t ln = L[n], rn = R[n];
    Gemm<T> a;  // dM = dH(X~_{n+1}) H(Y_{n+1})^T
    a.A = dX;
    a.lda = cols;
    a.a_kc = true;
    a.B = Y[n];
    a.ldb = cols;
    a.b_kc = true;
    a.C = dM;
    a.ldc = rn;
    a.M = ln;
    a.N = rn;
    a.K = cols;
    TTR_TRY(gemm(c, a));
    Gemm<T> b;  // dH(Y_{n+1}) = M_n^T dH(X~_{n+1})
    b.A = mm[n];
    b.lda = rn;
    b.a_kc = false;
    b.B = dX;
    b.ldb = cols;
    b.b_kc = false;
    b.C = gin[n];
    b.ldc = cols;
    b.M = rn;
    b.N = cols;
    b.K = ln;
    TTR_TRY(gemm(c, b));
    if (!c.dry) TTR_TRY(copy2d<T>(dQ, 1, gout[n - 1], 1, m * ln, 1, 1.0, 0.0, c.s));
    Gemm<T> d;  // dQ += Z_n dM^T
    d.A = xt[n];
    d.lda = rn;
    d.a_kc = true;
    d.B = dM;
    d.ldb = rn;
    d.b_kc = true;
    d.C = dQ;
    d.ldc = ln;
    d.M = m;
    d.N = ln;
    d.K = rn;
    d.beta = T(1);
    TTR_TRY(gemm(c, d));
    T *dZ = (n == 1) ? gin[0] : dxb[n & 1];
    Gemm<T> e;  // dZ = Q_n dM
    e.A = q[n];
    e.lda = ln;
    e.a_kc = true;
    e.B = dM;
    e.ldb = rn;
    e.b_kc = false;
    e.C = dZ;
    e.ldc = rn;
    e.M = m;
    e.N = rn;
    e.K = ln;
    TTR_TRY(gemm(c, e));
    Gemm<T> f;  // Mq = dQ^T Q
    f.A = dQ;
    f.lda = ln;
    f.a_kc = false;
    f.B = q[n];
    f.ldb = ln;
    f.b_kc = false;
    f.C = Mq;
    f.ldc = ln;
    f.M = ln;
    f.N = ln;
    f.K = m;
    TTR_TRY(gemm(c, f));
    if (!c.dry) TTR_TRY(copyltu<T>(Cq, Mq, ln, -1.0, c.s));
    Gemm<T> g;  // dQ += Q copyltu(-dQ^T Q)
    g.A = q[n];
    g.lda = ln;
    g.a_kc = true;
    g.B = Cq;
    g.ldb = ln;
    g.b_kc = false;
    g.C = dQ;
    g.ldc = ln;
    g.M = m;
    g.N = ln;
    g.K = ln;
    g.beta = T(1);
    TTR_TRY(gemm(c, g));
    GemmX hx;  // dY_n = dQ R^{-T}
    hx.A = dQ;
    hx.lda = ln;
    hx.a_kc = true;
    hx.ta = p.store;
    hx.B = (sizeof(T) == 4) ? (const void *)rinvf[n] : (const void *)rinv[n];
    hx.ldb = ln;
    hx.b_kc = true;
    hx.tb = p.store;
    hx.C = dYs;
    hx.ldc = ln;
    hx.tc = p.store;
    hx.M = m;
    hx.N = ln;
    hx.K = ln;
    hx.math = p.store;
    TTR_TRY(gemm(c, hx));
    Gemm<T> i2;  // dZ += dY_n W_n^T
    i2.A = dYs;
    i2.lda = ln;
    i2.a_kc = true;
    i2.B = W[n];
    i2.ldb = ln;
    i2.b_kc = true;
    i2.C = dZ;
    i2.ldc = rn;
    i2.M = m;
    i2.N = rn;
    i2.K = ln;
    i2.beta = T(1);
    TTR_TRY(gemm(c, i2));
    Gemm<T> j2;  // dW_n = Z_n^T dY_n
    j2.A = xt[n];
    j2.lda = rn;
    j2.a_kc = false;
    j2.B = dYs;
    j2.ldb = ln;
    j2.b_kc = false;
    j2.C = dW[n];
    j2.ldc = ln;
    j2.M = rn;
    j2.N = ln;
    j2.K = m;
    TTR_TRY(gemm(c, j2));
    dX = dZ;
  }
  // ---- reverse W chain
  int64_t zc_max = 1;
  for (int n = 1; n <= N - 2; ++n) zc_max = std::max(zc_max, R[n] * dims[n] * L[n + 1]);
  T *dZc = c.arena.take<T>((size_t)zc_max);
  for (int n = 1; n <= N - 2; ++n) {
    if (p.renorm && !c.dry) TTR_TRY(scale_dev<T>(dW[n], R[n] * L[n], fac + n, c.s));
    const int64_t I = dims[n];
    GemmX a;  // dZc (R_n x I L_{n+1}) = dW_n H(S_{n+1})
    a.A = dW[n];
    a.lda = L[n];
    a.a_kc = true;
    a.ta = p.store;
    a.B = Sk[n];
    a.ldb = I * L[n + 1];
    a.b_kc = false;
    a.tb = p.sk;
    a.C = dZc;
    a.ldc = I * L[n + 1];
    a.tc = p.store;
    a.M = R[n];
    a.N = I * L[n + 1];
    a.K = L[n];
    a.math = p.wmath;
    TTR_TRY(gemm(c, a));
    Gemm<T> b;  // dV(Y_{n+1}) += dV(Zc) W_{n+1}^T
    b.A = dZc;
    b.lda = L[n + 1];
    b.a_kc = true;
    b.B = W[n + 1];
    b.ldb = L[n + 1];
    b.b_kc = true;
    b.C = gin[n];
    b.ldc = R[n + 1];
    b.M = R[n] * I;
    b.N = R[n + 1];
    b.K = L[n + 1];
    b.beta = T(1);
    TTR_TRY(gemm(c, b));
    Gemm<T> d;  // dW_{n+1} += V(Y_{n+1})^T dV(Zc)
    d.A = Y[n];
    d.lda = R[n + 1];
    d.a_kc = false;
    d.B = dZc;
    d.ldb = L[n + 1];
    d.b_kc = false;
    d.C = dW[n + 1];
    d.ldc = L[n + 1];
    d.M = R[n + 1];
    d.N = L[n + 1];
    d.K = R[n] * I;
    d.beta = T(1);
    TTR_TRY(gemm(c, d));
  }
  if (p.renorm && !c.dry) TTR_TRY(scale_dev<T>(dW[N - 1], R[N - 1] * L[N - 1], fac + N - 1, c.s));
  GemmX z;  // dH(Y_N) += dW_{N-1} H(S_N)
  z.A = dW[N - 1];
  z.lda = L[N - 1];
  z.a_kc = true;
  z.ta = p.store;
  z.B = Sk[N - 1];
  z.ldb = dims[N - 1];
  z.b_kc = false;
  z.tb = p.sk;
  z.C = gin[N - 1];
  z.ldc = dims[N - 1];
  z.tc = p.store;
  z.M = R[N - 1];
  z.N = dims[N - 1];
  z.K = L[N - 1];
  z.beta = 1.0;
  z.math = p.wmath;
  TTR_TRY(gemm(c, z));
  if (c.dry) return TT_OK;
  // a numerically singular R_n (a rank-deficient sketch Y_n) leaves the
  // adjoint of the thin QR undefined: report it
  int bad = 0;
  TTR_HIP(hipMemcpyAsync(&bad, cflag, sizeof(int), hipMemcpyDeviceToHost, c.s));
  TTR_HIP(hipStreamSynchronize(c.s));
  if (bad)
    return fail(TT_ENUMERIC, "tt_round_rand_backward: a sketched matrix Y_n = Z_n W_n is "
                             "numerically rank deficient (its R factor is singular)");
  return TT_OK;
}

// ---------------------------------------------------------------- Algorithm 1
// Right-to-left orthogonalisation of the working cores xs[1..N] (each buffer
// large enough for any core of the train; ranks left[0..N], updated),
// rr = the ranks after it.  Core n = N..2 with H = H(X_n) (c x m,
// m = I_n r_n):
//   m >= c: thin QR of H^T (transposed into a tall panel) gives Q; the new
//           core is Q^T, and R^T = H Q is carried into X_{n-1};
//   m <  c: the rank drops to m; Q is the QR factor of the leading m x m
//           block of H^T (its first m rows of H, transposed), the new core
//           Q^T, and R^T = H Q is carried into X_{n-1}.
template <typename T>
int orth_rl(Ctx &c, int N, const int64_t *dims, const std::vector<int64_t> &rr,
            std::vector<T *> &xs, T *&spare, T *pan, T *qb, T *rt, QrScratch &qs,
            std::vector<int64_t> &left) {
  for (int n = N; n >= 2; --n) {
    const int64_t cc = left[n - 1], I = dims[n - 1], m = I * rr[n];
    const int64_t rows_prev = left[n - 2] * dims[n - 2];
    const int64_t q = std::min(m, cc);  // columns of Q, the new bond rank
    c.partial_need = std::max(c.partial_need, qr_partial_elems(m, q) * sizeof(double));
    if (!c.dry) {
      // tall panel H^T (m x cc), or the leading square block (m x m)
      if (m >= cc)
        TTR_TRY(transpose<T>(pan, xs[n], cc, m, c.s));
      else
        TTR_TRY(transpose<T>(pan, xs[n], m, m, c.s));
      qs.partial = c.partial;
      TTR_TRY(qr_thin<T>(pan, qb, m, q, qs, c.s));
    }
    Gemm<T> g;  // R^T = H Q  (cc x q)
    g.A = xs[n];
    g.lda = m;
    g.a_kc = true;
    g.B = qb;
    g.ldb = q;
    g.b_kc = false;
    g.C = rt;
    g.ldc = q;
    g.M = cc;
    g.N = q;
    g.K = m;
    TTR_TRY(gemm(c, g));
    if (!c.dry) TTR_TRY(transpose<T>(xs[n], qb, m, q, c.s));  // new core: Q^T
    Gemm<T> h;  // V(X_{n-1}) <- V(X_{n-1}) R^T
    h.A = xs[n - 1];
    h.lda = cc;
    h.a_kc = true;
    h.B = rt;
    h.ldb = q;
    h.b_kc = false;
    h.C = spare;
    h.ldc = q;
    h.M = rows_prev;
    h.N = q;
    h.K = cc;
    TTR_TRY(gemm(c, h));
    std::swap(xs[n - 1], spare);
    left[n - 1] = q;
  }
  return TT_OK;
}

// ---------------------------------------------------------------- TT-SVD
// Deterministic rounding: Algorithm 1 (right-to-left orthogonalisation)
// followed by Algorithm 2 (left-to-right truncation).
//
// Algorithm 1: orth_rl.
// Algorithm 2, core n = 1..N-1: with A = V(X_n) (m x c), the SVD of the QR
// factor R of A has the right singular vectors and singular values of the
// Gram A^T A = R^T R; with its leading eigenpairs (V_k, s_k^2):
//   V(X_n) <- A V_k s_k^-1 (= Q U_k),   H(X_{n+1}) <- s_k V_k^T H(X_{n+1}),
// so no explicit Q is formed.  The rank is fixed (k = min(max_rank, c, m))
// or chosen on the device by the eps rule and read back by the host.
struct SvdPlan {
  int N = 0;
  std::vector<int64_t> dims, R;   // input ranks
  std::vector<int64_t> rr;        // ranks after Algorithm 1
  std::vector<int64_t> kmax;      // output rank bounds
  int64_t max_rank = 0;
  int64_t max_c = 1;              // widest Gram / QR panel
};

int make_svd_plan(SvdPlan &P, int N, const int64_t *dims, const int64_t *ranks,
                  int64_t max_rank) {
  TTR_TRY(check_shape(N, dims, ranks, "tt_round_svd"));
  P.N = N;
  P.dims.assign(dims, dims + N);
  P.R.assign(ranks, ranks + N + 1);
  P.max_rank = max_rank;
  P.rr.assign(N + 1, 1);
  for (int n = N; n >= 2; --n) P.rr[n - 1] = std::min(P.R[n - 1], dims[n - 1] * P.rr[n]);
  P.kmax.assign(N + 1, 1);
  P.max_c = 1;
  for (int n = 1; n <= N - 1; ++n) {
    int64_t k = std::min(P.rr[n], P.kmax[n - 1] * dims[n - 1]);
    if (max_rank > 0) k = std::min(k, max_rank);
    P.kmax[n] = k;
    P.max_c = std::max(P.max_c, P.rr[n]);
  }
  for (int n = N; n >= 2; --n)
    if (dims[n - 1] * P.rr[n] >= P.R[n - 1]) P.max_c = std::max(P.max_c, P.R[n - 1]);
  if (N > 1 && P.max_c > TT_MAX_SKETCH_RANK)
    return fail(TT_EUNSUPPORTED, "tt_round_svd: a bond rank above TT_MAX_SKETCH_RANK");
  return TT_OK;
}

template <typename T>
int svd_exec(Ctx &c, const SvdPlan &P, const T *const *Y, double eps0, T *const *out,
             int64_t *out_ranks) {
  const int N = P.N;
  const int64_t *dims = P.dims.data();
  const DType dt = DTypeOf<T>::value;
  int64_t core_max = 1, pan_max = 1;
  for (int n = 0; n < N; ++n) {
    core_max = std::max(core_max, P.R[n] * dims[n] * P.R[n + 1]);
    pan_max = std::max(pan_max, P.R[n] * dims[n] * P.R[n + 1]);
  }
  std::vector<T *> xs(N + 1, nullptr);
  for (int n = 1; n <= N; ++n) xs[n] = c.arena.take<T>((size_t)core_max);
  T *spare = c.arena.take<T>((size_t)core_max);
  T *pan = c.arena.take<T>((size_t)pan_max);
  T *qb = c.arena.take<T>((size_t)core_max);
  const int64_t lc = P.max_c;
  T *rt = c.arena.take<T>((size_t)(lc * lc));
  T *cbuf = c.arena.take<T>((size_t)(lc * lc));
  double *gbuf = c.arena.take<double>((size_t)(lc * lc));
  double *lam = c.arena.take<double>((size_t)lc + 1);
  double *U = c.arena.take<double>((size_t)(lc * lc));
  T *Pf = c.arena.take<T>((size_t)(lc * lc));
  T *Sf = c.arena.take<T>((size_t)(lc * lc));
  double *tails = c.arena.take<double>((size_t)N + 1);
  double *dnorm = c.arena.take<double>(1);
  int *eflag = c.arena.take<int>(4);
  int *dk = c.arena.take<int>((size_t)N + 1);
  double *escr = c.arena.take<double>(eig_trunc_scratch(lc, lc));
  QrScratch qs;
  qs.gram = c.arena.take<double>((size_t)std::max(lc * lc, 2 * lc));
  qs.rinv = c.arena.take<double>((size_t)std::max(lc * lc, 2 * lc));
  if (sizeof(T) == 4) qs.rinv_f = c.arena.take<float>((size_t)(lc * lc));
  qs.q1 = c.arena.take<T>((size_t)pan_max);
  qs.flag = c.arena.take<int>(4);

  // working copies of the cores
  for (int n = 1; n <= N; ++n)
    if (!c.dry)
      TTR_TRY(copy2d<T>(xs[n], 1, Y[n - 1], 1, P.R[n - 1] * dims[n - 1] * P.R[n], 1, 1.0, 0.0,
                        c.s));
  std::vector<int64_t> left(P.R.begin(), P.R.end());  // current bond ranks
  // ---- Algorithm 1
  TTR_TRY(orth_rl<T>(c, N, dims, P.rr, xs, spare, pan, qb, rt, qs, left));
  // ||Y|| = ||X_1||_F once the other cores are orthonormal
  if (!c.dry && eps0 > 0.0) TTR_TRY(frob_norm<T>(xs[1], dims[0] * left[1], dnorm, c.s));
  // ---- Algorithm 2
  std::vector<int64_t> k(N + 1, 1);
  for (int n = 1; n <= N - 1; ++n) {
    const int64_t cc = left[n], m = k[n - 1] * dims[n - 1];
    const int64_t kcap = std::min(P.kmax[n], m);
    GemmX g;  // Gram A^T A (cc x cc), FP64
    g.A = xs[n];
    g.lda = cc;
    g.a_kc = false;
    g.ta = dt;
    g.B = xs[n];
    g.ldb = cc;
    g.b_kc = false;
    g.tb = dt;
    g.C = gbuf;
    g.ldc = cc;
    g.tc = DType::F64;
    g.M = cc;
    g.N = cc;
    g.K = m;
    g.math = DType::F64;
    TTR_TRY(gemm(c, g));
    const int64_t keig = eps0 > 0.0 ? cc : kcap;
    if (!c.dry) TTR_TRY(eig_trunc<T>(gbuf, cc, keig, lam, U, Pf, Sf, tails + n, eflag, escr, c.s));
    int64_t kn = kcap;
    if (eps0 > 0.0 && !c.dry) {
      TTR_TRY(select_rank(lam, (int)cc, dnorm, eps0, N, (int)kcap, dk + n, tails + n, c.s));
      int hk = 0;
      TTR_HIP(hipMemcpyAsync(&hk, dk + n, sizeof(int), hipMemcpyDeviceToHost, c.s));
      TTR_HIP(hipStreamSynchronize(c.s));
      if (hk < 1 || hk > kcap) return fail(TT_ENUMERIC, "tt_round_svd: invalid truncation rank");
      kn = hk;
    }
    k[n] = kn;
    // B = A S_k^T (m x kn); B = Q' R' (thin QR, restores orthonormality lost
    // to the squared conditioning of the Gram); V(X_n) <- Q';
    // H(X_{n+1}) <- (R' P_k^T) H(X_{n+1})
    const int64_t cols = dims[n] * left[n + 1];
    auto issue = [&](int64_t kk) -> int {
      Gemm<T> a;
      a.A = xs[n];
      a.lda = cc;
      a.a_kc = true;
      a.B = Sf;
      a.ldb = cc;
      a.b_kc = true;
      a.C = spare;
      a.ldc = kk;
      a.M = m;
      a.N = kk;
      a.K = cc;
      TTR_TRY(gemm(c, a));
      c.partial_need = std::max(c.partial_need, qr_partial_elems(m, kk) * sizeof(double));
      if (!c.dry) {
        qs.partial = c.partial;
        TTR_TRY(qr_thin<T>(spare, qb, m, kk, qs, c.s));
      }
      Gemm<T> r;  // R' = Q'^T B (kk x kk)
      r.A = qb;
      r.lda = kk;
      r.a_kc = false;
      r.B = spare;
      r.ldb = kk;
      r.b_kc = false;
      r.C = rt;
      r.ldc = kk;
      r.M = kk;
      r.N = kk;
      r.K = m;
      TTR_TRY(gemm(c, r));
      Gemm<T> q;  // C = R' P_k^T (kk x cc)
      q.A = rt;
      q.lda = kk;
      q.a_kc = true;
      q.B = Pf;
      q.ldb = keig;
      q.b_kc = true;
      q.C = cbuf;
      q.ldc = cc;
      q.M = kk;
      q.N = cc;
      q.K = kk;
      TTR_TRY(gemm(c, q));
      Gemm<T> b;  // H(X_{n+1}) <- C H(X_{n+1})  (kk x cols)
      b.A = cbuf;
      b.lda = cc;
      b.a_kc = true;
      b.B = xs[n + 1];
      b.ldb = cols;
      b.b_kc = false;
      b.C = spare;
      b.ldc = cols;
      b.M = kk;
      b.N = cols;
      b.K = cc;
      return gemm(c, b);
    };
    if (c.dry) {
      for (int64_t kk = 1; kk <= kcap; ++kk) TTR_TRY(issue(kk));  // any eps rank
    } else {
      TTR_TRY(issue(kn));
      std::swap(xs[n], qb);     // Q' is the new core n
      std::swap(xs[n + 1], spare);
    }
  }
  for (int n = 1; n <= N; ++n) {
    const int64_t cnt = k[n - 1] * dims[n - 1] * (n == N ? 1 : k[n]);
    if (!c.dry) TTR_TRY(copy2d<T>(out[n - 1], 1, xs[n], 1, cnt, 1, 1.0, 0.0, c.s));
  }
  if (out_ranks)
    for (int n = 0; n <= N; ++n) out_ranks[n] = k[n];
  return TT_OK;
}

// Sketch cores in the workspace, in the mode's sketch storage type.

int sketch_exec(Ctx &c, const Problem &P, const Prec &p, std::vector<void *> &Sk);

// ---------------------------------------------------------------- TT-GMRES
// Section 4.2: right-preconditioned GMRES on TTs whose sums are rounded by
// Algorithm 7 to a tolerance (the section 3.2 remark after Algorithm 5).
// With x_0 = 0, beta = ||f||, V_1 = f / beta, step k:
//   Y = (P x I ... x I) V_k
//   W = round(sum_t (A_{t,1} x ... x A_{t,N}) Y)        sketch seed + 2k - 1
//   h_jk = <V_j, W>, j = 1..k                           (Algorithm 3 + first cores)
//   Z = round(W - sum_j h_jk V_j),  V_{k+1} = Z / ||Z||  sketch seed + 2k
// (||Z|| is the norm of Z's first core: the truncation leaves cores 2..N
// right-orthogonal), Givens rotations of the Hessenberg column on the host
// (k+1 scalars), residual estimate |g_{k+1}| / beta; at the end
// x = (P x I ..) round(sum_j y_j V_j) (seed + 2m + 1).
struct GmresSpec {
  int N = 0, T = 0;
  std::vector<int64_t> dims;
  const void *const *mats = nullptr;  // [T * N], null = identity
  const void *precond = nullptr;      // I_1 x I_1 or null
  std::vector<int64_t> fr;            // ranks of f
  const void *const *f = nullptr;
  int64_t lmax = 0;
  double round_eps = 0.0, tol = 0.0;
  int max_iter = 0;
  uint64_t seed = 0;
};

// out (caller buffers of capacity l x I x l) = sum_j coeffs[j] X_j rounded to
// eps0 (sketch rank lmax); ranks to out_ranks.  Scratch is rolled back.
template <typename T>
int round_eps_into(Ctx &c, int N, const int64_t *dims, const std::vector<const T *> &cores,
                   const std::vector<std::vector<int64_t>> &ranks,
                   const std::vector<double> &coeffs, int64_t lmax, double eps0, uint64_t seed,
                   T *const *out, std::vector<int64_t> &out_ranks) {
  const int s = (int)ranks.size();
  std::vector<int64_t> flat;
  for (const auto &r : ranks) flat.insert(flat.end(), r.begin(), r.end());
  Problem P;
  TTR_TRY(make_problem(P, s, N, dims, flat.data(), lmax, 0, coeffs.data()));
  out_ranks.assign(N + 1, 1);
  P.eps_mode = true;
  P.eps0 = eps0;
  P.truncate = true;
  P.ranks_out = out_ranks.data();
  Prec pc;
  TTR_TRY(prec_cfg(TT_PREC_F64, pc));
  const size_t mark = c.arena.off;
  std::vector<void *> Skw;
  TTR_TRY(sketch_exec(c, P, pc, Skw));
  if (!c.dry)
    TTR_TRY(sketch_generate(seed, N, P.dims.data(), P.ell.data(), (int)pc.sk,
                            (void *const *)Skw.data(), c.s));
  TTR_TRY(round_exec<T>(c, P, pc, cores.data(), (const void *const *)Skw.data(), out));
  c.peak = std::max(c.peak, c.arena.off);
  c.arena.off = mark;
  return TT_OK;
}

// out[j] = <X_j, Y> (device) for s TTs X_j against one TT Y
template <typename T>
int tt_dots(Ctx &c, int N, const int64_t *dims, const std::vector<const T *> &X,
            const std::vector<std::vector<int64_t>> &xr, const T *const *Y,
            const std::vector<int64_t> &yr, double *out) {
  const int s = (int)xr.size();
  if (s > kFirstDotsMax) return fail(TT_EINVAL, "internal: too many inner products");
  const size_t mark = c.arena.off;
  std::vector<T *> W(N, nullptr);
  for (int n = 1; n <= N - 1; ++n) {
    int64_t rows = 0;
    for (int j = 0; j < s; ++j) rows += xr[j][n];
    W[n] = c.arena.take<T>((size_t)(rows * yr[n]));
  }
  Prec pc;
  TTR_TRY(prec_cfg(TT_PREC_F64, pc));
  std::vector<const int64_t *> Rj(s);
  for (int j = 0; j < s; ++j) Rj[j] = xr[j].data();
  TTR_TRY(wchain<T>(c, pc, false, N, dims, s, Rj.data(), X.data(), yr.data(),
                    (const void *const *)Y, W.data()));
  if (!c.dry) {
    FirstDots<T> a;
    int64_t off = 0;
    for (int j = 0; j < s; ++j) {
      a.X[j] = X[(size_t)j * N];
      a.W[j] = W[1] + off * yr[1];
      a.r[j] = (int)xr[j][1];
      off += xr[j][1];
    }
    a.Y = Y[0];
    a.I = (int)dims[0];
    a.ry = (int)yr[1];
    a.out = out;
    TTR_TRY(first_dots<T>(a, s, c.s));
  }
  c.peak = std::max(c.peak, c.arena.off);
  c.arena.off = mark;
  return TT_OK;
}

// core n (r0 x I x r1) <- M core n along the mode index (batched over r0)
template <typename T>
int apply_mode(Ctx &c, const T *M, const T *core, T *dst, int64_t r0, int64_t I, int64_t r1) {
  Gemm<T> g;
  g.A = M;
  g.lda = I;
  g.a_kc = true;
  g.B = core;
  g.ldb = r1;
  g.b_kc = false;
  g.C = dst;
  g.ldc = r1;
  g.M = I;
  g.N = r1;
  g.K = I;
  g.batch = r0;
  g.sA = 0;
  g.sB = I * r1;
  g.sC = I * r1;
  return gemm(c, g);
}

template <typename T>
int gmres_exec(Ctx &c, const GmresSpec &S, T *const *x_out, int64_t *x_ranks, double *res,
               int32_t *iters) {
  const int N = S.N, m = S.max_iter, Tn = S.T;
  const int64_t *dims = S.dims.data();
  const int64_t l = S.lmax;
  int64_t Imax = 1;
  for (int n = 0; n < N; ++n) Imax = std::max(Imax, dims[n]);
  int64_t fmax = 1;
  for (int n = 0; n < N; ++n) fmax = std::max(fmax, S.fr[n] * dims[n] * S.fr[n + 1]);
  const size_t cap = (size_t)std::max<int64_t>(l * l * Imax, fmax);
  std::vector<std::vector<T *>> V(m + 2, std::vector<T *>(N, nullptr));
  for (int k = 1; k <= m + 1; ++k)
    for (int n = 0; n < N; ++n) V[k][n] = c.arena.take<T>(cap);
  std::vector<T *> Wc(N), terms((size_t)Tn * N, nullptr);
  for (int n = 0; n < N; ++n) Wc[n] = c.arena.take<T>(cap);
  for (int t = 0; t < Tn; ++t)
    for (int n = 0; n < N; ++n)
      if (S.mats[(size_t)t * N + n]) terms[(size_t)t * N + n] = c.arena.take<T>(cap);
  T *y1 = c.arena.take<T>(cap), *u1 = c.arena.take<T>(cap);
  double *dots = c.arena.take<double>((size_t)m + 2);
  std::vector<std::vector<int64_t>> vr(m + 2);
  // beta = ||f|| and V_1 = f / beta
  std::vector<const T *> fc(N);
  for (int n = 0; n < N; ++n) fc[n] = static_cast<const T *>(S.f[n]);
  double beta = 1.0;
  {
    TTR_TRY(tt_dots<T>(c, N, dims, fc, {S.fr}, fc.data(), S.fr, dots));
    if (!c.dry) {
      TTR_HIP(hipMemcpyAsync(&beta, dots, sizeof(double), hipMemcpyDeviceToHost, c.s));
      TTR_HIP(hipStreamSynchronize(c.s));
      if (!(beta > 0.0) || !std::isfinite(beta)) return fail(TT_EINVAL, "tt_gmres: f is zero");
      beta = std::sqrt(beta);
    }
    for (int n = 0; n < N; ++n)
      if (!c.dry)
        TTR_TRY(copy2d<T>(V[1][n], 1, fc[n], 1, S.fr[n] * dims[n] * S.fr[n + 1], 1,
                          n == 0 ? 1.0 / beta : 1.0, 0.0, c.s));
    vr[1] = S.fr;
  }
  std::vector<double> Hc((size_t)(m + 1) * m, 0.0), cs(m, 0.0), sn(m, 0.0), g(m + 1, 0.0);
  g[0] = beta;
  if (res) res[0] = 1.0;
  int done = 0;
  for (int k = 1; k <= m; ++k) {
    // Y = (P x I ..) V_k
    const T *Ycore0 = V[k][0];
    if (S.precond) {
      TTR_TRY(apply_mode<T>(c, static_cast<const T *>(S.precond), V[k][0], y1, 1, dims[0],
                            vr[k][1]));
      Ycore0 = y1;
    }
    // operator terms and W
    std::vector<const T *> tc((size_t)Tn * N);
    std::vector<std::vector<int64_t>> tr(Tn, vr[k]);
    for (int t = 0; t < Tn; ++t)
      for (int n = 0; n < N; ++n) {
        const T *src = n == 0 ? Ycore0 : V[k][n];
        const T *M = static_cast<const T *>(S.mats[(size_t)t * N + n]);
        if (M) {
          TTR_TRY(apply_mode<T>(c, M, src, terms[(size_t)t * N + n], vr[k][n], dims[n],
                                vr[k][n + 1]));
          src = terms[(size_t)t * N + n];
        }
        tc[(size_t)t * N + n] = src;
      }
    std::vector<int64_t> wr;
    TTR_TRY(round_eps_into<T>(c, N, dims, tc, tr, std::vector<double>(Tn, 1.0), l, S.round_eps,
                              S.seed + 2 * (uint64_t)k - 1, Wc.data(), wr));
    // h_jk = <V_j, W>
    std::vector<const T *> vc;
    std::vector<std::vector<int64_t>> vrs;
    for (int j = 1; j <= k; ++j) {
      for (int n = 0; n < N; ++n) vc.push_back(V[j][n]);
      vrs.push_back(vr[j]);
    }
    TTR_TRY(tt_dots<T>(c, N, dims, vc, vrs, Wc.data(), wr, dots));
    std::vector<double> h(k + 1, 0.0);
    if (!c.dry) {
      TTR_HIP(hipMemcpyAsync(h.data(), dots, sizeof(double) * k, hipMemcpyDeviceToHost, c.s));
      TTR_HIP(hipStreamSynchronize(c.s));
    }
    // Z = W - sum_j h_jk V_j, into V_{k+1}
    std::vector<const T *> zc;
    std::vector<std::vector<int64_t>> zr;
    std::vector<double> zco;
    for (int n = 0; n < N; ++n) zc.push_back(Wc[n]);
    zr.push_back(wr);
    zco.push_back(1.0);
    for (int j = 1; j <= k; ++j) {
      for (int n = 0; n < N; ++n) zc.push_back(V[j][n]);
      zr.push_back(vr[j]);
      zco.push_back(-h[j - 1]);
    }
    TTR_TRY(round_eps_into<T>(c, N, dims, zc, zr, zco, l, S.round_eps, S.seed + 2 * (uint64_t)k,
                              V[k + 1].data(), vr[k + 1]));
    double hz = 1.0;
    if (!c.dry) {
      TTR_TRY(frob_norm<T>(V[k + 1][0], dims[0] * vr[k + 1][1], dots, c.s));
      TTR_HIP(hipMemcpyAsync(&hz, dots, sizeof(double), hipMemcpyDeviceToHost, c.s));
      TTR_HIP(hipStreamSynchronize(c.s));
      if (!(hz > 0.0) || !std::isfinite(hz)) hz = 0.0;
      if (hz > 0.0)
        TTR_TRY(copy2d<T>(V[k + 1][0], 1, V[k + 1][0], 1, dims[0] * vr[k + 1][1], 1, 1.0 / hz,
                          0.0, c.s));
    }
    h[k] = hz;
    // Givens rotations of the new Hessenberg column
    for (int j = 0; j < k - 1; ++j) {
      const double a = h[j], b = h[j + 1];
      h[j] = cs[j] * a + sn[j] * b;
      h[j + 1] = -sn[j] * a + cs[j] * b;
    }
    const double r = std::hypot(h[k - 1], h[k]);
    cs[k - 1] = r > 0.0 ? h[k - 1] / r : 1.0;
    sn[k - 1] = r > 0.0 ? h[k] / r : 0.0;
    h[k - 1] = r;
    h[k] = 0.0;
    for (int j = 0; j <= k; ++j) Hc[(size_t)j * m + (k - 1)] = h[j];
    g[k] = -sn[k - 1] * g[k - 1];
    g[k - 1] = cs[k - 1] * g[k - 1];
    const double est = std::fabs(g[k]) / beta;
    if (res) res[k] = est;
    done = k;
    if (!c.dry && (est <= S.tol || hz == 0.0)) break;
  }
  // y from the triangular system, x = (P x I ..) round(sum_j y_j V_j)
  std::vector<double> y(done, 0.0);
  for (int i = done - 1; i >= 0; --i) {
    double acc = g[i];
    for (int j = i + 1; j < done; ++j) acc -= Hc[(size_t)i * m + j] * y[j];
    const double d = Hc[(size_t)i * m + i];
    y[i] = d != 0.0 ? acc / d : 0.0;
  }
  std::vector<const T *> uc;
  std::vector<std::vector<int64_t>> ur;
  for (int j = 1; j <= done; ++j) {
    for (int n = 0; n < N; ++n) uc.push_back(V[j][n]);
    ur.push_back(vr[j]);
  }
  std::vector<T *> uout(N);
  uout[0] = S.precond ? u1 : x_out[0];
  for (int n = 1; n < N; ++n) uout[n] = x_out[n];
  std::vector<int64_t> xr;
  TTR_TRY(round_eps_into<T>(c, N, dims, uc, ur, y, l, S.round_eps, S.seed + 2 * (uint64_t)done + 1,
                            uout.data(), xr));
  if (S.precond)
    TTR_TRY(apply_mode<T>(c, static_cast<const T *>(S.precond), u1, x_out[0], 1, dims[0], xr[1]));
  if (x_ranks)
    for (int n = 0; n <= N; ++n) x_ranks[n] = xr[n];
  if (iters) *iters = done;
  return TT_OK;
}

// ---------------------------------------------------------------- Algorithm 4
// Orthogonalize-then-Randomize: Algorithm 1 on working copies of the input,
// then the sweep of Algorithm 5 with the Gaussian matrices Omega_n (R_n x
// l_n, drawn on the device like a sketch core keyed by seed + n) in place of
// the partial contractions, then the same truncation.
struct OrthPlan {
  int N = 0;
  std::vector<int64_t> dims, R, rr;
  int64_t core_max = 1, max_c = 1;
};

int make_orth_plan(OrthPlan &P, int N, const int64_t *dims, const int64_t *ranks) {
  TTR_TRY(check_shape(N, dims, ranks, "tt_round_orth_rand"));
  P.N = N;
  P.dims.assign(dims, dims + N);
  P.R.assign(ranks, ranks + N + 1);
  P.rr.assign(N + 1, 1);
  for (int n = N; n >= 2; --n) P.rr[n - 1] = std::min(P.R[n - 1], dims[n - 1] * P.rr[n]);
  for (int n = 0; n < N; ++n) {
    P.core_max = std::max(P.core_max, P.R[n] * dims[n] * P.R[n + 1]);
    P.max_c = std::max(P.max_c, P.R[n]);
  }
  if (N > 1 && P.max_c > TT_MAX_SKETCH_RANK)
    return fail(TT_EUNSUPPORTED, "tt_round_orth_rand: a bond rank above TT_MAX_SKETCH_RANK");
  return TT_OK;
}

template <typename T>
int orth_rand_exec(Ctx &c, const OrthPlan &O, const Problem &P2, const Prec &p,
                   const T *const *Y, uint64_t seed, T *const *out) {
  const int N = O.N;
  const int64_t *dims = O.dims.data();
  std::vector<T *> xs(N + 1, nullptr);
  for (int n = 1; n <= N; ++n) xs[n] = c.arena.take<T>((size_t)O.core_max);
  T *spare = c.arena.take<T>((size_t)O.core_max);
  T *pan = c.arena.take<T>((size_t)O.core_max);
  T *qb = c.arena.take<T>((size_t)O.core_max);
  const int64_t lc = O.max_c;
  T *rt = c.arena.take<T>((size_t)(lc * lc));
  QrScratch qs;
  qs.gram = c.arena.take<double>((size_t)std::max(lc * lc, 2 * lc));
  qs.rinv = c.arena.take<double>((size_t)std::max(lc * lc, 2 * lc));
  if (sizeof(T) == 4) qs.rinv_f = c.arena.take<float>((size_t)(lc * lc));
  qs.q1 = c.arena.take<T>((size_t)O.core_max);
  qs.flag = c.arena.take<int>(4);
  for (int n = 1; n <= N; ++n)
    if (!c.dry)
      TTR_TRY(copy2d<T>(xs[n], 1, Y[n - 1], 1, O.R[n - 1] * dims[n - 1] * O.R[n], 1, 1.0, 0.0,
                        c.s));
  std::vector<int64_t> left(O.R.begin(), O.R.end());
  TTR_TRY(orth_rl<T>(c, N, dims, O.rr, xs, spare, pan, qb, rt, qs, left));
  // Omega_n (R_n x l_n), n = 1..N-1
  std::vector<T *> om(N, nullptr);
  for (int n = 1; n <= N - 1; ++n) {
    const int64_t cnt = O.rr[n] * P2.ell[n];
    om[n] = c.arena.take<T>((size_t)cnt);
    if (!c.dry) {
      const int64_t d1[1] = {cnt}, r1[2] = {1, 1};
      void *ptr = om[n];
      TTR_TRY(sketch_generate(seed + (uint64_t)n, 1, d1, r1, (int)p.store, &ptr, c.s));
    }
  }
  std::vector<const T *> cores(N);
  for (int n = 0; n < N; ++n) cores[n] = xs[n + 1];
  return round_exec<T>(c, P2, p, cores.data(), nullptr, out, om.data());
}

int sketch_exec(Ctx &c, const Problem &P, const Prec &p, std::vector<void *> &Sk) {
  Sk.assign(P.N, nullptr);
  for (int n = 0; n < P.N; ++n)
    Sk[n] = c.arena.take<char>((size_t)(P.ell[n] * P.dims[n] * P.ell[n + 1]) * dtype_bytes(p.sk));
  return TT_OK;
}

// Runs `body(ctx)` twice: dry to size the split-K buffer, then for real with
// the partial buffer first in the workspace.
template <typename F>
int run_with_workspace(void *workspace, size_t ws_bytes, hipStream_t s, F body) {
  read_env();  // the query and the run see the same path choices
  Ctx dry;
  dry.dry = true;
  TTR_TRY(body(dry));
  const size_t partial_bytes = (dry.partial_need + 255) & ~size_t(255);
  const size_t need = partial_bytes + std::max(dry.arena.off, dry.peak);
  if (!workspace && need > 0) return fail(TT_EINVAL, "null workspace");
  if (ws_bytes < need)
    return fail(TT_ENOMEM, "workspace too small: need " + std::to_string(need) + " bytes");
  if (reinterpret_cast<uintptr_t>(workspace) % 256 != 0)
    return fail(TT_EINVAL, "workspace must be 256-byte aligned");
  Ctx real;
  real.dry = false;
  real.s = s;
  real.arena.base = static_cast<char *>(workspace);
  real.partial = real.arena.take<char>(dry.partial_need);
  real.partial_cap = dry.partial_need;
  real.arena.off = partial_bytes;
  return body(real);
}

template <typename F>
int measure_workspace(F body, size_t *bytes) {
  if (!bytes) return fail(TT_EINVAL, "null bytes pointer");
  read_env();
  Ctx dry;
  dry.dry = true;
  TTR_TRY(body(dry));
  *bytes = ((dry.partial_need + 255) & ~size_t(255)) + std::max(dry.arena.off, dry.peak);
  return TT_OK;
}

}  // namespace
}  // namespace ttr

using namespace ttr;

extern "C" {

const char *tt_last_error(void) { return g_err.c_str(); }

int tt_version(void) { return 100; }

int tt_round_rand_plan(int32_t N, const int64_t *dims, const int64_t *ranks, int64_t target_rank,
                       int64_t oversample, int64_t *sketch_ranks, int64_t *out_ranks) {
  TTR_TRY(check_shape(N, dims, ranks, "tt_round_rand_plan"));
  if (target_rank < 1) return fail(TT_EINVAL, "target_rank must be >= 1");
  if (oversample < 0) return fail(TT_EINVAL, "oversample must be >= 0");
  if (!sketch_ranks || !out_ranks) return fail(TT_EINVAL, "null output arrays");
  std::vector<int64_t> ell, out;
  plan_ranks(N, dims, ranks, target_rank, oversample, ell, out);
  for (int n = 0; n <= N; ++n) {
    sketch_ranks[n] = ell[n];
    out_ranks[n] = out[n];
  }
  return TT_OK;
}

int tt_round_rand_workspace(int32_t N, const int64_t *dims, const int64_t *ranks,
                            int64_t target_rank, int64_t oversample, int32_t prec, size_t *bytes) {
  return tt_sum_round_workspace(1, N, dims, ranks, target_rank, oversample, prec, bytes);
}

static int sum_round_workspace_mode(int32_t s, int32_t N, const int64_t *dims,
                                    const int64_t *ranks, int64_t target_rank,
                                    int64_t oversample, int32_t prec, bool eps_mode,
                                    size_t *bytes) {
  Problem P;
  TTR_TRY(make_problem(P, s, N, dims, ranks, target_rank, oversample, nullptr));
  if (eps_mode) {
    P.eps_mode = true;
    P.truncate = true;
  }
  Prec pc;
  TTR_TRY(prec_cfg(prec, pc));
  if (!bytes) return fail(TT_EINVAL, "null bytes pointer");
  if (N == 1) {
    *bytes = 0;
    return TT_OK;
  }
  return measure_workspace(
      [&](Ctx &c) -> int {
        std::vector<void *> Sk;
        TTR_TRY(sketch_exec(c, P, pc, Sk));
        if (pc.store == DType::F64) {
          std::vector<const double *> Y((size_t)s * N, nullptr);
          std::vector<double *> out(N, nullptr);
          return round_exec<double>(c, P, pc, Y.data(), (const void *const *)Sk.data(),
                                    out.data());
        }
        std::vector<const float *> Y((size_t)s * N, nullptr);
        std::vector<float *> out(N, nullptr);
        return round_exec<float>(c, P, pc, Y.data(), (const void *const *)Sk.data(), out.data());
      },
      bytes);
}
int tt_sum_round_workspace(int32_t s, int32_t N, const int64_t *dims, const int64_t *ranks,
                           int64_t target_rank, int64_t oversample, int32_t prec,
                           size_t *bytes) {
  return sum_round_workspace_mode(s, N, dims, ranks, target_rank, oversample, prec, false, bytes);
}
int tt_sum_round_eps_workspace(int32_t s, int32_t N, const int64_t *dims, const int64_t *ranks,
                               int64_t max_rank, int32_t prec, size_t *bytes) {
  return sum_round_workspace_mode(s, N, dims, ranks, max_rank, 0, prec, true, bytes);
}
int tt_round_rand_eps_workspace(int32_t N, const int64_t *dims, const int64_t *ranks,
                                int64_t max_rank, int32_t prec, size_t *bytes) {
  return sum_round_workspace_mode(1, N, dims, ranks, max_rank, 0, prec, true, bytes);
}

int tt_make_sketch(uint64_t seed, int32_t N, const int64_t *dims, const int64_t *sketch_ranks,
                   int32_t dtype, void *const *cores, void *stream) {
  TTR_TRY(check_shape(N, dims, sketch_ranks, "tt_make_sketch"));
  TTR_TRY(check_ptrs(N, cores, "tt_make_sketch"));
  if (dtype != TT_F64 && dtype != TT_F32 && dtype != TT_BF16)
    return fail(TT_EINVAL, "unknown dtype");
  return sketch_generate(seed, N, dims, sketch_ranks, dtype, cores, (hipStream_t)stream);
}

}  // extern "C"

namespace ttr {
namespace {

// The speculative form synchronises with its stream at the end: not under
// stream capture, not in tolerance mode (which reads back ranks per bond and
// keeps its second pass), not for callers that set g_spec_off, and not with
// TT_SPECULATE=0 in the environment.
bool speculation_allowed(const Problem &P, hipStream_t s) {
  if (P.eps_mode || g_spec_off) return false;
  const char *e = std::getenv("TT_SPECULATE");
  if (e && !std::strcmp(e, "0")) return false;
  hipStreamCaptureStatus st = hipStreamCaptureStatusNone;
  if (hipStreamIsCapturing(s, &st) != hipSuccess) return false;
  return st == hipStreamCaptureStatusNone;
}

template <typename T>
int round_typed(const Problem &P, const Prec &pc, const void *const *cores, bool gen,
                       uint64_t seed, const void *const *sketch_cores, void *const *out_cores,
                       void *workspace, size_t ws_bytes, hipStream_t st) {
  const int N = P.N, s = P.s;
  if (N == 1) {
    // a single core: the (weighted) sum itself
    const int64_t cnt = P.dims[0];
    T *dst = (T *)out_cores[0];
    for (int j = 0; j < s; ++j)
      TTR_TRY(copy2d<T>(dst, cnt, (const T *)cores[j], cnt, 1, cnt, P.coeffs[j],
                        j == 0 ? 0.0 : 1.0, st));
    return TT_OK;
  }
  const T *const *Y = (const T *const *)cores;
  T *const *out = (T *const *)out_cores;
  return run_with_workspace(workspace, ws_bytes, st, [&](Ctx &c) -> int {
    std::vector<void *> Skw;
    TTR_TRY(sketch_exec(c, P, pc, Skw));  // same layout with a given sketch
    std::vector<const void *> Sk(N, nullptr);
    if (gen) {
      if (!c.dry)
        TTR_TRY(sketch_generate(seed, N, P.dims.data(), P.ell.data(), (int)pc.sk,
                                (void *const *)Skw.data(), c.s));
      for (int n = 0; n < N; ++n) Sk[n] = Skw[n];
    } else if (pc.sk == pc.store) {
      for (int n = 0; n < N; ++n) Sk[n] = sketch_cores[n];
    } else {
      // caller's FP32 sketch rounded to the BF16 the partial contractions read
      for (int n = 0; n < N; ++n) {
        if (!c.dry)
          TTR_TRY(round_to_bf16((__bf16 *)Skw[n], (const float *)sketch_cores[n],
                                P.ell[n] * P.dims[n] * P.ell[n + 1], c.s));
        Sk[n] = Skw[n];
      }
    }
    // Speculative form when the call may wait for its stream: the rescue
    // launches that a well-conditioned input never needs are left out, the
    // flags are read back after the sweep and after the truncation, and a
    // phase with a set flag is redone guarded (round_exec).  Under stream
    // capture, in tolerance mode and for callers that cannot wait, the guarded
    // form runs directly.
    Problem Q = P;
    Q.spec = speculation_allowed(P, c.s);
    return round_exec<T>(c, Q, pc, Y, Sk.data(), out);
  });
}

// with eps0 >= 0: tolerance-driven rounding (target_rank = the largest rank
// l, no oversampling; the ranks chosen go to ranks_out)
void set_eps_mode(Problem &P, double eps0, int64_t *ranks_out) {
  P.eps_mode = eps0 > 0.0;
  P.eps0 = eps0;
  P.truncate = P.eps_mode;
  P.ranks_out = ranks_out;
}

int round_common(int32_t s, int32_t N, const int64_t *dims, const int64_t *ranks,
                        const void *const *cores, const double *coeffs, int32_t dtype,
                        int64_t target_rank, int64_t oversample, bool gen, uint64_t seed,
                        const int64_t *sketch_ranks, const void *const *sketch_cores,
                        int32_t prec, void *const *out_cores, void *workspace, size_t ws_bytes,
                        void *stream, double eps0 = -1.0, int64_t *ranks_out = nullptr) {
  read_env();
  Problem P;
  TTR_TRY(make_problem(P, s, N, dims, ranks, target_rank, oversample, coeffs));
  if (eps0 >= 0.0) {
    if (!(eps0 < 1.0)) return fail(TT_EINVAL, "eps0 must lie in [0, 1)");
    if (!ranks_out) return fail(TT_EINVAL, "null out_ranks");
    set_eps_mode(P, eps0, ranks_out);
    if (N == 1) {
      ranks_out[0] = ranks_out[1] = 1;
    }
  }
  Prec pc;
  TTR_TRY(prec_cfg(prec, pc));
  TTR_TRY(check_dtype(dtype, pc));
  TTR_TRY(check_ptrs(s * N, cores, "input cores"));
  TTR_TRY(check_ptrs(N, out_cores, "output cores"));
  if (!gen) {
    if (!sketch_ranks) return fail(TT_EINVAL, "null sketch ranks");
    for (int n = 0; n <= N; ++n)
      if (sketch_ranks[n] != P.ell[n])
        return fail(TT_EINVAL, "sketch ranks differ from the plan's sketch ranks");
    TTR_TRY(check_ptrs(N, sketch_cores, "sketch cores"));
  }
  hipStream_t st = (hipStream_t)stream;
  if (pc.store == DType::F64)
    return round_typed<double>(P, pc, cores, gen, seed, sketch_cores, out_cores, workspace,
                               ws_bytes, st);
  return round_typed<float>(P, pc, cores, gen, seed, sketch_cores, out_cores, workspace,
                            ws_bytes, st);
}

// ---------------------------------------------------------------- Algorithm 6
// Two-Sided-Randomization (generalized Nystrom) in FP64.  Ranks: l_n from
// plan_ranks with no oversampling (the output ranks), right sketch ranks
// rho_n = ceil(3 l_n / 2) capped by I_{n+1} ... I_N.
void plan_two_sided(int N, const int64_t *dims, const int64_t *R, int64_t target,
                    std::vector<int64_t> &ell, std::vector<int64_t> &rho) {
  std::vector<int64_t> out;
  plan_ranks(N, dims, R, target, 0, ell, out);
  const int64_t big = int64_t(1) << 40;
  std::vector<int64_t> w(N + 1, 1);
  for (int n = N - 1; n >= 1; --n) w[n] = std::min(big, dims[n] * w[n + 1]);
  rho.assign(N + 1, 1);
  for (int n = 1; n <= N - 1; ++n) rho[n] = std::min((3 * ell[n] + 1) / 2, w[n]);
}

constexpr double kNystromRcond = 1e-6;

// Y (ranks R) -> X (ranks L) with left sketch SkL (ranks L) and right sketch
// SkR (ranks P); every step is a GEMM except the eigensolve and the scaling.
int two_sided_exec(Ctx &c, const Prec &p, int N, const int64_t *dims, const int64_t *R,
                   const double *const *Y, const int64_t *L, const int64_t *P,
                   const double *const *SkL, const double *const *SkR, double *const *out) {
  typedef double T;
  std::vector<T *> WR(N, nullptr), WL(N, nullptr), Lf(N, nullptr), Rf(N, nullptr);
  int64_t lmax = 1, pmax = 1, zmax = 1, tmax = 1;
  for (int n = 1; n <= N - 1; ++n) {
    WR[n] = c.arena.take<T>((size_t)(R[n] * P[n]));
    WL[n] = c.arena.take<T>((size_t)(L[n] * R[n]));
    Lf[n] = c.arena.take<T>((size_t)(R[n] * L[n]));
    Rf[n] = c.arena.take<T>((size_t)(L[n] * R[n]));
    lmax = std::max(lmax, L[n]);
    pmax = std::max(pmax, P[n]);
    if (n >= 2) {
      zmax = std::max(zmax, L[n - 1] * dims[n - 1] * R[n]);
      tmax = std::max(tmax, R[n - 1] * dims[n - 1] * L[n]);
    }
  }
  T *zb = c.arena.take<T>((size_t)zmax);
  T *tb = c.arena.take<T>((size_t)tmax);
  // per-bond slots (bond n in slot n - 1) of the factor computation, so
  // that the eigensolves of all bonds run in one launch each
  const int nbond = N - 1;
  const int64_t sC = lmax * pmax, sG = lmax * lmax;
  T *Cb = c.arena.take<T>((size_t)(sC * nbond));
  T *Bb = c.arena.take<T>((size_t)(sC * nbond));
  T *Gb = c.arena.take<T>((size_t)(sG * nbond));
  T *lam = c.arena.take<T>((size_t)(lmax * nbond));
  T *U1 = c.arena.take<T>((size_t)(sG * nbond));
  T *U2 = c.arena.take<T>((size_t)(sG * nbond));
  T *Ub = c.arena.take<T>((size_t)(sG * nbond));
  T *A1 = c.arena.take<T>((size_t)(sG * nbond));
  T *A2 = c.arena.take<T>((size_t)(sG * nbond));
  T *Eb = c.arena.take<T>((size_t)(pmax * lmax));
  std::vector<int> nl(nbond);
  for (int n = 1; n <= N - 1; ++n) nl[n - 1] = (int)L[n];
  auto mm = [&](const T *A, int64_t lda, bool a_kc, const T *B, int64_t ldb, bool b_kc, T *C,
                int64_t ldc, int64_t M, int64_t Nn, int64_t K) {
    Gemm<T> g;
    g.A = A;
    g.lda = lda;
    g.a_kc = a_kc;
    g.B = B;
    g.ldb = ldb;
    g.b_kc = b_kc;
    g.C = C;
    g.ldc = ldc;
    g.M = M;
    g.N = Nn;
    g.K = K;
    return gemm(c, g);
  };

  // ---- W^R_n = H(Y_{n+1:N}) H(SkR_{n+1:N})^T (Algorithm 3), R_n x rho_n
  {
    const int64_t *Rj[1] = {R};
    TTR_TRY(wchain<T>(c, p, false, N, dims, 1, Rj, Y, P, (const void *const *)SkR, WR.data()));
  }
  // ---- W^L_n = V(SkL_{1:n})^T V(Y_{1:n}), l_n x R_n (the mirror of Algorithm 3)
  TTR_TRY(mm(SkL[0], L[1], false, Y[0], R[1], false, WL[1], R[1], L[1], R[1], dims[0]));
  for (int n = 2; n <= N - 1; ++n) {
    const int64_t I = dims[n - 1];
    // Z = W^L_{n-1} H(Y_n), read as V(Z): (l_{n-1} I_n) x R_n
    TTR_TRY(mm(WL[n - 1], R[n - 1], true, Y[n - 1], I * R[n], false, zb, I * R[n], L[n - 1],
               I * R[n], R[n - 1]));
    // W^L_n = V(SkL_n)^T V(Z)
    TTR_TRY(mm(SkL[n - 1], L[n], false, zb, R[n], false, WL[n], R[n], L[n], R[n],
               L[n - 1] * I));
  }
  // ---- factors of equation (LnRn) at every bond.  Left singular vectors of
  // C = W^L W^R in two passes: the eigenvectors U1 of C C^T, then those (U2)
  // of B B^T with B = U1^T C, whose rows are already nearly orthogonal, so
  // that Jacobi (with its relative test only) resolves the small singular
  // values to their own relative accuracy instead of that of s_1^2;
  // U = U1 U2, s^2 = eig(B B^T).
  for (int n = 1; n <= N - 1; ++n) {
    const int64_t l = L[n], rho = P[n], r = R[n], o = n - 1;
    TTR_TRY(mm(WL[n], r, true, WR[n], rho, false, Cb + o * sC, rho, l, rho, r));  // C
    TTR_TRY(mm(Cb + o * sC, rho, true, Cb + o * sC, rho, true, Gb + o * sG, l, l, l, rho));
  }
  if (!c.dry) TTR_TRY(sym_eig_batch(Gb, sG, lam, lmax, U1, sG, nl.data(), nbond, false, c.s));
  for (int n = 1; n <= N - 1; ++n) {
    const int64_t l = L[n], rho = P[n], o = n - 1;
    TTR_TRY(mm(U1 + o * sG, l, false, Cb + o * sC, rho, false, Bb + o * sC, rho, l, rho,
               l));  // B = U1^T C
    TTR_TRY(mm(Bb + o * sC, rho, true, Bb + o * sC, rho, true, Gb + o * sG, l, l, l, rho));
  }
  if (!c.dry) TTR_TRY(sym_eig_batch(Gb, sG, lam, lmax, U2, sG, nl.data(), nbond, true, c.s));
  for (int n = 1; n <= N - 1; ++n) {
    const int64_t l = L[n], rho = P[n], r = R[n], o = n - 1;
    T *a1 = A1 + o * sG, *a2 = A2 + o * sG;
    TTR_TRY(mm(U1 + o * sG, l, true, U2 + o * sG, l, false, Ub + o * sG, l, l, l, l));
    if (!c.dry) TTR_TRY(nystrom_scale(lam + o * lmax, Ub + o * sG, l, kNystromRcond, a1, a2, c.s));
    TTR_TRY(mm(Cb + o * sC, rho, false, a1, l, false, Eb, l, rho, l, l));  // E = C^T U diag(h/s)
    TTR_TRY(mm(WR[n], rho, true, Eb, l, false, Lf[n], l, r, l, rho));     // L_n = W^R E
    TTR_TRY(mm(a2, l, true, WL[n], r, false, Rf[n], r, l, r, l));         // R_n = diag(h) U^T W^L
  }
  // ---- cores, each independent of the others
  TTR_TRY(mm(Y[0], R[1], true, Lf[1], L[1], false, out[0], L[1], dims[0], L[1], R[1]));
  for (int n = 2; n <= N - 1; ++n) {
    const int64_t I = dims[n - 1];
    // V(T) = V(Y_n) L_n, then H(X_n) = R_{n-1} H(T)
    TTR_TRY(mm(Y[n - 1], R[n], true, Lf[n], L[n], false, tb, L[n], R[n - 1] * I, L[n], R[n]));
    TTR_TRY(mm(Rf[n - 1], R[n - 1], true, tb, I * L[n], false, out[n - 1], I * L[n], L[n - 1],
               I * L[n], R[n - 1]));
  }
  TTR_TRY(mm(Rf[N - 1], R[N - 1], true, Y[N - 1], dims[N - 1], false, out[N - 1], dims[N - 1],
             L[N - 1], dims[N - 1], R[N - 1]));
  return TT_OK;
}

int two_sided_check(int32_t N, const int64_t *dims, const int64_t *ranks, int64_t target,
                    std::vector<int64_t> &ell, std::vector<int64_t> &rho) {
  TTR_TRY(check_shape(N, dims, ranks, "tt_round_two_sided"));
  if (target < 1) return fail(TT_EINVAL, "target_rank must be >= 1");
  plan_two_sided(N, dims, ranks, target, ell, rho);
  for (int n = 0; n <= N; ++n)
    if (N > 1 && (ell[n] > TT_MAX_SKETCH_RANK || rho[n] > TT_MAX_SKETCH_RANK))
      return fail(TT_EUNSUPPORTED, "sketch rank above TT_MAX_SKETCH_RANK");
  return TT_OK;
}

// Sketch cores in the workspace, then two_sided_exec.
int two_sided_body(Ctx &c, int N, const int64_t *dims, const int64_t *ranks,
                   const std::vector<int64_t> &ell, const std::vector<int64_t> &rho,
                   const double *const *Y, uint64_t seed_l, uint64_t seed_r,
                   double *const *out) {
  Prec p;
  TTR_TRY(prec_cfg(TT_PREC_F64, p));
  std::vector<double *> SkL(N), SkR(N);
  for (int n = 0; n < N; ++n) {
    SkL[n] = c.arena.take<double>((size_t)(ell[n] * dims[n] * ell[n + 1]));
    SkR[n] = c.arena.take<double>((size_t)(rho[n] * dims[n] * rho[n + 1]));
  }
  if (!c.dry) {
    TTR_TRY(sketch_generate(seed_l, N, dims, ell.data(), TT_F64, (void *const *)SkL.data(), c.s));
    TTR_TRY(sketch_generate(seed_r, N, dims, rho.data(), TT_F64, (void *const *)SkR.data(), c.s));
  }
  return two_sided_exec(c, p, N, dims, ranks, Y, ell.data(), rho.data(),
                        (const double *const *)SkL.data(), (const double *const *)SkR.data(),
                        out);
}

}  // namespace
}  // namespace ttr

extern "C" {

int tt_round_rand(int32_t N, const int64_t *dims, const int64_t *ranks, const void *const *cores,
                  int32_t dtype, int64_t target_rank, int64_t oversample, uint64_t sketch_seed,
                  int32_t prec, void *const *out_cores, void *workspace, size_t ws_bytes,
                  void *stream) {
  return round_common(1, N, dims, ranks, cores, nullptr, dtype, target_rank, oversample, true,
                      sketch_seed, nullptr, nullptr, prec, out_cores, workspace, ws_bytes,
                      stream);
}

int tt_round_rand_with_sketch(int32_t N, const int64_t *dims, const int64_t *ranks,
                              const void *const *cores, int32_t dtype, int64_t target_rank,
                              int64_t oversample, const int64_t *sketch_ranks,
                              const void *const *sketch_cores, int32_t prec,
                              void *const *out_cores, void *workspace, size_t ws_bytes,
                              void *stream) {
  return round_common(1, N, dims, ranks, cores, nullptr, dtype, target_rank, oversample, false, 0,
                      sketch_ranks, sketch_cores, prec, out_cores, workspace, ws_bytes, stream);
}

int tt_sum_round(int32_t s, int32_t N, const int64_t *dims, const int64_t *ranks,
                 const void *const *cores, const double *coeffs, int32_t dtype,
                 int64_t target_rank, int64_t oversample, uint64_t sketch_seed, int32_t prec,
                 void *const *out_cores, void *workspace, size_t ws_bytes, void *stream) {
  return round_common(s, N, dims, ranks, cores, coeffs, dtype, target_rank, oversample, true,
                      sketch_seed, nullptr, nullptr, prec, out_cores, workspace, ws_bytes,
                      stream);
}

int tt_round_rand_eps(int32_t N, const int64_t *dims, const int64_t *ranks,
                      const void *const *cores, int32_t dtype, int64_t max_rank, double eps0,
                      uint64_t sketch_seed, int32_t prec, void *const *out_cores,
                      int64_t *out_ranks, void *workspace, size_t ws_bytes, void *stream) {
  return round_common(1, N, dims, ranks, cores, nullptr, dtype, max_rank, 0, true, sketch_seed,
                      nullptr, nullptr, prec, out_cores, workspace, ws_bytes, stream, eps0,
                      out_ranks);
}

int tt_sum_round_eps(int32_t s, int32_t N, const int64_t *dims, const int64_t *ranks,
                     const void *const *cores, const double *coeffs, int32_t dtype,
                     int64_t max_rank, double eps0, uint64_t sketch_seed, int32_t prec,
                     void *const *out_cores, int64_t *out_ranks, void *workspace,
                     size_t ws_bytes, void *stream) {
  return round_common(s, N, dims, ranks, cores, coeffs, dtype, max_rank, 0, true, sketch_seed,
                      nullptr, nullptr, prec, out_cores, workspace, ws_bytes, stream, eps0,
                      out_ranks);
}

int tt_round_svd_plan(int32_t N, const int64_t *dims, const int64_t *ranks, int64_t max_rank,
                      int64_t *out_ranks) {
  if (!out_ranks) return fail(TT_EINVAL, "null out_ranks");
  SvdPlan P;
  TTR_TRY(make_svd_plan(P, N, dims, ranks, max_rank));
  for (int n = 0; n <= N; ++n) out_ranks[n] = (N == 1) ? 1 : P.kmax[n];
  return TT_OK;
}

static int svd_prec(int32_t prec, DType &store) {
  if (prec == TT_PREC_F64) store = DType::F64;
  else if (prec == TT_PREC_F32) store = DType::F32;
  else if (prec == TT_PREC_MIXED_BF16)
    return fail(TT_EUNSUPPORTED, "tt_round_svd has no mixed-precision mode");
  else return fail(TT_EINVAL, "unknown prec");
  return TT_OK;
}

int tt_round_svd_workspace(int32_t N, const int64_t *dims, const int64_t *ranks,
                           int64_t max_rank, int32_t prec, size_t *bytes) {
  SvdPlan P;
  TTR_TRY(make_svd_plan(P, N, dims, ranks, max_rank));
  DType st;
  TTR_TRY(svd_prec(prec, st));
  if (!bytes) return fail(TT_EINVAL, "null bytes pointer");
  if (N == 1) {
    *bytes = 0;
    return TT_OK;
  }
  return measure_workspace(
      [&](Ctx &c) -> int {
        if (st == DType::F64) {
          std::vector<const double *> Y(N, nullptr);
          std::vector<double *> out(N, nullptr);
          return svd_exec<double>(c, P, Y.data(), 1.0, out.data(), nullptr);
        }
        std::vector<const float *> Y(N, nullptr);
        std::vector<float *> out(N, nullptr);
        return svd_exec<float>(c, P, Y.data(), 1.0, out.data(), nullptr);
      },
      bytes);
}

int tt_round_svd(int32_t N, const int64_t *dims, const int64_t *ranks, const void *const *cores,
                 int32_t dtype, double eps0, int64_t max_rank, int32_t prec,
                 void *const *out_cores, int64_t *out_ranks, void *workspace, size_t ws_bytes,
                 void *stream) {
  read_env();
  SvdPlan P;
  TTR_TRY(make_svd_plan(P, N, dims, ranks, max_rank));
  DType st;
  TTR_TRY(svd_prec(prec, st));
  if (dtype != (int32_t)st) return fail(TT_EINVAL, "dtype does not match the precision mode");
  if (!(eps0 >= 0.0) || !std::isfinite(eps0)) return fail(TT_EINVAL, "eps0 must be finite and >= 0");
  if (!out_ranks) return fail(TT_EINVAL, "null out_ranks");
  TTR_TRY(check_ptrs(N, cores, "input cores"));
  TTR_TRY(check_ptrs(N, out_cores, "output cores"));
  hipStream_t sm = (hipStream_t)stream;
  if (N == 1) {
    const int64_t cnt = dims[0];
    if (st == DType::F64)
      TTR_TRY(copy2d<double>((double *)out_cores[0], 1, (const double *)cores[0], 1, cnt, 1, 1.0,
                             0.0, sm));
    else
      TTR_TRY(copy2d<float>((float *)out_cores[0], 1, (const float *)cores[0], 1, cnt, 1, 1.0,
                            0.0, sm));
    out_ranks[0] = out_ranks[1] = 1;
    return TT_OK;
  }
  return run_with_workspace(workspace, ws_bytes, sm, [&](Ctx &c) -> int {
    if (st == DType::F64)
      return svd_exec<double>(c, P, (const double *const *)cores, eps0, (double *const *)out_cores,
                              c.dry ? nullptr : out_ranks);
    return svd_exec<float>(c, P, (const float *const *)cores, eps0, (float *const *)out_cores,
                           c.dry ? nullptr : out_ranks);
  });
}

static int backward_prec(int32_t prec, Prec &pc) {
  TTR_TRY(prec_cfg(prec, pc));
  if (prec == TT_PREC_MIXED_BF16)
    return fail(TT_EUNSUPPORTED, "the adjoint supports TT_PREC_F64 and TT_PREC_F32");
  return TT_OK;
}

int tt_round_rand_backward_workspace(int32_t N, const int64_t *dims, const int64_t *ranks,
                                     int64_t target_rank, int64_t oversample, int32_t prec,
                                     size_t *bytes) {
  Problem P;
  TTR_TRY(make_problem(P, 1, N, dims, ranks, target_rank, oversample, nullptr));
  Prec pc;
  TTR_TRY(backward_prec(prec, pc));
  if (!bytes) return fail(TT_EINVAL, "null bytes pointer");
  if (P.truncate)
    return fail(TT_EUNSUPPORTED, "the adjoint covers roundings without truncation");
  if (N == 1) {
    *bytes = 0;
    return TT_OK;
  }
  return measure_workspace(
      [&](Ctx &c) -> int {
        std::vector<void *> Sk;
        TTR_TRY(sketch_exec(c, P, pc, Sk));
        if (pc.store == DType::F64) {
          std::vector<const double *> Y(N, nullptr), go(N, nullptr);
          std::vector<double *> gi(N, nullptr);
          return backward_exec<double>(c, P, pc, Y.data(), (const void *const *)Sk.data(),
                                       go.data(), gi.data());
        }
        std::vector<const float *> Y(N, nullptr), go(N, nullptr);
        std::vector<float *> gi(N, nullptr);
        return backward_exec<float>(c, P, pc, Y.data(), (const void *const *)Sk.data(), go.data(),
                                    gi.data());
      },
      bytes);
}

int tt_round_rand_backward(int32_t N, const int64_t *dims, const int64_t *ranks,
                           const void *const *cores, int32_t dtype, int64_t target_rank,
                           int64_t oversample, uint64_t sketch_seed, int32_t prec,
                           const void *const *grad_out, void *const *grad_in, void *workspace,
                           size_t ws_bytes, void *stream) {
  read_env();
  Problem P;
  TTR_TRY(make_problem(P, 1, N, dims, ranks, target_rank, oversample, nullptr));
  Prec pc;
  TTR_TRY(backward_prec(prec, pc));
  TTR_TRY(check_dtype(dtype, pc));
  if (P.truncate)
    return fail(TT_EUNSUPPORTED, "the adjoint covers roundings without truncation");
  TTR_TRY(check_ptrs(N, cores, "input cores"));
  TTR_TRY(check_ptrs(N, grad_out, "output cotangents"));
  TTR_TRY(check_ptrs(N, grad_in, "input gradients"));
  hipStream_t st = (hipStream_t)stream;
  if (N == 1) {
    const int64_t cnt = dims[0];
    if (pc.store == DType::F64)
      return copy2d<double>((double *)grad_in[0], 1, (const double *)grad_out[0], 1, cnt, 1, 1.0,
                            0.0, st);
    return copy2d<float>((float *)grad_in[0], 1, (const float *)grad_out[0], 1, cnt, 1, 1.0, 0.0,
                         st);
  }
  return run_with_workspace(workspace, ws_bytes, st, [&](Ctx &c) -> int {
    std::vector<void *> Skw;
    TTR_TRY(sketch_exec(c, P, pc, Skw));
    if (!c.dry)
      TTR_TRY(sketch_generate(sketch_seed, N, P.dims.data(), P.ell.data(), (int)pc.sk,
                              (void *const *)Skw.data(), c.s));
    if (pc.store == DType::F64)
      return backward_exec<double>(c, P, pc, (const double *const *)cores,
                                   (const void *const *)Skw.data(),
                                   (const double *const *)grad_out, (double *const *)grad_in);
    return backward_exec<float>(c, P, pc, (const float *const *)cores,
                                (const void *const *)Skw.data(), (const float *const *)grad_out,
                                (float *const *)grad_in);
  });
}

int tt_timing_start(int32_t site, int32_t capacity) {
  if (site < TT_SITE_WCHAIN_Z || site > TT_SITE_WCHAIN_FUSED) return fail(TT_EINVAL, "unknown site");
  if (capacity < 1 || capacity > (1 << 20)) return fail(TT_EINVAL, "capacity out of range");
  for (hipEvent_t e : g_timer.ev) (void)hipEventDestroy(e);
  g_timer.ev.assign(2 * (size_t)capacity, nullptr);
  for (hipEvent_t &e : g_timer.ev) TTR_HIP(hipEventCreate(&e));
  g_timer.reps.clear();
  g_timer.used = 0;
  g_timer.site = site;
  return TT_OK;
}

int tt_timing_stop(double *total_ms, int32_t *launches) {
  if (!total_ms || !launches) return fail(TT_EINVAL, "null output");
  double t = 0.0;
  for (size_t i = 0; i + 1 < g_timer.used; i += 2) {
    TTR_HIP(hipEventSynchronize(g_timer.ev[i + 1]));
    float ms = 0.f;
    TTR_HIP(hipEventElapsedTime(&ms, g_timer.ev[i], g_timer.ev[i + 1]));
    t += ms / g_timer.reps[i / 2];
  }
  *total_ms = t;
  *launches = (int32_t)(g_timer.used / 2);
  for (hipEvent_t e : g_timer.ev) (void)hipEventDestroy(e);
  g_timer.ev.clear();
  g_timer.reps.clear();
  g_timer.used = 0;
  g_timer.site = -1;
  return TT_OK;
}

int tt_partial_contractions_rl_workspace(int32_t N, const int64_t *dims, const int64_t *ranks_x,
                                         const int64_t *ranks_y, int32_t prec, size_t *bytes) {
  TTR_TRY(check_shape(N, dims, ranks_x, "X"));
  TTR_TRY(check_shape(N, dims, ranks_y, "Y"));
  if (N < 2) return fail(TT_EINVAL, "partial contractions need N >= 2");
  read_env();
  Prec pc;
  TTR_TRY(prec_cfg(prec, pc));
  pc.sk = pc.store;
  return measure_workspace(
      [&](Ctx &c) -> int {
        std::vector<void *> W(N, nullptr), X(N, nullptr);
        std::vector<const void *> Yc(N, nullptr);
        if (pc.store == DType::F64)
          return wchain<double>(c, pc, false, N, dims, 1, &ranks_x, (const double *const *)X.data(),
                                ranks_y, Yc.data(), (double *const *)W.data());
        return wchain<float>(c, pc, false, N, dims, 1, &ranks_x, (const float *const *)X.data(),
                             ranks_y, Yc.data(), (float *const *)W.data());
      },
      bytes);
}

int tt_partial_contractions_rl(int32_t N, const int64_t *dims, const int64_t *ranks_x,
                               const void *const *x_cores, const int64_t *ranks_y,
                               const void *const *y_cores, int32_t prec, void *const *W_out,
                               void *workspace, size_t ws_bytes, void *stream) {
  TTR_TRY(check_shape(N, dims, ranks_x, "X"));
  TTR_TRY(check_shape(N, dims, ranks_y, "Y"));
  if (N < 2) return fail(TT_EINVAL, "partial contractions need N >= 2");
  read_env();
  Prec pc;
  TTR_TRY(prec_cfg(prec, pc));
  pc.sk = pc.store;
  TTR_TRY(check_ptrs(N, x_cores, "X cores"));
  TTR_TRY(check_ptrs(N, y_cores, "Y cores"));
  TTR_TRY(check_ptrs(N - 1, W_out, "W"));
  std::vector<void *> W(N, nullptr);
  for (int n = 1; n <= N - 1; ++n) W[n] = W_out[n - 1];
  return run_with_workspace(workspace, ws_bytes, (hipStream_t)stream, [&](Ctx &c) -> int {
    if (pc.store == DType::F64)
      return wchain<double>(c, pc, false, N, dims, 1, &ranks_x, (const double *const *)x_cores,
                            ranks_y, y_cores, (double *const *)W.data());
    return wchain<float>(c, pc, false, N, dims, 1, &ranks_x, (const float *const *)x_cores,
                         ranks_y, y_cores, (float *const *)W.data());
  });
}

}  // extern "C"

extern "C" {

int tt_round_two_sided_plan(int32_t N, const int64_t *dims, const int64_t *ranks,
                            int64_t target_rank, int64_t *left_ranks, int64_t *right_ranks) {
  std::vector<int64_t> ell, rho;
  TTR_TRY(two_sided_check(N, dims, ranks, target_rank, ell, rho));
  if (!left_ranks || !right_ranks) return fail(TT_EINVAL, "null output arrays");
  for (int n = 0; n <= N; ++n) {
    left_ranks[n] = ell[n];
    right_ranks[n] = rho[n];
  }
  return TT_OK;
}

int tt_round_two_sided_workspace(int32_t N, const int64_t *dims, const int64_t *ranks,
                                 int64_t target_rank, size_t *bytes) {
  std::vector<int64_t> ell, rho;
  TTR_TRY(two_sided_check(N, dims, ranks, target_rank, ell, rho));
  if (!bytes) return fail(TT_EINVAL, "null bytes pointer");
  if (N == 1) {
    *bytes = 0;
    return TT_OK;
  }
  std::vector<const double *> Y(N, nullptr);
  std::vector<double *> out(N, nullptr);
  return measure_workspace(
      [&](Ctx &c) -> int {
        return two_sided_body(c, N, dims, ranks, ell, rho, Y.data(), 0, 0, out.data());
      },
      bytes);
}

int tt_round_two_sided(int32_t N, const int64_t *dims, const int64_t *ranks,
                       const void *const *cores, int32_t dtype, int64_t target_rank,
                       uint64_t seed_left, uint64_t seed_right, void *const *out_cores,
                       void *workspace, size_t ws_bytes, void *stream) {
  std::vector<int64_t> ell, rho;
  TTR_TRY(two_sided_check(N, dims, ranks, target_rank, ell, rho));
  if (dtype != TT_F64) return fail(TT_EUNSUPPORTED, "two-sided rounding takes FP64 cores");
  TTR_TRY(check_ptrs(N, cores, "input cores"));
  TTR_TRY(check_ptrs(N, out_cores, "output cores"));
  hipStream_t st = (hipStream_t)stream;
  if (N == 1)
    return copy2d<double>((double *)out_cores[0], dims[0], (const double *)cores[0], dims[0], 1,
                          dims[0], 1.0, 0.0, st);
  return run_with_workspace(workspace, ws_bytes, st, [&](Ctx &c) -> int {
    return two_sided_body(c, N, dims, ranks, ell, rho, (const double *const *)cores, seed_left,
                          seed_right, (double *const *)out_cores);
  });
}

}  // extern "C"

extern "C" {

int tt_round_orth_rand_plan(int32_t N, const int64_t *dims, const int64_t *ranks,
                            int64_t target_rank, int64_t oversample, int64_t *sketch_ranks,
                            int64_t *out_ranks) {
  OrthPlan O;
  TTR_TRY(make_orth_plan(O, N, dims, ranks));
  return tt_round_rand_plan(N, dims, O.rr.data(), target_rank, oversample, sketch_ranks,
                            out_ranks);
}

static int orth_common(int32_t N, const int64_t *dims, const int64_t *ranks,
                       const void *const *cores, int32_t dtype, int64_t target_rank,
                       int64_t oversample, uint64_t seed, int32_t prec, void *const *out_cores,
                       void *workspace, size_t ws_bytes, void *stream, size_t *bytes) {
  read_env();
  OrthPlan O;
  TTR_TRY(make_orth_plan(O, N, dims, ranks));
  Problem P2;
  TTR_TRY(make_problem(P2, 1, N, dims, O.rr.data(), target_rank, oversample, nullptr));
  Prec pc;
  TTR_TRY(prec_cfg(prec, pc));
  if (prec == TT_PREC_MIXED_BF16)
    return fail(TT_EUNSUPPORTED, "tt_round_orth_rand: TT_PREC_F64 or TT_PREC_F32");
  // the workspace query runs the same sequence without buffers
  std::vector<const void *> no_in(N, nullptr);
  std::vector<void *> no_out(N, nullptr);
  const void *const *in = cores ? cores : no_in.data();
  void *const *outp = out_cores ? out_cores : no_out.data();
  auto body = [&](Ctx &c) -> int {
    if (pc.store == DType::F64)
      return orth_rand_exec<double>(c, O, P2, pc, (const double *const *)in, seed,
                                    (double *const *)outp);
    return orth_rand_exec<float>(c, O, P2, pc, (const float *const *)in, seed,
                                 (float *const *)outp);
  };
  if (bytes) {
    if (N == 1) {
      *bytes = 0;
      return TT_OK;
    }
    return measure_workspace(body, bytes);
  }
  TTR_TRY(check_dtype(dtype, pc));
  TTR_TRY(check_ptrs(N, cores, "input cores"));
  TTR_TRY(check_ptrs(N, out_cores, "output cores"));
  hipStream_t st = (hipStream_t)stream;
  if (N == 1) {
    const int64_t cnt = dims[0];
    if (pc.store == DType::F64)
      return copy2d<double>((double *)out_cores[0], 1, (const double *)cores[0], 1, cnt, 1, 1.0,
                            0.0, st);
    return copy2d<float>((float *)out_cores[0], 1, (const float *)cores[0], 1, cnt, 1, 1.0, 0.0,
                         st);
  }
  return run_with_workspace(workspace, ws_bytes, st, body);
}

int tt_round_orth_rand_workspace(int32_t N, const int64_t *dims, const int64_t *ranks,
                                 int64_t target_rank, int64_t oversample, int32_t prec,
                                 size_t *bytes) {
  if (!bytes) return fail(TT_EINVAL, "null bytes pointer");
  return orth_common(N, dims, ranks, nullptr, prec == TT_PREC_F64 ? TT_F64 : TT_F32,
                     target_rank, oversample, 0, prec, nullptr, nullptr, 0, nullptr, bytes);
}

int tt_round_orth_rand(int32_t N, const int64_t *dims, const int64_t *ranks,
                       const void *const *cores, int32_t dtype, int64_t target_rank,
                       int64_t oversample, uint64_t seed, int32_t prec, void *const *out_cores,
                       void *workspace, size_t ws_bytes, void *stream) {
  return orth_common(N, dims, ranks, cores, dtype, target_rank, oversample, seed, prec,
                     out_cores, workspace, ws_bytes, stream, nullptr);
}

}  // extern "C"

extern "C" {

static int gmres_common(int32_t N, const int64_t *dims, int32_t T, const void *const *op_mats,
                        const void *precond, const int64_t *f_ranks, const void *const *f_cores,
                        int32_t dtype, int64_t max_rank, double round_eps, double tol,
                        int32_t max_iter, uint64_t seed, void *const *x_cores, int64_t *x_ranks,
                        double *residuals, int32_t *iterations, void *workspace,
                        size_t ws_bytes, void *stream, size_t *bytes) {
  read_env();
  TTR_TRY(check_shape(N, dims, f_ranks, "tt_gmres: f"));
  if (N < 2) return fail(TT_EUNSUPPORTED, "tt_gmres: order N >= 2");
  if (T < 1) return fail(TT_EINVAL, "tt_gmres: at least one operator term");
  if (max_iter < 1 || max_iter + 1 > kFirstDotsMax)
    return fail(TT_EUNSUPPORTED, "tt_gmres: max_iter in 1 .. 63");
  if (!(round_eps > 0.0 && round_eps < 1.0)) return fail(TT_EINVAL, "tt_gmres: round_eps in (0, 1)");
  if (!(tol > 0.0)) return fail(TT_EINVAL, "tt_gmres: tol > 0");
  if (max_rank < 1 || max_rank > TT_MAX_SKETCH_RANK)
    return fail(TT_EUNSUPPORTED, "tt_gmres: max_rank in 1 .. TT_MAX_SKETCH_RANK");
  for (int n = 1; n < N; ++n)
    if (f_ranks[n] > max_rank) return fail(TT_EINVAL, "tt_gmres: f ranks above max_rank");
  if (dtype != TT_F64) return fail(TT_EUNSUPPORTED, "tt_gmres: TT_F64 storage only");
  GmresSpec S;
  S.N = N;
  S.T = T;
  S.dims.assign(dims, dims + N);
  std::vector<const void *> no_mats;
  if (!op_mats && bytes) {
    no_mats.assign((size_t)T * N, nullptr);
    S.mats = no_mats.data();
  } else {
    if (!op_mats) return fail(TT_EINVAL, "tt_gmres: null operator matrix array");
    S.mats = op_mats;
  }
  S.precond = precond;
  S.fr.assign(f_ranks, f_ranks + N + 1);
  std::vector<const void *> no_f(N, nullptr);
  S.f = f_cores ? f_cores : no_f.data();
  S.lmax = max_rank;
  S.round_eps = round_eps;
  S.tol = tol;
  S.max_iter = max_iter;
  S.seed = seed;
  std::vector<void *> no_x(N, nullptr);
  void *const *xo = x_cores ? x_cores : no_x.data();
  auto body = [&](Ctx &c) -> int {
    return gmres_exec<double>(c, S, (double *const *)xo, c.dry ? nullptr : x_ranks,
                              c.dry ? nullptr : residuals, c.dry ? nullptr : iterations);
  };
  if (bytes) {
    // the sizes do not depend on the operator matrices being set
    if (!op_mats) {
      // treat every matrix as present for the sizing
      static const char dummy = 0;
      no_mats.assign((size_t)T * N, &dummy);
      S.mats = no_mats.data();
      if (!precond) S.precond = &dummy;
    }
    return measure_workspace(body, bytes);
  }
  TTR_TRY(check_ptrs(N, f_cores, "tt_gmres: f cores"));
  TTR_TRY(check_ptrs(N, x_cores, "tt_gmres: x cores"));
  if (!x_ranks || !residuals || !iterations) return fail(TT_EINVAL, "tt_gmres: null output");
  return run_with_workspace(workspace, ws_bytes, (hipStream_t)stream, body);
}

int tt_gmres_workspace(int32_t N, const int64_t *dims, int32_t T, const int64_t *f_ranks,
                       int64_t max_rank, int32_t max_iter, size_t *bytes) {
  if (!bytes) return fail(TT_EINVAL, "null bytes pointer");
  return gmres_common(N, dims, T, nullptr, nullptr, f_ranks, nullptr, TT_F64, max_rank, 0.5, 1.0,
                      max_iter, 0, nullptr, nullptr, nullptr, nullptr, nullptr, 0, nullptr,
                      bytes);
}

int tt_gmres(int32_t N, const int64_t *dims, int32_t T, const void *const *op_mats,
             const void *precond, const int64_t *f_ranks, const void *const *f_cores,
             int32_t dtype, int64_t max_rank, double round_eps, double tol, int32_t max_iter,
             uint64_t seed, void *const *x_cores, int64_t *x_ranks, double *residuals,
             int32_t *iterations, void *workspace, size_t ws_bytes, void *stream) {
  return gmres_common(N, dims, T, op_mats, precond, f_ranks, f_cores, dtype, max_rank, round_eps,
                      tol, max_iter, seed, x_cores, x_ranks, residuals, iterations, workspace,
                      ws_bytes, stream, nullptr);
}

}  // extern "C"
