// Batched randomized rounding: many independent TTs (any orders, mode sizes
// and ranks) rounded together, Algorithm 5 on every item in lock step.
//
// Every step of the method is one *grouped* launch over all items that are
// still active at that step: a grouped GEMM (workgroups dealt to the items'
// tiles through a prefix table), one workgroup per item for the Cholesky,
// Householder, renormalisation and eigen-solver kernels.  The one-workgroup
// factorisations, which bound a single rounding by their latency, then run
// side by side on as many compute units as there are items.
//
// Schedule (s = step index, items with fewer cores drop out early):
//   W chain   s = 0..      W_{N-1}, then Zc = V(Y_n) W_n, W_{n-1} = H(Zc) H(Sk_n)^T
//   sweep     n = 1..      Y_n = Z_n W_n, CholeskyQR2 (FP64 Gram and Cholesky,
//                          Householder fallback gated on the pivot flag),
//                          M_n = Q^T Z_n, next core M_n H(Y_{n+1})
//   truncate  n = N..2     FP64 Gram, eigenpairs, H(X_n) <- S H(X_n), X_{n-1} <- X_{n-1} P
// All shapes and pointers are fixed when the batch is created, so the
// descriptor tables are built once, uploaded into the caller's workspace,
// and the whole sequence can be captured into one hipGraph and replayed.
// The tile shape of each grouped GEMM is chosen by timing every variant on
// the batch itself (the variants differ only in how output tiles are dealt
// to wavefronts; every output element is summed in the same order, so the
// choice never changes the results).
#include <algorithm>
#include <cstring>
#include <memory>

#include "tt_internal.h"

namespace ttr {
namespace {

enum OpKind { OP_SKETCH, OP_GEMM, OP_CHOL, OP_HH, OP_EIG, OP_SCALE };

struct Op {
  OpKind kind = OP_GEMM;
  size_t tab_off = 0;  // byte offset of the table inside the table region
  int count = 0;
  // OP_GEMM
  std::vector<GemmX> gx;
  int variant = 3;
  int64_t total_wgs = 0;
  bool reduce = false;  // some entry is split over K
  int64_t max_mn = 0;
  // OP_CHOL / OP_EIG: largest n; OP_EIG: largest kw; OP_HH: LDS bytes
  int nmax = 0, kwmax = 0;
  size_t lds = 0;
  // host copies of the small descriptor tables
  std::vector<CholGroupDesc> chol;
  std::vector<HhGroupDesc> hh;
  std::vector<EigGroupDesc> eig;
  std::vector<ScaleGroupDesc> scale;
  // OP_SKETCH: item index
  int item = -1;
};

struct Item {
  Problem P;
  std::vector<const void *> Y;
  std::vector<void *> out;
  uint64_t seed = 0;
  // workspace
  std::vector<void *> Sk, W, xs, xb;
  void *ys = nullptr, *mbuf = nullptr, *q1 = nullptr;
  double *gram = nullptr, *rinv = nullptr, *fac = nullptr;
  float *rinv_f = nullptr;
  int *qflag = nullptr;
  void *zc = nullptr;
  double *tg = nullptr, *lam = nullptr, *U = nullptr, *tails = nullptr, *escr = nullptr;
  int *eflag = nullptr;
  void *Pf = nullptr, *Sf = nullptr, *tb[2] = {nullptr, nullptr};
  // split-K partials of this item's grouped products
  void *part = nullptr;
  size_t part_need = 0;
};

size_t elem_bytes(DType t) { return t == DType::F64 ? 8 : (t == DType::F32 ? 4 : 2); }

}  // namespace

struct Batch {
  Prec pc;
  std::vector<Item> items;
  std::vector<Op> ops;
  char *tables = nullptr;  // device table region (start of the workspace)
  size_t table_bytes = 0;
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
  int launches = 0;
};

namespace {

void *take_bytes(Arena &a, size_t bytes) { return a.take<char>(bytes); }

// Per-item workspace layout (mirrors the single-TT path).
void layout_item(Item &it, const Prec &p, Arena &a) {
  const Problem &P = it.P;
  const int N = P.N;
  const int64_t *dims = P.dims.data();
  const std::vector<int64_t> &L = P.ell, &R = P.R[0];
  const size_t es = elem_bytes(p.store), ks = elem_bytes(p.sk);
  it.Sk.assign(N, nullptr);
  for (int n = 0; n < N; ++n) it.Sk[n] = take_bytes(a, (size_t)(L[n] * dims[n] * L[n + 1]) * ks);
  it.W.assign(N, nullptr);
  for (int n = 1; n <= N - 1; ++n) it.W[n] = take_bytes(a, (size_t)(R[n] * L[n]) * es);
  it.fac = a.take<double>((size_t)N + 1);
  int64_t zmax = 1;
  for (int n = 2; n <= N - 1; ++n) zmax = std::max(zmax, R[n - 1] * dims[n - 1] * L[n]);
  it.zc = take_bytes(a, (size_t)zmax * es);
  int64_t ys_max = 1, x_max = 1, m_max = 1, lm = 1;
  for (int n = 1; n <= N - 1; ++n) {
    ys_max = std::max(ys_max, L[n - 1] * dims[n - 1] * L[n]);
    m_max = std::max(m_max, L[n] * R[n]);
    if (n + 1 <= N - 1) x_max = std::max(x_max, L[n] * dims[n] * R[n + 1]);
  }
  for (int n = 0; n <= N; ++n) lm = std::max(lm, L[n]);
  it.ys = take_bytes(a, (size_t)ys_max * es);
  it.mbuf = take_bytes(a, (size_t)m_max * es);
  it.xb.assign(2, nullptr);
  it.xb[0] = take_bytes(a, (size_t)x_max * es);
  it.xb[1] = take_bytes(a, (size_t)x_max * es);
  it.q1 = take_bytes(a, (size_t)ys_max * es);
  it.gram = a.take<double>((size_t)std::max(lm * lm, 2 * lm));
  it.rinv = a.take<double>((size_t)std::max(lm * lm, 2 * lm));
  if (p.store == DType::F32) it.rinv_f = a.take<float>((size_t)(lm * lm));
  it.qflag = a.take<int>(4);
  it.xs.assign(N + 1, nullptr);
  for (int n = 1; n <= N; ++n)
    it.xs[n] = take_bytes(a, (size_t)(L[n - 1] * dims[n - 1] * L[n]) * es);
  it.tg = a.take<double>((size_t)(lm * lm));
  it.lam = a.take<double>((size_t)lm);
  it.U = a.take<double>((size_t)(lm * lm));
  it.tails = a.take<double>((size_t)N + 1);
  it.eflag = a.take<int>(4);
  it.escr = a.take<double>(eig_trunc_scratch(lm, lm));
  it.Pf = take_bytes(a, (size_t)(lm * lm) * es);
  it.Sf = take_bytes(a, (size_t)(lm * lm) * es);
  int64_t tmax = 1;
  for (int n = 2; n <= N - 1; ++n) tmax = std::max(tmax, L[n - 1] * dims[n - 1] * P.out[n]);
  it.tb[0] = take_bytes(a, (size_t)tmax * es);
  it.tb[1] = take_bytes(a, (size_t)tmax * es);
}

GemmX mk(const Prec &p, DType math, const void *A, int64_t lda, bool akc, DType ta, const void *B,
         int64_t ldb, bool bkc, DType tb, void *C, int64_t ldc, DType tc, int64_t M, int64_t N,
         int64_t K, double beta = 0.0) {
  (void)p;
  GemmX g;
  g.A = A;
  g.lda = lda;
  g.a_kc = akc;
  g.ta = ta;
  g.B = B;
  g.ldb = ldb;
  g.b_kc = bkc;
  g.tb = tb;
  g.C = C;
  g.ldc = ldc;
  g.tc = tc;
  g.M = M;
  g.N = N;
  g.K = K;
  g.math = math;
  g.beta = beta;
  return g;
}

// Long contractions are split over K into the item's partial buffer.
GemmX split(Item &it, GemmX g) {
  const int sp = gemm_group_splits(g);
  if (sp > 1) {
    g.splits = sp;
    g.partial = it.part;
    it.part_need = std::max(it.part_need, (size_t)sp * g.M * g.N * gemm_acc_bytes(g.math));
  }
  return g;
}

template <typename... A>
GemmX mks(Item &it, A &&...args) {
  return split(it, mk(std::forward<A>(args)...));
}

// Builds the op list; table offsets are assigned by assign_tables().
int build_ops(Batch &b) {
  const Prec &p = b.pc;
  const DType st = p.store;
  std::vector<Op> &ops = b.ops;
  int maxN = 0;
  for (const Item &it : b.items) maxN = std::max(maxN, it.P.N);
  auto gemm_op = [&](std::vector<GemmX> &&g) {
    if (g.empty()) return;
    Op o;
    o.kind = OP_GEMM;
    o.gx = std::move(g);
    o.count = (int)o.gx.size();
    for (const GemmX &x : o.gx) {
      if (x.splits > 1) o.reduce = true;
      o.max_mn = std::max(o.max_mn, x.M * x.N);
    }
    ops.push_back(std::move(o));
  };
  // sketches
  for (int i = 0; i < (int)b.items.size(); ++i) {
    Op o;
    o.kind = OP_SKETCH;
    o.item = i;
    ops.push_back(o);
  }
  // ---- W chains
  for (int s = 0; s <= maxN - 2; ++s) {
    std::vector<GemmX> z, w;
    Op sc;
    sc.kind = OP_SCALE;
    for (Item &it : b.items) {
      const int N = it.P.N;
      const int64_t *dims = it.P.dims.data();
      const std::vector<int64_t> &L = it.P.ell, &R = it.P.R[0];
      if (s == 0) {
        w.push_back(mks(it, p, p.wmath, it.Y[N - 1], dims[N - 1], true, st, it.Sk[N - 1], dims[N - 1],
                       true, p.sk, it.W[N - 1], L[N - 1], st, R[N - 1], L[N - 1], dims[N - 1]));
        sc.scale.push_back({it.W[N - 1], R[N - 1] * L[N - 1], it.fac + N - 1});
      } else {
        const int n = N - s;
        if (n < 2) continue;
        const int64_t I = dims[n - 1];
        z.push_back(mks(it, p, p.wmath, it.Y[n - 1], R[n], true, st, it.W[n], L[n], false, st, it.zc,
                       L[n], st, R[n - 1] * I, L[n], R[n]));
        w.push_back(mks(it, p, p.wmath, it.zc, I * L[n], true, st, it.Sk[n - 1], I * L[n], true, p.sk,
                       it.W[n - 1], L[n - 1], st, R[n - 1], L[n - 1], I * L[n]));
        sc.scale.push_back({it.W[n - 1], R[n - 1] * L[n - 1], it.fac + n - 1});
      }
    }
    gemm_op(std::move(z));
    gemm_op(std::move(w));
    if (p.renorm && !sc.scale.empty()) {
      sc.count = (int)sc.scale.size();
      ops.push_back(std::move(sc));
    }
  }
  // ---- sweep
  for (int n = 1; n <= maxN - 1; ++n) {
    std::vector<GemmX> gy, g1, q1, g2, q2, gm, gn;
    Op c1, c2, hh;
    c1.kind = c2.kind = OP_CHOL;
    hh.kind = OP_HH;
    for (Item &it : b.items) {
      const int N = it.P.N;
      if (n > N - 1) continue;
      const int64_t *dims = it.P.dims.data();
      const std::vector<int64_t> &L = it.P.ell, &R = it.P.R[0];
      const int64_t m = L[n - 1] * dims[n - 1], ln = L[n];
      const void *cur = (n == 1) ? it.Y[0] : it.xb[(n - 1) & 1];
      void *dst = (n + 1 == N) ? it.xs[N] : it.xb[n & 1];
      gy.push_back(mks(it, p, st, cur, R[n], true, st, it.W[n], ln, false, st, it.ys, ln, st, m, ln,
                      R[n]));
      const void *rinv_t = (st == DType::F32) ? (const void *)it.rinv_f : (const void *)it.rinv;
      g1.push_back(mks(it, p, DType::F64, it.ys, ln, false, st, it.ys, ln, false, st, it.gram, ln,
                      DType::F64, ln, ln, m));
      c1.chol.push_back({it.gram, it.rinv, it.rinv_f, (int)ln, it.qflag, 0});
      q1.push_back(mks(it, p, st, it.ys, ln, true, st, rinv_t, ln, false, st, it.q1, ln, st, m, ln, ln));
      g2.push_back(mks(it, p, DType::F64, it.q1, ln, false, st, it.q1, ln, false, st, it.gram, ln,
                      DType::F64, ln, ln, m));
      c2.chol.push_back({it.gram, it.rinv, it.rinv_f, (int)ln, it.qflag, 1});
      q2.push_back(mks(it, p, st, it.q1, ln, true, st, rinv_t, ln, false, st, it.xs[n], ln, st, m, ln,
                      ln));
      QrScratch qs;
      qs.gram = it.gram;
      qs.rinv = it.rinv;
      qs.rinv_f = it.rinv_f;
      qs.q1 = it.q1;
      qs.flag = it.qflag;
      HhGroupDesc d;
      const size_t need = hh_group_desc(it.ys, it.xs[n], m, ln, qs, 0, elem_bytes(st), &d);
      hh.hh.push_back(d);
      hh.lds = std::max(hh.lds, need);
      c1.nmax = c2.nmax = std::max(c1.nmax, (int)ln);
      gm.push_back(mks(it, p, st, it.xs[n], ln, false, st, cur, R[n], false, st, it.mbuf, R[n], st, ln,
                      R[n], m));
      const int64_t cols = dims[n] * R[n + 1];
      gn.push_back(mks(it, p, st, it.mbuf, R[n], true, st, it.Y[n], cols, false, st, dst, cols, st, ln,
                      cols, R[n]));
    }
    if (gy.empty()) continue;
    gemm_op(std::move(gy));
    gemm_op(std::move(g1));
    c1.count = (int)c1.chol.size();
    ops.push_back(std::move(c1));
    gemm_op(std::move(q1));
    gemm_op(std::move(g2));
    c2.count = (int)c2.chol.size();
    ops.push_back(std::move(c2));
    gemm_op(std::move(q2));
    hh.count = (int)hh.hh.size();
    ops.push_back(std::move(hh));
    gemm_op(std::move(gm));
    gemm_op(std::move(gn));
  }
  // ---- truncation (right to left)
  for (int t = 0; t <= maxN - 2; ++t) {
    std::vector<GemmX> gg, gs, gp;
    Op eg;
    eg.kind = OP_EIG;
    for (Item &it : b.items) {
      const int N = it.P.N;
      const int n = N - t;
      if (n < 2) continue;
      const int64_t *dims = it.P.dims.data();
      const std::vector<int64_t> &L = it.P.ell;
      const int64_t rr = (n == N) ? 1 : it.P.out[n];
      const int64_t lr = L[n - 1], k = it.P.out[n - 1], cols = dims[n - 1] * rr;
      const void *hsrc = (n == N) ? it.xs[N] : it.tb[(n + 1) & 1];
      gg.push_back(mks(it, p, DType::F64, hsrc, cols, true, st, hsrc, cols, true, st, it.tg, lr,
                      DType::F64, lr, lr, cols));
      EigGroupDesc d;
      if (!eig_group_desc(it.tg, lr, k, it.lam, it.U, it.Pf, it.Sf, it.tails + n - 1, it.eflag,
                          it.escr, &d))
        return fail(TT_EUNSUPPORTED, "batched rounding: a sketch rank above 76");
      eg.eig.push_back(d);
      eg.nmax = std::max(eg.nmax, (int)lr);
      eg.kwmax = std::max(eg.kwmax, d.kw);
      gs.push_back(mks(it, p, st, it.Sf, lr, true, st, hsrc, cols, false, st, it.out[n - 1], cols, st, k,
                      cols, lr));
      const int64_t rows = L[n - 2] * dims[n - 2];
      void *dst = (n - 1 == 1) ? it.out[0] : it.tb[n & 1];
      gp.push_back(mks(it, p, st, it.xs[n - 1], lr, true, st, it.Pf, k, false, st, dst, k, st, rows, k,
                      lr));
    }
    if (gg.empty()) continue;
    gemm_op(std::move(gg));
    eg.count = (int)eg.eig.size();
    ops.push_back(std::move(eg));
    gemm_op(std::move(gs));
    gemm_op(std::move(gp));
  }
  return TT_OK;
}

size_t table_bytes_of(const Op &o) {
  switch (o.kind) {
    case OP_GEMM: return sizeof(GemmGroupEntry) * o.count;
    case OP_CHOL: return sizeof(CholGroupDesc) * o.count;
    case OP_HH: return sizeof(HhGroupDesc) * o.count;
    case OP_EIG: return sizeof(EigGroupDesc) * o.count;
    case OP_SCALE: return sizeof(ScaleGroupDesc) * o.count;
    default: return 0;
  }
}

size_t assign_tables(Batch &b) {
  size_t off = 0;
  for (Op &o : b.ops) {
    off = (off + 255) & ~size_t(255);
    o.tab_off = off;
    off += table_bytes_of(o);
  }
  return (off + 255) & ~size_t(255);
}

int fill_gemm_table(const Op &o, int v, std::vector<GemmGroupEntry> &tab, int64_t *total) {
  tab.resize(o.count);
  int64_t wg = 0;
  for (int i = 0; i < o.count; ++i) {
    TTR_TRY(gemm_group_fill(o.gx[i], v, wg, &tab[i]));
    wg += gemm_group_wgs(tab[i]);
  }
  *total = wg;
  return TT_OK;
}

int upload_tables(Batch &b) {
  std::vector<char> host(b.table_bytes, 0);
  for (Op &o : b.ops) {
    char *dst = host.data() + o.tab_off;
    switch (o.kind) {
      case OP_GEMM: {
        std::vector<GemmGroupEntry> tab;
        TTR_TRY(fill_gemm_table(o, o.variant, tab, &o.total_wgs));
        std::memcpy(dst, tab.data(), sizeof(GemmGroupEntry) * tab.size());
        break;
      }
      case OP_CHOL: std::memcpy(dst, o.chol.data(), sizeof(CholGroupDesc) * o.count); break;
      case OP_HH: std::memcpy(dst, o.hh.data(), sizeof(HhGroupDesc) * o.count); break;
      case OP_EIG: std::memcpy(dst, o.eig.data(), sizeof(EigGroupDesc) * o.count); break;
      case OP_SCALE: std::memcpy(dst, o.scale.data(), sizeof(ScaleGroupDesc) * o.count); break;
      default: break;
    }
  }
  TTR_HIP(hipMemcpy(b.tables, host.data(), b.table_bytes, hipMemcpyHostToDevice));
  return TT_OK;
}

int launch_op(Batch &b, const Op &o, hipStream_t s) {
  const void *tab = b.tables + o.tab_off;
  const bool f32 = b.pc.store == DType::F32;
  switch (o.kind) {
    case OP_SKETCH: {
      const Item &it = b.items[o.item];
      return sketch_generate(it.seed, it.P.N, it.P.dims.data(), it.P.ell.data(), (int)b.pc.sk,
                             (void *const *)it.Sk.data(), s);
    }
    case OP_GEMM:
      TTR_TRY(gemm_group_run(o.gx[0], o.variant, (const GemmGroupEntry *)tab, o.count,
                             o.total_wgs, s));
      if (o.reduce)
        TTR_TRY(gemm_group_reduce(o.gx[0], (const GemmGroupEntry *)tab, o.count, o.max_mn, s));
      return TT_OK;
    case OP_CHOL: return chol_group_run((const CholGroupDesc *)tab, o.count, o.nmax, s);
    case OP_HH:
      return f32 ? householder_group_run<float>((const HhGroupDesc *)tab, o.count, o.lds, s)
                 : householder_group_run<double>((const HhGroupDesc *)tab, o.count, o.lds, s);
    case OP_EIG:
      return f32 ? eig_trunc_group<float>((const EigGroupDesc *)tab, o.count, o.nmax, o.kwmax, s)
                 : eig_trunc_group<double>((const EigGroupDesc *)tab, o.count, o.nmax, o.kwmax, s);
    case OP_SCALE:
      return f32 ? scale_pow2_group<float>((const ScaleGroupDesc *)tab, o.count, s)
                 : scale_pow2_group<double>((const ScaleGroupDesc *)tab, o.count, s);
  }
  return TT_OK;
}

int run_ops(Batch &b, hipStream_t s) {
  for (const Op &o : b.ops) TTR_TRY(launch_op(b, o, s));
  return TT_OK;
}

// Times every tile variant of every grouped GEMM on the batch's own shapes
// (the operands hold whatever the workspace holds; only timing matters) and
// keeps the fastest.  The default variant is the one with least padding for
// the largest product.
int autotune(Batch &b, hipStream_t s) {
  hipEvent_t e0, e1;
  TTR_HIP(hipEventCreate(&e0));
  TTR_HIP(hipEventCreate(&e1));
  int rc = TT_OK;
  std::vector<GemmGroupEntry> tab;
  for (Op &o : b.ops) {
    if (o.kind != OP_GEMM) continue;
    float best = 1e30f;
    int best_v = o.variant;
    for (int v = 0; v < gemm_variant_count() && rc == TT_OK; ++v) {
      int64_t total = 0;
      rc = fill_gemm_table(o, v, tab, &total);
      if (rc != TT_OK) break;
      if (hipMemcpy(b.tables + o.tab_off, tab.data(), sizeof(GemmGroupEntry) * tab.size(),
                    hipMemcpyHostToDevice) != hipSuccess) {
        rc = fail(TT_EHIP, "autotune upload");
        break;
      }
      const GemmGroupEntry *d = (const GemmGroupEntry *)(b.tables + o.tab_off);
      rc = gemm_group_run(o.gx[0], v, d, o.count, total, s);  // warm-up
      if (rc != TT_OK) break;
      (void)hipEventRecord(e0, s);
      for (int r = 0; r < 3 && rc == TT_OK; ++r) rc = gemm_group_run(o.gx[0], v, d, o.count, total, s);
      (void)hipEventRecord(e1, s);
      (void)hipEventSynchronize(e1);
      float ms = 0.f;
      (void)hipEventElapsedTime(&ms, e0, e1);
      if (ms < best) {
        best = ms;
        best_v = v;
      }
    }
    o.variant = best_v;
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  return rc;
}

int default_variants(Batch &b) {
  for (Op &o : b.ops) {
    if (o.kind != OP_GEMM) continue;
    int64_t bestM = 0, bestN = 0;
    for (const GemmX &g : o.gx)
      if (g.M * g.N > bestM * bestN) {
        bestM = g.M;
        bestN = g.N;
      }
    // least padded work for the largest product; ties to the smaller tile
    int best = 0;
    double cost = 1e300;
    for (int v = 0; v < gemm_variant_count(); ++v) {
      int64_t bm, bn;
      gemm_variant_tile(o.gx[0].math, v, &bm, &bn);
      const double c = double((bestM + bm - 1) / bm * bm) * double((bestN + bn - 1) / bn * bn) *
                       (1.0 + 1e-3 * v);
      if (c < cost) {
        cost = c;
        best = v;
      }
    }
    o.variant = best;
  }
  return TT_OK;
}

struct BatchArgs {
  int B = 0;
  const int32_t *orders = nullptr;
  const int64_t *dims = nullptr, *ranks = nullptr, *target = nullptr, *over = nullptr;
};

int make_items(Batch &b, const BatchArgs &a, char *base, size_t *item_bytes,
               const std::vector<size_t> *needs) {
  if (a.B < 1) return fail(TT_EINVAL, "batch needs at least one TT");
  if (!a.orders || !a.dims || !a.ranks || !a.target || !a.over)
    return fail(TT_EINVAL, "null batch description array");
  b.items.resize(a.B);
  size_t doff = 0, roff = 0;
  Arena arena;
  arena.base = base;
  for (int i = 0; i < a.B; ++i) {
    const int N = a.orders[i];
    if (N < 2) return fail(TT_EINVAL, "batched TTs need order >= 2");
    Item &it = b.items[i];
    TTR_TRY(make_problem(it.P, 1, N, a.dims + doff, a.ranks + roff, a.target[i], a.over[i],
                         nullptr));
    for (int n = 0; n <= N; ++n)
      if (it.P.ell[n] > 76) return fail(TT_EUNSUPPORTED, "batched rounding: sketch rank above 76");
    layout_item(it, b.pc, arena);
    if (needs) it.part = take_bytes(arena, (*needs)[i]);
    it.Y.assign(N, nullptr);  // filled by tt_batch_create
    it.out.assign(N, nullptr);
    doff += N;
    roff += N + 1;
  }
  *item_bytes = arena.off;
  return TT_OK;
}

}  // namespace
}  // namespace ttr

using namespace ttr;

struct tt_batch_s {
  Batch b;
  hipStream_t cap = nullptr;
};

namespace {

// Two passes: the first sizes the launch tables and every item's split-K
// partial buffer, the second lays the items out behind the tables.
int batch_layout(Batch &b, const BatchArgs &a, char *base, size_t *total) {
  size_t item_bytes = 0;
  TTR_TRY(make_items(b, a, nullptr, &item_bytes, nullptr));
  b.ops.clear();
  TTR_TRY(build_ops(b));
  b.table_bytes = assign_tables(b);
  std::vector<size_t> needs;
  for (const Item &it : b.items) needs.push_back(it.part_need);
  b.ops.clear();
  TTR_TRY(make_items(b, a, base ? base + b.table_bytes : nullptr, &item_bytes, &needs));
  *total = b.table_bytes + item_bytes;
  return TT_OK;
}

}  // namespace

extern "C" {

int tt_batch_workspace(int32_t B, const int32_t *orders, const int64_t *dims,
                       const int64_t *ranks, const int64_t *target_ranks,
                       const int64_t *oversample, int32_t prec, size_t *bytes) {
  if (!bytes) return fail(TT_EINVAL, "null bytes pointer");
  Batch b;
  TTR_TRY(prec_cfg(prec, b.pc));
  BatchArgs a{B, orders, dims, ranks, target_ranks, oversample};
  return batch_layout(b, a, nullptr, bytes);
}

int tt_batch_create(int32_t B, const int32_t *orders, const int64_t *dims, const int64_t *ranks,
                    const int64_t *target_ranks, const int64_t *oversample,
                    const uint64_t *seeds, int32_t dtype, int32_t prec,
                    const void *const *cores, void *const *out_cores, void *workspace,
                    size_t ws_bytes, int32_t flags, void *stream, tt_batch *batch) {
  read_env();
  if (!batch) return fail(TT_EINVAL, "null batch handle pointer");
  *batch = nullptr;
  if (!seeds) return fail(TT_EINVAL, "null seeds");
  if (flags & ~(TT_BATCH_GRAPH | TT_BATCH_AUTOTUNE)) return fail(TT_EINVAL, "unknown flags");
  std::unique_ptr<tt_batch_s> h(new tt_batch_s());
  Batch &b = h->b;
  TTR_TRY(prec_cfg(prec, b.pc));
  TTR_TRY(check_dtype(dtype, b.pc));
  BatchArgs a{B, orders, dims, ranks, target_ranks, oversample};
  size_t need = 0;
  TTR_TRY(batch_layout(b, a, nullptr, &need));
  if (!workspace) return fail(TT_EINVAL, "null workspace");
  if (ws_bytes < need)
    return fail(TT_ENOMEM, "workspace too small: need " + std::to_string(need) + " bytes");
  if (reinterpret_cast<uintptr_t>(workspace) % 256 != 0)
    return fail(TT_EINVAL, "workspace must be 256-byte aligned");
  char *base = static_cast<char *>(workspace);
  TTR_TRY(batch_layout(b, a, base, &need));
  int total_cores = 0;
  for (int i = 0; i < B; ++i) total_cores += orders[i];
  TTR_TRY(check_ptrs(total_cores, cores, "input cores"));
  TTR_TRY(check_ptrs(total_cores, out_cores, "output cores"));
  int off = 0;
  for (int i = 0; i < B; ++i) {
    Item &it = b.items[i];
    it.Y.assign(cores + off, cores + off + orders[i]);
    it.out.assign(out_cores + off, out_cores + off + orders[i]);
    it.seed = seeds[i];
    off += orders[i];
  }
  b.ops.clear();
  TTR_TRY(build_ops(b));
  b.table_bytes = assign_tables(b);
  b.tables = base;
  TTR_TRY(default_variants(b));
  hipStream_t st = (hipStream_t)stream;
  if (flags & TT_BATCH_AUTOTUNE) TTR_TRY(autotune(b, st));
  TTR_TRY(upload_tables(b));
  b.launches = 0;
  for (const Op &o : b.ops) b.launches += (o.kind == OP_EIG) ? 3 : (o.reduce ? 2 : 1);
  if (flags & TT_BATCH_GRAPH) {
    // one eager pass (first-use kernel attributes are set outside capture)
    TTR_TRY(run_ops(b, st));
    TTR_HIP(hipStreamSynchronize(st));
    TTR_HIP(hipStreamCreateWithFlags(&h->cap, hipStreamNonBlocking));
    TTR_HIP(hipStreamBeginCapture(h->cap, hipStreamCaptureModeThreadLocal));
    const int rc = run_ops(b, h->cap);
    hipGraph_t g = nullptr;
    const hipError_t ec = hipStreamEndCapture(h->cap, &g);
    if (rc != TT_OK) {
      if (g) (void)hipGraphDestroy(g);
      return rc;
    }
    if (ec != hipSuccess) return fail(TT_EHIP, std::string("graph capture: ") + hipGetErrorString(ec));
    b.graph = g;
    TTR_HIP(hipGraphInstantiate(&b.exec, b.graph, nullptr, nullptr, 0));
  }
  *batch = h.release();
  return TT_OK;
}

int tt_batch_run(tt_batch batch, void *stream) {
  if (!batch) return fail(TT_EINVAL, "null batch");
  Batch &b = batch->b;
  hipStream_t st = (hipStream_t)stream;
  if (b.exec) {
    TTR_HIP(hipGraphLaunch(b.exec, st));
    return TT_OK;
  }
  return run_ops(b, st);
}

int tt_batch_info(tt_batch batch, int32_t *launches, int32_t *gemm_groups,
                  int32_t *variant_count) {
  if (!batch || !launches || !gemm_groups || !variant_count)
    return fail(TT_EINVAL, "null argument");
  Batch &b = batch->b;
  *launches = b.launches;
  int gg = 0;
  for (int v = 0; v < 4; ++v) variant_count[v] = 0;
  for (const Op &o : b.ops)
    if (o.kind == OP_GEMM) {
      ++gg;
      variant_count[o.variant]++;
    }
  *gemm_groups = gg;
  return TT_OK;
}

int tt_batch_destroy(tt_batch batch) {
  if (!batch) return TT_OK;
  Batch &b = batch->b;
  if (b.exec) (void)hipGraphExecDestroy(b.exec);
  if (b.graph) (void)hipGraphDestroy(b.graph);
  if (batch->cap) (void)hipStreamDestroy(batch->cap);
  delete batch;
  return TT_OK;
}

}  // extern "C"
