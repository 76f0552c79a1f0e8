// Internal declarations shared by the HIP translation units of libttround.
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>
#include <string>
#include <vector>

#include "../../include/tt_round.h"

namespace ttr {

// ---------------------------------------------------------------- errors
void set_error(const std::string &msg);
int fail(int status, const std::string &msg);

struct Status {
  int code = TT_OK;
  std::string msg;
};

#define TTR_HIP(call)                                                        \
  do {                                                                       \
    hipError_t e_ = (call);                                                  \
    if (e_ != hipSuccess)                                                    \
      return ::ttr::fail(TT_EHIP, std::string(#call) + ": " +                \
                                     hipGetErrorString(e_));                 \
  } while (0)

#define TTR_TRY(expr)            \
  do {                           \
    int s_ = (expr);             \
    if (s_ != TT_OK) return s_;  \
  } while (0)

// ---------------------------------------------------------------- workspace
// Bump allocator over the caller's workspace.  With base == nullptr it only
// measures (used by the *_workspace queries), so the query and the run share
// one layout function.
struct Arena {
  char *base = nullptr;
  size_t off = 0;
  size_t cap = 0;
  template <typename T>
  T *take(size_t count) {
    off = (off + 255) & ~size_t(255);
    T *p = base ? reinterpret_cast<T *>(base + off) : nullptr;
    off += count * sizeof(T);
    return p;
  }
};

// ---------------------------------------------------------------- GEMM
enum class DType : int { F64 = 0, F32 = 1, BF16 = 2 };

template <typename T>
struct DTypeOf;
template <>
struct DTypeOf<double> {
  static constexpr DType value = DType::F64;
};
template <>
struct DTypeOf<float> {
  static constexpr DType value = DType::F32;
};
template <>
struct DTypeOf<__bf16> {
  static constexpr DType value = DType::BF16;
};

// C(m,n) = alpha * sum_k A(m,k) B(k,n) + beta * C(m,n), C row-major (ldc).
// A(m,k) = a_kc ? A[m*lda + k] : A[k*lda + m]
// B(k,n) = b_kc ? B[n*ldb + k] : B[k*ldb + n]
// ta/tb/tc: storage types; math: MFMA arithmetic (F64, F32 or BF16 with F32
// accumulation).  With splits > 1 the K range is cut into chunks whose
// partial products (accumulator type) go to `partial` (splits*M*N elements)
// and are summed in chunk order by a second kernel (deterministic).
struct GemmX {
  const void *A = nullptr;
  int64_t lda = 0;
  bool a_kc = true;
  DType ta = DType::F64;
  const void *B = nullptr;
  int64_t ldb = 0;
  bool b_kc = false;
  DType tb = DType::F64;
  void *C = nullptr;
  int64_t ldc = 0;
  DType tc = DType::F64;
  int64_t M = 0, N = 0, K = 0;
  double alpha = 1, beta = 0;
  DType math = DType::F64;
  int splits = 1;
  void *partial = nullptr;
  // batch of independent products: operand pointers advance by sA/sB/sC
  // elements per batch entry (split-K is not combined with batching)
  int64_t batch = 1;
  int64_t sA = 0, sB = 0, sC = 0;
  // device gate: with `gate` set the launch does nothing unless
  // (*gate != 0) == (gate_on != 0) (decided on the device, no host sync)
  const int *gate = nullptr;
  int gate_on = 1;
  // device operand selection: with `sel` set and *sel != 0 the product reads
  // A2 and B2 (same types, shapes and layouts) instead of A and B
  const int *sel = nullptr;
  const void *A2 = nullptr, *B2 = nullptr;
};
__device__ inline bool gemm_gated_off(const GemmX &g) {
  return g.gate && ((*g.gate != 0) != (g.gate_on != 0));
}

// One entry of a grouped GEMM launch (device table): the product, its tile
// grid for the launch's tile variant and its first workgroup.
struct GemmGroupEntry {
  GemmX g;
  int64_t tiles_m = 0, tiles_n = 0, kchunk = 0;
  int64_t wg_begin = 0;
};
int gemm_variant_count();
void gemm_variant_tile(DType math, int v, int64_t *bm, int64_t *bn);
// split count for a grouped product (entries carry g.splits and g.partial;
// the partials of entries with splits > 1 are summed by gemm_group_reduce)
int gemm_group_splits(const GemmX &g);
int gemm_group_fill(const GemmX &g, int v, int64_t wg_begin, GemmGroupEntry *e);
int gemm_group_reduce(const GemmX &rep, const GemmGroupEntry *d_tab, int count, int64_t max_mn,
                      hipStream_t s);
int64_t gemm_group_wgs(const GemmGroupEntry &e);
// launches count products (table in device memory) in one grid of total_wgs
// workgroups; rep gives the common types and layouts
int gemm_group_run(const GemmX &rep, int v, const GemmGroupEntry *d_tab, int count,
                   int64_t total_wgs, hipStream_t s);

int gemm_pick_splits(int64_t M, int64_t N, int64_t K, DType math);
// number of split-K partials gemmx_run writes for g (1 = none, C written)
int gemm_used_splits(const GemmX &g);
size_t gemm_acc_bytes(DType math);
int gemmx_run(const GemmX &g, hipStream_t s);
// C = alpha * (sum of the g.splits partials [split][M][N] in g.partial) +
// beta * C, summed in a fixed order (accumulator type of g.math)
int gemm_reduce_splits(const GemmX &g, hipStream_t s);

// One level of the W chain (Algorithm 3) for every summand in one kernel:
// C_j = H(V(Y_j) W_j) H(Sk)^T for Y_j (R0_j x I x R1_j), W_j (R1_j x L1,
// ld L1), Sk (L0 x I x L1), C_j (R0_j x L0, ld L0); F64 or F32 arithmetic on
// operands of that type, or BF16 products with FP32 accumulation on FP32
// cores and a BF16 or FP32 sketch.  wfuse_supported tells whether the
// shapes fit the kernel (every R1_j a multiple of 4, L1 and L0 at most 128,
// W_j^T within the LDS); wfuse_aligned whether every Y_j is 16-byte aligned,
// which it also needs.  wfuse_partial_elems is the split buffer it needs
// (elements of t).  wfuse_run launches the kernel (up to 24 summands per
// launch) writing C_j or its i-range splits; wfuse_sum then adds the splits.
struct WFuseItem {
  const void *Y = nullptr, *W = nullptr;
  void *C = nullptr;
  int64_t R0 = 0, R1 = 0;
};
struct WFuse {
  const void *Sk = nullptr;
  DType t = DType::F64;     // storage of Y_j, W_j and C_j
  DType math = DType::F64;  // arithmetic: t, or BF16 with FP32 storage
  DType sk = DType::F64;    // storage of Sk: t (BF16 arithmetic: BF16 or FP32)
  int64_t I = 0, L1 = 0, L0 = 0;
  std::vector<WFuseItem> items;
};
bool wfuse_supported(const WFuse &f);
bool wfuse_aligned(const WFuse &f);
int64_t wfuse_partial_elems(const WFuse &f);
int wfuse_run(const WFuse &f, void *partial, size_t partial_bytes, hipStream_t s);
int wfuse_sum(const WFuse &f, void *partial, hipStream_t s);

// same-type convenience form
template <typename T>
struct Gemm {
  const T *A = nullptr;
  int64_t lda = 0;
  bool a_kc = true;
  const T *B = nullptr;
  int64_t ldb = 0;
  bool b_kc = false;
  T *C = nullptr;
  int64_t ldc = 0;
  int64_t M = 0, N = 0, K = 0;
  T alpha = 1, beta = 0;
  int splits = 1;
  T *partial = nullptr;
  int64_t batch = 1;
  int64_t sA = 0, sB = 0, sC = 0;
  GemmX x() const {
    GemmX g;
    g.A = A;
    g.lda = lda;
    g.a_kc = a_kc;
    g.ta = DTypeOf<T>::value;
    g.B = B;
    g.ldb = ldb;
    g.b_kc = b_kc;
    g.tb = DTypeOf<T>::value;
    g.C = C;
    g.ldc = ldc;
    g.tc = DTypeOf<T>::value;
    g.M = M;
    g.N = N;
    g.K = K;
    g.alpha = alpha;
    g.beta = beta;
    g.math = DTypeOf<T>::value;
    g.splits = splits;
    g.partial = partial;
    g.batch = batch;
    g.sA = sA;
    g.sB = sB;
    g.sC = sC;
    return g;
  }
};
template <typename T>
int gemm_run(const Gemm<T> &g, hipStream_t s) {
  return gemmx_run(g.x(), s);
}

// Round a finite FP32 value to the nearest bfloat16, ties to even, in integer
// arithmetic on its bits (the compiler may not fuse it with an earlier
// FP64 -> FP32 rounding, which would change the result at double-rounding
// ties).
__device__ inline __bf16 bf16_rne(float f) {
  uint32_t u = __float_as_uint(f);
  u += 0x7FFFu + ((u >> 16) & 1u);
  return __builtin_bit_cast(__bf16, (uint16_t)(u >> 16));
}

// ---------------------------------------------------------------- problems
// Arithmetic of one rounding.  F64: everything in FP64.  F32: FP32 storage
// and MFMA, FP64 Gram matrices (thin QR and truncation) and Cholesky/eigen
// solves.  MIXED_BF16: as F32, but the partial contractions (Algorithm 3) run
// on the BF16 MFMA with FP32 accumulation against a BF16 sketch.  Non-FP64
// modes renormalise each W_n by a power of two (exact; keeps the chain inside
// the FP32 exponent range for long trains).
struct Prec {
  DType store = DType::F64;  // cores, W_n, sweep buffers, outputs
  DType wmath = DType::F64;  // partial-contraction MFMA arithmetic
  DType sk = DType::F64;     // sketch storage inside the rounding
  bool renorm = false;
};

// Problem description shared by single-TT and sum rounding.  A single TT is
// a sum with s = 1.
struct Problem {
  int N = 0, s = 1;
  std::vector<int64_t> dims;
  std::vector<std::vector<int64_t>> R;  // per summand, N+1 ranks
  std::vector<int64_t> Rsum;            // formal ranks
  std::vector<int64_t> ell, out;
  std::vector<double> coeffs;
  bool truncate = false;
  int64_t max_ell = 1;
  // tolerance-driven truncation (section 3.2, remark after Algorithm 5):
  // out holds the upper bounds l_n, the ranks chosen by the eps rule of
  // Algorithm 2 are written to ranks_out (host, N+1 entries)
  bool eps_mode = false;
  double eps0 = 0.0;
  int64_t *ranks_out = nullptr;
  // speculative form: the guarded rescue launches (third CholeskyQR pass,
  // Householder fallback, second truncation pass) are left out and every
  // core's QR flag and every bond's truncation control is kept for the
  // caller to read back; a set one means the rounding must be redone guarded
  bool spec = false;
};

// Set by callers that must not synchronise or read back (the no-allocation
// entry point): roundings on this thread take the guarded form only.
extern thread_local bool g_spec_off;

int check_shape(int32_t N, const int64_t *dims, const int64_t *ranks, const char *what);
int check_ptrs(int32_t N, const void *const *p, const char *what);
void plan_ranks(int N, const int64_t *dims, const int64_t *R, int64_t target, int64_t over,
                std::vector<int64_t> &ell, std::vector<int64_t> &out);
int prec_cfg(int32_t prec, Prec &p);
int check_dtype(int32_t dtype, const Prec &p);
size_t dtype_bytes(DType t);
void read_env();
int make_problem(Problem &P, int s, int N, const int64_t *dims, const int64_t *ranks,
                 int64_t target, int64_t over, const double *coeffs);

// ---------------------------------------------------------------- sketch
int sketch_generate(uint64_t seed, int N, const int64_t *dims, const int64_t *sranks,
                    int dtype, void *const *cores, hipStream_t s);

// ---------------------------------------------------------------- QR
// Thin QR of the m x n row-major matrix Y (n <= TT_MAX_SKETCH_RANK, m >= n),
// Q written row-major m x n to Q (may not alias Y), diag(R) >= 0.
// The Gram matrix and its Cholesky factor are always FP64; with FP32 storage
// R^-1 is also written rounded to FP32 (rinv_f) for the Q = Y R^-1 product.
struct QrScratch {
  double *gram = nullptr;      // n*n
  double *rinv = nullptr;      // max(n*n, 2n)
  float *rinv_f = nullptr;     // n*n (FP32 storage only)
  void *q1 = nullptr;          // m*n elements of the storage type
  int *flag = nullptr;         // 1 int
  void *partial = nullptr;     // split-K partials
  bool speculative = false;    // leave out the third pass and the Householder rescue
  int *go = nullptr;           // speculative: launches run while *go != 0; a pivot
                               // breakdown clears it (the caller redoes the sweep)
};
size_t qr_partial_elems(int64_t m, int64_t n);
// FP64 Gram of a tall panel: G = A^T A (n x n, ld ldg) for A(k, m) stored
// K x n row-major (a_kc false, leading dimension lda) or n x K row-major
// (a_kc true); n <= 128, K <= 16384 (gram_supported).  Needs
// gram_partial_elems doubles of split buffer when K > 64.  gram_set_mode(1)
// makes the callers use the split-K GEMM instead.
bool gram_supported(int64_t n, int64_t K);
size_t gram_partial_elems(int64_t n, int64_t K);
int gram_run(const void *A, DType ta, bool a_kc, int64_t lda, int64_t n, int64_t K, double *G,
             int64_t ldg, void *partial, size_t partial_bytes, hipStream_t s,
             const int *gate = nullptr);
void gram_set_mode(int mode);
bool gram_enabled(int64_t n, int64_t K);
// Q = Y R (Y, Q: K x n row-major in the storage type ts, FP64 or FP32; R:
// n x n upper triangular, FP64; FP64 arithmetic) and G = Q^T Q of Q as
// stored, from the same launch (n <= 96; the split buffer as for gram_run)
bool apply_gram_supported(int64_t n, int64_t K);
int apply_gram_run(const void *Y, DType ts, const double *R, void *Q, int64_t n, int64_t K,
                   double *G, int64_t ldg, void *partial, size_t partial_bytes, hipStream_t s,
                   const int *gate = nullptr);
template <typename T>
int qr_thin(const T *Y, T *Q, int64_t m, int64_t n, QrScratch &ws, hipStream_t s);
void qr_set_mode(int mode);  // 0 auto, 1 force householder, 2 force cholqr2
// truncation eigensolver: 0 tridiagonal (Jacobi when it fails), 1 Jacobi always
void eig_set_mode(int mode);
// R^{-1} of the upper Cholesky factor of the n x n FP64 matrix G (n <= 96),
// row-major; Rinv_f (optional) receives it rounded to FP32; *flag = 1 on a
// pivot breakdown
int chol_inverse(const double *G, int64_t n, double *Rinv, float *Rinv_f, int *flag,
                 hipStream_t s);

// Grouped forms of the one-workgroup kernels: one launch, one workgroup (or
// a fixed set of them) per entry of a device table.
struct CholGroupDesc {
  const double *G;
  double *Rinv;
  float *Rinv_f;
  int n;
  int *flag;
  int or_flag;
};
int chol_group_run(const CholGroupDesc *d_tab, int count, int nmax, hipStream_t s);

struct HhGroupDesc {
  const void *Y;
  void *Q;
  void *work;
  double *rdiag, *tau;
  int64_t m;
  int n;
  const int *flag;
  int always;
  int use_lds;
};
// fills the scratch assignment of one panel (m x n) exactly as qr_thin's
// Householder path does; returns the LDS bytes it needs
size_t hh_group_desc(const void *Y, void *Q, int64_t m, int64_t n, QrScratch &ws, int always,
                     size_t elem, HhGroupDesc *d);
template <typename T>
int householder_group_run(const HhGroupDesc *d_tab, int count, size_t lds_bytes, hipStream_t s);

// ---------------------------------------------------------------- eigen
// Symmetric eigendecomposition of an n x n matrix (n <= TT_MAX_SKETCH_RANK)
// by cyclic Jacobi: eigenvalues descending to `lam`, eigenvectors as the
// columns of U (row-major n x n); *info (optional) receives the sweep count.
// With a gate pointer the kernel returns at once unless *gate != 0.  With
// `relative` every off-diagonal entry is rotated until it is small relative
// to its two diagonal entries (no absolute floor at the rounding level of
// the largest one): for Grams of nearly orthogonal rows.
int sym_eig(const double *G, double *lam, double *U, int64_t n, hipStream_t s,
            int *info = nullptr, const int *gate = nullptr, bool relative = false);

// `count` independent sym_eig problems in one launch (one workgroup each):
// problem b reads G + b sG and writes lam + b sl and U + b sU, order n[b]
// (host array).
int sym_eig_batch(const double *G, int64_t sG, double *lam, int64_t sl, double *U, int64_t sU,
                  const int *n, int count, bool relative, hipStream_t s);

// Truncation factors from (lam, U): P = U_k sqrt(lam_k) (n x k, row-major),
// S = sqrt(lam_k)^-1 U_k^T (k x n, row-major), tail = sum_{j>=k} max(lam_j,0).
template <typename T>
int trunc_factors(const double *lam, const double *U, int64_t n, int64_t k, T *P, T *S,
                  double *tail, hipStream_t s, const int *gate = nullptr);

// Leading k eigenpairs of the symmetric n x n G and the truncation factors
// P, S and tail as above: tridiagonalisation + multisection + twisted
// factorisation for n <= 76 with a device-flagged Jacobi fallback, Jacobi for
// larger n.  lam (n) and U (n x n) are scratch/outputs; flag is one int;
// scratch holds eig_trunc_scratch(n, k) doubles.
//
// With ctl (4 device ints) the solve also decides whether the kept directions
// need the second pass of trunc_refine_*: ctl[0] = 1 when the smallest kept
// eigenvalue is below tau times the largest, ctl[1] = the number w of kept
// eigenvalues at or above that level (only their eigenvectors are then
// checked and returned accurately), ctl[3] = the leading dimension of U,
// and when ctl[0] = 1 it writes U1 (n x n): an orthonormal basis whose first
// ctl[1] columns are those eigenvectors and the rest their complement.
template <typename T>
int eig_trunc(const double *G, int64_t n, int64_t k, double *lam, double *U, T *P, T *S,
              double *tail, int *flag, double *scratch, hipStream_t s, int *ctl = nullptr,
              double tau = 0.0, double *U1 = nullptr);
size_t eig_trunc_scratch(int64_t n, int64_t k);

// Second pass of the truncation at one bond (kernels return at once unless
// ctl[0] = 1): after the caller has formed B = U1^T H and G2 = B B^T (FP64)
// from eig_trunc's U1, trunc_refine_solve writes F (k x n) and
// P (n x k) with F B orthonormal rows spanning the k leading right singular
// directions of H and P F B = H projected onto them; kept directions at the
// rounding level of B get zero rows of F and zero columns of P, nullmask[j]
// = 1 and ctl[2] = their count; trunc_refine_complete then writes
// orthonormal rows into those rows of the core C = F B (cols >= k;
// scratch: trunc_complete_scratch doubles).  scratch of the solve:
// trunc_refine_scratch doubles.  n <= TT_MAX_SKETCH_RANK.
template <typename T>
int trunc_refine_solve(const double *G2, const double *U1, int64_t n, int64_t k, int *ctl,
                       int *nullmask, double *scratch, T *F, T *P, hipStream_t s);
template <typename T>
int trunc_refine_complete(T *C, int64_t k, int64_t cols, const int *ctl, const int *nullmask,
                          double *scratch, hipStream_t s);
size_t trunc_complete_scratch(int64_t k, int64_t cols);
size_t trunc_refine_scratch(int64_t n, int64_t k);
// the same in two steps for the tolerance mode: trunc_refine_eps forms the
// weak-block eigenpairs (when ctl[0] = 1) and writes lamc (n): the spectrum
// to choose the rank from (first-pass eigenvalues above the split, the
// weak block's below it; lam itself when ctl[0] = 0); trunc_refine_final
// then forms F and P for the chosen k
template <typename T>
int trunc_refine_eps(const double *G2, const double *U1, int64_t n, int *ctl, int *nullmask,
                     double *scratch, const double *lam, double *lamc, hipStream_t s);
template <typename T>
int trunc_refine_final(const double *G2, const double *U1, int64_t n, int64_t k, int *ctl,
                       int *nullmask, double *scratch, T *F, T *P, hipStream_t s);
int trunc_refine_ctl(const double *lam, const double *U, int64_t n, int64_t k, double tau,
                     int *ctl, double *U1, hipStream_t s);
// after the kept rank k is chosen below the rank the solve was run for:
// ctl[0] = (k > ctl[1]) (the second pass is needed only if a kept
// eigenvalue is below the split)
int trunc_refine_setk(int *ctl, int64_t k, hipStream_t s);

struct EigGroupDesc {
  const double *G;
  int n, k, kw;
  double *d, *e, *sc, *Vr, *taus, *lamw, *Uz;
  double *lam, *U;
  void *P, *S;
  double *tail;
  int *flag;
};
// descriptor of one eig_trunc problem (same scratch layout); false when the
// problem is outside the grouped fast path (n > 76)
bool eig_group_desc(const double *G, int64_t n, int64_t k, double *lam, double *U, void *P,
                    void *S, double *tail, int *flag, double *scratch, EigGroupDesc *d);
template <typename T>
int eig_trunc_group(const EigGroupDesc *d_tab, int count, int nmax, int kwmax, hipStream_t s);

// ---------------------------------------------------------------- misc
// dst[r*ldd + c] = alpha * src[r*lds + c] + beta * dst[r*ldd + c]
template <typename T>
int copy2d(T *dst, int64_t ldd, const T *src, int64_t lds, int64_t rows, int64_t cols,
           double alpha, double beta, hipStream_t s);

// x <- x * 2^-floor(log2 max|x|) (exact; one workgroup, count small); the
// factor applied (1 if none) goes to *fout when fout is not null
template <typename T>
int scale_pow2(T *x, int64_t count, hipStream_t s, double *fout = nullptr);
struct ScaleGroupDesc {
  void *x;
  int64_t count;
  double *fout;
};
template <typename T>
int scale_pow2_group(const ScaleGroupDesc *d_tab, int count, hipStream_t s);
// x *= *f, f on the device
template <typename T>
int scale_dev(T *x, int64_t count, const double *f, hipStream_t s);
// C = alpha (tril(M) + tril(M, -1)^T), k x k row-major
template <typename T>
int copyltu(T *C, const T *M, int64_t k, double alpha, hipStream_t s);

// Generalized Nystrom scalings (Algorithm 6, equation (LnRn)) from the
// eigenpairs of G = C C^T (lam descending, U's columns the eigenvectors,
// n x n row-major): with s_j = sqrt(lam_j) and h_j = s_j^-1/2 where
// s_j > rcond s_1 (else 0), A1 = U diag(h_j / s_j) and A2 = diag(h) U^T.
int nystrom_scale(const double *lam, const double *U, int64_t n, double rcond, double *A1,
                  double *A2, hipStream_t s);

// X = R^{-1} of the upper-triangular n x n FP64 R (row-major); Xf (optional)
// the same rounded to FP32; *flag = (first ? 0 : *flag) | (R numerically
// singular: a diagonal entry at or below 64 u max |R_ii|, or a non-finite
// result)
int tri_inv_upper(const double *R, int64_t n, double *X, float *Xf, int *flag, bool first,
                  hipStream_t s);

// Inner products <X_j, Y> of TTs from their first cores (1 x I x r_j and
// 1 x I x ry) and the partial contractions W_1^(j) (r_j x ry, leading
// dimension ry): out[j] (device, FP64), up to kFirstDotsMax per launch.
constexpr int kFirstDotsMax = 64;
template <typename T>
struct FirstDots {
  const T *X[kFirstDotsMax];
  const T *W[kFirstDotsMax];
  int r[kFirstDotsMax];
  const T *Y = nullptr;
  int I = 0, ry = 0;
  double *out = nullptr;
};
template <typename T>
int first_dots(const FirstDots<T> &a, int count, hipStream_t s);

// dst = RNE_bf16(src)
int round_to_bf16(__bf16 *dst, const float *src, int64_t count, hipStream_t s);

// dst (cols x rows) = src (rows x cols)^T, row-major
template <typename T>
int transpose(T *dst, const T *src, int64_t rows, int64_t cols, hipStream_t s);
// dst = I (m x m)
template <typename T>
int fill_identity(T *dst, int64_t m, hipStream_t s);
// *out = ||x||_F (FP64, deterministic)
template <typename T>
int frob_norm(const T *x, int64_t count, double *out, hipStream_t s);
// eps-truncation rank from descending eigenvalues lam of a Gram matrix:
// smallest k >= 1 with sum_{j>=k} lam_j <= (eps0 norm)^2/(N-1), capped by kmax
// Next core of a sum, slice-wise for every summand in one launch (Algorithm
// 7): X(:, i, offn_j + c) = M(:, offm_j + k) Y_j(k, i, c) summed over k < r_j,
// for all summands j and mode indices i < I1.  M: L x ldm row-major (the
// summands' columns side by side), Y_j: r_j x I1 x r1_j, X: L x I1 x rs1.
// Storage T (FP64 or FP32), arithmetic in T.  sum_next_fits (elem =
// sizeof(T)) is false when the shapes do not fit (more than kSumNextMax
// summands, or the operands of one summand beyond the LDS budget); the caller
// then takes one GEMM per summand.
constexpr int kSumNextMax = 24;
struct SumNextEntry {
  const void *Y;
  int64_t offm, offn;
  int32_t rj, rj1;
};
bool sum_next_fits(size_t elem, int64_t L, int64_t I1, const SumNextEntry *e, int count);
template <typename T>
int sum_next_run(const T *M, int64_t ldm, T *X, int64_t L, int64_t I1, int64_t rs1,
                 const SumNextEntry *e, int count, const int *gate, hipStream_t s);
int select_rank(const double *lam, int n, const double *norm, double eps0, int N, int kmax,
                int *k_out, double *tail_out, hipStream_t s);

}  // namespace ttr
