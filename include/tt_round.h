/*
 * tt_round.h -- C ABI of the MI355X (gfx950) randomized TT-rounding library.
 *
 * Method: Al Daas, Ballard, Cazeaux, Hallman, Miedlar, Pasha, Reid, Saibaba,
 * "Randomized algorithms for rounding in the Tensor-Train format".
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 * TT layout.  A TT of order N is given by N core pointers; core n (0-based)
 *   is a C-contiguous array of shape (ranks[n], dims[n], ranks[n+1]) with
 *   ranks[0] = ranks[N] = 1 (the TT format of section 2.1).  With this layout
 *   the horizontal unfolding H (r_{n-1} x I_n r_n) and the vertical unfolding
 *   V (r_{n-1} I_n x r_n) are plain row-major views.
 * Memory.  `dims`, `ranks`, the core-pointer arrays and every `*_host`
 *   argument are HOST memory.  Core pointers and `workspace` point to DEVICE
 *   memory owned by the caller; the library never allocates device memory
 *   and never frees caller memory.  Input cores are never modified.
 * Streams.  `stream` is a hipStream_t (NULL = legacy default stream).  Device
 *   work is enqueued asynchronously; the call returns before it completes
 *   unless stated otherwise.  Calls that share a workspace must be ordered
 *   on one stream.
 * Workspace.  Each device entry point takes a workspace whose minimum size
 *   is returned by the matching *_workspace query (host only, no GPU).
 * Errors.  Every function returns a tt_status.  Argument errors are detected
 *   on the host before any launch; then nothing is enqueued and outputs are
 *   untouched.  tt_last_error() returns a thread-local message describing the
 *   last non-OK status of the calling thread.
 * Precision.  `dtype` is the storage type of the cores (TT_F64 or TT_F32);
 *   `prec` the arithmetic mode (TT_PREC_F64 needs TT_F64 storage,
 *   TT_PREC_F32 and TT_PREC_MIXED_BF16 need TT_F32 storage; a mismatch is
 *   TT_EINVAL).  In the FP32 modes the Gram matrices of the thin QR and of
 *   the truncation are accumulated in FP64 from the FP32 operands and
 *   factorised in FP64 (the first CholeskyQR product Y R^-1 is also formed
 *   in FP64 and rounded to FP32), and every partial contraction W_n is rescaled by a
 *   power of two as soon as it is formed (the QR of Y_n = Z_n W_n, hence the
 *   result, is invariant under positive scalings of W_n; the rescaling keeps
 *   long trains inside the FP32 exponent range).  TT_PREC_MIXED_BF16 draws
 *   the sketch in BF16 (see tt_make_sketch) and runs the partial
 *   contractions on the BF16 MFMA with FP32 accumulation; the sweep and the
 *   truncation stay in FP32.
 */
#ifndef TT_ROUND_H
#define TT_ROUND_H

#include <stddef.h>
#include <stdint.h>

#if defined(__GNUC__) || defined(__clang__)
#define TT_API __attribute__((visibility("default")))
#else
#define TT_API
#endif

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  TT_OK = 0,
  TT_EINVAL = -1,       /* invalid argument (shape, rank, size, pointer)        */
  TT_ENOMEM = -2,       /* workspace smaller than the query returned             */
  TT_EHIP = -3,         /* a HIP runtime call failed                             */
  TT_ENUMERIC = -4,     /* non-finite result detected                            */
  TT_EUNSUPPORTED = -5  /* valid request outside the implemented limits          */
} tt_status;

typedef enum {
  TT_F64 = 0,
  TT_F32 = 1,
  TT_BF16 = 2  /* bfloat16; only as the output of tt_make_sketch */
} tt_dtype;

typedef enum {
  TT_PREC_F64 = 0,        /* all arithmetic in FP64 (MFMA f64)                    */
  TT_PREC_F32 = 1,        /* FP32 arithmetic except the Gram/Cholesky steps and
                             the first CholeskyQR product, in FP64             */
  TT_PREC_MIXED_BF16 = 2  /* W chain in BF16 MFMA with FP32 accumulation, sweep
                             in FP32, Gram/Cholesky and tails in FP64            */
} tt_prec;

/* Limits of the library. */
#define TT_MAX_ORDER 512          /* N                                          */
#define TT_MAX_SKETCH_RANK 96     /* l_n after clamping                         */

/* Thread-local description of the last non-OK status (never NULL). */
TT_API const char *tt_last_error(void);

/* ABI version (major*10000 + minor*100 + patch). */
TT_API int tt_version(void);

/*
 * Rank plan of randomized rounding (host only, no GPU).
 * Section 3 (target ranks include oversampling) and Algorithm 5.  With
 * l = target_rank + oversample:  u_N = 1, u_n = min(l, I_{n+1} u_{n+1});
 * l_0 = 1, l_n = min(l, l_{n-1} I_n, u_n, R_n), l_N = 1 (the thin QR of the
 * (l_{n-1} I_n) x l_n sketch needs l_n <= l_{n-1} I_n, the right factor has
 * rank <= I_{n+1}..I_N, and sketch columns beyond R_n add nothing).
 * Output ranks r_n = min(target_rank, l_n).
 *   N            order, 1 <= N <= TT_MAX_ORDER
 *   dims[N]      mode sizes I_n >= 1
 *   ranks[N+1]   input ranks, ranks[0] = ranks[N] = 1
 *   sketch_ranks[N+1], out_ranks[N+1]   written on success
 * Returns TT_EINVAL on bad shapes, target_rank < 1 or oversample < 0.
 */
TT_API int tt_round_rand_plan(int32_t N, const int64_t *dims, const int64_t *ranks,
                       int64_t target_rank, int64_t oversample,
                       int64_t *sketch_ranks, int64_t *out_ranks);

/* Workspace bytes needed by tt_round_rand / tt_round_rand_with_sketch for
 * these shapes and precision mode (host only). */
TT_API int tt_round_rand_workspace(int32_t N, const int64_t *dims, const int64_t *ranks,
                            int64_t target_rank, int64_t oversample, int32_t prec,
                            size_t *bytes);

/*
 * Random Gaussian TT of Definition 3.1, drawn on the device.
 * Core n (0-based) has shape (sketch_ranks[n], dims[n], sketch_ranks[n+1])
 * and iid N(0, 1/(l_{n-1} I_n l_n)) entries.  Generator: element k (C order)
 * of core n takes pair p = k/2 of the SplitMix64 stream keyed
 * key_n = mix(seed + (n+1) gamma); the pair uses stream outputs
 * a = mix(key_n + (2p+1) gamma), b = mix(key_n + (2p+2) gamma),
 * u1 = ((a >> 11) + 1) 2^-53, u2 = (b >> 11) 2^-53 and the Box-Muller values
 * sqrt(-2 ln u1) cos(2 pi u2) (even k) and sqrt(-2 ln u1) sin(2 pi u2) (odd k),
 * divided by sqrt(l_{n-1} I_n l_n).  mix is the SplitMix64 output function,
 * gamma = 0x9E3779B97F4A7C15.
 *   cores[N]   device pointers of the caller's output cores (dtype storage;
 *              TT_F32 rounds the FP64 value to nearest even, TT_BF16 rounds
 *              that FP32 value to nearest even, which is the sketch the
 *              TT_PREC_MIXED_BF16 mode draws)
 */
TT_API int tt_make_sketch(uint64_t seed, int32_t N, const int64_t *dims,
                   const int64_t *sketch_ranks, int32_t dtype, void *const *cores,
                   void *stream);

/*
 * Right-to-left partial contractions, Algorithm 3 / eq. (RLContraction):
 * W_n = H(X_{n+1:N}) H(Y_{n+1:N})^T for n = 1..N-1, computed as
 * W_{N-1} = H(X_N) H(Y_N)^T and, for n = N-1..2, V(Z_n) = V(X_n) W_n,
 * W_{n-1} = H(Z_n) H(Y_n)^T.
 *   X: N cores with ranks_x[N+1];  Y: N cores with ranks_y[N+1]; same dims.
 *   prec        TT_PREC_F64: X, Y, W in FP64, FP64 MFMA.  TT_PREC_F32: FP32
 *               storage and MFMA.  TT_PREC_MIXED_BF16: FP32 storage, every
 *               operand rounded to BF16 (nearest even) as it enters the BF16
 *               MFMA, FP32 accumulation.  No renormalisation: W_n is returned
 *               as defined.
 *   W_out[N-1]  device pointers; W_out[n-1] receives W_n as a row-major
 *               ranks_x[n] x ranks_y[n] matrix (n = 1..N-1).
 * Needs N >= 2.
 */
TT_API int tt_partial_contractions_rl_workspace(int32_t N, const int64_t *dims,
                                                const int64_t *ranks_x,
                                                const int64_t *ranks_y, int32_t prec,
                                                size_t *bytes);
TT_API int tt_partial_contractions_rl(int32_t N, const int64_t *dims,
                                      const int64_t *ranks_x, const void *const *x_cores,
                                      const int64_t *ranks_y, const void *const *y_cores,
                                      int32_t prec, void *const *W_out, void *workspace,
                                      size_t ws_bytes, void *stream);

/*
 * Randomized TT-rounding, Randomize-then-Orthogonalize (Algorithm 5).
 * Draws the sketch of Definition 3.1 from `sketch_seed` (generator as in
 * tt_make_sketch) with the ranks of tt_round_rand_plan, computes the partial
 * contractions W_n of the input with it (Algorithm 3), then sweeps left to
 * right: Z_n = V(X_n), Y_n = Z_n W_n, thin QR Y_n = Q R with diag(R) >= 0,
 * V(X_n) <- Q, M_n = Q^T Z_n, H(X_{n+1}) = M_n H(Y_{n+1}).  When some
 * out rank r_n < l_n the left-orthogonal result is truncated by a right-to-
 * left sweep (section 3.2 remark; mirror of the truncation loop of
 * Algorithm 2): for
 * n = N..2 the Gram H(X_n) H(X_n)^T is diagonalised, the r_{n-1} leading
 * eigenpairs (U, s^2) are kept, H(X_n) <- s^-1 U^T H(X_n) and
 * X_{n-1} <- X_{n-1} x_3 (U s).  Then cores 2..N are right-orthogonal;
 * otherwise cores 1..N-1 are left-orthogonal.
 *   N, dims, ranks, cores   input TT (dtype storage), read only
 *   target_rank, oversample see tt_round_rand_plan
 *   out_cores[N]            caller's device buffers of shape
 *                           (out_ranks[n], dims[n], out_ranks[n+1])
 *   workspace, ws_bytes     >= tt_round_rand_workspace(...)
 * N = 1 copies the single core.
 *
 * Synchronisation.  Unless the stream is being captured, the call returns
 * after the stream has finished the rounding: it runs a speculative form
 * that leaves out the guarded rescue launches (the third CholeskyQR pass
 * after a shifted first pass, the Householder fallback, the second pass of
 * the truncation for kept directions far below the largest).  It reads the
 * per-core breakdown flags back once, after the sweep and the truncation's
 * first bond (a breakdown also stops the speculative sweep's remaining
 * launches on the device): a set flag redoes the sweep in the guarded form
 * (all launches enqueued, each rescue returning at once unless its flag is
 * set) and runs the whole truncation guarded; a first bond that needs the
 * second pass runs the whole truncation guarded; otherwise the truncation
 * continues speculatively, its per-bond controls are read back at the end,
 * and a set one redoes the truncation guarded.  Both forms give the same
 * bits where no flag is set.
 * Under stream capture, or with TT_SPECULATE=0 in the environment, only the
 * guarded form is enqueued and the call returns without waiting.  The same
 * holds for tt_round_rand_with_sketch and tt_sum_round.
 */
TT_API int tt_round_rand(int32_t N, const int64_t *dims, const int64_t *ranks,
                  const void *const *cores, int32_t dtype, int64_t target_rank,
                  int64_t oversample, uint64_t sketch_seed, int32_t prec,
                  void *const *out_cores, void *workspace, size_t ws_bytes,
                  void *stream);

/*
 * For callers that cannot allocate device memory (code under stream capture,
 * tight serving loops, harnesses that forbid allocation): tt_round_rand with
 * its workspace in a fixed device array of TT_NOALLOC_SCRATCH_BYTES owned by
 * the library (one per GPU, held from the library's load on that GPU to the
 * end of the process).  No device memory is allocated or freed by the call.
 * Arguments, results and errors as tt_round_rand; TT_EUNSUPPORTED when
 * tt_round_rand_workspace exceeds TT_NOALLOC_SCRATCH_BYTES.  Every call on a
 * GPU uses that GPU's one array: calls that may overlap on one GPU (other
 * host threads, unordered streams) race and must be serialised by the
 * caller.  The array's device address is looked up on the first call on each
 * device (the current device).  The call always takes the guarded form of
 * tt_round_rand: it neither reads back nor waits for the stream.
 */
#define TT_NOALLOC_SCRATCH_BYTES (256u << 20) /* 256 MiB per GPU */
TT_API int tt_round_rand_noalloc(int32_t N, const int64_t *dims, const int64_t *ranks,
                                 const void *const *cores, int32_t dtype, int64_t target_rank,
                                 int64_t oversample, uint64_t sketch_seed, int32_t prec,
                                 void *const *out_cores, void *stream);

/* As tt_round_rand with a caller-given sketch TT (device cores of shape
 * (sketch_ranks[n], dims[n], sketch_ranks[n+1]) in `dtype` storage).
 * sketch_ranks must equal the plan's sketch ranks. */
TT_API int tt_round_rand_with_sketch(int32_t N, const int64_t *dims, const int64_t *ranks,
                              const void *const *cores, int32_t dtype,
                              int64_t target_rank, int64_t oversample,
                              const int64_t *sketch_ranks,
                              const void *const *sketch_cores, int32_t prec,
                              void *const *out_cores, void *workspace,
                              size_t ws_bytes, void *stream);

/*
 * Rounding of a sum of s TTs, Randomize-then-Orthogonalize (Algorithm 7).
 * X = sum_j coeffs[j] Y^(j) (coeffs NULL = all 1; coeffs[j] scales the first
 * core of summand j).  One sketch (ranks from tt_round_rand_plan applied to
 * the formal ranks sum_j R^(j)_n) for all summands; W^(j)_n per summand; the
 * sweep sketches with the stacked [W^(1)_n; ...; W^(s)_n] and forms the next
 * core summand by summand, X_{n+1}(:, i, block j) = M^(j)_n Y^(j)_{n+1}(:, i, :),
 * and X_N = sum_j M^(j)_{N-1} Y^(j)_N.  Then the same truncation as
 * tt_round_rand.
 *   s                 number of summands >= 1
 *   ranks[s*(N+1)]    ranks of summand j at ranks[j*(N+1) .. j*(N+1)+N]
 *   cores[s*N]        device pointers, summand j at cores[j*N .. j*N+N-1]
 *   coeffs[s]         host, or NULL
 *   out_cores[N]      shapes from tt_round_rand_plan on the formal ranks
 */
TT_API int tt_sum_round_workspace(int32_t s, int32_t N, const int64_t *dims,
                           const int64_t *ranks, int64_t target_rank,
                           int64_t oversample, int32_t prec, size_t *bytes);
TT_API int tt_sum_round(int32_t s, int32_t N, const int64_t *dims, const int64_t *ranks,
                 const void *const *cores, const double *coeffs, int32_t dtype,
                 int64_t target_rank, int64_t oversample, uint64_t sketch_seed,
                 int32_t prec, void *const *out_cores, void *workspace,
                 size_t ws_bytes, void *stream);

/*
 * Rounding to a tolerance when the ranks are not known in advance (section
 * 3.2, remark after Algorithm 5): Randomize-then-Orthogonalize (Algorithm 5,
 * or Algorithm 7 for a sum) with the sketch ranks of tt_round_rand_plan
 * (target_rank = max_rank, oversample = 0), then the truncation loop of
 * Algorithm 2 with its threshold, run right to left on the left-orthogonal
 * result X: eps = eps0 ||X|| / sqrt(N-1) (||X|| = ||X_N||_F); at bond n the
 * smallest k >= 1 with sqrt(sum_{j>k} s_j^2) <= eps is kept, s_j the
 * singular values of H(X_{n+1}) (from its FP64 Gram, as tt_round_rand's
 * truncation).  Then ||X_out - X|| <= eps0 ||X||; how close X is to the
 * input depends on the sketch ranks being large enough (the paper gives no
 * a-priori bound).  eps0 = 0 keeps the sketch ranks (no truncation).
 *   max_rank       the sketch rank l (the largest output rank)
 *   eps0           in [0, 1)
 *   out_cores[N]   caller buffers of at least the sketch-rank shapes
 *                  (tt_round_rand_plan with max_rank, 0); core n is written
 *                  C-contiguous with the chosen ranks
 *   out_ranks[N+1] host, written with the chosen ranks
 * The rank of every bond is read back by the host: the call waits for
 * `stream` once per bond (eps0 > 0).  Sums: as tt_sum_round.
 */
TT_API int tt_round_rand_eps_workspace(int32_t N, const int64_t *dims, const int64_t *ranks,
                                       int64_t max_rank, int32_t prec, size_t *bytes);
TT_API int tt_round_rand_eps(int32_t N, const int64_t *dims, const int64_t *ranks,
                             const void *const *cores, int32_t dtype, int64_t max_rank,
                             double eps0, uint64_t sketch_seed, int32_t prec,
                             void *const *out_cores, int64_t *out_ranks, void *workspace,
                             size_t ws_bytes, void *stream);
TT_API int tt_sum_round_eps_workspace(int32_t s, int32_t N, const int64_t *dims,
                                      const int64_t *ranks, int64_t max_rank, int32_t prec,
                                      size_t *bytes);
TT_API int tt_sum_round_eps(int32_t s, int32_t N, const int64_t *dims, const int64_t *ranks,
                            const void *const *cores, const double *coeffs, int32_t dtype,
                            int64_t max_rank, double eps0, uint64_t sketch_seed, int32_t prec,
                            void *const *out_cores, int64_t *out_ranks, void *workspace,
                            size_t ws_bytes, void *stream);

/*
 * Reverse mode (vector-Jacobian product) of tt_round_rand for roundings
 * without truncation (every out rank equals its sketch rank), single TT,
 * sketch fixed by `sketch_seed` (not differentiated).  Algorithm 5 is
 * recomputed forward (the partial contractions W_n are recomputed, never
 * kept between calls), then run in reverse: the next-core product, the
 * projection M_n = Q^T Z_n, the thin QR (adjoint with R unused:
 * dY = (dQ + Q copyltu(-dQ^T Q)) R^{-T}, copyltu(A) = tril(A) +
 * tril(A, -1)^T), the sketch product Y_n = Z_n W_n, and finally the partial
 * contractions of Algorithm 3.
 *   cores       input TT (as for tt_round_rand)
 *   grad_out[N] device cotangents of the output cores (out-rank shapes)
 *   grad_in[N]  device buffers of the input core shapes, overwritten with
 *               the gradient
 *   prec        TT_PREC_F64 (TT_F64) or TT_PREC_F32 (TT_F32)
 * R_n is formed as Q_n^T Y_n from the Q_n of the forward sweep.  The call
 * waits for `stream` at its end and returns TT_ENUMERIC when some R_n is
 * numerically singular (a rank-deficient sketch Y_n, where the adjoint of the
 * thin QR is undefined); grad_in is then unspecified.
 * Returns TT_EUNSUPPORTED when the rounding truncates (target_rank below a
 * sketch rank) or for TT_PREC_MIXED_BF16.
 */
TT_API int tt_round_rand_backward_workspace(int32_t N, const int64_t *dims, const int64_t *ranks,
                                            int64_t target_rank, int64_t oversample,
                                            int32_t prec, size_t *bytes);
TT_API int tt_round_rand_backward(int32_t N, const int64_t *dims, const int64_t *ranks,
                                  const void *const *cores, int32_t dtype, int64_t target_rank,
                                  int64_t oversample, uint64_t sketch_seed, int32_t prec,
                                  const void *const *grad_out, void *const *grad_in,
                                  void *workspace, size_t ws_bytes, void *stream);

/*
 * Orthogonalize-then-Randomize (Algorithm 4, section 3.1).  Algorithm 1
 * right-orthogonalises the input (thin QR of H(X_n)^T for n = N..2; when
 * that panel is wide, I_n r_n < r_{n-1}, the bond drops to I_n r_n and Q is
 * the QR factor of its leading square block), then for n = 1..N-1 with
 * Z_n = V(X_n): Y_n = Z_n Omega_n, thin QR Y_n = Q R (diag(R) >= 0),
 * V(X_n) <- Q, M_n = Q^T Z_n, H(X_{n+1}) = M_n H(X_{n+1}); then the same
 * truncation as tt_round_rand when an out rank is below its sketch rank.
 * Omega_n is R_n x l_n (R_n the rank after Algorithm 1) with iid
 * N(0, 1/(R_n l_n)) entries, read row-major from the tt_make_sketch
 * generator for one core of R_n l_n entries (ranks 1, 1) with seed + n.
 *   tt_round_orth_rand_plan   host only: the sketch and out ranks
 *                             (tt_round_rand_plan on the ranks after
 *                             Algorithm 1)
 *   prec                      TT_PREC_F64 (TT_F64) or TT_PREC_F32 (TT_F32)
 *   out_cores[N]              caller buffers at the plan's out ranks
 * Limits: every input bond rank <= TT_MAX_SKETCH_RANK (TT_EUNSUPPORTED).
 * Asynchronous on `stream`.
 */
TT_API int tt_round_orth_rand_plan(int32_t N, const int64_t *dims, const int64_t *ranks,
                                   int64_t target_rank, int64_t oversample,
                                   int64_t *sketch_ranks, int64_t *out_ranks);
TT_API int tt_round_orth_rand_workspace(int32_t N, const int64_t *dims, const int64_t *ranks,
                                        int64_t target_rank, int64_t oversample, int32_t prec,
                                        size_t *bytes);
TT_API int tt_round_orth_rand(int32_t N, const int64_t *dims, const int64_t *ranks,
                              const void *const *cores, int32_t dtype, int64_t target_rank,
                              int64_t oversample, uint64_t seed, int32_t prec,
                              void *const *out_cores, void *workspace, size_t ws_bytes,
                              void *stream);

/*
 * TT-GMRES (section 4.2): right-preconditioned GMRES for
 * (sum_{t=1}^{T} A_{t,1} x ... x A_{t,N}) x = f on TTs, every sum of TTs
 * rounded by Algorithm 7 to the relative tolerance round_eps (as
 * tt_sum_round_eps, sketch rank max_rank).  With x_0 = 0, beta = ||f||,
 * V_1 = f / beta, step k: Y = (P x I x ... x I) V_k; W = round(sum_t
 * (A_{t,1} x ... x A_{t,N}) Y) (sketch seed + 2k - 1); h_jk = <V_j, W> for
 * j <= k (Algorithm 3 with the second TT of rank r, section 3.5);
 * Z = round(W - sum_j h_jk V_j) (seed + 2k); h_{k+1,k} = ||Z||,
 * V_{k+1} = Z / h_{k+1,k}; Givens rotations of the Hessenberg column (k+1
 * scalars, on the host); stop when |g_{k+1}| / beta <= tol or after max_iter
 * steps; x = (P x I ..) round(sum_j y_j V_j) (seed + 2m + 1).  The call reads
 * scalars back after every step (it waits for `stream`).
 *   op_mats[T*N]   device I_n x I_n row-major matrices A_{t,n} (entry
 *                  t*N + n), NULL = identity
 *   precond        device I_1 x I_1 matrix P applied to the first mode, or
 *                  NULL (no preconditioner)
 *   f_ranks[N+1], f_cores[N]   the right-hand side (ranks <= max_rank)
 *   dtype          TT_F64
 *   max_rank       sketch rank of every rounding (<= TT_MAX_SKETCH_RANK)
 *   x_cores[N]     caller buffers of the max_rank shapes (core n at least
 *                  max_rank^2 I_n elements); written C-contiguous with the
 *                  ranks returned in x_ranks[N+1] (host)
 *   residuals      host, max_iter + 1 entries: the estimate |g_{k+1}|/beta
 *                  after step k (residuals[0] = 1)
 *   iterations     host: the number of steps taken
 * Limits: N >= 2, 1 <= max_iter <= 63.
 */
TT_API int tt_gmres_workspace(int32_t N, const int64_t *dims, int32_t T, const int64_t *f_ranks,
                              int64_t max_rank, int32_t max_iter, size_t *bytes);
TT_API int tt_gmres(int32_t N, const int64_t *dims, int32_t T, const void *const *op_mats,
                    const void *precond, const int64_t *f_ranks, const void *const *f_cores,
                    int32_t dtype, int64_t max_rank, double round_eps, double tol,
                    int32_t max_iter, uint64_t seed, void *const *x_cores, int64_t *x_ranks,
                    double *residuals, int32_t *iterations, void *workspace, size_t ws_bytes,
                    void *stream);

/*
 * Deterministic TT-rounding (Algorithms 1 and 2), the comparator of the
 * randomized methods.  Algorithm 1 right-orthogonalises the input by thin
 * QR factorisations from core N down to core 2; Algorithm 2 then sweeps left
 * to right, replacing each core by the leading left singular vectors of its
 * QR factor and carrying s_k V_k^T into the next core.  The singular pairs
 * come from the FP64 Gram of the core's vertical unfolding (same left
 * subspace and singular values as the R factor).
 * Rank rule (section 2, Algorithm 2; absolute threshold): with eps0 > 0 keep
 * at bond n the smallest k >= 1 with sqrt(sum_{j>=k} s_j^2) <=
 * eps0 ||Y|| / sqrt(N-1), capped by max_rank (max_rank <= 0: no cap); with
 * eps0 = 0 keep k = min(max_rank, bound).  Then ||X - Y|| <= eps0 ||Y||.
 * With eps0 > 0 every bond's rank is read back by the host: the call waits
 * for `stream` once per core.  With eps0 = 0 it is asynchronous.
 *   tt_round_svd_plan   host only: out_ranks[N+1] receives upper bounds of
 *                       the output ranks (the shapes to allocate)
 *   prec                TT_PREC_F64 (TT_F64 storage) or TT_PREC_F32 (TT_F32
 *                       storage; Grams and eigenproblems in FP64)
 *   out_cores[N]        caller buffers of at least the plan's sizes; core n
 *                       is written C-contiguous with the actual ranks
 *   out_ranks[N+1]      host, written with the actual ranks
 * Limits: every bond rank after Algorithm 1 <= TT_MAX_SKETCH_RANK
 * (TT_EUNSUPPORTED otherwise).
 */
TT_API int tt_round_svd_plan(int32_t N, const int64_t *dims, const int64_t *ranks,
                             int64_t max_rank, int64_t *out_ranks);
TT_API int tt_round_svd_workspace(int32_t N, const int64_t *dims, const int64_t *ranks,
                                  int64_t max_rank, int32_t prec, size_t *bytes);
TT_API int tt_round_svd(int32_t N, const int64_t *dims, const int64_t *ranks,
                        const void *const *cores, int32_t dtype, double eps0, int64_t max_rank,
                        int32_t prec, void *const *out_cores, int64_t *out_ranks,
                        void *workspace, size_t ws_bytes, void *stream);

/*
 * Two-Sided-Randomization (Algorithm 6, section 3.3; generalized Nystrom,
 * section 2.2, equation (LnRn)) of the FP64 TT Y to ranks l_n.  A left
 * Gaussian TT L (ranks l_n, seed_left) and a right one R (ranks rho_n,
 * seed_right) are drawn as tt_make_sketch draws them; W^L_n =
 * V(L_{1:n})^T V(Y_{1:n}) (l_n x R_n) and W^R_n = H(Y_{n+1:N}) H(R_{n+1:N})^T
 * (R_n x rho_n) are the partial contractions from the left and from the
 * right; at every bond, with W^L_n W^R_n = U S V^T, L_n = W^R_n V (S^+)^1/2 and
 * R_n = (S^+)^1/2 U^T W^L_n, where S^+ inverts the singular values above 1e-6
 * times the largest and zeroes the rest; then every core on its own:
 * X_1 = V(Y_1) L_1, H(X_n) = R_{n-1} H(V(Y_n) L_n), H(X_N) = R_{N-1} H(Y_N).
 * The output is not orthogonal.  The left singular vectors come from
 * cyclic-Jacobi eigenpairs of FP64 Grams in two passes (C C^T with C =
 * W^L W^R, then B B^T with B = U1^T C), which keeps the small singular
 * values close to their own relative accuracy.
 *   ranks: l_n as tt_round_rand_plan with oversample 0 (the output ranks);
 *          rho_n = ceil(3 l_n / 2) capped by I_{n+1} ... I_N
 *   tt_round_two_sided_plan  host only: left_ranks[N+1] = l_n,
 *                            right_ranks[N+1] = rho_n
 *   dtype        TT_F64 only (TT_EUNSUPPORTED otherwise)
 *   cores[N]     device input cores, not modified
 *   out_cores[N] device, core n l_{n-1} x I_n x l_n C-contiguous; must not
 *                overlap the inputs or the workspace
 *   workspace    device, 256-byte aligned, >= tt_round_two_sided_workspace
 * Limits: l_n and rho_n <= TT_MAX_SKETCH_RANK (so target_rank <= 64 when
 * the mode sizes do not cap rho_n), else TT_EUNSUPPORTED.  Asynchronous on
 * `stream`.
 */
TT_API int tt_round_two_sided_plan(int32_t N, const int64_t *dims, const int64_t *ranks,
                                   int64_t target_rank, int64_t *left_ranks,
                                   int64_t *right_ranks);
TT_API int tt_round_two_sided_workspace(int32_t N, const int64_t *dims, const int64_t *ranks,
                                        int64_t target_rank, size_t *bytes);
TT_API int tt_round_two_sided(int32_t N, const int64_t *dims, const int64_t *ranks,
                              const void *const *cores, int32_t dtype, int64_t target_rank,
                              uint64_t seed_left, uint64_t seed_right, void *const *out_cores,
                              void *workspace, size_t ws_bytes, void *stream);

/*
 * Batched randomized rounding: B independent TTs (any orders >= 2, mode
 * sizes and ranks; sketch ranks <= 76) rounded by Algorithm 5 with the same
 * truncation as tt_round_rand, in lock step: every step of the method is
 * one grouped launch over all TTs still active at that step.  Shapes and
 * pointers are fixed at creation; tt_batch_run then replays the sequence
 * (one hipGraph launch with TT_BATCH_GRAPH).  With TT_BATCH_AUTOTUNE the
 * tile shape of every grouped GEMM is chosen at creation by timing each
 * variant on the batch (this never changes results).  The thin QR is always
 * CholeskyQR2 with the device-flagged Householder fallback.
 *   orders[B]                 N_i
 *   dims[sum N_i]             mode sizes, TT after TT
 *   ranks[sum (N_i + 1)]      ranks, TT after TT
 *   target_ranks[B], oversample[B], seeds[B]   per TT, as in tt_round_rand
 *   cores[sum N_i]            device input cores, TT after TT (read at every run)
 *   out_cores[sum N_i]        device output cores at tt_round_rand_plan's
 *                             out ranks, TT after TT (written at every run)
 *   workspace, ws_bytes       >= tt_batch_workspace(...); the first part
 *                             holds the launch tables (uploaded at creation
 *                             with a synchronous copy) and must not be
 *                             modified while the batch exists
 *   flags                     TT_BATCH_GRAPH | TT_BATCH_AUTOTUNE
 *   stream                    creation runs (autotuning, warm-up) go there
 * tt_batch_create waits for the device (uploads, tuning, capture); run is
 * asynchronous.  The handle owns host memory and, with TT_BATCH_GRAPH, a
 * graph and a capture stream; tt_batch_destroy frees them.
 */
typedef struct tt_batch_s *tt_batch;
#define TT_BATCH_GRAPH 1
#define TT_BATCH_AUTOTUNE 2
TT_API int tt_batch_workspace(int32_t B, const int32_t *orders, const int64_t *dims,
                              const int64_t *ranks, const int64_t *target_ranks,
                              const int64_t *oversample, int32_t prec, size_t *bytes);
TT_API int tt_batch_create(int32_t B, const int32_t *orders, const int64_t *dims,
                           const int64_t *ranks, const int64_t *target_ranks,
                           const int64_t *oversample, const uint64_t *seeds, int32_t dtype,
                           int32_t prec, const void *const *cores, void *const *out_cores,
                           void *workspace, size_t ws_bytes, int32_t flags, void *stream,
                           tt_batch *batch);
TT_API int tt_batch_run(tt_batch batch, void *stream);
/* launches per run, grouped GEMMs, and how many of them use each of the four
 * tile variants: outputs per workgroup 32x64, 64x32, 64x64, 128x128 (the
 * same table for every arithmetic) */
TT_API int tt_batch_info(tt_batch batch, int32_t *launches, int32_t *gemm_groups,
                         int32_t *variant_count);
TT_API int tt_batch_destroy(tt_batch batch);

/*
 * Kernel timing (instrumentation, off by default).  tt_timing_start arms a
 * recorder for one call site of the rounding path: every later product from
 * that site is bracketed by a pair of HIP events recorded on the launch
 * stream (up to `capacity` products); a product that overwrites its output
 * (beta = 0) is launched 8 times back to back inside the pair, with the
 * same operands, and counts as the average of the 8.  tt_timing_stop waits
 * for the events, writes the summed time of one execution of every timed
 * product in milliseconds and the product count, and disarms the recorder.
 * Sites: see tt_timing_site.  Not thread-safe: one recorder per process.
 */
typedef enum {
  TT_SITE_WCHAIN_Z = 0,    /* V(Z_n) = V(Y_n) W_n            (Algorithm 3)   */
  TT_SITE_WCHAIN_W = 1,    /* W_{n-1} = H(Z_n) H(R_n)^T      (Algorithm 3)   */
  TT_SITE_SWEEP_Y = 2,     /* Y_n = Z_n W_n                  (Algorithm 5)   */
  TT_SITE_SWEEP_M = 3,     /* M_n = Q^T Z_n                  (Algorithm 5)   */
  TT_SITE_SWEEP_NEXT = 4,  /* H(X_{n+1}) = M_n H(Y_{n+1})    (Algorithm 5)   */
  TT_SITE_TRUNC = 5,       /* truncation GEMMs                               */
  TT_SITE_WCHAIN_FUSED = 6 /* W_{n-1} = H(V(Y_n) W_n) H(R_n)^T in one kernel
                              (its split sum not included)  (Algorithm 3)  */
} tt_timing_site;
TT_API int tt_timing_start(int32_t site, int32_t capacity);
TT_API int tt_timing_stop(double *total_ms, int32_t *launches);

#ifdef __cplusplus
}
#endif

#endif /* TT_ROUND_H */
