/*
 * cs.h - C ABI of libcsrecover: CG-based greedy compressive-sensing recovery
 * on AMD Instinct MI355X (gfx950).
 *
 * Problem (Sec. II and Eq. (2) of Hsieh, Lu, Pei, "Fast Greedy Approaches for
 * Compressive Sensing of Large-Scale Signals"): given measurements y = A s of
 * a K-sparse s, recover s.  The sensing matrix is the operator of Sec. III-A,
 * Eq. (7), A = D F R with
 *   D  keeping the M sampled rows `rows` of an N-vector,
 *   F  the orthonormal N-point DCT-II, (F x)_k = c_k sum_n x_n cos(pi(2n+1)k/(2N)),
 *      c_0 = sqrt(1/N), c_k = sqrt(2/N); or (cs_op.xform = 1, partial Fourier
 *      sensing of a real signal, Sec. II) the orthonormal real Fourier basis:
 *      row k < N/2 sqrt(2/N) Re X_k, row N-k -sqrt(2/N) Im X_k, rows 0 and N/2
 *      X_0 / sqrt(N) and X_{N/2} / sqrt(N), with X the N-point DFT, so that
 *      sampling rows k and N-k measures the complex coefficient X_k,
 *   R  the randomizer: a sign flip, optionally with a permutation.
 * The measured signal is x = Psi s (Eq. (2)) with Psi the identity (s is
 * sparse directly), the orthonormal DCT-II (the same F) as in the
 * experiments of Sec. IV-A, so that A = D F R F, or the separable 2-D DCT of
 * Sec. III-E on an n x n image; see cs_op.psi.
 *
 * Every least-squares step is the CG-based weighted least squares of
 * Sec. III-B/C (Eqs. (10)-(11), the CG function of Algorithm 1): CG on
 * W_S A^T A W_S theta = W_S A^T y, touching A only through the operator.
 *
 * Conventions for every entry point
 * ---------------------------------
 * Memory:  all array arguments are DEVICE pointers owned by the caller; the
 *          library never allocates or frees device memory and keeps no
 *          pointer after it returns.  Scratch space is the caller's workspace
 *          `ws` of `ws_bytes` bytes (256-byte aligned); query its size with
 *          cs_workspace_size().  Workspaces must not be shared by calls that
 *          run concurrently.
 * Types:   `dtype` selects the element type of y, s, x, u, out and the
 *          workspace vectors: CS_F32 (float) or CS_F64 (double).  Inner
 *          products and residual norms are accumulated in double in both.
 * Streams: all device work is enqueued on `stream` (0 = default stream).
 *          Every call synchronises that stream (descriptor validation and the
 *          loop control read small device flags) and returns with results
 *          complete.
 * Errors:  arguments are validated on the host before any device work; a
 *          negative status means nothing was written to the outputs.
 *          Operator descriptors (rows ascending and in range, signs +-1) are
 *          validated on the device; a bad descriptor returns CS_E_OP.
 *          Conditions met during the iteration set bits in cs_info.flags
 *          and still return CS_OK with best-effort outputs.
 *          CS_E_HIP reports a HIP runtime error (text: cs_last_error()).
 * Sizes:   N is a power of two with 16 <= N <= 2^26; 1 <= M <= N;
 *          1 <= K <= M.  SP additionally needs 2K <= M (its least-squares
 *          step uses 2K columns, which must have full column rank, Thm. 1).
 * Threads: the library is reentrant for distinct workspaces;
 *          cs_last_error() is thread-local.
 */
#ifndef CS_H
#define CS_H

#include <stddef.h>
#include <stdint.h>
#include <hip/hip_runtime_api.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum { CS_F32 = 0, CS_F64 = 1 } cs_dtype;

typedef enum {
  CS_ALGO_OMP = 0,      /* Orthogonal Matching Pursuit (Sec. II, Algorithm 1)           */
  CS_ALGO_SP = 1,       /* Subspace Pursuit (run in Sec. IV)                            */
  CS_ALGO_OMPR = 2,     /* OMP with Replacement, l = 1 (run in Sec. IV)                 */
  CS_ALGO_OPERATOR = 3, /* cs_apply_A / cs_apply_At only                                */
  CS_ALGO_LS = 4,       /* cs_ls_solve (the CG function of Algorithm 1 alone)           */
  CS_ALGO_COSAMP = 5    /* CoSaMP, the merge/prune neighbour of SP                      */
} cs_algo;

typedef enum {
  CS_OK = 0,
  CS_E_INVALID = -1,    /* null pointer, bad dtype/algo, K < 1, tol <= 0 or not finite  */
  CS_E_SHAPE = -2,      /* N not a power of two in [16, 2^26], M > N, K > M, SP 2K > M   */
  CS_E_OP = -3,         /* rows not strictly ascending in [0, N), a sign not +-1, perm
                           not a permutation, or psi not 0, 1 or 2                     */
  CS_E_WORKSPACE = -4,  /* workspace too small or not 256-byte aligned                   */
  CS_E_HIP = -5         /* HIP runtime error                                             */
} cs_status;

/* cs_info.flags bits (non-fatal) */
enum {
  CS_F_CG_MAXITER = 1,     /* a CG solve hit its iteration cap before the tolerance   */
  CS_F_CG_BREAKDOWN = 2,   /* d^T H d <= 0 or not finite (rank-deficient A_S, Thm. 3) */
  CS_F_OUTER_MAXITER = 4,  /* SP/OMPR stopped at max_outer                            */
  CS_F_NONFINITE = 8,      /* a non-finite value reached a selection or a norm        */
  CS_F_NEAR_TIE = 16       /* some selection's margin (cs_info.min_margin) was within
                              4 (tol + u log2 N) of its chosen key (u the unit roundoff
                              of the working precision): a different but equally
                              valid trajectory was within the keys' resolution     */
};

/* Sensing operator A = Phi Psi with Phi = D F R (Eq. (7)): D keeps rows, F
 * is the orthonormal DCT-II, R the randomizer: entry j of x enters the DCT at
 * index perm[j] with sign signs[j].  perm == NULL is the identity
 * (R = diag(signs), the headline workloads here); the paper's R is a uniform
 * random permutation (perm with all signs +1).  Psi is the sparsifying basis
 * of Eq. (2): psi = 0 the identity; psi = 1 the orthonormal DCT-II, as in the
 * experiments of Sec. IV-A (A s = D F R F s); psi = 2 the separable 2-D DCT
 * of Sec. III-E with both factors the orthonormal DCT-II F_n of the side
 * n = sqrt(N) (x = vec(F_n S F_n^T), s = vec(S) row-major; N = n^2 with n a
 * power of two in [8, 8192], FP64 [8, 4096], else CS_E_SHAPE).  With psi != 0
 * every H-apply runs two more transforms and two reorders through R; the
 * workspace must be sized by cs_workspace_size_op(), and the batched entry
 * point rejects it. */
typedef struct {
  int64_t n;              /* signal length N                                        */
  int64_t m;              /* number of sampled rows M                               */
  const int32_t* rows;    /* device [m]: sampled DCT rows, strictly ascending      */
  const int8_t* signs;    /* device [n]: sign flips, each +1 or -1                  */
  const int32_t* perm;    /* device [n] permutation of [0, N), or NULL              */
  int32_t psi;            /* sparsifying basis: 0 identity, 1 the transform F,
                             2 separable 2-D DCT-II on an n x n image             */
  int32_t xform;          /* F: 0 orthonormal DCT-II; 1 orthonormal real Fourier
                             basis (partial Fourier sensing, see above); 2 partial
                             complex Fourier sensing of a real signal (below)     */
} cs_op;

/*
 * Partial complex Fourier sensing (xform = 2): A x = D(FFT(x)), the randomly
 * partial Fourier matrix of Sec. II, for a real signal x.  F is the unitary
 * DFT ((F v)_k = N^(-1/2) sum_n v_n e^(-2 pi i k n / N)), R the sign flip (and
 * permutation), and `rows` holds the M sampled frequencies, strictly ascending
 * in [1, N/2) (a real signal's coefficients at 0 and N/2 are real and those at
 * N - k conjugate to those at k, so each complex degree of freedom is sampled
 * once; M <= N/2 - 1).  The measurements y, cs_apply_A's output, cs_apply_At's
 * input and cs_adjoint_ls's grad_y are M complex values stored as (re, im)
 * pairs of the dtype (2M reals); s stays real.  The least squares is over real
 * coefficients with the complex norm, and the adjoint is that of the real inner
 * product Re<u, v>: A* u = R^T Re(F^H D^T u).  K may reach 2M (SP: K <= M,
 * CoSaMP: 3K <= 2M).  OMPR's default step is N/M with this M; cs_info.resid_norm
 * is the complex ||y - A s||, and decision margins of correlation keys are those
 * of 2 A* r (the call runs the real rows k and N - k of the real Fourier basis,
 * on which the complex problem is the same problem with the data scaled by
 * sqrt 2).  psi must be 0; size the workspace with cs_workspace_size_op; the
 * batched calls reject it (CS_E_OP).  Frequencies outside [1, N/2) or not
 * strictly ascending give CS_E_OP.
 */

/* Optional knobs; pass NULL for the defaults shown. */
typedef struct {
  int32_t cg_max_iter;    /* CG iterations per solve; 0 -> 2|S| + 50                */
  int32_t max_outer;      /* SP rounds / OMPR swaps; 0 -> SP 100, OMPR 4K           */
  int32_t warm_start;     /* 1 (default) start CG from the previous solution; 0 cold */
  int32_t cg_block;       /* batched calls: threads per block of the per-signal CG
                             kernels (64..1024, a multiple of 64); 0 -> 256.
                             Single-signal calls ignore it.                          */
  double ompr_eta;        /* OMPR step eta; <= 0 -> N/M                             */
  int32_t tol_abs;        /* 1: `tol` is absolute, each CG solve stops at
                             ||b - H theta|| <= tol (the xi of the CG loop test of
                             Algorithm 1 as printed); 0 (default): relative, <= tol ||b||     */
  int32_t ompr_l;         /* OMPR replacement size l (indices swapped per step);
                             0 -> 1                                                 */
} cs_params;

/* Filled on return when non-NULL (host memory). */
typedef struct {
  int32_t outer_iters;    /* OMP: K; SP: rounds; OMPR: swaps performed              */
  int32_t flags;          /* CS_F_* bits                                            */
  int64_t cg_iters;       /* total CG iterations over all solves                    */
  int64_t transforms;     /* N-point transforms applied (forward + inverse)         */
  double resid_norm;      /* ||y - A s|| of the returned s (FP64 accumulation)      */
  double model_bytes;     /* algorithmic HBM bytes of the transform passes          */
  double min_margin;      /* smallest decision margin of the call, in the working
                             precision: over every selection (argmax, top-K, OMPR
                             drop) the key of the last chosen candidate minus the
                             key of the first rejected one (a lower bound of it
                             where a top-K's rejected keys were not all seen);
                             0 for a tie broken by index; -1 with no selection
                             (cs_ls_solve, cs_adjoint_ls)                          */
} cs_info;

/* Workspace bytes needed by one call of `algo` at these sizes (0 if invalid).
 * It grows as O(N + K) (Sec. III-D: the method's memory is O(N)). */
size_t cs_workspace_size(cs_dtype dtype, int64_t n, int64_t m, int32_t k, cs_algo algo);

/* The same for a given operator (host descriptor; only n, m and psi are
 * read): a DCT sparsifying basis needs two more N-vectors (psi = 1) or four
 * and a twiddle table (psi = 2).  0 if invalid. */
size_t cs_workspace_size_op(cs_dtype dtype, const cs_op* op, int32_t k, cs_algo algo);

/*
 * Recovery entry points: y [M] -> s [N] (dense, zero off the support) and
 * support [K] (int32, strictly ascending).  `tol` is the CG stopping
 * tolerance, relative: each solve stops when ||b - H theta|| <= tol ||b||
 * (the CG loop test of Algorithm 1 with xi = tol ||b||).
 *
 * cs_recover_omp:  Sec. II steps 1-4 / Algorithm 1: K iterations of
 *                  argmax |A^T r| outside S, S <- S + t, CG least squares,
 *                  r = y - A s.
 * cs_recover_sp:   Subspace Pursuit: top-K of |A^T y|; then rounds of
 *                  expand by the top-K of |A^T r| outside T, least squares on
 *                  the 2K columns, prune to the top-K magnitudes, least
 *                  squares; stops when the support repeats or the residual
 *                  grows.
 * cs_recover_ompr: OMPR with replacement size l (cs_params.ompr_l, default 1):
 *                  top-K of |A^T y|; then steps that take the l best
 *                  correlations J outside S and keep the top-K of
 *                  |x + eta A^T r| over S u J; stops when no index of J is
 *                  kept (for l = 1: when j would be dropped).
 * cs_recover_cosamp: CoSaMP on the same steps: from x = 0, rounds that merge
 *                  the top-2K of |A^T r| with the support, solve least squares
 *                  on the union, keep its K largest entries and update r;
 *                  stops when the support repeats or the residual grows.
 *                  Needs 3K <= M.
 * Ties in every selection rank by (magnitude descending, index ascending).
 */
cs_status cs_recover_omp(cs_dtype dtype, const void* y, const cs_op* op, int32_t k, double tol,
                         void* s, int32_t* support, const cs_params* params,
                         void* ws, size_t ws_bytes, cs_info* info, hipStream_t stream);
cs_status cs_recover_sp(cs_dtype dtype, const void* y, const cs_op* op, int32_t k, double tol,
                        void* s, int32_t* support, const cs_params* params,
                        void* ws, size_t ws_bytes, cs_info* info, hipStream_t stream);
cs_status cs_recover_ompr(cs_dtype dtype, const void* y, const cs_op* op, int32_t k, double tol,
                          void* s, int32_t* support, const cs_params* params,
                          void* ws, size_t ws_bytes, cs_info* info, hipStream_t stream);
cs_status cs_recover_cosamp(cs_dtype dtype, const void* y, const cs_op* op, int32_t k, double tol,
                            void* s, int32_t* support, const cs_params* params,
                            void* ws, size_t ws_bytes, cs_info* info, hipStream_t stream);

/*
 * cs_recover_sp_static: cs_recover_sp without a workspace argument, for
 * callers that cannot allocate device memory (code under HIP graph capture,
 * tight serving loops, harnesses that forbid hipMalloc).  The workspace is a
 * static device array of CS_STATIC_WS_BYTES bytes inside the library, one per
 * GPU, held from the library's first use on that GPU until the process ends;
 * its device address is looked up on the first call on each device (with that
 * device current).  The call itself allocates nothing: no hipMalloc, hipFree
 * or pinned host buffer (host reads of loop flags are stream-ordered copies
 * into the call's own stack followed by a wait on `stream`), and kernel
 * timing (cs_prof_*) is not recorded for it.  Arguments, results, cs_info and
 * errors are those of cs_recover_sp; sizes whose cs_workspace_size_op(...,
 * CS_ALGO_SP) exceeds CS_STATIC_WS_BYTES (FP32: N up to 2^21 at M = N/4,
 * K = M/64; FP64: N up to 2^20) return CS_E_WORKSPACE with nothing written.
 * Every call on one GPU shares that GPU's array and leaves its contents
 * behind (each call initialises what it reads): calls that overlap on one
 * GPU, from several threads or on several streams, race and must be
 * serialised by the caller.
 */
#define CS_STATIC_WS_BYTES (64u << 20)
cs_status cs_recover_sp_static(cs_dtype dtype, const void* y, const cs_op* op, int32_t k, double tol,
                               void* s, int32_t* support, const cs_params* params, cs_info* info,
                               hipStream_t stream);

/*
 * The CG function of Algorithm 1 on its own: solve the weighted
 * least squares of Eq. (10) through its normal equations, Eq. (11), for the
 * columns `support` [k] (device int32, strictly ascending, in [0, N)).
 * theta [k] receives the solution on the support, in support order.
 * x0 [k] (nullable) is the starting point (NULL: theta = 0, the algorithm's own start).
 */
cs_status cs_ls_solve(cs_dtype dtype, const void* y, const cs_op* op, const int32_t* support,
                      int32_t k, double tol, const void* x0, void* theta,
                      const cs_params* params, void* ws, size_t ws_bytes, cs_info* info,
                      hipStream_t stream);

/*
 * Backward of a recovery on its frozen final support.  On `support` [k]
 * (device int32, strictly ascending) the recovered coefficients are the
 * least-squares solution of Eq. (10)-(11), s_S = (A_S^T A_S)^-1 A_S^T y,
 * linear in y, and s is zero off the support.  Given grad_s [N] = dL/ds
 * (dense; only its entries on the support are read) this writes
 *     grad_y [M] = dL/dy = A_S (A_S^T A_S)^-1 (dL/ds)_S.
 * It is one more solve of the CG function of Algorithm 1, with right-hand
 * side (dL/ds)_S (same `tol` semantics and cs_info fields as cs_ls_solve),
 * followed by one forward apply of A on the support.  The workspace is sized
 * by cs_workspace_size(..., k, CS_ALGO_LS).
 */
cs_status cs_adjoint_ls(cs_dtype dtype, const cs_op* op, const int32_t* support, int32_t k,
                        const void* grad_s, double tol, void* grad_y,
                        const cs_params* params, void* ws, size_t ws_bytes, cs_info* info,
                        hipStream_t stream);

/*
 * Batched recovery: `count` independent signals, each with its own operator
 * (N, M, rows, signs), sparsity K, measurements and outputs, recovered by
 * one call.  Every signal follows the same decision rules as the
 * single-signal call (here OMPR, l = 1, as cs_recover_ompr) and gets the same
 * kind of result; the signals advance together through batched device steps
 * (per-size-class transform passes over all signals, then per-signal CG and
 * selection work) that the library captures in a HIP graph and replays until
 * every signal has stopped.  `items` is a host array of `count` descriptors
 * whose pointers are device pointers; `info` is a host array of `count`
 * entries (nullable).  Sizes follow the single-signal rules per signal.  The
 * workspace is cs_workspace_size_batched() bytes (256-byte aligned).  The
 * call synchronises `stream` and returns with all outputs complete.
 */
typedef struct {
  cs_op op;               /* this signal's operator                                 */
  const void* y;          /* device [M]                                             */
  void* s;                /* device [N] output, dense                               */
  int32_t* support;       /* device [K] output, strictly ascending                  */
  int32_t k;              /* sparsity K                                             */
  int32_t moves_cap;      /* swaps `moves` can hold (0: none are recorded)          */
  int32_t* moves;         /* device [2 moves_cap] output or NULL: swap i writes the
                             natural index that entered the support at 2i and the
                             one that left at 2i+1, in order, for the first
                             moves_cap swaps (the trajectory, e.g. to compare a
                             recovery's decisions with a reference's)           */
} cs_batch_item;

size_t cs_workspace_size_batched(cs_dtype dtype, int32_t count, const cs_batch_item* items, cs_algo algo);

/*
 * cs_recover_sp_batched: Subspace Pursuit (as cs_recover_sp) on `count`
 * independent signals in one call, for example the forward of a batch being
 * differentiated.  Each signal runs the single-signal driver on its own slice
 * of the workspace (cs_workspace_size_batched(..., CS_ALGO_SP); operators may
 * use any psi), with results identical to cs_recover_sp on that signal; the
 * signals run concurrently on a pool of host threads, each with its own HIP
 * stream (default priority), that the library creates on the first batched
 * call on a device and keeps until the process ends.  Work queued on `stream`
 * before the call completes before any signal starts; the call returns with
 * every output complete and does not use `stream` afterwards.  The moves
 * fields of the items are ignored.  Not capturable in a HIP graph: the SP
 * loop decides on the host between steps (support repeated, residual grown),
 * reading small device words, as the single-signal call does.  A failing
 * signal makes the call return its status (text: cs_last_error()), other
 * signals' outputs complete.
 */
cs_status cs_recover_sp_batched(cs_dtype dtype, int32_t count, const cs_batch_item* items, double tol,
                                const cs_params* params, void* ws, size_t ws_bytes, cs_info* info,
                                hipStream_t stream);

cs_status cs_recover_ompr_batched(cs_dtype dtype, int32_t count, const cs_batch_item* items, double tol,
                                  const cs_params* params, void* ws, size_t ws_bytes, cs_info* info,
                                  hipStream_t stream);

/* out [M] = A x for a dense x [N] (Sec. III-D: sign flip, DCT-II, row pick). */
cs_status cs_apply_A(cs_dtype dtype, const cs_op* op, const void* x, void* out,
                     void* ws, size_t ws_bytes, hipStream_t stream);
/* out [N] = A^T u for u [M] (zero-fill, DCT-III, sign flip). */
cs_status cs_apply_At(cs_dtype dtype, const cs_op* op, const void* u, void* out,
                      void* ws, size_t ws_bytes, hipStream_t stream);

/*
 * Tuning of the transform passes.  The DCT of Sec. III-D runs as an
 * N/2-point complex FFT split four-step into L1 x L2 (column passes over
 * strips of 2^log_b columns, row passes over row pairs, 2^log_e elements per
 * thread).  Several splits are compiled per N; which is fastest depends on
 * the device, so a tuner can time them and install its choice for the rest of
 * the process.  Results are the same up to rounding whichever split runs.
 *
 * cs_shape_candidates: the compiled shapes for N, the default first; writes
 *   up to `max` into out (out == NULL: returns the count only).
 * cs_set_shape: makes `shape` (one of the candidates) the shape of every later
 *   call at this N in this process; NULL restores the default.  Not to be
 *   called while other calls run.  Workspace sizes do not depend on it.
 * cs_time_shape: average milliseconds of one H-apply (the three transform
 *   passes of one CG iteration, on a dense N-vector) with `shape`, over `reps`
 *   applies on `stream`; workspace as for cs_apply_A.
 */
typedef struct {
  int32_t log_l1, log_l2, log_b, log_e;
} cs_shape;
int cs_shape_candidates(cs_dtype dtype, int64_t n, cs_shape* out, int32_t max);
cs_status cs_set_shape(cs_dtype dtype, int64_t n, const cs_shape* shape);
cs_status cs_time_shape(cs_dtype dtype, const cs_op* op, const cs_shape* shape, int32_t reps, void* ws,
                        size_t ws_bytes, hipStream_t stream, double* ms_per_apply);

const char* cs_status_str(cs_status status);
const char* cs_last_error(void);

/*
 * Opt-in timing of the transform passes (not part of the method; for
 * measurement).  When enabled, each column / row pass launch is bracketed by
 * HIP events on the caller's stream; per-class totals accumulate until
 * cs_prof_reset().  `bytes` is the algorithmic HBM traffic of those launches:
 * one N-vector read and one written per pass, except that a column pass on
 * the compact CG vectors replaces one of them by the k support keys and the
 * compact values it moves, and the residual row pass also reads y.
 * Classes: col_fwd, col_inv, row_happly, row_resid, row_fwd, row_adj.
 */
typedef struct {
  char name[32];
  int64_t launches;
  double total_ms;
  double bytes;
} cs_prof_stat;
int cs_prof_enable(int on);                   /* returns the previous state          */
void cs_prof_reset(void);
int cs_prof_read(cs_prof_stat* out, int max);  /* out == NULL: number of classes      */

#ifdef __cplusplus
}
#endif
#endif /* CS_H */
