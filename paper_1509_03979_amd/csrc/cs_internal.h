// Internal declarations shared by the libcsrecover translation units.
//
// Data layout (all device memory, inside the caller's workspace):
//  * "v-order" dense N-vectors.  The DCT-II of x is computed through the
//    real sequence v (v_n = x_{2n}, v_{N-1-n} = x_{2n+1}, n < N/2) packed as
//    N/2 complex values z_m = v_{2m} + i v_{2m+1}.  Dense spatial-domain
//    buffers store v directly, so x_j lives at position vpos(j) and the
//    transform reads z with no permutation pass.
//  * four-step split of the N/2-point complex FFT: L = L1 * L2, z viewed as
//    an L1 x L2 row-major array (z[L2 n1 + n2]).  Column FFTs (length L1) run
//    in place over strips of B adjacent columns; row FFTs (length L2) run over
//    mirror row pairs (k1, L1-k1) so that the DCT post/pre-processing, which
//    couples Z_k with Z_{L-k}, happens inside one workgroup.
//  * "freq-layout": one slot per complex bin Z_k, stored in the order the row
//    pass visits them (slot f = (k mod L1) * L2 + k / L1).  Slot k owns the
//    two DCT outputs X_k and X_{N-k} (slot 0 owns X_0 and X_{N/2}).  The row
//    mask of D and the measurements y are kept in this layout.
#pragma once

#include <hip/hip_runtime.h>
#include <algorithm>
#include <cstdint>
#include <cstddef>
#include <string>
#include <stdexcept>
#include <vector>

#include "../../include/cs.h"

namespace csr {

// ------------------------------------------------------------------ errors
struct Error : std::runtime_error {
  cs_status status;
  Error(cs_status s, const std::string& m) : std::runtime_error(m), status(s) {}
};

void hip_check(hipError_t e, const char* what, const char* file, int line);
#define CS_HIP(x) ::csr::hip_check((x), #x, __FILE__, __LINE__)
#define CS_LAUNCH_CHECK() ::csr::hip_check(hipGetLastError(), "kernel launch", __FILE__, __LINE__)

// ------------------------------------------------------------------ complex
template <typename T>
struct alignas(2 * sizeof(T)) Cx {
  T re, im;
};

template <typename T>
__device__ __forceinline__ Cx<T> cx(T r, T i) { Cx<T> c; c.re = r; c.im = i; return c; }
template <typename T>
__device__ __forceinline__ Cx<T> operator+(Cx<T> a, Cx<T> b) { return cx(a.re + b.re, a.im + b.im); }
template <typename T>
__device__ __forceinline__ Cx<T> operator-(Cx<T> a, Cx<T> b) { return cx(a.re - b.re, a.im - b.im); }
template <typename T>
__device__ __forceinline__ Cx<T> cmul(Cx<T> a, Cx<T> b) {
  return cx(a.re * b.re - a.im * b.im, a.re * b.im + a.im * b.re);
}
// a * conj(b)
template <typename T>
__device__ __forceinline__ Cx<T> cmulc(Cx<T> a, Cx<T> b) {
  return cx(a.re * b.re + a.im * b.im, a.im * b.re - a.re * b.im);
}
template <typename T>
__device__ __forceinline__ Cx<T> conj(Cx<T> a) { return cx(a.re, -a.im); }
template <typename T>
__device__ __forceinline__ Cx<T> scale(Cx<T> a, T s) { return cx(a.re * s, a.im * s); }

// ------------------------------------------------------------------ plan
// Four-step shape of the N/2-point complex FFT: L1 = 2^logL1 rows of
// L2 = 2^logL2, column strips of 2^logB columns, 2^logE elements per thread.
struct Shape {
  int logL1, logL2, logB;
  int logE;               // log2 of the elements each thread holds (caps the radix)
};

// Everything the transform kernels need for one N, passed by value.
struct Plan {
  int64_t n, m;
  int64_t words;          // 32-bit words of an N-bit bitmap
  int logn;
  int64_t L;              // N/2 complex points
  int logL;
  int L1, L2, logL1, logL2;
  int B, logB;            // column strip width of the column passes
  int logE;               // log2 elements per thread in the LDS FFTs
  int alt;                // 1 when an alternative (tuning) shape is in use
  int nt_col, nt_row;     // threads per workgroup of the column / row passes
  size_t lds_col, lds_row;
  const void* tw_lo;      // W_{4N}^i, i in [0, 4096)          (Cx<T>)
  const void* tw_hi;      // W_{4N}^{4096 h}, h in [0, 4N/4096) (Cx<T>)
  const void* tw_step;    // W_{4N}^{i L1 nt_row} (i < 16), then W_{4N}^{4 i L1 nt_row}: the row pass's
                          // per-item Makhoul twiddle steps (Cx<T>, 2 kTwStepHalf entries)
  const uint32_t* mask;   // N bits in freq-layout: bit 2f+h = row sampled
  const int32_t* perm;    // randomizer permutation: entry j enters the DCT at perm[j] (null: identity)
  const int32_t* pinv;    // its inverse (null with perm)
  int keynat;             // 1: candidates are keyed by their natural index (2-D DCT basis)
  int fourier;            // 1: F is the orthonormal real Fourier basis instead of the DCT-II
};

constexpr int kTwStage = 8192;   // entries reserved for one stage-twiddle table (size 2^13 needs 8176)
constexpr int kTwLo = 4096;
constexpr int kTwStepHalf = 16;
constexpr int kTwLoLog = 12;

// v-order position of natural index j, and its inverse.
__host__ __device__ __forceinline__ int64_t vpos(int64_t j, int64_t n) {
  return (j & 1) ? (n - 1 - (j >> 1)) : (j >> 1);
}
__host__ __device__ __forceinline__ int64_t vinv(int64_t p, int64_t n) {
  return (p < (n >> 1)) ? (2 * p) : (2 * (n - 1 - p) + 1);
}
// Position of transform input q in the packed N-vector: v-order for the DCT
// (Makhoul's reordering), natural for the real Fourier basis.
__host__ __device__ __forceinline__ int64_t xpos(int64_t q, const Plan& pl) {
  return pl.fourier ? q : vpos(q, pl.n);
}
__host__ __device__ __forceinline__ int64_t xinv(int64_t p, const Plan& pl) {
  return pl.fourier ? p : vinv(p, pl.n);
}
// freq-layout float position of DCT output index q.
__host__ __device__ __forceinline__ int64_t fpos(int64_t q, const Plan& p) {
  int64_t k, h;
  if (q == 0) { k = 0; h = 0; }
  else if (q == p.L) { k = 0; h = 1; }
  else if (q < p.L) { k = q; h = 0; }
  else { k = p.n - q; h = 1; }
  int64_t f = (k & (p.L1 - 1)) * p.L2 + (k >> p.logL1);
  return 2 * f + h;
}

// Key order.  The greedy drivers index candidates by key, an order that
// follows the column passes: position p (complex element m = p/2 = n1 L2 + c,
// half h = p mod 2) belongs to strip g = c / B; keys number strips first, then
// rows, then the strip's columns, then the half, so the support bits and the
// correlation values one column workgroup touches are contiguous.
__host__ __device__ __forceinline__ int64_t key_of_pos(int64_t p, const Plan& pl) {
  const int64_t m = p >> 1, h = p & 1;
  const int64_t n1 = m >> pl.logL2, c = m & (pl.L2 - 1);
  const int64_t g = c >> pl.logB, b = c & (pl.B - 1);
  return ((((g << pl.logL1) + n1) << pl.logB | b) << 1) | h;
}
__host__ __device__ __forceinline__ int64_t pos_of_key(int64_t k, const Plan& pl) {
  const int64_t h = k & 1;
  int64_t t = k >> 1;
  const int64_t b = t & (pl.B - 1);
  t >>= pl.logB;
  const int64_t n1 = t & (pl.L1 - 1), g = t >> pl.logL1;
  return (((n1 << pl.logL2) + (g << pl.logB) + b) << 1) | h;
}
// Natural index j of x <-> DCT input index (through the randomizer's
// permutation, device tables) <-> key.
__device__ __forceinline__ int64_t nat_of_key(int64_t k, const Plan& pl) {
  if (pl.keynat) return k;
  const int64_t q = xinv(pos_of_key(k, pl), pl);
  return pl.pinv ? (int64_t)pl.pinv[q] : q;
}
__device__ __forceinline__ int64_t key_of_nat(int64_t j, const Plan& pl) {
  if (pl.keynat) return j;
  const int64_t q = pl.perm ? (int64_t)pl.perm[j] : j;
  return key_of_pos(xpos(q, pl), pl);
}

// W_{4N}^idx = exp(-2 pi i idx / (4N)), idx in [0, 4N), from the two-level table.
template <typename T>
__device__ __forceinline__ Cx<T> tw4n(const Plan& p, uint32_t idx) {
  const Cx<T>* lo = (const Cx<T>*)p.tw_lo;
  const Cx<T>* hi = (const Cx<T>*)p.tw_hi;
  return cmul(lo[idx & (kTwLo - 1)], hi[idx >> kTwLoLog]);
}

// XCD-aware block order: dispatch sends block b to XCD b % 8; give each XCD
// a contiguous range of work items so neighbours share its L2.
__device__ __forceinline__ int xcd_order(int b, int nb) {
  if (nb & 7) return b;
  return (b & 7) * (nb >> 3) + (b >> 3);
}

// ------------------------------------------------------------------ compact column-pass I/O
// The CG works on compact vectors indexed by the support's rank in key order
// (key_of_pos).  Its support is an ascending key list plus an N-bit key bitmap
// with, per 32-bit word, the number of set bits in all earlier words (wpre):
// the compact slot of key k is wpre[k/32] + popcount(bits below k in its
// word), which gives each column strip its range of slots.  The CG runs in
// sign-flipped coordinates (x' = R x for the diagonal sign flip R), which
// leaves every inner product unchanged and lets the column passes move raw
// values.
enum ColMode {
  COL_DENSE = 0,   // forward: read a dense v-order input; inverse: write dense v-order output
  COL_X = 1,       // forward: input = x on the support
  COL_DIR = 2,     // forward: d = r + beta d (d = r at iteration 0), input = d
                   //   (fused: first x += alpha d, r -= alpha q of the previous iteration)
  COL_Q = 3,       // inverse: q = output on the support, partial d^T q per workgroup
                   //   (fused: partials of d^T q, r^T r, r^T q, q^T q for the step kernel)
  COL_R = 4,       // inverse: r = b - output, d = r, partial r^T r per workgroup
  COL_KEY = 5      // inverse: write dense key-order output
};

template <typename T>
struct ColIO {
  int mode;
  int it;                  // COL_DIR / COL_Q: iteration index
  int max_iter;            // COL_Q (fused): iteration cap
  int fused;               // COL_DIR / COL_Q: the CG vector and scalar updates ride on the passes
  int kcap;                // compact length; slots at or beyond it are ignored
  const uint32_t* sbits;   // support bitmap over keys
  const uint32_t* wpre;    // per-word exclusive prefix counts of sbits
  const int32_t* list;     // ascending support keys (kcap of them)
  T* x;
  T* r;
  T* d;
  T* q;
  const T* b;
  double* pout;            // COL_Q / COL_R: one partial per workgroup (fused COL_Q: four, by rows of G)
  struct CgScalars* cg;    // nullable: no early exit, no scalar updates
};

// ------------------------------------------------------------------ context
// Per-call state: plan, workspace carving, device scalars.
struct CgScalars {
  double rr[2];           // r^T r, ping-pong by iteration parity
  double bb;              // b^T b
  double tol2;            // tol^2
  double resid2;          // ||y - A x||^2 of the last residual pass
  int32_t differ;         // set by bits_differ; read back with resid2
  int32_t pad0;
  double dq;              // d^T H d of the current iteration
  double beta;            // next direction update coefficient
  double alpha;           // step of the last iteration (fused passes: applied by the next one)
  double ref;             // the stopping test is r^T r <= tol2 * ref: ref = b^T b (relative) or 1 (absolute)
  int32_t done;
  int32_t iters;
  int32_t flags;
  int32_t pad1;
};

struct SelHead {           // radix state between the passes of a top-K
  uint64_t prefix, pmask;  // key prefix found so far
  int64_t need;            // how many of the keys matching the prefix to take
  int32_t mode;            // candidate source
  int32_t bit;             // unresolved low key bits
  int32_t tie;             // 1 if more keys equal the threshold than are needed
  int32_t pending;         // 1 if the previous pass left histogram rows to pick from
};

struct SelState {          // top-K selection state
  SelHead head[2];         // double-buffered by pass parity
  int64_t k;               // K of the current selection
  uint64_t t_lo, t_hi;     // candidate band of the dense split
  uint64_t tau;            // threshold key of the last selection
  int32_t tie_out;         // whether the last selection broke a tie by index
  int32_t nonfinite;
  uint64_t below;          // largest key below the threshold seen by the final pass (0: none)
  double mmin;             // smallest decision margin of the call so far (+inf: none)
  double mrel;             // the smallest margin relative to its decision's key
};

// Dense top-K split: one workgroup of kSplitThreads per block of `per_block`
// elements (a multiple of 4 kSplitThreads), each with `cap` candidate slots.
constexpr int kSplitBlocks = 1024;
constexpr int kSplitThreads = 512;
struct SplitLayout {
  int blocks;
  int64_t per_block;
  int cap;
};
inline SplitLayout split_layout(int64_t n) {
  constexpr int64_t r = 4 * kSplitThreads;
  int64_t g = std::min<int64_t>(kSplitBlocks, (n + r - 1) / r);
  const int64_t eb = ((n + g - 1) / g + r - 1) / r * r;
  g = (n + eb - 1) / eb;
  return SplitLayout{(int)g, eb, (int)(eb / 8 + 64)};
}
constexpr int kPassBlocks = 128;  // workgroups of a radix pass
constexpr int kSelDigit = 13;     // radix digit width of the top-K passes
constexpr int kSelBins = 1 << kSelDigit;

struct ArgKey {            // argmax key: (magnitude bits + 1, ~index)
  uint64_t hi;
  uint32_t lo;
  uint32_t pad;
};

template <typename T>
struct Ctx {
  hipStream_t stream;
  Plan plan;
  const int8_t* signs;     // natural order, on the greedy candidates (null: all +1)
  // Sparsifying basis Psi = DCT-II (psi = 1): the candidates index s, whose
  // transform has no randomizer (plan.perm/pinv and signs are null); the
  // randomizer R sits between Psi's output and Phi's input, applied by the
  // reorder kernels through rsigns/rperm/rpinv.
  int psi = 0;
  const int8_t* rsigns = nullptr;
  const int32_t* rperm = nullptr;
  const int32_t* rpinv = nullptr;
  T* P1 = nullptr;         // psi: freq-layout N-vector (Psi output / Psi^T input); psi 2: x in natural order
  T* P2 = nullptr;         // psi: v-order N-vector (Phi input / output)
  // psi = 2, the separable 2-D DCT basis on an n x n image (n = 2^dct_log):
  T* P3 = nullptr;         // the support scattered into a zero image (fixed within a CG solve)
  T* P4 = nullptr;         // row-pass intermediate
  Cx<T>* tw_dct = nullptr; // stage twiddles of the n/2-point row FFTs
  int dct_log = 0;
  const int32_t* rows;
  // Partial complex Fourier sensing (cs_op.xform = 2): the M sampled
  // frequencies k in [1, N/2) become the 2M rows k and N - k of the real
  // Fourier basis (rows_x, ascending), and complex data enter and leave
  // through ybuf (2M reals) by the row pairing of cplx_in / cplx_out.
  int cplx = 0;
  const int32_t* freq = nullptr;   // caller's frequencies (device, M)
  int32_t* rows_x = nullptr;       // expanded rows (workspace, 2M)
  T* ybuf = nullptr;               // expanded real data (workspace, 2M)
  int kmax;                // largest support handled by the compact buffers
  // dense N-vectors (v-order unless noted)
  Cx<T>* W;                // transform work buffer (L complex)
  T* Dd;                   // dense scratch (operator input)
  T* Cc;                   // correlation F^T D^T r, key order (shares Dd's memory)
  T* C0;                   // F^T D^T y (A^T y before the sign flip), key order
  T* Yf;                   // y in freq-layout (N reals)
  // twiddles, masks
  Cx<T>* tw_col; Cx<T>* tw_row;   // stage twiddles of the L1- and L2-point FFTs
  Cx<T>* tw_lo; Cx<T>* tw_hi;
  Cx<T>* tw_step;
  uint32_t* mask;          // row mask of D, freq-layout bits
  int32_t* pinv;           // inverse of the randomizer's permutation (N entries)
  // supports: key bitmaps, ascending key lists and per-word prefix counts
  uint32_t* bits[3];
  int32_t* list[3];
  uint32_t* wpre[3];
  uint32_t* nbits;         // natural-index bitmap for the output support
  // compact buffers (kmax each, key order, sign-flipped coordinates)
  T *cb, *cx, *cr, *cd, *cq, *cx2, *cx3;
  // reductions
  double* partial;         // 4 * kRedBlocks doubles
  double* partial2;        // row-pass partials (L1/2)
  double* pgrid;           // column-pass partials (one per column workgroup)
  ArgKey* argpart;         // kArgBlocks
  void* rkey;              // dense top-K candidates: keys (width of T), positions and
  uint32_t* rpos;          //   per-block (count, selected count) pairs
  int32_t* rcnt;
  uint32_t* hrows;         // radix histograms: three rows of kSelBins counts (pass p adds into
                           //   row p mod 3, picks from row p-1 mod 3, clears row p+1 mod 3)
  int32_t* ibuf;           // small int scratch (>= 64)
  uint32_t* blockcnt;      // bitmap compaction block counts
  CgScalars* cg;
  SelState* sel;
  double ynorm = 0;        // ||y||, FP64 accumulation
  int32_t last_differ = 0; // CgScalars::differ as read back by the last resid_corr
  int tol_abs = 0;         // CG tolerance absolute (||r|| <= tol) instead of relative
  // host-side counters
  int64_t transforms = 0;
  int64_t cg_iters = 0;
  // iterations of the last solves by support size and start (cold or warm),
  // to size a solve's first queued chunk of iterations (most recent first)
  struct CgHint {
    int k = -1;
    int warm = 0;
    int it = 0;
  } hint[4];
  int last_warm_it = -1;   // iterations of the most recent warm-started solve
  double model_bytes = 0;
  int32_t flags = 0;
};

// ------------------------------------------------------------------ batched recovery
// Per-signal phase of the batched OMPR driver.  One batched step moves every
// signal one stage along: a warm-started CG solve (WARM, then ITER per
// iteration), the residual and correlation (RESID), the OMPR swap (SELECT).
enum BPhase { BP_WARM = 0, BP_ITER = 1, BP_RESID = 2, BP_SELECT = 3, BP_DONE = 4 };

struct BState {
  int32_t phase;
  int32_t cur;            // list / x slot of the current support (0 or 1)
  int32_t it;             // CG iteration within the current solve
  int32_t swaps;          // OMPR swaps done
  int32_t k, max_outer, cg_cap, flags;
  int32_t warm, jd[2], tol_abs;
  int64_t cg_iters, transforms;
  double rn, bb, tol2, eta, ynorm, model_bytes;
  double mmin, mrel;      // decision margins (as SelState's)
};

template <typename T>
struct BSig {              // device-side view of one signal of a batch
  Plan plan;
  Cx<T>* W;
  T* Cc;
  T* C0;
  T* Yf;
  const Cx<T>* tw_col;
  const Cx<T>* tw_row;
  uint32_t* bits;          // support key bitmap
  uint32_t* wpre[2];
  int32_t* list[2];
  T* cb;
  T* cx[2];
  T *cr, *cd, *cq;
  double* pgrid;           // column-pass partials
  double* prow;            // row-pass partials
  ArgKey* argpart;
  uint32_t* blockcnt;
  CgScalars* cg;
  BState* st;
  int32_t* moves;          // swap log (entered, left) per swap, or null
  int32_t moves_cap;
};

// A support as the CG sees it.
struct Supp {
  const uint32_t* bits;    // key bitmap
  const uint32_t* wpre;    // per-word exclusive prefix counts
  const int32_t* list;     // ascending keys
  int k;
};

constexpr int kRedBlocks = 256;   // blocks of the compact reductions
constexpr int kRedThreads = 256;
constexpr int kArgBlocks = 1024;
constexpr int kBitsPerBlockWords = 1024;  // words per block in bitmap compaction

// ------------------------------------------------------------------ profiling
enum ProfClass { PC_COL_FWD = 0, PC_COL_INV, PC_ROW_HAPPLY, PC_ROW_RESID, PC_ROW_FWD, PC_ROW_ADJ, PC_COUNT };
bool prof_on();
int prof_begin(hipStream_t s, hipEvent_t* ev);
int prof_end(int cls, double bytes, hipEvent_t start, hipStream_t s);   // record index
void prof_discard(int idx);   // drop a recorded launch (it exited early: no work done)
void prof_flush();

// ------------------------------------------------------------------ plan/workspace
// Plan for N: the shape given in `force`, else the process-wide choice for
// this N (set_shape_override), else the default.  False if N or the shape is
// unsupported.
bool choose_plan(cs_dtype dt, int64_t n, int64_t m, Plan& p, const Shape* force = nullptr);
// Compiled shapes for L = 2^l, the default first; returns how many (<= max).
int shape_candidates(cs_dtype dt, int l, Shape* out, int max);
// Installs (s != nullptr) or clears the process-wide shape for L = 2^l.
bool set_shape_override(cs_dtype dt, int l, const Shape* s);
size_t workspace_bytes(cs_dtype dt, int64_t n, int64_t m, int32_t k, cs_algo algo, int psi = 0, int cplx = 0);

template <typename T>
void ctx_init(Ctx<T>& c, const cs_op* op, int kmax, void* ws, size_t ws_bytes, hipStream_t s,
              const Shape* force = nullptr);

// ------------------------------------------------------------------ transform launchers
enum RowMode { ROW_HAPPLY = 0, ROW_RESID = 1, ROW_FWD = 2, ROW_ADJ = 3,
               ROW_FWD_ALL = 4 };   // ROW_FWD without the row mask (a full DCT-II: the DCT basis)

template <typename T> void setup_operator(Ctx<T>& c);                  // twiddles, masks (+ validation)
template <typename T> void scatter_freq(Ctx<T>& c, const T* u, T* outf); // u [M] -> freq layout
// y -> Yf (freq layout), ||y|| -> ynorm, F^T D^T y (key order) -> C0
template <typename T> void load_measurements(Ctx<T>& c, const T* y);
template <typename T> void gather_freq(Ctx<T>& c, const T* inf, T* out); // freq layout -> [M]
// Partial complex Fourier: M complex values (re, im pairs) <-> the 2M real
// rows k, N - k.  cplx_in writes ybuf[i] = a Re u_i and ybuf[2M-1-i] = b Im u_i;
// cplx_out writes out_i = (a r_i) + i (b r_{2M-1-i}) from r = ybuf.
template <typename T> void cplx_in(Ctx<T>& c, const T* u, double a, double b);
template <typename T> void cplx_out(Ctx<T>& c, T* out, double a, double b);
template <typename T> void fill(T* p, int64_t count, T v, hipStream_t s);
// Reads `bytes` (a multiple of 4, at most 1016) of device memory on the host:
// a one-block kernel copies them into a pinned, device-mapped host buffer
// (one per calling thread, kept for the life of the process) once the queued
// work before it is done, and the host waits for that.  Cheaper than a
// pageable device-to-host copy.
void dev_read(hipStream_t s, const void* dev, void* host, size_t bytes);
// The same read split in two: dev_post queues the copy into mailbox slot
// `slot` (1..3) and returns its sequence number without waiting, so more work
// can be queued behind it; dev_wait(slot, seq) waits for that copy.  Posts to
// one slot land in stream order and a wait matches only its own sequence
// number, so a post that is never collected does no harm.  Not available
// while a NoAllocScope lives (no mailbox then).
uint32_t dev_post(hipStream_t s, const void* dev, size_t bytes, int slot);
void dev_wait(hipStream_t s, int slot, uint32_t seq, void* host, size_t bytes);
// While a NoAllocScope lives on the calling thread, host reads are
// stream-ordered copies into the caller's host memory followed by a stream
// wait (the pinned mailbox allocates on its first use), and kernel timing is
// not recorded (its events are created on demand): the library then makes no
// allocation of its own.
bool no_alloc_mode();
struct NoAllocScope {
  NoAllocScope();
  ~NoAllocScope();
};
// Sums the row pass's residual partials into *r2 on the device (no read).
void dev_sum_resid(hipStream_t s, const double* partial, int np, double* r2);
void dev_read_resid(hipStream_t s, const double* partial, int np, double* r2, const int32_t* flag, double* r2_host,
                    int32_t* flag_host);
template <typename T> double norm2_host(Ctx<T>& c, const T* v, int64_t count);   // ||v||, synchronises
void fill_u32(uint32_t* p, int64_t count, uint32_t v, hipStream_t s);
void sum_partials_to(const double* partial, int np, double* out, hipStream_t s);   // *out = sum (one block)

// Launch a transform pass; returns its algorithmic bytes.  With `rec` the
// profiling record index (or -1) is stored there.
template <typename T> double launch_col(Ctx<T>& c, const Cx<T>* in, Cx<T>* out, bool inv, const ColIO<T>& io,
                                        int* rec = nullptr);
template <typename T> double launch_row(Ctx<T>& c, int mode, const T* fin, T* fout, double* partial, const int* done,
                                        int* rec = nullptr);
template <typename T> ColIO<T> col_io(Ctx<T>& c, int mode, const Supp* S);   // compact I/O on support S
template <typename T> void transform_fwd(Ctx<T>& c, const T* in, T* outf, bool all = false); // outf = DCT in freq layout, masked unless all
// out = F^T (freq input), in v-order or (key_order) key order
template <typename T> void transform_adj(Ctx<T>& c, const T* inf, T* out, bool key_order);
template <typename T> void perm_in(Ctx<T>& c, const T* x, T* dense);      // dense[vpos(perm j)] = sign_j x_j
template <typename T> void perm_out(Ctx<T>& c, const T* dense, T* x);     // x_j = sign_j dense[vpos(perm j)]
// DCT sparsifying basis: R from Psi's freq-layout output to Phi's v-order
// input, R^T back; the middle of an H-apply and of a residual pass.
template <typename T> void rand_in(Ctx<T>& c, const T* fin, T* vout, const int* done);
template <typename T> void rand_out(Ctx<T>& c, const T* vin, T* fout, const int* done);
template <typename T> double psi_middle(Ctx<T>& c, CgScalars* cg, int* rec);   // rec: 5 entries or null
template <typename T> void psi_resid_middle(Ctx<T>& c);
// psi = 2: natural-order x (instead of freq layout) through R and back
template <typename T> void rand_in_nat(Ctx<T>& c, const T* xin, T* vout, const int* done);
template <typename T> void rand_out_nat(Ctx<T>& c, const T* vin, T* xout, const int* done);
// separable 2-D DCT basis: out = vec(F S F^T) (inv: vec(F^T S F)); tmp an N-vector
constexpr int kDct2dMinLog = 3;      // image sides 8 ..
constexpr int kDct2dMaxLog32 = 13;   // .. 8192 (FP32)
constexpr int kDct2dMaxLog64 = 12;   // .. 4096 (FP64)
int dct2d_side_log(cs_dtype dt, int64_t n);   // log2 of the side, or -1 if N is not a supported square
template <typename T> void dct2d(Ctx<T>& c, bool inv, const T* in, T* tmp, T* out, const int* done);
template <typename T> void dct2d_setup(Ctx<T>& c);
template <typename T> void psi2_happly(Ctx<T>& c, CgScalars* cg, T* sout);   // image in P3 -> F^T(...)F into sout
template <typename T> void psi2_resid(Ctx<T>& c, T* cout);                  // image in P3 -> A^T (y - A x)
template <typename T> void psi2_forward(Ctx<T>& c, const T* img, T* outf);
template <typename T> void psi2_adjoint(Ctx<T>& c, const T* inf, T* out);
template <typename T> void prepare_kernels();                             // LDS limits, once per process

// ------------------------------------------------------------------ selection
// argmax of |dense| outside `excl` into *out_j (natural index; -1: none).  With
// r2 non-null the selection is gated on the device by the residual: *r2 <=
// thr2 gives *out_j = -2 and notes no margin.
template <typename T>
void argmax_excl(Ctx<T>& c, const T* dense, const uint32_t* excl, int32_t* out_j, const double* r2 = nullptr,
                 double thr2 = 0.0);
// A decision is a near-tie when its margin is within the resolution its keys
// are computed to: relative to the chosen key, kNearTie (tol + u log2 N), with
// tol the CG tolerance relative to ||b|| and u the working precision's unit
// roundoff.
constexpr double kNearTie = 4.0;
inline bool near_tie(double mrel, double tol_rel, bool f32, int logn) {
  const double u = f32 ? 0x1p-24 : 0x1p-53;
  return mrel <= kNearTie * (tol_rel + u * (double)logn);   // false for +inf (no decision)
}
// Decision margins: cleared per call; read back as (smallest margin, smallest
// margin relative to its key).
template <typename T> void sel_reset(Ctx<T>& c);
template <typename T> void margins_read(Ctx<T>& c, double* mmin, double* mrel);
template <typename T> void topk_dense(Ctx<T>& c, const T* dense, const uint32_t* excl, int k, uint32_t* out_bits);
template <typename T> void topk_compact(Ctx<T>& c, const T* vals, const int32_t* list, int count, int k, uint32_t* out_bits);
template <typename T> int bits_to_list(Ctx<T>& c, const uint32_t* bits, int32_t* list, int expect, uint32_t* wpre);
void bits_or(const uint32_t* a, const uint32_t* b, uint32_t* out, int64_t words, hipStream_t s);
int bits_equal(const uint32_t* a, const uint32_t* b, int64_t words, int32_t* scratch, hipStream_t s);
// The same comparison posted to mailbox slot `slot` without waiting (see
// dev_post): the flag (nonzero when the sets differ) is collected by dev_wait.
uint32_t bits_differ_post(const uint32_t* a, const uint32_t* b, int64_t words, int32_t* scratch, int slot,
                          hipStream_t s);
// *flag = 1 if the bitmaps differ, else 0 (no host read)
void bits_differ(const uint32_t* a, const uint32_t* b, int64_t words, int32_t* flag, hipStream_t s);

// ------------------------------------------------------------------ CG
// Solves the weighted normal equations on support S; x (compact, key order,
// sign-flipped coordinates) is the start point when `warm`, and receives the
// solution.  The right-hand side is gathered from C0 unless `b_ready` (then
// the caller has put it in cb).  With `r0_corr` the warm start's residual
// b - H x is taken from the correlation in Cc instead of a transform: valid
// when S contains the support of the solution Cc was computed from and x is
// that solution (zero on the new keys).
template <typename T>
int cg_solve(Ctx<T>& c, const Supp& S, T* x, bool warm, double tol, int max_iter, bool b_ready = false,
             bool r0_corr = false);

// outf (freq layout, N reals) = masked DCT of the compact x placed on S: the
// forward operator on the support, before the row pick.
template <typename T>
void apply_support(Ctx<T>& c, const Supp& S, const T* x, T* outf);

// r = y - A x and F^T D^T r (key order, in Cc) for the solution x on S;
// returns ||r|| (synchronises).  resid_corr_queue queues the same work and
// leaves ||r||^2 on the device (CgScalars::resid2) without waiting.
template <typename T>
double resid_corr(Ctx<T>& c, const Supp& S, const T* x);
template <typename T>
void resid_corr_queue(Ctx<T>& c, const Supp& S, const T* x);

// out[i] = x[slot of to[i] in from] or 0 when absent (both ascending key lists).
template <typename T>
void remap(Ctx<T>& c, const int32_t* from, const T* x, int kfrom, const int32_t* to, T* out, int kto);

// ------------------------------------------------------------------ drivers
template <typename T>
void run_omp(Ctx<T>& c, int k, double tol, const cs_params& prm, T* s_out, int32_t* supp_out, cs_info* info);
template <typename T>
void run_sp(Ctx<T>& c, int k, double tol, const cs_params& prm, T* s_out, int32_t* supp_out, cs_info* info);
template <typename T>
void run_ompr(Ctx<T>& c, int k, double tol, const cs_params& prm, T* s_out, int32_t* supp_out, cs_info* info);
template <typename T>
void run_cosamp(Ctx<T>& c, int k, double tol, const cs_params& prm, T* s_out, int32_t* supp_out, cs_info* info);
template <typename T>
void write_output(Ctx<T>& c, const int32_t* list, const T* x, int k, T* s_out, int32_t* supp_out);

// Batched OMPR: workspace layout (per-signal offsets appended to offs when
// non-null; returns the total bytes, 0 if a size is unsupported) and driver.
size_t batch_layout(cs_dtype dt, int count, const cs_batch_item* items, std::vector<size_t>* offs);
// Concurrent batches (cs_pool.hip): per-signal workspace slices for `algo`
// (offsets appended to offs), and the run of `one` (a single-signal
// recovery) over every signal on the per-device worker pool.
size_t batch_layout_algo(cs_dtype dt, int count, const cs_batch_item* items, cs_algo algo,
                         std::vector<size_t>* offs);
void recover_batched_pool(cs_algo algo, cs_dtype dt, int count, const cs_batch_item* items, double tol,
                          const cs_params* params, void* ws, size_t ws_bytes, cs_info* infos, hipStream_t stream,
                          void (*one)(cs_algo, cs_dtype, const void*, const cs_op*, int32_t, double, void*,
                                      int32_t*, const cs_params*, void*, size_t, cs_info*, hipStream_t));
template <typename T>
void run_ompr_batched(int count, const cs_batch_item* items, double tol, const cs_params& prm, int cg_threads,
                      void* ws, size_t ws_bytes, cs_info* infos, hipStream_t stream);

}  // namespace csr
