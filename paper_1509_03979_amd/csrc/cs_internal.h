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
#include <cstdint>
#include <cstddef>
#include <string>
#include <stdexcept>

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
  const uint32_t* mask;   // N bits in freq-layout: bit 2f+h = row sampled
};

constexpr int kTwStage = 8192;   // entries reserved for one stage-twiddle table (size 2^13 needs 8176)
constexpr int kTwLo = 4096;
constexpr int kTwLoLog = 12;

// v-order position of natural index j, and its inverse.
__host__ __device__ __forceinline__ int64_t vpos(int64_t j, int64_t n) {
  return (j & 1) ? (n - 1 - (j >> 1)) : (j >> 1);
}
__host__ __device__ __forceinline__ int64_t vinv(int64_t p, int64_t n) {
  return (p < (n >> 1)) ? (2 * p) : (2 * (n - 1 - p) + 1);
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

// ------------------------------------------------------------------ context
// Per-call state: plan, workspace carving, device scalars.
struct CgScalars {
  double rr[2];           // r^T r, ping-pong by iteration parity
  double bb;              // b^T b
  double tol2;            // tol^2
  double resid2;          // ||y - A x||^2 of the last residual pass
  int32_t done;
  int32_t iters;
  int32_t flags;
  int32_t pad;
};

struct SelState {          // radix select state
  uint64_t prefix, pmask;  // key prefix found so far
  int64_t need;            // how many of the keys equal to the final prefix to take
  int64_t count_eq;        // how many keys equal the final prefix
  uint32_t jprefix, jmask; // tie-break prefix over indices
  int64_t jneed;
  uint32_t hist[256];
  int32_t tie;             // 1 if the index tie-break is active
  int32_t nonfinite;
};

struct ArgKey {            // argmax key: (magnitude bits + 1, ~index)
  uint64_t hi;
  uint32_t lo;
  uint32_t pad;
};

template <typename T>
struct Ctx {
  hipStream_t stream;
  Plan plan;
  const int8_t* signs;     // natural order
  const int32_t* rows;
  int kmax;                // largest support handled by the compact buffers
  // dense N-vectors (v-order unless noted)
  Cx<T>* W;                // transform work buffer (L complex)
  T* Dd;                   // CG direction, dense
  T* Dx;                   // current solution, dense
  T* C0;                   // A^T y (raw, unsigned by the sign flip), dense
  T* Yf;                   // y in freq-layout (N reals)
  // twiddles and mask
  Cx<T>* tw_col; Cx<T>* tw_row;   // stage twiddles of the L1- and L2-point FFTs
  Cx<T>* tw_lo; Cx<T>* tw_hi;
  uint32_t* mask;
  // bitmaps over natural indices (N bits each)
  uint32_t* bits[3];
  // compact buffers (kmax each)
  int32_t* list[3];
  T *cb, *cx, *cr, *cd, *cq, *cx2, *cx3;
  // reductions
  double* partial;         // >= 2 * kRedBlocks doubles
  double* partial2;
  ArgKey* argpart;         // kArgBlocks
  int32_t* ibuf;           // small int scratch (>= 64)
  uint32_t* blockcnt;      // bitmap compaction block counts
  CgScalars* cg;
  SelState* sel;
  double ynorm = 0;        // ||y||, FP64 accumulation
  // host-side counters
  int64_t transforms = 0;
  int64_t cg_iters = 0;
  double model_bytes = 0;
  int32_t flags = 0;
};

constexpr int kRedBlocks = 256;   // blocks of the compact reductions
constexpr int kRedThreads = 256;
constexpr int kArgBlocks = 1024;
constexpr int kBitsPerBlockWords = 1024;  // words per block in bitmap compaction

// ------------------------------------------------------------------ profiling
enum ProfClass { PC_COL_FWD = 0, PC_COL_INV, PC_ROW_HAPPLY, PC_ROW_RESID, PC_ROW_FWD, PC_ROW_ADJ, PC_COUNT };
bool prof_on();
int prof_begin(hipStream_t s, hipEvent_t* ev);
void prof_end(int cls, double bytes, hipEvent_t start, hipStream_t s);
void prof_flush();

// ------------------------------------------------------------------ plan/workspace
bool choose_plan(cs_dtype dt, int64_t n, int64_t m, Plan& p);
size_t workspace_bytes(cs_dtype dt, int64_t n, int64_t m, int32_t k, cs_algo algo);

template <typename T>
void ctx_init(Ctx<T>& c, const cs_op* op, int kmax, void* ws, size_t ws_bytes, hipStream_t s);

// ------------------------------------------------------------------ transform launchers
enum RowMode { ROW_HAPPLY = 0, ROW_RESID = 1, ROW_FWD = 2, ROW_ADJ = 3 };

template <typename T> void setup_operator(Ctx<T>& c);                  // twiddles + mask (+ validation)
template <typename T> void scatter_freq(Ctx<T>& c, const T* u, T* outf); // u [M] -> freq layout
template <typename T> void gather_freq(Ctx<T>& c, const T* inf, T* out); // freq layout -> [M]
// dense v-order `in` -> W -> (row pass mode) -> W (v-order result unless FWD/ADJ)
template <typename T> void transform_happly(Ctx<T>& c, const T* in, const int* done);
template <typename T> void transform_resid(Ctx<T>& c, const T* in);      // W = A^T(y - A x), resid2 partials
template <typename T> void transform_fwd(Ctx<T>& c, const T* in, T* outf); // outf = masked DCT in freq layout
template <typename T> void perm_in(Ctx<T>& c, const T* x, T* dense);      // dense[vpos(j)] = sign_j x_j
template <typename T> void perm_out(Ctx<T>& c, const T* dense, T* x);     // x_j = sign_j dense[vpos(j)]
template <typename T> void prepare_kernels();                             // LDS limits, once per process
template <typename T> void transform_adj(Ctx<T>& c, const T* inf, T* out); // out = F^T (freq input), v-order
template <typename T> void fill(T* p, int64_t count, T v, hipStream_t s);
// Reads `bytes` (a multiple of 4, at most 4096) of device memory on the host:
// a one-block kernel copies them into a pinned, device-mapped host buffer
// (one per calling thread, kept for the life of the process), then the stream
// is synchronised.  Cheaper than a pageable device-to-host copy.
void dev_read(hipStream_t s, const void* dev, void* host, size_t bytes);
template <typename T> double norm2_host(Ctx<T>& c, const T* v, int64_t count);   // ||v||, synchronises
void fill_u32(uint32_t* p, int64_t count, uint32_t v, hipStream_t s);

// ------------------------------------------------------------------ compact <-> dense
template <typename T> void scatter_signed(Ctx<T>& c, T* dense, const int32_t* list, const T* vals, int k);
template <typename T> void scatter_zero(Ctx<T>& c, T* dense, const int32_t* list, int k);
template <typename T> void gather_signed(Ctx<T>& c, const T* dense, const int32_t* list, T* vals, int k);

// ------------------------------------------------------------------ selection
template <typename T> void argmax_excl(Ctx<T>& c, const T* dense, const uint32_t* excl, int32_t* out_j);
template <typename T> void topk_dense(Ctx<T>& c, const T* dense, const uint32_t* excl, int k, uint32_t* out_bits);
template <typename T> void topk_compact(Ctx<T>& c, const T* vals, const int32_t* list, int count, int k, uint32_t* out_bits);
template <typename T> int bits_to_list(Ctx<T>& c, const uint32_t* bits, int32_t* list, int expect);
void bits_or(const uint32_t* a, const uint32_t* b, uint32_t* out, int64_t words, hipStream_t s);
void bits_set_list(uint32_t* bits, const int32_t* list, int k, hipStream_t s);
int bits_equal(const uint32_t* a, const uint32_t* b, int64_t words, int32_t* scratch, hipStream_t s);

// ------------------------------------------------------------------ CG
template <typename T>
int cg_solve(Ctx<T>& c, const int32_t* list, int k, T* x, bool warm, double tol, int max_iter);

// residual + correlation for the solution (list, x): updates Dx, leaves
// c = raw A^T (y - A x) in W (v-order) and returns ||y - A x|| on the host.
template <typename T>
double resid_corr(Ctx<T>& c, const int32_t* old_list, int old_k, const int32_t* list, const T* x, int k);

// ------------------------------------------------------------------ drivers
template <typename T>
void run_omp(Ctx<T>& c, int k, double tol, const cs_params& prm, T* s_out, int32_t* supp_out, cs_info* info);
template <typename T>
void run_sp(Ctx<T>& c, int k, double tol, const cs_params& prm, T* s_out, int32_t* supp_out, cs_info* info);
template <typename T>
void run_ompr(Ctx<T>& c, int k, double tol, const cs_params& prm, T* s_out, int32_t* supp_out, cs_info* info);
template <typename T>
void write_output(Ctx<T>& c, const int32_t* list, const T* x, int k, T* s_out, int32_t* supp_out);

}  // namespace csr
