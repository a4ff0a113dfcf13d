// Transform subsystem: the operator A = D F R of Eq. (7) and the CG matrix
// H = W_S A^T A W_S of Eq. (11), evaluated with the FFT-based DCT that
// Sec. III-D calls for ("DCT can be speeded by FFT").
//
// DCT-II of length N through an N/2-point complex FFT (Makhoul's even/odd
// reordering): with v as in cs_internal.h and Z = FFT_{N/2}(z),
//   V_k = E_k + W_N^k O_k,  E_k = (Z_k + conj Z_{L-k})/2,  O_k = (Z_k - conj Z_{L-k})/(2i)
//   X_k = c_k Re(e^{-i pi k/(2N)} V_k),  X_{N-k} = -c_k Im(e^{-i pi k/(2N)} V_k).
// The DCT-III (transpose) inverts each step.  Both directions meet in the
// row pass, so one H-apply is three passes over HBM:
//   column FFTs -> [row FFT, post-process, mask/residual, pre-process,
//   inverse row FFT] -> inverse column FFTs.
#include "cs_internal.h"
#include "cs_kernels.h"

#include <algorithm>
#include <atomic>
#include <chrono>
#include <mutex>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>

namespace csr {

void hip_check(hipError_t e, const char* what, const char* file, int line) {
  if (e != hipSuccess) {
    throw Error(CS_E_HIP, std::string(what) + " failed: " + hipGetErrorString(e) + " (" + file + ":" +
                              std::to_string(line) + ")");
  }
}

// ------------------------------------------------------------------ plan
namespace {
std::mutex g_shape_mu;
Shape g_shape_over[2][kMaxL + 1];   // [FP64][log2 L]; logL1 == 0: no override
}  // namespace

static bool same_shape(const Shape& a, const Shape& b) {
  return a.logL1 == b.logL1 && a.logL2 == b.logL2 && a.logB == b.logB && a.logE == b.logE;
}

static bool shape_compiled(cs_dtype dt, const Shape& s) {
  if (s.logL1 + s.logL2 < kMinL || s.logL1 + s.logL2 > kMaxL) return false;
  if (same_shape(s, shape_for(dt == CS_F64, s.logL1 + s.logL2))) return true;
  return (dt == CS_F32) ? kernels_alt<float>(s) != nullptr : kernels_alt<double>(s) != nullptr;
}

int shape_candidates(cs_dtype dt, int l, Shape* out, int max) {
  if (max < 1 || l < kMinL || l > kMaxL) return 0;
  out[0] = shape_for(dt == CS_F64, l);
  int cnt = max - 1;
  const Shape probe{l / 2, l - l / 2, 0, 0};
  if (dt == CS_F32) kernels_alt<float>(probe, out + 1, &cnt);
  else kernels_alt<double>(probe, out + 1, &cnt);
  return 1 + cnt;
}

bool set_shape_override(cs_dtype dt, int l, const Shape* s) {
  if (l < kMinL || l > kMaxL) return false;
  if (s && (s->logL1 + s->logL2 != l || !shape_compiled(dt, *s))) return false;
  std::lock_guard<std::mutex> g(g_shape_mu);
  g_shape_over[dt == CS_F64][l] = s ? *s : Shape{0, 0, 0, 0};
  return true;
}

bool choose_plan(cs_dtype dt, int64_t n, int64_t m, Plan& p, const Shape* force) {
  if (n < 16 || n > (int64_t(1) << 26) || (n & (n - 1))) return false;
  p = Plan{};
  p.n = n;
  p.m = m;
  p.words = (n + 31) / 32;
  p.logn = 0;
  while ((int64_t(1) << p.logn) < n) ++p.logn;
  p.L = n / 2;
  p.logL = p.logn - 1;
  const Shape def = shape_for(dt == CS_F64, p.logL);
  Shape sh = def;
  {
    // process-wide choice (the autotuner's), else the default
    std::lock_guard<std::mutex> g(g_shape_mu);
    const Shape& o = g_shape_over[dt == CS_F64][p.logL];
    if (o.logL1 != 0) sh = o;
  }
  if (force) {
    if (force->logL1 + force->logL2 != p.logL || !shape_compiled(dt, *force)) return false;
    sh = *force;
  }
  if (!same_shape(sh, def)) p.alt = 1;
  // Tuning override "logL1,logL2,logB,logE" (must multiply to this L and be instantiated).
  if (const char* ov = std::getenv("CS_SHAPE")) {
    Shape o{0, 0, 0, 0};
    if (!force && std::sscanf(ov, "%d,%d,%d,%d", &o.logL1, &o.logL2, &o.logB, &o.logE) == 4 &&
        o.logL1 + o.logL2 == p.logL && !same_shape(o, def)) {
      const bool ok = (dt == CS_F32) ? kernels_alt<float>(o) != nullptr : kernels_alt<double>(o) != nullptr;
      if (ok) { sh = o; p.alt = 1; }
    }
  }
  p.logL1 = sh.logL1;
  p.logL2 = sh.logL2;
  p.logB = sh.logB;
  p.logE = sh.logE;
  p.L1 = 1 << p.logL1;
  p.L2 = 1 << p.logL2;
  p.B = 1 << p.logB;
  const size_t cs = (dt == CS_F32) ? 8 : 16;
  const int ecol = p.B * p.L1, erow = 2 * p.L2;
  p.nt_col = nt_for(ecol, p.logE);
  p.nt_row = nt_for(erow, p.logE);
  p.lds_col = cs * lp_size(ecol);
  p.lds_row = cs * lp_size(erow);
  return true;
}

// ------------------------------------------------------------------ setup kernels
// W_{n}^k for k in [0, count) with W = exp(-2 pi i k / n), in FP64 then rounded.
template <typename T>
__global__ void k_twiddle(Cx<T>* out, int64_t count, int64_t n, int64_t step) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= count) return;
  // angle = 2 pi (i*step mod n) / n, reduced exactly in integers
  int64_t a = (i * step) % n;
  double sv, cv;
  sincospi(2.0 * (double)a / (double)n, &sv, &cv);
  out[i] = cx<T>((T)cv, (T)(-sv));
}

// The freq-layout mask of D straight from the sampled rows: row q sets bit
// fpos(q) (slot f = (k mod L1) L2 + k / L1, half h: DCT output k or N - k, or
// L for k = 0); the mask starts clear.  Flags rows out of range or not
// strictly ascending.
__global__ void k_mask_from_rows(const int32_t* __restrict__ rows, int64_t m, const Plan p,
                                 uint32_t* __restrict__ mask, int32_t* bad) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= m) return;
  const int64_t q = rows[i];
  const bool ok = (q >= 0 && q < p.n) && (i == 0 || rows[i - 1] < q);
  if (!ok) {
    atomicOr(bad, 1);
    return;
  }
  const int64_t b = fpos(q, p);
  atomicOr(&mask[b >> 5], 1u << (b & 31));
}

// The mask in two passes for shapes with L1 a multiple of 32 and L2 of 64.
// First the natural-order bitmap of the rows (cleared beforehand): thread i
// checks row i (in range, above row i-1) and the rows of a wave, ascending,
// OR their bits per word with a segmented shuffle scan, so each word takes one
// atomic per wave.
__global__ void k_rows_bitmap(const int32_t* __restrict__ rows, int64_t m, int64_t n, uint32_t* __restrict__ nb,
                              int32_t* bad) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int lane = threadIdx.x & 63;
  uint32_t w = 0xFFFFFFFFu, v = 0u;
  if (i < m) {
    const int64_t q = rows[i];
    if ((q >= 0 && q < n) && (i == 0 || rows[i - 1] < q)) {
      w = (uint32_t)(q >> 5);
      v = 1u << (q & 31);
    } else {
      atomicOr(bad, 1);
    }
  }
  for (int off = 1; off < 64; off <<= 1) {
    const uint32_t w2 = __shfl_up(w, off, 64), v2 = __shfl_up(v, off, 64);
    if (lane >= off && w2 == w) v |= v2;
  }
  const uint32_t wn = __shfl_down(w, 1, 64);
  if (w != 0xFFFFFFFFu && (lane == 63 || wn != w)) atomicOr(&nb[w], v);
}

__device__ __forceinline__ uint32_t spread16(uint32_t x) {   // bit i -> bit 2i
  x &= 0xFFFFu;
  x = (x | (x << 8)) & 0x00FF00FFu;
  x = (x | (x << 4)) & 0x0F0F0F0Fu;
  x = (x | (x << 2)) & 0x33333333u;
  x = (x | (x << 1)) & 0x55555555u;
  return x;
}

// Then the transpose into the freq layout: slot f = a L2 + b holds row
// k = b L1 + a (half 0) and row N - k (half 1; row L for k = 0).  One wave per
// tile of 32 a-values by 64 b-values: lane b holds the word of rows b L1 + a0 ..
// + 31 and the two words around N - b L1 - a0; one ballot per a and half gives
// 64 slots, interleaved into four mask words.
__global__ __launch_bounds__(64) void k_mask_transpose(const uint32_t* __restrict__ nb, const Plan p,
                                                       uint32_t* __restrict__ mask) {
  const int lane = threadIdx.x;
  const int64_t a0 = (int64_t)blockIdx.x * 32, b0 = (int64_t)blockIdx.y * 64, b = b0 + lane;
  const int64_t L1 = p.L1, L2 = p.L2, n = p.n;
  const uint32_t w0 = nb[(b * L1 + a0) >> 5];
  const int64_t hi = n - b * L1 - a0;               // the row of half 1 at a = a0 (n: the k = 0 case)
  const int64_t lo = hi - 31;
  const uint32_t wlo = nb[lo >> 5];
  const uint32_t whi = nb[(hi < n ? hi : n - 1) >> 5];
  const bool k0 = (b == 0 && a0 == 0);
  const uint32_t rowL = (nb[p.L >> 5] >> (p.L & 31)) & 1u;
  for (int a = 0; a < 32; ++a) {
    const bool h0 = (w0 >> a) & 1u;
    const int64_t r1 = hi - a;
    bool h1;
    if (k0 && a == 0) h1 = rowL != 0;
    else h1 = ((((r1 >> 5) == (lo >> 5)) ? wlo : whi) >> (r1 & 31)) & 1u;
    const uint64_t m0 = __ballot(h0), m1 = __ballot(h1);
    if (lane < 4) {
      const uint32_t x0 = (uint32_t)(m0 >> (16 * lane)), x1 = (uint32_t)(m1 >> (16 * lane));
      mask[(((a0 + a) * L2 + b0) >> 4) + lane] = spread16(x0) | (spread16(x1) << 1);
    }
  }
}

// Inverse of the randomizer's permutation; flags an entry out of range or a
// repeated one (pinv starts at -1).
__global__ void k_perm_inverse(const int32_t* __restrict__ perm, int64_t n, int32_t* __restrict__ pinv, int32_t* bad) {
  int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= n) return;
  const int32_t q = perm[j];
  if (q < 0 || q >= n) { atomicOr(bad, 4); return; }
  if (atomicCAS(&pinv[q], -1, (int32_t)j) != -1) atomicOr(bad, 4);
}

// Sixteen signs per thread (N is a multiple of 16; the array 16-byte aligned),
// or one per thread for an unaligned array.
__global__ void k_check_signs1(const int8_t* __restrict__ s, int64_t n, int32_t* bad) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const int8_t v = s[i];
  if (v != 1 && v != -1) atomicOr(bad, 2);
}
__global__ void k_check_signs(const int8_t* __restrict__ s, int64_t n, int32_t* bad) {
  const int64_t i = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) * 16;
  if (i >= n) return;
  const uint4 w = *reinterpret_cast<const uint4*>(s + i);
  const uint32_t v[4] = {w.x, w.y, w.z, w.w};
  bool okall = true;
#pragma unroll
  for (int j = 0; j < 4; ++j)
#pragma unroll
    for (int b = 0; b < 4; ++b) {
      const uint32_t c = (v[j] >> (8 * b)) & 0xFFu;   // +1 = 0x01, -1 = 0xFF
      okall &= (c == 0x01u || c == 0xFFu);
    }
  if (!okall) atomicOr(bad, 2);
}

template <typename T>
__global__ void k_fill(T* __restrict__ p, int64_t count, T v) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  int64_t st = (int64_t)gridDim.x * blockDim.x;
  for (; i < count; i += st) p[i] = v;
}

template <typename T>
void fill(T* p, int64_t count, T v, hipStream_t s) {
  if (count <= 0) return;
  int64_t blocks = std::min<int64_t>((count + 255) / 256, 4096);
  hipLaunchKernelGGL(k_fill<T>, dim3((unsigned)blocks), dim3(256), 0, s, p, count, v);
  CS_LAUNCH_CHECK();
}
void fill_u32(uint32_t* p, int64_t count, uint32_t v, hipStream_t s) { fill<uint32_t>(p, count, v, s); }

static inline unsigned nblk(int64_t n, int t) { return (unsigned)std::max<int64_t>(1, (n + t - 1) / t); }

// Partial complex Fourier sensing (cs_op.xform = 2).  For a real signal the
// unitary DFT coefficient k in (0, N/2) is (row k - i row N-k) / sqrt 2 of the
// orthonormal real Fourier basis, so the complex operator is the real one on
// the rows k and N - k with the data paired by cplx_in / cplx_out; the rows
// are [k_0 .. k_{M-1}, N - k_{M-1} .. N - k_0] (ascending when the k are).
__global__ void k_expand_rows(const int32_t* __restrict__ freq, int64_t m, int64_t n, int32_t* __restrict__ rows) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= m) return;
  const int32_t k = freq[i];
  rows[i] = k;
  rows[2 * m - 1 - i] = (int32_t)(n - k);
}

template <typename T>
void setup_operator(Ctx<T>& c) {
  const Plan& p = c.plan;
  hipStream_t s = c.stream;
  if (c.cplx) {   // the rows (validated with the mask below) from the sampled frequencies
    hipLaunchKernelGGL(k_expand_rows, dim3(nblk(p.m / 2, 256)), dim3(256), 0, s, c.freq, p.m / 2, p.n, c.rows_x);
    CS_LAUNCH_CHECK();
  }
  hipLaunchKernelGGL(k_stage_twiddles<T>, dim3(nblk(tw_table_count(p.logL1, p.logE), 256)), dim3(256), 0, s,
                     c.tw_col, p.logL1, p.logE);
  CS_LAUNCH_CHECK();
  hipLaunchKernelGGL(k_stage_twiddles<T>, dim3(nblk(tw_table_count(p.logL2, p.logE), 256)), dim3(256), 0, s,
                     c.tw_row, p.logL2, p.logE);
  CS_LAUNCH_CHECK();
  const int64_t n4 = 4 * p.n;
  hipLaunchKernelGGL(k_twiddle<T>, dim3(nblk(kTwLo, 256)), dim3(256), 0, s, c.tw_lo, (int64_t)kTwLo, n4,
                     (int64_t)1);
  CS_LAUNCH_CHECK();
  const int64_t nhi = std::max<int64_t>(1, n4 / kTwLo);
  hipLaunchKernelGGL(k_twiddle<T>, dim3(nblk(nhi, 256)), dim3(256), 0, s, c.tw_hi, nhi, n4, (int64_t)kTwLo);
  CS_LAUNCH_CHECK();
  const int64_t st = (int64_t)p.L1 * p.nt_row;   // the row pass's item stride in bins
  hipLaunchKernelGGL(k_twiddle<T>, dim3(1), dim3(kTwStepHalf), 0, s, c.tw_step, (int64_t)kTwStepHalf, n4, st);
  CS_LAUNCH_CHECK();
  hipLaunchKernelGGL(k_twiddle<T>, dim3(1), dim3(kTwStepHalf), 0, s, c.tw_step + kTwStepHalf, (int64_t)kTwStepHalf,
                     n4, 4 * st);
  CS_LAUNCH_CHECK();
  fill<int32_t>(c.ibuf, 1, 0, s);
  if (p.L1 % 32 == 0 && p.L2 % 64 == 0) {
    // natural row bitmap in nbits (free until the output), then the transpose
    fill_u32(c.nbits, p.words, 0u, s);
    hipLaunchKernelGGL(k_rows_bitmap, dim3(nblk(p.m, 256)), dim3(256), 0, s, c.rows, p.m, p.n, c.nbits, c.ibuf);
    CS_LAUNCH_CHECK();
    hipLaunchKernelGGL(k_mask_transpose, dim3((unsigned)(p.L1 / 32), (unsigned)(p.L2 / 64)), dim3(64), 0, s,
                       (const uint32_t*)c.nbits, p, c.mask);
    CS_LAUNCH_CHECK();
  } else {
    fill_u32(c.mask, p.words, 0u, s);
    hipLaunchKernelGGL(k_mask_from_rows, dim3(nblk(p.m, 256)), dim3(256), 0, s, c.rows, p.m, p, c.mask, c.ibuf);
    CS_LAUNCH_CHECK();
  }
  if (((uintptr_t)c.rsigns & 15u) == 0)
    hipLaunchKernelGGL(k_check_signs, dim3(nblk((p.n + 15) / 16, 256)), dim3(256), 0, s, c.rsigns, p.n, c.ibuf);
  else hipLaunchKernelGGL(k_check_signs1, dim3(nblk(p.n, 256)), dim3(256), 0, s, c.rsigns, p.n, c.ibuf);
  CS_LAUNCH_CHECK();
  if (c.psi == 2) dct2d_setup<T>(c);
  if (c.rperm) {
    fill<int32_t>(c.pinv, p.n, -1, s);
    hipLaunchKernelGGL(k_perm_inverse, dim3(nblk(p.n, 256)), dim3(256), 0, s, c.rperm, p.n, c.pinv, c.ibuf);
    CS_LAUNCH_CHECK();
  }
  int32_t bad = 0;
  dev_read(s, c.ibuf, &bad, sizeof(int32_t));
  if (bad & 1)
    throw Error(CS_E_OP, c.cplx ? "operator frequencies must be strictly ascending in [1, N/2)"
                                : "operator rows must be strictly ascending in [0, N)");
  if (bad & 2) throw Error(CS_E_OP, "operator signs must be +1 or -1");
  if (bad & 4) throw Error(CS_E_OP, "operator perm must be a permutation of [0, N)");
}

// ------------------------------------------------------------------ host reads
// A pinned, coherent host mailbox per host thread: word 0 is a sequence
// number, the payload follows from word 2.  k_post copies the payload, makes
// it visible system-wide, then publishes the sequence number; the host spins
// on that word instead of waiting for the stream (a stream wait adds the
// runtime's completion signalling to every read of the greedy and CG loops).
// A read that does not arrive within a bound falls back to a stream wait,
// which also reports any error of the queued work.  The mailbox has slots of
// kSlotWords: slot 0 for the reads that wait at once, the others for reads
// posted ahead of more queued work and collected later (dev_post / dev_wait).
constexpr int kBoxWords = 1024;
constexpr int kBoxHead = 2;
constexpr int kBoxSlots = 4;
constexpr int kSlotWords = kBoxWords / kBoxSlots;

__global__ void k_post(const uint32_t* __restrict__ src, uint32_t* __restrict__ box, int words, uint32_t seq) {
  for (int i = threadIdx.x; i < words; i += blockDim.x) box[kBoxHead + i] = src[i];
  __threadfence_system();
  __syncthreads();
  if (threadIdx.x == 0) __hip_atomic_store(box, seq, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_SYSTEM);
}

namespace {
struct HostBox {
  uint32_t* h = nullptr;
  uint32_t* d = nullptr;
  uint32_t seq = 0;
};
thread_local HostBox g_box;
}  // namespace

// The residual read: sums the row pass's partials of ||y - A x||^2 (fixed
// order), stores the sum at `r2` on the device, and posts {r2, *flag} to the
// mailbox in the same launch.
__global__ void k_post_resid(const double* __restrict__ partial, int np, double* __restrict__ r2,
                             const int32_t* __restrict__ flag, uint32_t* __restrict__ box, uint32_t seq) {
  __shared__ double red[16];
  double s = 0.0;
  for (int i = threadIdx.x; i < np; i += blockDim.x) s += partial[i];
  for (int off = 32; off > 0; off >>= 1) s += __shfl_down(s, off, 64);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = s;
  __syncthreads();
  if (threadIdx.x == 0) {
    double t = 0.0;
    for (int i = 0; i < (int)(blockDim.x >> 6); ++i) t += red[i];
    *r2 = t;
    const uint64_t bits = (uint64_t)__double_as_longlong(t);
    if (box) {
      box[kBoxHead] = (uint32_t)bits;
      box[kBoxHead + 1] = (uint32_t)(bits >> 32);
    }
    if (box) {   // null: the caller copies r2 and the flag itself
      box[kBoxHead + 2] = (uint32_t)*flag;
      __threadfence_system();
      __hip_atomic_store(box, seq, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_SYSTEM);
    }
  }
}

namespace {
void box_init() {
  if (!g_box.h) {
    void* h = nullptr;
    CS_HIP(hipHostMalloc(&h, 4 * kBoxWords, hipHostMallocMapped | hipHostMallocCoherent));
    void* d = nullptr;
    CS_HIP(hipHostGetDevicePointer(&d, h, 0));
    g_box.h = (uint32_t*)h;
    g_box.d = (uint32_t*)d;
    __atomic_store_n(g_box.h, 0u, __ATOMIC_RELEASE);
  }
}
uint32_t box_next() { return ++g_box.seq == 0 ? ++g_box.seq : g_box.seq; }   // never 0 (the initial word)
// spin until the sequence word of `slot` shows `want` (bounded; then a stream
// wait, which also reports any error of the queued work), and copy the payload out
void box_wait(hipStream_t s, int slot, uint32_t want, void* host, size_t bytes) {
  const uint32_t* w = g_box.h + slot * kSlotWords;
  bool arrived = false;
  const auto t0 = std::chrono::steady_clock::now();
  for (uint32_t spin = 0;; ++spin) {
    if (__atomic_load_n(w, __ATOMIC_ACQUIRE) == want) {
      arrived = true;
      break;
    }
    if ((spin & 1023u) == 1023u && std::chrono::steady_clock::now() - t0 > std::chrono::milliseconds(20)) break;
  }
  if (!arrived) {
    CS_HIP(hipStreamSynchronize(s));
    if (__atomic_load_n(w, __ATOMIC_ACQUIRE) != want) throw Error(CS_E_HIP, "device read did not arrive");
  }
  std::memcpy(host, w + kBoxHead, bytes);
}
}  // namespace

namespace {
thread_local int g_no_alloc = 0;
}  // namespace

bool no_alloc_mode() { return g_no_alloc != 0; }
NoAllocScope::NoAllocScope() { ++g_no_alloc; }
NoAllocScope::~NoAllocScope() { --g_no_alloc; }

void dev_read_resid(hipStream_t s, const double* partial, int np, double* r2, const int32_t* flag, double* r2_host,
                    int32_t* flag_host) {
  if (no_alloc_mode()) {
    hipLaunchKernelGGL(k_post_resid, dim3(1), dim3(1024), 0, s, partial, np, r2, flag, nullptr, 0u);
    CS_LAUNCH_CHECK();
    CS_HIP(hipMemcpyAsync(r2_host, r2, sizeof(double), hipMemcpyDeviceToHost, s));
    CS_HIP(hipMemcpyAsync(flag_host, flag, sizeof(int32_t), hipMemcpyDeviceToHost, s));
    CS_HIP(hipStreamSynchronize(s));
    return;
  }
  box_init();
  const uint32_t want = box_next();
  hipLaunchKernelGGL(k_post_resid, dim3(1), dim3(1024), 0, s, partial, np, r2, flag, g_box.d, want);
  CS_LAUNCH_CHECK();
  struct { double r2; int32_t flag, pad; } h{};
  box_wait(s, 0, want, &h, sizeof(h));
  *r2_host = h.r2;
  *flag_host = h.flag;
}

void dev_sum_resid(hipStream_t s, const double* partial, int np, double* r2) {
  hipLaunchKernelGGL(k_post_resid, dim3(1), dim3(1024), 0, s, partial, np, r2, nullptr, nullptr, 0u);
  CS_LAUNCH_CHECK();
}

void dev_read(hipStream_t s, const void* dev, void* host, size_t bytes) {
  if (bytes % 4 || bytes > 4 * (kSlotWords - kBoxHead)) throw Error(CS_E_INVALID, "dev_read size");
  if (no_alloc_mode()) {
    CS_HIP(hipMemcpyAsync(host, dev, bytes, hipMemcpyDeviceToHost, s));
    CS_HIP(hipStreamSynchronize(s));
    return;
  }
  box_init();
  const uint32_t want = box_next();
  hipLaunchKernelGGL(k_post, dim3(1), dim3(64), 0, s, (const uint32_t*)dev, g_box.d, (int)(bytes / 4), want);
  CS_LAUNCH_CHECK();
  box_wait(s, 0, want, host, bytes);
}

uint32_t dev_post(hipStream_t s, const void* dev, size_t bytes, int slot) {
  if (bytes % 4 || bytes > 4 * (kSlotWords - kBoxHead) || slot < 1 || slot >= kBoxSlots || no_alloc_mode())
    throw Error(CS_E_INVALID, "dev_post");
  box_init();
  const uint32_t want = box_next();
  hipLaunchKernelGGL(k_post, dim3(1), dim3(64), 0, s, (const uint32_t*)dev, g_box.d + slot * kSlotWords,
                     (int)(bytes / 4), want);
  CS_LAUNCH_CHECK();
  return want;
}

void dev_wait(hipStream_t s, int slot, uint32_t seq, void* host, size_t bytes) {
  if (bytes % 4 || bytes > 4 * (kSlotWords - kBoxHead) || slot < 1 || slot >= kBoxSlots)
    throw Error(CS_E_INVALID, "dev_wait");
  box_wait(s, slot, seq, host, bytes);
}

// ------------------------------------------------------------------ freq-layout scatter / gather
template <typename T>
__global__ void k_scatter_freq(const T* __restrict__ u, const int32_t* __restrict__ rows, int64_t m,
                               T* __restrict__ outf, Plan p) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= m) return;
  outf[fpos(rows[i], p)] = u[i];
}
template <typename T>
__global__ void k_gather_freq(const T* __restrict__ inf, const int32_t* __restrict__ rows, int64_t m,
                              T* __restrict__ out, Plan p) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= m) return;
  out[i] = inf[fpos(rows[i], p)];
}

// ---- partial complex Fourier (cs_op.xform = 2): the data pairing of the
// rows k and N - k (k_expand_rows above)
template <typename T>
__global__ void k_cplx_in(const T* __restrict__ u, int64_t m, T a, T b, T* __restrict__ out) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= m) return;
  out[i] = a * u[2 * i];
  out[2 * m - 1 - i] = b * u[2 * i + 1];
}
template <typename T>
__global__ void k_cplx_out(const T* __restrict__ r, int64_t m, T a, T b, T* __restrict__ out) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= m) return;
  out[2 * i] = a * r[i];
  out[2 * i + 1] = b * r[2 * m - 1 - i];
}
template <typename T>
void cplx_in(Ctx<T>& c, const T* u, double a, double b) {
  const int64_t m = c.plan.m / 2;
  hipLaunchKernelGGL(k_cplx_in<T>, dim3(nblk(m, 256)), dim3(256), 0, c.stream, u, m, (T)a, (T)b, c.ybuf);
  CS_LAUNCH_CHECK();
}
template <typename T>
void cplx_out(Ctx<T>& c, T* out, double a, double b) {
  const int64_t m = c.plan.m / 2;
  hipLaunchKernelGGL(k_cplx_out<T>, dim3(nblk(m, 256)), dim3(256), 0, c.stream, (const T*)c.ybuf, m, (T)a, (T)b, out);
  CS_LAUNCH_CHECK();
}

template <typename T>
void scatter_freq(Ctx<T>& c, const T* u, T* outf) {
  fill<T>(outf, c.plan.n, (T)0, c.stream);
  hipLaunchKernelGGL(k_scatter_freq<T>, dim3(nblk(c.plan.m, 256)), dim3(256), 0, c.stream, u, c.rows,
                     c.plan.m, outf, c.plan);
  CS_LAUNCH_CHECK();
}
template <typename T>
void gather_freq(Ctx<T>& c, const T* inf, T* out) {
  hipLaunchKernelGGL(k_gather_freq<T>, dim3(nblk(c.plan.m, 256)), dim3(256), 0, c.stream, inf, c.rows,
                     c.plan.m, out, c.plan);
  CS_LAUNCH_CHECK();
}

// ------------------------------------------------------------------ reductions
__global__ void k_sum_partials(const double* __restrict__ partial, int np, double* __restrict__ out) {
  __shared__ double red[16];
  double s = 0.0;
  for (int i = threadIdx.x; i < np; i += blockDim.x) s += partial[i];
  for (int off = 32; off > 0; off >>= 1) s += __shfl_down(s, off, 64);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = s;
  __syncthreads();
  if (threadIdx.x == 0) {
    double t = 0.0;
    for (int i = 0; i < (int)(blockDim.x >> 6); ++i) t += red[i];
    *out = t;
  }
}

template <typename T>
__global__ void k_sumsq_partial(const T* __restrict__ v, int64_t count, double* __restrict__ partial) {
  __shared__ double red[4];
  double s = 0.0;
  const int64_t st = (int64_t)gridDim.x * blockDim.x;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < count; i += st) {
    const double x = (double)v[i];
    s += x * x;
  }
  for (int off = 32; off > 0; off >>= 1) s += __shfl_down(s, off, 64);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = s;
  __syncthreads();
  if (threadIdx.x == 0) partial[blockIdx.x] = red[0] + red[1] + red[2] + red[3];
}

void sum_partials_to(const double* partial, int np, double* out, hipStream_t s) {
  hipLaunchKernelGGL(k_sum_partials, dim3(1), dim3(1024), 0, s, partial, np, out);
  CS_LAUNCH_CHECK();
}

template <typename T>
double norm2_host(Ctx<T>& c, const T* v, int64_t count) {
  const unsigned grid = (unsigned)std::min<int64_t>(kRedBlocks, nblk(count, 256));
  hipLaunchKernelGGL(k_sumsq_partial<T>, dim3(grid), dim3(256), 0, c.stream, v, count, c.partial2);
  CS_LAUNCH_CHECK();
  hipLaunchKernelGGL(k_sum_partials, dim3(1), dim3(1024), 0, c.stream, c.partial2, (int)grid, &c.cg->resid2);
  CS_LAUNCH_CHECK();
  double r2 = 0.0;
  dev_read(c.stream, &c.cg->resid2, &r2, sizeof(double));
  return std::sqrt(r2);
}

// Loads y: freq-layout copy, ||y||, and F^T D^T y (key order) into C0.
template <typename T>
void load_measurements(Ctx<T>& c, const T* y) {
  scatter_freq<T>(c, y, c.Yf);
  c.ynorm = norm2_host<T>(c, y, c.plan.m);
  if (!c.psi) {
    transform_adj<T>(c, c.Yf, c.C0, true);
    return;
  }
  if (c.psi == 2) {
    psi2_adjoint<T>(c, c.Yf, c.C0);
    return;
  }
  // A^T y = F^T R^T F^T D^T y: Phi^T into v-order, R^T, then Psi^T into key order
  transform_adj<T>(c, c.Yf, c.P2, false);
  rand_out<T>(c, c.P2, c.P1, nullptr);
  transform_adj<T>(c, c.P1, c.C0, true);
}

// ------------------------------------------------------------------ launchers
template <typename T>
ColIO<T> col_io(Ctx<T>& c, int mode, const Supp* S) {
  ColIO<T> io{};
  io.mode = mode;
  if (S) {
    io.sbits = S->bits;
    io.wpre = S->wpre;
    io.list = S->list;
    io.kcap = S->k;
  }
  return io;
}

template <typename T>
double launch_col(Ctx<T>& c, const Cx<T>* in, Cx<T>* out, bool inv, const ColIO<T>& io, int* rec) {
  const Plan& p = c.plan;
  const KernelSet<T>& ks = kernels_plan<T>(p);
  const unsigned grid = (unsigned)(p.L2 >> p.logB);
  // A dense pass reads and writes one N-vector.  A compact side replaces one
  // of them by the k support keys and the compact vectors it moves: x read
  // (COL_X); r, d read and d written (COL_DIR); d read and q written (COL_Q);
  // b read, r and d written (COL_R).  With the CG update fused, COL_DIR also
  // reads x and q and writes x and r, and COL_Q also reads r.
  double bytes = 2.0 * (double)p.n * sizeof(T);
  if (io.mode != COL_DENSE && io.mode != COL_KEY) {
    static const int vec[6] = {0, 1, 3, 2, 3, 0};
    const int nv = io.fused ? (io.mode == COL_DIR ? 7 : (io.mode == COL_Q ? 3 : vec[io.mode])) : vec[io.mode];
    bytes = (double)p.n * sizeof(T) + (double)io.kcap * (4.0 + nv * (double)sizeof(T));
  }
  hipEvent_t ev = nullptr;
  const bool prof = prof_on();
  if (prof) prof_begin(c.stream, &ev);
  auto fn = inv ? ks.col_inv : ks.col_fwd;
  fn<<<dim3(grid), dim3(ks.nt_col), p.lds_col, c.stream>>>(in, out, p, io, c.tw_col);
  CS_LAUNCH_CHECK();
  const int r = prof ? prof_end(inv ? PC_COL_INV : PC_COL_FWD, bytes, ev, c.stream) : -1;
  if (rec) *rec = r;
  c.model_bytes += bytes;
  return bytes;
}

template <typename T>
double launch_row(Ctx<T>& c, int mode, const T* fin, T* fout, double* partial, const int* done, int* rec) {
  const Plan& p = c.plan;
  const KernelSet<T>& ks = kernels_plan<T>(p);
  const unsigned grid = (unsigned)(p.L1 >> 1);
  // read and write one N-vector; the residual pass also reads y (N reals in freq layout)
  double bytes = 2.0 * (double)p.n * sizeof(T);
  if (mode == ROW_RESID) bytes += (double)p.n * sizeof(T);
  hipEvent_t ev = nullptr;
  const bool prof = prof_on();
  if (prof) prof_begin(c.stream, &ev);
  ks.row<<<dim3(grid), dim3(ks.nt_row), p.lds_row, c.stream>>>(c.W, p, mode, fin, fout, partial, done, c.tw_row);
  CS_LAUNCH_CHECK();
  const int cls = mode == ROW_FWD_ALL ? PC_ROW_FWD : PC_ROW_HAPPLY + mode;
  const int r = prof ? prof_end(cls, bytes, ev, c.stream) : -1;
  if (rec) *rec = r;
  c.model_bytes += bytes;
  return bytes;
}

template <typename T>
void transform_fwd(Ctx<T>& c, const T* in, T* outf, bool all) {
  launch_col<T>(c, (const Cx<T>*)in, c.W, false, col_io<T>(c, COL_DENSE, nullptr));
  launch_row<T>(c, all ? ROW_FWD_ALL : ROW_FWD, nullptr, outf, nullptr, nullptr);
  c.transforms += 1;
}

template <typename T>
void transform_adj(Ctx<T>& c, const T* inf, T* out, bool key_order) {
  launch_row<T>(c, ROW_ADJ, inf, nullptr, nullptr, nullptr);
  launch_col<T>(c, c.W, (Cx<T>*)out, true, col_io<T>(c, key_order ? COL_KEY : COL_DENSE, nullptr));
  c.transforms += 1;
}

template <typename T>
__global__ void k_perm_in(const T* __restrict__ x, T* __restrict__ dense, const int8_t* __restrict__ signs,
                          const Plan pl) {
  int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= pl.n) return;
  const int64_t q = pl.perm ? (int64_t)pl.perm[j] : j;
  dense[xpos(q, pl)] = (signs && signs[j] < 0) ? -x[j] : x[j];
}
template <typename T>
__global__ void k_perm_out(const T* __restrict__ dense, T* __restrict__ x, const int8_t* __restrict__ signs,
                           const Plan pl) {
  int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= pl.n) return;
  const int64_t q = pl.perm ? (int64_t)pl.perm[j] : j;
  const T v = dense[xpos(q, pl)];
  x[j] = (signs && signs[j] < 0) ? -v : v;
}
template <typename T>
void perm_in(Ctx<T>& c, const T* x, T* dense) {
  hipLaunchKernelGGL(k_perm_in<T>, dim3(nblk(c.plan.n, 256)), dim3(256), 0, c.stream, x, dense, c.signs, c.plan);
  CS_LAUNCH_CHECK();
}
template <typename T>
void perm_out(Ctx<T>& c, const T* dense, T* x) {
  hipLaunchKernelGGL(k_perm_out<T>, dim3(nblk(c.plan.n, 256)), dim3(256), 0, c.stream, dense, x, c.signs, c.plan);
  CS_LAUNCH_CHECK();
}

// ------------------------------------------------------------------ DCT sparsifying basis
// With Psi = F the signal is x = F s: index i of x is output i of Psi's DCT
// (freq-layout float fpos(i)) and enters Phi's DCT at input perm[i] with sign
// signs[i] (v-order position vpos(perm[i])).  Both reorders write their
// destination in order and gather the source.

// freq-layout float position -> DCT output index (inverse of fpos)
__device__ __forceinline__ int64_t fpos_inv(int64_t P, const Plan& p) {
  const int64_t f = P >> 1, h = P & 1;
  const int64_t k = (f & (p.L2 - 1)) * p.L1 + (f >> p.logL2);
  if (!h) return k;
  return k == 0 ? p.L : p.n - k;
}

// v-order Phi input t <- R (Psi output): DCT input q at t, x index i = pinv[q]
// nat = 1: the source holds x in natural order (the 2-D DCT basis) instead of
// Psi's freq layout.
template <typename T>
__global__ void k_rand_in(const T* __restrict__ fin, T* __restrict__ vout, const int8_t* __restrict__ signs,
                          const int32_t* __restrict__ pinv, const Plan pl, const int* __restrict__ done, int nat) {
  if (done && *done) return;
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= pl.n) return;
  const int64_t q = xinv(t, pl);
  const int64_t i = pinv ? (int64_t)pinv[q] : q;
  const T v = fin[nat ? i : fpos(i, pl)];
  vout[t] = signs[i] < 0 ? -v : v;
}

// freq-layout Psi^T input P <- R^T (Phi^T output): x index i = fpos_inv(P),
// read at v-order position vpos(perm[i])
template <typename T>
__global__ void k_rand_out(const T* __restrict__ vin, T* __restrict__ fout, const int8_t* __restrict__ signs,
                           const int32_t* __restrict__ perm, const Plan pl, const int* __restrict__ done, int nat) {
  if (done && *done) return;
  const int64_t P = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (P >= pl.n) return;
  const int64_t i = nat ? P : fpos_inv(P, pl);
  const int64_t q = perm ? (int64_t)perm[i] : i;
  const T v = vin[xpos(q, pl)];
  fout[P] = signs[i] < 0 ? -v : v;
}

template <typename T>
void rand_in(Ctx<T>& c, const T* fin, T* vout, const int* done) {
  hipLaunchKernelGGL(k_rand_in<T>, dim3(nblk(c.plan.n, 256)), dim3(256), 0, c.stream, fin, vout, c.rsigns, c.rpinv,
                     c.plan, done, 0);
  CS_LAUNCH_CHECK();
}
template <typename T>
void rand_in_nat(Ctx<T>& c, const T* xin, T* vout, const int* done) {
  hipLaunchKernelGGL(k_rand_in<T>, dim3(nblk(c.plan.n, 256)), dim3(256), 0, c.stream, xin, vout, c.rsigns, c.rpinv,
                     c.plan, done, 1);
  CS_LAUNCH_CHECK();
}
template <typename T>
void rand_out(Ctx<T>& c, const T* vin, T* fout, const int* done) {
  hipLaunchKernelGGL(k_rand_out<T>, dim3(nblk(c.plan.n, 256)), dim3(256), 0, c.stream, vin, fout, c.rsigns, c.rperm,
                     c.plan, done, 0);
  CS_LAUNCH_CHECK();
}
template <typename T>
void rand_out_nat(Ctx<T>& c, const T* vin, T* xout, const int* done) {
  hipLaunchKernelGGL(k_rand_out<T>, dim3(nblk(c.plan.n, 256)), dim3(256), 0, c.stream, vin, xout, c.rsigns, c.rperm,
                     c.plan, done, 1);
  CS_LAUNCH_CHECK();
}

// Between the two column passes of an H-apply on Psi's transform (W holds
// Psi's column stage): finish F s (row pass into P1), R into Phi's input,
// Phi^T Phi = three passes with the row mask, R^T, and Psi^T's row pass
// back into W.  `cg` (nullable) makes every launch exit once CG is done.
template <typename T>
double psi_middle(Ctx<T>& c, CgScalars* cg, int* rec) {
  const int* done = cg ? &cg->done : nullptr;
  ColIO<T> fwd = col_io<T>(c, COL_DENSE, nullptr), inv = col_io<T>(c, COL_DENSE, nullptr);
  fwd.cg = cg;
  inv.cg = cg;
  double bytes = 0.0;
  bytes += launch_row<T>(c, ROW_FWD_ALL, nullptr, c.P1, nullptr, done, rec ? &rec[0] : nullptr);
  rand_in<T>(c, c.P1, c.P2, done);
  bytes += launch_col<T>(c, (const Cx<T>*)c.P2, c.W, false, fwd, rec ? &rec[1] : nullptr);
  bytes += launch_row<T>(c, ROW_HAPPLY, nullptr, nullptr, nullptr, done, rec ? &rec[2] : nullptr);
  bytes += launch_col<T>(c, c.W, (Cx<T>*)c.P2, true, inv, rec ? &rec[3] : nullptr);
  rand_out<T>(c, c.P2, c.P1, done);
  bytes += launch_row<T>(c, ROW_ADJ, c.P1, nullptr, nullptr, done, rec ? &rec[4] : nullptr);
  c.transforms += 2;
  return bytes;
}

// ---- separable 2-D DCT basis (psi = 2): the s-space image lives in natural
// order, so the 2-D transform runs as two row passes on either side of Phi.

// H-apply on the image in P3 (the support's values, zero elsewhere): x = F S F^T,
// R, Phi^T Phi with the row mask, R^T, and F^T X F into `sout` (an N-vector,
// natural order).  `cg` (nullable) makes every launch exit once CG is done.
template <typename T>
void psi2_happly(Ctx<T>& c, CgScalars* cg, T* sout) {
  const int* done = cg ? &cg->done : nullptr;
  ColIO<T> fwd = col_io<T>(c, COL_DENSE, nullptr), inv = col_io<T>(c, COL_DENSE, nullptr);
  fwd.cg = cg;
  inv.cg = cg;
  dct2d<T>(c, false, c.P3, c.P4, c.P1, done);
  rand_in_nat<T>(c, c.P1, c.P2, done);
  launch_col<T>(c, (const Cx<T>*)c.P2, c.W, false, fwd);
  launch_row<T>(c, ROW_HAPPLY, nullptr, nullptr, nullptr, done);
  launch_col<T>(c, c.W, (Cx<T>*)c.P2, true, inv);
  rand_out_nat<T>(c, c.P2, c.P1, done);
  dct2d<T>(c, true, c.P1, c.P4, sout, done);
  c.transforms += 4;
}

// Residual on the image in P3: r = y - A x masked (norm partials into
// partial2) and A^T r into `cout` (natural order).
template <typename T>
void psi2_resid(Ctx<T>& c, T* cout) {
  dct2d<T>(c, false, c.P3, c.P4, c.P1, nullptr);
  rand_in_nat<T>(c, c.P1, c.P2, nullptr);
  launch_col<T>(c, (const Cx<T>*)c.P2, c.W, false, col_io<T>(c, COL_DENSE, nullptr));
  launch_row<T>(c, ROW_RESID, c.Yf, nullptr, c.partial2, nullptr);
  launch_col<T>(c, c.W, (Cx<T>*)c.P2, true, col_io<T>(c, COL_DENSE, nullptr));
  rand_out_nat<T>(c, c.P2, c.P1, nullptr);
  dct2d<T>(c, true, c.P1, c.P4, cout, nullptr);
  c.transforms += 4;
}

// A s for an image `img` (natural order) into freq layout (masked).
template <typename T>
void psi2_forward(Ctx<T>& c, const T* img, T* outf) {
  dct2d<T>(c, false, img, c.P4, c.P1, nullptr);
  rand_in_nat<T>(c, c.P1, c.P2, nullptr);
  transform_fwd<T>(c, c.P2, outf);
  c.transforms += 1;
}

// A^T u for u in freq layout (zero off the rows) into `out` (natural order).
template <typename T>
void psi2_adjoint(Ctx<T>& c, const T* inf, T* out) {
  transform_adj<T>(c, inf, c.P2, false);
  rand_out_nat<T>(c, c.P2, c.P1, nullptr);
  dct2d<T>(c, true, c.P1, c.P4, out, nullptr);
  c.transforms += 1;
}

// y-side of the residual with a DCT basis: W holds Psi's column stage of x.
// Forms r = y - A x (masked, with its norm partials) and leaves Psi^T's row
// pass of A^T r in W for the inverse column pass.
template <typename T>
void psi_resid_middle(Ctx<T>& c) {
  launch_row<T>(c, ROW_FWD_ALL, nullptr, c.P1, nullptr, nullptr);
  rand_in<T>(c, c.P1, c.P2, nullptr);
  launch_col<T>(c, (const Cx<T>*)c.P2, c.W, false, col_io<T>(c, COL_DENSE, nullptr));
  launch_row<T>(c, ROW_RESID, c.Yf, nullptr, c.partial2, nullptr);
  launch_col<T>(c, c.W, (Cx<T>*)c.P2, true, col_io<T>(c, COL_DENSE, nullptr));
  rand_out<T>(c, c.P2, c.P1, nullptr);
  launch_row<T>(c, ROW_ADJ, c.P1, nullptr, nullptr, nullptr);
  c.transforms += 2;
}

template <typename T>
void prepare_kernels() {
  static std::atomic<int> ready{0};   // per instantiation; setting the attribute twice is harmless
  if (ready.load()) return;
  const int lim = 140 * 1024;          // largest padded dynamic LDS any shape asks for
  for (int l = kMinL; l <= kMaxL; ++l) {
    const KernelSet<T>& ks = kernels_for<T>(l);
    CS_HIP(hipFuncSetAttribute((const void*)ks.col_fwd, hipFuncAttributeMaxDynamicSharedMemorySize, lim));
    CS_HIP(hipFuncSetAttribute((const void*)ks.col_inv, hipFuncAttributeMaxDynamicSharedMemorySize, lim));
    CS_HIP(hipFuncSetAttribute((const void*)ks.row, hipFuncAttributeMaxDynamicSharedMemorySize, lim));
    CS_HIP(hipFuncSetAttribute((const void*)ks.col_fwd_b, hipFuncAttributeMaxDynamicSharedMemorySize, lim));
    CS_HIP(hipFuncSetAttribute((const void*)ks.col_inv_b, hipFuncAttributeMaxDynamicSharedMemorySize, lim));
    CS_HIP(hipFuncSetAttribute((const void*)ks.row_b, hipFuncAttributeMaxDynamicSharedMemorySize, lim));
  }
  for (int a = 1; a <= 14; ++a)
    for (int b = 1; b <= 13; ++b)
      for (int lb = 0; lb <= 4; ++lb)
        for (int le = 1; le <= 4; ++le)
        if (const KernelSet<T>* ks = kernels_alt<T>(Shape{a, b, lb, le})) {
          CS_HIP(hipFuncSetAttribute((const void*)ks->col_fwd, hipFuncAttributeMaxDynamicSharedMemorySize, lim));
          CS_HIP(hipFuncSetAttribute((const void*)ks->col_inv, hipFuncAttributeMaxDynamicSharedMemorySize, lim));
          CS_HIP(hipFuncSetAttribute((const void*)ks->row, hipFuncAttributeMaxDynamicSharedMemorySize, lim));
          CS_HIP(hipFuncSetAttribute((const void*)ks->col_fwd_b, hipFuncAttributeMaxDynamicSharedMemorySize, lim));
          CS_HIP(hipFuncSetAttribute((const void*)ks->col_inv_b, hipFuncAttributeMaxDynamicSharedMemorySize, lim));
          CS_HIP(hipFuncSetAttribute((const void*)ks->row_b, hipFuncAttributeMaxDynamicSharedMemorySize, lim));
        }
  ready.store(1);
}

// ------------------------------------------------------------------ instantiations
#define CS_INST(T)                                                                      \
  template void fill<T>(T*, int64_t, T, hipStream_t);                                   \
  template double norm2_host<T>(Ctx<T>&, const T*, int64_t);                            \
  template void setup_operator<T>(Ctx<T>&);                                             \
  template void scatter_freq<T>(Ctx<T>&, const T*, T*);                                 \
  template void gather_freq<T>(Ctx<T>&, const T*, T*);                                  \
  template ColIO<T> col_io<T>(Ctx<T>&, int, const Supp*);                               \
  template double launch_col<T>(Ctx<T>&, const Cx<T>*, Cx<T>*, bool, const ColIO<T>&, int*); \
  template double launch_row<T>(Ctx<T>&, int, const T*, T*, double*, const int*, int*);      \
  template void transform_fwd<T>(Ctx<T>&, const T*, T*, bool);                                \
  template void load_measurements<T>(Ctx<T>&, const T*);                                \
  template void cplx_in<T>(Ctx<T>&, const T*, double, double);                          \
  template void cplx_out<T>(Ctx<T>&, T*, double, double);                               \
  template void transform_adj<T>(Ctx<T>&, const T*, T*, bool);                              \
  template void perm_in<T>(Ctx<T>&, const T*, T*);                                      \
  template void perm_out<T>(Ctx<T>&, const T*, T*);                                     \
  template void rand_in<T>(Ctx<T>&, const T*, T*, const int*);                          \
  template void rand_out<T>(Ctx<T>&, const T*, T*, const int*);                         \
  template void rand_in_nat<T>(Ctx<T>&, const T*, T*, const int*);                      \
  template void rand_out_nat<T>(Ctx<T>&, const T*, T*, const int*);                     \
  template double psi_middle<T>(Ctx<T>&, CgScalars*, int*);                             \
  template void psi_resid_middle<T>(Ctx<T>&);                                           \
  template void psi2_happly<T>(Ctx<T>&, CgScalars*, T*);                                \
  template void psi2_resid<T>(Ctx<T>&, T*);                                             \
  template void psi2_forward<T>(Ctx<T>&, const T*, T*);                                 \
  template void psi2_adjoint<T>(Ctx<T>&, const T*, T*);                                 \
  template void prepare_kernels<T>();
CS_INST(float)
CS_INST(double)
template void fill<int32_t>(int32_t*, int64_t, int32_t, hipStream_t);
template void fill<uint32_t>(uint32_t*, int64_t, uint32_t, hipStream_t);

}  // namespace csr
