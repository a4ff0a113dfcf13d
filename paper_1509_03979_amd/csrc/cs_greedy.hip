// Greedy drivers: OMP (Sec. II steps 1-4, Algorithm 1 lines 01-10), SP and
// OMPR (the other two greedy algorithms of Sec. IV), all built from the same
// three steps: correlation A^T r, support selection, CG least squares.
//
// State lives on the device: supports as sorted int32 lists plus N-bit
// bitmaps, solutions as compact vectors, the current solution also scattered
// (sign-flipped, v-order) into the dense buffer Dx that the residual pass
// reads.  Warm starts gather the previous solution from Dx, which is zero off
// the previous support, so new indices start at 0.
//
// Decision rules follow the SP/OMPR readings documented with the oracle:
//   SP:   stop with T' when T' == T; stop with (T, x) when ||r'|| > ||r||.
//   OMPR: l = 1, z = x + eta A^T r on I u {j}; stop when j ranks last.
#include "cs_internal.h"

#include <algorithm>
#include <cmath>
#include <utility>

namespace csr {

static inline unsigned nblk(int64_t n, int t) { return (unsigned)std::max<int64_t>(1, (n + t - 1) / t); }

// out[i] = vals[position of sub[i] in sup] (sub is a subset of sup, both ascending)
template <typename T>
__global__ void k_subset_gather(const int32_t* __restrict__ sup, const T* __restrict__ vals, int ksup,
                                const int32_t* __restrict__ sub, T* __restrict__ out, int ksub) {
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= ksub) return;
  const int32_t key = sub[i];
  int lo = 0, hi = ksup - 1;
  T v = (T)0;
  while (lo <= hi) {
    const int mid = (lo + hi) >> 1;
    const int32_t m = sup[mid];
    if (m == key) { v = vals[mid]; break; }
    if (m < key) lo = mid + 1; else hi = mid - 1;
  }
  out[i] = v;
}

// OMPR drop step.  Candidates I u {j}: z_i = x_i + eta (A^T r)_i, z_j = eta (A^T r)_j.
// The dropped element is the last under (|z| desc, index asc): the smallest
// |z|, ties to the larger index.  Packed as a max-reduction over
// (~bits(|z|), index).
template <typename T> __device__ __forceinline__ uint64_t mag_bits2(T v);
template <> __device__ __forceinline__ uint64_t mag_bits2<float>(float v) { return (uint64_t)__float_as_uint(fabsf(v)); }
template <> __device__ __forceinline__ uint64_t mag_bits2<double>(double v) {
  return (uint64_t)__double_as_longlong(fabs(v));
}

__device__ __forceinline__ bool dkey_gt(uint64_t ah, uint32_t al, uint64_t bh, uint32_t bl) {
  return ah > bh || (ah == bh && al > bl);
}

template <typename T>
__global__ void k_ompr_drop(const T* __restrict__ x, const int32_t* __restrict__ list, int k,
                            const T* __restrict__ Wv, const int8_t* __restrict__ signs, int64_t n, T eta,
                            const int32_t* __restrict__ jptr, int32_t* __restrict__ out) {
  // single block of 1024 threads
  __shared__ uint64_t sh_h[16];
  __shared__ uint32_t sh_l[16];
  uint64_t bh = 0;
  uint32_t bl = 0;
  const int32_t jn = *jptr;
  for (int i = threadIdx.x; i <= k; i += blockDim.x) {
    int64_t j;
    T z;
    if (i < k) {
      j = list[i];
      const T cv = signs[j] < 0 ? -Wv[vpos(j, n)] : Wv[vpos(j, n)];
      z = x[i] + eta * cv;
    } else {
      j = jn;
      if (j < 0) continue;
      const T cv = signs[j] < 0 ? -Wv[vpos(j, n)] : Wv[vpos(j, n)];
      z = eta * cv;
    }
    const uint64_t h = ~mag_bits2(z);
    const uint32_t l = (uint32_t)j;
    if (dkey_gt(h, l, bh, bl)) { bh = h; bl = l; }
  }
  for (int off = 32; off > 0; off >>= 1) {
    const uint64_t oh = __shfl_down((unsigned long long)bh, off, 64);
    const uint32_t ol = __shfl_down(bl, off, 64);
    if (dkey_gt(oh, ol, bh, bl)) { bh = oh; bl = ol; }
  }
  if ((threadIdx.x & 63) == 0) { sh_h[threadIdx.x >> 6] = bh; sh_l[threadIdx.x >> 6] = bl; }
  __syncthreads();
  if (threadIdx.x == 0) {
    for (int w = 1; w < (int)(blockDim.x >> 6); ++w)
      if (dkey_gt(sh_h[w], sh_l[w], bh, bl)) { bh = sh_h[w]; bl = sh_l[w]; }
    out[0] = (int32_t)bl;
  }
}

__global__ void k_swap_bits(uint32_t* bits, const int32_t* __restrict__ jd) {
  // jd[0] = j to set, jd[1] = index to clear
  if (threadIdx.x == 0 && blockIdx.x == 0) {
    const uint32_t j = (uint32_t)jd[0], d = (uint32_t)jd[1];
    bits[d >> 5] &= ~(1u << (d & 31));
    bits[j >> 5] |= 1u << (j & 31);
  }
}

__global__ void k_set_bit_dev(uint32_t* bits, const int32_t* __restrict__ jp) {
  if (threadIdx.x == 0 && blockIdx.x == 0) {
    const int32_t j = *jp;
    if (j >= 0) bits[(uint32_t)j >> 5] |= 1u << ((uint32_t)j & 31);
  }
}

template <typename T>
__global__ void k_scatter_plain(T* __restrict__ s, const int32_t* __restrict__ list, const T* __restrict__ x, int k) {
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < k) s[list[i]] = x[i];
}

template <typename T>
void write_output(Ctx<T>& c, const int32_t* list, const T* x, int k, T* s_out, int32_t* supp_out) {
  fill<T>(s_out, c.plan.n, (T)0, c.stream);
  hipLaunchKernelGGL(k_scatter_plain<T>, dim3(nblk(k, 256)), dim3(256), 0, c.stream, s_out, list, x, k);
  CS_LAUNCH_CHECK();
  CS_HIP(hipMemcpyAsync(supp_out, list, sizeof(int32_t) * k, hipMemcpyDeviceToDevice, c.stream));
}

static inline int cg_cap(const cs_params& prm, int k) {
  return prm.cg_max_iter > 0 ? prm.cg_max_iter : 2 * k + 50;
}

// ------------------------------------------------------------------ OMP
template <typename T>
void run_omp(Ctx<T>& c, int K, double tol, const cs_params& prm, T* s_out, int32_t* supp_out, cs_info* info) {
  hipStream_t s = c.stream;
  const int64_t words = c.plan.words;
  uint32_t* bitsS = c.bits[0];
  int32_t* cur = c.list[0];
  int32_t* nxt = c.list[1];
  T* x = c.cx;
  fill_u32(bitsS, words, 0u, s);
  fill<T>(c.Dx, c.plan.n, (T)0, s);
  double rn = 0.0;
  for (int i = 1; i <= K; ++i) {
    // the first correlation is A^T r_0 = A^T y, already in C0
    argmax_excl<T>(c, i == 1 ? (const T*)c.C0 : (const T*)c.W, bitsS, c.ibuf);   // line 03
    hipLaunchKernelGGL(k_set_bit_dev, dim3(1), dim3(64), 0, s, bitsS, (const int32_t*)c.ibuf);   // line 04
    CS_LAUNCH_CHECK();
    bits_to_list<T>(c, bitsS, nxt, i);
    const bool warm = prm.warm_start != 0 && i > 1;
    if (warm) gather_signed<T>(c, c.Dx, nxt, x, i);
    cg_solve<T>(c, nxt, i, x, warm, tol, cg_cap(prm, i));              // line 06
    rn = resid_corr<T>(c, cur, i - 1, nxt, x, i);                       // line 07 (+ next line 03's A^T r)
    std::swap(cur, nxt);
  }
  write_output<T>(c, cur, x, K, s_out, supp_out);
  if (info) { info->outer_iters = K; info->resid_norm = rn; }
}

// ------------------------------------------------------------------ SP
template <typename T>
void run_sp(Ctx<T>& c, int K, double tol, const cs_params& prm, T* s_out, int32_t* supp_out, cs_info* info) {
  hipStream_t s = c.stream;
  const int64_t words = c.plan.words;
  uint32_t* bT = c.bits[0];
  uint32_t* bU = c.bits[1];   // T u D
  uint32_t* bN = c.bits[2];   // D, then T'
  int32_t* lT = c.list[0];
  int32_t* lU = c.list[1];
  int32_t* lN = c.list[2];
  T* xT = c.cx;               // on T
  T* xU = c.cx2;              // on T u D
  T* xN = c.cx3;              // on T'
  const bool warm = prm.warm_start != 0;
  const int max_outer = prm.max_outer > 0 ? prm.max_outer : 100;

  fill<T>(c.Dx, c.plan.n, (T)0, s);
  topk_dense<T>(c, c.C0, nullptr, K, bT);
  bits_to_list<T>(c, bT, lT, K);
  cg_solve<T>(c, lT, K, xT, false, tol, cg_cap(prm, K));
  double rn = resid_corr<T>(c, nullptr, 0, lT, xT, K);
  int rounds = 0;
  bool stopped = false;
  for (int l = 1; l <= max_outer; ++l) {
    rounds = l;
    topk_dense<T>(c, (const T*)c.W, bT, K, bN);          // D: top-K of |A^T r| outside T
    bits_or(bT, bN, bU, words, s);
    bits_to_list<T>(c, bU, lU, 2 * K);
    if (warm) gather_signed<T>(c, c.Dx, lU, xU, 2 * K);
    cg_solve<T>(c, lU, 2 * K, xU, warm, tol, cg_cap(prm, 2 * K));
    topk_compact<T>(c, xU, lU, 2 * K, K, bN);             // T': top-K of |x~| over T u D
    bits_to_list<T>(c, bN, lN, K);
    if (warm)
      hipLaunchKernelGGL(k_subset_gather<T>, dim3(nblk(K, 256)), dim3(256), 0, s, lU, xU, 2 * K, lN, xN, K);
    CS_LAUNCH_CHECK();
    cg_solve<T>(c, lN, K, xN, warm, tol, cg_cap(prm, K));
    const bool same = bits_equal(bN, bT, words, c.ibuf + 8, s);
    const double rn2 = resid_corr<T>(c, lT, K, lN, xN, K);
    if (same) {
      std::swap(lT, lN); std::swap(bT, bN); std::swap(xT, xN);
      rn = rn2;
      stopped = true;
      break;
    }
    if (rn2 > rn) {   // keep the previous (T, x)
      stopped = true;
      break;
    }
    std::swap(lT, lN); std::swap(bT, bN); std::swap(xT, xN);
    rn = rn2;
  }
  if (!stopped) c.flags |= CS_F_OUTER_MAXITER;
  write_output<T>(c, lT, xT, K, s_out, supp_out);
  if (info) { info->outer_iters = rounds; info->resid_norm = rn; }
}

// ------------------------------------------------------------------ OMPR
template <typename T>
void run_ompr(Ctx<T>& c, int K, double tol, const cs_params& prm, T* s_out, int32_t* supp_out, cs_info* info) {
  hipStream_t s = c.stream;
  uint32_t* bI = c.bits[0];
  int32_t* lI = c.list[0];
  int32_t* lN = c.list[1];
  T* xI = c.cx;
  T* xN = c.cx3;
  const bool warm = prm.warm_start != 0;
  const int max_outer = prm.max_outer > 0 ? prm.max_outer : 4 * K;
  const double eta = prm.ompr_eta > 0 ? prm.ompr_eta : (double)c.plan.n / (double)c.plan.m;

  fill<T>(c.Dx, c.plan.n, (T)0, s);
  topk_dense<T>(c, c.C0, nullptr, K, bI);
  bits_to_list<T>(c, bI, lI, K);
  cg_solve<T>(c, lI, K, xI, false, tol, cg_cap(prm, K));
  double rn = resid_corr<T>(c, nullptr, 0, lI, xI, K);
  int swaps = 0;
  bool stopped = false;
  int32_t jd[2];
  for (int t = 1; t <= max_outer; ++t) {
    if (rn <= 1e-12 * c.ynorm) { stopped = true; break; }
    argmax_excl<T>(c, (const T*)c.W, bI, c.ibuf);
    hipLaunchKernelGGL(k_ompr_drop<T>, dim3(1), dim3(1024), 0, s, xI, lI, K, (const T*)c.W, c.signs, c.plan.n,
                       (T)eta, (const int32_t*)c.ibuf, c.ibuf + 1);
    CS_LAUNCH_CHECK();
    dev_read(s, c.ibuf, jd, 2 * sizeof(int32_t));
    if (jd[0] < 0 || jd[1] == jd[0]) { stopped = true; break; }
    hipLaunchKernelGGL(k_swap_bits, dim3(1), dim3(64), 0, s, bI, (const int32_t*)c.ibuf);
    CS_LAUNCH_CHECK();
    bits_to_list<T>(c, bI, lN, K);
    if (warm) gather_signed<T>(c, c.Dx, lN, xN, K);
    cg_solve<T>(c, lN, K, xN, warm, tol, cg_cap(prm, K));
    rn = resid_corr<T>(c, lI, K, lN, xN, K);
    std::swap(lI, lN); std::swap(xI, xN);
    ++swaps;
  }
  if (!stopped) c.flags |= CS_F_OUTER_MAXITER;
  write_output<T>(c, lI, xI, K, s_out, supp_out);
  if (info) { info->outer_iters = swaps; info->resid_norm = rn; }
}

#define CS_INST(T)                                                                                   \
  template void run_omp<T>(Ctx<T>&, int, double, const cs_params&, T*, int32_t*, cs_info*);       \
  template void run_sp<T>(Ctx<T>&, int, double, const cs_params&, T*, int32_t*, cs_info*);        \
  template void run_ompr<T>(Ctx<T>&, int, double, const cs_params&, T*, int32_t*, cs_info*);      \
  template void write_output<T>(Ctx<T>&, const int32_t*, const T*, int, T*, int32_t*);
CS_INST(float)
CS_INST(double)

}  // namespace csr
