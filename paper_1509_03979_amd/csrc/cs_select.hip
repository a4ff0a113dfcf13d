// Selection subsystem: support detection (Eq. (6), Algorithm 1 line 03) and
// the top-K selections of SP and OMPR.
//
// Every selection ranks candidates by (magnitude descending, index ascending).
// Candidates live at keys k (the key order of the column passes; natural index
// j = nat_of_key(k)); sets of selected candidates are N-bit bitmaps over keys,
// and the natural index decides ties.
// Magnitudes are compared through their IEEE bit patterns, which order like the
// values for non-negative numbers; a key of 0 marks an excluded candidate and
// every admissible key is bits(|v|) + 1.
//  * argmax: packed keys (bits + 1, ~index) reduced with wavefront shuffles.
//  * top-K: MSB-first radix select, 8 bits per pass, on the magnitude key;
//    if the K-th key is shared by more candidates than are still needed, a
//    second radix select over the indices (ascending) keeps the lowest ones.
//    Selected indices are marked in an N-bit bitmap and compacted to a sorted
//    list with a block prefix sum, so supports come out ascending.
#include "cs_device.h"

#include <algorithm>

namespace csr {

static inline unsigned nblk(int64_t n, int t) { return (unsigned)std::max<int64_t>(1, (n + t - 1) / t); }

// ------------------------------------------------------------------ argmax outside a set
template <typename T>
__global__ void k_argmax_partial(const T* __restrict__ dense, const uint32_t* __restrict__ excl, const Plan pl,
                                 ArgKey* __restrict__ part, SelState* sel) {
  const int64_t n = pl.n;
  ArgKey best{0, 0, 0};
  bool bad = false;
  const int64_t st = (int64_t)gridDim.x * blockDim.x;
  for (int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; p < n; p += st) {
    if (excl && bit_of(excl, p)) continue;
    const int64_t j = nat_of_key(p, pl);
    const T v = dense[p];
    bad |= !finite_v(v);
    ArgKey k{mag_bits(v) + 1, 0xFFFFFFFFu - (uint32_t)j, 0};
    if (key_gt(k, best)) best = k;
  }
  if (bad) atomicOr(&sel->nonfinite, 1);
  best = block_max_key(best);
  if (threadIdx.x == 0) part[blockIdx.x] = best;
}

__global__ void k_argmax_final(const ArgKey* __restrict__ part, int np, int32_t* out_j) {
  ArgKey best{0, 0, 0};
  for (int i = threadIdx.x; i < np; i += blockDim.x)
    if (key_gt(part[i], best)) best = part[i];
  best = block_max_key(best);
  if (threadIdx.x == 0) *out_j = best.hi ? (int32_t)(0xFFFFFFFFu - best.lo) : -1;
}

template <typename T>
void argmax_excl(Ctx<T>& c, const T* dense, const uint32_t* excl, int32_t* out_j) {
  const int64_t n = c.plan.n;
  const unsigned grid = (unsigned)std::min<int64_t>(kArgBlocks, nblk(n, 256));
  hipLaunchKernelGGL(k_argmax_partial<T>, dim3(grid), dim3(256), 0, c.stream, dense, excl, c.plan, c.argpart, c.sel);
  CS_LAUNCH_CHECK();
  hipLaunchKernelGGL(k_argmax_final, dim3(1), dim3(1024), 0, c.stream, c.argpart, (int)grid, out_j);
  CS_LAUNCH_CHECK();
}

// ------------------------------------------------------------------ radix select
// Candidate sources.  Dense: key k of a key-order vector, excluded through a
// key bitmap.  Compact: entry i of vals at key list[i].  Both report the key
// (for marking) and the natural index (for ties).
struct DenseSrc {};
struct CompactSrc {};

template <typename T, typename S>
__device__ __forceinline__ void cand(const T* __restrict__ vals, const void* __restrict__ aux, int64_t i,
                                     const Plan& pl, uint64_t& key, uint32_t& j, uint32_t& pos, bool& bad) {
  if constexpr (std::is_same<S, DenseSrc>::value) {
    const uint32_t* excl = (const uint32_t*)aux;
    pos = (uint32_t)i;
    j = (uint32_t)nat_of_key(i, pl);
    if (excl && bit_of(excl, i)) { key = 0; return; }
    const T v = vals[i];
    bad |= !finite_v(v);
    key = mag_bits(v) + 1;
  } else {
    const int32_t* list = (const int32_t*)aux;
    pos = (uint32_t)list[i];
    j = (uint32_t)nat_of_key(pos, pl);
    const T v = vals[i];
    bad |= !finite_v(v);
    key = mag_bits(v) + 1;
  }
}

__global__ void k_sel_init(SelState* sel, int64_t need) {
  if (threadIdx.x == 0) {
    sel->prefix = 0; sel->pmask = 0; sel->need = need; sel->count_eq = 0;
    sel->jprefix = 0; sel->jmask = 0; sel->jneed = 0; sel->tie = 0; sel->nonfinite = 0;
  }
  for (int i = threadIdx.x; i < 256; i += blockDim.x) sel->hist[i] = 0;
}

// phase 0: histogram of key digit at `shift` among keys matching the prefix.
// phase 1: histogram of index digit among keys equal to the threshold whose
//          index matches the index prefix (only when the tie-break is active).
template <typename T, typename S, int PHASE>
__global__ void k_radix_hist(const T* __restrict__ vals, const void* __restrict__ aux, int64_t count, const Plan pl,
                             SelState* sel, int shift) {
  __shared__ uint32_t h[256];
  if (PHASE == 1 && !sel->tie) return;
  for (int i = threadIdx.x; i < 256; i += blockDim.x) h[i] = 0;
  __syncthreads();
  const uint64_t prefix = sel->prefix, pmask = sel->pmask;
  const uint32_t jprefix = sel->jprefix, jmask = sel->jmask;
  bool bad = false;
  const int64_t st = (int64_t)gridDim.x * blockDim.x;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < count; i += st) {
    uint64_t key; uint32_t j, pos;
    cand<T, S>(vals, aux, i, pl, key, j, pos, bad);
    if (PHASE == 0) {
      if ((key & pmask) == prefix) atomicAdd(&h[(key >> shift) & 255u], 1u);
    } else {
      if (key == prefix && (j & jmask) == jprefix) atomicAdd(&h[(j >> shift) & 255u], 1u);
    }
  }
  if (PHASE == 0 && bad) atomicOr(&sel->nonfinite, 1);
  __syncthreads();
  for (int i = threadIdx.x; i < 256; i += blockDim.x)
    if (h[i]) atomicAdd(&sel->hist[i], h[i]);
}

// One block of 256 threads: the histogram is staged in LDS with one load per
// thread and a suffix (phase 0, digits high to low) or prefix (phase 1,
// digits low to high) scan picks the digit that holds the `need`-th candidate.
template <int PHASE>
__global__ void k_radix_pick(SelState* sel, int shift) {
  __shared__ int64_t cum[256];
  __shared__ int64_t hist[256];
  const int t = threadIdx.x;
  if (PHASE == 1 && !sel->tie) {
    sel->hist[t] = 0;
    return;
  }
  const int64_t h = sel->hist[t];
  // phase 0 scans digits from 255 down: position q = 255 - digit
  const int q = (PHASE == 0) ? 255 - t : t;
  hist[q] = h;
  __syncthreads();
  // inclusive scan over q
  int64_t v = hist[t];
  cum[t] = v;
  __syncthreads();
  for (int off = 1; off < 256; off <<= 1) {
    const int64_t a = (t >= off) ? cum[t - off] : 0;
    __syncthreads();
    cum[t] += a;
    __syncthreads();
  }
  const int64_t need = (PHASE == 0) ? sel->need : sel->jneed;
  const int64_t incl = cum[t], excl = incl - hist[t];
  __syncthreads();
  if (excl < need && need <= incl) {          // exactly one q satisfies this (need >= 1)
    const int d = (PHASE == 0) ? 255 - t : t;
    if (PHASE == 0) {
      sel->need = need - excl;
      sel->prefix |= (uint64_t)d << shift;
      sel->pmask |= (uint64_t)255 << shift;
      if (shift == 0) {
        sel->count_eq = hist[t];
        sel->tie = (need - excl < hist[t]) ? 1 : 0;
        sel->jneed = need - excl;
      }
    } else {
      sel->jneed = need - excl;
      sel->jprefix |= (uint32_t)d << shift;
      sel->jmask |= 255u << shift;
    }
  }
  sel->hist[t] = 0;
}

template <typename T, typename S>
__global__ void k_radix_mark(const T* __restrict__ vals, const void* __restrict__ aux, int64_t count, const Plan pl,
                             const SelState* __restrict__ sel, uint32_t* __restrict__ bits) {
  const uint64_t tau = sel->prefix;
  const int tie = sel->tie;
  const uint32_t jt = sel->jprefix;
  bool bad = false;
  const int64_t st = (int64_t)gridDim.x * blockDim.x;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < count; i += st) {
    uint64_t key; uint32_t j, pos;
    cand<T, S>(vals, aux, i, pl, key, j, pos, bad);
    if (key == 0) continue;
    if (key > tau || (key == tau && (!tie || j <= jt))) atomicOr(&bits[pos >> 5], 1u << (pos & 31));
  }
}

template <typename T, typename S>
static void radix_topk(Ctx<T>& c, const T* vals, const void* aux, int64_t count, int k, uint32_t* out_bits) {
  hipStream_t s = c.stream;
  const Plan& pl = c.plan;
  const unsigned grid = (unsigned)std::min<int64_t>(1024, nblk(count, 256));
  fill_u32(out_bits, c.plan.words, 0u, s);
  hipLaunchKernelGGL(k_sel_init, dim3(1), dim3(256), 0, s, c.sel, (int64_t)k);
  CS_LAUNCH_CHECK();
  const int width = (sizeof(T) == 4) ? 32 : 64;
  for (int shift = width - 8; shift >= 0; shift -= 8) {
    hipLaunchKernelGGL((k_radix_hist<T, S, 0>), dim3(grid), dim3(256), 0, s, vals, aux, count, pl, c.sel, shift);
    CS_LAUNCH_CHECK();
    hipLaunchKernelGGL(k_radix_pick<0>, dim3(1), dim3(256), 0, s, c.sel, shift);
    CS_LAUNCH_CHECK();
  }
  for (int shift = 24; shift >= 0; shift -= 8) {
    hipLaunchKernelGGL((k_radix_hist<T, S, 1>), dim3(grid), dim3(256), 0, s, vals, aux, count, pl, c.sel, shift);
    CS_LAUNCH_CHECK();
    hipLaunchKernelGGL(k_radix_pick<1>, dim3(1), dim3(256), 0, s, c.sel, shift);
    CS_LAUNCH_CHECK();
  }
  hipLaunchKernelGGL((k_radix_mark<T, S>), dim3(grid), dim3(256), 0, s, vals, aux, count, pl, c.sel, out_bits);
  CS_LAUNCH_CHECK();
}

template <typename T>
void topk_dense(Ctx<T>& c, const T* dense, const uint32_t* excl, int k, uint32_t* out_bits) {
  radix_topk<T, DenseSrc>(c, dense, excl, c.plan.n, k, out_bits);
}

template <typename T>
void topk_compact(Ctx<T>& c, const T* vals, const int32_t* list, int count, int k, uint32_t* out_bits) {
  radix_topk<T, CompactSrc>(c, vals, list, count, k, out_bits);
}

// ------------------------------------------------------------------ bitmaps
__global__ void k_bits_or(const uint32_t* __restrict__ a, const uint32_t* __restrict__ b, uint32_t* __restrict__ o,
                          int64_t words) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < words) o[i] = a[i] | b[i];
}
void bits_or(const uint32_t* a, const uint32_t* b, uint32_t* out, int64_t words, hipStream_t s) {
  hipLaunchKernelGGL(k_bits_or, dim3(nblk(words, 256)), dim3(256), 0, s, a, b, out, words);
  CS_LAUNCH_CHECK();
}

__global__ void k_bits_set_list(uint32_t* __restrict__ bits, const int32_t* __restrict__ list, int k) {
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < k) {
    const uint32_t j = (uint32_t)list[i];
    atomicOr(&bits[j >> 5], 1u << (j & 31));
  }
}
void bits_set_list(uint32_t* bits, const int32_t* list, int k, hipStream_t s) {
  if (k <= 0) return;
  hipLaunchKernelGGL(k_bits_set_list, dim3(nblk(k, 256)), dim3(256), 0, s, bits, list, k);
  CS_LAUNCH_CHECK();
}

__global__ void k_bits_diff(const uint32_t* __restrict__ a, const uint32_t* __restrict__ b, int64_t words,
                            int32_t* flag) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < words && a[i] != b[i]) *flag = 1;
}
int bits_equal(const uint32_t* a, const uint32_t* b, int64_t words, int32_t* scratch, hipStream_t s) {
  fill<int32_t>(scratch, 1, 0, s);
  hipLaunchKernelGGL(k_bits_diff, dim3(nblk(words, 256)), dim3(256), 0, s, a, b, words, scratch);
  CS_LAUNCH_CHECK();
  int32_t h = 0;
  dev_read(s, scratch, &h, sizeof(int32_t));
  return h == 0;
}

__global__ void k_bits_count(const uint32_t* __restrict__ bits, int64_t words, uint32_t* __restrict__ cnt) {
  bits_count_body(bits, words, cnt, blockIdx.x);
}
__global__ void k_bits_scan(uint32_t* cnt, int nb) { bits_scan_body(cnt, nb); }
__global__ void k_bits_write(const uint32_t* __restrict__ bits, int64_t words, const uint32_t* __restrict__ cnt,
                             int32_t* __restrict__ list, int limit, uint32_t* __restrict__ wpre) {
  bits_write_body(bits, words, cnt, list, limit, wpre, blockIdx.x);
}

template <typename T>
int bits_to_list(Ctx<T>& c, const uint32_t* bits, int32_t* list, int expect, uint32_t* wpre) {
  const int64_t words = c.plan.words;
  const int nb = (int)((words + kBitsPerBlockWords - 1) / kBitsPerBlockWords);
  hipStream_t s = c.stream;
  hipLaunchKernelGGL(k_bits_count, dim3(nb), dim3(256), 0, s, bits, words, c.blockcnt);
  CS_LAUNCH_CHECK();
  hipLaunchKernelGGL(k_bits_scan, dim3(1), dim3(1024), 0, s, c.blockcnt, nb);
  CS_LAUNCH_CHECK();
  hipLaunchKernelGGL(k_bits_write, dim3(nb), dim3(256), 0, s, bits, words, c.blockcnt, list, expect, wpre);
  CS_LAUNCH_CHECK();
  return nb;   // total count is left in blockcnt[nb]
}

#define CS_INST(T)                                                                        \
  template void argmax_excl<T>(Ctx<T>&, const T*, const uint32_t*, int32_t*);           \
  template void topk_dense<T>(Ctx<T>&, const T*, const uint32_t*, int, uint32_t*);      \
  template void topk_compact<T>(Ctx<T>&, const T*, const int32_t*, int, int, uint32_t*); \
  template int bits_to_list<T>(Ctx<T>&, const uint32_t*, int32_t*, int, uint32_t*);
CS_INST(float)
CS_INST(double)

}  // namespace csr
