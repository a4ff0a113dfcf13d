// Selection subsystem: support detection (Eq. (6), Algorithm 1) and the
// top-K selections of SP and OMPR.
//
// Every selection ranks candidates by (magnitude descending, index ascending).
// Candidates live at keys k (the key order of the column passes; natural index
// j = nat_of_key(k)); sets of selected candidates are N-bit bitmaps over keys,
// and the natural index decides ties.
// Magnitudes are compared through their IEEE bit patterns, which order like the
// values for non-negative numbers; a key of 0 marks an excluded candidate and
// every admissible key is bits(|v|) + 1.
//  * argmax: packed keys (bits + 1, ~index) reduced with wavefront shuffles.
//  * top-K of a dense vector: order statistics of a sample bracket the K-th
//    key in a band; one streaming pass writes the bitmap of the keys above the band and
//    collects the keys inside it; an MSB-first radix select (13-bit digits)
//    over those candidates finds the threshold.  Each pass adds its
//    workgroup histograms into one global row with atomics (only the bins a
//    workgroup saw), and the next pass reads that row to fix the digit, so a
//    digit costs one row read and no extra launch; three rows rotate so that
//    each pass also clears the row two passes ahead.  If the K-th key is
//    shared by more candidates than are still needed, the ones with the
//    lowest natural indices are kept.  When the band misses (too many keys
//    above it, too few in it, or a full segment) the same radix passes run
//    over every key instead.  Top-K of a compact vector runs the radix passes
//    over its entries.  Supports are compacted from the bitmaps with a block
//    prefix sum, so they come out ascending.
#include "cs_device.h"

#include <algorithm>
#include <cstddef>
#include <cstdlib>
#include <type_traits>

namespace csr {

static inline unsigned nblk(int64_t n, int t) { return (unsigned)std::max<int64_t>(1, (n + t - 1) / t); }

// ------------------------------------------------------------------ argmax outside a set
// Each workgroup keeps its best two keys (part[2b], part[2b + 1]), so the
// final also has the runner-up: the decision's margin.
template <typename T>
__global__ void k_argmax_partial(const T* __restrict__ dense, const uint32_t* __restrict__ excl, const Plan pl,
                                 ArgKey* __restrict__ part, SelState* sel) {
  const int64_t n = pl.n;
  K2 t;
  bool bad = false;
  const int64_t st = (int64_t)gridDim.x * blockDim.x;
  for (int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; p < n; p += st) {
    if (excl && bit_of(excl, p)) continue;
    const int64_t j = nat_of_key(p, pl);
    const T v = dense[p];
    bad |= !finite_v(v);
    t.add(mag_bits(v) + 1, 0xFFFFFFFFu - (uint32_t)j);
  }
  if (bad) atomicOr(&sel->nonfinite, 1);
  block_max_key2(t);
  if (threadIdx.x == 0) {
    part[2 * blockIdx.x] = t.best();
    part[2 * blockIdx.x + 1] = t.second();
  }
}

// A residual gate (r2 non-null): when *r2 <= thr2 the selection is not made,
// out_j = -2 and no margin is noted (the caller stops on a zero residual).
template <typename T>
__global__ void k_argmax_final(const ArgKey* __restrict__ part, int np, int32_t* out_j, SelState* sel,
                               const double* __restrict__ r2, double thr2) {
  if (r2 && *r2 <= thr2) {
    if (threadIdx.x == 0) *out_j = -2;
    return;
  }
  K2 t;
  for (int i = threadIdx.x; i < np; i += blockDim.x) {
    const ArgKey a = part[2 * i], b = part[2 * i + 1];
    t.add(a.hi, a.lo, b.hi, b.lo);
  }
  block_max_key2(t);
  if (threadIdx.x == 0) {
    *out_j = t.bh ? (int32_t)(0xFFFFFFFFu - t.bl) : -1;
    if (t.bh && t.sh) {
      const double vb = key_value<T>(t.bh);
      note_margin(&sel->mmin, &sel->mrel, vb - key_value<T>(t.sh), vb);
    }
  }
}

template <typename T>
void argmax_excl(Ctx<T>& c, const T* dense, const uint32_t* excl, int32_t* out_j, const double* r2, double thr2) {
  const int64_t n = c.plan.n;
  const unsigned grid = (unsigned)std::min<int64_t>(kArgBlocks, nblk(n, 256));
  hipLaunchKernelGGL(k_argmax_partial<T>, dim3(grid), dim3(256), 0, c.stream, dense, excl, c.plan, c.argpart, c.sel);
  CS_LAUNCH_CHECK();
  hipLaunchKernelGGL(k_argmax_final<T>, dim3(1), dim3(1024), 0, c.stream, c.argpart, (int)grid, out_j, c.sel, r2,
                     thr2);
  CS_LAUNCH_CHECK();
}

// Start of a call: no margin yet, the radix rows cleared.
__global__ void k_sel_reset(SelState* sel, uint32_t* __restrict__ hrows) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < 3 * kSelBins) hrows[i] = 0u;
  if (i == 0) {
    sel->mmin = __builtin_huge_val();
    sel->mrel = __builtin_huge_val();
  }
}

template <typename T>
void sel_reset(Ctx<T>& c) {
  hipLaunchKernelGGL(k_sel_reset, dim3(nblk(3 * kSelBins, 256)), dim3(256), 0, c.stream, c.sel, c.hrows);
  CS_LAUNCH_CHECK();
}

template <typename T>
void margins_read(Ctx<T>& c, double* mmin, double* mrel) {
  double h[2];
  static_assert(offsetof(SelState, mrel) == offsetof(SelState, mmin) + sizeof(double), "layout");
  dev_read(c.stream, &c.sel->mmin, h, sizeof(h));
  *mmin = h[0];
  *mrel = h[1];
}

// ------------------------------------------------------------------ top-K
// Candidate sources of the radix passes (SelHead::mode).
enum : int32_t {
  SEL_DENSE = 0,   // every key of a dense key-order vector (excluded keys count as 0)
  SEL_SEG = 1,     // the candidate segments written by the dense split
  SEL_LIST = 2,    // a compact vector with its key list
  SEL_NONE = 3,    // the split already marked every selected key
};

constexpr int kSample = 2048;     // keys sampled to bracket the K-th key
constexpr int kDigit = kSelDigit;  // radix digit width of the passes
constexpr int kBins = kSelBins;
constexpr int kIdxDigit = 11;     // digit width of the radix select over tied indices
constexpr int kIdxBins = 1 << kIdxDigit;
static_assert(kBins % 1024 == 0, "bins per thread of the digit pick");
// rows rotate mod 3: after a selection of P passes only row (P - 1) mod 3 is
// left uncleared, and the next selection's first pass adds into row 0
static_assert((32 + kDigit - 1) / kDigit % 3 != 1 && (64 + kDigit - 1) / kDigit % 3 != 1, "row rotation");
constexpr int kTieCap = 4096;     // tied candidates sorted in LDS by the final pass

// Magnitude key of candidate i of a dense vector: 0 if excluded.
template <typename T>
__device__ __forceinline__ uint64_t dense_key(const T* __restrict__ vals, const uint32_t* __restrict__ excl,
                                              int64_t i) {
  if (excl && bit_of(excl, i)) return 0;
  return mag_bits(vals[i]) + 1;
}

__device__ __forceinline__ void load4(const float* p, float (&o)[4]) {
  const float4 v = *reinterpret_cast<const float4*>(p);
  o[0] = v.x; o[1] = v.y; o[2] = v.z; o[3] = v.w;
}
__device__ __forceinline__ void load4(const double* p, double (&o)[4]) {
  const double2 a = *reinterpret_cast<const double2*>(p);
  const double2 b = *reinterpret_cast<const double2*>(p + 2);
  o[0] = a.x; o[1] = a.y; o[2] = b.x; o[3] = b.y;
}

// Candidate records of the dense split store the key in the width of T.
template <typename T> using RecKey = typename std::conditional<sizeof(T) == 4, uint32_t, uint64_t>::type;

__device__ __forceinline__ uint64_t max_key(int keybits) { return keybits >= 64 ? ~0ull : (1ull << keybits) - 1; }

// Sorts LDS keys s[0, P) (P a power of two, <= 2 * blockDim.x * 2) with a
// bitonic network; ascending or descending.
__device__ void lds_bitonic(uint64_t* s, int P, bool descending) {
  for (int size = 2; size <= P; size <<= 1) {
    for (int str = size >> 1; str > 0; str >>= 1) {
      for (int q = threadIdx.x; q < (P >> 1); q += blockDim.x) {
        const int i = 2 * q - (q & (str - 1));
        const int j = i + str;
        const bool up = ((i & size) == 0) != descending;   // ascending run
        const uint64_t a = s[i], b = s[j];
        if ((a > b) == up) {
          s[i] = b;
          s[j] = a;
        }
      }
      __syncthreads();
    }
  }
}

// Inclusive prefix sum over the workgroup (any size up to 1024, a multiple of
// 64): wavefront shuffles, then the wavefront totals through LDS.
__device__ __forceinline__ int64_t block_incl_scan(int64_t v, int64_t* ws) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
#pragma unroll
  for (int off = 1; off < 64; off <<= 1) {
    const int64_t a = __shfl_up((long long)v, off, 64);
    if (lane >= off) v += a;
  }
  if (lane == 63) ws[wave] = v;
  __syncthreads();
  int64_t pre = 0;
  for (int i = 0; i < wave; ++i) pre += ws[i];
  __syncthreads();
  return v + pre;
}

// One workgroup of 1024 threads, two keys each: takes kSample keys at hashed
// offsets of equal strides (all keys when N <= kSample; padding keys are 0),
// finds two of their order statistics and sets the candidate band [t_lo,
// t_hi] so that, with high probability, fewer than K keys lie above t_hi and
// at least K lie at or above t_lo.  The band only steers the work: the first
// radix pass checks both counts and falls back to every key when either
// fails.  The ranking runs on the top 32 key bits (all of an FP32 key); for
// longer keys the band is widened to the edges of its 32-bit buckets.
template <typename T>
__global__ __launch_bounds__(1024) void k_sel_sample(const T* __restrict__ vals, const uint32_t* __restrict__ excl,
                                                     int64_t n, int64_t k, int keybits, SelState* sel) {
  const int t = threadIdx.x;
  const int S = (int)std::min<int64_t>(kSample, n);   // both powers of two
  const int64_t stride = n / S;
  const int kshift = keybits - 32;
  int64_t pos[2];
  T val[2];
  uint32_t xw[2];
#pragma unroll
  for (int h = 0; h < 2; ++h) {
    const int e = std::min(2 * t + h, S - 1);
    uint32_t x = (uint32_t)e * 0x9E3779B1u;
    x ^= x >> 16;
    x *= 0x85EBCA6Bu;
    x ^= x >> 13;
    pos[h] = (int64_t)e * stride + (int64_t)(x & (uint32_t)(stride - 1));
    val[h] = vals[pos[h]];
    xw[h] = excl ? excl[pos[h] >> 5] : 0u;
  }
  uint32_t v[2];
#pragma unroll
  for (int h = 0; h < 2; ++h) {
    const bool in = 2 * t + h < S && !((xw[h] >> (pos[h] & 31)) & 1u) && finite_v(val[h]);
    v[h] = in ? (uint32_t)((mag_bits(val[h]) + 1) >> kshift) : 0u;
  }
  // expected sample rank of the K-th key and a margin of four standard
  // deviations of a binomial count (none when the sample is every key)
  const double r = (double)k * (double)S / (double)n;
  const double margin = (S == n) ? 0.0 : 4.0 * sqrt(r) + 4.0;
  const int64_t rh = (int64_t)floor(r - margin), rl = (int64_t)ceil(r + margin);
  // the two keys needed, by descending rank among the kSample sample slots
  // (padding and excluded slots hold 0 and rank last): rank rh, or the
  // largest when no rank is safely above the K-th, and rank rl
  uint32_t want[2] = {(uint32_t)(rh >= 1 ? std::min<int64_t>(rh, S) : 1),
                      (uint32_t)(rl >= 1 && rl <= S ? rl : 1)};
  // MSB-first radix select of both ranks at once, 8-bit digits: per digit one
  // LDS histogram per rank over the keys that match its prefix, and one wave
  // per rank finds the digit whose descending cumulative count reaches it
  __shared__ uint32_t hist[2][256];
  __shared__ uint32_t sel_pref[2], sel_need[2];
  if (t < 2) {
    sel_pref[t] = 0u;
    sel_need[t] = want[t];
  }
#pragma unroll
  for (int shift = 24; shift >= 0; shift -= 8) {
    if (t < 512) hist[t >> 8][t & 255] = 0u;
    __syncthreads();
    const uint32_t hi = shift == 24 ? 0u : ~((1u << (shift + 8)) - 1u);   // the digits already fixed
    const uint32_t p0 = sel_pref[0], p1 = sel_pref[1];
#pragma unroll
    for (int h = 0; h < 2; ++h) {
      const uint32_t d = (v[h] >> shift) & 255u;
      if ((v[h] & hi) == p0) atomicAdd(&hist[0][d], 1u);
      if ((v[h] & hi) == p1) atomicAdd(&hist[1][d], 1u);
    }
    __syncthreads();
    const int wv = t >> 6, lane = t & 63;
    if (wv < 2) {
      // lane l holds digits 255 - 4l .. 252 - 4l (descending)
      uint32_t c[4], sum = 0;
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        c[q] = hist[wv][255 - 4 * lane - q];
        sum += c[q];
      }
      uint32_t incl = sum;   // inclusive prefix over lanes, in descending digit order
#pragma unroll
      for (int off = 1; off < 64; off <<= 1) {
        const uint32_t o = __shfl_up(incl, off, 64);
        if (lane >= off) incl += o;
      }
      const uint32_t need = sel_need[wv];
      const uint32_t excl = incl - sum;
      if (excl < need && need <= incl) {   // exactly one lane
        uint32_t above = excl;
        int q = 0;
#pragma unroll
        for (int qq = 0; qq < 3; ++qq)
          if (q == qq && above + c[qq] < need) {
            above += c[qq];
            q = qq + 1;
          }
        sel_pref[wv] |= (uint32_t)(255 - 4 * lane - q) << shift;
        sel_need[wv] = need - above;
      }
    }
    __syncthreads();
  }
  if (t == 0) {
    const uint32_t khi = sel_pref[0], klo = sel_pref[1];
    const uint64_t low = kshift ? (1ull << kshift) - 1 : 0ull;   // bits below the ranked ones
    uint64_t thi = max_key(keybits), tlo = 1;
    if (rh >= 1) thi = ((uint64_t)khi << kshift) | low;
    // no sample rank is safely above the K-th, but about N/S keys exceed the
    // sample's largest: with r >= 2 that is at most K/2 on average, so the
    // largest still bounds the band from above (the first pass checks it)
    else if (r >= 2.0 && khi != 0u) thi = ((uint64_t)khi << kshift) | low;
    if (rl >= 1 && rl <= S) tlo = std::max<uint64_t>(1, (uint64_t)klo << kshift);
    sel->t_lo = tlo;
    sel->t_hi = thi;
    sel->k = k;
    sel->nonfinite = 0;
  }
}

// Set bits of a wave-wide mask below this lane.
__device__ __forceinline__ uint32_t lane_prefix(uint64_t m) {
  return __builtin_amdgcn_mbcnt_hi((uint32_t)(m >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)m, 0u));
}

// Dense split (kSplitThreads per workgroup).  Workgroup b reads keys
// [b E, (b+1) E), four consecutive keys per lane, and writes the output bitmap words itself (keys above t_hi set,
// the rest clear), so no word needs clearing or atomics; keys inside the band
// go to the workgroup's candidate segment.  Per workgroup it records
// (candidates found, keys above the band).
template <typename T>
__device__ __forceinline__ void sel_split_body(const T* __restrict__ vals, const uint32_t* __restrict__ excl,
                                               int64_t n, int64_t eb, int cap, SelState* sel,
                                               RecKey<T>* __restrict__ rkey, uint32_t* __restrict__ rpos,
                                               int32_t* __restrict__ rcnt, uint32_t* __restrict__ out_bits) {
  __shared__ uint32_t s_mid;
  __shared__ uint32_t s_hi[kSplitThreads / 64];
  if (threadIdx.x == 0) s_mid = 0u;
  __syncthreads();
  const uint64_t t_lo = sel->t_lo, t_hi = sel->t_hi;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const uint64_t below = lane ? (~0ull >> (64 - lane)) : 0ull;
  const int64_t b0 = (int64_t)blockIdx.x * eb;
  const int64_t end = std::min<int64_t>(n, b0 + eb);
  RecKey<T>* bk = rkey + (int64_t)blockIdx.x * cap;
  uint32_t* bp = rpos + (int64_t)blockIdx.x * cap;
  uint32_t hcnt = 0;
  bool bad = false;
  constexpr int U = 4;                           // rounds in flight per iteration
  constexpr int R = kSplitThreads * 4;            // keys per round
  for (int64_t r0 = b0; r0 < end; r0 += U * R) {
    T v[U][4];
    uint32_t ex[U];
    // every load issued before any is used (a lane past the end re-reads the
    // last four keys and marks them excluded), so the rounds are in flight together
    uint32_t xw[U];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int64_t p = r0 + u * R + wave * 256 + lane * 4;
      const int64_t pc = p < end ? p : end - 4;
      load4(vals + pc, v[u]);
      xw[u] = excl ? excl[pc >> 5] : 0u;
    }
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int64_t p = r0 + u * R + wave * 256 + lane * 4;
      ex[u] = p < end ? (xw[u] >> (p & 31)) & 0xFu : 0xFu;
    }
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int64_t p = r0 + u * R + wave * 256 + lane * 4;
      uint64_t key[4];
      uint32_t hib = 0, midb = 0;
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        const bool x = (ex[u] >> e) & 1u;
        bad |= !x && !finite_v(v[u][e]);
        key[e] = x ? 0 : mag_bits(v[u][e]) + 1;
        if (key[e] > t_hi) hib |= 1u << e;
        else if (key[e] >= t_lo) midb |= 1u << e;
      }
      // eight lanes hold the 32 bits of one word
      uint32_t w = hib << ((lane & 7) * 4);
      w |= __shfl_xor(w, 1, 64);
      w |= __shfl_xor(w, 2, 64);
      w |= __shfl_xor(w, 4, 64);
      if ((lane & 7) == 0 && p < end) out_bits[p >> 5] = w;
      hcnt += __popc(hib);
      const uint64_t m0 = __ballot(midb & 1u), m1 = __ballot((midb >> 1) & 1u);
      const uint64_t m2 = __ballot((midb >> 2) & 1u), m3 = __ballot((midb >> 3) & 1u);
      const uint32_t c0 = __popcll(m0), c1 = __popcll(m1), c2 = __popcll(m2), c3 = __popcll(m3);
      const uint32_t tot = c0 + c1 + c2 + c3;
      if (tot) {
        uint32_t base = 0;
        if (lane == 0) base = atomicAdd(&s_mid, tot);
        base = __shfl(base, 0, 64);
        const uint32_t o[4] = {base + __popcll(m0 & below), base + c0 + __popcll(m1 & below),
                               base + c0 + c1 + __popcll(m2 & below), base + c0 + c1 + c2 + __popcll(m3 & below)};
#pragma unroll
        for (int e = 0; e < 4; ++e)
          if (((midb >> e) & 1u) && o[e] < (uint32_t)cap) {
            bk[o[e]] = (RecKey<T>)key[e];
            bp[o[e]] = (uint32_t)(p + e);
          }
      }
    }
  }
  for (int off = 32; off > 0; off >>= 1) hcnt += __shfl_xor(hcnt, off, 64);
  if (lane == 0) s_hi[wave] = hcnt;
  if (bad) atomicOr(&sel->nonfinite, 1);
  __syncthreads();
  if (threadIdx.x == 0) {
    rcnt[2 * blockIdx.x] = (int32_t)s_mid;
    uint32_t hsum = 0;
    for (int i = 0; i < kSplitThreads / 64; ++i) hsum += s_hi[i];
    rcnt[2 * blockIdx.x + 1] = (int32_t)hsum;
  }
}

template <typename T>
__global__ __launch_bounds__(kSplitThreads) void k_sel_split(const T* __restrict__ vals, const uint32_t* __restrict__ excl,
                                                             int64_t n, int64_t eb, int cap, SelState* sel,
                                                             RecKey<T>* __restrict__ rkey, uint32_t* __restrict__ rpos,
                                                             int32_t* __restrict__ rcnt, uint32_t* __restrict__ out_bits) {
  sel_split_body<T>(vals, excl, n, eb, cap, sel, rkey, rpos, rcnt, out_bits);
}
// OR of a value over each aligned group of eight lanes, by cross-lane moves
// within quads and the mirror within half-rows (no LDS round trip).
__device__ __forceinline__ uint32_t or8(uint32_t w) {
  w |= (uint32_t)__builtin_amdgcn_update_dpp(0, (int)w, 0xB1, 0xF, 0xF, false);    // quad lanes 1 0 3 2
  w |= (uint32_t)__builtin_amdgcn_update_dpp(0, (int)w, 0x4E, 0xF, 0xF, false);    // quad lanes 2 3 0 1
  w |= (uint32_t)__builtin_amdgcn_update_dpp(0, (int)w, 0x141, 0xF, 0xF, false);   // half-row mirror
  return w;
}

// The dense split for FP32 keys: the same work as sel_split_body with 32-bit
// keys, band and offsets within the workgroup's block (so address arithmetic
// stays 32-bit), the bitmap words assembled by cross-lane moves.
__global__ __launch_bounds__(kSplitThreads) void k_sel_split_f32(
    const float* __restrict__ vals, const uint32_t* __restrict__ excl, int64_t n, int64_t eb, int cap, SelState* sel,
    uint32_t* __restrict__ rkey, uint32_t* __restrict__ rpos, int32_t* __restrict__ rcnt,
    uint32_t* __restrict__ out_bits) {
  __shared__ uint32_t s_mid;
  __shared__ uint32_t s_hi[kSplitThreads / 64];
  if (threadIdx.x == 0) s_mid = 0u;
  __syncthreads();
  const uint32_t lo32 = (uint32_t)sel->t_lo, hi32 = (uint32_t)sel->t_hi;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int64_t b0 = (int64_t)blockIdx.x * eb;
  const uint32_t len = (uint32_t)(std::min<int64_t>(n, b0 + eb) - b0);   // a multiple of 32
  const float* __restrict__ vb = vals + b0;
  const uint32_t* __restrict__ xb = excl ? excl + (b0 >> 5) : nullptr;
  uint32_t* __restrict__ ob = out_bits + (b0 >> 5);
  uint32_t* __restrict__ bk = rkey + (int64_t)blockIdx.x * cap;
  uint32_t* __restrict__ bp = rpos + (int64_t)blockIdx.x * cap;
  uint32_t hcnt = 0;
  bool bad = false;
  constexpr int U = 4;                           // rounds in flight per iteration
  constexpr uint32_t R = kSplitThreads * 4;       // keys per round
  const uint32_t lo = (uint32_t)(wave * 256 + lane * 4);
  for (uint32_t r0 = 0; r0 < len; r0 += U * R) {
    float4 v[U];
    uint32_t xw[U];
#pragma unroll
    for (int u = 0; u < U; ++u) {     // a lane past the end re-reads the last four keys, marked excluded below
      const uint32_t off = r0 + u * R + lo;
      const uint32_t oc = off < len ? off : len - 4;
      v[u] = *reinterpret_cast<const float4*>(vb + oc);
      xw[u] = xb ? xb[oc >> 5] : 0u;
    }
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const uint32_t off = r0 + u * R + lo;
      const uint32_t ex = off < len ? (xw[u] >> (off & 31)) & 0xFu : 0xFu;
      const float vv[4] = {v[u].x, v[u].y, v[u].z, v[u].w};
      uint32_t key[4], hib = 0, midb = 0;
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        const uint32_t m = __float_as_uint(vv[e]) & 0x7FFFFFFFu;
        const bool x = (ex >> e) & 1u;
        bad |= !x && m >= 0x7F800000u;
        key[e] = x ? 0u : m + 1u;
        hib |= (uint32_t)(key[e] > hi32) << e;
        midb |= (uint32_t)(key[e] >= lo32 && key[e] <= hi32) << e;
      }
      // eight lanes hold the 32 bits of one word
      const uint32_t w = or8(hib << ((lane & 7) * 4));
      if ((lane & 7) == 0 && off < len) ob[off >> 5] = w;
      hcnt += __popc(hib);
      // each lane's band keys (at most four) at its exclusive prefix in the wave
      const uint32_t cnt = __popc(midb);
      if (__ballot(cnt != 0)) {
        const uint64_t c0 = __ballot(cnt & 1u), c1 = __ballot(cnt & 2u), c2 = __ballot(cnt & 4u);
        const uint32_t tot = (uint32_t)(__popcll(c0) + 2 * __popcll(c1) + 4 * __popcll(c2));
        uint32_t base = 0;
        if (lane == 0) base = atomicAdd(&s_mid, tot);
        base = __shfl(base, 0, 64);
        uint32_t o = base + lane_prefix(c0) + 2 * lane_prefix(c1) + 4 * lane_prefix(c2);
        const uint32_t pos = (uint32_t)b0 + off;
#pragma unroll
        for (int e = 0; e < 4; ++e)
          if ((midb >> e) & 1u) {
            if (o < (uint32_t)cap) {
              bk[o] = key[e];
              bp[o] = pos + (uint32_t)e;
            }
            ++o;
          }
      }
    }
  }
  for (int off = 32; off > 0; off >>= 1) hcnt += __shfl_xor(hcnt, off, 64);
  if (lane == 0) s_hi[wave] = hcnt;
  if (bad) atomicOr(&sel->nonfinite, 1);
  __syncthreads();
  if (threadIdx.x == 0) {
    rcnt[2 * blockIdx.x] = (int32_t)s_mid;
    uint32_t hsum = 0;
    for (int i = 0; i < kSplitThreads / 64; ++i) hsum += s_hi[i];
    rcnt[2 * blockIdx.x + 1] = (int32_t)hsum;
  }
}

// Dense source: totals of the split.  Candidates come from the segments when
// fewer than K keys lie above the band and the band holds the rest (or every
// admissible key), and no segment overflowed; otherwise from every key.
// Every thread of the workgroup calls it; thread 0 stores the result.
__device__ __forceinline__ void sel_decide(const SelState* sel, const int32_t* __restrict__ rcnt, int nseg, int cap,
                                           int keybits, bool force_dense, SelHead* out) {
  double mid = 0.0, hi = 0.0, over = 0.0;
  for (int i = threadIdx.x; i < nseg; i += blockDim.x) {
    const int32_t m = rcnt[2 * i], h = rcnt[2 * i + 1];
    mid += m;
    hi += h;
    over += (m > cap) ? 1.0 : 0.0;
  }
  mid = block_sum_any(mid);
  hi = block_sum_any(hi);
  over = block_sum_any(over);
  if (threadIdx.x != 0) return;
  SelHead& hd = *out;
  const uint64_t t_lo = sel->t_lo, t_hi = sel->t_hi;
  const int64_t K = sel->k, nh = (int64_t)hi, nm = (int64_t)mid;
  hd.tie = 0;
  hd.pending = 0;
  const bool ok = !force_dense && over == 0.0 && nh <= K && (nh + nm >= K || t_lo == 1);
  if (!ok) {
    hd.mode = SEL_DENSE;
    hd.need = K;
    hd.prefix = 0;
    hd.pmask = 0;
    hd.bit = keybits;
    return;
  }
  hd.need = std::min<int64_t>(K - nh, nm);
  hd.mode = hd.need == 0 ? SEL_NONE : SEL_SEG;
  hd.bit = 0;
  hd.prefix = t_hi;
  hd.pmask = ~0ull;
  if (hd.need == 0) return;
  const uint64_t x = t_lo ^ t_hi;   // bits above the highest differing one are shared by the band
  if (x == 0) {
    hd.tie = hd.need < nm ? 1 : 0;   // every candidate has the key t_hi
  } else {
    const int b = 64 - __clzll((long long)x);
    hd.bit = b;
    hd.pmask = b >= 64 ? 0ull : ~((1ull << b) - 1);
    hd.prefix = t_hi & hd.pmask;
  }
}

// Every workgroup (1024 threads, kBins / 1024 bins each) reads the histogram
// row of the previous pass and fixes the digit (high to low) that holds the
// need-th candidate; all workgroups reach the same state.
__device__ __forceinline__ void sel_pick(SelHead& hd, const uint32_t* __restrict__ row, int64_t* sc) {
  constexpr int BPT = kBins / 1024;
  const int w = hd.bit < kDigit ? hd.bit : kDigit, shift = hd.bit - w;
  const int nb = 1 << w;
  const int t = threadIdx.x;
  uint32_t c[BPT];
#pragma unroll
  for (int u = 0; u < BPT; ++u) {
    const int q = BPT * t + u;
    c[u] = q < nb ? row[nb - 1 - q] : 0u;
  }
  int64_t loc = 0;
#pragma unroll
  for (int u = 0; u < BPT; ++u) loc += c[u];
  const int64_t incl = block_incl_scan(loc, sc), need = hd.need;
  int64_t run = incl - loc;
  __syncthreads();   // every thread has read hd.need
  if (run < need && need <= incl) {
#pragma unroll
    for (int u = 0; u < BPT; ++u) {
      if (run < need && need <= run + c[u]) {
        const uint64_t d = (uint64_t)(nb - 1 - (BPT * t + u));
        const int64_t rest = need - run;
        hd.need = rest;
        hd.prefix |= d << shift;
        hd.pmask |= (uint64_t)(nb - 1) << shift;
        hd.bit = shift;
        if (shift == 0) hd.tie = rest < (int64_t)c[u] ? 1 : 0;
      }
      run += c[u];
    }
  }
  if (t == 0) hd.pending = 0;
  __syncthreads();
}

// Clears row r of the rotation (spread over the grid).
__device__ __forceinline__ void sel_clear_row(uint32_t* __restrict__ hrows, int r) {
  uint32_t* row = hrows + (int64_t)r * kBins;
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < kBins; i += gridDim.x * blockDim.x) row[i] = 0u;
}

// One radix pass p (1024 threads per workgroup, at most kPassBlocks
// workgroups).  Reads the state left by pass p-1, picks the digit its
// histogram row fixes, and if key bits remain unresolved adds the histogram of
// the next digit (up to kDigit bits) among the candidates matching the prefix
// into row p mod 3.  State is double-buffered by pass parity.
// init = 1 (first pass over a dense split) decides the source (init = 3: the
// same, but always every key: the fallback, for tests); init = 2 starts a
// selection over a list of k entries.  Segments are read one
// wavefront per segment.
template <typename T>
__global__ __launch_bounds__(1024) void k_sel_pass(const T* __restrict__ vals, const void* __restrict__ aux,
                                                   int64_t count, SelState* sel, const RecKey<T>* __restrict__ rkey,
                                                   const int32_t* __restrict__ rcnt, int nseg, int cap,
                                                   uint32_t* __restrict__ hrows, int p, int init, int64_t k,
                                                   int keybits) {
  __shared__ uint32_t h[kBins];
  __shared__ SelHead hd;
  __shared__ int64_t sc[16];
  if (init == 1 || init == 3) {
    sel_decide(sel, rcnt, nseg, cap, keybits, init == 3, &hd);
  } else if (threadIdx.x == 0) {
    if (init == 2) {
      hd.mode = SEL_LIST; hd.need = k; hd.prefix = 0; hd.pmask = 0; hd.bit = keybits; hd.tie = 0; hd.pending = 0;
    } else {
      hd = sel->head[p & 1];
    }
  }
  __syncthreads();
  if (hd.pending) sel_pick(hd, hrows + (int64_t)((p + 2) % 3) * kBins, sc);
  sel_clear_row(hrows, (p + 1) % 3);
  const bool active = hd.mode != SEL_NONE && hd.bit > 0;
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    SelHead o = hd;
    o.pending = active ? 1 : 0;
    sel->head[(p + 1) & 1] = o;
    if (init == 2) sel->nonfinite = 0;
    if (init) sel->below = 0;   // read by the final pass, a later launch
  }
  if (!active) return;
  const int mode = hd.mode;
  const int w = hd.bit < kDigit ? hd.bit : kDigit, shift = hd.bit - w;
  const uint32_t dm = (1u << w) - 1;
  for (uint32_t i = threadIdx.x; i <= dm; i += blockDim.x) h[i] = 0u;
  __syncthreads();
  const uint64_t prefix = hd.prefix, pmask = hd.pmask;
  auto add = [&](uint64_t key) {
    if ((key & pmask) == prefix) atomicAdd(&h[(uint32_t)(key >> shift) & dm], 1u);
  };
  if (mode == SEL_SEG) {
    const int lane = threadIdx.x & 63;
    const int nw = (int)(gridDim.x * (blockDim.x >> 6));
    for (int sg = blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6); sg < nseg; sg += nw) {
      const int c = std::min(rcnt[2 * sg], cap);
      const int64_t o = (int64_t)sg * cap;
      for (int i = lane; i < c; i += 64) add((uint64_t)rkey[o + i]);
    }
  } else {
    const int64_t st = (int64_t)gridDim.x * blockDim.x;
    if (mode == SEL_DENSE) {
      const uint32_t* excl = (const uint32_t*)aux;
      for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < count; i += st)
        add(dense_key(vals, excl, i));
    } else {
      for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < count; i += st) add(mag_bits(vals[i]) + 1);
    }
  }
  __syncthreads();
  uint32_t* row = hrows + (int64_t)(p % 3) * kBins;
  for (uint32_t i = threadIdx.x; i <= dm; i += blockDim.x) {
    const uint32_t v = h[i];
    if (v) atomicAdd(&row[i], v);
  }
}

// Final pass: picks the last digit, then marks the selected candidates: every
// key above the threshold tau, and the keys equal to tau (all of them, or, when
// more share tau than are still needed, the ones with the lowest natural
// indices).  Segments and lists set bits atomically; the dense source
// rewrites every word.  Ties are resolved by workgroup 0 alone: the tied
// candidates are collected and sorted by index in LDS, or, beyond kTieCap of
// them, found by a radix select over their indices.
template <typename T>
__global__ __launch_bounds__(1024) void k_sel_final(const T* __restrict__ vals, const void* __restrict__ aux,
                                                    int64_t count, int64_t words, const Plan pl, SelState* sel,
                                                    const RecKey<T>* __restrict__ rkey,
                                                    const uint32_t* __restrict__ rpos,
                                                    const int32_t* __restrict__ rcnt, int nseg, int cap,
                                                    uint32_t* __restrict__ hrows, int p, int jbits,
                                                    uint32_t* __restrict__ bits) {
  __shared__ SelHead hd;
  __shared__ int64_t sc[16];
  __shared__ uint64_t tb[kTieCap];
  __shared__ uint32_t th[kIdxBins];
  __shared__ uint32_t s_cnt, s_digit;
  __shared__ int64_t s_rest;
  if (threadIdx.x == 0) hd = sel->head[p & 1];
  __syncthreads();
  if (hd.pending) sel_pick(hd, hrows + (int64_t)((p + 2) % 3) * kBins, sc);
  sel_clear_row(hrows, (p + 1) % 3);
  const int mode = hd.mode;
  if (mode == SEL_NONE) return;
  const uint64_t tau = hd.prefix;
  const bool tie = hd.tie != 0;
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    sel->tau = tau;
    sel->tie_out = hd.tie;
  }
  const int lane = threadIdx.x & 63;
  const int nw = (int)(gridDim.x * (blockDim.x >> 6));
  const int64_t st = (int64_t)gridDim.x * blockDim.x;
  const uint32_t* excl = (const uint32_t*)aux;
  const int32_t* list = (const int32_t*)aux;
  // the largest admissible key below tau this thread sees (the first rejected
  // candidate, for the margin; not needed under a tie, whose margin is 0)
  uint64_t below = 0;
  auto seen = [&](uint64_t key) {
    if (key != 0 && key < tau && key > below) below = key;
  };
  // --- keys above tau (and equal to it without a tie)
  if (mode == SEL_DENSE) {
    if (tie && blockIdx.x != 0) return;   // workgroup 0 owns every word when it also resolves the tie
    const int64_t w0 = tie ? threadIdx.x : (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t ws = tie ? blockDim.x : st;
    for (int64_t w = w0; w < words; w += ws) {
      uint32_t word = 0;
      for (int e = 0; e < 32; ++e) {
        const int64_t q = w * 32 + e;
        if (q < count) {
          const uint64_t key = dense_key(vals, excl, q);
          seen(key);
          if (key != 0 && (key > tau || (key == tau && !tie))) word |= 1u << e;
        }
      }
      bits[w] = word;
    }
  } else if (mode == SEL_SEG) {
    for (int sg = blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6); sg < nseg; sg += nw) {
      const int c = std::min(rcnt[2 * sg], cap);
      const int64_t o = (int64_t)sg * cap;
      for (int i = lane; i < c; i += 64) {
        const uint64_t key = (uint64_t)rkey[o + i];
        seen(key);
        if (key > tau || (key == tau && !tie)) {
          const uint32_t q = rpos[o + i];
          atomicOr(&bits[q >> 5], 1u << (q & 31));
        }
      }
    }
  } else {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < count; i += st) {
      const uint64_t key = mag_bits(vals[i]) + 1;
      seen(key);
      if (key > tau || (key == tau && !tie)) {
        const uint32_t q = (uint32_t)list[i];
        atomicOr(&bits[q >> 5], 1u << (q & 31));
      }
    }
  }
  if (!tie) {
    for (int off = 32; off > 0; off >>= 1) {
      const uint64_t o = __shfl_down((unsigned long long)below, off, 64);
      below = o > below ? o : below;
    }
    // one atomic per workgroup: all of them target the same word
    __shared__ uint64_t s_below[16];
    if (lane == 0) s_below[threadIdx.x >> 6] = below;
    __syncthreads();
    if (threadIdx.x == 0) {
      uint64_t bm = 0;
      for (int i = 0; i < (int)(blockDim.x >> 6); ++i) bm = s_below[i] > bm ? s_below[i] : bm;
      if (bm) atomicMax((unsigned long long*)&sel->below, (unsigned long long)bm);
    }
  }
  if (!tie || blockIdx.x != 0 || tau == 0) return;   // key 0 (excluded) is never marked
  // --- tie: the need lowest natural indices among the keys equal to tau
  __syncthreads();
  __threadfence_block();
  const int64_t need = hd.need;
  // visits every (key, key position) of the source with this workgroup alone
  auto each = [&](auto&& f) {
    if (mode == SEL_SEG) {
      for (int sg = threadIdx.x >> 6; sg < nseg; sg += (int)(blockDim.x >> 6)) {
        const int c = std::min(rcnt[2 * sg], cap);
        const int64_t o = (int64_t)sg * cap;
        for (int i = lane; i < c; i += 64) f((uint64_t)rkey[o + i], rpos[o + i]);
      }
    } else if (mode == SEL_DENSE) {
      for (int64_t i = threadIdx.x; i < count; i += blockDim.x) f(dense_key(vals, excl, i), (uint32_t)i);
    } else {
      for (int64_t i = threadIdx.x; i < count; i += blockDim.x) f(mag_bits(vals[i]) + 1, (uint32_t)list[i]);
    }
  };
  if (threadIdx.x == 0) s_cnt = 0u;
  __syncthreads();
  each([&](uint64_t key, uint32_t q) {
    if (key == tau) {
      const uint32_t slot = atomicAdd(&s_cnt, 1u);
      if (slot < (uint32_t)kTieCap) tb[slot] = ((uint64_t)(uint32_t)nat_of_key(q, pl) << 32) | q;
    }
  });
  __syncthreads();
  const uint32_t nt = s_cnt;
  if (nt <= (uint32_t)kTieCap) {
    int P = 2;
    while (P < (int)nt) P <<= 1;
    for (int i = (int)nt + threadIdx.x; i < P; i += blockDim.x) tb[i] = ~0ull;
    __syncthreads();
    lds_bitonic(tb, P, false);
    for (int i = threadIdx.x; i < (int)need; i += blockDim.x) {
      const uint32_t q = (uint32_t)tb[i];
      atomicOr(&bits[q >> 5], 1u << (q & 31));
    }
    return;
  }
  // many tied keys: radix select (low indices first) over the tied indices
  uint32_t jprefix = 0u, jmask = 0u;
  int64_t rest = need;
  for (int bit = jbits; bit > 0;) {
    const int w = bit < kIdxDigit ? bit : kIdxDigit, shift = bit - w;
    const uint32_t dm = (1u << w) - 1;
    for (uint32_t i = threadIdx.x; i <= dm; i += blockDim.x) th[i] = 0u;
    __syncthreads();
    each([&](uint64_t key, uint32_t q) {
      if (key != tau) return;
      const uint32_t j = (uint32_t)nat_of_key(q, pl);
      if ((j & jmask) == jprefix) atomicAdd(&th[(j >> shift) & dm], 1u);
    });
    __syncthreads();
    const int t = threadIdx.x;
    int64_t c[2];
    c[0] = 2 * t <= (int)dm ? th[2 * t] : 0;
    c[1] = 2 * t + 1 <= (int)dm ? th[2 * t + 1] : 0;
    const int64_t loc = c[0] + c[1];
    const int64_t incl = block_incl_scan(loc, sc);
    int64_t run = incl - loc;
    if (run < rest && rest <= incl) {
#pragma unroll
      for (int u = 0; u < 2; ++u) {
        if (run < rest && rest <= run + c[u]) {
          s_digit = (uint32_t)(2 * t + u);
          s_rest = rest - run;
        }
        run += c[u];
      }
    }
    __syncthreads();
    const uint32_t d = s_digit;
    const int64_t nrest = s_rest;
    __syncthreads();
    jprefix |= d << shift;
    jmask |= dm << shift;
    rest = nrest;
    bit = shift;
  }
  each([&](uint64_t key, uint32_t q) {
    if (key == tau && (uint32_t)nat_of_key(q, pl) <= jprefix) atomicOr(&bits[q >> 5], 1u << (q & 31));
  });
}

static inline int index_bits(int64_t n) {
  int b = 0;
  while ((int64_t(1) << b) < n) ++b;
  return std::max(b, 1);
}

// The selection's margin: the K-th key minus the first rejected one (0 under a
// tie).  When the final pass saw no key below the threshold, a dense split's
// rejected keys all lie below the band, so tau minus the band's lower bound is
// a lower bound of the margin; a list or dense source had no rejected key.
// (A kernel of its own: a device-scope release in every workgroup of the final
// pass, so that its last one could note the margin, costs more than a launch.)
template <typename T>
__global__ void k_sel_margin(SelState* sel, int p) {
  if (threadIdx.x != 0) return;
  const SelHead hd = sel->head[p & 1];
  if (hd.mode == SEL_NONE || sel->tau == 0) return;
  const double vt = key_value<T>(sel->tau);
  if (sel->tie_out) {
    note_margin(&sel->mmin, &sel->mrel, 0.0, vt);
    return;
  }
  uint64_t b = sel->below;
  if (b == 0) {
    if (hd.mode != SEL_SEG) return;
    b = sel->t_lo;
  }
  note_margin(&sel->mmin, &sel->mrel, vt - key_value<T>(b), vt);
}

template <typename T>
static void sel_run(Ctx<T>& c, const T* vals, const void* aux, int64_t count, int init, int64_t k, int nseg,
                    int cap, unsigned grid, uint32_t* out_bits) {
  hipStream_t s = c.stream;
  const int keybits = 8 * (int)sizeof(T);
  const int passes = (keybits + kDigit - 1) / kDigit;
  for (int p = 0; p < passes; ++p) {
    hipLaunchKernelGGL((k_sel_pass<T>), dim3(grid), dim3(1024), 0, s, vals, aux, count, c.sel,
                       (const RecKey<T>*)c.rkey, c.rcnt, nseg, cap, c.hrows, p, p == 0 ? init : 0, k, keybits);
    CS_LAUNCH_CHECK();
  }
  hipLaunchKernelGGL((k_sel_final<T>), dim3(grid), dim3(1024), 0, s, vals, aux, count, c.plan.words, c.plan, c.sel,
                     (const RecKey<T>*)c.rkey, c.rpos, c.rcnt, nseg, cap, c.hrows, passes, index_bits(c.plan.n), out_bits);
  CS_LAUNCH_CHECK();
  hipLaunchKernelGGL((k_sel_margin<T>), dim3(1), dim3(64), 0, s, c.sel, passes);
  CS_LAUNCH_CHECK();
}

template <typename T>
void topk_dense(Ctx<T>& c, const T* dense, const uint32_t* excl, int k, uint32_t* out_bits) {
  hipStream_t s = c.stream;
  const int64_t n = c.plan.n;
  const SplitLayout sl = split_layout(n);
  hipLaunchKernelGGL((k_sel_sample<T>), dim3(1), dim3(1024), 0, s, dense, excl, n, (int64_t)k, 8 * (int)sizeof(T),
                     c.sel);
  CS_LAUNCH_CHECK();
  if constexpr (sizeof(T) == 4)
    hipLaunchKernelGGL(k_sel_split_f32, dim3(sl.blocks), dim3(kSplitThreads), 0, s, (const float*)dense, excl, n,
                       sl.per_block, sl.cap, c.sel, (uint32_t*)c.rkey, c.rpos, c.rcnt, out_bits);
  else
    hipLaunchKernelGGL((k_sel_split<T>), dim3(sl.blocks), dim3(kSplitThreads), 0, s, dense, excl, n, sl.per_block,
                       sl.cap, c.sel, (RecKey<T>*)c.rkey, c.rpos, c.rcnt, out_bits);
  CS_LAUNCH_CHECK();
  const unsigned grid = (unsigned)std::min(kPassBlocks, sl.blocks);
  // CS_SELECT_DENSE set: take the every-key fallback regardless of the band
  // (a test hook; the band's own checks make the fallback rare)
  const bool force = std::getenv("CS_SELECT_DENSE") != nullptr;
  sel_run<T>(c, dense, excl, n, force ? 3 : 1, k, sl.blocks, sl.cap, grid, out_bits);
}

template <typename T>
void topk_compact(Ctx<T>& c, const T* vals, const int32_t* list, int count, int k, uint32_t* out_bits) {
  fill_u32(out_bits, c.plan.words, 0u, c.stream);
  const unsigned grid = (unsigned)std::min<int64_t>(kPassBlocks, nblk(count, 1024));
  sel_run<T>(c, vals, list, count, 2, k, 0, 0, grid, out_bits);
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
void bits_differ(const uint32_t* a, const uint32_t* b, int64_t words, int32_t* flag, hipStream_t s) {
  fill<int32_t>(flag, 1, 0, s);
  hipLaunchKernelGGL(k_bits_diff, dim3(nblk(words, 256)), dim3(256), 0, s, a, b, words, flag);
  CS_LAUNCH_CHECK();
}

uint32_t bits_differ_post(const uint32_t* a, const uint32_t* b, int64_t words, int32_t* scratch, int slot,
                          hipStream_t s) {
  fill<int32_t>(scratch, 1, 0, s);
  hipLaunchKernelGGL(k_bits_diff, dim3(nblk(words, 256)), dim3(256), 0, s, a, b, words, scratch);
  CS_LAUNCH_CHECK();
  return dev_post(s, scratch, sizeof(int32_t), slot);
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
__global__ void k_bits_write(const uint32_t* __restrict__ bits, int64_t words, uint32_t* __restrict__ cnt,
                             int32_t* __restrict__ list, int limit, uint32_t* __restrict__ wpre) {
  bits_write_body(bits, words, cnt, list, limit, wpre, blockIdx.x, gridDim.x);
}

template <typename T>
int bits_to_list(Ctx<T>& c, const uint32_t* bits, int32_t* list, int expect, uint32_t* wpre) {
  const int64_t words = c.plan.words;
  const int nb = (int)((words + kBitsPerBlockWords - 1) / kBitsPerBlockWords);
  hipStream_t s = c.stream;
  hipLaunchKernelGGL(k_bits_count, dim3(nb), dim3(256), 0, s, bits, words, c.blockcnt);
  CS_LAUNCH_CHECK();
  hipLaunchKernelGGL(k_bits_write, dim3(nb), dim3(256), 0, s, bits, words, c.blockcnt, list, expect, wpre);
  CS_LAUNCH_CHECK();
  return nb;   // total count is left in blockcnt[nb]
}

#define CS_INST(T)                                                                        \
  template void argmax_excl<T>(Ctx<T>&, const T*, const uint32_t*, int32_t*, const double*, double); \
  template void sel_reset<T>(Ctx<T>&);                                                  \
  template void margins_read<T>(Ctx<T>&, double*, double*);                             \
  template void topk_dense<T>(Ctx<T>&, const T*, const uint32_t*, int, uint32_t*);      \
  template void topk_compact<T>(Ctx<T>&, const T*, const int32_t*, int, int, uint32_t*); \
  template int bits_to_list<T>(Ctx<T>&, const uint32_t*, int32_t*, int, uint32_t*);
CS_INST(float)
CS_INST(double)

}  // namespace csr
