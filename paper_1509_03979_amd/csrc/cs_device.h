// Device helpers shared by the selection, CG and batched-driver units:
// magnitude keys, block reductions, and the bitmap-to-list compaction bodies.
#pragma once

#include "cs_internal.h"

namespace csr {

// IEEE bit pattern of |v|: orders like the value for non-negative numbers.
template <typename T> __device__ __forceinline__ uint64_t mag_bits(T v);
template <> __device__ __forceinline__ uint64_t mag_bits<float>(float v) { return (uint64_t)__float_as_uint(fabsf(v)); }
template <> __device__ __forceinline__ uint64_t mag_bits<double>(double v) {
  return (uint64_t)__double_as_longlong(fabs(v));
}
template <typename T> __device__ __forceinline__ bool finite_v(T v) { return isfinite(v); }

__device__ __forceinline__ bool bit_of(const uint32_t* __restrict__ b, int64_t j) {
  return (b[j >> 5] >> (j & 31)) & 1u;
}

__device__ __forceinline__ bool key_gt(const ArgKey& a, const ArgKey& b) {
  return a.hi > b.hi || (a.hi == b.hi && a.lo > b.lo);
}

__device__ __forceinline__ ArgKey shfl_down_key(ArgKey k, int off) {
  ArgKey r;
  r.hi = __shfl_down((unsigned long long)k.hi, off, 64);
  r.lo = __shfl_down(k.lo, off, 64);
  r.pad = 0;
  return r;
}

// Block-wide max of ArgKey (any block size up to 1024); result valid in thread 0.
__device__ __forceinline__ ArgKey block_max_key(ArgKey best) {
  __shared__ ArgKey sh[16];
  for (int off = 32; off > 0; off >>= 1) {
    ArgKey o = shfl_down_key(best, off);
    if (key_gt(o, best)) best = o;
  }
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  if (lane == 0) sh[wave] = best;
  __syncthreads();
  if (threadIdx.x == 0) {
    for (int i = 1; i < (int)(blockDim.x >> 6); ++i)
      if (key_gt(sh[i], best)) best = sh[i];
  }
  __syncthreads();
  return best;
}

// The best two (hi, lo) keys, held as scalars so they stay in registers (keys
// are distinct: the index part differs).  K2::add merges the pair (oh, ol) >=
// (o2h, o2l) into (best, second).
__device__ __forceinline__ bool kgt(uint64_t ah, uint32_t al, uint64_t bh, uint32_t bl) {
  return ah > bh || (ah == bh && al > bl);
}
struct K2 {
  uint64_t bh = 0, sh = 0;
  uint32_t bl = 0, sl = 0;
  __device__ __forceinline__ void add(uint64_t oh, uint32_t ol, uint64_t o2h = 0, uint32_t o2l = 0) {
    const bool gt = kgt(oh, ol, bh, bl);
    // new second: max(old best, o2) when o wins, else max(old second, o)
    const uint64_t ch = gt ? bh : sh, dh = gt ? o2h : oh;
    const uint32_t cl = gt ? bl : sl, dl = gt ? o2l : ol;
    const bool c = kgt(ch, cl, dh, dl);
    sh = c ? ch : dh;
    sl = c ? cl : dl;
    bh = gt ? oh : bh;
    bl = gt ? ol : bl;
  }
  __device__ __forceinline__ ArgKey best() const { return ArgKey{bh, bl, 0}; }
  __device__ __forceinline__ ArgKey second() const { return ArgKey{sh, sl, 0}; }
};

// Block-wide best two (any block size up to 1024); valid in thread 0.
__device__ __forceinline__ void block_max_key2(K2& t) {
  __shared__ uint64_t sbh[16], ssh[16];
  __shared__ uint32_t sbl[16], ssl[16];
  for (int off = 32; off > 0; off >>= 1) {
    const uint64_t oh = __shfl_down((unsigned long long)t.bh, off, 64);
    const uint32_t ol = __shfl_down(t.bl, off, 64);
    const uint64_t o2h = __shfl_down((unsigned long long)t.sh, off, 64);
    const uint32_t o2l = __shfl_down(t.sl, off, 64);
    t.add(oh, ol, o2h, o2l);
  }
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  if (lane == 0) {
    sbh[wave] = t.bh; sbl[wave] = t.bl;
    ssh[wave] = t.sh; ssl[wave] = t.sl;
  }
  __syncthreads();
  if (threadIdx.x == 0)
    for (int i = 1; i < (int)(blockDim.x >> 6); ++i) t.add(sbh[i], sbl[i], ssh[i], ssl[i]);
  __syncthreads();
}

// Value of a magnitude key (bits(|v|) + 1, 0: none) in the precision of T.
template <typename T> __device__ __forceinline__ double key_value(uint64_t key);
template <> __device__ __forceinline__ double key_value<float>(uint64_t key) {
  return key ? (double)__uint_as_float((uint32_t)(key - 1)) : 0.0;
}
template <> __device__ __forceinline__ double key_value<double>(uint64_t key) {
  return key ? __longlong_as_double((long long)(key - 1)) : 0.0;
}

// Records a decision margin (gap between the last chosen and the first
// rejected key) and its size relative to the chosen key (one thread).
__device__ __forceinline__ void note_margin(double* mmin, double* mrel, double margin, double key) {
  if (!(margin >= 0.0)) return;
  if (margin < *mmin) *mmin = margin;
  const double rel = key > 0.0 ? margin / key : (margin == 0.0 ? 0.0 : __builtin_huge_val());   // a tie is 0
  if (rel < *mrel) *mrel = rel;
}

// Block sum in a fixed order, broadcast to every thread (any block size up to
// 1024, a multiple of 64).
__device__ __forceinline__ double block_sum_any(double v) {
  __shared__ double sh[16];
  __shared__ double res;
  for (int off = 32; off > 0; off >>= 1) v += __shfl_down(v, off, 64);
  if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = v;
  __syncthreads();
  if (threadIdx.x == 0) {
    double s = 0.0;
    for (int i = 0; i < (int)(blockDim.x >> 6); ++i) s += sh[i];
    res = s;
  }
  __syncthreads();
  const double r = res;
  __syncthreads();
  return r;
}

// ------------------------------------------------------------------ OMPR drop step
// Candidates I u {j}: z_i = x'_i + eta c_i on the support (compact x' and the
// key-order correlation c = F^T D^T r, sign-flipped coordinates), z_j = eta
// c_j for the entering index j (natural, < 0: none).  The dropped element is
// the last under (|z| desc, index asc): the smallest |z|, ties to the larger
// index, found as a max-reduction over (~bits(|z|), index).  Returns the
// dropped natural index in thread 0 (any block size up to 1024).
__device__ __forceinline__ bool dkey_gt(uint64_t ah, uint32_t al, uint64_t bh, uint32_t bl) {
  return ah > bh || (ah == bh && al > bl);
}

// With margin/mkey non-null, thread 0 also stores the gap between the
// smallest and the next smallest |z| (the drop decision's margin) and that
// next smallest |z|.
template <typename T>
__device__ __forceinline__ int32_t ompr_drop_body(const T* __restrict__ x, const int32_t* __restrict__ list, int k,
                                                  const T* __restrict__ cc, const Plan& pl, T eta, int32_t jn,
                                                  double* margin = nullptr, double* mkey = nullptr) {
  K2 t;   // best two of (~bits(|z|), index): the smallest |z|, then the next
  // Rounds of U slots per thread: the list and x loads of a round, then its
  // correlation loads, are all issued before any is used, and none sits under
  // a per-lane branch (a slot past the end reads slot k - 1 or key 0 and is
  // dropped afterwards), so the round waits on two load latencies, not 2U.
  constexpr int U = 4;
  const int bd = blockDim.x;
  const int64_t kjn = jn >= 0 ? key_of_nat(jn, pl) : 0;
  for (int i0 = threadIdx.x; i0 <= k; i0 += U * bd) {
    int64_t key[U];
    T xv[U];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int i = i0 + u * bd;
      const int li = i < k ? i : k - 1;
      const int64_t kl = list[li];
      const T xl = x[li];
      key[u] = i < k ? kl : kjn;
      xv[u] = i < k ? xl : (T)0;
    }
    T cv[U];
#pragma unroll
    for (int u = 0; u < U; ++u) cv[u] = cc[key[u]];   // sign_j (A^T r)_j
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int i = i0 + u * bd;
      if (i < k || (i == k && jn >= 0)) {
        const int64_t j = i < k ? nat_of_key(key[u], pl) : (int64_t)jn;
        t.add(~mag_bits(xv[u] + eta * cv[u]), (uint32_t)j);
      }
    }
  }
  block_max_key2(t);
  __shared__ uint32_t s_drop;
  if (threadIdx.x == 0) {
    s_drop = t.bl;
    if (margin && t.sh != 0) {   // a second candidate exists (0 is never a real ~bits key)
      const double zmin = key_value<T>(~t.bh + 1), z2 = key_value<T>(~t.sh + 1);
      *margin = z2 - zmin;
      *mkey = z2;
    } else if (margin) {
      *margin = -1.0;
    }
  }
  __syncthreads();
  const uint32_t bl = s_drop;
  return (int32_t)bl;
}

// ------------------------------------------------------------------ bitmap -> ascending index list
// Block b covers words [1024 b, 1024 b + 1024): count its set bits (256 threads).
__device__ __forceinline__ void bits_count_body(const uint32_t* __restrict__ bits, int64_t words,
                                                uint32_t* __restrict__ cnt, int b) {
  __shared__ uint32_t red[4];
  const int64_t w0 = (int64_t)b * kBitsPerBlockWords;
  uint32_t s = 0;
  for (int i = threadIdx.x; i < kBitsPerBlockWords; i += blockDim.x) {
    const int64_t w = w0 + i;
    if (w < words) s += __popc(bits[w]);
  }
  for (int off = 32; off > 0; off >>= 1) s += __shfl_down(s, off, 64);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = s;
  __syncthreads();
  if (threadIdx.x == 0) cnt[b] = red[0] + red[1] + red[2] + red[3];
}

// Block b (256 threads, 4 words each) writes the indices of its set bits at
// their ranks (at most `limit` of them) and, per word, the number of set bits
// in all earlier words (wpre, nullable).  The block's first rank is the sum of
// the earlier blocks' counts cnt[0..b), taken here rather than by a scan pass;
// the last block (b = nb - 1) also stores the total in cnt[nb].
__device__ __forceinline__ void bits_write_body(const uint32_t* __restrict__ bits, int64_t words,
                                                uint32_t* __restrict__ cnt, int32_t* __restrict__ list,
                                                int limit, uint32_t* __restrict__ wpre, int b, int nb) {
  __shared__ uint32_t sh[256];
  __shared__ uint32_t wsum[4];
  const int64_t w0 = (int64_t)b * kBitsPerBlockWords + threadIdx.x * 4;
  uint32_t wv[4];
  uint32_t mine = 0;
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    wv[q] = (w0 + q < words) ? bits[w0 + q] : 0u;
    mine += __popc(wv[q]);
  }
  uint32_t pre = 0;
  for (int i = threadIdx.x; i < b; i += blockDim.x) pre += cnt[i];
  for (int off = 32; off > 0; off >>= 1) pre += __shfl_down(pre, off, 64);
  if ((threadIdx.x & 63) == 0) wsum[threadIdx.x >> 6] = pre;
  sh[threadIdx.x] = mine;
  __syncthreads();
  const uint32_t base = wsum[0] + wsum[1] + wsum[2] + wsum[3];
  for (int off = 1; off < 256; off <<= 1) {
    uint32_t t = (threadIdx.x >= (unsigned)off) ? sh[threadIdx.x - off] : 0u;
    __syncthreads();
    sh[threadIdx.x] += t;
    __syncthreads();
  }
  if (b == nb - 1 && threadIdx.x == 255) cnt[nb] = base + sh[255];
  uint32_t pos = base + sh[threadIdx.x] - mine;
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    if (wpre && w0 + q < words) wpre[w0 + q] = pos;
    uint32_t v = wv[q];
    while (v) {
      const int bit = __ffs(v) - 1;
      v &= v - 1;
      if ((int)pos < limit) list[pos] = (int32_t)((w0 + q) * 32 + bit);
      ++pos;
    }
  }
}

// ------------------------------------------------------------------ fused CG step
// Four workgroup sums at once, valid in thread 0: shuffle trees within each
// wave, then across the waves' totals in wave 0 (NW <= 16 waves).
// A wave that holds no data (`wave_has` false, uniform per wave) skips its
// shuffles and contributes zeros.
template <int NW>
__device__ __forceinline__ double4 wg_sum4(double a, double b, double c, double d, double (&red)[4][NW],
                                           bool wave_has = true) {
  if (wave_has) {
    for (int off = 32; off > 0; off >>= 1) {
      a += __shfl_down(a, off, 64);
      b += __shfl_down(b, off, 64);
      c += __shfl_down(c, off, 64);
      d += __shfl_down(d, off, 64);
    }
  }
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  if (lane == 0) {
    red[0][w] = a;
    red[1][w] = b;
    red[2][w] = c;
    red[3][w] = d;
  }
  __syncthreads();
  double4 s = make_double4(0.0, 0.0, 0.0, 0.0);
  if (w == 0) {
    if (lane < NW) s = make_double4(red[0][lane], red[1][lane], red[2][lane], red[3][lane]);
    for (int off = 8; off > 0; off >>= 1) {
      s.x += __shfl_down(s.x, off, 64);
      s.y += __shfl_down(s.y, off, 64);
      s.z += __shfl_down(s.z, off, 64);
      s.w += __shfl_down(s.w, off, 64);
    }
  }
  __syncthreads();
  return s;
}

// The scalar CG step of iteration `it` from the inner products of its current
// residual r and direction d with q = H d (sum = {d^T q, r^T r, r^T q, q^T q}):
// alpha = r^T r / d^T q, and the next residual's norm without a second pass,
// |r - alpha q|^2 = r^T r - 2 alpha r^T q + alpha^2 q^T q.  r^T r is summed
// afresh every iteration, so the expansion's rounding never accumulates.
// alpha is rounded to the vector precision first, since that is the step the
// vectors take.  Breakdown (d^T q not positive) stops with alpha = 0.
template <typename T>
__device__ __forceinline__ void cg_step_fused(CgScalars* cg, double4 sum, int it, int max_iter, T) {
  const double dq = sum.x, rr = sum.y;
  cg->dq = dq;
  cg->rr[it & 1] = rr;
  if (!(dq > 0.0) || !isfinite(dq)) {            // H not positive on d (Theorem 3's condition fails)
    cg->alpha = 0.0;
    cg->flags |= CS_F_CG_BREAKDOWN;
    cg->done = 1;
    return;
  }
  const double alpha = (double)(T)(rr / dq);
  double rr_new = rr - 2.0 * alpha * sum.z + alpha * alpha * sum.w;
  if (rr_new < 0.0) rr_new = 0.0;                // rounding below an exact zero residual
  const bool fin = isfinite(rr_new);
  cg->alpha = alpha;
  cg->rr[(it + 1) & 1] = rr_new;
  cg->beta = rr > 0.0 ? rr_new / rr : 0.0;
  cg->iters = it + 1;
  if (!fin) cg->flags |= CS_F_NONFINITE;
  if (!fin || rr_new <= cg->tol2 * cg->ref || it + 1 >= max_iter) cg->done = 1;
}

}  // namespace csr
