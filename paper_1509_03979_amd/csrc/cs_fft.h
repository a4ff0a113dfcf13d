// Workgroup-cooperative FFTs held in LDS, with every size, stride and thread
// count fixed at compile time.
//
// A set of CNT independent length-N FFTs sits in LDS.  Two layouts are used:
//   column-major (CM): element e of FFT f at e * CNT + f  (column strips)
//   row-major:         element e of FFT f at e + f * N    (row pairs)
// The transform is a sequence of Stockham autosort stages (Govindaraju et al.,
// SC'08 formulation): the stage of span NS reads the R inputs of butterfly j
// at j + r N/R, multiplies input r by W_{NS R}^{r (j mod NS)}, does an R-point
// DFT in registers and writes output r to (j / NS) NS R + (j mod NS) + r NS.
// Radix 16 (or the per-thread element count, if smaller) while enough bits
// remain, then one smaller stage.  A stage
// reads all its inputs into registers, synchronises, then writes in place.
// Output is in natural order.  Forward uses exp(-2 pi i ...), inverse
// exp(+2 pi i ...), both unnormalised.
//
// LDS addresses are padded by one element every 16 (lp): radix-16 writes
// have a 16-element lane stride, which unpadded sends a wave's lanes to the
// same banks.  Because every displacement used below is either a multiple
// of 16 or smaller than 16 from a 16-aligned base, lp(base + d) = lp(base)
// + d + d/16, so each access is a per-thread base plus an immediate offset.
//
// Stage twiddles come from a per-size table laid out stage after stage, each
// stage as [k][r-1] = W_{NS R}^{r k} (k < NS, 1 <= r < R), so the R-1 factors
// of a butterfly are contiguous.
#pragma once

#include "cs_internal.h"

namespace csr {

__device__ __forceinline__ int lp(int a) { return a + (a >> 4); }
__host__ __device__ constexpr int lp_size(int n) { return n + (n >> 4) + 1; }

// Radix of the stage at span 2^logns: the largest of 16 / 8 / 4 / 2 that does not
// exceed 2^loge (the elements each thread holds) or the bits that remain.
__host__ __device__ constexpr int stage_lr(int logn, int logns, int loge) {
  const int cap = loge < 4 ? loge : 4;
  return (logn - logns) >= cap ? cap : (logn - logns);
}
__host__ __device__ constexpr int tw_stage_count(int logn, int logns, int loge) {
  return logns == 0 ? 0 : (1 << logns) * ((1 << stage_lr(logn, logns, loge)) - 1);
}
// offset of stage `logns` in the table of size-2^logn FFTs
__host__ __device__ constexpr int tw_stage_offset(int logn, int logns, int loge) {
  int off = 0, ns = 0;
  while (ns < logns) {
    off += tw_stage_count(logn, ns, loge);
    ns += stage_lr(logn, ns, loge);
  }
  return off;
}
__host__ __device__ constexpr int tw_table_count(int logn, int loge) { return tw_stage_offset(logn, logn, loge); }

// threads per workgroup for E elements at 2^loge per thread (one wave to 1024 threads)
__host__ __device__ constexpr int nt_for(int e, int loge) {
  return (e >> loge) < 64 ? 64 : ((e >> loge) > 1024 ? 1024 : (e >> loge));
}

template <typename T, bool INV>
__device__ __forceinline__ Cx<T> mul_mi(Cx<T> a) {   // a * (-i) forward, a * (+i) inverse
  return INV ? cx(-a.im, a.re) : cx(a.im, -a.re);
}

template <typename T, bool INV>
__device__ __forceinline__ void dft2(Cx<T>& a0, Cx<T>& a1) {
  Cx<T> t = a0 - a1;
  a0 = a0 + a1;
  a1 = t;
}

template <typename T, bool INV>
__device__ __forceinline__ void dft4(Cx<T>& a0, Cx<T>& a1, Cx<T>& a2, Cx<T>& a3) {
  Cx<T> t0 = a0 + a2, t1 = a0 - a2, t2 = a1 + a3, t3 = mul_mi<T, INV>(a1 - a3);
  a0 = t0 + t2;
  a2 = t0 - t2;
  a1 = t1 + t3;
  a3 = t1 - t3;
}

// 8-point DFT: two 4-point DFTs on the even/odd inputs, combined with W_8^k.
template <typename T, bool INV>
__device__ __forceinline__ void dft8(Cx<T>* a) {
  const T h = (T)0.70710678118654752440;
  dft4<T, INV>(a[0], a[2], a[4], a[6]);
  dft4<T, INV>(a[1], a[3], a[5], a[7]);
  Cx<T> o1 = a[3], o2 = a[5], o3 = a[7];
  // W_8^1 = (1 - i)/sqrt2 forward, (1 + i)/sqrt2 inverse
  o1 = INV ? cx(h * (o1.re - o1.im), h * (o1.re + o1.im)) : cx(h * (o1.re + o1.im), h * (o1.im - o1.re));
  o2 = mul_mi<T, INV>(o2);
  // W_8^3 = (-1 - i)/sqrt2 forward, (-1 + i)/sqrt2 inverse
  o3 = INV ? cx(-h * (o3.re + o3.im), h * (o3.re - o3.im)) : cx(h * (o3.im - o3.re), -h * (o3.re + o3.im));
  Cx<T> e0 = a[0], e1 = a[2], e2 = a[4], e3 = a[6], o0 = a[1];
  a[0] = e0 + o0; a[4] = e0 - o0;
  a[1] = e1 + o1; a[5] = e1 - o1;
  a[2] = e2 + o2; a[6] = e2 - o2;
  a[3] = e3 + o3; a[7] = e3 - o3;
}

// 16-point DFT: two 8-point DFTs on even/odd inputs, combined with W_16^k.
template <typename T, bool INV>
__device__ __forceinline__ void dft16(Cx<T>* a) {
  Cx<T> e[8], o[8];
#pragma unroll
  for (int i = 0; i < 8; ++i) { e[i] = a[2 * i]; o[i] = a[2 * i + 1]; }
  dft8<T, INV>(e);
  dft8<T, INV>(o);
  const T c1 = (T)0.92387953251128675613, s1 = (T)0.38268343236508977173;
  const T h = (T)0.70710678118654752440;
  const T sg = INV ? (T)1 : (T)-1;   // W_16^k = cos(2 pi k/16) + sg i sin(2 pi k/16)
  const T cr[8] = {(T)1, c1, h, s1, (T)0, -s1, -h, -c1};
  const T ci[8] = {(T)0, s1, h, c1, (T)1, c1, h, s1};
#pragma unroll
  for (int k = 0; k < 8; ++k) {
    Cx<T> t;
    if (k == 0) t = o[0];
    else if (k == 4) t = mul_mi<T, INV>(o[4]);
    else t = cmul(o[k], cx(cr[k], sg * ci[k]));
    a[k] = e[k] + t;
    a[k + 8] = e[k] - t;
  }
}

template <typename T, int R, bool INV>
__device__ __forceinline__ void dft_r(Cx<T>* a) {
  if constexpr (R == 2) dft2<T, INV>(a[0], a[1]);
  else if constexpr (R == 4) dft4<T, INV>(a[0], a[1], a[2], a[3]);
  else if constexpr (R == 8) dft8<T, INV>(a);
  else dft16<T, INV>(a);
}

template <typename T, bool INV, int NT, int LOGN, int LOGCNT, bool CM, int LOGE, int LOGNS>
__device__ __forceinline__ void ct_stage(Cx<T>* buf, const Cx<T>* __restrict__ tw) {
  constexpr int N = 1 << LOGN, CNT = 1 << LOGCNT;
  constexpr int LR = stage_lr(LOGN, LOGNS, LOGE), R = 1 << LR;
  constexpr int NB = N >> LR, TOTAL = NB * CNT;
  constexpr int MAXB = (TOTAL + NT - 1) / NT;
  constexpr int NS = 1 << LOGNS;
  constexpr int ES = CM ? CNT : 1, FS = CM ? 1 : N;
  constexpr int TWOFF = tw_stage_offset(LOGN, LOGNS, LOGE);
  constexpr bool RD_FAST = ((NB * ES) % 16) == 0;
  constexpr bool WR_FAST = ((NS * ES) % 16) == 0;
  constexpr bool WR_SMALL = (NS == 1) && (ES == 1) && (R == 16) && (FS % 16 == 0);
  const int tid = threadIdx.x;
  Cx<T> v[MAXB][R];
#pragma unroll
  for (int q = 0; q < MAXB; ++q) {
    const int w = tid + q * NT;
    if (TOTAL % NT == 0 || w < TOTAL) {
      int j, f;
      if (CM) { f = w & (CNT - 1); j = w >> LOGCNT; }
      else { j = w & (NB - 1); f = w >> (LOGN - LR); }
      const int base = j * ES + f * FS;
      if (RD_FAST) {
        const int pb = lp(base);
#pragma unroll
        for (int r = 0; r < R; ++r) v[q][r] = buf[pb + r * NB * ES + ((r * NB * ES) >> 4)];
      } else {
#pragma unroll
        for (int r = 0; r < R; ++r) v[q][r] = buf[lp(base + r * NB * ES)];
      }
      if (LOGNS > 0) {
        const int k = j & (NS - 1);
        const Cx<T>* tp = tw + TWOFF + k * (R - 1);
#pragma unroll
        for (int r = 1; r < R; ++r) {
          const Cx<T> t = tp[r - 1];
          v[q][r] = INV ? cmulc(v[q][r], t) : cmul(v[q][r], t);
        }
      }
      dft_r<T, R, INV>(v[q]);
    }
  }
  __syncthreads();
#pragma unroll
  for (int q = 0; q < MAXB; ++q) {
    const int w = tid + q * NT;
    if (TOTAL % NT == 0 || w < TOTAL) {
      int j, f;
      if (CM) { f = w & (CNT - 1); j = w >> LOGCNT; }
      else { j = w & (NB - 1); f = w >> (LOGN - LR); }
      const int k = j & (NS - 1);
      const int d = ((j >> LOGNS) << (LOGNS + LR)) + k;
      const int base = d * ES + f * FS;
      if (WR_FAST) {
        const int pb = lp(base);
#pragma unroll
        for (int r = 0; r < R; ++r) buf[pb + r * NS * ES + ((r * NS * ES) >> 4)] = v[q][r];
      } else if (WR_SMALL) {
        const int pb = lp(base);           // base is a multiple of 16 and r < 16
#pragma unroll
        for (int r = 0; r < R; ++r) buf[pb + r] = v[q][r];
      } else {
#pragma unroll
        for (int r = 0; r < R; ++r) buf[lp(base + r * NS * ES)] = v[q][r];
      }
    }
  }
  __syncthreads();
}

template <typename T, bool INV, int NT, int LOGN, int LOGCNT, bool CM, int LOGE, int LOGNS = 0, int LOGEND = LOGN>
__device__ __forceinline__ void ct_fft(Cx<T>* buf, const Cx<T>* __restrict__ tw) {
  if constexpr (LOGNS < LOGEND) {
    ct_stage<T, INV, NT, LOGN, LOGCNT, CM, LOGE, LOGNS>(buf, tw);
    ct_fft<T, INV, NT, LOGN, LOGCNT, CM, LOGE, LOGNS + stage_lr(LOGN, LOGNS, LOGE), LOGEND>(buf, tw);
  }
}

// Register-resident first and last stages, for row-major sets of FFTs where
// every stage is radix R = 2^LOGE and each thread owns exactly one butterfly
// per stage (NT butterflies: CNT N / R == NT).  Thread tid owns FFT
// f = tid / (N/R) and butterfly j = tid mod (N/R); its first stage reads
// elements j + r N/R (r < R) of FFT f, and its last stage produces elements
// j + r N/R as well.  So the caller can load the input straight from global
// memory into v[] (in that order) and store the output from v[], saving an
// LDS round trip and a barrier at each end.
template <int LOGN, int LOGCNT, int LOGE, int NT>
struct RegIO {
  static constexpr int R = 1 << LOGE;
  static constexpr bool ok = (LOGN % LOGE == 0) && LOGN >= 2 * LOGE && ((1 << (LOGN + LOGCNT)) >> LOGE) == NT;
};

// v holds the inputs of the first stage; runs every stage, output in LDS (natural order).
template <typename T, bool INV, int NT, int LOGN, int LOGCNT, int LOGE>
__device__ __forceinline__ void ct_fft_from_regs(Cx<T>* buf, const Cx<T>* __restrict__ tw, Cx<T> (&v)[1 << LOGE]) {
  constexpr int R = 1 << LOGE, N = 1 << LOGN;
  dft_r<T, R, INV>(v);
  // first stage (span 1): butterfly j writes output r to j R + r of its FFT
  const int tid = threadIdx.x;
  const int j = tid & ((N >> LOGE) - 1), f = tid >> (LOGN - LOGE);
  const int base = j * R + f * N;          // a multiple of 16 (R >= 16) or, below, generic
  if constexpr (R == 16) {
    const int pb = lp(base);
#pragma unroll
    for (int r = 0; r < R; ++r) buf[pb + r] = v[r];
  } else {
#pragma unroll
    for (int r = 0; r < R; ++r) buf[lp(base + r)] = v[r];
  }
  __syncthreads();
  ct_fft<T, INV, NT, LOGN, LOGCNT, false, LOGE, LOGE>(buf, tw);
}

// Runs every stage of the FFTs held in LDS but keeps the last stage's outputs
// in v (element j + r N/R of FFT f in v[r]); the LDS is free on return.
template <typename T, bool INV, int NT, int LOGN, int LOGCNT, int LOGE>
__device__ __forceinline__ void ct_fft_to_regs(Cx<T>* buf, const Cx<T>* __restrict__ tw, Cx<T> (&v)[1 << LOGE]) {
  constexpr int R = 1 << LOGE, N = 1 << LOGN;
  constexpr int LAST = LOGN - LOGE;            // span of the last stage
  ct_fft<T, INV, NT, LOGN, LOGCNT, false, LOGE, 0, LAST>(buf, tw);
  constexpr int NB = N >> LOGE, NS = 1 << LAST;
  constexpr int TWOFF = tw_stage_offset(LOGN, LAST, LOGE);
  const int tid = threadIdx.x;
  const int j = tid & (NB - 1), f = tid >> (LOGN - LOGE);
  const int pb = lp(j + f * N);
#pragma unroll
  for (int r = 0; r < R; ++r) v[r] = buf[pb + r * NB + ((r * NB) >> 4)];
  const int k = j & (NS - 1);
  const Cx<T>* tp = tw + TWOFF + k * (R - 1);
#pragma unroll
  for (int r = 1; r < R; ++r) {
    const Cx<T> t = tp[r - 1];
    v[r] = INV ? cmulc(v[r], t) : cmul(v[r], t);
  }
  dft_r<T, R, INV>(v);
  __syncthreads();
}

// Column-major sets (CNT interleaved FFTs, element n of FFT f at n CNT + f).
// First stage from registers: when that stage has exactly NT butterflies,
// thread tid owns butterfly (f = tid mod CNT, j = tid / CNT), whose inputs
// j + r N/R are what a strided load e = tid + r NT visits (element e / CNT of
// FFT e mod CNT).  v holds them; every stage runs, output in LDS.
template <typename T, bool INV, int NT, int LOGN, int LOGCNT, int LOGE>
__device__ __forceinline__ void ct_fft_cm_from_regs(Cx<T>* buf, const Cx<T>* __restrict__ tw,
                                                    Cx<T> (&v)[1 << stage_lr(LOGN, 0, LOGE)]) {
  constexpr int LR = stage_lr(LOGN, 0, LOGE), R = 1 << LR, CNT = 1 << LOGCNT;
  static_assert(((1 << (LOGN + LOGCNT)) >> LR) == NT, "one first-stage butterfly per thread");
  dft_r<T, R, INV>(v);
  const int tid = threadIdx.x;
  const int f = tid & (CNT - 1), j = tid >> LOGCNT;
  const int base = j * R * CNT + f;   // output r of butterfly j is element j R + r
#pragma unroll
  for (int r = 0; r < R; ++r) buf[lp(base + r * CNT)] = v[r];
  __syncthreads();
  ct_fft<T, INV, NT, LOGN, LOGCNT, true, LOGE, LR>(buf, tw);
}

}  // namespace csr
