// Workgroup-cooperative FFTs held in LDS.
//
// A set of `count` independent length-n FFTs sits in LDS; element e of FFT f
// is at buf[e * es + f * fs].  The transform runs as a sequence of Stockham
// autosort stages (radix 16/8/4/2, Govindaraju et al., SC'08 formulation):
// stage with span Ns reads the R inputs of butterfly j at j + r n/R, applies
// twiddles W_{Ns R}^{r (j mod Ns)}, does an R-point DFT in registers and
// writes output r to (j / Ns) Ns R + (j mod Ns) + r Ns.  Each stage reads all
// its inputs into registers, synchronises, then writes in place, so one LDS
// buffer suffices.  Output is in natural order.
//
// Forward = exp(-2 pi i ...) kernel, inverse = exp(+2 pi i ...), unnormalised.
#pragma once

#include "cs_internal.h"

namespace csr {

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
  // odd outputs times W_8^k, k = 0..3
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
    Cx<T> w = cx(cr[k], sg * ci[k]);
    Cx<T> t = (k == 0) ? o[0] : cmul(o[k], w);
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

template <int R> struct LogR;
template <> struct LogR<2> { static constexpr int v = 1; };
template <> struct LogR<4> { static constexpr int v = 2; };
template <> struct LogR<8> { static constexpr int v = 3; };
template <> struct LogR<16> { static constexpr int v = 4; };

// One radix-R Stockham stage.  F_FAST selects the thread-to-butterfly map:
// true  -> consecutive threads take consecutive FFTs (use when fs == 1),
// false -> consecutive threads take consecutive butterflies (use when es == 1).
template <typename T, int R, bool INV, bool F_FAST, int MAXB>
__device__ __forceinline__ void fft_stage(Cx<T>* buf, int logn, int logNs, int logcount, int es, int fs,
                                          const Cx<T>* __restrict__ twsub) {
  constexpr int LR = LogR<R>::v;
  const int lognb = logn - LR;
  const int nb = 1 << lognb;
  const int total = nb << logcount;
  const int tid = threadIdx.x, nt = blockDim.x;
  const int Ns = 1 << logNs;
  // twiddle W_{Ns R}^{m} = W_{8192}^{m * 8192 / (Ns R)}
  const int twshift = kTwSubLog - (logNs + LR);
  Cx<T> v[MAXB][R];
#pragma unroll
  for (int q = 0; q < MAXB; ++q) {
    const int w = tid + q * nt;
    if (w < total) {
      int j, f;
      if (F_FAST) { f = w & ((1 << logcount) - 1); j = w >> logcount; }
      else { j = w & (nb - 1); f = w >> lognb; }
      const int base = j * es + f * fs;
#pragma unroll
      for (int r = 0; r < R; ++r) v[q][r] = buf[base + r * nb * es];
      if (logNs > 0) {
        const int k = j & (Ns - 1);
#pragma unroll
        for (int r = 1; r < R; ++r) {
          Cx<T> t = twsub[(r * k) << twshift];
          v[q][r] = INV ? cmulc(v[q][r], t) : cmul(v[q][r], t);
        }
      }
      dft_r<T, R, INV>(v[q]);
    }
  }
  __syncthreads();
#pragma unroll
  for (int q = 0; q < MAXB; ++q) {
    const int w = tid + q * nt;
    if (w < total) {
      int j, f;
      if (F_FAST) { f = w & ((1 << logcount) - 1); j = w >> logcount; }
      else { j = w & (nb - 1); f = w >> lognb; }
      const int k = j & (Ns - 1);
      const int d = ((j >> logNs) << (logNs + LR)) + k;
      const int base = d * es + f * fs;
#pragma unroll
      for (int r = 0; r < R; ++r) buf[base + r * Ns * es] = v[q][r];
    }
  }
  __syncthreads();
}

// Full FFT of `1 << logcount` length-2^logn sequences in LDS, EPT elements per
// thread at most (blockDim.x * EPT >= 2^(logn + logcount)).
template <typename T, bool INV, bool F_FAST, int EPT>
__device__ __forceinline__ void lds_fft(Cx<T>* buf, int logn, int logcount, int es, int fs,
                                        const Cx<T>* __restrict__ twsub) {
  int logNs = 0;
  int rem = logn;
  while (rem > 0) {
    if (rem >= 4 && EPT >= 16) {
      fft_stage<T, 16, INV, F_FAST, (EPT >= 16 ? EPT / 16 : 1)>(buf, logn, logNs, logcount, es, fs, twsub);
      rem -= 4; logNs += 4;
    } else if (rem >= 3) {
      fft_stage<T, 8, INV, F_FAST, EPT / 8>(buf, logn, logNs, logcount, es, fs, twsub);
      rem -= 3; logNs += 3;
    } else if (rem == 2) {
      fft_stage<T, 4, INV, F_FAST, EPT / 4>(buf, logn, logNs, logcount, es, fs, twsub);
      rem -= 2; logNs += 2;
    } else {
      fft_stage<T, 2, INV, F_FAST, EPT / 2>(buf, logn, logNs, logcount, es, fs, twsub);
      rem -= 1; logNs += 1;
    }
  }
}

}  // namespace csr
