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
#include "cs_fft.h"

#include <algorithm>
#include <cmath>

namespace csr {

void hip_check(hipError_t e, const char* what, const char* file, int line) {
  if (e != hipSuccess) {
    throw Error(CS_E_HIP, std::string(what) + " failed: " + hipGetErrorString(e) + " (" + file + ":" +
                              std::to_string(line) + ")");
  }
}

// ------------------------------------------------------------------ plan
bool choose_plan(cs_dtype dt, int64_t n, int64_t m, Plan& p) {
  if (n < 16 || n > (int64_t(1) << 26) || (n & (n - 1))) return false;
  p = Plan{};
  p.n = n;
  p.m = m;
  p.logn = 0;
  while ((int64_t(1) << p.logn) < n) ++p.logn;
  p.words = (n + 31) / 32;
  p.L = n / 2;
  p.logL = p.logn - 1;
  const int l = p.logL;
  const int maxL2 = (dt == CS_F32) ? 13 : 12;          // two rows of L2 fit in 128 KB LDS
  const int maxE = (dt == CS_F32) ? 16384 : 8192;      // column strip elements per workgroup
  int logL1;
  if (l >= 22) logL1 = l - maxL2;
  else logL1 = std::max(l - maxL2, l / 2);
  logL1 = std::max(logL1, 1);
  p.logL1 = logL1;
  p.logL2 = l - logL1;
  if (p.logL2 < 1 || p.logL2 > maxL2) return false;
  p.L1 = 1 << p.logL1;
  p.L2 = 1 << p.logL2;
  int B = std::min({p.L2, maxE / p.L1, 16});
  while (B > 4 && (p.L2 / B) < 256) B >>= 1;
  B = std::max(B, 1);
  p.B = B;
  p.logB = 0;
  while ((1 << p.logB) < B) ++p.logB;
  const size_t cs = (dt == CS_F32) ? 8 : 16;
  const int ecol = B * p.L1, erow = 2 * p.L2;
  p.nt_col = std::max(64, std::min(1024, ecol / 16));
  p.nt_row = std::max(64, std::min(1024, erow / 16));
  if ((int64_t)p.nt_col * 16 < ecol || (int64_t)p.nt_row * 16 < erow) return false;
  p.lds_col = cs * ecol;
  p.lds_row = cs * erow;
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

// Builds the freq-layout row mask and validates the descriptor.
// bad[0] |= 1: rows not strictly ascending or out of range; |= 2: a sign not +-1.
__global__ void k_mask_rows(const int32_t* __restrict__ rows, int64_t m, uint32_t* __restrict__ mask,
                            Plan p, int32_t* bad) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= m) return;
  int64_t q = rows[i];
  bool ok = (q >= 0 && q < p.n) && (i == 0 || rows[i - 1] < q);
  if (!ok) { atomicOr(bad, 1); return; }
  int64_t fp = fpos(q, p);
  atomicOr(&mask[fp >> 5], 1u << (fp & 31));
}

__global__ void k_check_signs(const int8_t* __restrict__ s, int64_t n, int32_t* bad) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  int8_t v = s[i];
  if (v != 1 && v != -1) atomicOr(bad, 2);
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

template <typename T>
void setup_operator(Ctx<T>& c) {
  const Plan& p = c.plan;
  hipStream_t s = c.stream;
  hipLaunchKernelGGL(k_twiddle<T>, dim3(nblk(kTwSub, 256)), dim3(256), 0, s, c.tw_sub, (int64_t)kTwSub,
                     (int64_t)kTwSub, (int64_t)1);
  CS_LAUNCH_CHECK();
  const int64_t n4 = 4 * p.n;
  hipLaunchKernelGGL(k_twiddle<T>, dim3(nblk(kTwLo, 256)), dim3(256), 0, s, c.tw_lo, (int64_t)kTwLo, n4,
                     (int64_t)1);
  CS_LAUNCH_CHECK();
  const int64_t nhi = std::max<int64_t>(1, n4 / kTwLo);
  hipLaunchKernelGGL(k_twiddle<T>, dim3(nblk(nhi, 256)), dim3(256), 0, s, c.tw_hi, nhi, n4, (int64_t)kTwLo);
  CS_LAUNCH_CHECK();
  fill_u32(c.mask, p.words, 0u, s);
  fill<int32_t>(c.ibuf, 1, 0, s);
  hipLaunchKernelGGL(k_mask_rows, dim3(nblk(p.m, 256)), dim3(256), 0, s, c.rows, p.m, c.mask, p, c.ibuf);
  CS_LAUNCH_CHECK();
  hipLaunchKernelGGL(k_check_signs, dim3(nblk(p.n, 256)), dim3(256), 0, s, c.signs, p.n, c.ibuf);
  CS_LAUNCH_CHECK();
  int32_t bad = 0;
  CS_HIP(hipMemcpyAsync(&bad, c.ibuf, sizeof(int32_t), hipMemcpyDeviceToHost, s));
  CS_HIP(hipStreamSynchronize(s));
  if (bad & 1) throw Error(CS_E_OP, "operator rows must be strictly ascending in [0, N)");
  if (bad & 2) throw Error(CS_E_OP, "operator signs must be +1 or -1");
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

// ------------------------------------------------------------------ column passes
// Forward column FFTs: z (L1 x L2, row-major) -> Y[k1][n2] = sum_n1 z[n1][n2] W_L1^{n1 k1}.
// One workgroup owns a strip of B adjacent columns; LDS holds it row-major.
template <typename T, bool INV>
__global__ __launch_bounds__(1024) void k_col(const Cx<T>* __restrict__ in, Cx<T>* __restrict__ out, Plan p,
                                              const int* __restrict__ done) {
  if (done && *done) return;
  extern __shared__ __align__(16) unsigned char smem_raw[];
  Cx<T>* buf = (Cx<T>*)smem_raw;
  const int g = xcd_order(blockIdx.x, gridDim.x);
  const int c0 = g << p.logB;
  const int E = p.B << p.logL1;
  for (int e = threadIdx.x; e < E; e += blockDim.x) {
    const int n1 = e >> p.logB, b = e & (p.B - 1);
    buf[e] = in[(size_t)n1 * p.L2 + c0 + b];
  }
  __syncthreads();
  lds_fft<T, INV, true, 16>(buf, p.logL1, p.logB, p.B, 1, (const Cx<T>*)p.tw_sub);
  for (int e = threadIdx.x; e < E; e += blockDim.x) {
    const int n1 = e >> p.logB, b = e & (p.B - 1);
    out[(size_t)n1 * p.L2 + c0 + b] = buf[e];
  }
}

// ------------------------------------------------------------------ row pass
// Workgroup w owns rows ra = w, rb = L1 - w (w >= 1) or ra = 0, rb = L1/2 (w = 0).
// Row r, element k2 holds Z[r + L1 k2]; the mirror bin L - k of k = r + L1 k2
// is row L1 - r, element L2 - 1 - k2 (r >= 1) or row 0, element L2 - k2 (r = 0).
//
// Item t enumerates the bin pairs {k, L-k} of the two rows:
//   w >= 1: t in [0, L2): (ra, t) with (rb, L2-1-t)
//   w == 0: t in [0, L2/2]: (0, t) with (0, (L2-t) mod L2); t = 0 is bin 0;
//           t in (L2/2, L2]: (rb, t') with (rb, L2-1-t'), t' = t - L2/2 - 1.
struct RowItem {
  int sa, sb;       // LDS slots (row select * stride + element) of self and partner
  int64_t fa, fb;   // freq-layout slots of self and partner
  int64_t k;        // bin index of self
  bool zero;        // bin 0 (self-contained)
};

__device__ __forceinline__ RowItem row_item(int t, int w, int ra, int rb, const Plan& p, int stride) {
  RowItem it;
  const int L2 = p.L2;
  int rsel, k2, rsel2, k22, rowA, rowB;
  if (w > 0) {
    rsel = 0; k2 = t; rsel2 = 1; k22 = L2 - 1 - t;
  } else if (t <= L2 / 2) {
    rsel = 0; k2 = t; rsel2 = 0; k22 = (L2 - t) & (L2 - 1);
  } else {
    const int tt = t - L2 / 2 - 1;
    rsel = 1; k2 = tt; rsel2 = 1; k22 = L2 - 1 - tt;
  }
  rowA = rsel ? rb : ra;
  rowB = rsel2 ? rb : ra;
  it.sa = rsel * stride + k2;
  it.sb = rsel2 * stride + k22;
  it.fa = (int64_t)rowA * L2 + k2;
  it.fb = (int64_t)rowB * L2 + k22;
  it.k = (int64_t)rowA + (int64_t)p.L1 * k2;
  it.zero = (it.k == 0);
  return it;
}

__device__ __forceinline__ uint32_t mask2(const uint32_t* __restrict__ mask, int64_t f) {
  return (mask[(2 * f) >> 5] >> ((2 * f) & 31)) & 3u;
}

template <typename T, int MODE>
__global__ __launch_bounds__(1024) void k_row(Cx<T>* __restrict__ buf, Plan p, const T* __restrict__ fin,
                                              T* __restrict__ fout, double* __restrict__ partial,
                                              const int* __restrict__ done) {
  if (done && *done) return;
  extern __shared__ __align__(16) unsigned char smem_raw[];
  Cx<T>* lds = (Cx<T>*)smem_raw;
  __shared__ double red[32];
  const int w = blockIdx.x;
  const int ra = w, rb = (w == 0) ? (p.L1 >> 1) : (p.L1 - w);
  const int L2 = p.L2, stride = p.L2;
  const uint32_t Lmask = (uint32_t)(p.L - 1);
  const Cx<T>* twsub = (const Cx<T>*)p.tw_sub;
  const T c = (T)sqrt(2.0 / (double)p.n);
  const T rsn = (T)(1.0 / sqrt((double)p.n));
  const T h = (T)0.70710678118654752440;

  if (MODE != ROW_ADJ) {
    for (int e = threadIdx.x; e < 2 * L2; e += blockDim.x) {
      const int rs = e >> p.logL2, n2 = e & (L2 - 1);
      const int r = rs ? rb : ra;
      Cx<T> v = buf[(size_t)r * L2 + n2];
      const uint32_t m = ((uint32_t)n2 * (uint32_t)r) & Lmask;   // W_L^{n2 r} = W_4N^{8 m}
      lds[rs * stride + n2] = cmul(v, tw4n<T>(p, m << 3));
    }
    __syncthreads();
    lds_fft<T, false, false, 16>(lds, p.logL2, 1, 1, stride, twsub);
  }

  double acc = 0.0;
  const int nitems = (w > 0) ? L2 : (L2 + 1);
  for (int t = threadIdx.x; t < nitems; t += blockDim.x) {
    const RowItem it = row_item(t, w, ra, rb, p, stride);
    T xa0, xa1, xb0, xb1;   // X_k, X_{N-k} (self slot) and X_{L-k}, X_{L+k} (partner slot)
    Cx<T> wk, WN;
    if (MODE != ROW_ADJ) {
      const Cx<T> Zk = lds[it.sa];
      if (it.zero) {
        xa0 = (Zk.re + Zk.im) * rsn;
        xa1 = (Zk.re - Zk.im) * rsn;
        xb0 = xb1 = (T)0;
      } else {
        const Cx<T> Zm = lds[it.sb];
        const Cx<T> E = scale(Zk + conj(Zm), (T)0.5);
        const Cx<T> D = Zk - conj(Zm);
        const Cx<T> O = cx(D.im * (T)0.5, -D.re * (T)0.5);   // D / (2i)
        wk = tw4n<T>(p, (uint32_t)it.k);
        WN = tw4n<T>(p, (uint32_t)(4 * it.k));
        const Cx<T> WO = cmul(WN, O);
        const Cx<T> Vk = E + WO;
        const Cx<T> Vm = conj(E - WO);
        const Cx<T> wm = cx(h * (wk.re - wk.im), -h * (wk.re + wk.im));  // e^{-i pi/4} conj(wk)
        const Cx<T> a = cmul(wk, Vk), b = cmul(wm, Vm);
        xa0 = c * a.re; xa1 = -c * a.im;
        xb0 = c * b.re; xb1 = -c * b.im;
      }
    } else {
      xa0 = fin[2 * it.fa]; xa1 = fin[2 * it.fa + 1];
      xb0 = fin[2 * it.fb]; xb1 = fin[2 * it.fb + 1];
      if (!it.zero) {
        wk = tw4n<T>(p, (uint32_t)it.k);
        WN = tw4n<T>(p, (uint32_t)(4 * it.k));
      }
    }
    if (MODE == ROW_HAPPLY || MODE == ROW_RESID || MODE == ROW_FWD) {
      const uint32_t ma = mask2(p.mask, it.fa);
      const uint32_t mb = it.zero ? 0u : mask2(p.mask, it.fb);
      if (MODE == ROW_RESID) {
        xa0 = fin[2 * it.fa] - xa0;
        xa1 = fin[2 * it.fa + 1] - xa1;
        xb0 = it.zero ? (T)0 : fin[2 * it.fb] - xb0;
        xb1 = it.zero ? (T)0 : fin[2 * it.fb + 1] - xb1;
      }
      xa0 = (ma & 1u) ? xa0 : (T)0;
      xa1 = (ma & 2u) ? xa1 : (T)0;
      xb0 = (mb & 1u) ? xb0 : (T)0;
      xb1 = (mb & 2u) ? xb1 : (T)0;
      if (MODE == ROW_RESID) {
        // a self-paired bin (k = L/2) has fa == fb: count its two outputs once
        const bool self = (!it.zero) && (it.fa == it.fb);
        acc += (double)xa0 * xa0 + (double)xa1 * xa1;
        if (!self) acc += (double)xb0 * xb0 + (double)xb1 * xb1;
      }
      if (MODE == ROW_FWD) {
        fout[2 * it.fa] = xa0; fout[2 * it.fa + 1] = xa1;
        if (!it.zero) { fout[2 * it.fb] = xb0; fout[2 * it.fb + 1] = xb1; }
        continue;
      }
    }
    // pre-process for the inverse
    if (it.zero) {
      lds[it.sa] = cx((xa0 + xa1) * rsn, (xa0 - xa1) * rsn);
    } else {
      const Cx<T> wm = cx(h * (wk.re - wk.im), -h * (wk.re + wk.im));
      const Cx<T> Vk = scale(cmulc(cx(xa0, -xa1), wk), c);    // conj(wk) (Xk - i X_{N-k}) c
      const Cx<T> Vm = scale(cmulc(cx(xb0, -xb1), wm), c);
      const Cx<T> E = scale(Vk + conj(Vm), (T)0.5);
      const Cx<T> O = scale(cmulc(Vk - conj(Vm), WN), (T)0.5);
      lds[it.sa] = cx(E.re - O.im, E.im + O.re);               // E + i O
      lds[it.sb] = cx(E.re + O.im, -E.im + O.re);              // conj(E) + i conj(O)
    }
  }
  if (MODE == ROW_RESID) {
    // workgroup reduction of acc -> partial[w]
    for (int off = 32; off > 0; off >>= 1) acc += __shfl_down(acc, off, 64);
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    if (lane == 0) red[wave] = acc;
    __syncthreads();
    if (threadIdx.x == 0) {
      double s = 0.0;
      for (int i = 0; i < (int)(blockDim.x + 63) / 64; ++i) s += red[i];
      partial[w] = s;
    }
  }
  if (MODE == ROW_FWD) return;
  __syncthreads();
  lds_fft<T, true, false, 16>(lds, p.logL2, 1, 1, stride, twsub);
  for (int e = threadIdx.x; e < 2 * L2; e += blockDim.x) {
    const int rs = e >> p.logL2, n2 = e & (L2 - 1);
    const int r = rs ? rb : ra;
    const uint32_t m = ((uint32_t)n2 * (uint32_t)r) & Lmask;
    buf[(size_t)r * L2 + n2] = cmulc(lds[rs * stride + n2], tw4n<T>(p, m << 3));
  }
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

template <typename T>
double norm2_host(Ctx<T>& c, const T* v, int64_t count) {
  const unsigned grid = (unsigned)std::min<int64_t>(kRedBlocks, nblk(count, 256));
  hipLaunchKernelGGL(k_sumsq_partial<T>, dim3(grid), dim3(256), 0, c.stream, v, count, c.partial2);
  CS_LAUNCH_CHECK();
  hipLaunchKernelGGL(k_sum_partials, dim3(1), dim3(1024), 0, c.stream, c.partial2, (int)grid, &c.cg->resid2);
  CS_LAUNCH_CHECK();
  double r2 = 0.0;
  CS_HIP(hipMemcpyAsync(&r2, &c.cg->resid2, sizeof(double), hipMemcpyDeviceToHost, c.stream));
  CS_HIP(hipStreamSynchronize(c.stream));
  return std::sqrt(r2);
}

// ------------------------------------------------------------------ launchers
template <typename T>
static void launch_col(Ctx<T>& c, const Cx<T>* in, Cx<T>* out, bool inv, const int* done) {
  const Plan& p = c.plan;
  const unsigned grid = (unsigned)(p.L2 >> p.logB);
  const double bytes = 2.0 * (double)p.n * sizeof(T);   // read and write one N-vector
  hipEvent_t ev = nullptr;
  const bool prof = prof_on();
  if (prof) prof_begin(c.stream, &ev);
  if (inv)
    hipLaunchKernelGGL((k_col<T, true>), dim3(grid), dim3(p.nt_col), p.lds_col, c.stream, in, out, p, done);
  else
    hipLaunchKernelGGL((k_col<T, false>), dim3(grid), dim3(p.nt_col), p.lds_col, c.stream, in, out, p, done);
  CS_LAUNCH_CHECK();
  if (prof) prof_end(inv ? PC_COL_INV : PC_COL_FWD, bytes, ev, c.stream);
  c.model_bytes += bytes;
}

template <typename T, int MODE>
static void launch_row(Ctx<T>& c, const T* fin, T* fout, double* partial, const int* done) {
  const Plan& p = c.plan;
  const unsigned grid = (unsigned)(p.L1 >> 1);
  // read and write one N-vector; the residual pass also reads y (N reals in freq layout)
  double bytes = 2.0 * (double)p.n * sizeof(T);
  if (MODE == ROW_RESID) bytes += (double)p.n * sizeof(T);
  hipEvent_t ev = nullptr;
  const bool prof = prof_on();
  if (prof) prof_begin(c.stream, &ev);
  hipLaunchKernelGGL((k_row<T, MODE>), dim3(grid), dim3(p.nt_row), p.lds_row, c.stream, c.W, p, fin, fout,
                     partial, done);
  CS_LAUNCH_CHECK();
  if (prof) prof_end(PC_ROW_HAPPLY + MODE, bytes, ev, c.stream);
  c.model_bytes += bytes;
}

template <typename T>
void transform_happly(Ctx<T>& c, const T* in, const int* done) {
  launch_col<T>(c, (const Cx<T>*)in, c.W, false, done);
  launch_row<T, ROW_HAPPLY>(c, nullptr, nullptr, nullptr, done);
  launch_col<T>(c, c.W, c.W, true, done);
  c.transforms += 2;
}

template <typename T>
void transform_resid(Ctx<T>& c, const T* in) {
  launch_col<T>(c, (const Cx<T>*)in, c.W, false, nullptr);
  launch_row<T, ROW_RESID>(c, c.Yf, nullptr, c.partial2, nullptr);
  launch_col<T>(c, c.W, c.W, true, nullptr);
  hipLaunchKernelGGL(k_sum_partials, dim3(1), dim3(1024), 0, c.stream, c.partial2, c.plan.L1 >> 1,
                     &c.cg->resid2);
  CS_LAUNCH_CHECK();
  c.transforms += 2;
}

template <typename T>
void transform_fwd(Ctx<T>& c, const T* in, T* outf) {
  launch_col<T>(c, (const Cx<T>*)in, c.W, false, nullptr);
  launch_row<T, ROW_FWD>(c, nullptr, outf, nullptr, nullptr);
  c.transforms += 1;
}

template <typename T>
void transform_adj(Ctx<T>& c, const T* inf) {
  launch_row<T, ROW_ADJ>(c, inf, nullptr, nullptr, nullptr);
  launch_col<T>(c, c.W, c.W, true, nullptr);
  c.transforms += 1;
}

// ------------------------------------------------------------------ compact <-> dense
template <typename T>
__global__ void k_scatter_signed(T* __restrict__ dense, const int32_t* __restrict__ list,
                                 const T* __restrict__ vals, int k, const int8_t* __restrict__ signs, int64_t n) {
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= k) return;
  const int64_t j = list[i];
  dense[vpos(j, n)] = signs[j] < 0 ? -vals[i] : vals[i];
}
template <typename T>
__global__ void k_scatter_zero(T* __restrict__ dense, const int32_t* __restrict__ list, int k, int64_t n) {
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= k) return;
  dense[vpos(list[i], n)] = (T)0;
}
template <typename T>
__global__ void k_gather_signed(const T* __restrict__ dense, const int32_t* __restrict__ list,
                                T* __restrict__ vals, int k, const int8_t* __restrict__ signs, int64_t n) {
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= k) return;
  const int64_t j = list[i];
  const T v = dense[vpos(j, n)];
  vals[i] = signs[j] < 0 ? -v : v;
}

template <typename T>
void scatter_signed(Ctx<T>& c, T* dense, const int32_t* list, const T* vals, int k) {
  if (k <= 0) return;
  hipLaunchKernelGGL(k_scatter_signed<T>, dim3(nblk(k, 256)), dim3(256), 0, c.stream, dense, list, vals, k,
                     c.signs, c.plan.n);
  CS_LAUNCH_CHECK();
}
template <typename T>
void scatter_zero(Ctx<T>& c, T* dense, const int32_t* list, int k) {
  if (k <= 0) return;
  hipLaunchKernelGGL(k_scatter_zero<T>, dim3(nblk(k, 256)), dim3(256), 0, c.stream, dense, list, k, c.plan.n);
  CS_LAUNCH_CHECK();
}
template <typename T>
void gather_signed(Ctx<T>& c, const T* dense, const int32_t* list, T* vals, int k) {
  if (k <= 0) return;
  hipLaunchKernelGGL(k_gather_signed<T>, dim3(nblk(k, 256)), dim3(256), 0, c.stream, dense, list, vals, k,
                     c.signs, c.plan.n);
  CS_LAUNCH_CHECK();
}

template <typename T>
__global__ void k_perm_in(const T* __restrict__ x, T* __restrict__ dense, const int8_t* __restrict__ signs,
                          int64_t n) {
  int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= n) return;
  dense[vpos(j, n)] = signs[j] < 0 ? -x[j] : x[j];
}
template <typename T>
__global__ void k_perm_out(const T* __restrict__ dense, T* __restrict__ x, const int8_t* __restrict__ signs,
                           int64_t n) {
  int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= n) return;
  const T v = dense[vpos(j, n)];
  x[j] = signs[j] < 0 ? -v : v;
}
template <typename T>
void perm_in(Ctx<T>& c, const T* x, T* dense) {
  hipLaunchKernelGGL(k_perm_in<T>, dim3(nblk(c.plan.n, 256)), dim3(256), 0, c.stream, x, dense, c.signs, c.plan.n);
  CS_LAUNCH_CHECK();
}
template <typename T>
void perm_out(Ctx<T>& c, const T* dense, T* x) {
  hipLaunchKernelGGL(k_perm_out<T>, dim3(nblk(c.plan.n, 256)), dim3(256), 0, c.stream, dense, x, c.signs, c.plan.n);
  CS_LAUNCH_CHECK();
}

template <typename T>
void prepare_kernels() {
  static bool done = false;   // per instantiation; benign race (idempotent calls)
  if (done) return;
  const int lim = 128 * 1024;   // largest dynamic LDS any plan asks for (static LDS comes on top)
  CS_HIP(hipFuncSetAttribute((const void*)k_col<T, false>, hipFuncAttributeMaxDynamicSharedMemorySize, lim));
  CS_HIP(hipFuncSetAttribute((const void*)k_col<T, true>, hipFuncAttributeMaxDynamicSharedMemorySize, lim));
  CS_HIP(hipFuncSetAttribute((const void*)k_row<T, ROW_HAPPLY>, hipFuncAttributeMaxDynamicSharedMemorySize, lim));
  CS_HIP(hipFuncSetAttribute((const void*)k_row<T, ROW_RESID>, hipFuncAttributeMaxDynamicSharedMemorySize, lim));
  CS_HIP(hipFuncSetAttribute((const void*)k_row<T, ROW_FWD>, hipFuncAttributeMaxDynamicSharedMemorySize, lim));
  CS_HIP(hipFuncSetAttribute((const void*)k_row<T, ROW_ADJ>, hipFuncAttributeMaxDynamicSharedMemorySize, lim));
  done = true;
}

// ------------------------------------------------------------------ instantiations
#define CS_INST(T)                                                              \
  template void fill<T>(T*, int64_t, T, hipStream_t);                           \
  template double norm2_host<T>(Ctx<T>&, const T*, int64_t);                    \
  template void setup_operator<T>(Ctx<T>&);                                     \
  template void scatter_freq<T>(Ctx<T>&, const T*, T*);                         \
  template void gather_freq<T>(Ctx<T>&, const T*, T*);                          \
  template void transform_happly<T>(Ctx<T>&, const T*, const int*);             \
  template void transform_resid<T>(Ctx<T>&, const T*);                          \
  template void transform_fwd<T>(Ctx<T>&, const T*, T*);                        \
  template void transform_adj<T>(Ctx<T>&, const T*);                            \
  template void perm_in<T>(Ctx<T>&, const T*, T*);                              \
  template void perm_out<T>(Ctx<T>&, const T*, T*);                             \
  template void prepare_kernels<T>();                                           \
  template void scatter_signed<T>(Ctx<T>&, T*, const int32_t*, const T*, int); \
  template void scatter_zero<T>(Ctx<T>&, T*, const int32_t*, int);             \
  template void gather_signed<T>(Ctx<T>&, const T*, const int32_t*, T*, int);
CS_INST(float)
CS_INST(double)
template void fill<int32_t>(int32_t*, int64_t, int32_t, hipStream_t);
template void fill<uint32_t>(uint32_t*, int64_t, uint32_t, hipStream_t);

}  // namespace csr
