// Separable 2-D DCT sparsifying basis (Sec. III-E: Psi = Psi_2 (x) Psi_1 with
// x = vec(Psi_1 S Psi_2^T)), here with both factors the orthonormal DCT-II F_n
// of the image side n = sqrt(N):  x = vec(F_n S F_n^T) (row-major vec), and
// Psi^T x = vec(F_n^T X F_n).
//
// Each 2-D transform is two launches of one kernel that transforms every row
// of an n x n image and writes the result transposed: applied twice it gives
// F S F^T (forward, DCT-II rows) or F^T X F (inverse, DCT-III rows).  A row's
// DCT runs through an n/2-point complex FFT in LDS (Makhoul's even/odd
// reordering, as for the N-point transform): z_m = v_2m + i v_2m+1 with
// v_m = x_2m, v_{n-1-m} = x_2m+1; Z = FFT(z); the DCT outputs of k and n-k
// come from Z_k and Z_{n/2-k}.  The inverse runs these steps backwards.
#include "cs_kernels.h"

namespace csr {

// rows per workgroup: up to 4096 (FP32) / 2048 (FP64) complex LDS elements
template <typename T>
__host__ __device__ constexpr int dct2d_logr(int logc) {
  const int cap = sizeof(T) == 4 ? 12 : 11;
  const int logh = logc - 1;
  const int r = cap - logh;
  return r < 0 ? 0 : (r > logc ? logc : r);
}
template <typename T, int LOGC>
__host__ __device__ constexpr int dct2d_nt() {
  return nt_for((1 << dct2d_logr<T>(LOGC)) << (LOGC - 1), 2);
}

template <typename T, int LOGC, bool INV>
__global__ __launch_bounds__((dct2d_nt<T, LOGC>())) void k_dct_rows(const T* __restrict__ in, T* __restrict__ out,
                                                                   const Plan p, const Cx<T>* __restrict__ tw,
                                                                   const int* __restrict__ done) {
  if (done && *done) return;
  constexpr int C = 1 << LOGC, H = C >> 1, LOGH = LOGC - 1;
  constexpr int LOGR = dct2d_logr<T>(LOGC), RPW = 1 << LOGR;
  constexpr int NT = dct2d_nt<T, LOGC>();
  __shared__ Cx<T> lds[lp_size(RPW * H)];
  T* ldr = reinterpret_cast<T*>(lds);
  const int tid = threadIdx.x;
  const int r0 = blockIdx.x * RPW;
  const T c0 = (T)sqrt(1.0 / (double)C), c1 = (T)sqrt(2.0 / (double)C);
  // W_{4N}^i with N = C^2: W_C^k = W_{4N}^{4Ck}, e^{-i pi k / (2C)} = W_{4N}^{Ck}
  if (!INV) {
    // x_j of row f -> v position vp -> z slot vp / 2, half vp % 2
    for (int e = tid; e < RPW * C; e += NT) {
      const int f = e >> LOGC, j = e & (C - 1);
      const int vp = (j & 1) ? (C - 1 - (j >> 1)) : (j >> 1);
      ldr[2 * lp(f * H + (vp >> 1)) + (vp & 1)] = in[(size_t)(r0 + f) * C + j];
    }
    __syncthreads();
    ct_fft<T, false, NT, LOGH, LOGR, false, 2>(lds, tw);
    // item (f, k), k in [0, H/2]: outputs k, C-k and (for k' = H-k != k) k', C-k'
    constexpr int NI = (H >> 1) + 1;
    for (int t = tid; t < RPW * NI; t += NT) {
      const int f = t & (RPW - 1), k = t >> LOGR;
      const size_t col = (size_t)(r0 + f);
      const Cx<T> Zk = lds[lp(f * H + (k == 0 ? 0 : k))];
      if (k == 0) {
        out[col] = c0 * (Zk.re + Zk.im);                              // X_0
        out[(size_t)H * C + col] = c0 * (Zk.re - Zk.im);              // X_H = c_H (re - im) / sqrt 2
        continue;
      }
#pragma unroll
      for (int s = 0; s < 2; ++s) {
        const int kk = s ? H - k : k;
        if (s && kk == k) break;
        const Cx<T> A = lds[lp(f * H + kk)], B = lds[lp(f * H + H - kk)];
        const Cx<T> E = scale(A + conj(B), (T)0.5);
        const Cx<T> D = A - conj(B);
        const Cx<T> O = cx(D.im * (T)0.5, -D.re * (T)0.5);          // D / (2i)
        const Cx<T> V = E + cmul(tw4n<T>(p, (uint32_t)(4 * C * kk)), O);
        const Cx<T> a = cmul(tw4n<T>(p, (uint32_t)(C * kk)), V);
        out[(size_t)kk * C + col] = c1 * a.re;                        // X_kk
        out[(size_t)(C - kk) * C + col] = -c1 * a.im;                 // X_{C-kk}
      }
    }
  } else {
    // X_j of row f in natural order at complex slot j / 2, half j % 2
    for (int e = tid; e < RPW * C; e += NT) {
      const int f = e >> LOGC, j = e & (C - 1);
      ldr[2 * lp(f * H + (j >> 1)) + (j & 1)] = in[(size_t)(r0 + f) * C + j];
    }
    __syncthreads();
    // item (f, k), k in [0, H/2]: Z_k and Z_{H-k} from X_k, X_{C-k}, X_{H+k}, X_{H-k}
    constexpr int NI = (H >> 1) + 1;
    constexpr int MAXQ = (RPW * NI + NT - 1) / NT;
    auto xat = [&](int f, int j) -> T { return ldr[2 * lp(f * H + (j >> 1)) + (j & 1)]; };
    Cx<T> za[MAXQ], zb[MAXQ];
#pragma unroll
    for (int q = 0; q < MAXQ; ++q) {
      const int t = tid + q * NT;
      if (t >= RPW * NI) break;
      const int f = t & (RPW - 1), k = t >> LOGR;
      // V(j) = e^{i pi j / (2C)} (X_j / c_j - i X_{C-j} / c_{C-j}), V(0) = X_0 / c_0
      auto V = [&](int j) -> Cx<T> {
        if (j == 0) return cx(xat(f, 0) / c0, (T)0);
        const Cx<T> u = cx(xat(f, j) / c1, -xat(f, C - j) / c1);
        return cmulc(u, tw4n<T>(p, (uint32_t)(C * j)));               // times conj(W_{4C}^j)
      };
#pragma unroll
      for (int s = 0; s < 2; ++s) {
        const int kk = s ? H - k : k;
        Cx<T> z = cx((T)0, (T)0);
        if (!(s && (kk == k || k == 0))) {
          const Cx<T> a = V(kk), b = V(kk + H);
          const Cx<T> E = scale(a + b, (T)0.5);
          const Cx<T> O = cmulc(scale(a - b, (T)0.5), tw4n<T>(p, (uint32_t)(4 * C * kk)));   // times e^{+2 pi i kk / C}
          z = cx(E.re - O.im, E.im + O.re);                           // E + i O
        }
        if (s) zb[q] = z; else za[q] = z;
      }
    }
    __syncthreads();
#pragma unroll
    for (int q = 0; q < MAXQ; ++q) {
      const int t = tid + q * NT;
      if (t >= RPW * NI) break;
      const int f = t & (RPW - 1), k = t >> LOGR;
      lds[lp(f * H + k)] = za[q];
      if (k != 0 && H - k != k) lds[lp(f * H + H - k)] = zb[q];
    }
    __syncthreads();
    ct_fft<T, true, NT, LOGH, LOGR, false, 2>(lds, tw);
    const T sc = (T)(1.0 / (double)H);
    for (int t = tid; t < RPW * C; t += NT) {
      const int f = t & (RPW - 1), j = t >> LOGR;
      const int vp = (j & 1) ? (C - 1 - (j >> 1)) : (j >> 1);
      const Cx<T> z = lds[lp(f * H + (vp >> 1))];
      out[(size_t)j * C + (r0 + f)] = sc * ((vp & 1) ? z.im : z.re);
    }
  }
}

// ------------------------------------------------------------------ host
template <typename T, int LOGC>
static void dct_launch(bool inv, const T* in, T* out, const Plan& p, const Cx<T>* tw, const int* done,
                       hipStream_t s) {
  constexpr int blocks = (1 << LOGC) >> dct2d_logr<T>(LOGC);
  constexpr int nt = dct2d_nt<T, LOGC>();
  if (inv) hipLaunchKernelGGL((k_dct_rows<T, LOGC, true>), dim3(blocks), dim3(nt), 0, s, in, out, p, tw, done);
  else hipLaunchKernelGGL((k_dct_rows<T, LOGC, false>), dim3(blocks), dim3(nt), 0, s, in, out, p, tw, done);
  CS_LAUNCH_CHECK();
}

int dct2d_side_log(cs_dtype dt, int64_t n) {
  int l = 0;
  while ((int64_t(1) << l) < n) ++l;
  if ((int64_t(1) << l) != n || (l & 1)) return -1;
  const int h = l / 2;
  if (h < kDct2dMinLog || h > (dt == CS_F64 ? kDct2dMaxLog64 : kDct2dMaxLog32)) return -1;
  return h;
}

// One row pass: rows of `in` (n x n) transformed, written transposed to `out`.
template <typename T>
static void dct_rows(Ctx<T>& c, bool inv, const T* in, T* out, const int* done) {
  const int h = c.dct_log;
  const Plan& p = c.plan;
  hipStream_t s = c.stream;
  switch (h) {
    case 3: dct_launch<T, 3>(inv, in, out, p, c.tw_dct, done, s); break;
    case 4: dct_launch<T, 4>(inv, in, out, p, c.tw_dct, done, s); break;
    case 5: dct_launch<T, 5>(inv, in, out, p, c.tw_dct, done, s); break;
    case 6: dct_launch<T, 6>(inv, in, out, p, c.tw_dct, done, s); break;
    case 7: dct_launch<T, 7>(inv, in, out, p, c.tw_dct, done, s); break;
    case 8: dct_launch<T, 8>(inv, in, out, p, c.tw_dct, done, s); break;
    case 9: dct_launch<T, 9>(inv, in, out, p, c.tw_dct, done, s); break;
    case 10: dct_launch<T, 10>(inv, in, out, p, c.tw_dct, done, s); break;
    case 11: dct_launch<T, 11>(inv, in, out, p, c.tw_dct, done, s); break;
    case 12: dct_launch<T, 12>(inv, in, out, p, c.tw_dct, done, s); break;
    case 13:
      if constexpr (sizeof(T) == 4) dct_launch<T, 13>(inv, in, out, p, c.tw_dct, done, s);
      else throw Error(CS_E_SHAPE, "the FP64 2-D DCT basis takes n <= 4096");
      break;
    default: throw Error(CS_E_SHAPE, "unsupported 2-D DCT side");
  }
}

// out = vec(F S F^T) (inv = false) or vec(F^T S F) (inv = true); tmp is an N-vector.
template <typename T>
void dct2d(Ctx<T>& c, bool inv, const T* in, T* tmp, T* out, const int* done) {
  dct_rows<T>(c, inv, in, tmp, done);
  dct_rows<T>(c, inv, tmp, out, done);
}

template <typename T>
void dct2d_setup(Ctx<T>& c) {
  const int logh = c.dct_log - 1;
  hipLaunchKernelGGL(k_stage_twiddles<T>, dim3(std::max(1, (tw_table_count(logh, 2) + 255) / 256)), dim3(256), 0,
                     c.stream, c.tw_dct, logh, 2);
  CS_LAUNCH_CHECK();
}

template void dct2d<float>(Ctx<float>&, bool, const float*, float*, float*, const int*);
template void dct2d<double>(Ctx<double>&, bool, const double*, double*, double*, const int*);
template void dct2d_setup<float>(Ctx<float>&);
template void dct2d_setup<double>(Ctx<double>&);

static_assert(tw_table_count(12, 2) <= kTwStage, "2-D DCT stage table");

}  // namespace csr
