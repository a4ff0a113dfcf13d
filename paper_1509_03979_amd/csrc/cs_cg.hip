// CG subsystem: the CG function of Algorithm 1 (lines 11-24) on the weighted
// normal equations of Eq. (11),
//     H theta = b,   H = W_S A^T A W_S,   b = W_S A^T y,
// restricted to the support S (the rows and columns of H off S are zero, so
// the iteration lives on compact |S|-vectors, Theorem 5's argument).
//
//   r_0 = b - H x_0 (x_0 = 0: r_0 = b), d_0 = r_0
//   alpha = r^T r / d^T H d;  x += alpha d;  r -= alpha H d
//   beta = r_new^T r_new / r^T r;  d = r_new + beta d
// until ||r|| <= tol ||b|| (relative form of the line-15 test).
//
// H d is one pass of the transform subsystem over the dense direction buffer
// (sign flip and scatter of d onto S are fused into the update kernel that
// produces d).  Inner products are accumulated in FP64 with a fixed-order
// two-level reduction (per-block partials, then every consumer block sums the
// partials in the same order), so results are run-to-run deterministic.
// Scalars stay on the device; the host queues iterations in chunks and reads
// the `done` flag between chunks.
#include "cs_internal.h"

#include <algorithm>
#include <cmath>

namespace csr {

static inline int red_blocks(int k) { return std::max(1, std::min(kRedBlocks, (k + kRedThreads - 1) / kRedThreads)); }

// Block sum broadcast to all threads (blockDim.x == kRedThreads).
__device__ __forceinline__ double block_sum(double v) {
  __shared__ double sh[kRedThreads / 64];
  __shared__ double res;
  for (int off = 32; off > 0; off >>= 1) v += __shfl_down(v, off, 64);
  if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = v;
  __syncthreads();
  if (threadIdx.x == 0) {
    double s = 0.0;
    for (int i = 0; i < kRedThreads / 64; ++i) s += sh[i];
    res = s;
  }
  __syncthreads();
  return res;
}

__device__ __forceinline__ double sum_partials(const double* __restrict__ p, int np) {
  double s = 0.0;
  for (int i = threadIdx.x; i < np; i += blockDim.x) s += p[i];
  return block_sum(s);
}

template <typename T>
__device__ __forceinline__ T sgn_apply(int8_t s, T v) { return s < 0 ? -v : v; }

// b_i = sign_j * C0[vpos(j)], j = S_i;  partial b^T b
template <typename T>
__global__ void k_cg_gather_b(const T* __restrict__ C0, const int32_t* __restrict__ list, int k,
                              const int8_t* __restrict__ signs, int64_t n, T* __restrict__ b,
                              double* __restrict__ pbb) {
  double acc = 0.0;
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < k; i += gridDim.x * blockDim.x) {
    const int64_t j = list[i];
    const T v = sgn_apply(signs[j], C0[vpos(j, n)]);
    b[i] = v;
    acc += (double)v * (double)v;
  }
  acc = block_sum(acc);
  if (threadIdx.x == 0) pbb[blockIdx.x] = acc;
}

// x = 0, r = d = b, Dd[vpos(S_i)] = sign * d_i;  partial r^T r
template <typename T>
__global__ void k_cg_init_cold(const T* __restrict__ b, T* __restrict__ x, T* __restrict__ r, T* __restrict__ d,
                               T* __restrict__ Dd, const int32_t* __restrict__ list, int k,
                               const int8_t* __restrict__ signs, int64_t n, double* __restrict__ prr) {
  double acc = 0.0;
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < k; i += gridDim.x * blockDim.x) {
    const T v = b[i];
    x[i] = (T)0;
    r[i] = v;
    d[i] = v;
    const int64_t j = list[i];
    Dd[vpos(j, n)] = sgn_apply(signs[j], v);
    acc += (double)v * (double)v;
  }
  acc = block_sum(acc);
  if (threadIdx.x == 0) prr[blockIdx.x] = acc;
}

// After W = H x0 (v-order): r = b - (H x0)_S, d = r, Dd = sign * d on S.
template <typename T>
__global__ void k_cg_init_warm(const T* __restrict__ Wv, const T* __restrict__ b, T* __restrict__ r,
                               T* __restrict__ d, T* __restrict__ Dd, const int32_t* __restrict__ list, int k,
                               const int8_t* __restrict__ signs, int64_t n, double* __restrict__ prr) {
  double acc = 0.0;
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < k; i += gridDim.x * blockDim.x) {
    const int64_t j = list[i];
    const int64_t p = vpos(j, n);
    const int8_t s = signs[j];
    const T v = b[i] - sgn_apply(s, Wv[p]);
    r[i] = v;
    d[i] = v;
    Dd[p] = sgn_apply(s, v);
    acc += (double)v * (double)v;
  }
  acc = block_sum(acc);
  if (threadIdx.x == 0) prr[blockIdx.x] = acc;
}

__global__ void k_cg_start(CgScalars* cg, const double* __restrict__ prr, const double* __restrict__ pbb, int np,
                           double tol2, int max_iter) {
  const double rr = sum_partials(prr, np);
  const double bb = sum_partials(pbb, np);
  if (threadIdx.x == 0) {
    cg->rr[0] = rr;
    cg->rr[1] = rr;
    cg->bb = bb;
    cg->tol2 = tol2;
    cg->iters = 0;
    cg->flags = 0;
    const bool fin = isfinite(rr) && isfinite(bb);
    if (!fin) cg->flags |= CS_F_NONFINITE;
    cg->done = (!fin || rr <= tol2 * bb || max_iter <= 0) ? 1 : 0;
  }
}

// q_i = sign * W[vpos(S_i)];  partial d^T q
template <typename T>
__global__ void k_cg_q(const T* __restrict__ Wv, const int32_t* __restrict__ list, int k,
                       const int8_t* __restrict__ signs, int64_t n, const T* __restrict__ d, T* __restrict__ q,
                       double* __restrict__ pdq, const CgScalars* __restrict__ cg) {
  if (cg->done) return;
  double acc = 0.0;
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < k; i += gridDim.x * blockDim.x) {
    const int64_t j = list[i];
    const T v = sgn_apply(signs[j], Wv[vpos(j, n)]);
    q[i] = v;
    acc += (double)d[i] * (double)v;
  }
  acc = block_sum(acc);
  if (threadIdx.x == 0) pdq[blockIdx.x] = acc;
}

// alpha = rr / dq; x += alpha d; r -= alpha q; partial r^T r
template <typename T>
__global__ void k_cg_xr(T* __restrict__ x, T* __restrict__ r, const T* __restrict__ d, const T* __restrict__ q,
                        int k, const double* __restrict__ pdq, double* __restrict__ prr, CgScalars* cg, int np,
                        int it) {
  if (cg->done) return;
  const double dq = sum_partials(pdq, np);
  const double rr = cg->rr[it & 1];
  if (!(dq > 0.0) || !isfinite(dq)) {           // H not positive on d (Theorem 3 fails)
    if (blockIdx.x == 0 && threadIdx.x == 0) {
      cg->flags |= CS_F_CG_BREAKDOWN;
      cg->done = 1;
    }
    return;
  }
  const T alpha = (T)(rr / dq);
  double acc = 0.0;
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < k; i += gridDim.x * blockDim.x) {
    x[i] += alpha * d[i];
    const T rv = r[i] - alpha * q[i];
    r[i] = rv;
    acc += (double)rv * (double)rv;
  }
  acc = block_sum(acc);
  if (threadIdx.x == 0) prr[blockIdx.x] = acc;
}

// beta = rr_new / rr; d = r + beta d; Dd = sign * d on S; convergence test.
template <typename T>
__global__ void k_cg_d(const T* __restrict__ r, T* __restrict__ d, T* __restrict__ Dd,
                       const int32_t* __restrict__ list, int k, const int8_t* __restrict__ signs, int64_t n,
                       const double* __restrict__ prr, CgScalars* cg, int np, int it, int max_iter) {
  if (cg->done) return;
  const double rr_new = sum_partials(prr, np);
  const double rr = cg->rr[it & 1];
  const T beta = (T)(rr_new / rr);
  const bool conv = rr_new <= cg->tol2 * cg->bb;
  if (!conv) {
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < k; i += gridDim.x * blockDim.x) {
      const T dv = r[i] + beta * d[i];
      d[i] = dv;
      const int64_t j = list[i];
      Dd[vpos(j, n)] = sgn_apply(signs[j], dv);
    }
  }
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    cg->rr[(it + 1) & 1] = rr_new;
    cg->iters = it + 1;
    if (!isfinite(rr_new)) cg->flags |= CS_F_NONFINITE;
    if (conv || !isfinite(rr_new) || it + 1 >= max_iter) cg->done = 1;
  }
}

template <typename T>
int cg_solve(Ctx<T>& c, const int32_t* list, int k, T* x, bool warm, double tol, int max_iter) {
  hipStream_t s = c.stream;
  const int64_t n = c.plan.n;
  const int nb = red_blocks(k);
  double* prr = c.partial;
  double* pbb = c.partial + kRedBlocks;
  double* pdq = c.partial + 2 * kRedBlocks;
  fill<T>(c.Dd, n, (T)0, s);
  hipLaunchKernelGGL(k_cg_gather_b<T>, dim3(nb), dim3(kRedThreads), 0, s, c.C0, list, k, c.signs, n, c.cb, pbb);
  CS_LAUNCH_CHECK();
  if (warm) {
    scatter_signed<T>(c, c.Dd, list, x, k);
    transform_happly<T>(c, c.Dd, nullptr);
    hipLaunchKernelGGL(k_cg_init_warm<T>, dim3(nb), dim3(kRedThreads), 0, s, (const T*)c.W, c.cb, c.cr, c.cd,
                       c.Dd, list, k, c.signs, n, prr);
  } else {
    hipLaunchKernelGGL(k_cg_init_cold<T>, dim3(nb), dim3(kRedThreads), 0, s, c.cb, x, c.cr, c.cd, c.Dd, list, k,
                       c.signs, n, prr);
  }
  CS_LAUNCH_CHECK();
  hipLaunchKernelGGL(k_cg_start, dim3(1), dim3(kRedThreads), 0, s, c.cg, prr, pbb, nb, tol * tol, max_iter);
  CS_LAUNCH_CHECK();
  const int* done = &c.cg->done;
  // Iterations are queued in chunks; the host reads the device flags between
  // chunks.  After the first chunk the next one is sized from the observed
  // geometric rate of r^T r so that few early-exit launches are queued.
  int it = 0;
  int chunk = std::min(4, std::max(max_iter, 1));
  CgScalars host{};
  double rr_prev = -1.0;
  int it_prev = 0;
  while (it < max_iter) {
    const int q = std::min(chunk, max_iter - it);
    for (int u = 0; u < q; ++u, ++it) {
      transform_happly<T>(c, c.Dd, done);
      hipLaunchKernelGGL(k_cg_q<T>, dim3(nb), dim3(kRedThreads), 0, s, (const T*)c.W, list, k, c.signs, n, c.cd,
                         c.cq, pdq, c.cg);
      CS_LAUNCH_CHECK();
      hipLaunchKernelGGL(k_cg_xr<T>, dim3(nb), dim3(kRedThreads), 0, s, x, c.cr, c.cd, c.cq, k, pdq, prr, c.cg,
                         nb, it);
      CS_LAUNCH_CHECK();
      hipLaunchKernelGGL(k_cg_d<T>, dim3(nb), dim3(kRedThreads), 0, s, c.cr, c.cd, c.Dd, list, k, c.signs, n, prr,
                         c.cg, nb, it, max_iter);
      CS_LAUNCH_CHECK();
    }
    dev_read(s, c.cg, &host, sizeof(CgScalars));
    if (host.done) break;
    const double rr_now = host.rr[host.iters & 1];
    const double target = host.tol2 * host.bb;
    const double rr_ref = (rr_prev > 0.0) ? rr_prev : host.rr[0];
    const int span = (rr_prev > 0.0) ? (host.iters - it_prev) : host.iters;
    int next = 2;
    if (span > 0 && rr_ref > 0.0 && rr_now > 0.0 && rr_now < rr_ref && target > 0.0) {
      const double rate = std::log(rr_now / rr_ref) / span;      // log decrease per iteration (< 0)
      const double need = std::log(target / rr_now) / rate;      // iterations still needed
      if (std::isfinite(need)) next = (int)std::ceil(need);
    }
    chunk = std::max(1, std::min(next, 64));
    rr_prev = rr_now;
    it_prev = host.iters;
  }
  if (!host.done) dev_read(s, c.cg, &host, sizeof(CgScalars));
  const bool conv = host.rr[host.iters & 1] <= host.tol2 * host.bb;
  if (!conv && !(host.flags & CS_F_CG_BREAKDOWN)) c.flags |= CS_F_CG_MAXITER;
  c.flags |= host.flags;
  c.cg_iters += host.iters;
  return host.iters;
}

template <typename T>
double resid_corr(Ctx<T>& c, const int32_t* old_list, int old_k, const int32_t* list, const T* x, int k) {
  if (old_list && old_k > 0) scatter_zero<T>(c, c.Dx, old_list, old_k);
  scatter_signed<T>(c, c.Dx, list, x, k);
  transform_resid<T>(c, c.Dx);
  double r2 = 0.0;
  dev_read(c.stream, &c.cg->resid2, &r2, sizeof(double));
  return std::sqrt(r2);
}

template int cg_solve<float>(Ctx<float>&, const int32_t*, int, float*, bool, double, int);
template int cg_solve<double>(Ctx<double>&, const int32_t*, int, double*, bool, double, int);
template double resid_corr<float>(Ctx<float>&, const int32_t*, int, const int32_t*, const float*, int);
template double resid_corr<double>(Ctx<double>&, const int32_t*, int, const int32_t*, const double*, int);

}  // namespace csr
