// CG subsystem: the CG function of Algorithm 1 on the weighted
// normal equations of Eq. (11),
//     H theta = b,   H = W_S A^T A W_S,   b = W_S A^T y,
// restricted to the support S (rows and columns of H off S are zero, so the
// iteration lives on compact |S|-vectors, as in the proof of Theorem 5).
//
//   r_0 = b - H x_0 (x_0 = 0: r_0 = b), d_0 = r_0
//   alpha = r^T r / d^T H d;  x += alpha d;  r -= alpha H d
//   beta = r_new^T r_new / r^T r;  d = r_new + beta d
// until ||r|| <= tol ||b|| (relative form of the CG loop test of Algorithm 1).
//
// Compact vectors are ordered by key (the order of the column passes) and
// hold sign-flipped coordinates theta' = R theta, R = diag(+-1) the sign flip
// of the operator: H' = R H R and b' = R b give the same inner products, so the
// iterates are those of the plain CG, and the column passes move raw values.
// One iteration is four launches, the vector update riding on the passes:
//   1. forward column pass in COL_DIR mode: the previous iteration's
//      x += alpha d, r -= alpha q, then d = r + beta d on the support;
//   2. row pass (DCT post-processing, row mask of D, pre-processing);
//   3. inverse column pass in COL_Q mode: q = (H d)_S and per-workgroup FP64
//      partials of d^T q, r^T r, r^T q, q^T q;
//   4. one-workgroup step kernel: the partials summed in index order, alpha,
//      the next r^T r by expansion, beta and the stopping test.
// A finish kernel applies the last step once the solve has stopped.  Results
// are deterministic (fixed summation order).  Scalars stay on the device;
// every kernel of an iteration exits early once `done` is set, and the host
// reads the flags between chunks of queued iterations.
#include "cs_device.h"

#include <algorithm>
#include <cmath>
#include <vector>

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

// b'_i = (F^T D^T y)[k_i] for the support keys k_i; partial b^T b
template <typename T>
__global__ void k_cg_gather_b(const T* __restrict__ C0, const int32_t* __restrict__ list, int k,
                              T* __restrict__ b, double* __restrict__ pbb) {
  double acc = 0.0;
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < k; i += gridDim.x * blockDim.x) {
    const T v = C0[list[i]];
    b[i] = v;
    acc += (double)v * (double)v;
  }
  acc = block_sum(acc);
  if (threadIdx.x == 0) pbb[blockIdx.x] = acc;
}

// Both of the above in one pass when a warm start on a grown support also
// gathers b: b'_i = C0[k_i] (partial b^T b) and r = d = Cc[k_i] (partial r^T r).
template <typename T>
__global__ void k_cg_gather_b_corr(const T* __restrict__ C0, const T* __restrict__ cc,
                                   const int32_t* __restrict__ list, int k, T* __restrict__ b, T* __restrict__ r,
                                   T* __restrict__ d, double* __restrict__ pbb, double* __restrict__ prr) {
  double ab = 0.0, ar = 0.0;
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < k; i += gridDim.x * blockDim.x) {
    const int32_t key = list[i];
    const T v = C0[key], w = cc[key];
    b[i] = v;
    r[i] = w;
    d[i] = w;
    ab += (double)v * (double)v;
    ar += (double)w * (double)w;
  }
  ab = block_sum(ab);
  ar = block_sum(ar);
  if (threadIdx.x == 0) {
    pbb[blockIdx.x] = ab;
    prr[blockIdx.x] = ar;
  }
}

// partial b^T b of a right-hand side already in place
template <typename T>
__global__ void k_cg_bnorm(const T* __restrict__ b, int k, double* __restrict__ pbb) {
  double acc = 0.0;
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < k; i += gridDim.x * blockDim.x) {
    const double v = (double)b[i];
    acc += v * v;
  }
  acc = block_sum(acc);
  if (threadIdx.x == 0) pbb[blockIdx.x] = acc;
}

// warm start on a superset of the previous support: with x_0 the previous
// solution (zero on the new keys), A x_0 is the previous fit, so
// b - H x_0 = A_S^T (y - A x_prev) = the stored correlation on S.
// r = d = Cc[keys]; partial r^T r.
template <typename T>
__global__ void k_cg_init_corr(const T* __restrict__ cc, const int32_t* __restrict__ list, int k, T* __restrict__ r,
                               T* __restrict__ d, double* __restrict__ prr) {
  double acc = 0.0;
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < k; i += gridDim.x * blockDim.x) {
    const T v = cc[list[i]];
    r[i] = v;
    d[i] = v;
    acc += (double)v * (double)v;
  }
  acc = block_sum(acc);
  if (threadIdx.x == 0) prr[blockIdx.x] = acc;
}

// cold start: x = 0, r = b; partial r^T r
template <typename T>
__global__ void k_cg_init_cold(const T* __restrict__ b, T* __restrict__ x, T* __restrict__ r, int k,
                               double* __restrict__ prr) {
  double acc = 0.0;
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < k; i += gridDim.x * blockDim.x) {
    const T v = b[i];
    x[i] = (T)0;
    r[i] = v;
    acc += (double)v * (double)v;
  }
  acc = block_sum(acc);
  if (threadIdx.x == 0) prr[blockIdx.x] = acc;
}

__global__ void k_cg_start(CgScalars* cg, const double* __restrict__ prr, int nrr, const double* __restrict__ pbb,
                           int nbb, double tol2, int max_iter, int tol_abs) {
  const double rr = sum_partials(prr, nrr);
  const double bb = sum_partials(pbb, nbb);
  if (threadIdx.x == 0) {
    cg->rr[0] = rr;
    cg->rr[1] = rr;
    cg->bb = bb;
    cg->ref = tol_abs ? 1.0 : bb;
    cg->tol2 = tol2;
    cg->iters = 0;
    cg->flags = 0;
    cg->alpha = 0.0;
    const bool fin = isfinite(rr) && isfinite(bb);
    if (!fin) cg->flags |= CS_F_NONFINITE;
    cg->done = (!fin || rr <= tol2 * cg->ref || max_iter <= 0) ? 1 : 0;
  }
}

// Blocks of the compact element-wise kernels: kUpdUnroll elements per thread.
constexpr int kUpdUnroll = 8;
static inline int upd_blocks(int k) {
  const int per = kRedThreads * kUpdUnroll;
  return std::max(1, std::min(kRedBlocks, (k + per - 1) / per));
}

// The scalar CG step from the inverse pass's four partials per workgroup,
// summed in a fixed order (the kernel boundary makes them visible).
template <typename T>
__global__ void k_cg_step(CgScalars* cg, const double* __restrict__ part, int g, int it, int max_iter) {
  if (cg->done) return;
  __shared__ double red4[4][kRedThreads / 64];
  double v[4] = {0.0, 0.0, 0.0, 0.0};
  for (int i = threadIdx.x; i < g; i += blockDim.x) {
#pragma unroll
    for (int j = 0; j < 4; ++j) v[j] += part[j * g + i];
  }
  const double4 t = wg_sum4<kRedThreads / 64>(v[0], v[1], v[2], v[3], red4);
  if (threadIdx.x == 0) cg_step_fused(cg, t, it, max_iter, (T)0);
}

// The last iteration's x += alpha d, r -= alpha q when the column passes carry
// the CG update (they apply each iteration's step at the start of the next
// one, and no pass runs after the solve has stopped).  alpha = 0 when no step
// is pending (no iteration, or a breakdown).
template <typename T>
__global__ void k_cg_finish(T* __restrict__ x, T* __restrict__ r, const T* __restrict__ d, const T* __restrict__ q,
                            int k, const CgScalars* __restrict__ cg) {
  const T alpha = (T)cg->alpha;
  if (alpha == (T)0) return;
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < k; i += gridDim.x * blockDim.x) {
    x[i] = x[i] + alpha * d[i];
    r[i] = r[i] - alpha * q[i];
  }
}

// ---- separable 2-D DCT basis: compact vectors <-> the support of the
// zero-padded image P3 (keys are natural indices; the support is fixed within
// a solve, so P3 is cleared once per solve)
template <typename T>
__global__ void k_s2_scatter(const T* __restrict__ v, const int32_t* __restrict__ list, int k, T* __restrict__ img) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < k) img[list[i]] = v[i];
}

// d = r (iteration 0) or r + beta d on the support, scattered into the image;
// from iteration 1 on, first the previous step x += alpha d, r -= alpha q (as
// the forward column pass does for the four-step operator)
template <typename T>
__global__ void k_s2_dir(T* __restrict__ x, T* __restrict__ r, T* __restrict__ d, const T* __restrict__ q,
                         const int32_t* __restrict__ list, int k, T* __restrict__ img,
                         const CgScalars* __restrict__ cg, int it) {
  if (cg->done) return;
  const T beta = it == 0 ? (T)0 : (T)cg->beta;
  const T alpha = it == 0 ? (T)0 : (T)cg->alpha;
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < k; i += gridDim.x * blockDim.x) {
    T v = r[i];
    if (it > 0) {
      const T dv = d[i];
      x[i] = x[i] + alpha * dv;
      v = v - alpha * q[i];
      r[i] = v;
      v = v + beta * dv;
    }
    d[i] = v;
    img[list[i]] = v;
  }
}

// q = (H d)_S gathered from the transformed image, with per-block partials of
// d^T q, r^T r, r^T q and q^T q (rows of gridDim.x) for the step kernel.
template <typename T>
__global__ void k_s2_q(const T* __restrict__ sout, const int32_t* __restrict__ list, int k, const T* __restrict__ d,
                       const T* __restrict__ r, T* __restrict__ q, double* __restrict__ part,
                       const CgScalars* __restrict__ cg) {
  if (cg->done) return;
  double a_dq = 0.0, a_rr = 0.0, a_rq = 0.0, a_qq = 0.0;
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < k; i += gridDim.x * blockDim.x) {
    const T v = sout[list[i]];
    q[i] = v;
    const double qv = (double)v, dv = (double)d[i], rv = (double)r[i];
    a_dq += dv * qv;
    a_rr += rv * rv;
    a_rq += rv * qv;
    a_qq += qv * qv;
  }
  __shared__ double red4[4][kRedThreads / 64];
  const double4 t = wg_sum4<kRedThreads / 64>(a_dq, a_rr, a_rq, a_qq, red4);
  if (threadIdx.x == 0) {
    const int g = (int)gridDim.x;
    part[blockIdx.x] = t.x;
    part[g + blockIdx.x] = t.y;
    part[2 * g + blockIdx.x] = t.z;
    part[3 * g + blockIdx.x] = t.w;
  }
}

// warm start: r = b - (H x0)_S, d = r, partial r^T r per block
template <typename T>
__global__ void k_s2_r(const T* __restrict__ sout, const int32_t* __restrict__ list, int k, const T* __restrict__ b,
                       T* __restrict__ r, T* __restrict__ d, double* __restrict__ prr) {
  double acc = 0.0;
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < k; i += gridDim.x * blockDim.x) {
    const T v = b[i] - sout[list[i]];
    r[i] = v;
    d[i] = v;
    acc += (double)v * (double)v;
  }
  acc = block_sum(acc);
  if (threadIdx.x == 0) prr[blockIdx.x] = acc;
}

template <typename T>
static void s2_scatter(Ctx<T>& c, const Supp& S, const T* v) {
  hipLaunchKernelGGL(k_s2_scatter<T>, dim3(std::max(1, (S.k + 255) / 256)), dim3(256), 0, c.stream, v, S.list, S.k,
                     c.P3);
  CS_LAUNCH_CHECK();
}

template <typename T>
int cg_solve(Ctx<T>& c, const Supp& S, T* x, bool warm, double tol, int max_iter, bool b_ready, bool r0_corr) {
  hipStream_t s = c.stream;
  const int k = S.k;
  const int nb = red_blocks(k);
  const int ncol = (int)(c.plan.L2 >> c.plan.logB);   // column-pass workgroups
  double* prr = c.partial;
  double* pbb = c.partial + kRedBlocks;
  double* pdq = c.pgrid;
  const bool corr = warm && r0_corr;
  if (b_ready) hipLaunchKernelGGL(k_cg_bnorm<T>, dim3(nb), dim3(kRedThreads), 0, s, c.cb, k, pbb);
  else if (corr)
    hipLaunchKernelGGL(k_cg_gather_b_corr<T>, dim3(nb), dim3(kRedThreads), 0, s, c.C0, (const T*)c.Cc, S.list, k,
                       c.cb, c.cr, c.cd, pbb, prr);
  else hipLaunchKernelGGL(k_cg_gather_b<T>, dim3(nb), dim3(kRedThreads), 0, s, c.C0, S.list, k, c.cb, pbb);
  CS_LAUNCH_CHECK();
  if (corr) {
    if (b_ready) {
      hipLaunchKernelGGL(k_cg_init_corr<T>, dim3(nb), dim3(kRedThreads), 0, s, (const T*)c.Cc, S.list, k, c.cr,
                         c.cd, prr);
      CS_LAUNCH_CHECK();
    }
    hipLaunchKernelGGL(k_cg_start, dim3(1), dim3(kRedThreads), 0, s, c.cg, prr, nb, pbb, nb, tol * tol, max_iter,
                       c.tol_abs);
  } else if (warm && c.psi == 2) {
    fill<T>(c.P3, c.plan.n, (T)0, s);
    s2_scatter<T>(c, S, x);
    psi2_happly<T>(c, nullptr, c.P1);
    hipLaunchKernelGGL(k_s2_r<T>, dim3(nb), dim3(kRedThreads), 0, s, (const T*)c.P1, S.list, k, (const T*)c.cb, c.cr,
                       c.cd, prr);
    CS_LAUNCH_CHECK();
    hipLaunchKernelGGL(k_cg_start, dim3(1), dim3(kRedThreads), 0, s, c.cg, prr, nb, pbb, nb, tol * tol, max_iter,
                       c.tol_abs);
  } else if (warm) {
    // r = b - H x0, d = r through the transform, partial r^T r per column workgroup
    ColIO<T> in = col_io<T>(c, COL_X, &S);
    in.x = x;
    launch_col<T>(c, nullptr, c.W, false, in);
    if (c.psi) psi_middle<T>(c, nullptr, nullptr);
    else launch_row<T>(c, ROW_HAPPLY, nullptr, nullptr, nullptr, nullptr);
    ColIO<T> out = col_io<T>(c, COL_R, &S);
    out.r = c.cr;
    out.d = c.cd;
    out.b = c.cb;
    out.pout = c.pgrid;
    launch_col<T>(c, c.W, nullptr, true, out);
    c.transforms += 2;
    hipLaunchKernelGGL(k_cg_start, dim3(1), dim3(kRedThreads), 0, s, c.cg, c.pgrid, ncol, pbb, nb, tol * tol,
                       max_iter, c.tol_abs);
  } else {
    hipLaunchKernelGGL(k_cg_init_cold<T>, dim3(nb), dim3(kRedThreads), 0, s, c.cb, x, c.cr, k, prr);
    CS_LAUNCH_CHECK();
    hipLaunchKernelGGL(k_cg_start, dim3(1), dim3(kRedThreads), 0, s, c.cg, prr, nb, pbb, nb, tol * tol, max_iter, c.tol_abs);
  }
  CS_LAUNCH_CHECK();

  // The CG update is fused into the passes around each H-apply: the inverse
  // pass (or the gather from the 2-D basis image) writes per-workgroup
  // partials, a one-workgroup step kernel takes the scalar step, and the next
  // forward pass (or scatter) moves x, r and d; a finish kernel applies the
  // last step once the solve has stopped.
  const bool fused = c.psi != 2;   // (the column-pass I/O below; the 2-D basis has its own kernels)
  ColIO<T> dir = col_io<T>(c, COL_DIR, &S);
  dir.r = c.cr;
  dir.d = c.cd;
  dir.cg = c.cg;
  dir.fused = fused;
  dir.x = x;
  dir.q = c.cq;
  ColIO<T> qio = col_io<T>(c, COL_Q, &S);
  qio.q = c.cq;
  qio.d = c.cd;
  qio.r = c.cr;
  qio.pout = pdq;
  qio.cg = c.cg;
  qio.fused = fused;
  qio.max_iter = max_iter;

  const int* done = &c.cg->done;

  // Iterations are queued in chunks; the host reads the flags after each
  // chunk.  After the first read the chunks are sized from the observed
  // geometric rate of r^T r so that few early-exit launches are queued.
  int it = 0;
  // The first chunk: the iterations the last solve of this size and start
  // took, plus one (early-exiting kernels cost less than a host round trip);
  // else 4 from a cold start and 2 from a warm one.  A warm start is capped
  // by the most recent warm solve plus two: once the greedy support settles,
  // warm starts converge in few iterations (or none), whatever the same-size
  // solve of an earlier round took, and queued iterations would all exit.
  int first = warm ? 2 : 4;
  bool hinted = false;
  for (int h = 0; h < 4; ++h)
    if (c.hint[h].k == k && c.hint[h].warm == (int)warm) {
      first = std::max(1, c.hint[h].it + 1);
      hinted = true;
      break;
    }
  if (warm && c.last_warm_it >= 0) first = std::min(first, c.last_warm_it + 2);
  CgScalars host{};
  double rr_prev = -1.0;
  int it_prev = 0;
  // Queued iterations past convergence exit at once; their launches are taken
  // out of the counters and the timing records once the count is known.
  // With a DCT basis the H-apply runs on Psi's column passes with Phi^T Phi
  // (and the two reorders through R) in between.
  struct Queued { int rec[7]; double bytes; };
  std::vector<Queued> queued;
  const int per_it = c.psi ? 4 : 2;   // transforms per iteration
  if (c.psi == 2 && !(warm && !r0_corr)) fill<T>(c.P3, c.plan.n, (T)0, s);   // (cleared above otherwise)
  auto queue_chunk = [&](int q) {
    for (int u = 0; u < q; ++u, ++it) {
      dir.it = it;
      qio.it = it;
      Queued qd{{-1, -1, -1, -1, -1, -1, -1}, 0.0};
      int nparts = ncol;
      if (c.psi == 2) {
        hipLaunchKernelGGL(k_s2_dir<T>, dim3(nb), dim3(kRedThreads), 0, s, x, c.cr, c.cd, (const T*)c.cq, S.list, k,
                           c.P3, (const CgScalars*)c.cg, it);
        CS_LAUNCH_CHECK();
        psi2_happly<T>(c, c.cg, c.P1);
        hipLaunchKernelGGL(k_s2_q<T>, dim3(nb), dim3(kRedThreads), 0, s, (const T*)c.P1, S.list, k, (const T*)c.cd,
                           (const T*)c.cr, c.cq, pdq, (const CgScalars*)c.cg);
        CS_LAUNCH_CHECK();
        nparts = nb;
      } else {
        qd.bytes += launch_col<T>(c, nullptr, c.W, false, dir, &qd.rec[0]);
        if (c.psi) qd.bytes += psi_middle<T>(c, c.cg, &qd.rec[1]);
        else qd.bytes += launch_row<T>(c, ROW_HAPPLY, nullptr, nullptr, nullptr, done, &qd.rec[1]);
        qd.bytes += launch_col<T>(c, c.W, nullptr, true, qio, &qd.rec[6]);
      }
      hipLaunchKernelGGL(k_cg_step<T>, dim3(1), dim3(kRedThreads), 0, s, c.cg, (const double*)pdq, nparts, it,
                         max_iter);
      CS_LAUNCH_CHECK();
      queued.push_back(qd);
      if (c.psi == 2) continue;
      c.transforms += 2;   // (psi_middle counts Phi's two)
    }
  };
  // Iterations still needed after the last read (host.iters), from the
  // observed geometric rate of r^T r over the last read span.
  auto predict = [&]() {
    const double rr_now = host.rr[host.iters & 1];
    const double target = host.tol2 * host.ref;
    const double rr_ref = (rr_prev > 0.0) ? rr_prev : host.rr[0];
    const int span = (rr_prev > 0.0) ? (host.iters - it_prev) : host.iters;
    int next = 2;
    if (span > 0 && rr_ref > 0.0 && rr_now > 0.0 && rr_now < rr_ref && target > 0.0) {
      const double rate = std::log(rr_now / rr_ref) / span;      // log decrease per iteration (< 0)
      const double need = std::log(target / rr_now) / rate;      // iterations still needed
      if (std::isfinite(need)) next = (int)std::ceil(need);
    }
    rr_prev = rr_now;
    it_prev = host.iters;
    return std::max(1, std::min(next, 64));
  };
  // With the mailbox, each chunk's scalars are posted behind it and the next
  // chunk is queued before they are read, so the device does not idle across
  // the read: chunk i + 1 runs while the host reads chunk i.  The run-ahead
  // chunk is sized from the rate seen so far; before the first read only a
  // cold start without a hint runs ahead (warm starts often converge at once).
  const bool ahead = !no_alloc_mode();
  struct Posted { int slot; uint32_t seq; };
  Posted pend[2] = {};
  int npend = 0, slot_next = 1;
  auto post = [&]() {
    pend[npend++] = Posted{slot_next, dev_post(s, c.cg, sizeof(CgScalars), slot_next)};
    slot_next = 3 - slot_next;   // slots 1 and 2 alternate: at most two posts wait
  };
  // When the last warm solve took no step, this one likely starts converged:
  // its start is read before any iteration is queued (one read instead of a
  // chunk of launches that would all exit at once).
  bool settled = false;
  if (warm && c.last_warm_it == 0 && max_iter > 0) {
    dev_read(s, c.cg, &host, sizeof(CgScalars));
    settled = host.done != 0;
  }
  if (max_iter > 0 && !settled) {
    queue_chunk(std::min(first, max_iter));
    if (ahead) post();
  }
  bool known = false;
  int need = 0;   // iterations still needed after host.iters at the last read
  while (max_iter > 0 && !settled) {
    if (ahead) {
      if (npend < 2 && it < max_iter) {
        const int more = known ? need - (it - host.iters) : ((!warm && !hinted) ? 2 : 0);
        if (more > 0) {
          queue_chunk(std::min(more, max_iter - it));
          post();
        }
      }
      dev_wait(s, pend[0].slot, pend[0].seq, &host, sizeof(CgScalars));
      pend[0] = pend[1];
      --npend;
    } else {
      dev_read(s, c.cg, &host, sizeof(CgScalars));
    }
    known = true;
    if (host.done) break;
    need = predict();
    if (npend == 0) {   // nothing queued beyond the read: queue the predicted rest now
      if (it >= max_iter) break;
      queue_chunk(std::min(std::max(1, need - (it - host.iters)), max_iter - it));
      if (ahead) post();
    }
  }
  if (!host.done) dev_read(s, c.cg, &host, sizeof(CgScalars));
  if (host.iters > 0) {
    hipLaunchKernelGGL(k_cg_finish<T>, dim3(upd_blocks(k)), dim3(kRedThreads), 0, s, x, c.cr, (const T*)c.cd,
                       (const T*)c.cq, k, (const CgScalars*)c.cg);
    CS_LAUNCH_CHECK();
  }
  const bool conv = host.rr[host.iters & 1] <= host.tol2 * host.ref;
  if (!conv && !(host.flags & CS_F_CG_BREAKDOWN)) c.flags |= CS_F_CG_MAXITER;
  c.flags |= host.flags;
  c.cg_iters += host.iters;
  for (size_t i = (size_t)std::max(host.iters, 0); i < queued.size(); ++i) {
    c.transforms -= per_it;
    c.model_bytes -= queued[i].bytes;
    for (int r : queued[i].rec) prof_discard(r);
  }
  int h = 0;
  while (h < 3 && !(c.hint[h].k == k && c.hint[h].warm == (int)warm)) ++h;
  for (; h > 0; --h) c.hint[h] = c.hint[h - 1];   // move (or insert) to the front
  c.hint[0].k = k;
  c.hint[0].warm = warm;
  c.hint[0].it = host.iters;
  if (warm) c.last_warm_it = host.iters;
  return host.iters;
}

template <typename T>
static void resid_corr_passes(Ctx<T>& c, const Supp& S, const T* x) {
  if (c.psi == 2) {
    fill<T>(c.P3, c.plan.n, (T)0, c.stream);
    s2_scatter<T>(c, S, x);
    psi2_resid<T>(c, c.Cc);
  } else {
  ColIO<T> in = col_io<T>(c, COL_X, &S);
  in.x = const_cast<T*>(x);
  launch_col<T>(c, nullptr, c.W, false, in);
  if (c.psi) psi_resid_middle<T>(c);
  else launch_row<T>(c, ROW_RESID, c.Yf, nullptr, c.partial2, nullptr);
  launch_col<T>(c, c.W, (Cx<T>*)c.Cc, true, col_io<T>(c, COL_KEY, nullptr));
  c.transforms += 2;
  }
}

template <typename T>
void resid_corr_queue(Ctx<T>& c, const Supp& S, const T* x) {
  resid_corr_passes<T>(c, S, x);
  dev_sum_resid(c.stream, c.partial2, (int)(c.plan.L1 >> 1), &c.cg->resid2);
}

template <typename T>
double resid_corr(Ctx<T>& c, const Supp& S, const T* x) {
  resid_corr_passes<T>(c, S, x);
  // one launch sums ||r||^2 and posts it with the support-comparison flag queued before it
  double r2 = 0.0;
  int32_t differ = 0;
  dev_read_resid(c.stream, c.partial2, (int)(c.plan.L1 >> 1), &c.cg->resid2, &c.cg->differ, &r2, &differ);
  c.last_differ = differ;
  return std::sqrt(r2);
}

template <typename T>
void apply_support(Ctx<T>& c, const Supp& S, const T* x, T* outf) {
  if (c.psi == 2) {
    fill<T>(c.P3, c.plan.n, (T)0, c.stream);
    s2_scatter<T>(c, S, x);
    psi2_forward<T>(c, c.P3, outf);
    return;
  }
  ColIO<T> in = col_io<T>(c, COL_X, &S);
  in.x = const_cast<T*>(x);
  launch_col<T>(c, nullptr, c.W, false, in);
  if (c.psi) {   // F s into freq layout, R, then Phi's forward transform
    launch_row<T>(c, ROW_FWD_ALL, nullptr, c.P1, nullptr, nullptr);
    rand_in<T>(c, c.P1, c.P2, nullptr);
    launch_col<T>(c, (const Cx<T>*)c.P2, c.W, false, col_io<T>(c, COL_DENSE, nullptr));
    c.transforms += 1;
  }
  launch_row<T>(c, ROW_FWD, nullptr, outf, nullptr, nullptr);
  c.transforms += 1;
}

// out[i] = x[slot of to[i] in from] or 0 (both lists ascending)
template <typename T>
__global__ void k_remap(const int32_t* __restrict__ from, const T* __restrict__ x, int kfrom,
                        const int32_t* __restrict__ to, T* __restrict__ out, int kto) {
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= kto) return;
  const int32_t key = to[i];
  int lo = 0, hi = kfrom - 1;
  T v = (T)0;
  while (lo <= hi) {
    const int mid = (lo + hi) >> 1;
    const int32_t m = from[mid];
    if (m == key) { v = x[mid]; break; }
    if (m < key) lo = mid + 1; else hi = mid - 1;
  }
  out[i] = v;
}

template <typename T>
void remap(Ctx<T>& c, const int32_t* from, const T* x, int kfrom, const int32_t* to, T* out, int kto) {
  if (kto <= 0) return;
  hipLaunchKernelGGL(k_remap<T>, dim3((kto + 255) / 256), dim3(256), 0, c.stream, from, x, kfrom, to, out, kto);
  CS_LAUNCH_CHECK();
}

#define CS_INST(T)                                                                    \
  template int cg_solve<T>(Ctx<T>&, const Supp&, T*, bool, double, int, bool, bool); \
  template void apply_support<T>(Ctx<T>&, const Supp&, const T*, T*);               \
  template double resid_corr<T>(Ctx<T>&, const Supp&, const T*);                    \
  template void resid_corr_queue<T>(Ctx<T>&, const Supp&, const T*);                \
  template void remap<T>(Ctx<T>&, const int32_t*, const T*, int, const int32_t*, T*, int);
CS_INST(float)
CS_INST(double)

}  // namespace csr
