// Greedy drivers: OMP (Sec. II steps 1-4, the outer loop of Algorithm 1), SP and
// OMPR (the other two greedy algorithms of Sec. IV), all built from the same
// three steps: correlation A^T r, support selection, CG least squares.
//
// State lives on the device: supports as N-bit bitmaps over keys (the order
// of the column passes), with ascending key lists and per-word prefix counts
// that the column passes use to find a key's compact slot; solutions are
// compact vectors in that order, in sign-flipped coordinates (x'_j = sign_j
// x_j; the correlations kept are F^T D^T r, so x' + eta F^T D^T r = sign (x +
// eta A^T r) and every magnitude the selections compare is unchanged).  Warm
// starts carry the previous solution over to the new support by key (new
// indices start at 0).  Selection breaks ties by natural index.
//
// Decision rules follow the SP/OMPR readings documented with the oracle:
//   SP:   stop with T' when T' == T; stop with (T, x) when ||r'|| > ||r||.
//   OMPR: l = 1, z = x + eta A^T r on I u {j}; stop when j ranks last.
#include "cs_device.h"

#include <algorithm>
#include <cmath>
#include <utility>

namespace csr {

static inline unsigned nblk(int64_t n, int t) { return (unsigned)std::max<int64_t>(1, (n + t - 1) / t); }

// OMPR drop step (one block of 1024 threads): out[0] = dropped natural index.
template <typename T>
__global__ void k_ompr_drop(const T* __restrict__ x, const int32_t* __restrict__ list, int k,
                            const T* __restrict__ cc, const Plan pl, T eta, const int32_t* __restrict__ jptr,
                            int32_t* __restrict__ out, SelState* sel) {
  if (*jptr == -2) {   // the residual gate stopped the step: no drop, no margin
    if (threadIdx.x == 0) out[0] = -2;
    return;
  }
  double m = -1.0, mk = 0.0;
  const int32_t d = ompr_drop_body<T>(x, list, k, cc, pl, eta, *jptr, &m, &mk);
  if (threadIdx.x == 0) {
    out[0] = d;
    note_margin(&sel->mmin, &sel->mrel, m, mk);
  }
}

// key bitmap update for a swap: jd[0] = index to add, jd[1] = index to drop
// (natural); no change when the step stops (no index to add, or it is the one dropped)
__global__ void k_swap_bits(uint32_t* bits, const int32_t* __restrict__ jd, const Plan pl) {
  if (threadIdx.x == 0 && blockIdx.x == 0 && jd[0] >= 0 && jd[1] >= 0 && jd[0] != jd[1]) {
    const uint32_t pj = (uint32_t)key_of_nat(jd[0], pl), pd = (uint32_t)key_of_nat(jd[1], pl);
    bits[pd >> 5] &= ~(1u << (pd & 31));
    bits[pj >> 5] |= 1u << (pj & 31);
  }
}

// add the natural index *jp to a key bitmap
__global__ void k_set_bit_dev(uint32_t* bits, const int32_t* __restrict__ jp, const Plan pl) {
  if (threadIdx.x == 0 && blockIdx.x == 0) {
    const int32_t j = *jp;
    if (j >= 0) {
      const uint32_t p = (uint32_t)key_of_nat(j, pl);
      bits[p >> 5] |= 1u << (p & 31);
    }
  }
}

// dense output s[j] = sign_j x'_i for j = nat_of_key(list[i]), and the
// natural-index bitmap of the support
template <typename T>
__global__ void k_output(T* __restrict__ s, uint32_t* __restrict__ nbits, const int32_t* __restrict__ list,
                         const T* __restrict__ x, int k, const Plan pl, const int8_t* __restrict__ signs) {
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < k) {
    const uint32_t j = (uint32_t)nat_of_key(list[i], pl);
    s[j] = (signs && signs[j] < 0) ? -x[i] : x[i];
    atomicOr(&nbits[j >> 5], 1u << (j & 31));
  }
}

template <typename T>
void write_output(Ctx<T>& c, const int32_t* list, const T* x, int k, T* s_out, int32_t* supp_out) {
  fill<T>(s_out, c.plan.n, (T)0, c.stream);
  fill_u32(c.nbits, c.plan.words, 0u, c.stream);
  hipLaunchKernelGGL(k_output<T>, dim3(nblk(k, 256)), dim3(256), 0, c.stream, s_out, c.nbits, list, x, k, c.plan, c.signs);
  CS_LAUNCH_CHECK();
  bits_to_list<T>(c, c.nbits, supp_out, k, nullptr);   // ascending natural indices
}

static inline int cg_cap(const cs_params& prm, int k) {
  return prm.cg_max_iter > 0 ? prm.cg_max_iter : 2 * k + 50;
}

// ------------------------------------------------------------------ OMP
template <typename T>
void run_omp(Ctx<T>& c, int K, double tol, const cs_params& prm, T* s_out, int32_t* supp_out, cs_info* info) {
  hipStream_t s = c.stream;
  uint32_t* bits = c.bits[0];            // support so far (keys)
  int cur = 0, nxt = 1;                   // list / prefix slots of the old and new support
  T* xc = c.cx;
  T* xn = c.cx3;
  fill_u32(bits, c.plan.words, 0u, s);
  double rn = 0.0;
  for (int i = 1; i <= K; ++i) {
    // selection: the first correlation is A^T r_0 = A^T y, already in C0
    argmax_excl<T>(c, i == 1 ? (const T*)c.C0 : (const T*)c.Cc, bits, c.ibuf);
    hipLaunchKernelGGL(k_set_bit_dev, dim3(1), dim3(64), 0, s, bits, (const int32_t*)c.ibuf, c.plan);  // S = S u {j}
    CS_LAUNCH_CHECK();
    bits_to_list<T>(c, bits, c.list[nxt], i, c.wpre[nxt]);
    const Supp S{bits, c.wpre[nxt], c.list[nxt], i};
    const bool warm = prm.warm_start != 0 && i > 1;
    if (warm) remap<T>(c, c.list[cur], xc, i - 1, c.list[nxt], xn, i);
    // least squares on S; the support only grew, so the warm start's residual is the stored correlation
    cg_solve<T>(c, S, xn, warm, tol, cg_cap(prm, i), false, true);
    // residual update (+ the next iteration's A^T r); OMP runs exactly K
    // iterations, so only the last residual norm is read back
    if (i == K) rn = resid_corr<T>(c, S, xn);
    else resid_corr_queue<T>(c, S, xn);
    std::swap(cur, nxt);
    std::swap(xc, xn);
  }
  write_output<T>(c, c.list[cur], xc, K, s_out, supp_out);
  if (info) { info->outer_iters = K; info->resid_norm = rn; }
}

// ------------------------------------------------------------------ SP
template <typename T>
void run_sp(Ctx<T>& c, int K, double tol, const cs_params& prm, T* s_out, int32_t* supp_out, cs_info* info) {
  hipStream_t s = c.stream;
  const int64_t words = c.plan.words;
  int iT = 0, iU = 1, iN = 2;   // slots: current T, T u D, T'
  T* xT = c.cx;
  T* xU = c.cx2;
  T* xN = c.cx3;
  const bool warm = prm.warm_start != 0;
  const int max_outer = prm.max_outer > 0 ? prm.max_outer : 100;
  auto supp = [&](int i, int k) { return Supp{c.bits[i], c.wpre[i], c.list[i], k}; };

  topk_dense<T>(c, c.C0, nullptr, K, c.bits[iT]);
  bits_to_list<T>(c, c.bits[iT], c.list[iT], K, c.wpre[iT]);
  cg_solve<T>(c, supp(iT, K), xT, false, tol, cg_cap(prm, K));
  double rn = resid_corr<T>(c, supp(iT, K), xT);
  int rounds = 0;
  bool stopped = false;
  for (int l = 1; l <= max_outer; ++l) {
    rounds = l;
    topk_dense<T>(c, (const T*)c.Cc, c.bits[iT], K, c.bits[iN]);   // D: top-K of |A^T r| outside T
    bits_or(c.bits[iT], c.bits[iN], c.bits[iU], words, s);
    bits_to_list<T>(c, c.bits[iU], c.list[iU], 2 * K, c.wpre[iU]);
    if (warm) remap<T>(c, c.list[iT], xT, K, c.list[iU], xU, 2 * K);
    // T u D contains T and Cc holds A^T r for (T, x): no transform for the warm residual
    cg_solve<T>(c, supp(iU, 2 * K), xU, warm, tol, cg_cap(prm, 2 * K), false, true);
    topk_compact<T>(c, xU, c.list[iU], 2 * K, K, c.bits[iN]);     // T': top-K of |x~| over T u D
    // T' = T: the round ends the recovery with (T, x), x already the least
    // squares on T, so neither that solve nor the residual is repeated.  The
    // comparison is read after T''s list (and warm start) are queued behind
    // it; they are left unused when the sets are equal.
    bool same;
    if (no_alloc_mode()) {
      same = bits_equal(c.bits[iN], c.bits[iT], words, c.ibuf + 8, s) != 0;
      if (!same) {
        bits_to_list<T>(c, c.bits[iN], c.list[iN], K, c.wpre[iN]);
        if (warm) remap<T>(c, c.list[iU], xU, 2 * K, c.list[iN], xN, K);
      }
    } else {
      const uint32_t seq = bits_differ_post(c.bits[iN], c.bits[iT], words, c.ibuf + 8, 3, s);
      bits_to_list<T>(c, c.bits[iN], c.list[iN], K, c.wpre[iN]);
      if (warm) remap<T>(c, c.list[iU], xU, 2 * K, c.list[iN], xN, K);
      int32_t differ = 0;
      dev_wait(s, 3, seq, &differ, sizeof(differ));
      same = differ == 0;
    }
    if (same) {
      stopped = true;
      break;
    }
    double rn2;
    if (warm) {
      // the residual at the warm start (x~ on T') first: its correlation is the
      // solve's initial residual, so the solve starts without an H-apply, and
      // when the solve takes no step it is the round's residual as well
      rn2 = resid_corr<T>(c, supp(iN, K), xN);
      if (cg_solve<T>(c, supp(iN, K), xN, true, tol, cg_cap(prm, K), false, true) > 0)
        rn2 = resid_corr<T>(c, supp(iN, K), xN);
    } else {
      cg_solve<T>(c, supp(iN, K), xN, false, tol, cg_cap(prm, K));
      rn2 = resid_corr<T>(c, supp(iN, K), xN);
    }
    if (rn2 > rn) {   // keep the previous (T, x)
      stopped = true;
      break;
    }
    std::swap(iT, iN);
    std::swap(xT, xN);
    rn = rn2;
  }
  if (!stopped) c.flags |= CS_F_OUTER_MAXITER;
  write_output<T>(c, c.list[iT], xT, K, s_out, supp_out);
  if (info) { info->outer_iters = rounds; info->resid_norm = rn; }
}

// OMPR candidates I u J for l > 1: keys (the support keys, then J's) and
// z = x + eta c on I, eta c on J.
template <typename T>
__global__ void k_ompr_cand(const T* __restrict__ x, const int32_t* __restrict__ list, int k,
                            int32_t* __restrict__ keys, int l, const T* __restrict__ cc, T eta, T* __restrict__ z) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < k) {
    const int32_t key = list[i];
    keys[i] = key;
    z[i] = x[i] + eta * cc[key];
  } else if (i < k + l) {
    z[i] = eta * cc[keys[i]];      // J's keys are already in place
  }
}

// One OMPR step with replacement size l > 1 (J = top-l outside I, keep the
// top-K of |z| over I u J): writes the kept set into bits_new and returns
// whether it differs from bits_cur.
template <typename T>
static bool ompr_step_l(Ctx<T>& c, int K, int l, T eta, const int32_t* list_cur, const T* x_cur,
                        const uint32_t* bits_cur, uint32_t* bits_j, uint32_t* bits_new) {
  hipStream_t s = c.stream;
  int32_t* keys = c.list[2];
  T* z = c.cx2;
  topk_dense<T>(c, (const T*)c.Cc, bits_cur, l, bits_j);
  bits_to_list<T>(c, bits_j, keys + K, l, nullptr);
  hipLaunchKernelGGL(k_ompr_cand<T>, dim3(nblk(K + l, 256)), dim3(256), 0, s, x_cur, list_cur, K, keys, l,
                     (const T*)c.Cc, eta, z);
  CS_LAUNCH_CHECK();
  topk_compact<T>(c, z, keys, K + l, K, bits_new);
  return !bits_equal(bits_new, bits_cur, c.plan.words, c.ibuf + 8, s);
}

// ------------------------------------------------------------------ OMPR
template <typename T>
void run_ompr(Ctx<T>& c, int K, double tol, const cs_params& prm, T* s_out, int32_t* supp_out, cs_info* info) {
  hipStream_t s = c.stream;
  uint32_t* bits = c.bits[0];
  int cur = 0, nxt = 1;
  T* xI = c.cx;
  T* xN = c.cx3;
  const bool warm = prm.warm_start != 0;
  const int max_outer = prm.max_outer > 0 ? prm.max_outer : 4 * K;
  const double eta = prm.ompr_eta > 0 ? prm.ompr_eta : (double)c.plan.n / (double)c.plan.m;

  topk_dense<T>(c, c.C0, nullptr, K, bits);
  bits_to_list<T>(c, bits, c.list[cur], K, c.wpre[cur]);
  cg_solve<T>(c, Supp{bits, c.wpre[cur], c.list[cur], K}, xI, false, tol, cg_cap(prm, K));
  double rn = resid_corr<T>(c, Supp{bits, c.wpre[cur], c.list[cur], K}, xI);
  int swaps = 0;
  bool stopped = false;
  int32_t jd[2];
  const int l = prm.ompr_l > 0 ? prm.ompr_l : 1;
  // l = 1: the residual test runs on the device (the argmax is skipped, j = -2,
  // once ||r|| <= 1e-12 ||y||), so the residual is not read back each step;
  // and the step's (j, i) is read after the swap, T''s list and the warm
  // start are queued behind it (they change nothing when the step stops)
  const double thr = 1e-12 * c.ynorm;
  const bool ahead = !no_alloc_mode();
  for (int t = 1; t <= max_outer; ++t) {
    if (l > 1 && rn <= thr) { stopped = true; break; }
    if (l > 1) {
      // general replacement size: the kept set goes to bits[2], then becomes the support
      if (!ompr_step_l<T>(c, K, l, (T)eta, c.list[cur], xI, bits, c.bits[1], c.bits[2])) { stopped = true; break; }
      std::swap(c.bits[0], c.bits[2]);
      bits = c.bits[0];
      bits_to_list<T>(c, bits, c.list[nxt], K, c.wpre[nxt]);
      const Supp S{bits, c.wpre[nxt], c.list[nxt], K};
      if (warm) remap<T>(c, c.list[cur], xI, K, c.list[nxt], xN, K);
      cg_solve<T>(c, S, xN, warm, tol, cg_cap(prm, K));
      rn = resid_corr<T>(c, S, xN);
      std::swap(cur, nxt);
      std::swap(xI, xN);
      ++swaps;
      continue;
    }
    argmax_excl<T>(c, (const T*)c.Cc, bits, c.ibuf, &c.cg->resid2, thr * thr);
    hipLaunchKernelGGL(k_ompr_drop<T>, dim3(1), dim3(1024), 0, s, xI, c.list[cur], K, (const T*)c.Cc, c.plan,
                       (T)eta, (const int32_t*)c.ibuf, c.ibuf + 1, c.sel);
    CS_LAUNCH_CHECK();
    auto queue_swap = [&]() {
      hipLaunchKernelGGL(k_swap_bits, dim3(1), dim3(64), 0, s, bits, (const int32_t*)c.ibuf, c.plan);
      CS_LAUNCH_CHECK();
      bits_to_list<T>(c, bits, c.list[nxt], K, c.wpre[nxt]);
      if (warm) remap<T>(c, c.list[cur], xI, K, c.list[nxt], xN, K);
    };
    if (ahead) {
      const uint32_t seq = dev_post(s, c.ibuf, 2 * sizeof(int32_t), 3);
      queue_swap();
      dev_wait(s, 3, seq, jd, 2 * sizeof(int32_t));
    } else {
      dev_read(s, c.ibuf, jd, 2 * sizeof(int32_t));
    }
    if (jd[0] < 0 || jd[1] == jd[0]) { stopped = true; break; }
    if (!ahead) queue_swap();
    const Supp S{bits, c.wpre[nxt], c.list[nxt], K};
    cg_solve<T>(c, S, xN, warm, tol, cg_cap(prm, K));
    resid_corr_queue<T>(c, S, xN);   // ||r||^2 stays on the device for the next step's gate
    rn = -1.0;
    std::swap(cur, nxt);
    std::swap(xI, xN);
    ++swaps;
  }
  if (rn < 0.0) {   // the last residual of the l = 1 steps is on the device
    double r2 = 0.0;
    dev_read(s, &c.cg->resid2, &r2, sizeof(double));
    rn = std::sqrt(r2);
  }
  if (!stopped) c.flags |= CS_F_OUTER_MAXITER;
  write_output<T>(c, c.list[cur], xI, K, s_out, supp_out);
  if (info) { info->outer_iters = swaps; info->resid_norm = rn; }
}

// ------------------------------------------------------------------ CoSaMP
// Each round: merge the top-2K of |A^T r| with the support, least squares on
// the union (2K..3K columns), prune to the K largest entries (no second
// solve), residual.  Stops with the new (T, x) when the support repeats and
// with the previous one when ||r|| grows (from the second round on).
template <typename T>
void run_cosamp(Ctx<T>& c, int K, double tol, const cs_params& prm, T* s_out, int32_t* supp_out, cs_info* info) {
  hipStream_t s = c.stream;
  const int64_t words = c.plan.words;
  int iT = 0, iU = 1, iN = 2;   // slots: current T, merged U, pruned T'
  T* xT = c.cx;
  T* xU = c.cx2;
  T* xN = c.cx3;
  const bool warm = prm.warm_start != 0;
  const int max_outer = prm.max_outer > 0 ? prm.max_outer : 100;
  double rn = c.ynorm;
  int rounds = 0;
  bool stopped = false;
  for (int it = 1; it <= max_outer; ++it) {
    rounds = it;
    topk_dense<T>(c, it == 1 ? (const T*)c.C0 : (const T*)c.Cc, nullptr, 2 * K, c.bits[iU]);
    if (it > 1) bits_or(c.bits[iU], c.bits[iT], c.bits[iU], words, s);
    const int nb = bits_to_list<T>(c, c.bits[iU], c.list[iU], 3 * K, c.wpre[iU]);
    uint32_t ku = 0;
    dev_read(s, c.blockcnt + nb, &ku, sizeof(uint32_t));
    const int kU = (int)std::min<uint32_t>(ku, (uint32_t)(3 * K));
    const Supp SU{c.bits[iU], c.wpre[iU], c.list[iU], kU};
    const bool w = warm && it > 1;
    if (w) remap<T>(c, c.list[iT], xT, K, c.list[iU], xU, kU);
    cg_solve<T>(c, SU, xU, w, tol, cg_cap(prm, kU), false, true);   // U contains T, Cc is A^T r of (T, x)
    topk_compact<T>(c, xU, c.list[iU], kU, K, c.bits[iN]);
    bits_to_list<T>(c, c.bits[iN], c.list[iN], K, c.wpre[iN]);
    remap<T>(c, c.list[iU], xU, kU, c.list[iN], xN, K);
    if (it > 1) bits_differ(c.bits[iN], c.bits[iT], words, &c.cg->differ, s);
    const Supp SN{c.bits[iN], c.wpre[iN], c.list[iN], K};
    const double rn2 = resid_corr<T>(c, SN, xN);               // also reads the flag back
    const bool same = it > 1 && c.last_differ == 0;
    if (same) {
      std::swap(iT, iN);
      std::swap(xT, xN);
      rn = rn2;
      stopped = true;
      break;
    }
    if (it > 1 && rn2 > rn) {   // keep the previous (T, x)
      stopped = true;
      break;
    }
    std::swap(iT, iN);
    std::swap(xT, xN);
    rn = rn2;
  }
  if (!stopped) c.flags |= CS_F_OUTER_MAXITER;
  write_output<T>(c, c.list[iT], xT, K, s_out, supp_out);
  if (info) { info->outer_iters = rounds; info->resid_norm = rn; }
}

#define CS_INST(T)                                                                                   \
  template void run_omp<T>(Ctx<T>&, int, double, const cs_params&, T*, int32_t*, cs_info*);       \
  template void run_sp<T>(Ctx<T>&, int, double, const cs_params&, T*, int32_t*, cs_info*);        \
  template void run_ompr<T>(Ctx<T>&, int, double, const cs_params&, T*, int32_t*, cs_info*);      \
  template void run_cosamp<T>(Ctx<T>&, int, double, const cs_params&, T*, int32_t*, cs_info*);    \
  template void write_output<T>(Ctx<T>&, const int32_t*, const T*, int, T*, int32_t*);
CS_INST(float)
CS_INST(double)

}  // namespace csr
