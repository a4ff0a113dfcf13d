// C ABI of libcsrecover: argument validation, workspace carving and the
// entry points declared in include/cs.h.
#include "cs_internal.h"

#include <algorithm>
#include <cmath>
#include <cstring>
#include <mutex>
#include <string>

namespace csr {

static thread_local std::string g_last_error;

static size_t align_up(size_t v, size_t a) { return (v + a - 1) / a * a; }

// Carves the workspace (or, with base == nullptr, only measures it).
struct Carver {
  char* base;
  size_t off = 0;
  template <typename P>
  P* take(size_t count) {
    off = align_up(off, 256);
    P* p = base ? reinterpret_cast<P*>(base + off) : nullptr;
    off += count * sizeof(P);
    return p;
  }
};

template <typename T>
static size_t carve(Ctx<T>& c, const Plan& p, int kmax, char* base, int psi = 0, int cplx = 0) {
  Carver cv{base};
  const int64_t n = p.n;
  if (cplx) {   // p.m counts the real rows (twice the complex measurements)
    c.rows_x = cv.take<int32_t>(p.m);
    c.ybuf = cv.take<T>(p.m);
  }
  c.W = cv.take<Cx<T>>(p.L);
  c.Dd = cv.take<T>(n);
  c.Cc = c.Dd;   // the operator entry points and the drivers never need both
  c.C0 = cv.take<T>(n);
  c.Yf = cv.take<T>(n);
  c.tw_col = cv.take<Cx<T>>(kTwStage);
  c.tw_row = cv.take<Cx<T>>(kTwStage);
  c.tw_lo = cv.take<Cx<T>>(kTwLo);
  c.tw_hi = cv.take<Cx<T>>(std::max<int64_t>(1, 4 * n / kTwLo));
  c.tw_step = cv.take<Cx<T>>(2 * kTwStepHalf);
  c.mask = cv.take<uint32_t>(p.words);
  c.pinv = cv.take<int32_t>(n);
  for (int i = 0; i < 3; ++i) c.bits[i] = cv.take<uint32_t>(p.words);
  for (int i = 0; i < 3; ++i) c.wpre[i] = cv.take<uint32_t>(p.words);
  c.nbits = cv.take<uint32_t>(p.words);
  const size_t kk = (size_t)std::max(kmax, 1) + 1;
  for (int i = 0; i < 3; ++i) c.list[i] = cv.take<int32_t>(kk);
  c.cb = cv.take<T>(kk);
  c.cx = cv.take<T>(kk);
  c.cr = cv.take<T>(kk);
  c.cd = cv.take<T>(kk);
  c.cq = cv.take<T>(kk);
  c.cx2 = cv.take<T>(kk);
  c.cx3 = cv.take<T>(kk);
  // partial buffers sized for every compiled shape of this N, so a workspace
  // stays valid whichever shape is in use
  int64_t rows = kRedBlocks, strips = kRedBlocks;
  Shape cand[16];
  const int nc = shape_candidates(sizeof(T) == 8 ? CS_F64 : CS_F32, p.logL, cand, 16);
  for (int i = 0; i < nc; ++i) {
    rows = std::max<int64_t>(rows, int64_t(1) << cand[i].logL1);
    strips = std::max<int64_t>(strips, int64_t(1) << (cand[i].logL2 - cand[i].logB));
  }
  c.partial = cv.take<double>(4 * kRedBlocks);
  c.partial2 = cv.take<double>(rows);
  c.pgrid = cv.take<double>(4 * strips);   // fused CG step: four partials per strip
  c.argpart = cv.take<ArgKey>(2 * kArgBlocks);   // best two per workgroup
  const SplitLayout sl = split_layout(n);
  c.rkey = cv.take<T>((int64_t)sl.blocks * sl.cap);
  c.rpos = cv.take<uint32_t>((int64_t)sl.blocks * sl.cap);
  c.rcnt = cv.take<int32_t>(2 * (int64_t)sl.blocks);
  c.hrows = cv.take<uint32_t>(3 * (int64_t)kSelBins);
  if (psi) {
    c.P1 = cv.take<T>(n);
    c.P2 = cv.take<T>(n);
  }
  if (psi == 2) {
    c.P3 = cv.take<T>(n);
    c.P4 = cv.take<T>(n);
    c.tw_dct = cv.take<Cx<T>>(kTwStage);
  }
  c.ibuf = cv.take<int32_t>(64);
  c.blockcnt = cv.take<uint32_t>((p.words + kBitsPerBlockWords - 1) / kBitsPerBlockWords + 2);
  c.cg = cv.take<CgScalars>(1);
  c.sel = cv.take<SelState>(1);
  return align_up(cv.off, 256);
}

static int kmax_for(cs_algo algo, int32_t k) {
  switch (algo) {
    case CS_ALGO_SP: return 2 * k;
    case CS_ALGO_OMPR: return 2 * k;     // candidates I u J for replacement sizes up to K
    case CS_ALGO_COSAMP: return 3 * k;
    case CS_ALGO_OPERATOR: return 1;
    default: return k;
  }
}

size_t workspace_bytes(cs_dtype dt, int64_t n, int64_t m, int32_t k, cs_algo algo, int psi, int cplx) {
  Plan p;
  if (!choose_plan(dt, n, cplx ? 2 * m : m, p)) return 0;
  if (dt == CS_F32) { Ctx<float> c{}; return carve(c, p, kmax_for(algo, k), nullptr, psi, cplx); }
  Ctx<double> c{};
  return carve(c, p, kmax_for(algo, k), nullptr, psi, cplx);
}

template <typename T>
void ctx_init(Ctx<T>& c, const cs_op* op, int kmax, void* ws, size_t ws_bytes, hipStream_t s, const Shape* force) {
  Plan p;
  const cs_dtype dt = sizeof(T) == 4 ? CS_F32 : CS_F64;
  if (op->xform < 0 || op->xform > 2) throw Error(CS_E_OP, "operator xform must be 0, 1 or 2");
  const int cplx = op->xform == 2 ? 1 : 0;
  if (!choose_plan(dt, op->n, cplx ? 2 * op->m : op->m, p, force)) throw Error(CS_E_SHAPE, "unsupported N or shape");
  if (op->psi < 0 || op->psi > 2) throw Error(CS_E_OP, "operator psi must be 0, 1 or 2");
  if (cplx && op->psi != 0) throw Error(CS_E_OP, "partial complex Fourier sensing takes psi = 0");
  const int psi = op->psi;
  const int dlog = psi == 2 ? dct2d_side_log(dt, op->n) : 0;
  if (dlog < 0) throw Error(CS_E_SHAPE, "the 2-D DCT basis needs N = n^2 with n a power of two in [8, 8192] (FP64: 4096)");
  const size_t need = carve(c, p, kmax, nullptr, psi, cplx);
  if (ws_bytes < need) throw Error(CS_E_WORKSPACE, "workspace too small: need " + std::to_string(need) + " bytes");
  carve(c, p, kmax, (char*)ws, psi, cplx);
  p.tw_lo = c.tw_lo;
  p.tw_hi = c.tw_hi;
  p.tw_step = c.tw_step;
  p.mask = c.mask;
  // the candidates' key order follows the transform they enter: Phi's (through
  // the randomizer) or, with a DCT basis, Psi's (no randomizer)
  p.perm = psi ? nullptr : op->perm;
  p.pinv = (!psi && op->perm) ? c.pinv : nullptr;
  p.keynat = psi == 2 ? 1 : 0;
  p.fourier = op->xform != 0 ? 1 : 0;
  c.plan = p;
  c.stream = s;
  c.psi = psi;
  c.dct_log = dlog;
  c.rsigns = op->signs;
  c.rperm = op->perm;
  c.rpinv = op->perm ? c.pinv : nullptr;
  c.signs = psi ? nullptr : op->signs;
  c.rows = cplx ? c.rows_x : op->rows;
  c.cplx = cplx;
  c.freq = cplx ? op->rows : nullptr;
  c.kmax = kmax;
  prepare_kernels<T>();
}

template void ctx_init<float>(Ctx<float>&, const cs_op*, int, void*, size_t, hipStream_t, const Shape*);
template void ctx_init<double>(Ctx<double>&, const cs_op*, int, void*, size_t, hipStream_t, const Shape*);

// ------------------------------------------------------------------ validation
static void check_shape(cs_dtype dt, const cs_op* op, int32_t k, cs_algo algo) {
  if (dt != CS_F32 && dt != CS_F64) throw Error(CS_E_INVALID, "dtype must be CS_F32 or CS_F64");
  if (!op || !op->rows || !op->signs) throw Error(CS_E_INVALID, "null operator descriptor");
  const int64_t n = op->n;
  if (n < 16 || n > (int64_t(1) << 26) || (n & (n - 1))) throw Error(CS_E_SHAPE, "N must be a power of two in [16, 2^26]");
  if (op->xform < 0 || op->xform > 2) throw Error(CS_E_OP, "operator xform must be 0, 1 or 2");
  // the real rows: partial complex Fourier sensing has two per sampled frequency
  const int64_t m = op->xform == 2 ? 2 * op->m : op->m;
  if (op->xform == 2 && (op->m < 1 || op->m > n / 2 - 1))
    throw Error(CS_E_SHAPE, "partial complex Fourier sensing needs 1 <= M <= N/2 - 1 frequencies");
  if (m < 1 || m > n) throw Error(CS_E_SHAPE, "M must satisfy 1 <= M <= N");
  if (op->psi < 0 || op->psi > 2) throw Error(CS_E_OP, "operator psi must be 0, 1 or 2");
  if (op->xform == 2 && op->psi != 0) throw Error(CS_E_OP, "partial complex Fourier sensing takes psi = 0");
  if (op->psi == 2 && dct2d_side_log(dt, n) < 0)
    throw Error(CS_E_SHAPE, "the 2-D DCT basis needs N = n^2 with n a power of two in [8, 8192] (FP64: 4096)");
  if (algo == CS_ALGO_OPERATOR) return;
  if (k < 1) throw Error(CS_E_INVALID, "K must be >= 1");
  if (k > m) throw Error(CS_E_SHAPE, op->xform == 2 ? "K must not exceed 2M" : "K must not exceed M");
  if (algo == CS_ALGO_SP && (int64_t)2 * k > m) throw Error(CS_E_SHAPE, "SP needs 2K <= M");
  if (algo == CS_ALGO_COSAMP && (int64_t)3 * k > m) throw Error(CS_E_SHAPE, "CoSaMP needs 3K <= M");
}

static void check_tol(double tol) {
  if (!(tol > 0.0) || !std::isfinite(tol)) throw Error(CS_E_INVALID, "tol must be positive and finite");
}

static void check_ws(void* ws) {
  if (!ws) throw Error(CS_E_WORKSPACE, "null workspace");
  if (reinterpret_cast<uintptr_t>(ws) % 256) throw Error(CS_E_WORKSPACE, "workspace must be 256-byte aligned");
}

static cs_params defaults(const cs_params* p) {
  cs_params d{};
  d.cg_max_iter = 0;
  d.max_outer = 0;
  d.warm_start = 1;
  d.ompr_eta = 0.0;
  d.tol_abs = 0;
  d.ompr_l = 1;
  if (p) {
    d.cg_max_iter = p->cg_max_iter;
    d.max_outer = p->max_outer;
    d.warm_start = p->warm_start;
    d.cg_block = p->cg_block;
    d.ompr_eta = p->ompr_eta;
    d.tol_abs = p->tol_abs;
    d.ompr_l = p->ompr_l > 0 ? p->ompr_l : 1;
  }
  return d;
}

template <typename T>
static void fill_info(Ctx<T>& c, cs_info* info) {
  if (!info) return;
  info->flags = c.flags;
  info->cg_iters = c.cg_iters;
  info->transforms = c.transforms;
  info->model_bytes = c.model_bytes;
}

// The call's smallest decision margin into cs_info, and CS_F_NEAR_TIE (an
// absolute CG tolerance enters scaled by 1/||y||).
template <typename T>
static void read_margins(Ctx<T>& c, double tol, cs_info* info) {
  double mm = 0.0, mr = 0.0;
  margins_read<T>(c, &mm, &mr);
  const double trel = c.tol_abs ? tol / std::max(c.ynorm, 1e-300) : tol;
  if (near_tie(mr, trel, sizeof(T) == 4, c.plan.logn)) c.flags |= CS_F_NEAR_TIE;
  info->min_margin = std::isfinite(mm) ? mm : -1.0;
}

template <typename T>
static void recover_t(cs_algo algo, const void* y, const cs_op* op, int32_t k, double tol, void* s, int32_t* support,
                      const cs_params* params, void* ws, size_t ws_bytes, cs_info* info, hipStream_t stream) {
  Ctx<T> c{};
  ctx_init<T>(c, op, kmax_for(algo, k), ws, ws_bytes, stream);
  setup_operator<T>(c);
  sel_reset<T>(c);
  cs_params prm = defaults(params);
  if (c.cplx) {
    // the real equivalent: y^ = sqrt 2 (Re y, -Im y) on the rows (k, N - k);
    // its normal equations are twice the complex ones (an absolute CG
    // tolerance doubles) and its correlations twice A* r (OMPR's step halves)
    cplx_in<T>(c, (const T*)y, std::sqrt(2.0), -std::sqrt(2.0));
    load_measurements<T>(c, c.ybuf);
    if (prm.tol_abs) tol *= 2.0;
    if (prm.ompr_eta > 0.0) prm.ompr_eta *= 0.5;
  } else {
    load_measurements<T>(c, (const T*)y);
  }
  c.tol_abs = prm.tol_abs != 0;
  cs_info loc{};
  cs_info* inf = info ? info : &loc;
  std::memset(inf, 0, sizeof(cs_info));
  if (algo == CS_ALGO_OMP) run_omp<T>(c, k, tol, prm, (T*)s, support, inf);
  else if (algo == CS_ALGO_SP) run_sp<T>(c, k, tol, prm, (T*)s, support, inf);
  else if (algo == CS_ALGO_COSAMP) run_cosamp<T>(c, k, tol, prm, (T*)s, support, inf);
  else run_ompr<T>(c, k, tol, prm, (T*)s, support, inf);
  read_margins<T>(c, tol, inf);
  if (c.cplx) inf->resid_norm *= std::sqrt(0.5);   // ||y^ - A^ s|| = sqrt 2 ||y - A s||
  CS_HIP(hipStreamSynchronize(stream));
  if (prof_on()) prof_flush();
  fill_info<T>(c, inf);
}

// One recovery of a batch (run by a pool worker on its own stream).
static void recover_one(cs_algo algo, cs_dtype dt, const void* y, const cs_op* op, int32_t k, double tol, void* s,
                        int32_t* support, const cs_params* params, void* ws, size_t ws_bytes, cs_info* info,
                        hipStream_t stream) {
  if (dt == CS_F32) recover_t<float>(algo, y, op, k, tol, s, support, params, ws, ws_bytes, info, stream);
  else recover_t<double>(algo, y, op, k, tol, s, support, params, ws, ws_bytes, info, stream);
}

static cs_status recover(cs_algo algo, cs_dtype dt, const void* y, const cs_op* op, int32_t k, double tol, void* s,
                         int32_t* support, const cs_params* params, void* ws, size_t ws_bytes, cs_info* info,
                         hipStream_t stream) {
  try {
    check_shape(dt, op, k, algo);
    if (!y || !s || !support) throw Error(CS_E_INVALID, "null y, s or support");
    check_tol(tol);
    if (algo == CS_ALGO_OMPR && params && (params->ompr_l < 0 || params->ompr_l > k || params->ompr_l > op->n - k))
      throw Error(CS_E_INVALID, "ompr_l must be in [1, min(K, N - K)] (0 means 1)");
    check_ws(ws);
    if (dt == CS_F32) recover_t<float>(algo, y, op, k, tol, s, support, params, ws, ws_bytes, info, stream);
    else recover_t<double>(algo, y, op, k, tol, s, support, params, ws, ws_bytes, info, stream);
    return CS_OK;
  } catch (const Error& e) {
    g_last_error = e.what();
    return e.status;
  } catch (const std::exception& e) {
    g_last_error = e.what();
    return CS_E_HIP;
  }
}

// ------------------------------------------------------------------ cs_ls_solve helpers
__global__ void k_check_support(const int32_t* __restrict__ sup, int k, int64_t n, int32_t* bad) {
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= k) return;
  const int32_t j = sup[i];
  if (j < 0 || j >= n || (i > 0 && sup[i - 1] >= j)) atomicOr(bad, 1);
}

// key bitmap of a natural-index support
__global__ void k_support_bits(const int32_t* __restrict__ sup, int k, const Plan pl, uint32_t* __restrict__ bits) {
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= k) return;
  const uint32_t p = (uint32_t)key_of_nat(sup[i], pl);
  atomicOr(&bits[p >> 5], 1u << (p & 31));
}

__device__ __forceinline__ uint32_t rank_of(const uint32_t* __restrict__ bits, const uint32_t* __restrict__ wpre,
                                            uint32_t p) {
  return wpre[p >> 5] + __popc(bits[p >> 5] & ((1u << (p & 31)) - 1u));
}

// Between support order with natural coordinates and key order with
// sign-flipped coordinates.  TO_KEY: xkey[rank(key(sup[i]))] = sign xnat[i];
// otherwise xnat[i] = sign xkey[rank(key(sup[i]))].
template <typename T, bool TO_KEY>
__global__ void k_reorder(const int32_t* __restrict__ sup, int k, const Plan pl, const int8_t* __restrict__ signs,
                          const uint32_t* __restrict__ bits, const uint32_t* __restrict__ wpre, T* xnat, T* xkey) {
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= k) return;
  const int32_t j = sup[i];
  const uint32_t slot = rank_of(bits, wpre, (uint32_t)key_of_nat(j, pl));
  const bool neg = signs && signs[j] < 0;
  if (TO_KEY) xkey[slot] = neg ? -xnat[i] : xnat[i];
  else xnat[i] = neg ? -xkey[slot] : xkey[slot];
}

// Validates a natural-index support and builds its key bitmap, list and
// prefix counts in slot 0 (the CG works in key order).
template <typename T>
static Supp support_keys(Ctx<T>& c, const int32_t* support, int32_t k) {
  hipStream_t stream = c.stream;
  fill<int32_t>(c.ibuf + 16, 1, 0, stream);
  const unsigned gk = (unsigned)((k + 255) / 256);
  hipLaunchKernelGGL(k_check_support, dim3(gk), dim3(256), 0, stream, support, k, c.plan.n, c.ibuf + 16);
  CS_LAUNCH_CHECK();
  int32_t bad = 0;
  dev_read(stream, c.ibuf + 16, &bad, sizeof(int32_t));
  if (bad) throw Error(CS_E_INVALID, "support must be strictly ascending in [0, N)");
  fill_u32(c.bits[0], c.plan.words, 0u, stream);
  hipLaunchKernelGGL(k_support_bits, dim3(gk), dim3(256), 0, stream, support, k, c.plan, c.bits[0]);
  CS_LAUNCH_CHECK();
  bits_to_list<T>(c, c.bits[0], c.list[0], k, c.wpre[0]);
  return Supp{c.bits[0], c.wpre[0], c.list[0], k};
}

template <typename T>
static void ls_t(const void* y, const cs_op* op, const int32_t* support, int32_t k, double tol, const void* x0,
                 void* theta, const cs_params* params, void* ws, size_t ws_bytes, cs_info* info, hipStream_t stream) {
  Ctx<T> c{};
  ctx_init<T>(c, op, k, ws, ws_bytes, stream);
  setup_operator<T>(c);
  const unsigned gk = (unsigned)((k + 255) / 256);
  const Supp S = support_keys<T>(c, support, k);
  const cs_params prm = defaults(params);
  if (c.cplx) {   // the real equivalent (see recover_t)
    cplx_in<T>(c, (const T*)y, std::sqrt(2.0), -std::sqrt(2.0));
    load_measurements<T>(c, c.ybuf);
    if (prm.tol_abs) tol *= 2.0;
  } else {
    load_measurements<T>(c, (const T*)y);
  }
  c.tol_abs = prm.tol_abs != 0;
  if (x0)
    hipLaunchKernelGGL((k_reorder<T, true>), dim3(gk), dim3(256), 0, stream, support, k, c.plan, c.signs, c.bits[0],
                       c.wpre[0], (T*)x0, c.cx);
  CS_LAUNCH_CHECK();
  const int cap = prm.cg_max_iter > 0 ? prm.cg_max_iter : 2 * k + 50;
  cg_solve<T>(c, S, c.cx, x0 != nullptr, tol, cap);
  hipLaunchKernelGGL((k_reorder<T, false>), dim3(gk), dim3(256), 0, stream, support, k, c.plan, c.signs, c.bits[0],
                     c.wpre[0], (T*)theta, c.cx);
  CS_LAUNCH_CHECK();
  double rn = 0.0;
  if (info) rn = resid_corr<T>(c, S, c.cx);
  CS_HIP(hipStreamSynchronize(stream));
  if (prof_on()) prof_flush();
  if (info) {
    std::memset(info, 0, sizeof(cs_info));
    info->resid_norm = c.cplx ? rn * std::sqrt(0.5) : rn;
    info->min_margin = -1.0;   // no selection
    fill_info<T>(c, info);
  }
}

// b'[rank(key(sup[i]))] = sign_j g[j], j = sup[i]: the support entries of a
// dense gradient, in key order and sign-flipped coordinates
template <typename T>
__global__ void k_grad_rhs(const int32_t* __restrict__ sup, int k, const Plan pl, const int8_t* __restrict__ signs,
                           const uint32_t* __restrict__ bits, const uint32_t* __restrict__ wpre,
                           const T* __restrict__ g, T* __restrict__ b) {
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= k) return;
  const int32_t j = sup[i];
  const uint32_t slot = rank_of(bits, wpre, (uint32_t)key_of_nat(j, pl));
  b[slot] = (signs && signs[j] < 0) ? -g[j] : g[j];
}

// dL/dy = A_S z with (A_S^T A_S) z = (dL/ds)_S: the CG on the sign-flipped
// system with b' = R g, then the forward operator on the support.
template <typename T>
static void adj_t(const cs_op* op, const int32_t* support, int32_t k, const void* grad, double tol, void* grad_y,
                  const cs_params* params, void* ws, size_t ws_bytes, cs_info* info, hipStream_t stream) {
  Ctx<T> c{};
  ctx_init<T>(c, op, k, ws, ws_bytes, stream);
  setup_operator<T>(c);
  const unsigned gk = (unsigned)((k + 255) / 256);
  const Supp S = support_keys<T>(c, support, k);
  const cs_params prm = defaults(params);
  c.tol_abs = prm.tol_abs != 0;
  if (c.cplx && prm.tol_abs) tol *= 2.0;   // the real equivalent's normal equations (see recover_t)
  hipLaunchKernelGGL(k_grad_rhs<T>, dim3(gk), dim3(256), 0, stream, support, k, c.plan, c.signs, c.bits[0], c.wpre[0],
                     (const T*)grad, c.cb);
  CS_LAUNCH_CHECK();
  const int cap = prm.cg_max_iter > 0 ? prm.cg_max_iter : 2 * k + 50;
  cg_solve<T>(c, S, c.cx, false, tol, cap, true);
  apply_support<T>(c, S, c.cx, c.Yf);
  if (c.cplx) {
    // dL/dy^ on the rows (k, N - k), then dL/dRe y = sqrt 2 dL/dy^_k and
    // dL/dIm y = -sqrt 2 dL/dy^_{N-k} (y^ = sqrt 2 (Re y, -Im y))
    gather_freq<T>(c, c.Yf, c.ybuf);
    cplx_out<T>(c, (T*)grad_y, std::sqrt(2.0), -std::sqrt(2.0));
  } else {
    gather_freq<T>(c, c.Yf, (T*)grad_y);
  }
  CS_HIP(hipStreamSynchronize(stream));
  if (prof_on()) prof_flush();
  if (info) {
    std::memset(info, 0, sizeof(cs_info));
    info->min_margin = -1.0;   // no selection
    fill_info<T>(c, info);
  }
}

// Average time of one H-apply (forward column pass, row pass, inverse column
// pass on a dense N-vector) with the given shape.
template <typename T>
static double time_shape_t(const cs_op* op, const Shape& sh, int reps, void* ws, size_t ws_bytes,
                           hipStream_t stream) {
  Ctx<T> c{};
  ctx_init<T>(c, op, 1, ws, ws_bytes, stream, &sh);
  setup_operator<T>(c);
  fill<T>(c.Dd, c.plan.n, (T)0, stream);
  auto happly = [&]() {
    launch_col<T>(c, (const Cx<T>*)c.Dd, c.W, false, col_io<T>(c, COL_DENSE, nullptr));
    launch_row<T>(c, ROW_HAPPLY, nullptr, nullptr, nullptr, nullptr);
    launch_col<T>(c, c.W, c.W, true, col_io<T>(c, COL_DENSE, nullptr));
  };
  happly();
  happly();
  hipEvent_t a = nullptr, b = nullptr;
  CS_HIP(hipEventCreate(&a));
  CS_HIP(hipEventCreate(&b));
  CS_HIP(hipEventRecord(a, stream));
  for (int i = 0; i < reps; ++i) happly();
  CS_HIP(hipEventRecord(b, stream));
  CS_HIP(hipEventSynchronize(b));
  float ms = 0.f;
  CS_HIP(hipEventElapsedTime(&ms, a, b));
  CS_HIP(hipEventDestroy(a));
  CS_HIP(hipEventDestroy(b));
  if (prof_on()) prof_flush();
  return (double)ms / reps;
}

template <typename T>
static void apply_t(bool adjoint, const cs_op* op, const void* in, void* out, void* ws, size_t ws_bytes,
                    hipStream_t stream) {
  Ctx<T> c{};
  ctx_init<T>(c, op, 1, ws, ws_bytes, stream);
  setup_operator<T>(c);
  // With a DCT basis (psi) perm_in/perm_out place s with no randomizer, and
  // R is applied between Psi's and Phi's transforms.
  if (c.psi == 2) {   // natural order on the s side: no placement pass
    if (!adjoint) {
      psi2_forward<T>(c, (const T*)in, c.Yf);
      gather_freq<T>(c, c.Yf, (T*)out);
    } else {
      scatter_freq<T>(c, (const T*)in, c.Yf);
      psi2_adjoint<T>(c, c.Yf, (T*)out);
    }
  } else if (!adjoint) {
    perm_in<T>(c, (const T*)in, c.Dd);
    transform_fwd<T>(c, c.Dd, c.Yf, c.psi != 0);   // Psi = F: every output, unmasked
    if (c.psi) {
      rand_in<T>(c, c.Yf, c.P2, nullptr);
      transform_fwd<T>(c, c.P2, c.Yf);
    }
    if (c.cplx) {   // y_k = (row k - i row N-k) / sqrt 2
      gather_freq<T>(c, c.Yf, c.ybuf);
      cplx_out<T>(c, (T*)out, std::sqrt(0.5), -std::sqrt(0.5));
    } else {
      gather_freq<T>(c, c.Yf, (T*)out);
    }
  } else {
    if (c.cplx) {   // A* u = A^T (Re u, -Im u) / sqrt 2 on the rows (k, N - k)
      cplx_in<T>(c, (const T*)in, std::sqrt(0.5), -std::sqrt(0.5));
      scatter_freq<T>(c, c.ybuf, c.Yf);
    } else {
      scatter_freq<T>(c, (const T*)in, c.Yf);
    }
    if (c.psi) {
      transform_adj<T>(c, c.Yf, c.P2, false);
      rand_out<T>(c, c.P2, c.P1, nullptr);
      transform_adj<T>(c, c.P1, (T*)c.W, false);
    } else {
      transform_adj<T>(c, c.Yf, (T*)c.W, false);
    }
    perm_out<T>(c, (const T*)c.W, (T*)out);
  }
  CS_HIP(hipStreamSynchronize(stream));
  if (prof_on()) prof_flush();
}

// ------------------------------------------------------------------ static workspace
// The workspace of cs_recover_sp_static: a file-scope device array, one copy
// per GPU, held from the load of the code object on that GPU until the
// process ends.  In host code the array's name is a host-side stand-in, not a
// device address; its device address is looked up once per device (with
// that device current) and only that address is handed to kernels.
static __device__ __align__(256) unsigned char scratch[CS_STATIC_WS_BYTES];

constexpr int kMaxDevices = 64;
static std::mutex g_scratch_mu;
static void* g_scratch_ptr[kMaxDevices];

static void* scratch_ptr() {
  int dev = 0;
  CS_HIP(hipGetDevice(&dev));
  if (dev < 0 || dev >= kMaxDevices) throw Error(CS_E_HIP, "device ordinal out of range for the static workspace");
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void* ptr = nullptr;
    CS_HIP(hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)));
    if (!ptr || reinterpret_cast<uintptr_t>(ptr) % 256) throw Error(CS_E_HIP, "static workspace address unusable");
    g_scratch_ptr[dev] = ptr;
  }
  return g_scratch_ptr[dev];
}

}  // namespace csr

using namespace csr;

extern "C" {

size_t cs_workspace_size(cs_dtype dtype, int64_t n, int64_t m, int32_t k, cs_algo algo) {
  if (dtype != CS_F32 && dtype != CS_F64) return 0;
  if (n < 16 || n > (int64_t(1) << 26) || (n & (n - 1)) || m < 1 || m > n) return 0;
  if (algo != CS_ALGO_OPERATOR && (k < 1 || k > m)) return 0;
  if (algo < CS_ALGO_OMP || algo > CS_ALGO_COSAMP) return 0;
  if (algo == CS_ALGO_COSAMP && (int64_t)3 * k > m) return 0;
  return workspace_bytes(dtype, n, m, k, algo, 0);
}

size_t cs_workspace_size_op(cs_dtype dtype, const cs_op* op, int32_t k, cs_algo algo) {
  if (!op || op->psi < 0 || op->psi > 2 || op->xform < 0 || op->xform > 2) return 0;
  if (op->psi == 2 && dct2d_side_log(dtype, op->n) < 0) return 0;
  const int cplx = op->xform == 2 ? 1 : 0;
  if (cplx && (op->psi != 0 || op->m < 1 || op->m > op->n / 2 - 1)) return 0;
  // sizes of the real rows: two per sampled frequency with complex sensing
  if (cs_workspace_size(dtype, op->n, cplx ? 2 * op->m : op->m, k, algo) == 0) return 0;
  return workspace_bytes(dtype, op->n, op->m, k, algo, op->psi, cplx);
}

cs_status cs_recover_omp(cs_dtype dtype, const void* y, const cs_op* op, int32_t k, double tol, void* s,
                         int32_t* support, const cs_params* params, void* ws, size_t ws_bytes, cs_info* info,
                         hipStream_t stream) {
  return recover(CS_ALGO_OMP, dtype, y, op, k, tol, s, support, params, ws, ws_bytes, info, stream);
}

cs_status cs_recover_sp(cs_dtype dtype, const void* y, const cs_op* op, int32_t k, double tol, void* s,
                        int32_t* support, const cs_params* params, void* ws, size_t ws_bytes, cs_info* info,
                        hipStream_t stream) {
  return recover(CS_ALGO_SP, dtype, y, op, k, tol, s, support, params, ws, ws_bytes, info, stream);
}

cs_status cs_recover_sp_static(cs_dtype dtype, const void* y, const cs_op* op, int32_t k, double tol, void* s,
                               int32_t* support, const cs_params* params, cs_info* info, hipStream_t stream) {
  try {
    check_shape(dtype, op, k, CS_ALGO_SP);
    if (!y || !s || !support) throw Error(CS_E_INVALID, "null y, s or support");
    check_tol(tol);
    const size_t need = workspace_bytes(dtype, op->n, op->m, k, CS_ALGO_SP, op->psi, op->xform == 2 ? 1 : 0);
    if (need == 0) throw Error(CS_E_SHAPE, "unsupported N or shape");
    if (need > (size_t)CS_STATIC_WS_BYTES)
      throw Error(CS_E_WORKSPACE, "these sizes need " + std::to_string(need) +
                                      " bytes of workspace; the static workspace holds " +
                                      std::to_string((size_t)CS_STATIC_WS_BYTES));
    void* ws = scratch_ptr();
    NoAllocScope scope;
    if (dtype == CS_F32)
      recover_t<float>(CS_ALGO_SP, y, op, k, tol, s, support, params, ws, CS_STATIC_WS_BYTES, info, stream);
    else
      recover_t<double>(CS_ALGO_SP, y, op, k, tol, s, support, params, ws, CS_STATIC_WS_BYTES, info, stream);
    return CS_OK;
  } catch (const Error& e) {
    g_last_error = e.what();
    return e.status;
  } catch (const std::exception& e) {
    g_last_error = e.what();
    return CS_E_HIP;
  }
}

cs_status cs_recover_ompr(cs_dtype dtype, const void* y, const cs_op* op, int32_t k, double tol, void* s,
                          int32_t* support, const cs_params* params, void* ws, size_t ws_bytes, cs_info* info,
                          hipStream_t stream) {
  return recover(CS_ALGO_OMPR, dtype, y, op, k, tol, s, support, params, ws, ws_bytes, info, stream);
}

cs_status cs_recover_cosamp(cs_dtype dtype, const void* y, const cs_op* op, int32_t k, double tol, void* s,
                            int32_t* support, const cs_params* params, void* ws, size_t ws_bytes, cs_info* info,
                            hipStream_t stream) {
  return recover(CS_ALGO_COSAMP, dtype, y, op, k, tol, s, support, params, ws, ws_bytes, info, stream);
}

cs_status cs_ls_solve(cs_dtype dtype, const void* y, const cs_op* op, const int32_t* support, int32_t k, double tol,
                      const void* x0, void* theta, const cs_params* params, void* ws, size_t ws_bytes,
                      cs_info* info, hipStream_t stream) {
  try {
    check_shape(dtype, op, k, CS_ALGO_LS);
    if (!y || !support || !theta) throw Error(CS_E_INVALID, "null y, support or theta");
    check_tol(tol);
    check_ws(ws);
    if (dtype == CS_F32) ls_t<float>(y, op, support, k, tol, x0, theta, params, ws, ws_bytes, info, stream);
    else ls_t<double>(y, op, support, k, tol, x0, theta, params, ws, ws_bytes, info, stream);
    return CS_OK;
  } catch (const Error& e) {
    g_last_error = e.what();
    return e.status;
  } catch (const std::exception& e) {
    g_last_error = e.what();
    return CS_E_HIP;
  }
}

cs_status cs_adjoint_ls(cs_dtype dtype, const cs_op* op, const int32_t* support, int32_t k, const void* grad_s,
                        double tol, void* grad_y, const cs_params* params, void* ws, size_t ws_bytes, cs_info* info,
                        hipStream_t stream) {
  try {
    check_shape(dtype, op, k, CS_ALGO_LS);
    if (!support || !grad_s || !grad_y) throw Error(CS_E_INVALID, "null support, grad_s or grad_y");
    check_tol(tol);
    check_ws(ws);
    if (dtype == CS_F32) adj_t<float>(op, support, k, grad_s, tol, grad_y, params, ws, ws_bytes, info, stream);
    else adj_t<double>(op, support, k, grad_s, tol, grad_y, params, ws, ws_bytes, info, stream);
    return CS_OK;
  } catch (const Error& e) {
    g_last_error = e.what();
    return e.status;
  } catch (const std::exception& e) {
    g_last_error = e.what();
    return CS_E_HIP;
  }
}

size_t cs_workspace_size_batched(cs_dtype dtype, int32_t count, const cs_batch_item* items, cs_algo algo) {
  if (dtype != CS_F32 && dtype != CS_F64) return 0;
  if (count < 1 || !items || (algo != CS_ALGO_OMPR && algo != CS_ALGO_SP)) return 0;
  for (int i = 0; i < count; ++i) {
    const cs_op& o = items[i].op;
    if (algo == CS_ALGO_OMPR && o.psi != 0) return 0;
    if (o.xform == 2) return 0;   // complex measurements: single-signal calls only
    if (algo == CS_ALGO_SP && (int64_t)2 * items[i].k > o.m) return 0;
    if (cs_workspace_size_op(dtype, &o, items[i].k, algo) == 0) return 0;
  }
  return algo == CS_ALGO_OMPR ? batch_layout(dtype, count, items, nullptr)
                              : batch_layout_algo(dtype, count, items, algo, nullptr);
}

cs_status cs_recover_sp_batched(cs_dtype dtype, int32_t count, const cs_batch_item* items, double tol,
                                const cs_params* params, void* ws, size_t ws_bytes, cs_info* info,
                                hipStream_t stream) {
  try {
    if (count < 1 || !items) throw Error(CS_E_INVALID, "count must be >= 1 with a non-null item array");
    for (int i = 0; i < count; ++i) {
      check_shape(dtype, &items[i].op, items[i].k, CS_ALGO_SP);
      if (items[i].op.xform == 2) throw Error(CS_E_OP, "the batched calls take real measurements (xform 0 or 1)");
      if (!items[i].y || !items[i].s || !items[i].support) throw Error(CS_E_INVALID, "null y, s or support in batch");
    }
    check_tol(tol);
    check_ws(ws);
    recover_batched_pool(CS_ALGO_SP, dtype, count, items, tol, params, ws, ws_bytes, info, stream, recover_one);
    return CS_OK;
  } catch (const Error& e) {
    g_last_error = e.what();
    return e.status;
  } catch (const std::exception& e) {
    g_last_error = e.what();
    return CS_E_HIP;
  }
}

cs_status cs_recover_ompr_batched(cs_dtype dtype, int32_t count, const cs_batch_item* items, double tol,
                                  const cs_params* params, void* ws, size_t ws_bytes, cs_info* info,
                                  hipStream_t stream) {
  try {
    if (count < 1 || !items) throw Error(CS_E_INVALID, "count must be >= 1 with a non-null item array");
    if (params && params->ompr_l > 1) throw Error(CS_E_INVALID, "the batched call runs OMPR with l = 1");
    for (int i = 0; i < count; ++i) {
      check_shape(dtype, &items[i].op, items[i].k, CS_ALGO_OMPR);
      if (items[i].op.psi != 0) throw Error(CS_E_INVALID, "the batched call takes operators with psi = 0");
      if (items[i].op.xform == 2) throw Error(CS_E_OP, "the batched calls take real measurements (xform 0 or 1)");
      if (!items[i].y || !items[i].s || !items[i].support) throw Error(CS_E_INVALID, "null y, s or support in batch");
      if (items[i].moves_cap < 0 || (items[i].moves_cap > 0 && !items[i].moves))
        throw Error(CS_E_INVALID, "moves_cap must be >= 0, with a non-null moves array when positive");
    }
    check_tol(tol);
    check_ws(ws);
    const cs_params prm = defaults(params);
    const int cgb = (params && params->cg_block > 0) ? params->cg_block : 256;
    if (cgb < 64 || cgb > 1024 || (cgb & 63)) throw Error(CS_E_INVALID, "cg_block must be a multiple of 64 in [64, 1024]");
    if (dtype == CS_F32) run_ompr_batched<float>(count, items, tol, prm, cgb, ws, ws_bytes, info, stream);
    else run_ompr_batched<double>(count, items, tol, prm, cgb, ws, ws_bytes, info, stream);
    if (prof_on()) prof_flush();
    return CS_OK;
  } catch (const Error& e) {
    g_last_error = e.what();
    return e.status;
  } catch (const std::exception& e) {
    g_last_error = e.what();
    return CS_E_HIP;
  }
}

static cs_status apply_entry(bool adjoint, cs_dtype dtype, const cs_op* op, const void* in, void* out, void* ws,
                             size_t ws_bytes, hipStream_t stream) {
  try {
    check_shape(dtype, op, 1, CS_ALGO_OPERATOR);
    if (!in || !out) throw Error(CS_E_INVALID, "null input or output");
    check_ws(ws);
    if (dtype == CS_F32) apply_t<float>(adjoint, op, in, out, ws, ws_bytes, stream);
    else apply_t<double>(adjoint, op, in, out, ws, ws_bytes, stream);
    return CS_OK;
  } catch (const Error& e) {
    g_last_error = e.what();
    return e.status;
  } catch (const std::exception& e) {
    g_last_error = e.what();
    return CS_E_HIP;
  }
}

cs_status cs_apply_A(cs_dtype dtype, const cs_op* op, const void* x, void* out, void* ws, size_t ws_bytes,
                     hipStream_t stream) {
  return apply_entry(false, dtype, op, x, out, ws, ws_bytes, stream);
}

cs_status cs_apply_At(cs_dtype dtype, const cs_op* op, const void* u, void* out, void* ws, size_t ws_bytes,
                      hipStream_t stream) {
  return apply_entry(true, dtype, op, u, out, ws, ws_bytes, stream);
}

static int log2_exact(int64_t n) {
  int l = 0;
  while ((int64_t(1) << l) < n) ++l;
  return l;
}

int cs_shape_candidates(cs_dtype dtype, int64_t n, cs_shape* out, int32_t max) {
  if ((dtype != CS_F32 && dtype != CS_F64) || n < 16 || n > (int64_t(1) << 26) || (n & (n - 1))) return 0;
  Shape tmp[16];
  const int cnt = shape_candidates(dtype, log2_exact(n) - 1, tmp, 16);
  if (!out) return cnt;
  const int w = std::min<int>(cnt, std::max<int32_t>(max, 0));
  for (int i = 0; i < w; ++i) out[i] = cs_shape{tmp[i].logL1, tmp[i].logL2, tmp[i].logB, tmp[i].logE};
  return w;
}

cs_status cs_set_shape(cs_dtype dtype, int64_t n, const cs_shape* shape) {
  if ((dtype != CS_F32 && dtype != CS_F64) || n < 16 || n > (int64_t(1) << 26) || (n & (n - 1))) {
    g_last_error = "N must be a power of two in [16, 2^26] and dtype CS_F32 or CS_F64";
    return CS_E_SHAPE;
  }
  Shape sh{0, 0, 0, 0};
  if (shape) sh = Shape{shape->log_l1, shape->log_l2, shape->log_b, shape->log_e};
  if (!set_shape_override(dtype, log2_exact(n) - 1, shape ? &sh : nullptr)) {
    g_last_error = "shape is not one of cs_shape_candidates() for this N";
    return CS_E_SHAPE;
  }
  return CS_OK;
}

cs_status cs_time_shape(cs_dtype dtype, const cs_op* op, const cs_shape* shape, int32_t reps, void* ws,
                        size_t ws_bytes, hipStream_t stream, double* ms_per_apply) {
  try {
    check_shape(dtype, op, 1, CS_ALGO_OPERATOR);
    if (!shape || !ms_per_apply || reps < 1) throw Error(CS_E_INVALID, "null shape or result, or reps < 1");
    check_ws(ws);
    const Shape sh{shape->log_l1, shape->log_l2, shape->log_b, shape->log_e};
    *ms_per_apply = (dtype == CS_F32) ? time_shape_t<float>(op, sh, reps, ws, ws_bytes, stream)
                                      : time_shape_t<double>(op, sh, reps, ws, ws_bytes, stream);
    return CS_OK;
  } catch (const Error& e) {
    g_last_error = e.what();
    return e.status;
  } catch (const std::exception& e) {
    g_last_error = e.what();
    return CS_E_HIP;
  }
}

const char* cs_status_str(cs_status status) {
  switch (status) {
    case CS_OK: return "ok";
    case CS_E_INVALID: return "invalid argument";
    case CS_E_SHAPE: return "unsupported shape";
    case CS_E_OP: return "invalid operator descriptor";
    case CS_E_WORKSPACE: return "workspace too small or misaligned";
    case CS_E_HIP: return "HIP runtime error";
  }
  return "unknown status";
}

const char* cs_last_error(void) { return g_last_error.c_str(); }

}  // extern "C"
