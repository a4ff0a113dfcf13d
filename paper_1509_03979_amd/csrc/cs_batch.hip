// Batched OMPR: many signals of uneven N, M and K recovered together.
//
// Every signal keeps its own device state (BState: phase, current support
// slot, CG iteration, swap count, counters) next to the workspace of a
// single-signal call.  One batched step moves every unfinished signal one
// stage along the OMPR loop of the single-signal driver:
//   WARM    r = b - H x (warm start), r^T r, CG set-up
//   ITER    one CG iteration (Algorithm 1 lines 16-23)
//   RESID   r = y - A x, ||r|| and the correlation F^T D^T r
//   SELECT  argmax outside the support, the drop step, the swap and the new
//           support's list, prefix counts, remapped x and right-hand side
// with the same decision rules, so each signal follows the path the
// single-signal OMPR takes.  A step is a fixed sequence of launches: the three
// transform passes once per size class (the signal in blockIdx.y, its shape a
// template parameter), then one CG kernel and the selection kernels over all
// signals, each returning at once for signals in another phase.  The host
// captures several steps in a HIP graph and replays it until a device counter
// of unfinished signals reads zero.
#include "cs_device.h"
#include "cs_kernels.h"

#include <algorithm>
#include <cmath>
#include <cstring>
#include <map>
#include <vector>

namespace csr {

constexpr int kBArgBlocks = 64;   // argmax blocks per signal
constexpr int kBSteps = 8;        // batched steps per graph replay

// x = 0 and b = C0 on the initial support; b^T b
template <typename T>
__global__ void k_b_start(const BSig<T>* __restrict__ sigs) {
  const BSig<T>& s = sigs[blockIdx.x];
  BState* st = s.st;
  const int k = st->k, cur = st->cur;
  const int32_t* list = s.list[cur];
  T* x = s.cx[cur];
  double acc = 0.0;
  for (int i = threadIdx.x; i < k; i += blockDim.x) {
    const T v = s.C0[list[i]];
    s.cb[i] = v;
    x[i] = (T)0;
    acc += (double)v * (double)v;
  }
  acc = block_sum_any(acc);
  if (threadIdx.x == 0) {
    st->bb = acc;
    st->phase = BP_WARM;
  }
}

// Per-signal scalar work after the transform passes of a step (one block per
// signal): the CG start (WARM), the CG update (ITER), the residual norm (RESID).
template <typename T>
__global__ void k_b_post(const BSig<T>* __restrict__ sigs) {
  const BSig<T>& s = sigs[blockIdx.x];
  BState* st = s.st;
  const int phase = st->phase;
  if (phase > BP_RESID) return;
  const Plan& p = s.plan;
  CgScalars* cg = s.cg;
  const int k = st->k;
  const int tid = threadIdx.x;
  const double nb = (double)p.n * sizeof(T), kb = (double)k, esz = (double)sizeof(T);
  if (phase == BP_WARM) {
    const int ncol = (int)(p.L2 >> p.logB);
    double rr = 0.0;
    for (int i = tid; i < ncol; i += blockDim.x) rr += s.pgrid[i];
    rr = block_sum_any(rr);
    if (tid == 0) {
      const double bb = st->bb;
      cg->rr[0] = rr;
      cg->rr[1] = rr;
      cg->bb = bb;
      cg->tol2 = st->tol2;
      cg->iters = 0;
      cg->flags = 0;
      cg->cnt_q = 0u;
      cg->cnt_u = 0u;
      const bool fin = isfinite(rr) && isfinite(bb);
      const bool conv = rr <= st->tol2 * bb;
      const bool done = !fin || conv || st->cg_cap <= 0;
      if (!fin) st->flags |= CS_F_NONFINITE;
      else if (done && !conv) st->flags |= CS_F_CG_MAXITER;
      cg->done = done ? 1 : 0;
      st->it = 0;
      st->phase = done ? BP_RESID : BP_ITER;
      st->transforms += 2;
      st->model_bytes += 4.0 * nb + kb * (4.0 + esz) + kb * (4.0 + 3.0 * esz);
    }
  } else if (phase == BP_ITER) {
    const int it = st->it;
    const double dq = cg->dq;
    const double rr = cg->rr[it & 1];
    if (tid == 0) {
      st->transforms += 2;
      st->model_bytes += 4.0 * nb + kb * (4.0 + 3.0 * esz) + kb * (4.0 + 2.0 * esz);
    }
    if (!(dq > 0.0) || !isfinite(dq)) {           // H not positive on d (Theorem 3's condition fails)
      if (tid == 0) {
        st->flags |= CS_F_CG_BREAKDOWN;
        cg->done = 1;
        st->phase = BP_RESID;
      }
      return;
    }
    const T alpha = (T)(rr / dq);
    T* x = s.cx[st->cur];
    double acc = 0.0;
    for (int i = tid; i < k; i += blockDim.x) {
      x[i] += alpha * s.cd[i];
      const T rv = s.cr[i] - alpha * s.cq[i];
      s.cr[i] = rv;
      acc += (double)rv * (double)rv;
    }
    const double rn = block_sum_any(acc);
    if (tid == 0) {
      const bool fin = isfinite(rn);
      cg->rr[(it + 1) & 1] = rn;
      cg->beta = rn / rr;
      cg->iters = it + 1;
      st->it = it + 1;
      st->cg_iters += 1;
      const bool conv = rn <= cg->tol2 * cg->bb;
      if (!fin) st->flags |= CS_F_NONFINITE;
      if (!fin || conv || it + 1 >= st->cg_cap) {
        if (fin && !conv) st->flags |= CS_F_CG_MAXITER;
        cg->done = 1;
        st->phase = BP_RESID;
      }
    }
  } else {
    const int nrow = (int)(p.L1 >> 1);
    double r2 = 0.0;
    for (int i = tid; i < nrow; i += blockDim.x) r2 += s.prow[i];
    r2 = block_sum_any(r2);
    if (tid == 0) {
      st->rn = sqrt(r2);
      st->phase = BP_SELECT;
      st->transforms += 2;
      st->model_bytes += (nb + kb * (4.0 + esz)) + 3.0 * nb + 2.0 * nb;
    }
  }
}

// argmax of |c| outside the support: per-signal partials
template <typename T>
__global__ void k_b_argmax(const BSig<T>* __restrict__ sigs) {
  const BSig<T>& s = sigs[blockIdx.y];
  if (s.st->phase != BP_SELECT) return;
  const Plan& pl = s.plan;
  ArgKey best{0, 0, 0};
  const int64_t stp = (int64_t)gridDim.x * blockDim.x;
  for (int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; q < pl.n; q += stp) {
    if (bit_of(s.bits, q)) continue;
    const int64_t j = nat_of_key(q, pl);
    ArgKey kk{mag_bits(s.Cc[q]) + 1, 0xFFFFFFFFu - (uint32_t)j, 0};
    if (key_gt(kk, best)) best = kk;
  }
  best = block_max_key(best);
  if (threadIdx.x == 0) s.argpart[blockIdx.x] = best;
}

// The OMPR decision of one swap (one block of 1024 threads per signal): the
// entering index j, the stop tests, the drop step and the bitmap update.
template <typename T>
__global__ void k_b_select(const BSig<T>* __restrict__ sigs) {
  const BSig<T>& s = sigs[blockIdx.x];
  BState* st = s.st;
  if (st->phase != BP_SELECT) return;
  __shared__ int32_t sj;
  __shared__ int go;
  ArgKey best{0, 0, 0};
  for (int i = threadIdx.x; i < kBArgBlocks; i += blockDim.x)
    if (key_gt(s.argpart[i], best)) best = s.argpart[i];
  best = block_max_key(best);
  if (threadIdx.x == 0) {
    const int32_t j = best.hi ? (int32_t)(0xFFFFFFFFu - best.lo) : -1;
    go = 0;
    if (st->swaps >= st->max_outer) {
      st->flags |= CS_F_OUTER_MAXITER;
      st->phase = BP_DONE;
    } else if (st->rn <= 1e-12 * st->ynorm || j < 0) {
      st->phase = BP_DONE;
    } else {
      go = 1;
    }
    sj = j;
  }
  __syncthreads();
  if (!go) return;
  const int cur = st->cur;
  const int32_t d = ompr_drop_body<T>(s.cx[cur], s.list[cur], st->k, s.Cc, s.plan, (T)st->eta, sj);
  if (threadIdx.x == 0) {
    st->jd[0] = sj;
    st->jd[1] = d;
    if (d == sj) {
      st->phase = BP_DONE;
    } else {
      const uint32_t pj = (uint32_t)key_of_nat(sj, s.plan), pd = (uint32_t)key_of_nat(d, s.plan);
      s.bits[pd >> 5] &= ~(1u << (pd & 31));
      s.bits[pj >> 5] |= 1u << (pj & 31);
      st->swaps += 1;
    }
  }
}

// new support list and prefix counts in slot cur ^ 1
template <typename T>
__global__ void k_b_bits_count(const BSig<T>* __restrict__ sigs) {
  const BSig<T>& s = sigs[blockIdx.y];
  if (s.st->phase != BP_SELECT) return;
  const int64_t words = s.plan.words;
  if ((int64_t)blockIdx.x * kBitsPerBlockWords >= words) return;
  bits_count_body(s.bits, words, s.blockcnt, blockIdx.x);
}
template <typename T>
__global__ void k_b_bits_scan(const BSig<T>* __restrict__ sigs) {
  const BSig<T>& s = sigs[blockIdx.x];
  if (s.st->phase != BP_SELECT) return;
  bits_scan_body(s.blockcnt, (int)((s.plan.words + kBitsPerBlockWords - 1) / kBitsPerBlockWords));
}
template <typename T>
__global__ void k_b_bits_write(const BSig<T>* __restrict__ sigs) {
  const BSig<T>& s = sigs[blockIdx.y];
  const BState* st = s.st;
  if (st->phase != BP_SELECT) return;
  const int64_t words = s.plan.words;
  if ((int64_t)blockIdx.x * kBitsPerBlockWords >= words) return;
  const int nxt = st->cur ^ 1;
  bits_write_body(s.bits, words, s.blockcnt, s.list[nxt], st->k, s.wpre[nxt], blockIdx.x);
}

// warm start: x_new[i] = x_old at the same key, 0 for the new index
template <typename T>
__global__ void k_b_remap(const BSig<T>* __restrict__ sigs) {
  const BSig<T>& s = sigs[blockIdx.y];
  const BState* st = s.st;
  if (st->phase != BP_SELECT) return;
  const int k = st->k;
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= k) return;
  const int cur = st->cur, nxt = cur ^ 1;
  const int32_t* from = s.list[cur];
  const int32_t key = s.list[nxt][i];
  T v = (T)0;
  if (st->warm) {
    int lo = 0, hi = k - 1;
    while (lo <= hi) {
      const int mid = (lo + hi) >> 1;
      const int32_t m = from[mid];
      if (m == key) { v = s.cx[cur][mid]; break; }
      if (m < key) lo = mid + 1; else hi = mid - 1;
    }
  }
  s.cx[nxt][i] = v;
}

// switch to the new support: b = C0 on it, b^T b, next solve
template <typename T>
__global__ void k_b_finish(const BSig<T>* __restrict__ sigs) {
  const BSig<T>& s = sigs[blockIdx.x];
  BState* st = s.st;
  if (st->phase != BP_SELECT) return;
  const int k = st->k, nxt = st->cur ^ 1;
  const int32_t* list = s.list[nxt];
  double acc = 0.0;
  for (int i = threadIdx.x; i < k; i += blockDim.x) {
    const T v = s.C0[list[i]];
    s.cb[i] = v;
    acc += (double)v * (double)v;
  }
  acc = block_sum_any(acc);
  if (threadIdx.x == 0) {
    st->cur = nxt;
    st->bb = acc;
    st->phase = BP_WARM;
  }
}

__global__ void k_b_active(const BState* __restrict__ st, int count, int32_t* __restrict__ out) {
  __shared__ int32_t tot;
  if (threadIdx.x == 0) tot = 0;
  __syncthreads();
  int32_t n = 0;
  for (int i = threadIdx.x; i < count; i += blockDim.x) n += st[i].phase != BP_DONE;
  if (n) atomicAdd(&tot, n);
  __syncthreads();
  if (threadIdx.x == 0) *out = tot;
}

// ------------------------------------------------------------------ host driver
static size_t align256(size_t v) { return (v + 255) / 256 * 256; }

size_t batch_layout(cs_dtype dt, int count, const cs_batch_item* items, std::vector<size_t>* offs) {
  size_t off = 0;
  for (int i = 0; i < count; ++i) {
    const size_t sz = workspace_bytes(dt, items[i].op.n, items[i].op.m, items[i].k, CS_ALGO_OMPR);
    if (sz == 0) return 0;
    off = align256(off);
    if (offs) offs->push_back(off);
    off += sz;
  }
  off = align256(off) + align256((size_t)count * sizeof(BSig<double>));
  off += align256((size_t)count * sizeof(BState));
  off += align256((size_t)count * sizeof(int32_t));
  off += 256;   // unfinished-signal counter
  return off;
}

template <typename T>
void run_ompr_batched(int count, const cs_batch_item* items, double tol, const cs_params& prm, int cg_threads,
                      void* ws, size_t ws_bytes, cs_info* infos, hipStream_t stream) {
  const cs_dtype dt = sizeof(T) == 4 ? CS_F32 : CS_F64;
  std::vector<size_t> offs;
  const size_t need = batch_layout(dt, count, items, &offs);
  if (need == 0) throw Error(CS_E_SHAPE, "unsupported size in batch");
  if (ws_bytes < need) throw Error(CS_E_WORKSPACE, "workspace too small: need " + std::to_string(need) + " bytes");
  char* base = (char*)ws;
  size_t off = align256(offs.back() + workspace_bytes(dt, items[count - 1].op.n, items[count - 1].op.m,
                                                        items[count - 1].k, CS_ALGO_OMPR));
  BSig<T>* d_sigs = (BSig<T>*)(base + off);
  off += align256((size_t)count * sizeof(BSig<double>));
  BState* d_st = (BState*)(base + off);
  off += align256((size_t)count * sizeof(BState));
  int32_t* d_ids = (int32_t*)(base + off);
  off += align256((size_t)count * sizeof(int32_t));
  int32_t* d_active = (int32_t*)(base + off);

  // per-signal set-up on the single-signal code: operator tables, y, A^T y,
  // the initial top-K support
  std::vector<Ctx<T>> cs(count);
  std::vector<BSig<T>> hs(count);
  std::vector<BState> hst(count);
  int kmax = 1;
  int64_t nbw = 1;
  for (int i = 0; i < count; ++i) {
    const cs_batch_item& it = items[i];
    Ctx<T>& c = cs[i];
    ctx_init<T>(c, &it.op, it.k, base + offs[i], ws_bytes - offs[i], stream);
    setup_operator<T>(c);
    load_measurements<T>(c, (const T*)it.y);
    topk_dense<T>(c, c.C0, nullptr, it.k, c.bits[0]);
    bits_to_list<T>(c, c.bits[0], c.list[0], it.k, c.wpre[0]);
    BSig<T>& h = hs[i];
    h.plan = c.plan;
    h.W = c.W; h.Cc = c.Cc; h.C0 = c.C0; h.Yf = c.Yf;
    h.tw_col = c.tw_col; h.tw_row = c.tw_row;
    h.bits = c.bits[0];
    h.wpre[0] = c.wpre[0]; h.wpre[1] = c.wpre[1];
    h.list[0] = c.list[0]; h.list[1] = c.list[1];
    h.cb = c.cb; h.cx[0] = c.cx; h.cx[1] = c.cx3;
    h.cr = c.cr; h.cd = c.cd; h.cq = c.cq;
    h.pgrid = c.pgrid; h.prow = c.partial2;
    h.argpart = c.argpart; h.blockcnt = c.blockcnt;
    h.cg = c.cg;
    h.st = d_st + i;
    BState& b = hst[i];
    std::memset(&b, 0, sizeof(BState));
    b.phase = BP_WARM;
    b.k = it.k;
    b.max_outer = prm.max_outer > 0 ? prm.max_outer : 4 * it.k;
    b.cg_cap = prm.cg_max_iter > 0 ? prm.cg_max_iter : 2 * it.k + 50;
    b.warm = prm.warm_start != 0;
    b.tol2 = tol * tol;
    b.eta = prm.ompr_eta > 0 ? prm.ompr_eta : (double)it.op.n / (double)it.op.m;
    b.ynorm = c.ynorm;
    b.model_bytes = c.model_bytes;
    b.transforms = c.transforms;
    kmax = std::max(kmax, it.k);
    nbw = std::max<int64_t>(nbw, (c.plan.words + kBitsPerBlockWords - 1) / kBitsPerBlockWords);
  }
  // size classes: signals with the same N share the transform kernels
  std::map<int, std::vector<int32_t>> cls;
  for (int i = 0; i < count; ++i) cls[cs[i].plan.logn].push_back(i);
  std::vector<int32_t> ids;
  struct Cls { int first, cnt; Plan plan; };
  std::vector<Cls> cl;
  for (auto& kv : cls) {
    cl.push_back(Cls{(int)ids.size(), (int)kv.second.size(), cs[kv.second[0]].plan});
    ids.insert(ids.end(), kv.second.begin(), kv.second.end());
  }
  CS_HIP(hipMemcpyAsync(d_sigs, hs.data(), count * sizeof(BSig<T>), hipMemcpyHostToDevice, stream));
  CS_HIP(hipMemcpyAsync(d_st, hst.data(), count * sizeof(BState), hipMemcpyHostToDevice, stream));
  CS_HIP(hipMemcpyAsync(d_ids, ids.data(), count * sizeof(int32_t), hipMemcpyHostToDevice, stream));
  hipLaunchKernelGGL(k_b_start<T>, dim3(count), dim3(cg_threads), 0, stream, d_sigs);
  CS_LAUNCH_CHECK();
  CS_HIP(hipStreamSynchronize(stream));   // the host arrays above go out of scope only after the copies

  // capture kBSteps batched steps
  hipStream_t cap = nullptr;
  CS_HIP(hipStreamCreateWithFlags(&cap, hipStreamNonBlocking));
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
  CS_HIP(hipStreamBeginCapture(cap, hipStreamCaptureModeThreadLocal));
  const unsigned nsig = (unsigned)count;
  for (int stp = 0; stp < kBSteps; ++stp) {
    for (const Cls& c : cl) {
      const KernelSet<T>& ks = kernels_plan<T>(c.plan);
      ks.col_fwd_b<<<dim3((unsigned)(c.plan.L2 >> c.plan.logB), c.cnt), dim3(ks.nt_col), c.plan.lds_col, cap>>>(
          d_sigs, d_ids + c.first);
      CS_LAUNCH_CHECK();
    }
    for (const Cls& c : cl) {
      const KernelSet<T>& ks = kernels_plan<T>(c.plan);
      ks.row_b<<<dim3((unsigned)(c.plan.L1 >> 1), c.cnt), dim3(ks.nt_row), c.plan.lds_row, cap>>>(d_sigs,
                                                                                                  d_ids + c.first);
      CS_LAUNCH_CHECK();
    }
    for (const Cls& c : cl) {
      const KernelSet<T>& ks = kernels_plan<T>(c.plan);
      ks.col_inv_b<<<dim3((unsigned)(c.plan.L2 >> c.plan.logB), c.cnt), dim3(ks.nt_col), c.plan.lds_col, cap>>>(
          d_sigs, d_ids + c.first);
      CS_LAUNCH_CHECK();
    }
    hipLaunchKernelGGL(k_b_post<T>, dim3(nsig), dim3(cg_threads), 0, cap, d_sigs);
    hipLaunchKernelGGL(k_b_argmax<T>, dim3(kBArgBlocks, nsig), dim3(256), 0, cap, d_sigs);
    hipLaunchKernelGGL(k_b_select<T>, dim3(nsig), dim3(1024), 0, cap, d_sigs);
    hipLaunchKernelGGL(k_b_bits_count<T>, dim3((unsigned)nbw, nsig), dim3(256), 0, cap, d_sigs);
    hipLaunchKernelGGL(k_b_bits_scan<T>, dim3(nsig), dim3(1024), 0, cap, d_sigs);
    hipLaunchKernelGGL(k_b_bits_write<T>, dim3((unsigned)nbw, nsig), dim3(256), 0, cap, d_sigs);
    hipLaunchKernelGGL(k_b_remap<T>, dim3((unsigned)((kmax + 255) / 256), nsig), dim3(256), 0, cap, d_sigs);
    hipLaunchKernelGGL(k_b_finish<T>, dim3(nsig), dim3(cg_threads), 0, cap, d_sigs);
    CS_LAUNCH_CHECK();
  }
  hipLaunchKernelGGL(k_b_active, dim3(1), dim3(256), 0, cap, (const BState*)d_st, count, d_active);
  CS_LAUNCH_CHECK();
  CS_HIP(hipStreamEndCapture(cap, &graph));
  CS_HIP(hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0));

  // Replay until no signal is left.  Each swap takes at most cg_cap + 2 steps,
  // so the bound below is never reached by a run that terminates as designed.
  int64_t max_steps = 0;
  for (int i = 0; i < count; ++i)
    max_steps = std::max<int64_t>(max_steps, (int64_t)(hst[i].max_outer + 1) * (hst[i].cg_cap + 3) + 2);
  const int64_t max_replays = max_steps / kBSteps + 2;
  int32_t active = count;
  int64_t replays = 0;
  while (active > 0 && replays < max_replays) {
    CS_HIP(hipGraphLaunch(exec, stream));
    ++replays;
    dev_read(stream, d_active, &active, sizeof(int32_t));
  }
  CS_HIP(hipGraphExecDestroy(exec));
  CS_HIP(hipGraphDestroy(graph));
  CS_HIP(hipStreamDestroy(cap));

  CS_HIP(hipMemcpy(hst.data(), d_st, count * sizeof(BState), hipMemcpyDeviceToHost));
  for (int i = 0; i < count; ++i) {
    Ctx<T>& c = cs[i];
    const BState& b = hst[i];
    const int cur = b.cur;
    write_output<T>(c, c.list[cur], cur ? c.cx3 : c.cx, b.k, (T*)items[i].s, items[i].support);
    if (infos) {
      cs_info& inf = infos[i];
      std::memset(&inf, 0, sizeof(cs_info));
      inf.outer_iters = b.swaps;
      inf.flags = b.flags | (b.phase != BP_DONE ? CS_F_OUTER_MAXITER : 0);
      inf.cg_iters = b.cg_iters;
      inf.transforms = b.transforms;
      inf.resid_norm = b.rn;
      inf.model_bytes = b.model_bytes;
    }
  }
  CS_HIP(hipStreamSynchronize(stream));
}

template void run_ompr_batched<float>(int, const cs_batch_item*, double, const cs_params&, int, void*, size_t,
                                      cs_info*, hipStream_t);
template void run_ompr_batched<double>(int, const cs_batch_item*, double, const cs_params&, int, void*, size_t,
                                       cs_info*, hipStream_t);

}  // namespace csr
