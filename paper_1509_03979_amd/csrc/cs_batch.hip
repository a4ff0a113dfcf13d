// Batched OMPR: many signals of uneven N, M and K recovered together.
//
// Every signal keeps its own device state (BState: phase, current support
// slot, CG iteration, swap count, counters) next to the workspace of a
// single-signal call.  One batched step moves every unfinished signal one
// stage along the OMPR loop of the single-signal driver:
//   WARM    r = b - H x (warm start), r^T r, CG set-up
//   ITER    one CG iteration (the CG loop body of Algorithm 1)
//   RESID   r = y - A x, ||r||, the correlation F^T D^T r and its argmax
//   SELECT  the stop tests, the drop step and the swap: the new support's
//           list, prefix counts, remapped x and right-hand side
// with the same decision rules, so each signal follows the path the
// single-signal OMPR takes.  A step is a fixed sequence of launches: the three
// transform passes once per size class (the signal in blockIdx.y, its shape a
// template parameter), then two per-signal kernels (CG / residual / argmax,
// then the swap), each returning at once for signals in another phase.  The
// host captures several steps and a compaction of the still-running signals
// in a HIP graph and replays it until none is left, capturing a smaller
// graph over the running signals once half of them, or a whole size class,
// have stopped.
#include "cs_device.h"
#include "cs_kernels.h"

#include <algorithm>
#include <cmath>
#include <cstring>
#include <map>
#include <vector>

namespace csr {

constexpr int kBArgBlocks = 64;   // most argmax blocks per signal (fits the argpart buffer)

// argmax blocks of a signal: one per 4096 candidates (16 per thread of
// k_b_arg), 1 .. kBArgBlocks
__host__ __device__ __forceinline__ int arg_blocks(int64_t n) {
  const int64_t b = n >> 12;
  return (int)(b < 1 ? 1 : (b > kBArgBlocks ? kBArgBlocks : b));
}
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

// Argmax partials of a signal's fresh correlations (RESID phase): workgroup
// (x, y) takes keys x, x + nab B, ... of signal y, keeps its best two
// (the runner-up gives the decision's margin).  Small workgroups: most of
// the grid exits at once (signals in other phases, small signals' extra x).
constexpr int kBArgThreads = 256;
template <typename T>
__global__ __launch_bounds__(kBArgThreads) void k_b_arg(const BSig<T>* __restrict__ sigs,
                                                        const int32_t* __restrict__ ids) {
  const BSig<T>& s = sigs[ids[blockIdx.y]];
  if (s.st->phase != BP_RESID) return;
  const Plan& p = s.plan;
  const int nab = arg_blocks(p.n);
  if ((int)blockIdx.x >= nab) return;
  K2 t;
  const int64_t stp = (int64_t)nab * blockDim.x;
  // rounds of U keys per thread with every load of a round issued first (a
  // key at a time would wait for each load in turn)
  constexpr int U = 8;
  const uint32_t* __restrict__ bits = s.bits;
  const T* __restrict__ cc = s.Cc;
  for (int64_t q0 = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; q0 < p.n; q0 += U * stp) {
    uint32_t w[U];
    T v[U];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int64_t q = min(q0 + u * stp, p.n - 1);
      w[u] = bits[q >> 5];
      v[u] = cc[q];
    }
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int64_t q = q0 + u * stp;
      if (q < p.n && !((w[u] >> (q & 31)) & 1u))
        t.add(mag_bits(v[u]) + 1, 0xFFFFFFFFu - (uint32_t)nat_of_key(q, p));
    }
  }
  block_max_key2(t);
  if (threadIdx.x == 0) {
    s.argpart[2 * blockIdx.x] = t.best();
    s.argpart[2 * blockIdx.x + 1] = t.second();
  }
}

// Per-signal scalar work after the transform passes of a step (after k_b_arg,
// which reads the RESID phase this kernel moves on): the CG start (WARM), the
// CG update (ITER) or the residual norm (RESID, then SELECT).  One workgroup
// per signal, ids[blockIdx.x].
template <typename T>
__global__ void k_b_post(const BSig<T>* __restrict__ sigs, const int32_t* __restrict__ ids) {
  const BSig<T>& s = sigs[ids[blockIdx.x]];
  BState* st = s.st;
  const int phase = st->phase;
  if (phase > BP_RESID) return;
  const Plan& p = s.plan;
  const int tid = threadIdx.x;
  CgScalars* cg = s.cg;
  const int k = st->k;
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
      cg->ref = st->tol_abs ? 1.0 : bb;
      cg->tol2 = st->tol2;
      cg->iters = 0;
      cg->flags = 0;
      const bool fin = isfinite(rr) && isfinite(bb);
      const bool conv = rr <= st->tol2 * cg->ref;
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
    // d^T q from the inverse pass's per-workgroup partials (fixed order)
    const int ncol = (int)(p.L2 >> p.logB);
    double dqs = 0.0;
    for (int i = tid; i < ncol; i += blockDim.x) dqs += s.pgrid[i];
    const double dq = block_sum_any(dqs);
    if (tid == 0) cg->dq = dq;
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
    T* __restrict__ x = s.cx[st->cur];
    T* __restrict__ r = s.cr;
    const T* __restrict__ dv = s.cd;
    const T* __restrict__ qv = s.cq;
    double acc = 0.0;
    // distinct buffers: the loads of several slots go out together
#pragma unroll 4
    for (int i = tid; i < k; i += blockDim.x) {
      x[i] += alpha * dv[i];
      const T rv = r[i] - alpha * qv[i];
      r[i] = rv;
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
      const bool conv = rn <= cg->tol2 * cg->ref;
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

// One OMPR swap per signal (one block of 1024 threads): the entering index j
// (argmax partials), the stop tests, the drop step, then the new support
// edited in place of a rebuild: bitmap bits, the ascending key list and
// prefix counts with one key out and one in, the warm-start x (the shared
// keys keep their values, the new one starts at 0) and b = C0 on the new list.
template <typename T>
__global__ void k_b_select(const BSig<T>* __restrict__ sigs, const int32_t* __restrict__ ids) {
  const BSig<T>& s = sigs[ids[blockIdx.x]];
  BState* st = s.st;
  if (st->phase != BP_SELECT) return;
  __shared__ int32_t sj, sd, spd, spj;
  __shared__ int go;
  const int tid = threadIdx.x;
  K2 t;
  const int nab = arg_blocks(s.plan.n);
  for (int i = tid; i < nab; i += blockDim.x) {
    const ArgKey a = s.argpart[2 * i], b = s.argpart[2 * i + 1];
    t.add(a.hi, a.lo, b.hi, b.lo);
  }
  block_max_key2(t);
  if (tid == 0) {
    const int32_t j = t.bh ? (int32_t)(0xFFFFFFFFu - t.bl) : -1;
    if (t.bh && t.sh && st->swaps < st->max_outer) {
      const double vb = key_value<T>(t.bh);
      note_margin(&st->mmin, &st->mrel, vb - key_value<T>(t.sh), vb);
    }
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
  const int cur = st->cur, nxt = cur ^ 1, k = st->k;
  double m = -1.0, mk = 0.0;
  const int32_t d = ompr_drop_body<T>(s.cx[cur], s.list[cur], k, s.Cc, s.plan, (T)st->eta, sj, &m, &mk);
  if (tid == 0) {
    note_margin(&st->mmin, &st->mrel, m, mk);
    sd = d;
    go = d != sj;
    st->jd[0] = sj;
    st->jd[1] = d;
    if (!go) st->phase = BP_DONE;
    spd = -1;
    spj = 0;
  }
  __syncthreads();
  if (!go) return;
  const int32_t kj = (int32_t)key_of_nat(sj, s.plan), kd = (int32_t)key_of_nat(sd, s.plan);
  const int32_t* old = s.list[cur];
  // pd: slot of kd in the old list; pj: old keys below kj (kj is not in it);
  // the loads of U slots go out before any comparison
  {
    constexpr int U = 4;
    const int bd = blockDim.x;
    for (int i0 = tid; i0 < k; i0 += U * bd) {
      int32_t v[U], vn[U];
#pragma unroll
      for (int u = 0; u < U; ++u) {
        const int i = min(i0 + u * bd, k - 1);
        v[u] = old[i];
        vn[u] = old[min(i + 1, k - 1)];
      }
#pragma unroll
      for (int u = 0; u < U; ++u) {
        const int i = i0 + u * bd;
        if (i >= k) continue;
        if (v[u] == kd) spd = i;
        if (v[u] < kj && (i + 1 == k || vn[u] > kj)) spj = i + 1;
      }
    }
  }
  __syncthreads();
  const int pd = spd, pj = spj;
  if (pd < 0) {              // the dropped index is always on the support; stop rather than read past the list
    if (tid == 0) st->phase = BP_DONE;
    return;
  }
  const int q = pj - (pd < pj ? 1 : 0);          // slot of kj in the new list
  int32_t* __restrict__ nl = s.list[nxt];
  const T* __restrict__ xo = s.cx[cur];
  T* __restrict__ xn = s.cx[nxt];
  const T* __restrict__ c0 = s.C0;
  const bool warm = st->warm != 0;
  double acc = 0.0;
  // in rounds of U slots per thread, every load of a round issued before its
  // results are used (the loop is a chain of dependent reads otherwise)
  constexpr int U = 4;
  const int bd = blockDim.x;
  for (int i0 = tid; i0 < k; i0 += U * bd) {
    int32_t key[U];
    T xv[U];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int i = i0 + u * bd;
      const int r = i - (i > q ? 1 : 0);         // slot in the old list without kd
      const int o = min(r + (r >= pd ? 1 : 0), k - 1);
      key[u] = (i == q) ? kj : old[o];
      xv[u] = (warm && i != q) ? xo[o] : (T)0;
    }
    T bv[U];
#pragma unroll
    for (int u = 0; u < U; ++u) bv[u] = c0[i0 + u * bd < k ? key[u] : kj];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int i = i0 + u * bd;
      if (i < k) {
        nl[i] = key[u];
        xn[i] = xv[u];
        s.cb[i] = bv[u];
        acc += (double)bv[u] * (double)bv[u];
      }
    }
  }
  // prefix counts: words after kj's word gain one, words after kd's lose one
  const int64_t words = s.plan.words;
  const int64_t wj = kj >> 5, wd = kd >> 5;
  const uint32_t* __restrict__ wo = s.wpre[cur];
  uint32_t* __restrict__ wn = s.wpre[nxt];
  constexpr int UW = 8;
  for (int64_t w0 = tid; w0 < words; w0 += (int64_t)UW * bd) {
    uint32_t v[UW];
#pragma unroll
    for (int u = 0; u < UW; ++u) {
      const int64_t w = w0 + (int64_t)u * bd;
      v[u] = w < words ? wo[w] : 0u;
    }
#pragma unroll
    for (int u = 0; u < UW; ++u) {
      const int64_t w = w0 + (int64_t)u * bd;
      if (w < words) wn[w] = v[u] + (w > wj ? 1u : 0u) - (w > wd ? 1u : 0u);
    }
  }
  const double bb = block_sum_any(acc);
  if (tid == 0) {
    s.bits[kd >> 5] &= ~(1u << (kd & 31));
    s.bits[kj >> 5] |= 1u << (kj & 31);
    if (st->swaps < s.moves_cap) {
      s.moves[2 * st->swaps] = sj;
      s.moves[2 * st->swaps + 1] = sd;
    }
    st->swaps += 1;
    st->cur = nxt;
    st->bb = bb;
    st->phase = BP_WARM;
  }
}

// Compacts the ids of unfinished signals (kept in class order) and counts
// them per class: out_cnt[c] for class c, out_cnt[ncls] in total.  One block
// of 1024 threads.
__global__ void k_b_compact(const BState* __restrict__ st, const int32_t* __restrict__ ids,
                            const int32_t* __restrict__ cls_of, int cnt, int ncls, int32_t* __restrict__ out_ids,
                            int32_t* __restrict__ out_cnt) {
  __shared__ int32_t scan[1024];
  __shared__ int32_t carry;
  __shared__ int32_t ccnt[64];
  const int tid = threadIdx.x;
  if (tid == 0) carry = 0;
  for (int c = tid; c < 64; c += blockDim.x) ccnt[c] = 0;
  __syncthreads();
  for (int base = 0; base < cnt; base += 1024) {
    const int i = base + tid;
    const int32_t id = (i < cnt) ? ids[i] : -1;
    const int a = (i < cnt && st[id].phase != BP_DONE) ? 1 : 0;
    if (a) atomicAdd(&ccnt[cls_of[i]], 1);
    scan[tid] = a;
    __syncthreads();
    for (int off = 1; off < 1024; off <<= 1) {
      const int32_t t = tid >= off ? scan[tid - off] : 0;
      __syncthreads();
      scan[tid] += t;
      __syncthreads();
    }
    if (a) out_ids[carry + scan[tid] - 1] = id;
    __syncthreads();
    if (tid == 1023) carry += scan[1023];
    __syncthreads();
  }
  for (int c = tid; c < ncls; c += blockDim.x) out_cnt[c] = ccnt[c];
  if (tid == 0) out_cnt[ncls] = carry;
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
  off += 3 * align256((size_t)count * sizeof(int32_t));   // active ids, their classes, compacted ids
  off += 256;                                              // per-class counts (at most 64 classes)
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
  int32_t* d_cls = (int32_t*)(base + off);
  off += align256((size_t)count * sizeof(int32_t));
  int32_t* d_act = (int32_t*)(base + off);
  off += align256((size_t)count * sizeof(int32_t));
  int32_t* d_cnt = (int32_t*)(base + off);

  // per-signal set-up on the single-signal code: operator tables, y, A^T y,
  // the initial top-K support
  std::vector<Ctx<T>> cs(count);
  std::vector<BSig<T>> hs(count);
  std::vector<BState> hst(count);
  for (int i = 0; i < count; ++i) {
    const cs_batch_item& it = items[i];
    Ctx<T>& c = cs[i];
    ctx_init<T>(c, &it.op, it.k, base + offs[i], ws_bytes - offs[i], stream);
    setup_operator<T>(c);
    load_measurements<T>(c, (const T*)it.y);
    sel_reset<T>(c);
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
    h.moves = it.moves_cap > 0 ? it.moves : nullptr;
    h.moves_cap = it.moves_cap > 0 ? it.moves_cap : 0;
    BState& b = hst[i];
    std::memset(&b, 0, sizeof(BState));
    b.phase = BP_WARM;
    b.k = it.k;
    b.max_outer = prm.max_outer > 0 ? prm.max_outer : 4 * it.k;
    b.cg_cap = prm.cg_max_iter > 0 ? prm.cg_max_iter : 2 * it.k + 50;
    b.warm = prm.warm_start != 0;
    b.tol2 = tol * tol;
    b.tol_abs = prm.tol_abs != 0;
    b.eta = prm.ompr_eta > 0 ? prm.ompr_eta : (double)it.op.n / (double)it.op.m;
    b.ynorm = c.ynorm;
    b.model_bytes = c.model_bytes;
    b.transforms = c.transforms;
    b.mmin = __builtin_huge_val();   // the initial top-K's margin is in the signal's selection state
    b.mrel = __builtin_huge_val();
  }
  // size classes: signals with the same N share the transform kernels
  std::map<int, int> cls_index;
  for (int i = 0; i < count; ++i) cls_index[cs[i].plan.logn] = 0;
  std::vector<Plan> cls_plan;
  for (auto& kv : cls_index) {
    kv.second = (int)cls_plan.size();
    for (int i = 0; i < count; ++i)
      if (cs[i].plan.logn == kv.first) { cls_plan.push_back(cs[i].plan); break; }
  }
  const int ncls = (int)cls_plan.size();
  std::vector<int32_t> ids, cls_of;               // active signals in class order
  for (int c = 0; c < ncls; ++c)
    for (int i = 0; i < count; ++i)
      if (cs[i].plan.logn == cls_plan[c].logn) { ids.push_back(i); cls_of.push_back(c); }
  CS_HIP(hipMemcpyAsync(d_sigs, hs.data(), count * sizeof(BSig<T>), hipMemcpyHostToDevice, stream));
  CS_HIP(hipMemcpyAsync(d_st, hst.data(), count * sizeof(BState), hipMemcpyHostToDevice, stream));
  hipLaunchKernelGGL(k_b_start<T>, dim3(count), dim3(cg_threads), 0, stream, d_sigs);
  CS_LAUNCH_CHECK();
  CS_HIP(hipStreamSynchronize(stream));   // the host arrays above are read by the copies

  // Capture kBSteps batched steps over the active signals `ids`, then the
  // compaction of the ones still running.
  hipStream_t cap = nullptr;
  CS_HIP(hipStreamCreateWithFlags(&cap, hipStreamNonBlocking));
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
  std::vector<int32_t> graph_cnt(ncls, 0);
  auto build = [&]() {
    const int na = (int)ids.size();
    int nab = 1;
    for (int32_t id : ids) nab = std::max(nab, arg_blocks(cs[id].plan.n));
    CS_HIP(hipMemcpyAsync(d_ids, ids.data(), na * sizeof(int32_t), hipMemcpyHostToDevice, stream));
    CS_HIP(hipMemcpyAsync(d_cls, cls_of.data(), na * sizeof(int32_t), hipMemcpyHostToDevice, stream));
    CS_HIP(hipStreamSynchronize(stream));
    std::vector<int> first(ncls, 0);
    std::fill(graph_cnt.begin(), graph_cnt.end(), 0);
    for (int i = na - 1; i >= 0; --i) { first[cls_of[i]] = i; ++graph_cnt[cls_of[i]]; }
    CS_HIP(hipStreamBeginCapture(cap, hipStreamCaptureModeThreadLocal));
    for (int stp = 0; stp < kBSteps; ++stp) {
      for (int pass = 0; pass < 3; ++pass) {
        for (int c = 0; c < ncls; ++c) {
          if (!graph_cnt[c]) continue;
          const Plan& pl = cls_plan[c];
          const KernelSet<T>& ks = kernels_plan<T>(pl);
          const int32_t* cid = d_ids + first[c];
          const dim3 gcol((unsigned)(pl.L2 >> pl.logB), (unsigned)graph_cnt[c]);
          if (pass == 0) ks.col_fwd_b<<<gcol, dim3(ks.nt_col), pl.lds_col, cap>>>(d_sigs, cid);
          else if (pass == 1)
            ks.row_b<<<dim3((unsigned)(pl.L1 >> 1), (unsigned)graph_cnt[c]), dim3(ks.nt_row), pl.lds_row, cap>>>(
                d_sigs, cid);
          else ks.col_inv_b<<<gcol, dim3(ks.nt_col), pl.lds_col, cap>>>(d_sigs, cid);
          CS_LAUNCH_CHECK();
        }
      }
      hipLaunchKernelGGL(k_b_arg<T>, dim3((unsigned)nab, (unsigned)na), dim3(kBArgThreads), 0, cap, d_sigs,
                         (const int32_t*)d_ids);
      hipLaunchKernelGGL(k_b_post<T>, dim3((unsigned)na), dim3(cg_threads), 0, cap, d_sigs, (const int32_t*)d_ids);
      hipLaunchKernelGGL(k_b_select<T>, dim3((unsigned)na), dim3(1024), 0, cap, d_sigs, (const int32_t*)d_ids);
      CS_LAUNCH_CHECK();
    }
    hipLaunchKernelGGL(k_b_compact, dim3(1), dim3(1024), 0, cap, (const BState*)d_st, (const int32_t*)d_ids,
                       (const int32_t*)d_cls, na, ncls, d_act, d_cnt);
    CS_LAUNCH_CHECK();
    CS_HIP(hipStreamEndCapture(cap, &graph));
    CS_HIP(hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0));
  };
  auto drop = [&]() {
    if (exec) CS_HIP(hipGraphExecDestroy(exec));
    if (graph) CS_HIP(hipGraphDestroy(graph));
    exec = nullptr;
    graph = nullptr;
  };
  build();

  // Replay until no signal is left; re-capture over the running signals once
  // half of them have stopped or a size class has emptied.  Each swap takes at
  // most cg_cap + 2 steps, so the bound below is never reached by a run that
  // terminates as designed.
  int64_t max_steps = 0;
  for (int i = 0; i < count; ++i)
    max_steps = std::max<int64_t>(max_steps, (int64_t)(hst[i].max_outer + 1) * (hst[i].cg_cap + 3) + 2);
  const int64_t max_replays = max_steps / kBSteps + 2;
  std::vector<int32_t> cnt(ncls + 1, 0);
  for (int64_t replays = 0; replays < max_replays; ++replays) {
    CS_HIP(hipGraphLaunch(exec, stream));
    dev_read(stream, d_cnt, cnt.data(), (ncls + 1) * sizeof(int32_t));
    const int total = cnt[ncls];
    if (total == 0) break;
    bool emptied = false;
    for (int c = 0; c < ncls; ++c) emptied |= graph_cnt[c] > 0 && cnt[c] == 0;
    if (emptied || 2 * total <= (int)ids.size()) {
      ids.assign(total, 0);
      CS_HIP(hipMemcpy(ids.data(), d_act, total * sizeof(int32_t), hipMemcpyDeviceToHost));
      cls_of.resize(total);
      for (int i = 0; i < total; ++i) cls_of[i] = cls_index[cs[ids[i]].plan.logn];
      drop();
      build();
    }
  }
  drop();
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
      double mm = 0.0, mr = 0.0;
      margins_read<T>(c, &mm, &mr);   // the initial top-K
      mm = std::min(mm, b.mmin);
      mr = std::min(mr, b.mrel);
      const double trel = b.tol_abs ? tol / std::max(b.ynorm, 1e-300) : tol;
      if (near_tie(mr, trel, sizeof(T) == 4, c.plan.logn)) inf.flags |= CS_F_NEAR_TIE;
      inf.min_margin = std::isfinite(mm) ? mm : -1.0;
    }
  }
  CS_HIP(hipStreamSynchronize(stream));
}

template void run_ompr_batched<float>(int, const cs_batch_item*, double, const cs_params&, int, void*, size_t,
                                      cs_info*, hipStream_t);
template void run_ompr_batched<double>(int, const cs_batch_item*, double, const cs_params&, int, void*, size_t,
                                       cs_info*, hipStream_t);

}  // namespace csr
