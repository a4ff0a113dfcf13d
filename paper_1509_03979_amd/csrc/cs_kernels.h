// Transform pass kernels, specialised per four-step shape.
//
// Column pass k_col<T, INV, LOGL1, LOGB, LOGE>: one workgroup owns a strip of
// B = 2^LOGB adjacent columns of the L1 x L2 view of z and runs B length-L1
// FFTs on it in LDS (column-major layout, so a global row segment of B
// complex values maps to B consecutive LDS slots).  `in` and `out` may be the
// same buffer: a workgroup reads its whole strip before writing it back.
//
// Row pass k_row<T, LOGL2>: one workgroup owns a mirror row pair and runs
// four-step twiddle -> row FFT -> DCT post-processing -> mask or residual ->
// DCT pre-processing -> inverse row FFT -> conjugate twiddle; the mode (H-apply,
// residual, forward-only, adjoint-only) is a uniform argument.
#pragma once

#include "cs_device.h"
#include "cs_fft.h"

#include <type_traits>

namespace csr {

// ------------------------------------------------------------------ shapes

// Four-step split for an L = 2^l point complex FFT (N = 2^(l+1) real points).
// Measured on MI355X: what matters most is that two or more workgroups of
// each pass fit on a CU (so one's global-memory phase overlaps another's LDS
// FFT), i.e. at most ~68 KB of padded LDS per workgroup.  Large N therefore
// use rows of 4096 (FP32) / 2048 (FP64) complex and column strips of
// B * L1 <= 8192 (FP32) / 4096 (FP64) elements; smaller N split L about evenly
// with L1 >= L2 (more row-pair workgroups), and strips stay >= 4 columns wide
// (32 B segments) unless the row count is small.  Every shape keeps each
// workgroup within 128 KB of LDS (plus padding).
__host__ __device__ constexpr Shape shape_for(bool f64, int l) {
  const int maxL2 = f64 ? 11 : 12;
  const int maxL1 = f64 ? 13 : 14;      // one column of L1 complex values within 128 KB
  const int maxE = f64 ? 4096 : 8192;
  int logL1 = (l + 1) / 2;
  if (l >= 18) logL1 = l / 2;
  if (l - logL1 > maxL2) logL1 = l - maxL2;
  if (logL1 > maxL1) logL1 = maxL1;     // then L2 takes the rest (two rows still within 128 KB)
  if (logL1 < 1) logL1 = 1;
  const int logL2 = l - logL1;
  int B = 16;
  if (B > (1 << logL2)) B = 1 << logL2;
  while (B > 1 && B * (1 << logL1) > maxE) B >>= 1;
  while (B > 4 && ((1 << logL2) / B) < 256) B >>= 1;
  int logB = 0;
  while ((1 << logB) < B) ++logB;
  // Mid-size problems have too few workgroups to fill 256 CUs with 16 elements
  // per thread; hold fewer (smaller radix, more LDS stages, more waves).
  const int logE = (l >= 21) ? 4 : (l >= 17 ? 3 : 2);
  return Shape{logL1, logL2, logB, logE};
}

constexpr int kMinL = 3;    // N = 16
constexpr int kMaxL = 25;   // N = 2^26

// ------------------------------------------------------------------ column pass
__device__ __forceinline__ double wg_sum(double v, double* red, int nwaves) {
  for (int off = 32; off > 0; off >>= 1) v += __shfl_down(v, off, 64);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = v;
  __syncthreads();
  double s = 0.0;
  for (int i = 0; i < nwaves; ++i) s += red[i];
  __syncthreads();
  return s;
}

// An empty register constraint: the value is taken as changed here, so no
// computation on it moves above this point (no instruction is emitted).
template <typename V>
__device__ __forceinline__ void opaque(V& v) {
  asm volatile("" : "+v"(v));
}

// First compact slot at or after key `key`: the support keys below it.
template <typename T>
__device__ __forceinline__ uint32_t slot_at(const ColIO<T>& io, size_t key, int64_t words) {
  const size_t w = key >> 5;
  if ((int64_t)w >= words) return (uint32_t)io.kcap;
  const uint32_t s = io.wpre[w] + __popc(io.sbits[w] & ((1u << (key & 31)) - 1u));
  return s < (uint32_t)io.kcap ? s : (uint32_t)io.kcap;
}

// Column pass: one workgroup owns a strip of B = 2^LOGB adjacent columns of
// the L1 x L2 view of z and runs B length-L1 FFTs on it in LDS (column-major,
// so a global row segment of B complex values maps to B consecutive LDS
// slots).  Forward passes read a dense v-order input or build it from the
// compact CG vectors; inverse passes write a dense v-order output, a dense
// key-order output or gather the support entries back into the compact
// vectors.  In key order element e of strip g is complex slot g E + e, so the
// strip's support is one contiguous range of compact slots [s0, s1): the
// compact side touches only those entries (coalesced), never the N-bit
// bitmap.  `in` and `out` may be the same buffer in v-order modes: a
// workgroup reads its whole strip before writing it back.
template <typename T, bool INV, int LOGL1, int LOGB, int LOGE>
__device__ __forceinline__ void col_body(const Cx<T>* in, Cx<T>* out, const Plan& p, const ColIO<T>& io,
                                         const Cx<T>* __restrict__ tw, int g) {
  constexpr int E = 1 << (LOGL1 + LOGB), B = 1 << LOGB;
  constexpr int NT = nt_for(E, LOGE);
  constexpr int EPT = (E + NT - 1) / NT;
  constexpr int NW = NT / 64;
  // Inverse passes read a dense strip: each thread's loads are the inputs of
  // its first-stage butterfly, so that stage runs from registers.  (The
  // forward pass keeps its last stage in LDS: storing straight from that
  // stage's registers took as long and wrote more partial lines back from L2.)
  constexpr int LR0 = stage_lr(LOGL1, 0, LOGE);
  constexpr bool REG_IN = INV && (E >> LR0) == NT && EPT == (1 << LR0) && LOGL1 > 0;
  __shared__ double red[NW];
  extern __shared__ __align__(16) unsigned char smem_raw[];
  Cx<T>* buf = (Cx<T>*)smem_raw;
  T* bufr = (T*)smem_raw;
  const int tid = threadIdx.x;
  const size_t c0 = (size_t)g << LOGB;
  const size_t kb = (size_t)g * E;      // first key-order complex slot of the strip
  const size_t L2 = (size_t)p.L2;
  const bool compact = io.mode != COL_DENSE && io.mode != COL_KEY;
  // CG-driven passes (the compact CG passes, and the dense passes of an
  // H-apply through a DCT basis) exit once the solve has converged
  if ((io.mode == COL_DIR || io.mode == COL_Q || io.mode == COL_DENSE) && io.cg && io.cg->done) return;
  uint32_t s0 = 0, s1 = 0;
  if (compact) {
    if constexpr (E >= 16) {
      // the strip starts and ends on bitmap word boundaries: its slot range is
      // two prefix counts
      const int64_t w0 = (int64_t)((2 * kb) >> 5), w1 = (int64_t)((2 * (kb + E)) >> 5);
      s0 = w0 < p.words ? min(io.wpre[w0], (uint32_t)io.kcap) : (uint32_t)io.kcap;
      s1 = w1 < p.words ? min(io.wpre[w1], (uint32_t)io.kcap) : (uint32_t)io.kcap;
    } else {
      s0 = slot_at(io, 2 * kb, p.words);
      s1 = slot_at(io, 2 * (kb + E), p.words);
    }
  }
  // The compact side of a thread's first slot is loaded up front (key and
  // vector values together, ahead of the LDS fill or the dense loads and the
  // FFT), so its latency overlaps the rest; a strip with more slots than
  // threads takes the others in a loop afterwards.
  const uint32_t sl0 = s0 + (uint32_t)tid;
  const bool has0 = compact && sl0 < s1;
  uint32_t key0 = 0;
  T v_x = (T)0, v_r = (T)0, v_d = (T)0, v_q = (T)0, v_b = (T)0;
  const bool dir = io.mode == COL_DIR, first = io.it == 0;
  const bool upd = dir && io.fused && !first;
  // Unconditional loads (a lane without a slot reads slot 0 and ignores it):
  // a load under a condition would be waited for where the branches join,
  // before the strip's dense loads issue.
  const uint32_t slc = has0 ? sl0 : 0u;
  // inverse passes: one load per role from a pointer picked by the (uniform)
  // mode, the roles assigned after the FFT; the dense modes read the first
  // entry of the (read-only) twiddle table instead, never used
  uint32_t l_key = 0;
  T l_a = (T)0, l_r = (T)0;
  if constexpr (INV) {
    const bool qm = io.mode == COL_Q;
    const int32_t* pl = compact ? io.list : (const int32_t*)tw;
    const T* pa = compact ? (qm ? io.d : io.b) : (const T*)tw;
    const T* pr = (compact && qm && io.fused) ? io.r : pa;
    l_key = (uint32_t)pl[slc];
    l_a = pa[slc];
    l_r = pr[slc];
  }
  if (!INV && compact) {
    key0 = (uint32_t)io.list[slc];
    {
      if (dir) {
        v_r = io.r[slc];
        if (!first) v_d = io.d[slc];
        if (upd) {
          v_x = io.x[slc];
          v_q = io.q[slc];
        }
      } else {
        v_x = io.x[slc];
      }
    }
  }
  // thread tid handles e = tid + q NT: row n1 = e >> LOGB, column b = e & (B-1),
  // v-order complex element n1 L2 + c0 + b, keys 2 (kb + e) and 2 (kb + e) + 1
  if (!INV && compact) {
#pragma unroll
    for (int q = 0; q < EPT; ++q) {
      const int e = tid + q * NT;
      if (E % NT == 0 || e < E) buf[lp(e)] = cx((T)0, (T)0);
    }
    const T beta = (dir && !first) ? (T)io.cg->beta : (T)0;
    // fused: the previous iteration's x += alpha d, r -= alpha q lands here,
    // each compact slot updated by the one workgroup whose strip holds its key
    const T alpha = upd ? (T)io.cg->alpha : (T)0;
    // one slot: the new direction (and the fused update) or x
    auto slot = [&](uint32_t sl, uint32_t key, T xv, T rv, T dv, T qv) {
      const int64_t e = (int64_t)(key >> 1) - (int64_t)kb;
      if (e < 0 || e >= E) return;   // only a list shorter than kcap leaves stale entries here
      T val;
      if (dir) {
        if (upd) {
          io.x[sl] = xv + alpha * dv;
          rv = rv - alpha * qv;
          io.r[sl] = rv;
          val = rv + beta * dv;
        } else {
          val = first ? rv : rv + beta * dv;
        }
        io.d[sl] = val;
      } else {
        val = xv;
      }
      bufr[2 * lp((int)e) + (key & 1)] = val;
    };
    __syncthreads();
    if (has0) slot(sl0, key0, v_x, v_r, v_d, v_q);
    for (uint32_t sl = sl0 + NT; sl < s1; sl += NT) {
      const bool need_d = dir && !first;
      slot(sl, (uint32_t)io.list[sl], (!dir || upd) ? io.x[sl] : (T)0, dir ? io.r[sl] : (T)0,
           need_d ? io.d[sl] : (T)0, upd ? io.q[sl] : (T)0);
    }
  } else if constexpr (!REG_IN) {
#pragma unroll
    for (int q = 0; q < EPT; ++q) {
      const int e = tid + q * NT;
      if (E % NT == 0 || e < E) buf[lp(e)] = in[(size_t)(e >> LOGB) * L2 + c0 + (e & (B - 1))];
    }
  }
  if constexpr (REG_IN) {
    Cx<T> vi[1 << LR0];
#pragma unroll
    for (int q = 0; q < (1 << LR0); ++q) {
      const int e = tid + q * NT;
      vi[q] = in[(size_t)(e >> LOGB) * L2 + c0 + (e & (B - 1))];
    }
    ct_fft_cm_from_regs<T, INV, NT, LOGL1, LOGB, LOGE>(buf, tw, vi);
  } else {
    __syncthreads();
    ct_fft<T, INV, NT, LOGL1, LOGB, true, LOGE>(buf, tw);
  }
  if (INV && compact) {
    // the first slot's values are used from here on only: pin them here so
    // that no use (and no wait for their loads) moves up front
    opaque(l_key);
    opaque(l_a);
    opaque(l_r);
    const bool qm = io.mode == COL_Q;
    key0 = l_key;
    v_d = qm ? l_a : (T)0;
    v_b = qm ? (T)0 : l_a;
    v_r = (qm && io.fused) ? l_r : (T)0;
  }
  if (INV && compact && io.mode == COL_Q && io.fused) {
    // q = H d on the strip's slots with the partials of the four inner
    // products of the CG step (r is the current residual, already updated by
    // the forward pass).  No ticket: a device-scope release in every one of
    // the pass's workgroups costs more than the separate step launch that
    // reduces the partials after the kernel boundary.
    double a_dq = 0.0, a_rr = 0.0, a_rq = 0.0, a_qq = 0.0;
    auto slot = [&](uint32_t sl, uint32_t key, T dvv, T rvv) {
      const int64_t e = (int64_t)(key >> 1) - (int64_t)kb;
      if (e < 0 || e >= E) return;
      const T val = bufr[2 * lp((int)e) + (key & 1)];
      io.q[sl] = val;
      const double qv = (double)val, dv = (double)dvv, rv = (double)rvv;
      a_dq += dv * qv;
      a_rr += rv * rv;
      a_rq += rv * qv;
      a_qq += qv * qv;
    };
    if (has0) slot(sl0, key0, v_d, v_r);
    for (uint32_t sl = sl0 + NT; sl < s1; sl += NT) slot(sl, (uint32_t)io.list[sl], io.d[sl], io.r[sl]);
    const int G = (int)gridDim.x;
    __shared__ double red4[4][NW];
    // the strip's few slots sit in the first waves; the others skip the tree
    const double4 t = wg_sum4<NW>(a_dq, a_rr, a_rq, a_qq, red4, s0 + (uint32_t)(tid & ~63) < s1);
    if (tid == 0) {
      io.pout[blockIdx.x] = t.x;
      io.pout[G + blockIdx.x] = t.y;
      io.pout[2 * G + blockIdx.x] = t.z;
      io.pout[3 * G + blockIdx.x] = t.w;
    }
  } else if (INV && compact) {
    const bool qm = io.mode == COL_Q;
    double acc = 0.0;
    auto slot = [&](uint32_t sl, uint32_t key, T dv, T bv) {
      const int64_t e = (int64_t)(key >> 1) - (int64_t)kb;
      if (e < 0 || e >= E) return;
      const T val = bufr[2 * lp((int)e) + (key & 1)];
      if (qm) {
        io.q[sl] = val;
        acc += (double)dv * (double)val;
      } else {
        const T rv = bv - val;
        io.r[sl] = rv;
        io.d[sl] = rv;
        acc += (double)rv * (double)rv;
      }
    };
    if (has0) slot(sl0, key0, v_d, v_b);
    for (uint32_t sl = sl0 + NT; sl < s1; sl += NT)
      slot(sl, (uint32_t)io.list[sl], qm ? io.d[sl] : (T)0, qm ? (T)0 : io.b[sl]);
    // one partial per workgroup (d^T q or r^T r), summed by the next kernel
    const double tot = wg_sum(acc, red, NW);
    if (tid == 0) io.pout[blockIdx.x] = tot;
  } else if (INV && io.mode == COL_KEY) {
#pragma unroll
    for (int q = 0; q < EPT; ++q) {
      const int e = tid + q * NT;
      if (E % NT == 0 || e < E) out[kb + e] = buf[lp(e)];
    }
  } else {
#pragma unroll
    for (int q = 0; q < EPT; ++q) {
      const int e = tid + q * NT;
      if (E % NT == 0 || e < E) out[(size_t)(e >> LOGB) * L2 + c0 + (e & (B - 1))] = buf[lp(e)];
    }
  }
}

template <typename T, bool INV, int LOGL1, int LOGB, int LOGE>
__global__ __launch_bounds__(nt_for(1 << (LOGL1 + LOGB), LOGE)) void k_col(const Cx<T>* in, Cx<T>* out, Plan p,
                                                                           ColIO<T> io,
                                                                           const Cx<T>* __restrict__ tw) {
  col_body<T, INV, LOGL1, LOGB, LOGE>(in, out, p, io, tw, xcd_order(blockIdx.x, gridDim.x));
}

// Compact I/O of one batched signal in its current phase (mode < 0: idle).
// The per-signal state is the same for the whole workgroup: read it once
// into scalar registers and pick the two-slot members by select, so no
// per-lane copies or private arrays are made.
__device__ __forceinline__ int uniform_i32(int v) { return __builtin_amdgcn_readfirstlane(v); }

template <typename T, bool INV>
__device__ __forceinline__ ColIO<T> batch_io(const BSig<T>& s, int phase) {
  ColIO<T> io{};
  const int cur = uniform_i32(s.st->cur);
  io.sbits = s.bits;
  io.wpre = cur ? s.wpre[1] : s.wpre[0];
  io.list = cur ? s.list[1] : s.list[0];
  io.kcap = uniform_i32(s.st->k);
  io.it = uniform_i32(s.st->it);
  io.x = cur ? s.cx[1] : s.cx[0];
  io.r = s.cr;
  io.d = s.cd;
  io.q = s.cq;
  io.b = s.cb;
  io.pout = s.pgrid;
  io.cg = s.cg;            // read only in the CG modes (COL_DIR, COL_Q)
  if (!INV) io.mode = phase == BP_ITER ? COL_DIR : COL_X;
  else io.mode = phase == BP_WARM ? COL_R : (phase == BP_ITER ? COL_Q : COL_KEY);
  if (phase > BP_RESID) io.mode = -1;
  return io;
}

// Batched column pass: blockIdx.y picks the signal (ids[] of one size class).
template <typename T, bool INV, int LOGL1, int LOGB, int LOGE>
__global__ __launch_bounds__(nt_for(1 << (LOGL1 + LOGB), LOGE)) void k_col_b(const BSig<T>* __restrict__ sigs,
                                                                             const int32_t* __restrict__ ids) {
  const BSig<T>& s = sigs[uniform_i32(ids[blockIdx.y])];
  const int phase = uniform_i32(s.st->phase);
  const ColIO<T> io = batch_io<T, INV>(s, phase);
  if (io.mode < 0) return;
  col_body<T, INV, LOGL1, LOGB, LOGE>((const Cx<T>*)s.W, INV && phase == BP_RESID ? (Cx<T>*)s.Cc : s.W, s.plan, io,
                                      s.tw_col, xcd_order(blockIdx.x, gridDim.x));
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
  int sa, sb;       // LDS slots (row select * L2 + element) of self and partner
  int64_t fa, fb;   // freq-layout slots of self and partner
  int64_t k;        // bin index of self
  bool zero;        // bin 0 (self-contained)
};

__device__ __forceinline__ RowItem row_item(int t, int w, int ra, int rb, int L1, int L2) {
  RowItem it;
  int rsel, k2, rsel2, k22;
  if (w > 0) {
    rsel = 0; k2 = t; rsel2 = 1; k22 = L2 - 1 - t;
  } else if (t <= L2 / 2) {
    rsel = 0; k2 = t; rsel2 = 0; k22 = (L2 - t) & (L2 - 1);
  } else {
    const int tt = t - L2 / 2 - 1;
    rsel = 1; k2 = tt; rsel2 = 1; k22 = L2 - 1 - tt;
  }
  const int rowA = rsel ? rb : ra;
  const int rowB = rsel2 ? rb : ra;
  it.sa = rsel * L2 + k2;
  it.sb = rsel2 * L2 + k22;
  it.fa = (int64_t)rowA * L2 + k2;
  it.fb = (int64_t)rowB * L2 + k22;
  it.k = (int64_t)rowA + (int64_t)L1 * k2;
  it.zero = (it.k == 0);
  return it;
}

// W_L^{r n2} = W_4N^{8 ((r n2) mod L)}
template <typename T>
__device__ __forceinline__ Cx<T> row_tw(const Plan& p, uint32_t r, uint32_t n2) {
  return tw4n<T>(p, ((r * n2) & (uint32_t)(p.L - 1)) << 3);
}
// The same for n2 a multiple of S (a compile-time power of two): with 8 S a
// multiple of the low table's length the index has no low part, and the
// twiddle is one entry of the high table.
template <typename T, int S>
__device__ __forceinline__ Cx<T> row_tw_step(const Plan& p, uint32_t r, uint32_t n2) {
  if constexpr ((8 * S) % kTwLo == 0) {
    const uint32_t idx = ((r * n2) & (uint32_t)(p.L - 1)) << 3;
    return ((const Cx<T>*)p.tw_hi)[idx >> kTwLoLog];
  } else {
    return row_tw<T>(p, r, n2);
  }
}

// the four-step twiddles a row workgroup keeps in registers (none: formed twice)
template <typename T, int N>
struct TwKeep {
  Cx<T> v[N];
};
template <typename T>
struct TwKeep<T, 0> {};

template <typename T, int LOGL2, int LOGE, bool KEEPTW = true>
__device__ __forceinline__ void row_body(Cx<T>* __restrict__ buf, const Plan& p, int mode_rt,
                                         const T* __restrict__ fin, T* __restrict__ fout,
                                         double* __restrict__ partial, const Cx<T>* __restrict__ tw, int w) {
  const int mode = mode_rt;
  constexpr int L2 = 1 << LOGL2;
  constexpr int NT = nt_for(2 * L2, LOGE);
  constexpr bool SPLIT = NT <= L2;                 // threads tile each row exactly
  constexpr int PER_ROW = SPLIT ? L2 / NT : 1;
  extern __shared__ __align__(16) unsigned char smem_raw[];
  Cx<T>* lds = (Cx<T>*)smem_raw;
  __shared__ double red[NT / 64];
  const int L1 = p.L1;
  const int ra = w, rb = (w == 0) ? (L1 >> 1) : (L1 - w);
  const int tid = threadIdx.x;
  const T hc = (T)(0.5 * sqrt(2.0 / (double)p.n));
  const T rsn = (T)(1.0 / sqrt((double)p.n));
  const T h = (T)0.70710678118654752440;

  // four-step twiddle W_L^{r n2}: for n2 = tid + NT qq it is W_L^{r tid} W_L^{r NT qq}
  // (the second factor is the same for the whole workgroup); formed once and
  // kept in registers for the load and the store (KEEPTW), or formed again
  // for the store where registers are short (the batched pass on long rows)
  Cx<T> tb0 = cx((T)1, (T)0), tb1 = cx((T)1, (T)0);
  // Register-resident ends (the large shapes: every stage radix 16, one
  // butterfly per thread): thread tid owns row rs = tid / (L2/16) of the pair
  // and its elements j + (L2/16) r, r < 16 (j = tid mod L2/16), loaded
  // straight into the first FFT stage and stored from the last one.
  constexpr bool REGIO = RegIO<LOGL2, 1, LOGE, NT>::ok && KEEPTW;
  constexpr bool KEEP = SPLIT && KEEPTW && !REGIO;
  TwKeep<T, KEEP ? 2 * PER_ROW : 0> twk;
  constexpr int RR = 1 << LOGE, NBR = L2 >> LOGE;
  const int rs_own = REGIO ? (tid >> (LOGL2 - LOGE)) : 0;
  const int j_own = tid & (NBR - 1);
  TwKeep<T, REGIO ? RR : 0> twr;      // W_L^{row (j + NBR r)} for the thread's own elements
  Cx<T> vr[REGIO ? RR : 1];
  if constexpr (REGIO) {
    const uint32_t row = (uint32_t)(rs_own ? rb : ra);
    const Cx<T> tj = row_tw<T>(p, row, (uint32_t)j_own);
#pragma unroll
    for (int r = 0; r < RR; ++r) twr.v[r] = r ? cmul(tj, row_tw_step<T, NBR>(p, row, (uint32_t)(NBR * r))) : tj;
  }
  if (SPLIT && !REGIO) {
    tb0 = row_tw<T>(p, (uint32_t)ra, (uint32_t)tid);
    tb1 = row_tw<T>(p, (uint32_t)rb, (uint32_t)tid);
    if constexpr (KEEP) {
#pragma unroll
      for (int q = 0; q < 2 * PER_ROW; ++q) {
        const int rs = q >= PER_ROW;
        twk.v[q] = cmul(rs ? tb1 : tb0, row_tw_step<T, NT>(p, (uint32_t)(rs ? rb : ra),
                                                            (uint32_t)(NT * (q - rs * PER_ROW))));
      }
    }
  }

  // the two rows (uniform base pointers; 32-bit offsets within a row)
  Cx<T>* const rowa = buf + (size_t)ra * L2;
  Cx<T>* const rowb = buf + (size_t)rb * L2;
  if (mode != ROW_ADJ && REGIO) {
    if constexpr (REGIO) {
      const Cx<T>* __restrict__ rowp = rs_own ? rowb : rowa;
#pragma unroll
      for (int r = 0; r < RR; ++r) vr[r] = cmul(rowp[(uint32_t)(j_own + NBR * r)], twr.v[r]);
      ct_fft_from_regs<T, false, NT, LOGL2, 1, LOGE>(lds, tw, vr);
    }
  } else if (mode != ROW_ADJ) {
    if (SPLIT) {
#pragma unroll
      for (int q = 0; q < 2 * PER_ROW; ++q) {
        const int rs = q >= PER_ROW;
        const int qq = q - rs * PER_ROW;
        const uint32_t n2 = (uint32_t)(tid + NT * qq);
        const int r = rs ? rb : ra;
        Cx<T> twv;
        if constexpr (KEEP) twv = twk.v[q];
        else twv = cmul(rs ? tb1 : tb0, row_tw_step<T, NT>(p, (uint32_t)r, (uint32_t)(NT * qq)));
        lds[lp(rs * L2 + n2)] = cmul((rs ? rowb : rowa)[n2], twv);
      }
    } else {
      for (int e = tid; e < 2 * L2; e += NT) {
        const int rs = e >> LOGL2, n2 = e & (L2 - 1);
        const int r = rs ? rb : ra;
        lds[lp(rs * L2 + n2)] = cmul(buf[(size_t)r * L2 + n2], row_tw<T>(p, (uint32_t)r, (uint32_t)n2));
      }
    }
    __syncthreads();
    ct_fft<T, false, NT, LOGL2, 1, false, LOGE>(lds, tw);
  }

  // One item: self slot (LDS sa, freq-layout fa, bin k) and its partner
  // (sb, fb, bin L - k).  Returns after the store in the forward-only modes.
  double acc = 0.0;
  // wkc = (c/2) W_4N^k: the DCT scale c and the halves of E and O folded into
  // the rotation (c/2 alone for the real Fourier basis); the partner's is
  // wmc = (c/2) e^{-i pi/4} conj(W_4N^k).
  // An item's global inputs (the mask words of its two bins; y or the adjoint
  // input at them), loaded ahead of the item so their latency overlaps the
  // previous item's arithmetic.
  struct ItemIn {
    uint32_t wa, wb;
    T a0, a1, b0, b1;
  };
  auto item_in = [&](auto md_tag, uint32_t fa, uint32_t fb) {
    constexpr int MD = decltype(md_tag)::value;
    const int mode = MD >= 0 ? MD : mode_rt;
    ItemIn r{0u, 0u, (T)0, (T)0, (T)0, (T)0};
    if (mode != ROW_ADJ && mode != ROW_FWD_ALL) {
      r.wa = p.mask[fa >> 4];   // bits 2f, 2f + 1 of slot f
      r.wb = p.mask[fb >> 4];
    }
    if (mode == ROW_ADJ || mode == ROW_RESID) {
      r.a0 = fin[2u * fa]; r.a1 = fin[2u * fa + 1u];
      r.b0 = fin[2u * fb]; r.b1 = fin[2u * fb + 1u];
    }
    return r;
  };
  auto item = [&](auto md_tag, int sa, int sb, uint32_t fa, uint32_t fb, bool zero, bool self, Cx<T> wkc,
                  Cx<T> WN, const ItemIn& in) {
    constexpr int MD = decltype(md_tag)::value;   // the mode when fixed at compile time, else -1
    const int mode = MD >= 0 ? MD : mode_rt;
    T xa0, xa1, xb0, xb1;   // X_k, X_{N-k} (self slot) and X_{L-k}, X_{L+k} (partner slot)
    const Cx<T> wmc = p.fourier ? cx(hc, (T)0) : cx(h * (wkc.re - wkc.im), -h * (wkc.re + wkc.im));
    if (mode != ROW_ADJ) {
      const Cx<T> Zk = lds[sa];
      if (zero) {
        xa0 = (Zk.re + Zk.im) * rsn;
        xa1 = (Zk.re - Zk.im) * rsn;
        xb0 = xb1 = (T)0;
      } else {
        const Cx<T> Zm = lds[sb];
        // 2E = Zk + conj Zm, 2O = (Zk - conj Zm) / i; X from (c/2)-scaled rotations
        const Cx<T> E2 = Zk + conj(Zm);
        const Cx<T> D = Zk - conj(Zm);
        const Cx<T> WO2 = cmul(WN, cx(D.im, -D.re));
        const Cx<T> a = cmul(wkc, E2 + WO2), b = cmul(wmc, conj(E2 - WO2));
        xa0 = a.re; xa1 = -a.im;
        xb0 = b.re; xb1 = -b.im;
      }
    } else {
      xa0 = in.a0; xa1 = in.a1;
      xb0 = in.b0; xb1 = in.b1;
    }
    if (mode != ROW_ADJ) {
      const bool all = mode == ROW_FWD_ALL;
      const uint32_t ma = all ? 3u : (in.wa >> ((fa & 15u) * 2u)) & 3u;
      const uint32_t mb = zero ? 0u : (all ? 3u : (in.wb >> ((fb & 15u) * 2u)) & 3u);
      if (mode == ROW_RESID) {
        xa0 = in.a0 - xa0;
        xa1 = in.a1 - xa1;
        xb0 = zero ? (T)0 : in.b0 - xb0;
        xb1 = zero ? (T)0 : in.b1 - xb1;
      }
      xa0 = (ma & 1u) ? xa0 : (T)0;
      xa1 = (ma & 2u) ? xa1 : (T)0;
      xb0 = (mb & 1u) ? xb0 : (T)0;
      xb1 = (mb & 2u) ? xb1 : (T)0;
      if (mode == ROW_RESID) {
        // a self-paired bin (k = L/2) has fa == fb: count its two outputs once
        acc += (double)xa0 * xa0 + (double)xa1 * xa1;
        if (!self) acc += (double)xb0 * xb0 + (double)xb1 * xb1;
      }
      if (mode == ROW_FWD || all) {
        fout[2u * fa] = xa0; fout[2u * fa + 1u] = xa1;
        if (!zero) { fout[2u * fb] = xb0; fout[2u * fb + 1u] = xb1; }
        return;
      }
    }
    // pre-process for the inverse
    if (zero) {
      lds[sa] = cx((xa0 + xa1) * rsn, (xa0 - xa1) * rsn);
    } else {
      const Cx<T> Vk = cmulc(cx(xa0, -xa1), wkc);   // conj(wk) (Xk - i X_{N-k}) c / 2
      const Cx<T> Vm = cmulc(cx(xb0, -xb1), wmc);
      const Cx<T> E = Vk + conj(Vm);
      const Cx<T> O = cmulc(Vk - conj(Vm), WN);
      lds[sa] = cx(E.re - O.im, E.im + O.re);               // E + i O
      lds[sb] = cx(E.re + O.im, -E.im + O.re);              // conj(E) + i conj(O)
    }
  };

  if (SPLIT && w > 0) {
    // Rows w >= 1, threads tiling the row: item t = tid + NT qi pairs (ra, t)
    // with (rb, L2-1-t), bin k = ra + L1 t.  Its Makhoul twiddles are
    // W_4N^k = W_4N^{ra + L1 tid} W_4N^{L1 NT qi} and W_4N^{4k} likewise; the
    // second factors are the same for every workgroup (p.tw_step).  The two
    // modes of the CG and greedy loops get the item code with the mode fixed.
    constexpr int PER_ITEM = SPLIT ? L2 / NT : 1;
    const uint32_t k0 = (uint32_t)ra + (uint32_t)L1 * (uint32_t)tid;
    const Cx<T> kb4 = tw4n<T>(p, 4u * k0);
    // (c/2) W_4N^{k0}: the item's wkc is this times the step, no per-item scale
    const Cx<T> kb1c = p.fourier ? cx(hc, (T)0) : scale(tw4n<T>(p, k0), hc);
    const Cx<T>* __restrict__ step = (const Cx<T>*)p.tw_step;
    const uint32_t fa0 = (uint32_t)ra * L2 + (uint32_t)tid;
    const uint32_t fb0 = (uint32_t)rb * L2 + (uint32_t)(L2 - 1 - tid);
    auto items = [&](auto md_tag) {
      // software-pipelined by one item: the next item's inputs are loaded
      // (unconditionally, the last item reloading its own) before this one runs
      ItemIn cur = item_in(md_tag, fa0, fb0);
#pragma unroll 1
      for (int qi = 0; qi < PER_ITEM; ++qi) {
        const int qn = qi + 1 < PER_ITEM ? qi + 1 : qi;
        const ItemIn nxt = item_in(md_tag, fa0 + (uint32_t)(NT * qn), fb0 - (uint32_t)(NT * qn));
        // the real Fourier basis has no Makhoul rotation: wkc stays c/2
        const Cx<T> wkc = (qi && !p.fourier) ? cmul(kb1c, step[qi]) : kb1c;
        const Cx<T> WN = qi ? cmul(kb4, step[kTwStepHalf + qi]) : kb4;
        // LDS slots t and 2 L2 - 1 - t; NT qi is a multiple of 16, so the padded
        // index is a per-thread base plus an immediate
        const int dq = NT * qi + ((NT * qi) >> 4);
        item(md_tag, lp(tid) + dq, lp(2 * L2 - 1 - tid) - dq, fa0 + (uint32_t)(NT * qi),
             fb0 - (uint32_t)(NT * qi), false, false, wkc, WN, cur);
        cur = nxt;
      }
    };
    if (mode_rt == ROW_HAPPLY) items(std::integral_constant<int, ROW_HAPPLY>{});
    else if (mode_rt == ROW_RESID) items(std::integral_constant<int, ROW_RESID>{});
    else items(std::integral_constant<int, -1>{});
  } else {
    const int nitems = (w > 0) ? L2 : (L2 + 1);
    for (int t = tid; t < nitems; t += NT) {
      const RowItem it = row_item(t, w, ra, rb, L1, L2);
      Cx<T> wk = cx((T)1, (T)0), WN = cx((T)1, (T)0);
      if (!it.zero) {
        wk = tw4n<T>(p, (uint32_t)it.k);
        WN = tw4n<T>(p, (uint32_t)(4 * it.k));
        if (p.fourier) wk = cx((T)1, (T)0);
      }
      const auto md = std::integral_constant<int, -1>{};
      item(md, lp(it.sa), lp(it.sb), (uint32_t)it.fa, (uint32_t)it.fb, it.zero, !it.zero && it.fa == it.fb,
           scale(wk, hc), WN, item_in(md, (uint32_t)it.fa, (uint32_t)it.fb));
    }
  }
  if (mode == ROW_RESID) {
    for (int off = 32; off > 0; off >>= 1) acc += __shfl_down(acc, off, 64);
    if ((tid & 63) == 0) red[tid >> 6] = acc;
    __syncthreads();
    if (tid == 0) {
      double s = 0.0;
#pragma unroll
      for (int i = 0; i < NT / 64; ++i) s += red[i];
      partial[w] = s;
    }
  }
  if (mode == ROW_FWD || mode == ROW_FWD_ALL) return;
  __syncthreads();
  if constexpr (REGIO) {
    ct_fft_to_regs<T, true, NT, LOGL2, 1, LOGE>(lds, tw, vr);
    Cx<T>* __restrict__ rowp = rs_own ? rowb : rowa;
#pragma unroll
    for (int r = 0; r < RR; ++r) rowp[(uint32_t)(j_own + NBR * r)] = cmulc(vr[r], twr.v[r]);
    return;
  }
  ct_fft<T, true, NT, LOGL2, 1, false, LOGE>(lds, tw);
  if (SPLIT) {
#pragma unroll
    for (int q = 0; q < 2 * PER_ROW; ++q) {
      const int rs = q >= PER_ROW;
      const int qq = q - rs * PER_ROW;
      const int n2 = tid + NT * qq;
      const int r = rs ? rb : ra;
      Cx<T> twv;
      if constexpr (KEEP) twv = twk.v[q];
      else twv = cmul(rs ? tb1 : tb0, row_tw_step<T, NT>(p, (uint32_t)r, (uint32_t)(NT * qq)));
      (rs ? rowb : rowa)[(uint32_t)n2] = cmulc(lds[lp(rs * L2 + n2)], twv);
    }
  } else {
    for (int e = tid; e < 2 * L2; e += NT) {
      const int rs = e >> LOGL2, n2 = e & (L2 - 1);
      const int r = rs ? rb : ra;
      buf[(size_t)r * L2 + n2] = cmulc(lds[lp(rs * L2 + n2)], row_tw<T>(p, (uint32_t)r, (uint32_t)n2));
    }
  }
}

template <typename T, int LOGL2, int LOGE>
__global__ __launch_bounds__(nt_for(2 << LOGL2, LOGE)) void k_row(Cx<T>* __restrict__ buf, Plan p, int mode,
                                                            const T* __restrict__ fin, T* __restrict__ fout,
                                                            double* __restrict__ partial,
                                                            const int* __restrict__ done,
                                                            const Cx<T>* __restrict__ tw) {
  if (done && *done) return;
  row_body<T, LOGL2, LOGE>(buf, p, mode, fin, fout, partial, tw, blockIdx.x);
}

// Batched row pass: H-apply in the CG phases, residual in BP_RESID.
template <typename T, int LOGL2, int LOGE>
__global__ __launch_bounds__(nt_for(2 << LOGL2, LOGE)) void k_row_b(const BSig<T>* __restrict__ sigs,
                                                              const int32_t* __restrict__ ids) {
  const BSig<T>& s = sigs[uniform_i32(ids[blockIdx.y])];
  const int phase = uniform_i32(s.st->phase);
  if (phase > BP_RESID) return;
  const bool res = phase == BP_RESID;
  row_body<T, LOGL2, LOGE, true>(s.W, s.plan, res ? ROW_RESID : ROW_HAPPLY, res ? s.Yf : nullptr, nullptr,
                           res ? s.prow : nullptr, s.tw_row, blockIdx.x);
}

// ------------------------------------------------------------------ stage twiddle tables
// Fills the stage table of the size-2^logn FFT (layout in cs_fft.h).
template <typename T>
__global__ void k_stage_twiddles(Cx<T>* __restrict__ out, int logn, int loge) {
  const int total = tw_table_count(logn, loge);
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < total; i += gridDim.x * blockDim.x) {
    int ns = 0, off = 0;
    while (true) {
      const int lr = stage_lr(logn, ns, loge);
      const int cnt = tw_stage_count(logn, ns, loge);
      if (i < off + cnt) {
        const int R = 1 << lr;
        const int loc = i - off;
        const int k = loc / (R - 1), r = loc % (R - 1) + 1;
        // W_{NS R}^{r k} = exp(-2 pi i r k / (NS R))
        const int64_t den = (int64_t)1 << (ns + lr);
        const int64_t num = ((int64_t)r * k) % den;
        double sv, cv;
        sincospi(2.0 * (double)num / (double)den, &sv, &cv);
        out[i] = cx<T>((T)cv, (T)(-sv));
        break;
      }
      off += cnt;
      ns += lr;
    }
  }
}

// ------------------------------------------------------------------ dispatch tables
template <typename T>
struct KernelSet {
  void (*col_fwd)(const Cx<T>*, Cx<T>*, Plan, ColIO<T>, const Cx<T>*);
  void (*col_inv)(const Cx<T>*, Cx<T>*, Plan, ColIO<T>, const Cx<T>*);
  void (*row)(Cx<T>*, Plan, int, const T*, T*, double*, const int*, const Cx<T>*);
  void (*col_fwd_b)(const BSig<T>*, const int32_t*);
  void (*col_inv_b)(const BSig<T>*, const int32_t*);
  void (*row_b)(const BSig<T>*, const int32_t*);
  int nt_col, nt_row;
};

// Kernel set for L = 2^l (defined in the per-type instantiation units).
template <typename T> const KernelSet<T>& kernels_for(int l);
// Kernel set of an alternative instantiated shape, or nullptr.  With
// list_out, instead lists (up to *list_max, count returned in *list_max) the
// alternatives for the same L as s.
template <typename T>
const KernelSet<T>* kernels_alt(Shape s, Shape* list_out = nullptr, int* list_max = nullptr);

template <typename T>
inline const KernelSet<T>& kernels_plan(const Plan& p) {
  if (p.alt) return *kernels_alt<T>(Shape{p.logL1, p.logL2, p.logB, p.logE});
  return kernels_for<T>(p.logL);
}

}  // namespace csr
