// Batched Subspace Pursuit: independent signals recovered concurrently.
//
// Each signal runs the single-signal SP driver (the same kernels and decision
// rules as cs_recover_sp) on its own slice of the caller's workspace.  The
// driver's loop control reads a few device words per step, so one signal
// leaves the GPU idle between its small launches; several signals in flight,
// each on its own stream and host thread, fill those gaps.  The threads and
// streams form a per-process pool per device, created on the first batched
// call and kept until the process ends (each worker keeps its pinned host
// mailbox too), so a call creates nothing but one event.
#include "cs_internal.h"

#include <algorithm>
#include <atomic>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <functional>
#include <memory>
#include <mutex>
#include <string>
#include <thread>
#include <vector>

namespace csr {

namespace {

struct DevicePool {
  int device = 0;
  std::mutex mu;
  std::condition_variable cv;
  std::deque<std::function<void(hipStream_t, hipError_t)>> jobs;
  std::vector<std::thread> threads;
  std::vector<hipStream_t> streams;
};

constexpr int kMaxPoolDevices = 64;
std::mutex g_pools_mu;
DevicePool* g_pools[kMaxPoolDevices];

int pool_width() {
  const unsigned hc = std::thread::hardware_concurrency();
  return (int)std::max(2u, std::min(16u, hc ? hc / 2 : 8u));
}

void worker(DevicePool* p, int w) {
  const hipError_t dev_err = hipSetDevice(p->device);   // reported by every job this worker takes
  for (;;) {
    std::function<void(hipStream_t, hipError_t)> job;
    {
      std::unique_lock<std::mutex> lk(p->mu);
      p->cv.wait(lk, [&] { return !p->jobs.empty(); });
      job = std::move(p->jobs.front());
      p->jobs.pop_front();
    }
    job(p->streams[w], dev_err);
  }
}

DevicePool* pool_for_current_device() {
  int dev = 0;
  CS_HIP(hipGetDevice(&dev));
  if (dev < 0 || dev >= kMaxPoolDevices) throw Error(CS_E_HIP, "device ordinal out of range for the worker pool");
  std::lock_guard<std::mutex> lk(g_pools_mu);
  if (!g_pools[dev]) {
    auto* p = new DevicePool();   // lives until the process ends (its threads never exit)
    p->device = dev;
    const int w = pool_width();
    for (int i = 0; i < w; ++i) {
      hipStream_t s = nullptr;
      CS_HIP(hipStreamCreateWithFlags(&s, hipStreamNonBlocking));   // default priority
      p->streams.push_back(s);
    }
    for (int i = 0; i < w; ++i) {
      p->threads.emplace_back(worker, p, i);
      p->threads.back().detach();
    }
    g_pools[dev] = p;
  }
  return g_pools[dev];
}

}  // namespace

size_t batch_layout_algo(cs_dtype dt, int count, const cs_batch_item* items, cs_algo algo,
                         std::vector<size_t>* offs) {
  size_t off = 0;
  for (int i = 0; i < count; ++i) {
    const size_t sz = workspace_bytes(dt, items[i].op.n, items[i].op.m, items[i].k, algo, items[i].op.psi);
    if (sz == 0) return 0;
    off = (off + 255) / 256 * 256;
    if (offs) offs->push_back(off);
    off += sz;
  }
  return (off + 255) / 256 * 256;
}

void recover_batched_pool(cs_algo algo, cs_dtype dt, int count, const cs_batch_item* items, double tol,
                          const cs_params* params, void* ws, size_t ws_bytes, cs_info* infos, hipStream_t stream,
                          void (*one)(cs_algo, cs_dtype, const void*, const cs_op*, int32_t, double, void*,
                                      int32_t*, const cs_params*, void*, size_t, cs_info*, hipStream_t)) {
  std::vector<size_t> offs;
  const size_t need = batch_layout_algo(dt, count, items, algo, &offs);
  if (need == 0) throw Error(CS_E_SHAPE, "unsupported size in batch");
  if (ws_bytes < need) throw Error(CS_E_WORKSPACE, "workspace too small: need " + std::to_string(need) + " bytes");
  DevicePool* p = pool_for_current_device();
  // the signals' inputs may come from work queued on the caller's stream
  hipEvent_t ready = nullptr;
  CS_HIP(hipEventCreateWithFlags(&ready, hipEventDisableTiming));
  CS_HIP(hipEventRecord(ready, stream));
  struct Shared {
    std::mutex mu;
    std::condition_variable cv;
    int left = 0;
    cs_status first = CS_OK;
    std::string msg;
  } sh;
  sh.left = count;
  std::vector<cs_info> loc(count);
  // largest signals first, so the pool ends on short ones
  std::vector<int> order(count);
  for (int i = 0; i < count; ++i) order[i] = i;
  std::stable_sort(order.begin(), order.end(), [&](int a, int b) {
    return items[a].op.n * (int64_t)items[a].k > items[b].op.n * (int64_t)items[b].k;
  });
  {
    std::lock_guard<std::mutex> lk(p->mu);
    for (int i : order) {
      p->jobs.emplace_back([&, i](hipStream_t s, hipError_t dev_err) {
        cs_status st = CS_OK;
        std::string m;
        try {
          CS_HIP(dev_err);
          CS_HIP(hipStreamWaitEvent(s, ready, 0));
          const cs_batch_item& it = items[i];
          one(algo, dt, it.y, &it.op, it.k, tol, it.s, it.support, params, (char*)ws + offs[i],
              (i + 1 < count ? offs[i + 1] : need) - offs[i], &loc[i], s);
        } catch (const Error& e) {
          st = e.status;
          m = e.what();
        } catch (const std::exception& e) {
          st = CS_E_HIP;
          m = e.what();
        }
        std::lock_guard<std::mutex> lk2(sh.mu);
        if (st != CS_OK && sh.first == CS_OK) {
          sh.first = st;
          sh.msg = "signal " + std::to_string(i) + ": " + m;
        }
        if (--sh.left == 0) sh.cv.notify_all();
      });
    }
  }
  p->cv.notify_all();
  {
    std::unique_lock<std::mutex> lk(sh.mu);
    sh.cv.wait(lk, [&] { return sh.left == 0; });
  }
  (void)hipEventDestroy(ready);
  if (sh.first != CS_OK) throw Error(sh.first, sh.msg);
  if (infos) std::memcpy(infos, loc.data(), count * sizeof(cs_info));
}

}  // namespace csr
