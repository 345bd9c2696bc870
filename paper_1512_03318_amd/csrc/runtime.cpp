// Host runtime: error state, caching device allocator, precision staging.
#include <map>
#include <mutex>
#include <unordered_map>
#include <vector>

#include "runtime.hpp"

namespace mrd {

namespace {
thread_local std::string g_err;
}

int fail(int code, const std::string& msg) {
  g_err = msg;
  return code;
}

void set_last_error(const std::string& msg) { g_err = msg; }

namespace {

// Caching allocator for plan buffers (device) and upload staging (pinned host).  A DMRG
// sweep creates and destroys one plan per bond with similar sizes; reusing freed blocks
// avoids hipMalloc / hipFree (each of which can cost milliseconds) on every bond.
// Blocks are rounded up to 1/8 of their power of two, kept per device, and released
// beyond 24 GiB cached.  A block is returned either when no kernel uses it any more
// (put) or at a point of a stream (put_after): it is then reused only once an event
// recorded there has completed, so stream-ordered work never needs a host wait.
class BlockPool {
 public:
  explicit BlockPool(bool pinned) : pinned_(pinned) {}
  void* get(size_t bytes) {
    if (bytes == 0) return nullptr;
    const size_t r = round(bytes);
    int dev = 0;
    if (!pinned_) (void)hipGetDevice(&dev);
    {
      std::lock_guard<std::mutex> g(m_);
      reap_locked();
      auto& fl = free_[dev];
      auto it = fl.lower_bound(r);
      if (it != fl.end() && it->first <= r + r / 4) {
        void* p = it->second;
        cached_ -= it->first;
        fl.erase(it);
        return p;
      }
    }
    void* p = raw_alloc(r);
    if (!p) {
      trim(0);
      p = raw_alloc(r);
      if (!p)
        throw DmError{DM_ERR_ALLOC, std::string(pinned_ ? "hipHostMalloc" : "hipMalloc") + " of " +
                                        std::to_string(r) + " bytes failed"};
    }
    std::lock_guard<std::mutex> g(m_);
    size_[p] = {r, dev};
    return p;
  }
  void put(void* p) {
    if (!p) return;
    std::lock_guard<std::mutex> g(m_);
    put_locked(p);
    reap_locked();
  }
  void put_after(void* p, hipStream_t s) {
    if (!p) return;
    std::lock_guard<std::mutex> g(m_);
    hipEvent_t e = nullptr;
    if (!events_.empty()) {
      e = events_.back();
      events_.pop_back();
    } else if (hipEventCreateWithFlags(&e, hipEventDisableTiming) != hipSuccess) {
      (void)hipGetLastError();
      (void)hipStreamSynchronize(s);  // no event: wait here instead
      put_locked(p);
      return;
    }
    if (hipEventRecord(e, s) != hipSuccess) {
      (void)hipGetLastError();
      (void)hipStreamSynchronize(s);
      events_.push_back(e);
      put_locked(p);
      return;
    }
    pending_.push_back({e, p});
  }

 private:
  static constexpr size_t kMaxCached = size_t(24) << 30;
  static size_t round(size_t b) {
    if (b <= (size_t(1) << 20)) return (b + 4095) & ~size_t(4095);
    size_t top = size_t(1) << (63 - __builtin_clzll(b));
    const size_t step = top / 8;
    return (b + step - 1) / step * step;
  }
  void* raw_alloc(size_t r) {
    void* p = nullptr;
    const hipError_t e = pinned_ ? hipHostMalloc(&p, r, hipHostMallocDefault) : hipMalloc(&p, r);
    if (e != hipSuccess) {
      (void)hipGetLastError();
      return nullptr;
    }
    return p;
  }
  void raw_free(void* p) {
    if (pinned_) (void)hipHostFree(p);
    else (void)hipFree(p);
  }
  void put_locked(void* p) {
    auto it = size_.find(p);
    if (it == size_.end()) return;
    free_[it->second.second].emplace(it->second.first, p);
    cached_ += it->second.first;
    if (cached_ > kMaxCached) trim_locked(kMaxCached);
  }
  // blocks whose release point has been reached become free
  void reap_locked() {
    for (size_t i = 0; i < pending_.size();) {
      const hipError_t q = hipEventQuery(pending_[i].first);
      if (q == hipErrorNotReady) {
        ++i;
        continue;
      }
      if (q != hipSuccess) (void)hipGetLastError();
      events_.push_back(pending_[i].first);
      put_locked(pending_[i].second);
      pending_[i] = pending_.back();
      pending_.pop_back();
    }
  }
  void trim(size_t limit) {
    std::lock_guard<std::mutex> g(m_);
    trim_locked(limit);
  }
  void trim_locked(size_t limit) {
    for (auto& kv : free_) {
      auto& fl = kv.second;
      while (cached_ > limit && !fl.empty()) {
        auto last = std::prev(fl.end());
        raw_free(last->second);
        size_.erase(last->second);
        cached_ -= last->first;
        fl.erase(last);
      }
    }
  }
  const bool pinned_;
  std::mutex m_;
  std::map<int, std::multimap<size_t, void*>> free_;
  std::unordered_map<void*, std::pair<size_t, int>> size_;
  std::vector<std::pair<hipEvent_t, void*>> pending_;
  std::vector<hipEvent_t> events_;
  size_t cached_ = 0;
};

BlockPool& pool() {
  static BlockPool* p = new BlockPool(false);  // never destroyed: outlives static teardown
  return *p;
}
BlockPool& pinned_pool() {
  static BlockPool* p = new BlockPool(true);
  return *p;
}

}  // namespace

void* dev_alloc(size_t bytes) { return pool().get(bytes); }
void dev_free(void* p) { pool().put(p); }
void dev_free_after(void* p, hipStream_t s) { pool().put_after(p, s); }
void* pinned_alloc(size_t bytes) { return pinned_pool().get(bytes); }
void pinned_free_after(void* p, hipStream_t s) { pinned_pool().put_after(p, s); }
void pinned_free(void* p) { pinned_pool().put(p); }

namespace {
std::mutex g_ev_mu;
std::vector<std::pair<int, std::array<hipEvent_t, 5>>> g_ev_pool;  // (device, events)
}  // namespace

std::array<hipEvent_t, 5> timing_events_get() {
  int dev = 0;
  HIPCHK(hipGetDevice(&dev));
  {
    std::lock_guard<std::mutex> g(g_ev_mu);
    for (size_t i = g_ev_pool.size(); i-- > 0;)
      if (g_ev_pool[i].first == dev) {
        const std::array<hipEvent_t, 5> e = g_ev_pool[i].second;
        g_ev_pool.erase(g_ev_pool.begin() + (std::ptrdiff_t)i);
        return e;
      }
  }
  std::array<hipEvent_t, 5> e{};
  for (auto& x : e) HIPCHK(hipEventCreate(&x));
  return e;
}

void timing_events_put(const std::array<hipEvent_t, 5>& e) {
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) {  // no device context: release them instead
    for (hipEvent_t x : e) (void)hipEventDestroy(x);
    return;
  }
  std::lock_guard<std::mutex> g(g_ev_mu);
  g_ev_pool.push_back({dev, e});
}

size_t elem_bytes(int prec, bool real) { return (prec == DM_FP64 ? 16 : 8) / (real ? 2 : 1); }

bool take_real(int32_t& prec) {
  const bool real = (prec & DM_REAL) != 0;
  prec &= ~DM_REAL;
  return real;
}

void check_prec(int prec) {
  if (prec != DM_FP64 && prec != DM_FP32 && prec != DM_BF16X3)
    throw DmError{DM_ERR_DTYPE, "precision " + std::to_string(prec) + " not supported"};
}

void check_ly(int ly) {
  if (ly < 1) throw DmError{DM_ERR_ARG, "ly must be >= 1"};
}

void stage_in(const void* src, void* dst, int64_t n, int prec, hipStream_t s, bool real) {
  if (n == 0) return;
  const int64_t nr = real ? n : 2 * n;  // real values
  if (prec == DM_FP64)
    HIPCHK(hipMemcpyAsync(dst, src, (size_t)nr * 8, hipMemcpyDeviceToDevice, s));
  else
    HIPCHK(launch_cast_d2f((const double*)src, (float*)dst, nr, s));
}
void stage_out(const void* src, void* dst, int64_t n, int prec, hipStream_t s, bool real) {
  if (n == 0) return;
  const int64_t nr = real ? n : 2 * n;
  if (prec == DM_FP64)
    HIPCHK(hipMemcpyAsync(dst, src, (size_t)nr * 8, hipMemcpyDeviceToDevice, s));
  else
    HIPCHK(launch_cast_f2d((const float*)src, (double*)dst, nr, s));
}

hipError_t gemm_lp(int prec, const GemmStage& st, const float* A, const float* B, float* C,
                   float* part, hipStream_t s, const int32_t* skip,
                   const std::function<void()>& between) {
  if (prec == DM_BF16X3) return launch_gemm_bf16x3(st, A, B, C, part, s, skip, between);
  return launch_gemm<float>(st, A, B, C, part, s, skip, between);
}

}  // namespace mrd

extern "C" const char* dm_last_error(void) { return mrd::g_err.c_str(); }
