// Host runtime: error state, caching device allocator, precision staging.
#include <map>
#include <mutex>
#include <unordered_map>

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

// Caching device allocator for plan buffers.  A DMRG sweep creates and destroys one
// plan per bond with similar sizes; reusing freed blocks avoids hipMalloc / hipFree
// (each of which can cost milliseconds) on every bond.  Blocks are rounded up to 1/8 of
// their power of two, kept per device, and released with hipFree beyond 24 GiB cached.
// Callers guarantee that no kernel still uses a block when it is returned.
class DevicePool {
 public:
  void* get(size_t bytes) {
    if (bytes == 0) return nullptr;
    const size_t r = round(bytes);
    int dev = 0;
    (void)hipGetDevice(&dev);
    {
      std::lock_guard<std::mutex> g(m_);
      auto& fl = free_[dev];
      auto it = fl.lower_bound(r);
      if (it != fl.end() && it->first <= r + r / 4) {
        void* p = it->second;
        cached_ -= it->first;
        fl.erase(it);
        return p;
      }
    }
    void* p = nullptr;
    if (hipMalloc(&p, r) != hipSuccess) {
      (void)hipGetLastError();
      trim(0);
      if (hipMalloc(&p, r) != hipSuccess) {
        (void)hipGetLastError();
        throw DmError{DM_ERR_ALLOC, "hipMalloc of " + std::to_string(r) + " bytes failed"};
      }
    }
    std::lock_guard<std::mutex> g(m_);
    size_[p] = {r, dev};
    return p;
  }
  void put(void* p) {
    if (!p) return;
    std::lock_guard<std::mutex> g(m_);
    auto it = size_.find(p);
    if (it == size_.end()) return;
    free_[it->second.second].emplace(it->second.first, p);
    cached_ += it->second.first;
    if (cached_ > kMaxCached) trim_locked(kMaxCached);
  }

 private:
  static constexpr size_t kMaxCached = size_t(24) << 30;
  static size_t round(size_t b) {
    if (b <= (size_t(1) << 20)) return (b + 4095) & ~size_t(4095);
    size_t top = size_t(1) << (63 - __builtin_clzll(b));
    const size_t step = top / 8;
    return (b + step - 1) / step * step;
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
        (void)hipFree(last->second);
        size_.erase(last->second);
        cached_ -= last->first;
        fl.erase(last);
      }
    }
  }
  std::mutex m_;
  std::map<int, std::multimap<size_t, void*>> free_;
  std::unordered_map<void*, std::pair<size_t, int>> size_;
  size_t cached_ = 0;
};

DevicePool& pool() {
  static DevicePool* p = new DevicePool();  // never destroyed: outlives static teardown
  return *p;
}

}  // namespace

void* dev_alloc(size_t bytes) { return pool().get(bytes); }
void dev_free(void* p) { pool().put(p); }

size_t elem_bytes(int prec) { return prec == DM_FP64 ? 16 : 8; }

void check_prec(int prec) {
  if (prec != DM_FP64 && prec != DM_FP32 && prec != DM_BF16X3)
    throw DmError{DM_ERR_DTYPE, "precision " + std::to_string(prec) + " not supported"};
}

void check_ly(int ly) {
  if (ly < 1) throw DmError{DM_ERR_ARG, "ly must be >= 1"};
}

void stage_in(const void* src, void* dst, int64_t n, int prec, hipStream_t s) {
  if (n == 0) return;
  if (prec == DM_FP64)
    HIPCHK(hipMemcpyAsync(dst, src, (size_t)n * 16, hipMemcpyDeviceToDevice, s));
  else
    HIPCHK(launch_cast_d2f((const double*)src, (float*)dst, 2 * n, s));
}
void stage_out(const void* src, void* dst, int64_t n, int prec, hipStream_t s) {
  if (n == 0) return;
  if (prec == DM_FP64)
    HIPCHK(hipMemcpyAsync(dst, src, (size_t)n * 16, hipMemcpyDeviceToDevice, s));
  else
    HIPCHK(launch_cast_f2d((const float*)src, (double*)dst, 2 * n, s));
}

hipError_t gemm_lp(int prec, const GemmStage& st, const float* A, const float* B, float* C,
                   float* part, hipStream_t s, const int32_t* skip,
                   const std::function<void()>& between) {
  if (prec == DM_BF16X3) return launch_gemm_bf16x3(st, A, B, C, part, s, skip, between);
  return launch_gemm<float>(st, A, B, C, part, s, skip, between);
}

}  // namespace mrd

extern "C" const char* dm_last_error(void) { return mrd::g_err.c_str(); }
