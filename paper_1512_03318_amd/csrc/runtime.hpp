// Host runtime shared by the plan, Lanczos, environment and batch entry points:
// error handling, the caching device allocator, task-table uploads, precision staging
// and the effective-Hamiltonian plan object.
#pragma once

#include <array>
#include <cstdint>
#include <cstring>
#include <functional>
#include <future>
#include <string>
#include <system_error>
#include <vector>

#include "plan.hpp"

namespace mrd {

// Sets the thread-local message of dm_last_error() and returns code.
int fail(int code, const std::string& msg);

#define HIPCHK(expr)                                                                    \
  do {                                                                                  \
    hipError_t e_ = (expr);                                                             \
    if (e_ != hipSuccess)                                                               \
      throw ::mrd::DmError{DM_ERR_HIP, std::string(#expr) + ": " + hipGetErrorString(e_)}; \
  } while (0)

// Runs f, turning exceptions into error codes (no exception crosses the C ABI).
template <typename F>
int guarded(F&& f) {
  try {
    f();
    return DM_OK;
  } catch (const DmError& e) {
    return fail(e.code, e.msg);
  } catch (const std::bad_alloc&) {
    return fail(DM_ERR_ALLOC, "host allocation failed");
  } catch (const std::exception& e) {
    return fail(DM_ERR_ARG, e.what());
  }
}

// Runs f on a second thread, or later on the caller (at get()) when no thread can be
// started; the result and any exception come back through get().
template <class F>
std::future<void> run_beside(const F& f) {
  try {
    return std::async(std::launch::async, f);
  } catch (const std::system_error&) {
    return std::async(std::launch::deferred, f);
  }
}

// Waits for the work queued on a stream (errors ignored): called before an error
// leaves an entry point that had queued work, so none of it is still running when the
// caller reacts to the error.
inline void drain(dm_stream s) {
  if (hipStreamSynchronize((hipStream_t)s) != hipSuccess) (void)hipGetLastError();
}

// Complex FP64 vectors are read and written as 16-byte elements.
inline bool misaligned(const void* p) { return reinterpret_cast<uintptr_t>(p) % 16 != 0; }

// Caching allocators (runtime.cpp): blocks are reused across plans.  dev_free: no
// kernel uses the block any more; dev_free_after: reusable once stream s has passed
// this point (no host wait).  Pinned host blocks stage uploads.
void* dev_alloc(size_t bytes);
void dev_free(void* p);
void dev_free_after(void* p, hipStream_t s);
void* pinned_alloc(size_t bytes);
void pinned_free_after(void* p, hipStream_t s);
void pinned_free(void* p);  // no copy uses the block any more
// Timing events of the stage profiling (five per recorded matvec), reused across plans on
// the current device: a plan per bond update would otherwise create and destroy them on
// every bond.  put: every recorded event of the set has completed.
std::array<hipEvent_t, 5> timing_events_get();
void timing_events_put(const std::array<hipEvent_t, 5>& e);

// All task tables of one or more stages in one device block, uploaded with one copy.
struct TableUpload {
  struct Part {
    const void* src;
    size_t bytes, off;
    void** dst;
  };
  std::vector<Part> parts;
  size_t total = 0;
  template <typename T>
  void add(const std::vector<T>& v, T** dst) {
    *dst = nullptr;
    if (v.empty()) return;
    const size_t off = (total + 255) & ~size_t(255);
    parts.push_back({v.data(), v.size() * sizeof(T), off, (void**)dst});
    total = off + v.size() * sizeof(T);
  }
  void add(GemmStage& st) {
    add(st.segs, &st.d_segs);
    add(st.probs, &st.d_probs);
    add(st.tiles, &st.d_tiles);
    add(st.rows, &st.d_rows);
    add(st.red_tiles, &st.d_red_tiles);
  }
  void add(PsStage& st) {
    add(st.probs, &st.d_probs);
    add(st.tiles, &st.d_tiles);
    add(st.rows, &st.d_rows);
    add(st.red_tiles, &st.d_red_tiles);
    add(st.sk_tiles, &st.d_sk_tiles);
    add(st.sk_segs, &st.d_sk_segs);
    add(st.sk_jobs, &st.d_sk_jobs);
    add(st.sk_wg, &st.d_sk_wg);
    add(st.sk_red, &st.d_sk_red);
  }
  void add(MixStage& st) {
    add(st.tasks, &st.d_tasks);
    add(st.srcs, &st.d_srcs);
    add(st.wgs, &st.d_wgs);
    add(st.blks, &st.d_blks);
    add(st.stasks, &st.d_stasks);
    add(st.coefs, &st.d_coefs);
  }
  // Stream-ordered upload into a pool block: the host tables (which must stay unchanged
  // until commit) are copied straight into pinned staging, released after the copy on s;
  // returns the block (free it with dev_free / dev_free_after).
  void* commit(hipStream_t s) {
    if (parts.empty()) return nullptr;
    char* h = (char*)pinned_alloc(total);
    for (const Part& p : parts) std::memcpy(h + p.off, p.src, p.bytes);
    char* d = (char*)dev_alloc(total);
    const hipError_t e = hipMemcpyAsync(d, h, total, hipMemcpyHostToDevice, s);
    pinned_free_after(h, s);
    if (e != hipSuccess) {
      dev_free_after(d, s);
      HIPCHK(e);
    }
    for (const Part& p : parts) *p.dst = d + p.off;
    return d;
  }
  // Upload into a device block d of at least `total` bytes that the caller provides, from
  // pageable host memory (no pinned staging block): the copy has consumed the host
  // bytes when hipMemcpyAsync returns, and is ordered on s.
  void commit_pageable(void* dv, hipStream_t s) {
    if (parts.empty()) return;
    char* d = static_cast<char*>(dv);
    std::vector<char> h(total);
    for (const Part& p : parts) std::memcpy(h.data() + p.off, p.src, p.bytes);
    HIPCHK(hipMemcpyAsync(d, h.data(), total, hipMemcpyHostToDevice, s));
    for (const Part& p : parts) *p.dst = d + p.off;
  }
};

size_t elem_bytes(int prec, bool real = false);
void check_prec(int prec);
// Splits the DM_REAL bit off a precision argument (real: the eq. rot formulation, FP64
// or FP32 only).
bool take_real(int32_t& prec);
void check_ly(int ly);
// Copy (FP64) or cast (FP32 storage) n complex elements from a complex128 buffer, and back.
// n elements (complex, or real values when real is set) from FP64 into the precision's
// storage, and back
void stage_in(const void* src, void* dst, int64_t n, int prec, hipStream_t s, bool real = false);
void stage_out(const void* src, void* dst, int64_t n, int prec, hipStream_t s, bool real = false);
// FP32-storage GEMM stage: FP32 MFMA (DM_FP32) or bf16 hi/lo split MFMA (DM_BF16X3).
hipError_t gemm_lp(int prec, const GemmStage& st, const float* A, const float* B, float* C,
                   float* part, hipStream_t s, const int32_t* skip = nullptr,
                   const std::function<void()>& between = std::function<void()>());

}  // namespace mrd

// =====================================================================================
// Effective Hamiltonian plan
// =====================================================================================
struct dm_heff_plan {
  int ly = 1, prec = DM_FP64;
  mrd::Bond a, c;
  mrd::MpoSite w1, w2;
  mrd::ThetaLayout th;
  mrd::EnvLLayout L;
  mrd::EnvRLayout R;
  std::vector<int64_t> xoff;  // per a: X panel offset (rows = L.P.rows[a], cols = th.P.cols[a])
  std::vector<int> xld;       // per a: X panel leading dimension (cols rounded up to 16)
  int64_t xtotal = 0;
  mrd::GemmStage s1, s4;
  mrd::GemmStage s1f, s4f;  // DM_BF16X3: the stages in FP kernel shapes (FP64 Rayleigh quotient)
  const mrd::GemmStage& rq_s1() const { return prec == DM_BF16X3 ? s1f : s1; }
  const mrd::GemmStage& rq_s4() const { return prec == DM_BF16X3 ? s4f : s4; }
  mrd::MixStage mix;
  // DM_BF16X3 matvec on pre-split operands (bf16 planes): stages, the mixing that writes
  // Z split, the split jobs of L, R (plan creation) and theta (every matvec), and the
  // plane offsets (bf16 elements) per ket sector a (L, theta^T) and output sector c' (Z, R)
  mrd::PsStage s1p, s4p;
  mrd::MixStage mixp;
  std::vector<mrd::SplitJob> lsplit, rsplit, thsplit;
  mrd::SplitJob* d_lsplit = nullptr;
  mrd::SplitJob* d_rsplit = nullptr;
  mrd::SplitJob* d_thsplit = nullptr;
  int64_t lsplit_items = 0, rsplit_items = 0, thsplit_items = 0;
  std::vector<int64_t> lsoff, thsoff, zsoff, rsoff;
  std::vector<int32_t> zkp;  // padded K of each Z / R panel
  int64_t ls_total = 0, ths_total = 0, zs_total = 0, rs_total = 0;
  void* dLs = nullptr;
  void* dRs = nullptr;
  void* dThs = nullptr;
  void* dZs = nullptr;
  void* dSplitP = nullptr;  // K-split partial tiles of the pre-split (.).R stage
  bool real = false;        // real operands (eq. rot): FP64 or FP32
  bool presplit = false;    // BF16x3 matvec on the pre-split operands
  bool streamk = false;     // ... through the stream-K kernels
  int ncu = 1;              // compute units of the plan's device
  // the Lanczos kernels write an FP32 copy of v_j that the matvec reads
  bool staged_in() const { return prec == DM_FP32 || (prec == DM_BF16X3 && !presplit); }
  void* dTables = nullptr;      // all task tables (one pool block)
  hipEvent_t done = nullptr;    // recorded after every use; waited on before release
  double mix_flops = 0;
  std::vector<int64_t> zoff;  // per c': Z panel offset (rows zrows[c'], cols R.P.cols[c'])
  std::vector<int> zld;       // per c': Z panel leading dimension (cols rounded up to 16)
  std::vector<int> zrows;
  int64_t ztotal = 0;
  void* dZ = nullptr;
  void* dZ64 = nullptr;
  // device buffers (elements in the plan's precision)
  void* dL = nullptr;
  void* dR = nullptr;
  void* dL64 = nullptr;  // FP64 copies for the final Rayleigh quotient (low precision plans)
  void* dR64 = nullptr;
  void* dX = nullptr;
  void* dX64 = nullptr;
  void* dSplit = nullptr;    // K-split partial tiles of the (.)R stage
  void* dSplit64 = nullptr;
  void* dTin = nullptr;  // low-precision staging of theta in / out
  void* dTout = nullptr;
  // Lanczos workspace (FP64)
  double* dV = nullptr;       // Krylov basis, Vcap vectors of n
  int Vcap = 0;
  double* dW = nullptr;       // H v_j
  double* dVcur = nullptr;    // v_j (fixed address: the matvec input of every step)
  double* dPart = nullptr;    // per-block partial sums
  mrd::LzState* dState = nullptr;
  mrd::LzInst* dInst = nullptr;    // this plan as a one-instance Lanczos table
  mrd::LzInst* hInst = nullptr;    // pinned host copy (start vector pointer set per solve)
  mrd::LzGrid lzg;
  mrd::LzResult* dRes = nullptr;
  mrd::LzResult* hRes = nullptr;   // pinned
  hipGraph_t graph = nullptr; // one Lanczos step (matvec + projections), captured once
  hipGraphExec_t graph_exec = nullptr;
  hipStream_t cap_stream = nullptr;
  bool use_graph = true;
  // profiling: events around the three stages of each recorded matvec
  bool profiling = false;
  int32_t prof_stride = 1;  // record every prof_stride-th matvec
  int64_t prof_seen = 0;    // matvecs since profiling was enabled
  std::vector<std::array<hipEvent_t, 5>> ev;
  size_t ev_used = 0;
  ~dm_heff_plan() {
    if (done) {
      (void)hipEventSynchronize(done);  // no kernel of this plan may still run
      (void)hipEventDestroy(done);
    }
    for (auto& e : ev) mrd::timing_events_put(e);  // complete: `done` has been waited for
    mrd::dev_free(dTables);
    for (void* p : {dL, dR, dL64, dR64, dX, dX64, dSplit, dSplit64, dTin, dTout, dZ, dZ64, dLs, dRs, dThs, dZs,
                    dSplitP})
      mrd::dev_free(p);
    if (graph_exec) (void)hipGraphExecDestroy(graph_exec);
    if (graph) (void)hipGraphDestroy(graph);
    if (cap_stream) (void)hipStreamDestroy(cap_stream);
    for (double* p : {dV, dW, dVcur, dPart}) mrd::dev_free(p);
    mrd::dev_free(dState);
    mrd::dev_free(dInst);
    mrd::dev_free(dRes);
    mrd::pinned_free(hInst);  // the solves that copied them have synchronised
    mrd::pinned_free(hRes);
  }
  int64_t n() const { return th.P.total; }
  // complex elements of the Lanczos vectors (a real vector of n values is read as
  // ceil(n / 2) complex elements, the last one padded with a zero)
  int64_t nlz() const { return real ? (th.P.total + 1) / 2 : th.P.total; }
  // real values in theta (FP64 / FP32 casts)
  int64_t nreal() const { return real ? th.P.total : 2 * th.P.total; }
};


namespace mrd {
// theta_out = H_eff theta in the plan's precision (FP64 in / out); force64 uses the
// FP64 copies of L and R.  skip (may be null): device flag that turns the launches into
// no-ops.  capturing: no profiling events (inside HIP graph capture).  staged: an FP32 /
// BF16x3 plan's FP32 copy of theta is already in its input buffer (written by the
// Lanczos kernels that produced theta), so no cast is launched.
void heff_run(dm_heff_plan* p, const void* theta, void* theta_out, hipStream_t s, bool force64,
              const int32_t* skip = nullptr, bool capturing = false, bool staged = false);
// Lanczos workspace of a plan for up to max_iter steps.
void ensure_lanczos(dm_heff_plan* p, int max_iter);
}  // namespace mrd
