// Batched Lanczos over many independent effective Hamiltonians.
//
// The task tables of all plans are merged into one table per phase, so every phase of
// one Lanczos step (casts, L.theta GEMMs, MPO mixing, (.).R GEMMs, K-split reduction,
// the Lanczos vector kernels) is one launch over all instances: 14 launches per step
// whatever the batch size.  Offsets of the merged tables are rebased to one base
// address (the lowest buffer of the batch), so the kernels of the single-plan path run
// unchanged.  Merged GEMM tiles are ordered longest first (LPT list scheduling: the
// hardware dispatcher hands workgroups out in index order as compute units free up),
// interleaved over the eight XCDs so that every XCD receives its own longest-first
// list.  The instances run in lock step; each instance stops on its own rule (its
// remaining vector launches become no-ops) and its stop time is read from the device
// wall clock.
#include <sys/stat.h>
#include <unistd.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <fstream>
#include <map>
#include <memory>
#include <numeric>
#include <string>

#include "runtime.hpp"

using namespace mrd;

namespace {

// Host copy of the device XCD mapping of the GEMM kernels: block b runs tile xcd_tile(b).
int xcd_tile_host(int b, int n) {
  const int q = n >> 3, r = n & 7, x = b & 7;
  return x * q + std::min(x, r) + (b >> 3);
}

struct Shift {
  int64_t a = 0, b = 0, c = 0;  // complex elements, added to A, B and C offsets
};

// Work of one tile in staged K chunks (the kernel's run time is set by its K loop).
double tile_cost(const GemmStage& st, const GemmTile& t) {
  const GemmProb& p = st.probs[t.prob];
  double chunks = 0;
  for (int g = 0; g < p.nseg; ++g) chunks += (st.segs[p.seg0 + g].k + st.kc - 1) / st.kc;
  return chunks / std::max(1, p.nks);
}

// Concatenates the problems of all plans (offsets rebased); tiles are built per bucket.
GemmStage merge_problems(const std::vector<const GemmStage*>& in, const std::vector<Shift>& sh) {
  // merged stages work on the batch's FP32 staging copies of theta (cast for all
  // instances in one launch), so the FP64 output flag of the plans' own stages is dropped
  constexpr int32_t f64 = G_C_F64;
  GemmStage m;
  m.flags = in[0]->flags & ~f64;
  for (size_t i = 0; i < in.size(); ++i) {
    const GemmStage& st = *in[i];
    if ((st.flags & ~f64) != m.flags) throw DmError{DM_ERR_ARG, "batched plans have different stage kinds"};
    const int32_t seg0 = (int32_t)m.segs.size();
    const int32_t row0 = (int32_t)m.rows.size();
    for (GemmSeg g : st.segs) {
      g.a_off += sh[i].a;
      g.b_off += sh[i].b;
      m.segs.push_back(g);
    }
    for (int64_t r : st.rows) m.rows.push_back((m.flags & G_C_ROWMAP) ? r + sh[i].c : r);
    for (GemmProb p : st.probs) {
      if (!(m.flags & G_C_ROWMAP)) p.c_off += sh[i].c;
      p.seg0 += seg0;
      if (p.rowmap >= 0) p.rowmap += row0;
      m.probs.push_back(p);
    }
    m.flops += st.flops;
  }
  if (m.segs.size() > INT32_MAX || m.rows.size() > INT32_MAX)
    throw DmError{DM_ERR_ARG, "batched task table too large"};
  return m;
}

// Workgroup tile shape of a GEMM stage (the fields add_tiles and the launchers read).
struct Shape {
  int tm, tn;
  bool deep, split;
  int kc, split_min;
};

void set_shape(GemmStage& st, const Shape& sh) {
  st.tile_m = sh.tm;
  st.tile_n = sh.tn;
  st.deep = sh.deep;
  st.split = sh.split;
  st.kc = sh.kc;
  st.split_min = sh.split_min;
}

// Shapes the kernels provide for a stage (see launch_gemm / launch_gemm_bf16x3).
std::vector<Shape> candidates(int prec, int32_t flags) {
  const bool long_k = flags == (G_B_T | G_C_ROWMAP);
  if (prec == DM_BF16X3) {
    if (long_k)
      return {{128, 32, false, true, 32, 12}, {128, 32, false, true, 32, 6}, {64, 32, false, true, 32, 6},
              {64, 64, false, true, 32, 6}};
    return {{128, 64, false, false, 32, 4}, {64, 64, false, false, 32, 4}};
  }
  if (long_k) return {{32, 32, true, true, 64, 4}, {64, 64, false, false, 32, 4}};
  return {{64, 64, false, false, 32, 4}, {32, 32, true, false, 64, 4}};
}

// Problem buckets by output shape: rows (<= 64, > 64) x columns (<= 32, <= 64, > 64).
int bucket_of(const GemmProb& p) { return (p.M > 64 ? 3 : 0) + (p.N > 64 ? 2 : p.N > 32 ? 1 : 0); }
constexpr int kBuckets = 6;

// Tiles of the problems in `which` with shape sh, longest first (LPT), interleaved so
// that block b -- dispatched to XCD b % 8 -- starts the b-th longest tile.
void tile_bucket(GemmStage& st, const std::vector<int>& which, const Shape& sh) {
  set_shape(st, sh);
  st.tiles.clear();
  st.red_tiles.clear();
  st.nslots = 0;
  for (GemmProb& p : st.probs) {
    p.nks = 1;
    p.slot0 = -1;
  }
  for (int i : which) add_tiles(st, i, st.probs[i].M, st.probs[i].N);
  std::vector<std::pair<double, GemmTile>> tl;
  for (const GemmTile& t : st.tiles) tl.emplace_back(tile_cost(st, t), t);
  std::stable_sort(tl.begin(), tl.end(), [](const auto& x, const auto& y) { return x.first > y.first; });
  const int n = (int)tl.size();
  for (int b = 0; b < n; ++b) st.tiles[xcd_tile_host(b, n)] = tl[b].second;
  double f = 0;
  for (int i : which) {
    const GemmProb& p = st.probs[i];
    for (int q = 0; q < p.nseg; ++q) f += 8.0 * p.M * p.N * st.segs[p.seg0 + q].k;
  }
  st.flops = f;
}

// Mixing tasks are short and memory-bound: they keep each plan's own order (tasks that
// share source blocks are adjacent, and the kernel hands each XCD a contiguous run).
MixStage merge_mix(const std::vector<const MixStage*>& in, const std::vector<Shift>& sh) {
  MixStage m;
  for (size_t i = 0; i < in.size(); ++i) {
    const int32_t src0 = (int32_t)m.srcs.size();
    for (MixSrc s : in[i]->srcs) {
      s.off += sh[i].a;
      m.srcs.push_back(s);
    }
    for (MixTask t : in[i]->tasks) {
      t.dst += sh[i].c;
      t.src0 += src0;
      m.tasks.push_back(t);
    }
    m.flops += in[i]->flops;
  }
  // slab forms, if every plan has one of the same element size
  bool slabs = true;
  for (const MixStage* x : in) slabs = slabs && !x->wgs.empty() && x->slab_eb == in[0]->slab_eb;
  if (slabs) {
    m.slab_eb = in[0]->slab_eb;
    for (size_t i = 0; i < in.size(); ++i) {
      const int32_t b0 = (int32_t)m.blks.size(), t0 = (int32_t)m.stasks.size(), c0 = (int32_t)m.coefs.size();
      for (SlabBlk b : in[i]->blks) {
        b.off += sh[i].a;
        m.blks.push_back(b);
      }
      for (SlabTask t : in[i]->stasks) {
        t.dst += sh[i].c;
        t.c0 += c0;
        m.stasks.push_back(t);
      }
      m.coefs.insert(m.coefs.end(), in[i]->coefs.begin(), in[i]->coefs.end());
      for (SlabWG g : in[i]->wgs) {
        g.blk0 += b0;
        g.task0 += t0;
        m.wgs.push_back(g);
      }
      m.lds_bytes = std::max(m.lds_bytes, in[i]->lds_bytes);
    }
  }
  return m;
}

// One merged matvec: theta (per instance) -> w, all instances in one launch per phase.
struct MergedMatvec {
  std::vector<GemmStage> s1, s4;  // one stage per problem bucket, each with its tuned shape
  MixStage mix;
  char* base = nullptr;  // every offset counts elements from here
  void* split = nullptr; // K-split partial tiles (buckets run in stream order and share it)
  int prec = DM_FP64;
  std::vector<std::string> tuning;  // chosen shape per bucket, for reports
};

// Rebasing: offsets of instance i move by (buffer_i - base) / element size.
struct Rebase {
  size_t eb;
  char* base = nullptr;
  void note(const void* p) {
    if (p && (!base || (char*)p < base)) base = (char*)p;
  }
  int64_t shift(const void* p) const {
    if (!p) return 0;
    const ptrdiff_t d = (char*)p - base;
    if (d % (ptrdiff_t)eb) throw DmError{DM_ERR_ARG, "misaligned buffer in batch"};
    return (int64_t)(d / (ptrdiff_t)eb);
  }
};

}  // namespace

struct dm_batch {
  std::vector<dm_heff_plan*> plans;
  int prec = DM_FP64;
  bool built = false;
  MergedMatvec mv, mv64;        // mv64: FP64 matvec of the final Rayleigh quotient
  std::vector<CastJob> cout;    // FP32 results of each instance to its FP64 w
  int32_t cout_blocks = 0;
  CastJob* d_cout = nullptr;
  void* dTables = nullptr;
  int lz_cap = 0;               // max_iter the instance table is laid out for
  LzInst* dInst = nullptr;
  LzInst* hInst = nullptr;      // pinned
  LzGrid lzg;
  LzResult* dRes = nullptr;
  LzResult* hRes = nullptr;     // pinned
  hipEvent_t done = nullptr;
  hipGraph_t graph = nullptr;   // one batched Lanczos step (opt-in, as for single plans)
  hipGraphExec_t graph_exec = nullptr;
  hipStream_t cap_stream = nullptr;
  bool use_graph = false;
  bool tune = true;             // tile shape per problem bucket timed at the first solve
  ~dm_batch() {
    if (done) {
      (void)hipEventSynchronize(done);
      (void)hipEventDestroy(done);
    }
    if (graph_exec) (void)hipGraphExecDestroy(graph_exec);
    if (graph) (void)hipGraphDestroy(graph);
    if (cap_stream) (void)hipStreamDestroy(cap_stream);
    dev_free(dTables);
    dev_free(mv.split);
    dev_free(mv64.split);
    dev_free(dInst);
    dev_free(dRes);
    if (hInst) (void)hipHostFree(hInst);
    if (hRes) (void)hipHostFree(hRes);
  }
};

namespace {

// Merged tables of the step matvec (f64 = false) or of the FP64 Rayleigh quotient.
// Device time (ms, best of 3 after one warm-up) of one bucket stage on the batch's buffers.
double time_stage(GemmStage& t, int prec, char* base, size_t eb, hipStream_t s) {
  TableUpload up;
  up.add(t);
  void* tab = up.commit(s);
  void* part = dev_alloc((size_t)t.nslots * t.slot_elems() * eb);
  hipEvent_t e0 = nullptr, e1 = nullptr;
  double best = 1e30;
  try {
    HIPCHK(hipEventCreate(&e0));
    HIPCHK(hipEventCreate(&e1));
    for (int r = 0; r < 4; ++r) {
      HIPCHK(hipEventRecord(e0, s));
      if (prec == DM_FP64)
        HIPCHK(launch_gemm<double>(t, (double*)base, (double*)base, (double*)base, (double*)part, s));
      else
        HIPCHK(gemm_lp(prec, t, (float*)base, (float*)base, (float*)base, (float*)part, s));
      HIPCHK(hipEventRecord(e1, s));
      HIPCHK(hipEventSynchronize(e1));
      float ms = 0;
      HIPCHK(hipEventElapsedTime(&ms, e0, e1));
      if (r > 0) best = std::min(best, (double)ms);
    }
  } catch (...) {
    if (e0) (void)hipEventDestroy(e0);
    if (e1) (void)hipEventDestroy(e1);
    dev_free_after(tab, s);
    dev_free_after(part, s);
    throw;
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  dev_free(tab);   // the stream was synchronised above
  dev_free(part);
  return best;
}

// ---------------------------------------------------------------------------------
// Tile shapes chosen by timing are kept in a small text file, one line per key
//   <gfx arch> <precision> <stage flags> <bucket> <work class>  <candidate index>
// (work class: log2 of the bucket's algorithmic GFLOP, rounded), so later batches of the
// same kind skip the timing.  File: $MRDMRG_TUNE_CACHE, else $XDG_CACHE_HOME/mrdmrg/
// tile_shapes.txt, else ~/.cache/mrdmrg/tile_shapes.txt; MRDMRG_TUNE_CACHE=0 turns it
// off.  Written whole to a temporary file and renamed over the old one.
// ---------------------------------------------------------------------------------
std::string cache_path() {
  const char* e = getenv("MRDMRG_TUNE_CACHE");
  if (e && e[0] == '0' && e[1] == 0) return "";
  if (e && e[0]) return e;
  const char* x = getenv("XDG_CACHE_HOME");
  if (x && x[0]) return std::string(x) + "/mrdmrg/tile_shapes.txt";
  const char* h = getenv("HOME");
  if (h && h[0]) return std::string(h) + "/.cache/mrdmrg/tile_shapes.txt";
  return "";
}

std::map<std::string, int> cache_read(const std::string& path) {
  std::map<std::string, int> out;
  if (path.empty()) return out;
  std::ifstream f(path);
  std::string line;
  while (std::getline(f, line)) {
    const size_t cut = line.rfind(' ');
    if (cut == std::string::npos || cut == 0) continue;
    try {
      out[line.substr(0, cut)] = std::stoi(line.substr(cut + 1));
    } catch (const std::exception&) {  // a damaged line is ignored
    }
  }
  return out;
}

void cache_write(const std::string& path, const std::map<std::string, int>& add) {
  if (path.empty() || add.empty()) return;
  std::map<std::string, int> all = cache_read(path);
  for (const auto& kv : add) all[kv.first] = kv.second;
  const size_t slash = path.rfind('/');
  if (slash != std::string::npos) {
    std::string dir = path.substr(0, slash);
    for (size_t i = 1; i <= dir.size(); ++i)
      if (i == dir.size() || dir[i] == '/') (void)mkdir(dir.substr(0, i).c_str(), 0755);
  }
  const std::string tmp = path + ".tmp" + std::to_string((long)getpid());
  {
    std::ofstream f(tmp);
    if (!f) return;  // an unwritable cache only costs the timing next time
    for (const auto& kv : all) f << kv.first << ' ' << kv.second << '\n';
    if (!f) return;
  }
  (void)std::rename(tmp.c_str(), path.c_str());
}

std::string arch_name() {
  int dev = 0;
  hipDeviceProp_t p;
  if (hipGetDevice(&dev) != hipSuccess || hipGetDeviceProperties(&p, dev) != hipSuccess) return "unknown";
  std::string a = p.gcnArchName;
  const size_t colon = a.find(':');
  return colon == std::string::npos ? a : a.substr(0, colon);
}

// One stage per problem bucket; with tune, each bucket takes the fastest candidate shape
// (timed on the batch's own buffers, or read from the cache of earlier timings),
// otherwise the plans' default shape.
std::vector<GemmStage> tune_stage(const GemmStage& base, int prec, const Shape& dflt, bool tune,
                                  char* ptr, size_t eb, hipStream_t s, std::vector<std::string>& log) {
  std::vector<std::vector<int>> which(kBuckets);
  for (int i = 0; i < (int)base.probs.size(); ++i) which[bucket_of(base.probs[i])].push_back(i);
  const std::vector<Shape> cand = candidates(prec, base.flags);
  const std::string path = tune ? cache_path() : std::string();
  const std::map<std::string, int> cached = cache_read(path);
  std::map<std::string, int> learned;
  const std::string arch = tune ? arch_name() : std::string();
  std::vector<GemmStage> out;
  for (int bk = 0; bk < kBuckets; ++bk) {
    if (which[bk].empty()) continue;
    Shape best = dflt;
    bool from_cache = false;
    if (tune && cand.size() > 1) {
      double gf = 0;
      for (int i : which[bk]) {
        const GemmProb& p = base.probs[i];
        for (int q = 0; q < p.nseg; ++q) gf += 8.0 * p.M * p.N * base.segs[p.seg0 + q].k;
      }
      const int wclass = (int)std::lround(std::log2(std::max(gf * 1e-9, 1e-6)));
      const std::string key = arch + " " + std::to_string(prec) + " " + std::to_string(base.flags) + " " +
                              std::to_string(bk) + " " + std::to_string(wclass);
      auto it = cached.find(key);
      if (it != cached.end() && it->second >= 0 && it->second < (int)cand.size()) {
        best = cand[it->second];
        from_cache = true;
      } else {
        double tbest = 1e30;
        int ibest = 0;
        for (size_t ci = 0; ci < cand.size(); ++ci) {
          GemmStage t = base;
          tile_bucket(t, which[bk], cand[ci]);
          const double ms = time_stage(t, prec, ptr, eb, s);
          if (ms < tbest) {
            tbest = ms;
            best = cand[ci];
            ibest = (int)ci;
          }
        }
        learned[key] = ibest;
      }
    }
    GemmStage t = base;
    tile_bucket(t, which[bk], best);
    log.push_back("flags " + std::to_string(base.flags) + " bucket " + std::to_string(bk) + ": " +
                  std::to_string(which[bk].size()) + " problems, " + std::to_string(best.tm) + "x" +
                  std::to_string(best.tn) + (best.deep ? " deep" : "") + (best.split ? " split" : "") +
                  (from_cache ? " (cached)" : ""));
    out.push_back(std::move(t));
  }
  cache_write(path, learned);
  return out;
}

Shape shape_of(const GemmStage& st) {
  return {st.tile_m, st.tile_n, st.deep, st.split, st.kc, st.split_min};
}

// Merged tables of the step matvec (f64 = false) or of the FP64 Rayleigh quotient.
MergedMatvec build_merged(dm_batch& b, bool f64, hipStream_t s) {
  MergedMatvec m;
  m.prec = f64 ? DM_FP64 : b.prec;
  const bool low = m.prec != DM_FP64;
  Rebase rb{low ? size_t(8) : size_t(16)};
  struct Bufs {
    void *L, *R, *X, *Z, *in, *out;
  };
  std::vector<Bufs> bufs;
  for (dm_heff_plan* p : b.plans) {
    Bufs q;
    if (!low && b.prec != DM_FP64) {  // FP64 matvec of a low-precision plan
      q = {p->dL64, p->dR64, p->dX64, p->dZ64, p->dVcur, p->dW};
    } else if (!low) {
      q = {p->dL, p->dR, p->dX, p->dZ, p->dVcur, p->dW};
    } else {
      q = {p->dL, p->dR, p->dX, p->dZ, p->dTin, p->dTout};
    }
    for (void* x : {q.L, q.R, q.X, q.Z, q.in, q.out}) rb.note(x);
    bufs.push_back(q);
  }
  std::vector<const GemmStage*> s1, s4;
  std::vector<const MixStage*> mx;
  std::vector<Shift> sh1, sh4, shm;
  for (size_t i = 0; i < b.plans.size(); ++i) {
    const Bufs& q = bufs[i];
    s1.push_back(f64 ? &b.plans[i]->rq_s1() : &b.plans[i]->s1);
    s4.push_back(f64 ? &b.plans[i]->rq_s4() : &b.plans[i]->s4);
    mx.push_back(&b.plans[i]->mix);
    sh1.push_back({rb.shift(q.L), rb.shift(q.in), rb.shift(q.X)});
    shm.push_back({rb.shift(q.X), 0, rb.shift(q.Z)});
    sh4.push_back({rb.shift(q.Z), rb.shift(q.R), rb.shift(q.out)});
  }
  m.base = rb.base;
  // the once-per-solve FP64 Rayleigh-quotient matvec keeps the plans' shapes untuned
  const bool tune = b.tune && !f64;
  m.s1 = tune_stage(merge_problems(s1, sh1), m.prec, shape_of(*s1[0]), tune, m.base, rb.eb, s, m.tuning);
  m.mix = merge_mix(mx, shm);
  m.s4 = tune_stage(merge_problems(s4, sh4), m.prec, shape_of(*s4[0]), tune, m.base, rb.eb, s, m.tuning);
  size_t split = 0;
  for (const GemmStage& t : m.s4) split = std::max(split, (size_t)t.nslots * t.slot_elems() * rb.eb);
  m.split = dev_alloc(split);
  return m;
}

void run_merged(const MergedMatvec& m, hipStream_t s) {
  if (m.prec == DM_FP64) {
    double* base = (double*)m.base;
    for (const GemmStage& t : m.s1) HIPCHK(launch_gemm<double>(t, base, base, base, nullptr, s));
    HIPCHK(launch_mix<double>(m.mix, base, base, s));
    for (const GemmStage& t : m.s4) HIPCHK(launch_gemm<double>(t, base, base, base, (double*)m.split, s));
  } else {
    float* base = (float*)m.base;
    for (const GemmStage& t : m.s1) HIPCHK(gemm_lp(m.prec, t, base, base, base, nullptr, s));
    HIPCHK(launch_mix<float>(m.mix, base, base, s));
    for (const GemmStage& t : m.s4) HIPCHK(gemm_lp(m.prec, t, base, base, base, (float*)m.split, s));
  }
}

void build_batch(dm_batch& b, hipStream_t s) {
  b.mv = build_merged(b, false, s);
  if (b.prec != DM_FP64) {
    b.mv64 = build_merged(b, true, s);
    for (dm_heff_plan* p : b.plans) {
      b.cout.push_back({p->dTout, p->dW, 2 * p->n(), 0, 0});
    }
    b.cout_blocks = cast_layout(b.cout);
  }
  TableUpload up;
  for (MergedMatvec* m : {&b.mv, &b.mv64}) {
    for (GemmStage& t : m->s1) up.add(t);
    for (GemmStage& t : m->s4) up.add(t);
    up.add(m->mix);
  }
  up.add(b.cout, &b.d_cout);
  b.dTables = up.commit(s);
  b.built = true;
}

// One batched Lanczos step; nv_bound as for lz_launch_step_tail (step index + 1, or 0
// for the captured step).  The FP32 inputs of an FP32 / BF16x3 batch were written by
// the Lanczos kernels that produced v_j.
void batch_step(dm_batch& b, hipStream_t s, int32_t nv_bound) {
  run_merged(b.mv, s);
  if (b.prec != DM_FP64)
    HIPCHK(launch_cast_batch(false, b.d_cout, (int32_t)b.cout.size(), b.cout_blocks, s));
  HIPCHK(lz_launch_step_tail(b.dInst, b.lzg, nv_bound, s));
}

}  // namespace

extern "C" int dm_batch_create(int32_t n, dm_heff_plan* const* plans, dm_stream stream,
                               dm_batch** out) {
  (void)stream;
  return guarded([&] {
    if (!out || n <= 0 || !plans) throw DmError{DM_ERR_ARG, "dm_batch_create: bad arguments"};
    *out = nullptr;
    auto b = std::make_unique<dm_batch>();
    b->plans.assign(plans, plans + n);
    for (dm_heff_plan* p : b->plans) {
      if (!p) throw DmError{DM_ERR_ARG, "dm_batch_create: null plan"};
      if (p->n() == 0) throw DmError{DM_ERR_LAYOUT, "dm_batch_create: empty theta"};
      if (p->real) throw DmError{DM_ERR_ARG, "dm_batch_create: real (DM_REAL) plans are solved one by one"};
    }
    for (int i = 0; i < n; ++i)
      for (int j = 0; j < i; ++j)
        if (b->plans[i] == b->plans[j]) throw DmError{DM_ERR_ARG, "dm_batch_create: plan repeated"};
    b->prec = b->plans[0]->prec;
    for (dm_heff_plan* p : b->plans)
      if (p->prec != b->prec) throw DmError{DM_ERR_DTYPE, "dm_batch_create: plans differ in precision"};
    HIPCHK(hipEventCreateWithFlags(&b->done, hipEventDisableTiming));
    const char* g = getenv("MRDMRG_GRAPH");
    b->use_graph = g && g[0] == '1';
    const char* t = getenv("MRDMRG_TUNE");  // "0": keep the plans' tile shapes
    b->tune = !(t && t[0] == '0');
    *out = b.release();
  });
}

extern "C" void dm_batch_destroy(dm_batch* b) { delete b; }

extern "C" int64_t dm_batch_info(const dm_batch* b, char* buf, int64_t len) {
  if (!b) return 0;
  std::string t;
  for (const std::string& l : b->mv.tuning) t += l + "\n";
  if (buf && len > 0) {
    const int64_t n = std::min<int64_t>(len - 1, (int64_t)t.size());
    std::memcpy(buf, t.data(), (size_t)n);
    buf[n] = 0;
  }
  return (int64_t)t.size() + 1;
}

static int lanczos_ground_batched_impl(dm_batch* b, void* const* thetas, int32_t max_iter,
                                       double tol, double* energies, int32_t* iters,
                                       double* done_us, dm_stream stream);

extern "C" int lanczos_ground_batched(dm_batch* b, void* const* thetas, int32_t max_iter,
                                      double tol, double* energies, int32_t* iters,
                                      double* done_us, dm_stream stream) {
  // as lanczos_ground: an error returns only once the queued work has drained
  const int rc = lanczos_ground_batched_impl(b, thetas, max_iter, tol, energies, iters, done_us, stream);
  if (rc != DM_OK && b) drain(stream);
  return rc;
}

static int lanczos_ground_batched_impl(dm_batch* b, void* const* thetas, int32_t max_iter,
                                       double tol, double* energies, int32_t* iters,
                                       double* done_us, dm_stream stream) {
  return guarded([&] {
    if (!b || !thetas || !energies || !iters) throw DmError{DM_ERR_ARG, "null argument"};
    if (max_iter < 1 || max_iter > LZ_MAX) throw DmError{DM_ERR_ARG, "max_iter must be in 1..64"};
    const int n = (int)b->plans.size();
    for (int i = 0; i < n; ++i)
      if (!thetas[i]) throw DmError{DM_ERR_ARG, "null theta"};
      else if (misaligned(thetas[i])) throw DmError{DM_ERR_ARG, "theta must be 16-byte aligned"};
    hipStream_t s = (hipStream_t)stream;
    for (dm_heff_plan* p : b->plans) ensure_lanczos(p, max_iter);
    if (!b->built) build_batch(*b, s);
    if (b->lz_cap != max_iter) {
      if (b->graph_exec) (void)hipGraphExecDestroy(b->graph_exec);
      if (b->graph) (void)hipGraphDestroy(b->graph);
      b->graph_exec = nullptr;
      b->graph = nullptr;
      dev_free(b->dInst);
      dev_free(b->dRes);
      if (b->hInst) (void)hipHostFree(b->hInst);
      if (b->hRes) (void)hipHostFree(b->hRes);
      b->dInst = nullptr;
      b->dRes = nullptr;
      b->hInst = nullptr;
      b->hRes = nullptr;
      b->dInst = (LzInst*)dev_alloc(n * sizeof(LzInst));
      b->dRes = (LzResult*)dev_alloc(n * sizeof(LzResult));
      HIPCHK(hipHostMalloc((void**)&b->hInst, n * sizeof(LzInst), hipHostMallocDefault));
      HIPCHK(hipHostMalloc((void**)&b->hRes, n * sizeof(LzResult), hipHostMallocDefault));
      b->lz_cap = max_iter;
    }
    // the instance table is rebuilt every solve: Krylov buffers may have been regrown by
    // single-plan solves in between, and the start vectors change
    std::vector<LzInst> I(n);
    for (int i = 0; i < n; ++i) {
      dm_heff_plan* p = b->plans[i];
      I[i] = LzInst{p->dV, p->dW, p->dVcur, p->dPart, nullptr, (double*)thetas[i], p->dState,
                    p->n(), p->n()};
      I[i].tin = b->prec == DM_FP64 ? nullptr : (float*)p->dTin;
      I[i].xn = 2 * p->n();  // complex instances (real plans are not batched)
      I[i].real = 0;
    }
    LzGrid g = lz_layout(I, max_iter);
    g.vf32 = b->prec != DM_FP64;
    const bool same = b->graph_exec && std::equal(I.begin(), I.end(), b->hInst, [](const LzInst& x, const LzInst& y) {
      return x.V == y.V && x.w == y.w && x.vcur == y.vcur && x.part == y.part && x.st == y.st;
    });
    if (!same && b->graph_exec) {
      (void)hipGraphExecDestroy(b->graph_exec);
      (void)hipGraphDestroy(b->graph);
      b->graph_exec = nullptr;
      b->graph = nullptr;
    }
    std::copy(I.begin(), I.end(), b->hInst);  // previous solve synchronised: buffer free
    b->lzg = g;
    HIPCHK(hipMemcpyAsync(b->dInst, b->hInst, n * sizeof(LzInst), hipMemcpyHostToDevice, s));
    HIPCHK(lz_launch_init(b->dInst, b->lzg, max_iter, tol, s));
    HIPCHK(lz_launch_start(b->dInst, b->lzg, s));
    if (b->use_graph && !b->graph_exec) {
      if (!b->cap_stream) HIPCHK(hipStreamCreateWithFlags(&b->cap_stream, hipStreamNonBlocking));
      HIPCHK(hipStreamBeginCapture(b->cap_stream, hipStreamCaptureModeThreadLocal));
      try {
        batch_step(*b, b->cap_stream, 0);
      } catch (...) {
        hipGraph_t gr = nullptr;
        (void)hipStreamEndCapture(b->cap_stream, &gr);
        if (gr) (void)hipGraphDestroy(gr);
        throw;
      }
      HIPCHK(hipStreamEndCapture(b->cap_stream, &b->graph));
      HIPCHK(hipGraphInstantiate(&b->graph_exec, b->graph, nullptr, nullptr, 0));
    }
    for (int j = 0; j < max_iter; ++j) {
      if (b->use_graph)
        HIPCHK(hipGraphLaunch(b->graph_exec, s));
      else
        batch_step(*b, s, j + 1);
    }
    HIPCHK(lz_launch_finish(b->dInst, b->lzg, s));
    if (b->prec != DM_FP64) {
      run_merged(b->mv64, s);  // FP64 H vcur -> w for every instance
      HIPCHK(lz_launch_rq(b->dInst, b->lzg, s));
    }
    HIPCHK(lz_launch_results(b->dInst, b->lzg, b->dRes, s));
    HIPCHK(hipMemcpyAsync(b->hRes, b->dRes, n * sizeof(LzResult), hipMemcpyDeviceToHost, s));
    HIPCHK(hipEventRecord(b->done, s));
    for (dm_heff_plan* p : b->plans) HIPCHK(hipEventRecord(p->done, s));
    HIPCHK(hipStreamSynchronize(s));
    int rate_khz = 0;
    int dev = 0;
    HIPCHK(hipGetDevice(&dev));
    HIPCHK(hipDeviceGetAttribute(&rate_khz, hipDeviceAttributeWallClockRate, dev));
    bool bad = false;
    for (int i = 0; i < n; ++i) {
      const LzResult& r = b->hRes[i];
      energies[i] = r.energy;
      iters[i] = r.k;
      bad = bad || r.bad;
      if (done_us)
        done_us[i] = rate_khz > 0 ? (double)(r.t1 - r.t0) * 1e3 / rate_khz : 0.0;
    }
    if (bad) throw DmError{DM_ERR_NONFINITE, "Lanczos produced a zero, NaN or Inf norm"};
  });
}
