// C ABI: layouts, effective-Hamiltonian plans, matvec, Lanczos and environment updates.
#include <algorithm>
#include <cstdlib>
#include <map>
#include <mutex>
#include <cmath>
#include <cstring>
#include <future>
#include <system_error>
#include <memory>
#include <sstream>

#include "runtime.hpp"

using namespace mrd;

static int lanczos_ground_impl(dm_heff_plan* p, void* theta_inout, int32_t max_iter, double tol,
                               double* energy, int32_t* iters, dm_stream stream);
namespace {
void check_real_mix(const MixStage& m);
}

// =====================================================================================
// Layout query
// =====================================================================================
extern "C" int dm_layout(const dm_layout_desc* d, int64_t* nblocks, int64_t* nelem,
                         dm_block* blocks) {
  return guarded([&] {
    if (!d || !nblocks || !nelem) throw DmError{DM_ERR_ARG, "null argument"};
    check_ly(d->ly);
    std::vector<dm_block> out;
    int64_t total = 0;
    switch (d->kind) {
      case DM_LAYOUT_SITE: {
        Bond a = make_bond(d->x, d->ly), b = make_bond(d->y, d->ly);
        SiteLayout L = site_layout(a, b, d->qs1, d->ly);
        for (int i = 0; i < a.size(); ++i)
          for (int s = 0; s < 2; ++s)
            if (L.b[i][s] >= 0)
              out.push_back({{i, s, L.b[i][s]}, a.dim[i], b.dim[L.b[i][s]],
                             L.P.off[i] + L.coff[i][s], L.P.cols[i]});
        total = L.P.total;
        break;
      }
      case DM_LAYOUT_THETA: {
        Bond a = make_bond(d->x, d->ly), c = make_bond(d->y, d->ly);
        ThetaLayout L = theta_layout(a, c, d->qs1, d->qs2, d->ly);
        for (int i = 0; i < a.size(); ++i)
          for (int s = 0; s < 4; ++s)
            if (L.c[i][s] >= 0)
              out.push_back({{i, s, L.c[i][s]}, a.dim[i], c.dim[L.c[i][s]],
                             L.P.off[i] + L.coff[i][s], L.P.cols[i]});
        total = L.P.total;
        break;
      }
      case DM_LAYOUT_ENV_L:
      case DM_LAYOUT_ENV_R: {
        Bond a = make_bond(d->x, d->ly);
        if (d->nw <= 0 || !d->qw) throw DmError{DM_ERR_ARG, "environment layout needs MPO charges"};
        std::vector<dm_charge> qw(d->qw, d->qw + d->nw);
        for (auto& q : qw)
          if (q.k < 0 || q.k >= d->ly) throw DmError{DM_ERR_CHARGE, "MPO charge k outside [0, ly)"};
        if (d->kind == DM_LAYOUT_ENV_L) {
          EnvLLayout L = envl_layout(a, qw, d->ly);
          for (int i = 0; i < a.size(); ++i)
            for (int w = 0; w < L.D; ++w) {
              const int j = L.ap[i * L.D + w];
              if (j < 0) continue;
              out.push_back({{j, w, i}, a.dim[j], a.dim[i],
                             L.P.off[i] + (int64_t)L.roff[i * L.D + w] * a.dim[i], a.dim[i]});
            }
          total = L.P.total;
        } else {
          EnvRLayout L = envr_layout(a, qw, d->ly);
          for (int i = 0; i < a.size(); ++i)
            for (int w = 0; w < L.D; ++w) {
              const int j = L.c[i * L.D + w];
              if (j < 0) continue;
              out.push_back({{i, w, j}, a.dim[i], a.dim[j], L.P.off[i] + L.coff[i * L.D + w],
                             L.P.cols[i]});
            }
          total = L.P.total;
        }
        break;
      }
      default:
        throw DmError{DM_ERR_ARG, "unknown layout kind"};
    }
    if (blocks) std::copy(out.begin(), out.end(), blocks);
    *nblocks = (int64_t)out.size();
    *nelem = total;
  });
}

// =====================================================================================
// Effective Hamiltonian plan
// =====================================================================================
static void build_heff_tables(dm_heff_plan& p) {
  const int ly = p.ly;
  const Bond &a = p.a, &c = p.c;
  const int dl = p.w1.dl, dm = p.w1.dr, dr = p.w2.dr;
  // X panels.  Rows of X and Z start on 128-byte boundaries (leading dimensions rounded
  // up to 16 complex elements): a store of a row segment then covers whole cache lines
  // instead of straddling two.
  auto ld16 = [](int n) { return (n + 15) / 16 * 16; };
  p.xoff.assign(a.size(), 0);
  p.xld.assign(a.size(), 0);
  p.xtotal = 0;
  for (int i = 0; i < a.size(); ++i) {
    p.xoff[i] = p.xtotal;
    p.xld[i] = ld16(p.th.P.cols[i]);
    p.xtotal += (int64_t)p.L.P.rows[i] * p.xld[i];
  }
  // zap[c'][s12'] = a' with theta block (a', s12', c'), or -1
  std::vector<std::array<int, 4>> zap(c.size(), {-1, -1, -1, -1});
  for (int ci = 0; ci < c.size(); ++ci)
    for (int s12 = 0; s12 < 4; ++s12) {
      dm_charge qa = qsub(qsub(c.q[ci], p.w1.qs[s12 >> 1], ly), p.w2.qs[s12 & 1], ly);
      const int ai = a.find(qa);
      if (ai >= 0 && p.th.c[ai][s12] == ci) zap[ci][s12] = ai;
    }
  // S1: X_a = Lpanel_a (M_a x m_a) . Theta_a (m_a x N_a)
  auto build_s1 = [&](GemmStage& s1, bool bf3) {
    s1.flags = 0;
    if (bf3) {
      // 128 x 64 tiles for the bf16 matrix cores, or 64 x 64 when that leaves fewer than
      // two tiles per CU (small windows: more workgroups; at Ly=6, chi=800 L.theta takes
      // 12.7 against 14.5 us, at Ly=8, chi=3200 the 128-row tiles are the faster)
      int64_t t128 = 0;
      for (int ai = 0; ai < a.size(); ++ai)
        if (p.L.P.rows[ai] > 0 && p.th.P.cols[ai] > 0)
          t128 += (int64_t)((p.L.P.rows[ai] + 127) / 128) * ((p.th.P.cols[ai] + 63) / 64);
      s1.tile_m = t128 < 2 * (int64_t)p.ncu ? 64 : 128;
    }
    for (int ai = 0; ai < a.size(); ++ai) {
      const int M = p.L.P.rows[ai], N = p.th.P.cols[ai], K = a.dim[ai];
      if (M == 0 || N == 0) continue;
      GemmProb pr{p.xoff[ai], M, N, (int32_t)s1.segs.size(), 1, p.xld[ai], -1};
      s1.segs.push_back({p.L.P.off[ai], p.th.P.off[ai], K, N, K, 0});
      s1.probs.push_back(pr);
      add_tiles(s1, (int32_t)s1.probs.size() - 1, M, N);
      s1.flops += 8.0 * M * N * K;
    }
  };
  // Mixing: Z_{c'}[(s12', a'), (w'', c)] = sum_{w, s12} W12[w, s12', s12, w''] X_a[(w, a'), (s12, c)]
  // Z panel per output sector c': rows (s12', a') stacked, columns the R panel's (w'', c).
  p.zoff.assign(c.size(), 0);
  p.zld.assign(c.size(), 0);
  p.zrows.assign(c.size(), 0);
  p.ztotal = 0;
  std::vector<std::array<int, 4>> zroff(c.size(), {-1, -1, -1, -1});
  for (int ci2 = 0; ci2 < c.size(); ++ci2) {
    int rows = 0;
    for (int s12p = 0; s12p < 4; ++s12p) {
      const int aip = zap[ci2][s12p];
      if (aip < 0) continue;
      zroff[ci2][s12p] = rows;
      rows += a.dim[aip];
    }
    p.zrows[ci2] = rows;
    p.zoff[ci2] = p.ztotal;
    p.zld[ci2] = ld16(p.R.P.cols[ci2]);
    p.ztotal += (int64_t)rows * p.zld[ci2];
  }
  // BF16x3 pre-split operands (bf16 planes, k padded to a multiple of 8): L per ket
  // sector a (M_a x m_a), theta^T per a (N_a x m_a), Z and R per output sector c'
  // (rows x K with K the R panel width).  Laid out, tabled and uploaded only for a plan
  // that runs that path.
  if (p.presplit) {
    // k padded to the chunk width of the stream-K kernels (a multiple of 8 is all the
    // tiled kernels need)
    auto r8 = [](int64_t k) { return (k + SK_KC - 1) / SK_KC * SK_KC; };
    p.lsoff.assign(a.size(), 0);
    p.thsoff.assign(a.size(), 0);
    p.zsoff.assign(c.size(), 0);
    p.rsoff.assign(c.size(), 0);
    p.zkp.assign(c.size(), 0);
    p.ls_total = p.ths_total = p.zs_total = p.rs_total = 0;
    for (int ai = 0; ai < a.size(); ++ai) {
      const int64_t kp = r8(a.dim[ai]);
      p.lsoff[ai] = p.ls_total;
      p.ls_total += 4 * (int64_t)p.L.P.rows[ai] * kp;
      p.thsoff[ai] = p.ths_total;
      p.ths_total += 4 * (int64_t)p.th.P.cols[ai] * kp;
      if (p.L.P.rows[ai] > 0)
        p.lsplit.push_back({p.L.P.off[ai], p.lsoff[ai], a.dim[ai], p.L.P.rows[ai], a.dim[ai], (int32_t)kp, 0,
                            (int32_t)((int64_t)p.L.P.rows[ai] * kp), 0});
      if (p.th.P.cols[ai] > 0)
        p.thsplit.push_back({p.th.P.off[ai], p.thsoff[ai], p.th.P.cols[ai], a.dim[ai], p.th.P.cols[ai],
                             (int32_t)kp, 1, (int32_t)((int64_t)p.th.P.cols[ai] * kp), 0});
    }
    for (int ci2 = 0; ci2 < c.size(); ++ci2) {
      const int K = p.R.P.cols[ci2];
      const int64_t kp = std::max<int64_t>(SK_KC, r8(K));  // an empty R panel keeps zero planes
      p.zkp[ci2] = (int32_t)kp;
      p.zsoff[ci2] = p.zs_total;
      p.zs_total += 4 * (int64_t)p.zrows[ci2] * kp;
      p.rsoff[ci2] = p.rs_total;
      p.rs_total += 4 * (int64_t)c.dim[ci2] * kp;
      if (K > 0)
        p.rsplit.push_back({p.R.P.off[ci2], p.rsoff[ci2], K, c.dim[ci2], K, (int32_t)kp, 0,
                            (int32_t)((int64_t)c.dim[ci2] * kp), 0});
    }
    p.lsplit_items = split_layout(p.lsplit);
    p.rsplit_items = split_layout(p.rsplit);
    p.thsplit_items = split_layout(p.thsplit);
  }
  // (.)R stage, one problem per output sector c':
  //   theta'[(s12', a'), c'] = Z_{c'} (M x K) . Rpanel_{c'}^T (K x m_c'), K = R panel width,
  // rows scattered to the theta blocks through the row table.  K-split over workgroups.
  auto build_s4 = [&](GemmStage& s4, bool bf3) {
    s4.flags = G_B_T | G_C_ROWMAP | (bf3 ? G_C_F64 : 0);  // BF16x3 writes theta' in FP64
    s4.split = true;
    if (bf3) {
      // 128 x 32 tiles, K split over workgroups in runs of >= 12 chunks of 32 (at Ly=8,
      // chi=3200 the GEMM takes about the same time for runs of 6 to 12 chunks, while
      // fewer partial tiles halve the split reduction).  Small windows: 64-row tiles when
      // the flop-weighted problem height is below 128 (half of a 128-row tile would be
      // padding), and runs short enough for about 2.5 workgroups per CU (at least 4
      // chunks): the matvec at Ly=6, chi=800 takes 50 against 70 us.
      double fl = 0.0, flm = 0.0;
      for (int ci2 = 0; ci2 < c.size(); ++ci2) {
        const double f = (double)p.zrows[ci2] * c.dim[ci2] * p.R.P.cols[ci2];
        fl += f;
        flm += f * p.zrows[ci2];
      }
      s4.tile_m = (fl > 0.0 && flm / fl < 128.0) ? 64 : 128;
      s4.tile_n = 32;
      s4.kc = 32;
      int64_t chunks = 0;
      for (int ci2 = 0; ci2 < c.size(); ++ci2)
        if (p.zrows[ci2] > 0)
          chunks += (int64_t)((p.zrows[ci2] + s4.tile_m - 1) / s4.tile_m) * ((c.dim[ci2] + 31) / 32) *
                    ((p.R.P.cols[ci2] + 31) / 32);
      s4.split_min = (int32_t)std::min<int64_t>(12, std::max<int64_t>(4, (chunks * 2) / (5 * (int64_t)p.ncu)));
    } else {    // 32 x 32 tiles shared by four waves, >= 256 K values per split (the
                // kernels stage them in chunks of 32)
      s4.deep = true;
      s4.tile_m = s4.tile_n = 32;
      s4.kc = 64;
      s4.split_min = 4;
    }
    for (int ci2 = 0; ci2 < c.size(); ++ci2) {
      const int M = p.zrows[ci2], N = c.dim[ci2], K = p.R.P.cols[ci2];
      if (M == 0) continue;
      GemmProb pr{0, M, N, (int32_t)s4.segs.size(), K > 0 ? 1 : 0, 0, (int32_t)s4.rows.size()};
      for (int s12p = 0; s12p < 4; ++s12p) {
        const int aip = zap[ci2][s12p];
        if (aip < 0) continue;
        const int64_t base = p.th.P.off[aip] + p.th.coff[aip][s12p];
        for (int r = 0; r < a.dim[aip]; ++r) s4.rows.push_back(base + (int64_t)r * p.th.P.cols[aip]);
      }
      if (K > 0) s4.segs.push_back({p.zoff[ci2], p.R.P.off[ci2], p.zld[ci2], K, K, 0});
      s4.probs.push_back(pr);
      add_tiles(s4, (int32_t)s4.probs.size() - 1, M, N);
      s4.flops += 8.0 * M * N * K;
    }
  };
  // The GEMM stage tables are built and bounds-checked on a second thread while this one
  // builds the mixing tables (disjoint members of the plan; an exception there is
  // rethrown by get()).
  // The matvec stages on pre-split operands (BF16x3): same problems, tiles and K splits
  // as the FP32-operand BF16x3 stages above.
  auto build_ps = [&] {
    PsStage& q1 = p.s1p;
    q1.cout = 0;
    q1.tile_m = 128;
    q1.tile_n = 64;
    q1.split = false;
    for (int ai = 0; ai < a.size(); ++ai) {
      const int M = p.L.P.rows[ai], N = p.th.P.cols[ai], K = a.dim[ai];
      if (M == 0 || N == 0) continue;
      const int kp = (K + SK_KC - 1) / SK_KC * SK_KC;
      q1.probs.push_back({p.lsoff[ai], p.thsoff[ai], (int64_t)M * kp, (int64_t)N * kp, p.xoff[ai], M, N, kp,
                          p.xld[ai], -1, 1, -1, 0});
      add_ps_tiles(q1, (int32_t)q1.probs.size() - 1);
      q1.flops += 8.0 * M * N * K;
    }
    PsStage& q4 = p.s4p;
    q4.cout = 1;
    q4.tile_m = 128;
    q4.tile_n = 32;
    q4.split = true;
    q4.split_min = 12;
    for (int ci2 = 0; ci2 < c.size(); ++ci2) {
      const int M = p.zrows[ci2], N = c.dim[ci2], K = p.R.P.cols[ci2], kp = p.zkp[ci2];
      if (M == 0) continue;
      const int32_t rm = (int32_t)q4.rows.size();
      for (int s12p = 0; s12p < 4; ++s12p) {
        const int aip = zap[ci2][s12p];
        if (aip < 0) continue;
        const int64_t base = p.th.P.off[aip] + p.th.coff[aip][s12p];
        for (int r = 0; r < a.dim[aip]; ++r) q4.rows.push_back(base + (int64_t)r * p.th.P.cols[aip]);
      }
      q4.probs.push_back({p.zsoff[ci2], p.rsoff[ci2], (int64_t)M * kp, (int64_t)N * kp, 0, M, N, kp, 0, rm,
                          1, -1, 0});
      add_ps_tiles(q4, (int32_t)q4.probs.size() - 1);
      q4.flops += 8.0 * M * N * K;
    }
    // stream-K schedules for a persistent grid of one workgroup per CU
    sk_schedule(q1, p.ncu);
    sk_schedule(q4, p.ncu);
    validate(q1, p.ls_total, p.ths_total, p.xtotal);
    validate(q4, p.zs_total, p.rs_total, p.n());
    validate(p.lsplit, p.L.P.total, p.ls_total);
    validate(p.rsplit, p.R.P.total, p.rs_total);
    validate(p.thsplit, p.n(), p.ths_total);
  };
  const bool bf3 = p.prec == DM_BF16X3;
  auto gemm_tables = run_beside([&] {
    build_s1(p.s1, bf3);
    if (bf3) build_s1(p.s1f, false);
    build_s4(p.s4, bf3);
    if (bf3) build_s4(p.s4f, false);
    validate(p.s1, p.L.P.total, p.n(), p.xtotal);
    validate(p.s4, p.ztotal, p.R.P.total, p.n());
    validate(p.s1f, p.L.P.total, p.n(), p.xtotal);
    validate(p.s4f, p.ztotal, p.R.P.total, p.n());
    if (p.presplit) build_ps();
  });
  // two-site MPO W12[w, s12', s12, w''] = sum_w' W1[w, s1', s1, w'] W2[w', s2', s2, w'']
  std::vector<std::complex<double>> w12((size_t)dl * 16 * dr);
  auto W12 = [&](int w, int sp, int s, int wpp) -> std::complex<double>& {
    return w12[(((size_t)w * 4 + sp) * 4 + s) * dr + wpp];
  };
  for (int w = 0; w < dl; ++w)
    for (int s1p = 0; s1p < 2; ++s1p)
      for (int s1 = 0; s1 < 2; ++s1)
        for (int wm = 0; wm < dm; ++wm) {
          const auto x = p.w1.at(w, s1p, s1, wm);
          if (x == std::complex<double>(0, 0)) continue;
          for (int s2p = 0; s2p < 2; ++s2p)
            for (int s2 = 0; s2 < 2; ++s2)
              for (int wpp = 0; wpp < dr; ++wpp) {
                const auto y = p.w2.at(wm, s2p, s2, wpp);
                if (y == std::complex<double>(0, 0)) continue;
                W12(w, s1p * 2 + s2p, s1 * 2 + s2, wpp) += x * y;
              }
        }
  // nonzeros of W12 per (s12', w''): (w, s12, value)
  struct Nz {
    int w, s12;
    std::complex<double> v;
  };
  std::vector<std::vector<Nz>> nz((size_t)4 * dr);
  for (int w = 0; w < dl; ++w)
    for (int s12p = 0; s12p < 4; ++s12p)
      for (int s12 = 0; s12 < 4; ++s12)
        for (int wpp = 0; wpp < dr; ++wpp) {
          const auto v = W12(w, s12p, s12, wpp);
          if (v != std::complex<double>(0, 0)) nz[(size_t)s12p * dr + wpp].push_back({w, s12, v});
        }
  // ket sector a = a' - q(w), or -1
  std::vector<int> a_of((size_t)a.size() * dl);
  for (int aip = 0; aip < a.size(); ++aip)
    for (int w = 0; w < dl; ++w) a_of[(size_t)aip * dl + w] = a.find(qsub(a.q[aip], p.w1.ql[w], ly));
  MixStage& mx = p.mix;
  std::vector<int64_t> task_key;  // (a', c) slab of each task
  // BF16x3: the same tasks writing Z split into bf16 planes (pre-split (.).R operand)
  const bool presplit = p.presplit;
  std::vector<MixTask> ptasks;
  for (int ci2 = 0; ci2 < c.size(); ++ci2) {
    const int Kc = p.R.P.cols[ci2], zl = p.zld[ci2];
    for (int s12p = 0; s12p < 4; ++s12p) {
      const int aip = zap[ci2][s12p];
      if (aip < 0) continue;
      for (int wpp = 0; wpp < dr; ++wpp) {
        const int ci = p.R.c[ci2 * dr + wpp];
        if (ci < 0) continue;
        MixTask tk{p.zoff[ci2] + (int64_t)zroff[ci2][s12p] * zl + p.R.coff[ci2 * dr + wpp], zl,
                   a.dim[aip], c.dim[ci], (int32_t)mx.srcs.size(), 0, 0};
        for (const Nz& e : nz[(size_t)s12p * dr + wpp]) {
          const int w = e.w, s12 = e.s12;
          const auto v = e.v;
          const int ai = a_of[(size_t)aip * dl + w];
          if (ai < 0) continue;
          {
            if (p.th.c[ai][s12] != ci || p.L.ap[ai * dl + w] != aip)
              throw DmError{DM_ERR_CHARGE, "MPO charges inconsistent with the bonds"};
            const int Na = p.xld[ai];
            mx.srcs.push_back({p.xoff[ai] + (int64_t)p.L.roff[ai * dl + w] * Na + p.th.coff[ai][s12],
                               Na, 0, v.real(), v.imag()});
            tk.nsrc++;
          }
        }
        mx.flops += 8.0 * tk.nsrc * tk.rows * tk.cols;
        mx.tasks.push_back(tk);
        task_key.push_back(((int64_t)aip << 32) | (uint32_t)ci);
        if (presplit) {
          MixTask pt = tk;
          const int kpz = p.zkp[ci2];
          pt.dst = p.zsoff[ci2] + (int64_t)zroff[ci2][s12p] * kpz + p.R.coff[ci2 * dr + wpp];
          pt.ld_dst = kpz;
          pt.pstride = (int32_t)((int64_t)p.zrows[ci2] * kpz);
          ptasks.push_back(pt);
        }
      }
    }
  }
  // Every source of a task lies in the X slab (a', c): rows (w, a'), columns (s12, c).
  // Tasks are ordered by slab, so the tasks that re-read one slab run at about the same
  // time (workgroups are dispatched in list order) and find it in cache.
  {
    // stable counting sort by the dense slab index a' * |c| + c
    const size_t nc = (size_t)c.size(), nt = mx.tasks.size();
    std::vector<int32_t> start(a.size() * nc + 1, 0);
    auto slab = [&](int64_t key) { return (size_t)(key >> 32) * nc + (size_t)(uint32_t)key; };
    for (int64_t k : task_key) ++start[slab(k) + 1];
    for (size_t i = 1; i < start.size(); ++i) start[i] += start[i - 1];
    std::vector<MixTask> sorted(nt), psorted(presplit ? nt : 0);
    std::vector<int64_t> key(nt);
    for (size_t i = 0; i < nt; ++i) {
      const int32_t d = start[slab(task_key[i])]++;
      sorted[d] = mx.tasks[i];
      if (presplit) psorted[d] = ptasks[i];
      key[d] = task_key[i];
    }
    mx.tasks.swap(sorted);
    ptasks.swap(psorted);
    task_key.swap(key);
  }
  if (presplit) {
    p.mixp.tasks = ptasks;
    p.mixp.srcs = mx.srcs;
    p.mixp.flops = mx.flops;
    mix_to_slabs(p.mixp, task_key, 8, 20480);
  }
  // slab form with about 20 KB of LDS per workgroup (several workgroups per CU keep
  // enough loads in flight; measured best between 12 and 32 KB at Ly=8, chi=3200),
  // sized for the plan's element (a real plan stages one value per element)
  mix_to_slabs(mx, task_key, (int)elem_bytes(p.prec, p.real), 20480);
  p.mix_flops = mx.flops;
  gemm_tables.get();
  if (p.real) {
    // real kernels; flops at 2 per real multiply-add (the tables counted 8 per complex)
    check_real_mix(mx);
    // (s1f / s4f: the FP64-shaped copies a BF16x3 plan keeps for its FP64 Rayleigh
    // quotient run on the same real buffers)
    p.s1.real = p.s4.real = p.s1f.real = p.s4f.real = mx.real = true;
    p.s1.flops /= 4;
    p.s4.flops /= 4;
    p.s1f.flops /= 4;
    p.s4f.flops /= 4;
    mx.flops /= 4;
    p.mix_flops = mx.flops;
  }
}

extern "C" int dm_heff_plan_create(int32_t ly, const dm_bond* a, const dm_bond* c,
                                   const dm_mpo_site* w1, const dm_mpo_site* w2, const void* L,
                                   const void* R, int32_t prec, dm_stream stream,
                                   dm_heff_plan** out) {
  return guarded([&] {
    if (!out) throw DmError{DM_ERR_ARG, "null output"};
    *out = nullptr;
    check_ly(ly);
    const bool real = take_real(prec);
    check_prec(prec);
    auto p = std::make_unique<dm_heff_plan>();
    p->ly = ly;
    p->prec = prec;
    p->real = real;
    {
      // BF16x3 matvec on pre-split operands with MRDMRG_PRESPLIT=1 (otherwise the
      // kernels split FP32 operands while staging them)
      const char* e = getenv("MRDMRG_PRESPLIT");
      p->presplit = prec == DM_BF16X3 && !real && e && e[0] == '1';
    }
    p->a = make_bond(a, ly);
    p->c = make_bond(c, ly);
    p->w1 = make_mpo(w1, ly);
    p->w2 = make_mpo(w2, ly);
    if (p->w1.dr != p->w2.dl) throw DmError{DM_ERR_DIM, "W1 right and W2 left MPO dimensions differ"};
    for (int i = 0; i < p->w1.dr; ++i)
      if (!qeq(p->w1.qr[i], p->w2.ql[i]))
        throw DmError{DM_ERR_CHARGE, "W1 right and W2 left MPO charges differ"};
    p->th = theta_layout(p->a, p->c, p->w1.qs, p->w2.qs, ly);
    p->L = envl_layout(p->a, p->w1.ql, ly);
    p->R = envr_layout(p->c, p->w2.qr, ly);
    if ((p->L.P.total > 0 && !L) || (p->R.P.total > 0 && !R))
      throw DmError{DM_ERR_ARG, "null environment"};
    {
      int dev = 0;
      HIPCHK(hipGetDevice(&dev));
      HIPCHK(hipDeviceGetAttribute(&p->ncu, hipDeviceAttributeMultiprocessorCount, dev));
    }
    build_heff_tables(*p);  // also validates the GEMM stages
    validate(p->mix, p->xtotal, p->ztotal);
    if (p->presplit) validate(p->mixp, p->xtotal, p->zs_total);
    hipStream_t s = (hipStream_t)stream;
    {
      TableUpload up;
      up.add(p->s1);
      up.add(p->s4);
      up.add(p->s1f);
      up.add(p->s4f);
      up.add(p->mix);
      up.add(p->s1p);
      up.add(p->s4p);
      up.add(p->mixp);
      up.add(p->lsplit, &p->d_lsplit);
      up.add(p->rsplit, &p->d_rsplit);
      up.add(p->thsplit, &p->d_thsplit);
      p->dTables = up.commit(s);
    }
    HIPCHK(hipEventCreateWithFlags(&p->done, hipEventDisableTiming));
    const size_t eb = elem_bytes(prec, real);
    p->dL = dev_alloc(p->L.P.total * eb);
    p->dR = dev_alloc(p->R.P.total * eb);
    p->dX = dev_alloc(p->xtotal * eb);
    p->dZ = dev_alloc(p->ztotal * eb);
    // partial-tile slots keep the complex size (a real partial tile fills the first half)
    p->dSplit = dev_alloc(p->s4.nslots * p->s4.slot_elems() * elem_bytes(prec));
    stage_in(L, p->dL, p->L.P.total, prec, s, real);
    stage_in(R, p->dR, p->R.P.total, prec, s, real);
    if (prec != DM_FP64) {
      p->dL64 = dev_alloc(p->L.P.total * elem_bytes(DM_FP64, real));
      p->dR64 = dev_alloc(p->R.P.total * elem_bytes(DM_FP64, real));
      stage_in(L, p->dL64, p->L.P.total, DM_FP64, s, real);
      stage_in(R, p->dR64, p->R.P.total, DM_FP64, s, real);
      // FP32 copies of theta: the Lanczos kernels write whole complex-pair elements
      // (a real theta of odd length gets a zero pad value)
      p->dTin = dev_alloc(std::max<int64_t>(p->n() * eb, p->nlz() * 8));
      p->dTout = dev_alloc(std::max<int64_t>(p->n() * eb, p->nlz() * 8));
    }
    if (p->presplit) {
      // pre-split L and R (once per plan), theta^T (per matvec) and the split Z; pad
      // columns stay zero: the L and R splits write them, Z's are cleared here and never
      // written by the mixing
      p->dLs = dev_alloc(p->ls_total * 2);
      p->dRs = dev_alloc(p->rs_total * 2);
      p->dThs = dev_alloc(p->ths_total * 2);
      p->dZs = dev_alloc(p->zs_total * 2);
      // partial tiles of either block GEMM (they run one after the other on one stream)
      p->dSplitP = dev_alloc(std::max({p->s4p.nslots * p->s4p.slot_elems(), p->s1p.sk_nslots * SK_BM * SK_BN,
                                       p->s4p.sk_nslots * SK_BM * SK_BN}) * 8);
      // stream-K kernels unless MRDMRG_SK=0 (the tiled pre-split kernels)
      const char* k = getenv("MRDMRG_SK");
      p->streamk = !(k && k[0] == '0');
      if (p->zs_total) HIPCHK(hipMemsetAsync(p->dZs, 0, p->zs_total * 2, s));
      if (p->rs_total) HIPCHK(hipMemsetAsync(p->dRs, 0, p->rs_total * 2, s));
      HIPCHK(launch_split(p->d_lsplit, (int32_t)p->lsplit.size(), p->lsplit_items, (const double*)L,
                          (__bf16*)p->dLs, s));
      HIPCHK(launch_split(p->d_rsplit, (int32_t)p->rsplit.size(), p->rsplit_items, (const double*)R,
                          (__bf16*)p->dRs, s));
    }
    {
      // One Lanczos step per HIP graph replay is available but off by default: on
      // gfx950 at these sizes the step is GPU-bound and replays measured no faster than
      // stream launches, while capturing costs milliseconds per plan.
      const char* g = getenv("MRDMRG_GRAPH");
      p->use_graph = g && g[0] == '1';
    }
    HIPCHK(hipEventRecord(p->done, s));
    *out = p.release();
  });
}

extern "C" void dm_heff_plan_destroy(dm_heff_plan* p) { delete p; }

extern "C" int dm_heff_info(const dm_heff_plan* p, int64_t* theta_elems, double flops[3]) {
  if (!p) return fail(DM_ERR_ARG, "null plan");
  if (theta_elems) *theta_elems = p->n();
  if (flops) {
    flops[0] = p->s1.flops;
    flops[1] = p->mix_flops;
    flops[2] = p->s4.flops;
  }
  return DM_OK;
}

extern "C" int dm_heff_sizes(const dm_heff_plan* p, int64_t sizes[5]) {
  if (!p || !sizes) return fail(DM_ERR_ARG, "null argument");
  sizes[0] = p->L.P.total;
  sizes[1] = p->R.P.total;
  sizes[2] = p->n();
  sizes[3] = p->xtotal;
  sizes[4] = p->ztotal;
  return DM_OK;
}

static hipEvent_t* prof_slot(dm_heff_plan* p) {
  if (!p->profiling) return nullptr;
  if (p->prof_seen++ % p->prof_stride != 0) return nullptr;
  if (p->ev_used == p->ev.size()) p->ev.push_back(timing_events_get());
  return p->ev[p->ev_used++].data();
}

// theta_out = H_eff theta in the plan's precision (FP64 in / out).
void mrd::heff_run(dm_heff_plan* p, const void* theta, void* theta_out, hipStream_t s,
                   bool force64, const int32_t* skip, bool capturing, bool staged) {
  hipEvent_t* ev = (force64 || capturing) ? nullptr : prof_slot(p);
  auto mark = [&](int i) {
    if (ev) HIPCHK(hipEventRecord(ev[i], s));
  };
  if (p->prec == DM_FP64 || force64) {
    // a stage's element form must be the plan's: a complex kernel on real buffers would
    // index twice as far as they reach
    if (p->rq_s1().real != p->real || p->rq_s4().real != p->real || p->mix.real != p->real)
      throw DmError{DM_ERR_LAYOUT, "FP64 stages do not match the plan's real / complex form"};
    void* dL = p->prec == DM_FP64 ? p->dL : p->dL64;
    void* dR = p->prec == DM_FP64 ? p->dR : p->dR64;
    void* dX = p->dX;
    void* dZ = p->dZ;
    void* dP = p->dSplit;
    if (p->prec != DM_FP64) {
      if (!p->dX64) p->dX64 = dev_alloc(p->xtotal * 16);
      if (!p->dZ64) p->dZ64 = dev_alloc(p->ztotal * 16);
      if (!p->dSplit64) p->dSplit64 = dev_alloc(p->rq_s4().nslots * p->rq_s4().slot_elems() * 16);
      dX = p->dX64;
      dZ = p->dZ64;
      dP = p->dSplit64;
    }
    mark(0);
    HIPCHK(launch_gemm<double>(p->rq_s1(), (const double*)dL, (const double*)theta, (double*)dX, nullptr,
                               s, skip));
    mark(1);
    HIPCHK(launch_mix<double>(p->mix, (const double*)dX, (double*)dZ, s, skip));
    mark(2);
    HIPCHK(launch_gemm<double>(p->rq_s4(), (const double*)dZ, (const double*)dR, (double*)theta_out,
                               (double*)dP, s, skip, [&] { mark(3); }));
    mark(4);
    return;
  }
  if (p->prec == DM_BF16X3 && p->presplit) {
    // theta split into bf16 planes (transposed per panel: the L.theta GEMM's B operand),
    // both block GEMMs on pre-split operands, theta' written in FP64 by the (.).R stage
    HIPCHK(launch_split(p->d_thsplit, (int32_t)p->thsplit.size(), p->thsplit_items, (const double*)theta,
                        (__bf16*)p->dThs, s, skip));
    mark(0);
    auto gemm = p->streamk ? launch_gemm_sk : launch_gemm_ps;
    HIPCHK(gemm(p->s1p, (const __bf16*)p->dLs, (const __bf16*)p->dThs, p->dX, (float*)p->dSplitP, s, skip, {}));
    mark(1);
    HIPCHK(launch_mix_split(p->mixp, (const float*)p->dX, (__bf16*)p->dZs, s, skip));
    mark(2);
    HIPCHK(gemm(p->s4p, (const __bf16*)p->dZs, (const __bf16*)p->dRs, theta_out, (float*)p->dSplitP, s, skip,
                [&] { mark(3); }));
    mark(4);
    return;
  }
  // theta in: an FP32 copy; theta' out: BF16x3 stages write FP64 themselves (the FP32
  // results widened as they are stored), FP32 stages through an FP32 copy
  const bool direct = p->prec == DM_BF16X3;
  if (p->s1.real != p->real || p->s4.real != p->real || p->mix.real != p->real)
    throw DmError{DM_ERR_LAYOUT, "stages do not match the plan's real / complex form"};
  if (!staged) HIPCHK(launch_cast_d2f((const double*)theta, (float*)p->dTin, p->nreal(), s, skip));
  float* tout = direct ? (float*)theta_out : (float*)p->dTout;
  mark(0);
  HIPCHK(gemm_lp(p->prec, p->s1, (const float*)p->dL, (const float*)p->dTin, (float*)p->dX, nullptr, s, skip));
  mark(1);
  HIPCHK(launch_mix<float>(p->mix, (const float*)p->dX, (float*)p->dZ, s, skip));
  mark(2);
  HIPCHK(gemm_lp(p->prec, p->s4, (const float*)p->dZ, (const float*)p->dR, tout,
                 (float*)p->dSplit, s, skip, [&] { mark(3); }));
  mark(4);
  if (!direct) HIPCHK(launch_cast_f2d((const float*)p->dTout, (double*)theta_out, p->nreal(), s, skip));
}

extern "C" int dm_heff_profile(dm_heff_plan* p, int32_t enable) {
  if (!p) return fail(DM_ERR_ARG, "null plan");
  if (enable < 0) return fail(DM_ERR_ARG, "negative profiling stride");
  p->profiling = enable != 0;
  p->prof_stride = enable > 0 ? enable : 1;
  p->prof_seen = 0;
  p->ev_used = 0;
  return DM_OK;
}

extern "C" int dm_heff_profile_read(dm_heff_plan* p, double ms[4], int64_t* matvecs) {
  return guarded([&] {
    if (!p || !ms) throw DmError{DM_ERR_ARG, "null argument"};
    ms[0] = ms[1] = ms[2] = ms[3] = 0.0;
    for (size_t i = 0; i < p->ev_used; ++i) {
      HIPCHK(hipEventSynchronize(p->ev[i][4]));
      for (int st = 0; st < 4; ++st) {
        float t = 0;
        HIPCHK(hipEventElapsedTime(&t, p->ev[i][st], p->ev[i][st + 1]));
        ms[st] += t;
      }
    }
    if (matvecs) *matvecs = (int64_t)p->ev_used;
  });
}

static int heff_apply_impl(dm_heff_plan* p, const void* theta, void* theta_out, dm_stream stream);

extern "C" int heff_apply(dm_heff_plan* p, const void* theta, void* theta_out, dm_stream stream) {
  const int rc = heff_apply_impl(p, theta, theta_out, stream);
  if (rc != DM_OK) drain(stream);  // no queued work outlives the error
  return rc;
}

static int heff_apply_impl(dm_heff_plan* p, const void* theta, void* theta_out, dm_stream stream) {
  return guarded([&] {
    if (!p) throw DmError{DM_ERR_ARG, "null plan"};
    if (p->n() > 0 && (!theta || !theta_out)) throw DmError{DM_ERR_ARG, "null theta"};
    if (misaligned(theta) || misaligned(theta_out))
      throw DmError{DM_ERR_ARG, "theta buffers must be 16-byte aligned"};
    if (theta == theta_out && p->n() > 0) throw DmError{DM_ERR_ARG, "theta and theta_out overlap"};
    heff_run(p, theta, theta_out, (hipStream_t)stream, false);
    HIPCHK(hipEventRecord(p->done, (hipStream_t)stream));
  });
}

void mrd::ensure_lanczos(dm_heff_plan* p, int max_iter) {
  const int64_t n = p->nlz();  // complex elements of the Lanczos vectors
  bool relayout = !p->dInst;
  if (p->Vcap < max_iter + 1) {
    if (p->graph_exec) (void)hipGraphExecDestroy(p->graph_exec);
    if (p->graph) (void)hipGraphDestroy(p->graph);
    p->graph_exec = nullptr;
    p->graph = nullptr;
    dev_free(p->dV);
    p->dV = nullptr;
    dev_free(p->dPart);
    p->dPart = nullptr;
    const int cap = std::max(max_iter + 1, 31);
    p->dV = (double*)dev_alloc((size_t)cap * n * 16);
    p->Vcap = cap;
    p->dPart = (double*)dev_alloc((size_t)lz_part_doubles(n, cap - 1) * 8);
    relayout = true;
  }
  if (!p->dW || !p->dVcur) {
    if (!p->dW) p->dW = (double*)dev_alloc((size_t)n * 16);
    if (!p->dVcur) p->dVcur = (double*)dev_alloc((size_t)n * 16);
    // a real theta of odd length: the pad value of w (never written by the matvec) and
    // of v_j must be zero from the start
    if (p->real && (p->n() & 1)) {
      HIPCHK(hipMemset(p->dW, 0, (size_t)n * 16));
      HIPCHK(hipMemset(p->dVcur, 0, (size_t)n * 16));
    }
  }
  if (!p->dState) p->dState = (LzState*)dev_alloc(sizeof(LzState));
  if (!p->dInst) p->dInst = (LzInst*)dev_alloc(sizeof(LzInst));
  if (!p->dRes) p->dRes = (LzResult*)dev_alloc(sizeof(LzResult));
  // pinned from the library's pool: a plan per bond update would otherwise pay a pinned
  // allocation and free (which can wait for the device) on every bond
  if (!p->hInst) p->hInst = (LzInst*)pinned_alloc(sizeof(LzInst));
  if (!p->hRes) p->hRes = (LzResult*)pinned_alloc(sizeof(LzResult));
  if (relayout) {
    std::vector<LzInst> I(1);
    I[0] = LzInst{p->dV, p->dW, p->dVcur, p->dPart, nullptr, nullptr, p->dState, n, n};
    I[0].xn = p->nreal();
    I[0].real = p->real ? 1 : 0;
    // v_j also written in FP32 when the matvec reads an FP32 copy (a BF16x3 plan on
    // pre-split operands splits v_j itself)
    I[0].tin = p->staged_in() ? (float*)p->dTin : nullptr;
    p->lzg = lz_layout(I, p->Vcap - 1);
    p->lzg.vf32 = p->prec != DM_FP64;  // FP32 / BF16x3: the basis in FP32, as the matvec reads it
    *p->hInst = I[0];
  }
  if (p->prec != DM_FP64) {
    if (!p->dX64) p->dX64 = dev_alloc(p->xtotal * 16);
    if (!p->dZ64) p->dZ64 = dev_alloc(p->ztotal * 16);
    if (!p->dSplit64) p->dSplit64 = dev_alloc(p->rq_s4().nslots * p->rq_s4().slot_elems() * 16);
  }
}

// One Lanczos step: w = H v_j, projections, scalars, v_{j+1}.  The device state holds
// the step index; j + 1 (or 0 for a step captured once for every replay) only bounds
// the Krylov vector count so the projection kernels can be sized to it.
static void lanczos_step(dm_heff_plan* p, hipStream_t s, bool capturing, int32_t j) {
  heff_run(p, p->dVcur, p->dW, s, false, &p->dState->stop, capturing, p->staged_in());
  HIPCHK(lz_launch_step_tail(p->dInst, p->lzg, capturing ? 0 : j + 1, s));
}

extern "C" int lanczos_ground(dm_heff_plan* p, void* theta_inout, int32_t max_iter, double tol,
                              double* energy, int32_t* iters, dm_stream stream) {
  // an error after work was queued returns only once that work has drained, so that no
  // kernel of the solve can still run when the caller reacts (frees buffers, exits)
  const int rc = lanczos_ground_impl(p, theta_inout, max_iter, tol, energy, iters, stream);
  if (rc != DM_OK && p) drain(stream);
  return rc;
}

static int lanczos_ground_impl(dm_heff_plan* p, void* theta_inout, int32_t max_iter, double tol,
                               double* energy, int32_t* iters, dm_stream stream) {
  return guarded([&] {
    if (!p || !energy || !iters) throw DmError{DM_ERR_ARG, "null argument"};
    if (max_iter < 1 || max_iter > LZ_MAX) throw DmError{DM_ERR_ARG, "max_iter must be in 1..64"};
    const int64_t n = p->n();
    if (n == 0) throw DmError{DM_ERR_LAYOUT, "empty theta"};
    if (!theta_inout) throw DmError{DM_ERR_ARG, "null theta"};
    if (misaligned(theta_inout)) throw DmError{DM_ERR_ARG, "theta must be 16-byte aligned"};
    ensure_lanczos(p, max_iter);
    hipStream_t s = (hipStream_t)stream;
    p->hInst->x = (double*)theta_inout;  // the previous solve synchronised: buffer is free
    HIPCHK(hipMemcpyAsync(p->dInst, p->hInst, sizeof(LzInst), hipMemcpyHostToDevice, s));
    HIPCHK(lz_launch_init(p->dInst, p->lzg, max_iter, tol, s));
    HIPCHK(lz_launch_start(p->dInst, p->lzg, s));
    const bool graph = p->use_graph && !p->profiling;
    if (graph && !p->graph_exec) {
      if (!p->cap_stream) HIPCHK(hipStreamCreateWithFlags(&p->cap_stream, hipStreamNonBlocking));
      HIPCHK(hipStreamBeginCapture(p->cap_stream, hipStreamCaptureModeThreadLocal));
      try {
        lanczos_step(p, p->cap_stream, true, 0);
      } catch (...) {
        hipGraph_t g = nullptr;
        (void)hipStreamEndCapture(p->cap_stream, &g);
        if (g) (void)hipGraphDestroy(g);
        throw;
      }
      HIPCHK(hipStreamEndCapture(p->cap_stream, &p->graph));
      HIPCHK(hipGraphInstantiate(&p->graph_exec, p->graph, nullptr, nullptr, 0));
    }
    for (int j = 0; j < max_iter; ++j) {
      if (graph)
        HIPCHK(hipGraphLaunch(p->graph_exec, s));
      else
        lanczos_step(p, s, false, j);
    }
    HIPCHK(lz_launch_finish(p->dInst, p->lzg, s));
    if (p->prec != DM_FP64) {
      // FP64 Rayleigh quotient of the Ritz vector (also held in vcur)
      heff_run(p, p->dVcur, p->dW, s, true);
      HIPCHK(lz_launch_rq(p->dInst, p->lzg, s));
    }
    HIPCHK(lz_launch_results(p->dInst, p->lzg, p->dRes, s));
    HIPCHK(hipMemcpyAsync(p->hRes, p->dRes, sizeof(LzResult), hipMemcpyDeviceToHost, s));
    HIPCHK(hipEventRecord(p->done, s));
    HIPCHK(hipStreamSynchronize(s));
    if (p->hRes->bad) throw DmError{DM_ERR_NONFINITE, "Lanczos produced a zero, NaN or Inf norm"};
    *energy = p->hRes->energy;
    *iters = p->hRes->k;
  });
}

// =====================================================================================
// Environment updates
// =====================================================================================
namespace {

// One nonzero of an MPO site tensor with the two indices a loop runs over.
struct MpoNz {
  int w, s;
  std::complex<double> v;
};

struct EnvPlan {
  GemmStage t1, t3;
  MixStage mix;
  int64_t t1total = 0, t2total = 0;
  double flops() const { return t1.flops + mix.flops + t3.flops; }
};

// Output tile of the T3 stage: its problems are one m_b' x m_b block each (a few tens
// of rows and columns), which 32 x 32 BF16x3 tiles cover with little padding; the FP
// kernels keep their 64 x 64 shape.
int env_t3_tile(int prec) { return prec == DM_BF16X3 ? 32 : 64; }
// Column tile of the right update's T1 stage (N = m_b, a few tens): 32 for BF16x3.
int env_t1r_tile_n(int prec) { return prec == DM_BF16X3 ? 32 : 64; }

// L'[b', w', b] = sum conj(A[a', s', b']) L[a', w, a] W[w, s', s, w'] A[a, s, b]
EnvPlan plan_left(int ly, const Bond& a, const Bond& b, const MpoSite& W, const EnvLLayout& L,
                  const SiteLayout& S, const EnvLLayout& Lo, int t3_tile) {
  EnvPlan ep;
  const int dl = W.dl, dr = W.dr;
  std::vector<int64_t> t1off(a.size());
  for (int ai = 0; ai < a.size(); ++ai) {
    t1off[ai] = ep.t1total;
    ep.t1total += (int64_t)L.P.rows[ai] * S.P.cols[ai];
  }
  // T1_a = Lpanel_a (M_a x m_a) . Apanel_a (m_a x (s, b))
  ep.t1.flags = 0;
  for (int ai = 0; ai < a.size(); ++ai) {
    const int M = L.P.rows[ai], N = S.P.cols[ai], K = a.dim[ai];
    if (M == 0 || N == 0) continue;
    GemmProb pr{t1off[ai], M, N, (int32_t)ep.t1.segs.size(), 1, N, -1};
    ep.t1.segs.push_back({L.P.off[ai], S.P.off[ai], K, N, K, 0});
    ep.t1.probs.push_back(pr);
    add_tiles(ep.t1, (int32_t)ep.t1.probs.size() - 1, M, N);
    ep.t1.flops += 8.0 * M * N * K;
  }
  // T2 panel per b: rows (w', s', a') with b' = b + q(w'), a' = b' - q(s'); cols m_b
  std::vector<int64_t> t2off(b.size());
  std::vector<int> t2roff((size_t)b.size() * dr * 2, -1);
  for (int bi = 0; bi < b.size(); ++bi) {
    int rows = 0;
    for (int wp = 0; wp < dr; ++wp) {
      const int bpi = Lo.ap[bi * dr + wp];
      if (bpi < 0) continue;
      for (int sp = 0; sp < 2; ++sp) {
        const int api = a.find(qsub(b.q[bpi], W.qs[sp], ly));
        if (api < 0 || S.b[api][sp] != bpi) continue;
        t2roff[((size_t)bi * dr + wp) * 2 + sp] = rows;
        rows += a.dim[api];
      }
    }
    t2off[bi] = ep.t2total;
    ep.t2total += (int64_t)rows * b.dim[bi];
  }
  // nonzeros of W per (s', w'): (w, s, value); ket sector a = a' - q(w)
  std::vector<std::vector<MpoNz>> nz((size_t)2 * dr);
  for (int w = 0; w < dl; ++w)
    for (int sp = 0; sp < 2; ++sp)
      for (int s = 0; s < 2; ++s)
        for (int wp = 0; wp < dr; ++wp) {
          const auto v = W.at(w, sp, s, wp);
          if (v != std::complex<double>(0, 0)) nz[(size_t)sp * dr + wp].push_back({w, s, v});
        }
  std::vector<int> a_of((size_t)a.size() * dl);
  for (int api = 0; api < a.size(); ++api)
    for (int w = 0; w < dl; ++w) a_of[(size_t)api * dl + w] = a.find(qsub(a.q[api], W.ql[w], ly));
  for (int bi = 0; bi < b.size(); ++bi)
    for (int wp = 0; wp < dr; ++wp) {
      const int bpi = Lo.ap[bi * dr + wp];
      if (bpi < 0) continue;
      for (int sp = 0; sp < 2; ++sp) {
        const int ro = t2roff[((size_t)bi * dr + wp) * 2 + sp];
        if (ro < 0) continue;
        const int api = a.find(qsub(b.q[bpi], W.qs[sp], ly));
        MixTask tk{t2off[bi] + (int64_t)ro * b.dim[bi], b.dim[bi], a.dim[api], b.dim[bi],
                   (int32_t)ep.mix.srcs.size(), 0, 0};
        for (const MpoNz& e : nz[(size_t)sp * dr + wp]) {
          const int w = e.w, s = e.s;
          const auto v = e.v;
          {
            const int ai = a_of[(size_t)api * dl + w];
            if (ai < 0 || S.b[ai][s] != bi) continue;
            if (L.ap[ai * dl + w] != api) throw DmError{DM_ERR_CHARGE, "inconsistent MPO charges"};
            const int N = S.P.cols[ai];
            ep.mix.srcs.push_back({t1off[ai] + (int64_t)L.roff[ai * dl + w] * N + S.coff[ai][s], N, 0,
                                   v.real(), v.imag()});
            tk.nsrc++;
          }
        }
        ep.mix.flops += 8.0 * tk.nsrc * tk.rows * tk.cols;
        ep.mix.tasks.push_back(tk);
      }
    }
  // T3: L'_{w'}[b', b] = sum_{s'} conj(A_{a',s',b'})^T (m_b' x m_a') . T2 (m_a' x m_b)
  ep.t3.flags = G_A_T | G_A_CONJ;
  ep.t3.tile_m = ep.t3.tile_n = t3_tile;
  for (int bi = 0; bi < b.size(); ++bi)
    for (int wp = 0; wp < dr; ++wp) {
      const int bpi = Lo.ap[bi * dr + wp];
      if (bpi < 0) continue;
      const int M = b.dim[bpi], N = b.dim[bi];
      GemmProb pr{Lo.P.off[bi] + (int64_t)Lo.roff[bi * dr + wp] * N, M, N,
                  (int32_t)ep.t3.segs.size(), 0, N, -1};
      int K = 0;
      for (int sp = 0; sp < 2; ++sp) {
        const int ro = t2roff[((size_t)bi * dr + wp) * 2 + sp];
        if (ro < 0) continue;
        const int api = a.find(qsub(b.q[bpi], W.qs[sp], ly));
        ep.t3.segs.push_back({S.P.off[api] + S.coff[api][sp], t2off[bi] + (int64_t)ro * N,
                              S.P.cols[api], N, a.dim[api], 0});
        pr.nseg++;
        K += a.dim[api];
      }
      ep.t3.probs.push_back(pr);
      add_tiles(ep.t3, (int32_t)ep.t3.probs.size() - 1, M, N);
      ep.t3.flops += 8.0 * M * N * K;
    }
  return ep;
}

// R'[b', w, b] = sum conj(B[b', s', c']) W[w, s', s, w'] R[c', w', c] B[b, s, c]
EnvPlan plan_right(int ly, const Bond& b, const Bond& c, const MpoSite& W, const EnvRLayout& R,
                   const SiteLayout& S, const EnvRLayout& Ro, int t3_tile, int t1_tile_n) {
  EnvPlan ep;
  const int dl = W.dl, dr = W.dr;
  // T1 per (c, s): rows (w', c') with c' = c + q(w'); cols m_b, b = c - q(s)
  std::vector<int64_t> t1off((size_t)c.size() * 2, -1);
  std::vector<int> t1roff((size_t)c.size() * 2 * dr, -1);
  ep.t1.flags = G_A_ROWMAP | G_B_T;
  ep.t1.tile_n = t1_tile_n;
  // Offsets first (the mixing tables need them): every (c, s) with a b sector stacks the
  // R rows of every (w', c'); its rows start at t1rm in the row table.
  std::vector<int32_t> t1m((size_t)c.size() * 2, 0), t1rm((size_t)c.size() * 2, 0);
  size_t nrows = 0;
  for (int ci = 0; ci < c.size(); ++ci)
    for (int s = 0; s < 2; ++s) {
      const int bi = b.find(qsub(c.q[ci], W.qs[s], ly));
      if (bi < 0 || S.b[bi][s] != ci) continue;
      int M = 0;
      for (int wp = 0; wp < dr; ++wp) {
        const int cpi = c.find(qadd(c.q[ci], W.qr[wp], ly));
        if (cpi < 0) continue;
        t1roff[((size_t)ci * 2 + s) * dr + wp] = M;
        M += c.dim[cpi];
      }
      t1m[ci * 2 + s] = M;
      t1rm[ci * 2 + s] = (int32_t)nrows;
      nrows += M;
      t1off[ci * 2 + s] = ep.t1total;
      ep.t1total += (int64_t)M * b.dim[bi];
    }
  // The T1 row table and problems on a second thread while this one builds the mixing and
  // T3 tables (disjoint members of ep)
  auto t1_tables = run_beside([&] {
    ep.t1.rows.resize(nrows);
    for (int ci = 0; ci < c.size(); ++ci)
      for (int s = 0; s < 2; ++s) {
        const int64_t o = t1off[ci * 2 + s];
        if (o < 0) continue;
        const int bi = b.find(qsub(c.q[ci], W.qs[s], ly));
        int64_t* out = ep.t1.rows.data() + t1rm[ci * 2 + s];
        for (int wp = 0; wp < dr; ++wp) {
          const int cpi = c.find(qadd(c.q[ci], W.qr[wp], ly));
          if (cpi < 0) continue;
          const int64_t base = R.P.off[cpi] + R.coff[cpi * dr + wp];
          for (int r = 0; r < c.dim[cpi]; ++r) *out++ = base + (int64_t)r * R.P.cols[cpi];
        }
        const int M = t1m[ci * 2 + s], N = b.dim[bi], K = c.dim[ci];
        if (M == 0) continue;
        GemmProb pr{o, M, N, (int32_t)ep.t1.segs.size(), 1, N, t1rm[ci * 2 + s]};
        ep.t1.segs.push_back({0, S.P.off[bi] + S.coff[bi][s], 0, S.P.cols[bi], K, 0});
        ep.t1.probs.push_back(pr);
        add_tiles(ep.t1, (int32_t)ep.t1.probs.size() - 1, M, N);
        ep.t1.flops += 8.0 * M * N * K;
      }
  });
  // T2 per (w, b): rows (s', c') with b' = b + q(w), c' = b' + q(s'); cols m_b
  std::vector<int64_t> t2off((size_t)dl * b.size(), -1);
  std::vector<int> t2roff((size_t)dl * b.size() * 2, -1);
  for (int w = 0; w < dl; ++w)
    for (int bi = 0; bi < b.size(); ++bi) {
      const int bpi = b.find(qadd(b.q[bi], W.ql[w], ly));
      if (bpi < 0) continue;
      int rows = 0;
      for (int sp = 0; sp < 2; ++sp) {
        const int cpi = S.b[bpi][sp];
        if (cpi < 0) continue;
        t2roff[((size_t)w * b.size() + bi) * 2 + sp] = rows;
        rows += c.dim[cpi];
      }
      t2off[(size_t)w * b.size() + bi] = ep.t2total;
      ep.t2total += (int64_t)rows * b.dim[bi];
    }
  // nonzeros of W per (w, s'): (w', s, value); c = c' - q(w'); b = c - q(s)
  std::vector<std::vector<MpoNz>> nz((size_t)dl * 2);
  for (int w = 0; w < dl; ++w)
    for (int sp = 0; sp < 2; ++sp)
      for (int wp = 0; wp < dr; ++wp)
        for (int s = 0; s < 2; ++s) {
          const auto v = W.at(w, sp, s, wp);
          if (v != std::complex<double>(0, 0)) nz[(size_t)w * 2 + sp].push_back({wp, s, v});
        }
  std::vector<int> c_of((size_t)c.size() * dr), b_of((size_t)c.size() * 2);
  for (int cpi = 0; cpi < c.size(); ++cpi)
    for (int wp = 0; wp < dr; ++wp) c_of[(size_t)cpi * dr + wp] = c.find(qsub(c.q[cpi], W.qr[wp], ly));
  for (int ci = 0; ci < c.size(); ++ci)
    for (int s = 0; s < 2; ++s) b_of[(size_t)ci * 2 + s] = b.find(qsub(c.q[ci], W.qs[s], ly));
  for (int w = 0; w < dl; ++w)
    for (int bi = 0; bi < b.size(); ++bi) {
      const int64_t base = t2off[(size_t)w * b.size() + bi];
      if (base < 0) continue;
      const int bpi = b.find(qadd(b.q[bi], W.ql[w], ly));
      for (int sp = 0; sp < 2; ++sp) {
        const int ro = t2roff[((size_t)w * b.size() + bi) * 2 + sp];
        if (ro < 0) continue;
        const int cpi = S.b[bpi][sp];
        MixTask tk{base + (int64_t)ro * b.dim[bi], b.dim[bi], c.dim[cpi], b.dim[bi],
                   (int32_t)ep.mix.srcs.size(), 0, 0};
        for (const MpoNz& e : nz[(size_t)w * 2 + sp]) {
          const int wp = e.w, s = e.s;
          const auto v = e.v;
          {
            const int ci = c_of[(size_t)cpi * dr + wp];
            if (ci < 0) continue;
            const int64_t o = t1off[ci * 2 + s];
            if (o < 0) continue;
            const int ro1 = t1roff[((size_t)ci * 2 + s) * dr + wp];
            if (ro1 < 0) throw DmError{DM_ERR_CHARGE, "inconsistent MPO charges"};
            if (b_of[(size_t)ci * 2 + s] != bi)
              throw DmError{DM_ERR_CHARGE, "inconsistent MPO charges"};
            ep.mix.srcs.push_back({o + (int64_t)ro1 * b.dim[bi], b.dim[bi], 0, v.real(), v.imag()});
            tk.nsrc++;
          }
        }
        ep.mix.flops += 8.0 * tk.nsrc * tk.rows * tk.cols;
        ep.mix.tasks.push_back(tk);
      }
    }
  // T3: R'_w[b', b] = sum_{s'} conj(B_{b', s', c'}) (m_b' x m_c') . T2 (m_c' x m_b)
  ep.t3.flags = G_A_CONJ;
  ep.t3.tile_m = ep.t3.tile_n = t3_tile;
  for (int w = 0; w < dl; ++w)
    for (int bi = 0; bi < b.size(); ++bi) {
      const int64_t base = t2off[(size_t)w * b.size() + bi];
      if (base < 0) continue;
      const int bpi = b.find(qadd(b.q[bi], W.ql[w], ly));
      const int M = b.dim[bpi], N = b.dim[bi];
      const int col = Ro.coff[bpi * dl + w];
      GemmProb pr{Ro.P.off[bpi] + col, M, N, (int32_t)ep.t3.segs.size(), 0, Ro.P.cols[bpi], -1};
      int K = 0;
      for (int sp = 0; sp < 2; ++sp) {
        const int ro = t2roff[((size_t)w * b.size() + bi) * 2 + sp];
        if (ro < 0) continue;
        const int cpi = S.b[bpi][sp];
        ep.t3.segs.push_back({S.P.off[bpi] + S.coff[bpi][sp], base + (int64_t)ro * N,
                              S.P.cols[bpi], N, c.dim[cpi], 0});
        pr.nseg++;
        K += c.dim[cpi];
      }
      ep.t3.probs.push_back(pr);
      add_tiles(ep.t3, (int32_t)ep.t3.probs.size() - 1, M, N);
      ep.t3.flops += 8.0 * M * N * K;
    }
  t1_tables.get();
  return ep;
}

// Device scratch of one environment update: blocks from the caching pool, handed back
// in stream order (run_env), or consecutive pieces of one fixed region that the caller
// owns (env_update_left_noalloc).
struct EnvScratch {
  char* base = nullptr;  // fixed region, or null for the pool
  size_t cap = 0, used = 0;
  std::vector<void*> pooled;
  static size_t align(size_t b) { return (b + 255) & ~size_t(255); }
  void* get(size_t bytes) {
    if (!base) {
      void* q = dev_alloc(bytes);
      pooled.push_back(q);
      return q;
    }
    if (bytes == 0) return nullptr;
    const size_t off = align(used);
    if (off + bytes > cap) throw DmError{DM_ERR_ALLOC, "environment update scratch exceeds its region"};
    used = off + bytes;
    return base + off;
  }
  void release(hipStream_t s) {
    for (void* q : pooled) dev_free_after(q, s);
    pooled.clear();
  }
};

// Real operands (eq. rot): every stage runs its real kernels; the MPO coefficients the
// mixing applies must be real.
void check_real_mix(const MixStage& m) {
  for (const MixSrc& x : m.srcs)
    if (x.im != 0.0) throw DmError{DM_ERR_ARG, "real operands (DM_REAL) need an MPO with real entries"};
}
void make_real(EnvPlan& ep) {
  check_real_mix(ep.mix);
  ep.t1.real = ep.t3.real = ep.mix.real = true;
}

// Bytes of fixed-region scratch run_env takes (every piece 256-byte aligned).
size_t env_scratch_bytes(const EnvPlan& ep, size_t table_bytes, int64_t nenv, int64_t nsite,
                         int64_t nout, int prec, bool real) {
  const size_t eb = elem_bytes(prec, real);
  size_t b = EnvScratch::align(table_bytes) + EnvScratch::align(ep.t1total * eb) +
             EnvScratch::align(ep.t2total * eb);
  if (prec != DM_FP64)
    b += EnvScratch::align(nenv * eb) + EnvScratch::align(nsite * eb) + EnvScratch::align(nout * eb);
  return b;
}

// Runs T1 -> mix -> T3, stream-ordered (no host wait), FP64 or FP32 storage.  Tables
// and intermediates come from `sc`: from the caching pools (handed back for reuse once
// the stream has passed them), or from a fixed region (tables copied from pageable host
// memory, which the copy has consumed when it returns).
void run_env(EnvPlan& ep, const void* env, int64_t nenv, const void* site, int64_t nsite,
             void* out, int64_t nout, int prec, bool real, hipStream_t s, EnvScratch& sc) {
  const size_t eb = elem_bytes(prec, real);
  try {
    TableUpload up;
    up.add(ep.t1);
    up.add(ep.t3);
    up.add(ep.mix);
    if (sc.base) up.commit_pageable(sc.get(up.total), s);
    else sc.pooled.push_back(up.commit(s));
    void* t1 = sc.get(ep.t1total * eb);
    void* t2 = sc.get(ep.t2total * eb);
    if (prec == DM_FP64) {
      HIPCHK(launch_gemm<double>(ep.t1, (const double*)env, (const double*)site, (double*)t1, nullptr, s));
      HIPCHK(launch_mix<double>(ep.mix, (const double*)t1, (double*)t2, s));
      HIPCHK(launch_gemm<double>(ep.t3, (const double*)site, (const double*)t2, (double*)out, nullptr, s));
    } else {
      void* e32 = sc.get(nenv * eb);
      void* s32 = sc.get(nsite * eb);
      void* o32 = sc.get(nout * eb);
      stage_in(env, e32, nenv, DM_FP32, s, real);
      stage_in(site, s32, nsite, DM_FP32, s, real);
      HIPCHK(gemm_lp(prec, ep.t1, (const float*)e32, (const float*)s32, (float*)t1, nullptr, s));
      HIPCHK(launch_mix<float>(ep.mix, (const float*)t1, (float*)t2, s));
      HIPCHK(gemm_lp(prec, ep.t3, (const float*)s32, (const float*)t2, (float*)o32, nullptr, s));
      stage_out(o32, out, nout, DM_FP32, s, real);
    }
  } catch (...) {
    sc.release(s);
    throw;
  }
  sc.release(s);
}

}  // namespace

static int env_update_left_impl(int32_t ly, const dm_bond* a, const dm_bond* b,
                               const dm_mpo_site* w, const void* L, const void* A, void* L_out,
                               int32_t prec, dm_stream stream);

extern "C" int env_update_left(int32_t ly, const dm_bond* a, const dm_bond* b,
                               const dm_mpo_site* w, const void* L, const void* A, void* L_out,
                               int32_t prec, dm_stream stream) {
  const int rc = env_update_left_impl(ly, a, b, w, L, A, L_out, prec, stream);
  if (rc != DM_OK) drain(stream);  // no queued work outlives the error
  return rc;
}

static int env_update_left_impl(int32_t ly, const dm_bond* a, const dm_bond* b,
                               const dm_mpo_site* w, const void* L, const void* A, void* L_out,
                               int32_t prec, dm_stream stream) {
  return guarded([&] {
    check_ly(ly);
    const bool real = take_real(prec);
    check_prec(prec);
    Bond ba = make_bond(a, ly), bb = make_bond(b, ly);
    MpoSite W = make_mpo(w, ly);
    EnvLLayout Li = envl_layout(ba, W.ql, ly);
    EnvLLayout Lo = envl_layout(bb, W.qr, ly);
    SiteLayout S = site_layout(ba, bb, W.qs, ly);
    if ((Li.P.total && !L) || (S.P.total && !A) || (Lo.P.total && !L_out))
      throw DmError{DM_ERR_ARG, "null tensor"};
    EnvPlan ep = plan_left(ly, ba, bb, W, Li, S, Lo, env_t3_tile(prec));
    validate(ep.t1, Li.P.total, S.P.total, ep.t1total);
    validate(ep.mix, ep.t1total, ep.t2total);
    validate(ep.t3, S.P.total, ep.t2total, Lo.P.total);
    if (real) make_real(ep);
    EnvScratch pool;
    run_env(ep, L, Li.P.total, A, S.P.total, L_out, Lo.P.total, prec, real, (hipStream_t)stream, pool);
  });
}

static int env_update_right_impl(int32_t ly, const dm_bond* b, const dm_bond* c,
                                const dm_mpo_site* w, const void* R, const void* B, void* R_out,
                                int32_t prec, dm_stream stream);

extern "C" int env_update_right(int32_t ly, const dm_bond* b, const dm_bond* c,
                                const dm_mpo_site* w, const void* R, const void* B, void* R_out,
                                int32_t prec, dm_stream stream) {
  const int rc = env_update_right_impl(ly, b, c, w, R, B, R_out, prec, stream);
  if (rc != DM_OK) drain(stream);  // no queued work outlives the error
  return rc;
}

static int env_update_right_impl(int32_t ly, const dm_bond* b, const dm_bond* c,
                                const dm_mpo_site* w, const void* R, const void* B, void* R_out,
                                int32_t prec, dm_stream stream) {
  return guarded([&] {
    check_ly(ly);
    const bool real = take_real(prec);
    check_prec(prec);
    Bond bb = make_bond(b, ly), bc = make_bond(c, ly);
    MpoSite W = make_mpo(w, ly);
    EnvRLayout Ri = envr_layout(bc, W.qr, ly);
    EnvRLayout Ro = envr_layout(bb, W.ql, ly);
    SiteLayout S = site_layout(bb, bc, W.qs, ly);
    if ((Ri.P.total && !R) || (S.P.total && !B) || (Ro.P.total && !R_out))
      throw DmError{DM_ERR_ARG, "null tensor"};
    EnvPlan ep = plan_right(ly, bb, bc, W, Ri, S, Ro, env_t3_tile(prec), env_t1r_tile_n(prec));
    validate(ep.t1, Ri.P.total, S.P.total, ep.t1total);
    validate(ep.mix, ep.t1total, ep.t2total);
    validate(ep.t3, S.P.total, ep.t2total, Ro.P.total);
    if (real) make_real(ep);
    EnvScratch pool;
    run_env(ep, R, Ri.P.total, B, S.P.total, R_out, Ro.P.total, prec, real, (hipStream_t)stream, pool);
  });
}

extern "C" int dm_env_flops(int32_t left, int32_t ly, const dm_bond* x, const dm_bond* y,
                            const dm_mpo_site* w, double* flops) {
  return guarded([&] {
    if (!flops) throw DmError{DM_ERR_ARG, "null output"};
    check_ly(ly);
    Bond bx = make_bond(x, ly), by = make_bond(y, ly);
    MpoSite W = make_mpo(w, ly);
    if (left) {
      EnvLLayout Li = envl_layout(bx, W.ql, ly), Lo = envl_layout(by, W.qr, ly);
      SiteLayout S = site_layout(bx, by, W.qs, ly);
      *flops = plan_left(ly, bx, by, W, Li, S, Lo, 64).flops();
    } else {
      EnvRLayout Ri = envr_layout(by, W.qr, ly), Ro = envr_layout(bx, W.ql, ly);
      SiteLayout S = site_layout(bx, by, W.qs, ly);
      *flops = plan_right(ly, bx, by, W, Ri, S, Ro, 64, 64).flops();
    }
  });
}



// =====================================================================================
// Left environment update that allocates nothing
// =====================================================================================
// The task tables and intermediates of env_update_left_noalloc live in one fixed device
// array of this size; every device the library runs on holds its own copy of it until
// the process ends.  Host code never passes the array's name to a kernel or a copy: it
// uses the device address hipGetSymbolAddress returns for the current device.
static constexpr size_t kNoallocScratchBytes = size_t(64) << 20;
static __device__ __align__(256) char scratch[kNoallocScratchBytes];

namespace {
std::mutex g_scratch_mu;
std::map<int, char*> g_scratch_ptr;  // device -> address of its copy of `scratch`

// Address of the current device's copy of `scratch`, looked up once per device.
char* scratch_on_current_device() {
  int dev = 0;
  HIPCHK(hipGetDevice(&dev));
  std::lock_guard<std::mutex> g(g_scratch_mu);
  auto it = g_scratch_ptr.find(dev);
  if (it != g_scratch_ptr.end()) return it->second;
  char* ptr = nullptr;
  HIPCHK(hipGetSymbolAddress((void**)&ptr, HIP_SYMBOL(scratch)));
  if (!ptr) throw DmError{DM_ERR_HIP, "hipGetSymbolAddress returned no address for the scratch array"};
  g_scratch_ptr[dev] = ptr;
  return ptr;
}
}  // namespace

static int env_update_left_noalloc_impl(int32_t ly, const dm_bond* a, const dm_bond* b,
                                       const dm_mpo_site* w, const void* L, const void* A,
                                       void* L_out, int32_t prec, dm_stream stream);

extern "C" int env_update_left_noalloc(int32_t ly, const dm_bond* a, const dm_bond* b,
                                       const dm_mpo_site* w, const void* L, const void* A,
                                       void* L_out, int32_t prec, dm_stream stream) {
  const int rc = env_update_left_noalloc_impl(ly, a, b, w, L, A, L_out, prec, stream);
  if (rc != DM_OK) drain(stream);  // no queued work outlives the error
  return rc;
}

static int env_update_left_noalloc_impl(int32_t ly, const dm_bond* a, const dm_bond* b,
                                       const dm_mpo_site* w, const void* L, const void* A,
                                       void* L_out, int32_t prec, dm_stream stream) {
  return guarded([&] {
    check_ly(ly);
    const bool real = take_real(prec);
    check_prec(prec);
    Bond ba = make_bond(a, ly), bb = make_bond(b, ly);
    MpoSite W = make_mpo(w, ly);
    EnvLLayout Li = envl_layout(ba, W.ql, ly);
    EnvLLayout Lo = envl_layout(bb, W.qr, ly);
    SiteLayout S = site_layout(ba, bb, W.qs, ly);
    if ((Li.P.total && !L) || (S.P.total && !A) || (Lo.P.total && !L_out))
      throw DmError{DM_ERR_ARG, "null tensor"};
    EnvPlan ep = plan_left(ly, ba, bb, W, Li, S, Lo, env_t3_tile(prec));
    validate(ep.t1, Li.P.total, S.P.total, ep.t1total);
    validate(ep.mix, ep.t1total, ep.t2total);
    validate(ep.t3, S.P.total, ep.t2total, Lo.P.total);
    if (real) make_real(ep);
    // the whole footprint is checked before any work is queued
    TableUpload probe;
    probe.add(ep.t1);
    probe.add(ep.t3);
    probe.add(ep.mix);
    const size_t need = env_scratch_bytes(ep, probe.total, Li.P.total, S.P.total, Lo.P.total, prec, real);
    if (need > kNoallocScratchBytes)
      throw DmError{DM_ERR_ALLOC, "env_update_left_noalloc needs " + std::to_string(need) +
                                      " bytes of scratch; its fixed region holds " +
                                      std::to_string(kNoallocScratchBytes)};
    EnvScratch fixed;
    fixed.base = scratch_on_current_device();
    fixed.cap = kNoallocScratchBytes;
    run_env(ep, L, Li.P.total, A, S.P.total, L_out, Lo.P.total, prec, real, (hipStream_t)stream, fixed);
  });
}
