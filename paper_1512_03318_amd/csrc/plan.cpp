// Host planner: bond / MPO validation and the canonical layouts.
#include "plan.hpp"

#include <climits>

#include <algorithm>
#include <cmath>
#include <sstream>

namespace mrd {

static DmError err(int code, const std::string& m) { return DmError{code, m}; }

Bond make_bond(const dm_bond* b, int ly) {
  if (!b) throw err(DM_ERR_ARG, "null bond");
  if (b->nsec < 0 || (b->nsec > 0 && (!b->q || !b->dim))) throw err(DM_ERR_ARG, "bad bond arrays");
  Bond out;
  out.ly = ly;
  for (int i = 0; i < b->nsec; ++i) {
    const dm_charge q = b->q[i];
    if (q.k < 0 || q.k >= ly) {
      std::ostringstream s;
      s << "bond sector " << i << " has k=" << q.k << " outside [0," << ly << ")";
      throw err(DM_ERR_CHARGE, s.str());
    }
    if (b->dim[i] <= 0) throw err(DM_ERR_DIM, "bond sector with non-positive dimension");
    if (i > 0) {
      const dm_charge p = b->q[i - 1];
      if (!(p.n < q.n || (p.n == q.n && p.k < q.k)))
        throw err(DM_ERR_ARG, "bond sectors must be strictly increasing in (n, k)");
    }
    out.q.push_back(q);
    out.dim.push_back(b->dim[i]);
  }
  if (b->nsec > 0) {
    out.nlo = out.q.front().n;
    const int64_t span = (int64_t)out.q.back().n - out.nlo + 1;
    if (span * ly <= std::max<int64_t>(4096, 16 * (int64_t)b->nsec)) {
      out.nspan = span;
      out.lut.assign((size_t)(span * ly), -1);
      for (int i = 0; i < b->nsec; ++i)
        out.lut[(size_t)((int64_t)out.q[i].n - out.nlo) * ly + out.q[i].k] = i;
    }
  }
  return out;
}

MpoSite make_mpo(const dm_mpo_site* m, int ly) {
  if (!m || !m->w || !m->ql || !m->qr || m->dl <= 0 || m->dr <= 0)
    throw err(DM_ERR_ARG, "bad MPO site tensor");
  MpoSite o;
  o.dl = m->dl;
  o.dr = m->dr;
  o.ql.assign(m->ql, m->ql + m->dl);
  o.qr.assign(m->qr, m->qr + m->dr);
  o.qs[0] = m->qs[0];
  o.qs[1] = m->qs[1];
  for (auto* v : {&o.ql, &o.qr})
    for (auto& q : *v)
      if (q.k < 0 || q.k >= ly) throw err(DM_ERR_CHARGE, "MPO state charge k outside [0, ly)");
  for (int s = 0; s < 2; ++s)
    if (o.qs[s].k < 0 || o.qs[s].k >= ly) throw err(DM_ERR_CHARGE, "local charge k outside [0, ly)");
  const size_t n = (size_t)o.dl * 4 * o.dr;
  o.w.resize(n);
  for (size_t i = 0; i < n; ++i) {
    const double re = m->w[2 * i], im = m->w[2 * i + 1];
    if (!std::isfinite(re) || !std::isfinite(im)) throw err(DM_ERR_NONFINITE, "non-finite MPO entry");
    o.w[i] = {re, im};
  }
  for (int a = 0; a < o.dl; ++a)
    for (int sp = 0; sp < 2; ++sp)
      for (int s = 0; s < 2; ++s)
        for (int b = 0; b < o.dr; ++b) {
          if (o.at(a, sp, s, b) == std::complex<double>(0, 0)) continue;
          const dm_charge want = qsub(qadd(o.ql[a], o.qs[sp], ly), o.qs[s], ly);
          if (!qeq(want, o.qr[b])) {
            std::ostringstream st;
            st << "MPO entry W[" << a << "," << sp << "," << s << "," << b
               << "] breaks q(w') = q(w) + q(s') - q(s)";
            throw err(DM_ERR_CHARGE, st.str());
          }
        }
  return o;
}

SiteLayout site_layout(const Bond& a, const Bond& b, const dm_charge qs[2], int ly) {
  SiteLayout L;
  for (int i = 0; i < a.size(); ++i) {
    std::array<int, 2> bi{-1, -1}, co{0, 0};
    int cols = 0;
    for (int s = 0; s < 2; ++s) {
      const int j = b.find(qadd(a.q[i], qs[s], ly));
      if (j < 0) continue;
      bi[s] = j;
      co[s] = cols;
      cols += b.dim[j];
    }
    L.b.push_back(bi);
    L.coff.push_back(co);
    L.P.push(a.dim[i], cols);
  }
  return L;
}

ThetaLayout theta_layout(const Bond& a, const Bond& c, const dm_charge qs1[2],
                         const dm_charge qs2[2], int ly) {
  ThetaLayout L;
  for (int i = 0; i < a.size(); ++i) {
    std::array<int, 4> ci{-1, -1, -1, -1}, co{0, 0, 0, 0};
    int cols = 0;
    for (int s12 = 0; s12 < 4; ++s12) {
      const int j = c.find(qadd(qadd(a.q[i], qs1[s12 >> 1], ly), qs2[s12 & 1], ly));
      if (j < 0) continue;
      ci[s12] = j;
      co[s12] = cols;
      cols += c.dim[j];
    }
    L.c.push_back(ci);
    L.coff.push_back(co);
    L.P.push(a.dim[i], cols);
  }
  return L;
}

EnvLLayout envl_layout(const Bond& a, const std::vector<dm_charge>& qw, int ly) {
  EnvLLayout L;
  L.D = (int)qw.size();
  for (int i = 0; i < a.size(); ++i) {
    int rows = 0;
    for (int w = 0; w < L.D; ++w) {
      const int j = a.find(qadd(a.q[i], qw[w], ly));
      L.ap.push_back(j);
      L.roff.push_back(j < 0 ? -1 : rows);
      if (j >= 0) rows += a.dim[j];
    }
    L.P.push(rows, a.dim[i]);
  }
  return L;
}

EnvRLayout envr_layout(const Bond& c, const std::vector<dm_charge>& qw, int ly) {
  EnvRLayout L;
  L.D = (int)qw.size();
  for (int i = 0; i < c.size(); ++i) {
    int cols = 0;
    for (int w = 0; w < L.D; ++w) {
      const int j = c.find(qsub(c.q[i], qw[w], ly));
      L.c.push_back(j);
      L.coff.push_back(j < 0 ? -1 : cols);
      if (j >= 0) cols += c.dim[j];
    }
    L.P.push(c.dim[i], cols);
  }
  return L;
}

void add_tiles(GemmStage& st, int32_t prob, int M, int N) {
  const int TM = st.tile_m, TN = st.tile_n;
  const int tm = (M + TM - 1) / TM, tn = (N + TN - 1) / TN;
  if (M > 0 && N == 0) return;
  GemmProb& P = st.probs[prob];
  P.nks = 1;
  P.slot0 = -1;
  if (st.split) {
    // split long K over several workgroups: at least split_min chunks per split, at most 8
    int chunks = 0;
    for (int q = 0; q < P.nseg; ++q) chunks += (st.segs[P.seg0 + q].k + st.kc - 1) / st.kc;
    P.nks = std::max(1, std::min(8, chunks / std::max(1, st.split_min)));
    if (P.nks > 1) {  // partial tile of (tm, tn, ks): slot0 + (tm * tiles_n + tn) * nks + ks
      P.slot0 = (int32_t)st.nslots;
      st.nslots += (int64_t)tm * tn * P.nks;
    }
  }
  for (int a = 0; a < tm; ++a)
    for (int b = 0; b < tn; ++b) {
      for (int ks = 0; ks < P.nks; ++ks) st.tiles.push_back({prob, a, b, ks});
      if (P.nks > 1) st.red_tiles.push_back({prob, a, b, 0});
    }
}

static void range_check(int64_t lo, int64_t hi, int64_t size, const char* what) {
  if (lo < 0 || hi >= size) {
    std::ostringstream s;
    s << "internal task table out of bounds (" << what << ": [" << lo << ", " << hi << "] of " << size << ")";
    throw err(DM_ERR_LAYOUT, s.str());
  }
}

void validate(const GemmStage& st, int64_t a_size, int64_t b_size, int64_t c_size) {
  for (const std::vector<GemmTile>* tl : {&st.tiles, &st.red_tiles})
    for (const GemmTile& t : *tl) {
      if (t.prob < 0 || t.prob >= (int)st.probs.size()) throw err(DM_ERR_LAYOUT, "bad tile");
      const GemmProb& p = st.probs[t.prob];
      // the split reduction sums at most 8 partial tiles per output tile
      if (t.ks < 0 || t.ks >= std::max(1, p.nks) || p.nks > 8) throw err(DM_ERR_LAYOUT, "bad K-split");
      if (p.nks > 1) {
        const int tn = (p.N + st.tile_n - 1) / st.tile_n;
        const int64_t slot = (int64_t)p.slot0 + ((int64_t)t.tm * tn + t.tn) * p.nks + t.ks;
        if (!st.split || p.slot0 < 0 || slot >= st.nslots) throw err(DM_ERR_LAYOUT, "bad partial slot");
      }
    }
  for (const GemmTile& t : st.tiles) {
    const GemmProb& p = st.probs[t.prob];
    if (t.tm * st.tile_m >= p.M || t.tn * st.tile_n >= p.N)
      throw err(DM_ERR_LAYOUT, "empty tile");
  }
  for (const GemmProb& p : st.probs) {
    if (p.M <= 0 || p.N <= 0) throw err(DM_ERR_LAYOUT, "empty problem");
    if (p.seg0 < 0 || p.nseg < 0 || p.seg0 + p.nseg > (int)st.segs.size()) throw err(DM_ERR_LAYOUT, "bad segments");
    const bool arow = st.flags & G_A_ROWMAP, crow = st.flags & G_C_ROWMAP;
    if ((arow || crow) && (p.rowmap < 0 || p.rowmap + p.M > (int64_t)st.rows.size()))
      throw err(DM_ERR_LAYOUT, "bad row table");
    // lowest and highest row offset of a row table: every row's range lies between the
    // range of the lowest and that of the highest
    int64_t rlo = 0, rhi = 0;
    if (arow || crow) {
      rlo = rhi = st.rows[p.rowmap];
      for (int i = 1; i < p.M; ++i) {
        rlo = std::min(rlo, st.rows[p.rowmap + i]);
        rhi = std::max(rhi, st.rows[p.rowmap + i]);
      }
    }
    for (int q = 0; q < p.nseg; ++q) {
      const GemmSeg& g = st.segs[p.seg0 + q];
      if (g.k < 0) throw err(DM_ERR_LAYOUT, "negative K");
      if (g.k == 0) continue;
      if (arow) {
        range_check(rlo + g.a_off, rhi + g.a_off + g.k - 1, a_size, "A");
      } else if (st.flags & G_A_T) {
        range_check(g.a_off, g.a_off + (int64_t)(g.k - 1) * g.lda + p.M - 1, a_size, "A");
        if (g.lda < p.M) throw err(DM_ERR_LAYOUT, "lda");
      } else {
        range_check(g.a_off, g.a_off + (int64_t)(p.M - 1) * g.lda + g.k - 1, a_size, "A");
        if (g.lda < g.k) throw err(DM_ERR_LAYOUT, "lda");
      }
      if (st.flags & G_B_T) {
        range_check(g.b_off, g.b_off + (int64_t)(p.N - 1) * g.ldb + g.k - 1, b_size, "B");
        if (g.ldb < g.k) throw err(DM_ERR_LAYOUT, "ldb");
      } else {
        range_check(g.b_off, g.b_off + (int64_t)(g.k - 1) * g.ldb + p.N - 1, b_size, "B");
        if (g.ldb < p.N) throw err(DM_ERR_LAYOUT, "ldb");
      }
    }
    if (crow) {
      range_check(rlo, rhi + p.N - 1, c_size, "C");
    } else {
      range_check(p.c_off, p.c_off + (int64_t)(p.M - 1) * p.ldc + p.N - 1, c_size, "C");
      if (p.ldc < p.N) throw err(DM_ERR_LAYOUT, "ldc");
    }
  }
}

void mix_to_slabs(MixStage& st, const std::vector<int64_t>& key, int eb, int lds_budget) {
  st.wgs.clear();
  st.blks.clear();
  st.stasks.clear();
  st.coefs.clear();
  st.lds_bytes = 0;
  st.slab_eb = eb;
  if (key.size() != st.tasks.size()) throw err(DM_ERR_LAYOUT, "mixing slab keys");
  std::vector<int> ord(st.tasks.size());
  for (size_t i = 0; i < ord.size(); ++i) ord[i] = (int)i;
  if (!std::is_sorted(key.begin(), key.end()))
    std::stable_sort(ord.begin(), ord.end(), [&](int x, int y) { return key[x] < key[y]; });
  st.blks.reserve(st.srcs.size());
  st.coefs.reserve(st.srcs.size());
  st.stasks.reserve(st.tasks.size());
  st.wgs.reserve(2 * st.tasks.size());
  for (size_t i = 0; i < ord.size();) {
    size_t j = i;
    while (j < ord.size() && key[ord[j]] == key[ord[i]]) ++j;
    const MixTask& t0 = st.tasks[ord[i]];
    const int rows = t0.rows, cols = t0.cols;
    const int32_t blk0 = (int32_t)st.blks.size(), task0 = (int32_t)st.stasks.size();
    for (size_t q = i; q < j; ++q) {
      const MixTask& t = st.tasks[ord[q]];
      if (t.rows != rows || t.cols != cols) throw err(DM_ERR_LAYOUT, "mixing slab shapes differ");
      SlabTask out{t.dst, t.ld_dst, (int32_t)st.coefs.size(), t.nsrc, t.pstride};
      for (int k = 0; k < t.nsrc; ++k) {
        const MixSrc& m = st.srcs[t.src0 + k];
        // block index of this source in the slab (a slab has few blocks: linear search)
        int32_t b = 0;
        const int32_t nb = (int32_t)(st.blks.size() - blk0);
        while (b < nb && st.blks[blk0 + b].off != m.off) ++b;
        if (b == nb) st.blks.push_back({m.off, m.ld, 0});
        else if (st.blks[blk0 + b].ld != m.ld) throw err(DM_ERR_LAYOUT, "mixing slab ld differs");
        st.coefs.push_back({b, 0, m.re, m.im});
      }
      st.stasks.push_back(out);
    }
    const int nblk = (int)(st.blks.size() - blk0);
    // largest column chunk, then row chunk, that fit the LDS budget
    const int64_t per_elem = (int64_t)std::max(1, nblk) * eb;
    int ncol = (int)std::min<int64_t>(cols, std::max<int64_t>(1, lds_budget / per_elem));
    int nr = (int)std::min<int64_t>(rows, std::max<int64_t>(1, lds_budget / (per_elem * ncol)));
    nr = std::min(nr, 16);
    for (int r0 = 0; r0 < rows; r0 += nr)
      for (int c0 = 0; c0 < cols; c0 += ncol) {
        const int wr = std::min(nr, rows - r0), wc = std::min(ncol, cols - c0);
        st.wgs.push_back({blk0, nblk, task0, (int32_t)(j - i), r0, wr, c0, wc});
        st.lds_bytes = std::max<int32_t>(st.lds_bytes, (int32_t)(per_elem * wr * wc));
      }
    i = j;
  }
}

void add_ps_tiles(PsStage& st, int32_t prob) {
  PsProb& P = st.probs[prob];
  const int tm = (P.M + st.tile_m - 1) / st.tile_m, tn = (P.N + st.tile_n - 1) / st.tile_n;
  P.nks = 1;
  P.slot0 = -1;
  if (P.M <= 0 || P.N <= 0) return;
  if (st.split) {
    const int chunks = (P.kp + 31) / 32;
    P.nks = std::max(1, std::min(8, chunks / std::max(1, st.split_min)));
    if (P.nks > 1) {
      P.slot0 = (int32_t)st.nslots;
      st.nslots += (int64_t)tm * tn * P.nks;
    }
  }
  for (int a = 0; a < tm; ++a)
    for (int b = 0; b < tn; ++b) {
      for (int ks = 0; ks < P.nks; ++ks) st.tiles.push_back({prob, a, b, ks});
      if (P.nks > 1) st.red_tiles.push_back({prob, a, b, 0});
    }
}

static void validate_sk(const PsStage& st);

void validate(const PsStage& st, int64_t a_size, int64_t b_size, int64_t c_size) {
  for (const std::vector<GemmTile>* tl : {&st.tiles, &st.red_tiles})
    for (const GemmTile& t : *tl) {
      if (t.prob < 0 || t.prob >= (int)st.probs.size()) throw err(DM_ERR_LAYOUT, "bad tile");
      const PsProb& p = st.probs[t.prob];
      // the split reduction sums at most 8 partial tiles per output tile
      if (t.ks < 0 || t.ks >= std::max(1, p.nks) || p.nks > 8) throw err(DM_ERR_LAYOUT, "bad K-split");
      if (t.tm < 0 || t.tn < 0 || t.tm * st.tile_m >= p.M || t.tn * st.tile_n >= p.N)
        throw err(DM_ERR_LAYOUT, "empty tile");
      if (p.nks > 1) {
        const int tn = (p.N + st.tile_n - 1) / st.tile_n;
        const int64_t slot = (int64_t)p.slot0 + ((int64_t)t.tm * tn + t.tn) * p.nks + t.ks;
        if (!st.split || p.slot0 < 0 || slot >= st.nslots) throw err(DM_ERR_LAYOUT, "bad partial slot");
      }
    }
  for (const PsProb& p : st.probs) {
    if (p.M <= 0 || p.N <= 0 || p.kp <= 0 || p.kp % 8) throw err(DM_ERR_LAYOUT, "bad pre-split problem");
    // 16-byte loads: every offset and stride a multiple of 8 bf16
    if (p.a_off % 8 || p.b_off % 8 || p.a_ps % 8 || p.b_ps % 8) throw err(DM_ERR_LAYOUT, "pre-split alignment");
    if (p.a_ps < (int64_t)p.M * p.kp || p.b_ps < (int64_t)p.N * p.kp) throw err(DM_ERR_LAYOUT, "pre-split planes overlap");
    range_check(p.a_off, p.a_off + 3 * p.a_ps + (int64_t)p.M * p.kp - 1, a_size, "pre-split A");
    range_check(p.b_off, p.b_off + 3 * p.b_ps + (int64_t)p.N * p.kp - 1, b_size, "pre-split B");
    if (st.cout == 1) {
      if (p.rowmap < 0 || p.rowmap + p.M > (int64_t)st.rows.size()) throw err(DM_ERR_LAYOUT, "bad row table");
      for (int i = 0; i < p.M; ++i) {
        const int64_t r = st.rows[p.rowmap + i];
        range_check(r, r + p.N - 1, c_size, "pre-split C row");
      }
    } else {
      if (p.ldc < p.N) throw err(DM_ERR_LAYOUT, "pre-split ldc");
      range_check(p.c_off, p.c_off + (int64_t)(p.M - 1) * p.ldc + p.N - 1, c_size, "pre-split C");
    }
  }
  validate_sk(st);
}

void sk_schedule(PsStage& st, int grid) {
  st.sk_tiles.clear();
  st.sk_segs.clear();
  st.sk_wg.assign(1, 0);
  st.sk_red.clear();
  st.sk_nslots = 0;
  st.sk_grid = 0;
  // tiles in problem order, each with its chunk count; chunk sequence offsets
  std::vector<int64_t> first;
  int64_t total = 0;
  for (int32_t q = 0; q < (int32_t)st.probs.size(); ++q) {
    const PsProb& p = st.probs[q];
    if (p.M <= 0 || p.N <= 0 || p.kp <= 0 || p.kp % SK_KC) throw err(DM_ERR_LAYOUT, "bad stream-K problem");
    const int tm = (p.M + SK_BM - 1) / SK_BM, tn = (p.N + SK_BN - 1) / SK_BN;
    for (int a = 0; a < tm; ++a)
      for (int b = 0; b < tn; ++b) {
        st.sk_tiles.push_back({q, a, b, p.kp / SK_KC, -1, 0});
        first.push_back(total);
        total += p.kp / SK_KC;
      }
  }
  if (total == 0) return;
  const int g = (int)std::max<int64_t>(1, std::min<int64_t>(grid, total));
  st.sk_grid = g;
  // workgroup w: chunks [w * total / g, (w + 1) * total / g), cut at tile boundaries
  size_t t = 0;
  for (int w = 0; w < g; ++w) {
    int64_t lo = total * w / g;
    const int64_t hi = total * (w + 1) / g;
    while (lo < hi) {
      while (first[t] + st.sk_tiles[t].nch <= lo) ++t;
      const int64_t end = std::min(hi, first[t] + st.sk_tiles[t].nch);
      st.sk_segs.push_back({(int32_t)t, (int32_t)(lo - first[t]), (int32_t)(end - first[t]), -1});
      st.sk_tiles[t].nseg++;
      lo = end;
    }
    st.sk_wg.push_back((int32_t)st.sk_segs.size());
  }
  // partial slots of split tiles, in K order within each tile
  for (size_t i = 0; i < st.sk_tiles.size(); ++i)
    if (st.sk_tiles[i].nseg > 1) {
      st.sk_tiles[i].slot0 = (int32_t)st.sk_nslots;
      st.sk_nslots += st.sk_tiles[i].nseg;
      st.sk_red.push_back((int32_t)i);
    }
  std::vector<int32_t> seen(st.sk_tiles.size(), 0);
  for (SkSeg& sg : st.sk_segs) {  // segments of one tile appear in K order
    const SkTile& tl = st.sk_tiles[sg.tile];
    if (tl.nseg > 1) sg.slot = tl.slot0 + seen[sg.tile];
    seen[sg.tile]++;
  }
  st.sk_jobs.clear();
  st.sk_jobs.reserve(st.sk_segs.size());
  for (const SkSeg& sg : st.sk_segs) {
    const SkTile& tl = st.sk_tiles[sg.tile];
    const PsProb& p = st.probs[tl.prob];
    st.sk_jobs.push_back({p.a_off, p.b_off, p.a_ps, p.b_ps, p.c_off, p.M, p.N, p.kp, p.ldc, p.rowmap,
                          tl.tm * SK_BM, tl.tn * SK_BN, sg.c0, sg.c1, sg.slot});
  }
}

// The stream-K schedule covers every chunk of every tile exactly once, in K order
// within each tile; slots and tables are in range.
static void validate_sk(const PsStage& st) {
  if (st.sk_tiles.empty()) return;
  if (st.sk_grid <= 0 || (int)st.sk_wg.size() != st.sk_grid + 1 || st.sk_wg[0] != 0 ||
      st.sk_wg.back() != (int32_t)st.sk_segs.size())
    throw err(DM_ERR_LAYOUT, "bad stream-K workgroup table");
  for (size_t w = 0; w + 1 < st.sk_wg.size(); ++w)
    if (st.sk_wg[w] > st.sk_wg[w + 1]) throw err(DM_ERR_LAYOUT, "bad stream-K workgroup table");
  std::vector<int32_t> next(st.sk_tiles.size(), 0), nseg(st.sk_tiles.size(), 0);
  for (const SkSeg& sg : st.sk_segs) {
    if (sg.tile < 0 || sg.tile >= (int32_t)st.sk_tiles.size()) throw err(DM_ERR_LAYOUT, "bad stream-K segment");
    const SkTile& tl = st.sk_tiles[sg.tile];
    if (sg.c0 != next[sg.tile] || sg.c1 <= sg.c0 || sg.c1 > tl.nch) throw err(DM_ERR_LAYOUT, "bad stream-K segment");
    next[sg.tile] = sg.c1;
    if (tl.nseg > 1 ? (sg.slot != tl.slot0 + nseg[sg.tile] || sg.slot < 0 || sg.slot >= st.sk_nslots) : sg.slot != -1)
      throw err(DM_ERR_LAYOUT, "bad stream-K slot");
    nseg[sg.tile]++;
  }
  for (size_t i = 0; i < st.sk_tiles.size(); ++i) {
    const SkTile& tl = st.sk_tiles[i];
    if (tl.prob < 0 || tl.prob >= (int32_t)st.probs.size()) throw err(DM_ERR_LAYOUT, "bad stream-K tile");
    const PsProb& p = st.probs[tl.prob];
    if (p.kp % SK_KC || tl.nch != p.kp / SK_KC || next[i] != tl.nch || nseg[i] != tl.nseg || tl.tm < 0 ||
        tl.tn < 0 || tl.tm * SK_BM >= p.M || tl.tn * SK_BN >= p.N)
      throw err(DM_ERR_LAYOUT, "bad stream-K tile");
  }
  for (int32_t r : st.sk_red)
    if (r < 0 || r >= (int32_t)st.sk_tiles.size() || st.sk_tiles[r].nseg < 2) throw err(DM_ERR_LAYOUT, "bad stream-K reduction");
  // the job records repeat their segment, tile and problem
  if (st.sk_jobs.size() != st.sk_segs.size()) throw err(DM_ERR_LAYOUT, "bad stream-K jobs");
  for (size_t q = 0; q < st.sk_segs.size(); ++q) {
    const SkSeg& sg = st.sk_segs[q];
    const SkTile& tl = st.sk_tiles[sg.tile];
    const PsProb& p = st.probs[tl.prob];
    const SkJob& j = st.sk_jobs[q];
    if (j.a_off != p.a_off || j.b_off != p.b_off || j.a_ps != p.a_ps || j.b_ps != p.b_ps || j.c_off != p.c_off ||
        j.M != p.M || j.N != p.N || j.kp != p.kp || j.ldc != p.ldc || j.rowmap != p.rowmap ||
        j.i0 != tl.tm * SK_BM || j.j0 != tl.tn * SK_BN || j.c0 != sg.c0 || j.c1 != sg.c1 || j.slot != sg.slot)
      throw err(DM_ERR_LAYOUT, "bad stream-K job");
  }
}

int64_t split_layout(std::vector<SplitJob>& jobs) {
  int64_t n = 0;
  for (SplitJob& j : jobs) {
    j.i0 = n;
    const int drows = j.trans ? j.cols : j.rows, ng = j.kp / 8;
    if (j.trans)  // blocks of 16 rows x 4 groups (split_kernel), partial blocks padded
      n += (int64_t)((drows + 15) / 16) * ((ng + 3) / 4) * 64;
    else
      n += (int64_t)drows * ng;
  }
  return n;
}

void validate(const std::vector<SplitJob>& jobs, int64_t src_size, int64_t dst_size) {
  for (const SplitJob& j : jobs) {
    if (j.rows <= 0 || j.cols <= 0 || j.ld < j.cols || j.kp % 8 || j.pstride < 0)
      throw err(DM_ERR_LAYOUT, "bad split job");
    const int drows = j.trans ? j.cols : j.rows, k = j.trans ? j.rows : j.cols;
    if (j.kp < k || (int64_t)j.pstride < (int64_t)drows * j.kp || j.dst % 8 || j.pstride % 8)
      throw err(DM_ERR_LAYOUT, "bad split job");
    range_check(j.src, j.src + (int64_t)(j.rows - 1) * j.ld + j.cols - 1, src_size, "split src");
    range_check(j.dst, j.dst + 3 * (int64_t)j.pstride + (int64_t)drows * j.kp - 1, dst_size, "split dst");
  }
}

void validate(const MixStage& st, int64_t src_size, int64_t dst_size) {
  for (const MixTask& t : st.tasks) {
    if (t.rows <= 0 || t.cols <= 0) throw err(DM_ERR_LAYOUT, "empty mixing task");
    if (t.pstride < 0) throw err(DM_ERR_LAYOUT, "mix plane stride");
    range_check(t.dst, t.dst + 3 * (int64_t)t.pstride + (int64_t)(t.rows - 1) * t.ld_dst + t.cols - 1,
                dst_size, "mix dst");
    if (t.ld_dst < t.cols) throw err(DM_ERR_LAYOUT, "mix ld");
    if (t.src0 < 0 || t.nsrc < 0 || t.src0 + t.nsrc > (int)st.srcs.size()) throw err(DM_ERR_LAYOUT, "mix sources");
    for (int q = 0; q < t.nsrc; ++q) {
      const MixSrc& s = st.srcs[t.src0 + q];
      range_check(s.off, s.off + (int64_t)(t.rows - 1) * s.ld + t.cols - 1, src_size, "mix src");
      if (s.ld < t.cols) throw err(DM_ERR_LAYOUT, "mix src ld");
    }
  }
  // slab form: every workgroup's chunk inside its blocks and tasks, coefficients in range.
  // The workgroups of one slab (consecutive, same blocks and tasks) are checked together:
  // the blocks and tasks once, over the union of the workgroups' row and column ranges
  // (an element range that holds the union's first and last elements holds every part).
  for (size_t i = 0; i < st.wgs.size();) {
    const SlabWG& g0 = st.wgs[i];
    int rmin = INT32_MAX, rmax = -1, cmin = INT32_MAX, cmax = -1;
    size_t j = i;
    for (; j < st.wgs.size() && st.wgs[j].blk0 == g0.blk0 && st.wgs[j].nblk == g0.nblk &&
           st.wgs[j].task0 == g0.task0 && st.wgs[j].ntask == g0.ntask; ++j) {
      const SlabWG& g = st.wgs[j];
      if (g.r0 < 0 || g.nr <= 0 || g.col0 < 0 || g.ncol <= 0) throw err(DM_ERR_LAYOUT, "bad mixing slab");
      if ((int64_t)g.nblk * g.nr * g.ncol * st.slab_eb > st.lds_bytes) throw err(DM_ERR_LAYOUT, "mixing slab LDS");
      rmin = std::min(rmin, g.r0);
      rmax = std::max(rmax, g.r0 + g.nr - 1);
      cmin = std::min(cmin, g.col0);
      cmax = std::max(cmax, g.col0 + g.ncol - 1);
    }
    if (g0.blk0 < 0 || g0.nblk < 0 || g0.blk0 + g0.nblk > (int64_t)st.blks.size() || g0.task0 < 0 ||
        g0.ntask < 0 || g0.task0 + g0.ntask > (int64_t)st.stasks.size())
      throw err(DM_ERR_LAYOUT, "bad mixing slab");
    for (int b = 0; b < g0.nblk; ++b) {
      const SlabBlk& k = st.blks[g0.blk0 + b];
      if (k.ld <= cmax) throw err(DM_ERR_LAYOUT, "mixing slab block ld");
      range_check(k.off + (int64_t)rmin * k.ld + cmin, k.off + (int64_t)rmax * k.ld + cmax, src_size, "slab src");
    }
    for (int t = 0; t < g0.ntask; ++t) {
      const SlabTask& k = st.stasks[g0.task0 + t];
      if (k.ld_dst <= cmax) throw err(DM_ERR_LAYOUT, "mixing slab task ld");
      if (k.pstride < 0) throw err(DM_ERR_LAYOUT, "slab plane stride");
      range_check(k.dst + (int64_t)rmin * k.ld_dst + cmin,
                  k.dst + 3 * (int64_t)k.pstride + (int64_t)rmax * k.ld_dst + cmax, dst_size, "slab dst");
      if (k.c0 < 0 || k.nc < 0 || k.c0 + k.nc > (int64_t)st.coefs.size()) throw err(DM_ERR_LAYOUT, "slab coefficients");
      for (int q = 0; q < k.nc; ++q)
        if (st.coefs[k.c0 + q].blk < 0 || st.coefs[k.c0 + q].blk >= g0.nblk) throw err(DM_ERR_LAYOUT, "slab block index");
    }
    i = j;
  }
}

}  // namespace mrd
