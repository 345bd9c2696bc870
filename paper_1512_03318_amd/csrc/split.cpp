// Two-site split: block SVD truncation of theta at its middle bond (dm_theta_split).
//
// theta[a, s1, s2, c] is a matrix M_b[(a, s1), (s2, c)] per middle charge q(b) = q(a) +
// q(s1) (Sec. III C: the Schmidt states carry (N, k)).  Each sector matrix is gathered
// from theta's blocks into a column-major workspace (transposed and conjugated when it
// is wider than tall), factorised by the one-sided Jacobi kernel (svd.hip), and the
// kept singular vectors are scattered into the two new site tensors.  Which values are
// kept is decided on the host from the singular values alone: the chi largest over all
// sectors, ties broken by (sector, rank within the sector), none at or below the
// cutoff, renormalised to a unit sum of squares (the same rule as the oracle's split).
#include <algorithm>
#include <cmath>
#include <map>
#include <tuple>

#include "runtime.hpp"
#include "svd.hpp"

using namespace mrd;

namespace {

struct Sector {
  dm_charge q;
  std::vector<std::pair<int, int>> rows;  // (a sector, s1), increasing
  std::vector<std::pair<int, int>> cols;  // (s2, c sector), increasing
  std::vector<int> roff, coff;
  int m = 0, n = 0;                       // rows, columns of M
  bool trans = false;                      // workspace holds M^H
  int64_t w_off = 0, v_off = 0, sig_off = 0;
  int wm() const { return trans ? n : m; }  // workspace rows
  int wn() const { return trans ? m : n; }  // workspace columns (<= rows)
};

// Host check that every element a copy job touches lies inside its buffers (sizes in
// complex elements; perm / scale tables of the given lengths, permuted indices in range).
void validate_copies(const std::vector<CopyJob>& jobs, int64_t src_size, int64_t dst_size,
                     const std::vector<int32_t>& perm, size_t nscale, int64_t src_rows, int64_t src_cols) {
  for (const CopyJob& j : jobs) {
    if (j.rows < 0 || j.cols < 0) throw DmError{DM_ERR_LAYOUT, "bad copy job"};
    if (j.rows == 0 || j.cols == 0) continue;
    auto span = [](int64_t off, int64_t a, int64_t b, int64_t na, int64_t nb) {
      // first and last offsets of off + i a + j b over i < na, j < nb (a, b >= 0)
      return std::make_pair(off, off + (na - 1) * a + (nb - 1) * b);
    };
    if (j.s_r < 0 || j.s_c < 0 || j.d_r < 0 || j.d_c < 0) throw DmError{DM_ERR_LAYOUT, "bad copy strides"};
    int64_t nr = j.rows, nc = j.cols;
    if (j.rperm >= 0) {
      if ((size_t)j.rperm + j.rows > perm.size()) throw DmError{DM_ERR_LAYOUT, "copy row table"};
      int64_t mx = 0;
      for (int i = 0; i < j.rows; ++i) {
        const int32_t v = perm[j.rperm + i];
        if (v < 0 || v >= src_cols) throw DmError{DM_ERR_LAYOUT, "copy row index"};
        mx = std::max<int64_t>(mx, v);
      }
      nr = mx + 1;
    }
    if (j.cperm >= 0) {
      if ((size_t)j.cperm + j.cols > perm.size()) throw DmError{DM_ERR_LAYOUT, "copy column table"};
      int64_t mx = 0;
      for (int i = 0; i < j.cols; ++i) {
        const int32_t v = perm[j.cperm + i];
        if (v < 0 || v >= src_cols) throw DmError{DM_ERR_LAYOUT, "copy column index"};
        mx = std::max<int64_t>(mx, v);
      }
      nc = mx + 1;
    }
    (void)src_rows;
    const auto s = span(j.src, j.s_r, j.s_c, nr, nc), d = span(j.dst, j.d_r, j.d_c, j.rows, j.cols);
    if (s.first < 0 || s.second >= src_size) throw DmError{DM_ERR_LAYOUT, "copy source out of bounds"};
    if (d.first < 0 || d.second >= dst_size) throw DmError{DM_ERR_LAYOUT, "copy target out of bounds"};
    if ((j.rscale >= 0 && (size_t)j.rscale + j.rows > nscale) || (j.cscale >= 0 && (size_t)j.cscale + j.cols > nscale))
      throw DmError{DM_ERR_LAYOUT, "copy scale table"};
  }
}

}  // namespace

extern "C" int dm_theta_split(int32_t ly, const dm_bond* a_, const dm_bond* c_, const dm_charge qs1[2],
                              const dm_charge qs2[2], const void* theta, int32_t chi, double cutoff,
                              int32_t move_right, dm_stream stream, dm_split** out) {
  return guarded([&] {
    if (!out || !qs1 || !qs2) throw DmError{DM_ERR_ARG, "null argument"};
    *out = nullptr;
    check_ly(ly);
    if (chi < 1) throw DmError{DM_ERR_ARG, "chi must be positive"};
    if (!(cutoff >= 0.0)) throw DmError{DM_ERR_ARG, "cutoff must be non-negative"};
    Bond a = make_bond(a_, ly), c = make_bond(c_, ly);
    for (int s = 0; s < 2; ++s)
      for (const dm_charge* q : {&qs1[s], &qs2[s]})
        if (q->k < 0 || q->k >= ly) throw DmError{DM_ERR_CHARGE, "local charge k outside [0, ly)"};
    ThetaLayout th = theta_layout(a, c, qs1, qs2, ly);
    if (th.P.total > 0 && !theta) throw DmError{DM_ERR_ARG, "null theta"};
    if (misaligned(theta)) throw DmError{DM_ERR_ARG, "theta must be 16-byte aligned"};
    hipStream_t s = (hipStream_t)stream;

    // sectors of the middle bond and their row / column groups
    std::map<std::pair<int, int>, Sector> sec;  // key (n, k)
    for (int ai = 0; ai < a.size(); ++ai)
      for (int s12 = 0; s12 < 4; ++s12) {
        const int ci = th.c[ai][s12];
        if (ci < 0) continue;
        const int s1 = s12 >> 1, s2 = s12 & 1;
        const dm_charge qb = qadd(a.q[ai], qs1[s1], ly);
        Sector& S = sec[{qb.n, qb.k}];
        S.q = qb;
        if (S.rows.empty() || S.rows.back() != std::make_pair(ai, s1)) S.rows.push_back({ai, s1});
        S.cols.push_back({s2, ci});
      }
    std::vector<Sector*> order;
    int64_t wtot = 0, stot = 0;
    for (auto& kv : sec) {
      Sector& S = kv.second;
      std::sort(S.rows.begin(), S.rows.end());
      S.rows.erase(std::unique(S.rows.begin(), S.rows.end()), S.rows.end());
      std::sort(S.cols.begin(), S.cols.end());
      S.cols.erase(std::unique(S.cols.begin(), S.cols.end()), S.cols.end());
      for (auto& r : S.rows) {
        S.roff.push_back(S.m);
        S.m += a.dim[r.first];
      }
      for (auto& q : S.cols) {
        S.coff.push_back(S.n);
        S.n += c.dim[q.second];
      }
      S.trans = S.m < S.n;
      S.w_off = wtot;
      wtot += (int64_t)S.m * S.n;
      S.v_off = wtot;
      wtot += (int64_t)S.wn() * S.wn();
      S.sig_off = stot;
      stot += S.wn();
      order.push_back(&S);
    }
    auto split = std::make_unique<dm_split>();
    split->ly = ly;
    std::vector<void*> scratch;
    auto release = [&] {
      for (void* p : scratch) dev_free_after(p, s);
    };
    try {
      void* work = dev_alloc(wtot * 16);
      scratch.push_back(work);
      void* sig = dev_alloc(stot * 8);
      scratch.push_back(sig);
      if (wtot) HIPCHK(hipMemsetAsync(work, 0, wtot * 16, s));
      // gather theta's blocks into the sector workspaces
      std::vector<CopyJob> gather;
      std::vector<SvdJob> svd;
      for (Sector* S : order) {
        for (size_t ri = 0; ri < S->rows.size(); ++ri) {
          const int ai = S->rows[ri].first, s1 = S->rows[ri].second;
          for (size_t cj = 0; cj < S->cols.size(); ++cj) {
            const int s2 = S->cols[cj].first, ci = S->cols[cj].second;
            const int s12 = s1 * 2 + s2;
            if (th.c[ai][s12] != ci) continue;
            CopyJob J{};
            J.src = th.P.off[ai] + th.coff[ai][s12];
            J.s_r = th.P.cols[ai];
            J.s_c = 1;
            J.rows = a.dim[ai];
            J.cols = c.dim[ci];
            J.rperm = J.cperm = J.rscale = J.cscale = -1;
            if (!S->trans) {  // W = M, column-major m x n
              J.dst = S->w_off + S->roff[ri] + (int64_t)S->coff[cj] * S->m;
              J.d_r = 1;
              J.d_c = S->m;
            } else {  // W = M^H, column-major n x m
              J.dst = S->w_off + S->coff[cj] + (int64_t)S->roff[ri] * S->n;
              J.d_r = S->n;
              J.d_c = 1;
              J.conj = 1;
            }
            gather.push_back(J);
          }
        }
        svd.push_back({S->w_off, S->v_off, S->sig_off, S->wm(), S->wn()});
      }
      for (const SvdJob& J : svd)
        if (J.n > J.m || J.m <= 0 || J.n <= 0 || J.w_off + (int64_t)J.m * J.n > wtot || J.v_off + (int64_t)J.n * J.n > wtot ||
            J.sig_off + J.n > stot)
          throw DmError{DM_ERR_LAYOUT, "split: SVD workspace out of bounds"};
      validate_copies(gather, th.P.total, wtot, {}, 0, 0, 0);
      const int64_t ng = copy_layout(gather);
      TableUpload up;
      CopyJob* d_gather = nullptr;
      SvdJob* d_svd = nullptr;
      up.add(gather, &d_gather);
      up.add(svd, &d_svd);
      scratch.push_back(up.commit(s));
      HIPCHK(launch_block_copy(d_gather, (int32_t)gather.size(), ng, nullptr, nullptr, (const double*)theta,
                               (double*)work, s));
      HIPCHK(launch_svd_jacobi(d_svd, (int32_t)svd.size(), (double*)work, (double*)sig, 60, s));
      std::vector<double> hs(stot);
      if (stot) HIPCHK(hipMemcpyAsync(hs.data(), sig, stot * 8, hipMemcpyDeviceToHost, s));
      HIPCHK(hipStreamSynchronize(s));
      for (double v : hs)
        if (!std::isfinite(v)) throw DmError{DM_ERR_NONFINITE, "singular value is not finite"};

      // selection: per sector the values in descending order (ties by column), then the
      // chi largest overall, ties by (sector, rank)
      std::vector<std::vector<int>> rank(order.size());
      std::vector<std::tuple<double, int, int>> cand;  // (-sigma, sector, rank)
      double total = 0.0;
      for (size_t q = 0; q < order.size(); ++q) {
        const Sector& S = *order[q];
        std::vector<int>& r = rank[q];
        for (int j = 0; j < S.wn(); ++j) r.push_back(j);
        std::stable_sort(r.begin(), r.end(), [&](int x, int y) { return hs[S.sig_off + x] > hs[S.sig_off + y]; });
        for (int k = 0; k < S.wn(); ++k) {
          const double v = hs[S.sig_off + r[k]];
          cand.emplace_back(-v, (int)q, k);
          total += v * v;
        }
      }
      std::sort(cand.begin(), cand.end());
      std::vector<int> keep(order.size(), 0);
      double kept = 0.0;
      for (size_t i = 0; i < cand.size() && (int)i < chi; ++i) {
        const double v = -std::get<0>(cand[i]);
        if (!(v > cutoff)) break;
        keep[std::get<1>(cand[i])] = std::max(keep[std::get<1>(cand[i])], std::get<2>(cand[i]) + 1);
        kept += v * v;
      }
      if (!(kept > 0.0)) throw DmError{DM_ERR_NONFINITE, "no singular value above the cutoff"};
      const double norm = std::sqrt(kept);
      split->discarded = std::max(0.0, 1.0 - kept / total);
      // new bond and per-sector tables: permutation (kept workspace columns in
      // descending order) and the scale sigma / norm
      std::vector<int32_t> perm;
      std::vector<double> scl;
      std::vector<int32_t> p0(order.size(), -1);
      for (size_t q = 0; q < order.size(); ++q) {
        if (keep[q] == 0) continue;
        const Sector& S = *order[q];
        split->bq.push_back(S.q);
        split->bdim.push_back(keep[q]);
        p0[q] = (int32_t)perm.size();
        for (int k = 0; k < keep[q]; ++k) {
          perm.push_back(rank[q][k]);
          const double v = hs[S.sig_off + rank[q][k]] / norm;
          scl.push_back(v);
          split->schmidt.push_back(v);
        }
      }
      dm_bond bb{(int32_t)split->bq.size(), split->bq.data(), split->bdim.data()};
      Bond b = make_bond(&bb, ly);
      SiteLayout Lt = site_layout(a, b, qs1, ly), Rt = site_layout(b, c, qs2, ly);
      split->nleft = Lt.P.total;
      split->nright = Rt.P.total;
      split->left = dev_alloc(Lt.P.total * 16);
      split->right = dev_alloc(Rt.P.total * 16);
      if (Lt.P.total) HIPCHK(hipMemsetAsync(split->left, 0, Lt.P.total * 16, s));
      if (Rt.P.total) HIPCHK(hipMemsetAsync(split->right, 0, Rt.P.total * 16, s));
      // M = P diag(sigma) Q^H with P = U_W, Q = V_W (W = M) or P = V_W, Q = U_W (W = M^H)
      std::vector<CopyJob> lj, rj;
      int bi = 0;
      for (size_t q = 0; q < order.size(); ++q) {
        if (keep[q] == 0) continue;
        const Sector& S = *order[q];
        const int64_t p_base = S.trans ? S.v_off : S.w_off, q_base = S.trans ? S.w_off : S.v_off;
        const int64_t p_ld = S.m, q_ld = S.n;  // rows of P (= m) and of Q (= n), column-major
        for (size_t ri = 0; ri < S.rows.size(); ++ri) {
          const int ai = S.rows[ri].first, s1 = S.rows[ri].second;
          if (Lt.b[ai][s1] != bi) throw DmError{DM_ERR_LAYOUT, "split: left layout mismatch"};
          CopyJob J{};
          J.src = p_base + S.roff[ri];
          J.s_r = 1;
          J.s_c = p_ld;
          J.dst = Lt.P.off[ai] + Lt.coff[ai][s1];
          J.d_r = Lt.P.cols[ai];
          J.d_c = 1;
          J.rows = a.dim[ai];
          J.cols = keep[q];
          J.rperm = -1;
          J.cperm = p0[q];
          J.rscale = -1;
          J.cscale = move_right ? -1 : p0[q];
          lj.push_back(J);
        }
        for (size_t cj = 0; cj < S.cols.size(); ++cj) {
          const int s2 = S.cols[cj].first, ci = S.cols[cj].second;
          if (Rt.b[bi][s2] != ci) throw DmError{DM_ERR_LAYOUT, "split: right layout mismatch"};
          CopyJob J{};
          J.src = q_base + S.coff[cj];
          J.s_r = q_ld;
          J.s_c = 1;
          J.dst = Rt.P.off[bi] + Rt.coff[bi][s2];
          J.d_r = Rt.P.cols[bi];
          J.d_c = 1;
          J.rows = keep[q];
          J.cols = c.dim[ci];
          J.rperm = p0[q];
          J.cperm = -1;
          J.rscale = move_right ? p0[q] : -1;
          J.cscale = -1;
          J.conj = 1;
          rj.push_back(J);
        }
        ++bi;
      }
      // permuted indices are workspace columns: below the largest column count
      int32_t maxw = 0;
      for (const Sector* S : order) maxw = std::max(maxw, S->wn());
      validate_copies(lj, wtot, Lt.P.total, perm, scl.size(), 0, maxw);
      validate_copies(rj, wtot, Rt.P.total, perm, scl.size(), 0, maxw);
      const int64_t nl = copy_layout(lj), nr = copy_layout(rj);
      TableUpload up2;
      CopyJob* d_lj = nullptr;
      CopyJob* d_rj = nullptr;
      int32_t* d_perm = nullptr;
      double* d_scl = nullptr;
      up2.add(lj, &d_lj);
      up2.add(rj, &d_rj);
      up2.add(perm, &d_perm);
      up2.add(scl, &d_scl);
      scratch.push_back(up2.commit(s));
      HIPCHK(launch_block_copy(d_lj, (int32_t)lj.size(), nl, d_perm, d_scl, (const double*)work,
                               (double*)split->left, s));
      HIPCHK(launch_block_copy(d_rj, (int32_t)rj.size(), nr, d_perm, d_scl, (const double*)work,
                               (double*)split->right, s));
    } catch (...) {
      release();
      throw;
    }
    release();
    *out = split.release();
  });
}

extern "C" int dm_split_bond(const dm_split* sp, int32_t* nsec, dm_charge* q, int32_t* dim) {
  if (!sp || !nsec) return fail(DM_ERR_ARG, "null argument");
  *nsec = (int32_t)sp->bq.size();
  if (q) std::copy(sp->bq.begin(), sp->bq.end(), q);
  if (dim) std::copy(sp->bdim.begin(), sp->bdim.end(), dim);
  return DM_OK;
}

extern "C" int dm_split_tensors(const dm_split* sp, const void** left, int64_t* nleft, const void** right,
                                int64_t* nright) {
  if (!sp) return fail(DM_ERR_ARG, "null split");
  if (left) *left = sp->left;
  if (nleft) *nleft = sp->nleft;
  if (right) *right = sp->right;
  if (nright) *nright = sp->nright;
  return DM_OK;
}

extern "C" int dm_split_schmidt(const dm_split* sp, double* values, double* discarded) {
  if (!sp) return fail(DM_ERR_ARG, "null split");
  if (values) std::copy(sp->schmidt.begin(), sp->schmidt.end(), values);
  if (discarded) *discarded = sp->discarded;
  return DM_OK;
}

extern "C" int dm_split_copy(const dm_split* sp, void* left, void* right, dm_stream stream) {
  return guarded([&] {
    if (!sp || (sp->nleft && !left) || (sp->nright && !right)) throw DmError{DM_ERR_ARG, "null argument"};
    hipStream_t s = (hipStream_t)stream;
    if (sp->nleft) HIPCHK(hipMemcpyAsync(left, sp->left, sp->nleft * 16, hipMemcpyDeviceToDevice, s));
    if (sp->nright) HIPCHK(hipMemcpyAsync(right, sp->right, sp->nright * 16, hipMemcpyDeviceToDevice, s));
  });
}

extern "C" void dm_split_destroy(dm_split* sp) { delete sp; }
