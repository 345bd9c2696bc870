// Finite two-site DMRG sweeps on the device (dm_mps, dm_dmrg_sweeps).
//
// The paper runs (i)DMRG on the mixed-basis MPO (Sec. I, III A) and does not restate the
// sweep.  This is the textbook finite two-site sweep around the hot path: at bond
// (i, i+1) the two-site tensor theta = M_i M_{i+1} (block GEMMs) is the start vector of
// the Lanczos ground state of H_eff (the plan of L_i, W_i, W_{i+1}, R_{i+2}); theta is
// split by the block SVD truncation (dm_theta_split) into a left-canonical A_i and S V^H
// (sweeping right) or U S and a right-canonical B_{i+1} (sweeping left), and the
// environment the sweep leaves behind is updated (env_update_left / env_update_right).
// One sweep is a pass right over bonds 0 .. n-2 and back left over n-2 .. 0.  Site
// tensors and environments stay on the device; the host keeps the bonds and decides the
// truncation from the singular values.
#include <algorithm>
#include <cmath>
#include <memory>

#include "runtime.hpp"
#include "svd.hpp"

using namespace mrd;

struct dm_mps {
  int ly = 1, n = 0;
  std::vector<std::vector<dm_charge>> bq;  // bond i: charges (increasing) and dims
  std::vector<std::vector<int32_t>> bd;
  std::vector<std::array<dm_charge, 2>> qs;
  std::vector<void*> t;      // site tensors, SITE layout of (bond i, bond i+1, qs[i])
  std::vector<int64_t> nt;
  std::vector<std::vector<double>> schmidt;  // per bond: Schmidt values of its last split
  dm_bond bond(int i) const { return dm_bond{(int32_t)bq[i].size(), bq[i].data(), bd[i].data()}; }
  ~dm_mps() {
    for (void* p : t) dev_free(p);
  }
};

namespace {

void set_bond(dm_mps& m, int i, const dm_bond& b) {
  m.bq[i].assign(b.q, b.q + b.nsec);
  m.bd[i].assign(b.dim, b.dim + b.nsec);
}

// theta[a, s1, s2, c] = sum_b M1[a, s1, b] M2[b, s2, c] into the THETA layout: one
// block GEMM per (a, s1): the M1 block (a, s1, b) times the whole M2 panel of b, whose
// columns (s2, c) are theta's columns (s1 s2, c) of panel a, in the same order.
void contract_two_site(int ly, const Bond& a, const Bond& b, const Bond& c, const dm_charge qs1[2],
                       const dm_charge qs2[2], const void* m1, const void* m2, void* theta, hipStream_t s,
                       std::vector<void*>& scratch) {
  SiteLayout S1 = site_layout(a, b, qs1, ly), S2 = site_layout(b, c, qs2, ly);
  ThetaLayout th = theta_layout(a, c, qs1, qs2, ly);
  if (th.P.total) HIPCHK(hipMemsetAsync(theta, 0, th.P.total * 16, s));
  GemmStage st;
  st.flags = 0;
  for (int ai = 0; ai < a.size(); ++ai)
    for (int s1 = 0; s1 < 2; ++s1) {
      const int bi = S1.b[ai][s1];
      if (bi < 0) continue;
      const int N = S2.P.cols[bi], M = a.dim[ai], K = b.dim[bi];
      if (N == 0) continue;
      int first = -1;
      for (int s2 = 0; s2 < 2; ++s2)
        if (first < 0 && th.c[ai][2 * s1 + s2] >= 0) first = 2 * s1 + s2;
      if (first < 0) throw DmError{DM_ERR_LAYOUT, "two-site contraction: theta columns missing"};
      GemmProb pr{th.P.off[ai] + th.coff[ai][first], M, N, (int32_t)st.segs.size(), 1, th.P.cols[ai], -1};
      st.segs.push_back({S1.P.off[ai] + S1.coff[ai][s1], S2.P.off[bi], S1.P.cols[ai], N, K, 0});
      st.probs.push_back(pr);
      add_tiles(st, (int32_t)st.probs.size() - 1, M, N);
      st.flops += 8.0 * M * N * K;
    }
  validate(st, S1.P.total, S2.P.total, th.P.total);
  TableUpload up;
  up.add(st);
  scratch.push_back(up.commit(s));
  HIPCHK(launch_gemm<double>(st, (const double*)m1, (const double*)m2, (double*)theta, nullptr, s));
}

// A one-element environment holding 1 (the MPO boundary state).
void* unit_env(hipStream_t s) {
  void* p = dev_alloc(16);
  const double one[2] = {1.0, 0.0};
  HIPCHK(hipMemcpyAsync(p, one, 16, hipMemcpyHostToDevice, s));
  HIPCHK(hipStreamSynchronize(s));  // the host source is a local
  return p;
}

int check(int rc) {
  if (rc != DM_OK) throw DmError{rc, dm_last_error()};
  return rc;
}

}  // namespace

extern "C" int dm_mps_create(int32_t ly, int32_t n, const dm_bond* bonds, const dm_charge* qs,
                             const void* const* tensors, dm_stream stream, dm_mps** out) {
  return guarded([&] {
    if (!out || n < 2 || !bonds || !qs || !tensors) throw DmError{DM_ERR_ARG, "dm_mps_create: bad arguments"};
    *out = nullptr;
    check_ly(ly);
    auto m = std::make_unique<dm_mps>();
    m->ly = ly;
    m->n = n;
    m->bq.resize(n + 1);
    m->bd.resize(n + 1);
    m->schmidt.resize(n + 1);
    for (int i = 0; i <= n; ++i) {
      make_bond(&bonds[i], ly);  // validates
      set_bond(*m, i, bonds[i]);
    }
    hipStream_t s = (hipStream_t)stream;
    for (int i = 0; i < n; ++i) {
      const dm_charge q2[2] = {qs[2 * i], qs[2 * i + 1]};
      m->qs.push_back({q2[0], q2[1]});
      Bond bl = make_bond(&bonds[i], ly), br = make_bond(&bonds[i + 1], ly);
      SiteLayout L = site_layout(bl, br, q2, ly);
      if (L.P.total > 0 && !tensors[i]) throw DmError{DM_ERR_ARG, "null site tensor"};
      void* p = dev_alloc(L.P.total * 16);
      m->t.push_back(p);
      m->nt.push_back(L.P.total);
      if (L.P.total) HIPCHK(hipMemcpyAsync(p, tensors[i], L.P.total * 16, hipMemcpyDeviceToDevice, s));
    }
    HIPCHK(hipStreamSynchronize(s));
    *out = m.release();
  });
}

extern "C" void dm_mps_destroy(dm_mps* m) { delete m; }

extern "C" int dm_mps_bond(const dm_mps* m, int32_t i, int32_t* nsec, dm_charge* q, int32_t* dim) {
  if (!m || !nsec || i < 0 || i > m->n) return fail(DM_ERR_ARG, "dm_mps_bond: bad arguments");
  *nsec = (int32_t)m->bq[i].size();
  if (q) std::copy(m->bq[i].begin(), m->bq[i].end(), q);
  if (dim) std::copy(m->bd[i].begin(), m->bd[i].end(), dim);
  return DM_OK;
}

extern "C" int dm_mps_tensor(const dm_mps* m, int32_t i, const void** data, int64_t* nelem) {
  if (!m || i < 0 || i >= m->n) return fail(DM_ERR_ARG, "dm_mps_tensor: bad arguments");
  if (data) *data = m->t[i];
  if (nelem) *nelem = m->nt[i];
  return DM_OK;
}

extern "C" int dm_mps_copy(const dm_mps* m, int32_t i, void* dst, dm_stream stream) {
  return guarded([&] {
    if (!m || i < 0 || i >= m->n || (m->nt[i] && !dst)) throw DmError{DM_ERR_ARG, "dm_mps_copy: bad arguments"};
    if (m->nt[i])
      HIPCHK(hipMemcpyAsync(dst, m->t[i], m->nt[i] * 16, hipMemcpyDeviceToDevice, (hipStream_t)stream));
  });
}

extern "C" int dm_mps_schmidt(const dm_mps* m, int32_t i, double* values, int64_t* count) {
  if (!m || i < 0 || i > m->n || !count) return fail(DM_ERR_ARG, "dm_mps_schmidt: bad arguments");
  *count = (int64_t)m->schmidt[i].size();
  if (values) std::copy(m->schmidt[i].begin(), m->schmidt[i].end(), values);
  return DM_OK;
}

extern "C" int dm_dmrg_sweeps(dm_mps* psi, const dm_mpo_site* w, int32_t nsweeps, int32_t chi,
                              int32_t max_iter, double cutoff, int32_t prec, double* energies,
                              dm_stream stream) {
  return guarded([&] {
    if (!psi || !w || nsweeps < 1 || !energies) throw DmError{DM_ERR_ARG, "dm_dmrg_sweeps: bad arguments"};
    check_prec(prec);
    const int n = psi->n, ly = psi->ly;
    hipStream_t s = (hipStream_t)stream;
    std::vector<MpoSite> W;
    for (int i = 0; i < n; ++i) {
      W.push_back(make_mpo(&w[i], ly));
      if (!qeq(W[i].qs[0], psi->qs[i][0]) || !qeq(W[i].qs[1], psi->qs[i][1]))
        throw DmError{DM_ERR_CHARGE, "MPO local charges differ from the MPS"};
      if (i > 0 && W[i].dl != W[i - 1].dr) throw DmError{DM_ERR_DIM, "MPO bond dimensions differ"};
    }
    if (W[0].dl != 1 || W[n - 1].dr != 1) throw DmError{DM_ERR_DIM, "MPO boundary dimensions must be 1"};
    // environments: L[i] on bond i (MPO states w[i].ql), R[i] on bond i (w[i-1].qr)
    std::vector<void*> L(n + 1, nullptr), R(n + 1, nullptr);
    std::vector<void*> scratch;
    auto free_env = [&](void*& p) {
      dev_free_after(p, s);
      p = nullptr;
    };
    auto env_elems = [&](int kind, int i, const std::vector<dm_charge>& qw) {
      dm_bond b = psi->bond(i);
      dm_layout_desc d{};
      d.kind = kind;
      d.ly = ly;
      d.x = &b;
      d.nw = (int32_t)qw.size();
      d.qw = qw.data();
      int64_t nb = 0, ne = 0;
      check(dm_layout(&d, &nb, &ne, nullptr));
      return ne;
    };
    try {
      if (env_elems(DM_LAYOUT_ENV_L, 0, W[0].ql) != 1 || env_elems(DM_LAYOUT_ENV_R, n, W[n - 1].qr) != 1)
        throw DmError{DM_ERR_CHARGE, "boundary bonds do not meet the MPO boundary states"};
      L[0] = unit_env(s);
      R[n] = unit_env(s);
      for (int i = n - 1; i >= 2; --i) {
        R[i] = dev_alloc(env_elems(DM_LAYOUT_ENV_R, i, W[i].ql) * 16);
        dm_bond bi = psi->bond(i), bj = psi->bond(i + 1);
        check(env_update_right(ly, &bi, &bj, &w[i], R[i + 1], psi->t[i], R[i], DM_FP64, stream));
      }
      double e = 0.0;
      for (int sweep = 0; sweep < nsweeps; ++sweep) {
        for (int dir = 0; dir < 2; ++dir) {
          const bool right = dir == 0;
          for (int step = 0; step < n - 1; ++step) {
            const int i = right ? step : n - 2 - step;
            dm_bond ba = psi->bond(i), bb = psi->bond(i + 1), bc = psi->bond(i + 2);
            Bond a = make_bond(&ba, ly), b = make_bond(&bb, ly), c = make_bond(&bc, ly);
            const dm_charge* q1 = psi->qs[i].data();
            const dm_charge* q2 = psi->qs[i + 1].data();
            ThetaLayout th = theta_layout(a, c, q1, q2, ly);
            void* theta = dev_alloc(std::max<int64_t>(1, th.P.total) * 16);
            scratch.push_back(theta);
            contract_two_site(ly, a, b, c, q1, q2, psi->t[i], psi->t[i + 1], theta, s, scratch);
            dm_heff_plan* plan = nullptr;
            check(dm_heff_plan_create(ly, &ba, &bc, &w[i], &w[i + 1], L[i], R[i + 2], prec, stream, &plan));
            std::unique_ptr<dm_heff_plan, void (*)(dm_heff_plan*)> hold(plan, dm_heff_plan_destroy);
            int32_t k = 0;
            check(lanczos_ground(plan, theta, max_iter, 1e-14, &e, &k, stream));
            hold.reset();
            dm_split* sp = nullptr;
            check(dm_theta_split(ly, &ba, &bc, q1, q2, theta, chi, cutoff, right ? 1 : 0, stream, &sp));
            std::unique_ptr<dm_split, void (*)(dm_split*)> spl(sp, dm_split_destroy);
            // the split's tensors become the MPS's
            free_env(psi->t[i]);
            free_env(psi->t[i + 1]);
            psi->t[i] = sp->left;
            psi->nt[i] = sp->nleft;
            psi->t[i + 1] = sp->right;
            psi->nt[i + 1] = sp->nright;
            sp->left = sp->right = nullptr;
            psi->bq[i + 1] = sp->bq;
            psi->bd[i + 1] = sp->bdim;
            psi->schmidt[i + 1] = sp->schmidt;
            dm_bond nb = psi->bond(i + 1);
            if (right) {
              free_env(L[i + 1]);
              L[i + 1] = dev_alloc(env_elems(DM_LAYOUT_ENV_L, i + 1, W[i].qr) * 16);
              check(env_update_left(ly, &ba, &nb, &w[i], L[i], psi->t[i], L[i + 1], DM_FP64, stream));
            } else {
              free_env(R[i + 1]);
              R[i + 1] = dev_alloc(env_elems(DM_LAYOUT_ENV_R, i + 1, W[i + 1].ql) * 16);
              check(env_update_right(ly, &nb, &bc, &w[i + 1], R[i + 2], psi->t[i + 1], R[i + 1], DM_FP64, stream));
            }
            for (void* p : scratch) dev_free_after(p, s);
            scratch.clear();
          }
        }
        energies[sweep] = e;
      }
      HIPCHK(hipStreamSynchronize(s));
    } catch (...) {
      (void)hipStreamSynchronize(s);
      for (void* p : scratch) dev_free(p);
      for (void*& p : L) dev_free(p);
      for (void*& p : R) dev_free(p);
      throw;
    }
    for (void*& p : L) dev_free(p);
    for (void*& p : R) dev_free(p);
  });
}

extern "C" int dm_entanglement(const double* values, int64_t count, double* entropy, double* energies) {
  if ((count > 0 && !values) || count < 0) return fail(DM_ERR_ARG, "dm_entanglement: bad arguments");
  double S = 0.0;
  for (int64_t i = 0; i < count; ++i) {
    const double l = values[i];
    if (!(l > 0.0)) return fail(DM_ERR_ARG, "dm_entanglement: Schmidt values must be positive");
    S -= l * l * std::log(l * l);
    if (energies) energies[i] = -2.0 * std::log(l);
  }
  if (entropy) *entropy = S;
  return DM_OK;
}
