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

// The bond steps of two-site sweeps over the orbitals of an MPS held by the library,
// with the environments at its two ends in L[0] and R[n] (device, owned here, freed
// with every other environment when the sweeper goes).  Environment L[i] lives on bond
// i with the MPO states of w[i].ql, R[i] on bond i with those of w[i - 1].qr.
struct Sweeper {
  dm_mps& psi;
  std::vector<dm_mpo_site> w;
  int ly, n;
  hipStream_t s;
  int32_t prec, chi, max_iter;
  double cutoff;
  bool real;  // the eigensolves run DM_REAL plans on the real parts (eq. rot form)
  std::vector<void*> L, R, scratch;
  double e = 0.0;
  int64_t theta_n = 0;  // elements of the last theta_of

  Sweeper(dm_mps& p, std::vector<dm_mpo_site> sites, int32_t prec_, int32_t chi_, int32_t max_iter_,
          double cutoff_, hipStream_t st, bool real_ = false)
      : psi(p), w(std::move(sites)), ly(p.ly), n(p.n), s(st), prec(prec_), chi(chi_), max_iter(max_iter_),
        cutoff(cutoff_), real(real_), L(p.n + 1, nullptr), R(p.n + 1, nullptr) {}
  ~Sweeper() {
    (void)hipStreamSynchronize(s);
    for (void* p : scratch) dev_free(p);
    for (void*& p : L) dev_free(p);
    for (void*& p : R) dev_free(p);
  }

  void release(void*& p) {
    dev_free_after(p, s);
    p = nullptr;
  }
  void flush() {
    for (void* p : scratch) dev_free_after(p, s);
    scratch.clear();
  }
  int64_t env_elems(int kind, int i, const std::vector<dm_charge>& qw) const {
    dm_bond b = psi.bond(i);
    dm_layout_desc d{};
    d.kind = kind;
    d.ly = ly;
    d.x = &b;
    d.nw = (int32_t)qw.size();
    d.qw = qw.data();
    int64_t nb = 0, ne = 0;
    check(dm_layout(&d, &nb, &ne, nullptr));
    return ne;
  }
  std::vector<dm_charge> ql(int i) const { return std::vector<dm_charge>(w[i].ql, w[i].ql + w[i].dl); }
  std::vector<dm_charge> qr(int i) const { return std::vector<dm_charge>(w[i].qr, w[i].qr + w[i].dr); }

  // L[i + 1] from L[i] and the (left-canonical) tensor i
  void update_left(int i) {
    release(L[i + 1]);
    L[i + 1] = dev_alloc(std::max<int64_t>(1, env_elems(DM_LAYOUT_ENV_L, i + 1, qr(i))) * 16);
    dm_bond ba = psi.bond(i), bb = psi.bond(i + 1);
    check(env_update_left(ly, &ba, &bb, &w[i], L[i], psi.t[i], L[i + 1], DM_FP64, (dm_stream)s));
  }
  // R[i + 1] from R[i + 2] and the (right-canonical) tensor i + 1
  void update_right(int i) {
    release(R[i + 1]);
    R[i + 1] = dev_alloc(std::max<int64_t>(1, env_elems(DM_LAYOUT_ENV_R, i + 1, ql(i + 1))) * 16);
    dm_bond bb = psi.bond(i + 1), bc = psi.bond(i + 2);
    check(env_update_right(ly, &bb, &bc, &w[i + 1], R[i + 2], psi.t[i + 1], R[i + 1], DM_FP64, (dm_stream)s));
  }
  // theta = M_i M_{i+1} (scratch until flush)
  void* theta_of(int i) {
    dm_bond ba = psi.bond(i), bb = psi.bond(i + 1), bc = psi.bond(i + 2);
    Bond a = make_bond(&ba, ly), b = make_bond(&bb, ly), c = make_bond(&bc, ly);
    const dm_charge* q1 = psi.qs[i].data();
    const dm_charge* q2 = psi.qs[i + 1].data();
    ThetaLayout th = theta_layout(a, c, q1, q2, ly);
    void* theta = dev_alloc(std::max<int64_t>(1, th.P.total) * 16);
    scratch.push_back(theta);
    theta_n = th.P.total;
    contract_two_site(ly, a, b, c, q1, q2, psi.t[i], psi.t[i + 1], theta, s, scratch);
    return theta;
  }
  // lowest eigenpair of H_eff(L[i], w[i], w[i+1], R[i+2]) from theta (theta_of(i)), in
  // place.  Real form: the state, the environments and the MPO are real (held complex with
  // zero imaginary parts), so their real parts go to a DM_REAL plan and back.
  void solve(int i, void* theta) {
    dm_bond ba = psi.bond(i), bc = psi.bond(i + 2);
    const void* Lp = L[i];
    const void* Rp = R[i + 2];
    void* th = theta;
    if (real) {
      const int64_t nl = env_elems(DM_LAYOUT_ENV_L, i, ql(i)), nr = env_elems(DM_LAYOUT_ENV_R, i + 2, qr(i + 1));
      double* lr = (double*)dev_alloc(std::max<int64_t>(1, nl) * 8);
      scratch.push_back(lr);
      double* rr = (double*)dev_alloc(std::max<int64_t>(1, nr) * 8);
      scratch.push_back(rr);
      double* tr = (double*)dev_alloc(std::max<int64_t>(1, theta_n) * 8);
      scratch.push_back(tr);
      HIPCHK(launch_re_take((const double*)L[i], lr, nl, s));
      HIPCHK(launch_re_take((const double*)R[i + 2], rr, nr, s));
      HIPCHK(launch_re_take((const double*)theta, tr, theta_n, s));
      Lp = lr;
      Rp = rr;
      th = tr;
    }
    dm_heff_plan* plan = nullptr;
    check(dm_heff_plan_create(ly, &ba, &bc, &w[i], &w[i + 1], Lp, Rp, prec | (real ? DM_REAL : 0), (dm_stream)s,
                              &plan));
    std::unique_ptr<dm_heff_plan, void (*)(dm_heff_plan*)> hold(plan, dm_heff_plan_destroy);
    int32_t k = 0;
    check(lanczos_ground(plan, th, max_iter, 1e-14, &e, &k, (dm_stream)s));
    if (real) HIPCHK(launch_re_put((const double*)th, (double*)theta, theta_n, s));
  }
  std::unique_ptr<dm_split, void (*)(dm_split*)> split(int i, const void* theta, bool right) {
    dm_bond ba = psi.bond(i), bc = psi.bond(i + 2);
    dm_split* sp = nullptr;
    check(dm_theta_split(ly, &ba, &bc, psi.qs[i].data(), psi.qs[i + 1].data(), theta, chi, cutoff, right ? 1 : 0,
                         (dm_stream)s, &sp));
    return std::unique_ptr<dm_split, void (*)(dm_split*)>(sp, dm_split_destroy);
  }
  // the split's two tensors and middle bond become the MPS's
  void take(int i, dm_split& sp) {
    release(psi.t[i]);
    release(psi.t[i + 1]);
    psi.t[i] = sp.left;
    psi.nt[i] = sp.nleft;
    psi.t[i + 1] = sp.right;
    psi.nt[i + 1] = sp.nright;
    sp.left = sp.right = nullptr;
    psi.bq[i + 1] = sp.bq;
    psi.bd[i + 1] = sp.bdim;
    psi.schmidt[i + 1] = sp.schmidt;
  }
  // one bond of a sweep: theta, its Lanczos ground state (eig), the split, and the
  // environment behind the move
  void step(int i, bool right, bool eig) {
    void* theta = theta_of(i);
    if (eig) solve(i, theta);
    auto sp = split(i, theta, right);
    take(i, *sp);
    if (right)
      update_left(i);
    else
      update_right(i);
    flush();
  }
};

// A bond with every charge moved by d (N exactly, k modulo ly), in increasing order;
// perm[j] = position of old sector j in the moved bond.
void moved_bond(const dm_mps& m, int i, dm_charge d, std::vector<dm_charge>& q, std::vector<int32_t>& dim,
                std::vector<int>& perm) {
  const int ns = (int)m.bq[i].size(), ly = m.ly;
  std::vector<std::pair<dm_charge, int>> v;
  for (int j = 0; j < ns; ++j) {
    const dm_charge c = m.bq[i][j];
    v.push_back({dm_charge{c.n + d.n, ((c.k + d.k) % ly + ly) % ly}, j});
  }
  std::sort(v.begin(), v.end(), [](const auto& x, const auto& y) {
    return x.first.n < y.first.n || (x.first.n == y.first.n && x.first.k < y.first.k);
  });
  q.clear();
  dim.clear();
  perm.assign(ns, -1);
  for (int j = 0; j < ns; ++j) {
    q.push_back(v[j].first);
    dim.push_back(m.bd[i][v[j].second]);
    perm[v[j].second] = j;
  }
}

// Copies every panel of `from` (data src) to panel perm[j] of `to` (data dst): the
// same tensor with its bond charges moved, whose panels keep their shapes.
void permute_panels(const Panels& from, const Panels& to, const std::vector<int>& perm, const void* src, void* dst,
                    hipStream_t s) {
  if (from.off.size() != perm.size() || to.off.size() != perm.size() || from.total != to.total)
    throw DmError{DM_ERR_LAYOUT, "moved tensor: panel count or size differs"};
  for (size_t j = 0; j < perm.size(); ++j) {
    const int t = perm[j];
    if (t < 0 || t >= (int)to.off.size() || to.rows[t] != from.rows[j] || to.cols[t] != from.cols[j])
      throw DmError{DM_ERR_LAYOUT, "moved tensor: panel shape differs"};
    const int64_t ne = (int64_t)from.rows[j] * from.cols[j];
    if (ne)
      HIPCHK(hipMemcpyAsync((char*)dst + to.off[t] * 16, (const char*)src + from.off[j] * 16, ne * 16,
                            hipMemcpyDeviceToDevice, s));
  }
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
    const bool real = take_real(prec);
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
    Sweeper sw(*psi, std::vector<dm_mpo_site>(w, w + n), prec, chi, max_iter, cutoff, s, real);
    if (sw.env_elems(DM_LAYOUT_ENV_L, 0, W[0].ql) != 1 || sw.env_elems(DM_LAYOUT_ENV_R, n, W[n - 1].qr) != 1)
      throw DmError{DM_ERR_CHARGE, "boundary bonds do not meet the MPO boundary states"};
    sw.L[0] = unit_env(s);
    sw.R[n] = unit_env(s);
    for (int i = n - 1; i >= 2; --i) sw.update_right(i - 1);
    for (int sweep = 0; sweep < nsweeps; ++sweep) {
      for (int step = 0; step < n - 1; ++step) sw.step(step, true, true);
      for (int step = 0; step < n - 1; ++step) sw.step(n - 2 - step, false, true);
      energies[sweep] = sw.e;
    }
    HIPCHK(hipStreamSynchronize(s));
  });
}

extern "C" int dm_idmrg(dm_mps* psi, const dm_mpo_site* cell, dm_charge d, const void* L0, const void* R0,
                        int32_t n_iter, int32_t sweeps, int32_t chi, int32_t max_iter, double cutoff,
                        int32_t prec, double* energies, dm_stream stream) {
  return guarded([&] {
    if (!psi || !cell || !L0 || !R0 || n_iter < 1 || sweeps < 1 || !energies || psi->n < 2 || psi->n % 2)
      throw DmError{DM_ERR_ARG, "dm_idmrg: bad arguments"};
    const bool real = take_real(prec);
    check_prec(prec);
    const int n2 = psi->n, n = n2 / 2, ly = psi->ly;
    if (d.k < 0 || d.k >= ly) throw DmError{DM_ERR_CHARGE, "dm_idmrg: charge of two cells has k outside [0, ly)"};
    hipStream_t s = (hipStream_t)stream;
    std::vector<MpoSite> W;
    for (int i = 0; i < n; ++i) {
      W.push_back(make_mpo(&cell[i], ly));
      for (int c = 0; c < 2; ++c)
        for (int x = 0; x < 2; ++x)
          if (!qeq(W[i].qs[x], psi->qs[i + c * n][x]))
            throw DmError{DM_ERR_CHARGE, "MPO cell's local charges differ from the MPS"};
      if (i > 0 && W[i].dl != W[i - 1].dr) throw DmError{DM_ERR_DIM, "MPO bond dimensions differ"};
    }
    if (W[n - 1].dr != W[0].dl) throw DmError{DM_ERR_DIM, "MPO cell does not close (D_n != D_0)"};
    for (int a = 0; a < W[0].dl; ++a)
      if (!qeq(W[n - 1].qr[a], W[0].ql[a])) throw DmError{DM_ERR_CHARGE, "MPO cell's end states differ from its first"};
    {  // the two cells' last bond is their first moved by d
      std::vector<dm_charge> q;
      std::vector<int32_t> dim;
      std::vector<int> perm;
      moved_bond(*psi, 0, d, q, dim, perm);
      bool same = q.size() == psi->bq[n2].size();
      for (size_t j = 0; same && j < q.size(); ++j) same = qeq(q[j], psi->bq[n2][j]) && dim[j] == psi->bd[n2][j];
      if (!same) throw DmError{DM_ERR_CHARGE, "dm_idmrg: last bond is not the first moved by d"};
    }
    std::vector<dm_mpo_site> w2(cell, cell + n);
    w2.insert(w2.end(), cell, cell + n);
    Sweeper sw(*psi, w2, prec, chi, max_iter, cutoff, s, real);
    const size_t nl = (size_t)sw.env_elems(DM_LAYOUT_ENV_L, 0, W[0].ql), nr = (size_t)sw.env_elems(DM_LAYOUT_ENV_R, n2, W[0].ql);
    sw.L[0] = dev_alloc(std::max<size_t>(1, nl) * 16);
    sw.R[n2] = dev_alloc(std::max<size_t>(1, nr) * 16);
    if (nl) HIPCHK(hipMemcpyAsync(sw.L[0], L0, nl * 16, hipMemcpyDeviceToDevice, s));
    if (nr) HIPCHK(hipMemcpyAsync(sw.R[n2], R0, nr * 16, hipMemcpyDeviceToDevice, s));
    for (int it = 0; it < n_iter; ++it) {
      // right-canonical form: splits moving left, no eigensolve
      for (int i = n2 - 2; i >= 0; --i) sw.step(i, false, false);
      for (int sweep = 0; sweep < sweeps; ++sweep) {
        for (int i = 0; i < n2 - 1; ++i) sw.step(i, true, true);
        const int stop = sweep == sweeps - 1 ? n : 0;
        for (int i = n2 - 2; i >= stop; --i) sw.step(i, false, true);
      }
      // the bond between the cells: one SVD, both gauges
      void* theta = sw.theta_of(n - 1);
      sw.solve(n - 1, theta);
      auto spr = sw.split(n - 1, theta, true);   // U | S V^H
      auto spl = sw.split(n - 1, theta, false);  // U S | V^H
      sw.take(n - 1, *spr);
      energies[it] = sw.e;
      if (it + 1 == n_iter) {
        sw.flush();
        break;
      }
      // the left cell joins the left block, the right cell (V^H) the right block
      sw.update_left(n - 1);  // L[n]
      // device buffers of the next two cells and environments, released in stream order if
      // anything below fails (psi itself is then left unspecified)
      void* rn = nullptr;
      void* rm = nullptr;
      std::vector<void*> t(n2, nullptr);
      std::vector<std::vector<dm_charge>> bq(n2 + 1);
      std::vector<std::vector<int32_t>> bd(n2 + 1);
      std::vector<std::vector<double>> sch(n2 + 1);
      std::vector<int64_t> nt(n2, 0);
      try {
        rn = dev_alloc(std::max<int64_t>(1, sw.env_elems(DM_LAYOUT_ENV_R, n, W[0].ql)) * 16);
        {
          dm_bond bb = psi->bond(n), bc = psi->bond(n + 1);
          check(env_update_right(ly, &bb, &bc, &sw.w[n], sw.R[n + 1], spl->right, rn, DM_FP64, stream));
        }
        // next two cells: the right cell, then the left cell moved by d; the right block's
        // environment moves with it
        for (int i = 0; i <= n; ++i) {
          bq[i] = psi->bq[n + i];
          bd[i] = psi->bd[n + i];
          sch[i] = psi->schmidt[n + i];
        }
        std::vector<int> perm_c;  // the centre bond moved (the new right end)
        for (int i = 1; i <= n; ++i) {
          std::vector<int> perm;
          moved_bond(*psi, i, d, bq[n + i], bd[n + i], perm);
          if (i == n) perm_c = perm;
          sch[n + i] = psi->schmidt[i];
        }
        for (int i = 0; i < n; ++i) {
          t[i] = psi->t[n + i];
          nt[i] = psi->nt[n + i];
          psi->t[n + i] = nullptr;
        }
        for (int i = 0; i < n; ++i) {
          dm_bond oa = psi->bond(i), ob = psi->bond(i + 1);
          const Bond ba = make_bond(&oa, ly), bb = make_bond(&ob, ly);
          std::vector<int> perm;
          std::vector<dm_charge> qa;
          std::vector<int32_t> da;
          moved_bond(*psi, i, d, qa, da, perm);
          dm_bond na{(int32_t)qa.size(), qa.data(), da.data()};
          dm_bond nb{(int32_t)bq[n + i + 1].size(), bq[n + i + 1].data(), bd[n + i + 1].data()};
          const SiteLayout from = site_layout(ba, bb, psi->qs[i].data(), ly);
          const SiteLayout to = site_layout(make_bond(&na, ly), make_bond(&nb, ly), psi->qs[i].data(), ly);
          if (from.P.total != psi->nt[i]) throw DmError{DM_ERR_LAYOUT, "dm_idmrg: site tensor size"};
          t[n + i] = dev_alloc(std::max<int64_t>(1, to.P.total) * 16);
          nt[n + i] = to.P.total;
          permute_panels(from.P, to.P, perm, psi->t[i], t[n + i], s);
          sw.release(psi->t[i]);
        }
        {
          dm_bond oc = psi->bond(n);
          dm_bond nc{(int32_t)bq[n2].size(), bq[n2].data(), bd[n2].data()};
          const EnvRLayout from = envr_layout(make_bond(&oc, ly), W[0].ql, ly);
          const EnvRLayout to = envr_layout(make_bond(&nc, ly), W[0].ql, ly);
          if (from.P.total != sw.env_elems(DM_LAYOUT_ENV_R, n, W[0].ql))
            throw DmError{DM_ERR_LAYOUT, "dm_idmrg: environment size"};
          rm = dev_alloc(std::max<int64_t>(1, to.P.total) * 16);
          permute_panels(from.P, to.P, perm_c, rn, rm, s);
          sw.release(rn);
          void* ln = sw.L[n];
          sw.L[n] = nullptr;
          for (void*& p : sw.L) sw.release(p);
          for (void*& p : sw.R) sw.release(p);
          sw.L[0] = ln;
          sw.R[n2] = rm;
          rm = nullptr;
        }
      } catch (...) {
        sw.release(rn);
        sw.release(rm);
        for (void*& p : t) sw.release(p);
        throw;
      }
      psi->bq = bq;
      psi->bd = bd;
      psi->schmidt = sch;
      psi->t = t;
      psi->nt = nt;
      sw.flush();
    }
    HIPCHK(hipStreamSynchronize(s));
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
