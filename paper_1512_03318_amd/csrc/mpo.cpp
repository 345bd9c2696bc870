// Hofstadter-cylinder MPO from a finite-state machine (Sec. IV A-D of arXiv:1512.03318).
//
// Each term of eq. H is a path R -> ... -> F through the machine; the transition taken
// at orbital i places the term's local operator there (identity on R -> R, F -> F).
// A state in the middle of a path is labelled by (term family, the family's fixed
// parameters, which of the term's operators are already placed, and the charge they
// carry); for the mixed basis the charge includes the momentum modulo Ly, which is the
// role of the momentum-labelled states A_mu(k), C_mu(k) of Sec. IV D.  States exist only
// along actual term paths (the trimming of Sec. IV D).  Proportional states are then
// merged exactly (column / row deparallelisation).
//
// Fermion signs follow eq. JW: operators are placed in chain order; placing an operator
// while an earlier operator of the written product is still unplaced exchanges two
// fermions (factor -1); the local operator is the product of the operators placed on
// that orbital (written order) times Z = (-1)^n when an odd number of the term's
// fermion operators remain to the right; orbitals without operators carry Z or 1 by the
// same rule.
#include <algorithm>
#include <array>
#include <cmath>
#include <complex>
#include <map>
#include <memory>
#include <string>
#include <unordered_map>
#include <vector>

#include "../../include/mrdmrg.h"
#include "internal.hpp"

namespace {

using cplx = std::complex<double>;
using Mat2 = std::array<cplx, 4>;  // <s'|op|s> at [s' * 2 + s]

const Mat2 kI = {1, 0, 0, 1};
const Mat2 kZ = {1, 0, 0, -1};
const Mat2 kCdag = {0, 0, 1, 0};  // |1><0|
const Mat2 kC = {0, 1, 0, 0};     // |0><1|
const Mat2 kN = {0, 0, 0, 1};

Mat2 mul(const Mat2& a, const Mat2& b) {
  return {a[0] * b[0] + a[1] * b[2], a[0] * b[1] + a[1] * b[3], a[2] * b[0] + a[3] * b[2],
          a[2] * b[1] + a[3] * b[3]};
}

struct Op {
  int site;
  char kind;  // '+', '-', 'n'
};

struct Term {
  std::vector<Op> ops;
  std::array<int, 4> fam;  // family id and its fixed parameters
  cplx fam_coef;
  std::vector<cplx> role_f;
  std::vector<std::array<int, 2>> charge;  // (dN, dk) per operator
};

// State key: family (4 ints), placed-operator mask, dN, dk.  R and F are special.
using Key = std::array<int, 7>;
const Key kR = {-1, 0, 0, 0, 0, 0, 0};
const Key kF = {-2, 0, 0, 0, 0, 0, 0};

struct KeyHash {
  size_t operator()(const Key& k) const {
    size_t h = 1469598103934665603ull;
    for (int v : k) h = (h ^ (size_t)(uint32_t)v) * 1099511628211ull;
    return h;
  }
};

struct Trans {
  Key in, out;
  Mat2 m;
};

class Builder {
 public:
  Builder(int n, int ly) : n_(n), ly_(ly), trans_(n) {}

  void add(const Term& t) {
    const int nr = (int)t.ops.size();
    int lo = n_, hi = -1;
    for (auto& o : t.ops) {
      lo = std::min(lo, o.site);
      hi = std::max(hi, o.site);
    }
    int placed = 0, dN = 0, dk = 0;
    Key key = kR;
    for (int i = lo; i <= hi; ++i) {
      std::vector<int> here;
      for (int r = 0; r < nr; ++r)
        if (t.ops[r].site == i) here.push_back(r);
      if (here.empty()) {
        int rem = 0;
        for (int r = 0; r < nr; ++r)
          if (!(placed >> r & 1) && t.ops[r].kind != 'n') ++rem;
        reg(i, key, key, key, rem % 2 ? kZ : kI);
        continue;
      }
      int after = placed;
      for (int r : here) after |= 1 << r;
      Mat2 m = kI;
      for (int r : here) m = mul(m, t.ops[r].kind == '+' ? kCdag : t.ops[r].kind == '-' ? kC : kN);
      int rem = 0;
      for (int r = 0; r < nr; ++r)
        if (!(after >> r & 1) && t.ops[r].kind != 'n') ++rem;
      if (rem % 2) m = mul(m, kZ);
      double sign = 1.0;
      for (int r : here) {
        if (t.ops[r].kind == 'n') continue;
        int earlier = 0;
        for (int q = 0; q < r; ++q)
          if (!(after >> q & 1) && t.ops[q].kind != 'n') ++earlier;
        if (earlier % 2) sign = -sign;
      }
      cplx coef = sign * (placed == 0 ? t.fam_coef : cplx(1.0));
      for (int r : here) {
        coef *= t.role_f[r];
        dN += t.charge[r][0];
        dk += t.charge[r][1];
      }
      for (auto& v : m) v *= coef;
      if (after == (1 << nr) - 1) {
        Key kid = {-3, t.fam[0], t.fam[1], t.fam[2], t.fam[3], 0, 0};
        reg(i, key, kid, kF, m);
        key = kF;
      } else {
        Key nk = {t.fam[0], t.fam[1], t.fam[2], t.fam[3], after, dN, ((dk % ly_) + ly_) % ly_};
        reg(i, key, nk, nk, m);
        key = nk;
      }
      placed = after;
    }
  }

  dm_mpo* finish(const std::vector<int>& mom, int pair_family);

 private:
  void reg(int site, const Key& in, const Key& kid, const Key& out, const Mat2& m) {
    auto& tab = trans_[site];
    auto& inner = tab[in];
    auto it = inner.find(kid);
    if (it != inner.end()) {
      for (int q = 0; q < 4; ++q)
        if (std::abs(it->second.m[q] - m[q]) > 1e-12)
          throw std::runtime_error("inconsistent FSM transition");
      return;
    }
    inner.emplace(kid, Trans{in, out, m});
  }

  int n_, ly_;
  std::vector<std::unordered_map<Key, std::unordered_map<Key, Trans, KeyHash>, KeyHash>> trans_;
};

}  // namespace

struct dm_mpo {
  int ly = 1;
  std::vector<int> D;                                // n + 1 bond dimensions
  std::vector<std::vector<dm_charge>> q;             // per bond
  std::vector<std::vector<double>> w;                // per site: [dl][2][2][dr] interleaved
  std::vector<std::array<dm_charge, 2>> qs;          // per site
};

namespace {

dm_charge key_charge(const Key& k) {
  if (k == kR || k == kF) return {0, 0};
  return {k[5], k[6]};
}

bool key_less(const Key& a, const Key& b) {
  auto rank = [](const Key& k) { return k == kR ? 0 : (k == kF ? 2 : 1); };
  if (rank(a) != rank(b)) return rank(a) < rank(b);
  dm_charge qa = key_charge(a), qb = key_charge(b);
  if (qa.n != qb.n) return qa.n < qb.n;
  if (qa.k != qb.k) return qa.k < qb.k;
  return a < b;
}

// Dense MPO: per site W[a][sp][s][b] complex, with bond charges; merges proportional
// columns / rows (exact rewriting) until nothing changes.
struct Dense {
  std::vector<std::vector<cplx>> W;  // [dl*4*dr]
  std::vector<int> D;
  std::vector<std::vector<dm_charge>> q;
  std::vector<std::vector<char>> keep_fixed;  // R / F flags per bond state
  cplx& at(int i, int a, int x, int b) { return W[i][((size_t)a * 4 + x) * D[i + 1] + b]; }
};

// Rounding in the phase products leaves about 1e-17 where an entry is zero (a cosine of
// a right angle, the imaginary part of e^{ia} e^{-ia}); such components are set to
// exact zeros, so that proportionality is decided on the true nonzero pattern.
void snap(std::vector<cplx>& w) {
  double mx = 0;
  for (auto& v : w) mx = std::max(mx, std::abs(v));
  const double tol = 1e-14 * mx;
  for (auto& v : w) v = cplx(std::abs(v.real()) <= tol ? 0.0 : v.real(), std::abs(v.imag()) <= tol ? 0.0 : v.imag());
}

// true with lambda when v_j = lambda v_k: the same nonzero pattern (components above
// 1e-14 of each vector's largest), lambda taken at v_j's largest component, and the
// difference within 1e-13 of v_j's largest.  Patterns are compared with thresholds so
// that rounding residue (left by merges and phase products) never defines lambda.
bool parallel(const std::vector<cplx>& vj, const std::vector<cplx>& vk, cplx* lam) {
  double mj = 0, mk = 0;
  size_t p = 0;
  for (size_t i = 0; i < vj.size(); ++i) {
    if (std::abs(vj[i]) > mj) {
      mj = std::abs(vj[i]);
      p = i;
    }
    mk = std::max(mk, std::abs(vk[i]));
  }
  if (mj == 0 || mk == 0) return false;
  for (size_t i = 0; i < vj.size(); ++i)
    if ((std::abs(vj[i]) > 1e-14 * mj) != (std::abs(vk[i]) > 1e-14 * mk)) return false;
  const cplx l = vj[p] / vk[p];
  for (size_t i = 0; i < vj.size(); ++i)
    if (std::abs(vj[i] - l * vk[i]) > 1e-13 * mj) return false;
  *lam = l;
  return true;
}

void deparallelise(Dense& d) {
  const int n = (int)d.W.size();
  for (int round = 0; round < 50; ++round) {
    bool changed = false;
    // columns of W[i] (states at bond i + 1)
    for (int i = 0; i + 1 < n; ++i) {
      const int dl = d.D[i], dm = d.D[i + 1], dr = d.D[i + 2];
      std::vector<std::vector<cplx>> col(dm, std::vector<cplx>((size_t)dl * 4));
      for (int a = 0; a < dl; ++a)
        for (int x = 0; x < 4; ++x)
          for (int b = 0; b < dm; ++b) col[b][(size_t)a * 4 + x] = d.at(i, a, x, b);
      std::vector<int> keep;
      std::vector<std::vector<cplx>> next = {};
      std::vector<cplx> rows_next(d.W[i + 1]);
      auto rn = [&](int a, int x, int b) -> cplx& { return rows_next[((size_t)a * 4 + x) * dr + b]; };
      for (int j = 0; j < dm; ++j) {
        bool zero = true;
        for (auto& v : col[j]) zero = zero && v == cplx(0);
        if (zero && !d.keep_fixed[i + 1][j]) {
          changed = true;
          continue;
        }
        bool merged = false;
        if (!d.keep_fixed[i + 1][j])
          for (int k : keep) {
            if (d.q[i + 1][k].n != d.q[i + 1][j].n || d.q[i + 1][k].k != d.q[i + 1][j].k) continue;
            cplx lam;
            if (parallel(col[j], col[k], &lam)) {
              for (int x = 0; x < 4; ++x)
                for (int b = 0; b < dr; ++b) rn(k, x, b) += lam * rn(j, x, b);
              merged = true;
              changed = true;
              break;
            }
          }
        if (!merged) keep.push_back(j);
      }
      if ((int)keep.size() == dm) continue;
      const int nm = (int)keep.size();
      std::vector<cplx> A((size_t)dl * 4 * nm), B((size_t)nm * 4 * dr);
      for (int a = 0; a < dl; ++a)
        for (int x = 0; x < 4; ++x)
          for (int b = 0; b < nm; ++b) A[((size_t)a * 4 + x) * nm + b] = d.at(i, a, x, keep[b]);
      for (int a = 0; a < nm; ++a)
        for (int x = 0; x < 4; ++x)
          for (int b = 0; b < dr; ++b) B[((size_t)a * 4 + x) * dr + b] = rn(keep[a], x, b);
      std::vector<dm_charge> nq;
      std::vector<char> nf;
      for (int k : keep) {
        nq.push_back(d.q[i + 1][k]);
        nf.push_back(d.keep_fixed[i + 1][k]);
      }
      snap(A);
      snap(B);
      d.W[i] = A;
      d.W[i + 1] = B;
      d.D[i + 1] = nm;
      d.q[i + 1] = nq;
      d.keep_fixed[i + 1] = nf;
    }
    // rows of W[i] (states at bond i), right to left
    for (int i = n - 1; i >= 1; --i) {
      const int dl = d.D[i - 1], dm = d.D[i], dr = d.D[i + 1];
      std::vector<std::vector<cplx>> row(dm, std::vector<cplx>((size_t)4 * dr));
      for (int a = 0; a < dm; ++a)
        for (int x = 0; x < 4; ++x)
          for (int b = 0; b < dr; ++b) row[a][(size_t)x * dr + b] = d.at(i, a, x, b);
      std::vector<cplx> prev(d.W[i - 1]);
      auto pv = [&](int a, int x, int b) -> cplx& { return prev[((size_t)a * 4 + x) * dm + b]; };
      std::vector<int> keep;
      for (int j = 0; j < dm; ++j) {
        bool zero = true;
        for (auto& v : row[j]) zero = zero && v == cplx(0);
        if (zero && !d.keep_fixed[i][j]) {
          changed = true;
          continue;
        }
        bool merged = false;
        if (!d.keep_fixed[i][j])
          for (int k : keep) {
            if (d.q[i][k].n != d.q[i][j].n || d.q[i][k].k != d.q[i][j].k) continue;
            cplx lam;
            if (parallel(row[j], row[k], &lam)) {
              for (int a = 0; a < dl; ++a)
                for (int x = 0; x < 4; ++x) pv(a, x, k) += lam * pv(a, x, j);
              merged = true;
              changed = true;
              break;
            }
          }
        if (!merged) keep.push_back(j);
      }
      if ((int)keep.size() == dm) continue;
      const int nm = (int)keep.size();
      std::vector<cplx> A((size_t)dl * 4 * nm), B((size_t)nm * 4 * dr);
      for (int a = 0; a < dl; ++a)
        for (int x = 0; x < 4; ++x)
          for (int b = 0; b < nm; ++b) A[((size_t)a * 4 + x) * nm + b] = pv(a, x, keep[b]);
      for (int a = 0; a < nm; ++a)
        for (int x = 0; x < 4; ++x)
          for (int b = 0; b < dr; ++b) B[((size_t)a * 4 + x) * dr + b] = d.at(i, keep[a], x, b);
      std::vector<dm_charge> nq;
      std::vector<char> nf;
      for (int k : keep) {
        nq.push_back(d.q[i][k]);
        nf.push_back(d.keep_fixed[i][k]);
      }
      snap(A);
      snap(B);
      d.W[i - 1] = A;
      d.W[i] = B;
      d.D[i] = nm;
      d.q[i] = nq;
      d.keep_fixed[i] = nf;
    }
    if (!changed) break;
  }
}

}  // namespace

dm_mpo* Builder::finish(const std::vector<int>& mom, int pair_family) {
  for (int i = 0; i < n_; ++i) {
    reg(i, kR, kR, kR, kI);
    reg(i, kF, kF, kF, kI);
  }
  // states per bond, reachable from R at bond 0 and co-reachable to F at bond n
  std::vector<std::vector<Key>> fwd(n_ + 1), bwd(n_ + 1);
  std::vector<std::unordered_map<Key, char, KeyHash>> live(n_ + 1);
  {
    std::vector<std::unordered_map<Key, char, KeyHash>> f(n_ + 1), b(n_ + 1);
    f[0][kR] = 1;
    for (int i = 0; i < n_; ++i)
      for (auto& kv : trans_[i])
        if (f[i].count(kv.first))
          for (auto& t : kv.second) f[i + 1][t.second.out] = 1;
    b[n_][kF] = 1;
    for (int i = n_ - 1; i >= 0; --i)
      for (auto& kv : trans_[i])
        for (auto& t : kv.second)
          if (b[i + 1].count(t.second.out)) {
            b[i][kv.first] = 1;
            break;
          }
    for (int i = 0; i <= n_; ++i)
      for (auto& kv : f[i])
        if (b[i].count(kv.first)) live[i][kv.first] = 1;
  }
  Dense d;
  std::vector<std::unordered_map<Key, int, KeyHash>> idx(n_ + 1);
  d.D.resize(n_ + 1);
  d.q.resize(n_ + 1);
  d.keep_fixed.resize(n_ + 1);
  for (int i = 0; i <= n_; ++i) {
    std::vector<Key> ks;
    for (auto& kv : live[i]) ks.push_back(kv.first);
    std::sort(ks.begin(), ks.end(), key_less);
    for (size_t j = 0; j < ks.size(); ++j) {
      idx[i][ks[j]] = (int)j;
      d.q[i].push_back(key_charge(ks[j]));
      d.keep_fixed[i].push_back(ks[j] == kR || ks[j] == kF);
    }
    d.D[i] = (int)ks.size();
  }
  d.W.resize(n_);
  for (int i = 0; i < n_; ++i) {
    d.W[i].assign((size_t)d.D[i] * 4 * d.D[i + 1], cplx(0));
    for (auto& kv : trans_[i]) {
      auto ia = idx[i].find(kv.first);
      if (ia == idx[i].end()) continue;
      for (auto& t : kv.second) {
        auto ib = idx[i + 1].find(t.second.out);
        if (ib == idx[i + 1].end()) continue;
        for (int x = 0; x < 4; ++x) d.at(i, ia->second, x, ib->second) += t.second.m[x];
      }
    }
  }
  for (auto& w : d.W) snap(w);
  if (pair_family > 0) {
    // Eq. rot: the two phase branches s = +1, -1 of family `pair_family` (key[2] = s)
    // carry conjugate phases, so with the bond basis change that maps each pair (p, m)
    // to ((e_p + e_m) / sqrt 2, i (e_p - e_m) / sqrt 2) every W[i] = T_i^-1 W[i] T_{i+1}
    // becomes real; a pair shares its charge, so the block structure is unchanged.
    std::vector<std::vector<std::pair<int, int>>> pairs(n_ + 1);
    for (int b = 0; b <= n_; ++b)
      for (auto& kv : idx[b]) {
        const Key& k = kv.first;
        if (k[0] != pair_family || k[2] != 1) continue;
        Key q = k;
        q[2] = -1;
        auto it = idx[b].find(q);
        if (it == idx[b].end()) throw std::runtime_error("eq. rot: a phase branch state has no partner");
        pairs[b].push_back({kv.second, it->second});
      }
    const double r2 = 1.0 / std::sqrt(2.0);
    const cplx I(0.0, 1.0);
    for (int i = 0; i < n_; ++i) {
      for (auto& pm : pairs[i + 1])  // columns: times T_{i+1}
        for (int a = 0; a < d.D[i]; ++a)
          for (int x = 0; x < 4; ++x) {
            const cplx cp = d.at(i, a, x, pm.first), cm = d.at(i, a, x, pm.second);
            d.at(i, a, x, pm.first) = (cp + cm) * r2;
            d.at(i, a, x, pm.second) = I * (cp - cm) * r2;
          }
      for (auto& pm : pairs[i])  // rows: T_i^-1 from the left
        for (int x = 0; x < 4; ++x)
          for (int b = 0; b < d.D[i + 1]; ++b) {
            const cplx rp = d.at(i, pm.first, x, b), rm = d.at(i, pm.second, x, b);
            d.at(i, pm.first, x, b) = (rp + rm) * r2;
            d.at(i, pm.second, x, b) = I * (rm - rp) * r2;
          }
      double mx = 0, mi = 0;
      for (auto& v : d.W[i]) {
        mx = std::max(mx, std::abs(v));
        mi = std::max(mi, std::abs(v.imag()));
      }
      if (mi > 1e-12 * std::max(1.0, mx)) throw std::runtime_error("eq. rot: rotated MPO is not real");
      for (auto& v : d.W[i]) v = cplx(v.real(), 0.0);
      snap(d.W[i]);
    }
  }
  deparallelise(d);
  auto* m = new dm_mpo;
  m->ly = ly_;
  m->D = d.D;
  m->q = d.q;
  for (int i = 0; i < n_; ++i) {
    std::vector<double> w((size_t)d.D[i] * 4 * d.D[i + 1] * 2);
    for (size_t e = 0; e < d.W[i].size(); ++e) {
      w[2 * e] = d.W[i][e].real();
      w[2 * e + 1] = d.W[i][e].imag();
    }
    m->w.push_back(std::move(w));
    m->qs.push_back({dm_charge{0, 0}, dm_charge{1, mom[i] % ly_}});
  }
  return m;
}

namespace {
void mpo_error(const std::string& m) { mrd::set_last_error(m); }

enum Fam { ONSITE = 1, HOP, INTRA, INTER, RXHOP, RYHOP, RXINT, RYINT };

void add_mixed(Builder& B, int Ly, int Lx, double phi, double t, double V) {
  const double al = 2.0 * M_PI / Ly;
  auto o = [&](int x, int m) { return x * Ly + m; };
  for (int x = 0; x < Lx; ++x) {
    for (int m = 0; m < Ly; ++m)  // -2t cos(k + x phi) n_{x,k}  (eq. H_kin)
      B.add({{{o(x, m), 'n'}}, {ONSITE, x, 0, 0}, 1.0, {-2.0 * t * std::cos(al * m + x * phi)}, {{0, 0}}});
    if (x + 1 < Lx)
      for (int m = 0; m < Ly; ++m) {  // -t (c+_{x,k} c_{x+1,k} + h.c.)
        B.add({{{o(x, m), '+'}, {o(x + 1, m), '-'}}, {HOP, x, 1, 0}, -t, {1.0, 1.0},
               {{1, m}, {-1, (Ly - m) % Ly}}});
        B.add({{{o(x + 1, m), '+'}, {o(x, m), '-'}}, {HOP, x, -1, 0}, -t, {1.0, 1.0},
               {{1, m}, {-1, (Ly - m) % Ly}}});
      }
    // (V/L) sum_q cos q n_{x,q} n_{x,-q}, cos q = (e^{iq} + e^{-iq}) / 2 on the first bilinear
    for (int s : {1, -1})
      for (int a = 0; a < Ly; ++a)
        for (int b = 0; b < Ly; ++b)
          for (int c = 0; c < Ly; ++c) {
            const int d = ((a - b + c) % Ly + Ly) % Ly;
            B.add({{{o(x, a), '+'}, {o(x, b), '-'}, {o(x, c), '+'}, {o(x, d), '-'}},
                   {INTRA, x, s, 0},
                   V / (2.0 * Ly),
                   {std::polar(1.0, s * al * a), std::polar(1.0, -s * al * b), 1.0, 1.0},
                   {{1, a}, {-1, (Ly - b) % Ly}, {1, c}, {-1, (Ly - d) % Ly}}});
          }
    // (V/L) sum_q n_{x+1,q} n_{x,-q}
    if (x + 1 < Lx)
      for (int a = 0; a < Ly; ++a)
        for (int b = 0; b < Ly; ++b)
          for (int c = 0; c < Ly; ++c) {
            const int d = ((a - b + c) % Ly + Ly) % Ly;
            B.add({{{o(x + 1, a), '+'}, {o(x + 1, b), '-'}, {o(x, c), '+'}, {o(x, d), '-'}},
                   {INTER, x, 0, 0},
                   V / Ly,
                   {1.0, 1.0, 1.0, 1.0},
                   {{1, a}, {-1, (Ly - b) % Ly}, {1, c}, {-1, (Ly - d) % Ly}}});
          }
  }
}

void add_real(Builder& B, int Ly, int Lx, double phi, double t, double V) {
  auto o = [&](int x, int y) { return x * Ly + y; };
  for (int x = 0; x < Lx; ++x) {
    const cplx ph = std::polar(1.0, x * phi);
    for (int y = 0; y < Ly; ++y) {
      const int yp = (y + 1) % Ly;
      if (x + 1 < Lx) {
        B.add({{{o(x, y), '+'}, {o(x + 1, y), '-'}}, {RXHOP, x, y, 1}, -t, {1.0, 1.0}, {{1, 0}, {-1, 0}}});
        B.add({{{o(x + 1, y), '+'}, {o(x, y), '-'}}, {RXHOP, x, y, -1}, -t, {1.0, 1.0}, {{1, 0}, {-1, 0}}});
        B.add({{{o(x, y), 'n'}, {o(x + 1, y), 'n'}}, {RXINT, x, y, 0}, V, {1.0, 1.0}, {{0, 0}, {0, 0}}});
      }
      B.add({{{o(x, y), '+'}, {o(x, yp), '-'}}, {RYHOP, x, y, 1}, -t * ph, {1.0, 1.0}, {{1, 0}, {-1, 0}}});
      B.add({{{o(x, yp), '+'}, {o(x, y), '-'}}, {RYHOP, x, y, -1}, -t * std::conj(ph), {1.0, 1.0},
             {{1, 0}, {-1, 0}}});
      B.add({{{o(x, y), 'n'}, {o(x, yp), 'n'}}, {RYINT, x, y, 0}, V, {1.0, 1.0}, {{0, 0}, {0, 0}}});
    }
  }
}
}  // namespace

extern "C" int dm_mpo_hofstadter(int32_t Ly, int32_t Lx, int32_t p, int32_t q, double t,
                                 double V, int32_t basis, dm_mpo** out) {
  if (!out) {
    mpo_error("null output");
    return DM_ERR_ARG;
  }
  *out = nullptr;
  if (Ly < 3 || Lx < 1 || q == 0 || basis < 0 || basis > 2) {
    mpo_error("need Ly >= 3, Lx >= 1, q != 0, basis 0, 1 or 2");
    return DM_ERR_ARG;
  }
  try {
    const int n = Ly * Lx;
    const bool mixed = basis != 1;
    const int ly = mixed ? Ly : 1;
    const double phi = 2.0 * M_PI * (double)p / (double)q;
    Builder B(n, ly);
    if (mixed)
      add_mixed(B, Ly, Lx, phi, t, V);
    else
      add_real(B, Ly, Lx, phi, t, V);
    std::vector<int> mom(n);
    for (int i = 0; i < n; ++i) mom[i] = mixed ? i % Ly : 0;
    *out = B.finish(mom, basis == 2 ? INTRA : 0);
    return DM_OK;
  } catch (const std::exception& e) {
    mpo_error(e.what());
    return DM_ERR_ARG;
  }
}

extern "C" int dm_mpo_n_sites(const dm_mpo* m) { return m ? (int)m->w.size() : 0; }

extern "C" int dm_mpo_site_get(const dm_mpo* m, int32_t i, dm_mpo_site* out) {
  if (!m || !out || i < 0 || i >= (int)m->w.size()) {
    mpo_error("dm_mpo_site_get: bad handle or site index");
    return DM_ERR_ARG;
  }
  out->dl = m->D[i];
  out->dr = m->D[i + 1];
  out->ql = m->q[i].data();
  out->qr = m->q[i + 1].data();
  out->qs[0] = m->qs[i][0];
  out->qs[1] = m->qs[i][1];
  out->w = m->w[i].data();
  return DM_OK;
}

extern "C" void dm_mpo_destroy(dm_mpo* m) { delete m; }
