// Host planner: charge matching of block-sparse tensors into GEMM / mixing task tables.
#pragma once

#include <array>
#include <complex>
#include <cstdint>
#include <string>
#include <vector>

#include "../../include/mrdmrg.h"
#include "internal.hpp"

namespace mrd {

struct DmError {
  int code;
  std::string msg;
};

inline dm_charge qadd(dm_charge a, dm_charge b, int ly) {
  return {a.n + b.n, ((a.k + b.k) % ly + ly) % ly};
}
inline dm_charge qsub(dm_charge a, dm_charge b, int ly) {
  return {a.n - b.n, ((a.k - b.k) % ly + ly) % ly};
}
inline bool qeq(dm_charge a, dm_charge b) { return a.n == b.n && a.k == b.k; }

// A validated virtual bond.
struct Bond {
  int ly = 1;
  std::vector<dm_charge> q;  // strictly increasing in (n, k)
  std::vector<int> dim;
  // Sector lookup (the planners call it tens of thousands of times per bond update): a
  // dense table over (n - nlo) * ly + k when the range of n is small, else a binary
  // search of the sorted charges.
  int nlo = 0;
  int64_t nspan = 0;
  std::vector<int32_t> lut;
  int size() const { return (int)q.size(); }
  int find(dm_charge c) const {
    if (c.k < 0 || c.k >= ly) return -1;
    if (!lut.empty()) {
      const int64_t d = (int64_t)c.n - nlo;
      return (d < 0 || d >= nspan) ? -1 : lut[(size_t)d * ly + c.k];
    }
    int lo = 0, hi = size();
    while (lo < hi) {
      const int mid = (lo + hi) >> 1;
      if (q[mid].n < c.n || (q[mid].n == c.n && q[mid].k < c.k)) lo = mid + 1;
      else hi = mid;
    }
    return (lo < size() && q[lo].n == c.n && q[lo].k == c.k) ? lo : -1;
  }
  int64_t total() const {
    int64_t s = 0;
    for (int d : dim) s += d;
    return s;
  }
};
Bond make_bond(const dm_bond* b, int ly);  // throws DmError

// A validated MPO site tensor, dense on the host.
struct MpoSite {
  int dl = 0, dr = 0;
  std::vector<dm_charge> ql, qr;
  dm_charge qs[2];
  std::vector<std::complex<double>> w;  // [dl][2][2][dr]
  std::complex<double> at(int a, int sp, int s, int b) const {
    return w[(((size_t)a * 2 + sp) * 2 + s) * dr + b];
  }
};
MpoSite make_mpo(const dm_mpo_site* m, int ly);  // throws DmError (charge rule checked)

// Panels: one row-major matrix per sector, stored back to back.
struct Panels {
  std::vector<int64_t> off;
  std::vector<int> rows, cols;
  int64_t total = 0;
  void push(int r, int c) {
    off.push_back(total);
    rows.push_back(r);
    cols.push_back(c);
    total += (int64_t)r * c;
  }
};

// SITE layout A[a, s, b]: panel per a, columns (s, b).
struct SiteLayout {
  Panels P;
  std::vector<std::array<int, 2>> b, coff;
};
SiteLayout site_layout(const Bond& a, const Bond& b, const dm_charge qs[2], int ly);

// THETA layout theta[a, s1, s2, c]: panel per a, columns (s1 s2, c).
struct ThetaLayout {
  Panels P;
  std::vector<std::array<int, 4>> c, coff;
};
ThetaLayout theta_layout(const Bond& a, const Bond& c, const dm_charge qs1[2],
                         const dm_charge qs2[2], int ly);

// ENV_L layout L[a', w, a]: panel per ket a, rows (w, a').
struct EnvLLayout {
  Panels P;
  int D = 0;
  std::vector<int> ap, roff;  // [a * D + w]
};
EnvLLayout envl_layout(const Bond& a, const std::vector<dm_charge>& qw, int ly);

// ENV_R layout R[c', w, c]: panel per bra c', columns (w, c).
struct EnvRLayout {
  Panels P;
  int D = 0;
  std::vector<int> c, coff;  // [c' * D + w]
};
EnvRLayout envr_layout(const Bond& c, const std::vector<dm_charge>& qw, int ly);

// Appends the output tiles of problem `prob` (already in st.probs) and sets its
// K-split fields.
void add_tiles(GemmStage& st, int32_t prob, int M, int N);

// Host check that every access of a stage stays inside its buffers (sizes in complex
// elements); throws DmError(DM_ERR_LAYOUT) otherwise.  Run on every table before upload.
void validate(const GemmStage& st, int64_t a_size, int64_t b_size, int64_t c_size);
// Builds the slab form of a mixing stage from its task list.  key[t] names the slab of
// task t (tasks of one slab share rows, cols and source blocks); eb = bytes per complex
// element; each workgroup stages at most lds_budget bytes.
void mix_to_slabs(MixStage& st, const std::vector<int64_t>& key, int eb, int lds_budget);
void validate(const MixStage& st, int64_t src_size, int64_t dst_size);
// Pre-split stages: tiles (and K splits) of problem `prob`; bounds of every access
// (A and B sizes in bf16 elements, C in complex elements).
void add_ps_tiles(PsStage& st, int32_t prob);
void validate(const PsStage& st, int64_t a_size, int64_t b_size, int64_t c_size);
void validate(const std::vector<SplitJob>& jobs, int64_t src_size, int64_t dst_size);

}  // namespace mrd
