// Block SVD truncation and the two-site sweep: device job tables (svd.hip) and the
// host side of the split (split.cpp).
#pragma once

#include <cstdint>
#include <vector>

#include <hip/hip_runtime.h>

#include "../../include/mrdmrg.h"

namespace mrd {

// Strided complex FP64 copy of a rows x cols block (svd.hip, block_copy_kernel):
//   dst(i, j) = scale * op(src(I, J)),  I = rperm < 0 ? i : perm[rperm + i],
//   J = cperm < 0 ? j : perm[cperm + j],  src(I, J) at src + I * s_r + J * s_c,
//   dst(i, j) at dst + i * d_r + j * d_c,  scale = scale[rscale + i] (rscale >= 0),
//   scale[cscale + j] (cscale >= 0) or 1,  op = conj when conj.  i0: first flat item.
struct CopyJob {
  int64_t src, dst;
  int64_t s_r, s_c, d_r, d_c;
  int32_t rows, cols;
  int32_t rperm, cperm, rscale, cscale;
  int32_t conj, pad;
  int64_t i0;
};
int64_t copy_layout(std::vector<CopyJob>& jobs);  // fills i0, returns the total items
hipError_t launch_block_copy(const CopyJob* jobs, int32_t njobs, int64_t nitems, const int32_t* perm,
                             const double* scale, const double* src, double* dst, hipStream_t s);

// One Jacobi SVD problem: W (m x n, n <= m, column-major) at w_off and V (n x n) at v_off
// in the work buffer (complex elements), singular values at sig_off (doubles).
struct SvdJob {
  int64_t w_off, v_off, sig_off;
  int32_t m, n;
};
hipError_t launch_svd_jacobi(const SvdJob* jobs, int32_t njobs, double* work, double* sig,
                             int32_t max_sweeps, hipStream_t s);

void dev_free(void* p);  // runtime.cpp

}  // namespace mrd

// Result of dm_theta_split: the new middle bond, the two site tensors (pool blocks, freed
// with the split unless taken over) and the kept Schmidt values.
struct dm_split {
  int ly = 1;
  std::vector<dm_charge> bq;   // new middle bond, increasing charges
  std::vector<int32_t> bdim;
  void* left = nullptr;        // SITE layout of (a, b, qs1), complex128
  int64_t nleft = 0;
  void* right = nullptr;       // SITE layout of (b, c, qs2)
  int64_t nright = 0;
  std::vector<double> schmidt;  // kept values per sector in bond order, descending
  double discarded = 0.0;
  ~dm_split() {
    mrd::dev_free(left);
    mrd::dev_free(right);
  }
};
