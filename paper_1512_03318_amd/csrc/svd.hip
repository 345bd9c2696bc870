// Block SVD of a two-site wavefunction for the DMRG truncation, FP64 on the device.
//
// The paper reads the Schmidt decomposition off the two-site tensor with every Schmidt
// state labelled by (N, k) (Sec. III C); the decomposition is block diagonal in the
// charge of the middle bond, q(b) = q(a) + q(s1), so it is one SVD per middle sector of
// the matrix M_b[(a, s1), (s2, c)].  Each sector matrix is factorised by one-sided
// (Hestenes) Jacobi in one workgroup: the columns of W (W = M, or W = M^H when M is
// wider than tall, so that W has no more columns than rows) are made mutually
// orthogonal by complex plane rotations, in round-robin order (n/2 disjoint pairs per
// round, n - 1 rounds per sweep, sweeps until no pair has |a_p^H a_q| > eps |a_p||a_q|);
// then sigma_j = |a_j|, u_j = a_j / sigma_j, and the accumulated rotations are V.
// One-sided Jacobi gives singular values to high relative accuracy (Demmel, Veselic,
// "Jacobi's method is more accurate than QR", SIAM J. Matrix Anal. Appl. 13 (1992)).
//
// Rotation of the pair (p, q) with a = |a_p|^2, b = |a_q|^2, g = a_p^H a_q = |g| e^{i phi}:
// the phase is moved into a_q (a_q e^{-i phi}), then the real rotation that diagonalises
// [[a, |g|], [|g|, b]]: zeta = (b - a) / (2 |g|), t = sign(zeta) / (|zeta| + sqrt(1 +
// zeta^2)), c = 1 / sqrt(1 + t^2), s = c t; a_p <- c a_p - s a_q', a_q <- s a_p + c a_q'.
//
// The data movement around it (sector matrices gathered from theta's blocks, the new
// site tensors scattered from the kept singular vectors) is one generic strided copy.
#include "device.hpp"
#include "svd.hpp"

namespace mrd {

// ---------------------------------------------------------------------------------
// dst(i, j) = scale * op(src(i, j)) over rows x cols (complex FP64), with
//   src(i, j) at src + I * s_r + J * s_c, I = rperm ? rperm[i] : i, J = cperm ? cperm[j] : j
//   dst(i, j) at dst + i * d_r + j * d_c,   scale = rscale[i] or cscale[j] or 1,
//   op = conj when conj != 0.  Offsets in complex elements; perm / scale arrays index
//   the copy's own tables (-1: none).
// ---------------------------------------------------------------------------------
__global__ void __launch_bounds__(256) block_copy_kernel(const CopyJob* __restrict__ jobs,
                                                         int32_t njobs, int64_t nitems,
                                                         const int32_t* __restrict__ perm,
                                                         const double* __restrict__ scale,
                                                         const double* __restrict__ src,
                                                         double* __restrict__ dst) {
  const int64_t it = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (it >= nitems) return;
  int lo = 0, hi = njobs - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (jobs[mid].i0 <= it) lo = mid;
    else hi = mid - 1;
  }
  const CopyJob J = jobs[lo];
  const int64_t local = it - J.i0;
  if (local < 0 || local >= (int64_t)J.rows * J.cols) return;
  const int i = (int)(local / J.cols), j = (int)(local % J.cols);
  const int I = J.rperm >= 0 ? perm[J.rperm + i] : i;
  const int Jc = J.cperm >= 0 ? perm[J.cperm + j] : j;
  Cplx<double> v = ldc(src, J.src + (int64_t)I * J.s_r + (int64_t)Jc * J.s_c);
  if (J.conj) v.im = -v.im;
  double f = 1.0;
  if (J.rscale >= 0) f = scale[J.rscale + i];
  if (J.cscale >= 0) f = scale[J.cscale + j];
  stc(dst, J.dst + (int64_t)i * J.d_r + (int64_t)j * J.d_c, f * v.re, f * v.im);
}

int64_t copy_layout(std::vector<CopyJob>& jobs) {
  int64_t n = 0;
  for (CopyJob& j : jobs) {
    j.i0 = n;
    n += (int64_t)j.rows * j.cols;
  }
  return n;
}

hipError_t launch_block_copy(const CopyJob* jobs, int32_t njobs, int64_t nitems, const int32_t* perm,
                             const double* scale, const double* src, double* dst, hipStream_t s) {
  if (nitems == 0) return hipSuccess;
  const int64_t nb = (nitems + 255) / 256;
  if (nb > INT32_MAX) return hipErrorInvalidValue;
  hipLaunchKernelGGL(block_copy_kernel, dim3((uint32_t)nb), dim3(256), 0, s, jobs, njobs, nitems, perm, scale,
                     src, dst);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------------
// One-sided Jacobi SVD of one m x n complex matrix per workgroup (column-major W at
// w_off, n <= m), V (n x n, column-major) at v_off, singular values at sig_off (in
// column order, unsorted).  On return W holds U (unit columns; a column with sigma = 0
// is left as it is).  One wave per column pair of a round: the lanes stride over the
// rows (coalesced), the pair's norms and overlap are wave sums that every lane takes
// from lane 0, so the rotation and the convergence decision are the same in all lanes.
// (One thread per pair walked its two columns row by row, each step waiting on a
// global-memory load: about 10 ms per split at chi = 800.)
// ---------------------------------------------------------------------------------
constexpr int SVD_THREADS = 1024;

__device__ __forceinline__ double svd_wave_total(double x) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) x += __shfl_xor(x, o, 64);
  return __shfl(x, 0, 64);
}

__global__ void __launch_bounds__(SVD_THREADS) svd_jacobi_kernel(const SvdJob* __restrict__ jobs,
                                                                 double* __restrict__ work,
                                                                 double* __restrict__ sig,
                                                                 int32_t max_sweeps) {
  const SvdJob J = jobs[blockIdx.x];
  const int m = J.m, n = J.n;
  double* W = work + 2 * J.w_off;
  double* V = work + 2 * J.v_off;
  __shared__ int rotated;
  for (int64_t e = threadIdx.x; e < (int64_t)n * n; e += blockDim.x) {
    const int r = (int)(e % n), c = (int)(e / n);
    V[2 * e] = r == c ? 1.0 : 0.0;
    V[2 * e + 1] = 0.0;
  }
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6, nwv = blockDim.x >> 6;
  const int np = n + (n & 1);  // round-robin over an even count (one dummy when n is odd)
  constexpr double eps = 1e-15;
  for (int sweep = 0; sweep < max_sweeps; ++sweep) {
    if (threadIdx.x == 0) rotated = 0;
    __syncthreads();
    for (int round = 0; round < np - 1; ++round) {
      for (int k = wv; k < np / 2; k += nwv) {  // uniform over the wave
        // position i of the round: 0 stays, the others rotate by `round`
        auto at = [&](int i) { return i == 0 ? 0 : (i - 1 + round) % (np - 1) + 1; };
        int p = at(k), q = at(np - 1 - k);
        if (p > q) {
          const int t = p;
          p = q;
          q = t;
        }
        if (q >= n) continue;  // the dummy column
        double* ap = W + 2 * (int64_t)p * m;
        double* aq = W + 2 * (int64_t)q * m;
        double a = 0, b = 0, gr = 0, gi = 0;
        for (int r = lane; r < m; r += 64) {
          const double xr = ap[2 * r], xi = ap[2 * r + 1], yr = aq[2 * r], yi = aq[2 * r + 1];
          a += xr * xr + xi * xi;
          b += yr * yr + yi * yi;
          gr += xr * yr + xi * yi;  // conj(x) y
          gi += xr * yi - xi * yr;
        }
        a = svd_wave_total(a);
        b = svd_wave_total(b);
        gr = svd_wave_total(gr);
        gi = svd_wave_total(gi);
        const double g = sqrt(gr * gr + gi * gi);
        if (!(g > eps * sqrt(a) * sqrt(b))) continue;
        if (lane == 0) rotated = 1;
        const double er = gr / g, ei = -gi / g;  // e^{-i phi}
        const double zeta = (b - a) / (2.0 * g);
        const double t = (zeta >= 0 ? 1.0 : -1.0) / (fabs(zeta) + sqrt(1.0 + zeta * zeta));
        const double c = 1.0 / sqrt(1.0 + t * t), s = c * t;
        for (int r = lane; r < m; r += 64) {
          const double xr = ap[2 * r], xi = ap[2 * r + 1];
          const double yr = aq[2 * r] * er - aq[2 * r + 1] * ei, yi = aq[2 * r] * ei + aq[2 * r + 1] * er;
          ap[2 * r] = c * xr - s * yr;
          ap[2 * r + 1] = c * xi - s * yi;
          aq[2 * r] = s * xr + c * yr;
          aq[2 * r + 1] = s * xi + c * yi;
        }
        double* vp = V + 2 * (int64_t)p * n;
        double* vq = V + 2 * (int64_t)q * n;
        for (int r = lane; r < n; r += 64) {
          const double xr = vp[2 * r], xi = vp[2 * r + 1];
          const double yr = vq[2 * r] * er - vq[2 * r + 1] * ei, yi = vq[2 * r] * ei + vq[2 * r + 1] * er;
          vp[2 * r] = c * xr - s * yr;
          vp[2 * r + 1] = c * xi - s * yi;
          vq[2 * r] = s * xr + c * yr;
          vq[2 * r + 1] = s * xi + c * yi;
        }
      }
      __syncthreads();  // the next round's pairs read the columns this round wrote
    }
    const int any = rotated;
    __syncthreads();  // every thread has read the flag before it is cleared again
    if (!any) break;
  }
  for (int j = wv; j < n; j += nwv) {  // one wave per column
    double* aj = W + 2 * (int64_t)j * m;
    double nn = 0;
    for (int r = lane; r < m; r += 64) nn += aj[2 * r] * aj[2 * r] + aj[2 * r + 1] * aj[2 * r + 1];
    const double sgm = sqrt(svd_wave_total(nn));
    if (lane == 0) sig[J.sig_off + j] = sgm;
    if (sgm > 0) {
      const double inv = 1.0 / sgm;
      for (int r = lane; r < m; r += 64) {
        aj[2 * r] *= inv;
        aj[2 * r + 1] *= inv;
      }
    }
  }
}

hipError_t launch_svd_jacobi(const SvdJob* jobs, int32_t njobs, double* work, double* sig,
                             int32_t max_sweeps, hipStream_t s) {
  if (njobs == 0) return hipSuccess;
  hipLaunchKernelGGL(svd_jacobi_kernel, dim3(njobs), dim3(SVD_THREADS), 0, s, jobs, work, sig, max_sweeps);
  return hipGetLastError();
}

}  // namespace mrd
