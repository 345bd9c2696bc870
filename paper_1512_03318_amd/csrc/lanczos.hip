// Device-resident Lanczos (FP64) for the lowest eigenpair of the two-site H_eff.
//
// Textbook Lanczos with full reorthogonalisation by classical Gram-Schmidt applied
// twice, the tridiagonal eigenproblem solved on the device:
//
//   v_0 = theta / |theta|
//   step j:  w = H v_j
//            h1 = V^H w,  alpha_j = Re h1_j            (V = [v_0 .. v_j])
//            w1 = w - V h1,  h2 = V^H w1        (four streaming passes over V)
//            beta_j = |w1 - V h2| = sqrt(|w1|^2 - |h2|^2)
//            stop if beta_j <= tol * |T| (|T| = max_i |alpha_i| + beta_i + beta_{i-1})
//            or j = max_iter - 1;  else v_{j+1} = (w1 - V h2) / beta_j
//   lowest eigenpair (E, y) of T_k by multisection on Sturm counts and inverse
//   iteration, Ritz vector V y.
//
// All scalars live in LzState on the device.  Every kernel of one step reads the step
// index and the stop flag from there, so the launches of a step have fixed arguments
// (the step can be captured once as a HIP graph and replayed) and a breakdown turns
// the remaining launches into no-ops without a host round trip.  Partial sums are
// reduced in a fixed order: results are reproducible run to run.
#include <algorithm>

#include "internal.hpp"

namespace mrd {

constexpr int LZ_EPT = 4;                 // elements per thread in streaming kernels
constexpr int LZ_CHUNK = 256 * LZ_EPT;

int lz_nblk(int64_t n) { return (int)((n + LZ_CHUNK - 1) / LZ_CHUNK); }
int lz_nblk1(int64_t n) { return (int)((n + 255) / 256); }
// dot-product blocks along the vector: about 16 elements per thread
static int lz_dots_nblk(int64_t n) { return (int)std::max<int64_t>(1, (n + 4095) / 4096); }

__device__ __forceinline__ double wave_sum(double v) {
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
  return v;
}

// Block-sum of one value per thread; result valid in thread 0.  `sh` holds 4 doubles.
__device__ __forceinline__ double block_sum(double v, double* sh) {
  v = wave_sum(v);
  const int wv = threadIdx.x >> 6, lane = threadIdx.x & 63;
  __syncthreads();
  if (lane == 0) sh[wv] = v;
  __syncthreads();
  return (sh[0] + sh[1]) + (sh[2] + sh[3]);
}

__global__ void lz_init_kernel(LzState* st, int32_t max_iter, double tol) {
  if (threadIdx.x != 0 || blockIdx.x != 0) return;
  st->iter = 0;
  st->k = 0;
  st->stop = 0;
  st->bad = 0;
  st->max_iter = max_iter;
  st->tol = tol;
  st->tnorm = 0.0;
  st->energy = 0.0;
}

// partial[blk] = sum over the block's chunk of |x|^2
__global__ void __launch_bounds__(256) lz_norm_kernel(const double* __restrict__ x, int64_t n,
                                                      double* __restrict__ partial) {
  __shared__ double sh[4];
  double s = 0;
#pragma unroll
  for (int q = 0; q < LZ_EPT; ++q) {
    const int64_t e = (int64_t)blockIdx.x * LZ_CHUNK + q * 256 + threadIdx.x;
    if (e < n) s += x[2 * e] * x[2 * e] + x[2 * e + 1] * x[2 * e + 1];
  }
  s = block_sum(s, sh);
  if (threadIdx.x == 0) partial[blockIdx.x] = s;
}

// out[c] = sum_b partial[b * ncomp + c] in a fixed order, c < ncomp.
// ncomp = fixed if >= 0, else 2 * (st->iter + 1) + extra (the current step's width).
// With at_2nv, the result goes to out + 2 * (st->iter + 1) (the |w|^2 slot of h2).
__global__ void __launch_bounds__(256) lz_reduce_kernel(const double* __restrict__ partial,
                                                        int32_t nblk, int32_t fixed, int32_t extra,
                                                        const LzState* __restrict__ st,
                                                        double* __restrict__ out, int32_t at_2nv) {
  __shared__ double sm[256];
  if ((fixed < 0 || at_2nv) && st->stop) return;
  if (at_2nv) out += 2 * (st->iter + 1);
  const int ncomp = fixed >= 0 ? fixed : 2 * (st->iter + 1) + extra;
  const int c = blockIdx.x;
  if (c >= ncomp) return;
  double s = 0;
  for (int b = threadIdx.x; b < nblk; b += 256) s += partial[(int64_t)b * ncomp + c];
  sm[threadIdx.x] = s;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if (threadIdx.x < w) sm[threadIdx.x] += sm[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) out[c] = sm[0];
}

// v_0 = x / |x| into V[0] and vcur; |x|^2 in st->scal0.
__global__ void lz_start_scale_kernel(const double* __restrict__ x, int64_t n,
                                      LzState* __restrict__ st, double* __restrict__ v0,
                                      double* __restrict__ vcur) {
  const double nrm2 = st->scal0;
  if (!(nrm2 > 0.0) || !isfinite(nrm2)) {
    if (blockIdx.x == 0 && threadIdx.x == 0) {
      st->bad = 1;
      st->stop = 1;
    }
    return;
  }
  const double s = 1.0 / sqrt(nrm2);
  const int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (e >= n) return;
  const double a = x[2 * e] * s, b = x[2 * e + 1] * s;
  v0[2 * e] = a;
  v0[2 * e + 1] = b;
  vcur[2 * e] = a;
  vcur[2 * e + 1] = b;
}

constexpr int LZ_G = 4;  // Krylov vectors per dot-product block

// Block sums of NVAL per-thread values with one barrier (wave shuffles, then the four
// wave partials in a fixed order); out[c] for c < nval.
template <int NVAL>
__device__ __forceinline__ void block_sums(const double (&v)[NVAL], int nval, double* sh,
                                           double* out) {
  const int wv = threadIdx.x >> 6, lane = threadIdx.x & 63;
#pragma unroll
  for (int c = 0; c < NVAL; ++c) {
    const double x = wave_sum(v[c]);
    if (lane == 0) sh[c * 4 + wv] = x;
  }
  __syncthreads();
  if (threadIdx.x < nval) {
    const int c = threadIdx.x;
    out[c] = (sh[c * 4] + sh[c * 4 + 1]) + (sh[c * 4 + 2] + sh[c * 4 + 3]);
  }
}

// partial[blockIdx.y][2i + {0,1}] = sum of conj(V_i) x over the elements
// e = (blockIdx.y + gridDim.y q) * 256 + thread, q = 0, 1, ..., for the LZ_G vectors
// i = LZ_G * blockIdx.x + g < nv (nv = iter + 1).  Each thread accumulates many
// elements before the single block reduction; consecutive blocks (same y, next group)
// read the same x elements, which stay in L2.
__global__ void __launch_bounds__(256) lz_dots_kernel(const double* __restrict__ V, int64_t ld,
                                                      const double* __restrict__ x, int64_t n,
                                                      const LzState* __restrict__ st,
                                                      double* __restrict__ partial) {
  __shared__ double sh[4 * 2 * LZ_G];
  if (st->stop) return;
  const int nv = st->iter + 1;
  const int i0 = blockIdx.x * LZ_G;
  if (i0 >= nv) return;
  const double2* xv = reinterpret_cast<const double2*>(x);
  const double2* vv[LZ_G];
#pragma unroll
  for (int g = 0; g < LZ_G; ++g)
    vv[g] = reinterpret_cast<const double2*>(V) + (int64_t)min(i0 + g, nv - 1) * ld;
  double acc[2 * LZ_G];
#pragma unroll
  for (int c = 0; c < 2 * LZ_G; ++c) acc[c] = 0.0;
  const int64_t stride = (int64_t)gridDim.y * 256;
  for (int64_t e = (int64_t)blockIdx.y * 256 + threadIdx.x; e < n; e += stride) {
    const double2 xe = xv[e];
#pragma unroll
    for (int g = 0; g < LZ_G; ++g) {
      const double2 v = vv[g][e];
      acc[2 * g] += v.x * xe.x + v.y * xe.y;
      acc[2 * g + 1] += v.x * xe.y - v.y * xe.x;
    }
  }
  block_sums(acc, 2 * min(LZ_G, nv - i0), sh, partial + blockIdx.y * (int64_t)(2 * nv) + 2 * i0);
}

// w -= V h1 over the nv = iter + 1 Krylov vectors; partial[chunk] = |w_new|^2 over the chunk.
__global__ void __launch_bounds__(256) lz_sub_kernel(const double* __restrict__ V, int64_t ld,
                                                     double* __restrict__ w, int64_t n,
                                                     const LzState* __restrict__ st,
                                                     double* __restrict__ partial) {
  __shared__ double sh[4];
  if (st->stop) return;
  const int nv = st->iter + 1;
  const double* h1 = st->h1;
  double nn = 0;
#pragma unroll
  for (int q = 0; q < LZ_EPT; ++q) {
    const int64_t e = (int64_t)blockIdx.x * LZ_CHUNK + q * 256 + threadIdx.x;
    if (e >= n) continue;
    double wr = w[2 * e], wi = w[2 * e + 1];
    for (int i = 0; i < nv; ++i) {
      const double hr = h1[2 * i], hi = h1[2 * i + 1];
      const double vr = V[2 * ((int64_t)i * ld + e)], vi = V[2 * ((int64_t)i * ld + e) + 1];
      wr -= hr * vr - hi * vi;
      wi -= hr * vi + hi * vr;
    }
    w[2 * e] = wr;
    w[2 * e + 1] = wi;
    nn += wr * wr + wi * wi;
  }
  nn = block_sum(nn, sh);
  if (threadIdx.x == 0) partial[blockIdx.x] = nn;
}

// Scalar part of step j = st->iter: alpha_j, beta_j, |T|, stopping rule.
__global__ void lz_scalar_kernel(LzState* st) {
  if (threadIdx.x != 0 || blockIdx.x != 0 || st->stop) return;
  const int j = st->iter, nv = j + 1;
  const double alpha = st->h1[2 * j];
  double hh = 0;
  for (int i = 0; i < 2 * nv; ++i) hh += st->h2[i] * st->h2[i];
  const double nrm2 = st->h2[2 * nv];
  if (!isfinite(alpha) || !isfinite(nrm2)) {
    st->bad = 1;
    st->stop = 1;
    return;
  }
  const double beta = sqrt(fmax(nrm2 - hh, 0.0));
  st->alpha[j] = alpha;
  st->k = nv;
  const double row = fabs(alpha) + beta + (j > 0 ? st->beta[j - 1] : 0.0);
  st->tnorm = fmax(st->tnorm, row);
  if (beta <= st->tol * st->tnorm || j == st->max_iter - 1) {
    st->stop = 1;
    return;
  }
  st->beta[j] = beta;
  st->inv_beta = 1.0 / beta;
  st->iter = j + 1;
}

// v_{j+1} = (w - V h2) / beta_j into V[j+1] and vcur (runs only if the step continued).
__global__ void __launch_bounds__(256) lz_next_kernel(double* __restrict__ V, int64_t ld,
                                                      const double* __restrict__ w, int64_t n,
                                                      const LzState* __restrict__ st,
                                                      double* __restrict__ vcur) {
  if (st->stop) return;
  const int nv = st->iter;  // already advanced: vectors 0 .. j
  const int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (e >= n) return;
  double wr = w[2 * e], wi = w[2 * e + 1];
  const double* h2 = st->h2;
  for (int i = 0; i < nv; ++i) {
    const double hr = h2[2 * i], hi = h2[2 * i + 1];
    const double vr = V[2 * ((int64_t)i * ld + e)], vi = V[2 * ((int64_t)i * ld + e) + 1];
    wr -= hr * vr - hi * vi;
    wi -= hr * vi + hi * vr;
  }
  const double s = st->inv_beta;
  wr *= s;
  wi *= s;
  double* out = V + 2 * (int64_t)nv * ld;
  out[2 * e] = wr;
  out[2 * e + 1] = wi;
  vcur[2 * e] = wr;
  vcur[2 * e + 1] = wi;
}

// Sturm count: number of eigenvalues of T_k below x.
__device__ int lz_sturm(const double* al, const double* be, int k, double x) {
  int cnt = 0;
  double d = 1.0;
  for (int i = 0; i < k; ++i) {
    const double b2 = i ? be[i - 1] * be[i - 1] : 0.0;
    d = (al[i] - x) - (i ? b2 / d : 0.0);
    if (d == 0.0) d = -1e-300;
    if (d < 0) ++cnt;
  }
  return cnt;
}

// Lowest eigenpair of T_k.  One wavefront brackets the lowest eigenvalue by
// multisection: each lane counts (Sturm sequence) the eigenvalues below its own point
// of a 64-point grid of the current interval, so every round shrinks it 65-fold; then
// lane 0 runs inverse iteration with partial pivoting (four sweeps).  Writes st->energy
// and st->y.
__global__ void __launch_bounds__(64) lz_tridiag_kernel(LzState* st) {
  __shared__ int cnt[64];
  __shared__ double bounds[2];
  __shared__ double dd[LZ_MAX], du[LZ_MAX], du2[LZ_MAX], dl[LZ_MAX], b[LZ_MAX], ys[LZ_MAX];
  const int lane = threadIdx.x;
  const int k = st->k;
  const double* al = st->alpha;
  const double* be = st->beta;
  double* y = st->y;
  if (k <= 0) return;
  if (k == 1) {
    if (lane == 0) {
      st->energy = al[0];
      y[0] = 1.0;
    }
    return;
  }
  if (lane == 0) {
    double lo = al[0], hi = al[0];
    for (int i = 0; i < k; ++i) {
      const double r = (i ? fabs(be[i - 1]) : 0.0) + (i < k - 1 ? fabs(be[i]) : 0.0);
      lo = fmin(lo, al[i] - r);
      hi = fmax(hi, al[i] + r);
    }
    bounds[0] = lo;
    bounds[1] = hi;
  }
  __syncthreads();
  const double scale = fmax(fabs(bounds[0]), fabs(bounds[1]));
  for (int round = 0; round < 64; ++round) {
    const double lo = bounds[0], hi = bounds[1];
    if (!(hi - lo > 2e-16 * scale)) break;
    const double x = lo + (hi - lo) * (double)(lane + 1) / 65.0;
    cnt[lane] = lz_sturm(al, be, k, x);
    __syncthreads();
    if (lane == 0) {
      // first grid point with at least one eigenvalue below it
      int m = 64;
      for (int q = 0; q < 64; ++q)
        if (cnt[q] >= 1) {
          m = q;
          break;
        }
      const double nlo = m == 0 ? lo : lo + (hi - lo) * (double)m / 65.0;
      const double nhi = m == 64 ? hi : lo + (hi - lo) * (double)(m + 1) / 65.0;
      bounds[0] = nlo;
      bounds[1] = nhi;
    }
    __syncthreads();
    if (bounds[0] == lo && bounds[1] == hi) break;  // no progress at this precision
  }
  if (lane != 0) return;
  const double lam = 0.5 * (bounds[0] + bounds[1]);
  st->energy = lam;
  for (int i = 0; i < k; ++i) ys[i] = 1.0 / sqrt((double)k);
  for (int sweep = 0; sweep < 4; ++sweep) {
    for (int i = 0; i < k; ++i) {
      dd[i] = al[i] - lam;
      du[i] = i < k - 1 ? be[i] : 0.0;
      dl[i] = i < k - 1 ? be[i] : 0.0;
      du2[i] = 0.0;
      b[i] = ys[i];
    }
    for (int i = 0; i < k - 1; ++i) {
      if (fabs(dd[i]) >= fabs(dl[i])) {
        if (dd[i] == 0.0) dd[i] = 1e-300 * scale + 1e-300;
        const double f = dl[i] / dd[i];
        dd[i + 1] -= f * du[i];
        b[i + 1] -= f * b[i];
      } else {
        const double f = dd[i] / dl[i];
        dd[i] = dl[i];
        const double t = dd[i + 1];
        dd[i + 1] = du[i] - f * t;
        if (i < k - 2) {
          du2[i] = du[i + 1];
          du[i + 1] = -f * du2[i];
        }
        du[i] = t;
        const double tb = b[i];
        b[i] = b[i + 1];
        b[i + 1] = tb - f * b[i];
      }
    }
    if (dd[k - 1] == 0.0) dd[k - 1] = 1e-300 * scale + 1e-300;
    b[k - 1] /= dd[k - 1];
    b[k - 2] = (b[k - 2] - du[k - 2] * b[k - 1]) / dd[k - 2];
    for (int i = k - 3; i >= 0; --i) b[i] = (b[i] - du[i] * b[i + 1] - du2[i] * b[i + 2]) / dd[i];
    double nrm = 0;
    for (int i = 0; i < k; ++i) nrm += b[i] * b[i];
    nrm = sqrt(nrm);
    for (int i = 0; i < k; ++i) ys[i] = b[i] / nrm;
  }
  for (int i = 0; i < k; ++i) y[i] = ys[i];
}

// out = sum_{i < k} y_i V_i
__global__ void lz_combine_kernel(const double* __restrict__ V, int64_t ld, int64_t n,
                                  const LzState* __restrict__ st, double* __restrict__ out) {
  const int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (e >= n) return;
  const int k = st->k;
  double r = 0, im = 0;
  for (int i = 0; i < k; ++i) {
    const double yi = st->y[i];
    r += yi * V[2 * ((int64_t)i * ld + e)];
    im += yi * V[2 * ((int64_t)i * ld + e) + 1];
  }
  out[2 * e] = r;
  out[2 * e + 1] = im;
}

// partial[blk] = (Re <x, w>, |x|^2) over the chunk (Rayleigh quotient).
__global__ void __launch_bounds__(256) lz_rq_kernel(const double* __restrict__ x,
                                                    const double* __restrict__ w, int64_t n,
                                                    double* __restrict__ partial) {
  __shared__ double sh[4];
  double s = 0, q2 = 0;
#pragma unroll
  for (int q = 0; q < LZ_EPT; ++q) {
    const int64_t e = (int64_t)blockIdx.x * LZ_CHUNK + q * 256 + threadIdx.x;
    if (e < n) {
      s += x[2 * e] * w[2 * e] + x[2 * e + 1] * w[2 * e + 1];
      q2 += x[2 * e] * x[2 * e] + x[2 * e + 1] * x[2 * e + 1];
    }
  }
  s = block_sum(s, sh);
  q2 = block_sum(q2, sh);
  if (threadIdx.x == 0) {
    partial[2 * blockIdx.x] = s;
    partial[2 * blockIdx.x + 1] = q2;
  }
}

__global__ void lz_rq_final_kernel(LzState* st) {
  if (threadIdx.x != 0 || blockIdx.x != 0) return;
  const double e = st->rq[0] / st->rq[1];
  if (!isfinite(e)) st->bad = 1;
  st->energy = e;
}

// ---------------------------------------------------------------------------------
static dim3 g1(int64_t n) { return dim3((uint32_t)((n + 255) / 256)); }

hipError_t lz_launch_init(LzState* st, int32_t max_iter, double tol, hipStream_t s) {
  hipLaunchKernelGGL(lz_init_kernel, dim3(1), dim3(64), 0, s, st, max_iter, tol);
  return hipGetLastError();
}

hipError_t lz_launch_start(const double* x, int64_t n, LzState* st, double* partial, double* V,
                           double* vcur, hipStream_t s) {
  const int nb = lz_nblk(n);
  hipLaunchKernelGGL(lz_norm_kernel, dim3(nb), dim3(256), 0, s, x, n, partial);
  hipLaunchKernelGGL(lz_reduce_kernel, dim3(1), dim3(256), 0, s, partial, nb, 1, 0, st, &st->scal0, 0);
  hipLaunchKernelGGL(lz_start_scale_kernel, g1(n), dim3(256), 0, s, x, n, st, V, vcur);
  return hipGetLastError();
}

hipError_t lz_launch_step_tail(double* V, int64_t ld, double* w, int64_t n, LzState* st,
                               double* partial, double* vcur, int32_t max_iter, hipStream_t s) {
  const int nb = lz_nblk(n), nb1 = lz_dots_nblk(n);
  const int maxc = 2 * max_iter + 1;
  const dim3 gd((max_iter + LZ_G - 1) / LZ_G, nb1);
  double* pnorm = partial + (size_t)nb1 * maxc;
  hipLaunchKernelGGL(lz_dots_kernel, gd, dim3(256), 0, s, V, ld, w, n, st, partial);
  hipLaunchKernelGGL(lz_reduce_kernel, dim3(maxc), dim3(256), 0, s, partial, nb1, -1, 0, st, st->h1, 0);
  hipLaunchKernelGGL(lz_sub_kernel, dim3(nb), dim3(256), 0, s, V, ld, w, n, st, pnorm);
  hipLaunchKernelGGL(lz_dots_kernel, gd, dim3(256), 0, s, V, ld, w, n, st, partial);
  hipLaunchKernelGGL(lz_reduce_kernel, dim3(maxc), dim3(256), 0, s, partial, nb1, -1, 0, st, st->h2, 0);
  hipLaunchKernelGGL(lz_reduce_kernel, dim3(1), dim3(256), 0, s, pnorm, nb, 1, 0, st, st->h2, 1);
  hipLaunchKernelGGL(lz_scalar_kernel, dim3(1), dim3(64), 0, s, st);
  hipLaunchKernelGGL(lz_next_kernel, g1(n), dim3(256), 0, s, V, ld, w, n, st, vcur);
  return hipGetLastError();
}

hipError_t lz_launch_finish(const double* V, int64_t ld, int64_t n, LzState* st, double* out,
                            hipStream_t s) {
  hipLaunchKernelGGL(lz_tridiag_kernel, dim3(1), dim3(64), 0, s, st);
  hipLaunchKernelGGL(lz_combine_kernel, g1(n), dim3(256), 0, s, V, ld, n, st, out);
  return hipGetLastError();
}

hipError_t lz_launch_rq(const double* x, const double* w, int64_t n, LzState* st, double* partial,
                        hipStream_t s) {
  const int nb = lz_nblk(n);
  hipLaunchKernelGGL(lz_rq_kernel, dim3(nb), dim3(256), 0, s, x, w, n, partial);
  hipLaunchKernelGGL(lz_reduce_kernel, dim3(2), dim3(256), 0, s, partial, nb, 2, 0, st, st->rq, 0);
  hipLaunchKernelGGL(lz_rq_final_kernel, dim3(1), dim3(64), 0, s, st);
  return hipGetLastError();
}

}  // namespace mrd
