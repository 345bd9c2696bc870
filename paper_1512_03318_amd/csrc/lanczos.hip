// Device-resident Lanczos (FP64) for the lowest eigenpair of the two-site H_eff.
//
// Textbook Lanczos with full reorthogonalisation by classical Gram-Schmidt applied
// twice, the tridiagonal eigenproblem solved on the device:
//
//   v_0 = theta / |theta|
//   step j:  w = H v_j
//            h1 = V^H w,  alpha_j = Re h1_j            (V = [v_0 .. v_j])
//            w1 = w - V h1,  h2 = V^H w1
//            beta_j = |w1 - V h2| = sqrt(|w1|^2 - |h2|^2)
//            stop if beta_j <= tol * |T| (|T| = max_i |alpha_i| + beta_i + beta_{i-1})
//            or j = max_iter - 1;  else v_{j+1} = (w1 - V h2) / beta_j
//   lowest eigenpair (E, y) of T_k by bisection on Sturm counts and inverse iteration,
//   Ritz vector V y.
//
// All scalars live in LzState on the device.  Every kernel of one step reads the step
// index and the stop flag from there, so the launches of a step have fixed arguments
// (the step can be captured once as a HIP graph and replayed) and a breakdown turns
// the remaining launches into no-ops without a host round trip.  Partial sums are
// reduced in a fixed order: results are reproducible run to run.
#include "internal.hpp"

namespace mrd {

constexpr int LZ_EPT = 4;                 // elements per thread in streaming kernels
constexpr int LZ_CHUNK = 256 * LZ_EPT;
constexpr int LZ_REG = 32;                // Krylov vectors cached in registers

int lz_nblk(int64_t n) { return (int)((n + LZ_CHUNK - 1) / LZ_CHUNK); }
int lz_nblk1(int64_t n) { return (int)((n + 255) / 256); }

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
__global__ void __launch_bounds__(256) lz_reduce_kernel(const double* __restrict__ partial,
                                                        int32_t nblk, int32_t fixed, int32_t extra,
                                                        const LzState* __restrict__ st,
                                                        double* __restrict__ out) {
  __shared__ double sm[256];
  if (fixed < 0 && st->stop) return;
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

// partial[blk][2i + {0,1}] = sum over the chunk of conj(V_i) w, i <= iter.
__global__ void __launch_bounds__(256) lz_dots_kernel(const double* __restrict__ V, int64_t ld,
                                                      const double* __restrict__ w, int64_t n,
                                                      const LzState* __restrict__ st,
                                                      double* __restrict__ partial) {
  __shared__ double sh[4];
  if (st->stop) return;
  const int nv = st->iter + 1;
  double wr[LZ_EPT], wi[LZ_EPT];
#pragma unroll
  for (int q = 0; q < LZ_EPT; ++q) {
    const int64_t e = (int64_t)blockIdx.x * LZ_CHUNK + q * 256 + threadIdx.x;
    wr[q] = e < n ? w[2 * e] : 0.0;
    wi[q] = e < n ? w[2 * e + 1] : 0.0;
  }
  for (int i = 0; i < nv; ++i) {
    const double* v = V + 2 * (int64_t)i * ld;
    double sr = 0, si = 0;
#pragma unroll
    for (int q = 0; q < LZ_EPT; ++q) {
      const int64_t e = (int64_t)blockIdx.x * LZ_CHUNK + q * 256 + threadIdx.x;
      if (e < n) {
        const double vr = v[2 * e], vi = v[2 * e + 1];
        sr += vr * wr[q] + vi * wi[q];
        si += vr * wi[q] - vi * wr[q];
      }
    }
    sr = block_sum(sr, sh);
    si = block_sum(si, sh);
    if (threadIdx.x == 0) {
      partial[(int64_t)blockIdx.x * 2 * nv + 2 * i] = sr;
      partial[(int64_t)blockIdx.x * 2 * nv + 2 * i + 1] = si;
    }
  }
}

// One element per thread.  w -= V h1 (written back), then the partial projections
// conj(V_i) w and |w|^2 (component 2 nv).  The first LZ_REG Krylov elements of the
// thread are kept in registers between the two passes, so V is read once from memory.
__global__ void __launch_bounds__(256) lz_project_kernel(const double* __restrict__ V, int64_t ld,
                                                         double* __restrict__ w, int64_t n,
                                                         const LzState* __restrict__ st,
                                                         double* __restrict__ partial) {
  __shared__ double sh[4];
  if (st->stop) return;
  const int nv = st->iter + 1;
  const int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x;
  const bool in = e < n;
  double wr = in ? w[2 * e] : 0.0, wi = in ? w[2 * e + 1] : 0.0;
  double vr[LZ_REG], vi[LZ_REG];
#pragma unroll
  for (int i = 0; i < LZ_REG; ++i) {
    vr[i] = 0.0;
    vi[i] = 0.0;
    if (i < nv && in) {
      vr[i] = V[2 * ((int64_t)i * ld + e)];
      vi[i] = V[2 * ((int64_t)i * ld + e) + 1];
    }
  }
  const double* h1 = st->h1;
#pragma unroll
  for (int i = 0; i < LZ_REG; ++i) {
    if (i < nv) {
      const double hr = h1[2 * i], hi = h1[2 * i + 1];
      wr -= hr * vr[i] - hi * vi[i];
      wi -= hr * vi[i] + hi * vr[i];
    }
  }
  for (int i = LZ_REG; i < nv; ++i) {
    const double hr = h1[2 * i], hi = h1[2 * i + 1];
    const double ar = in ? V[2 * ((int64_t)i * ld + e)] : 0.0, ai = in ? V[2 * ((int64_t)i * ld + e) + 1] : 0.0;
    wr -= hr * ar - hi * ai;
    wi -= hr * ai + hi * ar;
  }
  if (in) {
    w[2 * e] = wr;
    w[2 * e + 1] = wi;
  }
  const int ncomp = 2 * nv + 1;
  double* out = partial + (int64_t)blockIdx.x * ncomp;
#pragma unroll
  for (int i = 0; i < LZ_REG; ++i) {
    if (i < nv) {
      const double sr = block_sum(vr[i] * wr + vi[i] * wi, sh);
      const double si = block_sum(vr[i] * wi - vi[i] * wr, sh);
      if (threadIdx.x == 0) {
        out[2 * i] = sr;
        out[2 * i + 1] = si;
      }
    }
  }
  for (int i = LZ_REG; i < nv; ++i) {
    const double ar = in ? V[2 * ((int64_t)i * ld + e)] : 0.0, ai = in ? V[2 * ((int64_t)i * ld + e) + 1] : 0.0;
    const double sr = block_sum(ar * wr + ai * wi, sh);
    const double si = block_sum(ar * wi - ai * wr, sh);
    if (threadIdx.x == 0) {
      out[2 * i] = sr;
      out[2 * i + 1] = si;
    }
  }
  const double nn = block_sum(wr * wr + wi * wi, sh);
  if (threadIdx.x == 0) out[2 * nv] = nn;
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

// Lowest eigenpair of T_k (one thread): bisection to full precision, then inverse
// iteration with partial pivoting (four sweeps).  Writes st->energy and st->y.
__global__ void lz_tridiag_kernel(LzState* st) {
  if (threadIdx.x != 0 || blockIdx.x != 0) return;
  const int k = st->k;
  const double* al = st->alpha;
  const double* be = st->beta;
  double* y = st->y;
  if (k <= 0) return;
  if (k == 1) {
    st->energy = al[0];
    y[0] = 1.0;
    return;
  }
  double lo = al[0], hi = al[0];
  for (int i = 0; i < k; ++i) {
    const double r = (i ? fabs(be[i - 1]) : 0.0) + (i < k - 1 ? fabs(be[i]) : 0.0);
    lo = fmin(lo, al[i] - r);
    hi = fmax(hi, al[i] + r);
  }
  const double scale = fmax(fabs(lo), fabs(hi));
  for (int it = 0; it < 2000 && hi - lo > 2e-16 * scale; ++it) {
    const double mid = 0.5 * (lo + hi);
    if (mid <= lo || mid >= hi) break;
    if (lz_sturm(al, be, k, mid) >= 1)
      hi = mid;
    else
      lo = mid;
  }
  const double lam = 0.5 * (lo + hi);
  st->energy = lam;
  double dd[LZ_MAX], du[LZ_MAX], du2[LZ_MAX], dl[LZ_MAX], b[LZ_MAX];
  for (int i = 0; i < k; ++i) y[i] = 1.0 / sqrt((double)k);
  for (int sweep = 0; sweep < 4; ++sweep) {
    for (int i = 0; i < k; ++i) {
      dd[i] = al[i] - lam;
      du[i] = i < k - 1 ? be[i] : 0.0;
      dl[i] = i < k - 1 ? be[i] : 0.0;
      du2[i] = 0.0;
      b[i] = y[i];
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
    for (int i = 0; i < k; ++i) y[i] = b[i] / nrm;
  }
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
  hipLaunchKernelGGL(lz_reduce_kernel, dim3(1), dim3(256), 0, s, partial, nb, 1, 0, st, &st->scal0);
  hipLaunchKernelGGL(lz_start_scale_kernel, g1(n), dim3(256), 0, s, x, n, st, V, vcur);
  return hipGetLastError();
}

hipError_t lz_launch_step_tail(double* V, int64_t ld, double* w, int64_t n, LzState* st,
                               double* partial, double* vcur, int32_t max_iter, hipStream_t s) {
  const int nb = lz_nblk(n), nb1 = lz_nblk1(n);
  const int maxc = 2 * max_iter + 1;
  hipLaunchKernelGGL(lz_dots_kernel, dim3(nb), dim3(256), 0, s, V, ld, w, n, st, partial);
  hipLaunchKernelGGL(lz_reduce_kernel, dim3(maxc), dim3(256), 0, s, partial, nb, -1, 0, st, st->h1);
  hipLaunchKernelGGL(lz_project_kernel, dim3(nb1), dim3(256), 0, s, V, ld, w, n, st, partial);
  hipLaunchKernelGGL(lz_reduce_kernel, dim3(maxc), dim3(256), 0, s, partial, nb1, -1, 1, st, st->h2);
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
  hipLaunchKernelGGL(lz_reduce_kernel, dim3(2), dim3(256), 0, s, partial, nb, 2, 0, st, st->rq);
  hipLaunchKernelGGL(lz_rq_final_kernel, dim3(1), dim3(64), 0, s, st);
  return hipGetLastError();
}

}  // namespace mrd
