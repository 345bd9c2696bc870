// HIP kernels for gfx950 (CDNA4): grouped complex block GEMMs on MFMA, sparse MPO
// mixing, precision casts and the FP64 Lanczos vector kernels.
//
// Complex data is interleaved (re, im).  A complex product on real MFMA is four real
// products: Cr += Ar Br - Ai Bi, Ci += Ar Bi + Ai Br.
#include "internal.hpp"

namespace mrd {

typedef double v4d __attribute__((ext_vector_type(4)));
typedef float v4f __attribute__((ext_vector_type(4)));

template <typename T>
struct Mfma;

// Result rows differ between the two 16x16x4 variants (measured on gfx950): the FP64
// form puts row lane/16 + 4r in register r, the FP32 form row 4 (lane/16) + r.
template <>
struct Mfma<double> {
  typedef v4d acc_t;
  static __device__ __forceinline__ acc_t mac(double a, double b, acc_t c) {
    return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
  }
  static __device__ __forceinline__ int row(int lk, int r) { return lk + 4 * r; }
};

template <>
struct Mfma<float> {
  typedef v4f acc_t;
  static __device__ __forceinline__ acc_t mac(float a, float b, acc_t c) {
    return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
  }
  static __device__ __forceinline__ int row(int lk, int r) { return 4 * lk + r; }
};

template <typename T>
struct Cplx {
  T re, im;
};

template <typename T>
__device__ __forceinline__ Cplx<T> ldc(const T* base, int64_t off) {
  // one complex element = two consecutive reals
  typedef T v2 __attribute__((ext_vector_type(2)));
  v2 v = *reinterpret_cast<const v2*>(base + 2 * off);
  return {v.x, v.y};
}

template <typename T>
__device__ __forceinline__ void stc(T* base, int64_t off, T re, T im) {
  typedef T v2 __attribute__((ext_vector_type(2)));
  v2 v;
  v.x = re;
  v.y = im;
  *reinterpret_cast<v2*>(base + 2 * off) = v;
}

// ---------------------------------------------------------------------------------
// Grouped complex GEMM.  One wavefront computes one 32 x 32 output tile as 2 x 2
// MFMA 16x16x4 blocks.  Operands are read straight from global memory (the blocks are
// small, K is short, and L1/L2 serve the reuse between the waves of a tile column);
// the next K-step is prefetched into registers while the current one is multiplied.
//
// MFMA 16x16x4 operand layout (one element per lane): A(i, k) with i = lane % 16,
// k = lane / 16; B(k, j) with j = lane % 16, k = lane / 16.  Result: lane holds four
// rows (Mfma<T>::row) of column lane % 16.
// ---------------------------------------------------------------------------------
template <typename T, int FLAGS>
__global__ void __launch_bounds__(256) gemm_kernel(const GemmSeg* __restrict__ segs,
                                                   const GemmProb* __restrict__ probs,
                                                   const GemmTile* __restrict__ tiles,
                                                   int32_t ntiles,
                                                   const int64_t* __restrict__ rows,
                                                   const T* __restrict__ A,
                                                   const T* __restrict__ B,
                                                   T* __restrict__ C) {
  typedef typename Mfma<T>::acc_t acc_t;
  const int lane = threadIdx.x & 63;
  const int t = blockIdx.x * 4 + (threadIdx.x >> 6);
  if (t >= ntiles) return;
  const GemmTile tile = tiles[t];
  const GemmProb P = probs[tile.prob];
  const int i0 = tile.tm * TILE_M;
  const int j0 = tile.tn * TILE_N;
  const int li = lane & 15;
  const int lk = lane >> 4;

  acc_t cre[2][2], cim[2][2];
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int b = 0; b < 2; ++b) {
      cre[a][b] = acc_t{0, 0, 0, 0};
      cim[a][b] = acc_t{0, 0, 0, 0};
    }

  const int ia0 = i0 + li, ia1 = i0 + 16 + li;
  const int jb0 = j0 + li, jb1 = j0 + 16 + li;
  const bool va0 = ia0 < P.M, va1 = ia1 < P.M;
  const bool vb0 = jb0 < P.N, vb1 = jb1 < P.N;
  int64_t arow0 = 0, arow1 = 0;
  if (FLAGS & G_A_ROWMAP) {
    if (va0) arow0 = rows[P.rowmap + ia0];
    if (va1) arow1 = rows[P.rowmap + ia1];
  }

  for (int sgi = 0; sgi < P.nseg; ++sgi) {
    const GemmSeg S = segs[P.seg0 + sgi];
    auto addrA = [&](int i, int64_t arow, int k) -> int64_t {
      if (FLAGS & G_A_ROWMAP) return arow + S.a_off + k;
      if (FLAGS & G_A_T) return S.a_off + (int64_t)k * S.lda + i;
      return S.a_off + (int64_t)i * S.lda + k;
    };
    auto addrB = [&](int k, int j) -> int64_t {
      if (FLAGS & G_B_T) return S.b_off + (int64_t)j * S.ldb + k;
      return S.b_off + (int64_t)k * S.ldb + j;
    };
    auto load = [&](int k0, Cplx<T>& a0, Cplx<T>& a1, Cplx<T>& b0, Cplx<T>& b1) {
      const int k = k0 + lk;
      const bool vk = k < S.k;
      a0 = (vk && va0) ? ldc(A, addrA(ia0, arow0, k)) : Cplx<T>{0, 0};
      a1 = (vk && va1) ? ldc(A, addrA(ia1, arow1, k)) : Cplx<T>{0, 0};
      b0 = (vk && vb0) ? ldc(B, addrB(k, jb0)) : Cplx<T>{0, 0};
      b1 = (vk && vb1) ? ldc(B, addrB(k, jb1)) : Cplx<T>{0, 0};
    };
    Cplx<T> a0, a1, b0, b1;
    load(0, a0, a1, b0, b1);
    for (int k0 = 0; k0 < S.k; k0 += 4) {
      Cplx<T> na0, na1, nb0, nb1;
      if (k0 + 4 < S.k) load(k0 + 4, na0, na1, nb0, nb1);
      const T ai0 = (FLAGS & G_A_CONJ) ? -a0.im : a0.im;
      const T ai1 = (FLAGS & G_A_CONJ) ? -a1.im : a1.im;
      const Cplx<T> av[2] = {{a0.re, ai0}, {a1.re, ai1}};
      const Cplx<T> bv[2] = {b0, b1};
#pragma unroll
      for (int a = 0; a < 2; ++a)
#pragma unroll
        for (int b = 0; b < 2; ++b) {
          cre[a][b] = Mfma<T>::mac(av[a].re, bv[b].re, cre[a][b]);
          cim[a][b] = Mfma<T>::mac(av[a].re, bv[b].im, cim[a][b]);
        }
#pragma unroll
      for (int a = 0; a < 2; ++a)
#pragma unroll
        for (int b = 0; b < 2; ++b) {
          cre[a][b] = Mfma<T>::mac(-av[a].im, bv[b].im, cre[a][b]);
          cim[a][b] = Mfma<T>::mac(av[a].im, bv[b].re, cim[a][b]);
        }
      a0 = na0;
      a1 = na1;
      b0 = nb0;
      b1 = nb1;
    }
  }

#pragma unroll
  for (int a = 0; a < 2; ++a) {
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int i = i0 + a * 16 + Mfma<T>::row(lk, r);
      if (i >= P.M) continue;
      const int64_t rb = (FLAGS & G_C_ROWMAP) ? rows[P.rowmap + i] : P.c_off + (int64_t)i * P.ldc;
#pragma unroll
      for (int b = 0; b < 2; ++b) {
        const int j = j0 + b * 16 + li;
        if (j < P.N) stc(C, rb + j, cre[a][b][r], cim[a][b][r]);
      }
    }
  }
}

template <typename T>
hipError_t launch_gemm(const GemmStage& st, const T* A, const T* B, T* C, hipStream_t s) {
  const int32_t nt = (int32_t)st.tiles.size();
  if (nt == 0) return hipSuccess;
  dim3 grid((nt + 3) / 4), block(256);
#define MRD_GEMM_CASE(F)                                                                \
  case F:                                                                               \
    hipLaunchKernelGGL((gemm_kernel<T, F>), grid, block, 0, s, st.d_segs, st.d_probs,   \
                       st.d_tiles, nt, st.d_rows, A, B, C);                             \
    break;
  switch (st.flags) {
    MRD_GEMM_CASE(0)
    MRD_GEMM_CASE(G_B_T | G_C_ROWMAP)
    MRD_GEMM_CASE(G_A_T | G_A_CONJ)
    MRD_GEMM_CASE(G_A_ROWMAP | G_B_T)
    MRD_GEMM_CASE(G_A_CONJ)
    default:
      return hipErrorInvalidValue;
  }
#undef MRD_GEMM_CASE
  return hipGetLastError();
}

template hipError_t launch_gemm<double>(const GemmStage&, const double*, const double*, double*,
                                        hipStream_t);
template hipError_t launch_gemm<float>(const GemmStage&, const float*, const float*, float*,
                                       hipStream_t);

// ---------------------------------------------------------------------------------
// Sparse MPO mixing: each workgroup owns one destination sub-block and sums its few
// scaled source sub-blocks.  Consecutive threads walk consecutive columns.
// ---------------------------------------------------------------------------------
template <typename T>
__global__ void __launch_bounds__(256) mix_kernel(const MixTask* __restrict__ tasks,
                                                  const MixSrc* __restrict__ srcs,
                                                  const T* __restrict__ src,
                                                  T* __restrict__ dst) {
  const MixTask tk = tasks[blockIdx.x];
  const int n = tk.rows * tk.cols;
  for (int e = threadIdx.x; e < n; e += blockDim.x) {
    const int r = e / tk.cols;
    const int c = e - r * tk.cols;
    T re = 0, im = 0;
    for (int q = 0; q < tk.nsrc; ++q) {
      const MixSrc sr = srcs[tk.src0 + q];
      const Cplx<T> x = ldc(src, sr.off + (int64_t)r * sr.ld + c);
      const T cr = (T)sr.re, ci = (T)sr.im;
      re += cr * x.re - ci * x.im;
      im += cr * x.im + ci * x.re;
    }
    stc(dst, tk.dst + (int64_t)r * tk.ld_dst + c, re, im);
  }
}

template <typename T>
hipError_t launch_mix(const MixStage& st, const T* src, T* dst, hipStream_t s) {
  if (st.tasks.empty()) return hipSuccess;
  hipLaunchKernelGGL((mix_kernel<T>), dim3((uint32_t)st.tasks.size()), dim3(256), 0, s,
                     st.d_tasks, st.d_srcs, src, dst);
  return hipGetLastError();
}
template hipError_t launch_mix<double>(const MixStage&, const double*, double*, hipStream_t);
template hipError_t launch_mix<float>(const MixStage&, const float*, float*, hipStream_t);

// ---------------------------------------------------------------------------------
// Precision casts.
// ---------------------------------------------------------------------------------
__global__ void cast_d2f_kernel(const double* __restrict__ in, float* __restrict__ out, int64_t n) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x)
    out[i] = (float)in[i];
}
__global__ void cast_f2d_kernel(const float* __restrict__ in, double* __restrict__ out, int64_t n) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x)
    out[i] = (double)in[i];
}
static dim3 grid_for(int64_t n) {
  int64_t b = (n + 255) / 256;
  if (b > 8192) b = 8192;
  if (b < 1) b = 1;
  return dim3((uint32_t)b);
}
hipError_t launch_cast_d2f(const double* in, float* out, int64_t n, hipStream_t s) {
  if (n == 0) return hipSuccess;
  hipLaunchKernelGGL(cast_d2f_kernel, grid_for(n), dim3(256), 0, s, in, out, n);
  return hipGetLastError();
}
hipError_t launch_cast_f2d(const float* in, double* out, int64_t n, hipStream_t s) {
  if (n == 0) return hipSuccess;
  hipLaunchKernelGGL(cast_f2d_kernel, grid_for(n), dim3(256), 0, s, in, out, n);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------------
// Lanczos vector kernels, FP64 complex.  Each workgroup owns a contiguous chunk of
// LZ_CHUNK elements; per-workgroup partial sums are reduced afterwards in a fixed
// order, so results are bitwise reproducible run to run.
// ---------------------------------------------------------------------------------
constexpr int LZ_EPT = 4;
constexpr int LZ_CHUNK = 256 * LZ_EPT;

int lz_nblk(int64_t n) { return (int)((n + LZ_CHUNK - 1) / LZ_CHUNK); }

__device__ __forceinline__ double wave_sum(double v) {
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
  return v;
}

// partial[blk * (2*nv) + 2*i + {0,1}] = sum over the chunk of conj(V_i[e]) w[e]
__global__ void __launch_bounds__(256) lz_dots_kernel(const double* __restrict__ V, int64_t ld,
                                                      int32_t nv, const double* __restrict__ w,
                                                      int64_t n, double* __restrict__ partial) {
  __shared__ double red[4][2];
  const int64_t e0 = (int64_t)blockIdx.x * LZ_CHUNK + threadIdx.x;
  double wr[LZ_EPT], wi[LZ_EPT];
#pragma unroll
  for (int q = 0; q < LZ_EPT; ++q) {
    const int64_t e = e0 + q * 256;
    wr[q] = e < n ? w[2 * e] : 0.0;
    wi[q] = e < n ? w[2 * e + 1] : 0.0;
  }
  const int wv = threadIdx.x >> 6, lane = threadIdx.x & 63;
  for (int i = 0; i < nv; ++i) {
    const double* v = V + 2 * (int64_t)i * ld;
    double sr = 0, si = 0;
#pragma unroll
    for (int q = 0; q < LZ_EPT; ++q) {
      const int64_t e = e0 + q * 256;
      if (e < n) {
        const double vr = v[2 * e], vi = v[2 * e + 1];
        sr += vr * wr[q] + vi * wi[q];
        si += vr * wi[q] - vi * wr[q];
      }
    }
    sr = wave_sum(sr);
    si = wave_sum(si);
    if (lane == 0) {
      red[wv][0] = sr;
      red[wv][1] = si;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
      partial[(int64_t)blockIdx.x * 2 * nv + 2 * i] = (red[0][0] + red[1][0]) + (red[2][0] + red[3][0]);
      partial[(int64_t)blockIdx.x * 2 * nv + 2 * i + 1] = (red[0][1] + red[1][1]) + (red[2][1] + red[3][1]);
    }
    __syncthreads();
  }
}

// out[c] = sum over blocks of partial[blk * ncomp + c], fixed pairwise order.
__global__ void __launch_bounds__(256) lz_reduce_kernel(const double* __restrict__ partial,
                                                        int32_t nblk, int32_t ncomp,
                                                        double* __restrict__ out) {
  __shared__ double sm[256];
  const int c = blockIdx.x;
  double s = 0;
  for (int b = threadIdx.x; b < nblk; b += 256) s += partial[(int64_t)b * ncomp + c];
  sm[threadIdx.x] = s;
  __syncthreads();
  for (int st = 128; st > 0; st >>= 1) {
    if (threadIdx.x < st) sm[threadIdx.x] += sm[threadIdx.x + st];
    __syncthreads();
  }
  if (threadIdx.x == 0) out[c] = sm[0];
}

// w[e] -= sum_i h_i V_i[e]; then partial dots conj(V_i) w_new and |w_new|^2 (slot nv).
__global__ void __launch_bounds__(256) lz_update_dots_kernel(const double* __restrict__ V,
                                                             int64_t ld, int32_t nv,
                                                             double* __restrict__ w, int64_t n,
                                                             const double* __restrict__ h,
                                                             double* __restrict__ partial) {
  __shared__ double red[4][2];
  const int64_t e0 = (int64_t)blockIdx.x * LZ_CHUNK + threadIdx.x;
  double wr[LZ_EPT], wi[LZ_EPT];
#pragma unroll
  for (int q = 0; q < LZ_EPT; ++q) {
    const int64_t e = e0 + q * 256;
    wr[q] = e < n ? w[2 * e] : 0.0;
    wi[q] = e < n ? w[2 * e + 1] : 0.0;
  }
  for (int i = 0; i < nv; ++i) {
    const double* v = V + 2 * (int64_t)i * ld;
    const double hr = h[2 * i], hi = h[2 * i + 1];
#pragma unroll
    for (int q = 0; q < LZ_EPT; ++q) {
      const int64_t e = e0 + q * 256;
      if (e < n) {
        const double vr = v[2 * e], vi = v[2 * e + 1];
        wr[q] -= hr * vr - hi * vi;
        wi[q] -= hr * vi + hi * vr;
      }
    }
  }
#pragma unroll
  for (int q = 0; q < LZ_EPT; ++q) {
    const int64_t e = e0 + q * 256;
    if (e < n) {
      w[2 * e] = wr[q];
      w[2 * e + 1] = wi[q];
    }
  }
  const int wv = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int ncomp = 2 * nv + 1;
  for (int i = 0; i <= nv; ++i) {
    double sr = 0, si = 0;
    if (i < nv) {
      const double* v = V + 2 * (int64_t)i * ld;
#pragma unroll
      for (int q = 0; q < LZ_EPT; ++q) {
        const int64_t e = e0 + q * 256;
        if (e < n) {
          const double vr = v[2 * e], vi = v[2 * e + 1];
          sr += vr * wr[q] + vi * wi[q];
          si += vr * wi[q] - vi * wr[q];
        }
      }
    } else {
#pragma unroll
      for (int q = 0; q < LZ_EPT; ++q) sr += wr[q] * wr[q] + wi[q] * wi[q];
    }
    sr = wave_sum(sr);
    si = wave_sum(si);
    if (lane == 0) {
      red[wv][0] = sr;
      red[wv][1] = si;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
      partial[(int64_t)blockIdx.x * ncomp + 2 * i] = (red[0][0] + red[1][0]) + (red[2][0] + red[3][0]);
      if (i < nv)
        partial[(int64_t)blockIdx.x * ncomp + 2 * i + 1] =
            (red[0][1] + red[1][1]) + (red[2][1] + red[3][1]);
    }
    __syncthreads();
  }
}

// out[e] = (w[e] - sum_i h_i V_i[e]) * scal[0]
__global__ void __launch_bounds__(256) lz_update_scale_kernel(const double* __restrict__ V,
                                                              int64_t ld, int32_t nv,
                                                              const double* __restrict__ w,
                                                              int64_t n,
                                                              const double* __restrict__ h,
                                                              const double* __restrict__ scal,
                                                              double* __restrict__ out) {
  const int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (e >= n) return;
  double wr = w[2 * e], wi = w[2 * e + 1];
  for (int i = 0; i < nv; ++i) {
    const double* v = V + 2 * (int64_t)i * ld;
    const double hr = h[2 * i], hi = h[2 * i + 1];
    const double vr = v[2 * e], vi = v[2 * e + 1];
    wr -= hr * vr - hi * vi;
    wi -= hr * vi + hi * vr;
  }
  const double s = scal[0];
  out[2 * e] = wr * s;
  out[2 * e + 1] = wi * s;
}

__global__ void lz_scale_kernel(const double* __restrict__ x, int64_t n,
                                const double* __restrict__ scal, double* __restrict__ out) {
  const int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (e >= n) return;
  const double s = scal[0];
  out[2 * e] = x[2 * e] * s;
  out[2 * e + 1] = x[2 * e + 1] * s;
}

// out[e] = sum_i y_i V_i[e] (real coefficients)
__global__ void lz_combine_kernel(const double* __restrict__ V, int64_t ld, int32_t nv, int64_t n,
                                  const double* __restrict__ y, double* __restrict__ out) {
  const int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (e >= n) return;
  double r = 0, im = 0;
  for (int i = 0; i < nv; ++i) {
    const double* v = V + 2 * (int64_t)i * ld;
    r += y[i] * v[2 * e];
    im += y[i] * v[2 * e + 1];
  }
  out[2 * e] = r;
  out[2 * e + 1] = im;
}

hipError_t launch_lz_dots(const double* V, int64_t ld, int32_t nv, const double* w, int64_t n,
                          double* partial, int32_t nblk, hipStream_t s) {
  hipLaunchKernelGGL(lz_dots_kernel, dim3(nblk), dim3(256), 0, s, V, ld, nv, w, n, partial);
  return hipGetLastError();
}
hipError_t launch_lz_reduce(const double* partial, int32_t nblk, int32_t ncomp, double* out,
                            hipStream_t s) {
  hipLaunchKernelGGL(lz_reduce_kernel, dim3(ncomp), dim3(256), 0, s, partial, nblk, ncomp, out);
  return hipGetLastError();
}
hipError_t launch_lz_update_dots(const double* V, int64_t ld, int32_t nv, double* w, int64_t n,
                                 const double* h, double* partial, int32_t nblk, hipStream_t s) {
  hipLaunchKernelGGL(lz_update_dots_kernel, dim3(nblk), dim3(256), 0, s, V, ld, nv, w, n, h,
                     partial);
  return hipGetLastError();
}
hipError_t launch_lz_update_scale(const double* V, int64_t ld, int32_t nv, const double* w,
                                  int64_t n, const double* h, const double* scal, double* out,
                                  hipStream_t s) {
  hipLaunchKernelGGL(lz_update_scale_kernel, grid_for(n).x < 1 ? dim3(1) : dim3((uint32_t)((n + 255) / 256)),
                     dim3(256), 0, s, V, ld, nv, w, n, h, scal, out);
  return hipGetLastError();
}
hipError_t launch_lz_scale(const double* x, int64_t n, const double* scal, double* out,
                           hipStream_t s) {
  hipLaunchKernelGGL(lz_scale_kernel, dim3((uint32_t)((n + 255) / 256)), dim3(256), 0, s, x, n,
                     scal, out);
  return hipGetLastError();
}
hipError_t launch_lz_combine(const double* V, int64_t ld, int32_t nv, int64_t n, const double* y,
                             double* out, hipStream_t s) {
  hipLaunchKernelGGL(lz_combine_kernel, dim3((uint32_t)((n + 255) / 256)), dim3(256), 0, s, V, ld,
                     nv, n, y, out);
  return hipGetLastError();
}

}  // namespace mrd
