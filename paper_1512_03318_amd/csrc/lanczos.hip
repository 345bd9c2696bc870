// Device-resident Lanczos (FP64) for the lowest eigenpair of the two-site H_eff.
//
// Textbook Lanczos with full reorthogonalisation by classical Gram-Schmidt applied
// twice, the tridiagonal eigenproblem solved on the device:
//
//   v_0 = theta / |theta|
//   step j:  w = H v_j
//            h1 = V^H w,  alpha_j = Re h1_j            (V = [v_0 .. v_j])
//            w1 = w - V h1,  h2 = V^H w1        (three streaming passes over V up to
//                                                LZ_FUSE vectors, four beyond)
//            beta_j = |w1 - V h2| = sqrt(|w1|^2 - |h2|^2)
//            stop if beta_j <= tol * |T| (|T| = max_i |alpha_i| + beta_i + beta_{i-1})
//            or j = max_iter - 1;  else v_{j+1} = (w1 - V h2) / beta_j
//   lowest eigenpair (E, y) of T_k by multisection on Sturm counts and inverse
//   iteration, Ritz vector V y.
//
// Plans whose matvec reads FP32 (DM_FP32, DM_BF16X3) keep V in complex FP32 (LzGrid::vf32):
// each v_j is rounded once when it is formed and widened to FP64 wherever it is used.
//
// All scalars live in LzState on the device.  Every kernel of one step reads the step
// index and the stop flag from there, so the launches of a step have fixed arguments
// (the step can be captured once as a HIP graph and replayed) and a breakdown turns
// the remaining launches into no-ops without a host round trip.  Partial sums are
// reduced in a fixed order: results are reproducible run to run.
//
// Each kernel runs over a table of independent instances (LzInst): one launch per
// phase serves a single plan or a whole batch of them.
#include <algorithm>

#include "device.hpp"

namespace mrd {

// complex FP64 element (re, im) as a native vector: 16-byte loads through global pointers
typedef double lzc __attribute__((ext_vector_type(2)));
typedef float lzf __attribute__((ext_vector_type(2)));

// Krylov basis storage: complex FP64, or (F32) complex FP32 for plans whose matvec reads
// an FP32 copy of v_j anyway.  Every vector is rounded once as it is formed, v_j in the
// basis is then exactly the matvec's input, and all arithmetic on it stays FP64.
template <bool F32>
struct LzV {
  typedef lzc T;
};
template <>
struct LzV<true> {
  typedef lzf T;
};
__device__ __forceinline__ lzc lz_wide(lzc v) { return v; }
__device__ __forceinline__ lzc lz_wide(lzf v) { return lzc{(double)v.x, (double)v.y}; }
// x rounded to the storage (in place) and returned in storage form
template <bool F32>
__device__ __forceinline__ typename LzV<F32>::T lz_round(lzc& x) {
  if constexpr (F32) {
    const lzf r = lzf{(float)x.x, (float)x.y};
    x = lz_wide(r);
    return r;
  } else {
    return x;
  }
}

constexpr int LZ_EPT = 4;                 // elements per thread in streaming kernels
constexpr int LZ_CHUNK = 256 * LZ_EPT;

static int lz_nblk(int64_t n) { return (int)((n + LZ_CHUNK - 1) / LZ_CHUNK); }
static int lz_nblk256(int64_t n) { return (int)((n + 255) / 256); }
// projection partials: one row of at most 2 max_iter + 1 doubles per chunk, then the
// norm partials
int64_t lz_part_doubles(int64_t n, int32_t max_iter) {
  return (int64_t)lz_nblk(n) * (2 * max_iter + 1) + 2 * (int64_t)lz_nblk(n);
}

LzGrid lz_layout(std::vector<LzInst>& I, int32_t max_iter) {
  LzGrid g;
  g.nins = (int32_t)I.size();
  g.max_iter = max_iter;
  for (auto& x : I) {
    x.nb = lz_nblk(x.n);
    x.pnorm = x.part + (int64_t)x.nb * (2 * max_iter + 1);
    x.c0 = g.nchunk;
    x.g0 = g.n256;
    g.nchunk += x.nb;
    g.n256 += lz_nblk256(x.n);
  }
  return g;
}

// Instance owning flat block b of a grid laid out by the offsets F (0: c0, 1: g0).
template <int F>
__device__ __forceinline__ int lz_find(const LzInst* __restrict__ I, int nins, int b) {
  int lo = 0, hi = nins - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    const int v = F == 0 ? I[mid].c0 : I[mid].g0;
    if (v <= b) lo = mid;
    else hi = mid - 1;
  }
  return lo;
}

// One DPP row operation on a double (two 32-bit moves); lanes of rows outside ROWS
// receive 0.
template <int CTRL, int ROWS>
__device__ __forceinline__ double dpp_d(double v) {
  const int lo = __builtin_amdgcn_update_dpp(0, __double2loint(v), CTRL, ROWS, 0xf, false);
  const int hi = __builtin_amdgcn_update_dpp(0, __double2hiint(v), CTRL, ROWS, 0xf, false);
  return __hiloint2double(hi, lo);
}

// Sum over the 64 lanes of a wave in a fixed order, returned in every lane.  Register
// moves between lanes (DPP) instead of LDS permutes: pairs, quads, half rows (mirror),
// rows of 16 (mirror), then row 0 into row 1 and row 2 into row 3 (broadcast of lane
// 15 of each row), then rows 0-1 into rows 2-3 (broadcast of lane 31); lane 63 holds
// the total.  Every lane of the wave must be active.
__device__ __forceinline__ double wave_sum(double v) {
  v += dpp_d<0xb1, 0xf>(v);   // quad_perm [1,0,3,2]
  v += dpp_d<0x4e, 0xf>(v);   // quad_perm [2,3,0,1]
  v += dpp_d<0x141, 0xf>(v);  // row_half_mirror
  v += dpp_d<0x140, 0xf>(v);  // row_mirror
  v += dpp_d<0x142, 0xa>(v);  // row_bcast:15 into rows 1, 3
  v += dpp_d<0x143, 0xc>(v);  // row_bcast:31 into rows 2, 3
  const int lo = __builtin_amdgcn_readlane(__double2loint(v), 63);
  const int hi = __builtin_amdgcn_readlane(__double2hiint(v), 63);
  return __hiloint2double(hi, lo);
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


__global__ void lz_init_kernel(const LzInst* __restrict__ I, int32_t max_iter, double tol) {
  if (threadIdx.x != 0) return;
  LzState* st = I[blockIdx.x].st;
  st->iter = 0;
  st->k = 0;
  st->stop = 0;
  st->bad = 0;
  st->max_iter = max_iter;
  st->tol = tol;
  st->tnorm = 0.0;
  st->energy = 0.0;
  st->t0 = wall_clock64();
  st->t1 = st->t0;
}

__device__ __forceinline__ void lz_mark_stop(LzState* st) {
  st->stop = 1;
  st->t1 = wall_clock64();
}

// pnorm[chunk] = sum over the chunk of |x|^2 (start vector)
__global__ void __launch_bounds__(256) lz_norm_kernel(const LzInst* __restrict__ I, int nins) {
  __shared__ double sh[4];
  const int q0 = lz_find<0>(I, nins, blockIdx.x);
  const LzInst& in = I[q0];
  const int blk = blockIdx.x - in.c0;
  const auto x = glb(in.x);
  double s = 0;
#pragma unroll
  for (int q = 0; q < LZ_EPT; ++q) {
    const int64_t e = (int64_t)blk * LZ_CHUNK + q * 256 + threadIdx.x;
    if (e >= in.n) continue;
    s += x[2 * e] * x[2 * e];
    if (2 * e + 1 < in.xn) s += x[2 * e + 1] * x[2 * e + 1];  // a real x of odd length ends here
  }
  s = block_sum(s, sh);
  if (threadIdx.x == 0) glb(in.pnorm)[blk] = s;
}

enum LzReduce : int32_t {
  LZR_SCAL0 = 0,  // sum of pnorm -> scal0
  LZR_H1 = 1,     // chunk partials -> h1 (2 nv components)
  LZR_H2 = 2,     // chunk partials -> h2
  LZR_NORM = 3,   // sum of pnorm -> h2[2 nv] (|w1|^2)
  LZR_RQ = 4,     // pnorm pairs -> rq[0..1]
  LZR_H2N = 5,    // chunk partials -> h2 and |w1|^2 (2 nv + 1 components)
};

// Fixed-order reduction of one component (blockIdx.x) of instance blockIdx.y.
__global__ void __launch_bounds__(256) lz_reduce_kernel(const LzInst* __restrict__ I, int32_t mode) {
  __shared__ double sm[256];
  const LzInst& in = I[blockIdx.y];
  LzState* st = in.st;
  const bool step = mode != LZR_SCAL0 && mode != LZR_RQ;
  if (step && st->stop) return;
  const int nv = st->iter + 1;
  const double* src;
  int nblk, ncomp;
  double* out;
  switch (mode) {
    case LZR_SCAL0: src = in.pnorm; nblk = in.nb; ncomp = 1; out = &st->scal0; break;
    case LZR_H1: src = in.part; nblk = in.nb; ncomp = 2 * nv; out = st->h1; break;
    case LZR_H2: src = in.part; nblk = in.nb; ncomp = 2 * nv; out = st->h2; break;
    case LZR_NORM: src = in.pnorm; nblk = in.nb; ncomp = 1; out = st->h2 + 2 * nv; break;
    case LZR_H2N: src = in.part; nblk = in.nb; ncomp = 2 * nv + 1; out = st->h2; break;
    default: src = in.pnorm; nblk = in.nb; ncomp = 2; out = st->rq; break;
  }
  const int c = blockIdx.x;
  if (c >= ncomp) return;
  if (in.real && (mode == LZR_H1 || mode == LZR_H2 || mode == LZR_H2N) && (c & 1) && c < 2 * nv) {
    if (threadIdx.x == 0) out[c] = 0.0;  // real instance: real projection coefficients
    return;
  }
  double s = 0;
  const auto sp = glb(src);
  for (int b = threadIdx.x; b < nblk; b += 256) s += sp[(int64_t)b * ncomp + c];
  sm[threadIdx.x] = s;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if (threadIdx.x < w) sm[threadIdx.x] += sm[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) out[c] = sm[0];
}

// v_0 = x / |x| into V[0] and vcur.
template <bool F32>
__global__ void lz_start_scale_kernel(const LzInst* __restrict__ I, int nins) {
  const int q0 = lz_find<1>(I, nins, blockIdx.x);
  const LzInst& in = I[q0];
  LzState* st = in.st;
  const double nrm2 = st->scal0;
  if (!(nrm2 > 0.0) || !isfinite(nrm2)) {
    if (blockIdx.x == in.g0 && threadIdx.x == 0) {
      st->bad = 1;
      lz_mark_stop(st);
    }
    return;
  }
  const double s = 1.0 / sqrt(nrm2);
  const int64_t e = (int64_t)(blockIdx.x - in.g0) * 256 + threadIdx.x;
  if (e >= in.n) return;
  const auto xr = glb(in.x);
  const double x0 = xr[2 * e], x1 = 2 * e + 1 < in.xn ? xr[2 * e + 1] : 0.0;
  lzc v = lzc{x0 * s, x1 * s};
  glb(reinterpret_cast<typename LzV<F32>::T*>(in.V))[e] = lz_round<F32>(v);
  glb(reinterpret_cast<lzc*>(in.vcur))[e] = v;
  if (in.tin) glb(reinterpret_cast<lzf*>(in.tin))[e] = lzf{(float)v.x, (float)v.y};
}

constexpr int LZ_G = 8;  // Krylov vectors per dot-product block

// Block sums of NVAL per-thread values with one barrier (wave shuffles, then the four
// wave partials in a fixed order); out[c] for c < nval.
template <int NVAL>
__device__ __forceinline__ void block_sums(const double (&v)[NVAL], int nval, double* sh,
                                           MRD_GLOBAL double* out) {
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

// part[blk][2i + {0,1}] = sum over chunk blk of conj(V_i) w for every i < nv (nv =
// iter + 1).  Chunk blk holds the elements blk * LZ_CHUNK + q * 256 + thread, q < LZ_EPT.
// One block per chunk keeps its w elements in registers and walks the basis in groups
// of LZ_G vectors; a group's loads are all issued before its products (measured at 30
// vectors of 660k elements: 56 us against 74 us with one block per chunk and group,
// which re-read w and ended after one round of loads).
template <int NG, bool F32>
__device__ __forceinline__ void lz_dots_group(const LzInst& in, const lzc (&xe)[LZ_EPT],
                                              int64_t e0, bool full, int i0, int nv, int blk,
                                              double* sh) {
  typedef typename LzV<F32>::T VT;
  const auto v0 = glb(reinterpret_cast<const VT*>(in.V));
  MRD_GLOBAL const VT* vv[NG];
#pragma unroll
  for (int g = 0; g < NG; ++g) vv[g] = v0 + (int64_t)(i0 + g) * in.ld;
  double acc[2 * NG];
#pragma unroll
  for (int c = 0; c < 2 * NG; ++c) acc[c] = 0.0;
  if (full) {
    VT v[NG][LZ_EPT];
#pragma unroll
    for (int g = 0; g < NG; ++g)
#pragma unroll
      for (int q = 0; q < LZ_EPT; ++q) v[g][q] = vv[g][e0 + q * 256];
#pragma unroll
    for (int q = 0; q < LZ_EPT; ++q)
#pragma unroll
      for (int g = 0; g < NG; ++g) {
        acc[2 * g] += v[g][q].x * xe[q].x + v[g][q].y * xe[q].y;
        acc[2 * g + 1] += v[g][q].x * xe[q].y - v[g][q].y * xe[q].x;
      }
  } else {
#pragma unroll
    for (int q = 0; q < LZ_EPT; ++q) {
      const int64_t e = e0 + q * 256;
      if (e < in.n) {
#pragma unroll
        for (int g = 0; g < NG; ++g) {
          const lzc v = lz_wide(vv[g][e]);
          acc[2 * g] += v.x * xe[q].x + v.y * xe[q].y;
          acc[2 * g + 1] += v.x * xe[q].y - v.y * xe[q].x;
        }
      }
    }
  }
  block_sums(acc, 2 * NG, sh, glb(in.part) + (int64_t)blk * (2 * nv) + 2 * i0);
}

template <bool F32>
__global__ void __launch_bounds__(256) lz_dots_kernel(const LzInst* __restrict__ I, int nins) {
  __shared__ double sh[4 * 2 * LZ_G];
  const int q0 = lz_find<0>(I, nins, blockIdx.x);
  const LzInst& in = I[q0];
  const auto sg = glb(in.st);
  if (sg->stop) return;
  const int nv = sg->iter + 1;
  const int blk = blockIdx.x - in.c0;
  const int64_t e0 = (int64_t)blk * LZ_CHUNK + threadIdx.x;
  const bool full = e0 + (LZ_EPT - 1) * 256 < in.n;  // every element of this thread in range
  const auto xv = glb(reinterpret_cast<const lzc*>(in.w));
  lzc xe[LZ_EPT];
#pragma unroll
  for (int q = 0; q < LZ_EPT; ++q) xe[q] = e0 + q * 256 < in.n ? xv[e0 + q * 256] : lzc{0.0, 0.0};
  for (int i0 = 0; i0 < nv; i0 += LZ_G) {
    if (i0 > 0) __syncthreads();  // the previous group's sums have been read from sh
    switch (min(LZ_G, nv - i0)) {  // uniform over the block
      case 1: lz_dots_group<1, F32>(in, xe, e0, full, i0, nv, blk, sh); break;
      case 2: lz_dots_group<2, F32>(in, xe, e0, full, i0, nv, blk, sh); break;
      case 3: lz_dots_group<3, F32>(in, xe, e0, full, i0, nv, blk, sh); break;
      case 4: lz_dots_group<4, F32>(in, xe, e0, full, i0, nv, blk, sh); break;
      case 5: lz_dots_group<5, F32>(in, xe, e0, full, i0, nv, blk, sh); break;
      case 6: lz_dots_group<6, F32>(in, xe, e0, full, i0, nv, blk, sh); break;
      case 7: lz_dots_group<7, F32>(in, xe, e0, full, i0, nv, blk, sh); break;
      default: lz_dots_group<LZ_G, F32>(in, xe, e0, full, i0, nv, blk, sh); break;
    }
  }
}

constexpr int LZ_U = 4;  // basis vectors loaded together in the subtraction loops

// x -= sum_{i < nv} h_i V_i[e] (h complex, interleaved), subtracted in index order;
// the loads of LZ_U vectors are issued before their products.
template <typename VT>
__device__ __forceinline__ void lz_sub_basis(lzc& x, MRD_GLOBAL const VT* V, int64_t ld,
                                             int64_t e, const MRD_GLOBAL double* h, int nv) {
  int i = 0;
  for (; i + LZ_U <= nv; i += LZ_U) {
    VT vs[LZ_U];
#pragma unroll
    for (int u = 0; u < LZ_U; ++u) vs[u] = V[(int64_t)(i + u) * ld + e];
#pragma unroll
    for (int u = 0; u < LZ_U; ++u) {
      const lzc v = lz_wide(vs[u]);
      const double hr = h[2 * (i + u)], hi = h[2 * (i + u) + 1];
      x.x -= hr * v.x - hi * v.y;
      x.y -= hr * v.y + hi * v.x;
    }
  }
  for (; i < nv; ++i) {
    const double hr = h[2 * i], hi = h[2 * i + 1];
    const lzc v = lz_wide(V[(int64_t)i * ld + e]);
    x.x -= hr * v.x - hi * v.y;
    x.y -= hr * v.y + hi * v.x;
  }
}

// w -= V h1 over the nv = iter + 1 Krylov vectors; pnorm[chunk] = |w_new|^2 over the chunk.
template <bool F32>
__global__ void __launch_bounds__(256) lz_sub_kernel(const LzInst* __restrict__ I, int nins) {
  __shared__ double sh[4];
  const int q0 = lz_find<0>(I, nins, blockIdx.x);
  const LzInst& in = I[q0];
  const MRD_GLOBAL LzState* st = glb(in.st);
  if (st->stop) return;
  const int nv = st->iter + 1;
  const MRD_GLOBAL double* h1 = st->h1;
  const auto V = glb(reinterpret_cast<const typename LzV<F32>::T*>(in.V));
  const auto w = glb(reinterpret_cast<lzc*>(in.w));
  const int64_t ld = in.ld;
  const int blk = blockIdx.x - in.c0;
  double nn = 0;
#pragma unroll
  for (int q = 0; q < LZ_EPT; ++q) {
    const int64_t e = (int64_t)blk * LZ_CHUNK + q * 256 + threadIdx.x;
    if (e >= in.n) continue;
    lzc x = w[e];
    lz_sub_basis(x, V, ld, e, h1, nv);
    w[e] = x;
    nn += x.x * x.x + x.y * x.y;
  }
  nn = block_sum(nn, sh);
  if (threadIdx.x == 0) glb(in.pnorm)[blk] = nn;
}

// Fused pass for bases of at most LZ_FUSE vectors, specialised on a bound NVB >= nv of
// the vector count (nv = iter + 1; the host passes the step's bound rounded up to a
// multiple of 8), so that the per-thread registers, and with them the occupancy, follow
// the basis size.  Vectors i >= nv are skipped by branches uniform over the block.
// Beyond 24 vectors the registers (about 280 per thread) leave one wave per SIMD, and
// the separate subtraction and grouped projection passes stream faster.
constexpr int LZ_FUSE = 24;

// Fixed-order block sums of the first ncomp of NV per-thread values (wave shuffles, then
// the four wave partials) into out[c]; value `last` goes to out[ncomp - 1] when given.
template <int NV>
__device__ __forceinline__ void block_sums_n(const double (&acc)[NV], int ncomp, int last,
                                            double* sh, MRD_GLOBAL double* out) {
  const int wv = threadIdx.x >> 6, lane = threadIdx.x & 63;
#pragma unroll
  for (int c = 0; c < NV; ++c) {
    if (c < ncomp || c == last) {
      const double t = wave_sum(acc[c]);
      if (lane == 0) sh[c * 4 + wv] = t;
    }
  }
  __syncthreads();
  const int c = threadIdx.x;
  if (c < ncomp) {
    const int src = (last >= 0 && c == ncomp - 1) ? last : c;
    out[c] = (sh[src * 4] + sh[src * 4 + 1]) + (sh[src * 4 + 2] + sh[src * 4 + 3]);
  }
}

// A bound below the actual vector count cannot happen (the step index bounds iter); if
// it did, the solve is flagged and stopped rather than computed on part of the basis.
__device__ __forceinline__ bool lz_over_bound(LzState* st, int nv, int nvb) {
  if (nv <= nvb) return false;
  if (threadIdx.x == 0) {
    st->bad = 1;
    lz_mark_stop(st);
  }
  return true;
}

// The subtraction and the second projection in one pass over the basis: w1 = w - V h1,
// then part[blk][2i + {0,1}] = sum of conj(V_i) w1 and part[blk][2 nv] = sum of |w1|^2
// over the chunk.  Each thread holds its element of every vector in registers between
// the subtraction and the products, so the basis is read once for both.
template <int NVB, bool F32>
__global__ void __launch_bounds__(256) lz_subdots_kernel(const LzInst* __restrict__ I, int nins) {
  __shared__ double sh[4 * (2 * NVB + 1)];
  const int q0 = lz_find<0>(I, nins, blockIdx.x);
  const LzInst& in = I[q0];
  LzState* st = in.st;
  if (glb(st)->stop) return;
  const int nv = glb(st)->iter + 1;
  if (lz_over_bound(st, nv, NVB)) return;
  const int blk = blockIdx.x - in.c0;
  const auto h1 = glb(st->h1);
  const auto w = glb(reinterpret_cast<lzc*>(in.w));
  const auto V = glb(reinterpret_cast<const typename LzV<F32>::T*>(in.V));
  const int64_t ld = in.ld;
  double acc[2 * NVB + 1];
#pragma unroll
  for (int c = 0; c < 2 * NVB + 1; ++c) acc[c] = 0.0;
#pragma unroll 1
  for (int q = 0; q < LZ_EPT; ++q) {
    const int64_t e = (int64_t)blk * LZ_CHUNK + q * 256 + threadIdx.x;
    if (e >= in.n) break;
    lzc v[NVB];
#pragma unroll
    for (int i = 0; i < NVB; ++i)
      if (i < nv) v[i] = lz_wide(V[i * ld + e]);
    lzc x = w[e];
#pragma unroll
    for (int i = 0; i < NVB; ++i)
      if (i < nv) {
        const double hr = h1[2 * i], hi = h1[2 * i + 1];
        x.x -= hr * v[i].x - hi * v[i].y;
        x.y -= hr * v[i].y + hi * v[i].x;
      }
    w[e] = x;
#pragma unroll
    for (int i = 0; i < NVB; ++i)
      if (i < nv) {
        acc[2 * i] += v[i].x * x.x + v[i].y * x.y;
        acc[2 * i + 1] += v[i].x * x.y - v[i].y * x.x;
      }
    acc[2 * NVB] += x.x * x.x + x.y * x.y;
  }
  block_sums_n(acc, 2 * nv + 1, 2 * NVB, sh, glb(in.part) + (int64_t)blk * (2 * nv + 1));
}

// Scalar part of step j = st->iter of instance blockIdx.x: alpha_j, beta_j, |T|, stopping rule.
__global__ void lz_scalar_kernel(const LzInst* __restrict__ I) {
  LzState* st = I[blockIdx.x].st;
  if (threadIdx.x != 0 || st->stop) return;
  const int j = st->iter, nv = j + 1;
  const double alpha = st->h1[2 * j];
  double hh = 0;
  for (int i = 0; i < 2 * nv; ++i) hh += st->h2[i] * st->h2[i];
  const double nrm2 = st->h2[2 * nv];
  if (!isfinite(alpha) || !isfinite(nrm2)) {
    st->bad = 1;
    lz_mark_stop(st);
    return;
  }
  const double beta = sqrt(fmax(nrm2 - hh, 0.0));
  st->alpha[j] = alpha;
  st->k = nv;
  const double row = fabs(alpha) + beta + (j > 0 ? st->beta[j - 1] : 0.0);
  st->tnorm = fmax(st->tnorm, row);
  if (beta <= st->tol * st->tnorm || j == st->max_iter - 1) {
    lz_mark_stop(st);
    return;
  }
  st->beta[j] = beta;
  st->inv_beta = 1.0 / beta;
  st->iter = j + 1;
}

// v_{j+1} = (w - V h2) / beta_j into V[j+1] and vcur (runs only if the step continued).
template <bool F32>
__global__ void __launch_bounds__(256) lz_next_kernel(const LzInst* __restrict__ I, int nins) {
  const int q0 = lz_find<1>(I, nins, blockIdx.x);
  const LzInst& in = I[q0];
  const MRD_GLOBAL LzState* st = glb(in.st);
  if (st->stop) return;
  const int nv = st->iter;  // already advanced: vectors 0 .. j
  const int64_t e = (int64_t)(blockIdx.x - in.g0) * 256 + threadIdx.x;
  if (e >= in.n) return;
  const auto V = glb(reinterpret_cast<typename LzV<F32>::T*>(in.V));
  const int64_t ld = in.ld;
  lzc x = glb(reinterpret_cast<const lzc*>(in.w))[e];
  lz_sub_basis(x, (MRD_GLOBAL const typename LzV<F32>::T*)V, ld, e, st->h2, nv);
  const double s = st->inv_beta;
  x.x *= s;
  x.y *= s;
  V[(int64_t)nv * ld + e] = lz_round<F32>(x);
  glb(reinterpret_cast<lzc*>(in.vcur))[e] = x;
  if (in.tin) glb(reinterpret_cast<lzf*>(in.tin))[e] = lzf{(float)x.x, (float)x.y};
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
__global__ void __launch_bounds__(64) lz_tridiag_kernel(const LzInst* __restrict__ I) {
  LzState* st = I[blockIdx.x].st;
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

// Ritz vector sum_{i < k} y_i V_i into x and vcur.
template <bool F32>
__global__ void lz_combine_kernel(const LzInst* __restrict__ I, int nins) {
  const int q0 = lz_find<1>(I, nins, blockIdx.x);
  const LzInst& in = I[q0];
  const int64_t e = (int64_t)(blockIdx.x - in.g0) * 256 + threadIdx.x;
  if (e >= in.n) return;
  const MRD_GLOBAL LzState* st = glb(in.st);
  const int k = st->k;
  typedef typename LzV<F32>::T VT;
  const auto V = glb(reinterpret_cast<const VT*>(in.V));
  const MRD_GLOBAL double* y = st->y;
  double r = 0, im = 0;
  int i = 0;
  for (; i + LZ_U <= k; i += LZ_U) {  // loads first, then the sums in index order
    VT vs[LZ_U];
#pragma unroll
    for (int u = 0; u < LZ_U; ++u) vs[u] = V[(int64_t)(i + u) * in.ld + e];
#pragma unroll
    for (int u = 0; u < LZ_U; ++u) {
      const lzc v = lz_wide(vs[u]);
      r += y[i + u] * v.x;
      im += y[i + u] * v.y;
    }
  }
  for (; i < k; ++i) {
    const lzc v = lz_wide(V[(int64_t)i * in.ld + e]);
    r += y[i] * v.x;
    im += y[i] * v.y;
  }
  glb(in.x)[2 * e] = r;
  if (2 * e + 1 < in.xn) glb(in.x)[2 * e + 1] = im;
  glb(reinterpret_cast<lzc*>(in.vcur))[e] = lzc{r, im};
}

// pnorm[2 chunk + {0,1}] = (Re <vcur, w>, |vcur|^2) over the chunk (Rayleigh quotient).
__global__ void __launch_bounds__(256) lz_rq_kernel(const LzInst* __restrict__ I, int nins) {
  __shared__ double sh[4];
  const int q0 = lz_find<0>(I, nins, blockIdx.x);
  const LzInst& in = I[q0];
  const int blk = blockIdx.x - in.c0;
  const auto x = glb(reinterpret_cast<const lzc*>(in.vcur));
  const auto w = glb(reinterpret_cast<const lzc*>(in.w));
  double s = 0, q2 = 0;
#pragma unroll
  for (int q = 0; q < LZ_EPT; ++q) {
    const int64_t e = (int64_t)blk * LZ_CHUNK + q * 256 + threadIdx.x;
    if (e < in.n) {
      const lzc xe = x[e], we = w[e];
      s += xe.x * we.x + xe.y * we.y;
      q2 += xe.x * xe.x + xe.y * xe.y;
    }
  }
  s = block_sum(s, sh);
  q2 = block_sum(q2, sh);
  if (threadIdx.x == 0) {
    glb(in.pnorm)[2 * blk] = s;
    glb(in.pnorm)[2 * blk + 1] = q2;
  }
}

__global__ void lz_rq_final_kernel(const LzInst* __restrict__ I) {
  if (threadIdx.x != 0) return;
  LzState* st = I[blockIdx.x].st;
  const double e = st->rq[0] / st->rq[1];
  if (!isfinite(e)) st->bad = 1;
  st->energy = e;
}

__global__ void lz_results_kernel(const LzInst* __restrict__ I, LzResult* __restrict__ out) {
  if (threadIdx.x != 0) return;
  const LzState* st = I[blockIdx.x].st;
  LzResult r;
  r.energy = st->energy;
  r.k = st->k;
  r.bad = st->bad;
  r.t0 = st->t0;
  r.t1 = st->t1;
  out[blockIdx.x] = r;
}

// ---------------------------------------------------------------------------------
hipError_t lz_launch_init(const LzInst* I, const LzGrid& g, int32_t max_iter, double tol,
                          hipStream_t s) {
  if (max_iter < 1 || max_iter > g.max_iter) return hipErrorInvalidValue;
  hipLaunchKernelGGL(lz_init_kernel, dim3(g.nins), dim3(64), 0, s, I, max_iter, tol);
  return hipGetLastError();
}

hipError_t lz_launch_start(const LzInst* I, const LzGrid& g, hipStream_t s) {
  hipLaunchKernelGGL(lz_norm_kernel, dim3(g.nchunk), dim3(256), 0, s, I, g.nins);
  hipLaunchKernelGGL(lz_reduce_kernel, dim3(1, g.nins), dim3(256), 0, s, I, (int32_t)LZR_SCAL0);
  if (g.vf32) hipLaunchKernelGGL(lz_start_scale_kernel<true>, dim3(g.n256), dim3(256), 0, s, I, g.nins);
  else hipLaunchKernelGGL(lz_start_scale_kernel<false>, dim3(g.n256), dim3(256), 0, s, I, g.nins);
  return hipGetLastError();
}

template <bool F32>
static void lz_step_tail(const LzInst* I, const LzGrid& g, int32_t nv_bound, hipStream_t s) {
  const int maxc = 2 * g.max_iter + 1;
  // nv <= max_iter at every step; without a bound from the caller (a step captured once
  // for every replay) the capacity bounds it
  const int b = (nv_bound > 0 && nv_bound < g.max_iter) ? nv_bound : g.max_iter;
  const dim3 gd(g.nchunk);  // projections: one block per chunk over the whole basis
  hipLaunchKernelGGL(lz_dots_kernel<F32>, gd, dim3(256), 0, s, I, g.nins);
  hipLaunchKernelGGL(lz_reduce_kernel, dim3(maxc, g.nins), dim3(256), 0, s, I, (int32_t)LZR_H1);
  // the fused pass is bound by latency, not bytes: over an FP32 basis it runs no faster
  // than over an FP64 one (15.5 / 36 us at 8 / 16 vectors) and at 24 vectors slower
  // (86 against 62 us), while the separate passes stream half the bytes; so an FP32
  // basis fuses up to 16 vectors only
  if (b <= (F32 ? 16 : LZ_FUSE)) {
    // one pass for w1, h2 and |w1|^2
    if (b <= 8) hipLaunchKernelGGL((lz_subdots_kernel<8, F32>), dim3(g.nchunk), dim3(256), 0, s, I, g.nins);
    else if (F32 || b <= 16) hipLaunchKernelGGL((lz_subdots_kernel<16, F32>), dim3(g.nchunk), dim3(256), 0, s, I, g.nins);
    else hipLaunchKernelGGL((lz_subdots_kernel<LZ_FUSE, false>), dim3(g.nchunk), dim3(256), 0, s, I, g.nins);
    hipLaunchKernelGGL(lz_reduce_kernel, dim3(maxc, g.nins), dim3(256), 0, s, I, (int32_t)LZR_H2N);
  } else {
    hipLaunchKernelGGL(lz_sub_kernel<F32>, dim3(g.nchunk), dim3(256), 0, s, I, g.nins);
    hipLaunchKernelGGL(lz_dots_kernel<F32>, gd, dim3(256), 0, s, I, g.nins);
    hipLaunchKernelGGL(lz_reduce_kernel, dim3(maxc, g.nins), dim3(256), 0, s, I, (int32_t)LZR_H2);
    hipLaunchKernelGGL(lz_reduce_kernel, dim3(1, g.nins), dim3(256), 0, s, I, (int32_t)LZR_NORM);
  }
  hipLaunchKernelGGL(lz_scalar_kernel, dim3(g.nins), dim3(64), 0, s, I);
  hipLaunchKernelGGL(lz_next_kernel<F32>, dim3(g.n256), dim3(256), 0, s, I, g.nins);
}

hipError_t lz_launch_step_tail(const LzInst* I, const LzGrid& g, int32_t nv_bound, hipStream_t s) {
  if (g.vf32) lz_step_tail<true>(I, g, nv_bound, s);
  else lz_step_tail<false>(I, g, nv_bound, s);
  return hipGetLastError();
}

hipError_t lz_launch_finish(const LzInst* I, const LzGrid& g, hipStream_t s) {
  hipLaunchKernelGGL(lz_tridiag_kernel, dim3(g.nins), dim3(64), 0, s, I);
  if (g.vf32) hipLaunchKernelGGL(lz_combine_kernel<true>, dim3(g.n256), dim3(256), 0, s, I, g.nins);
  else hipLaunchKernelGGL(lz_combine_kernel<false>, dim3(g.n256), dim3(256), 0, s, I, g.nins);
  return hipGetLastError();
}

hipError_t lz_launch_rq(const LzInst* I, const LzGrid& g, hipStream_t s) {
  hipLaunchKernelGGL(lz_rq_kernel, dim3(g.nchunk), dim3(256), 0, s, I, g.nins);
  hipLaunchKernelGGL(lz_reduce_kernel, dim3(2, g.nins), dim3(256), 0, s, I, (int32_t)LZR_RQ);
  hipLaunchKernelGGL(lz_rq_final_kernel, dim3(g.nins), dim3(64), 0, s, I);
  return hipGetLastError();
}

hipError_t lz_launch_results(const LzInst* I, const LzGrid& g, LzResult* out, hipStream_t s) {
  hipLaunchKernelGGL(lz_results_kernel, dim3(g.nins), dim3(64), 0, s, I, out);
  return hipGetLastError();
}

}  // namespace mrd
