// Split-precision (BF16x3) grouped complex GEMM for gfx950.
//
// Operands stay FP32 in HBM.  While a chunk is staged into LDS every FP32 value x is
// split into two bfloat16 parts, hi = bf16(x) and lo = bf16(x - hi) (round to nearest
// even both times), so that x = hi + lo up to a relative 2^-17.  A real product is then
// taken as three bf16 products on the 16x16x32 bf16 MFMA with FP32 accumulation,
//   x y  ~  xh yh + xh yl + xl yh,
// dropping xl yl (relative <= 2^-18) -- about 16 significant bits per product instead of
// FP32's 24, at the rate of the bf16 matrix cores.  The complex product takes four real
// products (Cr += Ar Br - Ai Bi, Ci += Ar Bi + Ai Br), so twelve MFMAs per 16x16x32
// complex sub-block.
//
// Because the bf16 matrix cores are fast, these tiles are larger than those of the
// FP32/FP64 kernels (more reuse of every staged element): BM x BN per workgroup of four
// waves arranged WM x WN, each wave (BM/WM) x (BN/WN) in 16 x 16 MFMA blocks, K staged
// in chunks of 32.  With SPLIT the K range of a problem is divided over nks workgroups
// (chunks ks, ks + nks, ...) that write partial tiles, summed in split order by
// gemm_split_reduce_kernel.
//
// MFMA 16x16x32 bf16 operands (8 bf16 per lane): A(i, k) with i = lane % 16 and
// k = 8 (lane / 16) + t, B(k, j) with j = lane % 16 and the same k; result row
// 4 (lane / 16) + r, column lane % 16 (measured on gfx950).  LDS therefore holds each
// operand as [row][k] planes (k contiguous), one plane per part: re_hi, re_lo, im_hi,
// im_lo; a lane reads its 8 k values with one 16-byte load.
//
// REAL (the real formulation of eq. rot): operands and results are real FP32 (results FP64
// with G_C_F64); two LDS planes per operand (hi, lo) and three MFMAs per 16x16x32 block.
//
// LDS rows: an operand staged along k (its quads are four consecutive k of one row, eight
// lanes per row) has 64-byte rows with 16-byte group g of row r stored at slot
// g ^ f(r), f(r) = ((r >> 1) ^ (r >> 3)) & 3.  A pass of 32 lanes storing 8 bytes each
// then covers four whole rows = all 64 banks once, and a fragment read (16 consecutive
// rows, one group) puts rows r, r + 4, r + 8, r + 12 (same banks without the XOR) in four
// different slots: no bank conflicts either way.  An operand staged across rows (quads
// along k of one column of consecutive lanes' rows) keeps rows of 40 bf16 (80 bytes), which
// keeps its fragment reads conflict-free.
#include "device.hpp"

namespace mrd {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef __bf16 bf16x4 __attribute__((ext_vector_type(4)));
typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));

__device__ __forceinline__ f32x4 mfma_bf16(bf16x8 a, bf16x8 b, f32x4 c) {
  return __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, c, 0, 0, 0);
}

__device__ __forceinline__ bf16x8 neg8(bf16x8 v) {
  u32x4 u = __builtin_bit_cast(u32x4, v);
  u ^= 0x80008000u;
  return __builtin_bit_cast(bf16x8, u);
}

// bf16 offset of element (row r, k) in an LDS plane of K-chunk rows (see above)
template <bool KCONTIG>
__device__ __forceinline__ int lds_rk(int r, int k) {
  if (KCONTIG) return r * 32 + ((((k >> 3) ^ (((r >> 1) ^ (r >> 3)) & 3)) << 3) | (k & 7));
  return r * 40 + k;
}

template <int FLAGS, int BM, int BN, int WM, int WN, bool REAL = false>
struct Bf3Cfg {
  static constexpr int PARTS = REAL ? 2 : 4;    // bf16 planes per operand
  static constexpr int KC = 32;                // K chunk = one bf16 MFMA step
  static constexpr int QA = BM * KC / 4 / 256;  // k-quads of A staged per thread
  static constexpr int QB = BN * KC / 4 / 256;
  static constexpr int XB = BM / WM / 16, YB = BN / WN / 16;  // MFMA blocks per wave
  static constexpr bool A_KC = !(FLAGS & G_A_T);
  static constexpr bool B_KC = (FLAGS & G_B_T) != 0;
  // bf16 per plane: rows of 32 (swizzled) or 40 (padded) bf16
  static constexpr int PLANE_A = BM * (A_KC ? 32 : 40), PLANE_B = BN * (B_KC ? 32 : 40);
  static constexpr int SMEM = 2 * PARTS * (PLANE_A + PLANE_B);  // bytes: PARTS planes of bf16
  static_assert(WM * WN == 4 && QA >= 1 && QB >= 1 && XB >= 1 && YB >= 1, "tile shape");
};

// quad q of this thread -> (row, first k of the quad) of an R x KC chunk
template <bool KCONTIG, int R, int KC>
__device__ __forceinline__ void quad_rk(int tid, int q, int& r, int& k) {
  const int e = tid + 256 * q;
  if (KCONTIG) { r = e / (KC / 4); k = 4 * (e % (KC / 4)); }
  else { r = e % R; k = 4 * (e / R); }
}

// split four complex values into the four bf16 planes of one LDS row segment
__device__ __forceinline__ void split_store(const Cplx<float> (&v)[4], __bf16* plane, int plane_sz,
                                            int off) {
  bf16x4 rh, rl, ih, il;
#pragma unroll
  for (int t = 0; t < 4; ++t) {
    const __bf16 a = (__bf16)v[t].re, b = (__bf16)v[t].im;
    rh[t] = a;
    rl[t] = (__bf16)(v[t].re - (float)a);
    ih[t] = b;
    il[t] = (__bf16)(v[t].im - (float)b);
  }
  *reinterpret_cast<bf16x4*>(plane + off) = rh;
  *reinterpret_cast<bf16x4*>(plane + plane_sz + off) = rl;
  *reinterpret_cast<bf16x4*>(plane + 2 * plane_sz + off) = ih;
  *reinterpret_cast<bf16x4*>(plane + 3 * plane_sz + off) = il;
}

// the real form: four real values (in .re) into the two planes hi, lo
__device__ __forceinline__ void split_store_real(const Cplx<float> (&v)[4], __bf16* plane, int plane_sz,
                                                 int off) {
  bf16x4 rh, rl;
#pragma unroll
  for (int t = 0; t < 4; ++t) {
    const __bf16 a = (__bf16)v[t].re;
    rh[t] = a;
    rl[t] = (__bf16)(v[t].re - (float)a);
  }
  *reinterpret_cast<bf16x4*>(plane + off) = rh;
  *reinterpret_cast<bf16x4*>(plane + plane_sz + off) = rl;
}

template <int FLAGS, int BM, int BN, int WM, int WN, bool SPLIT, bool REAL = false>
__global__ void __launch_bounds__(256) gemm_bf3_kernel(const GemmSeg* __restrict__ segs,
                                                       const GemmProb* __restrict__ probs,
                                                       const GemmTile* __restrict__ tiles,
                                                       const int64_t* __restrict__ rows,
                                                       const float* __restrict__ A,
                                                       const float* __restrict__ B,
                                                       float* __restrict__ C,
                                                       float* __restrict__ part,
                                                       const int32_t* __restrict__ skip) {
  if (skip && *skip) return;
  typedef Bf3Cfg<FLAGS, BM, BN, WM, WN, REAL> G;
  constexpr int KC = G::KC, QA = G::QA, QB = G::QB, XB = G::XB, YB = G::YB, NP = G::PARTS;
  __shared__ __attribute__((aligned(16))) char smem[G::SMEM];
  __bf16* sA = reinterpret_cast<__bf16*>(smem);          // [NP parts][BM rows]
  __bf16* sB = sA + NP * G::PLANE_A;                     // [NP parts][BN rows]

  const int tid = threadIdx.x;
  const int wave = tid >> 6, lane = tid & 63;
  const int li = lane & 15, lk = lane >> 4;
  const GemmTile tile = tiles[xcd_tile(blockIdx.x, gridDim.x)];
  const GemmProb P = probs[tile.prob];
  const int i0 = tile.tm * BM, j0 = tile.tn * BN;
  const int kfirst = SPLIT ? tile.ks * KC : 0;
  const int kstep = SPLIT ? P.nks * KC : KC;

  int64_t arow[QA];
#pragma unroll
  for (int q = 0; q < QA; ++q) {
    int r, k;
    quad_rk<G::A_KC, BM, KC>(tid, q, r, k);
    arow[q] = 0;
    if ((FLAGS & G_A_ROWMAP) && i0 + r < P.M) arow[q] = rows[P.rowmap + i0 + r];
  }

  Cplx<float> ra[QA][4], rb[QB][4];
  auto load_chunk = [&](const GemmSeg& S, int k0) {
    const int kc = min(KC, S.k - k0);
#pragma unroll
    for (int q = 0; q < QA; ++q) {
      int r, k;
      quad_rk<G::A_KC, BM, KC>(tid, q, r, k);
      const int i = i0 + r;
#pragma unroll
      for (int t = 0; t < 4; ++t) {
        Cplx<float> v{0.f, 0.f};
        if (i < P.M && k + t < kc) {
          const int kk = k0 + k + t;
          const int64_t ix = (FLAGS & G_A_ROWMAP) ? arow[q] + S.a_off + kk
                             : (FLAGS & G_A_T)    ? S.a_off + (int64_t)kk * S.lda + i
                                                  : S.a_off + (int64_t)i * S.lda + kk;
          if constexpr (REAL) {
            v.re = A[ix];
          } else {
            v = ldc(A, ix);
            if (FLAGS & G_A_CONJ) v.im = -v.im;
          }
        }
        ra[q][t] = v;
      }
    }
#pragma unroll
    for (int q = 0; q < QB; ++q) {
      int c, k;
      quad_rk<G::B_KC, BN, KC>(tid, q, c, k);
      const int j = j0 + c;
#pragma unroll
      for (int t = 0; t < 4; ++t) {
        Cplx<float> v{0.f, 0.f};
        if (j < P.N && k + t < kc) {
          const int kk = k0 + k + t;
          const int64_t ix = (FLAGS & G_B_T) ? S.b_off + (int64_t)j * S.ldb + kk : S.b_off + (int64_t)kk * S.ldb + j;
          if constexpr (REAL) v.re = B[ix];
          else v = ldc(B, ix);
        }
        rb[q][t] = v;
      }
    }
  };

  f32x4 cre[XB][YB], cim[XB][YB];
#pragma unroll
  for (int x = 0; x < XB; ++x)
#pragma unroll
    for (int y = 0; y < YB; ++y) {
      cre[x][y] = f32x4{0, 0, 0, 0};
      cim[x][y] = f32x4{0, 0, 0, 0};
    }
  const int wr = (wave % WM) * (BM / WM);
  const int wc = (wave / WM) * (BN / WN);

  int sg = 0, k0 = kfirst;
  GemmSeg S;
  while (sg < P.nseg) {
    S = segs[P.seg0 + sg];
    if (k0 < S.k) break;
    ++sg;
    k0 = kfirst;
  }
  if (sg < P.nseg) load_chunk(S, k0);
  while (sg < P.nseg) {
    __syncthreads();  // previous chunk fully consumed
#pragma unroll
    for (int q = 0; q < QA; ++q) {
      int r, k;
      quad_rk<G::A_KC, BM, KC>(tid, q, r, k);
      if constexpr (REAL) split_store_real(ra[q], sA, G::PLANE_A, lds_rk<G::A_KC>(r, k));
      else split_store(ra[q], sA, G::PLANE_A, lds_rk<G::A_KC>(r, k));
    }
#pragma unroll
    for (int q = 0; q < QB; ++q) {
      int c, k;
      quad_rk<G::B_KC, BN, KC>(tid, q, c, k);
      if constexpr (REAL) split_store_real(rb[q], sB, G::PLANE_B, lds_rk<G::B_KC>(c, k));
      else split_store(rb[q], sB, G::PLANE_B, lds_rk<G::B_KC>(c, k));
    }
    // the staging registers are free again: the next chunk's loads go out before the
    // barrier and stay in flight during it and the products of this chunk
    k0 += kstep;
    while (k0 >= S.k) {
      if (++sg >= P.nseg) break;
      S = segs[P.seg0 + sg];
      k0 = kfirst;
    }
    if (sg < P.nseg) load_chunk(S, k0);
    __syncthreads();
    // k positions beyond the chunk's valid range were staged as zeros
    bf16x8 b[YB][NP];
#pragma unroll
    for (int y = 0; y < YB; ++y)
#pragma unroll
      for (int p = 0; p < NP; ++p)
        b[y][p] = *reinterpret_cast<const bf16x8*>(sB + p * G::PLANE_B + lds_rk<G::B_KC>(wc + y * 16 + li, 8 * lk));
#pragma unroll
    for (int x = 0; x < XB; ++x) {
      bf16x8 a[NP];
#pragma unroll
      for (int p = 0; p < NP; ++p)
        a[p] = *reinterpret_cast<const bf16x8*>(sA + p * G::PLANE_A + lds_rk<G::A_KC>(wr + x * 16 + li, 8 * lk));
      if constexpr (REAL) {  // parts: 0 hi, 1 lo; small products first
#pragma unroll
        for (int y = 0; y < YB; ++y) {
          cre[x][y] = mfma_bf16(a[1], b[y][0], cre[x][y]);
          cre[x][y] = mfma_bf16(a[0], b[y][1], cre[x][y]);
          cre[x][y] = mfma_bf16(a[0], b[y][0], cre[x][y]);
        }
      } else {
      // parts: 0 re_hi, 1 re_lo, 2 im_hi, 3 im_lo
      const bf16x8 nih = neg8(a[2]), nil = neg8(a[3]);
#pragma unroll
      for (int y = 0; y < YB; ++y) {
        cre[x][y] = mfma_bf16(a[1], b[y][0], cre[x][y]);
        cim[x][y] = mfma_bf16(a[1], b[y][2], cim[x][y]);
        cre[x][y] = mfma_bf16(a[0], b[y][1], cre[x][y]);
        cim[x][y] = mfma_bf16(a[0], b[y][3], cim[x][y]);
        cre[x][y] = mfma_bf16(nil, b[y][2], cre[x][y]);
        cim[x][y] = mfma_bf16(a[3], b[y][0], cim[x][y]);
        cre[x][y] = mfma_bf16(nih, b[y][3], cre[x][y]);
        cim[x][y] = mfma_bf16(a[2], b[y][1], cim[x][y]);
        cre[x][y] = mfma_bf16(a[0], b[y][0], cre[x][y]);
        cim[x][y] = mfma_bf16(a[0], b[y][2], cim[x][y]);
        cre[x][y] = mfma_bf16(nih, b[y][2], cre[x][y]);
        cim[x][y] = mfma_bf16(a[2], b[y][0], cim[x][y]);
      }
      }
    }
  }

  if (SPLIT && P.nks > 1) {
    // partial tile of this K split, summed later by gemm_split_reduce_kernel
    const int tiles_n = (P.N + BN - 1) / BN;
    float* dst = part + 2 * ((int64_t)P.slot0 + ((int64_t)tile.tm * tiles_n + tile.tn) * P.nks + tile.ks) * (BM * BN);
#pragma unroll
    for (int x = 0; x < XB; ++x)
#pragma unroll
      for (int r = 0; r < 4; ++r)
#pragma unroll
        for (int y = 0; y < YB; ++y) {
          const int e = (wr + x * 16 + 4 * lk + r) * BN + wc + y * 16 + li;
          if constexpr (REAL) dst[e] = cre[x][y][r];  // first half of the slot, as the reduction reads it
          else stc(dst, e, cre[x][y][r], cim[x][y][r]);
        }
    return;
  }
#pragma unroll
  for (int x = 0; x < XB; ++x) {
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int i = i0 + wr + x * 16 + 4 * lk + r;
      if (i >= P.M) continue;
      const int64_t rbase = (FLAGS & G_C_ROWMAP) ? rows[P.rowmap + i] : P.c_off + (int64_t)i * P.ldc;
#pragma unroll
      for (int y = 0; y < YB; ++y) {
        const int j = j0 + wc + y * 16 + li;
        if (j >= P.N) continue;
        if constexpr (REAL) {
          if (FLAGS & G_C_F64) reinterpret_cast<double*>(C)[rbase + j] = (double)cre[x][y][r];
          else C[rbase + j] = cre[x][y][r];
        } else if (FLAGS & G_C_F64) {
          stc(reinterpret_cast<double*>(C), rbase + j, (double)cre[x][y][r], (double)cim[x][y][r]);
        } else {
          stc(C, rbase + j, cre[x][y][r], cim[x][y][r]);
        }
      }
    }
  }
}

hipError_t launch_gemm_bf16x3(const GemmStage& st, const float* A, const float* B, float* C,
                              float* part, hipStream_t s, const int32_t* skip,
                              const std::function<void()>& between) {
  const int32_t nt = (int32_t)st.tiles.size();
  if (nt == 0) return hipSuccess;
  if (st.nslots > 0 && !part) return hipErrorInvalidValue;
  dim3 grid(nt), block(256);
#define MRD_BF3_CASE(F, TM, TN, WM, WN, SP)                                                     \
  if (st.flags == (F) && st.tile_m == (TM) && st.tile_n == (TN) && st.split == (SP)) {          \
    if (st.real)                                                                                \
      hipLaunchKernelGGL((gemm_bf3_kernel<F, TM, TN, WM, WN, SP, true>), grid, block, 0, s,     \
                         st.d_segs, st.d_probs, st.d_tiles, st.d_rows, A, B, C, part, skip);    \
    else                                                                                        \
      hipLaunchKernelGGL((gemm_bf3_kernel<F, TM, TN, WM, WN, SP>), grid, block, 0, s,           \
                         st.d_segs, st.d_probs, st.d_tiles, st.d_rows, A, B, C, part, skip);    \
    if (between) between();                                                                     \
    if (SP && !st.red_tiles.empty()) {                                                          \
      if (st.real)                                                                              \
        hipLaunchKernelGGL((gemm_split_reduce_kernel<float, F, GemmProb, true>),                \
                           dim3(st.red_tiles.size(), (TM * TN + 1023) / 1024), block, 0, s,     \
                           st.d_probs, st.d_red_tiles, st.d_rows, part, C, TM, TN, skip);       \
      else                                                                                      \
        hipLaunchKernelGGL((gemm_split_reduce_kernel<float, F>),                                \
                           dim3(st.red_tiles.size(), (TM * TN + 1023) / 1024), block, 0, s,     \
                           st.d_probs, st.d_red_tiles, st.d_rows, part, C, TM, TN, skip);       \
    }                                                                                           \
    return hipGetLastError();                                                                   \
  }
  // short-K stages: 128 x 64 (L.theta) or 64 x 64 tiles; long-K stages: 128 x 32 with
  // the K range split over workgroups
  MRD_BF3_CASE(0, 128, 64, 2, 2, false)
  MRD_BF3_CASE(0, 64, 64, 2, 2, false)
  MRD_BF3_CASE(G_A_T | G_A_CONJ, 64, 64, 2, 2, false)
  MRD_BF3_CASE(G_A_T | G_A_CONJ, 32, 32, 2, 2, false)
  MRD_BF3_CASE(G_A_ROWMAP | G_B_T, 64, 64, 2, 2, false)
  MRD_BF3_CASE(G_A_ROWMAP | G_B_T, 64, 32, 4, 1, false)
  MRD_BF3_CASE(G_A_CONJ, 64, 64, 2, 2, false)
  MRD_BF3_CASE(G_A_CONJ, 32, 32, 2, 2, false)
  MRD_BF3_CASE(G_B_T | G_C_ROWMAP, 128, 32, 4, 1, true)
  MRD_BF3_CASE(G_B_T | G_C_ROWMAP | G_C_F64, 128, 32, 4, 1, true)
  MRD_BF3_CASE(G_B_T | G_C_ROWMAP | G_C_F64, 64, 32, 4, 1, true)
  // further shapes for the batched tile tuning
  MRD_BF3_CASE(G_B_T | G_C_ROWMAP, 64, 32, 4, 1, true)
  MRD_BF3_CASE(G_B_T | G_C_ROWMAP, 64, 64, 2, 2, true)
#undef MRD_BF3_CASE
  return hipErrorInvalidValue;
}

}  // namespace mrd
