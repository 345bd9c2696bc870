// HIP kernels for gfx950 (CDNA4): grouped complex block GEMMs on MFMA, sparse MPO
// mixing and precision casts.
//
// Complex data is interleaved (re, im).  A complex product on real MFMA is four real
// products: Cr += Ar Br - Ai Bi, Ci += Ar Bi + Ai Br.
#include "device.hpp"

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

// ---------------------------------------------------------------------------------
// Grouped complex GEMM on MFMA 16x16x4 with LDS staging.
//
// A workgroup (4 waves) owns one BM x BN output tile of one problem and walks the
// problem's K-segments in chunks of KC (8 WIDE, 32 DEEP).  Each chunk of A (BM x KC) and B (KC x BN)
// is loaded cooperatively with coalesced accesses -- consecutive threads read
// consecutive elements along the operand's contiguous dimension -- then stored to LDS
// as separate real / imaginary planes indexed [k][row], so that MFMA operands are
// conflict-free LDS reads.  The global loads of the next chunk are issued before the
// current chunk is multiplied.
//
//   WIDE (BM = BN = 64): waves own the four 32 x 32 quadrants and run the full K.
//   DEEP (BM = BN = 32): every wave runs the whole 32 x 32 tile on its own quarter of
//        each chunk (k in [16w, 16w + 16)); the four partial tiles are summed in fixed
//        order (wave 0 + 1 + 2 + 3) through LDS, so results are reproducible.
//
// MFMA 16x16x4 operand layout (one element per lane): A(i, k) with i = lane % 16,
// k = lane / 16; B(k, j) with j = lane % 16, k = lane / 16.  Result: lane holds four
// rows (Mfma<T>::row) of column lane % 16.  Complex product: Cr += Ar Br - Ai Bi,
// Ci += Ar Bi + Ai Br (A already conjugated when staged, for A_CONJ).
// ---------------------------------------------------------------------------------
template <typename T, int FLAGS, bool DEEP>
struct GemmCfg {
  // K chunk staged per step: short chunks keep the staging planes and registers small
  // (WIDE with chunks of 8: FP64 four waves per SIMD, FP32 seven; DEEP with 32: FP64
  // three, FP32 five -- against two and four with the chunks of 32 / 64 of before)
  static constexpr int KC = DEEP ? 32 : 8;
  static constexpr int BM = DEEP ? 32 : 64;
  static constexpr int BN = DEEP ? 32 : 64;
  static constexpr int NA = BM * KC / 256;  // A elements staged per thread per chunk
  static constexpr int NB = KC * BN / 256;
  // K-contiguous A (row-major, row table, mixed): consecutive threads walk k
  static constexpr bool A_KC = !(FLAGS & G_A_T);
  static constexpr bool B_KC = (FLAGS & G_B_T) != 0;
};

// REAL: real operands and result (the eq. rot formulation): one value per element, one
// product per MFMA step, only the first LDS plane used.
template <typename T, int FLAGS, bool DEEP, bool REAL = false>
__global__ void __launch_bounds__(256) gemm_kernel(const GemmSeg* __restrict__ segs,
                                                   const GemmProb* __restrict__ probs,
                                                   const GemmTile* __restrict__ tiles,
                                                   const int64_t* __restrict__ rows,
                                                   const T* __restrict__ A,
                                                   const T* __restrict__ B,
                                                   T* __restrict__ C,
                                                   T* __restrict__ part,
                                                   const int32_t* __restrict__ skip) {
  if (skip && *skip) return;
  typedef GemmCfg<T, FLAGS, DEEP> G;
  typedef typename Mfma<T>::acc_t acc_t;
  constexpr int BM = G::BM, BN = G::BN, NA = G::NA, NB = G::NB, KC = G::KC;
  // staging planes sA[2][KC][BM + 1], sB[2][KC][BN + 1]; DEEP reuses the space for the
  // cross-wave reduction red[3][32][64] after the K loop
  constexpr int SA = 2 * KC * (BM + 1), SB = 2 * KC * (BN + 1), SR = DEEP ? 3 * 32 * 64 : 0;
  __shared__ T smem[(SA + SB) > SR ? (SA + SB) : SR];
  T (*sA)[KC][BM + 1] = reinterpret_cast<T (*)[KC][BM + 1]>(smem);
  T (*sB)[KC][BN + 1] = reinterpret_cast<T (*)[KC][BN + 1]>(smem + SA);

  const int tid = threadIdx.x;
  const int wave = tid >> 6, lane = tid & 63;
  const int li = lane & 15, lk = lane >> 4;
  const GemmTile tile = tiles[xcd_tile(blockIdx.x, gridDim.x)];
  const GemmProb P = probs[tile.prob];
  const int i0 = tile.tm * BM, j0 = tile.tn * BN;
  // K-split (DEEP): in every segment this workgroup takes chunks ks, ks + nks, ...
  const int kfirst = DEEP ? tile.ks * KC : 0;
  const int kstep = DEEP ? P.nks * KC : KC;
  constexpr int KW = KC / 4;  // DEEP: k range of one wave inside a chunk

  // element e = tid + 256 q of a chunk -> (row, k) of A and (k, col) of B
  auto a_rk = [&](int q, int& r, int& k) {
    const int e = tid + 256 * q;
    if (G::A_KC) { r = e / KC; k = e % KC; } else { k = e / BM; r = e % BM; }
  };
  auto b_kc = [&](int q, int& k, int& c) {
    const int e = tid + 256 * q;
    if (G::B_KC) { c = e / KC; k = e % KC; } else { k = e / BN; c = e % BN; }
  };
  int64_t arow[NA];
#pragma unroll
  for (int q = 0; q < NA; ++q) {
    int r, k;
    a_rk(q, r, k);
    arow[q] = 0;
    if ((FLAGS & G_A_ROWMAP) && i0 + r < P.M) arow[q] = rows[P.rowmap + i0 + r];
  }

  Cplx<T> ra[NA], rb[NB];
  auto load_chunk = [&](const GemmSeg& S, int k0) {
    const int kc = min(KC, S.k - k0);
#pragma unroll
    for (int q = 0; q < NA; ++q) {
      int r, k;
      a_rk(q, r, k);
      const int i = i0 + r;
      Cplx<T> v{0, 0};
      if (i < P.M && k < kc) {
        const int kk = k0 + k;
        const int64_t off = (FLAGS & G_A_ROWMAP) ? arow[q] + S.a_off + kk
                            : (FLAGS & G_A_T)    ? S.a_off + (int64_t)kk * S.lda + i
                                                 : S.a_off + (int64_t)i * S.lda + kk;
        if constexpr (REAL) {
          v.re = A[off];
        } else {
          v = ldc(A, off);
          if (FLAGS & G_A_CONJ) v.im = -v.im;
        }
      }
      ra[q] = v;
    }
#pragma unroll
    for (int q = 0; q < NB; ++q) {
      int k, c;
      b_kc(q, k, c);
      const int j = j0 + c;
      Cplx<T> v{0, 0};
      if (j < P.N && k < kc) {
        const int kk = k0 + k;
        const int64_t off = (FLAGS & G_B_T) ? S.b_off + (int64_t)j * S.ldb + kk : S.b_off + (int64_t)kk * S.ldb + j;
        if constexpr (REAL)
          v.re = B[off];
        else
          v = ldc(B, off);
      }
      rb[q] = v;
    }
  };

  acc_t cre[2][2], cim[2][2];
#pragma unroll
  for (int x = 0; x < 2; ++x)
#pragma unroll
    for (int y = 0; y < 2; ++y) {
      cre[x][y] = acc_t{0, 0, 0, 0};
      cim[x][y] = acc_t{0, 0, 0, 0};
    }
  // sub-tile of this wave
  const int wr = DEEP ? 0 : (wave & 1) * 32;
  const int wc = DEEP ? 0 : (wave >> 1) * 32;

  // first (segment, chunk) of this workgroup
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
    const int kc = min(KC, S.k - k0);
    __syncthreads();  // previous chunk fully consumed
#pragma unroll
    for (int q = 0; q < NA; ++q) {
      int r, k;
      a_rk(q, r, k);
      sA[0][k][r] = ra[q].re;
      if constexpr (!REAL) sA[1][k][r] = ra[q].im;
    }
#pragma unroll
    for (int q = 0; q < NB; ++q) {
      int k, c;
      b_kc(q, k, c);
      sB[0][k][c] = rb[q].re;
      if constexpr (!REAL) sB[1][k][c] = rb[q].im;
    }
    // advance and prefetch the next chunk (the staging registers are free again): the
    // loads stay in flight during the barrier and the products of this chunk
    k0 += kstep;
    while (k0 >= S.k) {
      if (++sg >= P.nseg) break;
      S = segs[P.seg0 + sg];
      k0 = kfirst;
    }
    if (sg < P.nseg) load_chunk(S, k0);
    __syncthreads();
    const int kbeg = DEEP ? wave * KW : 0;
    const int kend = DEEP ? min(kbeg + KW, kc) : kc;
    for (int kb = kbeg; kb < kend; kb += 4) {
      const int k = kb + lk;
      if constexpr (REAL) {
        T a[2], b[2];
#pragma unroll
        for (int x = 0; x < 2; ++x) a[x] = sA[0][k][wr + x * 16 + li];
#pragma unroll
        for (int y = 0; y < 2; ++y) b[y] = sB[0][k][wc + y * 16 + li];
#pragma unroll
        for (int x = 0; x < 2; ++x)
#pragma unroll
          for (int y = 0; y < 2; ++y) cre[x][y] = Mfma<T>::mac(a[x], b[y], cre[x][y]);
        continue;
      }
      T are[2], aim[2], bre[2], bim[2];
#pragma unroll
      for (int x = 0; x < 2; ++x) {
        are[x] = sA[0][k][wr + x * 16 + li];
        aim[x] = sA[1][k][wr + x * 16 + li];
      }
#pragma unroll
      for (int y = 0; y < 2; ++y) {
        bre[y] = sB[0][k][wc + y * 16 + li];
        bim[y] = sB[1][k][wc + y * 16 + li];
      }
#pragma unroll
      for (int x = 0; x < 2; ++x)
#pragma unroll
        for (int y = 0; y < 2; ++y) {
          cre[x][y] = Mfma<T>::mac(are[x], bre[y], cre[x][y]);
          cim[x][y] = Mfma<T>::mac(are[x], bim[y], cim[x][y]);
        }
#pragma unroll
      for (int x = 0; x < 2; ++x)
#pragma unroll
        for (int y = 0; y < 2; ++y) {
          cre[x][y] = Mfma<T>::mac(-aim[x], bim[y], cre[x][y]);
          cim[x][y] = Mfma<T>::mac(aim[x], bre[y], cim[x][y]);
        }
    }
  }

  if constexpr (DEEP) {
    // fixed-order reduction of the four partial tiles
    T (*red)[32][64] = reinterpret_cast<T (*)[32][64]>(smem);
    __syncthreads();  // staging buffers are no longer read
    if (wave > 0) {
#pragma unroll
      for (int x = 0; x < 2; ++x)
#pragma unroll
        for (int y = 0; y < 2; ++y)
#pragma unroll
          for (int r = 0; r < 4; ++r) {
            red[wave - 1][((x * 2 + y) * 4 + r) * 2][lane] = cre[x][y][r];
            if constexpr (!REAL) red[wave - 1][((x * 2 + y) * 4 + r) * 2 + 1][lane] = cim[x][y][r];
          }
    }
    __syncthreads();
    if (wave != 0) return;
#pragma unroll
    for (int x = 0; x < 2; ++x)
#pragma unroll
      for (int y = 0; y < 2; ++y)
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const int e = ((x * 2 + y) * 4 + r) * 2;
          cre[x][y][r] = ((cre[x][y][r] + red[0][e][lane]) + red[1][e][lane]) + red[2][e][lane];
          if constexpr (!REAL)
            cim[x][y][r] = ((cim[x][y][r] + red[0][e + 1][lane]) + red[1][e + 1][lane]) + red[2][e + 1][lane];
        }
    if (P.nks > 1) {
      // partial tile of this K-split, summed later by gemm_split_reduce_kernel
      const int tiles_n = (P.N + BN - 1) / BN;
      T* dst = part + 2 * ((int64_t)P.slot0 + ((int64_t)tile.tm * tiles_n + tile.tn) * P.nks + tile.ks) * 1024;
#pragma unroll
      for (int x = 0; x < 2; ++x)
#pragma unroll
        for (int r = 0; r < 4; ++r)
#pragma unroll
          for (int y = 0; y < 2; ++y) {
            const int rr = x * 16 + Mfma<T>::row(lk, r), cc = y * 16 + li;
            if constexpr (REAL)
              dst[rr * 32 + cc] = cre[x][y][r];  // first half of the slot
            else
              stc(dst, rr * 32 + cc, cre[x][y][r], cim[x][y][r]);
          }
      return;
    }
  }
  // store this wave's 32 x 32 sub-tile
#pragma unroll
  for (int x = 0; x < 2; ++x) {
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int i = i0 + wr + x * 16 + Mfma<T>::row(lk, r);
      if (i >= P.M) continue;
      const int64_t rbase = (FLAGS & G_C_ROWMAP) ? rows[P.rowmap + i] : P.c_off + (int64_t)i * P.ldc;
#pragma unroll
      for (int y = 0; y < 2; ++y) {
        const int j = j0 + wc + y * 16 + li;
        if (j >= P.N) continue;
        if constexpr (REAL)
          C[rbase + j] = cre[x][y][r];
        else
          stc(C, rbase + j, cre[x][y][r], cim[x][y][r]);
      }
    }
  }
}

template <typename T>
hipError_t launch_gemm(const GemmStage& st, const T* A, const T* B, T* C, T* part, hipStream_t s,
                       const int32_t* skip, const std::function<void()>& between) {
  const int32_t nt = (int32_t)st.tiles.size();
  if (nt == 0) return hipSuccess;
  if (st.nslots > 0 && !part) return hipErrorInvalidValue;
  dim3 grid(nt), block(256);
#define MRD_GEMM_CASE(F, D)                                                                   \
  if (st.flags == (F) && st.deep == (D) && st.tile_m == (D ? 32 : 64) &&                     \
      st.tile_n == (D ? 32 : 64) && (D || !st.split)) {                                       \
    if (st.real)                                                                              \
      hipLaunchKernelGGL((gemm_kernel<T, F, D, true>), grid, block, 0, s, st.d_segs,          \
                         st.d_probs, st.d_tiles, st.d_rows, A, B, C, part, skip);             \
    else                                                                                      \
      hipLaunchKernelGGL((gemm_kernel<T, F, D, false>), grid, block, 0, s, st.d_segs,         \
                         st.d_probs, st.d_tiles, st.d_rows, A, B, C, part, skip);             \
    if (between) between();                                                                   \
    if (D && !st.red_tiles.empty()) {                                                         \
      if (st.real)                                                                            \
        hipLaunchKernelGGL((gemm_split_reduce_kernel<T, F, GemmProb, true>),                  \
                           dim3(st.red_tiles.size(), 1), block, 0, s, st.d_probs,             \
                           st.d_red_tiles, st.d_rows, part, C, 32, 32, skip);                 \
      else                                                                                    \
        hipLaunchKernelGGL((gemm_split_reduce_kernel<T, F>), dim3(st.red_tiles.size(), 1),    \
                           block, 0, s, st.d_probs, st.d_red_tiles, st.d_rows, part, C, 32,   \
                           32, skip);                                                         \
    }                                                                                         \
    return hipGetLastError();                                                                 \
  }
  MRD_GEMM_CASE(0, false)
  MRD_GEMM_CASE(G_A_T | G_A_CONJ, false)
  MRD_GEMM_CASE(G_A_ROWMAP | G_B_T, false)
  MRD_GEMM_CASE(G_A_CONJ, false)
  MRD_GEMM_CASE(G_B_T | G_C_ROWMAP, true)
  // further shapes for the batched tile tuning
  MRD_GEMM_CASE(0, true)
  MRD_GEMM_CASE(G_B_T | G_C_ROWMAP, false)
#undef MRD_GEMM_CASE
  return hipErrorInvalidValue;
}

template hipError_t launch_gemm<double>(const GemmStage&, const double*, const double*, double*,
                                        double*, hipStream_t, const int32_t*,
                                        const std::function<void()>&);
template hipError_t launch_gemm<float>(const GemmStage&, const float*, const float*, float*, float*,
                                       hipStream_t, const int32_t*, const std::function<void()>&);

// ---------------------------------------------------------------------------------
// Sparse MPO mixing: each workgroup owns one destination sub-block and sums its few
// scaled source sub-blocks.  Consecutive threads walk consecutive columns.
// ---------------------------------------------------------------------------------
template <typename T, bool REAL = false>
__global__ void __launch_bounds__(256) mix_kernel(const MixTask* __restrict__ tasks,
                                                  const MixSrc* __restrict__ srcs,
                                                  const T* __restrict__ src,
                                                  T* __restrict__ dst,
                                                  const int32_t* __restrict__ skip) {
  if (skip && *skip) return;
  const MixTask tk = tasks[blockIdx.x];
  const int n = tk.rows * tk.cols;
  // 1024 elements per pass, four per thread (e = base + 256 t + thread); the source
  // descriptors are read once per pass and the four loads of a source are independent
  for (int base = 0; base < n; base += 1024) {
    int r[4], c[4];
    T re[4], im[4];
#pragma unroll
    for (int t = 0; t < 4; ++t) {
      const int e = base + 256 * t + threadIdx.x;
      r[t] = e / tk.cols;
      c[t] = e - r[t] * tk.cols;
      re[t] = 0;
      im[t] = 0;
    }
    for (int q = 0; q < tk.nsrc; ++q) {
      const MixSrc sr = srcs[tk.src0 + q];
      const T cr = (T)sr.re, ci = (T)sr.im;
#pragma unroll
      for (int t = 0; t < 4; ++t) {
        if (r[t] >= tk.rows) continue;
        if constexpr (REAL) {  // real coefficients (checked on the host)
          re[t] += cr * src[sr.off + (int64_t)r[t] * sr.ld + c[t]];
        } else {
          const Cplx<T> x = ldc(src, sr.off + (int64_t)r[t] * sr.ld + c[t]);
          re[t] += cr * x.re - ci * x.im;
          im[t] += cr * x.im + ci * x.re;
        }
      }
    }
#pragma unroll
    for (int t = 0; t < 4; ++t) {
      if (r[t] >= tk.rows) continue;
      if constexpr (REAL)
        dst[tk.dst + (int64_t)r[t] * tk.ld_dst + c[t]] = re[t];
      else
        stc(dst, tk.dst + (int64_t)r[t] * tk.ld_dst + c[t], re[t], im[t]);
    }
  }
}

// The workgroup's part of a slab: per = rows x ncol elements, thread t starting at
// (r0, c0) and advancing by (step_r, step_c) per 256 elements.
struct MixPart {
  int per, ncol, r0, c0, step_r, step_c;
};

// Output element store of the mixing: complex in the element type (OT = T), or split
// into four bf16 planes pstride apart (OT = __bf16; see internal.hpp, PsProb).
template <typename T, typename OT>
__device__ __forceinline__ void mix_store(OT* obase, int64_t off, int32_t pstride, T re, T im) {
  if constexpr (sizeof(OT) == 2) {
    const float fr = (float)re, fi = (float)im;
    const __bf16 hr = (__bf16)fr, hi = (__bf16)fi;
    obase[off] = hr;
    obase[off + pstride] = (__bf16)(fr - (float)hr);
    obase[off + 2 * (int64_t)pstride] = hi;
    obase[off + 3 * (int64_t)pstride] = (__bf16)(fi - (float)hi);
  } else {
    stc(obase, off, re, im);
  }
}

// One output task of a slab with NC coefficients, all read once before the element
// loop (the generic loop reads the coefficient of every term of every element and waits
// for it); the terms are summed in the same order.  REAL: one T per element and real
// coefficients (the eq. rot form).
template <typename T, typename OT, int NC, bool REAL>
__device__ __forceinline__ void mix_slab_task(const SlabTask& k, const SlabCoef* __restrict__ coefs,
                                              const T* lds, OT* obase, const MixPart& p) {
  T cr[NC], ci[NC];
  int bo[NC];
#pragma unroll
  for (int q = 0; q < NC; ++q) {
    const SlabCoef w = coefs[k.c0 + q];
    cr[q] = (T)w.re;
    ci[q] = (T)w.im;
    bo[q] = w.blk * p.per;
  }
  int r = p.r0, c = p.c0;
  for (int e = threadIdx.x; e < p.per; e += 256) {
    T re = 0, im = 0;
#pragma unroll
    for (int q = 0; q < NC; ++q) {
      if constexpr (REAL) {
        re += cr[q] * lds[(int64_t)bo[q] + e];
      } else {
        const T* x = lds + 2 * ((int64_t)bo[q] + e);
        re += cr[q] * x[0] - ci[q] * x[1];
        im += cr[q] * x[1] + ci[q] * x[0];
      }
    }
    if constexpr (REAL) obase[(int64_t)r * k.ld_dst + c] = re;
    else mix_store<T, OT>(obase, (int64_t)r * k.ld_dst + c, k.pstride, re, im);
    r += p.step_r;
    c += p.step_c;
    if (c >= p.ncol) {
      c -= p.ncol;
      ++r;
    }
  }
}

// Slab form: stage the workgroup's part (rows r0.., columns col0..) of every source block
// of its slab in LDS (planes [block][row][col], interleaved complex, or one T per element
// when REAL), then produce that part of each task of the slab from LDS.  Elements e of
// the part map to (row, col) with a running (row, col) pair instead of a division per
// element.  OT: output element type (T, or __bf16 for an output split into planes).
template <typename T, typename OT, bool REAL = false>
__global__ void __launch_bounds__(256) mix_slab_kernel(const SlabWG* __restrict__ wgs,
                                                       const SlabBlk* __restrict__ blks,
                                                       const SlabTask* __restrict__ tasks,
                                                       const SlabCoef* __restrict__ coefs,
                                                       const T* __restrict__ src,
                                                       OT* __restrict__ dst,
                                                       const int32_t* __restrict__ skip) {
  static_assert(!REAL || sizeof(OT) == sizeof(T), "real mixing writes its own element type");
  constexpr int EW = REAL ? 1 : 2;  // T values per element
  if (skip && *skip) return;
  extern __shared__ __attribute__((aligned(16))) char mix_lds[];
  T* lds = reinterpret_cast<T*>(mix_lds);
  const SlabWG g = wgs[blockIdx.x];
  const int per = g.nr * g.ncol;
  const int step_r = 256 / g.ncol, step_c = 256 - step_r * g.ncol;
  const int r_init = threadIdx.x / g.ncol, c_init = threadIdx.x - r_init * g.ncol;
  // The blocks of a slab share the part's (row, col) walk: the same element of MIX_G
  // blocks is loaded at once (a group's missing blocks re-read its last one, in range of
  // the slab's block table, and are not stored), so every thread has MIX_G loads in
  // flight instead of one.
  constexpr int MIX_G = 8;
  for (int b0 = 0; b0 < g.nblk; b0 += MIX_G) {
    const int nb = min(MIX_G, g.nblk - b0);
    const T* base[MIX_G];
    int64_t ld[MIX_G];
#pragma unroll
    for (int u = 0; u < MIX_G; ++u) {
      const SlabBlk k = blks[g.blk0 + b0 + min(u, nb - 1)];
      base[u] = src + EW * (k.off + (int64_t)g.r0 * k.ld + g.col0);
      ld[u] = k.ld;
    }
    int r = r_init, c = c_init;
    for (int e = threadIdx.x; e < per; e += 256) {
      if constexpr (REAL) {
        T v[MIX_G];
#pragma unroll
        for (int u = 0; u < MIX_G; ++u) v[u] = base[u][(int64_t)r * ld[u] + c];
#pragma unroll
        for (int u = 0; u < MIX_G; ++u)
          if (u < nb) lds[(int64_t)(b0 + u) * per + e] = v[u];
      } else {
        Cplx<T> v[MIX_G];
#pragma unroll
        for (int u = 0; u < MIX_G; ++u) v[u] = ldc(base[u], (int64_t)r * ld[u] + c);
#pragma unroll
        for (int u = 0; u < MIX_G; ++u)
          if (u < nb) {
            T* out = lds + 2 * ((int64_t)(b0 + u) * per + e);
            out[0] = v[u].re;
            out[1] = v[u].im;
          }
      }
      r += step_r;
      c += step_c;
      if (c >= g.ncol) {
        c -= g.ncol;
        ++r;
      }
    }
  }
  __syncthreads();
  for (int t = 0; t < g.ntask; ++t) {
    const SlabTask k = tasks[g.task0 + t];
    // elements of T (complex: two T each) or bf16 elements of one plane
    OT* obase = dst + (sizeof(OT) == 2 ? 1 : EW) * (k.dst + (int64_t)g.r0 * k.ld_dst + g.col0);
    const MixPart part{per, g.ncol, r_init, c_init, step_r, step_c};
    switch (k.nc) {  // uniform over the workgroup
      case 1: mix_slab_task<T, OT, 1, REAL>(k, coefs, lds, obase, part); continue;
      case 2: mix_slab_task<T, OT, 2, REAL>(k, coefs, lds, obase, part); continue;
      case 3: mix_slab_task<T, OT, 3, REAL>(k, coefs, lds, obase, part); continue;
      case 4: mix_slab_task<T, OT, 4, REAL>(k, coefs, lds, obase, part); continue;
      case 5: mix_slab_task<T, OT, 5, REAL>(k, coefs, lds, obase, part); continue;
      case 6: mix_slab_task<T, OT, 6, REAL>(k, coefs, lds, obase, part); continue;
      case 7: mix_slab_task<T, OT, 7, REAL>(k, coefs, lds, obase, part); continue;
      case 8: mix_slab_task<T, OT, 8, REAL>(k, coefs, lds, obase, part); continue;
      default: break;
    }
    int r = r_init, c = c_init;
    for (int e = threadIdx.x; e < per; e += 256) {
      T re = 0, im = 0;
      for (int q = 0; q < k.nc; ++q) {
        const SlabCoef w = coefs[k.c0 + q];
        const T cr = (T)w.re, ci = (T)w.im;
        if constexpr (REAL) {
          re += cr * lds[(int64_t)w.blk * per + e];
        } else {
          const T* x = lds + 2 * ((int64_t)w.blk * per + e);
          re += cr * x[0] - ci * x[1];
          im += cr * x[1] + ci * x[0];
        }
      }
      if constexpr (REAL) obase[(int64_t)r * k.ld_dst + c] = re;
      else mix_store<T, OT>(obase, (int64_t)r * k.ld_dst + c, k.pstride, re, im);
      r += step_r;
      c += step_c;
      if (c >= g.ncol) {
        c -= g.ncol;
        ++r;
      }
    }
  }
}

template <typename T>
hipError_t launch_mix(const MixStage& st, const T* src, T* dst, hipStream_t s, const int32_t* skip) {
  if (st.tasks.empty()) return hipSuccess;
  if (st.real) {  // slab form if its tables were sized for real elements, else task form
    if (!st.wgs.empty() && st.slab_eb == (int)sizeof(T))
      hipLaunchKernelGGL((mix_slab_kernel<T, T, true>), dim3((uint32_t)st.wgs.size()), dim3(256),
                         (uint32_t)st.lds_bytes, s, st.d_wgs, st.d_blks, st.d_stasks, st.d_coefs, src,
                         dst, skip);
    else
      hipLaunchKernelGGL((mix_kernel<T, true>), dim3((uint32_t)st.tasks.size()), dim3(256), 0, s,
                         st.d_tasks, st.d_srcs, src, dst, skip);
    return hipGetLastError();
  }
  if (!st.wgs.empty() && st.slab_eb == (int)(2 * sizeof(T))) {
    hipLaunchKernelGGL((mix_slab_kernel<T, T>), dim3((uint32_t)st.wgs.size()), dim3(256),
                       (uint32_t)st.lds_bytes, s, st.d_wgs, st.d_blks, st.d_stasks, st.d_coefs, src,
                       dst, skip);
    return hipGetLastError();
  }
  hipLaunchKernelGGL((mix_kernel<T>), dim3((uint32_t)st.tasks.size()), dim3(256), 0, s,
                     st.d_tasks, st.d_srcs, src, dst, skip);
  return hipGetLastError();
}
hipError_t launch_mix_split(const MixStage& st, const float* src, __bf16* dst, hipStream_t s,
                            const int32_t* skip) {
  if (st.tasks.empty()) return hipSuccess;
  if (st.wgs.empty() || st.slab_eb != 8) return hipErrorInvalidValue;
  hipLaunchKernelGGL((mix_slab_kernel<float, __bf16>), dim3((uint32_t)st.wgs.size()), dim3(256),
                     (uint32_t)st.lds_bytes, s, st.d_wgs, st.d_blks, st.d_stasks, st.d_coefs, src,
                     dst, skip);
  return hipGetLastError();
}

template hipError_t launch_mix<double>(const MixStage&, const double*, double*, hipStream_t,
                                       const int32_t*);
template hipError_t launch_mix<float>(const MixStage&, const float*, float*, hipStream_t,
                                      const int32_t*);

// ---------------------------------------------------------------------------------
// Precision casts.
// ---------------------------------------------------------------------------------
__global__ void cast_d2f_kernel(const double* __restrict__ in, float* __restrict__ out, int64_t n,
                                const int32_t* __restrict__ skip) {
  if (skip && *skip) return;
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x)
    out[i] = (float)in[i];
}
__global__ void cast_f2d_kernel(const float* __restrict__ in, double* __restrict__ out, int64_t n,
                                const int32_t* __restrict__ skip) {
  if (skip && *skip) return;
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
// Real parts of n complex128 values (interleaved) into n doubles, and back (imaginary
// parts zero): a state held complex with zero imaginary parts handed to a real plan.
__global__ void re_take_kernel(const double* __restrict__ c, double* __restrict__ r, int64_t n) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x)
    r[i] = c[2 * i];
}
__global__ void re_put_kernel(const double* __restrict__ r, double* __restrict__ c, int64_t n) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x) {
    c[2 * i] = r[i];
    c[2 * i + 1] = 0.0;
  }
}
hipError_t launch_re_take(const double* c, double* r, int64_t n, hipStream_t s) {
  if (n == 0) return hipSuccess;
  hipLaunchKernelGGL(re_take_kernel, grid_for(n), dim3(256), 0, s, c, r, n);
  return hipGetLastError();
}
hipError_t launch_re_put(const double* r, double* c, int64_t n, hipStream_t s) {
  if (n == 0) return hipSuccess;
  hipLaunchKernelGGL(re_put_kernel, grid_for(n), dim3(256), 0, s, r, c, n);
  return hipGetLastError();
}
hipError_t launch_cast_d2f(const double* in, float* out, int64_t n, hipStream_t s,
                           const int32_t* skip) {
  if (n == 0) return hipSuccess;
  hipLaunchKernelGGL(cast_d2f_kernel, grid_for(n), dim3(256), 0, s, in, out, n, skip);
  return hipGetLastError();
}
hipError_t launch_cast_f2d(const float* in, double* out, int64_t n, hipStream_t s,
                           const int32_t* skip) {
  if (n == 0) return hipSuccess;
  hipLaunchKernelGGL(cast_f2d_kernel, grid_for(n), dim3(256), 0, s, in, out, n, skip);
  return hipGetLastError();
}

// One launch over many (src, dst, n) conversion jobs; block b serves the job whose first
// block c0 is the largest one <= b, 1024 reals per block.
template <bool D2F>
__global__ void __launch_bounds__(256) cast_batch_kernel(const CastJob* __restrict__ jobs, int njobs) {
  int lo = 0, hi = njobs - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (jobs[mid].c0 <= (int)blockIdx.x) lo = mid;
    else hi = mid - 1;
  }
  const CastJob j = jobs[lo];
  const int64_t base = (int64_t)(blockIdx.x - j.c0) * 1024 + threadIdx.x;
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    const int64_t i = base + 256 * q;
    if (i >= j.n) break;
    if (D2F) glb(static_cast<float*>(j.dst))[i] = (float)glb(static_cast<const double*>(j.src))[i];
    else glb(static_cast<double*>(j.dst))[i] = (double)glb(static_cast<const float*>(j.src))[i];
  }
}

int32_t cast_layout(std::vector<CastJob>& jobs) {
  int32_t nb = 0;
  for (auto& j : jobs) {
    j.c0 = nb;
    nb += (int32_t)((j.n + 1023) / 1024);
  }
  return nb;
}

hipError_t launch_cast_batch(bool d2f, const CastJob* jobs, int32_t njobs, int32_t nblocks,
                             hipStream_t s) {
  if (nblocks == 0) return hipSuccess;
  if (d2f)
    hipLaunchKernelGGL(cast_batch_kernel<true>, dim3(nblocks), dim3(256), 0, s, jobs, njobs);
  else
    hipLaunchKernelGGL(cast_batch_kernel<false>, dim3(nblocks), dim3(256), 0, s, jobs, njobs);
  return hipGetLastError();
}

}  // namespace mrd
