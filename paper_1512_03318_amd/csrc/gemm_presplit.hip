// Split-precision (BF16x3) grouped complex GEMM on operands that are already split.
//
// Both operands arrive as four bf16 planes (re_hi, re_lo, im_hi, im_lo), k contiguous
// and padded to a multiple of 8 (internal.hpp, PsProb), so the kernel does no
// conversion arithmetic at all: a chunk of 32 k values is moved from HBM to LDS with
// 16-byte loads and stores, and the MFMA fragments are 16-byte LDS reads.  The product
// is the same as that of gemm_bf3_kernel on the FP32 values the planes were split from:
// three bf16 products per real product (lo x lo dropped), FP32 accumulation, the same
// twelve v_mfma_f32_16x16x32_bf16 per 16 x 16 x 32 complex block in the same order, and
// the same chunk sequence and K splits, so the results are the same bit for bit.
//
// Who splits: L and R once per effective Hamiltonian (plan creation), theta once per
// matvec (launch_split), and the MPO mixing writes its output Z split (kernels.hip), so
// both block GEMMs of the matvec run on pre-split operands.
//
// LDS holds one chunk per plane as rows of 64 bytes (4 groups of 8 k), no padding; the
// 16-byte group g of row r sits at position g ^ f(r), f(r) = ((r >> 1) ^ (r >> 3)) & 3.
// The fragment read of one MFMA block (16 rows, one group each, 16 bytes per lane) then
// hits 16 distinct 16-byte bank slots, and the staging stores (4 groups of each row,
// rows in lane order) as well.
#include "device.hpp"

namespace mrd {

namespace {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
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

__device__ __forceinline__ int swz(int r) { return ((r >> 1) ^ (r >> 3)) & 3; }

}  // namespace

template <int BM, int BN, int WM, int WN, bool SPLIT, int COUT>
__global__ void __launch_bounds__(256) gemm_ps_kernel(const PsProb* __restrict__ probs,
                                                      const GemmTile* __restrict__ tiles,
                                                      const int64_t* __restrict__ rows,
                                                      const __bf16* __restrict__ A,
                                                      const __bf16* __restrict__ B,
                                                      void* __restrict__ C,
                                                      float* __restrict__ part,
                                                      const int32_t* __restrict__ skip) {
  if (skip && *skip) return;
  constexpr int KC = 32;
  constexpr int GA = BM * 4, GB = BN * 4;  // 16-byte groups of one plane per chunk
  constexpr int NA = 4 * GA / 256, NB = 4 * GB / 256;  // staging loads per thread
  constexpr int XB = BM / WM / 16, YB = BN / WN / 16;  // MFMA blocks per wave
  static_assert(WM * WN == 4 && NA >= 1 && NB >= 1 && XB >= 1 && YB >= 1, "tile shape");
  __shared__ u32x4 sA[4 * GA];
  __shared__ u32x4 sB[4 * GB];

  const int tid = threadIdx.x;
  const int wave = tid >> 6, lane = tid & 63;
  const int li = lane & 15, lk = lane >> 4;
  const GemmTile tile = tiles[xcd_tile(blockIdx.x, gridDim.x)];
  const PsProb P = probs[tile.prob];
  const int i0 = tile.tm * BM, j0 = tile.tn * BN;
  const int nchunk = (P.kp + KC - 1) / KC;
  const int cstep = SPLIT ? P.nks : 1;
  int ch = SPLIT ? tile.ks : 0;

  // staging item q of this thread: group g of row r of plane p (groups fastest, so a
  // wave reads whole 64-byte row segments)
  u32x4 ra[NA], rb[NB];
  auto load_chunk = [&](int c) {
    const int k0 = c * KC;
#pragma unroll
    for (int q = 0; q < NA; ++q) {
      const int e = tid + 256 * q, g = e & 3, r = (e >> 2) % BM, p = e / GA;
      const int i = i0 + r, k = k0 + 8 * g;
      u32x4 v = {0u, 0u, 0u, 0u};
      if (i < P.M && k < P.kp)
        v = *reinterpret_cast<const u32x4*>(A + P.a_off + p * P.a_ps + (int64_t)i * P.kp + k);
      ra[q] = v;
    }
#pragma unroll
    for (int q = 0; q < NB; ++q) {
      const int e = tid + 256 * q, g = e & 3, r = (e >> 2) % BN, p = e / GB;
      const int j = j0 + r, k = k0 + 8 * g;
      u32x4 v = {0u, 0u, 0u, 0u};
      if (j < P.N && k < P.kp)
        v = *reinterpret_cast<const u32x4*>(B + P.b_off + p * P.b_ps + (int64_t)j * P.kp + k);
      rb[q] = v;
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

  if (ch < nchunk) load_chunk(ch);
  while (ch < nchunk) {
    __syncthreads();  // previous chunk fully consumed
#pragma unroll
    for (int q = 0; q < NA; ++q) {
      const int e = tid + 256 * q, g = e & 3, r = (e >> 2) % BM, p = e / GA;
      sA[p * GA + r * 4 + (g ^ swz(r))] = ra[q];
    }
#pragma unroll
    for (int q = 0; q < NB; ++q) {
      const int e = tid + 256 * q, g = e & 3, r = (e >> 2) % BN, p = e / GB;
      sB[p * GB + r * 4 + (g ^ swz(r))] = rb[q];
    }
    // the staging registers are free again: the next chunk's loads are in flight during
    // the barrier and the products of this chunk
    ch += cstep;
    if (ch < nchunk) load_chunk(ch);
    __syncthreads();
    bf16x8 b[YB][4];
#pragma unroll
    for (int y = 0; y < YB; ++y) {
      const int r = wc + y * 16 + li;
#pragma unroll
      for (int p = 0; p < 4; ++p) b[y][p] = __builtin_bit_cast(bf16x8, sB[p * GB + r * 4 + (lk ^ swz(r))]);
    }
#pragma unroll
    for (int x = 0; x < XB; ++x) {
      const int r = wr + x * 16 + li;
      bf16x8 a[4];
#pragma unroll
      for (int p = 0; p < 4; ++p) a[p] = __builtin_bit_cast(bf16x8, sA[p * GA + r * 4 + (lk ^ swz(r))]);
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

  if (SPLIT && P.nks > 1) {
    // partial tile of this K split, summed in split order by the reduction kernel
    const int tiles_n = (P.N + BN - 1) / BN;
    float* dst = part + 2 * ((int64_t)P.slot0 + ((int64_t)tile.tm * tiles_n + tile.tn) * P.nks + tile.ks) * (BM * BN);
#pragma unroll
    for (int x = 0; x < XB; ++x)
#pragma unroll
      for (int r = 0; r < 4; ++r)
#pragma unroll
        for (int y = 0; y < YB; ++y)
          stc(dst, (wr + x * 16 + 4 * lk + r) * BN + wc + y * 16 + li, cre[x][y][r], cim[x][y][r]);
    return;
  }
#pragma unroll
  for (int x = 0; x < XB; ++x) {
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int i = i0 + wr + x * 16 + 4 * lk + r;
      if (i >= P.M) continue;
      const int64_t rbase = COUT == 1 ? rows[P.rowmap + i] : P.c_off + (int64_t)i * P.ldc;
#pragma unroll
      for (int y = 0; y < YB; ++y) {
        const int j = j0 + wc + y * 16 + li;
        if (j >= P.N) continue;
        if (COUT == 1)
          stc(static_cast<double*>(C), rbase + j, (double)cre[x][y][r], (double)cim[x][y][r]);
        else
          stc(static_cast<float*>(C), rbase + j, cre[x][y][r], cim[x][y][r]);
      }
    }
  }
}

hipError_t launch_gemm_ps(const PsStage& st, const __bf16* A, const __bf16* B, void* C, float* part,
                          hipStream_t s, const int32_t* skip, const std::function<void()>& between) {
  const int32_t nt = (int32_t)st.tiles.size();
  if (nt == 0) return hipSuccess;
  if (st.nslots > 0 && !part) return hipErrorInvalidValue;
  dim3 grid(nt), block(256);
#define MRD_PS_CASE(TM, TN, WM, WN, SP, CO)                                                       \
  if (st.tile_m == (TM) && st.tile_n == (TN) && st.split == (SP) && st.cout == (CO)) {            \
    hipLaunchKernelGGL((gemm_ps_kernel<TM, TN, WM, WN, SP, CO>), grid, block, 0, s, st.d_probs,   \
                       st.d_tiles, st.d_rows, A, B, C, part, skip);                                \
    if (between) between();                                                                       \
    if (SP && !st.red_tiles.empty())                                                              \
      hipLaunchKernelGGL((gemm_split_reduce_kernel<float, (CO == 1 ? (G_C_ROWMAP | G_C_F64) : 0), \
                                                   PsProb>),                                      \
                         dim3(st.red_tiles.size(), (TM * TN + 1023) / 1024), block, 0, s,         \
                         st.d_probs, st.d_red_tiles, st.d_rows, part, static_cast<float*>(C), TM,  \
                         TN, skip);                                                               \
    return hipGetLastError();                                                                     \
  }
  MRD_PS_CASE(128, 64, 2, 2, false, 0)
  MRD_PS_CASE(128, 32, 4, 1, true, 1)
#undef MRD_PS_CASE
  return hipErrorInvalidValue;
}

// ---------------------------------------------------------------------------------
// Stream-K persistent form (schedule: internal.hpp, SkTile / SkSeg).  One workgroup per
// CU walks its run of chunks through SK_NS LDS stages filled by direct global-to-LDS
// loads (global_load_lds_dwordx4: lane l of a wave writes 16 bytes at the stage address
// + 16 l, so the swizzle is applied by choosing which global group each lane loads).
// Eight waves (a 4 x 2 grid of 32 x 32 sub-tiles) share the stages, two per SIMD.
// While chunk i is multiplied, the loads of chunks i + 1 .. i + SK_NS - 1 are in flight,
// across tile boundaries too: no staging registers, no per-tile pipeline start.
//
// Ordering: each wave issues exactly SK_LPC load instructions per chunk, and vector
// memory operations complete in issue order, so "my loads of chunk i have landed" is
// vmcnt <= SK_LPC x (chunks issued after i); the stores at a segment end only add to
// that count.  Every wave waits so (and for its own LDS reads of the previous chunk),
// then the workgroup barrier makes the stage complete for all waves, and only after it
// is the stage of chunk i - 1 refilled.  Rows past M or N load the last valid row (their
// results are never stored); kp is a multiple of the chunk width, so no k is out of range.
// The products and their order within a chunk are those of gemm_ps_kernel; the K order
// within a tile is the chunk order, split at segment boundaries and summed in K order.
// ---------------------------------------------------------------------------------
#define MRD_LDS __attribute__((address_space(3)))

namespace {

constexpr int SK_NS = 3;                       // LDS stages
constexpr int SK_SA = 16 * SK_BM;              // 16-byte slots of A per stage (4 planes x rows x 4)
constexpr int SK_SB = 16 * SK_BN;
constexpr int SK_STAGE = SK_SA + SK_SB;
constexpr int SK_WAVES = 8;                    // two waves per SIMD hide each other's LDS and MFMA waits
constexpr int SK_LPC = (SK_BM + SK_BN) / 4 / SK_WAVES;  // load instructions per wave per chunk
constexpr int SK_WM = 4, SK_WN = 2;            // wave grid over the tile
constexpr int SK_XB = SK_BM / SK_WM / 16, SK_YB = SK_BN / SK_WN / 16;
static_assert(SK_BM % 64 == 0 && SK_BN % 64 == 0 && SK_KC == 32 && SK_WM * SK_WN == SK_WAVES &&
              (SK_BM / 4) % SK_WAVES == 0 && (SK_BN / 4) % SK_WAVES == 0, "stream-K tile");
static_assert((SK_NS - 2) * SK_LPC <= 63, "vmcnt range");

// s_waitcnt with vmcnt <= vm, lgkmcnt = 0, expcnt unconstrained (gfx9 encoding)
template <int VM>
__device__ __forceinline__ void sk_waitcnt() {
  __builtin_amdgcn_s_waitcnt((VM & 15) | ((VM >> 4) << 14) | (7 << 4));
}

// All waves: this wave's loads of the chunk about to be used (all but the last `after`
// chunks it issued) and its LDS reads have completed; then the workgroup barrier.
// (sched_barrier keeps the compiler from moving any instruction across the wait and the
// barrier; an inline-asm memory clobber would do the same but makes the compiler wait
// for every load in flight.)
__device__ __forceinline__ void sk_sync(int after) {
  __builtin_amdgcn_sched_barrier(0);
  if (after <= 0)
    sk_waitcnt<0>();
  else
    sk_waitcnt<SK_LPC * (SK_NS - 2)>();  // after == SK_NS - 2 (the pipeline's steady state)
  __builtin_amdgcn_s_barrier();
  __builtin_amdgcn_sched_barrier(0);
}

__device__ __forceinline__ void sk_issue(MRD_LDS u32x4* __restrict__ st, const SkJob& J, int k0,
                                         const __bf16* __restrict__ A, const __bf16* __restrict__ B, int wave,
                                         int lane) {
  const int rl = lane >> 2, sl = lane & 3;
#pragma unroll
  for (int t = 0; t < SK_BM / 4 / SK_WAVES; ++t) {  // A: blocks of 16 rows of one plane
    const int q = wave + SK_WAVES * t, p = q / (SK_BM / 16), rb = q % (SK_BM / 16);
    const int r = rb * 16 + rl, g = sl ^ swz(r);
    const int i = min(J.i0 + r, J.M - 1);
    const __bf16* src = A + J.a_off + p * J.a_ps + (int64_t)i * J.kp + k0 + 8 * g;
    __builtin_amdgcn_global_load_lds((const MRD_GLOBAL void*)src, (MRD_LDS void*)(st + p * SK_BM * 4 + rb * 64),
                                     16, 0, 0);
  }
#pragma unroll
  for (int t = 0; t < SK_BN / 4 / SK_WAVES; ++t) {  // B
    const int q = wave + SK_WAVES * t, p = q / (SK_BN / 16), rb = q % (SK_BN / 16);
    const int r = rb * 16 + rl, g = sl ^ swz(r);
    const int j = min(J.j0 + r, J.N - 1);
    const __bf16* src = B + J.b_off + p * J.b_ps + (int64_t)j * J.kp + k0 + 8 * g;
    __builtin_amdgcn_global_load_lds((const MRD_GLOBAL void*)src,
                                     (MRD_LDS void*)(st + SK_SA + p * SK_BN * 4 + rb * 64), 16, 0, 0);
  }
}

__device__ __forceinline__ void sk_mma(const MRD_LDS u32x4* __restrict__ st, f32x4 (&cre)[SK_XB][SK_YB],
                                       f32x4 (&cim)[SK_XB][SK_YB], int wr, int wc, int li, int lk) {
  bf16x8 b[SK_YB][4];
#pragma unroll
  for (int y = 0; y < SK_YB; ++y) {
    const int r = wc + y * 16 + li;
#pragma unroll
    for (int p = 0; p < 4; ++p) b[y][p] = __builtin_bit_cast(bf16x8, st[SK_SA + p * SK_BN * 4 + r * 4 + (lk ^ swz(r))]);
  }
#pragma unroll
  for (int x = 0; x < SK_XB; ++x) {
    const int r = wr + x * 16 + li;
    bf16x8 a[4];
#pragma unroll
    for (int p = 0; p < 4; ++p) a[p] = __builtin_bit_cast(bf16x8, st[p * SK_BM * 4 + r * 4 + (lk ^ swz(r))]);
    const bf16x8 nih = neg8(a[2]), nil = neg8(a[3]);
#pragma unroll
    for (int y = 0; y < SK_YB; ++y) {
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

// One stream-K step: wait for chunk i's stage, refill the stage of chunk i - 1 with
// chunk i + SK_NS - 1 (when there is one), multiply chunk i.
__device__ __forceinline__ void sk_step(const MRD_LDS u32x4* __restrict__ cur, MRD_LDS u32x4* __restrict__ nxt,
                                        int after, bool refill, const SkJob& Jn, int k0n,
                                        const __bf16* __restrict__ A, const __bf16* __restrict__ B,
                                        f32x4 (&cre)[SK_XB][SK_YB], f32x4 (&cim)[SK_XB][SK_YB], int wave,
                                        int lane, int wr, int wc, int li, int lk) {
  sk_sync(after);
  if (refill) sk_issue(nxt, Jn, k0n, A, B, wave, lane);
  sk_mma(cur, cre, cim, wr, wc, li, lk);
}

}  // namespace

template <int COUT>
__global__ void __launch_bounds__(64 * SK_WAVES) gemm_sk_kernel(const SkJob* __restrict__ jobs,
                                                               const int32_t* __restrict__ wgseg,
                                                               const int64_t* __restrict__ rows,
                                                               const __bf16* __restrict__ A,
                                                               const __bf16* __restrict__ B,
                                                               void* __restrict__ C, float* __restrict__ part,
                                                               const int32_t* __restrict__ skip) {
  if (skip && *skip) return;
  __shared__ u32x4 lds_raw[SK_NS * SK_STAGE];
  MRD_LDS u32x4* const lds = (MRD_LDS u32x4*)lds_raw;
  const int w = xcd_tile(blockIdx.x, gridDim.x);  // consecutive runs (neighbouring tiles) share an XCD
  const int sb = wgseg[w], se = wgseg[w + 1];
  if (sb >= se) return;
  const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
  const int li = lane & 15, lk = lane >> 4;
  const int wr = (wave % SK_WM) * (SK_BM / SK_WM), wc = (wave / SK_WM) * (SK_BN / SK_WN);
  int total = 0;
  for (int q = sb; q < se; ++q) total += jobs[q].c1 - jobs[q].c0;

  // issue cursor: job `is` (a copy in `ji`, the next one prefetched in `jn`), chunk `ic`
  int is = sb, issued = 0;
  SkJob ji = jobs[sb];
  SkJob jn = jobs[min(sb + 1, se - 1)];
  int ic = ji.c0;
  auto advance = [&] {
    ++issued;
    if (++ic == ji.c1 && ++is < se) {
      ji = jn;
      ic = ji.c0;
      jn = jobs[min(is + 1, se - 1)];
    }
  };
  for (int q = 0; q < SK_NS - 1 && issued < total; ++q) {
    sk_issue(lds + q * SK_STAGE, ji, ic * SK_KC, A, B, wave, lane);
    advance();
  }

  f32x4 cre[SK_XB][SK_YB], cim[SK_XB][SK_YB];
  auto zero = [&] {
#pragma unroll
    for (int x = 0; x < SK_XB; ++x)
#pragma unroll
      for (int y = 0; y < SK_YB; ++y) {
        cre[x][y] = f32x4{0, 0, 0, 0};
        cim[x][y] = f32x4{0, 0, 0, 0};
      }
  };
  zero();
  int cs = sb, cend = jobs[sb].c1 - jobs[sb].c0;  // compute cursor: job, chunks left in it
  for (int i = 0; i < total; ++i) {
    const int after = issued - (i + 1);  // chunks issued after chunk i
    const bool refill = issued < total;
    const int sc = i % SK_NS, sn = (i + SK_NS - 1) % SK_NS;
    sk_step(lds + sc * SK_STAGE, lds + sn * SK_STAGE, after, refill, ji, ic * SK_KC, A, B, cre, cim, wave, lane,
            wr, wc, li, lk);
    if (refill) advance();
    if (--cend > 0) continue;
    // end of a job: store the tile (slot < 0) or its partial, then start the next
    const SkJob J = jobs[cs];
    if (J.slot >= 0) {
      float* dst = part + 2 * (int64_t)J.slot * (SK_BM * SK_BN);
#pragma unroll
      for (int x = 0; x < SK_XB; ++x)
#pragma unroll
        for (int r = 0; r < 4; ++r)
#pragma unroll
          for (int y = 0; y < SK_YB; ++y)
            stc(dst, (wr + x * 16 + 4 * lk + r) * SK_BN + wc + y * 16 + li, cre[x][y][r], cim[x][y][r]);
    } else {
#pragma unroll
      for (int x = 0; x < SK_XB; ++x)
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const int gi = J.i0 + wr + x * 16 + 4 * lk + r;
          if (gi >= J.M) continue;
          const int64_t rbase = COUT == 1 ? rows[J.rowmap + gi] : J.c_off + (int64_t)gi * J.ldc;
#pragma unroll
          for (int y = 0; y < SK_YB; ++y) {
            const int gj = J.j0 + wc + y * 16 + li;
            if (gj >= J.N) continue;
            if (COUT == 1)
              stc(static_cast<double*>(C), rbase + gj, (double)cre[x][y][r], (double)cim[x][y][r]);
            else
              stc(static_cast<float*>(C), rbase + gj, cre[x][y][r], cim[x][y][r]);
          }
        }
    }
    // FP64 output: let the row-table loads and stores finish here, once per job
    // (otherwise the compiler waits for every load in flight at each step)
    if (COUT == 1) sk_waitcnt<0>();
    zero();
    if (++cs < se) cend = jobs[cs].c1 - jobs[cs].c0;
  }
}

// Sums the partial tiles of each split tile in K order and stores the result.  Block
// (x, y): split tile sk_red[x], elements [1024 y, 1024 y + 1024) of the tile.
template <int COUT>
__global__ void __launch_bounds__(256) gemm_sk_reduce_kernel(const PsProb* __restrict__ probs,
                                                             const SkTile* __restrict__ tiles,
                                                             const int32_t* __restrict__ red,
                                                             const int64_t* __restrict__ rows,
                                                             const float* __restrict__ part, void* __restrict__ C,
                                                             const int32_t* __restrict__ skip) {
  if (skip && *skip) return;
  const SkTile t = tiles[red[blockIdx.x]];
  const PsProb P = probs[t.prob];
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    const int e = blockIdx.y * 1024 + q * 256 + threadIdx.x;
    if (e >= SK_BM * SK_BN) break;
    const int r = e / SK_BN, c = e - r * SK_BN;
    const int i = t.tm * SK_BM + r, j = t.tn * SK_BN + c;
    if (i >= P.M || j >= P.N) continue;
    float re = 0.f, im = 0.f;
    for (int k = 0; k < t.nseg; ++k) {
      const Cplx<float> v = ldc(part, (int64_t)(t.slot0 + k) * (SK_BM * SK_BN) + e);
      re += v.re;
      im += v.im;
    }
    const int64_t rb = COUT == 1 ? rows[P.rowmap + i] : P.c_off + (int64_t)i * P.ldc;
    if (COUT == 1)
      stc(static_cast<double*>(C), rb + j, (double)re, (double)im);
    else
      stc(static_cast<float*>(C), rb + j, re, im);
  }
}

hipError_t launch_gemm_sk(const PsStage& st, const __bf16* A, const __bf16* B, void* C, float* part,
                          hipStream_t s, const int32_t* skip, const std::function<void()>& between) {
  if (st.sk_grid == 0) return hipSuccess;
  if (st.sk_nslots > 0 && !part) return hipErrorInvalidValue;
  if (st.cout == 1) {
    hipLaunchKernelGGL(gemm_sk_kernel<1>, dim3(st.sk_grid), dim3(64 * SK_WAVES), 0, s, st.d_sk_jobs, st.d_sk_wg,
                       st.d_rows, A, B, C, part, skip);
  } else {
    hipLaunchKernelGGL(gemm_sk_kernel<0>, dim3(st.sk_grid), dim3(64 * SK_WAVES), 0, s, st.d_sk_jobs, st.d_sk_wg,
                       st.d_rows, A, B, C, part, skip);
  }
  if (between) between();
  if (!st.sk_red.empty()) {
    const dim3 grid((uint32_t)st.sk_red.size(), (SK_BM * SK_BN + 1023) / 1024);
    if (st.cout == 1)
      hipLaunchKernelGGL(gemm_sk_reduce_kernel<1>, grid, dim3(256), 0, s, st.d_probs, st.d_sk_tiles, st.d_sk_red,
                         st.d_rows, part, C, skip);
    else
      hipLaunchKernelGGL(gemm_sk_reduce_kernel<0>, grid, dim3(256), 0, s, st.d_probs, st.d_sk_tiles, st.d_sk_red,
                         st.d_rows, part, C, skip);
  }
  return hipGetLastError();
}

// ---------------------------------------------------------------------------------
// FP64 complex -> split planes.  One item: eight consecutive k values of one
// destination row (16 bytes per plane).  With trans = 0 the k values are consecutive
// source columns (one 128-byte read per item); with trans = 1 the destination row is a
// source column, and consecutive items walk consecutive columns, so every source row is
// read contiguously across the threads of a wave.
// ---------------------------------------------------------------------------------
__global__ void __launch_bounds__(256) split_kernel(const SplitJob* __restrict__ jobs, int32_t njobs,
                                                    int64_t nitems, const double* __restrict__ src,
                                                    __bf16* __restrict__ dst,
                                                    const int32_t* __restrict__ skip) {
  if (skip && *skip) return;
  const int64_t it = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (it >= nitems) return;
  int lo = 0, hi = njobs - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (jobs[mid].i0 <= it) lo = mid;
    else hi = mid - 1;
  }
  const SplitJob J = jobs[lo];
  const int64_t local = it - J.i0;
  const int ng = J.kp / 8;
  const int drows = J.trans ? J.cols : J.rows, kmax = J.trans ? J.rows : J.cols;
  int row, g;
  if (J.trans) {
    // blocks of 16 destination rows x 4 groups per wave, groups fastest: the four lanes
    // of a row write its 64 contiguous bytes per plane, and each of the wave's loads
    // reads 16 neighbouring source columns (256 bytes) for each of 4 k values
    const int nrb = (drows + 15) / 16;
    const int64_t blk = local >> 6;
    const int l = (int)(local & 63);
    row = (int)(blk % nrb) * 16 + (l >> 2);
    g = (int)(blk / nrb) * 4 + (l & 3);
    if (row >= drows || g >= ng) return;
  } else {
    row = (int)(local / ng);
    g = (int)(local % ng);
  }
  bf16x8 rh, rl, ih, il;
#pragma unroll
  for (int t = 0; t < 8; ++t) {
    const int k = 8 * g + t;
    float re = 0.f, im = 0.f;
    if (k < kmax) {
      const int64_t e = J.trans ? J.src + (int64_t)k * J.ld + row : J.src + (int64_t)row * J.ld + k;
      const Cplx<double> v = ldc(src, e);
      re = (float)v.re;
      im = (float)v.im;
    }
    const __bf16 a = (__bf16)re, b = (__bf16)im;
    rh[t] = a;
    rl[t] = (__bf16)(re - (float)a);
    ih[t] = b;
    il[t] = (__bf16)(im - (float)b);
  }
  __bf16* out = dst + J.dst + (int64_t)row * J.kp + 8 * g;
  *reinterpret_cast<bf16x8*>(out) = rh;
  *reinterpret_cast<bf16x8*>(out + J.pstride) = rl;
  *reinterpret_cast<bf16x8*>(out + 2 * (int64_t)J.pstride) = ih;
  *reinterpret_cast<bf16x8*>(out + 3 * (int64_t)J.pstride) = il;
}

hipError_t launch_split(const SplitJob* jobs, int32_t njobs, int64_t nitems, const double* src,
                        __bf16* dst, hipStream_t s, const int32_t* skip) {
  if (nitems == 0) return hipSuccess;
  const int64_t nb = (nitems + 255) / 256;
  if (nb > INT32_MAX) return hipErrorInvalidValue;
  hipLaunchKernelGGL(split_kernel, dim3((uint32_t)nb), dim3(256), 0, s, jobs, njobs, nitems, src, dst, skip);
  return hipGetLastError();
}

}  // namespace mrd
