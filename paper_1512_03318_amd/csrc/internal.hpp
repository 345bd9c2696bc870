// Internal declarations shared by the host planner (api.hip) and the kernels (kernels.hip).
#pragma once

#include <hip/hip_runtime.h>
#include <hip/hip_complex.h>

#include <cstdint>
#include <functional>
#include <string>
#include <vector>

namespace mrd {

// ---------------------------------------------------------------------------------
// Grouped complex GEMM descriptors.
//
// One problem computes C[M x N] = sum over its K-segments of op(A_seg) op(B_seg):
//   A(i, k): affine      a_off + i * lda + k          (A_T: a_off + k * lda + i)
//            row table   arow[a_rowmap + i] + a_off + k
//   B(k, j): affine      b_off + k * ldb + j          (B_T: b_off + j * ldb + k)
//   C(i, j): affine      c_off + i * ldc + j,  row table crow[c_rowmap + i] + j
// All offsets count complex elements.  A_CONJ conjugates A.  The K-segments of one
// problem are summed in order into one accumulator; C is overwritten.
enum GemmFlags : int32_t {
  G_A_T = 1,
  G_A_CONJ = 2,
  G_B_T = 4,
  G_A_ROWMAP = 8,
  G_C_ROWMAP = 16,
  G_C_F64 = 128,  // BF16x3: C is complex128, the FP32 results widened as they are stored
};

struct GemmSeg {
  int64_t a_off;
  int64_t b_off;
  int32_t lda, ldb;
  int32_t k;
  int32_t pad;
};

struct GemmProb {
  int64_t c_off;
  int32_t M, N;
  int32_t seg0, nseg;
  int32_t ldc;
  int32_t rowmap;  // start in the row table (A or C, by flags), -1 if none
  int32_t nks;     // DEEP: K-splits; split ks takes segments ks, ks + nks, ...
  int32_t slot0;   // DEEP with nks > 1: first partial-tile slot of this problem
};

// One output tile of one problem: rows [tm*TM, ...), cols [tn*TN, ...) with the tile
// size of the stage (gemm_tile_m / gemm_tile_n); ks = K-split index (DEEP).
struct GemmTile {
  int32_t prob;
  int32_t tm, tn;
  int32_t ks;
};

// Sparse mixing: dst[r, c] = sum_s coef_s * src_s[r, c] over a rows x cols sub-block.
// pstride > 0: the destination is split into four bf16 planes (re_hi, re_lo, im_hi,
// im_lo) pstride elements apart, dst and ld_dst counting bf16 elements of one plane.
struct MixTask {
  int64_t dst;
  int32_t ld_dst, rows, cols;
  int32_t src0, nsrc;
  int32_t pstride;
};
struct MixSrc {
  int64_t off;
  int32_t ld;
  int32_t pad;
  double re, im;
};

// Host-side task table of one contraction stage, with its device copy.
struct GemmStage {
  int32_t flags = 0;
  bool real = false;  // real operands and result (eq. rot formulation)
  bool deep = false;  // one workgroup per tile, K-segments split over its 4 waves
  std::vector<GemmSeg> segs;
  std::vector<GemmProb> probs;
  std::vector<GemmTile> tiles;
  std::vector<int64_t> rows;  // row table
  // Output tile of one workgroup and the K split.  FP32/FP64 kernels: 64 x 64 tiles,
  // or DEEP 32 x 32 tiles whose four waves share the K range; BF16x3 kernel: 64 x 64,
  // 128 x 64, or 128 x 32 with split.  With split, a problem's K range is divided over
  // up to 8 workgroups, at least split_min chunks of kc each.
  int32_t tile_m = 64, tile_n = 64;
  bool split = false;
  int32_t kc = 32, split_min = 4;
  std::vector<GemmTile> red_tiles;  // split: tiles whose K-split partials are summed
  int64_t nslots = 0;               // split: partial tiles (tile_m x tile_n each)
  int64_t slot_elems() const { return (int64_t)tile_m * tile_n; }
  double flops = 0.0;         // algorithmic: 8 * M * N * K per problem (+ mixing MACs)
  // device
  GemmSeg* d_segs = nullptr;
  GemmProb* d_probs = nullptr;
  GemmTile* d_tiles = nullptr;
  int64_t* d_rows = nullptr;
  GemmTile* d_red_tiles = nullptr;
};

// Slab form of a mixing stage.  All sources of a task lie in one slab: a set of
// equally shaped source blocks (rows x cols).  A workgroup stages rows [r0, r0 + nr)
// and columns [col0, col0 + ncol) of every block of its slab in LDS once, then writes
// that part of every task of the slab, so each source element is read from memory once.
struct SlabWG {
  int32_t blk0, nblk;    // the slab's blocks
  int32_t task0, ntask;  // the slab's tasks
  int32_t r0, nr, col0, ncol;
};
struct SlabBlk {
  int64_t off;  // source element (0, 0) of the block
  int32_t ld, pad;
};
struct SlabTask {
  int64_t dst;  // destination element (0, 0) of the task
  int32_t ld_dst;
  int32_t c0, nc;  // coefficients [c0, c0 + nc)
  int32_t pstride;  // as MixTask::pstride
};
struct SlabCoef {
  int32_t blk, pad;  // block index within the slab
  double re, im;
};

struct MixStage {
  bool real = false;            // real data and coefficients (eq. rot form)
  std::vector<MixTask> tasks;   // in launch order
  std::vector<MixSrc> srcs;
  double flops = 0.0;  // 8 flops per complex multiply-add
  MixTask* d_tasks = nullptr;
  MixSrc* d_srcs = nullptr;
  // slab form (used by launch_mix when present)
  std::vector<SlabWG> wgs;
  std::vector<SlabBlk> blks;
  std::vector<SlabTask> stasks;
  std::vector<SlabCoef> coefs;
  int32_t lds_bytes = 0;  // largest LDS footprint of one workgroup
  int32_t slab_eb = 0;    // bytes per element the slab form was sized for (one real value
                          // per element for a real plan); a launch in another precision
                          // uses the task form
  SlabWG* d_wgs = nullptr;
  SlabBlk* d_blks = nullptr;
  SlabTask* d_stasks = nullptr;
  SlabCoef* d_coefs = nullptr;
};

// Kernel launchers (kernels.hip).  T = double or float (complex interleaved).
// part: scratch of st.nslots * st.slot_elems() complex elements (stages with K splits).
// skip (may be null): the kernels return at once when *skip != 0 (a stopped Lanczos).
// between (may be empty) runs on the host after the main kernel is enqueued and before
// the K-split reduction (used to record a profiling event).
template <typename T>
hipError_t launch_gemm(const GemmStage& st, const T* A, const T* B, T* C, T* part, hipStream_t s,
                       const int32_t* skip = nullptr,
                       const std::function<void()>& between = std::function<void()>());
// BF16x3 form of launch_gemm on FP32 operands (gemm_bf16x3.hip); same tables and tiles.
hipError_t launch_gemm_bf16x3(const GemmStage& st, const float* A, const float* B, float* C,
                              float* part, hipStream_t s, const int32_t* skip = nullptr,
                              const std::function<void()>& between = std::function<void()>());
template <typename T>
hipError_t launch_mix(const MixStage& st, const T* src, T* dst, hipStream_t s,
                      const int32_t* skip = nullptr);
// Mixing whose output is split into bf16 planes (tasks with pstride > 0, slab form).
hipError_t launch_mix_split(const MixStage& st, const float* src, __bf16* dst, hipStream_t s,
                            const int32_t* skip = nullptr);

// ---------------------------------------------------------------------------------
// Pre-split operands (BF16x3).  A complex matrix of R rows and K columns is stored as
// four bf16 planes re_hi, re_lo, im_hi, im_lo (x = hi + lo, hi = bf16(x), lo =
// bf16(x - hi), both round to nearest even, x the FP32 value), each R x kp with k
// contiguous, kp = K rounded up to a multiple of 8, the padding zero.
// One problem: C[M x N] = A (M x kp planes) . B^T (B: N x kp planes), in chunks of 32
// along k (K-split: split ks takes chunks ks, ks + nks, ...).  C is complex FP32 at
// c_off + i * ldc + j (COUT 0) or complex FP64 at row-table offsets (COUT 1).
struct PsProb {
  int64_t a_off, b_off;  // bf16 elements: plane 0, row 0 of A and of B
  int64_t a_ps, b_ps;    // plane strides (bf16 elements)
  int64_t c_off;
  int32_t M, N, kp;
  int32_t ldc;
  int32_t rowmap;  // start in the row table (COUT 1), -1 if none
  int32_t nks, slot0;
  int32_t pad;
};
// Stream-K schedule of a pre-split stage for a persistent grid: the K chunks of all
// output tiles form one sequence (tile after tile, chunks in K order), cut into equal
// runs, one per workgroup.  A run is a list of segments (chunks [c0, c1) of one tile); a
// tile that lies in one segment is stored directly (slot -1), otherwise each of its
// segments writes a partial tile to its own slot (slot0 + segment index, in K order) and
// a reduction sums them in that order.
struct SkTile {
  int32_t prob, tm, tn, nch;  // nch: chunks of 32 k values (kp / 32)
  int32_t slot0, nseg;
};
struct SkSeg {
  int32_t tile, c0, c1, slot;
};
// One segment as the kernel reads it: everything its loads and its store need, in one
// record (no dependent table lookups in the chunk loop).
struct SkJob {
  int64_t a_off, b_off, a_ps, b_ps, c_off;  // as PsProb
  int32_t M, N, kp, ldc, rowmap;
  int32_t i0, j0;   // first row and column of the tile
  int32_t c0, c1;   // chunks
  int32_t slot;     // partial slot, or -1: store the tile
};
struct PsStage {
  int32_t cout = 0;  // 0: FP32 affine C; 1: FP64 C through the row table
  int32_t tile_m = 128, tile_n = 64;
  bool split = false;
  int32_t split_min = 12;  // chunks of 32 per K split at least (at most 8 splits)
  std::vector<PsProb> probs;
  std::vector<GemmTile> tiles;
  std::vector<int64_t> rows;
  std::vector<GemmTile> red_tiles;
  int64_t nslots = 0;
  double flops = 0.0;
  int64_t slot_elems() const { return (int64_t)tile_m * tile_n; }
  PsProb* d_probs = nullptr;
  GemmTile* d_tiles = nullptr;
  int64_t* d_rows = nullptr;
  GemmTile* d_red_tiles = nullptr;
  // stream-K schedule (sk_schedule; tiles of SK_BM x SK_BN)
  int32_t sk_grid = 0;
  std::vector<SkTile> sk_tiles;
  std::vector<SkSeg> sk_segs;
  std::vector<SkJob> sk_jobs;   // per segment (same order)
  std::vector<int32_t> sk_wg;   // segments of workgroup g: [sk_wg[g], sk_wg[g + 1])
  std::vector<int32_t> sk_red;  // tiles with more than one segment
  int64_t sk_nslots = 0;
  SkTile* d_sk_tiles = nullptr;
  SkSeg* d_sk_segs = nullptr;
  SkJob* d_sk_jobs = nullptr;
  int32_t* d_sk_wg = nullptr;
  int32_t* d_sk_red = nullptr;
};
// Stream-K tile of the pre-split kernels (rows x columns) and chunk width.
constexpr int SK_BM = 128, SK_BN = 64, SK_KC = 32;
void sk_schedule(PsStage& st, int grid);  // needs every problem's kp a multiple of SK_KC
hipError_t launch_gemm_sk(const PsStage& st, const __bf16* A, const __bf16* B, void* C, float* part,
                          hipStream_t s, const int32_t* skip = nullptr,
                          const std::function<void()>& between = std::function<void()>());
hipError_t launch_gemm_ps(const PsStage& st, const __bf16* A, const __bf16* B, void* C, float* part,
                          hipStream_t s, const int32_t* skip = nullptr,
                          const std::function<void()>& between = std::function<void()>());

// Conversion of complex FP64 matrices into split planes.  Job: the source block is rows
// x cols at src + r * ld + c (complex elements); the destination rows are the source
// rows (trans 0) or the source columns (trans 1), each kp bf16 long (k = the other
// index, zero beyond it), planes pstride apart.  i0: first flat item (one item = eight
// k values of one destination row) of this job.
struct SplitJob {
  int64_t src, dst;
  int32_t ld, rows, cols, kp;
  int32_t trans, pstride;
  int64_t i0;
};
int64_t split_layout(std::vector<SplitJob>& jobs);  // fills i0, returns the total items
hipError_t launch_split(const SplitJob* jobs, int32_t njobs, int64_t nitems, const double* src,
                        __bf16* dst, hipStream_t s, const int32_t* skip = nullptr);

// c: n complex128 (interleaved); r: n doubles.  take: r = Re c; put: c = r + 0i.
hipError_t launch_re_take(const double* c, double* r, int64_t n, hipStream_t s);
hipError_t launch_re_put(const double* r, double* c, int64_t n, hipStream_t s);
hipError_t launch_cast_d2f(const double* in, float* out, int64_t n_real, hipStream_t s,
                           const int32_t* skip = nullptr);
hipError_t launch_cast_f2d(const float* in, double* out, int64_t n_real, hipStream_t s,
                           const int32_t* skip = nullptr);

// Device-resident Lanczos state (lanczos.hip), one per instance.
constexpr int LZ_MAX = 64;
struct LzState {
  double alpha[LZ_MAX + 1];
  double beta[LZ_MAX + 1];
  double h1[2 * (LZ_MAX + 1) + 2];  // <v_i, w>
  double h2[2 * (LZ_MAX + 1) + 2];  // second projection, then |w1|^2
  double y[LZ_MAX + 1];             // lowest eigenvector of T_k
  double rq[2];                     // Rayleigh quotient numerator / denominator
  double scal0;                     // |theta_0|^2
  double inv_beta, tnorm, tol, energy;
  int32_t iter, k, stop, max_iter, bad, pad;
  uint64_t t0, t1;                  // device wall clock at start and when the solve stopped
};

// One Lanczos instance of a (possibly batched) launch.  Every Lanczos kernel runs over
// all instances of its table at once: a flat grid whose blocks are assigned to
// instances by the first-block offsets c0 / g0 (found by binary search).
struct LzInst {
  double* V;       // Krylov basis, vector j at element j ld (complex FP64, or FP32 pairs
                   // when the launch grid says vf32)
  double* w;       // H v_j
  double* vcur;    // v_j (matvec input of every step)
  double* part;    // projection partials: nb x (2 max_iter + 1)
  double* pnorm;   // norm / Rayleigh-quotient partials: 2 nb
  double* x;       // caller's start vector in, Ritz vector out
  LzState* st;
  int64_t ld, n;   // n complex elements
  int32_t nb;      // chunk blocks (1024 elements)
  int32_t c0, g0;  // first chunk / 256-element block of this instance
  float* tin;      // or null: FP32 copy of v_j written with it (input of an FP32 /
                   // BF16x3 matvec, which then needs no cast of its own)
  // Real instances (eq. rot): the vectors hold 2 n - 1 or 2 n real values read as n
  // complex elements; xn is the number of doubles in the caller's x (2 n for a complex
  // instance), and the projection coefficients are kept real (their imaginary parts,
  // which pair unrelated components, are set to zero), so every update is the real one.
  int64_t xn;
  int32_t real;
};
// Launch shape of an instance table (host side).
struct LzGrid {
  int32_t nins = 0, nchunk = 0, n256 = 0;
  int32_t max_iter = 0;  // capacity: Krylov vectors - 1 of every instance
  // every instance keeps its Krylov basis in complex FP32 (V holds float pairs, same
  // element stride ld): plans whose matvec reads an FP32 copy of v_j
  bool vf32 = false;
};
struct LzResult {
  double energy;
  int32_t k, bad;
  uint64_t t0, t1;
};
// Fills nb, pnorm and the block offsets of I (V, w, vcur, part, x, st, ld, n set by
// the caller; part must hold nb (2 max_iter + 1) + 2 nb doubles, see lz_part_doubles).
LzGrid lz_layout(std::vector<LzInst>& I, int32_t max_iter);
int64_t lz_part_doubles(int64_t n, int32_t max_iter);
// Resets the states for a solve of at most max_iter (<= g.max_iter) steps.
hipError_t lz_launch_init(const LzInst* I, const LzGrid& g, int32_t max_iter, double tol,
                          hipStream_t s);
hipError_t lz_launch_start(const LzInst* I, const LzGrid& g, hipStream_t s);
// nv_bound: an upper bound of the Krylov vector count at this step (step index + 1),
// or 0 when unknown (a step captured once and replayed)
hipError_t lz_launch_step_tail(const LzInst* I, const LzGrid& g, int32_t nv_bound, hipStream_t s);
// Lowest Ritz pair; the Ritz vector goes to x and to vcur.
hipError_t lz_launch_finish(const LzInst* I, const LzGrid& g, hipStream_t s);
// energy = <vcur, w> / <vcur, vcur> (w = FP64 H vcur computed by the caller).
hipError_t lz_launch_rq(const LzInst* I, const LzGrid& g, hipStream_t s);
hipError_t lz_launch_results(const LzInst* I, const LzGrid& g, LzResult* out, hipStream_t s);

// Batched casts between FP64 and FP32 storage (kernels.hip): job i converts n reals.
struct CastJob {
  const void* src;
  void* dst;
  int64_t n;
  int32_t c0, pad;  // first block of this job
};
int32_t cast_layout(std::vector<CastJob>& jobs);  // fills c0, returns the total blocks
hipError_t launch_cast_batch(bool d2f, const CastJob* jobs, int32_t njobs, int32_t nblocks,
                             hipStream_t s);

// Thread-local message returned by dm_last_error().
void set_last_error(const std::string& msg);

}  // namespace mrd
