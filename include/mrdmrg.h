/*
 * mrdmrg -- MI355X (gfx950) hot path of mixed real/momentum-space cylinder DMRG.
 *
 * Motruk, Zaletel, Mong, Pollmann, "Density matrix renormalization group on a
 * cylinder in mixed real and momentum space", arXiv:1512.03318.
 *
 * The paper's method makes the ring momentum k an onsite Z_Ly charge (Sec. II: the
 * rotation T_y = prod exp(i k n_{x,k}) factorises over orbitals), so every DMRG tensor
 * is block sparse in (N, k mod Ly) (Sec. III B: this extra block structure is what
 * cuts time and memory).  This library runs the inner loop of the (i)DMRG sweep that
 * the paper relies on but does not restate (Sec. I, III A):
 *
 *   H_eff theta [a', s1', s2', c'] =
 *     sum L[a', w, a] W1[w, s1', s1, w'] W2[w', s2', s2, w''] R[c', w'', c] theta[a, s1, s2, c]
 *   L'[b', w', b] = sum conj(A[a', s', b']) L[a', w, a] W[w, s', s, w'] A[a, s, b]
 *   R'[b', w, b]  = sum conj(B[b', s', c']) W[w, s', s, w'] R[c', w', c] B[b, s, c]
 *
 * and the Lanczos ground-state solve around the first contraction.  W is the MPO of
 * eq. MPO (matrix of operators per orbital, built from the finite-state machine of
 * Sec. IV); its bond states carry the charge the operator string has placed so far.
 *
 * ---------------------------------------------------------------------------------
 * Conventions (all of them are checked; violations return an error code)
 *
 * Charges.  A charge is (n, k) with 0 <= k < ly; addition is (n1+n2, (k1+k2) mod ly).
 *   ly = 1 is a plain U(1) problem (the real-space basis).  A virtual bond carries the
 *   total charge left of it.  Local states |0>, |1> of an orbital carry qs[0], qs[1].
 *   Charge rules: A[a,s,b]: q(b) = q(a) + q(s).  theta: q(c) = q(a) + q(s1) + q(s2).
 *   W[w,s',s,w']: q(w') = q(w) + q(s') - q(s).  L[a',w,a]: q(a') = q(a) + q(w).
 *   R[c',w,c]: q(c') = q(c) + q(w).
 *
 * Bonds.  dm_bond lists sectors strictly increasing in (n, k) with positive dims.
 *
 * Data.  Every tensor passed to or returned from a compute call is device memory
 *   holding complex128 values, interleaved (re, im), in the canonical layout below.
 *   The caller owns all tensors; compute calls never keep a pointer to them after
 *   returning, except where stated.  dm_layout() returns every block's offset so a
 *   caller can pack and unpack data.  Layouts ("panel" = one row-major matrix):
 *
 *   DM_LAYOUT_SITE  (A or B, legs a, s, b): one panel per left sector a, in sector
 *       order; rows m_a; columns the concatenation over s = 0, 1 (when the sector
 *       b = a + q(s) exists) of m_b columns.  Block (a, s, b) has ld = panel width.
 *   DM_LAYOUT_THETA (legs a, s1, s2, c): one panel per left sector a; columns the
 *       concatenation over (s1, s2) = (0,0), (0,1), (1,0), (1,1) (when c exists).
 *   DM_LAYOUT_ENV_L (L[a', w, a], bra and ket on the same bond): one panel per ket
 *       sector a; columns m_a; rows the concatenation over MPO states w = 0..D-1 (when
 *       a' = a + q(w) exists) of m_a' rows.
 *   DM_LAYOUT_ENV_R (R[c', w, c]): one panel per bra sector c'; rows m_c'; columns the
 *       concatenation over w = 0..D-1 (when c = c' - q(w) exists) of m_c columns.
 *   Panels follow each other without padding.
 *
 * MPO site tensors are small host arrays: W[w][s'][s][w'] complex128 interleaved.
 *
 * Errors.  Every int-returning call returns DM_OK (0) or a negative DM_ERR_* code and
 *   sets a thread-local message readable with dm_last_error().  No C++ exception
 *   crosses this boundary.  GPU work is enqueued on the given stream; only the Lanczos
 *   calls synchronise (they return host scalars).  Library scratch is released in
 *   stream order (reused once the stream has passed the work that used it).
 *
 * Threads.  The library's device and pinned-host pools are locked: distinct plans and
 *   batches may be created and used from different host threads at once (each on its
 *   own stream).  Calls on one plan, or on a batch and the plans it holds, must not
 *   overlap.  Plan creation and the right environment update run part of their host
 *   planning on a helper thread that they join before returning.
 * ---------------------------------------------------------------------------------
 */
#ifndef MRDMRG_H
#define MRDMRG_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct ihipStream_t* dm_stream; /* hipStream_t; NULL is the default stream */

#define DM_OK 0
#define DM_ERR_ARG (-1)       /* null pointer, negative size, bad enum           */
#define DM_ERR_CHARGE (-2)    /* a block violates its leg-charge rule            */
#define DM_ERR_DIM (-3)       /* bonds of two tensors disagree                   */
#define DM_ERR_LAYOUT (-4)    /* tensor does not match the plan                  */
#define DM_ERR_DTYPE (-5)     /* unsupported precision                           */
#define DM_ERR_ALLOC (-6)     /* device or host allocation failed                */
#define DM_ERR_HIP (-7)       /* a HIP runtime call failed                       */
#define DM_ERR_NONFINITE (-8) /* Lanczos produced a NaN or Inf                   */

/* Arithmetic of the block GEMMs.  Inputs and outputs stay complex128; Lanczos
 * scalars, reorthogonalisation and the tridiagonal solve are FP64 in every mode.  In
 * DM_FP32 and DM_BF16X3 the Krylov basis is stored in complex FP32: each Lanczos vector
 * is rounded once as it is formed (the FP32 value is what the matvec reads) and every
 * product and sum over the basis is FP64. */
#define DM_FP64 0
#define DM_FP32 1
#define DM_BF16X3 2 /* hi/lo bfloat16 split of FP32 operands, FP32 accumulation */
/* OR'ed into DM_FP64, DM_FP32 or DM_BF16X3 (dm_heff_plan_create, env_update_left / _right and the
 * allocation-free variant): real operands, the formulation of eq. rot (Sec. IV D) in
 * which the mixed-basis MPO (dm_mpo_hofstadter basis 2), theta and the environments are
 * real.  Every tensor argument is then an array of float64 values in the same block
 * layout as its complex128 form (dm_layout: element counts and offsets are unchanged,
 * each element is one double); the MPO site tensors are still passed as complex128 and
 * must have zero imaginary parts (DM_ERR_ARG otherwise).  A real plan's flop counts
 * (dm_heff_info) are 2 per real multiply-add.  Real plans are not batched; the sweeps
 * and iDMRG use them when their precision carries DM_REAL. */
#define DM_REAL 16

typedef struct {
  int32_t n;
  int32_t k;
} dm_charge;

typedef struct {
  int32_t nsec;
  const dm_charge* q; /* [nsec] */
  const int32_t* dim; /* [nsec] */
} dm_bond;

typedef struct {
  int32_t dl, dr;      /* MPO bond dimensions left / right of the orbital        */
  const dm_charge* ql; /* [dl] charge of each left MPO state                     */
  const dm_charge* qr; /* [dr]                                                   */
  dm_charge qs[2];     /* charges of |0> and |1>                                 */
  const double* w;     /* host [dl][2][2][dr] complex128 interleaved, W[w,s',s,w'] */
} dm_mpo_site;

#define DM_LAYOUT_SITE 0
#define DM_LAYOUT_THETA 1
#define DM_LAYOUT_ENV_L 2
#define DM_LAYOUT_ENV_R 3

typedef struct {
  int32_t kind;         /* DM_LAYOUT_*                                              */
  int32_t ly;           /* momentum modulus (>= 1)                                  */
  const dm_bond* x;     /* SITE, THETA: left bond; ENV_L, ENV_R: the bond         */
  const dm_bond* y;     /* SITE, THETA: right bond; unused for ENV_*                */
  int32_t nw;           /* ENV_*: number of MPO states                             */
  const dm_charge* qw;  /* ENV_*: [nw] MPO state charges                          */
  dm_charge qs1[2];     /* SITE: local charges; THETA: first orbital              */
  dm_charge qs2[2];     /* THETA: second orbital                                  */
} dm_layout_desc;

typedef struct {
  int32_t idx[3]; /* SITE (a, s, b); THETA (a, s1*2+s2, c); ENV_L (a', w, a); ENV_R (c', w, c) */
  int32_t rows, cols;
  int64_t off; /* element offset of the block's (0, 0) entry                        */
  int64_t ld;  /* elements between consecutive rows                                 */
} dm_block;

/* Canonical layout of a tensor (see above).  Writes the block count and the total
 * number of complex elements; fills blocks[0..nblocks) when blocks != NULL (the
 * caller provides room for *nblocks entries: call once with NULL to size it). */
int dm_layout(const dm_layout_desc* d, int64_t* nblocks, int64_t* nelem, dm_block* blocks);

/* ---- Two-site effective Hamiltonian -------------------------------------------
 * A plan binds the environments L (bond a, MPO states of w1's left leg) and R (bond c,
 * MPO states of w2's right leg) and the two MPO site tensors of the window.  It
 * precomputes the charge-matched block task table (which L block meets which theta
 * block, which MPO entries mix which intermediate blocks) and copies L and R into
 * plan-owned device buffers in the plan's precision (plus FP64 copies for the final
 * Rayleigh quotient in DM_FP32 / DM_BF16X3).  The copies are stream-ordered on
 * `stream` (the call does not wait for them): L and R may be freed or overwritten by
 * later work on the same stream (e.g. a stream-ordered allocator), or after that stream
 * has been synchronised.  The plan owns its device scratch.  Several plans may run
 * concurrently on different streams; one plan must not be used by two streams at the
 * same time. */
typedef struct dm_heff_plan dm_heff_plan;

int dm_heff_plan_create(int32_t ly, const dm_bond* a, const dm_bond* c,
                        const dm_mpo_site* w1, const dm_mpo_site* w2,
                        const void* L, const void* R, int32_t prec,
                        dm_stream stream, dm_heff_plan** out);
/* Waits for the plan's creation work, then hands its device buffers back to the
 * library's pool for reuse: work of the plan queued by heff_apply must have completed
 * (synchronise its stream first; lanczos_ground returns synchronised). */
void dm_heff_plan_destroy(dm_heff_plan* p);

/* Number of complex elements of theta for this plan, and algorithmic flop counts of
 * one matvec (8 real flops per complex multiply-add): flops[0] = L.theta block GEMMs,
 * flops[1] = MPO mixing, flops[2] = (.).R block GEMMs. */
int dm_heff_info(const dm_heff_plan* p, int64_t* theta_elems, double flops[3]);

/* Complex elements of the plan's operands and intermediates: sizes[0] = L, sizes[1] = R,
 * sizes[2] = theta, sizes[3] = X (L.theta panels), sizes[4] = Z (mixed panels).  The
 * algorithmic bytes of a stage follow from these (each element read or written once). */
int dm_heff_sizes(const dm_heff_plan* p, int64_t sizes[5]);

/* Device-time profile of the matvec stages.  With enable = k > 0, every k-th matvec of
 * the plan (heff_apply and the ones inside lanczos_ground, counted from this call)
 * records HIP events on its stream around each kernel (each recorded event costs the
 * stream a few microseconds, so k > 1 keeps the instrumented run close to an
 * uninstrumented one); dm_heff_profile_read synchronises and returns the accumulated
 * milliseconds of 0: the L.theta GEMM kernel, 1: the MPO mixing kernel, 2: the (.).R
 * GEMM kernel, 3: the reduction of its K-split partial tiles, and the number of
 * matvecs recorded.  enable = 0 stops recording and clears the totals; enable < 0 is
 * DM_ERR_ARG.  Profiling keeps lanczos_ground on plain stream launches (no graph
 * replay). */
int dm_heff_profile(dm_heff_plan* p, int32_t enable);
int dm_heff_profile_read(dm_heff_plan* p, double ms[4], int64_t* matvecs);

/* theta_out = H_eff theta.  Both are device complex128 in the THETA layout of (a, c,
 * w1.qs, w2.qs), 16-byte aligned (DM_ERR_ARG otherwise); they must not overlap.
 * Asynchronous on `stream`. */
int heff_apply(dm_heff_plan* p, const void* theta, void* theta_out, dm_stream stream);

/* Lanczos ground state of H_eff (textbook Lanczos, classical Gram-Schmidt against all
 * previous vectors applied twice, FP64 on the device; lowest eigenpair of the
 * tridiagonal matrix by bisection and inverse iteration on the device).
 * theta_inout: start vector in (need not be normalised), normalised Ritz vector out;
 * device complex128, 16-byte aligned (DM_ERR_ARG otherwise).  Stops after max_iter
 * (1..64) matvecs or when beta_j <= tol * |T|.  In DM_FP32 / DM_BF16X3 the energy is the
 * FP64 Rayleigh quotient <theta|H_eff|theta> of the Ritz vector (one extra FP64
 * matvec); in DM_FP64 it is the Ritz value.  Synchronises. */
int lanczos_ground(dm_heff_plan* p, void* theta_inout, int32_t max_iter, double tol,
                   double* energy, int32_t* iters, dm_stream stream);

/* ---- Environment updates ---------------------------------------------------------
 * L_out (bond b, MPO states w.qr) from L (bond a, states w.ql) and the left-canonical
 * site tensor A (SITE layout of a, b, w.qs).  R_out (bond b, states w.ql) from R
 * (bond c, states w.qr) and the right-canonical B (SITE layout of b, c, w.qs).
 * Outputs are overwritten.  Asynchronous on `stream`: the inputs must stay valid and
 * the output is complete only once the work queued there has run (same rule as for
 * dm_heff_plan_create).  Scratch comes from the library's caching pool and is reused
 * only after the stream has passed this update. */
int env_update_left(int32_t ly, const dm_bond* a, const dm_bond* b, const dm_mpo_site* w,
                    const void* L, const void* A, void* L_out, int32_t prec, dm_stream stream);
int env_update_right(int32_t ly, const dm_bond* b, const dm_bond* c, const dm_mpo_site* w,
                     const void* R, const void* B, void* R_out, int32_t prec, dm_stream stream);

/* env_update_left for callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): same arguments, kernels
 * and results as env_update_left, but the task tables and intermediates live in one fixed
 * device region of 64 MiB that the library holds per device from load until the process
 * ends, instead of the caching pool.  The call makes no device or pinned allocation
 * (tables go up from pageable host memory).  An update whose scratch does not fit
 * (tables + the L.A and mixed intermediates, plus FP32 copies of L, A and L_out in
 * DM_FP32 / DM_BF16X3) returns DM_ERR_ALLOC before queueing any work.  All calls on one
 * device share the region: two calls whose queued work overlaps in time (different
 * streams, or different host threads) race, so callers serialise them, e.g. on one
 * stream.  Asynchronous on `stream` like env_update_left. */
int env_update_left_noalloc(int32_t ly, const dm_bond* a, const dm_bond* b, const dm_mpo_site* w,
                            const void* L, const void* A, void* L_out, int32_t prec,
                            dm_stream stream);

/* Algorithmic flops of one environment update, 8 per complex multiply-add, counted on
 * the same task tables the update runs.  left = 1: env_update_left from bond x (= a) to
 * bond y (= b); left = 0: env_update_right from bond y (= c) to bond x (= b). */
int dm_env_flops(int32_t left, int32_t ly, const dm_bond* x, const dm_bond* y,
                 const dm_mpo_site* w, double* flops);

/* ---- Many independent problems -------------------------------------------------
 * A batch merges the task tables of n plans (same precision) so that every phase of
 * one Lanczos step runs as one launch over all instances (one per problem bucket for
 * the block GEMMs).  At the first solve the GEMM problems of all instances are grouped
 * into buckets by output shape (rows <= 64 / > 64, columns <= 32 / <= 64 / > 64) and each
 * bucket is timed with every tile shape the kernels provide; the fastest is kept (set
 * MRDMRG_TUNE=0 to keep the plans' own shapes).  Chosen shapes are remembered in a text
 * file keyed by (GPU architecture, precision, stage, bucket, log2 of the bucket's
 * GFLOP): later batches of the same kind read them instead of timing.  The file is
 * $MRDMRG_TUNE_CACHE, else $XDG_CACHE_HOME/mrdmrg/tile_shapes.txt, else
 * ~/.cache/mrdmrg/tile_shapes.txt; MRDMRG_TUNE_CACHE=0 disables it.  Tiles are issued
 * longest first.  With
 * MRDMRG_GRAPH=1 each Lanczos iteration of the whole batch is one HIP graph replay.
 * Plans must outlive the batch. */
typedef struct dm_batch dm_batch;
int dm_batch_create(int32_t n, dm_heff_plan* const* plans, dm_stream stream, dm_batch** out);
void dm_batch_destroy(dm_batch* b);
/* The tile shape chosen per bucket, as text (empty before the first solve).  Writes at
 * most len bytes including the terminating zero; returns the full length. */
int64_t dm_batch_info(const dm_batch* b, char* buf, int64_t len);
/* thetas[i]: device start vector / Ritz vector of instance i (16-byte aligned, as for
 * lanczos_ground).  energies, iters: host
 * arrays of n.  Same algorithm and stopping rule as lanczos_ground per instance (the
 * tuned tile shapes may sum in another order: results agree to rounding).
 * done_us (may be NULL): host array of n, microseconds from launch until instance i
 * stopped, read from the device clock.  Synchronises. */
int lanczos_ground_batched(dm_batch* b, void* const* thetas, int32_t max_iter, double tol,
                           double* energies, int32_t* iters, double* done_us, dm_stream stream);

/* ---- Two-site split (block SVD truncation) ------------------------------------------
 * theta (device complex128, THETA layout of a, c, qs1, qs2) is a block-diagonal matrix
 * over the charge of the middle bond, q(b) = q(a) + q(s1) (the Schmidt states carry
 * (N, k), Sec. III C): M_b[(a, s1), (s2, c)].  Each M_b is factorised U S V^H in FP64 on
 * the device (one-sided Jacobi, one workgroup per sector).  Kept: the chi largest
 * singular values over all sectors (ties broken by sector charge, then rank within the
 * sector), none <= cutoff, renormalised to a unit sum of squares.  The new bond b lists
 * the sectors that keep at least one value, with that count as their dimension.
 * move_right != 0: left = U (left-canonical A, SITE layout of a, b, qs1) and right =
 * S V^H (SITE layout of b, c, qs2); move_right = 0: left = U S, right = V^H
 * (right-canonical B).  Synchronises (the kept values are chosen on the host).  The
 * split owns the new bond and both device tensors until dm_split_destroy, which
 * requires the work that reads them to have completed.  DM_ERR_NONFINITE when no value
 * exceeds the cutoff or a value is not finite. */
typedef struct dm_split dm_split;
int dm_theta_split(int32_t ly, const dm_bond* a, const dm_bond* c, const dm_charge qs1[2],
                   const dm_charge qs2[2], const void* theta, int32_t chi, double cutoff,
                   int32_t move_right, dm_stream stream, dm_split** out);
/* The new bond: *nsec, then (when q and dim are not NULL, room for *nsec each) its
 * charges and dimensions. */
int dm_split_bond(const dm_split* sp, int32_t* nsec, dm_charge* q, int32_t* dim);
/* Device pointers and element counts of the two site tensors (valid until destroyed). */
int dm_split_tensors(const dm_split* sp, const void** left, int64_t* nleft, const void** right,
                     int64_t* nright);
/* Kept Schmidt values (normalised), sector by sector in bond order, descending within a
 * sector (sum of the bond's dimensions values), and the discarded weight
 * 1 - sum(kept^2) / sum(all^2).  Either pointer may be NULL. */
int dm_split_schmidt(const dm_split* sp, double* values, double* discarded);
/* Copies the two site tensors into caller buffers (nleft / nright complex128 elements),
 * stream-ordered. */
int dm_split_copy(const dm_split* sp, void* left, void* right, dm_stream stream);
void dm_split_destroy(dm_split* sp);

/* ---- Finite two-site DMRG on the device ------------------------------------------------
 * An MPS of n >= 2 orbitals held by the library: bonds[0..n] (bond 0 the vacuum charge,
 * bond n the total charge), local charges qs[2 i], qs[2 i + 1] of orbital i, and site
 * tensors (device complex128, SITE layout of bonds[i], bonds[i+1], qs of i), copied.
 * Synchronises. */
typedef struct dm_mps dm_mps;
int dm_mps_create(int32_t ly, int32_t n, const dm_bond* bonds, const dm_charge* qs,
                  const void* const* tensors, dm_stream stream, dm_mps** out);
void dm_mps_destroy(dm_mps* m);
/* Bond i (0..n): *nsec, then charges and dimensions as dm_split_bond. */
int dm_mps_bond(const dm_mps* m, int32_t i, int32_t* nsec, dm_charge* q, int32_t* dim);
/* Device pointer and element count of site tensor i (valid until the next sweep). */
int dm_mps_tensor(const dm_mps* m, int32_t i, const void** data, int64_t* nelem);
/* Copies site tensor i into a caller buffer of nelem complex128 elements, stream-ordered. */
int dm_mps_copy(const dm_mps* m, int32_t i, void* dst, dm_stream stream);
/* Schmidt values of bond i from its last split (layout as dm_split_schmidt): *count,
 * then the values when `values` is not NULL. */
int dm_mps_schmidt(const dm_mps* m, int32_t i, double* values, int64_t* count);
/* Two-site DMRG sweeps (the paper's (i)DMRG relies on them, Sec. I, III A): the MPS must
 * be right-canonical from orbital 1 on.  One sweep moves right over bonds (0,1) ..
 * (n-2, n-1) and back left; at every bond the two-site tensor is the start vector of
 * lanczos_ground (max_iter steps, the plan in precision prec), its Ritz vector is split by
 * dm_theta_split (chi, cutoff; left-canonical behind a right move, right-canonical behind
 * a left move) and the environment behind the move is updated (FP64).  w: the n MPO
 * site tensors (w[0] with one left state, w[n-1] with one right state, the boundary
 * states of eq. MPO).  energies[s]: the energy of the last bond update of sweep s.
 * prec may carry DM_REAL: the MPO (eq. rot form), the MPS and the environments are then
 * real, still held as complex128 with zero imaginary parts, and every eigensolve runs a
 * DM_REAL plan on their real parts (every other step keeps the imaginary parts zero).
 * Synchronises. */
int dm_dmrg_sweeps(dm_mps* psi, const dm_mpo_site* w, int32_t nsweeps, int32_t chi,
                   int32_t max_iter, double cutoff, int32_t prec, double* energies,
                   dm_stream stream);
/* Infinite-cylinder DMRG by unit-cell growth (the paper's iDMRG, Sec. I, III A, Fig. 3).
 * cell: the n MPO site tensors of one bulk cell (the MPO repeats every n orbitals:
 * cell[n-1]'s right states are cell[0]'s left states, same order and charges).  psi: the
 * 2n orbitals of two cells (local charges of cell i on orbitals i and n + i) whose last
 * bond is its first bond with every charge moved by d, the charge of the two cells
 * (N exactly, k modulo ly).  L0 (ENV_L on psi's bond 0, states cell[0].ql) and R0
 * (ENV_R on bond 2n, states cell[0].ql): device environments of the blocks left and
 * right of the two cells (read on `stream`; for instance contracted from the boundary
 * states R and F through one cell of random isometries each: a one-sector boundary
 * here would freeze the charge of the bond between the next two cells).
 * Iteration j: the two cells are brought to right-canonical form (dm_theta_split moving
 * left, no eigensolve), then `sweeps` two-site sweeps as dm_dmrg_sweeps (the last one
 * stops at bond n); at bond n theta's Lanczos ground state is split once with both
 * gauges, energies[j] = its energy (the total energy of the 2 (j + 1) cells between the
 * initial blocks), the left cell (left-canonical) joins the left block and the right
 * cell (right-canonical) the right block; the next two cells start from the right cell
 * (with the Schmidt values at its left) followed by the left cell, its charges moved by
 * d (the right block's environment moves with it).  (E_j - E_{j-1}) / 2n is the energy
 * per orbital.  On return psi holds the last iteration's two cells, A..A (S V^H) B..B,
 * and dm_mps_schmidt(psi, n) the Schmidt values between them.  Environments in FP64;
 * the plans in precision prec (DM_REAL as in dm_dmrg_sweeps).  Synchronises.  After an
 * error psi is unspecified (destroy it). */
int dm_idmrg(dm_mps* psi, const dm_mpo_site* cell, dm_charge d, const void* L0, const void* R0,
             int32_t n_iter, int32_t sweeps, int32_t chi, int32_t max_iter, double cutoff,
             int32_t prec, double* energies, dm_stream stream);
/* Entanglement spectrum of one cut (Sec. III C): energies[i] = -2 ln lambda_i (may be
 * NULL) and the entropy -sum lambda^2 ln lambda^2 of count positive Schmidt values. */
int dm_entanglement(const double* values, int64_t count, double* entropy, double* energies);

/* ---- Hofstadter MPO ----------------------------------------------------------------
 * Builds the exact MPO of eq. H (Sec. III A) on an Ly x Lx cylinder, open in x and
 * periodic in y, flux 2 pi p/q per plaquette, in the mixed basis of eqs. H_kin and
 * H_int (basis = 0; orbital x*Ly + m, charges (1, m) mod Ly) or the real-space basis of
 * eq. H_real (basis = 1; orbital x*Ly + y, charges (1, 0), ly = 1), by the finite-state
 * machine of Sec. IV with exact merging of proportional states.  basis = 2: the mixed
 * basis in the real form of eq. rot (Sec. IV D): the two phase branches of the
 * intra-ring interaction are rotated into cos / sin combinations at every bond, so every
 * entry is real (returned with zero imaginary parts); same charges and bond dimensions.  The MPO lives in the
 * library; query site tensors with dm_mpo_site_get (pointers stay valid until
 * dm_mpo_destroy). */
typedef struct dm_mpo dm_mpo;
int dm_mpo_hofstadter(int32_t Ly, int32_t Lx, int32_t p, int32_t q, double t, double V,
                      int32_t basis, dm_mpo** out);
int dm_mpo_n_sites(const dm_mpo* m);
int dm_mpo_site_get(const dm_mpo* m, int32_t i, dm_mpo_site* out);
void dm_mpo_destroy(dm_mpo* m);

const char* dm_last_error(void);

#ifdef __cplusplus
}
#endif
#endif /* MRDMRG_H */
