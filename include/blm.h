/*
 * blm.h - C ABI of libblm, the MI355X (gfx950) hot path of the blocked
 * linear method (BLM) for variational Monte Carlo optimisation:
 * Zhao & Neuscamman, arXiv:1702.01481, Sec. II.
 *
 * One optimisation step is, in this call order:
 *
 *   blm_begin_step     previous-update directions Theta (Eq. 9)
 *   blm_build_blocks*  first pass over the samples: every block's overlap S_b
 *                      and Hamiltonian H_b estimates (Eq. 3 on the one-block
 *                      basis of Eq. 4 / Eq. 10)
 *                      (or blm_replay_build: the same, recorded once as a
 *                      HIP graph by blm_capture_build)
 *   blm_solve_blocks   every block's shifted generalised eigenproblem, ranked,
 *                      kept directions B^(b) (Eq. 5 / Eq. 10, Eq. 6)
 *   blm_project*       second pass over the same samples: stage-two estimates
 *                      on the kept directions (Eq. 6, Eq. 7)
 *   blm_stage2         stage-two eigenproblem, energy and update (Eq. 7, Eq. 8)
 *
 * Every function returns a blm_status; nothing throws across the ABI.  On an
 * error, blm_last_error() describes it.  All device pointers are HIP device
 * memory on the device that was current at blm_create; all work runs on the
 * stream given to blm_create.
 *
 * Numbers and layouts
 *   - N_V parameters are split into N_B contiguous blocks by block_offsets
 *     (block b holds parameters [off[b], off[b+1])).
 *   - Per-sample arrays are sample-major: O[s * ld + x] is the derivative
 *     ratio <n|Psi^x>/<n|Psi> of parameter x at sample s, e[s * ld + x] is
 *     <n|H|Psi^x>/<n|Psi>, E_L[s] = <n|H|Psi>/<n|Psi> and w[s] the importance
 *     weight |<n|Psi>|^2 / P(n) (Eq. 3).  w == NULL means all weights are 1.
 *   - Estimates are normalised by the total weight, so S[0][0] = 1.
 *   - The diagonal shift (Sec. II.A) adds delta times the parameter-space
 *     Euclidean metric to H; the coordinate of Psi itself is never shifted.
 *   - Eigenvalues are ranked by real part.  A complex conjugate pair supplies
 *     two directions (real and imaginary parts of its eigenvector) and is
 *     never split at the N_K cut, so a block keeps N_K or N_K + 1 directions.
 */
#ifndef BLM_H
#define BLM_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct blm_ctx blm_ctx;

typedef enum {
  BLM_OK = 0,
  BLM_E_ARG = 1,        /* bad argument or unsupported size */
  BLM_E_STATE = 2,      /* call out of order, or pass 2 saw other samples than pass 1 */
  BLM_E_HIP = 3,        /* a HIP runtime call failed */
  BLM_E_NOMEM = 4,      /* device allocation failed */
  BLM_E_S_NOT_PD = 5,   /* an overlap matrix is not positive definite */
  BLM_E_NONFINITE = 6,  /* NaN or Inf reached an eigenproblem */
  BLM_E_NOCONV = 7,     /* the QR iteration did not converge */
  BLM_E_TIMEOUT = 8     /* workgroups sharing a block eigenproblem stopped waiting for each other */
} blm_status;

typedef enum {
  BLM_PREC_F64 = 0,     /* sample contractions in FP64 on FP64 matrix cores */
  BLM_PREC_BF16X2 = 1,  /* BF16 hi/lo pieces, 3 piece products, FP32 sums flushed to FP64 */
  BLM_PREC_BF16X3 = 2,  /* BF16 hi/mid/lo pieces, 6 piece products, FP32 sums flushed to FP64 */
  BLM_PREC_FP8 = 3,     /* e4m3 codes with power-of-two column scales and a BF16 residual:
                           the four piece products on BF16 matrix cores (codes converted
                           exactly), FP32 sums scaled and flushed to FP64 */
  BLM_PREC_FP8X2 = 4    /* the same codes and scales with two BF16 residuals r, t: the eight
                           piece products of q, r, t but t t on BF16 matrix cores */
} blm_precision;

typedef enum {
  BLM_LAYOUT_F64 = 0,        /* O, e: double [n][ld], sample-major */
  BLM_LAYOUT_BF16_SPLIT = 1, /* O, e: BF16 pieces, k-packed (see blm_pack_bf16) */
  BLM_LAYOUT_FP8_SCALED = 2  /* O, e: e4m3 codes, plus O_res/e_res and O_scale/e_scale
                                (see blm_pack_fp8) */
} blm_layout;

/* What a step minimises.
 * BLM_TARGET_ENERGY: the energy, the pencil of Eq. 1 on each basis (Eq. 3
 *   estimates: S = sum w obar obar^T, H = sum w obar ebar^T).
 * BLM_TARGET_OMEGA: the excited-state target Omega = <(omega - H)> /
 *   <(omega - H)^2> of Sec. III.D, whose minimum with omega inside the gap is
 *   the first eigenstate above omega.  The BLM applies to it unchanged with
 *   the Omega pencil on the same bases: with f_s = omega obar_s - ebar_s,
 *   A = sum w f obar^T = omega S - H^T ((omega - H) applied to the left basis
 *   function) and B = sum w f f^T = omega^2 S - omega (H + H^T) + E,
 *   E = sum w ebar ebar^T, all divided by the total weight; the solves take
 *   (A + delta P) c = lambda B c (B symmetric positive definite) and the
 *   energies returned are the estimates lambda of Omega.  The left
 *   application keeps an exact eigenstate in the span an exact eigenvector
 *   of the sampled pencil, as H c = E S c does for the energy.  E costs a
 *   second Gram pass over the same chunks inside each blm_build_blocks and
 *   blm_project. */
typedef enum {
  BLM_TARGET_ENERGY = 0,
  BLM_TARGET_OMEGA = 1
} blm_target;

/* Flags returned per shift by blm_stage2 (bit mask). */
enum {
  BLM_FLAG_COMPLEX_ENERGY = 1u,   /* the stage-two lowest eigenvalue is complex; energy = real part */
  BLM_FLAG_PAIR_KEPT = 2u,        /* some block kept a complex pair */
  BLM_FLAG_SMALL_ALPHA = 4u       /* |alpha| < 1e-8 |eigenvector|: the step is very long */
};

typedef struct {
  int64_t n_params;              /* N_V >= 1 */
  int32_t n_blocks;              /* N_B >= 1 */
  const int64_t* block_offsets;  /* host [N_B + 1]: 0 = off[0] < off[1] < ... < off[N_B] = N_V */
  int32_t n_keep;                /* N_K >= 1 directions kept per block (Sec. II.B) */
  int32_t n_old;                 /* N_O >= 0 previous updates used as Theta (Eq. 9); 1 + N_O N_B <= 512 */
  int32_t n_shifts;              /* >= 1 shifts solved together from one build */
  const double* shifts;          /* host [n_shifts], each >= 0 */
  int32_t precision;             /* blm_precision */
  int64_t max_samples;           /* most samples in one build / project call (sum over its chunks) */
  int32_t target;                /* blm_target (BLM_TARGET_ENERGY: 0) */
  double omega;                  /* BLM_TARGET_OMEGA: the energy shift omega (finite); else unused */
} blm_config;

typedef struct {                 /* one chunk of samples; device memory, caller-owned */
  int64_t n_samples;             /* >= 0 */
  int64_t ld;                    /* row stride of O and e in elements, >= N_V */
  const void* O;                 /* BLM_LAYOUT_F64: double [n_samples][ld]; split: piece 0 */
  const void* e;                 /* same layout as O */
  const double* E_L;             /* [n_samples] */
  const double* w;               /* [n_samples] >= 0, or NULL for all-ones (required for BF16, FP8) */
  int32_t layout;                /* blm_layout; must be BLM_LAYOUT_F64 for BLM_PREC_F64,
                                    BLM_LAYOUT_BF16_SPLIT for the BF16 precisions and
                                    BLM_LAYOUT_FP8_SCALED for BLM_PREC_FP8 and FP8X2 */
  int32_t pieces;                /* split layout: pieces stored (2 or 3; >= 3 for BF16X3) */
  int64_t piece_stride;          /* split layout: elements between pieces, multiple of 8 */
  const void* O_res;             /* FP8 layout: BF16 residuals of O (uint16, see blm_pack_fp8) */
  const void* e_res;             /* FP8 layout: BF16 residuals of e */
  const float* O_scale;          /* FP8 layout: [ld] power-of-two column scales of O */
  const float* e_scale;          /* FP8 layout: [ld] column scales of e */
  const void* O_res2;            /* FP8 layout, BLM_PREC_FP8X2: second BF16 residuals of O */
  const void* e_res2;            /* FP8 layout, BLM_PREC_FP8X2: second BF16 residuals of e */
} blm_chunk;

/* Producer-side utility: splits FP64 samples src [n][ld_src] (columns
 * 0..ncols-1) into `pieces` (2 or 3) BF16 pieces, hi = bf16(x), mid =
 * bf16(x - hi), lo = bf16(x - hi - mid), stored k-packed: element (s, x) of
 * piece p at dst[p * piece_stride + ((s / 8) * ld_dst + x) * 8 + s % 8]
 * (uint16 bit patterns).  Rows n .. 8*ceil(n/8)-1 are written as zeros.
 * dst needs pieces * piece_stride elements, piece_stride >= 8*ceil(n/8)*ld_dst,
 * a multiple of 8, and 16-byte alignment.  Asynchronous on `stream`. */
blm_status blm_pack_bf16(const double* src, int64_t n, int64_t ld_src, int64_t ncols, int32_t pieces,
                         uint16_t* dst, int64_t ld_dst, int64_t piece_stride, void* stream);

/* Producer-side utility: FP8 storage of FP64 samples src [n][ld_src]
 * (columns 0..ncols-1), each value x of column c as x = scale[c] (q + r)
 * or, with res2, x = scale[c] (q + r + t):
 *   scale[c]  the smallest power of two (2^-126 .. 2^127) with
 *             max_s |x| / scale[c] <= 448;
 *   q         x / scale[c] rounded to OCP e4m3 (nearest, ties to even,
 *             saturating at 448), stored as its code byte;
 *   r         the exact remainder x / scale[c] - q rounded to FP32 and then
 *             to BF16 (nearest even), stored as uint16 bits;
 *   t         (res2 != NULL) the exact remainder x / scale[c] - q - r rounded
 *             the same way.
 * The stored value is within 2^-13 (1 + 2^-14) |x| (one residual) or
 * 2^-22 (1 + 2^-14) |x| (two) of x in q's normal range.  Layouts (k-packed): code of (s, x) at
 * codes[((s / 16) * ld_dst + x) * 16 + s % 16], residuals at
 * res[((s / 8) * ld_dst + x) * 8 + s % 8] (res2 likewise); rows n .. up to
 * the next multiple of 16 (codes) or 8 (residuals) are zeros.  codes needs
 * 16 * ceil(n / 16) * ld_dst bytes, res and res2 8 * ceil(n / 8) * ld_dst
 * elements each, all 16-byte aligned; scale ncols floats.
 * (Reduced-precision storage of the samples of Eq. 3 is this library's
 * option; the paper works in FP64.)  Asynchronous on `stream`. */
blm_status blm_pack_fp8(const double* src, int64_t n, int64_t ld_src, int64_t ncols, uint8_t* codes,
                        uint16_t* res, uint16_t* res2, float* scale, int64_t ld_dst, void* stream);

/* Bytes of device memory blm_create will allocate for this configuration. */
blm_status blm_workspace_bytes(const blm_config* cfg, size_t* bytes);

/* The part of that workspace which holds the block estimates themselves
 * (Sec. II.B, Fig. 1): each block's H_b and S_b sums (S in whole tiles),
 * the aux Gram, and the coupling strips aux^T O, aux^T e and auxE^T O over
 * all parameters (plus the Omega target's sums of ebar ebar^T in the same
 * layout).  It is the storage the paper counts per process (N_V^2 / N_B +
 * 3 N_V N_O (N_B - 1) elements of 8 bytes, 0.5 GB at N_V = 30,000, N_B = 100,
 * N_O = 5), with whole S tiles and the aux columns padded to groups of 16.
 * Computes without allocating; errors as blm_workspace_bytes. */
blm_status blm_accumulator_bytes(const blm_config* cfg, size_t* bytes);

/* Allocates the context and its device workspace.  stream is a hipStream_t
 * (NULL = the null stream).  The library owns the workspace until
 * blm_destroy. */
blm_status blm_create(const blm_config* cfg, void* stream, blm_ctx** out);
blm_status blm_destroy(blm_ctx* ctx);

/* Starts a step: clears the accumulators and sets the previous-update
 * directions Theta_jk (Eq. 9).  d_old is device [N_O][N_V]: row j-1 is the
 * whole update of step n-j.  Each block's pieces are orthonormalised; zero or
 * dependent pieces are dropped.  NULL (or N_O == 0) means no Theta. */
blm_status blm_begin_step(blm_ctx* ctx, const double* d_old);

/* Pass 1: adds the chunks' contributions to every block's S_b and H_b
 * (Eq. 3 on the Eq. 10 basis).  Asynchronous on the context's stream; the
 * chunks must stay valid until the stream has passed the call.  May be
 * called any number of times per step. */
blm_status blm_build_blocks(blm_ctx* ctx, const blm_chunk* chunks, int32_t n_chunks);

/* Launch-shape autotuner for the block build.  The build's Gram kernel
 * splits the sample axis of every output tile into G groups of 4,096-sample
 * slices, summed afterwards in a fixed order; the best G depends on the
 * device, the blocks and the storage.  This call times the kernel on the
 * given chunks for each G in {1, 2, 3, 4, 6, 8, 12, 16, 24, 32, 48, 64} and
 * the default count, with G times the tile count up to 65,536 (one
 * settling launch and one timed launch each, HIP events on the context's
 * stream), and later builds of this context use the fastest.  For the FP64
 * build it also chooses the tile shape: one 64 x 64 tile per workgroup, or
 * two tiles that share their row tile (64 x 128, the row panels read once
 * for both); the mixed-precision builds always take pairs.  blm_create
 * sizes the partial tiles of the split for the default count; when the
 * candidates need more, this call allocates a larger buffer (up to 6.4 GB)
 * and frees the old one, dropping any recording made by blm_capture_build
 * (record after tuning), or, if the device has no room, tries only the
 * counts that fit.  It writes only the Theta projection of the chunks and
 * scratch tiles: the step's accumulated estimates are unchanged, so it may
 * run between blm_begin_step and the first blm_build_blocks, or between
 * builds.  Synchronises the stream.  h_groups (may be NULL): the chosen G.
 * Returns BLM_E_STATE outside a build phase, BLM_E_ARG for empty or bad
 * chunks. */
blm_status blm_autotune_build(blm_ctx* ctx, const blm_chunk* chunks, int32_t n_chunks, int32_t* h_groups);

/* A step's block build as one HIP graph (Eq. 3 on the Eq. 4 / Eq. 10 basis,
 * as blm_build_blocks).  When every step presents the same chunk buffers
 * (refilled with each step's samples), the build's launches (Theta
 * projection, aux packing, Gram tiles, their sums) have fixed shapes:
 * blm_capture_build records them for this chunk list, with device copies
 * of its own of the launch tables, into a graph held by the context,
 * without running anything and without changing the step's state; it
 * replaces any earlier recording and synchronises the stream.  The graph
 * holds kernel launches only.  blm_replay_build then runs it on the
 * context's stream, with the effect of blm_build_blocks on the recorded
 * chunks (same call-order rules; asynchronous).  The recorded chunk
 * buffers, and their layout, must stay as they were at the recording
 * while replays run; the autotuned launch shape is the one in force at
 * the recording.  Event timing (blm_set_timing) does not cover a replayed
 * build: its phases keep the last call-by-call build's times.  blm_replay_build returns BLM_E_STATE without a
 * recording; blm_capture_build returns BLM_E_ARG for empty or bad chunks
 * and BLM_E_HIP if the runtime refuses the capture; BLM_E_ARG too for a
 * context of the Omega target (its build makes a second pass). */
blm_status blm_capture_build(blm_ctx* ctx, const blm_chunk* chunks, int32_t n_chunks);
blm_status blm_replay_build(blm_ctx* ctx);

/* Solves every block's shifted pencil (H_b + delta P_b) c = lambda S_b c for
 * every shift, ranks the eigenvalues by real part and keeps the parameter
 * part of the best directions, orthonormalised, as B^(b) (Eq. 6).
 * Synchronises the stream.  Optional host outputs:
 *   h_evals [n_shifts][N_B][N_K + 1][2]  the N_K + 1 lowest eigenvalues by real part
 *                                       (re, im); NaN where a pencil has fewer
 *   h_kept  [n_shifts][N_B]             directions kept per block
 * Pencils of 256 or more dimensions are reduced to Hessenberg form by
 * several workgroups each, which meet at a barrier after every elimination
 * step; a wait there gives up after BLM_SYNC_SPIN_LIMIT polls (environment,
 * read by blm_create; default 4194304) and the call then returns
 * BLM_E_TIMEOUT.  The Cholesky factorisations of the overlaps run the same
 * way, one barrier per 16 columns.  BLM_HESS_WORKGROUPS (environment, read
 * by blm_create; default 8) caps the workgroups per pencil in both; 1 keeps
 * every pencil on one workgroup, with no cooperative launch.  Errors: BLM_E_S_NOT_PD, BLM_E_NONFINITE, BLM_E_NOCONV,
 * BLM_E_TIMEOUT name the first failing block. */
blm_status blm_solve_blocks(blm_ctx* ctx, double* h_evals, int32_t* h_kept);

/* Pass 2: projects the same samples onto every shift's kept directions and
 * accumulates the stage-two estimates (Eq. 7).  Asynchronous. */
blm_status blm_project(blm_ctx* ctx, const blm_chunk* chunks, int32_t n_chunks);

/* Solves each shift's stage-two pencil, lowest eigenvalue by real part, and
 * forms the update mu_{i,b} += [A B^(b)]_i / alpha (Eq. 8).  Synchronises.
 *   d_update  device [n_shifts][N_V] (may be NULL)
 *   h_energy  host [n_shifts] real part of the eigenvalue (may be NULL)
 *   h_alpha   host [n_shifts] |alpha| / |eigenvector| (may be NULL)
 *   h_flags   host [n_shifts] BLM_FLAG_* bits (may be NULL)
 * Returns BLM_E_STATE if pass 2 saw a different sample count or total
 * weight than pass 1. */
blm_status blm_stage2(blm_ctx* ctx, double* d_update, double* h_energy, double* h_alpha,
                      uint32_t* h_flags);

/* Batches: several independent optimisations (contexts) whose block solves
 * share one eigensolver launch, and whose stage-two solves share another
 * (Sec. II.B applied to each context on its own; nothing is shared between
 * their estimates).  Their block builds can share one Gram launch too
 * (blm_batch_build), and their projections one projection launch and one
 * stage-two Gram launch (blm_batch_project).
 *
 * blm_batch_create takes n >= 1 distinct contexts created on the same
 * device and stream (else BLM_E_ARG) and allocates the batch's job tables
 * (BLM_E_NOMEM on failure).  The contexts stay owned by the caller and must
 * outlive the batch; the batch keeps their order. */
typedef struct blm_batch blm_batch;
blm_status blm_batch_create(blm_ctx* const* ctxs, int32_t n, blm_batch** out);
blm_status blm_batch_destroy(blm_batch* batch);

/* blm_build_blocks for every context of the batch in one Gram launch (per
 * kind: the FP64 build's tiles, or a mixed-precision build's FP64 aux jobs
 * and then its BF16 or FP8 tile pairs): every context's jobs, each reading
 * its own context's chunks, with one slice-group count for all.  chunks[i]
 * (n_chunks[i] of them) are context i's, as for blm_build_blocks.  The
 * contexts must share one storage (precision) and the energy target, else
 * BLM_E_ARG; a context out of order returns BLM_E_STATE before anything
 * runs.  The estimates equal each context's own blm_build_blocks up to the
 * order of the FP64 sums over slice groups. */
blm_status blm_batch_build(blm_batch* batch, const blm_chunk* const* chunks, const int32_t* n_chunks);

/* blm_project for every context of the batch (Eq. 7 for each on its own):
 * one launch projects every context's chunks onto that context's kept
 * directions, and one Gram launch sums every context's stage-two estimates.
 * chunks and n_chunks as for blm_batch_build; same storage and energy
 * target, else BLM_E_ARG; a context whose block solves have not run returns
 * BLM_E_STATE before anything runs.  The estimates equal each context's own
 * blm_project up to the order of the FP64 sums over slice groups. */
blm_status blm_batch_project(blm_batch* batch, const blm_chunk* const* chunks, const int32_t* n_chunks);

/* blm_solve_blocks for every context of the batch.  h_evals and h_kept are
 * NULL or arrays of n host pointers (each NULL or as for blm_solve_blocks).
 * A context that is not ready returns BLM_E_STATE before anything runs;
 * after the launch every context gets its results and the first error
 * status is returned, its message in that context's blm_last_error. */
blm_status blm_batch_solve_blocks(blm_batch* batch, double* const* h_evals, int32_t* const* h_kept);

/* blm_stage2 for every context of the batch; each argument is NULL or an
 * array of n pointers as for blm_stage2.  Errors as for
 * blm_batch_solve_blocks. */
blm_status blm_batch_stage2(blm_batch* batch, double* const* d_update, double* const* h_energy,
                            double* const* h_alpha, uint32_t* const* h_flags);

/* Diagnostics (valid after blm_solve_blocks).  Block b's normalised matrices
 * on the basis [Psi, Psi^{i,b}, Theta_jk (k != b, kept j, k-major)], with
 * the shift of index `shift` added to H.  h_H, h_S: host [dim][dim] row-major;
 * *dim receives the dimension (call with h_H == NULL to query it).  For the
 * Omega target, the pencil solved: A + delta P in h_H and B in h_S. */
blm_status blm_get_block_matrices(blm_ctx* ctx, int32_t block, int32_t shift, double* h_H,
                                  double* h_S, int32_t* dim);

/* Kept directions of block b for a shift: host [*n_rows][M_b] orthonormal rows. */
blm_status blm_get_directions(blm_ctx* ctx, int32_t block, int32_t shift, double* h_B,
                              int32_t* n_rows);

/* Stage-two matrices of a shift (valid after blm_project + blm_stage2),
 * normalised, unshifted: basis [Psi, B^(0) rows, B^(1) rows, ...].  For the
 * Omega target, A2 in h_H2 and B2 in h_S2. */
blm_status blm_get_stage2_matrices(blm_ctx* ctx, int32_t shift, double* h_H2, double* h_S2,
                                   int32_t* dim);

/* Test hook: all eigenvalues of a dense pencil H c = lambda S c (device
 * [d][d] row-major inputs, S symmetric positive definite), computed by the
 * library's eigensolver; h_evals host [d][2] (re, im) in the solver's order. */
blm_status blm_debug_eigvals(const double* d_H, const double* d_S, int32_t d, double* h_evals,
                             void* stream);

/* For callers that cannot allocate device memory: code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc.  The same
 * eigenvalues as blm_debug_eigvals (same kernels, same order, bit for bit)
 * of a dense pencil H c = lambda S c with S symmetric positive definite,
 * without any device allocation: the solver's scratch (one pencil's
 * workspace, about 12.8 MB) is a static device array of the library, one
 * copy per device, held until the process ends.
 *   d_H, d_S   device [d][d] row-major, caller-owned, read only
 *   d          1 <= d <= BLM_STATIC_MAXD, else BLM_E_ARG (nothing runs)
 *   d_evals    device [d][2] (re, im) in the solver's order; NaN on failure
 *   d_status   device int32: the solve's blm_status (BLM_OK, BLM_E_S_NOT_PD,
 *              BLM_E_NONFINITE or BLM_E_NOCONV), written by the last kernel
 *   stream     hipStream_t of the device current at the call (NULL = null stream)
 * Asynchronous: returns after enqueueing three kernel launches (no copies,
 * no memsets, no synchronisation); the return value reports only argument
 * and launch errors.  The first call on a device resolves the scratch
 * array's device address there (hipGetSymbolAddress, with that device
 * current); a caller that captures graphs should make that first call
 * before capturing.  Every call on a device shares its scratch, and the
 * scratch keeps the last call's contents: calls that overlap on one device
 * (on different streams, or replayed graphs in flight together) race, so
 * serialise them on one stream. */
#define BLM_STATIC_MAXD 512
blm_status blm_pencil_eigvals_static(const double* d_H, const double* d_S, int32_t d, double* d_evals,
                                     int32_t* d_status, void* stream);

/* Per-phase timing with HIP events recorded on the context's stream
 * (off by default).  blm_get_timings synchronises the stream and writes, for
 * the most recent call of each kind, up to n of these durations in ms:
 *   [0] previous-direction projection   [1] block Gram kernel
 *   [2] block Gram reduction             [3] block pencil assembly
 *   [4] block eigensolves                [5] kept-direction projection
 *   [6] stage-two Gram kernel            [7] stage-two Gram reduction
 *   [8] stage-two assembly + eigensolve + update
 *   [9] FP64 strips of the mixed-precision build (with their reduction) */
#define BLM_N_TIMINGS 10
blm_status blm_set_timing(blm_ctx* ctx, int32_t enable);
blm_status blm_get_timings(blm_ctx* ctx, double* h_ms, int32_t n);

/* Statistics of the last blm_solve_blocks, 16 int32 per pencil in the order
 * [shift][block]: status, kept rows, pair flag, QR iterations, then 100 MHz
 * clock ticks of the solver phases (Cholesky, congruence, Hessenberg,
 * QR, selection, inverse iteration, back-transform, orthonormalisation),
 * then ticks spent in early deflation and in bulge chases, and the number
 * of early deflations and of bulge chases. */
blm_status blm_get_solver_stats(blm_ctx* ctx, int32_t* h_stats, int32_t n);

/* Checkpoint of pass 1 (Sec. II.B: the block estimates are running sums
 * over the samples, Eq. 3 on the one-block basis, so a step interrupted
 * between chunks can resume from them).  The state is the FP64 sums of
 * every block, the coupling strips and the aux Gram (Fig. 1; for the Omega
 * target also the second pass's sums), the sample count of pass 1, and a
 * fingerprint of the configuration and of the step's previous directions.
 *
 * blm_state_bytes: the size of the state of this context (host bytes).
 * blm_export_state: after blm_begin_step and any number of
 *   blm_build_blocks / blm_replay_build calls, before blm_solve_blocks
 *   (else BLM_E_STATE); writes the state to the host buffer h_buf of
 *   `bytes` >= blm_state_bytes (else BLM_E_ARG).  Synchronises the stream.
 * blm_import_state: into a context created with the same configuration,
 *   right after blm_begin_step with the same previous directions and before
 *   any build (else BLM_E_STATE; a state of another configuration is
 *   BLM_E_ARG).  Later builds add to the imported sums exactly as they
 *   would have to the exporting context's, so the step's results are the
 *   same bit for bit.  Synchronises the stream.  The buffer stays the
 *   caller's. */
blm_status blm_state_bytes(const blm_ctx* ctx, size_t* bytes);
blm_status blm_export_state(blm_ctx* ctx, void* h_buf, size_t bytes);
blm_status blm_import_state(blm_ctx* ctx, const void* h_buf, size_t bytes);

const char* blm_last_error(const blm_ctx* ctx);
const char* blm_status_string(blm_status s);

#ifdef __cplusplus
}
#endif
#endif /* BLM_H */
