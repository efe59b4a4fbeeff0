// Internal declarations shared by the libblm translation units (kernels and
// host API).  gfx950 only.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace blm {

// Global-address-space view of a pointer read from a job or slice table.
// Loads through generic (flat) pointers count against the LDS wait counter
// too, so waiting for LDS would also wait for in-flight global prefetches.
// (Device pass only: the host pass of a .hip file sees plain pointers.)
#if defined(__HIP_DEVICE_COMPILE__)
#define BLM_GLOBAL __attribute__((address_space(1)))
#else
#define BLM_GLOBAL
#endif
template <class T>
__device__ __forceinline__ BLM_GLOBAL T* as_global(T* p) {
  return (BLM_GLOBAL T*)p;
}
typedef BLM_GLOBAL double gdouble;

// ---------------------------------------------------------------- Gram ----
// Weighted Gram tiles  C = X^T diag(w) Y  over sample slices, FP64 MFMA.
constexpr int GT = 64;        // output tile edge
constexpr int GKS = 16;       // samples per LDS stage
constexpr int GTHREADS = 256; // 4 waves, 2x2 of 32x32 sub-tiles
constexpr int NAUX = 16;      // aux columns per group: [1 | Theta] and [E_L | Theta-energy]
constexpr int NAUX_MAX = 512; // aux columns in all (1 + N_O N_B, padded to whole groups)
constexpr int STRIP_GROUPS = 4;  // aux groups per strip-only job (one read of the tile's panels)
constexpr int SLICE = 4096;   // samples per slice (unit of split-K work)

enum JobKind : int32_t {
  JOB_OFF = 0,          // i < j: S_ij = O_i^T W O_j, H_ij = O_i^T W e_j, H_ji^T = e_i^T W O_j
  JOB_DIAG = 1,         // i == j: S_ii, H_ii, plus the first aux group's strips aux^T W O_i,
                        // aux^T W e_i, auxE^T W O_i
  JOB_DIAG_NOSTRIP = 2, // i == j without strips
  JOB_AUX = 3,          // aux x aux tile (i, j): Xa_i^T W Xa_j, Xa_i^T W Ya_j (from the aux arrays)
  JOB_STRIP = 4         // strips of up to STRIP_GROUPS aux groups over a diagonal tile's columns only
};

struct GramJob {
  int32_t kind;
  int32_t mi, nj;       // valid rows / cols of the tile (<= GT)
  int32_t ag;           // JOB_DIAG, JOB_STRIP: first aux column of the strips' group (multiple of NAUX)
  int32_t ng;           // JOB_STRIP: aux groups of NAUX columns from ag (1..STRIP_GROUPS)
  int32_t set;          // launches over several contexts: the job's slice set (index into the
                        // launch's table of (first slice, slice count)); 0 otherwise
  int64_t ci, cj;       // first source column of tile i / tile j
  int64_t s_off;        // destination of S tile (i,j): s_base[s_off + r*ld_out + c]
  int64_t h_off;        // destination of H tile (i,j)
  int64_t ht_off;       // destination of H tile (j,i) (JOB_OFF): h_base[ht_off + c*ld_out + r]
  int64_t ld_out;
  int64_t strip_col;    // JOB_DIAG, JOB_STRIP: global parameter column of the strip's first column
};

// Two tile jobs of the BF16 build that share their row tile (jb < 0: none).
struct PairJob {
  int32_t ja, jb;
};

// Sample storage: FP64 sample-major ([n][ld]), or BF16 split pieces in the
// k-packed layout: element (s, x) of piece p at base + p * pstride +
// ((s / 8) * ld + x) * 8 + s % 8, so that 8 consecutive samples of one
// parameter are 16 contiguous bytes (one matrix-core operand).
struct Slice {
  const void* O;        // main panels: FP64 (row stride ld) or BF16 pieces (k-packed)
  const void* e;
  const double* Xa;     // aux panels (row stride ald), already offset to the slice's first row
  const double* Ya;
  const double* w;      // weights of the slice's first row, or nullptr
  int64_t ld;
  int64_t n;            // samples in the slice
  int64_t pstride;      // BF16 pieces: elements between pieces
  int32_t pieces;       // 0: FP64 or FP8 storage; 2 or 3: BF16 split pieces
  int32_t ald;          // row stride of Xa, Ya: all aux columns, padded to whole groups
  // BF16 split storage only: the first aux group (Xa, Ya) as BF16 pieces in the
  // k-packed layout with ld = NAUX, from the slice's first 8-sample group;
  // piece p of Xa at Xp + p * apstride (Ya likewise at Yp)
  const uint16_t* Xp;
  const uint16_t* Yp;
  int64_t apstride;
  // FP8 storage only (O, e then hold the e4m3 codes, k-packed by 16 samples:
  // element (s, x) at ((s / 16) * ld + x) * 16 + s % 16 bytes, from the
  // slice's first sample): BF16 residuals k-packed by 8, and the chunk's
  // per-column power-of-two scales; the first aux group likewise with ld = NAUX
  const uint16_t* Or;
  const uint16_t* er;
  const float* Os;
  const float* es;
  const uint8_t* Xq;
  const uint8_t* Yq;
  const uint16_t* Xr;
  const uint16_t* Yr;
  const float* Xs;
  const float* Ys;
  // FP8 storage with two residuals: the second ones, laid out like Or / Xr
  const uint16_t* Ot;
  const uint16_t* et;
  const uint16_t* Xt;
  const uint16_t* Yt;
};

// ------------------------------------------------- direction projection ---
// out[s][1 + d0 + t] = dir_t . O[s, col0 : col0 + m] for every direction t of a block
struct DirBlock {
  int64_t col0;
  int32_t m;
  int32_t d0, nd;
  int32_t pad;
};

// one chunk of a projection launch: its samples go to output rows
// [row_base, row_base + n) of Xo and Yo; workgroups [tile0, tile0 + ceil(n /
// 64)) cover it.  The blocks, directions and outputs are per chunk, so that
// one launch can serve the chunks of several contexts.
struct ProjChunk {
  const DirBlock* blocks;
  const double* const* dir;   // the directions, indexed by DirBlock::d0 + t
  // the same directions as window rows (16-byte loads): each row starts at
  // the even column at or before its block's first one, with a zero there
  // for a block at an odd column, and is padded with zeros to an even width
  const double* const* dirw;
  double* Xo;                 // [rows][ldo]: column 0 is 1, then O . dir
  double* Yo;                 // [rows][ldo]: column 0 is E_L, then e . dir
  int64_t ldo;
  int32_t n_blocks;
  int32_t n_dirs;             // columns past 1 + n_dirs are written as zeros
  const void* O;
  const void* e;
  const double* EL;
  int64_t ld;
  int64_t n;
  int64_t row_base;
  int64_t pstride;
  int32_t tile0;
  int32_t pieces;       // 0: FP64 storage; 2 or 3: BF16 split pieces (k-packed)
  // FP8 storage (O, e are e4m3 codes k-packed by 16): residuals and scales
  const uint16_t* Or;
  const uint16_t* er;
  const float* Os;
  const float* es;
  const uint16_t* Ot;   // second residuals (FP8 storage with two), else nullptr
  const uint16_t* et;
};
// one direction row copied into its window row: dst[r] = src[r - sh] for
// sh <= r < sh + m, zero elsewhere in [0, mwp)
struct WinCopy {
  const double* src;
  double* dst;
  int32_t m, sh, mwp, pad;
};
void launch_window_copy(const WinCopy* d_tab, int n, int max_mwp, hipStream_t st);
// window width of a block of m columns starting at column col0
inline int window_width(int64_t col0, int m) { return (int)(((col0 & 1) + m + 1) & ~1); }

// sample storage of a projection launch
enum StoreKind : int32_t { STORE_F64 = 0, STORE_BF16 = 1, STORE_FP8 = 2 };
constexpr int PROJ_ROWS = 64;

// ------------------------------------------------------------ eigensolve --
enum EigMode : int32_t {
  EIG_BLOCK = 0,        // kept directions: beta parts, orthonormalised
  EIG_STAGE2 = 1,       // lowest eigenvector, full
  EIG_VALUES = 2        // all eigenvalues only
};

struct EigJob {
  int32_t d;            // pencil dimension
  int32_t mode;
  int32_t n_want;       // directions wanted (EIG_BLOCK); 1 for EIG_STAGE2
  int32_t beta0, nbeta; // beta part of each eigenvector: entries [beta0, beta0 + nbeta)
  int32_t mw0, mkw;     // launches with several workgroups per pencil: the pencil's first
                        // workgroup and its count (set by launch_eig_split)
  double* S;            // [d][d] overlap in, Cholesky factor out
  double* A;            // [d][d] shifted Hamiltonian in, destroyed
  double* Hq;           // [d][d] Hessenberg copy
  double* V;            // [d][d] Householder vectors (row k: reflector k)
  double* W;            // max(2 d^2, 16 d): complex LU, congruence and Hessenberg scratch, and
                        // the QR chase's transposed rows above its window (d^2 + d / 2)
  double* vec;          // [n_sel][2][d] complex eigenvectors
  double* wr;           // [d]
  double* wi;           // [d]
  double* tau;          // [d]
  double* out;          // EIG_BLOCK: [n_want + 1][nbeta] rows; EIG_STAGE2: [2][d] (re, im)
  double* out_evals;    // [n_want + 1][2] the lowest eigenvalues in rank order (NaN past the last)
  int32_t* info;        // [EIG_INFO]: [0] status, [1] rows/vectors produced, [2] flags,
                        // [3] QR iterations, [4..11] 100 MHz ticks per phase (Cholesky,
                        // congruence, Hessenberg, QR, selection, inverse iteration,
                        // back-transform, orthonormalisation), [12] ticks in early
                        // deflation, [13] ticks in bulge chases, [14] early
                        // deflations, [15] chases
};

constexpr int EIG_INFO = 16;

enum EigStatus : int32_t {
  EIG_OK = 0,
  EIG_NOT_PD = 1,
  EIG_NONFINITE = 2,
  EIG_NOCONV = 3,
  EIG_SYNC = 4  // a workgroup barrier of the distributed Hessenberg reduction ran past its bound
};

constexpr int EIG_THREADS = 1024;
constexpr int EIG_MAXD = 4096;
constexpr int EIG_MAXSEL = 16;   // eigenvalues selected per problem (N_K + 1 <= this)

// launchers (blm_kernels.hip / blm_eig.hip)
// split: strip and aux jobs of a mixed build; stage2: the stage-two Gram
// (its own kernel instantiation, named apart in traces)
// d_sets (nullptr: every job reads slices [0, n_slices)): per slice set,
// (first slice, slice count) in d_slices, for launches whose jobs belong to
// several contexts (GramJob::set)
void launch_gram(const GramJob* d_jobs, int n_jobs, const Slice* d_slices, int n_slices, int P,
                 bool vec, bool split, bool stage2, double* d_partial, hipStream_t st,
                 const int2* d_sets = nullptr);
// d_pairs: the n_strip_pairs pairs that start with a diagonal tile first,
// then the others (each group is a launch of its own)
void launch_gram_bf16(const PairJob* d_pairs, int n_strip_pairs, int n_pairs, const GramJob* d_jobs,
                      const Slice* d_slices, int n_slices, int P, int pieces, double* d_partial,
                      hipStream_t st, const int2* d_sets = nullptr);
void launch_pack_bf16(const double* src, int64_t n, int64_t ld_src, int64_t ncols, int pieces,
                      uint16_t* dst, int64_t ld_dst, int64_t pstride, hipStream_t st);
void launch_gram_reduce(const GramJob* d_jobs, int n_jobs, int P, const double* d_partial,
                        double* s_base, double* h_base, double* strip_base, int64_t strip_ld,
                        int strip_rows, hipStream_t st);
// FP64 block tiles in pairs sharing a row tile (blm_gram64.hip); d_pairs as
// for launch_gram_bf16, indices into d_jobs
void launch_gram64_pairs(const PairJob* d_pairs, int n_strip_pairs, int n_pairs, const GramJob* d_jobs,
                         const Slice* d_slices, int n_slices, int P, double* d_partial, hipStream_t st,
                         const int2* d_sets = nullptr);
// nres: residuals per value in the FP8 storage (1 or 2)
void launch_gram_fp8(const PairJob* d_pairs, int n_strip_pairs, int n_pairs, const GramJob* d_jobs,
                     const Slice* d_slices, int n_slices, int P, int nres, double* d_partial, hipStream_t st,
                     const int2* d_sets = nullptr);
// FP64 [n][ld_src] -> e4m3 codes (k-packed by 16), one or two BF16 residuals
// (k-packed by 8; res2 nullptr: one) and per-column power-of-two scales
// (blm_fp8.hip)
void launch_pack_fp8(const double* src, int64_t n, int64_t ld_src, int64_t ncols, uint8_t* codes,
                     uint16_t* res, uint16_t* res2, float* scale, int64_t ld_dst, hipStream_t st);
// max_nd: the most directions of any block of any chunk
void launch_dirproj(const ProjChunk* d_chunks, int n_chunks, int n_tiles, bool vec, int store, int max_nd,
                    hipStream_t st);
void launch_eig(const EigJob* d_jobs, int n_jobs, hipStream_t st);
// the same with each pencil's Hessenberg reduction spread over several
// workgroups (cooperative launch; d_bar: 2 n_jobs counters); returns false
// if it had to fall back to one workgroup per pencil
// h_jobs: the host copy of the n_jobs pencils, uploaded to d_jobs by this
// call (it fills their workgroup ranges first)
bool launch_eig_split(EigJob* h_jobs, EigJob* d_jobs, int n_jobs, int d_max, int n_cus, int max_kw,
                      unsigned* d_bar, unsigned spin_limit, hipStream_t st);

}  // namespace blm
