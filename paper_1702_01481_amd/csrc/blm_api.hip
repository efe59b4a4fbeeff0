// Host side of libblm: the C ABI declared in include/blm.h, the context and
// its device workspace, the tile and direction tables, and the small
// glue kernels (previous-direction orthonormalisation, pencil assembly,
// update assembly).
//
// Workspace layout in HBM (FP64 unless noted):
//   D        [N_O][N_V]        orthonormalised previous-update pieces (Eq. 9)
//   Xa, Ya   [max_samples][A]  per-sample aux columns [1, t_s] and [E_L, u_s], where
//                               A = 1 + N_O N_B rounded up to a multiple of 16
//   accS     per block M_b x M_b  sum_s w O_b O_b^T (upper tiles), then A x A aux Gram
//   accH     per block M_b x M_b  sum_s w O_b e_b^T, then A x A aux Gram (X^T W Y)
//   strips   [3][A][N_V]        aux^T W O, aux^T W e, auxE^T W O   (Fig. 1, coupling strips)
//   partial  per (tile job, slice group) 3 x 64 x 64 partial tiles
//   eig      per pencil: S, A, Hq, V (d^2 each), W (2 d^2), vectors, outputs
//   Yp, Zp   [max_samples][n2] stage-two projections [1, B O_b ...], [E_L, B e_b ...]
//   G2S, G2H [n2][n2]          stage-two accumulators
#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <string>
#include <vector>

#include "../../include/blm.h"
#include "blm_internal.h"

using namespace blm;

namespace {

constexpr int MAX_CHUNKS = 4096;   // chunks in one build / project call
constexpr int ST_CREATED = 0, ST_BEGUN = 1, ST_BUILT = 2, ST_SOLVED = 3, ST_PROJECTED = 4,
              ST_DONE = 5;

struct AsmJob {
  int32_t d, M, kind, n_aux;  // kind 0: block, 1: stage two
  int32_t b, pad;
  double delta;
  int64_t off_b;              // first parameter of the block
  int64_t acc_off;            // block accumulators in accS / accH
  const int32_t* aux_idx;     // block: aux column of each non-parameter basis entry
  const int32_t* idx2;        // stage two: joint column of each basis entry
  double* S;
  double* A;
};

struct UpdJob {
  const double* rows;   // kept directions of (shift, block): [n][M_b]
  int32_t n;
  int32_t pad;
};

}  // namespace

struct blm_ctx {
  // configuration
  int64_t NV = 0;
  int NB = 0, NK = 0, NO = 0, NS = 0, prec = 0;
  std::vector<int64_t> off;
  std::vector<double> shifts;
  int64_t max_samples = 0;
  hipStream_t st = nullptr;
  int device = 0;
  int n_cus = 0;                   // compute units of the device (0: unknown)
  unsigned* d_hbar = nullptr;      // block solves: barrier counter and flag per pencil
  unsigned spin_limit = 1u << 22;  // polls of a workgroup barrier before it gives up
  int hess_wg = 32;                // most workgroups per pencil in the distributed Cholesky and Hessenberg
  std::string err;
  int state = ST_CREATED;

  // derived sizes
  int64_t acc_elems = 0, aux_off = 0;
  int NAP = NAUX;                  // aux columns, padded to whole groups of NAUX
  std::vector<int64_t> acc_off;
  std::vector<int> dmax;           // per block: largest pencil dimension
  int d2max = 0, n2max = 0;        // stage two
  int Pcap1 = 1, Pcap2 = 1, PcapM = 1;
  int nd2max = 0;                  // most kept directions of any block (all shifts), last solve
  size_t partial_slots = 0;       // partial tiles allocated (3 x 64 x 64 doubles each)
  int P_tuned[6] = {0, 0, 0, 0, 0, 0};   // slice groups chosen by blm_autotune_build, per build kind (0: heuristic)
  int max_slices = 0;
  int64_t* d_off = nullptr;

  // device buffers
  std::vector<void*> allocs;
  double *D = nullptr, *Xa = nullptr, *Ya = nullptr, *accS = nullptr, *accH = nullptr;
  double *strips = nullptr, *partial = nullptr;
  int32_t* d_dkeep = nullptr;
  GramJob *d_jobs1 = nullptr, *d_jobs2 = nullptr;
  int n_jobs1 = 0, n_jobs2 = 0;
  // mixed precision: jobs1 = FP64 aux job + strips of the aux groups after the
  // first, jobsM = BF16 or FP8 main-product jobs (with the first group's strips)
  GramJob* d_jobsM = nullptr;
  int n_jobsM = 0;
  PairJob* d_pairsM = nullptr;   // BF16 build: pairs of main jobs sharing a row tile
  int n_pairsM = 0;
  int n_strip_pairsM = 0;        // the first n_strip_pairsM pairs start with a diagonal tile
  std::vector<GramJob> h_jobs1, h_jobsM, h_jobs2;   // host copies (batched calls merge them)
  std::vector<PairJob> h_pairsM;
  // FP64 build, second tile shape: the block tiles (the first n_main1 jobs
  // of d_jobs1) as pairs sharing a row tile (64 x 128 per workgroup), strip
  // pairs first; pairs64: build with them (chosen by blm_autotune_build)
  PairJob* d_pairs64 = nullptr;
  int n_main1 = 0, n_pairs64 = 0, n_strip_pairs64 = 0;
  bool pairs64 = false;
  uint16_t* auxP = nullptr;      // BF16 build: first aux group as BF16 pieces (k-packed, ld 16)
  int64_t aux_pstride = 0;       // elements between pieces of auxP (Xa pieces, then Ya pieces)
  int pieces = 0;                  // 0: FP64 path; 2 or 3: BF16 split pieces used
  bool fp8 = false;                // FP8 storage (e4m3 codes, BF16 residuals, column scales)
  int fp8_res = 0;                 // FP8 storage: BF16 residuals per value (1 or 2)
  uint8_t* auxQ = nullptr;         // FP8 build: first aux group's codes (k-packed by 16, ld 16), Xa then Ya
  uint16_t* auxR = nullptr;        // FP8 build: its residuals (k-packed by 8, ld 16), Xa then Ya
  uint16_t* auxT = nullptr;        // FP8 build with two residuals: the second ones, laid out like auxR
  float* auxS = nullptr;           // FP8 build: its column scales [chunk][Xa, Ya][16]
  int64_t auxq_stride = 0, auxr_stride = 0;   // bytes / elements from the Xa to the Ya part
  bool mixed() const { return pieces != 0 || fp8; }
  Slice* d_slices = nullptr;
  ProjChunk* d_pchunks = nullptr;
  // recorded build (blm_capture_build): its own device tables, since other
  // calls rewrite d_slices and d_pchunks; cap: launches are being recorded
  // and take their tables from g_*; dry: tables are built, nothing launched
  hipGraphExec_t gexec = nullptr;
  Slice* g_slices = nullptr;
  ProjChunk* g_pchunks = nullptr;
  int64_t g_total = 0;
  bool cap = false, dry = false;
  std::vector<ProjChunk> h_pchunks;
  bool offsets_even = false;
  DirBlock *d_theta_blk = nullptr, *d_dir2_blk = nullptr;
  const double **d_theta_ptr = nullptr, **d_dir2_ptr = nullptr;
  // the same directions as window rows for 16-byte loads (WinCopy), refreshed
  // by the step's Theta setup and by each block solve
  double *theta_win = nullptr, *dir2_win = nullptr;
  const double **d_theta_wptr = nullptr, **d_dir2_wptr = nullptr;
  WinCopy *d_theta_wcopy = nullptr, *d_dir2_wcopy = nullptr;
  int theta_maxw = 0, dir2_maxw = 0;
  int32_t* d_auxlist = nullptr;    // per block: [1 + N_O (N_B - 1)]
  int auxlist_stride = 0;
  // eigen workspace: block problems [NS][NB], stage two [NS]
  std::vector<EigJob> eig1, eig2;
  EigJob *d_eig1 = nullptr, *d_eig2 = nullptr;
  AsmJob *d_asm1 = nullptr, *d_asm2 = nullptr, *d_asm_x = nullptr;
  int32_t *d_info1 = nullptr, *d_info2 = nullptr;
  double *d_ev1 = nullptr, *d_ev2 = nullptr;
  double *Yp = nullptr, *Zp = nullptr, *G2S = nullptr, *G2H = nullptr;
  int32_t* d_idx2 = nullptr;       // [NS][n2max]
  double *exS = nullptr, *exA = nullptr;  // export scratch
  UpdJob* d_upd = nullptr;
  double* d_coef = nullptr;        // [NS][NB][EIG_MAXSEL]
  int32_t* d_blk_of = nullptr;     // [NV]
  double* d_wsum = nullptr;        // [2] pass-1 and pass-2 total weight
  // excited-state target: the sums of ebar ebar^T, laid out as accS (block
  // tiles and aux Gram), strips and G2S, from a second Gram pass
  int target = BLM_TARGET_ENERGY;
  double omega = 0.0;
  double *accE = nullptr, *stripsE = nullptr, *G2E = nullptr;
  std::vector<Slice> h_slices_e;   // slice table of the second pass

  // step state
  std::vector<int> dkeep;          // [NB][NO]
  std::vector<std::vector<int>> auxlist;   // per block
  std::vector<int> nkept;          // [NS][NB]
  std::vector<int> pairkept;       // [NS][NB]
  std::vector<int32_t> last_info1; // solver statistics of the last block solve
  int n2 = 0, ld2 = 0;               // stage-two columns; row stride of Yp / Zp (even)
  std::vector<std::vector<int>> idx2;   // per shift
  int64_t n_pass1 = 0, n_pass2 = 0;
  std::vector<Slice> h_slices;

  // optional phase timing: event pairs (start, end) per phase
  bool timing = false;
  hipEvent_t ev[2 * BLM_N_TIMINGS] = {};
  bool ev_used[BLM_N_TIMINGS] = {};
};

namespace {

blm_status fail(blm_ctx* c, blm_status s, const std::string& m) {
  if (c) c->err = m;
  return s;
}

// Records the start (end == false) or end of phase i on the context's stream.
// device tables of the launches being issued or recorded
Slice* slice_tab(const blm_ctx* c) { return c->cap ? c->g_slices : c->d_slices; }
ProjChunk* pchunk_tab(const blm_ctx* c) { return c->cap ? c->g_pchunks : c->d_pchunks; }

void mark(blm_ctx* c, int i, bool end) {
  if (!c->timing || c->cap) return;
  (void)hipEventRecord(c->ev[2 * i + (end ? 1 : 0)], c->st);
  if (end) c->ev_used[i] = true;
}

#define HIPCHK(ctx, call)                                                                   \
  do {                                                                                      \
    hipError_t e_ = (call);                                                                 \
    if (e_ != hipSuccess)                                                                   \
      return fail(ctx, BLM_E_HIP, std::string(#call) + ": " + hipGetErrorString(e_));        \
  } while (0)

// ------------------------------------------------------------- kernels ----

// Orthonormalises each block's pieces of the previous updates (Eq. 9):
// modified Gram-Schmidt over j = 1..N_O; zero or dependent pieces dropped.
__global__ __launch_bounds__(256) void theta_mgs_kernel(double* D, int64_t NV, int NO,
                                                        const int64_t* off, int32_t* keep) {
  __shared__ double red[4];
  const int k = blockIdx.x, tid = threadIdx.x;
  const int64_t o = off[k], m = off[k + 1] - off[k];
  auto bsum = [&](double v) {
    for (int s = 32; s > 0; s >>= 1) v += __shfl_xor(v, s, 64);
    __syncthreads();
    if ((tid & 63) == 0) red[tid >> 6] = v;
    __syncthreads();
    return red[0] + red[1] + red[2] + red[3];
  };
  for (int j = 0; j < NO; ++j) {
    double* r = D + (size_t)j * NV + o;
    double p = 0.0;
    for (int64_t i = tid; i < m; i += 256) p += r[i] * r[i];
    const double n0 = sqrt(bsum(p));
    for (int q = 0; q < j; ++q) {
      if (!keep[k * NO + q]) continue;
      const double* qv = D + (size_t)q * NV + o;
      double pd = 0.0;
      for (int64_t i = tid; i < m; i += 256) pd += qv[i] * r[i];
      const double dot = bsum(pd);
      for (int64_t i = tid; i < m; i += 256) r[i] -= dot * qv[i];
    }
    p = 0.0;
    for (int64_t i = tid; i < m; i += 256) p += r[i] * r[i];
    const double nr = sqrt(bsum(p));
    const bool ok = n0 > 0.0 && nr >= 1e-12 * n0;
    const double sc = ok ? 1.0 / nr : 0.0;
    for (int64_t i = tid; i < m; i += 256) r[i] *= sc;
    if (tid == 0) keep[k * NO + j] = ok ? 1 : 0;
    __syncthreads();
  }
}

// Where a pencil's entries come from: the block accumulators (and, for the
// Omega target, the sums of ebar ebar^T in the same layouts) and the
// stage-two Gram.
struct AsmSrc {
  const double *accS, *accH, *strips, *G2S, *G2H;
  const double *accE, *stripsE, *G2E;
  int64_t NV, aux_off, ld2;
  int32_t nap, target;
  double omega;
};

// Unnormalised S and H entries (x, y) of a pencil, from accumulators laid
// out as accS / accH / strips / G2S / G2H.
__device__ __forceinline__ void asm_fetch(const AsmJob& J, int x, int y, const double* __restrict__ accS,
                                          const double* __restrict__ accH, const double* __restrict__ strips,
                                          const double* __restrict__ G2S, const double* __restrict__ G2H,
                                          const AsmSrc& R, double& s, double& h) {
  if (J.kind == 1) {
    const int a = J.idx2[x], b = J.idx2[y];
    s = G2S[(size_t)std::min(a, b) * R.ld2 + std::max(a, b)];
    h = G2H[(size_t)a * R.ld2 + b];
    return;
  }
  const int M = J.M;
  const bool px = (x >= 1 && x <= M), py = (y >= 1 && y <= M);
  const int ax = (x == 0) ? J.aux_idx[0] : J.aux_idx[x > M ? x - M : 0];
  const int ay = (y == 0) ? J.aux_idx[0] : J.aux_idx[y > M ? y - M : 0];
  const int64_t p = x - 1, q = y - 1;
  const size_t S0 = 0, S1 = (size_t)R.nap * R.NV, S2 = 2 * (size_t)R.nap * R.NV;
  if (px && py) {
    s = accS[J.acc_off + std::min(p, q) * M + std::max(p, q)];
    h = accH[J.acc_off + p * M + q];
  } else if (!px && py) {
    s = strips[S0 + (size_t)ax * R.NV + J.off_b + q];
    h = strips[S1 + (size_t)ax * R.NV + J.off_b + q];
  } else if (px && !py) {
    s = strips[S0 + (size_t)ay * R.NV + J.off_b + p];
    h = strips[S2 + (size_t)ay * R.NV + J.off_b + p];
  } else {
    s = accS[R.aux_off + std::min(ax, ay) * R.nap + std::max(ax, ay)];
    h = accH[R.aux_off + ax * R.nap + ay];
  }
}

// Pencil assembly from the accumulators, normalised by the total weight,
// with the diagonal shift on every coordinate but Psi's.  Energy target:
// (H + delta P, S).  Omega target: (A + delta P, B) with A = omega S - H^T
// and B = omega^2 S - omega (H + H^T) + E, E from the second pass.
__global__ __launch_bounds__(256) void assemble_kernel(const AsmJob* __restrict__ jobs, AsmSrc R) {
  const AsmJob J = jobs[blockIdx.x];
  const int d = J.d;
  const size_t n = (size_t)d * d;
  const double W = (J.kind == 0) ? R.accS[R.aux_off] : R.G2S[0];
  const double inv = 1.0 / W;
  for (size_t t = (size_t)blockIdx.y * blockDim.x + threadIdx.x; t < n;
       t += (size_t)gridDim.y * blockDim.x) {
    const int x = (int)(t / d), y = (int)(t % d);
    double s, h;
    asm_fetch(J, x, y, R.accS, R.accH, R.strips, R.G2S, R.G2H, R, s, h);
    if (R.target == BLM_TARGET_OMEGA) {
      double s_t, h_t, e, e_h;
      asm_fetch(J, y, x, R.accS, R.accH, R.strips, R.G2S, R.G2H, R, s_t, h_t);   // h_t = H[y][x]
      asm_fetch(J, x, y, R.accE, R.accE, R.stripsE, R.G2E, R.G2E, R, e, e_h);   // e = E[x][y]
      const double w = R.omega;
      const double a = w * s - h_t;                       // A = omega S - H^T
      const double b = (w * w) * s - w * (h + h_t) + e;   // B = omega^2 S - omega (H + H^T) + E
      h = a;
      s = b;
    }
    s *= inv;
    h *= inv;
    if (x == y && x >= 1) h += J.delta;
    J.S[t] = s;
    J.A[t] = h;
  }
}

AsmSrc asm_src(const blm_ctx* c, int64_t ld2) {
  AsmSrc R{};
  R.accS = c->accS;
  R.accH = c->accH;
  R.strips = c->strips;
  R.G2S = c->G2S;
  R.G2H = c->G2H;
  R.accE = c->accE;
  R.stripsE = c->stripsE;
  R.G2E = c->G2E;
  R.NV = c->NV;
  R.aux_off = c->aux_off;
  R.ld2 = ld2;
  R.nap = c->NAP;
  R.target = c->target;
  R.omega = c->omega;
  return R;
}

// update[s][x] = sum_r coef[s][b][r] B^(s,b)_r[x - off_b]  (Eq. 8)
__global__ __launch_bounds__(256) void update_kernel(double* __restrict__ upd, int64_t NV, int NB,
                                                     int NS, const int64_t* __restrict__ off,
                                                     const int32_t* __restrict__ blk_of,
                                                     const UpdJob* __restrict__ uj,
                                                     const double* __restrict__ coef) {
  const int64_t x = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int s = blockIdx.y;
  if (x >= NV) return;
  const int b = blk_of[x];
  const UpdJob U = uj[s * NB + b];
  const int64_t M = off[b + 1] - off[b], i = x - off[b];
  double acc = 0.0;
  for (int r = 0; r < U.n; ++r) acc += coef[((size_t)s * NB + b) * EIG_MAXSEL + r] * U.rows[r * M + i];
  upd[(size_t)s * NV + x] = acc;
}

// ------------------------------------------------------------- planning ---

struct Plan {
  std::vector<std::pair<void**, size_t>> items;
};

size_t eig_bytes(int d, int nbeta, int nk) {
  const size_t dd = (size_t)d * d;
  return 8 * (4 * dd + std::max(2 * dd, (size_t)16 * d) + 2 * (size_t)EIG_MAXSEL * d + 3 * (size_t)d +
              (size_t)(nk + 2) * std::max(nbeta, 2 * d));
}

blm_status validate(const blm_config* cfg, blm_ctx* c) {
  if (!cfg) return fail(c, BLM_E_ARG, "config is NULL");
  if (cfg->n_params < 1 || cfg->n_blocks < 1 || !cfg->block_offsets)
    return fail(c, BLM_E_ARG, "n_params and n_blocks must be >= 1 and block_offsets set");
  if (cfg->n_keep < 1 || cfg->n_keep + 1 > EIG_MAXSEL)
    return fail(c, BLM_E_ARG, "n_keep must be in [1, 15]");
  if (cfg->n_old < 0 || 1 + (int64_t)cfg->n_old * cfg->n_blocks > NAUX_MAX)
    return fail(c, BLM_E_ARG, "1 + n_old * n_blocks must be <= 512");
  if (cfg->n_shifts < 1 || !cfg->shifts) return fail(c, BLM_E_ARG, "need at least one shift");
  for (int i = 0; i < cfg->n_shifts; ++i)
    if (!(cfg->shifts[i] >= 0.0) || !std::isfinite(cfg->shifts[i]))
      return fail(c, BLM_E_ARG, "shifts must be finite and >= 0");
  if (cfg->precision != BLM_PREC_F64 && cfg->precision != BLM_PREC_BF16X2 &&
      cfg->precision != BLM_PREC_BF16X3 && cfg->precision != BLM_PREC_FP8 && cfg->precision != BLM_PREC_FP8X2)
    return fail(c, BLM_E_ARG, "unsupported precision");
  if (cfg->max_samples < 1) return fail(c, BLM_E_ARG, "max_samples must be >= 1");
  if (cfg->target != BLM_TARGET_ENERGY && cfg->target != BLM_TARGET_OMEGA)
    return fail(c, BLM_E_ARG, "unknown target");
  if (cfg->target == BLM_TARGET_OMEGA && !std::isfinite(cfg->omega))
    return fail(c, BLM_E_ARG, "omega must be finite");
  if (cfg->block_offsets[0] != 0 || cfg->block_offsets[cfg->n_blocks] != cfg->n_params)
    return fail(c, BLM_E_ARG, "block_offsets must run from 0 to n_params");
  for (int b = 0; b < cfg->n_blocks; ++b) {
    if (cfg->block_offsets[b + 1] <= cfg->block_offsets[b])
      return fail(c, BLM_E_ARG, "block_offsets must be strictly ascending");
    const int64_t d = 1 + (cfg->block_offsets[b + 1] - cfg->block_offsets[b]) +
                      (int64_t)cfg->n_old * (cfg->n_blocks - 1);
    if (d > EIG_MAXD) return fail(c, BLM_E_ARG, "a block pencil exceeds 4096 dimensions");
  }
  const int64_t d2 = 1 + (int64_t)cfg->n_blocks * (cfg->n_keep + 1);
  if (d2 > EIG_MAXD) return fail(c, BLM_E_ARG, "the stage-two pencil exceeds 4096 dimensions");
  return BLM_OK;
}

constexpr int PARTIAL_SLOTS = 65536;   // partial tiles the block build's slice groups may use

// Fills the derived sizes and the list of allocations (pointer slot, bytes).
void plan(blm_ctx* c, Plan& P) {
  const int NB = c->NB, NO = c->NO, NK = c->NK, NS = c->NS;
  const int64_t NV = c->NV;
  c->acc_off.assign(NB, 0);
  int64_t run = 0;
  c->dmax.assign(NB, 0);
  int n_jobs1 = 0, n_diag = 0;
  for (int b = 0; b < NB; ++b) {
    const int64_t M = c->off[b + 1] - c->off[b];
    c->acc_off[b] = run;
    run += M * M;
    c->dmax[b] = (int)(1 + M + (int64_t)NO * (NB - 1));
    const int T = (int)((M + GT - 1) / GT);
    n_jobs1 += T * (T + 1) / 2;
    n_diag += T;
  }
  c->NAP = NAUX * ((1 + NO * NB + NAUX - 1) / NAUX);
  // strip-only jobs of the aux groups after the first, STRIP_GROUPS groups each
  const int n_xstrip = n_diag * ((c->NAP / NAUX - 1 + STRIP_GROUPS - 1) / STRIP_GROUPS);
  const int TA = (c->NAP + GT - 1) / GT;                  // aux Gram: TA x TA tile jobs
  c->aux_off = run;
  run += (int64_t)c->NAP * c->NAP;
  c->acc_elems = run;
  c->n_jobs1 = n_jobs1 + TA * TA + n_xstrip;
  c->n_jobsM = c->mixed() ? n_jobs1 : 0;
  // mixed precision: the first aux group's strips ride on the BF16 or FP8
  // diagonal jobs; the aux Gram and the other groups' strips stay on the
  // FP64 kernel
  if (c->mixed()) c->n_jobs1 = TA * TA + n_xstrip;
  const int64_t aux_groups = c->max_samples / 8 + MAX_CHUNKS;
  c->aux_pstride = c->pieces ? aux_groups * NAUX * 8 : 0;
  c->auxq_stride = c->fp8 ? (c->max_samples / 16 + MAX_CHUNKS) * NAUX * 16 : 0;
  c->auxr_stride = c->fp8 ? (c->max_samples / 8 + MAX_CHUNKS) * NAUX * 8 : 0;
  c->n2max = 1 + NS * NB * (NK + 1);
  c->d2max = 1 + NB * (NK + 1);
  const int T2 = (c->n2max + GT - 1) / GT;
  const int n_jobs2max = T2 * (T2 + 1) / 2;
  // slice groups the block build may take: the heuristic picks about 4,096
  // workgroups, and the workspace holds their partial tiles; the autotuner
  // may try up to 65,536 partial tiles (6.4 GB), growing the workspace then
  c->Pcap1 = std::max(1, std::min(64, (PARTIAL_SLOTS + c->n_jobs1 - 1) / c->n_jobs1));
  // stage two has few tiles (3 at 121 coordinates): up to one slice group
  // per 4,096-sample slice, so that its launch fills the chip
  c->Pcap2 = std::max(1, std::min(512, (4096 + n_jobs2max - 1) / n_jobs2max));
  c->PcapM = c->n_jobsM ? std::max(1, std::min(64, (PARTIAL_SLOTS + c->n_jobsM - 1) / c->n_jobsM)) : 1;
  const int Ph1 = std::max(1, std::min(c->Pcap1, (4096 + c->n_jobs1 - 1) / c->n_jobs1));
  const int PhM = c->n_jobsM ? std::max(1, std::min(c->PcapM, (4096 + c->n_jobsM - 1) / c->n_jobsM)) : 1;
  const size_t slots = std::max({(size_t)c->n_jobs1 * Ph1, (size_t)n_jobs2max * c->Pcap2,
                                 (size_t)c->n_jobsM * PhM});
  c->partial_slots = slots;
  c->max_slices = (int)(c->max_samples / SLICE) + 1024;
  c->auxlist_stride = 1 + NO * (NB - 1);

  auto add = [&](void** slot, size_t bytes) { P.items.push_back({slot, std::max<size_t>(bytes, 8)}); };
  add((void**)&c->D, 8 * (size_t)std::max(NO, 1) * NV);
  add((void**)&c->d_dkeep, 4 * (size_t)std::max(NO * NB, 1));
  add((void**)&c->Xa, 8 * (size_t)c->max_samples * c->NAP);
  add((void**)&c->Ya, 8 * (size_t)c->max_samples * c->NAP);
  add((void**)&c->accS, 8 * (size_t)c->acc_elems);
  add((void**)&c->accH, 8 * (size_t)c->acc_elems);
  add((void**)&c->strips, 8 * (size_t)3 * c->NAP * NV);
  const bool om = c->target == BLM_TARGET_OMEGA;
  add((void**)&c->accE, om ? 8 * (size_t)c->acc_elems : 0);
  add((void**)&c->stripsE, om ? 8 * (size_t)3 * c->NAP * NV : 0);
  add((void**)&c->G2E, om ? 8 * (size_t)c->n2max * c->n2max : 0);
  add((void**)&c->partial, 8 * slots * 3 * GT * GT);
  add((void**)&c->d_off, 8 * (size_t)(NB + 1));
  add((void**)&c->d_jobs1, sizeof(GramJob) * (size_t)c->n_jobs1);
  add((void**)&c->d_jobs2, sizeof(GramJob) * (size_t)n_jobs2max);
  add((void**)&c->d_jobsM, sizeof(GramJob) * (size_t)std::max(c->n_jobsM, 1));
  add((void**)&c->d_pairsM, sizeof(PairJob) * (size_t)std::max(c->n_jobsM, 1));
  add((void**)&c->d_pairs64, c->mixed() ? 0 : sizeof(PairJob) * (size_t)std::max(n_jobs1, 1));
  add((void**)&c->auxP, 2 * 2 * (size_t)c->pieces * c->aux_pstride);
  add((void**)&c->auxQ, 2 * (size_t)c->auxq_stride);
  add((void**)&c->auxR, 2 * 2 * (size_t)c->auxr_stride);
  add((void**)&c->auxT, c->fp8_res == 2 ? 2 * 2 * (size_t)c->auxr_stride : 0);
  add((void**)&c->auxS, c->fp8 ? 4 * (size_t)MAX_CHUNKS * 2 * NAUX : 0);
  add((void**)&c->d_slices, sizeof(Slice) * (size_t)c->max_slices);
  add((void**)&c->d_pchunks, sizeof(ProjChunk) * (size_t)MAX_CHUNKS);
  add((void**)&c->d_theta_blk, sizeof(DirBlock) * (size_t)NB);
  add((void**)&c->d_theta_ptr, sizeof(double*) * (size_t)std::max(NO * NB, 1));
  add((void**)&c->d_dir2_blk, sizeof(DirBlock) * (size_t)NB);
  add((void**)&c->d_dir2_ptr, sizeof(double*) * (size_t)c->n2max);
  {
    // window rows: N_O per block for Theta, up to n2max for the kept directions
    int64_t theta_win = 0;
    int maxw = 2;
    for (int k = 0; k < NB; ++k) {
      const int w = window_width(c->off[k], (int)(c->off[k + 1] - c->off[k]));
      theta_win += (int64_t)NO * w;
      maxw = std::max(maxw, w);
    }
    c->theta_maxw = c->dir2_maxw = maxw;
    add((void**)&c->theta_win, 8 * (size_t)std::max<int64_t>(theta_win, 2));
    add((void**)&c->d_theta_wptr, sizeof(double*) * (size_t)std::max(NO * NB, 1));
    add((void**)&c->d_theta_wcopy, sizeof(WinCopy) * (size_t)std::max(NO * NB, 1));
    add((void**)&c->dir2_win, 8 * (size_t)c->n2max * maxw);
    add((void**)&c->d_dir2_wptr, sizeof(double*) * (size_t)c->n2max);
    add((void**)&c->d_dir2_wcopy, sizeof(WinCopy) * (size_t)c->n2max);
  }
  add((void**)&c->d_auxlist, 4 * (size_t)NB * c->auxlist_stride);
  add((void**)&c->d_eig1, sizeof(EigJob) * (size_t)NS * NB);
  add((void**)&c->d_eig2, sizeof(EigJob) * (size_t)NS);
  add((void**)&c->d_asm1, sizeof(AsmJob) * (size_t)NS * NB);
  add((void**)&c->d_asm2, sizeof(AsmJob) * (size_t)NS);
  add((void**)&c->d_asm_x, sizeof(AsmJob));
  add((void**)&c->d_info1, 4 * EIG_INFO * (size_t)NS * NB);
  add((void**)&c->d_hbar, 4 * 2 * (size_t)NS * NB);
  add((void**)&c->d_info2, 4 * EIG_INFO * (size_t)NS);
  add((void**)&c->d_ev1, 16 * (size_t)NS * NB * (NK + 1));
  add((void**)&c->d_ev2, 16 * (size_t)NS * 2);
  add((void**)&c->Yp, 8 * (size_t)c->max_samples * (c->n2max + 1));
  add((void**)&c->Zp, 8 * (size_t)c->max_samples * (c->n2max + 1));
  add((void**)&c->G2S, 8 * (size_t)c->n2max * c->n2max);
  add((void**)&c->G2H, 8 * (size_t)c->n2max * c->n2max);
  add((void**)&c->d_idx2, 4 * (size_t)NS * c->n2max);
  int dx = c->d2max;
  for (int b = 0; b < NB; ++b) dx = std::max(dx, c->dmax[b]);
  add((void**)&c->exS, 8 * (size_t)dx * dx);
  add((void**)&c->exA, 8 * (size_t)dx * dx);
  add((void**)&c->d_upd, sizeof(UpdJob) * (size_t)NS * NB);
  add((void**)&c->d_coef, 8 * (size_t)NS * NB * EIG_MAXSEL);
  add((void**)&c->d_blk_of, 4 * (size_t)NV);
  add((void**)&c->d_wsum, 16);
}

size_t eig_total_bytes(const blm_ctx* c) {
  size_t t = 0;
  for (int s = 0; s < c->NS; ++s) {
    for (int b = 0; b < c->NB; ++b)
      t += eig_bytes(c->dmax[b], (int)(c->off[b + 1] - c->off[b]), c->NK);
    t += eig_bytes(c->d2max, c->d2max, 1);
  }
  return t;
}

// Carves one pencil's workspace from a contiguous allocation.
EigJob carve(double*& p, int d, int nbeta, int nk, int mode, int want, int beta0,
             int32_t* info, double* ev) {
  EigJob J{};
  const size_t dd = (size_t)d * d;
  J.d = d;
  J.mode = mode;
  J.n_want = want;
  J.beta0 = beta0;
  J.nbeta = nbeta;
  J.S = p; p += dd;
  J.A = p; p += dd;
  J.Hq = p; p += dd;
  J.V = p; p += dd;
  J.W = p; p += std::max(2 * dd, (size_t)16 * d);
  J.vec = p; p += 2 * (size_t)EIG_MAXSEL * d;
  J.wr = p; p += d;
  J.wi = p; p += d;
  J.tau = p; p += d;
  J.out = p; p += (size_t)(nk + 2) * std::max(nbeta, 2 * d);
  J.out_evals = ev;
  J.info = info;
  return J;
}

blm_status upload_gram_jobs1(blm_ctx* c) {
  std::vector<GramJob> jobs, main;
  for (int b = 0; b < c->NB; ++b) {
    const int64_t M = c->off[b + 1] - c->off[b];
    const int T = (int)((M + GT - 1) / GT);
    for (int ti = 0; ti < T; ++ti)
      for (int tj = ti; tj < T; ++tj) {
        GramJob J{};
        J.kind = (ti == tj) ? JOB_DIAG : JOB_OFF;
        J.mi = (int)std::min<int64_t>(GT, M - (int64_t)GT * ti);
        J.nj = (int)std::min<int64_t>(GT, M - (int64_t)GT * tj);
        J.ci = c->off[b] + (int64_t)GT * ti;
        J.cj = c->off[b] + (int64_t)GT * tj;
        J.s_off = c->acc_off[b] + (int64_t)GT * ti * M + (int64_t)GT * tj;
        J.h_off = J.s_off;
        J.ht_off = c->acc_off[b] + (int64_t)GT * tj * M + (int64_t)GT * ti;
        J.ld_out = M;
        J.strip_col = J.ci;
        if (!c->mixed()) jobs.push_back(J);
        else main.push_back(J);   // all products, first strips included, on the mixed-precision kernel
      }
  }
  // the aux Gram: every (i, j) tile (S is read from its upper triangle, H
  // is full)
  for (int a0 = 0; a0 < c->NAP; a0 += GT)
    for (int b0 = 0; b0 < c->NAP; b0 += GT) {
      GramJob A{};
      A.kind = JOB_AUX;
      A.mi = std::min(GT, c->NAP - a0);
      A.nj = std::min(GT, c->NAP - b0);
      A.ci = a0;
      A.cj = b0;
      A.s_off = A.h_off = c->aux_off + (int64_t)a0 * c->NAP + b0;
      A.ld_out = c->NAP;
      jobs.push_back(A);
    }
  // the strips of every aux group after the first, per diagonal tile, up to
  // STRIP_GROUPS groups per job (one read of the tile's panels)
  for (int b = 0; b < c->NB; ++b) {
    const int64_t M = c->off[b + 1] - c->off[b];
    for (int64_t c0 = 0; c0 < M; c0 += GT)
      for (int ag = NAUX; ag < c->NAP; ag += STRIP_GROUPS * NAUX) {
        GramJob X{};
        X.kind = JOB_STRIP;
        X.mi = X.nj = (int)std::min<int64_t>(GT, M - c0);
        X.ci = X.cj = c->off[b] + c0;
        X.ag = ag;
        X.ng = std::min(STRIP_GROUPS, (c->NAP - ag) / NAUX);
        X.ld_out = M;
        X.strip_col = X.ci;
        jobs.push_back(X);
      }
  }
  c->n_jobs1 = (int)jobs.size();
  c->n_jobsM = (int)main.size();
  c->h_jobs1 = jobs;
  c->h_jobsM = main;
  HIPCHK(c, hipMemcpy(c->d_jobs1, jobs.data(), sizeof(GramJob) * jobs.size(), hipMemcpyHostToDevice));
  if (!c->mixed()) {
    // the FP64 block tiles lead d_jobs1; consecutive tiles of one row tile
    // pair up, pairs that start with a diagonal tile first
    int nm = 0;
    while (nm < (int)jobs.size() && (jobs[nm].kind == JOB_DIAG || jobs[nm].kind == JOB_OFF)) ++nm;
    std::vector<PairJob> pairs;
    for (int k = 0; k < nm;) {
      PairJob pj{k, -1};
      if (k + 1 < nm && jobs[k + 1].ci == jobs[k].ci) pj.jb = k + 1;
      pairs.push_back(pj);
      k += (pj.jb >= 0) ? 2 : 1;
    }
    std::stable_partition(pairs.begin(), pairs.end(),
                          [&](const PairJob& pj) { return jobs[pj.ja].kind == JOB_DIAG; });
    c->n_main1 = nm;
    c->n_strip_pairs64 = 0;
    for (const PairJob& pj : pairs) c->n_strip_pairs64 += jobs[pj.ja].kind == JOB_DIAG;
    c->n_pairs64 = (int)pairs.size();
    if (!pairs.empty())
      HIPCHK(c, hipMemcpy(c->d_pairs64, pairs.data(), sizeof(PairJob) * pairs.size(), hipMemcpyHostToDevice));
  }
  if (!main.empty()) {
    HIPCHK(c, hipMemcpy(c->d_jobsM, main.data(), sizeof(GramJob) * main.size(), hipMemcpyHostToDevice));
    // consecutive main jobs of one row tile (same first column) pair up
    std::vector<PairJob> pairs;
    for (size_t k = 0; k < main.size();) {
      PairJob pj{(int32_t)k, -1};
      if (k + 1 < main.size() && main[k + 1].ci == main[k].ci) pj.jb = (int32_t)(k + 1);
      pairs.push_back(pj);
      k += (pj.jb >= 0) ? 2 : 1;
    }
    // pairs that start with a diagonal tile (coupling strips) first: the
    // two groups are separate launches of separate kernel instantiations
    std::stable_partition(pairs.begin(), pairs.end(),
                          [&](const PairJob& pj) { return main[pj.ja].kind == JOB_DIAG; });
    c->n_strip_pairsM = 0;
    for (const PairJob& pj : pairs) c->n_strip_pairsM += main[pj.ja].kind == JOB_DIAG;
    c->n_pairsM = (int)pairs.size();
    c->h_pairsM = pairs;
    HIPCHK(c, hipMemcpy(c->d_pairsM, pairs.data(), sizeof(PairJob) * pairs.size(), hipMemcpyHostToDevice));
  }
  return BLM_OK;
}

int choose_P(int cap, int n_jobs, int n_slices) {
  int P = (4096 + n_jobs - 1) / n_jobs;
  P = std::min(P, cap);
  P = std::min(P, std::max(1, n_slices));
  return std::max(P, 1);
}

blm_status check_chunks(blm_ctx* c, const blm_chunk* ch, int n, int64_t* total) {
  if (n < 0 || (n > 0 && !ch)) return fail(c, BLM_E_ARG, "bad chunk list");
  if (n > MAX_CHUNKS) return fail(c, BLM_E_ARG, "more than 4096 chunks in one call");
  int64_t t = 0;
  for (int i = 0; i < n; ++i) {
    if (ch[i].n_samples < 0) return fail(c, BLM_E_ARG, "negative n_samples");
    if (ch[i].n_samples == 0) continue;
    if (ch[i].ld < c->NV) return fail(c, BLM_E_ARG, "chunk ld < n_params");
    if (!ch[i].O || !ch[i].e || !ch[i].E_L) return fail(c, BLM_E_ARG, "chunk pointer is NULL");
    if (!c->mixed() && ch[i].layout != BLM_LAYOUT_F64)
      return fail(c, BLM_E_ARG, "the FP64 precision needs BLM_LAYOUT_F64 chunks");
    if (c->fp8) {
      if (ch[i].layout != BLM_LAYOUT_FP8_SCALED)
        return fail(c, BLM_E_ARG, "the FP8 precision needs BLM_LAYOUT_FP8_SCALED chunks");
      if (ch[i].w) return fail(c, BLM_E_ARG, "the FP8 precision needs uniform weights (w == NULL)");
      if (!ch[i].O_res || !ch[i].e_res || !ch[i].O_scale || !ch[i].e_scale)
        return fail(c, BLM_E_ARG, "FP8 chunk: residual or scale pointer is NULL");
      if (((uintptr_t)ch[i].O | (uintptr_t)ch[i].e | (uintptr_t)ch[i].O_res | (uintptr_t)ch[i].e_res) & 15)
        return fail(c, BLM_E_ARG, "FP8 chunk: codes and residuals need 16-byte alignment");
      if (c->fp8_res == 2) {
        if (!ch[i].O_res2 || !ch[i].e_res2)
          return fail(c, BLM_E_ARG, "the FP8X2 precision needs second residuals (O_res2, e_res2)");
        if (((uintptr_t)ch[i].O_res2 | (uintptr_t)ch[i].e_res2) & 15)
          return fail(c, BLM_E_ARG, "FP8 chunk: second residuals need 16-byte alignment");
      }
    }
    if (c->pieces) {
      if (ch[i].layout != BLM_LAYOUT_BF16_SPLIT || ch[i].pieces < c->pieces || ch[i].pieces > 3)
        return fail(c, BLM_E_ARG, "the BF16 precisions need split chunks with enough pieces");
      if (ch[i].w) return fail(c, BLM_E_ARG, "the BF16 precisions need uniform weights (w == NULL)");
      if ((ch[i].piece_stride & 7) || ch[i].piece_stride < 8 * ((ch[i].n_samples + 7) / 8) * ch[i].ld ||
          ((uintptr_t)ch[i].O & 15) || ((uintptr_t)ch[i].e & 15))
        return fail(c, BLM_E_ARG, "split chunk: piece_stride or alignment invalid");
    }
    t += ch[i].n_samples;
  }
  if (t > c->max_samples) return fail(c, BLM_E_ARG, "more samples in one call than max_samples");
  *total = t;
  return BLM_OK;
}

// The projection table entries of one context's chunks, appended to out:
// tiles and row bases count on from *tiles and 0; *vec is cleared when a
// chunk cannot take 16-byte loads.
void add_pchunks(const blm_ctx* c, const blm_chunk* ch, int n, const DirBlock* d_blocks, int n_blocks,
                 const double* const* d_ptr, const double* const* d_wptr, int n_dirs, double* Xo, double* Yo,
                 int64_t ldo, std::vector<ProjChunk>& out, int* tiles, bool* vec) {
  int64_t rb = 0;
  for (int i = 0; i < n; ++i) {
    const int64_t ns = ch[i].n_samples;
    if (ns == 0) continue;
    ProjChunk P{};
    P.blocks = d_blocks;
    P.dir = d_ptr;
    P.dirw = d_wptr;
    P.Xo = Xo;
    P.Yo = Yo;
    P.ldo = ldo;
    P.n_blocks = n_blocks;
    P.n_dirs = n_dirs;
    P.O = ch[i].O;
    P.e = ch[i].e;
    P.EL = ch[i].E_L;
    P.ld = ch[i].ld;
    P.n = ns;
    P.row_base = rb;
    P.tile0 = *tiles;
    P.pieces = c->pieces;
    P.pstride = ch[i].piece_stride;
    if (c->fp8) {
      P.Or = (const uint16_t*)ch[i].O_res;
      P.er = (const uint16_t*)ch[i].e_res;
      P.Os = ch[i].O_scale;
      P.es = ch[i].e_scale;
      if (c->fp8_res == 2) {
        P.Ot = (const uint16_t*)ch[i].O_res2;
        P.et = (const uint16_t*)ch[i].e_res2;
      }
    }
    out.push_back(P);
    *tiles += (int)((ns + PROJ_ROWS - 1) / PROJ_ROWS);
    rb += ns;
    if ((ch[i].ld & 1) || ((uintptr_t)ch[i].O & 15) || ((uintptr_t)ch[i].e & 15)) *vec = false;
  }
}

int store_kind(const blm_ctx* c) { return c->fp8 ? STORE_FP8 : c->pieces ? STORE_BF16 : STORE_F64; }

// One projection launch over all chunks of a call; returns via c->h_pchunks.
// max_nd: the most directions of any block
blm_status run_dirproj(blm_ctx* c, const blm_chunk* ch, int n, const DirBlock* d_blocks,
                       int n_blocks, const double* const* d_ptr, const double* const* d_wptr, int n_dirs,
                       int max_nd, double* Xo, double* Yo, int64_t ldo) {
  c->h_pchunks.clear();
  int tiles = 0;
  bool vec = true;
  add_pchunks(c, ch, n, d_blocks, n_blocks, d_ptr, d_wptr, n_dirs, Xo, Yo, ldo, c->h_pchunks, &tiles, &vec);
  if (c->h_pchunks.empty() || c->dry) return BLM_OK;
  if (!c->cap)
    HIPCHK(c, hipMemcpyAsync(c->d_pchunks, c->h_pchunks.data(), sizeof(ProjChunk) * c->h_pchunks.size(),
                             hipMemcpyHostToDevice, c->st));
  const int store = store_kind(c);
  launch_dirproj(pchunk_tab(c), (int)c->h_pchunks.size(), tiles, vec && store == STORE_F64, store, max_nd, c->st);
  HIPCHK(c, hipGetLastError());
  return BLM_OK;
}

// kind: 0 FP64 kernel on FP64 storage, 1 FP64 kernel on split storage
// (strips), 2 BF16 matrix-core kernel on split storage (main products),
// 3 FP8 + BF16 matrix-core kernel on FP8 storage (main products),
// 4 FP64 kernel, stage two, 5 FP64 pair kernel on FP64 storage (block tiles
// in pairs sharing a row tile): the Gram launch of one kind over the slice
// table on the device, into the partial tiles
void launch_build_gram(blm_ctx* c, int kind, const GramJob* d_jobs, int n_jobs, int n_slices, int P, bool vec) {
  if (kind == 5)
    launch_gram64_pairs(c->d_pairs64, c->n_strip_pairs64, c->n_pairs64, d_jobs, slice_tab(c), n_slices, P,
                        c->partial, c->st);
  else if (kind == 2)
    launch_gram_bf16(c->d_pairsM, c->n_strip_pairsM, c->n_pairsM, d_jobs, slice_tab(c), n_slices, P, c->pieces,
                     c->partial, c->st);
  else if (kind == 3)
    launch_gram_fp8(c->d_pairsM, c->n_strip_pairsM, c->n_pairsM, d_jobs, slice_tab(c), n_slices, P, c->fp8_res,
                    c->partial, c->st);
  else
    launch_gram(d_jobs, n_jobs, slice_tab(c), n_slices, P, vec && (kind == 0 || kind == 4), kind == 1, kind == 4,
                c->partial, c->st);
}

// tuned: the block build's main Gram launch, which takes the slice-group
// count found by blm_autotune_build (the aux and stage-two Gram launches
// keep the heuristic)
blm_status run_gram(blm_ctx* c, GramJob* d_jobs, int n_jobs, int cap, double* s_base,
                    double* h_base, double* strip_base, int phase, bool vec, int kind = 0,
                    bool tuned = false) {
  const int n_slices = (int)c->h_slices.size();
  if (n_slices == 0 || n_jobs == 0) return BLM_OK;
  for (const Slice& S : c->h_slices)
    if ((S.ld & 1) || ((uintptr_t)S.O & 15) || ((uintptr_t)S.e & 15)) vec = false;
  if (n_slices > c->max_slices) return fail(c, BLM_E_ARG, "too many slices in one call");
  if (!c->cap)
    HIPCHK(c, hipMemcpyAsync(c->d_slices, c->h_slices.data(), sizeof(Slice) * n_slices,
                             hipMemcpyHostToDevice, c->st));
  int P = choose_P(cap, n_jobs, n_slices);
  if (tuned && c->P_tuned[kind] > 0) P = std::max(1, std::min({c->P_tuned[kind], cap, std::max(1, n_slices)}));
  if (phase >= 0) mark(c, phase, false);
  launch_build_gram(c, kind, d_jobs, n_jobs, n_slices, P, vec);
  HIPCHK(c, hipGetLastError());
  if (phase >= 0) {
    mark(c, phase, true);
    mark(c, phase + 1, false);
  }
  launch_gram_reduce(d_jobs, n_jobs, P, c->partial, s_base, h_base, strip_base, c->NV, c->NAP, c->st);
  HIPCHK(c, hipGetLastError());
  if (phase >= 0) mark(c, phase + 1, true);
  return BLM_OK;
}

// The aux columns of the chunks (Theta projection) and the build's slice
// table (host side, c->h_slices), with the aux columns packed to the
// build's storage per chunk.
blm_status build_slices(blm_ctx* c, const blm_chunk* ch, int n) {
  blm_status s = run_dirproj(c, ch, n, c->d_theta_blk, c->NO > 0 ? c->NB : 0, c->d_theta_ptr, c->d_theta_wptr,
                             c->NO * c->NB,
                             c->NO, c->Xa, c->Ya, c->NAP);
  if (s != BLM_OK) return s;
  c->h_slices.clear();
  int64_t rb = 0, gbase = 0, g16base = 0;
  int ci = 0;
  for (int i = 0; i < n; ++i) {
    const int64_t ns = ch[i].n_samples;
    if (ns == 0) continue;
    uint8_t* xq = nullptr;
    uint16_t *xr = nullptr, *xt = nullptr;
    float* xs = nullptr;
    if (c->fp8) {
      xq = c->auxQ + g16base * NAUX * 16;
      xr = c->auxR + gbase * NAUX * 8;
      if (c->fp8_res == 2) xt = c->auxT + gbase * NAUX * 8;
      xs = c->auxS + (size_t)ci * 2 * NAUX;
    }
    if (c->fp8 && !c->dry) {
      // this chunk's first aux group in FP8 storage, with its own scales
      launch_pack_fp8(c->Xa + (size_t)rb * c->NAP, ns, c->NAP, NAUX, xq, xr, xt, xs, NAUX, c->st);
      launch_pack_fp8(c->Ya + (size_t)rb * c->NAP, ns, c->NAP, NAUX, xq + c->auxq_stride, xr + c->auxr_stride,
                      xt ? xt + c->auxr_stride : nullptr, xs + NAUX, NAUX, c->st);
      HIPCHK(c, hipGetLastError());
    }
    if (c->pieces && !c->dry) {
      // this chunk's first aux group as BF16 pieces, from an 8-sample group boundary
      uint16_t* xp = c->auxP + gbase * NAUX * 8;
      launch_pack_bf16(c->Xa + (size_t)rb * c->NAP, ns, c->NAP, NAUX, c->pieces, xp, NAUX, c->aux_pstride,
                       c->st);
      launch_pack_bf16(c->Ya + (size_t)rb * c->NAP, ns, c->NAP, NAUX, c->pieces,
                       xp + (size_t)c->pieces * c->aux_pstride, NAUX, c->aux_pstride, c->st);
      HIPCHK(c, hipGetLastError());
    }
    for (int64_t s0 = 0; s0 < ns; s0 += SLICE) {
      Slice S{};
      if (c->fp8) {
        // slice starts are multiples of 16 samples
        S.O = (const uint8_t*)ch[i].O + (size_t)(s0 / 16) * ch[i].ld * 16;
        S.e = (const uint8_t*)ch[i].e + (size_t)(s0 / 16) * ch[i].ld * 16;
        S.Or = (const uint16_t*)ch[i].O_res + (size_t)(s0 / 8) * ch[i].ld * 8;
        S.er = (const uint16_t*)ch[i].e_res + (size_t)(s0 / 8) * ch[i].ld * 8;
        S.Os = ch[i].O_scale;
        S.es = ch[i].e_scale;
        S.Xq = xq + (size_t)(s0 / 16) * NAUX * 16;
        S.Yq = S.Xq + c->auxq_stride;
        S.Xr = xr + (size_t)(s0 / 8) * NAUX * 8;
        S.Yr = S.Xr + c->auxr_stride;
        S.Xs = xs;
        S.Ys = xs + NAUX;
        if (c->fp8_res == 2) {
          S.Ot = (const uint16_t*)ch[i].O_res2 + (size_t)(s0 / 8) * ch[i].ld * 8;
          S.et = (const uint16_t*)ch[i].e_res2 + (size_t)(s0 / 8) * ch[i].ld * 8;
          S.Xt = xt + (size_t)(s0 / 8) * NAUX * 8;
          S.Yt = S.Xt + c->auxr_stride;
        }
      } else if (c->pieces) {
        // k-packed pieces: slice starts are multiples of 8 samples
        S.O = (const uint16_t*)ch[i].O + (size_t)(s0 / 8) * ch[i].ld * 8;
        S.e = (const uint16_t*)ch[i].e + (size_t)(s0 / 8) * ch[i].ld * 8;
        S.pstride = ch[i].piece_stride;
        S.pieces = c->pieces;
      } else {
        S.O = (const double*)ch[i].O + (size_t)s0 * ch[i].ld;
        S.e = (const double*)ch[i].e + (size_t)s0 * ch[i].ld;
      }
      S.Xa = c->Xa + (size_t)(rb + s0) * c->NAP;
      S.Ya = c->Ya + (size_t)(rb + s0) * c->NAP;
      S.ald = c->NAP;
      if (c->pieces) {
        S.Xp = c->auxP + (size_t)(gbase + s0 / 8) * NAUX * 8;
        S.Yp = S.Xp + (size_t)c->pieces * c->aux_pstride;
        S.apstride = c->aux_pstride;
      }
      S.w = ch[i].w ? ch[i].w + s0 : nullptr;
      S.ld = ch[i].ld;
      S.n = std::min<int64_t>(SLICE, ns - s0);
      c->h_slices.push_back(S);
    }
    rb += ns;
    gbase += (ns + 7) / 8;
    g16base += (ns + 15) / 16;
    ++ci;
  }
  return BLM_OK;
}

// (a replay may still run on the context's stream: it reads the tables)
void release_build_graph(blm_ctx* c) {
  if (c->gexec) (void)hipStreamSynchronize(c->st);
  if (c->gexec) (void)hipGraphExecDestroy(c->gexec);
  if (c->g_slices) (void)hipFree(c->g_slices);
  if (c->g_pchunks) (void)hipFree(c->g_pchunks);
  c->gexec = nullptr;
  c->g_slices = nullptr;
  c->g_pchunks = nullptr;
  c->g_total = 0;
}

}  // namespace

extern "C" {

const char* blm_status_string(blm_status s) {
  switch (s) {
    case BLM_OK: return "ok";
    case BLM_E_ARG: return "invalid argument";
    case BLM_E_STATE: return "call out of order or inconsistent passes";
    case BLM_E_HIP: return "HIP runtime error";
    case BLM_E_NOMEM: return "out of device memory";
    case BLM_E_S_NOT_PD: return "overlap matrix not positive definite";
    case BLM_E_NONFINITE: return "non-finite value in an eigenproblem";
    case BLM_E_NOCONV: return "QR iteration did not converge";
    case BLM_E_TIMEOUT: return "workgroups of a block eigenproblem timed out waiting for each other";
  }
  return "unknown status";
}

const char* blm_last_error(const blm_ctx* c) { return c ? c->err.c_str() : "no context"; }

blm_status blm_workspace_bytes(const blm_config* cfg, size_t* bytes) {
  blm_ctx tmp;
  blm_status s = validate(cfg, &tmp);
  if (s != BLM_OK) return s;
  if (!bytes) return BLM_E_ARG;
  tmp.NV = cfg->n_params;
  tmp.NB = cfg->n_blocks;
  tmp.NK = cfg->n_keep;
  tmp.NO = cfg->n_old;
  tmp.NS = cfg->n_shifts;
  tmp.off.assign(cfg->block_offsets, cfg->block_offsets + cfg->n_blocks + 1);
  tmp.max_samples = cfg->max_samples;
  tmp.pieces = cfg->precision == BLM_PREC_BF16X3 ? 3 : cfg->precision == BLM_PREC_BF16X2 ? 2 : 0;
  tmp.fp8 = cfg->precision == BLM_PREC_FP8 || cfg->precision == BLM_PREC_FP8X2;
  tmp.fp8_res = cfg->precision == BLM_PREC_FP8X2 ? 2 : tmp.fp8 ? 1 : 0;
  tmp.target = cfg->target;
  Plan P;
  plan(&tmp, P);
  size_t t = 0;
  for (auto& it : P.items) t += (it.second + 255) / 256 * 256;
  *bytes = t + eig_total_bytes(&tmp);
  return BLM_OK;
}

blm_status blm_accumulator_bytes(const blm_config* cfg, size_t* bytes) {
  blm_ctx tmp;
  blm_status s = validate(cfg, &tmp);
  if (s != BLM_OK) return s;
  if (!bytes) return BLM_E_ARG;
  tmp.NV = cfg->n_params;
  tmp.NB = cfg->n_blocks;
  tmp.NK = cfg->n_keep;
  tmp.NO = cfg->n_old;
  tmp.NS = cfg->n_shifts;
  tmp.off.assign(cfg->block_offsets, cfg->block_offsets + cfg->n_blocks + 1);
  tmp.max_samples = cfg->max_samples;
  tmp.target = cfg->target;
  Plan P;
  plan(&tmp, P);
  const size_t one = 8 * ((size_t)2 * tmp.acc_elems + (size_t)3 * tmp.NAP * tmp.NV);
  *bytes = tmp.target == BLM_TARGET_OMEGA ? one + 8 * ((size_t)tmp.acc_elems + (size_t)3 * tmp.NAP * tmp.NV) : one;
  return BLM_OK;
}

blm_status blm_pack_bf16(const double* src, int64_t n, int64_t ld_src, int64_t ncols, int32_t pieces,
                         uint16_t* dst, int64_t ld_dst, int64_t piece_stride, void* stream) {
  if (!src || !dst || n < 0 || ncols < 1 || ld_src < ncols || ld_dst < ncols) return BLM_E_ARG;
  if (pieces < 2 || pieces > 3 || (piece_stride & 7) || piece_stride < 8 * ((n + 7) / 8) * ld_dst ||
      ((uintptr_t)dst & 15))
    return BLM_E_ARG;
  launch_pack_bf16(src, n, ld_src, ncols, pieces, dst, ld_dst, piece_stride, (hipStream_t)stream);
  return hipGetLastError() == hipSuccess ? BLM_OK : BLM_E_HIP;
}

blm_status blm_pack_fp8(const double* src, int64_t n, int64_t ld_src, int64_t ncols, uint8_t* codes,
                        uint16_t* res, uint16_t* res2, float* scale, int64_t ld_dst, void* stream) {
  if (!src || !codes || !res || !scale || n < 0 || ncols < 1 || ld_src < ncols || ld_dst < ncols)
    return BLM_E_ARG;
  if (((uintptr_t)codes & 15) || ((uintptr_t)res & 15) || ((uintptr_t)res2 & 15)) return BLM_E_ARG;
  launch_pack_fp8(src, n, ld_src, ncols, codes, res, res2, scale, ld_dst, (hipStream_t)stream);
  return hipGetLastError() == hipSuccess ? BLM_OK : BLM_E_HIP;
}

}  // extern "C"

namespace {

// Header of an exported pass-1 state; the FP64 arrays follow it.
struct StateHeader {
  uint64_t magic;
  int64_t version, target, NV, NB, NK, NO, NS, pieces, fp8, fp8_res, NAP;
  double omega;
  uint64_t cfg_hash;     // block offsets and shifts
  uint64_t theta_hash;   // the step's previous directions after blm_begin_step
  int64_t n_pass1, acc_elems, strip_elems;
};
constexpr uint64_t STATE_MAGIC = 0x31544154534d4c42ull;   // "BLMSTAT1"

uint64_t fnv1a(uint64_t h, const void* p, size_t n) {
  const unsigned char* b = (const unsigned char*)p;
  for (size_t i = 0; i < n; ++i) {
    h ^= b[i];
    h *= 0x100000001b3ull;
  }
  return h;
}

int64_t state_strip_elems(const blm_ctx* c) { return (int64_t)3 * c->NAP * c->NV; }

size_t state_size(const blm_ctx* c) {
  const int64_t per = c->acc_elems * 2 + state_strip_elems(c);
  const int64_t om = c->target == BLM_TARGET_OMEGA ? c->acc_elems + state_strip_elems(c) : 0;
  return sizeof(StateHeader) + 8 * (size_t)(per + om);
}

// The header of this context's current step (theta_hash reads the step's
// previous directions back from the device).
blm_status state_header(blm_ctx* c, StateHeader* H) {
  *H = StateHeader{};
  H->magic = STATE_MAGIC;
  H->version = 1;
  H->target = c->target;
  H->NV = c->NV;
  H->NB = c->NB;
  H->NK = c->NK;
  H->NO = c->NO;
  H->NS = c->NS;
  H->pieces = c->pieces;
  H->fp8 = c->fp8;
  H->fp8_res = c->fp8_res;
  H->NAP = c->NAP;
  H->omega = c->omega;
  uint64_t h = 0xcbf29ce484222325ull;
  h = fnv1a(h, c->off.data(), 8 * c->off.size());
  h = fnv1a(h, c->shifts.data(), 8 * c->shifts.size());
  H->cfg_hash = h;
  uint64_t t = 0xcbf29ce484222325ull;
  if (c->NO > 0) {
    std::vector<double> D((size_t)c->NO * c->NV);
    HIPCHK(c, hipMemcpyAsync(D.data(), c->D, 8 * D.size(), hipMemcpyDeviceToHost, c->st));
    HIPCHK(c, hipStreamSynchronize(c->st));
    t = fnv1a(t, D.data(), 8 * D.size());
    t = fnv1a(t, c->dkeep.data(), sizeof(int) * c->dkeep.size());
  }
  H->theta_hash = t;
  H->n_pass1 = c->n_pass1;
  H->acc_elems = c->acc_elems;
  H->strip_elems = state_strip_elems(c);
  return BLM_OK;
}

}  // namespace

extern "C" {

blm_status blm_state_bytes(const blm_ctx* c, size_t* bytes) {
  if (!c || !bytes) return BLM_E_ARG;
  *bytes = state_size(c);
  return BLM_OK;
}

blm_status blm_export_state(blm_ctx* c, void* h_buf, size_t bytes) {
  if (!c) return BLM_E_ARG;
  if (!h_buf || bytes < state_size(c)) return fail(c, BLM_E_ARG, "state buffer missing or too small");
  if (c->state != ST_BEGUN && c->state != ST_BUILT)
    return fail(c, BLM_E_STATE, "blm_export_state needs a step in pass 1 (after blm_begin_step, before the solves)");
  StateHeader H;
  blm_status s = state_header(c, &H);
  if (s != BLM_OK) return s;
  std::memcpy(h_buf, &H, sizeof H);
  char* p = (char*)h_buf + sizeof H;
  auto put = [&](const double* d, int64_t n) -> blm_status {
    HIPCHK(c, hipMemcpyAsync(p, d, 8 * (size_t)n, hipMemcpyDeviceToHost, c->st));
    p += 8 * (size_t)n;
    return BLM_OK;
  };
  if ((s = put(c->accS, c->acc_elems)) != BLM_OK || (s = put(c->accH, c->acc_elems)) != BLM_OK ||
      (s = put(c->strips, H.strip_elems)) != BLM_OK)
    return s;
  if (c->target == BLM_TARGET_OMEGA &&
      ((s = put(c->accE, c->acc_elems)) != BLM_OK || (s = put(c->stripsE, H.strip_elems)) != BLM_OK))
    return s;
  HIPCHK(c, hipStreamSynchronize(c->st));
  return BLM_OK;
}

blm_status blm_import_state(blm_ctx* c, const void* h_buf, size_t bytes) {
  if (!c) return BLM_E_ARG;
  if (!h_buf || bytes < sizeof(StateHeader)) return fail(c, BLM_E_ARG, "state buffer missing or too small");
  if (c->state != ST_BEGUN || c->n_pass1 != 0)
    return fail(c, BLM_E_STATE, "blm_import_state needs blm_begin_step and no build since");
  StateHeader H, mine;
  std::memcpy(&H, h_buf, sizeof H);
  blm_status s = state_header(c, &mine);
  if (s != BLM_OK) return s;
  if (H.magic != mine.magic || H.version != mine.version || H.target != mine.target || H.NV != mine.NV ||
      H.NB != mine.NB || H.NK != mine.NK || H.NO != mine.NO || H.NS != mine.NS || H.pieces != mine.pieces ||
      H.fp8 != mine.fp8 || H.fp8_res != mine.fp8_res || H.NAP != mine.NAP || H.omega != mine.omega ||
      H.cfg_hash != mine.cfg_hash || H.acc_elems != mine.acc_elems || H.strip_elems != mine.strip_elems)
    return fail(c, BLM_E_ARG, "the state was exported from a context of another configuration");
  if (bytes < state_size(c)) return fail(c, BLM_E_ARG, "state buffer too small");
  if (H.theta_hash != mine.theta_hash)
    return fail(c, BLM_E_STATE, "the step's previous directions differ from the exporting step's");
  if (H.n_pass1 < 0) return fail(c, BLM_E_ARG, "the state's sample count is not valid");
  const char* p = (const char*)h_buf + sizeof H;
  auto get = [&](double* d, int64_t n) -> blm_status {
    HIPCHK(c, hipMemcpyAsync(d, p, 8 * (size_t)n, hipMemcpyHostToDevice, c->st));
    p += 8 * (size_t)n;
    return BLM_OK;
  };
  if ((s = get(c->accS, c->acc_elems)) != BLM_OK || (s = get(c->accH, c->acc_elems)) != BLM_OK ||
      (s = get(c->strips, H.strip_elems)) != BLM_OK)
    return s;
  if (c->target == BLM_TARGET_OMEGA &&
      ((s = get(c->accE, c->acc_elems)) != BLM_OK || (s = get(c->stripsE, H.strip_elems)) != BLM_OK))
    return s;
  HIPCHK(c, hipStreamSynchronize(c->st));
  c->n_pass1 = H.n_pass1;
  c->state = H.n_pass1 > 0 ? ST_BUILT : ST_BEGUN;
  return BLM_OK;
}

blm_status blm_get_solver_stats(blm_ctx* c, int32_t* h_stats, int32_t n) {
  if (!c || !h_stats || n < 0) return BLM_E_ARG;
  const int m = std::min<int>(n, (int)c->last_info1.size());
  std::copy(c->last_info1.begin(), c->last_info1.begin() + m, h_stats);
  return BLM_OK;
}

blm_status blm_set_timing(blm_ctx* c, int32_t enable) {
  if (!c) return BLM_E_ARG;
  if (enable && !c->timing) {
    for (auto& e : c->ev)
      if (!e) HIPCHK(c, hipEventCreate(&e));
  }
  c->timing = enable != 0;
  return BLM_OK;
}

blm_status blm_get_timings(blm_ctx* c, double* h_ms, int32_t n) {
  if (!c || !h_ms || n < 0) return BLM_E_ARG;
  HIPCHK(c, hipStreamSynchronize(c->st));
  for (int i = 0; i < n && i < BLM_N_TIMINGS; ++i) {
    h_ms[i] = -1.0;
    if (!c->ev_used[i]) continue;
    float ms = 0.f;
    if (hipEventElapsedTime(&ms, c->ev[2 * i], c->ev[2 * i + 1]) == hipSuccess) h_ms[i] = ms;
  }
  return BLM_OK;
}

blm_status blm_destroy(blm_ctx* c) {
  if (!c) return BLM_OK;
  release_build_graph(c);
  for (auto& e : c->ev)
    if (e) (void)hipEventDestroy(e);
  for (void* p : c->allocs) (void)hipFree(p);
  delete c;
  return BLM_OK;
}

blm_status blm_create(const blm_config* cfg, void* stream, blm_ctx** out) {
  if (!out) return BLM_E_ARG;
  *out = nullptr;
  blm_ctx* c = new blm_ctx();
  blm_status s = validate(cfg, c);
  if (s != BLM_OK) {
    delete c;
    return s;
  }
  c->NV = cfg->n_params;
  c->NB = cfg->n_blocks;
  c->NK = cfg->n_keep;
  c->NO = cfg->n_old;
  c->NS = cfg->n_shifts;
  c->prec = cfg->precision;
  c->pieces = cfg->precision == BLM_PREC_BF16X3 ? 3 : cfg->precision == BLM_PREC_BF16X2 ? 2 : 0;
  c->fp8 = cfg->precision == BLM_PREC_FP8 || cfg->precision == BLM_PREC_FP8X2;
  c->fp8_res = cfg->precision == BLM_PREC_FP8X2 ? 2 : c->fp8 ? 1 : 0;
  c->off.assign(cfg->block_offsets, cfg->block_offsets + cfg->n_blocks + 1);
  c->shifts.assign(cfg->shifts, cfg->shifts + cfg->n_shifts);
  c->max_samples = cfg->max_samples;
  c->target = cfg->target;
  c->omega = cfg->omega;
  c->st = (hipStream_t)stream;
  c->offsets_even = true;
  for (int64_t o : c->off)
    if (o & 1) c->offsets_even = false;
  if (hipGetDevice(&c->device) != hipSuccess) {
    delete c;
    return BLM_E_HIP;
  }
  if (hipDeviceGetAttribute(&c->n_cus, hipDeviceAttributeMultiprocessorCount, c->device) != hipSuccess)
    c->n_cus = 0;
  if (const char* e = getenv("BLM_SYNC_SPIN_LIMIT")) c->spin_limit = (unsigned)strtoul(e, nullptr, 10);
  if (const char* e = getenv("BLM_HESS_WORKGROUPS")) c->hess_wg = std::max(1, atoi(e));
  if (const char* e = getenv("BLM_FP64_PAIRS")) c->pairs64 = atoi(e) != 0;
  Plan P;
  plan(c, P);
  for (auto& it : P.items) {
    void* p = nullptr;
    if (hipMalloc(&p, it.second) != hipSuccess) {
      blm_destroy(c);
      return BLM_E_NOMEM;
    }
    c->allocs.push_back(p);
    *it.first = p;
  }
  // eigen workspaces
  {
    void* p = nullptr;
    if (hipMalloc(&p, eig_total_bytes(c)) != hipSuccess) {
      blm_destroy(c);
      return BLM_E_NOMEM;
    }
    c->allocs.push_back(p);
    double* q = (double*)p;
    for (int sh = 0; sh < c->NS; ++sh)
      for (int b = 0; b < c->NB; ++b) {
        const int M = (int)(c->off[b + 1] - c->off[b]);
        const int i = sh * c->NB + b;
        double* start = q;
        c->eig1.push_back(carve(q, c->dmax[b], M, c->NK, EIG_BLOCK, c->NK, 1, c->d_info1 + EIG_INFO * i,
                                c->d_ev1 + 2 * (size_t)i * (c->NK + 1)));
        q = start + eig_bytes(c->dmax[b], M, c->NK) / 8;
      }
    for (int sh = 0; sh < c->NS; ++sh) {
      double* start = q;
      c->eig2.push_back(carve(q, c->d2max, c->d2max, 1, EIG_STAGE2, 1, 0, c->d_info2 + EIG_INFO * sh,
                              c->d_ev2 + 4 * (size_t)sh));
      q = start + eig_bytes(c->d2max, c->d2max, 1) / 8;
    }
  }
  blm_status r = upload_gram_jobs1(c);
  if (r != BLM_OK) {
    blm_destroy(c);
    return r;
  }
  // static tables: block of each parameter, offsets
  {
    std::vector<int32_t> blk(c->NV);
    for (int b = 0; b < c->NB; ++b)
      for (int64_t x = c->off[b]; x < c->off[b + 1]; ++x) blk[x] = b;
    if (hipMemcpy(c->d_blk_of, blk.data(), 4 * (size_t)c->NV, hipMemcpyHostToDevice) != hipSuccess) {
      blm_destroy(c);
      return BLM_E_HIP;
    }
    (void)hipMemcpy(c->d_off, c->off.data(), 8 * (c->NB + 1), hipMemcpyHostToDevice);
    // theta direction table (fixed): block k, rows j of D
    std::vector<DirBlock> tb(c->NB);
    std::vector<const double*> tp((size_t)std::max(c->NO * c->NB, 1), nullptr);
    std::vector<const double*> tpw(tp.size(), nullptr);
    std::vector<WinCopy> tcw(tp.size());
    int64_t wbase = 0;
    for (int k = 0; k < c->NB; ++k) {
      tb[k].col0 = c->off[k];
      tb[k].m = (int)(c->off[k + 1] - c->off[k]);
      tb[k].d0 = k * c->NO;
      tb[k].nd = c->NO;
      const int w = window_width(tb[k].col0, tb[k].m);
      for (int j = 0; j < c->NO; ++j) {
        tp[k * c->NO + j] = c->D + (size_t)j * c->NV + c->off[k];
        double* dst = c->theta_win + wbase;
        tpw[k * c->NO + j] = dst;
        tcw[k * c->NO + j] = WinCopy{tp[k * c->NO + j], dst, tb[k].m, (int)(tb[k].col0 & 1), w, 0};
        wbase += w;
      }
    }
    (void)hipMemcpy(c->d_theta_blk, tb.data(), sizeof(DirBlock) * c->NB, hipMemcpyHostToDevice);
    (void)hipMemcpy(c->d_theta_ptr, tp.data(), sizeof(double*) * tp.size(), hipMemcpyHostToDevice);
    (void)hipMemcpy(c->d_theta_wptr, tpw.data(), sizeof(double*) * tpw.size(), hipMemcpyHostToDevice);
    (void)hipMemcpy(c->d_theta_wcopy, tcw.data(), sizeof(WinCopy) * tcw.size(), hipMemcpyHostToDevice);
  }
  *out = c;
  return BLM_OK;
}

static const int64_t* dev_offsets(const blm_ctx* c) { return c->d_off; }

blm_status blm_begin_step(blm_ctx* c, const double* d_old) {
  if (!c) return BLM_E_ARG;
  HIPCHK(c, hipMemsetAsync(c->accS, 0, 8 * (size_t)c->acc_elems, c->st));
  HIPCHK(c, hipMemsetAsync(c->accH, 0, 8 * (size_t)c->acc_elems, c->st));
  HIPCHK(c, hipMemsetAsync(c->strips, 0, 8 * (size_t)3 * c->NAP * c->NV, c->st));
  if (c->target == BLM_TARGET_OMEGA) {
    HIPCHK(c, hipMemsetAsync(c->accE, 0, 8 * (size_t)c->acc_elems, c->st));
    HIPCHK(c, hipMemsetAsync(c->stripsE, 0, 8 * (size_t)3 * c->NAP * c->NV, c->st));
  }
  c->dkeep.assign((size_t)c->NB * c->NO, 0);
  if (c->NO > 0) {
    if (d_old) {
      HIPCHK(c, hipMemcpyAsync(c->D, d_old, 8 * (size_t)c->NO * c->NV, hipMemcpyDeviceToDevice, c->st));
      hipLaunchKernelGGL(theta_mgs_kernel, dim3(c->NB), dim3(256), 0, c->st, c->D, c->NV, c->NO,
                         dev_offsets(c), c->d_dkeep);
      HIPCHK(c, hipGetLastError());
      std::vector<int32_t> k((size_t)c->NB * c->NO);
      HIPCHK(c, hipMemcpyAsync(k.data(), c->d_dkeep, 4 * k.size(), hipMemcpyDeviceToHost, c->st));
      HIPCHK(c, hipStreamSynchronize(c->st));
      for (size_t i = 0; i < k.size(); ++i) c->dkeep[i] = k[i];
    } else {
      HIPCHK(c, hipMemsetAsync(c->D, 0, 8 * (size_t)c->NO * c->NV, c->st));
    }
    launch_window_copy(c->d_theta_wcopy, c->NO * c->NB, c->theta_maxw, c->st);
    HIPCHK(c, hipGetLastError());
  }
  // per-block aux lists: [0] then Theta_(k,j) for k != b, k-major
  c->auxlist.assign(c->NB, {});
  std::vector<int32_t> flat((size_t)c->NB * c->auxlist_stride, 0);
  for (int b = 0; b < c->NB; ++b) {
    auto& L = c->auxlist[b];
    L.push_back(0);
    for (int k = 0; k < c->NB; ++k) {
      if (k == b) continue;
      for (int j = 0; j < c->NO; ++j)
        if (c->dkeep[k * c->NO + j]) L.push_back(1 + k * c->NO + j);
    }
    std::copy(L.begin(), L.end(), flat.begin() + (size_t)b * c->auxlist_stride);
  }
  HIPCHK(c, hipMemcpyAsync(c->d_auxlist, flat.data(), 4 * flat.size(), hipMemcpyHostToDevice, c->st));
  HIPCHK(c, hipStreamSynchronize(c->st));
  c->n_pass1 = c->n_pass2 = 0;
  c->state = ST_BEGUN;
  return BLM_OK;
}

// The launches of one block build on chunks already checked: aux columns
// and slice table, then the Gram launches (issued on c->st, or recorded).
// The slice table of the Omega target's second pass: e in place of O and
// the aux columns [E_L, u] in place of [1, t], in every storage, so that
// the Gram launches' first product, with its strips and the aux Gram, sums
// ebar ebar^T.
static void swap_to_e(std::vector<Slice>& v) {
  for (Slice& S : v) {
    S.O = S.e;
    S.Xa = S.Ya;
    S.Xp = S.Yp;
    S.Or = S.er;
    S.Os = S.es;
    S.Ot = S.et;
    S.Xq = S.Yq;
    S.Xr = S.Yr;
    S.Xs = S.Ys;
    S.Xt = S.Yt;
  }
}

// The Gram launches of one build pass into the given accumulators (h
// nullptr: the H products are not kept).
static blm_status build_grams(blm_ctx* c, double* accS, double* accH, double* strips, bool timed) {
  if (c->mixed()) {
    // FP64 aux Gram and further aux groups' strips (timed in the strips
    // slot), then the mixed-precision products and first strips
    if (timed) mark(c, 9, false);
    blm_status s = run_gram(c, c->d_jobs1, c->n_jobs1, c->Pcap1, accS, accH, strips, -1, false, 1);
    if (s != BLM_OK) return s;
    if (timed) mark(c, 9, true);
    return run_gram(c, c->d_jobsM, c->n_jobsM, c->PcapM, accS, accH, strips, timed ? 1 : -1, false,
                    c->fp8 ? 3 : 2, true);
  }
  if (c->pairs64 && c->n_pairs64 > 0) {
    // FP64 in tile pairs: aux Gram and further aux groups' strips on
    // gram_kernel (timed in the strips slot), then the block tiles
    if (timed) mark(c, 9, false);
    blm_status s = run_gram(c, c->d_jobs1 + c->n_main1, c->n_jobs1 - c->n_main1, c->Pcap1, accS, accH, strips, -1,
                            c->offsets_even, 0);
    if (s != BLM_OK) return s;
    if (timed) mark(c, 9, true);
    return run_gram(c, c->d_jobs1, c->n_main1, c->Pcap1, accS, accH, strips, timed ? 1 : -1, false, 5, true);
  }
  return run_gram(c, c->d_jobs1, c->n_jobs1, c->Pcap1, accS, accH, strips, timed ? 1 : -1, c->offsets_even, 0,
                  true);
}

static blm_status build_launches(blm_ctx* c, const blm_chunk* ch, int32_t n) {
  mark(c, 0, false);
  blm_status s = build_slices(c, ch, n);
  if (s != BLM_OK) return s;
  mark(c, 0, true);
  s = build_grams(c, c->accS, c->accH, c->strips, true);
  if (s != BLM_OK || c->target != BLM_TARGET_OMEGA) return s;
  // second pass over the same chunks: sum w ebar ebar^T (the table is
  // swapped in, not edited, so that the first pass's upload source stays
  // as it was)
  c->h_slices_e = c->h_slices;
  swap_to_e(c->h_slices_e);
  std::swap(c->h_slices, c->h_slices_e);
  s = build_grams(c, c->accE, nullptr, c->stripsE, false);
  std::swap(c->h_slices, c->h_slices_e);
  return s;
}

blm_status blm_build_blocks(blm_ctx* c, const blm_chunk* ch, int32_t n) {
  if (!c) return BLM_E_ARG;
  if (c->state != ST_BEGUN && c->state != ST_BUILT)
    return fail(c, BLM_E_STATE, "blm_build_blocks needs blm_begin_step first");
  int64_t total = 0;
  blm_status s = check_chunks(c, ch, n, &total);
  if (s != BLM_OK) return s;
  s = build_launches(c, ch, n);
  if (s != BLM_OK) return s;
  c->n_pass1 += total;
  c->state = ST_BUILT;
  return BLM_OK;
}

blm_status blm_capture_build(blm_ctx* c, const blm_chunk* ch, int32_t n) {
  if (!c) return BLM_E_ARG;
  if (c->target == BLM_TARGET_OMEGA) return fail(c, BLM_E_ARG, "recorded builds are for the energy target");
  int64_t total = 0;
  blm_status s = check_chunks(c, ch, n, &total);
  if (s != BLM_OK) return s;
  release_build_graph(c);
  // the tables, built without launching anything, into the graph's own
  // device copies
  c->dry = true;
  s = build_slices(c, ch, n);
  c->dry = false;
  if (s != BLM_OK) return s;
  if (c->h_slices.empty()) return fail(c, BLM_E_ARG, "blm_capture_build needs samples");
  if ((int)c->h_slices.size() > c->max_slices) return fail(c, BLM_E_ARG, "too many slices in one call");
  HIPCHK(c, hipStreamSynchronize(c->st));
  HIPCHK(c, hipMalloc((void**)&c->g_slices, sizeof(Slice) * c->h_slices.size()));
  HIPCHK(c, hipMalloc((void**)&c->g_pchunks, sizeof(ProjChunk) * std::max<size_t>(c->h_pchunks.size(), 1)));
  HIPCHK(c, hipMemcpy(c->g_slices, c->h_slices.data(), sizeof(Slice) * c->h_slices.size(),
                      hipMemcpyHostToDevice));
  if (!c->h_pchunks.empty())
    HIPCHK(c, hipMemcpy(c->g_pchunks, c->h_pchunks.data(), sizeof(ProjChunk) * c->h_pchunks.size(),
                        hipMemcpyHostToDevice));
  // record the launches on a stream of the library's own (the context's
  // stream may be the null stream, which cannot be captured)
  hipStream_t cs = nullptr;
  HIPCHK(c, hipStreamCreateWithFlags(&cs, hipStreamNonBlocking));
  hipStream_t saved = c->st;
  c->st = cs;
  c->cap = true;
  hipGraph_t g = nullptr;
  hipError_t e = hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal);
  if (e == hipSuccess) {
    s = build_launches(c, ch, n);
    e = hipStreamEndCapture(cs, &g);
  }
  c->cap = false;
  c->st = saved;
  if (e == hipSuccess && s == BLM_OK) e = hipGraphInstantiate(&c->gexec, g, nullptr, nullptr, 0);
  if (g) (void)hipGraphDestroy(g);
  (void)hipStreamDestroy(cs);
  if (s == BLM_OK && e != hipSuccess) {
    c->gexec = nullptr;
    s = fail(c, BLM_E_HIP, std::string("build capture: ") + hipGetErrorString(e));
  }
  if (s != BLM_OK) {
    release_build_graph(c);
    return s;
  }
  c->g_total = total;
  return BLM_OK;
}

blm_status blm_replay_build(blm_ctx* c) {
  if (!c) return BLM_E_ARG;
  if (!c->gexec) return fail(c, BLM_E_STATE, "blm_replay_build needs blm_capture_build first");
  if (c->state != ST_BEGUN && c->state != ST_BUILT)
    return fail(c, BLM_E_STATE, "blm_replay_build needs blm_begin_step first");
  HIPCHK(c, hipGraphLaunch(c->gexec, c->st));
  c->n_pass1 += c->g_total;
  c->state = ST_BUILT;
  return BLM_OK;
}

blm_status blm_autotune_build(blm_ctx* c, const blm_chunk* ch, int32_t n, int32_t* h_groups) {
  if (!c) return BLM_E_ARG;
  if (c->state != ST_BEGUN && c->state != ST_BUILT)
    return fail(c, BLM_E_STATE, "blm_autotune_build needs blm_begin_step first");
  int64_t total = 0;
  blm_status s = check_chunks(c, ch, n, &total);
  if (s != BLM_OK) return s;
  s = build_slices(c, ch, n);
  if (s != BLM_OK) return s;
  const int n_slices = (int)c->h_slices.size();
  if (n_slices == 0) return fail(c, BLM_E_ARG, "blm_autotune_build needs samples");
  if (n_slices > c->max_slices) return fail(c, BLM_E_ARG, "too many slices in one call");
  HIPCHK(c, hipMemcpyAsync(c->d_slices, c->h_slices.data(), sizeof(Slice) * n_slices, hipMemcpyHostToDevice,
                           c->st));
  const int kind = c->fp8 ? 3 : c->pieces ? 2 : 0;
  const GramJob* jobs = c->mixed() ? c->d_jobsM : c->d_jobs1;
  const int n_jobs = c->mixed() ? c->n_jobsM : c->n_jobs1;
  int cap = std::max(1, std::min(c->mixed() ? c->PcapM : c->Pcap1, n_slices));
  if ((size_t)n_jobs * cap > c->partial_slots) {
    // the candidates need more partial tiles than blm_create sized for the
    // heuristic: grow the workspace (a recorded build refers to the old one,
    // so it is dropped); if the device has no room, try fewer groups
    const size_t want = (size_t)n_jobs * cap;
    void* np = nullptr;
    HIPCHK(c, hipStreamSynchronize(c->st));
    if (hipMalloc(&np, 8 * want * 3 * GT * GT) == hipSuccess) {
      release_build_graph(c);
      for (void*& a : c->allocs)
        if (a == (void*)c->partial) {
          (void)hipFree(a);
          a = np;
        }
      c->partial = (double*)np;
      c->partial_slots = want;
    } else {
      (void)hipGetLastError();
      cap = std::max(1, (int)(c->partial_slots / n_jobs));
    }
  }
  bool vec = kind == 0 && c->offsets_even;
  for (const Slice& S : c->h_slices)
    if ((S.ld & 1) || ((uintptr_t)S.O & 15) || ((uintptr_t)S.e & 15)) vec = false;
  hipEvent_t ev[2] = {nullptr, nullptr};
  if (hipEventCreate(&ev[0]) != hipSuccess || hipEventCreate(&ev[1]) != hipSuccess) {
    if (ev[0]) (void)hipEventDestroy(ev[0]);
    return fail(c, BLM_E_HIP, "hipEventCreate failed");
  }
  // the candidates, and the heuristic's own count
  std::vector<int> cand = {1, 2, 3, 4, 6, 8, 12, 16, 24, 32, 48, 64};
  cand.push_back(choose_P(cap, n_jobs, n_slices));
  std::sort(cand.begin(), cand.end());
  cand.erase(std::unique(cand.begin(), cand.end()), cand.end());
  // tile shapes: the FP64 build also tries its block tiles in pairs that
  // share a row tile (64 x 128 per workgroup, kind 5) against one tile per
  // workgroup (64 x 64, kind 0); a pair launch is timed with the aux and
  // strip-only jobs it leaves to gram_kernel
  std::vector<int> shapes = {kind};
  if (kind == 0 && c->n_pairs64 > 0 && !getenv("BLM_FP64_PAIRS")) shapes.push_back(5);
  auto launch_shape = [&](int sk, int P) {
    if (sk == 5) {
      launch_build_gram(c, 0, c->d_jobs1 + c->n_main1, c->n_jobs1 - c->n_main1, n_slices, P, vec);
      launch_build_gram(c, 5, c->d_jobs1, c->n_main1, n_slices, P, false);
    } else {
      launch_build_gram(c, sk, jobs, n_jobs, n_slices, P, vec);
    }
  };
  int best = 0, best_kind = kind;
  float best_ms = 0.0f;
  blm_status r = BLM_OK;
  for (int sk : shapes) {
    for (int P : cand) {
      if (P > cap) break;
      // one launch to settle caches and clocks, one timed
      launch_shape(sk, P);
      float ms = 0.0f;
      if (hipEventRecord(ev[0], c->st) != hipSuccess) r = BLM_E_HIP;
      launch_shape(sk, P);
      if (r == BLM_OK && (hipGetLastError() != hipSuccess || hipEventRecord(ev[1], c->st) != hipSuccess ||
                          hipEventSynchronize(ev[1]) != hipSuccess ||
                          hipEventElapsedTime(&ms, ev[0], ev[1]) != hipSuccess))
        r = BLM_E_HIP;
      if (r != BLM_OK) break;
      if (getenv("BLM_AUTOTUNE_LOG"))
        fprintf(stderr, "blm_autotune_build: kind %d, %d slice groups: %.3f ms\n", sk, P, ms);
      if (best == 0 || ms < best_ms) {
        best = P;
        best_kind = sk;
        best_ms = ms;
      }
    }
    if (r != BLM_OK) break;
  }
  (void)hipEventDestroy(ev[0]);
  (void)hipEventDestroy(ev[1]);
  if (r != BLM_OK) return fail(c, r, "a tuning launch failed");
  if (shapes.size() > 1) c->pairs64 = best_kind == 5;
  c->P_tuned[best_kind] = best;
  if (h_groups) *h_groups = best;
  return BLM_OK;
}

static blm_status eig_status(blm_ctx* c, int st, const char* what) {
  if (st == EIG_OK) return BLM_OK;
  char buf[160];
  const char* m = st == EIG_NOT_PD      ? "overlap not positive definite"
                  : st == EIG_NONFINITE ? "non-finite values"
                  : st == EIG_SYNC      ? "a workgroup barrier timed out"
                                        : "QR did not converge";
  snprintf(buf, sizeof buf, "%s: %s", what, m);
  c->err = buf;
  return st == EIG_NOT_PD      ? BLM_E_S_NOT_PD
         : st == EIG_NONFINITE ? BLM_E_NONFINITE
         : st == EIG_SYNC      ? BLM_E_TIMEOUT
                               : BLM_E_NOCONV;
}

}  // extern "C"

namespace {

// Block solves in three parts, so that several contexts can share one
// eigensolver launch: assembly of the shifted pencils (jobs returned with
// their dimensions), the launch, then the results and the stage-two tables.
blm_status solve_begin(blm_ctx* c, std::vector<EigJob>& ej, int* dm_out) {
  if (c->state != ST_BUILT) return fail(c, BLM_E_STATE, "blm_solve_blocks needs blm_build_blocks first");
  const int NB = c->NB, NS = c->NS;
  std::vector<AsmJob> asmj;
  ej = c->eig1;
  int dm = 1;
  for (int sh = 0; sh < NS; ++sh)
    for (int b = 0; b < NB; ++b) {
      const int M = (int)(c->off[b + 1] - c->off[b]);
      const int d = 1 + M + (int)c->auxlist[b].size() - 1;
      AsmJob A{};
      A.d = d;
      A.M = M;
      A.kind = 0;
      A.b = b;
      A.n_aux = (int)c->auxlist[b].size();
      A.delta = c->shifts[sh];
      A.off_b = c->off[b];
      A.acc_off = c->acc_off[b];
      A.aux_idx = c->d_auxlist + (size_t)b * c->auxlist_stride;
      EigJob& J = ej[sh * NB + b];
      J.d = d;
      A.S = J.S;
      A.A = J.A;
      asmj.push_back(A);
      dm = std::max(dm, d);
    }
  HIPCHK(c, hipMemcpyAsync(c->d_asm1, asmj.data(), sizeof(AsmJob) * asmj.size(), hipMemcpyHostToDevice, c->st));
  const int gy = std::min(256, std::max(1, (int)(((size_t)dm * dm + 255) / 256 / 8)));
  mark(c, 3, false);
  hipLaunchKernelGGL(assemble_kernel, dim3((unsigned)asmj.size(), gy), dim3(256), 0, c->st, c->d_asm1,
                     asm_src(c, c->n2max));
  HIPCHK(c, hipGetLastError());
  mark(c, 3, true);
  *dm_out = dm;
  return BLM_OK;
}

blm_status solve_end(blm_ctx* c, double* h_evals, int32_t* h_kept) {
  const int NB = c->NB, NS = c->NS, NK = c->NK;
  std::vector<int32_t> info((size_t)EIG_INFO * NS * NB);
  std::vector<double> ev((size_t)2 * NS * NB * (NK + 1));
  HIPCHK(c, hipMemcpyAsync(info.data(), c->d_info1, 4 * info.size(), hipMemcpyDeviceToHost, c->st));
  HIPCHK(c, hipMemcpyAsync(ev.data(), c->d_ev1, 8 * ev.size(), hipMemcpyDeviceToHost, c->st));
  HIPCHK(c, hipStreamSynchronize(c->st));
  c->nkept.assign((size_t)NS * NB, 0);
  c->pairkept.assign((size_t)NS * NB, 0);
  for (int i = 0; i < NS * NB; ++i) {
    char what[64];
    snprintf(what, sizeof what, "block %d, shift %d", i % NB, i / NB);
    blm_status s = eig_status(c, info[EIG_INFO * i], what);
    if (s != BLM_OK) return s;
    c->nkept[i] = info[EIG_INFO * i + 1];
    c->pairkept[i] = info[EIG_INFO * i + 2];
  }
  c->last_info1 = info;
  if (h_evals) std::copy(ev.begin(), ev.end(), h_evals);
  if (h_kept) std::copy(c->nkept.begin(), c->nkept.end(), h_kept);

  // stage-two tables: joint directions ordered block, shift, row
  std::vector<DirBlock> db(NB);
  std::vector<const double*> dp;
  std::vector<std::vector<int>> pos((size_t)NS * NB);
  for (int k = 0; k < NB; ++k) {
    const int M = (int)(c->off[k + 1] - c->off[k]);
    db[k].col0 = c->off[k];
    db[k].m = M;
    db[k].d0 = (int)dp.size();
    for (int sh = 0; sh < NS; ++sh) {
      const EigJob& J = c->eig1[sh * NB + k];
      for (int r = 0; r < c->nkept[sh * NB + k]; ++r) {
        pos[sh * NB + k].push_back(1 + (int)dp.size());
        dp.push_back(J.out + (size_t)r * M);
      }
    }
    db[k].nd = (int)dp.size() - db[k].d0;
  }
  c->nd2max = 0;
  for (int k = 0; k < NB; ++k) c->nd2max = std::max(c->nd2max, db[k].nd);
  c->n2 = 1 + (int)dp.size();
  c->ld2 = (c->n2 + 1) & ~1;
  c->idx2.assign(NS, {});
  std::vector<int32_t> flat((size_t)NS * c->n2max, 0);
  for (int sh = 0; sh < NS; ++sh) {
    auto& I = c->idx2[sh];
    I.push_back(0);
    for (int k = 0; k < NB; ++k)
      for (int p : pos[sh * NB + k]) I.push_back(p);
    std::copy(I.begin(), I.end(), flat.begin() + (size_t)sh * c->n2max);
  }
  std::vector<GramJob> jobs;
  const int n2 = c->n2, T = (n2 + GT - 1) / GT;
  for (int ti = 0; ti < T; ++ti)
    for (int tj = ti; tj < T; ++tj) {
      GramJob J{};
      J.kind = (ti == tj) ? JOB_DIAG_NOSTRIP : JOB_OFF;
      J.mi = std::min(GT, n2 - GT * ti);
      J.nj = std::min(GT, n2 - GT * tj);
      J.ci = (int64_t)GT * ti;
      J.cj = (int64_t)GT * tj;
      J.s_off = (int64_t)GT * ti * n2 + (int64_t)GT * tj;
      J.h_off = J.s_off;
      J.ht_off = (int64_t)GT * tj * n2 + (int64_t)GT * ti;
      J.ld_out = n2;
      jobs.push_back(J);
    }
  c->n_jobs2 = (int)jobs.size();
  c->h_jobs2 = jobs;
  HIPCHK(c, hipMemcpyAsync(c->d_dir2_blk, db.data(), sizeof(DirBlock) * NB, hipMemcpyHostToDevice, c->st));
  HIPCHK(c, hipMemcpyAsync(c->d_dir2_ptr, dp.data(), sizeof(double*) * std::max<size_t>(dp.size(), 1),
                           hipMemcpyHostToDevice, c->st));
  {
    // the kept directions as window rows
    std::vector<const double*> dpw(dp.size());
    std::vector<WinCopy> wc(dp.size());
    int64_t wbase = 0;
    for (int k = 0; k < NB; ++k) {
      const int w = window_width(db[k].col0, db[k].m);
      for (int t = db[k].d0; t < db[k].d0 + db[k].nd; ++t) {
        double* dst = c->dir2_win + wbase;
        dpw[t] = dst;
        wc[t] = WinCopy{dp[t], dst, db[k].m, (int)(db[k].col0 & 1), w, 0};
        wbase += w;
      }
    }
    if (!dp.empty()) {
      HIPCHK(c, hipMemcpyAsync(c->d_dir2_wptr, dpw.data(), sizeof(double*) * dpw.size(), hipMemcpyHostToDevice,
                               c->st));
      HIPCHK(c, hipMemcpyAsync(c->d_dir2_wcopy, wc.data(), sizeof(WinCopy) * wc.size(), hipMemcpyHostToDevice,
                               c->st));
      launch_window_copy(c->d_dir2_wcopy, (int)wc.size(), c->dir2_maxw, c->st);
      HIPCHK(c, hipGetLastError());
    }
  }
  HIPCHK(c, hipMemcpyAsync(c->d_idx2, flat.data(), 4 * flat.size(), hipMemcpyHostToDevice, c->st));
  HIPCHK(c, hipMemcpyAsync(c->d_jobs2, jobs.data(), sizeof(GramJob) * jobs.size(), hipMemcpyHostToDevice, c->st));
  HIPCHK(c, hipMemsetAsync(c->G2S, 0, 8 * (size_t)n2 * n2, c->st));
  HIPCHK(c, hipMemsetAsync(c->G2H, 0, 8 * (size_t)n2 * n2, c->st));
  if (c->target == BLM_TARGET_OMEGA) HIPCHK(c, hipMemsetAsync(c->G2E, 0, 8 * (size_t)n2 * n2, c->st));
  HIPCHK(c, hipStreamSynchronize(c->st));
  c->n_pass2 = 0;
  c->state = ST_SOLVED;
  return BLM_OK;
}

}  // namespace

extern "C" {

blm_status blm_solve_blocks(blm_ctx* c, double* h_evals, int32_t* h_kept) {
  if (!c) return BLM_E_ARG;
  std::vector<EigJob> ej;
  int dm = 1;
  blm_status s = solve_begin(c, ej, &dm);
  if (s != BLM_OK) return s;
  mark(c, 4, false);
  launch_eig_split(ej.data(), c->d_eig1, (int)ej.size(), dm, c->n_cus, c->hess_wg, c->d_hbar, c->spin_limit, c->st);
  HIPCHK(c, hipGetLastError());
  mark(c, 4, true);
  return solve_end(c, h_evals, h_kept);
}

}  // extern "C"

namespace {

// The stage-two slice table (c->h_slices) over the projected samples of the
// chunks: rows of Yp (1, O . directions) and Zp (E_L, e . directions).
void proj_slices(blm_ctx* c, const blm_chunk* ch, int n) {
  const int64_t ldo = c->ld2;
  c->h_slices.clear();
  int64_t rb = 0;
  for (int i = 0; i < n; ++i) {
    const int64_t ns = ch[i].n_samples;
    if (ns == 0) continue;
    for (int64_t s0 = 0; s0 < ns; s0 += SLICE) {
      Slice S{};
      S.O = c->Yp + (size_t)(rb + s0) * ldo;
      S.e = c->Zp + (size_t)(rb + s0) * ldo;
      S.w = ch[i].w ? ch[i].w + s0 : nullptr;
      S.ld = ldo;
      S.n = std::min<int64_t>(SLICE, ns - s0);
      c->h_slices.push_back(S);
    }
    rb += ns;
  }
}

}  // namespace

extern "C" {

blm_status blm_project(blm_ctx* c, const blm_chunk* ch, int32_t n) {
  if (!c) return BLM_E_ARG;
  if (c->state != ST_SOLVED && c->state != ST_PROJECTED)
    return fail(c, BLM_E_STATE, "blm_project needs blm_solve_blocks first");
  int64_t total = 0;
  blm_status s = check_chunks(c, ch, n, &total);
  if (s != BLM_OK) return s;
  const int64_t ldo = c->ld2;
  mark(c, 5, false);
  s = run_dirproj(c, ch, n, c->d_dir2_blk, c->NB, c->d_dir2_ptr, c->d_dir2_wptr, c->n2 - 1, c->nd2max, c->Yp,
                  c->Zp, ldo);
  if (s != BLM_OK) return s;
  proj_slices(c, ch, n);
  mark(c, 5, true);
  s = run_gram(c, c->d_jobs2, c->n_jobs2, c->Pcap2, c->G2S, c->G2H, nullptr, 6, true, 4);
  if (s != BLM_OK) return s;
  if (c->target == BLM_TARGET_OMEGA) {
    // sum w zbar zbar^T: the projections of e on both sides
    c->h_slices_e = c->h_slices;
    for (Slice& S : c->h_slices_e) S.O = S.e;
    std::swap(c->h_slices, c->h_slices_e);
    s = run_gram(c, c->d_jobs2, c->n_jobs2, c->Pcap2, c->G2E, nullptr, nullptr, -1, true, 4);
    std::swap(c->h_slices, c->h_slices_e);
    if (s != BLM_OK) return s;
  }
  c->n_pass2 += total;
  c->state = ST_PROJECTED;
  return BLM_OK;
}

}  // extern "C"

namespace {

// Stage two in the same three parts as the block solves.
blm_status stage2_begin(blm_ctx* c, std::vector<EigJob>& ej, int* dm_out) {
  if (c->state != ST_PROJECTED) return fail(c, BLM_E_STATE, "blm_stage2 needs blm_project first");
  if (c->n_pass2 != c->n_pass1)
    return fail(c, BLM_E_STATE, "pass 2 saw a different number of samples than pass 1");
  const int NS = c->NS, NB = c->NB;
  double w1 = 0.0, w2 = 0.0;
  HIPCHK(c, hipMemcpyAsync(&w1, c->accS + c->aux_off, 8, hipMemcpyDeviceToHost, c->st));
  HIPCHK(c, hipMemcpyAsync(&w2, c->G2S, 8, hipMemcpyDeviceToHost, c->st));
  HIPCHK(c, hipStreamSynchronize(c->st));
  if (!(std::fabs(w1 - w2) <= 1e-12 * std::fabs(w1)) || !(w1 > 0.0))
    return fail(c, BLM_E_STATE, "pass 2 total weight differs from pass 1 (or is not positive)");
  std::vector<AsmJob> asmj;
  ej = c->eig2;
  int dm = 1;
  for (int sh = 0; sh < NS; ++sh) {
    const int d = (int)c->idx2[sh].size();
    AsmJob A{};
    A.d = d;
    A.kind = 1;
    A.delta = c->shifts[sh];
    A.idx2 = c->d_idx2 + (size_t)sh * c->n2max;
    ej[sh].d = d;
    A.S = ej[sh].S;
    A.A = ej[sh].A;
    asmj.push_back(A);
    dm = std::max(dm, d);
  }
  (void)NB;
  mark(c, 8, false);
  HIPCHK(c, hipMemcpyAsync(c->d_asm2, asmj.data(), sizeof(AsmJob) * NS, hipMemcpyHostToDevice, c->st));
  const int gy = std::min(64, std::max(1, (int)(((size_t)dm * dm + 255) / 256 / 8)));
  hipLaunchKernelGGL(assemble_kernel, dim3(NS, gy), dim3(256), 0, c->st, c->d_asm2, asm_src(c, c->n2));
  HIPCHK(c, hipGetLastError());
  *dm_out = dm;
  return BLM_OK;
}

blm_status stage2_end(blm_ctx* c, const std::vector<EigJob>& ej, double* d_update, double* h_energy,
                      double* h_alpha, uint32_t* h_flags) {
  const int NS = c->NS, NB = c->NB;
  std::vector<int32_t> info((size_t)EIG_INFO * NS);
  std::vector<double> ev((size_t)4 * NS);
  HIPCHK(c, hipMemcpyAsync(info.data(), c->d_info2, 4 * info.size(), hipMemcpyDeviceToHost, c->st));
  HIPCHK(c, hipMemcpyAsync(ev.data(), c->d_ev2, 8 * ev.size(), hipMemcpyDeviceToHost, c->st));
  std::vector<std::vector<double>> vecs(NS);
  for (int sh = 0; sh < NS; ++sh) {
    vecs[sh].resize(2 * (size_t)ej[sh].d);
    HIPCHK(c, hipMemcpyAsync(vecs[sh].data(), ej[sh].out, 8 * vecs[sh].size(), hipMemcpyDeviceToHost, c->st));
  }
  HIPCHK(c, hipStreamSynchronize(c->st));
  std::vector<double> coef((size_t)NS * NB * EIG_MAXSEL, 0.0);
  std::vector<UpdJob> uj((size_t)NS * NB);
  for (int sh = 0; sh < NS; ++sh) {
    char what[64];
    snprintf(what, sizeof what, "stage two, shift %d", sh);
    blm_status s = eig_status(c, info[EIG_INFO * sh], what);
    if (s != BLM_OK) return s;
    const int d = ej[sh].d;
    const double* vr = vecs[sh].data();
    const double* vi = vr + d;
    // alpha = c_0; coefficient of kept row = Re(c_i / alpha)
    const double ar = vr[0], ai = vi[0];
    const double den = ar * ar + ai * ai;
    double nrm = 0.0;
    for (int i = 0; i < d; ++i) nrm += vr[i] * vr[i] + vi[i] * vi[i];
    nrm = std::sqrt(nrm);
    int at = 1;
    for (int b = 0; b < NB; ++b) {
      const int nk = c->nkept[sh * NB + b];
      uj[sh * NB + b].rows = c->eig1[sh * NB + b].out;
      uj[sh * NB + b].n = nk;
      for (int r = 0; r < nk; ++r, ++at)
        coef[((size_t)sh * NB + b) * EIG_MAXSEL + r] = (vr[at] * ar + vi[at] * ai) / den;
    }
    uint32_t fl = 0;
    if (ev[4 * sh + 1] != 0.0) fl |= BLM_FLAG_COMPLEX_ENERGY;
    for (int b = 0; b < NB; ++b)
      if (c->pairkept[sh * NB + b]) fl |= BLM_FLAG_PAIR_KEPT;
    const double ra = std::sqrt(den) / (nrm > 0 ? nrm : 1.0);
    if (ra < 1e-8) fl |= BLM_FLAG_SMALL_ALPHA;
    if (h_energy) h_energy[sh] = ev[4 * sh];
    if (h_alpha) h_alpha[sh] = ra;
    if (h_flags) h_flags[sh] = fl;
  }
  if (d_update) {
    HIPCHK(c, hipMemcpyAsync(c->d_coef, coef.data(), 8 * coef.size(), hipMemcpyHostToDevice, c->st));
    HIPCHK(c, hipMemcpyAsync(c->d_upd, uj.data(), sizeof(UpdJob) * uj.size(), hipMemcpyHostToDevice, c->st));
    hipLaunchKernelGGL(update_kernel, dim3((unsigned)((c->NV + 255) / 256), NS), dim3(256), 0, c->st,
                       d_update, c->NV, NB, NS, dev_offsets(c), c->d_blk_of, c->d_upd, c->d_coef);
    HIPCHK(c, hipGetLastError());
  }
  mark(c, 8, true);
  HIPCHK(c, hipStreamSynchronize(c->st));
  c->state = ST_DONE;
  return BLM_OK;
}

}  // namespace

extern "C" {

blm_status blm_stage2(blm_ctx* c, double* d_update, double* h_energy, double* h_alpha,
                      uint32_t* h_flags) {
  if (!c) return BLM_E_ARG;
  std::vector<EigJob> ej;
  int dm = 1;
  blm_status s = stage2_begin(c, ej, &dm);
  if (s != BLM_OK) return s;
  HIPCHK(c, hipMemcpyAsync(c->d_eig2, ej.data(), sizeof(EigJob) * ej.size(), hipMemcpyHostToDevice, c->st));
  launch_eig(c->d_eig2, (int)ej.size(), c->st);
  HIPCHK(c, hipGetLastError());
  return stage2_end(c, ej, d_update, h_energy, h_alpha, h_flags);
}

blm_status blm_get_block_matrices(blm_ctx* c, int32_t block, int32_t shift, double* h_H, double* h_S,
                                  int32_t* dim) {
  if (!c || !dim) return BLM_E_ARG;
  if (block < 0 || block >= c->NB || shift < 0 || shift >= c->NS) return fail(c, BLM_E_ARG, "bad index");
  if (c->state < ST_BUILT) return fail(c, BLM_E_STATE, "no block estimates yet");
  const int M = (int)(c->off[block + 1] - c->off[block]);
  const int d = M + (int)c->auxlist[block].size();
  *dim = d;
  if (!h_H && !h_S) return BLM_OK;
  AsmJob A{};
  A.d = d;
  A.M = M;
  A.kind = 0;
  A.b = block;
  A.n_aux = (int)c->auxlist[block].size();
  A.delta = c->shifts[shift];
  A.off_b = c->off[block];
  A.acc_off = c->acc_off[block];
  A.aux_idx = c->d_auxlist + (size_t)block * c->auxlist_stride;
  A.S = c->exS;
  A.A = c->exA;
  HIPCHK(c, hipMemcpyAsync(c->d_asm_x, &A, sizeof A, hipMemcpyHostToDevice, c->st));
  hipLaunchKernelGGL(assemble_kernel, dim3(1, 64), dim3(256), 0, c->st, c->d_asm_x, asm_src(c, c->n2max));
  HIPCHK(c, hipGetLastError());
  if (h_H) HIPCHK(c, hipMemcpyAsync(h_H, c->exA, 8 * (size_t)d * d, hipMemcpyDeviceToHost, c->st));
  if (h_S) HIPCHK(c, hipMemcpyAsync(h_S, c->exS, 8 * (size_t)d * d, hipMemcpyDeviceToHost, c->st));
  HIPCHK(c, hipStreamSynchronize(c->st));
  return BLM_OK;
}

blm_status blm_get_directions(blm_ctx* c, int32_t block, int32_t shift, double* h_B, int32_t* n_rows) {
  if (!c || !n_rows) return BLM_E_ARG;
  if (block < 0 || block >= c->NB || shift < 0 || shift >= c->NS) return fail(c, BLM_E_ARG, "bad index");
  if (c->state < ST_SOLVED) return fail(c, BLM_E_STATE, "no directions yet");
  const int i = shift * c->NB + block;
  *n_rows = c->nkept[i];
  if (!h_B) return BLM_OK;
  const int M = (int)(c->off[block + 1] - c->off[block]);
  HIPCHK(c, hipMemcpyAsync(h_B, c->eig1[i].out, 8 * (size_t)c->nkept[i] * M, hipMemcpyDeviceToHost, c->st));
  HIPCHK(c, hipStreamSynchronize(c->st));
  return BLM_OK;
}

blm_status blm_get_stage2_matrices(blm_ctx* c, int32_t shift, double* h_H2, double* h_S2, int32_t* dim) {
  if (!c || !dim) return BLM_E_ARG;
  if (shift < 0 || shift >= c->NS) return fail(c, BLM_E_ARG, "bad index");
  if (c->state < ST_PROJECTED) return fail(c, BLM_E_STATE, "no stage-two estimates yet");
  const int d = (int)c->idx2[shift].size();
  *dim = d;
  if (!h_H2 && !h_S2) return BLM_OK;
  AsmJob A{};
  A.d = d;
  A.kind = 1;
  A.delta = 0.0;
  A.idx2 = c->d_idx2 + (size_t)shift * c->n2max;
  A.S = c->exS;
  A.A = c->exA;
  HIPCHK(c, hipMemcpyAsync(c->d_asm_x, &A, sizeof A, hipMemcpyHostToDevice, c->st));
  hipLaunchKernelGGL(assemble_kernel, dim3(1, 16), dim3(256), 0, c->st, c->d_asm_x, asm_src(c, c->n2));
  HIPCHK(c, hipGetLastError());
  if (h_H2) HIPCHK(c, hipMemcpyAsync(h_H2, c->exA, 8 * (size_t)d * d, hipMemcpyDeviceToHost, c->st));
  if (h_S2) HIPCHK(c, hipMemcpyAsync(h_S2, c->exS, 8 * (size_t)d * d, hipMemcpyDeviceToHost, c->st));
  HIPCHK(c, hipStreamSynchronize(c->st));
  return BLM_OK;
}

blm_status blm_debug_eigvals(const double* d_H, const double* d_S, int32_t d, double* h_evals, void* stream) {
  if (!d_H || !d_S || !h_evals || d < 1 || d > EIG_MAXD) return BLM_E_ARG;
  hipStream_t st = (hipStream_t)stream;
  const size_t bytes = eig_bytes(d, d, 1);
  void *ws = nullptr, *aux = nullptr;
  if (hipMalloc(&ws, bytes) != hipSuccess) return BLM_E_NOMEM;
  if (hipMalloc(&aux, 256 + sizeof(EigJob)) != hipSuccess) {
    (void)hipFree(ws);
    return BLM_E_NOMEM;
  }
  double* q = (double*)ws;
  int32_t* info = (int32_t*)aux;
  double* ev = (double*)((char*)aux + 64);
  EigJob J = carve(q, d, d, 1, EIG_VALUES, 1, 0, info, ev);
  EigJob* dJ = (EigJob*)((char*)aux + 256);
  blm_status r = BLM_OK;
  std::vector<double> wr(d), wi(d);
  int32_t hinfo[4] = {0, 0, 0, 0};
  if (hipMemcpyAsync(J.A, d_H, 8 * (size_t)d * d, hipMemcpyDeviceToDevice, st) != hipSuccess ||
      hipMemcpyAsync(J.S, d_S, 8 * (size_t)d * d, hipMemcpyDeviceToDevice, st) != hipSuccess ||
      hipMemcpyAsync(dJ, &J, sizeof J, hipMemcpyHostToDevice, st) != hipSuccess) {
    r = BLM_E_HIP;
  } else {
    launch_eig(dJ, 1, st);
    if (hipGetLastError() != hipSuccess ||
        hipMemcpyAsync(wr.data(), J.wr, 8 * (size_t)d, hipMemcpyDeviceToHost, st) != hipSuccess ||
        hipMemcpyAsync(wi.data(), J.wi, 8 * (size_t)d, hipMemcpyDeviceToHost, st) != hipSuccess ||
        hipMemcpyAsync(hinfo, info, 16, hipMemcpyDeviceToHost, st) != hipSuccess ||
        hipStreamSynchronize(st) != hipSuccess)
      r = BLM_E_HIP;
  }
  (void)hipFree(ws);
  (void)hipFree(aux);
  if (r != BLM_OK) return r;
  if (hinfo[0] == EIG_NOT_PD) return BLM_E_S_NOT_PD;
  if (hinfo[0] == EIG_NONFINITE) return BLM_E_NONFINITE;
  if (hinfo[0] == EIG_NOCONV) return BLM_E_NOCONV;
  for (int i = 0; i < d; ++i) {
    h_evals[2 * i] = wr[i];
    h_evals[2 * i + 1] = wi[i];
  }
  return BLM_OK;
}

// ------------------------------------------------------------------ batches --
// Several contexts (independent optimisations) whose block solves, and whose
// stage-two solves, share one eigensolver launch each.
struct blm_batch {
  std::vector<blm_ctx*> ctx;
  hipStream_t st = nullptr;
  int n_cus = 0;
  unsigned spin_limit = 1u << 22;
  int hess_wg = 32;
  EigJob* d_eig1 = nullptr;   // every context's block pencils
  EigJob* d_eig2 = nullptr;   // every context's stage-two pencils
  unsigned* d_hbar = nullptr; // barrier counter and flag per block pencil
  // one Gram launch for every context's build (same storage, energy target):
  // the contexts' job tables concatenated, each job tagged with its
  // context's slice set; partial tiles of all jobs in one buffer
  bool merged = false;
  int kind = 0;                 // 0 FP64, 2 BF16 split, 3 FP8
  int pieces = 0, fp8_res = 0, P = 1;
  GramJob *d_jobs1 = nullptr, *d_jobsM = nullptr;
  PairJob* d_pairsM = nullptr;
  int n_jobs1 = 0, n_jobsM = 0, n_pairsM = 0, n_strip_pairsM = 0;
  std::vector<int> off1, offM;  // first job of each context in the merged tables
  Slice* d_slices = nullptr;
  int max_slices = 0;
  int2* d_sets = nullptr;
  double* partial = nullptr;
  std::vector<Slice> h_slices;
  std::vector<int2> h_sets;
  // one projection launch and one stage-two Gram launch for every context
  ProjChunk* d_pchunks = nullptr;
  std::vector<ProjChunk> h_pchunks;
  GramJob* d_jobs2 = nullptr;   // the contexts' stage-two jobs, set per call
  int P2 = 1;                   // slice groups of the stage-two launch
  size_t partial_slots = 0;
};

blm_status blm_batch_create(blm_ctx* const* ctxs, int32_t n, blm_batch** out) {
  if (!ctxs || !out || n < 1) return BLM_E_ARG;
  *out = nullptr;
  int n1 = 0, n2 = 0;
  for (int i = 0; i < n; ++i) {
    if (!ctxs[i]) return BLM_E_ARG;
    if (ctxs[i]->st != ctxs[0]->st || ctxs[i]->device != ctxs[0]->device) return BLM_E_ARG;
    for (int j = 0; j < i; ++j)
      if (ctxs[j] == ctxs[i]) return BLM_E_ARG;
    n1 += ctxs[i]->NS * ctxs[i]->NB;
    n2 += ctxs[i]->NS;
  }
  blm_batch* b = new blm_batch;
  b->ctx.assign(ctxs, ctxs + n);
  b->st = ctxs[0]->st;
  b->n_cus = ctxs[0]->n_cus;
  b->spin_limit = ctxs[0]->spin_limit;
  b->hess_wg = ctxs[0]->hess_wg;
  if (hipMalloc((void**)&b->d_eig1, sizeof(EigJob) * n1) != hipSuccess ||
      hipMalloc((void**)&b->d_eig2, sizeof(EigJob) * n2) != hipSuccess ||
      hipMalloc((void**)&b->d_hbar, 4 * 2 * (size_t)n1) != hipSuccess) {
    (void)hipFree(b->d_eig1);
    (void)hipFree(b->d_eig2);
    (void)hipFree(b->d_hbar);
    delete b;
    return BLM_E_NOMEM;
  }
  // merged build tables when every context builds with the same kernels
  bool same = true;
  for (int i = 0; i < n; ++i) {
    const blm_ctx* c = ctxs[i];
    same = same && c->target == BLM_TARGET_ENERGY && c->pieces == ctxs[0]->pieces && c->fp8 == ctxs[0]->fp8 &&
           c->fp8_res == ctxs[0]->fp8_res;
  }
  if (same) {
    std::vector<GramJob> j1, jm;
    std::vector<PairJob> strip_pairs, plain_pairs;
    for (int i = 0; i < n; ++i) {
      const blm_ctx* c = ctxs[i];
      b->off1.push_back((int)j1.size());
      b->offM.push_back((int)jm.size());
      for (GramJob J : c->h_jobs1) {
        J.set = i;
        j1.push_back(J);
      }
      const int om = (int)jm.size();
      for (GramJob J : c->h_jobsM) {
        J.set = i;
        jm.push_back(J);
      }
      for (int k = 0; k < (int)c->h_pairsM.size(); ++k) {
        PairJob pj = c->h_pairsM[k];
        pj.ja += om;
        if (pj.jb >= 0) pj.jb += om;
        (k < c->n_strip_pairsM ? strip_pairs : plain_pairs).push_back(pj);
      }
      b->max_slices += c->max_slices;
    }
    std::vector<PairJob> pairs = strip_pairs;
    pairs.insert(pairs.end(), plain_pairs.begin(), plain_pairs.end());
    b->kind = ctxs[0]->fp8 ? 3 : ctxs[0]->pieces ? 2 : 0;
    b->pieces = ctxs[0]->pieces;
    b->fp8_res = ctxs[0]->fp8_res;
    b->n_jobs1 = (int)j1.size();
    b->n_jobsM = (int)jm.size();
    b->n_pairsM = (int)pairs.size();
    b->n_strip_pairsM = (int)strip_pairs.size();
    // slice groups: about 4,096 workgroups in the largest launch
    const int nj = std::max(b->n_jobs1, b->n_jobsM);
    b->P = std::max(1, std::min(64, (4096 + nj - 1) / nj));
    // stage two: at most every context's largest job table
    int nj2 = 0;
    for (int i = 0; i < n; ++i) {
      const int T2 = (ctxs[i]->n2max + GT - 1) / GT;
      nj2 += T2 * (T2 + 1) / 2;
    }
    b->P2 = std::max(1, std::min(512, (4096 + nj2 - 1) / nj2));
    const size_t slots = std::max((size_t)nj * b->P, (size_t)nj2 * b->P2);
    b->partial_slots = slots;
    size_t n_pchunks = 0;
    for (int i = 0; i < n; ++i) n_pchunks += MAX_CHUNKS;
    bool ok = hipMalloc((void**)&b->d_jobs1, sizeof(GramJob) * std::max<size_t>(j1.size(), 1)) == hipSuccess &&
              hipMalloc((void**)&b->d_jobsM, sizeof(GramJob) * std::max<size_t>(jm.size(), 1)) == hipSuccess &&
              hipMalloc((void**)&b->d_pairsM, sizeof(PairJob) * std::max<size_t>(pairs.size(), 1)) == hipSuccess &&
              hipMalloc((void**)&b->d_slices, sizeof(Slice) * (size_t)b->max_slices) == hipSuccess &&
              hipMalloc((void**)&b->d_sets, sizeof(int2) * (size_t)n) == hipSuccess &&
              hipMalloc((void**)&b->d_pchunks, sizeof(ProjChunk) * n_pchunks) == hipSuccess &&
              hipMalloc((void**)&b->d_jobs2, sizeof(GramJob) * (size_t)nj2) == hipSuccess &&
              hipMalloc((void**)&b->partial, 8 * slots * 3 * GT * GT) == hipSuccess;
    ok = ok && hipMemcpy(b->d_jobs1, j1.data(), sizeof(GramJob) * j1.size(), hipMemcpyHostToDevice) == hipSuccess;
    if (ok && !jm.empty())
      ok = hipMemcpy(b->d_jobsM, jm.data(), sizeof(GramJob) * jm.size(), hipMemcpyHostToDevice) == hipSuccess &&
           hipMemcpy(b->d_pairsM, pairs.data(), sizeof(PairJob) * pairs.size(), hipMemcpyHostToDevice) == hipSuccess;
    if (!ok) {
      (void)hipGetLastError();
      blm_batch_destroy(b);
      return BLM_E_NOMEM;
    }
    b->merged = true;
  }
  *out = b;
  return BLM_OK;
}

blm_status blm_batch_destroy(blm_batch* b) {
  if (!b) return BLM_E_ARG;
  (void)hipFree(b->d_eig1);
  (void)hipFree(b->d_eig2);
  (void)hipFree(b->d_hbar);
  (void)hipFree(b->d_jobs1);
  (void)hipFree(b->d_jobsM);
  (void)hipFree(b->d_pairsM);
  (void)hipFree(b->d_slices);
  (void)hipFree(b->d_sets);
  (void)hipFree(b->partial);
  (void)hipFree(b->d_pchunks);
  (void)hipFree(b->d_jobs2);
  delete b;
  return BLM_OK;
}

blm_status blm_batch_build(blm_batch* b, const blm_chunk* const* chunks, const int32_t* n_chunks) {
  if (!b || !chunks || !n_chunks) return BLM_E_ARG;
  const int n = (int)b->ctx.size();
  blm_ctx* c0 = b->ctx[0];
  if (!b->merged)
    return fail(c0, BLM_E_ARG, "a batched build needs contexts of one storage and the energy target");
  std::vector<int64_t> tot(n, 0);
  for (int i = 0; i < n; ++i) {
    blm_ctx* c = b->ctx[i];
    if (c->state != ST_BEGUN && c->state != ST_BUILT)
      return fail(c, BLM_E_STATE, "blm_batch_build needs blm_begin_step first");
    blm_status s = check_chunks(c, chunks[i], n_chunks[i], &tot[i]);
    if (s != BLM_OK) return s;
  }
  // every context's aux columns and slice table, then one table of all
  b->h_slices.clear();
  b->h_sets.assign(n, make_int2(0, 0));
  bool vec = true;
  for (int i = 0; i < n; ++i) {
    blm_ctx* c = b->ctx[i];
    blm_status s = build_slices(c, chunks[i], n_chunks[i]);
    if (s != BLM_OK) return s;
    b->h_sets[i] = make_int2((int)b->h_slices.size(), (int)c->h_slices.size());
    b->h_slices.insert(b->h_slices.end(), c->h_slices.begin(), c->h_slices.end());
    vec = vec && c->offsets_even;
  }
  for (const Slice& S : b->h_slices)
    if ((S.ld & 1) || ((uintptr_t)S.O & 15) || ((uintptr_t)S.e & 15)) vec = false;
  if ((int)b->h_slices.size() > b->max_slices) return fail(c0, BLM_E_ARG, "too many slices in one call");
  if (b->h_slices.empty()) return BLM_OK;
  HIPCHK(c0, hipMemcpyAsync(b->d_slices, b->h_slices.data(), sizeof(Slice) * b->h_slices.size(),
                            hipMemcpyHostToDevice, b->st));
  HIPCHK(c0, hipMemcpyAsync(b->d_sets, b->h_sets.data(), sizeof(int2) * n, hipMemcpyHostToDevice, b->st));
  const int P = b->P;
  const size_t tile = (size_t)3 * GT * GT;
  for (blm_ctx* c : b->ctx) mark(c, 1, false);
  // the FP64 jobs, or the mixed builds' FP64 aux and further-strip jobs
  launch_gram(b->d_jobs1, b->n_jobs1, b->d_slices, 0, P, b->kind == 0 && vec, b->kind != 0, false, b->partial,
              b->st, b->d_sets);
  HIPCHK(c0, hipGetLastError());
  for (int i = 0; i < n; ++i) {
    blm_ctx* c = b->ctx[i];
    launch_gram_reduce(c->d_jobs1, c->n_jobs1, P, b->partial + (size_t)b->off1[i] * P * tile, c->accS, c->accH,
                       c->strips, c->NV, c->NAP, b->st);
  }
  if (b->kind != 0 && b->n_pairsM > 0) {
    // the mixed-precision block tiles, in pairs
    if (b->kind == 2)
      launch_gram_bf16(b->d_pairsM, b->n_strip_pairsM, b->n_pairsM, b->d_jobsM, b->d_slices, 0, P, b->pieces,
                       b->partial, b->st, b->d_sets);
    else
      launch_gram_fp8(b->d_pairsM, b->n_strip_pairsM, b->n_pairsM, b->d_jobsM, b->d_slices, 0, P, b->fp8_res,
                      b->partial, b->st, b->d_sets);
    HIPCHK(c0, hipGetLastError());
    for (int i = 0; i < n; ++i) {
      blm_ctx* c = b->ctx[i];
      launch_gram_reduce(c->d_jobsM, c->n_jobsM, P, b->partial + (size_t)b->offM[i] * P * tile, c->accS, c->accH,
                         c->strips, c->NV, c->NAP, b->st);
    }
  }
  HIPCHK(c0, hipGetLastError());
  for (blm_ctx* c : b->ctx) mark(c, 1, true);
  for (int i = 0; i < n; ++i) {
    b->ctx[i]->n_pass1 += tot[i];
    b->ctx[i]->state = ST_BUILT;
  }
  return BLM_OK;
}

blm_status blm_batch_project(blm_batch* b, const blm_chunk* const* chunks, const int32_t* n_chunks) {
  if (!b || !chunks || !n_chunks) return BLM_E_ARG;
  const int n = (int)b->ctx.size();
  blm_ctx* c0 = b->ctx[0];
  if (!b->merged)
    return fail(c0, BLM_E_ARG, "a batched projection needs contexts of one storage and the energy target");
  std::vector<int64_t> tot(n, 0);
  for (int i = 0; i < n; ++i) {
    blm_ctx* c = b->ctx[i];
    if (c->state != ST_SOLVED && c->state != ST_PROJECTED)
      return fail(c, BLM_E_STATE, "blm_batch_project needs the block solves first");
    blm_status s = check_chunks(c, chunks[i], n_chunks[i], &tot[i]);
    if (s != BLM_OK) return s;
  }
  // every context's samples onto its kept directions, in one launch
  b->h_pchunks.clear();
  int tiles = 0, max_nd = 0;
  bool vec = true;
  for (int i = 0; i < n; ++i) {
    blm_ctx* c = b->ctx[i];
    add_pchunks(c, chunks[i], n_chunks[i], c->d_dir2_blk, c->NB, c->d_dir2_ptr, c->d_dir2_wptr, c->n2 - 1, c->Yp,
                c->Zp, c->ld2,
                b->h_pchunks, &tiles, &vec);
    max_nd = std::max(max_nd, c->nd2max);
  }
  for (blm_ctx* c : b->ctx) mark(c, 5, false);
  if (!b->h_pchunks.empty()) {
    HIPCHK(c0, hipMemcpyAsync(b->d_pchunks, b->h_pchunks.data(), sizeof(ProjChunk) * b->h_pchunks.size(),
                              hipMemcpyHostToDevice, b->st));
    const int store = store_kind(c0);
    launch_dirproj(b->d_pchunks, (int)b->h_pchunks.size(), tiles, vec && store == STORE_F64, store, max_nd, b->st);
    HIPCHK(c0, hipGetLastError());
  }
  for (blm_ctx* c : b->ctx) mark(c, 5, true);
  // the stage-two sums of every context in one Gram launch: each job reads
  // its own context's slices of projected samples
  b->h_slices.clear();
  b->h_sets.assign(n, make_int2(0, 0));
  std::vector<GramJob> jobs;
  std::vector<int> off(n, 0);
  for (int i = 0; i < n; ++i) {
    blm_ctx* c = b->ctx[i];
    proj_slices(c, chunks[i], n_chunks[i]);
    b->h_sets[i] = make_int2((int)b->h_slices.size(), (int)c->h_slices.size());
    b->h_slices.insert(b->h_slices.end(), c->h_slices.begin(), c->h_slices.end());
    off[i] = (int)jobs.size();
    for (GramJob J : c->h_jobs2) {
      J.set = i;
      jobs.push_back(J);
    }
  }
  bool vec2 = true;
  for (const Slice& S : b->h_slices)
    if ((S.ld & 1) || ((uintptr_t)S.O & 15) || ((uintptr_t)S.e & 15)) vec2 = false;
  if ((int)b->h_slices.size() > b->max_slices) return fail(c0, BLM_E_ARG, "too many slices in one call");
  const int P2 = std::max(1, std::min(b->P2, (4096 + (int)jobs.size() - 1) / std::max(1, (int)jobs.size())));
  if ((size_t)jobs.size() * P2 > b->partial_slots) return fail(c0, BLM_E_ARG, "stage-two tables exceed the plan");
  if (!b->h_slices.empty() && !jobs.empty()) {
    HIPCHK(c0, hipMemcpyAsync(b->d_slices, b->h_slices.data(), sizeof(Slice) * b->h_slices.size(),
                              hipMemcpyHostToDevice, b->st));
    HIPCHK(c0, hipMemcpyAsync(b->d_sets, b->h_sets.data(), sizeof(int2) * n, hipMemcpyHostToDevice, b->st));
    HIPCHK(c0, hipMemcpyAsync(b->d_jobs2, jobs.data(), sizeof(GramJob) * jobs.size(), hipMemcpyHostToDevice,
                              b->st));
    const size_t tile = (size_t)3 * GT * GT;
    for (blm_ctx* c : b->ctx) mark(c, 6, false);
    launch_gram(b->d_jobs2, (int)jobs.size(), b->d_slices, 0, P2, vec2, false, true, b->partial, b->st, b->d_sets);
    HIPCHK(c0, hipGetLastError());
    for (blm_ctx* c : b->ctx) {
      mark(c, 6, true);
      mark(c, 7, false);
    }
    for (int i = 0; i < n; ++i) {
      blm_ctx* c = b->ctx[i];
      launch_gram_reduce(c->d_jobs2, c->n_jobs2, P2, b->partial + (size_t)off[i] * P2 * tile, c->G2S, c->G2H,
                         nullptr, c->NV, c->NAP, b->st);
    }
    HIPCHK(c0, hipGetLastError());
    for (blm_ctx* c : b->ctx) mark(c, 7, true);
  }
  for (int i = 0; i < n; ++i) {
    b->ctx[i]->n_pass2 += tot[i];
    b->ctx[i]->state = ST_PROJECTED;
  }
  return BLM_OK;
}

blm_status blm_batch_solve_blocks(blm_batch* b, double* const* h_evals, int32_t* const* h_kept) {
  if (!b) return BLM_E_ARG;
  const int n = (int)b->ctx.size();
  std::vector<EigJob> all;
  int dm = 1;
  for (int i = 0; i < n; ++i) {
    std::vector<EigJob> ej;
    int d = 1;
    blm_status s = solve_begin(b->ctx[i], ej, &d);
    if (s != BLM_OK) return s;
    all.insert(all.end(), ej.begin(), ej.end());
    dm = std::max(dm, d);
  }
  blm_ctx* c0 = b->ctx[0];
  for (blm_ctx* c : b->ctx) mark(c, 4, false);
  launch_eig_split(all.data(), b->d_eig1, (int)all.size(), dm, b->n_cus, b->hess_wg, b->d_hbar, b->spin_limit,
                   b->st);
  HIPCHK(c0, hipGetLastError());
  for (blm_ctx* c : b->ctx) mark(c, 4, true);
  blm_status first = BLM_OK;
  for (int i = 0; i < n; ++i) {
    const blm_status s = solve_end(b->ctx[i], h_evals ? h_evals[i] : nullptr, h_kept ? h_kept[i] : nullptr);
    if (s != BLM_OK && first == BLM_OK) first = s;
  }
  return first;
}

blm_status blm_batch_stage2(blm_batch* b, double* const* d_update, double* const* h_energy,
                            double* const* h_alpha, uint32_t* const* h_flags) {
  if (!b) return BLM_E_ARG;
  const int n = (int)b->ctx.size();
  std::vector<std::vector<EigJob>> per(n);
  std::vector<EigJob> all;
  for (int i = 0; i < n; ++i) {
    int d = 1;
    blm_status s = stage2_begin(b->ctx[i], per[i], &d);
    if (s != BLM_OK) return s;
    all.insert(all.end(), per[i].begin(), per[i].end());
  }
  blm_ctx* c0 = b->ctx[0];
  HIPCHK(c0, hipMemcpyAsync(b->d_eig2, all.data(), sizeof(EigJob) * all.size(), hipMemcpyHostToDevice, b->st));
  launch_eig(b->d_eig2, (int)all.size(), b->st);
  HIPCHK(c0, hipGetLastError());
  blm_status first = BLM_OK;
  for (int i = 0; i < n; ++i) {
    const blm_status s = stage2_end(b->ctx[i], per[i], d_update ? d_update[i] : nullptr,
                                    h_energy ? h_energy[i] : nullptr, h_alpha ? h_alpha[i] : nullptr,
                                    h_flags ? h_flags[i] : nullptr);
    if (s != BLM_OK && first == BLM_OK) first = s;
  }
  return first;
}

}  // extern "C"
