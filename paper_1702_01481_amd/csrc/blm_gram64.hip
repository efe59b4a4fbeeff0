// Block build on FP64 samples, two tile jobs per workgroup (gfx950).
//
// The products are those of gram_kernel (Eq. 3 on the one-block basis of
// Eq. 4 / Eq. 10): for an off-diagonal tile (i, j), S_ij = O_i^T W O_j,
// H_ij = O_i^T W e_j and H_ji^T = e_i^T W O_j; for a diagonal tile S_ii,
// H_ii and the coupling strips of Fig. 1 for the first 16 aux columns
// (aux^T W O_i, aux^T W e_i, auxE^T W O_i).  One workgroup takes a pair of
// tile jobs that share their row tile i, as the mixed-precision kernels do:
// the row panels {O_i, e_i} are read once for both, so a sample stage reads
// six 64-column panels for two jobs instead of eight.  Samples are read
// through registers, two 16-sample stages ahead of the one in LDS, and the
// weights are applied (and ragged columns and rows past a slice zeroed)
// when a stage is stored.  FP64 matrix cores (v_mfma_f64_16x16x4f64),
// partial tiles per slice group as gram_kernel writes them, summed by the
// same fixed-order reduction.
#include "blm_internal.h"

namespace blm {
namespace {

typedef double d4p __attribute__((ext_vector_type(4)));

__device__ __forceinline__ d4p mfma64(double a, double b, d4p c) {
  // lane l supplies A[l%16][l/16] and B[l/16][l%16]; register r of lane l
  // holds D[4 r + l/16][l%16]
  return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
}

constexpr int PT = 512;     // threads: eight waves, 2 x 4 over 64 rows x 128 columns
constexpr int PK = 16;      // samples per stage

struct PairLds {
  double A[2][2][PK][GT];     // [buffer][O_i * w, e_i * w][sample][column]
  double B[2][4][PK][GT];     // [buffer][O_j, e_j, O_j', e_j'][sample][column]
  double X[2][2][PK][NAUX];   // [buffer][aux * w, auxE * w][sample][aux column] (strip pairs)
};

// One thread's share of a stage: sample row lr = tid / 32, columns
// 2 (tid % 32) and the next one of each of the six panels; for strip pairs
// one aux value (tid % 32 < 16: Xa, else Ya, column tid % 16).
struct PairRegs {
  double v[6][2];
  double x;
  double w;
  bool valid;
};

// two consecutive columns c, c + 1 of a sample row (clamped into the tile's
// valid columns [0, n)); one 16-byte load when aligned
__device__ __forceinline__ void ld_cols(const BLM_GLOBAL double* row, int64_t c0, int c, int n, bool al,
                                        double& x, double& y) {
  if (al && c + 1 < n) {
    const double2 t = *reinterpret_cast<const BLM_GLOBAL double2*>(row + c0 + c);
    x = t.x;
    y = t.y;
  } else {
    x = row[c0 + min(c, n - 1)];
    y = row[c0 + min(c + 1, n - 1)];
  }
}

struct PairCursor {
  Slice S;
  int si;
  int64_t ro;
};

__device__ __forceinline__ void pc_skip(PairCursor& c, const Slice* __restrict__ slices, int n_slices, int P) {
  while (c.si < n_slices) {
    c.S = slices[c.si];
    if (c.S.n > 0) return;
    c.si += P;
  }
}

__device__ __forceinline__ void pc_next(PairCursor& c, const Slice* __restrict__ slices, int n_slices, int P) {
  c.ro += PK;
  if (c.ro >= c.S.n) {
    c.ro = 0;
    c.si += P;
    pc_skip(c, slices, n_slices, P);
  }
}

template <bool STRIPS>
__global__ __launch_bounds__(PT, 1) void gram64_pair_kernel(const PairJob* __restrict__ pairs, int n_pairs,
                                                           const GramJob* __restrict__ jobs,
                                                           const Slice* __restrict__ slices, int n_slices,
                                                           int P, double* __restrict__ partial,
    const int2* __restrict__ sets) {
  __shared__ PairLds L;
  // XCD-aware order (as gram_kernel): each XCD takes a contiguous range of
  // (slice group, pair) work items
  const int G = gridDim.x, g = blockIdx.x;
  const int q = G >> 3, r = G & 7, xcd = g & 7, idx = g >> 3;
  const int wid = (xcd < r) ? xcd * (q + 1) + idx : r * (q + 1) + (xcd - r) * q + idx;
  const int p = wid / n_pairs, pid = wid % n_pairs;
  const PairJob PJ = pairs[pid];
  const GramJob JA = jobs[PJ.ja];
  const bool has_b = PJ.jb >= 0;
  const GramJob JB = jobs[has_b ? PJ.jb : PJ.ja];
  if (sets) {
    const int2 ss = sets[JA.set];
    slices += ss.x;
    n_slices = ss.y;
  }
  const bool pair_strips = STRIPS && JA.kind == JOB_DIAG;

  const int tid = threadIdx.x, lane = tid & 63;
  const int wv = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int i16 = lane & 15, k4 = lane >> 4;
  const int wr = wv & 1, wc = wv >> 1;          // 2 x 4 waves over 64 x 128
  const bool wave_b = wc >= 2;
  const bool wave_on = !wave_b || has_b;
  const bool strip = pair_strips && !wave_b;    // the diagonal tile's waves compute the strips
  const GramJob& JW = wave_b ? JB : JA;
  const bool third = JW.kind == JOB_OFF;

  // loads: this thread's sample row and column pair
  const int lr = tid >> 5, lc = 2 * (tid & 31);
  const int xcol = tid & 15;
  const bool xy = (tid & 31) >= 16;
  const int na = JA.mi, nb0 = JA.nj, nb1 = JB.nj;

  auto load = [&](const PairCursor& C, PairRegs& R) {
    const Slice& S = C.S;
    const int64_t row = C.ro + lr;
    R.valid = row < S.n;
    const int64_t rc = R.valid ? row : S.n - 1;
    R.w = S.w ? as_global(S.w)[rc] : 1.0;
    const BLM_GLOBAL double* rO = as_global((const double*)S.O) + rc * S.ld;
    const BLM_GLOBAL double* rE = as_global((const double*)S.e) + rc * S.ld;
    const bool al = ((S.ld & 1) == 0) && (((uintptr_t)S.O & 15) == 0) && (((uintptr_t)S.e & 15) == 0);
    const bool ala = al && (JA.ci & 1) == 0, alb0 = al && (JA.cj & 1) == 0, alb1 = al && (JB.cj & 1) == 0;
    ld_cols(rO, JA.ci, lc, na, ala, R.v[0][0], R.v[0][1]);
    ld_cols(rE, JA.ci, lc, na, ala, R.v[1][0], R.v[1][1]);
    ld_cols(rO, JA.cj, lc, nb0, alb0, R.v[2][0], R.v[2][1]);
    ld_cols(rE, JA.cj, lc, nb0, alb0, R.v[3][0], R.v[3][1]);
    ld_cols(rO, JB.cj, lc, nb1, alb1, R.v[4][0], R.v[4][1]);
    ld_cols(rE, JB.cj, lc, nb1, alb1, R.v[5][0], R.v[5][1]);
    if (pair_strips) R.x = as_global(xy ? S.Ya : S.Xa)[rc * S.ald + JA.ag + xcol];
  };
  auto store = [&](const PairRegs& R, int b) {
    const double w = R.valid ? R.w : 0.0;
    const bool oka0 = lc < na, oka1 = lc + 1 < na;
    L.A[b][0][lr][lc] = oka0 ? R.v[0][0] * w : 0.0;
    L.A[b][0][lr][lc + 1] = oka1 ? R.v[0][1] * w : 0.0;
    L.A[b][1][lr][lc] = oka0 ? R.v[1][0] * w : 0.0;
    L.A[b][1][lr][lc + 1] = oka1 ? R.v[1][1] * w : 0.0;
    const bool okb0 = lc < nb0, okb1 = lc + 1 < nb0, okc0 = lc < nb1, okc1 = lc + 1 < nb1;
    L.B[b][0][lr][lc] = okb0 ? R.v[2][0] : 0.0;
    L.B[b][0][lr][lc + 1] = okb1 ? R.v[2][1] : 0.0;
    L.B[b][1][lr][lc] = okb0 ? R.v[3][0] : 0.0;
    L.B[b][1][lr][lc + 1] = okb1 ? R.v[3][1] : 0.0;
    L.B[b][2][lr][lc] = okc0 ? R.v[4][0] : 0.0;
    L.B[b][2][lr][lc + 1] = okc1 ? R.v[4][1] : 0.0;
    L.B[b][3][lr][lc] = okc0 ? R.v[5][0] : 0.0;
    L.B[b][3][lr][lc + 1] = okc1 ? R.v[5][1] : 0.0;
    if (pair_strips) L.X[b][xy ? 1 : 0][lr][xcol] = R.x * w;
  };

  d4p P0[2][2], P1[2][2], P2[2][2];
#pragma unroll
  for (int x = 0; x < 2; ++x)
#pragma unroll
    for (int y = 0; y < 2; ++y) {
      P0[x][y] = d4p{0, 0, 0, 0};
      P1[x][y] = d4p{0, 0, 0, 0};
      P2[x][y] = d4p{0, 0, 0, 0};
    }
  // this wave's column panels: the pair's first or second column tile
  const int bo = wave_b ? 2 : 0;
  const int c0 = 32 * (wc & 1);
  auto compute = [&](int b) {
#pragma unroll
    for (int kk = 0; kk < PK; kk += 4) {
      const int kr = kk + k4;
      const double a0 = L.A[b][0][kr][32 * wr + i16], a1 = L.A[b][0][kr][32 * wr + 16 + i16];
      const double b0 = L.B[b][bo][kr][c0 + i16], b1 = L.B[b][bo][kr][c0 + 16 + i16];
      const double f0 = L.B[b][bo + 1][kr][c0 + i16], f1 = L.B[b][bo + 1][kr][c0 + 16 + i16];
      P0[0][0] = mfma64(a0, b0, P0[0][0]);
      P0[0][1] = mfma64(a0, b1, P0[0][1]);
      P0[1][0] = mfma64(a1, b0, P0[1][0]);
      P0[1][1] = mfma64(a1, b1, P0[1][1]);
      P1[0][0] = mfma64(a0, f0, P1[0][0]);
      P1[0][1] = mfma64(a0, f1, P1[0][1]);
      P1[1][0] = mfma64(a1, f0, P1[1][0]);
      P1[1][1] = mfma64(a1, f1, P1[1][1]);
      if (STRIPS && strip) {
        // strips, 16 aux rows x 32 columns each: wr = 0: aux^T W O_i (P2[0]),
        // aux^T W e_i (P2[1]); wr = 1: auxE^T W O_i (P2[0])
        const double xs = L.X[b][wr][kr][i16];
        P2[0][0] = mfma64(xs, b0, P2[0][0]);
        P2[0][1] = mfma64(xs, b1, P2[0][1]);
        P2[1][0] = mfma64(xs, f0, P2[1][0]);
        P2[1][1] = mfma64(xs, f1, P2[1][1]);
      } else {
        const double e0 = L.A[b][1][kr][32 * wr + i16], e1 = L.A[b][1][kr][32 * wr + 16 + i16];
        P2[0][0] = mfma64(e0, b0, P2[0][0]);
        P2[0][1] = mfma64(e0, b1, P2[0][1]);
        P2[1][0] = mfma64(e1, b0, P2[1][0]);
        P2[1][1] = mfma64(e1, b1, P2[1][1]);
      }
    }
  };

  int n_stages = 0;
  for (int s = p; s < n_slices; s += P) n_stages += (int)((slices[s].n + PK - 1) / PK);

  // two stages in registers ahead of the one in LDS (as gram_kernel)
  PairCursor cur;
  cur.si = p;
  cur.ro = 0;
  pc_skip(cur, slices, n_slices, P);
  PairRegs R0, R1;
  if (n_stages > 0) {
    load(cur, R0);
    pc_next(cur, slices, n_slices, P);
    store(R0, 0);
  }
  if (n_stages > 1) {
    load(cur, R1);
    pc_next(cur, slices, n_slices, P);
  }
  __syncthreads();
  int buf = 0, t = 0;
  for (; t + 2 < n_stages; t += 2) {
    load(cur, R0);                                // stage t + 2
    pc_next(cur, slices, n_slices, P);
    if (wave_on) compute(buf);
    store(R1, buf ^ 1);                           // stage t + 1
    __syncthreads();
    buf ^= 1;
    if (t + 3 < n_stages) {
      load(cur, R1);                              // stage t + 3
      pc_next(cur, slices, n_slices, P);
    }
    if (wave_on) compute(buf);
    store(R0, buf ^ 1);                           // stage t + 2
    __syncthreads();
    buf ^= 1;
  }
  if (t + 1 < n_stages) {
    if (wave_on) compute(buf);
    store(R1, buf ^ 1);
    __syncthreads();
    buf ^= 1;
  }
  if (n_stages > 0 && wave_on) compute(buf);

  if (!wave_on) return;
  const int jw = wave_b ? PJ.jb : PJ.ja;
  BLM_GLOBAL double* base = as_global(partial) + ((size_t)jw * P + p) * (size_t)(3 * GT * GT);
#pragma unroll
  for (int x = 0; x < 2; ++x)
#pragma unroll
    for (int y = 0; y < 2; ++y)
#pragma unroll
      for (int rr = 0; rr < 4; ++rr) {
        const int row = 32 * wr + 16 * x + 4 * rr + k4;
        const int col = c0 + 16 * y + i16;
        base[row * GT + col] = P0[x][y][rr];
        base[GT * GT + row * GT + col] = P1[x][y][rr];
        if (third) base[2 * GT * GT + row * GT + col] = P2[x][y][rr];
      }
  if (STRIPS && strip) {
    // strips [3][NAUX][GT] in the third slot: 0 aux^T O, 1 aux^T e, 2 auxE^T O
#pragma unroll
    for (int y = 0; y < 2; ++y)
#pragma unroll
      for (int rr = 0; rr < 4; ++rr) {
        const int a = 4 * rr + k4;
        const int col = c0 + 16 * y + i16;
        if (wr == 0) {
          base[2 * GT * GT + 0 * NAUX * GT + a * GT + col] = P2[0][y][rr];
          base[2 * GT * GT + 1 * NAUX * GT + a * GT + col] = P2[1][y][rr];
        } else {
          base[2 * GT * GT + 2 * NAUX * GT + a * GT + col] = P2[0][y][rr];
        }
      }
  }
}

}  // namespace

void launch_gram64_pairs(const PairJob* d_pairs, int n_strip_pairs, int n_pairs, const GramJob* d_jobs,
                         const Slice* d_slices, int n_slices, int P, double* d_partial, hipStream_t st,
                         const int2* d_sets) {
  const int n_plain = n_pairs - n_strip_pairs;
  if (n_strip_pairs > 0)
    hipLaunchKernelGGL(gram64_pair_kernel<true>, dim3(n_strip_pairs * P), dim3(PT), 0, st, d_pairs, n_strip_pairs,
                       d_jobs, d_slices, n_slices, P, d_partial, d_sets);
  if (n_plain > 0)
    hipLaunchKernelGGL(gram64_pair_kernel<false>, dim3(n_plain * P), dim3(PT), 0, st, d_pairs + n_strip_pairs,
                       n_plain, d_jobs, d_slices, n_slices, P, d_partial, d_sets);
}

}  // namespace blm
