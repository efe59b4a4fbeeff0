// Mixed-precision block build from FP8 storage on the matrix cores of gfx950.
//
// A sample value x of column c of a chunk is stored as x = s_c (q + r), or
// with a second BF16 residual t of what r leaves, x = s_c (q + r + t):
// s_c a power of two per column and chunk (the smallest with max |x| / s_c <=
// 448), q an OCP e4m3 code (round to nearest even, saturating at 448) and r
// the BF16 rounding of the exact remainder x / s_c - q.  The stored value is
// within 2^-13 of x relative (normal range of q).
//
// A product x y is s_x s_y (q_x q_y + q_x r_y + r_x q_y + r_x r_y), all four
// terms on the BF16 matrix core (v_mfma_f32_16x16x32_bf16) with q converted to
// BF16 exactly (every e4m3 value is a BF16 value).  The FP8 matrix core is not
// used for the code product: measured on gfx950, it sums its 32 products only
// to about 2^-12 of the largest one (unbiased), which moved the block matrices
// by about 4e-6, while the BF16 instruction sums to near FP32 accuracy (each
// piece product is exact in FP32).  FP32 accumulators are scaled by s_x s_y (exact) and added into FP64
// registers every 256 samples and at every slice boundary (scales change
// with the chunk).  These are the block estimates of Eq. 3 on the one-block basis
// (Eq. 4 / Eq. 10), including the coupling strips of Fig. 1 for the first 16
// aux columns (wave function and previous directions), which are stored the
// same way per chunk; the aux Gram and further aux groups' strips run on the
// FP64 kernel.
//
// Storage (k-packed): codes of (s, x) at ((s / 16) * ld + x) * 16 + s % 16
// bytes, residuals at ((s / 8) * ld + x) * 8 + s % 8 (uint16), so that one
// 16-byte granule holds 16 codes or 8 residuals of one column.
#include "blm_internal.h"

namespace blm {
namespace {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef __bf16 bf16x2 __attribute__((ext_vector_type(2)));
typedef float f4 __attribute__((ext_vector_type(4)));
typedef double d4b __attribute__((ext_vector_type(4)));
typedef unsigned int u4v __attribute__((ext_vector_type(4)));
typedef unsigned int u2v __attribute__((ext_vector_type(2)));

__device__ __forceinline__ f4 mma_bf16(bf16x8 a, bf16x8 b, f4 c) {
  // lane l supplies A[l%16][8(l/16) .. +7] and B[8(l/16) .. +7][l%16];
  // register r of lane l holds D[4(l/16) + r][l%16]
  return __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, c, 0, 0, 0);
}

// 8 e4m3 codes -> 8 BF16 values (exact: every e4m3 value is a BF16 value)
__device__ __forceinline__ bf16x8 e4m3x8_to_bf16(u2v q) {
  const bf16x2 p0 = __builtin_amdgcn_cvt_scalef32_pk_bf16_fp8(q[0], 1.0f, false);
  const bf16x2 p1 = __builtin_amdgcn_cvt_scalef32_pk_bf16_fp8(q[0], 1.0f, true);
  const bf16x2 p2 = __builtin_amdgcn_cvt_scalef32_pk_bf16_fp8(q[1], 1.0f, false);
  const bf16x2 p3 = __builtin_amdgcn_cvt_scalef32_pk_bf16_fp8(q[1], 1.0f, true);
  return bf16x8{p0[0], p0[1], p1[0], p1[1], p2[0], p2[1], p3[0], p3[1]};
}

__device__ __forceinline__ void lds_dma16(const BLM_GLOBAL void* src, void* lds_base) {
  __builtin_amdgcn_global_load_lds(src, (__attribute__((address_space(3))) void*)lds_base, 16, 0, 0);
}

// One workgroup computes a pair of 64 x 64 tile jobs sharing row tile i (the
// layout of the BF16 build): A side {O_i, e_i}, B side {O_j, e_j, O_j', e_j'},
// eight waves of 32 x 32 per product, operands copied into LDS by direct
// global->LDS loads, double-buffered.  Per 32-sample step a wave issues 48
// BF16 matrix-core products: 4 terms x 3 products x 2 x 2 sub-tiles.
constexpr int F8_THREADS = 512;
constexpr int F8_STEP = 32;               // samples per step
constexpr int F8_G8 = F8_STEP / 8;        // 8-sample residual groups per step
constexpr int F8_G16 = F8_STEP / 16;      // 16-sample code groups per step
// FP32 partials are added into FP64 every F8_FLUSH steps and at every slice
// boundary.  With one residual, every 8 steps (256 samples): the storage's
// own error (2^-13 per value) dominates, and flushing every 64 samples gave
// the same matrices (3.6e-6 against the oracle on the stored values) and
// energies within 1e-6 relative of these, at 50.9 instead of 45.5 ms.  With
// two residuals (2^-22 per value) every 2 steps (64 samples), as the BF16
// build; flushing every step moved the matrices by 4.8e-9 instead of 6.7e-9
// against the oracle on the stored values, so the FP32 partials are not what
// limits them.
template <int NRES>
constexpr int F8_FLUSH = NRES == 2 ? 2 : 8;

template <int NRES>
struct F8Lds {
  u4v qA[2][F8_G16][GT];          // [O or e][16-sample group][column]: 16 codes
  u4v rA[NRES][2][F8_G8][GT];     // [residual][O or e][8-sample group][column]: 8 residuals
  u4v qB[2][F8_G16][2 * GT];
  u4v rB[NRES][2][F8_G8][2 * GT];
  u4v qX[2][F8_G16][NAUX];        // aux columns [Xa or Ya]
  u4v rX[NRES][2][F8_G8][NAUX];
  float sA[2][GT];                // column scales of the step's chunk
  float sB[2][2 * GT];
  float sX[2][NAUX];
};

// NRES: residuals per stored value (1: four piece products; 2: eight, the
// four of one residual plus q t, t q, r t and t r; t t, below 2^-26 of the
// product, is left out).  STRIPS: the launch of the pairs whose first job is
// a diagonal tile (coupling strips); the other pairs run an instantiation
// without the strip logic, which needs fewer registers.
template <int NRES, bool STRIPS>
__global__ __launch_bounds__(F8_THREADS, 1) void gram_fp8_kernel(const PairJob* __restrict__ pairs,
                                                                int n_pairs,
                                                                const GramJob* __restrict__ jobs,
                                                                const Slice* __restrict__ slices,
                                                                int n_slices, int P,
                                                                double* __restrict__ partial,
    const int2* __restrict__ sets) {
  // wave instructions per step: A side codes (2 arrays x 2 groups) and
  // residuals (2 x 4); B side the same for two 64-column halves; diagonal
  // pairs also the aux columns (codes of both arrays in one, residuals one
  // per array)
  constexpr int NIA = 2 * F8_G16 + NRES * 2 * F8_G8;
  constexpr int NIB = 2 * NIA;
  constexpr int NIX = 1 + 2 * NRES;
  constexpr int NW = F8_THREADS / 64;
  constexpr int NSC = 2 * GT + 2 * 2 * GT + 2 * NAUX;   // scales per step, one per thread
  static_assert(NSC <= F8_THREADS, "one scale per thread");
  __shared__ F8Lds<NRES> L[2];

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

  // the wave index is provably uniform, so every per-wave choice is a scalar
  // branch: matrix-core instructions ignore the lane mask
  const int tid = threadIdx.x, lane = tid & 63;
  const int wv = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int i16 = lane & 15, k4 = lane >> 4;
  const int wr = wv & 1, wc = wv >> 1;
  const bool wave_b = wc >= 2;
  const bool wave_on = !wave_b || has_b;
  const bool third = (wave_b ? JB.kind : JA.kind) == JOB_OFF;
  const bool pair_strips = STRIPS && JA.kind == JOB_DIAG;
  const bool strip = pair_strips && !wave_b;
  const int n_instr = NIA + NIB + (pair_strips ? NIX : 0);

  const int acol = JA.ci + min(lane, JA.mi - 1);
  const int bcol0 = JA.cj + min(lane, JA.nj - 1);
  const int bcol1 = JB.cj + min(lane, JB.nj - 1);

  // this thread's scale: which array, which source column, where in LDS
  int sc_kind, sc_col, sc_off;
  if (tid < 2 * GT) {
    sc_kind = tid / GT;
    const int c = tid % GT;
    sc_col = JA.ci + min(c, JA.mi - 1);
    sc_off = (int)((const char*)&L[0].sA[sc_kind][c] - (const char*)&L[0]);
  } else if (tid < 2 * GT + 4 * GT) {
    const int u = tid - 2 * GT, c = u % GT, h = (u / GT) & 1;
    sc_kind = u / (2 * GT);
    sc_col = h ? JB.cj + min(c, JB.nj - 1) : JA.cj + min(c, JA.nj - 1);
    sc_off = (int)((const char*)&L[0].sB[sc_kind][GT * h + c] - (const char*)&L[0]);
  } else {
    const int u = min(tid - 6 * GT, 2 * NAUX - 1);
    sc_kind = 2 + u / NAUX;
    sc_col = u % NAUX;
    sc_off = (int)((const char*)&L[0].sX[u / NAUX][u % NAUX] - (const char*)&L[0]);
  }
  float sreg = 0.f;

  f4 acc[3][2][2];
  d4b a64[3][2][2];
#pragma unroll
  for (int t = 0; t < 3; ++t)
#pragma unroll
    for (int x = 0; x < 2; ++x)
#pragma unroll
      for (int y = 0; y < 2; ++y) {
        acc[t][x][y] = f4{0.f, 0.f, 0.f, 0.f};
        a64[t][x][y] = d4b{0.0, 0.0, 0.0, 0.0};
      }

  // copies step (slice sl, first 8-sample group g8) into LDS buffer buf; every
  // address is inside the slice (groups and columns clamped)
  auto issue = [&](int sl, int64_t g8, int buf) __attribute__((always_inline)) {
    const Slice S = slices[sl];
    const int64_t n8 = (S.n + 7) >> 3, n16 = (S.n + 15) >> 4;
    const int64_t g16 = g8 >> 1;
    const BLM_GLOBAL uint8_t* QO = as_global((const uint8_t*)S.O);
    const BLM_GLOBAL uint8_t* QE = as_global((const uint8_t*)S.e);
    const BLM_GLOBAL uint16_t* RO = as_global(S.Or);
    const BLM_GLOBAL uint16_t* RE = as_global(S.er);
    const BLM_GLOBAL uint16_t* TO = as_global(S.Ot);
    const BLM_GLOBAL uint16_t* TE = as_global(S.et);
#pragma unroll
    for (int ii = 0; ii < (NIA + NIB + NIX + NW - 1) / NW; ++ii) {
      const int in = wv + ii * NW;
      if (in >= n_instr) break;
      const BLM_GLOBAL void* src;
      void* dst;
      if (in < NIA + NIB) {
        const bool bside = in >= NIA;
        const int j = bside ? (in - NIA) >> 1 : in;
        const int half = bside ? ((in - NIA) & 1) : 0;
        // arithmetic, not a conditional: a conditional over the captured values
        // becomes a load through a selected address, which keeps them in memory
        const int col = acol + (int)bside * (bcol0 - acol + half * (bcol1 - bcol0));
        if (j < 2 * F8_G16) {
          const int arr = j / F8_G16, gi = j % F8_G16;
          const int64_t gg = min(g16 + gi, n16 - 1);
          src = (arr ? QE : QO) + (gg * S.ld + col) * 16;
          dst = bside ? (void*)&L[buf].qB[arr][gi][GT * half] : (void*)&L[buf].qA[arr][gi][0];
        } else {
          const int jj = j - 2 * F8_G16, pc = jj / (2 * F8_G8), arr = (jj / F8_G8) & 1, gi = jj % F8_G8;
          const int64_t gg = min(g8 + gi, n8 - 1);
          const BLM_GLOBAL uint16_t* rs = pc ? (arr ? TE : TO) : (arr ? RE : RO);
          src = rs + (gg * S.ld + col) * 8;
          dst = bside ? (void*)&L[buf].rB[pc][arr][gi][GT * half] : (void*)&L[buf].rA[pc][arr][gi][0];
        }
      } else if (in == NIA + NIB) {
        // aux codes: lane -> (array lane / 32, group (lane / 16) % 2, column lane % 16)
        const int arr = lane >> 5, gi = (lane >> 4) & 1, c = lane & 15;
        const int64_t gg = min(g16 + gi, n16 - 1);
        src = as_global(arr ? S.Yq : S.Xq) + (gg * NAUX + c) * 16;
        dst = &L[buf].qX[0][0][0];
      } else {
        // aux residuals of one array: lane -> (group lane / 16, column lane % 16)
        const int k = in - NIA - NIB - 1, pc = k >> 1, arr = k & 1, gi = lane >> 4, c = lane & 15;
        const int64_t gg = min(g8 + gi, n8 - 1);
        const uint16_t* rs = pc ? (arr ? S.Yt : S.Xt) : (arr ? S.Yr : S.Xr);
        src = as_global(rs) + (gg * NAUX + c) * 8;
        dst = &L[buf].rX[pc][arr][0][0];
      }
      lds_dma16(src, dst);
    }
    if (tid < NSC) {
      const float* sp = sc_kind == 0 ? S.Os : sc_kind == 1 ? S.es : sc_kind == 2 ? S.Xs : S.Ys;
      sreg = as_global(sp)[sc_col];
    }
  };
  // after this thread's loads have landed: its scale into LDS buffer buf
  auto put_scale = [&](int buf) __attribute__((always_inline)) {
    if (tid < NSC) *(float*)((char*)&L[buf] + sc_off) = sreg;
  };

  // third product of each wave: e_i^T O_j off the diagonal; on a diagonal
  // tile the coupling strips (x = 0: aux^T O_i, or auxE^T O_i on the wr = 1
  // waves; x = 1: aux^T e_i on the wr = 0 waves).  Its A operand is chosen
  // by LDS address, its B operand by a register select.
  const int q3_base = strip ? (int)((const char*)&L[0].qX[wr][k4 >> 1][i16] - (const char*)&L[0])
                            : (int)((const char*)&L[0].qA[1][k4 >> 1][32 * wr + i16] - (const char*)&L[0]);
  const int r3_base = strip ? (int)((const char*)&L[0].rX[0][wr][k4][i16] - (const char*)&L[0])
                            : (int)((const char*)&L[0].rA[0][1][k4][32 * wr + i16] - (const char*)&L[0]);
  // from a first residual to the second one of the same operand
  const int t3_step = strip ? (int)sizeof(L[0].rX[0]) : (int)sizeof(L[0].rA[0]);
  const int ab_x = strip ? 0 : 16 * (int)sizeof(u4v);          // next 16 rows
  const bool b3_e = strip && wr == 0;

  auto compute = [&](int buf, int64_t n8_left, bool flush) __attribute__((always_inline)) {
    // groups at or past the slice's end contribute nothing: on the last
    // step of a slice the A side is zeroed by a lane mask
    const bool partial = n8_left < F8_G8;
    const unsigned km = (k4 < n8_left) ? 0xFFFFFFFFu : 0u;
    const F8Lds<NRES>& Lb = L[buf];
    const char* lb = (const char*)&Lb;
    const int hb = 8 * (k4 & 1);                               // byte offset of this lane's 8 codes
    bf16x8 br[2][2], bqb[2][2];
#pragma unroll
    for (int arr = 0; arr < 2; ++arr)
#pragma unroll
      for (int y = 0; y < 2; ++y) {
        const int col = 32 * wc + 16 * y + i16;
        bqb[arr][y] = e4m3x8_to_bf16(*(const u2v*)((const char*)&Lb.qB[arr][k4 >> 1][col] + hb));
        br[arr][y] = __builtin_bit_cast(bf16x8, Lb.rB[0][arr][k4][col]);
      }
#pragma unroll
    for (int x = 0; x < 2; ++x) {
      const int row = 32 * wr + 16 * x + i16;
      u2v aq = *(const u2v*)((const char*)&Lb.qA[0][k4 >> 1][row] + hb);
      u4v ar = Lb.rA[0][0][k4][row];
      u2v a3q = *(const u2v*)(lb + q3_base + x * ab_x + hb);
      u4v a3r = *(const u4v*)(lb + r3_base + x * ab_x);
      if (partial) {
        aq &= km;
        ar &= km;
        a3q &= km;
        a3r &= km;
      }
      const bf16x8 aqb = e4m3x8_to_bf16(aq), arb = __builtin_bit_cast(bf16x8, ar);
      const bf16x8 a3qb = e4m3x8_to_bf16(a3q), a3rb = __builtin_bit_cast(bf16x8, a3r);
      const bool e3 = x == 1 && b3_e;
      if constexpr (NRES == 2) {
        // the second residuals: q t, t q, r t and t r for each of the three
        // products (dropping r t and t r would move the matrices by about
        // 3e-8 relative, as much as everything else together)
        u4v at = Lb.rA[1][0][k4][row];
        u4v a3t = *(const u4v*)(lb + r3_base + t3_step + x * ab_x);
        if (partial) {
          at &= km;
          a3t &= km;
        }
        const bf16x8 atb = __builtin_bit_cast(bf16x8, at), a3tb = __builtin_bit_cast(bf16x8, a3t);
#pragma unroll
        for (int y = 0; y < 2; ++y) {
          const int col = 32 * wc + 16 * y + i16;
          const bf16x8 bt0 = __builtin_bit_cast(bf16x8, Lb.rB[1][0][k4][col]);
          const bf16x8 bt1 = __builtin_bit_cast(bf16x8, Lb.rB[1][1][k4][col]);
          acc[0][x][y] = mma_bf16(aqb, bt0, acc[0][x][y]);
          acc[1][x][y] = mma_bf16(aqb, bt1, acc[1][x][y]);
          acc[2][x][y] = mma_bf16(a3qb, e3 ? bt1 : bt0, acc[2][x][y]);
          acc[0][x][y] = mma_bf16(atb, bqb[0][y], acc[0][x][y]);
          acc[1][x][y] = mma_bf16(atb, bqb[1][y], acc[1][x][y]);
          acc[2][x][y] = mma_bf16(a3tb, e3 ? bqb[1][y] : bqb[0][y], acc[2][x][y]);
          acc[0][x][y] = mma_bf16(arb, bt0, acc[0][x][y]);
          acc[1][x][y] = mma_bf16(arb, bt1, acc[1][x][y]);
          acc[2][x][y] = mma_bf16(a3rb, e3 ? bt1 : bt0, acc[2][x][y]);
          acc[0][x][y] = mma_bf16(atb, br[0][y], acc[0][x][y]);
          acc[1][x][y] = mma_bf16(atb, br[1][y], acc[1][x][y]);
          acc[2][x][y] = mma_bf16(a3tb, e3 ? br[1][y] : br[0][y], acc[2][x][y]);
        }
      }
#pragma unroll
      for (int y = 0; y < 2; ++y) {
        const bf16x8 b3r = e3 ? br[1][y] : br[0][y];
        const bf16x8 b3qb = e3 ? bqb[1][y] : bqb[0][y];
        acc[0][x][y] = mma_bf16(aqb, bqb[0][y], acc[0][x][y]);
        acc[1][x][y] = mma_bf16(aqb, bqb[1][y], acc[1][x][y]);
        acc[2][x][y] = mma_bf16(a3qb, b3qb, acc[2][x][y]);
        acc[0][x][y] = mma_bf16(aqb, br[0][y], acc[0][x][y]);
        acc[1][x][y] = mma_bf16(aqb, br[1][y], acc[1][x][y]);
        acc[2][x][y] = mma_bf16(a3qb, b3r, acc[2][x][y]);
        acc[0][x][y] = mma_bf16(arb, bqb[0][y], acc[0][x][y]);
        acc[1][x][y] = mma_bf16(arb, bqb[1][y], acc[1][x][y]);
        acc[2][x][y] = mma_bf16(a3rb, b3qb, acc[2][x][y]);
        acc[0][x][y] = mma_bf16(arb, br[0][y], acc[0][x][y]);
        acc[1][x][y] = mma_bf16(arb, br[1][y], acc[1][x][y]);
        acc[2][x][y] = mma_bf16(a3rb, b3r, acc[2][x][y]);
      }
    }
    if (!flush) return;
    // scale by s_row s_col (powers of two: exact) into FP64
#pragma unroll
    for (int x = 0; x < 2; ++x)
#pragma unroll
      for (int rr = 0; rr < 4; ++rr) {
        const int row = 32 * wr + 16 * x + 4 * k4 + rr;
        const double sO = Lb.sA[0][row];
        const double s3 = strip ? (double)Lb.sX[wr][4 * k4 + rr] : (double)Lb.sA[1][row];
#pragma unroll
        for (int y = 0; y < 2; ++y) {
          const int col = 32 * wc + 16 * y + i16;
          const double tO = Lb.sB[0][col], tE = Lb.sB[1][col];
          const double t3 = (x == 1 && b3_e) ? tE : tO;
          a64[0][x][y][rr] += (double)acc[0][x][y][rr] * (sO * tO);
          a64[1][x][y][rr] += (double)acc[1][x][y][rr] * (sO * tE);
          a64[2][x][y][rr] += (double)acc[2][x][y][rr] * (s3 * t3);
        }
      }
#pragma unroll
    for (int t = 0; t < 3; ++t)
#pragma unroll
      for (int x = 0; x < 2; ++x)
#pragma unroll
        for (int y = 0; y < 2; ++y) acc[t][x][y] = f4{0.f, 0.f, 0.f, 0.f};
  };

  int n_steps = 0;
  for (int sl = p; sl < n_slices; sl += P) n_steps += (int)((slices[sl].n + F8_STEP - 1) / F8_STEP);

  int si = p;                 // slice and first 8-sample group of the next step to copy
  while (si < n_slices && slices[si].n <= 0) si += P;
  int64_t g0 = 0;
  auto advance = [&]() __attribute__((always_inline)) {
    g0 += F8_G8;
    if (g0 * 8 >= slices[si].n) {
      g0 = 0;
      si += P;
      while (si < n_slices && slices[si].n <= 0) si += P;
    }
  };
  int csi = si;               // slice and first group of the step in LDS
  int64_t cg0 = 0;
  if (n_steps > 0) {
    issue(si, g0, 0);
    advance();
  }
  __builtin_amdgcn_s_waitcnt(0);
  put_scale(0);
  __syncthreads();
  int buf = 0;
  for (int t = 0; t < n_steps; ++t) {
    const bool more = t + 1 < n_steps;
    const int64_t n8_left = ((slices[csi].n + 7) >> 3) - cg0;
    const int nsi = si;
    const int64_t ng0 = g0;
    if (more) issue(si, g0, buf ^ 1);
    if (wave_on) compute(buf, n8_left, ((t + 1) % F8_FLUSH<NRES>) == 0 || !more || nsi != csi);
    if (more) advance();
    __builtin_amdgcn_s_waitcnt(0);   // this wave's copies of the next step have landed
    if (more) put_scale(buf ^ 1);
    __syncthreads();                 // ... and everyone's; the current buffer is free
    buf ^= 1;
    csi = nsi;
    cg0 = ng0;
  }

  if (!wave_on) return;
  const int jw = wave_b ? PJ.jb : PJ.ja;
  BLM_GLOBAL double* base = as_global(partial) + ((size_t)jw * P + p) * (size_t)(3 * GT * GT);
  const int c0 = 32 * (wc & 1);
  if (strip) {
    // strips [3][NAUX][GT] in the third slot: q = 0 aux^T O, 1 aux^T e, 2 auxE^T O
#pragma unroll
    for (int y = 0; y < 2; ++y)
#pragma unroll
      for (int rr = 0; rr < 4; ++rr) {
        const int a = 4 * k4 + rr;
        const int col = c0 + 16 * y + i16;
        if (wr == 0) {
          base[2 * GT * GT + 0 * NAUX * GT + a * GT + col] = a64[2][0][y][rr];
          base[2 * GT * GT + 1 * NAUX * GT + a * GT + col] = a64[2][1][y][rr];
        } else {
          base[2 * GT * GT + 2 * NAUX * GT + a * GT + col] = a64[2][0][y][rr];
        }
      }
  }
#pragma unroll
  for (int x = 0; x < 2; ++x)
#pragma unroll
    for (int y = 0; y < 2; ++y)
#pragma unroll
      for (int rr = 0; rr < 4; ++rr) {
        const int row = 32 * wr + 16 * x + 4 * k4 + rr;
        const int col = c0 + 16 * y + i16;
        base[row * GT + col] = a64[0][x][y][rr];
        base[GT * GT + row * GT + col] = a64[1][x][y][rr];
        if (third) base[2 * GT * GT + row * GT + col] = a64[2][x][y][rr];
      }
}

// ---------------------------------------------------------------------------
// FP64 -> e4m3 codes + BF16 residuals + per-column scales (producer side)
// ---------------------------------------------------------------------------

constexpr uint32_t F8_SCALE_MIN_BITS = 0x00800000u;   // 2^-126

// smallest power of two s with |v| / s <= 448, as FP32 bits (2^-126 .. 2^127)
__device__ __forceinline__ uint32_t fp8_scale_bits(double v) {
  const double a = fabs(v);
  if (!(a > 0.0)) return F8_SCALE_MIN_BITS;
  int E;
  const double f = frexp(a, &E);                         // a = f 2^E, f in [0.5, 1)
  int k = (f <= 0.875) ? E - 9 : E - 8;                  // 448 = 0.875 2^9
  k = max(-126, min(127, k));
  return (uint32_t)(k + 127) << 23;
}

__global__ __launch_bounds__(256) void fp8_scale_init_kernel(uint32_t* scale_bits, int64_t ncols) {
  const int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (c < ncols) scale_bits[c] = F8_SCALE_MIN_BITS;
}

// block (64 columns) x (4 row lanes) threads; grid.y row blocks
__global__ __launch_bounds__(256) void fp8_scale_max_kernel(const double* __restrict__ src, int64_t n,
                                                            int64_t ld_src, int64_t ncols,
                                                            uint32_t* __restrict__ scale_bits) {
  const int64_t c = (int64_t)blockIdx.x * 64 + (threadIdx.x & 63);
  if (c >= ncols) return;
  uint32_t m = F8_SCALE_MIN_BITS;
  for (int64_t s = (int64_t)blockIdx.y * 4 + (threadIdx.x >> 6); s < n; s += (int64_t)gridDim.y * 4)
    m = max(m, fp8_scale_bits(src[s * ld_src + c]));
  // positive FP32 bit patterns order like their values
  atomicMax(scale_bits + c, m);
}

// e4m3 (OCP: bias 7, 3 mantissa bits, no infinities, max 448) nearest to a,
// ties to even, saturated at 448; a >= 0 and finite
__device__ __forceinline__ double e4m3_round(double a, uint32_t* code) {
  if (a == 0.0) {
    *code = 0;
    return 0.0;
  }
  int E;
  frexp(a, &E);
  const int e = max(E - 1, -6);                          // binade (subnormals share -6)
  const double quantum = ldexp(1.0, e - 3);
  double qv = rint(a / quantum) * quantum;               // exact scaling, RNE
  if (qv > 448.0) qv = 448.0;
  if (qv == 0.0) {
    *code = 0;
    return 0.0;
  }
  int Eq;
  const double fq = frexp(qv, &Eq);                      // qv = fq 2^Eq
  if (Eq - 1 < -6) {
    *code = (uint32_t)(qv * 512.0);                      // subnormal: m 2^-9
  } else {
    *code = ((uint32_t)(Eq - 1 + 7) << 3) | (uint32_t)(fq * 16.0 - 8.0);
  }
  return qv;
}

__device__ __forceinline__ uint16_t f64_to_bf16_rne(double v) {
  // to FP32 (round to nearest), then to BF16 (round to nearest even)
  const uint32_t u = __float_as_uint((float)v);
  const uint32_t lsb = (u >> 16) & 1u;
  return (uint16_t)((u + 0x7FFFu + lsb) >> 16);
}

// thread -> (16-sample group, column): 16 codes and 16 residuals
__global__ __launch_bounds__(256) void fp8_quant_kernel(const double* __restrict__ src, int64_t n,
                                                        int64_t ld_src, int64_t ncols,
                                                        const float* __restrict__ scale,
                                                        uint8_t* __restrict__ codes,
                                                        uint16_t* __restrict__ res, uint16_t* __restrict__ res2,
                                                        int64_t ld_dst) {
  const int64_t n16 = (n + 15) >> 4;
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= n16 * ncols) return;
  const int64_t g = t / ncols, x = t % ncols;
  const double inv = 1.0 / (double)scale[x];             // a power of two: exact
  uint32_t cw[4] = {0, 0, 0, 0};
  uint32_t rw[8] = {0, 0, 0, 0, 0, 0, 0, 0};
  uint32_t tw[8] = {0, 0, 0, 0, 0, 0, 0, 0};
#pragma unroll
  for (int e = 0; e < 16; ++e) {
    const int64_t s = 16 * g + e;
    const double v = (s < n) ? src[s * ld_src + x] * inv : 0.0;
    uint32_t code;
    const double qv = e4m3_round(fabs(v), &code);
    if (v < 0.0 && code != 0) code |= 0x80u;
    const double rem = v - (v < 0.0 ? -qv : qv);           // exact
    const uint16_t rb = f64_to_bf16_rne(rem);
    // the second residual: what r leaves of the remainder (exact in FP64)
    const double rem2 = rem - (double)__uint_as_float((uint32_t)rb << 16);
    const uint16_t tb = f64_to_bf16_rne(rem2);
    cw[e >> 2] |= code << (8 * (e & 3));
    rw[e >> 1] |= (uint32_t)rb << (16 * (e & 1));
    tw[e >> 1] |= (uint32_t)tb << (16 * (e & 1));
  }
  *reinterpret_cast<uint4*>(codes + (g * ld_dst + x) * 16) = make_uint4(cw[0], cw[1], cw[2], cw[3]);
  // residuals come in 8-sample groups: the buffers hold ceil(n / 8) of them,
  // so the second group of the last 16 is written only if it exists
  const bool second = 2 * g + 1 < ((n + 7) >> 3);
  uint16_t* rp = res + ((2 * g) * ld_dst + x) * 8;
  *reinterpret_cast<uint4*>(rp) = make_uint4(rw[0], rw[1], rw[2], rw[3]);
  if (second) *reinterpret_cast<uint4*>(rp + ld_dst * 8) = make_uint4(rw[4], rw[5], rw[6], rw[7]);
  if (res2) {
    uint16_t* tp = res2 + ((2 * g) * ld_dst + x) * 8;
    *reinterpret_cast<uint4*>(tp) = make_uint4(tw[0], tw[1], tw[2], tw[3]);
    if (second) *reinterpret_cast<uint4*>(tp + ld_dst * 8) = make_uint4(tw[4], tw[5], tw[6], tw[7]);
  }
}

}  // namespace

void launch_gram_fp8(const PairJob* d_pairs, int n_strip_pairs, int n_pairs, const GramJob* d_jobs,
                     const Slice* d_slices, int n_slices, int P, int nres, double* d_partial, hipStream_t st,
                     const int2* d_sets) {
  const int n_plain = n_pairs - n_strip_pairs;
  if (nres == 2) {
    if (n_strip_pairs > 0)
      hipLaunchKernelGGL((gram_fp8_kernel<2, true>), dim3(n_strip_pairs * P), dim3(F8_THREADS), 0, st, d_pairs,
                         n_strip_pairs, d_jobs, d_slices, n_slices, P, d_partial, d_sets);
    if (n_plain > 0)
      hipLaunchKernelGGL((gram_fp8_kernel<2, false>), dim3(n_plain * P), dim3(F8_THREADS), 0, st,
                         d_pairs + n_strip_pairs, n_plain, d_jobs, d_slices, n_slices, P, d_partial, d_sets);
  } else {
    if (n_strip_pairs > 0)
      hipLaunchKernelGGL((gram_fp8_kernel<1, true>), dim3(n_strip_pairs * P), dim3(F8_THREADS), 0, st, d_pairs,
                         n_strip_pairs, d_jobs, d_slices, n_slices, P, d_partial, d_sets);
    if (n_plain > 0)
      hipLaunchKernelGGL((gram_fp8_kernel<1, false>), dim3(n_plain * P), dim3(F8_THREADS), 0, st,
                         d_pairs + n_strip_pairs, n_plain, d_jobs, d_slices, n_slices, P, d_partial, d_sets);
  }
}

void launch_pack_fp8(const double* src, int64_t n, int64_t ld_src, int64_t ncols, uint8_t* codes,
                     uint16_t* res, uint16_t* res2, float* scale, int64_t ld_dst, hipStream_t st) {
  if (ncols <= 0) return;
  uint32_t* bits = reinterpret_cast<uint32_t*>(scale);
  hipLaunchKernelGGL(fp8_scale_init_kernel, dim3((unsigned)((ncols + 255) / 256)), dim3(256), 0, st,
                     bits, ncols);
  if (n <= 0) return;
  const unsigned gy = (unsigned)std::min<int64_t>(1024, (n + 255) / 256);
  hipLaunchKernelGGL(fp8_scale_max_kernel, dim3((unsigned)((ncols + 63) / 64), gy), dim3(256), 0, st,
                     src, n, ld_src, ncols, bits);
  const int64_t work = ((n + 15) >> 4) * ncols;
  hipLaunchKernelGGL(fp8_quant_kernel, dim3((unsigned)((work + 255) / 256)), dim3(256), 0, st, src, n,
                     ld_src, ncols, scale, codes, res, res2, ld_dst);
}

}  // namespace blm
