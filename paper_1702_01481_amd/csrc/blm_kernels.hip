// Sample-streaming kernels of the blocked linear method on gfx950:
//
//  * gram_kernel: weighted Gram tiles C = X^T diag(w) Y over sample slices
//    on the FP64 matrix cores (v_mfma_f64_16x16x4).  This is the Monte Carlo
//    estimate of Eq. 3 restricted to each parameter block (the green
//    elements of Fig. 1: S_b and H_b of the one-block basis, Eq. 4 / Eq. 10),
//    their coupling strips and the aux Gram (the blue elements; strips of
//    aux groups after the first also on BF16 split and FP8 storage), and,
//    in the second pass, the stage-two estimates of Eq. 7.
//  * gram_reduce_kernel: fixed-order sum of the per-slice partial tiles into
//    the FP64 accumulators (no floating-point atomics: bitwise
//    reproducible).
//  * dirproj_kernel: projection of every sample onto per-block directions,
//    t_s = D . O_{s,k} (previous-update directions, Eq. 9) or y_s = B^(b) O_{s,b}
//    (kept directions, Eq. 6).
#include "blm_internal.h"

namespace blm {

typedef double d4 __attribute__((ext_vector_type(4)));

__device__ __forceinline__ d4 mfma_f64(double a, double b, d4 c) {
  // D[i][j] += sum_k A[i][k] B[k][j], 16x16x4; lane l supplies A[l%16][l/16]
  // and B[l/16][l%16]; D register r of lane l is D[4*r + l/16][l%16].
  return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
}

__device__ __forceinline__ double bf16_to_f64(uint16_t h) {
  return (double)__uint_as_float((uint32_t)h << 16);
}

// Element (row, col) of BF16 split storage (k-packed), as the exact FP64 sum
// of its pieces.
__device__ __forceinline__ double split_load(const void* base, int64_t ld, int64_t pstride,
                                             int pieces, int64_t row, int64_t col) {
  const BLM_GLOBAL uint16_t* b = as_global((const uint16_t*)base);
  const int64_t i = ((row >> 3) * ld + col) * 8 + (row & 7);
  double v = bf16_to_f64(b[i]);
  if (pieces > 1) v += bf16_to_f64(b[i + pstride]);
  if (pieces > 2) v += bf16_to_f64(b[i + 2 * pstride]);
  return v;
}

// The 8 samples of one 8-sample group of one column in BF16 split storage,
// each as the exact FP64 sum of its pieces: one 16-byte load per piece.
__device__ __forceinline__ void split_load8(const void* base, int64_t ld, int64_t pstride,
                                            int pieces, int64_t group, int64_t col, double* v) {
  const BLM_GLOBAL uint16_t* b = as_global((const uint16_t*)base) + (group * ld + col) * 8;
#pragma unroll
  for (int k = 0; k < 8; ++k) v[k] = 0.0;
  for (int pc = 0; pc < pieces; ++pc) {
    const uint4 w = *reinterpret_cast<const BLM_GLOBAL uint4*>(b + (size_t)pc * pstride);
    const uint32_t u[4] = {w.x, w.y, w.z, w.w};
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      v[2 * k] += (double)__uint_as_float(u[k] << 16);
      v[2 * k + 1] += (double)__uint_as_float(u[k] & 0xFFFF0000u);
    }
  }
}

// The 8 samples of one 8-sample group of one column in FP8 storage (e4m3
// codes k-packed by 16 samples, BF16 residuals by 8, power-of-two column
// scale), each as the exact FP64 value scale (q + r), or scale (q + r + t)
// with a second residual array res2 (nullptr: none).  The sums are exact:
// q, r and t together span fewer than 53 bits.
__device__ __forceinline__ void fp8_load8(const void* codes, const uint16_t* res, const uint16_t* res2,
                                          const float* scale, int64_t ld, int64_t group, int64_t col, double* v) {
  const BLM_GLOBAL uint8_t* qb =
      as_global((const uint8_t*)codes) + ((group >> 1) * ld + col) * 16 + 8 * (group & 1);
  const uint2 q = *reinterpret_cast<const BLM_GLOBAL uint2*>(qb);
  const uint4 r = *reinterpret_cast<const BLM_GLOBAL uint4*>(as_global(res) + (group * ld + col) * 8);
  uint4 t = make_uint4(0, 0, 0, 0);
  if (res2) t = *reinterpret_cast<const BLM_GLOBAL uint4*>(as_global(res2) + (group * ld + col) * 8);
  const double sc = as_global(scale)[col];
  const uint32_t qw[2] = {q.x, q.y};
  const uint32_t rw[4] = {r.x, r.y, r.z, r.w};
  const uint32_t tw[4] = {t.x, t.y, t.z, t.w};
  // codes to BF16 (exact), two per conversion, then to FP64
  const uint32_t pw[4] = {
      __builtin_bit_cast(uint32_t, __builtin_amdgcn_cvt_scalef32_pk_bf16_fp8(qw[0], 1.0f, false)),
      __builtin_bit_cast(uint32_t, __builtin_amdgcn_cvt_scalef32_pk_bf16_fp8(qw[0], 1.0f, true)),
      __builtin_bit_cast(uint32_t, __builtin_amdgcn_cvt_scalef32_pk_bf16_fp8(qw[1], 1.0f, false)),
      __builtin_bit_cast(uint32_t, __builtin_amdgcn_cvt_scalef32_pk_bf16_fp8(qw[1], 1.0f, true))};
#pragma unroll
  for (int k = 0; k < 4; ++k) {
    const uint32_t pb = pw[k];
    const double q0 = (double)__uint_as_float(pb << 16), q1 = (double)__uint_as_float(pb & 0xFFFF0000u);
    const double r0 = (double)__uint_as_float(rw[k] << 16), r1 = (double)__uint_as_float(rw[k] & 0xFFFF0000u);
    const double t0 = (double)__uint_as_float(tw[k] << 16), t1 = (double)__uint_as_float(tw[k] & 0xFFFF0000u);
    v[2 * k] = sc * ((q0 + r0) + t0);
    v[2 * k + 1] = sc * ((q1 + r1) + t1);
  }
}

// ---------------------------------------------------------------------------
// Gram tiles
// ---------------------------------------------------------------------------

// One sample row of a stage as held in registers between its global loads
// and its LDS store.  Values are raw; the sample weight is applied (and
// columns outside the tile are zeroed) when the stage is stored, so that no
// instruction uses a loaded value before the next stage's products.
struct StageRegs {
  double a[4], e[4], b[4], f[4];
  double x[STRIP_GROUPS], y[STRIP_GROUPS];   // aux (1, Theta), (E_L, Theta energy); one per group
  double w;             // sample weight (of the clamped row)
  bool valid;           // the row is inside the slice
};

// Load cursor: the slice whose stages are being loaded and its descriptor,
// kept in registers (re-read only when the cursor moves to another slice).
struct Cursor {
  Slice S;
  int si;
  int64_t ro;
};

__device__ __forceinline__ void cursor_skip_empty(Cursor& c, const Slice* __restrict__ slices,
                                                  int n_slices, int P) {
  while (c.si < n_slices) {
    c.S = slices[c.si];
    if (c.S.n > 0) return;
    c.si += P;
  }
}

__device__ __forceinline__ void cursor_next(Cursor& c, const Slice* __restrict__ slices,
                                            int n_slices, int P) {
  c.ro += GKS;
  if (c.ro >= c.S.n) {
    c.ro = 0;
    c.si += P;
    cursor_skip_empty(c, slices, n_slices, P);
  }
}

__device__ __forceinline__ void ld2(const BLM_GLOBAL double* p, double& x, double& y) {
  const double2 v = *reinterpret_cast<const BLM_GLOBAL double2*>(p);
  x = v.x;
  y = v.y;
}

// Global loads of one 16-sample stage.  Every load is unconditional: rows
// past the end of the slice read the slice's last row (and get weight 0),
// columns past a ragged tile edge read the tile's last column (and are
// zeroed at the store).  FULL: the tile is 64 x 64 and 16-byte aligned.
template <int KIND, bool FULL, bool SPLIT>
__device__ __forceinline__ void gram_load(const GramJob& J, const Slice& S, int64_t ro, int tid,
                                          StageRegs& R) {
  const int lr = tid >> 4;            // sample row within the stage (0..15)
  const int lc = (tid & 15) * 4;      // first of 4 tile columns
  const int64_t row = ro + lr;
  const bool valid = row < S.n;
  const int64_t rc = valid ? row : S.n - 1;
  R.w = S.w ? as_global(S.w)[rc] : 1.0;
  R.valid = valid;
  if constexpr (KIND == JOB_AUX) {
    const BLM_GLOBAL double* xa = as_global(S.Xa) + rc * S.ald;
    const BLM_GLOBAL double* ya = as_global(S.Ya) + rc * S.ald;
#pragma unroll
    for (int c = 0; c < 4; ++c) {
      const int64_t ca = J.ci + min(lc + c, J.mi - 1), cb = J.cj + min(lc + c, J.nj - 1);
      R.a[c] = xa[ca];
      R.b[c] = xa[cb];
      R.f[c] = ya[cb];
      R.e[c] = 0.0;
    }
  } else if constexpr (SPLIT) {
    // strip jobs on BF16 split or FP8 storage (uniform weights): thread ->
    // (panel, 8-sample group, column); 8 samples of one column of O (panel
    // 0) or e (panel 1) land in a[0..3], e[0..3]
    const int pnl = tid >> 7, g = (tid >> 6) & 1, c = tid & 63;
    const int64_t r0 = ro + 8 * g;
    const bool ok = r0 < S.n && c < J.nj;
    const int64_t grp = (r0 < S.n ? r0 : S.n - 1) >> 3;
    const int64_t col = J.cj + min(c, J.nj - 1);
    double v[8];
    if (S.pieces > 0) split_load8(pnl ? S.e : S.O, S.ld, S.pstride, S.pieces, grp, col, v);
    else fp8_load8(pnl ? S.e : S.O, pnl ? S.er : S.Or, pnl ? S.et : S.Ot, pnl ? S.es : S.Os, S.ld, grp, col, v);
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      R.a[k] = ok ? v[k] : 0.0;
      R.e[k] = ok ? v[4 + k] : 0.0;
    }
  } else {
    const BLM_GLOBAL double* rO = as_global((const double*)S.O) + rc * S.ld;
    const BLM_GLOBAL double* re = as_global((const double*)S.e) + rc * S.ld;
    constexpr bool LOAD_A = KIND != JOB_STRIP;
    constexpr bool LOAD_E = KIND == JOB_OFF;
    // diagonal tiles: the column panel is the row panel
    constexpr bool LOAD_B = KIND == JOB_OFF || KIND == JOB_STRIP;
    if constexpr (FULL) {
#pragma unroll
      for (int h = 0; h < 2; ++h) {
        const int col = lc + 2 * h;
        if (LOAD_A) ld2(rO + J.ci + col, R.a[2 * h], R.a[2 * h + 1]);
        if (LOAD_E) ld2(re + J.ci + col, R.e[2 * h], R.e[2 * h + 1]);
        if (LOAD_B) ld2(rO + J.cj + col, R.b[2 * h], R.b[2 * h + 1]);
        ld2(re + J.cj + col, R.f[2 * h], R.f[2 * h + 1]);
      }
    } else {
#pragma unroll
      for (int c = 0; c < 4; ++c) {
        const int ca = min(lc + c, J.mi - 1), cb = min(lc + c, J.nj - 1);
        if (LOAD_A) R.a[c] = rO[J.ci + ca];
        if (LOAD_E) R.e[c] = re[J.ci + ca];
        if (LOAD_B) R.b[c] = rO[J.cj + cb];
        R.f[c] = re[J.cj + cb];
      }
    }
  }
  if constexpr (KIND == JOB_DIAG) {
    const int acol = tid & 15;
    R.x[0] = as_global(S.Xa)[rc * S.ald + J.ag + acol];
    R.y[0] = as_global(S.Ya)[rc * S.ald + J.ag + acol];
  } else if constexpr (KIND == JOB_STRIP) {
    // the job's groups (a group past J.ng loads the last one again)
    const int acol = tid & 15;
#pragma unroll
    for (int g = 0; g < STRIP_GROUPS; ++g) {
      const int64_t col = J.ag + NAUX * min(g, J.ng - 1) + acol;
      R.x[g] = as_global(S.Xa)[rc * S.ald + col];
      R.y[g] = as_global(S.Ya)[rc * S.ald + col];
    }
  }
}

// Double-buffered LDS panels of one workgroup (declared once per kernel: the
// per-kind bodies share it).
struct GramLds {
  double A[2][GKS][GT];   // O_i * w
  double E[2][GKS][GT];   // e_i * w
  double B[2][GKS][GT];   // O_j
  double F[2][GKS][GT];   // e_j
  double X[2][GKS][NAUX]; // aux (1, Theta) * w
  double Y[2][GKS][NAUX]; // aux (E_L, Theta energy) * w
};

template <int KIND, bool FULL, bool SPLIT>
__device__ __forceinline__ void gram_body(GramLds& L, const GramJob& J,
                                          const Slice* __restrict__ slices, int n_slices, int P,
                                          int p, double* __restrict__ out) {
  auto& sA = L.A;
  auto& sE = L.E;
  auto& sB = L.B;
  auto& sF = L.F;
  auto& sX = L.X;
  auto& sY = L.Y;

  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  const int wr = wv >> 1, wc = wv & 1;
  const int i16 = lane & 15, k4 = lane >> 4;
  constexpr bool STRIPS = KIND == JOB_DIAG || KIND == JOB_STRIP;
  constexpr bool MAIN = KIND != JOB_STRIP;
  const int ng = (KIND == JOB_STRIP) ? __builtin_amdgcn_readfirstlane(J.ng) : 1;

  d4 P0[2][2], P1[2][2], P2[2][2];
#pragma unroll
  for (int x = 0; x < 2; ++x)
#pragma unroll
    for (int y = 0; y < 2; ++y) {
      P0[x][y] = d4{0, 0, 0, 0};
      P1[x][y] = d4{0, 0, 0, 0};
      P2[x][y] = d4{0, 0, 0, 0};
    }

  // register stage -> LDS buffer nb (weights applied, ragged columns zeroed)
  auto store = [&](const StageRegs& R, int nb) {
    const int lr = tid >> 4, lc = (tid & 15) * 4;
    if constexpr (SPLIT && KIND == JOB_STRIP) {
      const int pnl = tid >> 7, g = (tid >> 6) & 1, c = tid & 63;
      double(*dst)[GT] = pnl ? sF[nb] : sB[nb];
#pragma unroll
      for (int k = 0; k < 4; ++k) {
        dst[8 * g + k][c] = R.a[k];
        dst[8 * g + 4 + k][c] = R.e[k];
      }
    } else {
      const double w = R.valid ? R.w : 0.0;
      double a[4], e[4], b[4], f[4];
#pragma unroll
      for (int c = 0; c < 4; ++c) {
        const bool oka = FULL || lc + c < J.mi, okb = FULL || lc + c < J.nj;
        a[c] = oka ? R.a[c] * w : 0.0;
        e[c] = oka ? R.e[c] * w : 0.0;
        if constexpr (KIND == JOB_DIAG || KIND == JOB_DIAG_NOSTRIP) b[c] = okb ? R.a[c] : 0.0;
        else b[c] = okb ? R.b[c] : 0.0;
        f[c] = okb ? R.f[c] : 0.0;
      }
#pragma unroll
      for (int c = 0; c < 4; ++c) {
        if (MAIN) sA[nb][lr][lc + c] = a[c];
        if (KIND == JOB_OFF) sE[nb][lr][lc + c] = e[c];
        sB[nb][lr][lc + c] = b[c];
        sF[nb][lr][lc + c] = f[c];
      }
    }
    if constexpr (KIND == JOB_STRIP) {
      // a strip-only job has no row panels: its aux groups go where they
      // would be (64 columns, STRIP_GROUPS groups of 16)
      const double w = R.valid ? R.w : 0.0;
#pragma unroll
      for (int g = 0; g < STRIP_GROUPS; ++g) {
        sA[nb][lr][NAUX * g + (tid & 15)] = R.x[g] * w;
        sE[nb][lr][NAUX * g + (tid & 15)] = R.y[g] * w;
      }
    } else if constexpr (STRIPS) {
      const double w = R.valid ? R.w : 0.0;
      sX[nb][lr][tid & 15] = R.x[0] * w;
      sY[nb][lr][tid & 15] = R.y[0] * w;
    }
  };
  auto compute = [&](int buf) {
#pragma unroll
    for (int kk = 0; kk < GKS; kk += 4) {
      const int kr = kk + k4;
      if constexpr (MAIN) {
        const double a0 = sA[buf][kr][32 * wr + i16], a1 = sA[buf][kr][32 * wr + 16 + i16];
        const double b0 = sB[buf][kr][32 * wc + i16], b1 = sB[buf][kr][32 * wc + 16 + i16];
        const double f0 = sF[buf][kr][32 * wc + i16], f1 = sF[buf][kr][32 * wc + 16 + i16];
        P0[0][0] = mfma_f64(a0, b0, P0[0][0]);
        P0[0][1] = mfma_f64(a0, b1, P0[0][1]);
        P0[1][0] = mfma_f64(a1, b0, P0[1][0]);
        P0[1][1] = mfma_f64(a1, b1, P0[1][1]);
        P1[0][0] = mfma_f64(a0, f0, P1[0][0]);
        P1[0][1] = mfma_f64(a0, f1, P1[0][1]);
        P1[1][0] = mfma_f64(a1, f0, P1[1][0]);
        P1[1][1] = mfma_f64(a1, f1, P1[1][1]);
        if constexpr (KIND == JOB_OFF) {
          const double e0 = sE[buf][kr][32 * wr + i16], e1 = sE[buf][kr][32 * wr + 16 + i16];
          P2[0][0] = mfma_f64(e0, b0, P2[0][0]);
          P2[0][1] = mfma_f64(e0, b1, P2[0][1]);
          P2[1][0] = mfma_f64(e1, b0, P2[1][0]);
          P2[1][1] = mfma_f64(e1, b1, P2[1][1]);
        }
      }
      if constexpr (KIND == JOB_STRIP) {
        // group g's three products in the accumulators of sub-tile (g / 2, g % 2)
        const double bs = sB[buf][kr][16 * wv + i16], fs = sF[buf][kr][16 * wv + i16];
#pragma unroll
        for (int g = 0; g < STRIP_GROUPS; ++g) {
          if (g < ng) {
            const double xs = sA[buf][kr][NAUX * g + i16], ys = sE[buf][kr][NAUX * g + i16];
            P0[g >> 1][g & 1] = mfma_f64(xs, bs, P0[g >> 1][g & 1]);   // aux^T W O_i
            P1[g >> 1][g & 1] = mfma_f64(xs, fs, P1[g >> 1][g & 1]);   // aux^T W e_i
            P2[g >> 1][g & 1] = mfma_f64(ys, bs, P2[g >> 1][g & 1]);   // auxE^T W O_i
          }
        }
      } else if constexpr (STRIPS) {
        const double xs = sX[buf][kr][i16], ys = sY[buf][kr][i16];
        const double bs = sB[buf][kr][16 * wv + i16], fs = sF[buf][kr][16 * wv + i16];
        P2[0][0] = mfma_f64(xs, bs, P2[0][0]);   // aux^T W O_i
        P2[0][1] = mfma_f64(xs, fs, P2[0][1]);   // aux^T W e_i
        P2[1][0] = mfma_f64(ys, bs, P2[1][0]);   // auxE^T W O_i
      }
    }
  };

  // Number of 16-sample stages of this workgroup's slices.
  int n_stages = 0;
  for (int si = p; si < n_slices; si += P) n_stages += (int)((slices[si].n + GKS - 1) / GKS);

  // Two stages are in flight in registers while another is in LDS: the
  // global loads of stage t+2 are issued before stage t is computed (one
  // register stage hid less of the memory latency: 158 against 150 ms for
  // a 30,000-parameter chunk).  Stage t+1 is stored to the other LDS buffer
  // (last read before the previous barrier) before stage t's products, so
  // that its LDS writes go out between the matrix-core instructions instead
  // of after them (150 -> 142 ms).
  Cursor cur;
  cur.si = p;
  cur.ro = 0;
  cursor_skip_empty(cur, slices, n_slices, P);
  // two register stages: the loads of stage t+2 are issued before stage t
  // is computed, and stage t+1 (loaded one step earlier) is stored after it
  StageRegs R0, R1;
  if (n_stages > 0) {
    gram_load<KIND, FULL, SPLIT>(J, cur.S, cur.ro, tid, R0);
    cursor_next(cur, slices, n_slices, P);
    store(R0, 0);
  }
  if (n_stages > 1) {
    gram_load<KIND, FULL, SPLIT>(J, cur.S, cur.ro, tid, R1);
    cursor_next(cur, slices, n_slices, P);
  }
  __syncthreads();
  int buf = 0;
  int t = 0;
  for (; t + 2 < n_stages; t += 2) {
    gram_load<KIND, FULL, SPLIT>(J, cur.S, cur.ro, tid, R0);     // stage t + 2
    cursor_next(cur, slices, n_slices, P);
    store(R1, buf ^ 1);                                           // stage t + 1
    compute(buf);
    __syncthreads();
    buf ^= 1;
    if (t + 3 < n_stages) {
      gram_load<KIND, FULL, SPLIT>(J, cur.S, cur.ro, tid, R1);   // stage t + 3
      cursor_next(cur, slices, n_slices, P);
    }
    store(R0, buf ^ 1);                                           // stage t + 2
    compute(buf);
    __syncthreads();
    buf ^= 1;
  }
  // here t + 2 >= n_stages: stages t (in LDS) and, if t + 1 < n_stages, t + 1 (in R1)
  if (t + 1 < n_stages) {
    store(R1, buf ^ 1);
    compute(buf);
    __syncthreads();
    buf ^= 1;
  }
  if (n_stages > 0) compute(buf);

  BLM_GLOBAL double* base = as_global(out);
  if constexpr (MAIN) {
#pragma unroll
    for (int x = 0; x < 2; ++x)
#pragma unroll
      for (int y = 0; y < 2; ++y)
#pragma unroll
        for (int rr = 0; rr < 4; ++rr) {
          const int row = 32 * wr + 16 * x + 4 * rr + k4;
          const int col = 32 * wc + 16 * y + i16;
          base[row * GT + col] = P0[x][y][rr];
          base[GT * GT + row * GT + col] = P1[x][y][rr];
          if (KIND == JOB_OFF) base[2 * GT * GT + row * GT + col] = P2[x][y][rr];
        }
  }
  if constexpr (KIND == JOB_STRIP) {
    // strips of the job's groups: product q in slot q, [NAUX * ng][GT]
#pragma unroll
    for (int g = 0; g < STRIP_GROUPS; ++g) {
      if (g >= ng) continue;
#pragma unroll
      for (int rr = 0; rr < 4; ++rr) {
        const int a = NAUX * g + 4 * rr + k4;
        const int c = 16 * wv + i16;
        base[0 * GT * GT + a * GT + c] = P0[g >> 1][g & 1][rr];
        base[1 * GT * GT + a * GT + c] = P1[g >> 1][g & 1][rr];
        base[2 * GT * GT + a * GT + c] = P2[g >> 1][g & 1][rr];
      }
    }
  } else if constexpr (STRIPS) {
    // strips: [3][NAUX][GT] in the third slot
#pragma unroll
    for (int rr = 0; rr < 4; ++rr) {
      const int a = 4 * rr + k4;
      const int c = 16 * wv + i16;
      base[2 * GT * GT + 0 * NAUX * GT + a * GT + c] = P2[0][0][rr];
      base[2 * GT * GT + 1 * NAUX * GT + a * GT + c] = P2[0][1][rr];
      base[2 * GT * GT + 2 * NAUX * GT + a * GT + c] = P2[1][0][rr];
    }
  }
}

// VEC: every job's columns are 16-byte aligned (even leading dimension and
// tile origins, aligned panels), so full 64 x 64 tiles use 16-byte loads.
// SPLIT: the jobs are strip jobs on BF16 split or FP8 storage, plus the aux job.
// STAGE2: the stage-two Gram (same code; its own instantiation, so that
// kernel traces tell it from the block build by name).
template <bool VEC, bool SPLIT, bool STAGE2>
__global__ __launch_bounds__(GTHREADS, 2) void gram_kernel(const GramJob* __restrict__ jobs,
                                                           int n_jobs,
                                                           const Slice* __restrict__ slices,
                                                           int n_slices, int P,
                                                           double* __restrict__ partial,
                                                           const int2* __restrict__ sets) {
  // XCD-aware order: the hardware deals workgroups round-robin over the 8
  // XCDs; give each XCD a contiguous range of work items so that the tiles of
  // one block and one slice set (which share their sample panels) run on the
  // same L2.
  const int G = gridDim.x, g = blockIdx.x;
  const int q = G >> 3, r = G & 7, xcd = g & 7, idx = g >> 3;
  const int wid = (xcd < r) ? xcd * (q + 1) + idx : r * (q + 1) + (xcd - r) * q + idx;
  const int p = wid / n_jobs, jid = wid % n_jobs;
  const GramJob J = jobs[jid];
  if (sets) {
    const int2 ss = sets[J.set];
    slices += ss.x;
    n_slices = ss.y;
  }
  __shared__ GramLds L;
  double* out = partial + ((size_t)jid * P + p) * (size_t)(3 * GT * GT);
  const bool full = VEC && J.mi == GT && J.nj == GT;
  if constexpr (SPLIT) {
    if (J.kind == JOB_STRIP) gram_body<JOB_STRIP, false, true>(L, J, slices, n_slices, P, p, out);
    else gram_body<JOB_AUX, false, false>(L, J, slices, n_slices, P, p, out);
  } else {
    switch (J.kind) {
      case JOB_OFF:
        if (full) gram_body<JOB_OFF, VEC, false>(L, J, slices, n_slices, P, p, out);
        else gram_body<JOB_OFF, false, false>(L, J, slices, n_slices, P, p, out);
        break;
      case JOB_DIAG:
        if (full) gram_body<JOB_DIAG, VEC, false>(L, J, slices, n_slices, P, p, out);
        else gram_body<JOB_DIAG, false, false>(L, J, slices, n_slices, P, p, out);
        break;
      case JOB_DIAG_NOSTRIP:
        if (full) gram_body<JOB_DIAG_NOSTRIP, VEC, false>(L, J, slices, n_slices, P, p, out);
        else gram_body<JOB_DIAG_NOSTRIP, false, false>(L, J, slices, n_slices, P, p, out);
        break;
      case JOB_STRIP:
        if (full) gram_body<JOB_STRIP, VEC, false>(L, J, slices, n_slices, P, p, out);
        else gram_body<JOB_STRIP, false, false>(L, J, slices, n_slices, P, p, out);
        break;
      default:
        gram_body<JOB_AUX, false, false>(L, J, slices, n_slices, P, p, out);
        break;
    }
  }
}

__global__ __launch_bounds__(256) void gram_reduce_kernel(const GramJob* __restrict__ jobs, int P,
                                                          const double* __restrict__ partial,
                                                          double* __restrict__ s_base,
                                                          double* __restrict__ h_base,
                                                          double* __restrict__ strip_base,
                                                          int64_t strip_ld, int strip_rows) {
  const int jid = blockIdx.x, qd = blockIdx.y;
  const GramJob J = jobs[jid];
  if (J.kind == JOB_STRIP) {
    // product qd of the job's groups: [NAUX * ng][GT] in slot qd
    const int n_st = NAUX * J.ng * GT;
    for (int el = blockIdx.z * blockDim.x + threadIdx.x; el < n_st; el += blockDim.x * gridDim.z) {
      double sum = 0.0;
      for (int pp = 0; pp < P; ++pp)
        sum += partial[((size_t)jid * P + pp) * (size_t)(3 * GT * GT) + (size_t)qd * GT * GT + el];
      const int a = el / GT, c = el % GT;
      if (c < J.mi) strip_base[((size_t)qd * strip_rows + J.ag + a) * strip_ld + J.strip_col + c] += sum;
    }
    return;
  }
  const bool strips = J.kind == JOB_DIAG;
  if (qd == 2 && J.kind != JOB_OFF && !strips) return;
  if (!h_base && (qd == 1 || (qd == 2 && !strips))) return;   // H products not kept
  const int n_el = (qd == 2 && strips) ? 3 * NAUX * GT : GT * GT;
  for (int el = blockIdx.z * blockDim.x + threadIdx.x; el < n_el; el += blockDim.x * gridDim.z) {
    double sum = 0.0;
    for (int pp = 0; pp < P; ++pp)
      sum += partial[((size_t)jid * P + pp) * (size_t)(3 * GT * GT) + (size_t)qd * GT * GT + el];
    if (qd == 2 && strips) {
      const int sq = el / (NAUX * GT), a = (el / GT) % NAUX, c = el % GT;
      if (c < J.mi)
        strip_base[((size_t)sq * strip_rows + J.ag + a) * strip_ld + J.strip_col + c] += sum;
      continue;
    }
    const int row = el / GT, col = el % GT;
    if (row >= J.mi || col >= J.nj) continue;
    if (qd == 0) s_base[J.s_off + row * J.ld_out + col] += sum;
    else if (qd == 1) h_base[J.h_off + row * J.ld_out + col] += sum;
    else h_base[J.ht_off + col * J.ld_out + row] += sum;
  }
}

void launch_gram(const GramJob* d_jobs, int n_jobs, const Slice* d_slices, int n_slices, int P,
                 bool vec, bool split, bool stage2, double* d_partial, hipStream_t st, const int2* d_sets) {
  if (n_jobs <= 0) return;
  const dim3 grid(n_jobs * P), block(GTHREADS);
  if (split)
    hipLaunchKernelGGL((gram_kernel<false, true, false>), grid, block, 0, st, d_jobs, n_jobs, d_slices, n_slices, P,
                       d_partial, d_sets);
  else if (stage2 && vec)
    hipLaunchKernelGGL((gram_kernel<true, false, true>), grid, block, 0, st, d_jobs, n_jobs, d_slices, n_slices, P,
                       d_partial, d_sets);
  else if (stage2)
    hipLaunchKernelGGL((gram_kernel<false, false, true>), grid, block, 0, st, d_jobs, n_jobs, d_slices, n_slices,
                       P, d_partial, d_sets);
  else if (vec)
    hipLaunchKernelGGL((gram_kernel<true, false, false>), grid, block, 0, st, d_jobs, n_jobs, d_slices, n_slices,
                       P, d_partial, d_sets);
  else
    hipLaunchKernelGGL((gram_kernel<false, false, false>), grid, block, 0, st, d_jobs, n_jobs, d_slices, n_slices,
                       P, d_partial, d_sets);
}

void launch_gram_reduce(const GramJob* d_jobs, int n_jobs, int P, const double* d_partial,
                        double* s_base, double* h_base, double* strip_base, int64_t strip_ld,
                        int strip_rows, hipStream_t st) {
  if (n_jobs <= 0) return;
  // the elements of a tile split over gridDim.z when there are many slice
  // groups to sum (each element is still summed by one thread, in order)
  const int z = std::min(16, std::max(1, P / 8));
  hipLaunchKernelGGL(gram_reduce_kernel, dim3(n_jobs, 3, z), dim3(256), 0, st, d_jobs, P, d_partial,
                     s_base, h_base, strip_base, strip_ld, strip_rows);
}

// ---------------------------------------------------------------------------
// projection onto per-block directions
// ---------------------------------------------------------------------------

constexpr int PJ_ROWS = 64;   // samples per workgroup (16 per wave)
constexpr int PJ_P = 32;      // parameters per LDS stage
constexpr int PJ_D = 32;      // directions per pass (2 MFMA column groups)

struct PjRegs {
  double o[8], e[8], d[4];
};

// Stage loader: 64 samples x 32 parameters of O and e, and 32 directions x
// 32 parameters of the direction rows.  VEC: 16-byte loads (the caller has
// checked alignment); otherwise 8-byte loads.
template <bool VEC, int ST>
__device__ __forceinline__ void pj_load(const ProjChunk& C, int64_t s0, const DirBlock& B, int dg,
                                        int p0, const double* const* __restrict__ dir_ptr, int tid,
                                        PjRegs& R) {
  if (ST != STORE_F64) {
    // thread -> (8-sample group g, parameter col): 8 samples of O and of e
    const int col = tid & 31, g = tid >> 5;
    const int64_t r0 = s0 + 8 * g;
    const bool ok = r0 < C.n && p0 + col < B.m;
    if constexpr (ST == STORE_FP8) {
      // loads at a clamped (in-bounds) group and column, then zeros outside:
      // no divergent branch, whose merged values the compiler kept in scratch
      const int64_t grp = min(r0, C.n - 1) >> 3;
      const int64_t cc = B.col0 + min(p0 + col, B.m - 1);
      double o[8], e[8];
      fp8_load8(C.O, C.Or, C.Ot, C.Os, C.ld, grp, cc, o);
      fp8_load8(C.e, C.er, C.et, C.es, C.ld, grp, cc, e);
#pragma unroll
      for (int k = 0; k < 8; ++k) {
        R.o[k] = ok ? o[k] : 0.0;
        R.e[k] = ok ? e[k] : 0.0;
      }
    } else if (ok) {
      split_load8(C.O, C.ld, C.pstride, C.pieces, r0 >> 3, B.col0 + p0 + col, R.o);
      split_load8(C.e, C.ld, C.pstride, C.pieces, r0 >> 3, B.col0 + p0 + col, R.e);
    } else {
#pragma unroll
      for (int k = 0; k < 8; ++k) R.o[k] = R.e[k] = 0.0;
    }
  } else if (VEC) {
    const int c2 = (tid & 15) * 2;
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      const int row = (tid >> 4) + 16 * i;
      const int64_t s = s0 + row;
      const bool v = (s < C.n) && (p0 + c2 < B.m);
      if (v) {
        const double2 a = *reinterpret_cast<const BLM_GLOBAL double2*>(
            as_global((const double*)C.O) + s * C.ld + B.col0 + p0 + c2);
        const double2 b = *reinterpret_cast<const BLM_GLOBAL double2*>(
            as_global((const double*)C.e) + s * C.ld + B.col0 + p0 + c2);
        R.o[2 * i] = a.x;
        R.o[2 * i + 1] = a.y;
        R.e[2 * i] = b.x;
        R.e[2 * i + 1] = b.y;
      } else {
        R.o[2 * i] = R.o[2 * i + 1] = R.e[2 * i] = R.e[2 * i + 1] = 0.0;
      }
    }
  } else {
    const int col = tid & 31;
#pragma unroll
    for (int i = 0; i < 8; ++i) {
      const int row = (tid >> 5) + 8 * i;
      const int64_t s = s0 + row;
      const bool v = (s < C.n) && (p0 + col < B.m);
      R.o[i] = v ? as_global((const double*)C.O)[s * C.ld + B.col0 + p0 + col] : 0.0;
      R.e[i] = v ? as_global((const double*)C.e)[s * C.ld + B.col0 + p0 + col] : 0.0;
    }
  }
  const int col = tid & 31;
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    const int dr = (tid >> 5) + 8 * i;
    const int dd = dg + dr;
    R.d[i] = (dd < B.nd && p0 + col < B.m) ? as_global(dir_ptr[B.d0 + dd])[p0 + col] : 0.0;
  }
}

template <bool VEC, int ST>
__device__ __forceinline__ void pj_store(double (*sO)[PJ_P + 1], double (*sE)[PJ_P + 1],
                                         double (*sD)[PJ_P + 1], int tid, const PjRegs& R) {
  if (ST != STORE_F64) {
    const int col = tid & 31, g = tid >> 5;
#pragma unroll
    for (int k = 0; k < 8; ++k) {
      sO[8 * g + k][col] = R.o[k];
      sE[8 * g + k][col] = R.e[k];
    }
  } else if (VEC) {
    const int c2 = (tid & 15) * 2;
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      const int row = (tid >> 4) + 16 * i;
      sO[row][c2] = R.o[2 * i];
      sO[row][c2 + 1] = R.o[2 * i + 1];
      sE[row][c2] = R.e[2 * i];
      sE[row][c2 + 1] = R.e[2 * i + 1];
    }
  } else {
    const int col = tid & 31;
#pragma unroll
    for (int i = 0; i < 8; ++i) {
      const int row = (tid >> 5) + 8 * i;
      sO[row][col] = R.o[i];
      sE[row][col] = R.e[i];
    }
  }
  const int col = tid & 31;
#pragma unroll
  for (int i = 0; i < 4; ++i) sD[(tid >> 5) + 8 * i][col] = R.d[i];
}

template <bool VEC, int ST>
__global__ __launch_bounds__(256) void dirproj_kernel(const ProjChunk* __restrict__ chunks, int n_chunks) {
  __shared__ double sO[PJ_ROWS][PJ_P + 1];
  __shared__ double sE[PJ_ROWS][PJ_P + 1];
  __shared__ double sD[PJ_D][PJ_P + 1];
  // which chunk and which 64-sample tile of it
  int ci = 0;
  while (ci + 1 < n_chunks && chunks[ci + 1].tile0 <= (int)blockIdx.x) ++ci;
  const ProjChunk C = chunks[ci];
  const int64_t s0 = (int64_t)(blockIdx.x - C.tile0) * PJ_ROWS;
  const DirBlock* __restrict__ blocks = C.blocks;
  const double* const* __restrict__ dir_ptr = C.dir;
  const int n_blocks = C.n_blocks, n_dirs = C.n_dirs;
  const int64_t ldo = C.ldo;
  BLM_GLOBAL double* X = as_global(C.Xo) + C.row_base * ldo;
  BLM_GLOBAL double* Y = as_global(C.Yo) + C.row_base * ldo;
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  const int i16 = lane & 15, k4 = lane >> 4;

  // column 0 (the wave function itself: 1 and E_L) and the padding columns
  for (int t = tid; t < PJ_ROWS * (int)ldo; t += blockDim.x) {
    const int rr = t / (int)ldo, c = t % (int)ldo;
    const int64_t s = s0 + rr;
    if (s >= C.n) continue;
    if (c == 0) {
      X[s * ldo] = 1.0;
      Y[s * ldo] = as_global(C.EL)[s];
    } else if (c >= 1 + n_dirs) {
      X[s * ldo + c] = 0.0;
      Y[s * ldo + c] = 0.0;
    }
  }

  for (int bi = 0; bi < n_blocks; ++bi) {
    const DirBlock B = blocks[bi];
    for (int dg = 0; dg < B.nd; dg += PJ_D) {
      const bool two = (B.nd - dg) > 16;
      d4 aO0 = {0, 0, 0, 0}, aO1 = {0, 0, 0, 0}, aE0 = {0, 0, 0, 0}, aE1 = {0, 0, 0, 0};
      PjRegs R;
      pj_load<VEC, ST>(C, s0, B, dg, 0, dir_ptr, tid, R);
      for (int p0 = 0; p0 < B.m; p0 += PJ_P) {
        __syncthreads();   // everyone is done reading the previous stage
        pj_store<VEC, ST>(sO, sE, sD, tid, R);
        __syncthreads();
        // the next stage's global loads overlap this stage's matrix-core work
        if (p0 + PJ_P < B.m) pj_load<VEC, ST>(C, s0, B, dg, p0 + PJ_P, dir_ptr, tid, R);
#pragma unroll
        for (int kk = 0; kk < PJ_P; kk += 4) {
          const int kc = kk + k4;
          const double ao = sO[16 * wv + i16][kc], ae = sE[16 * wv + i16][kc];
          const double b0 = sD[i16][kc];
          aO0 = mfma_f64(ao, b0, aO0);
          aE0 = mfma_f64(ae, b0, aE0);
          if (two) {
            const double b1 = sD[16 + i16][kc];
            aO1 = mfma_f64(ao, b1, aO1);
            aE1 = mfma_f64(ae, b1, aE1);
          }
        }
      }
#pragma unroll
      for (int rr = 0; rr < 4; ++rr) {
        const int64_t s = s0 + 16 * wv + 4 * rr + k4;
        if (s >= C.n) continue;
        const int t0 = dg + i16, t1 = dg + 16 + i16;
        if (t0 < B.nd) {
          X[s * ldo + 1 + B.d0 + t0] = aO0[rr];
          Y[s * ldo + 1 + B.d0 + t0] = aE0[rr];
        }
        if (two && t1 < B.nd) {
          X[s * ldo + 1 + B.d0 + t1] = aO1[rr];
          Y[s * ldo + 1 + B.d0 + t1] = aE1[rr];
        }
      }
    }
  }
}

// Split or FP8 storage when every block has at most PJ_SMALL directions (the
// previous-step directions of Eq. 9, one or two per block): each thread
// keeps FP64 sums for its 8 samples and its column of every 32-parameter
// stage with plain FMAs, then one reduction over the 32 columns per block.
// The matrix-core kernel would spend 15/16 of its products on padding
// directions here (FP64 vector and matrix peaks are equal on this chip).
// No LDS and no barriers.
constexpr int PJ_SMALL = 2;

template <int ST>
__global__ __launch_bounds__(256) void dirproj_small_kernel(const ProjChunk* __restrict__ chunks, int n_chunks) {
  int ci = 0;
  while (ci + 1 < n_chunks && chunks[ci + 1].tile0 <= (int)blockIdx.x) ++ci;
  const ProjChunk C = chunks[ci];
  const int64_t s0 = (int64_t)(blockIdx.x - C.tile0) * PJ_ROWS;
  const DirBlock* __restrict__ blocks = C.blocks;
  const double* const* __restrict__ dir_ptr = C.dir;
  const int n_blocks = C.n_blocks, n_dirs = C.n_dirs;
  const int64_t ldo = C.ldo;
  BLM_GLOBAL double* X = as_global(C.Xo) + C.row_base * ldo;
  BLM_GLOBAL double* Y = as_global(C.Yo) + C.row_base * ldo;
  const int tid = threadIdx.x;
  // column 0 (the wave function itself: 1 and E_L) and the padding columns
  for (int t = tid; t < PJ_ROWS * (int)ldo; t += blockDim.x) {
    const int rr = t / (int)ldo, c = t % (int)ldo;
    const int64_t s = s0 + rr;
    if (s >= C.n) continue;
    if (c == 0) {
      X[s * ldo] = 1.0;
      Y[s * ldo] = as_global(C.EL)[s];
    } else if (c >= 1 + n_dirs) {
      X[s * ldo + c] = 0.0;
      Y[s * ldo + c] = 0.0;
    }
  }
  const int col = tid & 31, g = tid >> 5;
  const int64_t r0 = s0 + 8 * g;
  for (int bi = 0; bi < n_blocks; ++bi) {
    const DirBlock B = blocks[bi];
    if (B.nd <= 0) continue;
    double ao[PJ_SMALL][8], ae[PJ_SMALL][8];
#pragma unroll
    for (int dd = 0; dd < PJ_SMALL; ++dd)
#pragma unroll
      for (int k = 0; k < 8; ++k) ao[dd][k] = ae[dd][k] = 0.0;
    const BLM_GLOBAL double* dr[PJ_SMALL];
#pragma unroll
    for (int dd = 0; dd < PJ_SMALL; ++dd) dr[dd] = as_global(dir_ptr[B.d0 + min(dd, B.nd - 1)]);
    for (int p0 = 0; p0 < B.m; p0 += PJ_P) {
      double o[8], e[8], d[PJ_SMALL];
      const bool ok = r0 < C.n && p0 + col < B.m;
      if (ok) {
        if constexpr (ST == STORE_FP8) {
          fp8_load8(C.O, C.Or, C.Ot, C.Os, C.ld, r0 >> 3, B.col0 + p0 + col, o);
          fp8_load8(C.e, C.er, C.et, C.es, C.ld, r0 >> 3, B.col0 + p0 + col, e);
        } else {
          split_load8(C.O, C.ld, C.pstride, C.pieces, r0 >> 3, B.col0 + p0 + col, o);
          split_load8(C.e, C.ld, C.pstride, C.pieces, r0 >> 3, B.col0 + p0 + col, e);
        }
      } else {
#pragma unroll
        for (int k = 0; k < 8; ++k) o[k] = e[k] = 0.0;
      }
#pragma unroll
      for (int dd = 0; dd < PJ_SMALL; ++dd) d[dd] = (ok && dd < B.nd) ? dr[dd][p0 + col] : 0.0;
#pragma unroll
      for (int dd = 0; dd < PJ_SMALL; ++dd)
#pragma unroll
        for (int k = 0; k < 8; ++k) {
          ao[dd][k] += o[k] * d[dd];
          ae[dd][k] += e[k] * d[dd];
        }
    }
    // sums over the 32 columns (the lanes of one half wave)
#pragma unroll
    for (int dd = 0; dd < PJ_SMALL; ++dd)
#pragma unroll
      for (int k = 0; k < 8; ++k)
#pragma unroll
        for (int off = 16; off > 0; off >>= 1) {
          ao[dd][k] += __shfl_xor(ao[dd][k], off, 64);
          ae[dd][k] += __shfl_xor(ae[dd][k], off, 64);
        }
    if (col == 0) {
#pragma unroll
      for (int k = 0; k < 8; ++k) {
        const int64_t s = r0 + k;
        if (s >= C.n) continue;
#pragma unroll
        for (int dd = 0; dd < PJ_SMALL; ++dd)
          if (dd < B.nd) {
            X[s * ldo + 1 + B.d0 + dd] = ao[dd][k];
            Y[s * ldo + 1 + B.d0 + dd] = ae[dd][k];
          }
      }
    }
  }
}

// FP64 storage: each wave projects its own 16 samples with operands taken
// straight from global memory (no LDS, no barriers).  In matrix-core product
// j of a 32-parameter stage, lane group g = lane / 16 supplies parameter
// p0 + 8 g + j on both operand sides (the contraction runs over the same
// permutation of the parameters on both sides), so each lane reads 8
// consecutive parameters of its sample row, 64 contiguous bytes.  Loads are
// unconditional (rows clamped to the chunk, columns to the block) and the
// next stage is loaded before the current one is multiplied.
//
// VEC (even leading dimension, aligned arrays): every load is 16 bytes, in
// window coordinates: a block's window starts at the even column at or
// before its first one (sh = 1 for a block at an odd column) and is sh + m
// columns wide.  The directions come as window rows (zero at the column
// before an odd block, zero padding to an even width).  A sample row's last
// pair may reach one column past the block: the next block's first column,
// or the row's padding when N_V is odd (the leading dimension is even), so
// inside the [n][ld] array; sample values outside the window are zeroed in
// registers (the padding may hold anything).
struct Pj64Regs {
  double o[8], e[8], x0[8], x1[8];
};

// 8 values of a row from aligned column pairs starting at c0 (pairs past
// the last one, lp, repeat it)
__device__ __forceinline__ void pj64_row8_vec(const BLM_GLOBAL double* p, int c0, int lp, double* v) {
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    const int c = min(c0 + 2 * q, 2 * lp);
    const double2 t = *reinterpret_cast<const BLM_GLOBAL double2*>(p + c);
    v[2 * q] = t.x;
    v[2 * q + 1] = t.y;
  }
}

// 8 entries c0 .. c0 + 7 of a row, clamped to [0, m)
__device__ __forceinline__ void pj64_row8_scalar(const BLM_GLOBAL double* p, int c0, int m, double* v) {
#pragma unroll
  for (int q = 0; q < 8; ++q) v[q] = p[min(c0 + q, m - 1)];
}

// mw: the window width (sh + m with VEC, m without)
template <bool VEC>
__device__ __forceinline__ void pj64_load(const BLM_GLOBAL double* rO, const BLM_GLOBAL double* rE,
                                          const BLM_GLOBAL double* d0, const BLM_GLOBAL double* d1,
                                          bool two, int c0, int mw, Pj64Regs& R) {
  if constexpr (VEC) {
    const int lp = (mw - 1) >> 1;      // the last column pair holding a column of the block
    pj64_row8_vec(rO, c0, lp, R.o);
    pj64_row8_vec(rE, c0, lp, R.e);
    pj64_row8_vec(d0, c0, lp, R.x0);   // window rows: padded to an even width
    if (two) pj64_row8_vec(d1, c0, lp, R.x1);
  } else {
    pj64_row8_scalar(rO, c0, mw, R.o);
    pj64_row8_scalar(rE, c0, mw, R.e);
    pj64_row8_scalar(d0, c0, mw, R.x0);
    if (two) pj64_row8_scalar(d1, c0, mw, R.x1);
  }
}

// p: the window column of R's first value; the block holds window columns
// sh .. mw - 1.  MASK: sample values outside them are zeroed (a window with
// a column before the block or a pad column after it; otherwise every value
// loaded is the block's own, and those past mw meet zero directions)
template <bool MASK, bool TWO>
__device__ __forceinline__ void pj64_mul(const Pj64Regs& R, bool ok0, bool ok1, int p, int mw, int sh,
                                         d4& aO0, d4& aE0, d4& aO1, d4& aE1) {
#pragma unroll
  for (int j = 0; j < 8; ++j) {
    const bool inb = p + j < mw;
    const bool inw = inb && p + j >= sh;
    const double o = (MASK && !inw) ? 0.0 : R.o[j];
    const double e = (MASK && !inw) ? 0.0 : R.e[j];
    const double b0 = (ok0 && inb) ? R.x0[j] : 0.0;
    aO0 = mfma_f64(o, b0, aO0);
    aE0 = mfma_f64(e, b0, aE0);
    if constexpr (TWO) {
      const double b1 = (ok1 && inb) ? R.x1[j] : 0.0;
      aO1 = mfma_f64(o, b1, aO1);
      aE1 = mfma_f64(e, b1, aE1);
    }
  }
}

// All stages of one block for one direction group; two register stages
// alternate (stage t+1 is loaded while stage t is multiplied).  A window
// whose width is not a multiple of 64 multiplies one all-zero stage more.
template <bool VEC, bool MASK, bool TWO>
__device__ __forceinline__ void pj64_block(const BLM_GLOBAL double* rO, const BLM_GLOBAL double* rE,
                                           const BLM_GLOBAL double* d0, const BLM_GLOBAL double* d1,
                                           bool ok0, bool ok1, int mw, int sh, int g, d4& aO0, d4& aE0,
                                           d4& aO1, d4& aE1) {
  Pj64Regs Ra, Rb;
  pj64_load<VEC>(rO, rE, d0, d1, TWO, 8 * g, mw, Ra);
  for (int p0 = 0; p0 < mw; p0 += 2 * PJ_P) {
    pj64_load<VEC>(rO, rE, d0, d1, TWO, p0 + PJ_P + 8 * g, mw, Rb);
    pj64_mul<MASK, TWO>(Ra, ok0, ok1, p0 + 8 * g, mw, sh, aO0, aE0, aO1, aE1);
    pj64_load<VEC>(rO, rE, d0, d1, TWO, p0 + 2 * PJ_P + 8 * g, mw, Ra);
    pj64_mul<MASK, TWO>(Rb, ok0, ok1, p0 + PJ_P + 8 * g, mw, sh, aO0, aE0, aO1, aE1);
  }
}

template <bool VEC>
__global__ __launch_bounds__(256) void dirproj64_kernel(const ProjChunk* __restrict__ chunks, int n_chunks) {
  int ci = 0;
  while (ci + 1 < n_chunks && chunks[ci + 1].tile0 <= (int)blockIdx.x) ++ci;
  const ProjChunk C = chunks[ci];
  const int64_t s0 = (int64_t)(blockIdx.x - C.tile0) * PJ_ROWS;
  const DirBlock* __restrict__ blocks = C.blocks;
  const double* const* __restrict__ dir_ptr = C.dir;
  const int n_blocks = C.n_blocks, n_dirs = C.n_dirs;
  const int64_t ldo = C.ldo;
  BLM_GLOBAL double* X = as_global(C.Xo) + C.row_base * ldo;
  BLM_GLOBAL double* Y = as_global(C.Yo) + C.row_base * ldo;
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  const int i16 = lane & 15, g = lane >> 4;

  // column 0 (the wave function itself: 1 and E_L) and the padding columns
  for (int t = tid; t < PJ_ROWS * (int)ldo; t += blockDim.x) {
    const int rr = t / (int)ldo, c = t % (int)ldo;
    const int64_t s = s0 + rr;
    if (s >= C.n) continue;
    if (c == 0) {
      X[s * ldo] = 1.0;
      Y[s * ldo] = as_global(C.EL)[s];
    } else if (c >= 1 + n_dirs) {
      X[s * ldo + c] = 0.0;
      Y[s * ldo + c] = 0.0;
    }
  }

  const int64_t sw = s0 + 16 * wv;                      // first sample of this wave
  const int64_t sl = min(sw + i16, C.n - 1);            // this lane's (clamped) sample row
  const BLM_GLOBAL double* rowO = as_global((const double*)C.O) + sl * C.ld;
  const BLM_GLOBAL double* rowE = as_global((const double*)C.e) + sl * C.ld;
  for (int bi = 0; bi < n_blocks; ++bi) {
    const DirBlock B = blocks[bi];
    const int sh = VEC ? (int)(B.col0 & 1) : 0;    // window from the even column at or before the block
    const int mw = B.m + sh;
    const BLM_GLOBAL double* rO = rowO + B.col0 - sh;
    const BLM_GLOBAL double* rE = rowE + B.col0 - sh;
    const double* const* dtab = VEC ? C.dirw : dir_ptr;
    for (int dg = 0; dg < B.nd; dg += 32) {
      const bool two = (B.nd - dg) > 16;
      const int t0 = dg + i16, t1 = dg + 16 + i16;
      const bool ok0 = t0 < B.nd, ok1 = two && t1 < B.nd;
      const BLM_GLOBAL double* d0 = as_global(dtab[B.d0 + min(t0, B.nd - 1)]);
      const BLM_GLOBAL double* d1 = as_global(dtab[B.d0 + min(t1, B.nd - 1)]);
      d4 aO0 = {0, 0, 0, 0}, aO1 = {0, 0, 0, 0}, aE0 = {0, 0, 0, 0}, aE1 = {0, 0, 0, 0};
      const bool mask = VEC && (sh != 0 || (mw & 1) != 0);
      if (mask) {
        if (two) pj64_block<VEC, VEC, true>(rO, rE, d0, d1, ok0, ok1, mw, sh, g, aO0, aE0, aO1, aE1);
        else pj64_block<VEC, VEC, false>(rO, rE, d0, d1, ok0, ok1, mw, sh, g, aO0, aE0, aO1, aE1);
      } else {
        if (two) pj64_block<VEC, false, true>(rO, rE, d0, d1, ok0, ok1, mw, sh, g, aO0, aE0, aO1, aE1);
        else pj64_block<VEC, false, false>(rO, rE, d0, d1, ok0, ok1, mw, sh, g, aO0, aE0, aO1, aE1);
      }
      // lane holds D[4 rr + g][i16]: sample sw + 4 rr + g, direction dg + i16 (+16)
#pragma unroll
      for (int rr = 0; rr < 4; ++rr) {
        const int64_t s = sw + 4 * rr + g;
        if (s >= C.n) continue;
        if (ok0) {
          X[s * ldo + 1 + B.d0 + t0] = aO0[rr];
          Y[s * ldo + 1 + B.d0 + t0] = aE0[rr];
        }
        if (ok1) {
          X[s * ldo + 1 + B.d0 + t1] = aO1[rr];
          Y[s * ldo + 1 + B.d0 + t1] = aE1[rr];
        }
      }
    }
  }
}

__global__ __launch_bounds__(256) void window_copy_kernel(const WinCopy* __restrict__ tab, int n) {
  const WinCopy W = tab[blockIdx.y];
  for (int r = blockIdx.x * blockDim.x + threadIdx.x; r < W.mwp; r += gridDim.x * blockDim.x) {
    const int x = r - W.sh;
    as_global(W.dst)[r] = (x >= 0 && x < W.m) ? as_global(W.src)[x] : 0.0;
  }
}

void launch_window_copy(const WinCopy* d_tab, int n, int max_mwp, hipStream_t st) {
  if (n <= 0 || max_mwp <= 0) return;
  hipLaunchKernelGGL(window_copy_kernel, dim3((max_mwp + 255) / 256, n), dim3(256), 0, st, d_tab, n);
}

void launch_dirproj(const ProjChunk* d_chunks, int n_chunks, int n_tiles, bool vec, int store, int max_nd,
                    hipStream_t st) {
  if (n_tiles <= 0) return;
  if (store != STORE_F64 && max_nd <= PJ_SMALL) {
    if (store == STORE_BF16)
      hipLaunchKernelGGL((dirproj_small_kernel<STORE_BF16>), dim3(n_tiles), dim3(256), 0, st, d_chunks, n_chunks);
    else
      hipLaunchKernelGGL((dirproj_small_kernel<STORE_FP8>), dim3(n_tiles), dim3(256), 0, st, d_chunks, n_chunks);
  } else if (store == STORE_BF16)
    hipLaunchKernelGGL((dirproj_kernel<false, STORE_BF16>), dim3(n_tiles), dim3(256), 0, st, d_chunks, n_chunks);
  else if (store == STORE_FP8)
    hipLaunchKernelGGL((dirproj_kernel<false, STORE_FP8>), dim3(n_tiles), dim3(256), 0, st, d_chunks, n_chunks);
  else if (vec)
    hipLaunchKernelGGL((dirproj64_kernel<true>), dim3(n_tiles), dim3(256), 0, st, d_chunks, n_chunks);
  else
    hipLaunchKernelGGL((dirproj64_kernel<false>), dim3(n_tiles), dim3(256), 0, st, d_chunks, n_chunks);
}

}  // namespace blm
