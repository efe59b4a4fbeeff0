// Dense shifted generalised eigensolver for the BLM pencils, FP64
// (H' c = lambda S c, S symmetric positive definite, H' not symmetric).
// launch_eig runs every step on one 1024-thread workgroup per pencil;
// launch_eig_split runs steps 1 to 3 on several workgroups per pencil
// (cooperative launches for 1 and 3, independent slices for 2) and the
// rest on one:
//
//   1. S = L L^T (Cholesky)                      -> BLM_E_S_NOT_PD if it fails
//   2. A = L^-1 H' L^-T (two triangular solves)
//   3. A = Q Hs Q^T, Hs upper Hessenberg (Householder reflectors kept)
//   4. eigenvalues of Hs: Francis implicit double-shift QR sweeps on the
//      active window with deflation (Golub & Van Loan, Sec. 7.5)
//   5. rank by real part (ties: larger imaginary part first), take the
//      lowest ones: a complex conjugate pair is taken whole
//   6. eigenvectors of the chosen eigenvalues by inverse iteration on Hs
//      (complex shift for a pair), then back to the pencil: c = L^-T Q y
//   7. block problems: the parameter part of Re c (and Im c for a pair),
//      orthonormalised by modified Gram-Schmidt -> kept directions (Eq. 6);
//      stage two: the chosen eigenvector itself (Eq. 7, Eq. 8).
//
// The ranking of eigenvalues as update directions follows Sec. II.B of the
// paper (lowest eigenvalue = best direction).
#include <float.h>

#include "blm_internal.h"

namespace blm {

namespace {

constexpr int NT = EIG_THREADS;
constexpr int HKW_MAX = 32;           // workgroups per pencil in the distributed Cholesky and Hessenberg steps
// smallest pencil it takes (smaller ones stay on one workgroup); its
// workspace, 2 d + 2 kw d doubles, fits in the 2 d^2 of W
constexpr int HESS_MULTI_MIN = 256;
static_assert(2 * HESS_MULTI_MIN >= 2 + 2 * HKW_MAX, "workspace of the distributed reduction");
enum : int { PH_CHOL = 1, PH_HESS = 2, PH_BACK = 4, PH_CONG = 8, PH_ALL = 15 };
constexpr int NW = NT / 64;
constexpr double EPS = DBL_EPSILON;
constexpr double DROP_TOL = 1e-12;

constexpr int AEDMAX = 64;            // largest deflation window
constexpr int AEDLD = AEDMAX + 1;     // LDS row stride of the window arrays
constexpr int MAX_BULGES = 16;
// bulge chase: ticks per batch (8 measured as fast as 12 and faster than 16,
// whose register segments spill), largest diagonal window (at most
// CT + 4 m for m <= MAX_BULGES bulges), its LDS row stride
constexpr int CT = 8;
constexpr int CWMAX = CT + 4 * MAX_BULGES + 4;
constexpr int CWLD = CWMAX + 1;
static_assert(CWMAX >= CT + 4 * MAX_BULGES + 2, "a batch's window must fit");

struct ChaseRec {
  double v0, v1, v2, bt;              // reflector I - bt v v^T; bt = 0: none
};

struct Shared {
  union {
    // Cholesky, Hessenberg reduction, selection, inverse iteration
    struct {
      double v1[EIG_MAXD];
      double v2[EIG_MAXD];
      double v3[EIG_MAXD];
      double v4[EIG_MAXD];
    };
    // congruence (stage) and the QR phase (stage, and the deflation window,
    // its Schur vectors, the spike and the window's eigenvalues)
    struct {
      double stage[16][256];
      union {
        struct {
          double aT[AEDMAX][AEDLD];
          double aZ[AEDMAX][AEDLD];
        };
        double cw[CWMAX][CWLD];       // bulge chase: the diagonal window of a batch
      };
      double au[AEDMAX], av[AEDMAX];
      double ewr[AEDMAX], ewi[AEDMAX];
      ChaseRec rec[CT][MAX_BULGES];   // bulge chase: reflectors of a batch [tick][bulge]
    };
  };
  double red[NW];
  double sc[16];
  int isc[16];
  unsigned char mark[EIG_MAXD];
  double sel_r[EIG_MAXSEL], sel_i[EIG_MAXSEL];
  int sel_n;
  int widx[NW];
  // multishift QR: shifts of the trailing block and per-bulge state
  double T[32 * 32];
  double swr[32], swi[32], sre[32];
  double bsum[16], bprod[16];
  double bx[16][3];
  // QR statistics: 100 MHz ticks in early deflation and in bulge chases,
  // number of early deflations and of chases
  unsigned long long qst[4];
};

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
  return v;
}

// value of v in lane src (src the same in every lane)
__device__ __forceinline__ double lane_bcast(double v, int src) {
  const uint64_t b = __double_as_longlong(v);
  const uint32_t lo = __builtin_amdgcn_readlane((uint32_t)b, src);
  const uint32_t hi = __builtin_amdgcn_readlane((uint32_t)(b >> 32), src);
  return __longlong_as_double((long long)(((uint64_t)hi << 32) | lo));
}

// modulus of x + i y; |x| when y is zero
__device__ __forceinline__ double cmod(double x, double y) { return (y == 0.0) ? fabs(x) : hypot(x, y); }

__device__ __forceinline__ double wave_max(double v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v = fmax(v, __shfl_xor(v, off, 64));
  return v;
}

// Sum over the workgroup, same value returned to every thread, fixed order.
__device__ double block_sum(Shared& sh, double v) {
  v = wave_sum(v);
  if ((threadIdx.x & 63) == 0) sh.red[threadIdx.x >> 6] = v;
  __syncthreads();
  double t = 0.0;
#pragma unroll
  for (int i = 0; i < NW; ++i) t += sh.red[i];
  __syncthreads();
  return t;
}

__device__ double block_max(Shared& sh, double v) {
  v = wave_max(v);
  if ((threadIdx.x & 63) == 0) sh.red[threadIdx.x >> 6] = v;
  __syncthreads();
  double t = sh.red[0];
#pragma unroll
  for (int i = 1; i < NW; ++i) t = fmax(t, sh.red[i]);
  __syncthreads();
  return t;
}

// ---------------------------------------------------------------- step 1 --
__device__ int cholesky(Shared& sh, gdouble* S, int d) {
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  for (int k = 0; k < d; ++k) {
    if (tid == 0) {
      const double v = S[(size_t)k * d + k];
      int st = EIG_OK;
      if (!isfinite(v)) st = EIG_NONFINITE;
      else if (!(v > 0.0)) st = EIG_NOT_PD;
      sh.isc[0] = st;
      sh.sc[0] = st == EIG_OK ? sqrt(v) : 1.0;
      if (st == EIG_OK) S[(size_t)k * d + k] = sh.sc[0];
    }
    __syncthreads();
    const int st = sh.isc[0];
    const double piv = sh.sc[0];
    if (st != EIG_OK) return st;
    for (int i = k + 1 + tid; i < d; i += NT) {
      const double x = S[(size_t)i * d + k] / piv;
      S[(size_t)i * d + k] = x;
      sh.v1[i] = x;
    }
    __syncthreads();
    for (int i = k + 1 + wv; i < d; i += NW) {
      const double li = sh.v1[i];
      gdouble* Si = S + (size_t)i * d;
      for (int j = k + 1 + lane; j <= i; j += 64) Si[j] -= li * sh.v1[j];
    }
    __syncthreads();
  }
  return EIG_OK;
}

// ---------------------------------------------------------------- step 2 --
// In place X <- L^-1 X for an n x n row-major X (L in the lower triangle of
// Lm), 16 rows at a time: the block's rows are solved in turn, staged in LDS
// by column chunks, and subtracted from all rows below in one pass (each
// trailing element is read and written once per 16 rows of L).
constexpr int CB = 16;       // rows per block
constexpr int CCH = 256;     // columns per LDS chunk

__device__ void lower_solve_rows(Shared& sh, const gdouble* Lm, gdouble* X, int n) {
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  for (int k0 = 0; k0 < n; k0 += CB) {
    const int kb = min(CB, n - k0);
    // diagonal block: rows k0 .. k0+kb-1, in order
    for (int kk = k0; kk < k0 + kb; ++kk) {
      const double lkk = Lm[(size_t)kk * n + kk];
      for (int j = tid; j < n; j += NT) {
        double v = X[(size_t)kk * n + j];
        for (int m = k0; m < kk; ++m) v -= Lm[(size_t)kk * n + m] * X[(size_t)m * n + j];
        X[(size_t)kk * n + j] = v / lkk;
      }
      __syncthreads();
    }
    // trailing rows, by column chunks staged in LDS
    for (int c0 = 0; c0 < n; c0 += CCH) {
      const int cw = min(CCH, n - c0);
      for (int t = tid; t < kb * CCH; t += NT) {
        const int m = t / CCH, j = t % CCH;
        sh.stage[m][j] = (j < cw) ? X[(size_t)(k0 + m) * n + c0 + j] : 0.0;
      }
      __syncthreads();
      for (int i = k0 + kb + wv; i < n; i += NW) {
        double l[CB];
#pragma unroll
        for (int m = 0; m < CB; ++m) l[m] = (m < kb) ? Lm[(size_t)i * n + k0 + m] : 0.0;
        gdouble* Xi = X + (size_t)i * n + c0;
        for (int j = lane; j < cw; j += 64) {
          double acc = Xi[j];
#pragma unroll
          for (int m = 0; m < CB; ++m) acc -= l[m] * sh.stage[m][j];
          Xi[j] = acc;
        }
      }
      __syncthreads();
    }
  }
}

// B <- A^T for n x n row-major matrices (distinct buffers).
__device__ void transpose(const gdouble* A, gdouble* B, int n) {
  const int tid = threadIdx.x;
  for (size_t t = tid; t < (size_t)n * n; t += NT) {
    const int i = (int)(t / n), j = (int)(t % n);
    B[(size_t)j * n + i] = A[t];
  }
  __syncthreads();
}

// A <- L^-1 A L^-T, using W (n x n) as scratch: X = L^-1 A, then
// A^T = L^-1 X^T.
__device__ void congruence(Shared& sh, const gdouble* L, gdouble* A, gdouble* W, int d) {
  lower_solve_rows(sh, L, A, d);
  transpose(A, W, d);
  lower_solve_rows(sh, L, W, d);
  transpose(W, A, d);
}

// ---------------------------------------------------------------- step 3 --
// Householder reduction to upper Hessenberg form.  Reflector k acts on
// indices k+1..d-1 with vector v (v[k+1] = 1) stored in row k of V and
// scalar tau[k]: P_k = I - tau v v^T.  A = Q Hs Q^T with Q = P_0 P_1 ... .
//
// Both sides of step k: P A P = A - tau (p v^T + v q'^T) with p = A v,
// q = A^T v, beta = v^T p and q' = q - tau beta v (rows above k+1 only get
// p v^T).  One pass over the matrix per step: column k+1 after step k is
// formed first, which gives reflector k+1; the pass then writes step k's
// update and, from the values it has just written, accumulates step k+1's
// products p = A v (per row, one wave per row) and q = A^T v (per wave over
// its rows, summed in a fixed order through the Qs scratch, 16 x d).

// column value after a step: a - tau (p_i v_j + v_i q'_j)
__device__ __forceinline__ double hess_upd(double a, double tk, double pi, double vj, double vi,
                                           double qj) {
  return a - tk * (pi * vj + vi * qj);
}

// Reflector of step k from column values c[i] (rows k+1..d-1) held in
// vec[i]: on return vec holds v (zeros up to k, 1 at k+1), V row k and tau[k]
// are written; returns tau, and the new subdiagonal entry in *beta_h.
__device__ double hess_reflector(Shared& sh, double* vec, gdouble* V, gdouble* tau, int k, int d,
                                 double* beta_h) {
  const int tid = threadIdx.x;
  double part = 0.0;
  for (int i = k + 2 + tid; i < d; i += NT) part += vec[i] * vec[i];
  const double sigma = block_sum(sh, part);
  const double alpha = vec[k + 1];
  if (sigma == 0.0) {
    *beta_h = alpha;
    for (int i = tid; i < d; i += NT) {
      const double vi = (i == k + 1) ? 1.0 : 0.0;
      vec[i] = vi;
      if (i > k) V[(size_t)k * d + i] = vi;
    }
    if (tid == 0) tau[k] = 0.0;
    __syncthreads();
    return 0.0;
  }
  const double nrm = sqrt(alpha * alpha + sigma);
  const double bh = alpha <= 0.0 ? nrm : -nrm;
  const double v0 = alpha - bh;
  const double tk = (bh - alpha) / bh;
  for (int i = tid; i < d; i += NT) {
    const double vi = (i <= k) ? 0.0 : (i == k + 1) ? 1.0 : vec[i] / v0;
    vec[i] = vi;
    if (i > k) V[(size_t)k * d + i] = vi;
  }
  if (tid == 0) tau[k] = tk;
  __syncthreads();
  *beta_h = bh;
  return tk;
}

// One pass over rows 0..d-1, columns k+1..d-1.  UPD: apply step k (v = cv,
// p from Pg, q' = cq, scalar tk; column k set to beta_h e_(k+1)).  PROD:
// accumulate p_next = A' nv into pn (LDS, zeroed by the caller) and the
// per-wave partials of A'^T nv into Qs (columns k+2..d-1 when UPD, k+1..
// otherwise).  Two rows per wave at a time; loads unconditional (columns
// clamped), stores guarded.
template <bool UPD, bool PROD>
__device__ void hess_pass(Shared& sh, gdouble* A, int d, int k, double tk, double beta_h,
                          const double* cv, const gdouble* Pg, const double* cq, const double* nv,
                          double* pn, gdouble* Qs) {
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  constexpr int QCH = 4;                      // columns per lane per chunk (256 per chunk)
  const int j0 = k + 1, nj = d - j0;
  for (int c0 = 0; c0 < nj; c0 += 64 * QCH) {
    double qacc[QCH];
#pragma unroll
    for (int m = 0; m < QCH; ++m) qacc[m] = 0.0;
    for (int i = wv; i < d; i += 2 * NW) {
      const int i2 = i + NW;
      const bool has2 = i2 < d;
      gdouble* A1 = A + (size_t)i * d + j0;
      gdouble* A2 = A + (size_t)(has2 ? i2 : i) * d + j0;
      double a1[QCH], a2[QCH];
#pragma unroll
      for (int m = 0; m < QCH; ++m) {
        const int jc = min(c0 + lane + 64 * m, nj - 1);
        a1[m] = A1[jc];
        a2[m] = A2[jc];
      }
      double p1 = 0.0, p2 = 0.0;
      const double nv1 = PROD ? nv[i] : 0.0, nv2 = (PROD && has2) ? nv[i2] : 0.0;
      if (UPD) {
        const double pi1 = Pg[i], pi2 = has2 ? Pg[i2] : 0.0;
        const double vi1 = cv[i], vi2 = has2 ? cv[i2] : 0.0;
#pragma unroll
        for (int m = 0; m < QCH; ++m) {
          const int j = c0 + lane + 64 * m;
          const bool ok = j < nj;
          const double vj = ok ? cv[j0 + j] : 0.0, qj = ok ? cq[j0 + j] : 0.0;
          a1[m] = hess_upd(a1[m], tk, pi1, vj, vi1, qj);
          a2[m] = hess_upd(a2[m], tk, pi2, vj, vi2, qj);
          if (ok) {
            A1[j] = a1[m];
            if (has2) A2[j] = a2[m];
          }
        }
      }
      if (PROD) {
#pragma unroll
        for (int m = 0; m < QCH; ++m) {
          const int j = c0 + lane + 64 * m;
          const bool ok = j < nj;
          const double w = ok ? nv[j0 + j] : 0.0;
          const double x1 = ok ? a1[m] : 0.0, x2 = ok ? a2[m] : 0.0;
          p1 += x1 * w;
          p2 += x2 * w;
          qacc[m] += nv1 * x1 + nv2 * x2;
        }
        p1 = wave_sum(p1);
        p2 = wave_sum(p2);
        if (lane == 0) {
          pn[i] += p1;
          if (has2) pn[i2] += p2;
        }
      }
    }
    if (PROD) {
#pragma unroll
      for (int m = 0; m < QCH; ++m) {
        const int j = lane + 64 * m;
        if (c0 + j < nj) Qs[(size_t)wv * d + j0 + c0 + j] = qacc[m];
      }
    }
  }
  if (UPD) {
    for (int i = k + 1 + tid; i < d; i += NT) A[(size_t)i * d + k] = (i == k + 1) ? beta_h : 0.0;
  }
}

__device__ void hessenberg(Shared& sh, gdouble* A, gdouble* V, gdouble* tau, gdouble* W, int d) {
  const int tid = threadIdx.x;
  if (d < 3) return;
  gdouble* Qs = W;                            // [16][d] per-wave partials of A^T v
  gdouble* Pg = W + (size_t)NW * d;           // [d] p = A v of the current step
  // arrays: cv = v of step k, cq = q' of step k, nv = v of step k+1,
  // pn = p of step k+1 (accumulated by the pass)
  double* cv = sh.v1;
  double* pn = sh.v2;
  double* cq = sh.v3;
  double* nv = sh.v4;
  // step 0's reflector from column 0, and its products
  for (int i = tid; i < d; i += NT) {
    cv[i] = (i >= 1) ? A[(size_t)i * d] : 0.0;
    pn[i] = 0.0;
  }
  __syncthreads();
  double beta_h = 0.0;
  double tk = hess_reflector(sh, cv, V, tau, 0, d, &beta_h);
  hess_pass<false, true>(sh, A, d, 0, 0.0, 0.0, nullptr, nullptr, nullptr, cv, pn, Qs);
  __syncthreads();
  for (int k = 0; k + 2 < d; ++k) {
    // p of step k to global (the pass reuses pn for step k+1), beta = v^T p
    double bp = 0.0;
    for (int i = tid; i < d; i += NT) {
      const double pi = pn[i];
      Pg[i] = pi;
      if (i > k) bp += cv[i] * pi;
    }
    const double beta = block_sum(sh, bp);
    // q' = q - tau beta v (q summed over the waves in a fixed order)
    for (int j = k + 1 + tid; j < d; j += NT) {
      double q = 0.0;
#pragma unroll
      for (int w = 0; w < NW; ++w) q += Qs[(size_t)w * d + j];
      cq[j] = q - tk * beta * cv[j];
    }
    __syncthreads();
    const bool next = k + 3 < d;
    double tk_next = 0.0, bh_next = 0.0;
    if (next) {
      // column k+1 after step k (v[k+1] = 1), rows k+2..d-1: reflector k+1
      for (int i = tid; i < d; i += NT) {
        nv[i] = (i >= k + 2) ? hess_upd(A[(size_t)i * d + k + 1], tk, Pg[i], 1.0, cv[i], cq[k + 1]) : 0.0;
        pn[i] = 0.0;
      }
      __syncthreads();
      tk_next = hess_reflector(sh, nv, V, tau, k + 1, d, &bh_next);
      hess_pass<true, true>(sh, A, d, k, tk, beta_h, cv, Pg, cq, nv, pn, Qs);
    } else {
      hess_pass<true, false>(sh, A, d, k, tk, beta_h, cv, Pg, cq, nullptr, nullptr, Qs);
    }
    __syncthreads();
    // step k+1's vector becomes the current one
    double* t = cv;
    cv = nv;
    nv = t;
    tk = tk_next;
    beta_h = bh_next;
  }
}

// ------------------------------------------ step 4a: deflation window --
// Aggressive early deflation (Braman, Byers & Mathias, SIAM J. Matrix Anal.
// Appl. 23 (2002) 948) for the eigenvalue-only QR iteration below: the
// trailing nw x nw window W of the active block is brought to real Schur
// form W = Z S Z^T; the coupling column (the "spike", s times the first row
// of Z) shows which of S's trailing eigenvalues are already converged; those
// are deflated, the rest is returned to Hessenberg form and the window's
// unconverged eigenvalues serve as the next sweep's shifts.
//
// The window routines run on one wave with the window in LDS: the wave's LDS
// accesses complete in program order, so they need no barriers.

__device__ __forceinline__ int wave_max_i(int v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v = max(v, __shfl_xor(v, o, 64));
  return v;
}

// Householder reflector P = I - bt v v^T with P (x, y, z)^T = (beta, 0, 0)^T.
// The inputs are scaled by a power of two (exact) instead of by their sum,
// and bt = 2 / |v|^2 = 1 / (al v0) since |v|^2 = 2 al (al + x): one division
// and one square root, which are the latency of a bulge step.  Returns false
// (no reflector) if x = y = z = 0.
__device__ __forceinline__ bool house3(double x, double y, double z, double& v0, double& v1,
                                       double& v2, double& bt, double& beta) {
  const double m = fmax(fabs(x), fmax(fabs(y), fabs(z)));
  if (m == 0.0) return false;
  const int e = ilogb(m);
  const double xs = ldexp(x, -e), ys = ldexp(y, -e), zs = ldexp(z, -e);
  const double al = copysign(sqrt(xs * xs + ys * ys + zs * zs), xs);
  v0 = xs + al;
  v1 = ys;
  v2 = zs;
  bt = 1.0 / (al * v0);
  beta = -ldexp(al, e);
  return true;
}

// Real Schur form of the n x n upper Hessenberg T (n <= AEDMAX) by Francis
// double-shift QR with whole-row and whole-column updates, accumulating the
// transformations into Z (which enters as the identity): T_in = Z T_out Z^T.
// 2 x 2 diagonal blocks are left as they converge (not standardised).
// Returns false if the iteration did not converge.
__device__ bool wave_schur(double (*T)[AEDLD], double (*Z)[AEDLD], int n) {
  const int lane = threadIdx.x & 63;
  double part = 0.0;
  for (int r = lane; r < n; r += 64)
    for (int c = (r > 0 ? r - 1 : 0); c < n; ++c) part += fabs(T[r][c]);
  const double tnorm = wave_sum(part);
  int h = n - 1, its = 0, total = 0;
  while (h >= 0) {
    int cand = 0;
    for (int k = 1 + lane; k <= h; k += 64) {
      double sc = fabs(T[k - 1][k - 1]) + fabs(T[k][k]);
      if (sc == 0.0) sc = tnorm;
      if (fabs(T[k][k - 1]) <= EPS * sc) cand = max(cand, k);
    }
    const int l = wave_max_i(cand);
    if (l >= h - 1) {
      if (l > 0 && lane == 0) T[l][l - 1] = 0.0;
      h = l - 1;
      its = 0;
      continue;
    }
    if (++total > 30 * n) return false;
    ++its;
    double ssum, sprod;
    if (its % 10 == 0) {
      const double ex = fabs(T[h][h - 1]) + fabs(T[h - 1][h - 2]);
      const double x = T[h][h] + 0.75 * ex;
      ssum = 2.0 * x;
      sprod = x * x + 0.4375 * ex * ex;
    } else {
      ssum = T[h - 1][h - 1] + T[h][h];
      sprod = T[h - 1][h - 1] * T[h][h] - T[h - 1][h] * T[h][h - 1];
    }
    for (int K = l - 1; K <= h - 2; ++K) {
      const int nr = (K <= h - 3) ? 3 : 2;
      double x, y, z;
      if (K == l - 1) {
        const double h00 = T[l][l], h01 = T[l][l + 1], h10 = T[l + 1][l];
        const double h11 = T[l + 1][l + 1], h21 = T[l + 2][l + 1];
        x = h00 * h00 + h01 * h10 - ssum * h00 + sprod;
        y = h10 * (h00 + h11 - ssum);
        z = h10 * h21;
      } else {
        x = T[K + 1][K];
        y = T[K + 2][K];
        z = (nr == 3) ? T[K + 3][K] : 0.0;
      }
      if (nr == 2) z = 0.0;
      double v0, v1, v2, bt, beta;
      if (!house3(x, y, z, v0, v1, v2, bt, beta)) continue;
      // Z <- Z P does not depend on T: for n <= 32 the upper half-wave updates
      // Z's columns in the same instructions in which the lower half updates
      // T's rows (three elements at a stride: a row of T across, a column of
      // Z down)
      const bool zsplit = n <= 32;
      if (zsplit) {
        const bool zl = lane >= 32;
        const int c = zl ? lane - 32 : K + 1 + lane;
        if (c < n) {
          double* p0 = zl ? &Z[c][K + 1] : &T[K + 1][c];
          const int st = zl ? 1 : AEDLD;
          double tt = v0 * p0[0] + v1 * p0[st];
          if (nr == 3) tt += v2 * p0[2 * st];
          tt *= bt;
          p0[0] -= tt * v0;
          p0[st] -= tt * v1;
          if (nr == 3) p0[2 * st] -= tt * v2;
        }
      } else {
        for (int c = K + 1 + lane; c < n; c += 64) {
          double tt = v0 * T[K + 1][c] + v1 * T[K + 2][c];
          if (nr == 3) tt += v2 * T[K + 3][c];
          tt *= bt;
          T[K + 1][c] -= tt * v0;
          T[K + 2][c] -= tt * v1;
          if (nr == 3) T[K + 3][c] -= tt * v2;
        }
      }
      if (K >= l && lane == 0) {
        T[K + 1][K] = beta;
        T[K + 2][K] = 0.0;
        if (nr == 3) T[K + 3][K] = 0.0;
      }
      const int r1 = min(K + 4, h);
      for (int r = lane; r <= r1; r += 64) {
        double tt = T[r][K + 1] * v0 + T[r][K + 2] * v1;
        if (nr == 3) tt += T[r][K + 3] * v2;
        tt *= bt;
        T[r][K + 1] -= tt * v0;
        T[r][K + 2] -= tt * v1;
        if (nr == 3) T[r][K + 3] -= tt * v2;
      }
      for (int r = lane; r < n && !zsplit; r += 64) {
        double tt = Z[r][K + 1] * v0 + Z[r][K + 2] * v1;
        if (nr == 3) tt += Z[r][K + 3] * v2;
        tt *= bt;
        Z[r][K + 1] -= tt * v0;
        Z[r][K + 2] -= tt * v1;
        if (nr == 3) Z[r][K + 3] -= tt * v2;
      }
    }
  }
  return true;
}

// Deflation test of the window's Schur form (T, Z) against the spike s Z[0][:],
// from the bottom up: blocks whose spike entries are below ulp times the
// block's size are converged and deflate, up to the first one that is not.
// (Moving unconverged blocks up to test the ones above, as LAPACK does, found
// hardly any more on these pencils, whose spectra are mostly complex pairs,
// and cost more than it saved.)  Returns the number of deflated eigenvalues.
__device__ int wave_aed_deflate(double (*T)[AEDLD], double (*Z)[AEDLD], int n, double spike) {
  int ns = n;
  while (ns > 0) {
    const int k = ns - 1;
    const bool two = (k > 0) && T[k][k - 1] != 0.0;
    double foo = fabs(T[k][k]);
    if (two) foo += sqrt(fabs(T[k][k - 1])) * sqrt(fabs(T[k - 1][k]));
    if (foo == 0.0) foo = fabs(spike);
    double f = fabs(spike * Z[0][k]);
    if (two) f = fmax(f, fabs(spike * Z[0][k - 1]));
    if (!(f <= fmax(DBL_MIN, EPS * foo))) break;
    ns -= two ? 2 : 1;
  }
  return n - ns;
}

// Eigenvalues of the diagonal blocks of a quasi-triangular S (n x n): a
// 2 x 2 block sits where S[k][k-1] != 0.
__device__ void wave_block_eigs(double (*S)[AEDLD], int n, double* er, double* ei) {
  const int lane = threadIdx.x & 63;
  for (int k = lane; k < n; k += 64) {
    const bool top = (k + 1 < n) && S[k + 1][k] != 0.0;
    const bool bot = (k > 0) && S[k][k - 1] != 0.0;
    if (!top && !bot) {
      er[k] = S[k][k];
      ei[k] = 0.0;
      continue;
    }
    const int i = top ? k : k - 1;
    const double a = S[i][i], b = S[i][i + 1], c = S[i + 1][i], dd = S[i + 1][i + 1];
    const double p = 0.5 * (a - dd);
    const double disc = p * p + b * c;
    if (disc >= 0.0) {
      const double zz = p + copysign(sqrt(disc), p);
      const double e0 = dd + zz, e1 = (zz != 0.0) ? dd - b * c / zz : dd + zz;
      er[k] = top ? e0 : e1;
      ei[k] = 0.0;
    } else {
      er[k] = dd + p;
      ei[k] = top ? sqrt(-disc) : -sqrt(-disc);
    }
  }
}

// Returns the leading nu x nu block of T, whose first column carries the
// spike u (length nu) on the left, to Hessenberg form by Householder
// reflections H_k (k = -1 reflects the spike onto e_0): T <- H T H on the
// window (rows k+1..nu-1 from the left over all columns, columns k+1..nu-1
// from the right), Z <- Z H.  Returns the spike's remaining first entry.
__device__ double wave_rehess(double (*T)[AEDLD], double (*Z)[AEDLD], double* u, double* v, int nu,
                              int nw) {
  const int lane = threadIdx.x & 63;
  double spike0 = u[0];
  for (int k = -1; k <= nu - 3; ++k) {
    const int r0 = k + 1, len = nu - r0;
    // x = column k below the diagonal (the spike for k = -1)
    const double xi = (lane < len) ? (k < 0 ? u[r0 + lane] : T[r0 + lane][k]) : 0.0;
    const double alpha = __shfl(xi, 0, 64);
    const double xn2 = wave_sum(lane > 0 ? xi * xi : 0.0);
    if (xn2 == 0.0) continue;
    const double beta = -copysign(sqrt(alpha * alpha + xn2), alpha);
    const double tau = (beta - alpha) / beta;
    const double scal = 1.0 / (alpha - beta);
    if (lane < len) v[lane] = (lane == 0) ? 1.0 : xi * scal;
    // the reflected column becomes beta e_0
    if (k < 0) {
      if (lane < len) u[lane] = (lane == 0) ? beta : 0.0;
      spike0 = beta;
    } else if (lane < len) {
      T[r0 + lane][k] = (lane == 0) ? beta : 0.0;
    }
    // left: rows r0..nu-1, columns k+1..nw-1
    for (int c = k + 1 + lane; c < nw; c += 64) {
      double wsum = 0.0;
      for (int i = 0; i < len; ++i) wsum += v[i] * T[r0 + i][c];
      wsum *= tau;
      for (int i = 0; i < len; ++i) T[r0 + i][c] -= wsum * v[i];
    }
    // right: columns r0..nu-1, rows 0..nu-1 (rows below nu are zero there)
    for (int r = lane; r < nu; r += 64) {
      double wsum = 0.0;
      for (int i = 0; i < len; ++i) wsum += T[r][r0 + i] * v[i];
      wsum *= tau;
      for (int i = 0; i < len; ++i) T[r][r0 + i] -= wsum * v[i];
    }
    for (int r = lane; r < nw; r += 64) {
      double wsum = 0.0;
      for (int i = 0; i < len; ++i) wsum += Z[r][r0 + i] * v[i];
      wsum *= tau;
      for (int i = 0; i < len; ++i) Z[r][r0 + i] -= wsum * v[i];
    }
  }
  return spike0;
}

// ---------------------------------------------------------------- step 4 --
// Eigenvalues of the upper Hessenberg matrix A (row stride ld, destroyed)
// into wr, wi.  A conjugate pair is stored as (re, +im), (re, -im) at
// consecutive indices.
//
// Each sweep chases m double-shift bulges down the active window [l, h]
// (small-bulge multishift QR).  With MULTI, m pairs of shifts are the
// eigenvalues of the trailing 2m x 2m block of the window (found by this
// routine with MULTI off on an LDS copy); bulge b enters four rows after
// bulge b-1, so the bulges touch disjoint rows and columns in every tick.
// Left (row) and right (column) reflections commute, so all row updates
// of a tick run first, then all column updates.  Without MULTI (or after
// 10 sweeps without deflation) one bulge uses the trailing 2x2 block's
// eigenvalues, or an ad hoc pair.  Deflation: a subdiagonal entry below
// eps (|a_{i-1,i-1}| + |a_ii|) is set to zero.
// ------------------------------------------- step 4b: windowed bulge chase --
// One multishift sweep (m bulges, shifts in sh.bsum / sh.bprod) over the
// active block l..h, in batches of CT ticks.  At tick t bulge g sits at
// K = l - 1 + t - 4 g (active while l - 1 <= K <= h - 2) and applies its
// 3 x 3 reflector P = I - bt v v^T (2 x 2 at the bottom) to rows and to
// columns K+1..K+3.  Per batch:
//   1. the diagonal window that holds every element those reflectors reach
//      near the diagonal is copied to LDS; the ticks run there (reflector
//      from the window, its rows and columns updated inside the window) and
//      each reflector is recorded;
//   2. the window is written back, and the recorded reflectors are applied
//      outside it: from the left to the columns right of the window, from
//      the right to the rows above it.
// Every element receives the same reflectors in the same order as in a
// tick-by-tick sweep: where a leading and a trailing bulge touch the same
// rows (or columns), the leading bulge's reflector always comes first, so
// the far parts can take one bulge's reflectors after another.  They are
// read and written once per batch instead of once per tick.

// Bulge g's recorded reflectors (ticks 0..CT-1) applied to a segment of
// CT + 2 consecutive rows (or columns) that starts at the bulge's first one.
__device__ __forceinline__ void chase_apply(const Shared& sh, int g, double (&x)[CT + 2]) {
#pragma unroll
  for (int tau = 0; tau < CT; ++tau) {
    const ChaseRec R = sh.rec[tau][g];
    const double tt = R.bt * (R.v0 * x[tau] + R.v1 * x[tau + 1] + R.v2 * x[tau + 2]);
    x[tau] -= tt * R.v0;
    x[tau + 1] -= tt * R.v1;
    x[tau + 2] -= tt * R.v2;
  }
}

// The recorded reflectors of a batch (first tick t0) applied to one item
// outside the window: a column right of it (right = true: rows change) or
// a row above it (columns change).  Bulge g's segment starts at position
// l + t0 - 4 g; consecutive bulges' segments overlap, so the segment rolls
// through registers: 4 new entries loaded, 4 finished ones stored per bulge.
// Only positions inside the window [wlo, whi] can change; loads are clamped
// there and stores limited to it.  A is the matrix for a column right of the
// window (rows are positions) and its transposed copy for a row above it
// (columns are positions); either way position q of the item is A[q][item],
// and neighbouring lanes (neighbouring items) touch neighbouring addresses.
template <class Real>
__device__ void chase_far(const Shared& sh, Real* A, int ld, int wlo, int whi, int t0, int l, int m,
                          bool right, int item) {
  auto ptr = [&](int pos) -> Real* {
    const int q = min(max(pos, wlo), whi);
    return A + (size_t)q * ld + item;
  };
  double x[CT + 2];
  int B = l + t0;
#pragma unroll
  for (int i = 0; i < CT + 2; ++i) x[i] = *ptr(B + i);
  for (int g = 0; g < m; ++g) {
    chase_apply(sh, g, x);
    const int nfin = (g + 1 < m) ? 4 : CT + 2;     // entries final after this bulge
#pragma unroll
    for (int i = 0; i < CT + 2; ++i) {
      const int pos = B + i;
      if (i >= CT + 2 - nfin && pos >= wlo && pos <= whi) *ptr(pos) = x[i];
    }
    if (g + 1 < m) {
#pragma unroll
      for (int i = CT + 1; i >= 4; --i) x[i] = x[i - 4];
      B -= 4;
#pragma unroll
      for (int i = 0; i < 4; ++i) x[i] = *ptr(B + i);
    }
  }
}

// The rows above the window live in a transposed copy during a sweep, so
// that their far updates (one row per lane) read and write consecutive
// addresses across a wave.  Entry (r, c) moves to T[c][r] when column c is
// in a batch's window and row r above it: a column holds rows l .. tl - 1 in
// T, tl being the window's top row of the last batch that held the column
// (recorded in tlf[c]).  Nothing else reads those entries during the sweep
// (windows and right items take rows at or below the window's top), and at
// its end they go back to A.
template <class Real>
__device__ void chase_windowed(Shared& sh, Real* A, int ld, int l, int h, int m, Real* T,
                               BLM_GLOBAL int32_t* tlf) {
  const int tid = threadIdx.x;
  // group grp of G threads carries bulge grp
  const int mp = m <= 1 ? 1 : m <= 2 ? 2 : m <= 4 ? 4 : m <= 8 ? 8 : 16;
  const int G = NT / mp, grp = tid / G, lt = tid % G;
  const int ticks = (h - l) + 4 * (m - 1);
  int wlo_prev = l, whi_prev = l - 1;
  for (int t0 = 0; t0 < ticks; t0 += CT) {
    const int t1 = min(t0 + CT, ticks);
    // the batch's reflectors sit at K in [Kmin, Kmax]; they reach rows and
    // columns up to K + 4 near the diagonal
    const int Kmax = min(l - 1 + t1 - 1, h - 2);
    const int Kmin = min(max(l - 1, l - 1 + t0 - 4 * (m - 1)), h - 2);
    const int wlo = max(l, Kmin), whi = min(h, Kmax + 4);
    const int nw = whi - wlo + 1;                   // <= CT + 4 m <= CWMAX
    for (int e = tid; e < nw * nw; e += NT) {
      const int i = e / nw, j = e % nw;
      sh.cw[i][j] = A[(size_t)(wlo + i) * ld + wlo + j];
    }
    for (int e = tid; e < CT * MAX_BULGES; e += NT)
      sh.rec[e / MAX_BULGES][e % MAX_BULGES] = ChaseRec{0.0, 0.0, 0.0, 0.0};
    __syncthreads();
    auto W = [&](int i, int j) -> double& { return sh.cw[i - wlo][j - wlo]; };
    for (int t = t0; t < t1; ++t) {
      const int K = l - 1 + t - 4 * grp;
      const bool act = grp < m && K >= l - 1 && K <= h - 2;
      const int nr = (K <= h - 3) ? 3 : 2;
      double v0 = 0.0, v1 = 0.0, v2 = 0.0, bt = 0.0, newsub = 0.0;
      bool refl = false;
      if (act) {
        double x, y, z;
        if (K == l - 1) {
          const double ssum = sh.bsum[grp], sprod = sh.bprod[grp];
          const double h00 = W(l, l), h01 = W(l, l + 1), h10 = W(l + 1, l);
          const double h11 = W(l + 1, l + 1), h21 = W(l + 2, l + 1);
          x = h00 * h00 + h01 * h10 - ssum * h00 + sprod;
          y = h10 * (h00 + h11 - ssum);
          z = h10 * h21;
        } else {
          x = sh.bx[grp][0];
          y = sh.bx[grp][1];
          z = sh.bx[grp][2];
        }
        if (nr == 2) z = 0.0;
        refl = house3(x, y, z, v0, v1, v2, bt, newsub);
        if (refl && lt == 0) sh.rec[t - t0][grp] = ChaseRec{v0, v1, v2, bt};
      }
      // a bulge entering at the top read the window's first rows, which its
      // own group rewrites below: let every wave finish reading first
      if ((t & 3) == 0 && (t >> 2) < m) __syncthreads();
      if (act && refl) {
        // rows K+1..K+nr, window columns max(l, K+1)..whi; the bulge column
        // K is set directly
        const int c0 = (K >= l) ? K + 1 : l;
        for (int c = c0 + lt; c <= whi; c += G) {
          const double x0 = W(K + 1, c), x1 = W(K + 2, c), x2 = (nr == 3) ? W(K + 3, c) : 0.0;
          const double tt = bt * (v0 * x0 + v1 * x1 + v2 * x2);
          W(K + 1, c) = x0 - tt * v0;
          W(K + 2, c) = x1 - tt * v1;
          if (nr == 3) W(K + 3, c) = x2 - tt * v2;
        }
        if (K >= l && lt == 0) {
          W(K + 1, K) = newsub;
          W(K + 2, K) = 0.0;
          if (nr == 3) W(K + 3, K) = 0.0;
        }
      }
      __syncthreads();
      if (act) {
        // columns K+1..K+nr, window rows wlo..min(K+4, h); keep column K+1's
        // entries below the diagonal (the next bulge) for the next tick
        const int r1 = (K + 4 < h) ? K + 4 : h;
        for (int rr = wlo + lt; rr <= r1; rr += G) {
          const double y0 = W(rr, K + 1), y1 = W(rr, K + 2), y2 = (nr == 3) ? W(rr, K + 3) : 0.0;
          double n0 = y0;
          if (refl) {
            const double tt = bt * (y0 * v0 + y1 * v1 + y2 * v2);
            n0 = y0 - tt * v0;
            W(rr, K + 1) = n0;
            W(rr, K + 2) = y1 - tt * v1;
            if (nr == 3) W(rr, K + 3) = y2 - tt * v2;
          }
          if (rr >= K + 2) sh.bx[grp][rr - K - 2] = n0;
        }
        if (K + 4 > h && lt == 0) sh.bx[grp][2] = 0.0;
        if (K + 3 > h && lt == 0) sh.bx[grp][1] = 0.0;
      }
      __syncthreads();
    }
    // the window back; the batch's reflectors to the columns right of it
    // (from the left) and to the rows above it (from the right)
    for (int e = tid; e < nw * nw; e += NT) {
      const int i = e / nw, j = e % nw;
      A[(size_t)(wlo + i) * ld + wlo + j] = sh.cw[i][j];
    }
    // into T: rows wlo_prev .. wlo - 1 of the columns the last window also
    // held, rows l .. wlo - 1 of the entering ones (one row per thread)
    const int cold = min(whi, whi_prev);
    const int nold = max(0, cold - wlo + 1), nnew = whi - max(wlo, whi_prev + 1) + 1;
    const int cnew = max(wlo, whi_prev + 1);
    for (int e = tid; e < nold * (wlo - wlo_prev); e += NT) {
      const int c = wlo + e / (wlo - wlo_prev), r = wlo_prev + e % (wlo - wlo_prev);
      T[(size_t)c * ld + r] = A[(size_t)r * ld + c];
    }
    for (int r = l + tid; r < wlo; r += NT)
      for (int c = cnew; c < cnew + nnew; ++c) T[(size_t)c * ld + r] = A[(size_t)r * ld + c];
    for (int c = wlo + tid; c <= whi; c += NT) tlf[c] = wlo;
    wlo_prev = wlo;
    whi_prev = whi;
    __syncthreads();
    const int nright = h - whi, ntop = wlo - l;
    for (int it = tid; it < nright + ntop; it += NT) {
      if (it < nright)
        chase_far(sh, A, ld, wlo, whi, t0, l, m, true, whi + 1 + it);
      else
        chase_far(sh, T, ld, wlo, whi, t0, l, m, false, l + (it - nright));
    }
    __syncthreads();
  }
  // T back to A, through LDS in 64 x 64 tiles (reads of T and writes of A
  // both along consecutive addresses); tlf is nondecreasing in the column
  double (*tb)[65] = reinterpret_cast<double (*)[65]>(&sh.cw[0][0]);
  static_assert(64 * 65 <= CWMAX * CWLD, "transpose tile");
  for (int c0 = l; c0 <= h; c0 += 64) {
    const int c1 = min(c0 + 63, h);
    const int rmax = tlf[c1];                       // rows l .. rmax - 1 hold T entries in this column group
    for (int r0 = l; r0 < rmax; r0 += 64) {
      for (int e = tid; e < 64 * 64; e += NT) {
        const int i = e >> 6, j = e & 63;           // column c0 + i, row r0 + j
        const int c = c0 + i, r = r0 + j;
        if (c <= c1 && r < rmax) tb[i][j] = T[(size_t)c * ld + r];
      }
      __syncthreads();
      for (int e = tid; e < 64 * 64; e += NT) {
        const int j = e >> 6, i = e & 63;           // row r0 + j, column c0 + i
        const int c = c0 + i, r = r0 + j;
        if (c <= c1 && r < tlf[c]) A[(size_t)r * ld + c] = tb[i][j];
      }
      __syncthreads();
    }
  }
}

constexpr int AED_MIN_W = 75;   // active blocks at least this wide use early deflation
constexpr int AED_NIBBLE = 14;  // percent of the window deflated to skip a sweep
constexpr int CU = 4;           // chase: elements per thread whose loads go out together

template <bool MULTI, class Real>
__device__ int hqr(Shared& sh, Real* A, int ld, int d, Real* wr, Real* wi, int* iters, Real* Tw = nullptr) {
  const int tid = threadIdx.x;
  if (MULTI && tid == 0)
    for (int i = 0; i < 4; ++i) sh.qst[i] = 0;
  auto at = [&](int i, int j) -> double& { return A[(size_t)i * ld + j]; };
  double part = 0.0;
  for (int i = tid; i < d; i += NT)
    for (int j = (i > 0 ? i - 1 : 0); j < d; ++j) part += fabs(at(i, j));
  const double anorm = block_sum(sh, part);
  int h = d - 1, its = 0, total = 0;
  const int max_total = 40 * (d + 1);
  while (h >= 0) {
    if (tid == 0) sh.isc[1] = 0;
    __syncthreads();
    for (int i = 1 + tid; i <= h; i += NT) {
      double s = fabs(at(i - 1, i - 1)) + fabs(at(i, i));
      if (s == 0.0) s = anorm;
      if (fabs(at(i, i - 1)) <= EPS * s) atomicMax(&sh.isc[1], i);
    }
    __syncthreads();
    const int l = sh.isc[1];
    if (l == h) {
      if (tid == 0) {
        if (l > 0) at(l, l - 1) = 0.0;
        wr[h] = at(h, h);
        wi[h] = 0.0;
      }
      h -= 1;
      its = 0;
      __syncthreads();
      continue;
    }
    if (l == h - 1) {
      if (tid == 0) {
        if (l > 0) at(l, l - 1) = 0.0;
        const double a = at(h - 1, h - 1), b = at(h - 1, h);
        const double c = at(h, h - 1), dd = at(h, h);
        const double p = 0.5 * (a - dd);
        const double disc = p * p + b * c;
        if (disc >= 0.0) {
          const double z = p + copysign(sqrt(disc), p);
          wr[h - 1] = dd + z;
          wr[h] = (z != 0.0) ? dd - b * c / z : dd + z;
          wi[h - 1] = 0.0;
          wi[h] = 0.0;
        } else {
          wr[h - 1] = wr[h] = dd + p;
          const double im = sqrt(-disc);
          wi[h - 1] = im;
          wi[h] = -im;
        }
      }
      h -= 2;
      its = 0;
      __syncthreads();
      continue;
    }
    if (total >= max_total) {
      *iters = total;
      return EIG_NOCONV;
    }
    ++its;
    ++total;
    const int w = h - l + 1;
    int m = 1;
    bool shifts_set = false;
    const uint64_t t_aed = wall_clock64();
    if (MULTI && w >= AED_MIN_W && its % 10 != 0) {
      if (tid == 0) sh.qst[2] += 1;
      // aggressive early deflation on the trailing window
      const int ns = w < 150 ? 10 : w < 300 ? 16 : 24;
      const int nw = min(AEDMAX, ns);
      const int kwtop = h - nw + 1;
      const double spike = at(kwtop, kwtop - 1);
      for (int t = tid; t < nw * nw; t += NT) {
        const int i = t / nw, j = t % nw;
        sh.aT[i][j] = (j + 1 >= i) ? at(kwtop + i, kwtop + j) : 0.0;
        sh.aZ[i][j] = (i == j) ? 1.0 : 0.0;
      }
      __syncthreads();
      if (tid < 64) {
        const bool ok = wave_schur(sh.aT, sh.aZ, nw);
        const int nd = ok ? wave_aed_deflate(sh.aT, sh.aZ, nw, spike) : 0;
        wave_block_eigs(sh.aT, nw, sh.ewr, sh.ewi);
        const int nu = nw - nd;
        double beta = 0.0;
        if (ok && nd > 0 && nu > 0) {
          for (int i = tid; i < nu; i += 64) sh.au[i] = spike * sh.aZ[0][i];
          beta = wave_rehess(sh.aT, sh.aZ, sh.au, sh.av, nu, nw);
        }
        if (tid == 0) {
          sh.isc[6] = ok ? 1 : 0;
          sh.isc[7] = nd;
          sh.sc[8] = beta;
        }
      }
      __syncthreads();
      if (sh.isc[6]) {
        const int nd = sh.isc[7], nu = nw - nd;
        if (nd > 0) {
          for (int i = nu + tid; i < nw; i += NT) {
            wr[kwtop + i] = sh.ewr[i];
            wi[kwtop + i] = sh.ewi[i];
          }
          // rows of the active block above the window: A <- A Z
          const int lane = tid & 63, wv = tid >> 6;
          for (int r = l + wv; r < kwtop; r += NW) {
            if (lane < nw) sh.stage[wv][lane] = at(r, kwtop + lane);
            if (lane < nw) {
              double acc = 0.0;
              for (int i = 0; i < nw; ++i) acc += sh.stage[wv][i] * sh.aZ[i][lane];
              at(r, kwtop + lane) = acc;
            }
          }
          for (int t = tid; t < nw * nw; t += NT) {
            const int i = t / nw, j = t % nw;
            if (j + 1 >= i) at(kwtop + i, kwtop + j) = sh.aT[i][j];
          }
          if (tid == 0) at(kwtop, kwtop - 1) = (nu > 0) ? sh.sc[8] : 0.0;
          __syncthreads();
          h = kwtop + nu - 1;
          its = 0;
        }
        // skip the sweep when the window deflated enough
        if (nd > 0 && 100 * nd > AED_NIBBLE * nw) {
          if (MULTI && tid == 0) sh.qst[0] += wall_clock64() - t_aed;
          continue;
        }
        if (h - l + 1 < 3) {
          if (MULTI && tid == 0) sh.qst[0] += wall_clock64() - t_aed;
          continue;
        }
        if (tid == 0) {
          // shifts: the window's bottom-most unconverged eigenvalues
          int mm = 0, i = nu - 1;
          double rpend = 0.0;
          bool have_r = false;
          while (i >= 0 && mm < MAX_BULGES && mm * 2 < ns) {
            if (sh.ewi[i] != 0.0 && i > 0) {
              const double re = sh.ewr[i], im = sh.ewi[i];
              sh.bsum[mm] = 2.0 * re;
              sh.bprod[mm] = re * re + im * im;
              ++mm;
              i -= 2;
            } else {
              if (have_r) {
                sh.bsum[mm] = rpend + sh.ewr[i];
                sh.bprod[mm] = rpend * sh.ewr[i];
                ++mm;
                have_r = false;
              } else {
                rpend = sh.ewr[i];
                have_r = true;
              }
              i -= 1;
            }
          }
          sh.isc[5] = mm;
        }
        __syncthreads();
        m = sh.isc[5];
        shifts_set = m > 0;
      }
    }
    if (MULTI && !shifts_set && its % 10 != 0) {
      const int ns = w < 30 ? 2 : w < 60 ? 4 : w < 150 ? 10 : w < 590 ? 16 : 2 * MAX_BULGES;
      if (ns > 2) {
        const int o = h - ns + 1;
        for (int t = tid; t < ns * ns; t += NT) {
          const int i = t / ns, j = t % ns;
          sh.T[t] = (j + 1 >= i) ? at(o + i, o + j) : 0.0;
        }
        __syncthreads();
        int it2 = 0;
        const int st2 = hqr<false>(sh, sh.T, ns, ns, sh.swr, sh.swi, &it2);
        __syncthreads();
        if (st2 == EIG_OK) {
          if (tid == 0) {
            int mm = 0, nre = 0;
            double* re = sh.sre;
            for (int i = 0; i < ns; ++i) {
              if (!isfinite(sh.swr[i]) || !isfinite(sh.swi[i])) continue;
              if (sh.swi[i] > 0.0 && mm < MAX_BULGES) {
                sh.bsum[mm] = 2.0 * sh.swr[i];
                sh.bprod[mm] = sh.swr[i] * sh.swr[i] + sh.swi[i] * sh.swi[i];
                ++mm;
              } else if (sh.swi[i] == 0.0) {
                re[nre++] = sh.swr[i];
              }
            }
            for (int i = 0; i + 1 < nre && mm < MAX_BULGES; i += 2) {
              sh.bsum[mm] = re[i] + re[i + 1];
              sh.bprod[mm] = re[i] * re[i + 1];
              ++mm;
            }
            sh.isc[5] = mm;
          }
          __syncthreads();
          m = sh.isc[5];
        }
      }
    }
    if (m < 1) m = 1;
    if (m == 1 && tid == 0) {
      // one bulge: trailing 2x2 block's eigenvalues, or an ad hoc pair
      const double a = at(h - 1, h - 1), b = at(h - 1, h);
      const double c = at(h, h - 1), dd = at(h, h);
      if (its % 10 == 0) {
        const double ex = fabs(c) + fabs(at(h - 1, h - 2));
        const double x = dd + 0.75 * ex;
        sh.bsum[0] = 2.0 * x;
        sh.bprod[0] = x * x + 0.4375 * ex * ex;
      } else {
        sh.bsum[0] = a + dd;
        sh.bprod[0] = a * dd - b * c;
      }
    }
    __syncthreads();

    const uint64_t t_chase = wall_clock64();
    if (MULTI && tid == 0) {
      sh.qst[0] += t_chase - t_aed;
      sh.qst[3] += 1;
    }
    if constexpr (MULTI) {
      chase_windowed(sh, A, ld, l, h, m, Tw, reinterpret_cast<BLM_GLOBAL int32_t*>(Tw + (size_t)ld * d));
      if (tid == 0) sh.qst[1] += wall_clock64() - t_chase;
      continue;
    }
    // chase: group g of G threads carries bulge g
    const int mp = m <= 1 ? 1 : m <= 2 ? 2 : m <= 4 ? 4 : m <= 8 ? 8 : 16;
    const int G = NT / mp, grp = tid / G, lt = tid % G;
    const int ticks = (h - l) + 4 * (m - 1);
    for (int t = 0; t < ticks; ++t) {
      const int K = l - 1 + t - 4 * grp;
      const bool act = grp < m && K >= l - 1 && K <= h - 2;
      const int nr = (K <= h - 3) ? 3 : 2;
      double v0 = 0.0, v1 = 0.0, v2 = 0.0, bt = 0.0, newsub = 0.0;
      bool refl = false;
      if (act) {
        double x, y, z;
        if (K == l - 1) {
          const double ssum = sh.bsum[grp], sprod = sh.bprod[grp];
          const double h00 = at(l, l), h01 = at(l, l + 1), h10 = at(l + 1, l);
          const double h11 = at(l + 1, l + 1), h21 = at(l + 2, l + 1);
          x = h00 * h00 + h01 * h10 - ssum * h00 + sprod;
          y = h10 * (h00 + h11 - ssum);
          z = h10 * h21;
        } else {
          x = sh.bx[grp][0];
          y = sh.bx[grp][1];
          z = sh.bx[grp][2];
        }
        if (nr == 2) z = 0.0;
        refl = house3(x, y, z, v0, v1, v2, bt, newsub);
      }
      // a bulge entering at the top read the window's first rows, which its
      // own group rewrites below: let every wave finish reading first
      if ((t & 3) == 0 && (t >> 2) < m) __syncthreads();
      if (act && refl) {
        // rows K+1..K+nr, columns max(l, K+1)..h; the bulge column K is set
        // directly.  CU columns per thread per pass: their loads are issued
        // together (indices clamped into the row), the stores guarded.
        const int c0 = (K >= l) ? K + 1 : l;
        Real* r1p = A + (size_t)(K + 1) * ld;
        Real* r2p = r1p + ld;
        Real* r3p = r2p + ld;
        for (int cb = c0 + lt; cb <= h; cb += G * CU) {
          double x0[CU], x1[CU], x2[CU];
#pragma unroll
          for (int u = 0; u < CU; ++u) {
            const int c = min(cb + G * u, h);
            x0[u] = r1p[c];
            x1[u] = r2p[c];
            x2[u] = (nr == 3) ? r3p[c] : 0.0;
          }
#pragma unroll
          for (int u = 0; u < CU; ++u) {
            const int c = cb + G * u;
            if (c <= h) {
              const double tt = bt * (v0 * x0[u] + v1 * x1[u] + v2 * x2[u]);
              r1p[c] = x0[u] - tt * v0;
              r2p[c] = x1[u] - tt * v1;
              if (nr == 3) r3p[c] = x2[u] - tt * v2;
            }
          }
        }
        if (K >= l && lt == 0) {
          at(K + 1, K) = newsub;
          at(K + 2, K) = 0.0;
          if (nr == 3) at(K + 3, K) = 0.0;
        }
      }
      __syncthreads();
      if (act) {
        // columns K+1..K+nr, rows l..min(K+4, h); keep column K+1's entries
        // below the diagonal (the next bulge) for the next tick
        const int r1 = (K + 4 < h) ? K + 4 : h;
        for (int rb = l + lt; rb <= r1; rb += G * CU) {
          double y0[CU], y1[CU], y2[CU];
#pragma unroll
          for (int u = 0; u < CU; ++u) {
            const Real* q = A + (size_t)min(rb + G * u, r1) * ld + K + 1;
            y0[u] = q[0];
            y1[u] = q[1];
            y2[u] = (nr == 3) ? q[2] : 0.0;
          }
#pragma unroll
          for (int u = 0; u < CU; ++u) {
            const int rr = rb + G * u;
            if (rr > r1) continue;
            Real* q = A + (size_t)rr * ld + K + 1;
            double n0 = y0[u];
            if (refl) {
              const double tt = bt * (y0[u] * v0 + y1[u] * v1 + y2[u] * v2);
              n0 = y0[u] - tt * v0;
              q[0] = n0;
              q[1] = y1[u] - tt * v1;
              if (nr == 3) q[2] = y2[u] - tt * v2;
            }
            if (rr >= K + 2) sh.bx[grp][rr - K - 2] = n0;
          }
        }
        if (K + 4 > h && lt == 0) sh.bx[grp][2] = 0.0;
        if (K + 3 > h && lt == 0) sh.bx[grp][1] = 0.0;
      }
      __syncthreads();
    }
    if (MULTI && tid == 0) sh.qst[1] += wall_clock64() - t_chase;
  }
  *iters = total;
  for (int i = tid; i < d; i += NT)
    if (!isfinite(wr[i]) || !isfinite(wi[i])) sh.isc[2] = 1;
  return EIG_OK;
}

// ---------------------------------------------------------------- step 5 --
// Picks eigenvalues in rank order until `want` directions are held (a pair
// gives two).  Returns the number of picked eigenvalue entries in sh.sel_*
// (a pair is one entry with positive imaginary part).
__device__ int select_lowest(Shared& sh, const gdouble* wr, const gdouble* wi, int d, int want,
                             gdouble* out_evals, int max_entries) {
  const int tid = threadIdx.x;
  for (int i = tid; i < d; i += NT) sh.mark[i] = 0;
  if (tid == 0) sh.sel_n = 0;
  __syncthreads();
  // eigenvalues are ranked until max_entries are listed; those taken while
  // fewer than `want` directions are held are the selected ones
  int held = 0, n_sel = 0, n_ev = 0;
  while (n_ev < max_entries && (held >= want || n_sel < EIG_MAXSEL)) {
    const bool take = held < want;
    // argmin over unmarked of (wr asc, wi desc, index asc)
    double br = INFINITY, bi = -INFINITY;
    int bidx = d;
    for (int i = tid; i < d; i += NT) {
      if (sh.mark[i]) continue;
      const double r = wr[i], im = wi[i];
      if (r < br || (r == br && (im > bi || (im == bi && i < bidx)))) {
        br = r;
        bi = im;
        bidx = i;
      }
    }
    // wave then block reduction of (br, bi, bidx)
    for (int off = 32; off > 0; off >>= 1) {
      const double orr = __shfl_xor(br, off, 64), oi = __shfl_xor(bi, off, 64);
      const int ox = __shfl_xor(bidx, off, 64);
      if (orr < br || (orr == br && (oi > bi || (oi == bi && ox < bidx)))) {
        br = orr;
        bi = oi;
        bidx = ox;
      }
    }
    if ((tid & 63) == 0) {
      sh.v1[tid >> 6] = br;
      sh.v2[tid >> 6] = bi;
      sh.widx[tid >> 6] = bidx;
    }
    __syncthreads();
    if (tid == 0) {
      double r = sh.v1[0], im = sh.v2[0];
      int ix = sh.widx[0];
      for (int w = 1; w < NW; ++w) {
        const double orr = sh.v1[w], oi = sh.v2[w];
        const int ox = sh.widx[w];
        if (orr < r || (orr == r && (oi > im || (oi == im && ox < ix)))) {
          r = orr;
          im = oi;
          ix = ox;
        }
      }
      sh.isc[3] = ix;
    }
    __syncthreads();
    const int ix = sh.isc[3];
    if (ix >= d) break;
    const double r = wr[ix], im = wi[ix];
    if (tid == 0) {
      sh.mark[ix] = 1;
      if (take) {
        sh.sel_r[n_sel] = r;
        sh.sel_i[n_sel] = im;
      }
      out_evals[2 * n_ev] = r;
      out_evals[2 * n_ev + 1] = im;
      if (im != 0.0) {
        // partner: the conjugate, stored right after it
        for (int j = 0; j < d; ++j)
          if (!sh.mark[j] && wr[j] == r && wi[j] == -im) {
            sh.mark[j] = 1;
            break;
          }
        if (n_ev + 1 < max_entries) {
          out_evals[2 * n_ev + 2] = r;
          out_evals[2 * n_ev + 3] = -im;
        }
      }
    }
    __syncthreads();
    if (take) {
      n_sel += 1;
      held += (im != 0.0) ? 2 : 1;
    }
    n_ev += (im != 0.0) ? 2 : 1;
  }
  // a pencil with fewer eigenvalues than entries
  if (tid == 0)
    for (int i = n_ev; i < max_entries; ++i) out_evals[2 * i] = out_evals[2 * i + 1] = __builtin_nan("");
  if (tid == 0) sh.sel_n = n_sel;
  __syncthreads();
  return n_sel;
}

// ---------------------------------------------------------------- step 6 --
// Inverse iteration on the Hessenberg matrix Hq for eigenvalue (sr, si):
// LU of Hq - sigma I with adjacent-row pivoting, tiny pivots replaced by
// eps3, three solves from a vector of ones (the first with U alone).  Result
// (complex) in yr, yi.
//
// The factorisation runs in batches of IB steps.  Column j only changes in
// steps k < j, and the step's pivot needs only column k, so one wave takes
// the batch's IB columns through its steps (one column per lane, the carried
// row in registers, the next rows' entries loaded PF steps ahead) and
// records the multipliers and interchanges; then every thread takes one
// column to the right of the batch through the same steps.  The back
// substitution runs in blocks of IB rows from the bottom: all waves subtract
// the solved part from the block's right-hand side and stage the block's
// triangle in LDS; one wave solves the triangle.
constexpr int IB = 64;   // steps per batch, rows per back-substitution block
constexpr int PF = 8;    // steps whose row entries are loaded together
static_assert(IB * IB <= EIG_MAXD, "triangle staging in v3/v4");

// one factorisation step on a column: (c = carried row, f = fresh row) ->
// U entry t and the new carried value
__device__ __forceinline__ void lu_step(bool swp, double mr, double mi, double f_r, double f_i, double& c_r,
                                        double& c_i, double& t_r, double& t_i) {
  t_r = swp ? f_r : c_r;
  t_i = swp ? f_i : c_i;
  const double u_r = swp ? c_r : f_r, u_i = swp ? c_i : f_i;
  c_r = u_r - (mr * t_r - mi * t_i);
  c_i = u_i - (mr * t_i + mi * t_r);
}

__device__ void inverse_iteration(Shared& sh, const gdouble* Hq, gdouble* Wr, gdouble* Wi, int d,
                                  double sr, double si, double eps3, gdouble* yr, gdouble* yi) {
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  // carried row of the factorisation (row 0 of Hq - sigma I to start)
  double* cr = sh.v3;
  double* ci = sh.v4;
  for (int j = tid; j < d; j += NT) {
    cr[j] = Hq[j] - (j == 0 ? sr : 0.0);
    ci[j] = (j == 0) ? -si : 0.0;
  }
  __syncthreads();
  for (int k0 = 0; k0 < d; k0 += IB) {
    const int kend = min(k0 + IB, d - 1);   // steps k0 .. kend-1
    if (wv == 0) {
      const int jw = k0 + lane;
      const bool in = jw < d;
      double c_r = in ? cr[jw] : 0.0, c_i = in ? ci[jw] : 0.0;
      for (int kg = k0; kg < kend; kg += PF) {
        double fp[PF];
#pragma unroll
        for (int q = 0; q < PF; ++q) {
          const int k = kg + q;
          fp[q] = (in && k < kend && jw >= k) ? Hq[(size_t)(k + 1) * d + jw] : 0.0;
        }
#pragma unroll
        for (int q = 0; q < PF; ++q) {
          const int k = kg + q;
          if (k >= kend) break;
          const double f_r = (jw == k + 1) ? fp[q] - sr : fp[q];
          const double f_i = (jw == k + 1) ? -si : 0.0;
          const int src = k - k0;
          const double ar = lane_bcast(c_r, src), ai = lane_bcast(c_i, src);
          const double br = lane_bcast(f_r, src), bi = lane_bcast(f_i, src);
          const bool swp = cmod(br, bi) > cmod(ar, ai);
          double pr = swp ? br : ar, pi = swp ? bi : ai;
          const double orr = swp ? ar : br, oi = swp ? ai : bi;
          if (cmod(pr, pi) < eps3) {
            pr = eps3;
            pi = 0.0;
          }
          const double den = pr * pr + pi * pi;
          const double mr = (orr * pr + oi * pi) / den, mi = (oi * pr - orr * pi) / den;
          if (lane == 0) {
            sh.v1[k] = mr;
            sh.v2[k] = mi;
            sh.mark[k] = swp ? 1 : 0;
          }
          if (in && jw >= k) {
            double t_r, t_i;
            if (jw == k) {
              t_r = pr;
              t_i = pi;
              c_r = 0.0;
              c_i = 0.0;
            } else {
              lu_step(swp, mr, mi, f_r, f_i, c_r, c_i, t_r, t_i);
            }
            Wr[(size_t)k * d + jw] = t_r;
            Wi[(size_t)k * d + jw] = t_i;
          }
        }
      }
      if (jw == d - 1) {
        // the last pivot, after the last step
        if (cmod(c_r, c_i) < eps3) {
          c_r = eps3;
          c_i = 0.0;
        }
        Wr[(size_t)(d - 1) * d + d - 1] = c_r;
        Wi[(size_t)(d - 1) * d + d - 1] = c_i;
      }
    }
    __syncthreads();
    // the batch's steps on the columns right of it
    for (int j = k0 + IB + tid; j < d; j += NT) {
      double c_r = cr[j], c_i = ci[j];
      for (int kg = k0; kg < kend; kg += PF) {
        double fp[PF];
#pragma unroll
        for (int q = 0; q < PF; ++q) {
          const int k = kg + q;
          fp[q] = (k < kend) ? Hq[(size_t)(k + 1) * d + j] : 0.0;
        }
#pragma unroll
        for (int q = 0; q < PF; ++q) {
          const int k = kg + q;
          if (k >= kend) break;
          const double f_r = (j == k + 1) ? fp[q] - sr : fp[q];
          const double f_i = (j == k + 1) ? -si : 0.0;
          double t_r, t_i;
          lu_step(sh.mark[k] != 0, sh.v1[k], sh.v2[k], f_r, f_i, c_r, c_i, t_r, t_i);
          Wr[(size_t)k * d + j] = t_r;
          Wi[(size_t)k * d + j] = t_i;
        }
      }
      cr[j] = c_r;
      ci[j] = c_i;
    }
    __syncthreads();
  }
  // right-hand side in yr/yi (global)
  for (int i = tid; i < d; i += NT) {
    yr[i] = 1.0;
    yi[i] = 0.0;
  }
  __syncthreads();
  double* ub_r = sh.v3;   // a block's triangle: (l, q) at l * IB + (q ^ l)
  double* ub_i = sh.v4;
  double* part = sh.T;    // the block's right-hand side corrections (re, im)
  for (int it = 0; it < 3; ++it) {
    if (it > 0) {
      // apply L^-1 (interchanges and multipliers in order): one lane, from LDS
      for (int i = tid; i < d; i += NT) {
        sh.v3[i] = yr[i];
        sh.v4[i] = yi[i];
      }
      __syncthreads();
      if (tid == 0) {
        constexpr int LG = 8;   // steps whose operands are read together
        double r0 = sh.v3[0], i0 = sh.v4[0];
        for (int kg = 0; kg + 1 < d; kg += LG) {
          double nr[LG], ni[LG], mr[LG], mi[LG];
          bool sw[LG];
#pragma unroll
          for (int q = 0; q < LG; ++q) {
            const int k = min(kg + q, d - 2);
            nr[q] = sh.v3[k + 1];
            ni[q] = sh.v4[k + 1];
            mr[q] = sh.v1[k];
            mi[q] = sh.v2[k];
            sw[q] = sh.mark[k] != 0;
          }
#pragma unroll
          for (int q = 0; q < LG; ++q) {
            const int k = kg + q;
            if (k + 1 >= d) break;
            double r1 = nr[q], i1 = ni[q];
            if (sw[q]) {
              const double tr = r0, ti = i0;
              r0 = r1;
              i0 = i1;
              r1 = tr;
              i1 = ti;
            }
            r1 -= mr[q] * r0 - mi[q] * i0;
            i1 -= mr[q] * i0 + mi[q] * r0;
            yr[k] = r0;
            yi[k] = i0;
            r0 = r1;
            i0 = i1;
          }
        }
        yr[d - 1] = r0;
        yi[d - 1] = i0;
      }
      __syncthreads();
    }
    // back substitution U x = y, blocks of IB rows from the bottom
    for (int r0 = ((d - 1) / IB) * IB; r0 >= 0; r0 -= IB) {
      const int r1 = min(d, r0 + IB), nb = r1 - r0;
      for (int t = tid; t < IB * IB; t += NT) {
        const int l = t / IB, q = t % IB;
        const bool ok = l < nb && q < nb && q >= l;
        ub_r[l * IB + (q ^ l)] = ok ? Wr[(size_t)(r0 + l) * d + r0 + q] : 0.0;
        ub_i[l * IB + (q ^ l)] = ok ? Wi[(size_t)(r0 + l) * d + r0 + q] : 0.0;
      }
      {
        // rows wv, wv + NW, ... of the block together (IB / NW of them)
        constexpr int RW = IB / NW;
        double ar[RW], ai[RW];
#pragma unroll
        for (int h = 0; h < RW; ++h) ar[h] = ai[h] = 0.0;
        for (int j = r1 + lane; j < d; j += 64) {
          const double xr = yr[j], xi = yi[j];
#pragma unroll
          for (int h = 0; h < RW; ++h) {
            const int l = min(wv + h * NW, nb - 1);
            const double a = Wr[(size_t)(r0 + l) * d + j], b = Wi[(size_t)(r0 + l) * d + j];
            ar[h] += a * xr - b * xi;
            ai[h] += a * xi + b * xr;
          }
        }
#pragma unroll
        for (int h = 0; h < RW; ++h) {
          const int l = wv + h * NW;
          const double sr_ = wave_sum(ar[h]), si_ = wave_sum(ai[h]);
          if (lane == 0 && l < nb) {
            part[2 * l] = sr_;
            part[2 * l + 1] = si_;
          }
        }
      }
      __syncthreads();
      if (wv == 0) {
        double y_r = 0.0, y_i = 0.0, g_r = 1.0, g_i = 0.0;
        if (lane < nb) {
          y_r = yr[r0 + lane] - part[2 * lane];
          y_i = yi[r0 + lane] - part[2 * lane + 1];
          // 1 / u_ll = conj(u_ll) / |u_ll|^2
          const double ur = ub_r[lane * IB], ui = ub_i[lane * IB];
          const double den = ur * ur + ui * ui;
          g_r = ur / den;
          g_i = -ui / den;
        }
        for (int q = nb - 1; q >= 0; --q) {
          const double br = lane_bcast(y_r, q), bi = lane_bcast(y_i, q);
          const double hr = lane_bcast(g_r, q), hi = lane_bcast(g_i, q);
          const double xr = br * hr - bi * hi, xi = br * hi + bi * hr;
          if (lane == q) {
            y_r = xr;
            y_i = xi;
          } else if (lane < q) {
            const double a = ub_r[lane * IB + (q ^ lane)], b = ub_i[lane * IB + (q ^ lane)];
            y_r -= a * xr - b * xi;
            y_i -= a * xi + b * xr;
          }
        }
        if (lane < nb) {
          yr[r0 + lane] = y_r;
          yi[r0 + lane] = y_i;
        }
      }
      __syncthreads();
    }
    // normalise (largest modulus -> 1)
    double m = 0.0;
    for (int i = tid; i < d; i += NT) m = fmax(m, hypot(yr[i], yi[i]));
    m = block_max(sh, m);
    const double inv = (m > 0.0 && isfinite(m)) ? 1.0 / m : 1.0;
    for (int i = tid; i < d; i += NT) {
      yr[i] *= inv;
      yi[i] *= inv;
    }
    __syncthreads();
  }
}

// ---------------------------------------------------------------- step 6b --
// One wave per real vector z (length d, global): z <- L^-T Q z.
__device__ void back_transform_wave(const gdouble* V, const gdouble* tau, const gdouble* L, gdouble* z,
                                    int d) {
  const int lane = threadIdx.x & 63;
  for (int k = d - 3; k >= 0; --k) {
    const double tk = tau[k];
    if (tk == 0.0) continue;
    const gdouble* v = V + (size_t)k * d;
    double s = 0.0;
    for (int i = k + 1 + lane; i < d; i += 64) s += v[i] * z[i];
    s = wave_sum(s) * tk;
    for (int i = k + 1 + lane; i < d; i += 64) z[i] -= s * v[i];
  }
  // solve L^T c = z from the bottom; lane (k % 64) owns entry k
  for (int k = d - 1; k >= 0; --k) {
    double ck = 0.0;
    if ((k & 63) == lane) {
      ck = z[k] / L[(size_t)k * d + k];
      z[k] = ck;
    }
    ck = __shfl(ck, k & 63, 64);
    const gdouble* Lk = L + (size_t)k * d;
    for (int i = lane; i < k; i += 64) z[i] -= Lk[i] * ck;
  }
}

// An eigen-job with its buffers typed as global memory, so that every access
// is a global (not flat) memory instruction and LDS waits never wait for them.
// ------------------------------------- step 2, distributed over workgroups --
// The congruence A <- L^-1 A L^-T with no synchronisation inside a launch.
// The columns of X = L^-1 A are independent right-hand sides: the first
// launch gives each workgroup a slice of at most CSW columns.  Row i of
// A = X L^-T is L^-1 applied to row i of X: the second launch gives each
// workgroup the same slice of rows, which it transposes into those columns
// of W, solves and transposes back.  Blocking and summation order are those
// of lower_solve_rows.
constexpr int CSW = 64;   // columns per slice: one lane each

constexpr int CRCH = 128;  // trailing rows per LDS chunk of L
constexpr int CRW = CRCH / NW;   // of them per wave

struct CongShared {
  double xs[CB][CSW];     // the slice's rows of the current diagonal block
  double ld[CB][CB];      // diagonal block of L
  double lc[CRCH][CB + 1];  // L's entries left of the diagonal block for a chunk of trailing rows
};

// X[:, c0:c1] <- L^-1 X[:, c0:c1] for a row-major n x n X, c1 - c0 <= CSW
__device__ void lower_solve_slice(CongShared& cs, const gdouble* Lm, gdouble* X, int n, int c0, int c1) {
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  const int w = c1 - c0;
  for (int k0 = 0; k0 < n; k0 += CB) {
    const int kb = min(CB, n - k0);
    // diagonal block: wave 0, one lane per column, rows in order; the other
    // waves stage nothing and wait
    if (wv == 0) {
      for (int t = lane; t < CB * CB; t += 64) {
        const int m = t / CB, q = t % CB;
        cs.ld[m][q] = (m < kb && q <= m) ? Lm[(size_t)(k0 + m) * n + k0 + q] : 1.0;
      }
      for (int m = 0; m < CB; ++m)
        cs.xs[m][lane] = (m < kb && lane < w) ? X[(size_t)(k0 + m) * n + c0 + lane] : 0.0;
      __builtin_amdgcn_wave_barrier();
      for (int kk = 0; kk < kb; ++kk) {
        double v = cs.xs[kk][lane];
        for (int m = 0; m < kk; ++m) v -= cs.ld[kk][m] * cs.xs[m][lane];
        v /= cs.ld[kk][kk];
        cs.xs[kk][lane] = v;
        if (lane < w) X[(size_t)(k0 + kk) * n + c0 + lane] = v;
      }
    }
    __syncthreads();
    // trailing rows in chunks of CRCH: the chunk's L entries (columns of the
    // diagonal block, zero past kb) staged in LDS, then CRW rows per wave
    // with their loads issued together; lanes over the slice's columns
    const int jc = min(lane, w - 1);
    for (int r0 = k0 + kb; r0 < n; r0 += CRCH) {
      const int nr = min(CRCH, n - r0);
      for (int t = tid; t < nr * CB; t += NT) {
        const int r = t / CB, m = t % CB;
        cs.lc[r][m] = (m < kb) ? Lm[(size_t)(r0 + r) * n + k0 + m] : 0.0;
      }
      __syncthreads();
      double a[CRW];
#pragma unroll
      for (int j = 0; j < CRW; ++j) {
        const int i = min(r0 + wv + NW * j, n - 1);
        a[j] = X[(size_t)i * n + c0 + jc];
      }
#pragma unroll 1
      for (int m = 0; m < CB; ++m) {
        const double x = cs.xs[m][lane];
#pragma unroll
        for (int j = 0; j < CRW; ++j) a[j] -= cs.lc[wv + NW * j][m] * x;
      }
#pragma unroll
      for (int j = 0; j < CRW; ++j) {
        const int i = r0 + wv + NW * j;
        if (i < n && lane < w) X[(size_t)i * n + c0 + lane] = a[j];
      }
      __syncthreads();
    }
  }
}

__device__ __forceinline__ bool cong_slice(const EigJob& E, int n_jobs, int* job, int* c0, int* c1) {
  *job = blockIdx.x % n_jobs;
  const int part = blockIdx.x / n_jobs;
  const int d = E.d;
  if (d <= 0 || d > EIG_MAXD || E.info[0] != EIG_OK) return false;
  const int ns = (d + CSW - 1) / CSW;
  if (part >= ns) return false;
  *c0 = (int)((int64_t)d * part / ns);
  *c1 = (int)((int64_t)d * (part + 1) / ns);
  return true;
}

// first launch: X = L^-1 A in place, one column slice per workgroup
__global__ __launch_bounds__(NT) void cong_cols_kernel(const EigJob* __restrict__ jobs, int n_jobs) {
  __shared__ CongShared cs;
  const EigJob& E = jobs[blockIdx.x % n_jobs];
  int job, c0, c1;
  if (!cong_slice(E, n_jobs, &job, &c0, &c1)) return;
  const uint64_t t0 = wall_clock64();
  lower_solve_slice(cs, as_global(E.S), as_global(E.A), E.d, c0, c1);
  if (c0 == 0 && threadIdx.x == 0) as_global(E.info)[5] = (int32_t)(wall_clock64() - t0);
}

// second launch: rows c0..c1-1 of A <- (L^-1 (rows of X)^T)^T through W
__global__ __launch_bounds__(NT) void cong_rows_kernel(const EigJob* __restrict__ jobs, int n_jobs) {
  __shared__ CongShared cs;
  const EigJob& E = jobs[blockIdx.x % n_jobs];
  int job, c0, c1;
  if (!cong_slice(E, n_jobs, &job, &c0, &c1)) return;
  const uint64_t t0 = wall_clock64();
  const int d = E.d, w = c1 - c0, tid = threadIdx.x;
  gdouble* A = as_global(E.A);
  gdouble* W = as_global(E.W);
  for (int t = tid; t < d * CSW; t += NT) {
    const int j = t / CSW, i = t % CSW;
    if (i < w) W[(size_t)j * d + c0 + i] = A[(size_t)(c0 + i) * d + j];
  }
  __syncthreads();
  lower_solve_slice(cs, as_global(E.S), W, d, c0, c1);
  for (int t = tid; t < w * d; t += NT) {
    const int i = t / d, j = t % d;
    A[(size_t)(c0 + i) * d + j] = W[(size_t)j * d + c0 + i];
  }
  if (c0 == 0 && tid == 0) {
    BLM_GLOBAL int32_t* info = as_global(E.info);
    info[5] += (int32_t)(wall_clock64() - t0);
  }
}

// ------------------------------------- step 3, distributed over workgroups --
// The one-pass Hessenberg reduction of hessenberg() with each pencil's rows
// split over kw workgroups (a cooperative launch: all resident).  Per step
// every workgroup forms, redundantly and in the same order (so identically),
// beta = v^T p, q' and the next reflector from p (global, one entry per row,
// written by the row's owner), the per-workgroup partials of A^T v (global)
// and column k+1; then it updates its own rows and accumulates their part of
// the next step's products.  p and the partials are double-buffered by step
// parity; one barrier per step separates the steps.  The barrier is a
// counter per pencil in global memory with a bounded wait: past the bound
// the pencil's error flag is set and every workgroup leaves.

constexpr int HQCH = 4;  // column chunks of 64 per row pass

struct HessShared {
  double cv[EIG_MAXD];        // v of step k
  double cq[EIG_MAXD];        // q' of step k
  double nv[EIG_MAXD];        // v of step k+1
  double qw[NW][64 * HQCH];   // per-wave partials of A^T v for one column chunk
  double red[NW];
  int ok;
};

__device__ double hs_block_sum(HessShared& hs, double v) {
  v = wave_sum(v);
  if ((threadIdx.x & 63) == 0) hs.red[threadIdx.x >> 6] = v;
  __syncthreads();
  double t = 0.0;
#pragma unroll
  for (int w = 0; w < NW; ++w) t += hs.red[w];
  __syncthreads();
  return t;
}

// barrier among the kw workgroups of a pencil: cnt counts arrivals, err is
// the pencil's flag; returns false if the wait ran past its bound (or
// another workgroup's did)
__device__ bool pencil_barrier(int& ok_slot, unsigned* cnt, int* err, unsigned target, unsigned spin_limit) {
  __syncthreads();
  if (threadIdx.x == 0) {
    __threadfence();
    atomicAdd(cnt, 1u);
    int ok = 1;
    for (unsigned spins = 0;; ++spins) {
      if (__hip_atomic_load(cnt, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) >= target) break;
      if (__hip_atomic_load(err, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != 0 || spins >= spin_limit) {
        __hip_atomic_store(err, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        ok = 0;
        break;
      }
      __builtin_amdgcn_s_sleep(2);
    }
    __threadfence();
    ok_slot = ok;
  }
  __syncthreads();
  return ok_slot != 0;
}

// reflector of step k from column values in vec (rows k+1..d-1), as in
// hess_reflector; only `writer` stores V row k and tau[k]
__device__ double hess_reflector_hs(HessShared& hs, double* vec, gdouble* V, gdouble* tau, int k, int d,
                                    double* beta_h, bool writer) {
  const int tid = threadIdx.x;
  double part = 0.0;
  for (int i = k + 2 + tid; i < d; i += NT) part += vec[i] * vec[i];
  const double sigma = hs_block_sum(hs, part);
  const double alpha = vec[k + 1];
  double tk = 0.0, v0 = 1.0;
  if (sigma == 0.0) {
    *beta_h = alpha;
  } else {
    const double nrm = sqrt(alpha * alpha + sigma);
    const double bh = alpha <= 0.0 ? nrm : -nrm;
    v0 = alpha - bh;
    tk = (bh - alpha) / bh;
    *beta_h = bh;
  }
  for (int i = tid; i < d; i += NT) {
    const double vi = (i <= k) ? 0.0 : (i == k + 1) ? 1.0 : (sigma == 0.0 ? 0.0 : vec[i] / v0);
    vec[i] = vi;
    if (writer && i > k) V[(size_t)k * d + i] = vi;
  }
  if (writer && tid == 0) tau[k] = tk;
  __syncthreads();
  return tk;
}

// own rows [r0, r1): step k's update (UPD) and the next products (PROD)
template <bool UPD, bool PROD>
__device__ void hess_pass_rows(HessShared& hs, gdouble* A, int d, int k, int r0, int r1, double tk,
                               double beta_h, const double* cv, const gdouble* Pc, const double* cq,
                               const double* nv, gdouble* Pn, gdouble* Qn) {
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  constexpr int QCH = HQCH;
  const int j0 = k + 1, nj = d - j0;
  for (int c0 = 0; c0 < nj; c0 += 64 * QCH) {
    double qacc[QCH];
#pragma unroll
    for (int m = 0; m < QCH; ++m) qacc[m] = 0.0;
    for (int i = r0 + wv; i < r1; i += 2 * NW) {
      const int i2 = i + NW;
      const bool has2 = i2 < r1;
      gdouble* A1 = A + (size_t)i * d + j0;
      gdouble* A2 = A + (size_t)(has2 ? i2 : i) * d + j0;
      double a1[QCH], a2[QCH];
#pragma unroll
      for (int m = 0; m < QCH; ++m) {
        const int jc = min(c0 + lane + 64 * m, nj - 1);
        a1[m] = A1[jc];
        a2[m] = A2[jc];
      }
      if (UPD) {
        const double pi1 = Pc[i], pi2 = has2 ? Pc[i2] : 0.0;
        const double vi1 = cv[i], vi2 = has2 ? cv[i2] : 0.0;
#pragma unroll
        for (int m = 0; m < QCH; ++m) {
          const int j = c0 + lane + 64 * m;
          const bool ok = j < nj;
          const double vj = ok ? cv[j0 + j] : 0.0, qj = ok ? cq[j0 + j] : 0.0;
          a1[m] = hess_upd(a1[m], tk, pi1, vj, vi1, qj);
          a2[m] = hess_upd(a2[m], tk, pi2, vj, vi2, qj);
          // column k+1 below row k+1 is not stored while the next reflector
          // is formed: every workgroup reads its values from before this
          // step for that (unordered with this store: no barrier between),
          // and step k+1 overwrites them with beta and zeros
          const bool hold = PROD && j == 0;
          if (ok) {
            if (!(hold && i >= k + 2)) A1[j] = a1[m];
            if (has2 && !(hold && i2 >= k + 2)) A2[j] = a2[m];
          }
        }
      }
      if (PROD) {
        const double nv1 = nv[i], nv2 = has2 ? nv[i2] : 0.0;
        double p1 = 0.0, p2 = 0.0;
#pragma unroll
        for (int m = 0; m < QCH; ++m) {
          const int j = c0 + lane + 64 * m;
          const bool ok = j < nj;
          const double w = ok ? nv[j0 + j] : 0.0;
          const double x1 = ok ? a1[m] : 0.0, x2 = ok ? a2[m] : 0.0;
          p1 += x1 * w;
          p2 += x2 * w;
          qacc[m] += nv1 * x1 + nv2 * x2;
        }
        p1 = wave_sum(p1);
        p2 = wave_sum(p2);
        if (lane == 0) {
          Pn[i] = (c0 == 0 ? 0.0 : Pn[i]) + p1;
          if (has2) Pn[i2] = (c0 == 0 ? 0.0 : Pn[i2]) + p2;
        }
      }
    }
    if (PROD) {
      // the waves' partials of this chunk summed in LDS in a fixed order;
      // the workgroup's partial goes to global memory
#pragma unroll
      for (int m = 0; m < QCH; ++m) hs.qw[wv][lane + 64 * m] = qacc[m];
      __syncthreads();
      if (tid < 64 * QCH && c0 + tid < nj) {
        double q = 0.0;
#pragma unroll
        for (int w = 0; w < NW; ++w) q += hs.qw[w][tid];
        Qn[j0 + c0 + tid] = q;
      }
      __syncthreads();
    }
  }
  if (UPD) {
    for (int i = max(r0, k + 1) + tid; i < r1; i += NT) A[(size_t)i * d + k] = (i == k + 1) ? beta_h : 0.0;
  }
}

// The pencil of workgroup g of a launch with several workgroups per pencil
// (ranges [mw0, mw0 + mkw) in job order): binary search; *part: the
// workgroup's index within its pencil.
__device__ __forceinline__ int pencil_of(const EigJob* __restrict__ jobs, int n_jobs, int g, int* part) {
  int lo = 0, hi = n_jobs - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (jobs[mid].mw0 <= g) lo = mid;
    else hi = mid - 1;
  }
  *part = g - jobs[lo].mw0;
  return lo;
}

__global__ __launch_bounds__(NT) void hess_multi_kernel(const EigJob* __restrict__ jobs, int n_jobs,
                                                        unsigned* __restrict__ bar, unsigned spin_limit) {
  __shared__ HessShared hs;
  int part;
  const int job = pencil_of(jobs, n_jobs, blockIdx.x, &part);
  const EigJob& E = jobs[job];
  const int kw = E.mkw;
  const int d = E.d, tid = threadIdx.x;
  gdouble* A = as_global(E.A);
  gdouble* V = as_global(E.V);
  gdouble* tau = as_global(E.tau);
  gdouble* W = as_global(E.W);
  BLM_GLOBAL int32_t* info = as_global(E.info);
  if (d < HESS_MULTI_MIN || d > EIG_MAXD || info[0] != EIG_OK) return;
  const uint64_t t_start = wall_clock64();
  unsigned* cnt = bar + 2 * job;
  int* err = (int*)(bar + 2 * job + 1);
  const int r0 = (int)((int64_t)d * part / kw), r1 = (int)((int64_t)d * (part + 1) / kw);
  const bool writer = part == 0;
  // workspace: p [2][d], per-workgroup partials of A^T v [2][kw][d]
  gdouble* Pb[2] = {W, W + d};
  gdouble* Qb[2] = {W + 2 * (size_t)d, W + 2 * (size_t)d + (size_t)kw * d};
  double* cv = hs.cv;
  double* cq = hs.cq;
  double* nv = hs.nv;
  unsigned gen = 0;
  // step 0: reflector from column 0, its products over the own rows
  for (int i = tid; i < d; i += NT) cv[i] = (i >= 1) ? A[(size_t)i * d] : 0.0;
  __syncthreads();
  double beta_h = 0.0;
  double tk = hess_reflector_hs(hs, cv, V, tau, 0, d, &beta_h, writer);
  hess_pass_rows<false, true>(hs, A, d, 0, r0, r1, 0.0, 0.0, nullptr, nullptr, nullptr, cv, Pb[0],
                              Qb[0] + (size_t)part * d);
  if (!pencil_barrier(hs.ok, cnt, err, kw * ++gen, spin_limit)) {
    if (tid == 0) info[0] = EIG_SYNC;
    return;
  }
  for (int k = 0; k + 2 < d; ++k) {
    const int cur = k & 1, nxt = cur ^ 1;
    const gdouble* Pc = Pb[cur];
    const gdouble* Qc = Qb[cur];
    // beta = v^T p; q' = sum of the partials - tau beta v (fixed order);
    // all loads of a column are issued before the sums
    double bp = 0.0;
    for (int j = k + 1 + tid; j < d; j += NT) {
      bp += cv[j] * Pc[j];
      // the partials in order, 8 loads issued before their sums
      double q = 0.0;
      for (int w0 = 0; w0 < kw; w0 += 8) {
        double qp[8];
#pragma unroll
        for (int w = 0; w < 8; ++w) qp[w] = (w0 + w < kw) ? Qc[(size_t)(w0 + w) * d + j] : 0.0;
#pragma unroll
        for (int w = 0; w < 8; ++w)
          if (w0 + w < kw) q += qp[w];
      }
      cq[j] = q;
    }
    const double beta = hs_block_sum(hs, bp);
    for (int j = k + 1 + tid; j < d; j += NT) cq[j] -= tk * beta * cv[j];
    __syncthreads();
    const bool next = k + 3 < d;
    double tk_next = 0.0, bh_next = 0.0;
    if (next) {
      for (int i = tid; i < d; i += NT)
        nv[i] = (i >= k + 2) ? hess_upd(A[(size_t)i * d + k + 1], tk, Pc[i], 1.0, cv[i], cq[k + 1]) : 0.0;
      __syncthreads();
      tk_next = hess_reflector_hs(hs, nv, V, tau, k + 1, d, &bh_next, writer);
      hess_pass_rows<true, true>(hs, A, d, k, r0, r1, tk, beta_h, cv, Pc, cq, nv, Pb[nxt],
                                 Qb[nxt] + (size_t)part * d);
    } else {
      hess_pass_rows<true, false>(hs, A, d, k, r0, r1, tk, beta_h, cv, Pc, cq, nullptr, nullptr, nullptr);
    }
    if (!pencil_barrier(hs.ok, cnt, err, kw * ++gen, spin_limit)) {
      if (tid == 0) info[0] = EIG_SYNC;
      return;
    }
    double* t = cv;
    cv = nv;
    nv = t;
    tk = tk_next;
    beta_h = bh_next;
  }
  if (writer && tid == 0) info[6] = (int32_t)((wall_clock64() - t_start));
}

// ------------------------------------- step 1, distributed over workgroups --
// Cholesky factorisation S = L L^T of each pencil's overlap on kw workgroups
// (cooperative launch, row bands as in the Hessenberg reduction), blocked
// and left-looking: panel k0 holds columns k0..k0+CPB-1.  Every workgroup
// forms the panel's diagonal block D = S_kk - L_k,<k0 L_k,<k0^T and factors
// it in LDS in the same order, so every one takes the same pivots (and
// sees the same failure).  Each workgroup updates its own rows below the
// panel (S_ik -= L_i,<k0 L_k,<k0^T, in place) and solves them against the
// factor.  One barrier per panel makes those rows of L visible to the next
// panel; only after it do the owners of the panel's own rows write its
// factor over the diagonal block, which every workgroup has read by then.
// Within the diagonal block the operations and their order are those of the
// one-workgroup factorisation.
constexpr int CPB = 16;     // columns per panel
constexpr int CTOPW = 512;  // columns of the panel's top rows staged at a time

struct CholShared {
  double top[CPB][CTOPW];   // L[k0 + q][m0 + c]
  double dg[CPB][CPB];      // the diagonal block, then its factor
  double dsum[CPB * (CPB + 1) / 2];  // the diagonal block's sums over earlier columns
  int st;
  int ok;
};

__global__ __launch_bounds__(NT) void chol_multi_kernel(const EigJob* __restrict__ jobs, int n_jobs,
                                                        unsigned* __restrict__ bar, unsigned spin_limit) {
  __shared__ CholShared cs;
  int part;
  const int job = pencil_of(jobs, n_jobs, blockIdx.x, &part);
  const EigJob& E = jobs[job];
  const int kw = E.mkw;
  const int d = E.d, tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  gdouble* S = as_global(E.S);
  BLM_GLOBAL int32_t* info = as_global(E.info);
  if (d <= 0 || d > EIG_MAXD) return;
  const uint64_t t_start = wall_clock64();
  unsigned* cnt = bar + 2 * job;
  int* err = (int*)(bar + 2 * job + 1);
  const int r0 = (int)((int64_t)d * part / kw), r1 = (int)((int64_t)d * (part + 1) / kw);
  unsigned gen = 0;
  for (int k0 = 0; k0 < d; k0 += CPB) {
    const int kb = min(CPB, d - k0);
    // (a) D's lower triangle: pair t = (q, p), p <= q, t = q (q + 1) / 2 + p
    constexpr int NPAIR = CPB * (CPB + 1) / 2;
    for (int t = tid; t < NPAIR; t += NT) cs.dsum[t] = 0.0;
    const int rb0 = max(r0, k0 + kb);   // own rows below the panel
    for (int m0 = 0; m0 < k0; m0 += CTOPW) {
      const int cw = min(CTOPW, k0 - m0);
      __syncthreads();
      for (int t = tid; t < CPB * CTOPW; t += NT) {
        const int q = t / CTOPW, c = t % CTOPW;
        cs.top[q][c] = (q < kb && c < cw) ? S[(size_t)(k0 + q) * d + m0 + c] : 0.0;
      }
      __syncthreads();
      for (int t = wv; t < NPAIR; t += NW) {
        int q = 0;
        while ((q + 1) * (q + 2) / 2 <= t) ++q;
        const int pp = t - q * (q + 1) / 2;
        double ps = 0.0;
#pragma unroll 1
        for (int c = lane; c < cw; c += 64) ps += cs.top[q][c] * cs.top[pp][c];
        ps = wave_sum(ps);
        if (lane == 0) cs.dsum[t] += ps;
      }
      // own rows below the panel: S[i][k0 + q] -= L[i][m0..] . top[q][..]
      for (int iv = rb0 + wv; iv < r1; iv += NW) {
        const int i = __builtin_amdgcn_readfirstlane(iv);
        double acc[CPB];
#pragma unroll
        for (int q = 0; q < CPB; ++q) acc[q] = 0.0;
#pragma unroll 1
        for (int c = lane; c < cw; c += 64) {
          const double x = S[(size_t)i * d + m0 + c];
#pragma unroll
          for (int q = 0; q < CPB; ++q) acc[q] += x * cs.top[q][c];
        }
#pragma unroll
        for (int q = 0; q < CPB; ++q) acc[q] = wave_sum(acc[q]);
        if (lane < kb) {
          double mine = acc[0];
#pragma unroll
          for (int q = 1; q < CPB; ++q)
            if (lane == q) mine = acc[q];
          S[(size_t)i * d + k0 + lane] -= mine;
        }
      }
    }
    // D = S_kk - the sums; lower triangle in dg
    __syncthreads();
    for (int t = tid; t < NPAIR; t += NT) {
      int q = 0;
      while ((q + 1) * (q + 2) / 2 <= t) ++q;
      const int pp = t - q * (q + 1) / 2;
      cs.dg[q][pp] = (q < kb) ? S[(size_t)(k0 + q) * d + k0 + pp] - cs.dsum[t] : 0.0;
    }
    __syncthreads();
    // (b) factor D in LDS: wave 0, lanes over rows, columns in order
    if (wv == 0) {
      int st = EIG_OK;
      for (int j = 0; j < kb; ++j) {
        double v = cs.dg[j][j];
        for (int pp = 0; pp < j; ++pp) v -= cs.dg[j][pp] * cs.dg[j][pp];
        if (!isfinite(v)) st = EIG_NONFINITE;
        else if (!(v > 0.0)) st = EIG_NOT_PD;
        if (st != EIG_OK) break;
        const double piv = sqrt(v);
        double x = 0.0;
        if (lane > j && lane < kb) {
          x = cs.dg[lane][j];
          for (int pp = 0; pp < j; ++pp) x -= cs.dg[lane][pp] * cs.dg[j][pp];
          x /= piv;
        }
        __builtin_amdgcn_wave_barrier();
        if (lane > j && lane < kb) cs.dg[lane][j] = x;
        if (lane == 0) cs.dg[j][j] = piv;
        __builtin_amdgcn_wave_barrier();
      }
      if (lane == 0) cs.st = st;
    }
    __syncthreads();
    if (cs.st != EIG_OK) {
      if (part == 0 && tid == 0) info[0] = cs.st;
      return;
    }
    // (c) own rows below the panel: L[i][k0 + q] = (a_q - sum_p L[i][k0 + p] f[q][p]) / f[q][q],
    // one wave per row, lane q holding entry q, the terms subtracted in p order
    for (int iv = rb0 + wv; iv < r1; iv += NW) {
      const int i = __builtin_amdgcn_readfirstlane(iv);
      gdouble* Li = S + (size_t)i * d + k0;
      double x = (lane < kb) ? Li[lane] : 0.0;
      for (int q = 0; q < kb; ++q) {
        if (lane == q) x /= cs.dg[q][q];
        const double xq = lane_bcast(x, q);
        if (lane > q && lane < kb) x -= xq * cs.dg[lane][q];
      }
      if (lane < kb) Li[lane] = x;
    }
    if (!pencil_barrier(cs.ok, cnt, err, kw * ++gen, spin_limit)) {
      if (tid == 0) info[0] = EIG_SYNC;
      return;
    }
    // every workgroup has read the panel's diagonal block: its factor into
    // the rows this workgroup owns (nothing in this launch reads it back)
    for (int t = tid; t < CPB * CPB; t += NT) {
      const int q = t / CPB, pp = t % CPB;
      if (q < kb && pp <= q && k0 + q >= r0 && k0 + q < r1) S[(size_t)(k0 + q) * d + k0 + pp] = cs.dg[q][pp];
    }
    __syncthreads();
  }
  if (part == 0 && tid == 0) info[4] = (int32_t)(wall_clock64() - t_start);
}

__global__ void eig_info_init_kernel(const EigJob* __restrict__ jobs, int n_jobs) {
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t < n_jobs * EIG_INFO) as_global(jobs[t / EIG_INFO].info)[t % EIG_INFO] = 0;
}

struct GJob {
  int32_t d, mode, n_want, beta0, nbeta;
  gdouble *S, *A, *Hq, *V, *W, *vec, *wr, *wi, *tau, *out, *out_evals;
  BLM_GLOBAL int32_t* info;
};

__device__ __forceinline__ GJob global_view(const EigJob& E) {
  GJob J;
  J.d = E.d;
  J.mode = E.mode;
  J.n_want = E.n_want;
  J.beta0 = E.beta0;
  J.nbeta = E.nbeta;
  J.S = as_global(E.S);
  J.A = as_global(E.A);
  J.Hq = as_global(E.Hq);
  J.V = as_global(E.V);
  J.W = as_global(E.W);
  J.vec = as_global(E.vec);
  J.wr = as_global(E.wr);
  J.wi = as_global(E.wi);
  J.tau = as_global(E.tau);
  J.out = as_global(E.out);
  J.out_evals = as_global(E.out_evals);
  J.info = as_global(E.info);
  return J;
}

// Phase clock (100 MHz constant counter): info[4 + i] = ticks spent in phase i.
__device__ __forceinline__ void phase_mark(const GJob& J, uint64_t& t, int i) {
  const uint64_t now = wall_clock64();
  if (threadIdx.x == 0) J.info[4 + i] = (int32_t)(now - t);
  t = now;
}

// phases: PH_CHOL Cholesky, PH_CONG congruence, PH_HESS the Hessenberg
// reduction, PH_BACK the rest.  A launch runs the phases its mask names; a
// pencil whose status is already an error skips the later ones.
__global__ __launch_bounds__(NT) void eig_kernel(const EigJob* __restrict__ jobs, int phases) {
  __shared__ Shared sh;
  const GJob J = global_view(jobs[blockIdx.x]);
  const int d = J.d, tid = threadIdx.x, wv = tid >> 6;
  uint64_t clk = wall_clock64();
  if (tid == 0) sh.isc[2] = 0;
  if ((phases & PH_CHOL) && tid == 0)
    for (int i = 0; i < EIG_INFO; ++i) J.info[i] = 0;
  __syncthreads();
  if (d <= 0 || d > EIG_MAXD) return;
  if (!(phases & PH_CHOL) && J.info[0] != EIG_OK) return;

  int st = EIG_OK;
  if (phases & PH_CHOL) {
    st = cholesky(sh, J.S, d);
    if (st != EIG_OK) {
      if (tid == 0) J.info[0] = st;
      return;
    }
    phase_mark(J, clk, 0);
  }
  if (phases & PH_CONG) {
    congruence(sh, J.S, J.A, J.W, d);
    phase_mark(J, clk, 1);
  }
  // after a distributed reduction (PH_HESS not set) the small pencils it
  // left out are reduced here
  if ((phases & PH_HESS) || ((phases & PH_BACK) && d < HESS_MULTI_MIN)) {
    hessenberg(sh, J.A, J.V, J.tau, J.W, d);
    phase_mark(J, clk, 2);
  }
  if (!(phases & PH_BACK)) return;
  for (size_t i = tid; i < (size_t)d * d; i += NT) J.Hq[i] = J.A[i];
  __syncthreads();
  // norm of the Hessenberg matrix for the inverse-iteration pivot floor
  double part = 0.0;
  for (size_t i = tid; i < (size_t)d * d; i += NT) part += fabs(J.Hq[i]);
  const double hnorm = block_sum(sh, part);
  int iters = 0;
  st = hqr<true>(sh, J.A, d, d, J.wr, J.wi, &iters, J.W);   // W: the chase's transposed rows
  __syncthreads();
  phase_mark(J, clk, 3);
  if (tid == 0) {
    J.info[3] = iters;
    for (int i = 0; i < 4; ++i) J.info[12 + i] = (int32_t)sh.qst[i];
  }
  if (st == EIG_OK && sh.isc[2]) st = EIG_NONFINITE;
  if (st != EIG_OK) {
    if (tid == 0) J.info[0] = st;
    return;
  }
  if (J.mode == EIG_VALUES) return;

  const int want = (J.mode == EIG_STAGE2) ? 1 : J.n_want;
  const int max_entries = (J.mode == EIG_STAGE2) ? 2 : J.n_want + 1;
  const int n_sel = select_lowest(sh, J.wr, J.wi, d, want, J.out_evals, max_entries);
  const double eps3 = EPS * fmax(hnorm, 1e-300);

  // eigenvectors of the chosen eigenvalues, complex, into vec[s][0|1][d]
  phase_mark(J, clk, 4);
  for (int s = 0; s < n_sel; ++s) {
    gdouble* yr = J.vec + (size_t)(2 * s) * d;
    gdouble* yi = yr + d;
    inverse_iteration(sh, J.Hq, J.W, J.W + (size_t)d * d, d, sh.sel_r[s], sh.sel_i[s], eps3, yr, yi);
  }
  phase_mark(J, clk, 5);
  // back to the pencil's coordinates: one wave per real vector
  const int n_real = 2 * n_sel;
  for (int v = wv; v < n_real; v += NW) {
    const int s = v >> 1;
    if ((v & 1) && sh.sel_i[s] == 0.0) continue;
    back_transform_wave(J.V, J.tau, J.S, J.vec + (size_t)v * d, d);
  }
  __syncthreads();
  phase_mark(J, clk, 6);

  if (J.mode == EIG_STAGE2) {
    for (int i = tid; i < d; i += NT) {
      J.out[i] = J.vec[i];
      J.out[d + i] = (sh.sel_i[0] == 0.0) ? 0.0 : J.vec[(size_t)d + i];
    }
    if (tid == 0) {
      J.info[1] = n_sel;
      J.info[2] = (sh.sel_i[0] != 0.0) ? 1 : 0;
    }
    return;
  }

  // block: parameter parts of Re c (and Im c for a pair), MGS, kept rows
  const int nb = J.nbeta;
  int kept = 0, pair = 0;
  for (int s = 0; s < n_sel; ++s) {
    const int parts = (sh.sel_i[s] != 0.0) ? 2 : 1;
    if (parts == 2) pair = 1;
    for (int pc = 0; pc < parts; ++pc) {
      const gdouble* src = J.vec + (size_t)(2 * s + pc) * d + J.beta0;
      gdouble* dst = J.out + (size_t)kept * nb;
      double part0 = 0.0;
      for (int i = tid; i < nb; i += NT) {
        const double x = src[i];
        dst[i] = x;
        part0 += x * x;
      }
      const double n0 = sqrt(block_sum(sh, part0));
      for (int q = 0; q < kept; ++q) {
        const gdouble* qv = J.out + (size_t)q * nb;
        double pd = 0.0;
        for (int i = tid; i < nb; i += NT) pd += qv[i] * dst[i];
        const double dot = block_sum(sh, pd);
        for (int i = tid; i < nb; i += NT) dst[i] -= dot * qv[i];
        __syncthreads();
      }
      double pn = 0.0;
      for (int i = tid; i < nb; i += NT) pn += dst[i] * dst[i];
      const double nr = sqrt(block_sum(sh, pn));
      if (n0 > 0.0 && nr >= DROP_TOL * n0 && kept < nb) {
        const double inv = 1.0 / nr;
        for (int i = tid; i < nb; i += NT) dst[i] *= inv;
        __syncthreads();
        ++kept;
      }
    }
  }
  if (tid == 0) {
    J.info[1] = kept;
    J.info[2] = pair;
  }
  phase_mark(J, clk, 7);
}

}  // namespace

void launch_eig(const EigJob* d_jobs, int n_jobs, hipStream_t st) {
  if (n_jobs <= 0) return;
  hipLaunchKernelGGL(eig_kernel, dim3(n_jobs), dim3(NT), 0, st, d_jobs, (int)PH_ALL);
}

__global__ void fill_u32_kernel(unsigned* p, int n) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = 0u;
}

// Workgroups per pencil for the distributed Cholesky and Hessenberg steps:
// every pencil one, then the remaining CUs one at a time to the pencil whose
// estimated time is longest, d^3 / kw (its row passes) + 5e4 d (its
// barriers, one per step, in the same units), up to max_kw (32 for pencils
// of 1,536 or more, 16 from 1,024, 8 below, where a barrier among more
// workgroups costs more than their shorter bands save).  Returns the
// launch's workgroup count, 0 when there are too few CUs for two per pencil.
static int plan_split(EigJob* jobs, int n_jobs, int n_cus, int max_kw) {
  if (n_jobs <= 0 || max_kw < 2 || n_cus / n_jobs < 2) return 0;
  std::vector<int> kw(n_jobs, 1);
  auto t_est = [&](int j, int k) {
    const double d = jobs[j].d;
    return d * d * d / k + 5e4 * d;
  };
  auto cap = [&](int j) { return min(max_kw, jobs[j].d >= 1536 ? 32 : jobs[j].d >= 1024 ? 16 : 8); };
  for (int left = n_cus - n_jobs; left > 0; --left) {
    int best = -1;
    double tb = 0.0;
    for (int j = 0; j < n_jobs; ++j) {
      if (kw[j] >= cap(j)) continue;
      const double t = t_est(j, kw[j]);
      if (best < 0 || t > tb) {
        best = j;
        tb = t;
      }
    }
    if (best < 0) break;
    ++kw[best];
  }
  int g = 0;
  for (int j = 0; j < n_jobs; ++j) {
    jobs[j].mw0 = g;
    jobs[j].mkw = kw[j];
    g += kw[j];
  }
  return g;
}

bool launch_eig_split(EigJob* h_jobs, EigJob* d_jobs, int n_jobs, int d_max, int n_cus, int max_kw,
                      unsigned* d_bar, unsigned spin_limit, hipStream_t st) {
  if (n_jobs <= 0) return true;
  const int n_wg = plan_split(h_jobs, n_jobs, n_cus, min(HKW_MAX, max_kw));
  if (hipMemcpyAsync(d_jobs, h_jobs, sizeof(EigJob) * n_jobs, hipMemcpyHostToDevice, st) != hipSuccess) return false;
  bool chol_done = false;
  if (n_wg > 0) {
    hipLaunchKernelGGL(eig_info_init_kernel, dim3((n_jobs * EIG_INFO + 255) / 256), dim3(256), 0, st, d_jobs,
                       n_jobs);
    hipLaunchKernelGGL(fill_u32_kernel, dim3((2 * n_jobs + 255) / 256), dim3(256), 0, st, d_bar, 2 * n_jobs);
    int nj = n_jobs;
    void* args[] = {(void*)&d_jobs, (void*)&nj, (void*)&d_bar, (void*)&spin_limit};
    chol_done = hipLaunchCooperativeKernel((const void*)chol_multi_kernel, dim3(n_wg), dim3(NT), args, 0, st) ==
                hipSuccess;
    if (!chol_done) (void)hipGetLastError();
  }
  if (!chol_done) hipLaunchKernelGGL(eig_kernel, dim3(n_jobs), dim3(NT), 0, st, d_jobs, (int)PH_CHOL);
  const int ns = max(1, (min(d_max, EIG_MAXD) + CSW - 1) / CSW);
  hipLaunchKernelGGL(cong_cols_kernel, dim3(n_jobs * ns), dim3(NT), 0, st, d_jobs, n_jobs);
  hipLaunchKernelGGL(cong_rows_kernel, dim3(n_jobs * ns), dim3(NT), 0, st, d_jobs, n_jobs);
  if (n_wg == 0) {
    hipLaunchKernelGGL(eig_kernel, dim3(n_jobs), dim3(NT), 0, st, d_jobs, (int)(PH_HESS | PH_BACK));
    return true;
  }
  hipLaunchKernelGGL(fill_u32_kernel, dim3((2 * n_jobs + 255) / 256), dim3(256), 0, st, d_bar, 2 * n_jobs);
  int nj = n_jobs;
  void* args[] = {(void*)&d_jobs, (void*)&nj, (void*)&d_bar, (void*)&spin_limit};
  const hipError_t e = hipLaunchCooperativeKernel((const void*)hess_multi_kernel, dim3(n_wg), dim3(NT), args, 0, st);
  if (e != hipSuccess) {
    (void)hipGetLastError();
    // the workgroups cannot all be resident: the Hessenberg reduction one
    // workgroup per pencil
    hipLaunchKernelGGL(eig_kernel, dim3(n_jobs), dim3(NT), 0, st, d_jobs, (int)(PH_HESS | PH_BACK));
    return false;
  }
  hipLaunchKernelGGL(eig_kernel, dim3(n_jobs), dim3(NT), 0, st, d_jobs, (int)PH_BACK);
  return true;
}

}  // namespace blm
