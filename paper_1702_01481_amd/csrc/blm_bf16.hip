// Mixed-precision block build on the BF16 matrix cores of gfx950.
//
// Every sample value x is stored as BF16 pieces x = hi + mid + lo (or
// hi + lo) whose FP64 sum is exact.  A product x*y is taken as the sum of the
// piece products of total order <= pieces - 1 (hi*hi, hi*mid, mid*hi, hi*lo,
// lo*hi, mid*mid for three pieces; hi*hi, hi*lo, lo*hi for two), each on
// v_mfma_f32_16x16x32_bf16 (exact products, FP32 sums).  FP32 accumulators
// are added into FP64 registers after every 32 samples, and the slices are summed
// in FP64 by the same fixed-order reduction as the FP64 path.  These are the
// block estimates of Eq. 3 on the one-block basis (Eq. 4 / Eq. 10).  The
// first 16 aux columns (the wave function itself and previous directions)
// are packed to BF16 pieces per chunk, and diagonal pairs compute their
// coupling strips of Fig. 1 here; the aux Gram and further aux groups'
// strips run on the FP64 kernel.
//
// Storage ("k-packed"): element (s, x) of piece p is at
// base + p * pstride + ((s / 8) * ld + x) * 8 + s % 8.  A lane's matrix-core
// operand (8 consecutive samples of one parameter) is one 16-byte load.
#include "blm_internal.h"

namespace blm {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f4 __attribute__((ext_vector_type(4)));
typedef double d4b __attribute__((ext_vector_type(4)));
typedef unsigned int u4v __attribute__((ext_vector_type(4)));

// FP32 accumulators are added into FP64 every few 32-sample steps, so that
// each FP32 partial holds only a few steps' sums: flushing every 256 samples
// gave block estimates within 6e-8 of FP64, and the block eigenvectors
// amplified that into 2e-6 of the energy; every 32 samples gave 2e-8 and
// 5.5e-8.

__device__ __forceinline__ f4 mfma_bf16(const bf16x8& a, const bf16x8& b, f4 c) {
  // D[i][j] += sum_k A[i][k] B[k][j], 16x16x32; lane l supplies
  // A[l%16][8(l/16) .. 8(l/16)+7] and B[8(l/16) .. +7][l%16].
  return __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, c, 0, 0, 0);
}

// Row of the 16x16 result held in register r of lane l (probed on gfx950;
// it differs from the FP64 16x16x4 instruction's layout).
__device__ __forceinline__ int bf16_d_row(int lane, int r) { return 4 * (lane >> 4) + r; }

__device__ __forceinline__ bf16x8 load_frag(const BLM_GLOBAL uint16_t* p, bool v) {
  if (v) return *reinterpret_cast<const BLM_GLOBAL bf16x8*>(p);
  bf16x8 z;
#pragma unroll
  for (int e = 0; e < 8; ++e) z[e] = (__bf16)0.0f;
  return z;
}

// One workgroup computes a pair of 64 x 64 tile jobs that share their row
// tile i: the A side is {O_i, e_i} (64 parameters), the B side {O_j, e_j,
// O_j', e_j'} (128 parameters, j' = j + 1).  Per 32-sample step the pieces of
// both sides are copied once into LDS by direct global->LDS loads (no
// registers involved; double-buffered, 72 KB per buffer, one workgroup per
// CU).  Eight waves, two per SIMD: wave (wr, wc) owns rows 32 wr .. + 31 and
// columns 32 wc .. + 31 of the 64 x 128 output of each product, so while one
// wave of a SIMD adds its FP32 partial sums into FP64, the other keeps the
// matrix core busy.  Per step a wave reads 24 fragments from LDS for 72
// matrix-core products.
constexpr int BP_COLS = 2 * GT;                  // B-side columns of a pair
constexpr int BP_STEP = 32;                      // samples per step (one k-depth)
constexpr int BP_KG = BP_STEP / 8;               // 8-sample groups per step
constexpr int BP_THREADS = 512;
// FP32 accumulators are added into FP64 every BP_FLUSH steps (64 samples):
// each FP32 partial then holds 12 matrix-core results (6 piece products of
// 2 steps), within about 1e-7 of its FP64 sum.
constexpr int BP_FLUSH = 2;

template <int PIECES>
struct BpLds {
  u4v A[2][PIECES][BP_KG][GT];        // [O or e][piece][group][column]
  u4v B[2][PIECES][BP_KG][BP_COLS];
  u4v X[2][PIECES][BP_KG][NAUX];      // aux columns [Xa or Ya][piece][group][column]
};

__device__ __forceinline__ void lds_dma16(const BLM_GLOBAL void* src, u4v* lds_base) {
  __builtin_amdgcn_global_load_lds(src, (__attribute__((address_space(3))) void*)lds_base, 16, 0, 0);
}

// STRIPS: the launch holds the pairs whose first job is a diagonal tile
// (coupling strips and their aux copies); the pairs without are a launch of
// their own, whose kernel needs fewer registers (no strip selects): with
// the strip logic it kept a value in scratch, and the wait for that reload
// (a vector-memory count) also waited for the step's global-to-LDS copies,
// so copies and products no longer overlapped.
template <int PIECES, bool STRIPS>
__global__ __launch_bounds__(BP_THREADS, 1) void gram_bf16_kernel(const PairJob* __restrict__ pairs,
                                                                 int n_pairs,
                                                                 const GramJob* __restrict__ jobs,
                                                                 const Slice* __restrict__ slices,
                                                                 int n_slices, int P,
                                                                 double* __restrict__ partial,
    const int2* __restrict__ sets) {
  // wave instructions per step: one per (side, array, piece, group[, half]);
  // diagonal pairs also copy the aux columns (one per array and piece)
  constexpr int NIA = 2 * PIECES * BP_KG;              // A side, 64 columns each
  constexpr int NIB = 2 * PIECES * BP_KG * 2;          // B side, two 64-column halves
  constexpr int NIX = 2 * PIECES;                      // aux: 4 groups x 16 columns each
  constexpr int NW = BP_THREADS / 64;
  __shared__ BpLds<PIECES> L[2];

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

  // The wave index is made provably wave-uniform, so that every per-wave
  // choice below (which products, which job) is a scalar branch: a
  // matrix-core instruction is not masked by the lane mask, so it must
  // never sit under a divergent condition.
  const int tid = threadIdx.x, lane = tid & 63;
  const int wv = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int i16 = lane & 15, k4 = lane >> 4;
  const int wr = wv & 1, wc = wv >> 1;           // 2 x 4 waves over 64 x 128
  const bool wave_b = wc >= 2;
  const bool wave_on = !wave_b || has_b;
  const GramJob& JW = wave_b ? JB : JA;
  const bool third = JW.kind == JOB_OFF;
  // Diagonal job with strips: the waves of its tile (wc < 2) compute the
  // coupling strips of Fig. 1 in the third product's registers:
  // aux^T O_i and aux^T e_i (wr = 0), auxE^T O_i (wr = 1), 16 x 32 each.
  const bool pair_strips = STRIPS && JA.kind == JOB_DIAG;
  const bool strip = pair_strips && !wave_b;
  const int n_instr = NIA + NIB + (pair_strips ? NIX : 0);

  // this lane's global column in each 64-column half (clamped into the tile)
  const int acol = JA.ci + min(lane, JA.mi - 1);
  const int bcol0 = JA.cj + min(lane, JA.nj - 1);
  const int bcol1 = JB.cj + min(lane, JB.nj - 1);

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

  // copies step (slice sl, first group grp0) into LDS buffer buf: this wave
  // issues instructions wv, wv + NW, ...; every address is inside the slice
  // (columns and groups clamped), granules the pair does not use are never
  // multiplied
  auto issue = [&](int sl, int64_t grp0, int buf) {
    const Slice S = slices[sl];
    const int64_t n8 = (S.n + 7) >> 3;
    const BLM_GLOBAL uint16_t* O = as_global((const uint16_t*)S.O);
    const BLM_GLOBAL uint16_t* E = as_global((const uint16_t*)S.e);
#pragma unroll
    for (int ii = 0; ii < (NIA + NIB + NIX + NW - 1) / NW; ++ii) {
      const int in = wv + ii * NW;
      if (in >= n_instr) break;
      if (in >= NIA + NIB) {
        // aux columns: lane -> (group lane / 16, column lane % 16)
        const int ix = in - NIA - NIB, xarr = ix / PIECES, xpc = ix % PIECES;
        const int64_t gg = min(grp0 + (lane >> 4), n8 - 1);
        const BLM_GLOBAL uint16_t* xb = as_global(xarr ? S.Yp : S.Xp);
        lds_dma16(xb + (int64_t)xpc * S.apstride + (gg * NAUX + (lane & 15)) * 8,
                  &L[buf].X[xarr][xpc][0][0]);
        continue;
      }
      int arr, pc, grp, col;
      u4v* dst;
      if (in < NIA) {
        grp = in % BP_KG;
        pc = (in / BP_KG) % PIECES;
        arr = in / (BP_KG * PIECES);
        col = acol;
        dst = &L[buf].A[arr][pc][grp][0];
      } else {
        const int ib = in - NIA;
        const int half = ib & 1;
        grp = (ib >> 1) % BP_KG;
        pc = ((ib >> 1) / BP_KG) % PIECES;
        arr = (ib >> 1) / (BP_KG * PIECES);
        col = bcol0 + half * (bcol1 - bcol0);   // arithmetic: a conditional over captured
                                                // values would keep them in memory
        dst = &L[buf].B[arr][pc][grp][GT * half];
      }
      const int64_t gg = min(grp0 + grp, n8 - 1);
      const BLM_GLOBAL uint16_t* base = arr ? E : O;
      lds_dma16(base + (int64_t)pc * S.pstride + (gg * S.ld + col) * 8, dst);
    }
  };
  // Third product slot, fixed per wave: e_i^T O_j for an off-diagonal tile,
  // the coupling strips for a diagonal one (x = 0: aux^T O_i, or auxE^T O_i
  // on the wr = 1 waves; x = 1: aux^T e_i).  Its A operand is chosen by LDS
  // address and its B operand by a register select, so every wave runs the
  // same straight-line sequence of matrix-core instructions.
  const int a3_base = strip ? (int)((const char*)&L[0].X[wr][0][k4][i16] - (const char*)&L[0])
                            : (int)((const char*)&L[0].A[1][0][k4][32 * wr + i16] - (const char*)&L[0]);
  const int a3_x = strip ? 0 : 16 * (int)sizeof(u4v);                  // next 16 rows
  const int a3_p = strip ? BP_KG * NAUX * (int)sizeof(u4v) : BP_KG * GT * (int)sizeof(u4v);
  const bool b3_e = strip && wr == 0;                                  // x = 1 pairs with e_i
  auto compute = [&](int buf, int64_t n8_left, bool flush) {
    // groups at or past the slice's end contribute nothing: on the last step
    // of a slice the A side is zeroed by a lane mask
    const bool partial = n8_left < BP_KG;
    const unsigned km = (k4 < n8_left) ? 0xFFFFFFFFu : 0u;
    const BpLds<PIECES>& Lb = L[buf];
    const char* lb = (const char*)&Lb;
    bf16x8 bO[2][PIECES], bE[2][PIECES];
#pragma unroll
    for (int y = 0; y < 2; ++y)
#pragma unroll
      for (int pc = 0; pc < PIECES; ++pc) {
        const int col = 32 * wc + 16 * y + i16;
        bO[y][pc] = __builtin_bit_cast(bf16x8, Lb.B[0][pc][k4][col]);
        bE[y][pc] = __builtin_bit_cast(bf16x8, Lb.B[1][pc][k4][col]);
      }
#pragma unroll
    for (int pa = 0; pa < PIECES; ++pa) {
      bf16x8 aO[2], a3[2];
#pragma unroll
      for (int x = 0; x < 2; ++x) {
        const int row = 32 * wr + 16 * x + i16;
        u4v vo = Lb.A[0][pa][k4][row];
        u4v v3 = *(const u4v*)(lb + a3_base + x * a3_x + pa * a3_p);
        if (partial) {
          vo &= km;
          v3 &= km;
        }
        aO[x] = __builtin_bit_cast(bf16x8, vo);
        a3[x] = __builtin_bit_cast(bf16x8, v3);
      }
#pragma unroll
      for (int pb = 0; pb + pa < PIECES; ++pb)
#pragma unroll
        for (int x = 0; x < 2; ++x)
#pragma unroll
          for (int y = 0; y < 2; ++y) {
            acc[0][x][y] = mfma_bf16(aO[x], bO[y][pb], acc[0][x][y]);
            acc[1][x][y] = mfma_bf16(aO[x], bE[y][pb], acc[1][x][y]);
            const bf16x8 b3 = (x == 1 && b3_e) ? bE[y][pb] : bO[y][pb];
            acc[2][x][y] = mfma_bf16(a3[x], b3, acc[2][x][y]);
          }
    }
    if (!flush) return;
#pragma unroll
    for (int t = 0; t < 3; ++t)
#pragma unroll
      for (int x = 0; x < 2; ++x)
#pragma unroll
        for (int y = 0; y < 2; ++y)
#pragma unroll
          for (int rr = 0; rr < 4; ++rr) {
            a64[t][x][y][rr] += (double)acc[t][x][y][rr];
            acc[t][x][y][rr] = 0.f;
          }
  };

  // number of steps of this workgroup
  int n_steps = 0;
  for (int sl = p; sl < n_slices; sl += P) n_steps += (int)((slices[sl].n + BP_STEP - 1) / BP_STEP);

  int si = p;                 // cursor: slice and first group of the next step to copy
  while (si < n_slices && slices[si].n <= 0) si += P;
  int64_t g0 = 0;
  auto advance = [&]() {
    g0 += BP_KG;
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
  __syncthreads();
  int buf = 0;
  for (int t = 0; t < n_steps; ++t) {
    const bool more = t + 1 < n_steps;
    const int64_t n8_left = ((slices[csi].n + 7) >> 3) - cg0;
    const int nsi = si;
    const int64_t ng0 = g0;
    if (more) issue(si, g0, buf ^ 1);
    if (wave_on) compute(buf, n8_left, ((t + 1) % BP_FLUSH) == 0 || !more);
    if (more) advance();
    __builtin_amdgcn_s_waitcnt(0);   // this wave's copies of the next step have landed
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
        const int a = bf16_d_row(lane, rr);
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
        const int row = 32 * wr + 16 * x + bf16_d_row(lane, rr);
        const int col = c0 + 16 * y + i16;
        base[row * GT + col] = a64[0][x][y][rr];
        base[GT * GT + row * GT + col] = a64[1][x][y][rr];
        if (third) base[2 * GT * GT + row * GT + col] = a64[2][x][y][rr];
      }
}

void launch_gram_bf16(const PairJob* d_pairs, int n_strip_pairs, int n_pairs, const GramJob* d_jobs,
                      const Slice* d_slices, int n_slices, int P, int pieces, double* d_partial,
                      hipStream_t st, const int2* d_sets) {
  const int n_plain = n_pairs - n_strip_pairs;
  if (pieces == 3) {
    if (n_strip_pairs > 0)
      hipLaunchKernelGGL((gram_bf16_kernel<3, true>), dim3(n_strip_pairs * P), dim3(BP_THREADS), 0, st, d_pairs,
                         n_strip_pairs, d_jobs, d_slices, n_slices, P, d_partial, d_sets);
    if (n_plain > 0)
      hipLaunchKernelGGL((gram_bf16_kernel<3, false>), dim3(n_plain * P), dim3(BP_THREADS), 0, st,
                         d_pairs + n_strip_pairs, n_plain, d_jobs, d_slices, n_slices, P, d_partial, d_sets);
  } else {
    if (n_strip_pairs > 0)
      hipLaunchKernelGGL((gram_bf16_kernel<2, true>), dim3(n_strip_pairs * P), dim3(BP_THREADS), 0, st, d_pairs,
                         n_strip_pairs, d_jobs, d_slices, n_slices, P, d_partial, d_sets);
    if (n_plain > 0)
      hipLaunchKernelGGL((gram_bf16_kernel<2, false>), dim3(n_plain * P), dim3(BP_THREADS), 0, st,
                         d_pairs + n_strip_pairs, n_plain, d_jobs, d_slices, n_slices, P, d_partial, d_sets);
  }
}

// ---------------------------------------------------------------------------
// FP64 -> BF16 split pieces, k-packed (producer-side utility)
// ---------------------------------------------------------------------------

__device__ __forceinline__ uint16_t f64_to_bf16_rn(double v) {
  // to FP32 (round to nearest), then to BF16 (round to nearest even); the
  // next piece takes the exact FP64 remainder, so the double rounding only
  // moves bits between pieces
  const uint32_t u = __float_as_uint((float)v);
  const uint32_t lsb = (u >> 16) & 1u;
  return (uint16_t)((u + 0x7FFFu + lsb) >> 16);
}

__global__ __launch_bounds__(256) void pack_bf16_kernel(const double* __restrict__ src, int64_t n,
                                                        int64_t ld_src, int64_t ncols, int pieces,
                                                        uint16_t* __restrict__ dst, int64_t ld_dst,
                                                        int64_t pstride) {
  const int64_t n8 = (n + 7) >> 3;
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= n8 * ncols) return;
  const int64_t g = t / ncols, x = t % ncols;
  uint16_t out[3][8];
#pragma unroll
  for (int e = 0; e < 8; ++e) {
    const int64_t s = 8 * g + e;
    double v = (s < n) ? src[s * ld_src + x] : 0.0;
#pragma unroll
    for (int pc = 0; pc < 3; ++pc) {
      const uint16_t h = (pc < pieces) ? f64_to_bf16_rn(v) : (uint16_t)0;
      out[pc][e] = h;
      v -= (double)__uint_as_float((uint32_t)h << 16);
    }
  }
  for (int pc = 0; pc < pieces; ++pc) {
    uint4 w;
    w.x = (uint32_t)out[pc][0] | ((uint32_t)out[pc][1] << 16);
    w.y = (uint32_t)out[pc][2] | ((uint32_t)out[pc][3] << 16);
    w.z = (uint32_t)out[pc][4] | ((uint32_t)out[pc][5] << 16);
    w.w = (uint32_t)out[pc][6] | ((uint32_t)out[pc][7] << 16);
    *reinterpret_cast<uint4*>(dst + (size_t)pc * pstride + (g * ld_dst + x) * 8) = w;
  }
}

void launch_pack_bf16(const double* src, int64_t n, int64_t ld_src, int64_t ncols, int pieces,
                      uint16_t* dst, int64_t ld_dst, int64_t pstride, hipStream_t st) {
  const int64_t n8 = (n + 7) >> 3;
  const int64_t work = n8 * ncols;
  if (work <= 0) return;
  hipLaunchKernelGGL(pack_bf16_kernel, dim3((unsigned)((work + 255) / 256)), dim3(256), 0, st, src, n,
                     ld_src, ncols, pieces, dst, ld_dst, pstride);
}

}  // namespace blm
