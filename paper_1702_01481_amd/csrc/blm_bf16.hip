// Mixed-precision block build on the BF16 matrix cores of gfx950.
//
// Every sample value x is stored as BF16 pieces x = hi + mid + lo (or
// hi + lo) whose FP64 sum is exact.  A product x*y is taken as the sum of the
// piece products of total order <= pieces - 1 (hi*hi, hi*mid, mid*hi, hi*lo,
// lo*hi, mid*mid for three pieces; hi*hi, hi*lo, lo*hi for two), each on
// v_mfma_f32_16x16x32_bf16 (exact products, FP32 sums).  FP32 accumulators
// are added into FP64 registers after every 32 samples, and the slices are summed
// in FP64 by the same fixed-order reduction as the FP64 path.  These are the
// block estimates of Eq. 3 on the one-block basis (Eq. 4 / Eq. 10); the
// columns of the wave function itself and of the previous directions stay
// in FP64 (strip jobs of the FP64 kernel).
//
// Storage ("k-packed"): element (s, x) of piece p is at
// base + p * pstride + ((s / 8) * ld + x) * 8 + s % 8.  A lane's matrix-core
// operand (8 consecutive samples of one parameter) is one 16-byte load.
#include "blm_internal.h"

namespace blm {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f4 __attribute__((ext_vector_type(4)));
typedef double d4b __attribute__((ext_vector_type(4)));

// FP32 accumulators are added into FP64 after every 32-sample step: each
// FP32 partial then holds one step's sum, which keeps the block estimates
// within about 2e-8 of FP64 (flushing every 256 samples gave 6e-8, and the
// block eigenvectors amplify that into 2e-6 of the energy).

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

// Each wave loads its own operands straight from HBM/L2 (the k-packed
// layout makes every operand one 16-byte load per lane); wave (wr, wc) owns
// rows 32 wr .. +31 and columns 32 wc .. +31 of each product.  (A variant
// that staged the panels in LDS for all 8 waves of a tile ran slower: one
// workgroup per CU left the loads' latency exposed.)
template <int PIECES>
__global__ __launch_bounds__(GTHREADS, 2) void gram_bf16_kernel(const GramJob* __restrict__ jobs,
                                                                int n_jobs,
                                                                const Slice* __restrict__ slices,
                                                                int n_slices, int P,
                                                                double* __restrict__ partial) {
  const int G = gridDim.x, g = blockIdx.x;
  const int q = G >> 3, r = G & 7, xcd = g & 7, idx = g >> 3;
  const int wid = (xcd < r) ? xcd * (q + 1) + idx : r * (q + 1) + (xcd - r) * q + idx;
  const int p = wid / n_jobs, jid = wid % n_jobs;
  const GramJob J = jobs[jid];
  const bool off = (J.kind == JOB_OFF);

  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  const int wr = wv >> 1, wc = wv & 1;
  const int i16 = lane & 15, g4 = lane >> 4;
  int ca[2], cb[2];
  bool va[2], vb[2];
#pragma unroll
  for (int x = 0; x < 2; ++x) {
    ca[x] = 32 * wr + 16 * x + i16;
    cb[x] = 32 * wc + 16 * x + i16;
    va[x] = ca[x] < J.mi;
    vb[x] = cb[x] < J.nj;
  }

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
  for (int si = p; si < n_slices; si += P) {
    const Slice S = slices[si];
    const BLM_GLOBAL uint16_t* O = as_global((const uint16_t*)S.O);
    const BLM_GLOBAL uint16_t* E = as_global((const uint16_t*)S.e);
    const int64_t n8 = (S.n + 7) >> 3;
    for (int64_t g0 = 0; g0 < n8; g0 += 4) {
      const int64_t gg = g0 + g4;
      const bool gv = gg < n8;
      bf16x8 bO[2][PIECES], bE[2][PIECES];
#pragma unroll
      for (int pc = 0; pc < PIECES; ++pc)
#pragma unroll
        for (int y = 0; y < 2; ++y) {
          const int64_t o = (size_t)pc * S.pstride + (gg * S.ld + J.cj + cb[y]) * 8;
          bO[y][pc] = load_frag(O + o, gv && vb[y]);
          bE[y][pc] = load_frag(E + o, gv && vb[y]);
        }
#pragma unroll
      for (int pa = 0; pa < PIECES; ++pa) {
        bf16x8 aO[2], aE[2];
#pragma unroll
        for (int x = 0; x < 2; ++x) {
          const int64_t o = (size_t)pa * S.pstride + (gg * S.ld + J.ci + ca[x]) * 8;
          aO[x] = load_frag(O + o, gv && va[x]);
          aE[x] = load_frag(E + o, gv && va[x] && off);
        }
#pragma unroll
        for (int pb = 0; pb + pa < PIECES; ++pb)
#pragma unroll
          for (int x = 0; x < 2; ++x)
#pragma unroll
            for (int y = 0; y < 2; ++y) {
              acc[0][x][y] = mfma_bf16(aO[x], bO[y][pb], acc[0][x][y]);
              acc[1][x][y] = mfma_bf16(aO[x], bE[y][pb], acc[1][x][y]);
              if (off) acc[2][x][y] = mfma_bf16(aE[x], bO[y][pb], acc[2][x][y]);
            }
      }
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
    }
  }

  BLM_GLOBAL double* base = as_global(partial) + ((size_t)jid * P + p) * (size_t)(3 * GT * GT);
#pragma unroll
  for (int x = 0; x < 2; ++x)
#pragma unroll
    for (int y = 0; y < 2; ++y)
#pragma unroll
      for (int rr = 0; rr < 4; ++rr) {
        const int row = 32 * wr + 16 * x + bf16_d_row(lane, rr);
        const int col = 32 * wc + 16 * y + i16;
        base[row * GT + col] = a64[0][x][y][rr];
        base[GT * GT + row * GT + col] = a64[1][x][y][rr];
        if (off) base[2 * GT * GT + row * GT + col] = a64[2][x][y][rr];
      }
}

void launch_gram_bf16(const GramJob* d_jobs, int n_jobs, const Slice* d_slices, int n_slices, int P,
                      int pieces, double* d_partial, hipStream_t st) {
  if (n_jobs <= 0) return;
  if (pieces == 3)
    hipLaunchKernelGGL(gram_bf16_kernel<3>, dim3(n_jobs * P), dim3(GTHREADS), 0, st, d_jobs, n_jobs,
                       d_slices, n_slices, P, d_partial);
  else
    hipLaunchKernelGGL(gram_bf16_kernel<2>, dim3(n_jobs * P), dim3(GTHREADS), 0, st, d_jobs, n_jobs,
                       d_slices, n_slices, P, d_partial);
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
