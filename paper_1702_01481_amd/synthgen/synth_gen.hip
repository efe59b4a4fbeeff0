// libsynthgen: on-device generator of the synthetic Monte Carlo samples of
// the banded-G model (input generator only; it holds none of the blocked
// linear method's arithmetic and is not part of libblm):
//
//   O_s   = mu + L z_s + 0.1 xi_s
//   E_L,s = -10 + a . (O_s - mu) + sigma_E eps_s
//   e_s   = E_L,s O_s + G (O_s - mu) + 0.05 eta_s,   G symmetric, G_ij = 0 for |i - j| > band
//
// with z, xi, eps, eta standard normal.  Random bits come from SplitMix64
// (Steele, Lea and Flood, "Fast splittable pseudorandom number generators",
// OOPSLA 2014) used as a counter-based generator: draw n of a seed is the
// SplitMix64 output mix(seed + (n + 1) gamma), so every draw is addressed by
// (quantity, chunk, sample, column) and any chunk can be made on its own, in
// any order, with the same bytes every time.  Normals come from the
// Box-Muller transform (Box and Muller, 1958) of two 24-bit uniforms, in
// single precision with the hardware's fast log, sine and cosine.
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace {

constexpr int TPB = 256;        // threads per workgroup: one column each
constexpr int SG = 128;         // samples per workgroup
constexpr int ESTAGE = 8;       // samples per LDS stage of the e kernel

// quantity ids (the counter's top bits)
enum : uint64_t { Q_Z = 1, Q_XI = 2, Q_EPS = 3, Q_ETA = 4 };

// counter of a draw: quantity (4 bits), chunk, sample, column (20 bits each)
__device__ __forceinline__ uint64_t counter(uint64_t q, uint64_t chunk, uint64_t s, uint64_t col) {
  return (q << 60) | ((chunk & 0xFFFFF) << 40) | ((s & 0xFFFFF) << 20) | (col & 0xFFFFF);
}

// SplitMix64 output number n of `seed`
__device__ __forceinline__ uint64_t splitmix(uint64_t seed, uint64_t n) {
  uint64_t z = seed + (n + 1) * 0x9E3779B97F4A7C15ull;
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}

// Two standard normals from 64 random bits.
__device__ __forceinline__ void normals2(uint64_t x, double& n0, double& n1) {
  const float s = 5.9604644775390625e-08f;  // 2^-24
  const float u1 = ((float)(uint32_t)(x >> 40) + 1.0f) * s;            // (0, 1]
  const float u2 = (float)(uint32_t)((x >> 16) & 0xFFFFFFu) * s;       // [0, 1)
  const float r = sqrtf(-2.0f * __logf(u1));
  float sn, cs;
  __sincosf(6.283185307179586f * (u2 - 0.5f), &sn, &cs);
  n0 = (double)(r * cs);
  n1 = (double)(r * sn);
}

// O = mu + L z + 0.1 xi for a 256-column x 128-sample tile; part[s][tile] =
// sum over the tile's columns of a_j (O_sj - mu_j).
template <int R>
__global__ __launch_bounds__(TPB, 4) void gen_O_kernel(int64_t n, int64_t nv, const double* __restrict__ L,
                                                    const double* __restrict__ mu, const double* __restrict__ a,
                                                    uint64_t seed, int64_t chunk, double* __restrict__ O, int64_t ld,
                                                    double* __restrict__ part, int n_tiles) {
  __shared__ double zs[SG][R];
  __shared__ double red[TPB / 64][SG];
  const int tid = threadIdx.x, tile = blockIdx.x;
  const int64_t s0 = (int64_t)blockIdx.y * SG;
  const int64_t j = (int64_t)tile * TPB + tid;
  const bool col_ok = j < nv;
  // z of the group's samples: R normals per sample, 2 per draw
  for (int t = tid; t < SG * R / 2; t += TPB) {
    const int sl = t / (R / 2), q2 = t % (R / 2);
    double v0, v1;
    normals2(splitmix(seed, counter(Q_Z, chunk, s0 + sl, q2)), v0, v1);
    zs[sl][2 * q2] = v0;
    zs[sl][2 * q2 + 1] = v1;
  }
  double Lj[R];
#pragma unroll
  for (int k = 0; k < R; ++k) Lj[k] = col_ok ? L[j * R + k] : 0.0;
  const double muj = col_ok ? mu[j] : 0.0, aj = col_ok ? a[j] : 0.0;
  __syncthreads();
  for (int sl = 0; sl < SG; sl += 2) {
    double xi[2];
    normals2(splitmix(seed, counter(Q_XI, chunk, s0 + sl, j)), xi[0], xi[1]);   // samples s0+sl, +1
#pragma unroll
    for (int u = 0; u < 2; ++u) {
      const int64_t s = s0 + sl + u;
      double lz = 0.0;
#pragma unroll
      for (int k = 0; k < R; ++k) lz = fma(Lj[k], zs[sl + u][k], lz);
      const double dO = lz + 0.1 * xi[u];
      if (col_ok && s < n) O[s * ld + j] = muj + dO;
      // partial of a . (O_s - mu) over this wave's columns
      double pr = col_ok ? aj * dO : 0.0;
#pragma unroll
      for (int off = 32; off >= 1; off >>= 1) pr += __shfl_xor(pr, off);
      if ((tid & 63) == 0) red[tid >> 6][sl + u] = pr;
    }
  }
  __syncthreads();
  if (tid < SG && s0 + tid < n) {
    double t = 0.0;
#pragma unroll
    for (int w = 0; w < TPB / 64; ++w) t += red[w][tid];
    part[(s0 + tid) * n_tiles + tile] = t;
  }
}

// E_L,s = -10 + sum_tiles part[s][tile] + sigma_E eps_s
__global__ void gen_EL_kernel(int64_t n, const double* __restrict__ part, int n_tiles, double sigma_E, uint64_t seed,
                              int64_t chunk, double* __restrict__ EL) {
  const int64_t s2 = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) * 2;
  if (s2 >= n) return;
  double eps[2];
  normals2(splitmix(seed, counter(Q_EPS, chunk, s2, 0)), eps[0], eps[1]);
  for (int u = 0; u < 2 && s2 + u < n; ++u) {
    double t = 0.0;
    for (int k = 0; k < n_tiles; ++k) t += part[(s2 + u) * n_tiles + k];
    EL[s2 + u] = -10.0 + t + sigma_E * eps[u];
  }
}

// e_s,i = E_L,s O_s,i + sum_{|k| <= B} G_{i,i+k} (O_s,i+k - mu_i+k) + 0.05 eta_s,i
// gband[i][B + k] = G_{i,i+k} (zero where i + k is outside the parameters).
template <int B>
__global__ __launch_bounds__(TPB, 4) void gen_e_kernel(int64_t n, int64_t nv, const double* __restrict__ gband,
                                                    const double* __restrict__ mu, const double* __restrict__ EL,
                                                    const double* __restrict__ O, int64_t ld, uint64_t seed,
                                                    int64_t chunk, double* __restrict__ e) {
  constexpr int NB = 2 * B + 1, W = TPB + 2 * B;
  __shared__ double sd[ESTAGE][W];
  const int tid = threadIdx.x, tile = blockIdx.x;
  const int64_t s0 = (int64_t)blockIdx.y * SG;
  const int64_t c0 = (int64_t)tile * TPB;
  const int64_t i = c0 + tid;
  const bool col_ok = i < nv;
  double g[NB];
#pragma unroll
  for (int k = 0; k < NB; ++k) g[k] = col_ok ? gband[i * NB + k] : 0.0;
  for (int st = 0; st < SG; st += ESTAGE) {
    __syncthreads();
    // O - mu of the stage's samples over columns [c0 - B, c0 + TPB + B)
#pragma unroll 1
    for (int sl = 0; sl < ESTAGE; ++sl) {
      const int64_t s = s0 + st + sl;
      for (int cl = tid; cl < W; cl += TPB) {
        const int64_t col = c0 - B + cl;
        double v = 0.0;
        if (s < n && col >= 0 && col < nv) v = O[s * ld + col] - mu[col];
        sd[sl][cl] = v;
      }
    }
    __syncthreads();
    for (int sl = 0; sl < ESTAGE; sl += 2) {
      double eta[2];
      normals2(splitmix(seed, counter(Q_ETA, chunk, s0 + st + sl, i)), eta[0], eta[1]);
#pragma unroll
      for (int u = 0; u < 2; ++u) {
        const int64_t s = s0 + st + sl + u;
        double acc = 0.0;
#pragma unroll
        for (int k = 0; k < NB; ++k) acc = fma(g[k], sd[sl + u][tid + k], acc);
        if (col_ok && s < n) e[s * ld + i] = EL[s] * O[s * ld + i] + acc + 0.05 * eta[u];
      }
    }
  }
}

template <int R>
void launch_O(dim3 grid, hipStream_t st, int64_t n, int64_t nv, const double* L, const double* mu, const double* a,
              uint64_t seed, int64_t chunk, double* O, int64_t ld, double* part, int n_tiles) {
  hipLaunchKernelGGL(gen_O_kernel<R>, grid, dim3(TPB), 0, st, n, nv, L, mu, a, seed, chunk, O, ld, part, n_tiles);
}

template <int B>
void launch_e(dim3 grid, hipStream_t st, int64_t n, int64_t nv, const double* gband, const double* mu,
              const double* EL, const double* O, int64_t ld, uint64_t seed, int64_t chunk, double* e) {
  hipLaunchKernelGGL(gen_e_kernel<B>, grid, dim3(TPB), 0, st, n, nv, gband, mu, EL, O, ld, seed, chunk, e);
}

}  // namespace

extern "C" {

// One chunk of n samples (1 <= n < 2^20; chunk < 2^20) of the banded-G
// model, all pointers device memory: L [nv][r] (r in {8, 16, 32, 64}),
// mu [nv], a [nv], gband [nv][2 band + 1] (band 4 or 8), outputs
// O, e [n][ld] (ld >= nv, nv < 2^20), EL [n], and a scratch `part` of
// n * ceil(nv / 256) doubles.  Asynchronous on stream.  Returns 0, or 1 for
// a bad argument, 2 for a launch error.
int synth_gen_banded_chunk(int64_t n, int64_t nv, int32_t r, const double* L, const double* mu, const double* a,
                           int32_t band, const double* gband, double sigma_E, uint64_t seed, int64_t chunk, double* O,
                           double* e, int64_t ld, double* EL, double* part, void* stream) {
  const bool r_ok = r == 8 || r == 16 || r == 32 || r == 64;
  const bool b_ok = band == 4 || band == 8;
  if (n < 1 || n >= (1 << 20) || nv < 1 || nv >= (1 << 20) || chunk < 0 || chunk >= (1 << 20) || !r_ok || !b_ok ||
      ld < nv || !L || !mu || !a || !gband || !O || !e || !EL || !part)
    return 1;
  hipStream_t st = (hipStream_t)stream;
  const int n_tiles = (int)((nv + TPB - 1) / TPB);
  const dim3 grid(n_tiles, (unsigned)((n + SG - 1) / SG));
  switch (r) {
    case 8: launch_O<8>(grid, st, n, nv, L, mu, a, seed, chunk, O, ld, part, n_tiles); break;
    case 16: launch_O<16>(grid, st, n, nv, L, mu, a, seed, chunk, O, ld, part, n_tiles); break;
    case 32: launch_O<32>(grid, st, n, nv, L, mu, a, seed, chunk, O, ld, part, n_tiles); break;
    default: launch_O<64>(grid, st, n, nv, L, mu, a, seed, chunk, O, ld, part, n_tiles); break;
  }
  hipLaunchKernelGGL(gen_EL_kernel, dim3((unsigned)((n + 2 * 256 - 1) / (2 * 256))), dim3(256), 0, st, n, part,
                     n_tiles, sigma_E, seed, chunk, EL);
  if (band == 4) launch_e<4>(grid, st, n, nv, gband, mu, EL, O, ld, seed, chunk, e);
  else launch_e<8>(grid, st, n, nv, gband, mu, EL, O, ld, seed, chunk, e);
  return hipGetLastError() == hipSuccess ? 0 : 2;
}

}  // extern "C"
