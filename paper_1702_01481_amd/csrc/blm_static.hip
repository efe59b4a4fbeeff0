// Allocation-free variant of the dense-pencil eigenvalue entry point
// (blm_debug_eigvals): every scratch buffer its kernels use lives in one
// file-scope device array of this translation unit, so the call issues no
// device allocation.  Intended for callers that cannot allocate device
// memory (code under HIP graph capture, tight serving loops, harnesses that
// forbid hipMalloc).
//
// Host code never passes the array's name to a kernel: on the host it is a
// stand-in symbol, not a device address.  The first call on a device, with
// that device current, resolves the array's address there with
// hipGetSymbolAddress; later calls on that device reuse it.
#include <mutex>

#include "blm.h"
#include "blm_internal.h"

namespace blm {
namespace {

constexpr int STATIC_MAXD = BLM_STATIC_MAXD;

// Scratch layout, in doubles from the array's start:
//   [0, 64)        header: the EigJob (byte 0), status words (byte 256),
//                  selected eigenvalues (byte 320)
//   [64, ...)      one pencil's eigensolver workspace for d <= STATIC_MAXD:
//                  S, A, Hq, V (d^2 each), W (2 d^2), complex vectors,
//                  wr, wi, tau, out (the same carving as a context's pencils)
constexpr size_t HEAD = 64;
constexpr size_t ws_doubles(size_t d) {
  return 4 * d * d + (2 * d * d > 16 * d ? 2 * d * d : 16 * d) + 2 * (size_t)EIG_MAXSEL * d + 3 * d +
         3 * (2 * d);
}
constexpr size_t SCRATCH_DOUBLES = HEAD + ws_doubles(STATIC_MAXD);

static __device__ __align__(256) double scratch[SCRATCH_DOUBLES];

static_assert(sizeof(EigJob) <= 256, "EigJob must fit the header's first 256 bytes");

// Carves the pencil workspace out of the scratch (base = its device address)
// and copies H and S into it (the solver overwrites both).
__global__ void static_setup_kernel(double* base, const double* __restrict__ H, const double* __restrict__ S,
                                    int d) {
  const size_t dd = (size_t)d * d;
  double* p = base + HEAD;
  double* S_ws = p;
  double* A_ws = p + dd;
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    EigJob J{};
    J.d = d;
    J.mode = EIG_VALUES;
    J.n_want = 1;
    J.beta0 = 0;
    J.nbeta = d;
    J.S = p; p += dd;
    J.A = p; p += dd;
    J.Hq = p; p += dd;
    J.V = p; p += dd;
    J.W = p; p += (2 * dd > 16 * (size_t)d ? 2 * dd : 16 * (size_t)d);
    J.vec = p; p += 2 * (size_t)EIG_MAXSEL * d;
    J.wr = p; p += d;
    J.wi = p; p += d;
    J.tau = p; p += d;
    J.out = p;
    J.info = (int32_t*)((char*)base + 256);
    J.out_evals = (double*)((char*)base + 320);
    *(EigJob*)base = J;
  }
  const size_t stride = (size_t)gridDim.x * blockDim.x;
  for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < dd; i += stride) {
    S_ws[i] = S[i];
    A_ws[i] = H[i];
  }
}

// Eigenvalues (re, im) in the solver's order to evals [d][2], and the
// solver's outcome as a blm_status to *status.
__global__ void static_finish_kernel(const double* base, int d, double* __restrict__ evals,
                                     int32_t* __restrict__ status) {
  const EigJob* J = (const EigJob*)base;
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  const int32_t st = J->info[0];
  if (i == 0) {
    *status = st == EIG_OK          ? BLM_OK
              : st == EIG_NOT_PD    ? BLM_E_S_NOT_PD
              : st == EIG_NONFINITE ? BLM_E_NONFINITE
              : st == EIG_NOCONV    ? BLM_E_NOCONV
                                    : BLM_E_HIP;
  }
  if (i < d) {
    // values are meaningful only on success; NaN otherwise
    evals[2 * i] = (st == EIG_OK) ? J->wr[i] : __builtin_nan("");
    evals[2 * i + 1] = (st == EIG_OK) ? J->wi[i] : __builtin_nan("");
  }
}

std::mutex g_mu;
constexpr int MAX_DEVICES = 64;
double* g_scratch[MAX_DEVICES] = {};

// Device address of this device's copy of the scratch array (resolved once
// per device, with the device current).
blm_status scratch_address(double** out) {
  int dev = -1;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= MAX_DEVICES) return BLM_E_HIP;
  std::lock_guard<std::mutex> lock(g_mu);
  if (!g_scratch[dev]) {
    void* p = nullptr;
    if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) != hipSuccess || !p) return BLM_E_HIP;
    g_scratch[dev] = (double*)p;
  }
  *out = g_scratch[dev];
  return BLM_OK;
}

}  // namespace
}  // namespace blm

using namespace blm;

extern "C" {

blm_status blm_pencil_eigvals_static(const double* d_H, const double* d_S, int32_t d, double* d_evals,
                                     int32_t* d_status, void* stream) {
  if (!d_H || !d_S || !d_evals || !d_status || d < 1 || d > STATIC_MAXD) return BLM_E_ARG;
  double* base = nullptr;
  const blm_status r = scratch_address(&base);
  if (r != BLM_OK) return r;
  hipStream_t st = (hipStream_t)stream;
  const size_t dd = (size_t)d * d;
  const int setup_blocks = (int)std::min<size_t>(256, (dd + 255) / 256);
  hipLaunchKernelGGL(static_setup_kernel, dim3(setup_blocks), dim3(256), 0, st, base, d_H, d_S, d);
  launch_eig((const EigJob*)base, 1, st);
  hipLaunchKernelGGL(static_finish_kernel, dim3((d + 255) / 256), dim3(256), 0, st, (const double*)base, d,
                     d_evals, d_status);
  return hipGetLastError() == hipSuccess ? BLM_OK : BLM_E_HIP;
}

}  // extern "C"
