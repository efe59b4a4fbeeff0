"""Seeded synthetic Monte Carlo sample data shaped like the workloads of the
blocked linear method (BLM) paper, Zhao & Neuscamman, arXiv:1702.01481.

This module only draws random numbers.  It holds none of the method's
arithmetic (no overlap or Hamiltonian estimates, no eigensolves), so it can
feed both the CPU oracle and the HIP path with the same bytes.

Per-sample quantities (the derivative ratios of Eq. 3 of the paper) follow a
low-rank Gaussian model:

    O_s   = mu + L z_s + 0.1 xi_s                      mu ~ N(0, 0.1^2), L_ij ~ N(0, 0.3^2)
    E_L,s = -10 + a . (O_s - mu) + sigma_E eps_s       a ~ N(0, 0.2^2)
    e_s   = E_L,s O_s + G (O_s - mu) + 0.05 eta_s      G symmetric, G_ij ~ N(0, 0.1^2)

with z, xi, eps, eta standard normal.  G is dense, or banded (G_ij = 0 for
|i - j| > band) for the 30,000-parameter workload, whose dense G(O - mu)
term would cost 2 N_s N_V^2 flop per pass (7.2 PFLOP at 4M samples, far more
than the method's own work); the banded model is made on the device by a
fused generator (synthgen/libsynthgen.so: SplitMix64 counters, Box-Muller
normals), chunk by chunk, as fast as it is consumed.  Model parameters are drawn once per
seed; the sample draws of chunk c come from a generator seeded by
(seed, c), so any chunk can be regenerated on its own, in any order, on the
CPU or on a GPU.  CPU and GPU draws differ (torch's CPU and device
generators are different streams); a comparison always hands both sides the
same bytes.
"""
from __future__ import annotations

import dataclasses
import math
from typing import List, Optional, Sequence, Tuple

import numpy as np
import torch

# stream ids for the independent quantities of one seed
_S_MU, _S_L, _S_A, _S_G, _S_BLOCKS, _S_OLD, _S_W = 1, 2, 3, 4, 5, 6, 7
_S_CHUNK0 = 1 << 20


def _seed_of(seed: int, stream: int) -> int:
    # splitmix64 finaliser of (seed, stream): well-separated 63-bit seeds
    x = (seed * 0x9E3779B97F4A7C15 + stream * 0xBF58476D1CE4E5B9 + 0x94D049BB133111EB) & ((1 << 64) - 1)
    x ^= x >> 30
    x = (x * 0xBF58476D1CE4E5B9) & ((1 << 64) - 1)
    x ^= x >> 27
    x = (x * 0x94D049BB133111EB) & ((1 << 64) - 1)
    x ^= x >> 31
    return x & ((1 << 63) - 1)


def _gen(device, seed: int, stream: int) -> torch.Generator:
    g = torch.Generator(device=device)
    g.manual_seed(_seed_of(seed, stream))
    return g


# ----------------------------------------------------------------------------
# workloads
# ----------------------------------------------------------------------------

@dataclasses.dataclass
class Workload:
    """One synthetic optimization problem: sizes, partition and BLM knobs."""
    name: str
    n_params: int
    block_offsets: np.ndarray          # int64 [N_B + 1], contiguous, ascending
    n_samples: int
    chunk: int                          # samples per chunk (last chunk may be shorter)
    rank: int                           # rank of L
    n_keep: int                         # N_K
    n_old: int                          # N_O
    shifts: Tuple[float, ...]
    sigma_E: float = 0.5
    seed: int = 0
    band: Optional[int] = None          # half-bandwidth of G (None: dense)

    @property
    def n_blocks(self) -> int:
        return len(self.block_offsets) - 1

    def chunk_sizes(self) -> List[int]:
        full, tail = divmod(self.n_samples, self.chunk)
        return [self.chunk] * full + ([tail] if tail else [])

    def generator(self, device="cpu") -> "SampleGenerator":
        """The sample generator of this workload (its model, seed and G)."""
        return SampleGenerator(self.n_params, self.rank, self.seed, sigma_E=self.sigma_E, device=device,
                               band=self.band)


def uniform_offsets(n_params: int, n_blocks: int) -> np.ndarray:
    """Contiguous blocks of (nearly) equal size."""
    base, rem = divmod(n_params, n_blocks)
    sizes = [base + (1 if b < rem else 0) for b in range(n_blocks)]
    return np.concatenate([[0], np.cumsum(sizes)]).astype(np.int64)


def loguniform_offsets(n_params: int, n_blocks: int, lo: float, hi: float, seed: int) -> np.ndarray:
    """Block sizes drawn log-uniform in [lo, hi], rescaled to sum to n_params,
    floored, with the remainder given to the largest fractional parts; kept in
    draw order."""
    g = _gen("cpu", seed, _S_BLOCKS)
    u = torch.rand(n_blocks, generator=g, dtype=torch.float64).numpy()
    raw = np.exp(math.log(lo) + u * (math.log(hi) - math.log(lo)))
    scaled = raw * (n_params / raw.sum())
    sizes = np.floor(scaled).astype(np.int64)
    rem = n_params - int(sizes.sum())
    order = np.argsort(-(scaled - sizes), kind="stable")
    sizes[order[:rem]] += 1
    return np.concatenate([[0], np.cumsum(sizes)]).astype(np.int64)


def uniform_int_offsets(n_params: int, lo: int, hi: int, seed: int) -> np.ndarray:
    """Block sizes drawn as uniform integers in [lo, hi] until n_params is
    covered; the last block takes what is left, and a remainder below lo is
    merged into the block before it."""
    g = _gen("cpu", seed, _S_BLOCKS)
    sizes: List[int] = []
    left = n_params
    while left > 0:
        s = min(int(torch.randint(lo, hi + 1, (1,), generator=g).item()), left)
        sizes.append(s)
        left -= s
    if len(sizes) > 1 and sizes[-1] < lo:
        last = sizes.pop()
        sizes[-1] += last
    return np.concatenate([[0], np.cumsum(sizes)]).astype(np.int64)


UNEVEN_BAND = 8      # half-bandwidth of G in the 30,000-parameter workload

BATCH_SIZES = (2_000, 4_000, 6_000, 8_000, 10_000, 12_000, 16_000, 20_000)


def batched_workloads(seed: int = 0, n_samples: int = 1_000_000) -> List[Workload]:
    """Eight independent optimizations solved together: N_V from 2,000 to
    20,000 (78,000 parameters in all), blocks drawn as uniform integers in
    [500, 1,500], n_samples each (1,000,000 at full size) in 65,536-sample
    chunks, rank 32, N_K=4, N_O=0, delta=1e-3; problem p draws from seed + p."""
    return [Workload(f"batch{p}_{n}x{n_samples}", n, uniform_int_offsets(n, 500, 1500, seed + p), n_samples,
                     65_536, 32, 4, 0, (1e-3,), seed=seed + p)
            for p, n in enumerate(BATCH_SIZES)]


def workload(name: str, seed: int = 0) -> Workload:
    """The four single-problem synthetic workloads (sizes of the paper's
    problems and beyond; batched_workloads gives the eight-problem one).

    small     N_V=200 in 4x50, N_s=20,000 (one chunk), rank 8, N_K=3, delta=1e-3
    fp64      N_V=4,096 in 8x512, N_s=1,000,000 in 65,536-sample chunks, rank 32,
              N_K=5, N_O=1, delta in {1e-4, 1e-3, 1e-2}
    bf16      N_V=16,384 in 16x1,024, N_s=4,000,000, rank 64, N_K=5, N_O=1
    uneven    N_V=30,000 in 40 log-uniform blocks in [100, 2,000], N_s=4,000,000,
              rank 32, N_K=4, N_O=0, delta=1e-3; G banded (half-bandwidth 8)
    """
    if name == "small":
        return Workload("small_200x20k", 200, uniform_offsets(200, 4), 20_000, 65_536, 8, 3, 0,
                        (1e-3,), seed=seed)
    if name == "fp64":
        return Workload("fp64_4096x1M", 4096, uniform_offsets(4096, 8), 1_000_000, 65_536, 32, 5, 1,
                        (1e-4, 1e-3, 1e-2), seed=seed)
    if name == "bf16":
        return Workload("bf16_16384x4M", 16384, uniform_offsets(16384, 16), 4_000_000, 65_536, 64, 5, 1,
                        (1e-4, 1e-3, 1e-2), seed=seed)
    if name == "uneven":
        return Workload("uneven_30000x4M", 30000, loguniform_offsets(30000, 40, 100.0, 2000.0, seed),
                        4_000_000, 65_536, 32, 4, 0, (1e-3,), seed=seed, band=UNEVEN_BAND)
    raise KeyError(name)


# ----------------------------------------------------------------------------
# generator
# ----------------------------------------------------------------------------

class SampleGenerator:
    """Draws the model parameters (mu, L, a, G) once, then chunks on demand.

    band=None: dense G, everything drawn with torch generators on `device`.
    band=b: G banded with half-bandwidth b.  The model parameters are drawn
    on the CPU (the same values for every device) and the chunks are made
    by the fused generator on a GPU, or by plain torch operations on the CPU
    (other random streams: a comparison always hands both sides the same
    bytes)."""

    def __init__(self, n_params: int, rank: int, seed: int = 0, sigma_E: float = 0.5,
                 device: str | torch.device = "cpu", band: Optional[int] = None):
        self.n_params, self.rank, self.seed, self.sigma_E = n_params, rank, seed, sigma_E
        self.device = torch.device(device)
        self.band = band
        f64 = torch.float64
        n = n_params
        if band is not None:
            cpu = "cpu"
            self.mu = (0.1 * torch.randn(n, generator=_gen(cpu, seed, _S_MU), dtype=f64)).to(self.device)
            self.L = (0.3 * torch.randn(n, rank, generator=_gen(cpu, seed, _S_L), dtype=f64)).to(self.device)
            self.a = (0.2 * torch.randn(n, generator=_gen(cpu, seed, _S_A), dtype=f64)).to(self.device)
            self.gband = banded_G(n, band, seed).to(self.device)
            self.G = None
            self._part = None
            return
        dev = self.device
        self.mu = 0.1 * torch.randn(n, generator=_gen(dev, seed, _S_MU), dtype=f64, device=dev)
        self.L = 0.3 * torch.randn(n, rank, generator=_gen(dev, seed, _S_L), dtype=f64, device=dev)
        self.a = 0.2 * torch.randn(n, generator=_gen(dev, seed, _S_A), dtype=f64, device=dev)
        g = 0.1 * torch.randn(n, n, generator=_gen(dev, seed, _S_G), dtype=f64, device=dev)
        # symmetric: upper triangle (with diagonal) mirrored
        up = torch.triu(g)
        self.G = up + torch.triu(g, 1).transpose(0, 1)
        del g, up

    def chunk(self, index: int, n_rows: int, out_O: Optional[torch.Tensor] = None,
              out_e: Optional[torch.Tensor] = None, out_EL: Optional[torch.Tensor] = None):
        """Samples of chunk `index`: O [n_rows][N_V], e [n_rows][N_V], E_L [n_rows]
        (written into out_* when given: contiguous rows of N_V, or views with
        unit column stride)."""
        if self.band is not None:
            if self.device.type == "cuda":
                return self._chunk_banded_device(index, n_rows, out_O, out_e, out_EL)
            return self._chunk_banded_cpu(index, n_rows, out_O, out_e, out_EL)
        dev, f64 = self.device, torch.float64
        g = _gen(dev, self.seed, _S_CHUNK0 + index)
        n = self.n_params
        z = torch.randn(n_rows, self.rank, generator=g, dtype=f64, device=dev)
        dO = z @ self.L.T
        del z
        dO.add_(torch.randn(n_rows, n, generator=g, dtype=f64, device=dev), alpha=0.1)
        eps = torch.randn(n_rows, generator=g, dtype=f64, device=dev)
        EL = -10.0 + dO @ self.a + self.sigma_E * eps
        if out_EL is not None:
            out_EL.copy_(EL)
            EL = out_EL
        O = out_O if out_O is not None else torch.empty(n_rows, n, dtype=f64, device=dev)
        torch.add(dO, self.mu, out=O)
        e = out_e if out_e is not None else torch.empty(n_rows, n, dtype=f64, device=dev)
        torch.matmul(dO, self.G, out=e)          # G symmetric: rows of (O-mu) G = G (O-mu)
        del dO
        e.addcmul_(EL[:, None], O)
        e.add_(torch.randn(n_rows, n, generator=g, dtype=f64, device=dev), alpha=0.05)
        return O, e, EL

    def _chunk_banded_cpu(self, index, n_rows, out_O, out_e, out_EL):
        f64 = torch.float64
        g = _gen("cpu", self.seed, _S_CHUNK0 + index)
        n = self.n_params
        z = torch.randn(n_rows, self.rank, generator=g, dtype=f64)
        dO = z @ self.L.T
        dO.add_(torch.randn(n_rows, n, generator=g, dtype=f64), alpha=0.1)
        EL = -10.0 + dO @ self.a + self.sigma_E * torch.randn(n_rows, generator=g, dtype=f64)
        O = dO + self.mu
        e = EL[:, None] * O + band_matvec(self.gband, dO)
        e.add_(torch.randn(n_rows, n, generator=g, dtype=f64), alpha=0.05)
        if out_O is not None:
            out_O.copy_(O)
            O = out_O
        if out_e is not None:
            out_e.copy_(e)
            e = out_e
        if out_EL is not None:
            out_EL.copy_(EL)
            EL = out_EL
        return O, e, EL

    def _chunk_banded_device(self, index, n_rows, out_O, out_e, out_EL):
        import ctypes as C
        dev, f64 = self.device, torch.float64
        n = self.n_params
        O = out_O if out_O is not None else torch.empty(n_rows, n, dtype=f64, device=dev)
        e = out_e if out_e is not None else torch.empty(n_rows, n, dtype=f64, device=dev)
        EL = out_EL if out_EL is not None else torch.empty(n_rows, dtype=f64, device=dev)
        for t, name in ((O, "O"), (e, "e")):
            if t.shape[0] < n_rows or t.shape[1] < n or t.stride(1) != 1 or t.dtype != f64:
                raise ValueError(f"{name} must be float64 [>= {n_rows}][>= {n}] with unit column stride")
        if O.stride(0) != e.stride(0):
            raise ValueError("O and e must share their row stride")
        n_tiles = (n + 255) // 256
        if self._part is None or self._part.numel() < n_rows * n_tiles:
            self._part = torch.empty(n_rows * n_tiles, dtype=f64, device=dev)
        st = torch.cuda.current_stream(dev).cuda_stream
        r = _synthgen().synth_gen_banded_chunk(
            n_rows, n, self.rank, C.c_void_p(self.L.data_ptr()), C.c_void_p(self.mu.data_ptr()),
            C.c_void_p(self.a.data_ptr()), self.band, C.c_void_p(self.gband.data_ptr()), float(self.sigma_E),
            C.c_uint64(_seed_of(self.seed, _S_CHUNK0)), int(index), C.c_void_p(O.data_ptr()),
            C.c_void_p(e.data_ptr()), O.stride(0), C.c_void_p(EL.data_ptr()), C.c_void_p(self._part.data_ptr()),
            C.c_void_p(st))
        if r != 0:
            raise RuntimeError(f"synth_gen_banded_chunk failed ({r})")
        return O, e, EL


def banded_G(n: int, band: int, seed: int) -> torch.Tensor:
    """Symmetric banded G as its diagonals: gband[i][band + k] = G_{i,i+k} for
    |k| <= band (zero where i + k falls outside 0..n-1); G_{i,i+k} = G_{i+k,i}
    ~ N(0, 0.1^2), drawn once per diagonal k >= 0 and mirrored."""
    g = _gen("cpu", seed, _S_G)
    gb = torch.zeros(n, 2 * band + 1, dtype=torch.float64)
    for k in range(0, band + 1):
        if k >= n:
            break
        d = 0.1 * torch.randn(n - k, generator=g, dtype=torch.float64)
        gb[: n - k, band + k] = d          # G_{i, i+k}
        if k:
            gb[k:, band - k] = d           # G_{i, i-k} = G_{i-k, i}
    return gb


def band_matvec(gband: torch.Tensor, X: torch.Tensor) -> torch.Tensor:
    """Rows of X times the banded G (plain torch, for the CPU generator):
    out[s, i] = sum_k gband[i, band + k] X[s, i + k]."""
    n = X.shape[1]
    band = (gband.shape[1] - 1) // 2
    out = torch.zeros_like(X)
    for k in range(-band, band + 1):
        if abs(k) >= n:
            continue
        lo, hi = max(0, -k), min(n, n - k)      # columns i with 0 <= i + k < n
        out[:, lo:hi] += gband[lo:hi, band + k] * X[:, lo + k:hi + k]
    return out


_synthgen_lib = None


def _synthgen():
    """libsynthgen.so (built by build_lib next to this module)."""
    global _synthgen_lib
    if _synthgen_lib is None:
        import ctypes as C
        import os
        path = os.path.join(os.path.dirname(os.path.abspath(__file__)), "synthgen", "libsynthgen.so")
        if not os.path.exists(path):
            raise ImportError(f"{path} not built; run python -m paper_1702_01481_amd.build_lib")
        lib = C.CDLL(path)
        vp, i32, i64 = C.c_void_p, C.c_int32, C.c_int64
        lib.synth_gen_banded_chunk.argtypes = [i64, i64, i32, vp, vp, vp, i32, vp, C.c_double, C.c_uint64, i64,
                                               vp, vp, i64, vp, vp, vp]
        lib.synth_gen_banded_chunk.restype = C.c_int
        _synthgen_lib = lib
    return _synthgen_lib


def weights(n_rows: int, seed: int, index: int = 0, device="cpu") -> torch.Tensor:
    """Non-uniform positive importance weights in [0.5, 1.5) (tests only)."""
    g = _gen(device, seed, _S_W * 1000 + index)
    return 0.5 + torch.rand(n_rows, generator=g, dtype=torch.float64, device=device)


def old_directions(n_old: int, n_params: int, seed: int, device="cpu") -> torch.Tensor:
    """Seeded stand-ins for the previous N_O updates, [N_O][N_V]."""
    g = _gen(device, seed, _S_OLD)
    return torch.randn(n_old, n_params, generator=g, dtype=torch.float64, device=device)


def dyadic_chunk(n_rows: int, n_params: int, seed: int, index: int = 0):
    """Small-integer samples in [-7, 7] (CPU): every product and every partial
    sum of the contractions is exact in FP64, BF16 pieces and FP32, so all
    summation orders give bit-identical results."""
    g = _gen("cpu", seed, _S_CHUNK0 + 7919 * (index + 1))
    O = torch.randint(-7, 8, (n_rows, n_params), generator=g).to(torch.float64)
    e = torch.randint(-7, 8, (n_rows, n_params), generator=g).to(torch.float64)
    EL = torch.randint(-7, 8, (n_rows,), generator=g).to(torch.float64)
    return O, e, EL


def planted_zero_variance(dim_hilbert: int, n_params: int, seed: int, n_samples: int = 0):
    """planted_eigenstate(..., state=0) without the spectrum: the ground
    state planted; returns (O, e, EL, w, Delta, E0)."""
    O, e, EL, w, delta, evals = planted_eigenstate(dim_hilbert, n_params, seed, 0, n_samples)
    return O, e, EL, w, delta, float(evals[0])


def planted_eigenstate(dim_hilbert: int, n_params: int, seed: int, state: int = 0, n_samples: int = 0):
    """A finite Hilbert-space model whose tangent space holds an exact
    eigenstate, the ground state (state 0) or an excited one (the setting of
    the strong zero-variance principle).

    A random symmetric Hamiltonian matrix Hf on `dim_hilbert` basis states
    has eigenstates phi_k (energies E_k, ascending).  Psi is positive and
    bounded away from zero; the derivative vectors Psi^x are random except
    the last, which is solved for so that Psi + sum_x Delta_x Psi^x is
    phi_state (scaled) for a random Delta.
    Per basis state n: O[n, x] = Psi^x(n)/Psi(n), EL[n] = (Hf Psi)(n)/Psi(n),
    e[n, x] = (Hf Psi^x)(n)/Psi(n).

    n_samples == 0: exact enumeration, weights Psi(n)^2.
    n_samples > 0: states drawn uniformly, weights Psi(n)^2 / (1/dim).
    Returns (O, e, EL, w, Delta, evals) as float64 numpy arrays, evals the
    whole spectrum of Hf.
    """
    g = _gen("cpu", seed, 0xC0FFEE)
    f64 = torch.float64
    A = torch.randn(dim_hilbert, dim_hilbert, generator=g, dtype=f64).numpy()
    Hf = 0.5 * (A + A.T)
    evals, evecs = np.linalg.eigh(Hf)
    phi0 = evecs[:, state]
    psi = 1.0 + torch.rand(dim_hilbert, generator=g, dtype=f64).numpy()
    dpsi = 0.5 * torch.randn(n_params, dim_hilbert, generator=g, dtype=f64).numpy()
    delta = 0.3 * torch.randn(n_params, generator=g, dtype=f64).numpy()
    delta[-1] = 0.5 + abs(delta[-1])
    # scale phi0 so that the planted state is a modest step away from psi
    phi = phi0 * (np.linalg.norm(psi) / np.linalg.norm(phi0)) * np.sign(phi0 @ psi)
    dpsi[-1] = (phi - psi - delta[:-1] @ dpsi[:-1]) / delta[-1]
    O_all = (dpsi / psi).T
    EL_all = (Hf @ psi) / psi
    e_all = ((Hf @ dpsi.T).T / psi).T
    if n_samples == 0:
        w = psi ** 2
        return O_all, e_all, EL_all, w, delta, evals
    idx = torch.randint(0, dim_hilbert, (n_samples,), generator=g).numpy()
    w = psi[idx] ** 2 * dim_hilbert
    return O_all[idx], e_all[idx], EL_all[idx], w, delta, evals
