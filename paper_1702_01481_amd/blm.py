"""Thin ctypes binding of libblm (include/blm.h): argument marshalling only.

Every step of the path runs in the HIP library; torch tensors only carry
device memory and the stream.  Loading fails loudly when the library has not
been built (python -m paper_1702_01481_amd.build_lib).
"""
from __future__ import annotations

import ctypes as C
import os
from typing import Iterable, List, Optional, Sequence, Tuple

import numpy as np
import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
# BLM_LIBRARY: another build of the same library (the sanitized host build)
LIB_PATH = os.environ.get("BLM_LIBRARY") or os.path.join(_HERE, "libblm.so")

BLM_OK = 0
STATUS_NAMES = {0: "BLM_OK", 1: "BLM_E_ARG", 2: "BLM_E_STATE", 3: "BLM_E_HIP", 4: "BLM_E_NOMEM",
                5: "BLM_E_S_NOT_PD", 6: "BLM_E_NONFINITE", 7: "BLM_E_NOCONV", 8: "BLM_E_TIMEOUT"}
FLAG_COMPLEX_ENERGY, FLAG_PAIR_KEPT, FLAG_SMALL_ALPHA = 1, 2, 4

PRECISIONS = {"fp64": 0, "bf16x2": 1, "bf16x3": 2, "fp8": 3, "fp8x2": 4}

EXPORTED = ("blm_pack_bf16", "blm_pack_fp8", "blm_workspace_bytes", "blm_accumulator_bytes", "blm_create", "blm_destroy", "blm_begin_step",
            "blm_build_blocks", "blm_autotune_build", "blm_capture_build", "blm_replay_build",
            "blm_solve_blocks", "blm_project", "blm_stage2",
            "blm_get_block_matrices", "blm_get_directions", "blm_get_stage2_matrices",
            "blm_debug_eigvals", "blm_pencil_eigvals_static", "blm_set_timing", "blm_get_timings", "blm_get_solver_stats",
            "blm_state_bytes", "blm_export_state", "blm_import_state",
            "blm_batch_create", "blm_batch_destroy", "blm_batch_build", "blm_batch_project", "blm_batch_solve_blocks", "blm_batch_stage2",
            "blm_last_error",
            "blm_status_string")
TIMING_NAMES = ("theta_proj", "block_gram", "block_reduce", "block_assemble", "block_eig",
                "dir_proj", "stage2_gram", "stage2_reduce", "stage2_solve", "block_strips")


class BLMError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"{STATUS_NAMES.get(status, status)}: {msg}")
        self.status = status


class _Config(C.Structure):
    _fields_ = [("n_params", C.c_int64), ("n_blocks", C.c_int32),
                ("block_offsets", C.POINTER(C.c_int64)), ("n_keep", C.c_int32),
                ("n_old", C.c_int32), ("n_shifts", C.c_int32), ("shifts", C.POINTER(C.c_double)),
                ("precision", C.c_int32), ("max_samples", C.c_int64), ("target", C.c_int32),
                ("omega", C.c_double)]


TARGETS = {"energy": 0, "omega": 1}


class _Chunk(C.Structure):
    _fields_ = [("n_samples", C.c_int64), ("ld", C.c_int64), ("O", C.c_void_p), ("e", C.c_void_p),
                ("E_L", C.c_void_p), ("w", C.c_void_p), ("layout", C.c_int32), ("pieces", C.c_int32),
                ("piece_stride", C.c_int64), ("O_res", C.c_void_p), ("e_res", C.c_void_p),
                ("O_scale", C.c_void_p), ("e_scale", C.c_void_p), ("O_res2", C.c_void_p),
                ("e_res2", C.c_void_p)]


_lib = None


def load() -> C.CDLL:
    """Loads libblm.so from the package directory (raises if it is missing)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"libblm.so not built at {LIB_PATH}; run python -m paper_1702_01481_amd.build_lib")
    lib = C.CDLL(LIB_PATH)
    vp, i32, i64, dp = C.c_void_p, C.c_int32, C.c_int64, C.POINTER(C.c_double)
    lib.blm_pack_bf16.argtypes = [vp, i64, i64, i64, i32, vp, i64, i64, vp]
    lib.blm_pack_fp8.argtypes = [vp, i64, i64, i64, vp, vp, vp, vp, i64, vp]
    lib.blm_workspace_bytes.argtypes = [C.POINTER(_Config), C.POINTER(C.c_size_t)]
    lib.blm_accumulator_bytes.argtypes = [C.POINTER(_Config), C.POINTER(C.c_size_t)]
    lib.blm_create.argtypes = [C.POINTER(_Config), vp, C.POINTER(vp)]
    lib.blm_destroy.argtypes = [vp]
    lib.blm_begin_step.argtypes = [vp, vp]
    lib.blm_build_blocks.argtypes = [vp, C.POINTER(_Chunk), i32]
    lib.blm_solve_blocks.argtypes = [vp, dp, C.POINTER(i32)]
    lib.blm_autotune_build.argtypes = [vp, C.POINTER(_Chunk), i32, C.POINTER(i32)]
    lib.blm_capture_build.argtypes = [vp, C.POINTER(_Chunk), i32]
    lib.blm_replay_build.argtypes = [vp]
    lib.blm_project.argtypes = [vp, C.POINTER(_Chunk), i32]
    lib.blm_stage2.argtypes = [vp, vp, dp, dp, C.POINTER(C.c_uint32)]
    lib.blm_get_block_matrices.argtypes = [vp, i32, i32, dp, dp, C.POINTER(i32)]
    lib.blm_get_directions.argtypes = [vp, i32, i32, dp, C.POINTER(i32)]
    lib.blm_get_stage2_matrices.argtypes = [vp, i32, dp, dp, C.POINTER(i32)]
    lib.blm_debug_eigvals.argtypes = [vp, vp, i32, dp, vp]
    lib.blm_pencil_eigvals_static.argtypes = [vp, vp, i32, vp, vp, vp]
    lib.blm_get_solver_stats.argtypes = [vp, C.POINTER(i32), i32]
    lib.blm_set_timing.argtypes = [vp, i32]
    lib.blm_get_timings.argtypes = [vp, dp, i32]
    lib.blm_batch_create.argtypes = [C.POINTER(vp), i32, C.POINTER(vp)]
    lib.blm_batch_destroy.argtypes = [vp]
    lib.blm_batch_build.argtypes = [vp, C.POINTER(C.POINTER(_Chunk)), C.POINTER(i32)]
    lib.blm_batch_solve_blocks.argtypes = [vp, C.POINTER(dp), C.POINTER(C.POINTER(i32))]
    lib.blm_batch_stage2.argtypes = [vp, C.POINTER(vp), C.POINTER(dp), C.POINTER(dp),
                                     C.POINTER(C.POINTER(C.c_uint32))]
    lib.blm_last_error.argtypes = [vp]
    lib.blm_last_error.restype = C.c_char_p
    lib.blm_status_string.argtypes = [C.c_int]
    lib.blm_status_string.restype = C.c_char_p
    for name in EXPORTED:
        if name not in ("blm_last_error", "blm_status_string"):
            getattr(lib, name).restype = C.c_int
    _lib = lib
    return lib


def _dptr(a: np.ndarray):
    return a.ctypes.data_as(C.POINTER(C.c_double))


def _stream_handle(stream) -> int:
    if stream is None:
        stream = torch.cuda.current_stream()
    return int(stream.cuda_stream)


def _check_f64_dev(t: torch.Tensor, name: str):
    if t.dtype != torch.float64 or not t.is_cuda:
        raise TypeError(f"{name} must be a float64 device tensor")


class SplitSamples:
    """BF16 split storage (hi/lo or hi/mid/lo pieces, k-packed) of an FP64
    [n][>= ncols] device array, made by the library's blm_pack_bf16."""

    def __init__(self, src: torch.Tensor, pieces: int = 3, ncols: Optional[int] = None, stream=None):
        _check_f64_dev(src, "src")
        self._alloc(int(src.shape[0]), int(ncols if ncols is not None else src.shape[1]), pieces, src.device)
        self.pack(src, stream)

    def _alloc(self, n_max: int, ncols: int, pieces: int, device):
        self.n = self.n_max = n_max
        self.ncols = ncols
        self.ld = self.ncols + (self.ncols & 1)
        self.pieces = int(pieces)
        n8 = (self.n_max + 7) // 8
        self.piece_stride = n8 * 8 * self.ld
        self.data = torch.empty(self.pieces * self.piece_stride, dtype=torch.int16, device=device)

    @classmethod
    def empty(cls, n_max: int, ncols: int, pieces: int = 3, device="cuda") -> "SplitSamples":
        """Storage for up to n_max samples, filled later by pack()."""
        obj = cls.__new__(cls)
        obj._alloc(int(n_max), int(ncols), pieces, torch.device(device))
        return obj

    def pack(self, src: torch.Tensor, stream=None):
        """Refills the storage from FP64 samples src [n <= n_max][>= ncols]
        (asynchronous on the stream)."""
        _check_f64_dev(src, "src")
        if src.dim() != 2 or src.stride(1) != 1:
            raise ValueError("src must be [n][ld] with unit column stride")
        n = int(src.shape[0])
        if n > self.n_max or src.shape[1] < self.ncols:
            raise ValueError("src does not fit the storage")
        self.n = n
        st = load().blm_pack_bf16(C.c_void_p(src.data_ptr()), n, src.stride(0) if n else self.ncols,
                                  self.ncols, self.pieces, C.c_void_p(self.data.data_ptr()), self.ld,
                                  self.piece_stride, C.c_void_p(_stream_handle(stream)))
        if st != BLM_OK:
            raise BLMError(st, "blm_pack_bf16 failed")
        return self

    def to_numpy(self) -> np.ndarray:
        """Host copy of the pieces' sum (for checks): [n][ncols] float64."""
        raw = self.data.cpu().numpy().astype(np.uint16).astype(np.uint32) << 16
        pcs = raw.view(np.float32).astype(np.float64).reshape(self.pieces, -1)
        tot = pcs.sum(axis=0)
        n8 = self.piece_stride // (8 * self.ld)
        arr = tot.reshape(n8, self.ld, 8).transpose(0, 2, 1).reshape(n8 * 8, self.ld)
        return arr[: self.n, : self.ncols]


class Fp8Samples:
    """FP8 storage (e4m3 codes k-packed by 16 samples, one or two BF16
    residuals k-packed by 8, power-of-two column scales) of an FP64
    [n][>= ncols] device array, made by the library's blm_pack_fp8."""

    def __init__(self, src: torch.Tensor, ncols: Optional[int] = None, stream=None, residuals: int = 1):
        _check_f64_dev(src, "src")
        self._alloc(int(src.shape[0]), int(ncols if ncols is not None else src.shape[1]), residuals, src.device)
        self.pack(src, stream)

    def _alloc(self, n_max: int, ncols: int, residuals: int, device):
        if residuals not in (1, 2):
            raise ValueError("residuals must be 1 or 2")
        self.n = self.n_max = n_max
        self.ncols = ncols
        self.ld = self.ncols
        self.residuals = residuals
        n16, n8 = (self.n_max + 15) // 16, (self.n_max + 7) // 8
        self.codes = torch.empty(n16 * 16 * self.ld, dtype=torch.uint8, device=device)
        self.res = torch.empty(n8 * 8 * self.ld, dtype=torch.int16, device=device)
        self.res2 = torch.empty(n8 * 8 * self.ld, dtype=torch.int16, device=device) if residuals == 2 else None
        self.scale = torch.empty(self.ld, dtype=torch.float32, device=device)

    @classmethod
    def empty(cls, n_max: int, ncols: int, device="cuda", residuals: int = 1) -> "Fp8Samples":
        """Storage for up to n_max samples, filled later by pack()."""
        obj = cls.__new__(cls)
        obj._alloc(int(n_max), int(ncols), residuals, torch.device(device))
        return obj

    def pack(self, src: torch.Tensor, stream=None):
        """Refills the storage from FP64 samples src [n <= n_max][>= ncols]
        (asynchronous on the stream)."""
        _check_f64_dev(src, "src")
        if src.dim() != 2 or src.stride(1) != 1:
            raise ValueError("src must be [n][ld] with unit column stride")
        n = int(src.shape[0])
        if n > self.n_max or src.shape[1] < self.ncols:
            raise ValueError("src does not fit the storage")
        self.n = n
        st = load().blm_pack_fp8(C.c_void_p(src.data_ptr()), n, src.stride(0) if n else self.ncols,
                                 self.ncols, C.c_void_p(self.codes.data_ptr()), C.c_void_p(self.res.data_ptr()),
                                 C.c_void_p(self.res2.data_ptr() if self.res2 is not None else None),
                                 C.c_void_p(self.scale.data_ptr()), self.ld, C.c_void_p(_stream_handle(stream)))
        if st != BLM_OK:
            raise BLMError(st, "blm_pack_fp8 failed")
        return self

    def host_parts(self):
        """Host copies: codes [n][ncols] uint8, residual bits [n][ncols] uint16, scales [ncols]
        (and, with two residuals, the second residual bits after the first)."""
        n16, n8 = (self.n_max + 15) // 16, (self.n_max + 7) // 8
        q = self.codes.cpu().numpy().reshape(n16, self.ld, 16).transpose(0, 2, 1).reshape(n16 * 16, self.ld)

        def unpack(t):
            r = t.cpu().numpy().view(np.uint16).reshape(n8, self.ld, 8).transpose(0, 2, 1)
            return r.reshape(n8 * 8, self.ld)[: self.n, : self.ncols]

        out = (q[: self.n, : self.ncols], unpack(self.res), self.scale.cpu().numpy()[: self.ncols])
        if self.res2 is not None:
            out = out[:2] + (unpack(self.res2),) + out[2:]
        return out


def _chunk(O, e, EL, w, n_params) -> _Chunk:
    if isinstance(O, SplitSamples):
        if not isinstance(e, SplitSamples) or e.n != O.n or e.ld != O.ld or e.pieces != O.pieces:
            raise ValueError("O and e must be SplitSamples of the same shape")
        if O.ncols < n_params:
            raise ValueError("split chunk has too few columns")
        _check_f64_dev(EL, "E_L")
        if w is not None:
            raise ValueError("the BF16 path needs uniform weights")
        return _Chunk(O.n, O.ld, O.data.data_ptr(), e.data.data_ptr(), EL.data_ptr(), None, 1, O.pieces,
                      O.piece_stride, None, None, None, None, None, None)
    if isinstance(O, Fp8Samples):
        if not isinstance(e, Fp8Samples) or e.n != O.n or e.ld != O.ld:
            raise ValueError("O and e must be Fp8Samples of the same shape")
        if O.ncols < n_params:
            raise ValueError("FP8 chunk has too few columns")
        _check_f64_dev(EL, "E_L")
        if w is not None:
            raise ValueError("the FP8 path needs uniform weights")
        if O.residuals != e.residuals:
            raise ValueError("O and e must carry the same number of residuals")
        two = O.residuals == 2
        return _Chunk(O.n, O.ld, O.codes.data_ptr(), e.codes.data_ptr(), EL.data_ptr(), None, 2, 0, 0,
                      O.res.data_ptr(), e.res.data_ptr(), O.scale.data_ptr(), e.scale.data_ptr(),
                      O.res2.data_ptr() if two else None, e.res2.data_ptr() if two else None)
    _check_f64_dev(O, "O")
    _check_f64_dev(e, "e")
    _check_f64_dev(EL, "E_L")
    if O.dim() != 2 or O.shape != e.shape or O.stride(1) != 1 or e.stride(1) != 1 or O.stride(0) != e.stride(0):
        raise ValueError("O and e must be [n][>= N_V] with unit column stride and equal row stride")
    if O.shape[1] < n_params or EL.shape[0] != O.shape[0] or not EL.is_contiguous():
        raise ValueError("chunk shapes do not match")
    if w is not None:
        _check_f64_dev(w, "w")
        if w.shape[0] != O.shape[0] or not w.is_contiguous():
            raise ValueError("w must be contiguous [n]")
    return _Chunk(O.shape[0], O.stride(0) if O.shape[0] > 0 else O.shape[1], O.data_ptr(), e.data_ptr(),
                  EL.data_ptr(), w.data_ptr() if w is not None else None, 0, 0, 0, None, None, None, None,
                  None, None)


class BLM:
    """One BLM optimisation context (blm_create .. blm_destroy)."""

    def __init__(self, n_params: int, block_offsets: Sequence[int], n_keep: int, n_old: int,
                 shifts: Sequence[float], max_samples: int, stream=None, precision: str = "fp64",
                 target: str = "energy", omega: float = 0.0):
        """target "omega": the excited-state target with energy shift omega
        (blm_target in blm.h); energies are then estimates of Omega."""
        self.lib = load()
        self.n_params = int(n_params)
        self.offsets = np.ascontiguousarray(block_offsets, dtype=np.int64)
        self.n_blocks = len(self.offsets) - 1
        self.n_keep, self.n_old = int(n_keep), int(n_old)
        self.shifts = np.ascontiguousarray(shifts, dtype=np.float64)
        self.max_samples = int(max_samples)
        self.precision = precision
        self._cfg = _Config(self.n_params, self.n_blocks, self.offsets.ctypes.data_as(C.POINTER(C.c_int64)),
                            self.n_keep, self.n_old, len(self.shifts), _dptr(self.shifts),
                            PRECISIONS[precision], self.max_samples, TARGETS[target], float(omega))
        self.target, self.omega = target, float(omega)
        self.stream = stream if stream is not None else torch.cuda.current_stream()
        h = C.c_void_p()
        self._check(self.lib.blm_create(C.byref(self._cfg), C.c_void_p(_stream_handle(self.stream)), C.byref(h)),
                    ctx=None)
        self.h = h
        self._keep = []   # tensors that must outlive queued work

    # -- helpers ----------------------------------------------------------
    def _check(self, st: int, ctx="self"):
        if st != BLM_OK:
            msg = ""
            if ctx == "self" and getattr(self, "h", None):
                msg = self.lib.blm_last_error(self.h).decode()
            raise BLMError(st, msg or self.lib.blm_status_string(st).decode())

    @staticmethod
    def workspace_bytes(n_params, block_offsets, n_keep, n_old, shifts, max_samples,
                        precision: str = "fp64", target: str = "energy") -> int:
        lib = load()
        off = np.ascontiguousarray(block_offsets, dtype=np.int64)
        sh = np.ascontiguousarray(shifts, dtype=np.float64)
        cfg = _Config(n_params, len(off) - 1, off.ctypes.data_as(C.POINTER(C.c_int64)), n_keep, n_old,
                      len(sh), _dptr(sh), PRECISIONS[precision], max_samples, TARGETS[target], 0.0)
        out = C.c_size_t()
        st = lib.blm_workspace_bytes(C.byref(cfg), C.byref(out))
        if st != BLM_OK:
            raise BLMError(st, lib.blm_status_string(st).decode())
        return int(out.value)

    @staticmethod
    def accumulator_bytes(n_params, block_offsets, n_keep, n_old, shifts, max_samples,
                          precision: str = "fp64", target: str = "energy") -> int:
        """Bytes of the block estimates' accumulators (blm_accumulator_bytes)."""
        lib = load()
        off = np.ascontiguousarray(block_offsets, dtype=np.int64)
        sh = np.ascontiguousarray(shifts, dtype=np.float64)
        cfg = _Config(n_params, len(off) - 1, off.ctypes.data_as(C.POINTER(C.c_int64)), n_keep, n_old,
                      len(sh), _dptr(sh), PRECISIONS[precision], max_samples, TARGETS[target], 0.0)
        out = C.c_size_t()
        st = lib.blm_accumulator_bytes(C.byref(cfg), C.byref(out))
        if st != BLM_OK:
            raise BLMError(st, lib.blm_status_string(st).decode())
        return int(out.value)

    def close(self):
        if getattr(self, "h", None):
            self.lib.blm_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _chunks(self, chunks) -> Tuple[C.Array, int]:
        cs = []
        for ch in chunks:
            O, e, EL = ch[0], ch[1], ch[2]
            w = ch[3] if len(ch) > 3 else None
            cs.append(_chunk(O, e, EL, w, self.n_params))
            self._keep.append(ch)
        arr = (_Chunk * max(len(cs), 1))(*cs)
        return arr, len(cs)

    # -- the step ---------------------------------------------------------
    def begin_step(self, old: Optional[torch.Tensor] = None):
        self._keep = []
        if old is not None:
            _check_f64_dev(old, "old")
            if old.shape != (self.n_old, self.n_params) or not old.is_contiguous():
                raise ValueError("old must be contiguous [n_old][n_params]")
            self._keep.append(old)
        self._check(self.lib.blm_begin_step(self.h, C.c_void_p(old.data_ptr() if old is not None else None)))

    def build(self, chunks: Iterable):
        arr, n = self._chunks(chunks)
        self._check(self.lib.blm_build_blocks(self.h, arr, n))

    def drop_chunk_refs(self):
        """Forgets the chunks kept alive for queued work (they are otherwise
        held until the next begin_step); only once the stream has passed
        the calls that read them, e.g. after torch.cuda.synchronize()."""
        self._keep = [k for k in self._keep if isinstance(k, torch.Tensor)]   # the step's old directions

    def capture_build(self, chunks: Iterable):
        """Records the build of these chunks as a HIP graph (blm_capture_build);
        the chunks are kept alive with the recording."""
        n0 = len(self._keep)
        arr, n = self._chunks(chunks)
        self._graph_keep = self._keep[n0:]
        del self._keep[n0:]
        self._check(self.lib.blm_capture_build(self.h, arr, n))

    def replay_build(self):
        """Runs the recorded build (blm_replay_build)."""
        self._check(self.lib.blm_replay_build(self.h))

    def autotune(self, chunks: Iterable) -> int:
        """Times the build's Gram kernel on these chunks for each slice-group
        count and keeps the fastest for later builds; returns it."""
        arr, n = self._chunks(chunks)
        g = C.c_int32()
        self._check(self.lib.blm_autotune_build(self.h, arr, n, C.byref(g)))
        return int(g.value)

    def solve(self):
        """Returns (evals [n_shifts][N_B][N_K+1] complex, kept [n_shifts][N_B])."""
        ns, nb, nk = len(self.shifts), self.n_blocks, self.n_keep
        ev = np.zeros((ns, nb, nk + 1, 2))
        kept = np.zeros((ns, nb), dtype=np.int32)
        self._check(self.lib.blm_solve_blocks(self.h, _dptr(ev), kept.ctypes.data_as(C.POINTER(C.c_int32))))
        return ev[..., 0] + 1j * ev[..., 1], kept

    def project(self, chunks: Iterable):
        arr, n = self._chunks(chunks)
        self._check(self.lib.blm_project(self.h, arr, n))

    def stage2(self, want_update: bool = True):
        """Returns (update [n_shifts][N_V] device tensor or None, energy, alpha ratio, flags)."""
        ns = len(self.shifts)
        upd = torch.empty(ns, self.n_params, dtype=torch.float64, device="cuda") if want_update else None
        en = np.zeros(ns)
        al = np.zeros(ns)
        fl = np.zeros(ns, dtype=np.uint32)
        self._check(self.lib.blm_stage2(self.h, C.c_void_p(upd.data_ptr() if upd is not None else None),
                                        _dptr(en), _dptr(al), fl.ctypes.data_as(C.POINTER(C.c_uint32))))
        self._keep = []
        return upd, en, al, fl

    # -- diagnostics ------------------------------------------------------
    def set_timing(self, enable: bool = True):
        self._check(self.lib.blm_set_timing(self.h, 1 if enable else 0))

    def solver_stats(self) -> np.ndarray:
        """[n_shifts * N_B][16] int32 statistics of the last block solve."""
        n = len(self.shifts) * self.n_blocks * 16
        out = np.zeros(n, dtype=np.int32)
        self._check(self.lib.blm_get_solver_stats(self.h, out.ctypes.data_as(C.POINTER(C.c_int32)), n))
        return out.reshape(-1, 16)

    def timings(self) -> dict:
        """Durations (ms) of the last call of each phase, from HIP events."""
        out = np.full(len(TIMING_NAMES), -1.0)
        self._check(self.lib.blm_get_timings(self.h, _dptr(out), len(out)))
        return {k: float(v) for k, v in zip(TIMING_NAMES, out)}

    # -- checkpoint of pass 1 -----------------------------------------------
    def export_state(self) -> np.ndarray:
        """blm_export_state: the step's pass-1 sums and fingerprint, as bytes."""
        n = C.c_size_t()
        self._check(self.lib.blm_state_bytes(self.h, C.byref(n)))
        buf = np.empty(n.value, dtype=np.uint8)
        self._check(self.lib.blm_export_state(self.h, buf.ctypes.data_as(C.c_void_p), C.c_size_t(buf.nbytes)))
        return buf

    def import_state(self, buf: np.ndarray):
        """blm_import_state: right after begin_step, with the same previous directions."""
        buf = np.ascontiguousarray(buf, dtype=np.uint8)
        self._check(self.lib.blm_import_state(self.h, buf.ctypes.data_as(C.c_void_p), C.c_size_t(buf.nbytes)))

    def block_matrices(self, block: int, shift: int = 0):
        d = C.c_int32()
        self._check(self.lib.blm_get_block_matrices(self.h, block, shift, None, None, C.byref(d)))
        H = np.zeros((d.value, d.value))
        S = np.zeros((d.value, d.value))
        self._check(self.lib.blm_get_block_matrices(self.h, block, shift, _dptr(H), _dptr(S), C.byref(d)))
        return H, S

    def directions(self, block: int, shift: int = 0) -> np.ndarray:
        n = C.c_int32()
        self._check(self.lib.blm_get_directions(self.h, block, shift, None, C.byref(n)))
        M = int(self.offsets[block + 1] - self.offsets[block])
        B = np.zeros((n.value, M))
        self._check(self.lib.blm_get_directions(self.h, block, shift, _dptr(B), C.byref(n)))
        return B

    def stage2_matrices(self, shift: int = 0):
        d = C.c_int32()
        self._check(self.lib.blm_get_stage2_matrices(self.h, shift, None, None, C.byref(d)))
        H = np.zeros((d.value, d.value))
        S = np.zeros((d.value, d.value))
        self._check(self.lib.blm_get_stage2_matrices(self.h, shift, _dptr(H), _dptr(S), C.byref(d)))
        return H, S


class Batch:
    """Several contexts (independent optimisations on the same stream) whose
    block builds can share one Gram launch (build), whose block solves share
    one eigensolver launch, and whose stage-two solves share another
    (blm_batch_*).  Projections stay per context."""

    def __init__(self, ctxs: Sequence[BLM]):
        self.lib = load()
        self.ctxs = list(ctxs)
        n = len(self.ctxs)
        arr = (C.c_void_p * n)(*[c.h.value for c in self.ctxs])
        h = C.c_void_p()
        st = self.lib.blm_batch_create(arr, n, C.byref(h))
        if st != BLM_OK:
            raise BLMError(st, self.lib.blm_status_string(st).decode())
        self.h = h

    def _check(self, st: int):
        if st != BLM_OK:
            msgs = [f"context {i}: {c.lib.blm_last_error(c.h).decode()}" for i, c in enumerate(self.ctxs)]
            raise BLMError(st, "; ".join(m for m in msgs if not m.endswith(": ")))

    def _chunk_tables(self, chunk_lists):
        n = len(self.ctxs)
        assert len(chunk_lists) == n
        arrs, counts = [], (C.c_int32 * n)()
        for i, (ctx, chunks) in enumerate(zip(self.ctxs, chunk_lists)):
            arr, m = ctx._chunks(chunks)
            arrs.append(arr)
            counts[i] = m
        self._keepalive = arrs
        return (C.POINTER(_Chunk) * n)(*[C.cast(a, C.POINTER(_Chunk)) for a in arrs]), counts

    def build(self, chunk_lists: Sequence[Iterable]):
        """blm_batch_build: chunk_lists[i] holds context i's chunks."""
        self._check(self.lib.blm_batch_build(self.h, *self._chunk_tables(chunk_lists)))

    def project(self, chunk_lists: Sequence[Iterable]):
        """blm_batch_project: chunk_lists[i] holds context i's chunks."""
        self._check(self.lib.blm_batch_project(self.h, *self._chunk_tables(chunk_lists)))

    def solve(self):
        """[(evals, kept)] per context, as BLM.solve."""
        outs = []
        for c in self.ctxs:
            ns, nb, nk = len(c.shifts), c.n_blocks, c.n_keep
            outs.append((np.zeros((ns, nb, nk + 1, 2)), np.zeros((ns, nb), dtype=np.int32)))
        n = len(self.ctxs)
        evp = (C.POINTER(C.c_double) * n)(*[_dptr(ev) for ev, _ in outs])
        kp = (C.POINTER(C.c_int32) * n)(*[k.ctypes.data_as(C.POINTER(C.c_int32)) for _, k in outs])
        self._check(self.lib.blm_batch_solve_blocks(self.h, evp, kp))
        return [(ev[..., 0] + 1j * ev[..., 1], k) for ev, k in outs]

    def stage2(self, want_update: bool = True):
        """[(update or None, energy, alpha ratio, flags)] per context, as BLM.stage2."""
        outs = []
        for c in self.ctxs:
            ns = len(c.shifts)
            upd = torch.empty(ns, c.n_params, dtype=torch.float64, device="cuda") if want_update else None
            outs.append((upd, np.zeros(ns), np.zeros(ns), np.zeros(ns, dtype=np.uint32)))
        n = len(self.ctxs)
        up = (C.c_void_p * n)(*[o[0].data_ptr() if o[0] is not None else None for o in outs])
        ep = (C.POINTER(C.c_double) * n)(*[_dptr(o[1]) for o in outs])
        ap = (C.POINTER(C.c_double) * n)(*[_dptr(o[2]) for o in outs])
        fp = (C.POINTER(C.c_uint32) * n)(*[o[3].ctypes.data_as(C.POINTER(C.c_uint32)) for o in outs])
        self._check(self.lib.blm_batch_stage2(self.h, up, ep, ap, fp))
        for c in self.ctxs:
            c._keep = []
        return outs

    def close(self):
        if getattr(self, "h", None):
            self.lib.blm_batch_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def debug_eigvals(H: torch.Tensor, S: torch.Tensor, stream=None) -> np.ndarray:
    """All eigenvalues of the pencil (H, S) from the library's eigensolver."""
    lib = load()
    _check_f64_dev(H, "H")
    _check_f64_dev(S, "S")
    d = H.shape[0]
    H = H.contiguous()
    S = S.contiguous()
    out = np.zeros((d, 2))
    st = lib.blm_debug_eigvals(C.c_void_p(H.data_ptr()), C.c_void_p(S.data_ptr()), d, _dptr(out),
                               C.c_void_p(_stream_handle(stream)))
    if st != BLM_OK:
        raise BLMError(st, lib.blm_status_string(st).decode())
    return out[:, 0] + 1j * out[:, 1]


STATIC_MAXD = 512   # BLM_STATIC_MAXD


def pencil_eigvals_static(H: torch.Tensor, S: torch.Tensor, evals: torch.Tensor, status: torch.Tensor,
                          stream=None) -> None:
    """blm_pencil_eigvals_static: the eigenvalues of debug_eigvals into the
    caller's device tensors evals (float64 [d][2]) and status (int32 [1]),
    with no device allocation by the library.  Asynchronous on the stream."""
    lib = load()
    _check_f64_dev(H, "H")
    _check_f64_dev(S, "S")
    _check_f64_dev(evals, "evals")
    d = int(H.shape[0])
    for t, name in ((H, "H"), (S, "S")):
        if t.dim() != 2 or tuple(t.shape) != (d, d) or not t.is_contiguous():
            raise ValueError(f"{name} must be a contiguous [d][d] tensor")
    if tuple(evals.shape) != (d, 2) or not evals.is_contiguous():
        raise ValueError("evals must be a contiguous [d][2] tensor")
    if status.dtype != torch.int32 or not status.is_cuda or status.numel() < 1:
        raise TypeError("status must be an int32 device tensor")
    st = lib.blm_pencil_eigvals_static(C.c_void_p(H.data_ptr()), C.c_void_p(S.data_ptr()), d,
                                       C.c_void_p(evals.data_ptr()), C.c_void_p(status.data_ptr()),
                                       C.c_void_p(_stream_handle(stream)))
    if st != BLM_OK:
        raise BLMError(st, lib.blm_status_string(st).decode())
