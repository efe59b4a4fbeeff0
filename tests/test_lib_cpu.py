"""Host-side checks of the C ABI library (no GPU needed): it loads, exports
every function include/blm.h declares, and sizes its workspace."""
import ctypes
import os
import re

import numpy as np
import pytest

from paper_1702_01481_amd import blm

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    src = open(os.path.join(ROOT, "include", "blm.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(blm_[a-z0-9_]+)\s*\(", src)))


def test_library_exports_every_declared_symbol():
    if not os.path.exists(blm.LIB_PATH):
        pytest.skip("libblm.so not built")
    lib = ctypes.CDLL(blm.LIB_PATH)
    names = _declared()
    assert len(names) >= 14
    for n in names:
        assert hasattr(lib, n), n
    assert set(names) == set(blm.EXPORTED)


def test_workspace_bytes_and_argument_checks():
    if not os.path.exists(blm.LIB_PATH):
        pytest.skip("libblm.so not built")
    off = np.array([0, 512 * 1, 512 * 2, 512 * 3, 512 * 4, 512 * 5, 512 * 6, 512 * 7, 4096])
    b = blm.BLM.workspace_bytes(4096, off, 5, 1, [1e-4, 1e-3, 1e-2], 1_000_000)
    # dominated by the per-sample aux and stage-two projection buffers
    assert 1e9 < b < 2e10
    small = blm.BLM.workspace_bytes(4096, off, 5, 1, [1e-3], 65536)
    assert small < b
    # 1 + N_O N_B aux columns: 17 and 505 are taken, 513 is not
    assert blm.BLM.workspace_bytes(4096, off, 5, 2, [1e-3], 65536) > small
    assert blm.BLM.workspace_bytes(4096, off, 5, 63, [1e-3], 65536) > small
    with pytest.raises(blm.BLMError):
        blm.BLM.workspace_bytes(4096, off, 5, 64, [1e-3], 65536)     # 1 + N_O N_B = 513 > 512
    with pytest.raises(blm.BLMError):
        blm.BLM.workspace_bytes(4096, off[::-1].copy(), 5, 1, [1e-3], 65536)
    with pytest.raises(blm.BLMError):
        blm.BLM.workspace_bytes(4096, off, 5, 1, [-1.0], 65536)


def test_synthetic_partitions_cover_the_parameters():
    """Block partitions of the synthetic workloads: contiguous, ascending,
    from 0 to N_V; uniform-integer blocks within [lo, hi] except a merged
    remainder (below lo) on the last block."""
    from paper_1702_01481_amd import synth
    for w in synth.batched_workloads(n_samples=1):
        off = np.asarray(w.block_offsets)
        sz = np.diff(off)
        assert off[0] == 0 and off[-1] == w.n_params, (w.name, off[-1])
        assert sz.min() >= 500 and sz[:-1].max() <= 1500 and sz[-1] < 2000, (w.name, sz)
    assert sum(w.n_params for w in synth.batched_workloads(n_samples=1)) == 78_000
    off = synth.loguniform_offsets(30_000, 40, 100.0, 2000.0, 0)
    assert off[0] == 0 and off[-1] == 30_000 and len(off) == 41 and np.all(np.diff(off) > 0)


def test_recorded_build_keeps_its_chunks():
    """BLM.capture_build holds the recorded chunks for as long as the
    recording (they are read at every replay), apart from the chunks a
    step keeps until its next begin_step; no GPU call is made."""
    import types

    import torch
    old = torch.zeros(1, 4, dtype=torch.float64)
    o = types.SimpleNamespace(_keep=[old], h=None, _check=lambda st: None,
                              lib=types.SimpleNamespace(blm_capture_build=lambda *a: 0))

    def _chunks(chunks):
        o._keep.extend(chunks)
        return None, len(chunks)

    o._chunks = _chunks
    blm.BLM.capture_build(o, [("O0", "e0", "E0"), ("O1", "e1", "E1")])
    assert o._graph_keep == [("O0", "e0", "E0"), ("O1", "e1", "E1")]
    assert len(o._keep) == 1 and o._keep[0] is old
    blm.BLM.drop_chunk_refs(o)
    assert o._graph_keep and len(o._keep) == 1 and o._keep[0] is old


def test_static_eigvals_rejects_sizes_beyond_its_scratch():
    """blm_pencil_eigvals_static checks its arguments on the host before any
    device call: a pencil above BLM_STATIC_MAXD, or d < 1, or a missing
    pointer is BLM_E_ARG (no GPU needed)."""
    if not os.path.exists(blm.LIB_PATH):
        pytest.skip("libblm.so not built")
    lib = blm.load()
    fake = ctypes.c_void_p(256)      # never dereferenced: the size check comes first
    assert lib.blm_pencil_eigvals_static(fake, fake, blm.STATIC_MAXD + 1, fake, fake, None) == 1
    assert lib.blm_pencil_eigvals_static(fake, fake, 0, fake, fake, None) == 1
    assert lib.blm_pencil_eigvals_static(None, fake, 8, fake, fake, None) == 1
    assert lib.blm_pencil_eigvals_static(fake, fake, 8, fake, None, None) == 1


def test_accumulators_hold_the_papers_storage_count():
    """The block estimates' storage at the paper's setting (Sec. II.B:
    N_V = 30,000, N_B = 100, N_O = 5 gives 0.5 GB per process): the
    library's accumulators within 5% of the oracle's count of that storage
    (tests/golden/paper_memory.json pins the count itself); the library
    keeps whole S tiles and aux columns padded to groups of 16."""
    if not os.path.exists(blm.LIB_PATH):
        pytest.skip("libblm.so not built")
    import json

    from oracle import blm_oracle as orc
    g = json.load(open(os.path.join(ROOT, "tests", "golden", "paper_memory.json")))["blm"]
    off = np.linspace(0, g["n_params"], g["n_blocks"] + 1).astype(np.int64)
    lib_b = blm.BLM.accumulator_bytes(g["n_params"], off, 4, g["n_old"], [1e-3], 65536)
    paper_b = orc.blm_matrix_bytes(g["n_params"], g["n_blocks"], g["n_old"])
    assert abs(lib_b / paper_b - 1) <= 0.05, (lib_b, paper_b)
    assert round(lib_b / 1e9, g["digits"]) == g["gigabytes"]
    assert lib_b < blm.BLM.workspace_bytes(g["n_params"], off, 4, g["n_old"], [1e-3], 65536)


def test_omega_target_configuration():
    """The excited-state target: more workspace (the second pass's sums),
    unknown targets and a non-finite omega refused."""
    if not os.path.exists(blm.LIB_PATH):
        pytest.skip("libblm.so not built")
    off = np.array([0, 100, 250, 400])
    e = blm.BLM.workspace_bytes(400, off, 2, 1, [1e-3], 4096)
    o = blm.BLM.workspace_bytes(400, off, 2, 1, [1e-3], 4096, target="omega")
    assert o > e
    assert (blm.BLM.accumulator_bytes(400, off, 2, 1, [1e-3], 4096, target="omega")
            > blm.BLM.accumulator_bytes(400, off, 2, 1, [1e-3], 4096))
    lib = blm.load()
    sh = np.array([1e-3])
    offs = np.ascontiguousarray(off, dtype=np.int64)
    for target, omega in ((7, 0.0), (1, float("nan")), (1, float("inf"))):
        cfg = blm._Config(400, 3, offs.ctypes.data_as(ctypes.POINTER(ctypes.c_int64)), 2, 1, 1,
                          sh.ctypes.data_as(ctypes.POINTER(ctypes.c_double)), 0, 4096, target, omega)
        out = ctypes.c_size_t()
        assert lib.blm_workspace_bytes(ctypes.byref(cfg), ctypes.byref(out)) == 1   # BLM_E_ARG
