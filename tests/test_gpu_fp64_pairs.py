"""The FP64 build's second tile shape: two 64 x 64 tiles of one row tile per
workgroup (gram64_pair_kernel), the shape the autotuner may choose against
one tile per workgroup.  The same block estimates (Eq. 3 on the one-block
basis, with the coupling strips of Fig. 1) either way.

`BLM_FP64_PAIRS=1` at context creation forces the pair shape.  Checked on
even block offsets (16-byte loads) and odd ones (8-byte loads), with ragged
tiles, a previous direction (aux columns, so diagonal pairs carry strips) and
two chunks: every block pencil, which holds the tiles and the strips, within
1e-13 of the single-tile build (relative Frobenius; the two kernels add the
products of a 16-sample stage in different orders), and the step's energies
within 1e-12.
"""
import os

import numpy as np
import pytest
import torch

from paper_1702_01481_amd import synth

pytestmark = pytest.mark.gpu


def _step(ctx, chunks, old):
    ctx.begin_step(old)
    ctx.build(chunks)
    _, kept = ctx.solve()
    ctx.project(chunks)
    _, en, _, _ = ctx.stage2()
    torch.cuda.synchronize()
    return np.asarray(en), kept


@pytest.mark.parametrize("offsets", [[0, 128, 384, 512, 640], [0, 131, 390, 517, 651]])
def test_pair_shape_matches_single_tiles(offsets):
    from paper_1702_01481_amd import blm
    nv = offsets[-1]
    gen = synth.SampleGenerator(nv, 8, 31, sigma_E=0.5, device="cuda")
    chunks = [gen.chunk(0, 20_000), gen.chunk(1, 13_617)]
    old = synth.old_directions(1, nv, seed=5).cuda().contiguous()
    torch.cuda.synchronize()
    args = (nv, offsets, 2, 1, [1e-3], 33_617)
    single = blm.BLM(*args)
    os.environ["BLM_FP64_PAIRS"] = "1"
    try:
        paired = blm.BLM(*args)
    finally:
        del os.environ["BLM_FP64_PAIRS"]
    e1, k1 = _step(single, chunks, old)
    e2, k2 = _step(paired, chunks, old)
    worst = 0.0
    for b in range(len(offsets) - 1):
        H1, S1 = single.block_matrices(b, 0)
        H2, S2 = paired.block_matrices(b, 0)
        worst = max(worst, np.linalg.norm(S2 - S1) / np.linalg.norm(S1), np.linalg.norm(H2 - H1) / np.linalg.norm(H1))
    print(f"[fp64-pairs] offsets {offsets}: block pencils within {worst:.1e}; energy {e1[0]:.12f} vs {e2[0]:.12f}",
          flush=True)
    assert worst <= 1e-13, worst
    assert np.array_equal(k1, k2)
    assert abs(e1[0] - e2[0]) <= 1e-12 * abs(e1[0])
    single.close()
    paired.close()
