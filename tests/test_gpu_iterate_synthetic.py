"""Iterated BLM steps with history on the synthetic sample stream (Sec. II.B,
Eq. 9 and Eq. 10): N_V = 2,000 parameters, 65,536 samples of the rank-32
model with dense G, delta = 1e-3, all on the device.  The samples are held
fixed, so the traditional LM step on them (the library with one block, a
2,001-dimensional pencil) is the fixed point the iteration should approach:
each BLM step takes the N_O newest updates of the steps before it as Theta.

Checked:
- the fixed-point property: with Theta holding the LM update, the BLM step
  returns the LM update and energy (any partition, any N_K);
- with history, the iteration approaches the LM update;
- the trends of the paper's Tables I to III, here as the distance of the
  sixth update from the LM update: it grows with the number of blocks and
  shrinks with more kept directions and more history.  The table is printed.
"""
import numpy as np
import pytest
import torch

from paper_1702_01481_amd import synth

pytestmark = pytest.mark.gpu

NV, NS, DELTA, STEPS = 2000, 65_536, 1e-3, 6


@pytest.fixture(scope="module")
def data():
    gen = synth.SampleGenerator(NV, 32, seed=3, sigma_E=0.5, device="cuda")
    ch = [gen.chunk(0, NS)]
    del gen
    torch.cuda.synchronize()
    lm_upd, lm_en = _step(ch, 1, 1, 0, None)
    print(f"[iterate-synth] LM energy {lm_en:.12f}", flush=True)
    yield {"chunks": ch, "lm": lm_upd, "lm_energy": lm_en}


def _step(chunks, n_blocks, n_keep, n_old, old, ctx=None):
    from paper_1702_01481_amd import blm
    offsets = synth.uniform_offsets(NV, n_blocks)
    own = ctx is None
    if own:
        ctx = blm.BLM(NV, offsets, n_keep, n_old, [DELTA], NS)
    ctx.begin_step(None if old is None else torch.from_numpy(old).cuda().contiguous())
    ctx.build(chunks)
    ctx.solve()
    ctx.project(chunks)
    upd, en, _, _ = ctx.stage2()
    torch.cuda.synchronize()
    out = upd[0].cpu().numpy(), float(en[0])
    if own:
        ctx.close()
    return out


def _iterate(data, n_blocks, n_keep, n_old):
    from paper_1702_01481_amd import blm
    offsets = synth.uniform_offsets(NV, n_blocks)
    ctx = blm.BLM(NV, offsets, n_keep, n_old, [DELTA], NS)
    hist, err, gap = [], [], []
    for _ in range(STEPS):
        old = None
        if n_old:
            rows = hist[::-1][:n_old]
            old = np.stack(rows + [np.zeros(NV)] * (n_old - len(rows)))
        d, en = _step(data["chunks"], n_blocks, n_keep, n_old, old, ctx)
        hist.append(d)
        err.append(np.linalg.norm(d - data["lm"]) / np.linalg.norm(data["lm"]))
        gap.append(en - data["lm_energy"])
    ctx.close()
    print(f"[iterate-synth] N_B {n_blocks:2d} N_K {n_keep} N_O {n_old}: update distance to LM "
          + " ".join(f"{x:.2e}" for x in err) + f"; final energy gap {gap[-1]:+.2e}", flush=True)
    return err


def test_lm_update_is_a_fixed_point(data):
    for n_blocks, n_keep in ((10, 1), (20, 2)):
        d, en = _step(data["chunks"], n_blocks, n_keep, 1, data["lm"][None, :].copy())
        r = np.linalg.norm(d - data["lm"]) / np.linalg.norm(data["lm"])
        e = abs(en - data["lm_energy"]) / abs(data["lm_energy"])
        print(f"[iterate-synth] Theta = LM update, N_B {n_blocks}, N_K {n_keep}: update {r:.1e}, energy {e:.1e}",
              flush=True)
        assert r <= 1e-8, r
        assert e <= 1e-10, e


def test_iteration_trends(data):
    base = _iterate(data, 10, 2, 1)
    nk = {1: _iterate(data, 10, 1, 1), 2: base, 4: _iterate(data, 10, 4, 1)}
    no = {0: _iterate(data, 10, 2, 0), 1: base, 2: _iterate(data, 10, 2, 2), 4: _iterate(data, 10, 2, 4)}
    nb = {5: _iterate(data, 5, 2, 1), 10: base, 20: _iterate(data, 20, 2, 1)}
    # history brings the steps toward the LM step
    assert base[-1] < 0.5 * base[0], base
    assert max(no[0]) - min(no[0]) <= 1e-9 * no[0][0], no[0]     # no history: the same step
    fin = lambda d: [d[k][-1] for k in sorted(d)]
    print("[iterate-synth] final distance by N_K (1, 2, 4):", fin(nk), flush=True)
    print("[iterate-synth] final distance by N_O (0, 1, 2, 4):", fin(no), flush=True)
    print("[iterate-synth] final distance by N_B (5, 10, 20):", fin(nb), flush=True)
    assert fin(nk) == sorted(fin(nk), reverse=True), fin(nk)
    assert fin(no) == sorted(fin(no), reverse=True), fin(no)
    assert fin(nb) == sorted(fin(nb)), fin(nb)
