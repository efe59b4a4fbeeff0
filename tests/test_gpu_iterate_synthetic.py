"""BLM steps against the LM on the synthetic sample stream (Sec. II.B,
Eq. 9 and Eq. 10; the trends of Tables I to III): N_V = 2,000 parameters,
65,536 samples of the rank-32 model with dense G (made on the CPU, the same
bytes as the oracle-side study in the design notes), delta = 1, all steps
through the library.  The samples are held fixed, so the traditional LM
step on them (the library with one block, a 2,001-dimensional pencil) is
the yardstick.

Checked:
- the fixed-point property: with Theta holding the LM update, the BLM step
  returns the LM update and energy (two partitions and N_K);
- one step against the oracle's step on the same samples;
- the paper's trends for one step: the distance of the BLM update from the
  LM update grows with the number of blocks (5, 10, 20) and shrinks with
  more kept directions (1, 2, 4);
- iterations that feed the N_O newest updates back as Theta are printed as
  a table (N_O = 1, 2, 4).  On these fixed, noisy, non-symmetric estimates
  the LM step is a fixed point of that iteration but does not attract it
  (the distance oscillates above one), so no convergence is asserted; with
  no history every step is the same.  The planted symmetric model
  (tests/test_gpu_iterate.py) is where history drives the steps to the LM.
"""
import numpy as np
import pytest
import torch

from oracle import blm_oracle as orc
from paper_1702_01481_amd import synth

pytestmark = pytest.mark.gpu

NV, NS, DELTA = 2000, 65_536, 1.0


@pytest.fixture(scope="module")
def data():
    gen = synth.SampleGenerator(NV, 32, seed=3, sigma_E=0.5)
    host = [tuple(t.numpy() for t in gen.chunk(0, NS)) + (None,)]
    dev = [tuple(torch.from_numpy(a).cuda() for a in host[0][:3])]
    torch.cuda.synchronize()
    lm_upd, lm_en = _step(dev, 1, 1, 0, None)
    print(f"[iterate-synth] LM energy {lm_en:.12f}", flush=True)
    yield {"host": host, "chunks": dev, "lm": lm_upd, "lm_energy": lm_en}


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


def _dist(data, d):
    return float(np.linalg.norm(d - data["lm"]) / np.linalg.norm(data["lm"]))


def test_lm_update_is_a_fixed_point(data):
    for n_blocks, n_keep in ((10, 1), (20, 2)):
        d, en = _step(data["chunks"], n_blocks, n_keep, 1, data["lm"][None, :].copy())
        r = _dist(data, d)
        e = abs(en - data["lm_energy"]) / abs(data["lm_energy"])
        print(f"[iterate-synth] Theta = LM update, N_B {n_blocks}, N_K {n_keep}: update {r:.1e}, energy {e:.1e}",
              flush=True)
        assert r <= 1e-8, r
        assert e <= 1e-10, e


def test_one_step_matches_the_oracle(data):
    d, en = _step(data["chunks"], 10, 2, 0, None)
    r, _ = orc.blm_step(lambda: data["host"], synth.uniform_offsets(NV, 10), 2, [DELTA])
    st = r[0].step
    assert abs(en - st.energy) <= 1e-10 * abs(st.energy), (en, st.energy)
    assert np.linalg.norm(d - st.dmu) <= 1e-8 * np.linalg.norm(st.dmu)


def test_one_step_trends(data):
    nb = {k: _dist(data, _step(data["chunks"], k, 2, 0, None)[0]) for k in (5, 10, 20)}
    nk = {k: _dist(data, _step(data["chunks"], 10, k, 0, None)[0]) for k in (1, 2, 4)}
    print("[iterate-synth] one step, distance to the LM update by N_B (N_K 2):",
          " ".join(f"{k}: {v:.4e}" for k, v in nb.items()), flush=True)
    print("[iterate-synth] one step, distance to the LM update by N_K (N_B 10):",
          " ".join(f"{k}: {v:.4e}" for k, v in nk.items()), flush=True)
    assert nb[5] < nb[10] < nb[20], nb
    assert nk[1] > nk[2] > nk[4], nk


def _iterate(data, n_blocks, n_keep, n_old, steps=4):
    from paper_1702_01481_amd import blm
    ctx = blm.BLM(NV, synth.uniform_offsets(NV, n_blocks), n_keep, n_old, [DELTA], NS)
    hist, dist = [], []
    for _ in range(steps):
        old = None
        if n_old:
            rows = hist[::-1][:n_old]
            old = np.stack(rows + [np.zeros(NV)] * (n_old - len(rows)))
        d, _ = _step(data["chunks"], n_blocks, n_keep, n_old, old, ctx)
        hist.append(d)
        dist.append(_dist(data, d))
    ctx.close()
    print(f"[iterate-synth] N_B {n_blocks} N_K {n_keep} N_O {n_old}: distance to the LM update by step "
          + " ".join(f"{x:.3e}" for x in dist), flush=True)
    return dist


def test_iterations_with_history_table(data):
    for n_old in (1, 2, 4):
        _iterate(data, 10, 2, n_old)
    flat = _iterate(data, 10, 2, 0, steps=3)
    assert max(flat) - min(flat) <= 1e-9 * flat[0], flat    # no history: the same step every time
