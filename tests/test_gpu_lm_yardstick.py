"""The traditional linear method (Eq. 1 and Eq. 2, Sec. II.A) as the
accuracy yardstick, through the library at the largest pencil it takes:
N_V = 4,095 parameters in one block, so the block pencil is the LM's own
4,096-dimensional one, on 24,000 synthetic samples (rank-32 model, dense G),
delta = 1e-3.  With one block the BLM is the LM: the block solve keeps the
lowest eigenvector's parameter part, and stage two on [Psi, B] returns that
eigenvector again.

Against the oracle's LM on the same sample bytes (lm_matrices, lm_step):
the matrices within 1e-12 relative Frobenius, the energy within 1e-10
relative, the update's cosine at least 1 - 1e-9 (the FP64 tolerances).
"""
import numpy as np
import pytest
import torch

from oracle import blm_oracle as orc
from paper_1702_01481_amd import synth

pytestmark = pytest.mark.gpu

NV, NS, DELTA = 4095, 24_000, 1e-3


@pytest.mark.timeout(600)
def test_lm_at_4096_dimensions_matches_the_oracle():
    from paper_1702_01481_amd import blm
    gen = synth.SampleGenerator(NV, 32, seed=7, sigma_E=0.5, device="cuda")
    O, e, EL = gen.chunk(0, NS)
    del gen
    torch.cuda.synchronize()
    offsets = np.array([0, NV], dtype=np.int64)
    ctx = blm.BLM(NV, offsets, 1, 0, [DELTA], NS)
    ctx.set_timing(True)
    ctx.begin_step()
    ctx.build([(O, e, EL)])
    ctx.solve()
    ctx.project([(O, e, EL)])
    upd, en, _, _ = ctx.stage2()
    torch.cuda.synchronize()
    t = ctx.timings()
    print(f"[lm] library step done: block solve {t['block_eig']:.0f} ms, energy {en[0]:.12f}", flush=True)
    H_g, S_g = ctx.block_matrices(0, 0)
    ctx.close()

    host = [(O.cpu().numpy(), e.cpu().numpy(), EL.cpu().numpy(), None)]
    H, S, _ = orc.lm_matrices(host)
    print("[lm] oracle matrices done; its 4,096-dimensional solve follows", flush=True)
    st = orc.lm_step(H, S, DELTA)
    P = np.eye(NV + 1)
    P[0, 0] = 0.0
    eS = np.linalg.norm(S_g - S) / np.linalg.norm(S)
    eH = np.linalg.norm(H_g - DELTA * P - H) / np.linalg.norm(H)
    d = upd[0].cpu().numpy()
    e_rel = abs(en[0] - st.energy) / abs(st.energy)
    cos = d @ st.dmu / (np.linalg.norm(d) * np.linalg.norm(st.dmu))
    r = np.linalg.norm(d - st.dmu) / np.linalg.norm(st.dmu)
    print(f"[lm] matrices {eS:.1e} / {eH:.1e}; energy {en[0]:.12f} vs {st.energy:.12f} (rel {e_rel:.1e}); "
          f"update cosine 1 - {1 - cos:.1e}, relative difference {r:.1e}", flush=True)
    assert eS <= 1e-12 and eH <= 1e-12, (eS, eH)
    assert e_rel <= 1e-10, e_rel
    assert cos >= 1 - 1e-9, cos
