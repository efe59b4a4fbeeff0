"""The excited-state target Omega = <(omega - H)> / <(omega - H)^2> (Sec.
III.D; the BLM applies to it with the Omega pencil, Sec. II.B) through the
C ABI, against the oracle.

* Planted excited state (strong zero variance): a finite Hilbert space whose
  tangent space holds the first excited state; from sampled states with
  weights, the library's LM (one block) on Omega with omega inside the gap
  returns the planted step (1e-8 relative) and lambda = 1/(omega - E_1)
  (1e-10 relative), as the oracle's pins fix.
* Whole step on synthetic samples (600 parameters in three uneven blocks,
  N_K = 2, one previous direction, two shifts, 30,000 samples): every
  block's pencil (A + delta P, B) against the oracle's omega_blm_step
  matrices, the kept counts, the stage-two pencil after mapping direction
  bases, the Omega estimates (1e-10 relative) and updates (cosine
  >= 1 - 1e-9).  The library forms A = omega S - H^T and B = omega^2 S -
  omega (H + H^T) + E from sums that are each exact to FP64 rounding, the
  oracle sums f f^T directly, so the pencils are held to 1e-12 times the
  cancellation factor (|omega|^2 |S| + 2 |omega| |H| + |E|) / |B| of the
  block (Frobenius norms, from the oracle's energy estimates).
* The same step on BF16 hi/mid/lo pieces: update cosine >= 0.9999 against
  FP64, energy printed.
* A recorded build is refused for this target.
"""
import numpy as np
import pytest
import torch

from oracle import blm_oracle as orc
from paper_1702_01481_amd import synth

pytestmark = pytest.mark.gpu


def _step(ctx, chunks, old=None):
    ctx.begin_step(old)
    ctx.build(chunks)
    _, kept = ctx.solve()
    ctx.project(chunks)
    upd, en, _, _ = ctx.stage2()
    torch.cuda.synchronize()
    return upd.cpu().numpy(), np.asarray(en), kept


def test_planted_excited_state():
    from paper_1702_01481_amd import blm
    O, e, EL, w, delta, ev = synth.planted_eigenstate(200, 60, 4, 1, 20_000)
    omega = 0.5 * (ev[0] + ev[1])
    dev = [tuple(torch.from_numpy(np.ascontiguousarray(a)).cuda() for a in (O, e, EL, w))]
    ctx = blm.BLM(60, [0, 60], 1, 0, [0.0], 20_000, target="omega", omega=omega)
    upd, en, _ = _step(ctx, dev)
    ctx.close()
    lam = 1.0 / (omega - ev[1])
    r = np.linalg.norm(upd[0] - delta) / np.linalg.norm(delta)
    print(f"[omega] planted: lambda {en[0]:.12f} vs 1/(omega - E_1) {lam:.12f}; step {r:.1e}", flush=True)
    assert abs(en[0] - lam) <= 1e-10 * abs(lam)
    assert r <= 1e-8


def _synthetic():
    gen = synth.SampleGenerator(600, 8, 11, sigma_E=0.5, device="cuda")
    ch = [gen.chunk(0, 16_384), gen.chunk(1, 13_616)]
    torch.cuda.synchronize()
    return ch


def test_whole_step_against_the_oracle():
    from paper_1702_01481_amd import blm
    chunks = _synthetic()
    offsets = np.array([0, 150, 390, 600])
    shifts, omega, n_keep = [1e-3, 1e-2], -11.0, 2
    old = synth.old_directions(1, 600, seed=9).numpy()
    ctx = blm.BLM(600, offsets, n_keep, 1, shifts, 30_000, target="omega", omega=omega)
    upd, en, kept = _step(ctx, chunks, torch.from_numpy(old).cuda().contiguous())
    host = [(O.cpu().numpy(), e.cpu().numpy(), EL.cpu().numpy(), None) for O, e, EL in chunks]
    out, probs = orc.omega_blm_step(lambda: iter(host), offsets, n_keep, shifts, omega, old=old)
    eprobs, _ = orc.block_problems(host, offsets, orc.previous_directions(old, offsets))
    for b in range(3):
        A_g, B_g = ctx.block_matrices(b, 0)
        S, H = eprobs[b].S, eprobs[b].H
        E = probs[b].S - omega ** 2 * S + omega * (H + H.T)
        nB = np.linalg.norm(probs[b].S)
        cancel = (omega ** 2 * np.linalg.norm(S) + 2 * abs(omega) * np.linalg.norm(H) + np.linalg.norm(E)) / nB
        eA = np.linalg.norm(A_g - shifts[0] * probs[b].P - probs[b].H) / np.linalg.norm(probs[b].H)
        eB = np.linalg.norm(B_g - probs[b].S) / nB
        print(f"[omega] block {b}: A {eA:.1e}, B {eB:.1e} (cancellation factor {cancel:.0f})", flush=True)
        assert eA <= 1e-12 * cancel and eB <= 1e-12 * cancel, (b, eA, eB, cancel)
    for si, delta in enumerate(shifts):
        res = out[si]
        for b in range(3):
            assert kept[si][b] == res.blocks[b].B.shape[0], (si, b)
        Bg = [ctx.directions(b, si) for b in range(3)]
        A2, B2 = ctx.stage2_matrices(si)
        n2 = A2.shape[0]
        T = np.zeros((n2, n2))
        T[0, 0] = 1.0
        at = 1
        for b in range(3):
            k = Bg[b].shape[0]
            T[at:at + k, at:at + k] = res.blocks[b].B @ Bg[b].T
            at += k
        e2A = np.linalg.norm(T @ A2 @ T.T - res.H2) / np.linalg.norm(res.H2)
        e2B = np.linalg.norm(T @ B2 @ T.T - res.S2) / np.linalg.norm(res.S2)
        e_rel = abs(en[si] - res.step.energy) / abs(res.step.energy)
        cos = upd[si] @ res.step.dmu / (np.linalg.norm(upd[si]) * np.linalg.norm(res.step.dmu))
        print(f"[omega] shift {delta:g}: stage two {e2A:.1e} / {e2B:.1e}; Omega {en[si]:.12f} vs "
              f"{res.step.energy:.12f} (rel {e_rel:.1e}); update cosine 1 - {1 - cos:.1e}", flush=True)
        assert e2A <= 1e-9 and e2B <= 1e-9, (si, e2A, e2B)
        assert e_rel <= 1e-10, (si, e_rel)
        assert cos >= 1 - 1e-9, (si, cos)
    ctx.close()

    split = [(blm.SplitSamples(O, 3), blm.SplitSamples(e, 3), EL) for O, e, EL in chunks]
    torch.cuda.synchronize()
    c3 = blm.BLM(600, offsets, n_keep, 1, shifts, 30_000, precision="bf16x3", target="omega", omega=omega)
    u3, e3, k3 = _step(c3, split, torch.from_numpy(old).cuda().contiguous())
    c3.close()
    for si, delta in enumerate(shifts):
        cos = u3[si] @ upd[si] / (np.linalg.norm(u3[si]) * np.linalg.norm(upd[si]))
        rel = abs(e3[si] - en[si]) / abs(en[si])
        print(f"[omega] bf16x3 shift {delta:g}: Omega rel err {rel:.1e}, update cosine {cos:.10f}, "
              f"kept {k3[si].tolist()} vs {kept[si].tolist()}", flush=True)
        assert cos >= 0.9999, (si, cos)


def test_recorded_build_refused():
    from paper_1702_01481_amd import blm
    chunks = _synthetic()
    ctx = blm.BLM(600, [0, 300, 600], 2, 0, [1e-3], 30_000, target="omega", omega=-11.0)
    with pytest.raises(blm.BLMError):
        ctx.capture_build(chunks)
    ctx.close()
