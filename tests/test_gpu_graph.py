"""The block build recorded once as a HIP graph (blm_capture_build) and
replayed every step (blm_replay_build), against the same build issued call
by call on a second context with the same configuration: three steps in a
row, each with its own previous direction (Eq. 9), with eager work (the
other context's whole step) and synchronisations between the replays.  In
FP64 the recorded chunk buffers are refilled with fresh samples before each
step.  The graph runs the same kernels in the same order with the same
launch shapes, so block matrices, eigenvalues, energies and updates must be
equal bit for bit."""
import numpy as np
import pytest
import torch

from paper_1702_01481_amd import synth

pytestmark = pytest.mark.gpu

OFFSETS = [0, 100, 210, 300]
SHIFTS = [1e-3, 1e-2]
N, CUT = 20000, 13001


def _samples(step):
    g = synth.SampleGenerator(300, 8, 40 + step)
    return g.chunk(0, N)


def _step(ctx, chunks, old, replay):
    ctx.begin_step(old)
    if replay:
        ctx.replay_build()
    else:
        ctx.build(chunks)
    ev, kept = ctx.solve()
    ctx.project(chunks)
    upd, en, _, _ = ctx.stage2()
    torch.cuda.synchronize()
    mats = [ctx.block_matrices(b, si) for si in range(len(SHIFTS)) for b in range(len(OFFSETS) - 1)]
    return mats, ev, kept, upd.cpu().numpy(), en


@pytest.mark.parametrize("precision", ["fp64", "bf16x3", "fp8", "fp8x2"])
def test_replayed_build_equals_eager_build(precision):
    from paper_1702_01481_amd import blm
    print(f"[graph] {precision}", flush=True)
    O, e, EL = _samples(0)
    w = synth.weights(N, 3) if precision == "fp64" else None
    bufs = []
    for a, b in ((0, CUT), (CUT, N)):
        bufs.append([O[a:b].cuda().contiguous(), e[a:b].cuda().contiguous(), EL[a:b].cuda().contiguous(),
                     None if w is None else w[a:b].cuda().contiguous()])

    def chunks():
        if precision == "fp64":
            return [tuple(c) for c in bufs]
        return store

    if precision in ("fp8", "fp8x2"):
        res = 2 if precision == "fp8x2" else 1
        store = [(blm.Fp8Samples(c[0], residuals=res), blm.Fp8Samples(c[1], residuals=res), c[2]) for c in bufs]
    elif precision == "bf16x3":
        store = [(blm.SplitSamples(c[0], 3), blm.SplitSamples(c[1], 3), c[2]) for c in bufs]
    ctx_g = blm.BLM(300, OFFSETS, 3, 1, SHIFTS, N, precision=precision)
    ctx_e = blm.BLM(300, OFFSETS, 3, 1, SHIFTS, N, precision=precision)
    with pytest.raises(blm.BLMError):
        ctx_g.replay_build()                       # nothing recorded yet
    ctx_g.capture_build(chunks())
    old = None
    for step in range(3):
        if precision == "fp64" and step > 0:
            O, e, EL = _samples(step)
            for c, (a, b) in zip(bufs, ((0, CUT), (CUT, N))):
                c[0].copy_(O[a:b])
                c[1].copy_(e[a:b])
                c[2].copy_(EL[a:b])
        torch.cuda.synchronize()
        old_t = torch.zeros(1, 300, dtype=torch.float64, device="cuda") if old is None else old
        g = _step(ctx_g, chunks(), old_t, replay=True)
        r = _step(ctx_e, chunks(), old_t, replay=False)
        for (Hg, Sg), (He, Se) in zip(g[0], r[0]):
            assert np.array_equal(Hg, He) and np.array_equal(Sg, Se), step
        assert np.array_equal(g[1], r[1], equal_nan=True), step
        assert np.array_equal(g[2], r[2]), step
        assert np.array_equal(g[3], r[3]) and np.array_equal(g[4], r[4]), step
        print(f"[graph] {precision} step {step}: equal, energies {g[4]}", flush=True)
        old = torch.from_numpy(g[3][1:2] if step == 0 else synth.old_directions(1, 300, step).numpy()).cuda()
        old = old.contiguous()
    ctx_g.close()
    ctx_e.close()
