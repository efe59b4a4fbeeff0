"""Checkpoint of pass 1 (blm_export_state / blm_import_state).  The block
estimates are running sums over the samples (Eq. 3 on the one-block basis,
Sec. II.B), so a step stopped between chunks resumes from its FP64 sums:
a second context, given the same previous directions, imports them and
builds the remaining chunks, and the whole step (block pencils, kept counts,
stage two, energies and updates) equals the uninterrupted step bit for bit.

Also checked: the refusals (another configuration, other previous
directions, a build before the import, an export after the solves, a short
buffer), and the excited-state target, whose state also holds the second
pass's sums.
"""
import numpy as np
import pytest
import torch

from paper_1702_01481_amd import synth

pytestmark = pytest.mark.gpu

NV = 600
OFFSETS = [0, 150, 390, 600]
SHIFTS = [1e-3, 1e-2]


def _data(prec):
    from paper_1702_01481_amd import blm
    gen = synth.SampleGenerator(NV, 8, 17, sigma_E=0.5, device="cuda")
    chunks = [gen.chunk(i, n) for i, n in enumerate((12_288, 9_000, 8_712))]
    if prec == "bf16x3":
        chunks = [(blm.SplitSamples(O, 3), blm.SplitSamples(e, 3), EL) for O, e, EL in chunks]
    old = synth.old_directions(1, NV, seed=4).cuda().contiguous()
    torch.cuda.synchronize()
    return chunks, old


def _ctx(prec, **kw):
    from paper_1702_01481_amd import blm
    return blm.BLM(NV, OFFSETS, 2, 1, kw.pop("shifts", SHIFTS), 30_000, precision=prec, **kw)


def _finish(ctx, chunks):
    _, kept = ctx.solve()
    ctx.project(chunks)
    upd, en, _, _ = ctx.stage2()
    torch.cuda.synchronize()
    mats = [ctx.block_matrices(b, s) for s in range(len(SHIFTS)) for b in range(len(OFFSETS) - 1)]
    return mats, kept, np.asarray(en), upd.cpu().numpy()


@pytest.mark.parametrize("prec,kw", [("fp64", {}), ("bf16x3", {}), ("fp64", {"target": "omega", "omega": -11.0})])
def test_resumed_step_equals_the_uninterrupted_one(prec, kw):
    chunks, old = _data(prec)
    ref = _ctx(prec, **dict(kw))
    ref.begin_step(old)
    for ch in chunks:
        ref.build([ch])
    r = _finish(ref, chunks)

    first = _ctx(prec, **dict(kw))
    first.begin_step(old)
    first.build(chunks[:1])
    first.build(chunks[1:2])
    state = first.export_state()
    first.close()

    resumed = _ctx(prec, **dict(kw))
    resumed.begin_step(old)
    resumed.import_state(state)
    resumed.build(chunks[2:])
    q = _finish(resumed, chunks)
    print(f"[checkpoint] {prec} {kw}: state {state.nbytes / 1e6:.1f} MB; energies {r[2]} and {q[2]}", flush=True)
    for (H1, S1), (H2, S2) in zip(r[0], q[0]):
        assert np.array_equal(H1, H2) and np.array_equal(S1, S2)
    assert np.array_equal(r[1], q[1])
    assert np.array_equal(r[2], q[2])
    assert np.array_equal(r[3], q[3])
    ref.close()
    resumed.close()


def test_refusals():
    from paper_1702_01481_amd import blm
    chunks, old = _data("fp64")
    a = _ctx("fp64")
    a.begin_step(old)
    a.build(chunks[:1])
    state = a.export_state()

    def status(fn):
        with pytest.raises(blm.BLMError) as ei:
            fn()
        return ei.value.status

    # another configuration
    b = _ctx("fp64", shifts=[1e-3])
    b.begin_step(old)
    assert status(lambda: b.import_state(state)) == 1
    b.close()
    # other previous directions
    c = _ctx("fp64")
    c.begin_step(synth.old_directions(1, NV, seed=5).cuda().contiguous())
    assert status(lambda: c.import_state(state)) == 2
    # a build before the import
    c.begin_step(old)
    c.build(chunks[1:2])
    assert status(lambda: c.import_state(state)) == 2
    # a short buffer
    c.begin_step(old)
    assert status(lambda: c.import_state(state[: state.nbytes // 2])) == 1
    # the import itself, then an export after the solves
    c.import_state(state)
    c.solve()
    assert status(lambda: c.export_state()) == 2
    c.close()
    a.close()
