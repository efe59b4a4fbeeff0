"""One Gram launch for the block builds of several independent optimisations
(blm_batch_build): every context's tile jobs in one launch, each reading its
own context's chunks (Eq. 3 for each context on its own).

* Three contexts of different shapes (one to three blocks, one or two
  shifts), in FP64, BF16 x3 and FP8 with two residuals: every block matrix
  of the batched build equals the context's own build up to the order of
  the FP64 sums over slice groups (relative Frobenius 1e-13), and the rest
  of the step, through the batch's shared solves, gives the same energies
  (1e-10 relative) and updates (cosine 1 - 1e-10).
* The eight-problem workload (N_V from 2,000 to 20,000, 78,000 parameters)
  at 16,384 samples per problem: one FP64 build launch for all eight against
  eight builds (1e-13), with both timed and printed.
* A batch of contexts with different storages refuses a batched build.
"""
import time

import numpy as np
import pytest
import torch

from paper_1702_01481_amd import synth

pytestmark = pytest.mark.gpu

PROBLEMS = [  # (offsets, N_K, shifts, samples, seed)
    ([0, 300], 3, (1e-3,), 4096, 21),
    ([0, 50, 120, 200], 2, (1e-3, 1e-2), 3000, 22),
    ([0, 130, 400], 3, (1e-2,), 5000, 23),
]


def _data(problems):
    out = []
    for off, _, _, ns, seed in problems:
        g = synth.SampleGenerator(int(off[-1]), 4, seed, device="cuda")
        O, e, EL = g.chunk(0, ns)
        out.append((O.contiguous(), e.contiguous(), EL.contiguous()))
    torch.cuda.synchronize()
    return out


def _stored(blm, prec, O, e, EL):
    if prec == "fp64":
        return (O, e, EL)
    if prec == "bf16x3":
        return (blm.SplitSamples(O, 3), blm.SplitSamples(e, 3), EL)
    return (blm.Fp8Samples(O, residuals=2), blm.Fp8Samples(e, residuals=2), EL)


def _rel(a, b):
    return np.linalg.norm(a - b) / np.linalg.norm(b)


def _cos(a, b):
    return float(a @ b / (np.linalg.norm(a) * np.linalg.norm(b)))


@pytest.mark.parametrize("prec", ["fp64", "bf16x3", "fp8x2"])
def test_batched_build_equals_single_builds(prec):
    from paper_1702_01481_amd import blm
    data = [_stored(blm, prec, *d) for d in _data(PROBLEMS)]
    torch.cuda.synchronize()

    def contexts():
        return [blm.BLM(int(off[-1]), off, nk, 0, sh, ns, precision=prec) for off, nk, sh, ns, _ in PROBLEMS]

    single, batched = contexts(), contexts()
    for c, d in zip(single, data):
        c.begin_step()
        c.build([d])
    b = blm.Batch(batched)
    for c in batched:
        c.begin_step()
    b.build([[d] for d in data])
    torch.cuda.synchronize()
    worst = 0.0
    for (off, _, sh, _, _), c1, c2 in zip(PROBLEMS, single, batched):
        for blk in range(len(off) - 1):
            H1, S1 = c1.block_matrices(blk, 0)
            H2, S2 = c2.block_matrices(blk, 0)
            worst = max(worst, _rel(S2, S1), _rel(H2, H1))
    print(f"[batch-build] {prec}: block matrices of the batched build within {worst:.1e} of single builds",
          flush=True)
    assert worst <= 1e-13, worst
    # the rest of the step: single contexts on their own, the batch together
    res1 = []
    for c, d in zip(single, data):
        _, k = c.solve()
        c.project([d])
        u, en, _, _ = c.stage2()
        res1.append((u.cpu().numpy(), en, k))
    kept2 = [k for _, k in b.solve()]
    for c, d in zip(batched, data):
        c.project([d])
    out2 = b.stage2()
    torch.cuda.synchronize()
    for q, ((u1, e1, k1), (u2, e2, _, _), k2) in enumerate(zip(res1, out2, kept2)):
        assert np.array_equal(k1, k2), (q, k1, k2)
        u2 = u2.cpu().numpy()
        for s in range(len(e1)):
            assert abs(e1[s] - e2[s]) <= 1e-10 * abs(e1[s]), (q, s, e1[s], e2[s])
            assert _cos(u1[s], u2[s]) >= 1 - 1e-10, (q, s)
    b.close()
    for c in single + batched:
        c.close()


@pytest.mark.timeout(600)
def test_eight_problems_in_one_build_launch():
    from paper_1702_01481_amd import blm
    ns = 16_384
    ws = synth.batched_workloads(n_samples=ns)
    data = []
    for w in ws:
        g = synth.SampleGenerator(w.n_params, w.rank, w.seed, sigma_E=w.sigma_E, device="cuda")
        data.append(g.chunk(0, ns))
        del g
    torch.cuda.synchronize()

    def contexts():
        return [blm.BLM(w.n_params, w.block_offsets, w.n_keep, w.n_old, w.shifts, ns) for w in ws]

    single, batched = contexts(), contexts()
    b = blm.Batch(batched)
    times = {}
    for rep in range(2):           # the second pass is timed
        for c in single + batched:
            c.begin_step()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for c, d in zip(single, data):
            c.build([d])
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        b.build([[d] for d in data])
        torch.cuda.synchronize()
        t2 = time.perf_counter()
        times = {"single": (t1 - t0) * 1e3, "batched": (t2 - t1) * 1e3}
    worst = 0.0
    for w, c1, c2 in zip(ws, single, batched):
        for blk in range(w.n_blocks):
            H1, S1 = c1.block_matrices(blk, 0)
            H2, S2 = c2.block_matrices(blk, 0)
            worst = max(worst, _rel(S2, S1), _rel(H2, H1))
    print(f"[batch-build] eight problems, {sum(w.n_blocks for w in ws)} blocks, {ns} samples each: eight builds "
          f"{times['single']:.1f} ms, one batched build {times['batched']:.1f} ms; matrices within {worst:.1e}",
          flush=True)
    assert worst <= 1e-13, worst
    b.close()
    for c in single + batched:
        c.close()


def test_mixed_storages_refuse_a_batched_build():
    from paper_1702_01481_amd import blm
    off, nk, sh, ns, _ = PROBLEMS[1]
    (O, e, EL), = _data(PROBLEMS[1:2])
    a = blm.BLM(int(off[-1]), off, nk, 0, sh, ns)
    c = blm.BLM(int(off[-1]), off, nk, 0, sh, ns, precision="bf16x3")
    b = blm.Batch([a, c])
    a.begin_step()
    c.begin_step()
    with pytest.raises(blm.BLMError) as ei:
        b.build([[(O, e, EL)], [(blm.SplitSamples(O, 3), blm.SplitSamples(e, 3), EL)]])
    assert ei.value.status == 1
    b.close()
    a.close()
    c.close()
