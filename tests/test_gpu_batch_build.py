"""One Gram launch for the block builds of several independent optimisations
(blm_batch_build), and one projection launch plus one stage-two Gram launch
for their projections (blm_batch_project): every context's jobs in one
launch, each reading its own context's chunks (Eq. 3 and Eq. 7 for each
context on its own).

* Three contexts of different shapes (one to three blocks, one or two
  shifts), in FP64, BF16 x3 and FP8 with two residuals: every block matrix
  of the batched build, and every stage-two matrix of the batched
  projection, equals the context's own up to the order of the FP64 sums
  over slice groups (relative Frobenius 1e-13); the whole batched step
  gives the same energies (1e-10 relative) and updates (cosine 1 - 1e-10).
* The eight-problem workload (N_V from 2,000 to 20,000, 78,000 parameters)
  at 16,384 samples per problem: batched build and projection against eight
  of each (1e-13), with both timed and printed.
* A batch of contexts with different storages refuses a batched build and
  a batched projection.
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
    torch.cuda.synchronize()
    kept2 = [k for _, k in b.solve()]
    b.project([[d] for d in data])
    torch.cuda.synchronize()
    worst2 = 0.0
    for (_, _, sh, _, _), c1, c2 in zip(PROBLEMS, single, batched):
        for si in range(len(sh)):
            A1, B1 = c1.stage2_matrices(si)
            A2, B2 = c2.stage2_matrices(si)
            worst2 = max(worst2, _rel(A2, A1), _rel(B2, B1))
    print(f"[batch-build] {prec}: stage-two matrices of the batched projection within {worst2:.1e}", flush=True)
    assert worst2 <= 1e-13, worst2
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
    chunk_lists = [[d] for d in data]
    t = {}

    def clock(key, fn):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        fn()
        torch.cuda.synchronize()
        t[key] = (time.perf_counter() - t0) * 1e3

    for rep in range(2):           # the second pass is timed
        for c in single + batched:
            c.begin_step()
        clock("build1", lambda: [c.build([d]) for c, d in zip(single, data)])
        clock("buildB", lambda: b.build(chunk_lists))
    worst = worst2 = 0.0
    for w, c1, c2 in zip(ws, single, batched):
        for blk in range(w.n_blocks):
            H1, S1 = c1.block_matrices(blk, 0)
            H2, S2 = c2.block_matrices(blk, 0)
            worst = max(worst, _rel(S2, S1), _rel(H2, H1))
    # the projection on its own: both sides build and solve per context, so
    # that their kept directions are the same bits (a direction's sign, or
    # its rotation within a near-degenerate pair, follows the last bits of
    # the block matrices, which the order of the batched build's sums moves)
    for rep in range(2):
        for c in single + batched:
            c.begin_step()
        for c, d in zip(single + batched, data + data):
            c.build([d])
        for c in single + batched:
            c.solve()
        clock("proj1", lambda: [c.project([d]) for c, d in zip(single, data)])
        clock("projB", lambda: b.project(chunk_lists))
    for w, c1, c2 in zip(ws, single, batched):
        for si in range(len(w.shifts)):
            A1, B1 = c1.stage2_matrices(si)
            A2, B2 = c2.stage2_matrices(si)
            worst2 = max(worst2, _rel(A2, A1), _rel(B2, B1))
    print(f"[batch-build] eight problems, {sum(w.n_blocks for w in ws)} blocks, {ns} samples each: eight builds "
          f"{t['build1']:.1f} ms, one batched build {t['buildB']:.1f} ms (matrices within {worst:.1e}); eight "
          f"projections {t['proj1']:.1f} ms, one batched projection {t['projB']:.1f} ms (within {worst2:.1e})",
          flush=True)
    assert worst <= 1e-13, worst
    assert worst2 <= 1e-13, worst2
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
    lists = [[(O, e, EL)], [(blm.SplitSamples(O, 3), blm.SplitSamples(e, 3), EL)]]
    with pytest.raises(blm.BLMError) as ei:
        b.build(lists)
    assert ei.value.status == 1
    with pytest.raises(blm.BLMError) as ei:
        b.project(lists)
    assert ei.value.status == 1
    b.close()
    a.close()
    c.close()
