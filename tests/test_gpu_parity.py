"""Parity of the HIP path (through the C ABI) with the CPU oracle.

Same seeded input bytes go to both sides.  Tolerances: FP64 path, matrices
within 1e-12 relative Frobenius, energies within 1e-10 relative; kept
direction spans and the update are compared through quantities that do not
depend on the choice of basis inside a span (projectors, the update itself).
"""
import numpy as np
import pytest
import torch

from oracle import blm_oracle as orc
from paper_1702_01481_amd import synth

pytestmark = pytest.mark.gpu


def _blm():
    from paper_1702_01481_amd import blm
    return blm


def _rel(a, b):
    nb = np.linalg.norm(b)
    return np.linalg.norm(a - b) / (nb if nb > 0 else 1.0)


def _make(n_params, n_samples, rank, seed, chunk, weighted=False, sigma_E=0.5):
    g = synth.SampleGenerator(n_params, rank, seed, sigma_E=sigma_E)
    O, e, EL = g.chunk(0, n_samples)
    w = synth.weights(n_samples, seed) if weighted else None
    host, dev = [], []
    for a in range(0, n_samples, chunk):
        b = min(n_samples, a + chunk)
        wc = None if w is None else w[a:b]
        host.append((O[a:b].numpy(), e[a:b].numpy(), EL[a:b].numpy(), None if wc is None else wc.numpy()))
        dev.append((O[a:b].cuda().contiguous(), e[a:b].cuda().contiguous(), EL[a:b].cuda().contiguous(),
                    None if wc is None else wc.cuda().contiguous()))
    return host, dev


def _run_gpu(offsets, n_keep, n_old, shifts, dev_chunks, old=None, max_samples=None):
    blm = _blm()
    n_params = int(offsets[-1])
    tot = sum(c[0].shape[0] for c in dev_chunks)
    ctx = blm.BLM(n_params, offsets, n_keep, n_old, shifts, max_samples or tot)
    ctx.begin_step(None if old is None else torch.from_numpy(old).cuda().contiguous())
    ctx.build(dev_chunks)
    ev, kept = ctx.solve()
    ctx.project(dev_chunks)
    upd, en, al, fl = ctx.stage2()
    torch.cuda.synchronize()
    return ctx, ev, kept, upd.cpu().numpy(), en, al, fl


def _compare_step(offsets, n_keep, shifts, host, dev, old=None, n_old=0, mat_tol=1e-12, en_tol=1e-10):
    offsets = np.asarray(offsets)
    res, probs = orc.blm_step(lambda: host, offsets, n_keep, shifts, old=old)
    ctx, ev, kept, upd, en, al, fl = _run_gpu(offsets, n_keep, n_old, shifts, dev, old=old)
    nb = len(offsets) - 1
    for si, delta in enumerate(shifts):
        r = res[si]
        for b in range(nb):
            H, S = ctx.block_matrices(b, si)
            p = probs[b]
            assert H.shape == p.H.shape
            assert _rel(S, p.S) <= mat_tol, (b, si, _rel(S, p.S))
            assert _rel(H, p.H + delta * p.P) <= mat_tol, (b, si, _rel(H, p.H + delta * p.P))
            # the N_K + 1 lowest eigenvalues of the shifted pencil, ranked
            lam = r.blocks[b].evals[orc.rank_order(r.blocks[b].evals)][: n_keep + 1]
            got = ev[si, b, : len(lam)]
            scale = np.abs(r.blocks[b].evals).max()
            assert np.abs(got - lam).max() <= 1e-10 * scale, (b, si, got, lam)
            # kept span: same count, same projector
            B = ctx.directions(b, si)
            Bo = r.blocks[b].B
            assert B.shape == Bo.shape, (b, si, B.shape, Bo.shape)
            np.testing.assert_allclose(B @ B.T, np.eye(B.shape[0]), atol=1e-12)
            assert np.abs(B.T @ B - Bo.T @ Bo).max() < 1e-8, (b, si)
        # stage-two estimates on the GPU's own directions
        Bs = [ctx.directions(b, si) for b in range(nb)]
        H2o, S2o, _ = orc.stage2_matrices(host, offsets, Bs)
        H2, S2 = ctx.stage2_matrices(si)
        assert _rel(S2, S2o) <= mat_tol and _rel(H2, H2o) <= mat_tol, (si, _rel(S2, S2o), _rel(H2, H2o))
        # energy and update against the oracle's whole step
        assert abs(en[si] - r.step.energy) <= en_tol * abs(r.step.energy), (si, en[si], r.step.energy)
        cos = upd[si] @ r.step.dmu / (np.linalg.norm(upd[si]) * np.linalg.norm(r.step.dmu))
        assert cos > 1 - 1e-10, (si, cos)
        assert _rel(upd[si], r.step.dmu) < 1e-7, (si, _rel(upd[si], r.step.dmu))
    ctx.close()


def test_eigvals_match_lapack():
    blm = _blm()
    rng = np.random.default_rng(7)
    cases = [(d, "gauss") for d in (1, 2, 3, 5, 17, 51, 64, 65, 130, 257, 600)] + [(300, "rot")]
    for d, kind in cases:
        A = rng.standard_normal((d, d))
        S = A @ A.T / d + np.eye(d)
        if kind == "gauss":
            H = rng.standard_normal((d, d)) - 10.0 * np.eye(d)
        else:
            # mostly complex pairs: block rotations, similarity-transformed
            R = np.zeros((d, d))
            for i in range(0, d - 1, 2):
                a, b = rng.standard_normal(2)
                R[i:i + 2, i:i + 2] = [[a, b], [-b, a]]
            Q, _ = np.linalg.qr(rng.standard_normal((d, d)))
            H = Q @ R @ Q.T
        got = blm.debug_eigvals(torch.from_numpy(H).cuda(), torch.from_numpy(S).cuda())
        ref, _ = orc.generalized_eig(H, S)
        dist = np.abs(got[:, None] - ref[None, :])
        scale = np.abs(ref).max()
        assert dist.min(axis=1).max() < 1e-10 * scale, (d, kind, dist.min(axis=1).max())
        assert dist.min(axis=0).max() < 1e-10 * scale, (d, kind, dist.min(axis=0).max())


def test_small_workload_step():
    """The 200-parameter, 20,000-sample workload (4 blocks of 50, N_K = 3)."""
    w = synth.workload("small")
    host, dev = _make(w.n_params, w.n_samples, w.rank, 0, w.chunk)
    _compare_step(w.block_offsets, w.n_keep, list(w.shifts), host, dev)


@pytest.mark.parametrize("weighted", [False, True])
def test_previous_directions_ragged_chunks(weighted):
    """N_O = 1 and 2, uneven blocks, several shifts, chunks with a ragged tail."""
    offsets = [0, 37, 70, 130, 131, 200]
    host, dev = _make(200, 9000, 6, 4, 4000, weighted=weighted)
    old = synth.old_directions(2, 200, 9).numpy()
    old[1, 37:70] = 0.0                       # one dropped piece
    _compare_step(offsets, 2, [1e-4, 1e-3, 1e-2], host, dev, old=old, n_old=2)


def test_sixteen_aux_columns():
    """The most previous-step directions the library takes: 1 + N_O N_B = 16
    aux columns (five uneven blocks, N_O = 3, one piece dropped), so every
    block's pencil carries 12 Theta coordinates beside its own parameters."""
    offsets = [0, 23, 60, 61, 118, 160]
    host, dev = _make(160, 8000, 5, 8, 3000)
    old = synth.old_directions(3, 160, 21).numpy()
    old[2, 61:118] = 0.0
    _compare_step(offsets, 2, [1e-3, 1e-2], host, dev, old=old, n_old=3)


def test_uneven_blocks_with_a_large_pencil():
    """Uneven blocks as in the 40-block workload (sizes from about 100 to
    2,000): one block of 1,100 parameters (pencil dimension 1,103: QR with
    the widest early-deflation windows and 24 shifts a sweep), one previous
    direction, two shifts, and an empty chunk between two ragged ones."""
    offsets = [0, 107, 1207, 1500]
    host, dev = _make(1500, 24000, 16, 7, 13000)
    host.insert(1, tuple(None if a is None else a[:0] for a in host[0]))
    dev.insert(1, tuple(None if a is None else a[:0] for a in dev[0]))
    old = synth.old_directions(1, 1500, 5).numpy()
    _compare_step(offsets, 4, [1e-3, 1e-2], host, dev, old=old, n_old=1)


def test_multi_tile_blocks():
    """Blocks spanning several 64-wide tiles with ragged edges."""
    offsets = [0, 150, 341]
    host, dev = _make(341, 20000, 8, 5, 7777)
    old = synth.old_directions(1, 341, 2).numpy()
    _compare_step(offsets, 4, [1e-3], host, dev, old=old, n_old=1)


@pytest.mark.parametrize("weighted", [False, True])
def test_aligned_full_tiles(weighted):
    """Blocks of whole 64-wide tiles with an even leading dimension (the
    direct-to-LDS path of the build), weights, one previous direction, and
    chunks whose tails leave partial 16-sample stages."""
    offsets = [0, 128, 256, 384]
    host, dev = _make(384, 20007, 8, 6, 6151, weighted=weighted)
    old = synth.old_directions(1, 384, 4).numpy()
    _compare_step(offsets, 4, [1e-4, 1e-2], host, dev, old=old, n_old=1)


@pytest.mark.parametrize("weighted", [False, True])
def test_full_tiles_at_odd_and_even_origins(weighted):
    """Blocks starting at odd and at even columns, with an even leading
    dimension, full and ragged tiles in one launch (an odd block origin
    keeps the whole build on the general load path)."""
    offsets = [0, 65, 193, 322, 450]
    host, dev = _make(450, 20007, 8, 13, 7001, weighted=weighted)
    old = synth.old_directions(1, 450, 6).numpy()
    _compare_step(offsets, 4, [1e-3], host, dev, old=old, n_old=1)


def test_dyadic_inputs_are_bit_exact():
    """Small-integer samples: every partial sum is exact, so the block
    matrices must equal the oracle's bit for bit (N_s a power of two)."""
    n, nv = 4096, 96
    O, e, EL = synth.dyadic_chunk(n, nv, 3)
    offsets = [0, 40, 96]
    host = [(O.numpy(), e.numpy(), EL.numpy(), None)]
    dev = [(O.cuda(), e.cuda(), EL.cuda(), None)]
    blm = _blm()
    ctx = blm.BLM(nv, offsets, 2, 0, [0.0], n)
    ctx.begin_step()
    ctx.build(dev)
    D = orc.previous_directions(None, np.array(offsets))
    probs, _ = orc.block_problems(host, np.array(offsets), D)
    for b in range(2):
        H, S = ctx.block_matrices(b, 0)
        Sx = np.triu(probs[b].S) + np.triu(probs[b].S, 1).T
        assert np.array_equal(S, Sx)
        assert np.array_equal(H, probs[b].H)
    ctx.close()


def test_planted_exact_eigenstate():
    """Zero-variance model, exact enumeration, previous direction = planted
    step: the GPU path must return the planted update."""
    O, e, EL, w, delta, E0 = synth.planted_zero_variance(40, 12, 0)
    dev = [(torch.from_numpy(O).cuda().contiguous(), torch.from_numpy(e).cuda().contiguous(),
            torch.from_numpy(EL).cuda().contiguous(), torch.from_numpy(w).cuda().contiguous())]
    ctx, ev, kept, upd, en, al, fl = _run_gpu([0, 4, 8, 12], 1, 1, [0.0], dev, old=delta[None, :].copy())
    assert abs(en[0] - E0) < 1e-10 * abs(E0)
    np.testing.assert_allclose(upd[0], delta, rtol=1e-8, atol=1e-9)
    ctx.close()


def test_error_paths():
    blm = _blm()
    host, dev = _make(30, 500, 3, 1, 500)
    ctx = blm.BLM(30, [0, 15, 30], 2, 0, [1e-3], 1000)
    with pytest.raises(blm.BLMError) as ei:
        ctx.solve()
    assert ei.value.status == 2
    ctx.begin_step()
    ctx.build(dev)
    ctx.solve()
    O, e, EL, _ = dev[0]
    ctx.project([(O[:400], e[:400], EL[:400])])
    with pytest.raises(blm.BLMError) as ei:
        ctx.stage2()
    assert ei.value.status == 2
    # duplicated parameter columns: S not positive definite
    O2 = O.clone()
    O2[:, 1] = O2[:, 0]
    ctx.begin_step()
    ctx.build([(O2, e, EL)])
    with pytest.raises(blm.BLMError) as ei:
        ctx.solve()
    assert ei.value.status == 5
    # NaN in the samples
    e2 = e.clone()
    e2[3, 4] = float("nan")
    ctx.begin_step()
    ctx.build([(O, e2, EL)])
    with pytest.raises(blm.BLMError) as ei:
        ctx.solve()
    assert ei.value.status in (6, 7)
    # too many samples for the workspace
    with pytest.raises(blm.BLMError) as ei:
        ctx.begin_step()
        ctx.build([(O, e, EL), (O, e, EL), (O, e, EL)])
    assert ei.value.status == 1
    ctx.close()


def test_barrier_timeout_is_reported(monkeypatch):
    """A 301-dimensional pencil is reduced to Hessenberg form by several
    workgroups; with a poll bound of zero their first barrier gives up, every
    workgroup exits and the solve reports BLM_E_TIMEOUT.  A context with the
    default bound then solves the same samples."""
    blm = _blm()
    _, dev = _make(300, 3000, 4, 3, 3000)
    monkeypatch.setenv("BLM_SYNC_SPIN_LIMIT", "0")
    ctx = blm.BLM(300, [0, 300], 2, 0, [1e-3], 3000)
    monkeypatch.delenv("BLM_SYNC_SPIN_LIMIT")
    ctx.begin_step()
    ctx.build(dev)
    with pytest.raises(blm.BLMError) as ei:
        ctx.solve()
    assert ei.value.status == 8
    ctx.close()
    ctx = blm.BLM(300, [0, 300], 2, 0, [1e-3], 3000)
    ctx.begin_step()
    ctx.build(dev)
    ev, kept = ctx.solve()
    assert np.all(np.isfinite(ev)) and kept.min() >= 1
    ctx.close()


def test_single_workgroup_hessenberg_gives_the_same_step(monkeypatch):
    """BLM_HESS_WORKGROUPS=1 keeps every pencil on one workgroup (no
    cooperative launch); the step equals the default one's to FP64
    tolerances (only the rounding order of the reduction's sums differs)."""
    blm = _blm()
    _, dev = _make(300, 3000, 4, 5, 3000)
    out = []
    for env in (None, "1"):
        if env is None:
            monkeypatch.delenv("BLM_HESS_WORKGROUPS", raising=False)
        else:
            monkeypatch.setenv("BLM_HESS_WORKGROUPS", env)
        ctx = blm.BLM(300, [0, 300], 3, 0, [1e-3], 3000)
        monkeypatch.delenv("BLM_HESS_WORKGROUPS", raising=False)
        ctx.begin_step()
        ctx.build(dev)
        ev, kept = ctx.solve()
        ctx.project(dev)
        upd, en, _, _ = ctx.stage2()
        torch.cuda.synchronize()
        out.append((ev, kept, upd.cpu().numpy(), en))
        ctx.close()
    (ev1, k1, u1, e1), (ev2, k2, u2, e2) = out
    assert np.array_equal(k1, k2)
    assert np.abs(ev1 - ev2).max() <= 1e-10 * np.abs(ev1).max()
    assert abs(e1[0] - e2[0]) <= 1e-10 * abs(e1[0])
    assert u1[0] @ u2[0] / (np.linalg.norm(u1[0]) * np.linalg.norm(u2[0])) >= 1 - 1e-10


# --------------------------------------------------------- mixed precision --

def test_pack_bf16_split_is_accurate():
    blm = _blm()
    rng = np.random.default_rng(3)
    x = rng.standard_normal((37, 21)) * np.exp(rng.uniform(-8, 8, size=(37, 21)))
    for pieces, tol in ((3, 2.0 ** -22), (2, 2.0 ** -14)):
        sp = blm.SplitSamples(torch.from_numpy(x).cuda(), pieces)
        torch.cuda.synchronize()
        y = sp.to_numpy()
        assert np.all(np.abs(y - x) <= tol * np.abs(x)), (pieces, np.max(np.abs(y - x) / np.abs(x)))


@pytest.mark.parametrize("precision", ["bf16x3", "bf16x2"])
def test_mixed_build_is_exact_on_small_integers(precision):
    """Integers in [-7, 7] are exact in one BF16 piece and every partial sum
    is exact in FP32: the mixed build's parameter block and the rows and
    columns of the wave function (whose aux values 1 and E_L are integers
    too) must equal the oracle bit for bit.  The Theta columns (projections
    onto a previous direction, not integers) carry the pieces' precision:
    24 significant bits with three pieces, 16 with two."""
    blm = _blm()
    n, nv = 4096, 160
    O, e, EL = synth.dyadic_chunk(n, nv, 8)
    offsets = [0, 70, 160]
    host = [(O.numpy(), e.numpy(), EL.numpy(), None)]
    pieces = 3 if precision == "bf16x3" else 2
    dev = [(blm.SplitSamples(O.cuda(), pieces), blm.SplitSamples(e.cuda(), pieces), EL.cuda())]
    old = synth.dyadic_chunk(1, nv, 9)[0].numpy()
    ctx = blm.BLM(nv, offsets, 2, 1, [0.0], n, precision=precision)
    ctx.begin_step(torch.from_numpy(old).cuda())
    ctx.build(dev)
    D = orc.previous_directions(old, np.array(offsets))
    probs, _ = orc.block_problems(host, np.array(offsets), D)
    for b in range(2):
        H, S = ctx.block_matrices(b, 0)
        M = offsets[b + 1] - offsets[b]
        Sx = np.triu(probs[b].S) + np.triu(probs[b].S, 1).T
        # parameter block and the wave function's row and column: exact
        assert np.array_equal(S[1:1 + M, 1:1 + M], Sx[1:1 + M, 1:1 + M])
        assert np.array_equal(H[1:1 + M, 1:1 + M], probs[b].H[1:1 + M, 1:1 + M])
        assert np.array_equal(S[0, :1 + M], Sx[0, :1 + M])
        assert np.array_equal(H[0, :1 + M], probs[b].H[0, :1 + M])
        assert np.array_equal(H[:1 + M, 0], probs[b].H[:1 + M, 0])
        # Theta rows and columns: the pieces' precision
        tol = 1e-7 if pieces == 3 else 1e-4
        assert _rel(S, Sx) < tol and _rel(H, probs[b].H) < tol, (_rel(S, Sx), _rel(H, probs[b].H))
    ctx.close()


@pytest.mark.parametrize("precision,en_tol,cos_tol", [("bf16x3", 1e-6, 1e-6), ("bf16x2", 1e-4, 1e-4)])
def test_mixed_step_against_fp64_oracle(precision, en_tol, cos_tol):
    """Mixed precision on the 200-parameter workload: energy within en_tol
    relative of the FP64 oracle, update cosine above 1 - cos_tol."""
    blm = _blm()
    w = synth.workload("small")
    host, dev = _make(w.n_params, w.n_samples, w.rank, 0, w.chunk)
    shifts = [1e-3, 1e-2]
    res, probs = orc.blm_step(lambda: host, w.block_offsets, w.n_keep, shifts)
    pieces = 3 if precision == "bf16x3" else 2
    sdev = [(blm.SplitSamples(O, pieces), blm.SplitSamples(e, pieces), EL) for O, e, EL, _ in dev]
    ctx = blm.BLM(w.n_params, w.block_offsets, w.n_keep, 0, shifts, w.n_samples, precision=precision)
    ctx.begin_step()
    ctx.build(sdev)
    errs = []
    for b in range(w.n_blocks):
        H, S = ctx.block_matrices(b, 0)
        errs.append((_rel(S, probs[b].S), _rel(H, probs[b].H + shifts[0] * probs[b].P)))
    ctx.solve()
    ctx.project(sdev)
    upd, en, _, _ = ctx.stage2()
    upd = upd.cpu().numpy()
    print(precision, "max matrix rel errors (S, H):", np.max(errs, axis=0))
    for si in range(len(shifts)):
        ref = res[si].step
        rel_e = abs(en[si] - ref.energy) / abs(ref.energy)
        cos = upd[si] @ ref.dmu / (np.linalg.norm(upd[si]) * np.linalg.norm(ref.dmu))
        print(precision, "shift", shifts[si], "energy rel err", rel_e, "update cosine", cos)
        assert rel_e <= en_tol, (si, rel_e)
        assert cos >= 1 - cos_tol, (si, cos)
    ctx.close()


def test_autotuned_build_gives_the_same_step():
    """blm_autotune_build leaves the step's estimates alone and changes only
    how the build splits the sample axis; the build that follows sums the
    same terms in another grouping (FP64 tolerances against the default)."""
    blm = _blm()
    host, dev = _make(300, 70_000, 4, 6, 35_000)
    out = []
    for tune in (False, True):
        ctx = blm.BLM(300, [0, 100, 300], 3, 0, [1e-3], 70_000)
        ctx.begin_step()
        if tune:
            g = ctx.autotune(dev)
            assert g >= 1
            ctx.build(dev[:1])                  # tuning between builds is allowed too
            assert ctx.autotune(dev[1:]) >= 1
            ctx.build(dev[1:])
        else:
            ctx.build(dev)
        ctx.solve()
        ctx.project(dev)
        upd, en, _, _ = ctx.stage2()
        torch.cuda.synchronize()
        out.append((ctx.block_matrices(1, 0), upd.cpu().numpy(), en))
        ctx.close()
    (m1, u1, e1), (m2, u2, e2) = out
    assert _rel(m2[0], m1[0]) <= 1e-13 and _rel(m2[1], m1[1]) <= 1e-13
    assert abs(e1[0] - e2[0]) <= 1e-10 * abs(e1[0])
    assert u1[0] @ u2[0] / (np.linalg.norm(u1[0]) * np.linalg.norm(u2[0])) >= 1 - 1e-10
    ctx = blm.BLM(300, [0, 100, 300], 3, 0, [1e-3], 70_000)
    with pytest.raises(blm.BLMError) as ei:
        ctx.autotune(dev)                       # before blm_begin_step
    assert ei.value.status == 2
    ctx.close()


@pytest.mark.parametrize("precision", ["bf16x3", "fp8"])
def test_autotuned_mixed_build_gives_the_same_matrices(precision):
    """The tuned slice-group count of the BF16 and FP8 pair kernels regroups
    their FP64 sums of FP32 partials only: every block matrix equals the
    default build's to 1e-12 in relative Frobenius norm."""
    blm = _blm()
    _, dev = _make(300, 70_000, 4, 7, 35_000)
    if precision == "fp8":
        data = [(blm.Fp8Samples(O), blm.Fp8Samples(e), EL) for O, e, EL, _ in dev]
    else:
        data = [(blm.SplitSamples(O, 3), blm.SplitSamples(e, 3), EL) for O, e, EL, _ in dev]
    mats = []
    for tune in (False, True):
        ctx = blm.BLM(300, [0, 100, 300], 3, 0, [1e-3], 70_000, precision=precision)
        ctx.begin_step()
        if tune:
            assert ctx.autotune(data) >= 1
        ctx.build(data)
        ctx.solve()
        torch.cuda.synchronize()
        mats.append([ctx.block_matrices(b, 0) for b in range(2)])
        ctx.close()
    for (H1, S1), (H2, S2) in zip(*mats):
        assert _rel(H2, H1) <= 1e-12 and _rel(S2, S1) <= 1e-12, (_rel(H2, H1), _rel(S2, S1))
