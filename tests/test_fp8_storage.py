"""FP8 storage (e4m3 codes, one or two BF16 residuals, power-of-two column
scales).

CPU part: the oracle's definition of the storage is pinned to values the OCP
e4m3 format fixes (its code table, round-to-nearest-even ties, saturation),
to the scale rule, and to the error bounds that follow from the format:
2^-13 (1 + 2^-14) |x| with one residual, 2^-22 (1 + 2^-14) |x| with two (q in
its normal range; each residual is the BF16 rounding of what the previous
pieces leave, so it carries 8 more bits below a gap of about 5 bits).

GPU part (through the C ABI): the library's packer against the oracle bit
for bit, and the FP8 block build against the FP64 oracle run on the values
the storage stands for; the whole step with two residuals against the FP64
oracle at the mixed-precision tolerance (energy within 1e-6, update cosine
at least 0.9999), which one residual does not meet.
"""
import numpy as np
import pytest
import torch

from oracle import blm_oracle as orc
from oracle import fp8_storage as f8
from paper_1702_01481_amd import synth


# ------------------------------------------------------------- CPU pins ----

def test_e4m3_code_table():
    """Values fixed by the OCP e4m3 format (bias 7, 3 mantissa bits, no
    infinities, 0x7F / 0xFF NaN)."""
    assert f8.e4m3_value(0x38) == 1.0
    assert f8.e4m3_value(0x40) == 2.0
    assert f8.e4m3_value(0x3C) == 1.5
    assert f8.e4m3_value(0x7E) == 448.0
    assert f8.e4m3_value(0x08) == 2.0 ** -6          # smallest normal
    assert f8.e4m3_value(0x07) == 7 * 2.0 ** -9      # largest subnormal
    assert f8.e4m3_value(0x01) == 2.0 ** -9          # smallest subnormal
    assert f8.e4m3_value(0xB8) == -1.0
    assert f8.e4m3_value(0x80) == 0.0
    assert np.isnan(f8.e4m3_value(0x7F)) and np.isnan(f8.e4m3_value(0xFF))
    finite = [f8.e4m3_value(c) for c in range(0x7F)]
    assert len(set(finite)) == 0x7F and max(finite) == 448.0


@pytest.mark.parametrize("a,value,code", [
    (1.0625, 1.0, 0x38),        # halfway 1 / 1.125: even mantissa 0
    (1.1875, 1.25, 0x3A),       # halfway 1.125 / 1.25: even mantissa 2
    (17.0, 16.0, 0x58),         # halfway 16 / 18
    (19.0, 20.0, 0x5A),         # halfway 18 / 20
    (2.0 ** -10, 0.0, 0x00),    # halfway 0 / 2^-9
    (3 * 2.0 ** -10, 2.0 ** -8, 0x02),
    (1.01, 1.0, 0x38),
    (464.0, 448.0, 0x7E),       # beyond the largest finite value: saturate
    (1000.0, 448.0, 0x7E),
])
def test_e4m3_nearest_ties_to_even(a, value, code):
    v, c = f8.e4m3_nearest(np.array([a]))
    assert v[0] == value and c[0] == code


def test_column_scales():
    x = np.array([[448.0, 449.0, 1.0, 0.0, -3.0, 2.0 ** 200, 1e-300]])
    s = f8.column_scales(x)
    assert list(s[:5]) == [1.0, 2.0, 2.0 ** -8, 2.0 ** -126, 2.0 ** -7]
    assert s[5] == 2.0 ** 127 and s[6] == 2.0 ** -126


def test_fp8_store_error_bound():
    """|x - s (q + r)| <= 2^-13 (1 + 2^-14) |x| where q is in the normal range
    (|x| >= 2^-6 s), and <= 2^-19 s below it."""
    rng = np.random.default_rng(5)
    x = rng.standard_normal((2000, 9)) * np.exp(rng.uniform(-6, 6, size=(1, 9)))
    x[:, 3] *= np.exp(rng.uniform(-20, 0, size=2000))      # a column spanning many binades
    q, r, s = f8.fp8_store(x)
    y = f8.fp8_values(q, r, s)
    s64 = s.astype(np.float64)
    normal = np.abs(x) >= 2.0 ** -6 * s64
    bound = np.where(normal, 2.0 ** -13 * (1 + 2.0 ** -14) * np.abs(x), 2.0 ** -19 * s64 + 0 * x)
    assert np.all(np.abs(y - x) <= bound)
    assert np.all(np.abs(x) / s64 <= 448.0)
    assert np.all(np.log2(s) == np.round(np.log2(s)))
    assert not np.any((q & 0x7F) == 0x7F)


def test_fp8_store_small_integers_exact():
    rng = np.random.default_rng(6)
    x = rng.integers(-7, 8, size=(300, 12)).astype(np.float64)
    q, r, s = f8.fp8_store(x)
    assert np.array_equal(f8.fp8_values(q, r, s), x)
    assert np.all(r == 0)


def test_fp8_store_two_residuals_error_bound():
    """|x - s (q + r + t)| <= 2^-22 (1 + 2^-14) |x| with q in the normal range;
    the first residual is the one-residual storage's, and t is the BF16
    rounding of the exact remainder x / s - q - r."""
    rng = np.random.default_rng(15)
    x = rng.standard_normal((3000, 9)) * np.exp(rng.uniform(-6, 6, size=(1, 9)))
    x[:, 3] *= np.exp(rng.uniform(-20, 0, size=3000))
    q, r, t, s = f8.fp8_store(x, residuals=2)
    q1, r1, s1 = f8.fp8_store(x)
    assert np.array_equal(q, q1) and np.array_equal(r, r1) and np.array_equal(s, s1)
    y = f8.fp8_values(q, r, s, t)
    s64 = s.astype(np.float64)
    normal = np.abs(x) >= 2.0 ** -6 * s64
    assert np.all(np.abs(y - x)[normal] <= 2.0 ** -22 * (1 + 2.0 ** -14) * np.abs(x)[normal])
    # t is what r leaves: exactly the remainder where that fits in BF16
    rem2 = x / s64 - f8.fp8_values(q, r, np.ones_like(s))
    assert np.all(np.abs(f8.bf16_value(t) - rem2) <= 2.0 ** -8 * np.abs(rem2) + 1e-300)


def test_fp8_store_two_residuals_small_integers_exact():
    rng = np.random.default_rng(16)
    x = rng.integers(-7, 8, size=(300, 12)).astype(np.float64)
    q, r, t, s = f8.fp8_store(x, residuals=2)
    assert np.array_equal(f8.fp8_values(q, r, s, t), x)
    assert np.all(r == 0) and np.all(t == 0)


def test_pin_catches_dropped_second_residual():
    """Two-residual storage that forgets t is caught by its error bound."""
    rng = np.random.default_rng(18)
    x = rng.standard_normal((500, 4))
    q, r, t, s = f8.fp8_store(x, residuals=2)
    y = f8.fp8_values(q, r, s)
    assert np.max(np.abs(y - x) / np.abs(x)) > 2.0 ** -22 * (1 + 2.0 ** -14)


def test_pin_catches_dropped_residual():
    """A storage that forgets the residual is caught by the error bound."""
    rng = np.random.default_rng(8)
    x = rng.standard_normal((500, 4))
    q, r, s = f8.fp8_store(x)
    y = f8.fp8_values(q, np.zeros_like(r), s)
    assert np.max(np.abs(y - x) / np.abs(x)) > 2.0 ** -13


# ---------------------------------------------------------------- GPU -------

def _blm():
    from paper_1702_01481_amd import blm
    return blm


def _rel(a, b):
    return np.linalg.norm(a - b) / np.linalg.norm(b)


@pytest.mark.gpu
@pytest.mark.parametrize("residuals", [1, 2])
def test_pack_fp8_matches_oracle_bitwise(residuals):
    """Codes, residual bits and scales of blm_pack_fp8 equal the oracle's, on
    columns of every kind (wide range, zeros, tiny, large, negative), with a
    row count that leaves the last 16-sample group ragged."""
    blm = _blm()
    rng = np.random.default_rng(11)
    n, nc = 1000 + 7, 37
    x = rng.standard_normal((n, nc)) * np.exp(rng.uniform(-12, 12, size=(1, nc)))
    x[:, 0] = 0.0
    x[:, 1] *= np.exp(rng.uniform(-30, 0, size=n))
    x[:, 2] = -np.abs(x[:, 2]) * 1e30
    x[:, 3] = 1e-30 * rng.standard_normal(n)
    x[::5, 4] = 0.0
    x[:, 5] = rng.integers(-7, 8, size=n)
    src = torch.zeros(n, nc + 3, dtype=torch.float64)
    src[:, :nc] = torch.from_numpy(x)
    pk = blm.Fp8Samples(src.cuda(), ncols=nc, residuals=residuals)
    torch.cuda.synchronize()
    parts = pk.host_parts()
    ref = f8.fp8_store(x, residuals=residuals)
    if residuals == 2:
        bad = np.argwhere(parts[2] != ref[2])
        assert bad.size == 0, (bad[:5], parts[2][tuple(bad[0])], ref[2][tuple(bad[0])])
    q, r, s = parts[0], parts[1], parts[-1]
    qo, ro, so = ref[0], ref[1], ref[-1]
    assert np.array_equal(s, so), np.nonzero(s != so)
    bad = np.argwhere(q != qo)
    assert bad.size == 0, (bad[:5], q[tuple(bad[0])], qo[tuple(bad[0])])
    bad = np.argwhere(r != ro)
    assert bad.size == 0, (bad[:5], r[tuple(bad[0])], ro[tuple(bad[0])])
    # padding rows of the last groups are zeros
    n16 = (n + 15) // 16
    qall = pk.codes.cpu().numpy().reshape(n16, pk.ld, 16).transpose(0, 2, 1).reshape(-1, pk.ld)
    assert np.all(qall[n:] == 0)


def _fp8_values_of(x: torch.Tensor, residuals: int = 1) -> np.ndarray:
    parts = f8.fp8_store(x.numpy(), residuals=residuals)
    if residuals == 1:
        return f8.fp8_values(*parts)
    q, r, t, s = parts
    return f8.fp8_values(q, r, s, t)


@pytest.mark.gpu
@pytest.mark.parametrize("prec,residuals", [("fp8", 1), ("fp8x2", 2)])
def test_fp8_build_against_oracle_on_stored_values(prec, residuals):
    """The FP8 block build (strips included, with a previous direction) on
    two ragged chunks against the FP64 oracle run on the values the storage
    stands for (the oracle's own storage of the same inputs).  What remains
    is the arithmetic of the path: every piece product is exact in FP32 and
    summed on the BF16 matrix core, partial sums are FP32 over at most 256
    samples before they go to FP64 (each rounding within 2^-24 of the
    partial: at most 256 of them, about 1.5e-5 of a partial in the worst
    case), and the aux columns' own FP8 storage of the previous-direction
    coordinates."""
    blm = _blm()
    n_params, n, rank = 200, 20000, 8
    offsets = np.array([0, 50, 100, 150, 200])
    g = synth.SampleGenerator(n_params, rank, 0)
    O, e, EL = g.chunk(0, n)
    cuts = [0, 13001, n]
    old = synth.old_directions(1, n_params, 4).numpy()
    host, dev = [], []
    for a, b in zip(cuts[:-1], cuts[1:]):
        host.append((_fp8_values_of(O[a:b], residuals), _fp8_values_of(e[a:b], residuals), EL[a:b].numpy(),
                     None))
        dev.append((blm.Fp8Samples(O[a:b].cuda().contiguous(), residuals=residuals),
                    blm.Fp8Samples(e[a:b].cuda().contiguous(), residuals=residuals), EL[a:b].cuda().contiguous()))
    ctx = blm.BLM(n_params, offsets, 3, 1, [1e-3], n, precision=prec)
    ctx.begin_step(torch.from_numpy(old).cuda())
    ctx.build(dev)
    D = orc.previous_directions(old, offsets)
    probs, _ = orc.block_problems(host, offsets, D)
    worst = 0.0
    for b in range(len(offsets) - 1):
        H, S = ctx.block_matrices(b, 0)
        p = probs[b]
        Sx = np.triu(p.S) + np.triu(p.S, 1).T
        eS, eH = _rel(S, Sx), _rel(H, p.H + 1e-3 * p.P)
        worst = max(worst, eS, eH)
        print(f"{prec} block {b}: S rel {eS:.2e}, H rel {eH:.2e}")
    ctx.close()
    assert worst < 1.5e-5, worst


@pytest.mark.gpu
@pytest.mark.parametrize("prec,residuals", [("fp8", 1), ("fp8x2", 2)])
def test_fp8_build_is_exact_on_small_integers(prec, residuals):
    """Integers in [-7, 7] are exact in e4m3 (column scale 2^-6 or 2^-8), all
    code products are multiples of 2^12 and every partial sum is an integer
    below 2^24: the FP8 build's parameter block and the wave function's row
    and column equal the oracle bit for bit."""
    blm = _blm()
    n, nv = 4096, 160
    O, e, EL = synth.dyadic_chunk(n, nv, 8)
    offsets = [0, 70, 160]
    host = [(O.numpy(), e.numpy(), EL.numpy(), None)]
    dev = [(blm.Fp8Samples(O.cuda(), residuals=residuals), blm.Fp8Samples(e.cuda(), residuals=residuals),
            EL.cuda())]
    old = synth.dyadic_chunk(1, nv, 9)[0].numpy()
    ctx = blm.BLM(nv, offsets, 2, 1, [0.0], n, precision=prec)
    ctx.begin_step(torch.from_numpy(old).cuda())
    ctx.build(dev)
    D = orc.previous_directions(old, np.array(offsets))
    probs, _ = orc.block_problems(host, np.array(offsets), D)
    for b in range(2):
        H, S = ctx.block_matrices(b, 0)
        M = offsets[b + 1] - offsets[b]
        Sx = np.triu(probs[b].S) + np.triu(probs[b].S, 1).T
        assert np.array_equal(S[1:1 + M, 1:1 + M], Sx[1:1 + M, 1:1 + M])
        assert np.array_equal(H[1:1 + M, 1:1 + M], probs[b].H[1:1 + M, 1:1 + M])
        assert np.array_equal(S[0, :1 + M], Sx[0, :1 + M])
        assert np.array_equal(H[0, :1 + M], probs[b].H[0, :1 + M])
        assert np.array_equal(H[:1 + M, 0], probs[b].H[:1 + M, 0])
        # Theta rows and columns (projections, not integers): FP8 storage precision
        assert _rel(S, Sx) < 3e-4 and _rel(H, probs[b].H) < 3e-4, (_rel(S, Sx), _rel(H, probs[b].H))
    ctx.close()


def _fp8_step(prec, residuals):
    blm = _blm()
    w = synth.workload("small")
    g = synth.SampleGenerator(w.n_params, w.rank, 0)
    O, e, EL = g.chunk(0, w.n_samples)
    host = [(O.numpy(), e.numpy(), EL.numpy(), None)]
    shifts = [1e-3, 1e-2]
    res, _ = orc.blm_step(lambda: host, w.block_offsets, w.n_keep, shifts)
    dev = [(blm.Fp8Samples(O.cuda(), residuals=residuals), blm.Fp8Samples(e.cuda(), residuals=residuals),
            EL.cuda())]
    ctx = blm.BLM(w.n_params, w.block_offsets, w.n_keep, 0, shifts, w.n_samples, precision=prec)
    ctx.begin_step()
    ctx.build(dev)
    ctx.solve()
    ctx.project(dev)
    upd, en, _, _ = ctx.stage2()
    upd = upd.cpu().numpy()
    ctx.close()
    out = []
    for si in range(len(shifts)):
        ref = res[si].step
        rel_e = abs(en[si] - ref.energy) / abs(ref.energy)
        cos = upd[si] @ ref.dmu / (np.linalg.norm(upd[si]) * np.linalg.norm(ref.dmu))
        print(f"{prec} shift {shifts[si]}: energy rel err {rel_e:.2e}, update cosine {cos:.10f}")
        out.append((rel_e, cos))
    return out


@pytest.mark.gpu
def test_fp8x2_step_meets_the_mixed_tolerance():
    """The whole step with two residuals (22-bit storage) on the
    200-parameter workload against the FP64 oracle on the original values:
    energy within 1e-6 relative and update cosine at least 0.9999 at both
    shifts."""
    for rel_e, cos in _fp8_step("fp8x2", 2):
        assert rel_e <= 1e-6, rel_e
        assert cos >= 0.9999, cos


@pytest.mark.gpu
def test_fp8_step_storage_bound():
    """With one residual the storage moves each sample value by up to 2^-13
    relative; the step stays within 1e-4 in energy and 1e-3 in cosine, the
    storage's own scale on these pencils."""
    for rel_e, cos in _fp8_step("fp8", 1):
        assert rel_e <= 1e-4, rel_e
        assert cos >= 1 - 1e-3, cos


@pytest.mark.gpu
@pytest.mark.xfail(reason="one BF16 residual stores 13 significant bits: the storage alone moves the "
                          "energy by about 1e-5 (emulated on the CPU with exact products), above the "
                          "1e-6 mixed-precision tolerance; the two-residual storage meets it",
                   strict=False)
def test_fp8_step_meets_the_mixed_tolerance():
    for rel_e, cos in _fp8_step("fp8", 1):
        assert rel_e <= 1e-6, rel_e
        assert cos >= 0.9999, cos


@pytest.mark.gpu
@pytest.mark.parametrize("residuals", [1, 2])
def test_pack_fp8_writes_only_its_residual_groups(residuals):
    """Residual arrays hold ceil(n / 8) groups of 8 samples (blm.h): with n
    such that this count is odd, the packer must not write the last 16-sample
    block's second group past the end (a regression: it did, clobbering what
    followed the array)."""
    import ctypes
    blm = _blm()
    n, nc = 6999, 40                        # ceil(n / 8) = 875, odd
    n8, n16 = (n + 7) // 8, (n + 15) // 16
    src = torch.randn(n, nc, dtype=torch.float64, device="cuda")
    codes = torch.zeros(n16 * 16 * nc, dtype=torch.uint8, device="cuda")
    guard = 4096
    res = torch.full((n8 * 8 * nc + guard,), 0x5A5A, dtype=torch.int32, device="cuda").to(torch.int16)
    res2 = torch.full((n8 * 8 * nc + guard,), 0x3C3C, dtype=torch.int32, device="cuda").to(torch.int16)
    scale = torch.zeros(nc, dtype=torch.float32, device="cuda")
    st = blm.load().blm_pack_fp8(ctypes.c_void_p(src.data_ptr()), n, nc, nc, ctypes.c_void_p(codes.data_ptr()),
                                 ctypes.c_void_p(res.data_ptr()),
                                 ctypes.c_void_p(res2.data_ptr() if residuals == 2 else None),
                                 ctypes.c_void_p(scale.data_ptr()), nc, None)
    assert st == 0
    torch.cuda.synchronize()
    assert bool((res[n8 * 8 * nc:] == 0x5A5A).all())
    assert bool((res2[n8 * 8 * nc:] == 0x3C3C).all())
    if residuals == 1:
        assert bool((res2 == 0x3C3C).all())
