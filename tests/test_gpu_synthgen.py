"""The on-device generator of the banded-G synthetic model (input generator
of the 30,000-parameter workload, not part of the method): its chunks are
reproducible and independent, and the bytes it writes follow the model it
states, checked from the bytes themselves on the host:

    O_s = mu + L z_s + 0.1 xi_s,  E_L,s = -10 + a.(O_s - mu) + sigma_E eps_s,
    e_s = E_L,s O_s + G (O_s - mu) + 0.05 eta_s  (G banded)."""
import numpy as np
import pytest
import torch

from paper_1702_01481_amd import synth

pytestmark = pytest.mark.gpu


def _gen(n_params=3000, rank=32, band=8, seed=3):
    return synth.SampleGenerator(n_params, rank, seed, sigma_E=0.5, device="cuda", band=band)


def test_chunks_are_reproducible_and_distinct():
    g = _gen()
    print("synthgen: chunks 0, 0, 1 of 1,000 x 3,000", flush=True)
    a = [t.cpu().numpy() for t in g.chunk(0, 1000)]
    b = [t.cpu().numpy() for t in g.chunk(0, 1000)]
    c = [t.cpu().numpy() for t in g.chunk(1, 1000)]
    for x, y in zip(a, b):
        assert np.array_equal(x, y)
    for x, z in zip(a, c):
        assert not np.array_equal(x, z)
    # a shorter chunk is the prefix of the longer one (draws are addressed by sample)
    p = [t.cpu().numpy() for t in g.chunk(0, 333)]
    for x, y in zip(a, p):
        assert np.array_equal(x[:333], y)


def test_written_samples_follow_the_model():
    g = _gen()
    n = 16384
    print(f"synthgen: moments of a {n} x 3,000 chunk", flush=True)
    O, e, EL = (t.cpu().numpy() for t in g.chunk(5, n))
    mu, L, a = g.mu.cpu().numpy(), g.L.cpu().numpy(), g.a.cpu().numpy()
    gband = g.gband.cpu()
    dO = O - mu
    # noise of e: what is left after the model's deterministic part
    eta = e - EL[:, None] * O - synth.band_matvec(gband, torch.from_numpy(dO)).numpy()
    assert abs(eta.std() / 0.05 - 1) < 0.01, eta.std()
    assert abs(eta.mean()) < 1e-3
    # noise of E_L
    eps = EL - (-10.0 + dO @ a)
    assert abs(eps.std() / 0.5 - 1) < 0.03, eps.std()
    assert abs(eps.mean()) < 0.02
    # O - mu has covariance L L^T + 0.01 I: compare the trace and a projection
    cov_tr = (dO * dO).sum() / n
    assert abs(cov_tr / (np.sum(L * L) + 0.01 * O.shape[1]) - 1) < 0.02
    v = L[:, 0] / np.linalg.norm(L[:, 0])
    var_v = np.mean((dO @ v) ** 2)
    assert abs(var_v / (v @ L @ L.T @ v + 0.01) - 1) < 0.05
    # normality of the xi-driven part: the component of O - mu orthogonal to
    # L's columns is 0.1 xi projected; its fraction within one sigma
    Q, _ = np.linalg.qr(L)
    resid = dO[:2000] - (dO[:2000] @ Q) @ Q.T
    frac = np.mean(np.abs(resid) < 0.1)
    assert abs(frac - 0.6827) < 0.01, frac
