"""Pins of the oracle's excited-state target (Omega = <(omega - H)> /
<(omega - H)^2>, Sec. III.D; the BLM on it, Sec. II.B): what the
definition and the mathematics fix, on the CPU.

* Brute force: per-sample loops over the definition of the two estimates.
* Expansion: A = omega S - H^T and B = omega^2 S - omega (H + H^T) + E with
  the energy LM's S, H and E = sum w ebar ebar^T.
* Exact eigenstates (strong zero variance): a model whose tangent space holds
  the first excited state phi_1 returns it with lambda = 1/(omega - E_1) for
  omega inside the gap, from sampled states; with omega below the spectrum
  the ground state instead, with lambda = 1/(omega - E_0).
* A planted mistake, (omega - H) applied to the right function (omega S - H
  instead of omega S - H^T), breaks the sampled zero-variance pin.
* The BLM on Omega reduces to the LM on Omega: one block; every direction
  kept; Theta holding the LM step (the fixed point).
"""
import numpy as np

from oracle import blm_oracle as orc
from paper_1702_01481_amd import synth


def _rel(a, b):
    return np.linalg.norm(a - b) / np.linalg.norm(b)


def test_brute_force_definition():
    rng = np.random.default_rng(0)
    n, m, omega = 6, 3, -9.5
    O = rng.normal(size=(n, m))
    e = rng.normal(size=(n, m))
    EL = rng.normal(size=n) - 10
    w = rng.uniform(0.5, 1.5, size=n)
    A, B, W = orc.omega_lm_matrices([(O, e, EL, w)], omega)
    Ab = np.zeros((m + 1, m + 1))
    Bb = np.zeros((m + 1, m + 1))
    for s in range(n):
        ob = [1.0] + list(O[s])
        eb = [EL[s]] + list(e[s])
        for i in range(m + 1):
            fi = omega * ob[i] - eb[i]
            for j in range(m + 1):
                fj = omega * ob[j] - eb[j]
                Ab[i, j] += w[s] * fi * ob[j]
                Bb[i, j] += w[s] * fi * fj
    Ab /= w.sum()
    Bb /= w.sum()
    assert abs(W - w.sum()) <= 1e-14 * W
    np.testing.assert_allclose(A, Ab, rtol=1e-13, atol=1e-13)
    np.testing.assert_allclose(B, Bb, rtol=1e-13, atol=1e-13)
    assert np.allclose(B, B.T) and np.linalg.eigvalsh(B).min() > 0


def test_expansion_in_the_energy_estimates():
    O, e, EL, w, _, ev = synth.planted_eigenstate(30, 8, 1, 1, 500)
    omega = 0.5 * (ev[0] + ev[1])
    A, B, _ = orc.omega_lm_matrices([(O, e, EL, w)], omega)
    H, S, W = orc.lm_matrices([(O, e, EL, w)])
    Y = np.hstack([EL[:, None], e])
    E = (Y * w[:, None]).T @ Y / W
    np.testing.assert_allclose(A, omega * S - H.T, rtol=0, atol=1e-12 * np.abs(A).max())
    np.testing.assert_allclose(B, omega ** 2 * S - omega * (H + H.T) + E, rtol=0, atol=1e-11 * np.abs(B).max())


def test_planted_excited_state_is_returned_from_samples():
    O, e, EL, w, delta, ev = synth.planted_eigenstate(40, 12, 3, 1, 3000)
    omega = 0.5 * (ev[0] + ev[1])
    A, B, _ = orc.omega_lm_matrices([(O, e, EL, w)], omega)
    st = orc.lm_step(A, B, 0.0)
    assert abs(st.energy - 1 / (omega - ev[1])) <= 1e-10 * abs(st.energy)
    assert _rel(st.dmu, delta) <= 1e-10


def test_omega_below_the_spectrum_targets_the_ground_state():
    O, e, EL, w, delta, ev = synth.planted_eigenstate(40, 12, 3, 0, 3000)
    omega = ev[0] - 1.0
    A, B, _ = orc.omega_lm_matrices([(O, e, EL, w)], omega)
    st = orc.lm_step(A, B, 0.0)
    assert abs(st.energy - 1 / (omega - ev[0])) <= 1e-10 * abs(st.energy)
    assert _rel(st.dmu, delta) <= 1e-10


def test_pin_catches_omega_applied_to_the_right_function():
    O, e, EL, w, delta, ev = synth.planted_eigenstate(40, 12, 3, 1, 3000)
    omega = 0.5 * (ev[0] + ev[1])
    _, B, _ = orc.omega_lm_matrices([(O, e, EL, w)], omega)
    H, S, _ = orc.lm_matrices([(O, e, EL, w)])
    wrong = orc.lm_step(omega * S - H, B, 0.0)
    assert _rel(wrong.dmu, delta) > 1e-4


def _noisy(n_params=24, n_samples=4000, seed=5):
    gen = synth.SampleGenerator(n_params, 4, seed, sigma_E=0.5)
    O, e, EL = (t.numpy() for t in gen.chunk(0, n_samples))
    return [(O, e, EL, None)]


def test_blm_on_omega_reduces_to_the_lm():
    chunks = _noisy()
    n = chunks[0][0].shape[1]
    omega, delta = -11.0, 1e-3          # a real lowest eigenvalue (the fixed point needs one)
    A, B, _ = orc.omega_lm_matrices(chunks, omega)
    lm = orc.lm_step(A, B, delta)
    # one block
    r, _ = orc.omega_blm_step(lambda: chunks, [0, n], 2, [delta], omega)
    assert abs(r[0].step.energy - lm.energy) <= 1e-10 * abs(lm.energy)
    assert _rel(r[0].step.dmu, lm.dmu) <= 1e-8
    # every direction kept
    offs = [0, 7, 15, n]
    r, _ = orc.omega_blm_step(lambda: chunks, offs, n, [delta], omega)
    assert abs(r[0].step.energy - lm.energy) <= 1e-10 * abs(lm.energy)
    assert _rel(r[0].step.dmu, lm.dmu) <= 1e-8
    # Theta holding the LM step: the fixed point
    r, _ = orc.omega_blm_step(lambda: chunks, offs, 1, [delta], omega, old=lm.dmu[None, :])
    assert abs(r[0].step.energy - lm.energy) <= 1e-10 * abs(lm.energy)
    assert _rel(r[0].step.dmu, lm.dmu) <= 1e-8
    # and a plain BLM step (one direction per block, no history) is not the LM step
    r, _ = orc.omega_blm_step(lambda: chunks, offs, 1, [delta], omega)
    assert _rel(r[0].step.dmu, lm.dmu) > 1e-6
