"""Whole-step parity of the library's FP64 step with the oracle's own step.

Both sides get the same sample bytes (the device chunks, copied to the host
once) and each runs the whole method by itself (Sec. II.B): the oracle's
block estimates (Eq. 3 on the Eq. 10 basis), its shifted block solves and
kept directions (Eq. 5, Eq. 6), its second pass and stage-two solve (Eq. 7,
Eq. 8).  With a previous direction, both run the two-step protocol on their
own: step one without history at the middle shift, whose updates are
compared (relative difference <= 1e-9).  Step two, the one compared in
full, then takes the oracle's step-one update as its previous direction
(Eq. 9) on both sides: the two step-one updates differ by about 1e-11, and
the Theta columns built from them would carry that difference into the
block matrices.  Nothing the library computes enters the oracle.

Compared, at the FP64 tolerances:
* every block's full S_b and H_b: relative Frobenius error <= 1e-12;
* the number of directions each block keeps at each shift: equal;
* each block's kept span (the projector B^T B): within a bound derived from
  the oracle's own spectrum (below);
* the stage-two matrices, after mapping the library's direction basis onto
  the oracle's (each side orthonormalises its own kept vectors, so the bases
  of a span may differ by a rotation within it);
* energy per shift: relative error <= 1e-10; update cosine >= 1 - 1e-9.

Span bound.  A relative perturbation eta of the pencil moves an invariant
subspace by about eta kappa(S) ||H|| / gap, with gap the distance from the
kept eigenvalues to the rest (first-order perturbation of a separated
spectral set).  With eta = 1e-12 (the matrix tolerance) and a factor 100
for the non-normal eigenvector conditioning, the bound is
1e-10 kappa(S_b) ||H_b + delta P_b||_F / gap_b, and never below 1e-10.
"""
from __future__ import annotations

import numpy as np
import torch

from oracle import blm_oracle as orc

MAT_TOL = 1e-12
ENERGY_TOL = 1e-10
COS_TOL = 1e-9


def host_copy(chunks):
    """The device chunks' bytes on the host, once: [(O, e, EL, None)]."""
    out = []
    for O, e, EL in chunks:
        out.append((O.cpu().numpy(), e.cpu().numpy(), EL.cpu().numpy(), None))
    torch.cuda.synchronize()
    return out


def gpu_step(ctx, chunks, old):
    ctx.begin_step(old)
    ctx.build(chunks)
    ev, kept = ctx.solve()
    ctx.project(chunks)
    upd, en, _, _ = ctx.stage2()
    torch.cuda.synchronize()
    return upd.cpu().numpy(), np.asarray(en), kept


def _rel(a, b):
    return np.linalg.norm(a - b) / np.linalg.norm(b)


def _span_bound(res, prob, delta, kappa):
    """1e-10 kappa(S) ||H + delta P|| / gap, at least 1e-10 (module doc; the
    Frobenius norm stands in for the spectral norm, which it bounds)."""
    lam = res.evals
    rest_mask = np.ones(len(lam), dtype=bool)
    rest_mask[list(res.used)] = False
    kept, rest = lam[list(res.used)], lam[rest_mask]
    if len(rest) == 0 or len(kept) == 0:
        return 1e-10
    gap = np.min(np.abs(kept[:, None] - rest[None, :]))
    nH = np.linalg.norm(prob.H + delta * prob.P)
    return max(1e-10, 1e-10 * kappa * nH / max(gap, 1e-300))


def compare_step(tag, ctx, offsets, shifts, n_keep, gpu, oracle_out, probs, log=print):
    """gpu = (update [n_shifts][N_V], energies, kept [n_shifts][N_B]) of the
    library's step in ctx; oracle_out, probs from orc.blm_step on the same
    samples and history.  Asserts the module's tolerances."""
    upd, en, kept = gpu
    nb = len(offsets) - 1
    worst = 0.0
    for b in range(nb):
        H, S = ctx.block_matrices(b, 0)
        H_un = H - shifts[0] * probs[b].P
        eS, eH = _rel(S, probs[b].S), _rel(H_un, probs[b].H)
        worst = max(worst, eS, eH)
        assert eS <= MAT_TOL and eH <= MAT_TOL, (tag, b, eS, eH)
    log(f"[whole-step] {tag}: all {nb} block matrices within {worst:.2e} of the oracle's")
    kappas = []
    for b in range(nb):
        ev = np.linalg.eigvalsh(probs[b].S)
        kappas.append(ev[-1] / max(ev[0], 1e-300))
    for si, delta in enumerate(shifts):
        res = oracle_out[si]
        span_worst, span_tol_min = 0.0, np.inf
        Bg_all = []
        for b in range(nb):
            Bo = res.blocks[b].B
            assert kept[si][b] == Bo.shape[0], (tag, si, b, kept[si][b], Bo.shape[0])
            Bg = ctx.directions(b, si)
            Bg_all.append(Bg)
            tol = _span_bound(res.blocks[b], probs[b], delta, kappas[b])
            dev = np.abs(Bg.T @ Bg - Bo.T @ Bo).max()
            assert dev <= tol, (tag, si, b, dev, tol)
            span_worst = max(span_worst, dev)
            span_tol_min = min(span_tol_min, tol)
        # stage two: the library's matrices in the oracle's direction basis
        H2, S2 = ctx.stage2_matrices(si)
        n2 = H2.shape[0]
        T = np.zeros((n2, n2))
        T[0, 0] = 1.0
        at = 1
        for b in range(nb):
            k = Bg_all[b].shape[0]
            T[at:at + k, at:at + k] = res.blocks[b].B @ Bg_all[b].T
            at += k
        e2S = _rel(T @ S2 @ T.T, res.S2)
        e2H = _rel(T @ H2 @ T.T, res.H2)
        st = res.step
        e_rel = abs(en[si] - st.energy) / abs(st.energy)
        cos = upd[si] @ st.dmu / (np.linalg.norm(upd[si]) * np.linalg.norm(st.dmu))
        log(f"[whole-step] {tag} shift {delta:g}: kept spans within {span_worst:.2e} (tightest bound "
            f"{span_tol_min:.1e}); stage-two matrices {e2S:.2e} / {e2H:.2e}; energy {en[si]:.12f} vs "
            f"{st.energy:.12f} (rel {e_rel:.1e}); update cosine 1 - {1 - cos:.1e}")
        assert max(e2S, e2H) <= max(1e-10, 10 * span_worst), (tag, si, e2S, e2H)
        assert e_rel <= ENERGY_TOL, (tag, si, e_rel)
        assert cos >= 1 - COS_TOL, (tag, si, cos)


def _source(host):
    def src():
        for i, c in enumerate(host):
            print(f"[oracle] chunk {i} of {len(host)}", flush=True)
            yield c
    return src


def _say(msg):
    print(f"[oracle] {msg}", flush=True)


def oracle_history(host, offsets, n_keep, delta):
    """The oracle's own first step without history at shift delta: its
    update, as the one previous direction [1][N_V] of the next step."""
    first, _ = orc.blm_step(_source(host), offsets, n_keep, [delta], old=None, progress=_say)
    return first[0].step.dmu[None, :].copy()


def oracle_step(host, offsets, n_keep, shifts, old):
    """The oracle's own step on the host chunks with history old (or None):
    (results per shift, block problems)."""
    return orc.blm_step(_source(host), offsets, n_keep, shifts, old=old, progress=_say)
