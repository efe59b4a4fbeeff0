"""Plain FP64 CPU oracle of the blocked linear method (BLM).

Zhao & Neuscamman, "A Blocked Linear Method for Optimizing Large Parameter
Sets in Variational Monte Carlo", arXiv:1702.01481.

TEST INFRASTRUCTURE ONLY.  Nothing in the product path may import, call or
execute this module: only the tests, the smoke check and the CPU-baseline leg
of the benchmark use it.  It shares no code with the HIP implementation.

It is written to be read against the paper, not to be fast: NumPy FP64
matrix products accumulate the Monte Carlo estimates chunk by chunk, and
SciPy/LAPACK does the dense linear algebra.

Conventions (readings of points the paper leaves open; every one is listed
with its reason in the design notes of the repository):

* Sample quantities, per sample s: O[s, x] = <n|Psi^x>/<n|Psi>,
  e[s, x] = <n|H|Psi^x>/<n|Psi>, EL[s] = <n|H|Psi>/<n|Psi> and the weight
  w[s] = |<n|Psi>|^2 / P(n) (Eq. 3).  w=None means uniform weights.
* All matrices are divided by the total weight, so S[0, 0] = 1.
* The diagonal shift (Sec. II.A) adds delta * P to H, where P is the
  Euclidean metric of the parameter coordinates of the problem at hand:
  0 on the Psi coordinate, the identity on raw derivatives, Gram(D) on the
  previous-direction coordinates Theta (Eq. 9), B B^T on stage-two
  coordinates.  The (0, 0) element is never shifted.
* Eigenvalues are ranked by their real part (ties: larger imaginary part
  first).  A real eigenvalue contributes the real eigenvector; a complex
  conjugate pair contributes the real and imaginary parts of its eigenvector
  and is kept whole when it straddles the N_K cut.
* Kept block directions are the parameter (beta) part of those vectors,
  orthonormalised by modified Gram-Schmidt, dropping a vector whose residual
  norm falls below DROP_TOL of its own norm.

Parity status: every function here is pinned by the CPU tests (closed forms,
library routines, brute force, and the special cases in which the BLM reduces
to the traditional linear method exactly).  The generic BLM update (N_K < M_b,
noisy data, no previous direction equal to the LM step) is defined only by
the algorithm itself; it is pinned through those special cases of the same
code, not by an independent value.  The excited-state target's functions
(omega_*) are pinned the same way: brute force, the expansion in the energy
estimates, planted exact eigenstates (ground and first excited) and the
reductions of the BLM to the LM.
"""
from __future__ import annotations

from dataclasses import dataclass, field
from typing import Callable, Iterable, List, Optional, Sequence, Tuple

import numpy as np
import scipy.linalg as sla

DROP_TOL = 1e-12


# ---------------------------------------------------------------------------
# Monte Carlo estimates (Eq. 3)
# ---------------------------------------------------------------------------

def _weights(w, n):
    return np.ones(n) if w is None else np.asarray(w, dtype=np.float64)


def lm_matrices(chunks: Iterable[tuple]) -> Tuple[np.ndarray, np.ndarray, float]:
    """Traditional-LM Hamiltonian and overlap estimates on the basis
    [Psi, Psi^1 .. Psi^N_V] (Eq. 1 estimated by Eq. 3).

    H[x, y] = sum_s w_s obar_s[x] ebar_s[y],  S[x, y] = sum_s w_s obar_s[x] obar_s[y]
    with obar_s = [1, O_s] and ebar_s = [E_L,s, e_s]; both divided by sum_s w_s.
    Returns (H, S, total weight).  H is not symmetric for finite samples.
    """
    H = S = None
    W = 0.0
    for O, e, EL, w in chunks:
        n = O.shape[0]
        w = _weights(w, n)
        X = np.hstack([np.ones((n, 1)), O])
        Y = np.hstack([np.asarray(EL).reshape(n, 1), e])
        Xw = X * w[:, None]
        s_c, h_c = Xw.T @ X, Xw.T @ Y
        S = s_c if S is None else S + s_c
        H = h_c if H is None else H + h_c
        W += float(w.sum())
    return H / W, S / W, W


def mgs_rows(rows: Sequence[np.ndarray], tol: float = DROP_TOL) -> np.ndarray:
    """Modified Gram-Schmidt over the given rows, in order; a row whose
    residual norm is below tol times its original norm is dropped."""
    out: List[np.ndarray] = []
    for v in rows:
        v = np.asarray(v, dtype=np.float64)
        nv = np.linalg.norm(v)
        if nv == 0.0:
            continue
        r = v.copy()
        for q in out:
            r = r - (q @ r) * q
        nr = np.linalg.norm(r)
        if nr < tol * nv:
            continue
        out.append(r / nr)
    m = rows[0].shape[0] if len(rows) else 0
    return np.array(out).reshape(len(out), m)


def previous_directions(old: Optional[np.ndarray], offsets: np.ndarray) -> List[np.ndarray]:
    """The coefficient rows D_jk of the previous-update directions (Eq. 9).

    old[j-1] is the full update of iteration n-j (j = 1..N_O).  Theta_jk is
    block k's piece of it; each block's rows are orthonormalised (zero rows
    and dependent rows dropped).  Returns one array [n_k, M_k] per block.
    """
    nb = len(offsets) - 1
    if old is None or len(old) == 0:
        return [np.zeros((0, offsets[k + 1] - offsets[k])) for k in range(nb)]
    old = np.asarray(old, dtype=np.float64)
    return [mgs_rows([old[j, offsets[k]:offsets[k + 1]] for j in range(old.shape[0])])
            for k in range(nb)]


@dataclass
class BlockProblem:
    """Block b's estimates on the one-block basis of Eq. 4 / Eq. 10:
    [Psi, Psi^{i,b} (i = 1..M_b), Theta_jk (k != b, kept j; k-major)]."""
    H: np.ndarray
    S: np.ndarray
    P: np.ndarray          # shift metric (parameter-space Euclidean metric)
    M: int                 # M_b: parameter columns are 1 .. M
    theta: List[Tuple[int, int]] = field(default_factory=list)   # (k, j) of each Theta column


def block_problems(chunks: Iterable[tuple], offsets: np.ndarray,
                   D: List[np.ndarray]) -> Tuple[List[BlockProblem], float]:
    """Per-block H_b and S_b of Eq. 10 estimated with Eq. 3.

    For block b, obar = [1, O_{s,b}, t_{s,jk}] and ebar = [E_L,s, e_{s,b}, u_{s,jk}]
    with t_{s,jk} = D_jk . O_{s,k} and u_{s,jk} = D_jk . e_{s,k} for every
    other block k (the Theta derivative ratios follow from Eq. 9 by
    linearity).  Divided by the total weight.
    """
    nb = len(offsets) - 1
    acc_H = [None] * nb
    acc_S = [None] * nb
    W = 0.0
    for O, e, EL, w in chunks:
        n = O.shape[0]
        w = _weights(w, n)
        T = [O[:, offsets[k]:offsets[k + 1]] @ D[k].T for k in range(nb)]
        U = [e[:, offsets[k]:offsets[k + 1]] @ D[k].T for k in range(nb)]
        for b in range(nb):
            others = [k for k in range(nb) if k != b]
            X = np.hstack([np.ones((n, 1)), O[:, offsets[b]:offsets[b + 1]]] + [T[k] for k in others])
            Y = np.hstack([np.asarray(EL).reshape(n, 1), e[:, offsets[b]:offsets[b + 1]]]
                          + [U[k] for k in others])
            Xw = X * w[:, None]
            s_c, h_c = Xw.T @ X, Xw.T @ Y
            acc_S[b] = s_c if acc_S[b] is None else acc_S[b] + s_c
            acc_H[b] = h_c if acc_H[b] is None else acc_H[b] + h_c
        W += float(w.sum())
    probs = []
    for b in range(nb):
        M = int(offsets[b + 1] - offsets[b])
        theta = [(k, j) for k in range(nb) if k != b for j in range(D[k].shape[0])]
        d = 1 + M + len(theta)
        P = np.zeros((d, d))
        P[1:1 + M, 1:1 + M] = np.eye(M)
        # Gram of the Theta coefficient rows: blocks of different k have
        # disjoint support, so only same-k pairs are nonzero
        for a, (ka, ja) in enumerate(theta):
            for c, (kc, jc) in enumerate(theta):
                if ka == kc:
                    P[1 + M + a, 1 + M + c] = D[ka][ja] @ D[kc][jc]
        probs.append(BlockProblem(acc_H[b] / W, acc_S[b] / W, P, M, theta))
    return probs, W


# ---------------------------------------------------------------------------
# shifted generalized eigenproblem (Eq. 1, Eq. 5, Eq. 7, Eq. 10)
# ---------------------------------------------------------------------------

def generalized_eig(Hs: np.ndarray, S: np.ndarray) -> Tuple[np.ndarray, np.ndarray]:
    """All eigenpairs of Hs c = lambda S c with S symmetric positive definite.

    Route: S = L L^T (Cholesky), A = L^-1 Hs L^-T, A v = lambda v (LAPACK
    geev), c = L^-T v.  Raises numpy.linalg.LinAlgError if S is not positive
    definite.  Columns of the returned matrix are the eigenvectors.
    """
    L = np.linalg.cholesky(S)
    X = sla.solve_triangular(L, Hs, lower=True)            # L^-1 Hs
    A = sla.solve_triangular(L, X.T, lower=True).T          # (L^-1 (L^-1 Hs)^T)^T = L^-1 Hs L^-T
    lam, V = sla.eig(A)
    C = sla.solve_triangular(L.T, V, lower=False)
    return lam, C


def generalized_eig_qz(Hs: np.ndarray, S: np.ndarray) -> np.ndarray:
    """Eigenvalues of the same pencil by the QZ algorithm (cross-check)."""
    return sla.eigvals(Hs, S)


def rank_order(lam: np.ndarray) -> np.ndarray:
    """Indices by ascending real part; equal real parts: larger imaginary
    part first (so a conjugate pair appears as +Im then -Im)."""
    return np.lexsort((-lam.imag, lam.real))


def _phase_fix(c: np.ndarray) -> np.ndarray:
    k = int(np.argmax(np.abs(c)))
    return c * (np.conj(c[k]) / abs(c[k]))


def ranked_directions(lam: np.ndarray, C: np.ndarray, n_keep: int) -> Tuple[List[np.ndarray], List[int]]:
    """Walk the eigenpairs from the lowest real part up and collect real
    directions until at least n_keep are held (Sec. II.B: the lowest
    eigenvalues mark the best update directions).  A conjugate pair gives
    two directions, Re c and Im c, and is never split.  Returns the
    directions and the indices of the eigenvalues used."""
    order = rank_order(lam)
    dirs: List[np.ndarray] = []
    used: List[int] = []
    i = 0
    while len(dirs) < n_keep and i < len(order):
        idx = order[i]
        if lam[idx].imag == 0.0:
            dirs.append(np.real(C[:, idx]).copy())
            used.append(int(idx))
            i += 1
        else:
            c = _phase_fix(C[:, idx])
            dirs += [c.real.copy(), c.imag.copy()]
            used += [int(idx), int(order[i + 1])]
            i += 2
    return dirs, used


@dataclass
class BlockResult:
    evals: np.ndarray      # all eigenvalues of the shifted block pencil
    used: List[int]        # indices of the eigenvalues whose vectors were kept
    B: np.ndarray          # kept directions, orthonormal rows [n_b, M_b]


def solve_block(prob: BlockProblem, delta: float, n_keep: int) -> BlockResult:
    """Block b's shifted pencil (H_b + delta P_b) c = lambda S_b c, ranked;
    the beta part c[1 : 1+M_b] of the kept vectors forms B^(b) (Eq. 6)."""
    lam, C = generalized_eig(prob.H + delta * prob.P, prob.S)
    dirs, used = ranked_directions(lam, C, n_keep)
    B = mgs_rows([d[1:1 + prob.M] for d in dirs])
    return BlockResult(lam, used, B)


# ---------------------------------------------------------------------------
# stage two (Eq. 6, Eq. 7, Eq. 8)
# ---------------------------------------------------------------------------

def stage2_matrices(chunks: Iterable[tuple], offsets: np.ndarray,
                    Bs: List[np.ndarray]) -> Tuple[np.ndarray, np.ndarray, float]:
    """Eq. 7 estimates on the basis of Eq. 6: [Psi, sum_i B^(b)_ji Psi^{i,b}]
    over blocks b (block-major) and kept rows j, from a second pass over the
    same samples.  Divided by the total weight."""
    nb = len(offsets) - 1
    H = S = None
    W = 0.0
    for O, e, EL, w in chunks:
        n = O.shape[0]
        w = _weights(w, n)
        Y = np.hstack([np.ones((n, 1))] + [O[:, offsets[b]:offsets[b + 1]] @ Bs[b].T for b in range(nb)])
        Z = np.hstack([np.asarray(EL).reshape(n, 1)] + [e[:, offsets[b]:offsets[b + 1]] @ Bs[b].T for b in range(nb)])
        Yw = Y * w[:, None]
        s_c, h_c = Yw.T @ Y, Yw.T @ Z
        S = s_c if S is None else S + s_c
        H = h_c if H is None else H + h_c
        W += float(w.sum())
    return H / W, S / W, W


def stage2_metric(Bs: List[np.ndarray]) -> np.ndarray:
    """diag(0, blockdiag_b B^(b) B^(b)^T): the parameter-space metric of
    the stage-two coordinates."""
    blocks = [B @ B.T for B in Bs]
    n = 1 + sum(b.shape[0] for b in blocks)
    P = np.zeros((n, n))
    at = 1
    for g in blocks:
        m = g.shape[0]
        P[at:at + m, at:at + m] = g
        at += m
    return P


@dataclass
class StepResult:
    energy: float          # Re lambda of the chosen eigenpair
    energy_imag: float     # Im lambda (nonzero: complex lowest pair)
    dmu: np.ndarray        # parameter update [N_V]
    alpha: complex         # coefficient of Psi in the chosen eigenvector
    coeffs: np.ndarray     # full chosen eigenvector


def lowest_update(Hs: np.ndarray, S: np.ndarray) -> Tuple[complex, np.ndarray]:
    """Lowest-real-part eigenpair of Hs c = lambda S c."""
    lam, C = generalized_eig(Hs, S)
    idx = int(rank_order(lam)[0])
    return lam[idx], C[:, idx]


def stage2_solve(H2: np.ndarray, S2: np.ndarray, Bs: List[np.ndarray], offsets: np.ndarray,
                 delta: float) -> StepResult:
    """Lowest eigenvector (alpha, A) of the stage-two pencil (Eq. 7); the
    update of block b is [A B^(b)]/alpha (Eq. 8), real part."""
    P2 = stage2_metric(Bs)
    lam, c = lowest_update(H2 + delta * P2, S2)
    alpha = c[0]
    dmu = np.zeros(int(offsets[-1]))
    at = 1
    for b, B in enumerate(Bs):
        nbk = B.shape[0]
        A_b = c[at:at + nbk]
        dmu[offsets[b]:offsets[b + 1]] = np.real((A_b / alpha) @ B)
        at += nbk
    return StepResult(float(lam.real), float(lam.imag), dmu, complex(alpha), c)


# ---------------------------------------------------------------------------
# whole methods
# ---------------------------------------------------------------------------

def lm_step(H: np.ndarray, S: np.ndarray, delta: float) -> StepResult:
    """Traditional LM (Eq. 1 with the shift, Eq. 2): lowest eigenvector c of
    (H + delta P) c = lambda S c, P = diag(0, I); update c_x / c_0."""
    n = H.shape[0]
    P = np.eye(n)
    P[0, 0] = 0.0
    lam, c = lowest_update(H + delta * P, S)
    return StepResult(float(lam.real), float(lam.imag), np.real(c[1:] / c[0]), complex(c[0]), c)


@dataclass
class BLMResult:
    blocks: List[BlockResult]
    H2: np.ndarray
    S2: np.ndarray
    step: StepResult


def blm_step(chunk_source: Callable[[], Iterable[tuple]], offsets, n_keep: int,
             shifts: Sequence[float], old: Optional[np.ndarray] = None,
             progress: Optional[Callable[[str], None]] = None) -> Tuple[List[BLMResult], List[BlockProblem]]:
    """One BLM iteration per shift (Sec. II.B): block estimates (first pass
    over the samples), block solves and kept directions, stage-two estimates
    (second pass over the same samples), stage-two solve and update.
    chunk_source() must yield the same chunks each time it is called.
    progress (optional) is called with a line of text after each phase and
    each block solve; it does not change the result."""
    say = progress if progress is not None else (lambda msg: None)
    offsets = np.asarray(offsets, dtype=np.int64)
    D = previous_directions(old, offsets)
    probs, _ = block_problems(chunk_source(), offsets, D)
    say(f"block estimates of {len(probs)} blocks done")
    out = []
    for delta in shifts:
        blocks = []
        for b, p in enumerate(probs):
            blocks.append(solve_block(p, delta, n_keep))
            say(f"shift {delta:g}: block {b} (d = {p.H.shape[0]}) solved")
        Bs = [r.B for r in blocks]
        H2, S2, _ = stage2_matrices(chunk_source(), offsets, Bs)
        out.append(BLMResult(blocks, H2, S2, stage2_solve(H2, S2, Bs, offsets, delta)))
        say(f"shift {delta:g}: stage two done")
    return out, probs


# ---------------------------------------------------------------------------
# excited-state target Omega (Sec. II.B remark, Sec. III.D)
# ---------------------------------------------------------------------------
#
# Omega = <Psi|(omega - H)|Psi> / <Psi|(omega - H)^2|Psi>; with omega inside
# the gap its minimum is the first eigenstate above omega.  The BLM applies
# to it with the pencil of Eq. 1 replaced by the Omega pencil on the same
# basis: for basis functions Psi_i with sample ratios xbar_s (as obar_s for
# the energy) and ybar_s (H applied, as ebar_s), let f_s = omega xbar_s - ybar_s
# be the sample ratios of (omega - H) Psi_i.  Then
#   A_ij = <Psi_i|(omega - H)|Psi_j>   estimated as sum_s w_s f_s,i xbar_s,j
#          ((omega - H) applied to the left function),
#   B_ij = <Psi_i|(omega - H)^2|Psi_j> estimated as sum_s w_s f_s,i f_s,j,
# both divided by the total weight, and (A + delta P) c = lambda B c is solved
# for its lowest eigenvalues, lambda estimating Omega.  With the left
# application, an exact eigenstate in the span stays an exact eigenvector of
# the sampled pencil (zero variance), as H c = E S c does for the energy.

def _omega_pair(X, Y, w, omega):
    F = omega * X - Y
    Fw = F * w[:, None]
    return Fw.T @ X, Fw.T @ F


def omega_lm_matrices(chunks: Iterable[tuple], omega: float) -> Tuple[np.ndarray, np.ndarray, float]:
    """A and B of the Omega target on the basis [Psi, Psi^1 .. Psi^N_V]
    (the traditional LM's basis), divided by the total weight."""
    A = B = None
    W = 0.0
    for O, e, EL, w in chunks:
        n = O.shape[0]
        w = _weights(w, n)
        X = np.hstack([np.ones((n, 1)), O])
        Y = np.hstack([np.asarray(EL).reshape(n, 1), e])
        a_c, b_c = _omega_pair(X, Y, w, omega)
        A = a_c if A is None else A + a_c
        B = b_c if B is None else B + b_c
        W += float(w.sum())
    return A / W, B / W, W


def omega_block_problems(chunks: Iterable[tuple], offsets: np.ndarray, D: List[np.ndarray],
                         omega: float) -> Tuple[List[BlockProblem], float]:
    """Per-block Omega pencils on the basis of Eq. 10 (as block_problems):
    each BlockProblem holds A_b in place of H_b and B_b in place of S_b."""
    nb = len(offsets) - 1
    acc_A = [None] * nb
    acc_B = [None] * nb
    W = 0.0
    for O, e, EL, w in chunks:
        n = O.shape[0]
        w = _weights(w, n)
        T = [O[:, offsets[k]:offsets[k + 1]] @ D[k].T for k in range(nb)]
        U = [e[:, offsets[k]:offsets[k + 1]] @ D[k].T for k in range(nb)]
        for b in range(nb):
            others = [k for k in range(nb) if k != b]
            X = np.hstack([np.ones((n, 1)), O[:, offsets[b]:offsets[b + 1]]] + [T[k] for k in others])
            Y = np.hstack([np.asarray(EL).reshape(n, 1), e[:, offsets[b]:offsets[b + 1]]]
                          + [U[k] for k in others])
            a_c, b_c = _omega_pair(X, Y, w, omega)
            acc_A[b] = a_c if acc_A[b] is None else acc_A[b] + a_c
            acc_B[b] = b_c if acc_B[b] is None else acc_B[b] + b_c
        W += float(w.sum())
    probs = []
    for b in range(nb):
        M = int(offsets[b + 1] - offsets[b])
        theta = [(k, j) for k in range(nb) if k != b for j in range(D[k].shape[0])]
        d = 1 + M + len(theta)
        P = np.zeros((d, d))
        P[1:1 + M, 1:1 + M] = np.eye(M)
        for a, (ka, ja) in enumerate(theta):
            for c, (kc, jc) in enumerate(theta):
                if ka == kc:
                    P[1 + M + a, 1 + M + c] = D[ka][ja] @ D[kc][jc]
        probs.append(BlockProblem(acc_A[b] / W, acc_B[b] / W, P, M, theta))
    return probs, W


def omega_stage2_matrices(chunks: Iterable[tuple], offsets: np.ndarray, Bs: List[np.ndarray],
                          omega: float) -> Tuple[np.ndarray, np.ndarray, float]:
    """A2 and B2 of the Omega target on the stage-two basis of Eq. 6."""
    nb = len(offsets) - 1
    A = B = None
    W = 0.0
    for O, e, EL, w in chunks:
        n = O.shape[0]
        w = _weights(w, n)
        Y = np.hstack([np.ones((n, 1))] + [O[:, offsets[b]:offsets[b + 1]] @ Bs[b].T for b in range(nb)])
        Z = np.hstack([np.asarray(EL).reshape(n, 1)] + [e[:, offsets[b]:offsets[b + 1]] @ Bs[b].T for b in range(nb)])
        a_c, b_c = _omega_pair(Y, Z, w, omega)
        A = a_c if A is None else A + a_c
        B = b_c if B is None else B + b_c
        W += float(w.sum())
    return A / W, B / W, W


def omega_blm_step(chunk_source: Callable[[], Iterable[tuple]], offsets, n_keep: int, shifts: Sequence[float],
                   omega: float, old: Optional[np.ndarray] = None) -> Tuple[List[BLMResult], List[BlockProblem]]:
    """One BLM iteration for the Omega target per shift: the steps of
    blm_step with the Omega pencils.  step.energy is the stage-two estimate
    of Omega; BLMResult.H2 / S2 hold A2 / B2."""
    offsets = np.asarray(offsets, dtype=np.int64)
    D = previous_directions(old, offsets)
    probs, _ = omega_block_problems(chunk_source(), offsets, D, omega)
    out = []
    for delta in shifts:
        blocks = [solve_block(p, delta, n_keep) for p in probs]
        Bs = [r.B for r in blocks]
        A2, B2, _ = omega_stage2_matrices(chunk_source(), offsets, Bs, omega)
        out.append(BLMResult(blocks, A2, B2, stage2_solve(A2, B2, Bs, offsets, delta)))
    return out, probs


# ---------------------------------------------------------------------------
# storage counts quoted in the paper (Sec. II.A, Sec. II.B)
# ---------------------------------------------------------------------------

def lm_matrix_bytes(n_params: int, elem_bytes: int = 8) -> int:
    """H and S of the traditional LM, each (1 + N_V)^2 elements."""
    return 2 * (1 + n_params) ** 2 * elem_bytes


def blm_matrix_bytes(n_params: int, n_blocks: int, n_old: int, elem_bytes: int = 8) -> float:
    """Dominant BLM storage: H holds N_V^2/N_B + 2 N_V N_O (N_B - 1) elements
    (Sec. II.B); S, symmetric, needs one coupling strip: N_V^2/N_B +
    N_V N_O (N_B - 1)."""
    h = n_params ** 2 / n_blocks + 2 * n_params * n_old * (n_blocks - 1)
    s = n_params ** 2 / n_blocks + n_params * n_old * (n_blocks - 1)
    return (h + s) * elem_bytes
