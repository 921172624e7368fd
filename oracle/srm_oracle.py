"""Plain FP64 oracle of the probabilistic Shared Response Model EM sweep.

TEST INFRASTRUCTURE ONLY.  Nothing in the device library imports, links or
executes this file; only tests, the smoke check and the benchmark's CPU
baseline do.  It is deliberately slow and literal: NumPy FP64, one subject at
a time, the steps in the order of Algorithm 1 (D-SRM), each citing the
equation it follows.  Library routines (matmul, Cholesky, SVD, eigh, slogdet)
serve as steps; nothing is blocked, fused or reordered beyond what the
equations state.

Model (Sec. II-A, Eq. 1): x_it = W_i s_t + mu_i + eps_i, eps_i ~ N(0, rho_i^2 I),
s_t ~ N(0, Sigma_s), W_i^T W_i = I.

Readings of the paper used here (the paper is silent, ambiguous or garbled):
  R1  rho_i^2 update (Eq. 5 is garbled: one term lacks the 1/(T V) factor and
      V is the total voxel count).  Used: the exact maximiser of the expected
      complete-data log-likelihood for subject i,
      rho_i^2 = (c_i - 2 tr(W_i^T A_i) + t tr(Sigma_s_new)) / (t v_i),
      with c_i = ||Xhat_i||_F^2, A_i = Xhat_i S^T and the trace identity that
      follows Eq. 11.
  R2  the factor 1/2 in A_i (unnumbered line before Eq. 4) is dropped: the polar
      factor is scale invariant and R1 uses the unscaled A_i.
  R3  Sigma_s starts at I_k (Algorithm 1 states only W_i and rho_i^2 = 1).
  R4  W0_i is an explicit input (the random orthogonal start of Algorithm 1).
  R5  fixed iteration count (the stopping criterion is unspecified).
  R6  the returned S is the posterior mean of the last E-step (the one the
      final W_i were built from).
  R7  1/t after demeaning, as printed.
  R8  Sigma_s is symmetric; it is symmetrised after each update.
  R9  the log-likelihood (not given in the paper) is the marginal Gaussian
      log-density of xhat_t ~ N(0, Phi), Phi = W Sigma_s W^T + Psi, reduced with
      the inversion lemma (Eq. 7) and Eq. 8 -- see ``loglik``.
  R10 a rank-deficient A_i (lambda_min(A^T A) <= 1e-13 lambda_max) is an error.
  R11 inversions by Cholesky (Sec. II-C); a failure is an error.
  (R12 and R13 concern the device's storage format and polar method only.)
  R14 the data standardisation (z-score) named among the implementation's
      native helpers (Sec. IV-A) is taken per voxel over the samples, with the
      population standard deviation (1/t); a constant voxel (standard
      deviation 0) is only demeaned.  For float32 input the FP64 mean of a
      constant voxel is exact (its sum is an exact multiple), so "constant"
      needs no tolerance.

Pins (tests/test_oracle.py): naive V x V E-step (Eq. 2-3), the closed form
Sigma_s (I - rho0 M) = M, orthonormality, polar = SVD, the trace identity,
monotone log-likelihood, the N = 1 PPCA closed form, M-step = argmax of the
expected complete-data log-likelihood, planted recovery, rotation
equivariance, agreement with the t x t Gram form (list and streamed input
alike), the Philox generator against NumPy's implementation of the same
published generator, and the Haar start's orthonormality.
"""
from __future__ import annotations

import math
from typing import Callable, Iterable, List, Optional, Sequence

import numpy as np
import scipy.linalg as sla


class OracleRankError(ArithmeticError):
    """A_i^T A_i is numerically singular: the polar factor is undefined."""


class OracleNotPD(ArithmeticError):
    """A k x k matrix that must be positive definite is not."""


RANK_TOL = 1e-13


def _chol(a: np.ndarray) -> np.ndarray:
    try:
        return np.linalg.cholesky(a)
    except np.linalg.LinAlgError as exc:  # R11
        raise OracleNotPD(str(exc)) from exc


def demean(X: np.ndarray):
    """Algorithm 1 initialisation: mu_i = (1/T) sum_t x_it, xhat = x - mu.

    Returns (mu [v], Xhat [v x t] float64, c = ||Xhat||_F^2)."""
    X = np.asarray(X, dtype=np.float64)
    mu = X.mean(axis=1)
    Xh = X - mu[:, None]
    c = float(np.sum(Xh * Xh))  # trace(A^T A) of Sec. IV-A
    return mu, Xh, c


def zscore(X: np.ndarray):
    """Per-voxel standardisation of Sec. IV-A (R14): (x - mu) / sd with sd the
    population standard deviation over the samples.

    Returns (mu [v], Z [v x t] float64, scale [v] = 1/sd, or 1 for a constant
    voxel)."""
    X = np.asarray(X, dtype=np.float64)
    mu = X.mean(axis=1)
    D = X - mu[:, None]
    sd = np.sqrt(np.mean(D * D, axis=1))
    keep = sd > 0
    scale = np.where(keep, 1.0 / np.where(keep, sd, 1.0), 1.0)
    return mu, D * scale[:, None], scale


def posterior(Y: np.ndarray, rho2: np.ndarray, Sigma_s: np.ndarray):
    """E-step on the master (Eq. 7-10) from the reduced Y = sum rho_i^-2 W_i^T Xhat_i.

    Returns (S, M, rho0) with M = (Sigma_s^-1 + rho0 I)^-1 (Eq. 7 with Eq. 8)
    and S = Sigma_s [I - rho0 M] Y (Eq. 10)."""
    k = Sigma_s.shape[0]
    rho0 = float(np.sum(1.0 / rho2))  # Eq. 8
    L = _chol(Sigma_s)
    Sinv = sla.cho_solve((L, True), np.eye(k))  # Sigma_s^-1
    B = Sinv + rho0 * np.eye(k)  # Sigma_s^-1 + W^T Psi^-1 W, Eq. 7-8
    LB = _chol(B)
    M = sla.cho_solve((LB, True), np.eye(k))
    S = Sigma_s @ (np.eye(k) - rho0 * M) @ Y  # Eq. 10
    return S, M, rho0


def loglik(c: Sequence[float], v: Sequence[int], t: int, rho2: np.ndarray,
           Sigma_s: np.ndarray, Y: np.ndarray, M: np.ndarray, rho0: float) -> float:
    """Marginal log-likelihood of the demeaned data under the current params (R9).

    log|Phi| = sum_i v_i log rho_i^2 + log|I + rho0 Sigma_s| (determinant lemma
    with Eq. 8); sum_t xhat_t^T Phi^-1 xhat_t = sum_i c_i / rho_i^2 - tr(Y^T M Y)
    (inversion lemma, Eq. 7, with Y from Eq. 10)."""
    v = np.asarray(v, dtype=np.float64)
    c = np.asarray(c, dtype=np.float64)
    V = float(v.sum())
    k = Sigma_s.shape[0]
    _, ld = np.linalg.slogdet(np.eye(k) + rho0 * Sigma_s)
    quad = float(np.sum(c / rho2)) - float(np.sum(Y * (M @ Y)))
    return -0.5 * (t * V * math.log(2.0 * math.pi)
                   + t * float(np.sum(v * np.log(rho2))) + t * ld + quad)


def polar_svd(A: np.ndarray):
    """Eq. 4, W = A (A^T A)^-1/2, computed as U V^T of the economy SVD of A.

    Returns (W, sum of singular values = tr(W^T A))."""
    U, sig, Vt = np.linalg.svd(A, full_matrices=False)
    if sig[-1] ** 2 <= RANK_TOL * sig[0] ** 2:  # R10
        raise OracleRankError("A_i is rank deficient")
    return U @ Vt, float(sig.sum())


def m_step_subject(Xh: np.ndarray, c: float, S: np.ndarray, tau: float):
    """Per-subject M-step given the posterior mean S and tau = tr(Sigma_s_new).

    A_i = Xhat_i S^T (R2), W_i = polar(A_i) (Eq. 4),
    rho_i^2 = (c_i - 2 tr(W_i^T A_i) + t tau) / (t v_i) (R1)."""
    v, t = Xh.shape
    A = Xh @ S.T
    W, tr_wa = polar_svd(A)
    rho2 = (c - 2.0 * tr_wa + t * tau) / (t * v)
    return W, rho2


def em_fit(X: List[np.ndarray], k: int, n_iter: int, W0: List[np.ndarray],
           final_loglik: bool = False, record: bool = False,
           demeaned: bool = False):
    """Algorithm 1 (D-SRM) run serially: n_iter EM iterations from W0.

    With demeaned=True the X_i are taken as the already demeaned Xhat_i (used
    to feed the oracle exactly the values a reduced-precision store holds).
    Returns a dict with W (list), S, rho2, Sigma_s, mu, c and ll (the
    log-likelihood of the parameters entering each iteration; with
    final_loglik, one more value for the parameters leaving the last one)."""
    N = len(X)
    t = X[0].shape[1]
    mus, Xh, c = [], [], []
    for Xi in X:  # initialisation: demean per subject
        if demeaned:
            xh = np.asarray(Xi, dtype=np.float64)
            m, ci = np.zeros(xh.shape[0]), float(np.sum(xh * xh))
        else:
            m, xh, ci = demean(Xi)
        mus.append(m)
        Xh.append(xh)
        c.append(ci)
    v = [x.shape[0] for x in Xh]
    W = [np.array(w, dtype=np.float64) for w in W0]  # R4
    rho2 = np.ones(N)  # Algorithm 1: rho_i^2 = 1
    Sigma_s = np.eye(k)  # R3
    ll, trace = [], []
    S = None
    for _ in range(n_iter):  # R5
        # E-step: reduce sum_i rho_i^-2 W_i^T Xhat_i (Eq. 10, Algorithm 1)
        Y = np.zeros((k, t))
        for i in range(N):
            Y += (1.0 / rho2[i]) * (W[i].T @ Xh[i])
        S, M, rho0 = posterior(Y, rho2, Sigma_s)
        ll.append(loglik(c, v, t, rho2, Sigma_s, Y, M, rho0))
        # M-step on the master: Sigma_s (Eq. 11) and its trace
        Sigma_s = M + (S @ S.T) / t
        Sigma_s = 0.5 * (Sigma_s + Sigma_s.T)  # R8
        tau = float(np.trace(Sigma_s))
        # M-step per subject: W_i (Eq. 4) and rho_i^2 (R1)
        newW, newr = [], np.empty(N)
        for i in range(N):
            Wi, r = m_step_subject(Xh[i], c[i], S, tau)
            newW.append(Wi)
            newr[i] = r
        W, rho2 = newW, newr
        if record:
            trace.append({"S": S.copy(), "Sigma_s": Sigma_s.copy(),
                          "rho2": rho2.copy(), "M": M.copy(), "Y": Y.copy()})
    out = {"W": W, "S": S, "rho2": rho2, "Sigma_s": Sigma_s, "mu": mus,
           "c": np.array(c), "ll": ll, "v": v, "t": t}
    if final_loglik:
        Y = np.zeros((k, t))
        for i in range(N):
            Y += (1.0 / rho2[i]) * (W[i].T @ Xh[i])
        _, M, rho0 = posterior(Y, rho2, Sigma_s)
        out["ll_final"] = loglik(c, v, t, rho2, Sigma_s, Y, M, rho0)
    if record:
        out["trace"] = trace
    return out


def naive_estep(Xh: List[np.ndarray], W: List[np.ndarray], rho2: np.ndarray,
                Sigma_s: np.ndarray):
    """The original E-step (Eq. 2-3) with the full V x V Phi -- tiny inputs only.

    Returns (E[S] [k x t], sum_t E[s_t s_t^T] [k x k], log-likelihood)."""
    Wst = np.vstack(W)
    X = np.vstack(Xh)
    V, t = X.shape
    psi = np.concatenate([np.full(w.shape[0], r) for w, r in zip(W, rho2)])
    Phi = Wst @ Sigma_s @ Wst.T + np.diag(psi)
    L = np.linalg.cholesky(Phi)
    PhiInv_X = sla.cho_solve((L, True), X)
    ES = Sigma_s.T @ Wst.T @ PhiInv_X  # Eq. 2
    PhiInv_W = sla.cho_solve((L, True), Wst)
    cov = Sigma_s - Sigma_s.T @ Wst.T @ PhiInv_W @ Sigma_s  # Eq. 3, first terms
    Ess = t * cov + ES @ ES.T  # sum over t of Eq. 3
    logdet = 2.0 * np.sum(np.log(np.diag(L)))
    ll = -0.5 * (float(np.sum(X * PhiInv_X)) + t * logdet
                 + t * V * math.log(2.0 * math.pi))
    return ES, Ess, ll, cov


def gram_summary(Xi: np.ndarray, W0i: np.ndarray, demeaned: bool = False):
    """What one pass over subject i's data leaves for the t x t Gram form:
    (G_i = Xhat_i^T Xhat_i, c_i = ||Xhat_i||_F^2, v_i, W0_i^T Xhat_i).
    demeaned=True takes X_i as Xhat_i, as in em_fit."""
    if demeaned:
        xh = np.asarray(Xi, dtype=np.float64)
        ci = float(np.sum(xh * xh))
    else:
        _, xh, ci = demean(Xi)
    return xh.T @ xh, ci, xh.shape[0], np.asarray(W0i, dtype=np.float64).T @ xh


def fit_gram_summaries(summ: Iterable, k: int, n_iter: int, final_loglik: bool = False):
    """The same EM written on the t x t Gram G_i = Xhat_i^T Xhat_i.

    Exact algebra on Eq. 4, 10 and R1: with A_i = Xhat_i S^T,
    W_i^T Xhat_i = P_i S G_i and A_i^T A_i = S G_i S^T, where
    P_i = (A_i^T A_i)^-1/2 (eigh).  summ yields gram_summary() of every
    subject, in order; W_i = Xhat_i S^T P_i is left to the caller (w_of)."""
    G, c, v, Z = [], [], [], []
    for Gi, ci, vi, Z0i in summ:
        G.append(Gi)
        c.append(ci)
        v.append(vi)
        Z.append(Z0i)  # W_i^T Xhat_i for W_i = W0_i
    N = len(G)
    t = G[0].shape[0]
    rho2 = np.ones(N)
    Sigma_s = np.eye(k)
    ll = []
    P = [None] * N
    S = None
    for _ in range(n_iter):
        Y = np.zeros((k, t))
        for i in range(N):
            Y += (1.0 / rho2[i]) * Z[i]
        S, M, rho0 = posterior(Y, rho2, Sigma_s)
        ll.append(loglik(c, v, t, rho2, Sigma_s, Y, M, rho0))
        Sigma_s = M + (S @ S.T) / t
        Sigma_s = 0.5 * (Sigma_s + Sigma_s.T)
        tau = float(np.trace(Sigma_s))
        newr = np.empty(N)
        for i in range(N):
            SG = S @ G[i]
            Gk = SG @ S.T  # A_i^T A_i
            lam, U = np.linalg.eigh(Gk)
            if lam[0] <= RANK_TOL * lam[-1]:
                raise OracleRankError("A_i is rank deficient")
            P[i] = (U / np.sqrt(lam)) @ U.T
            tr_wa = float(np.sum(np.sqrt(lam)))
            newr[i] = (c[i] - 2.0 * tr_wa + t * tau) / (t * v[i])
            Z[i] = P[i] @ SG
        rho2 = newr
    out = {"S": S, "rho2": rho2, "Sigma_s": Sigma_s, "ll": ll, "c": np.array(c),
           "v": v, "t": t, "P": P}
    if final_loglik:
        Y = np.zeros((k, t))
        for i in range(N):
            Y += (1.0 / rho2[i]) * Z[i]
        _, M, rho0 = posterior(Y, rho2, Sigma_s)
        out["ll_final"] = loglik(c, v, t, rho2, Sigma_s, Y, M, rho0)
    return out


def w_of(fit: dict, i: int, Xi: np.ndarray, demeaned: bool = False) -> np.ndarray:
    """W_i = A_i P_i = Xhat_i S^T P_i of a Gram-form fit (Eq. 4)."""
    if demeaned:
        xh = np.asarray(Xi, dtype=np.float64)
    else:
        _, xh, _ = demean(Xi)
    return xh @ fit["S"].T @ fit["P"][i]


def fit_gram(X, k: int, n_iter: int, W0, final_loglik: bool = False,
             demeaned: bool = False):
    """fit_gram_summaries over lists (or iterables, read once) of X_i and W0_i;
    with X a sequence, W holds every W_i."""
    out = fit_gram_summaries((gram_summary(x, w, demeaned) for x, w in zip(X, W0)),
                             k, n_iter, final_loglik)
    if isinstance(X, Sequence):
        out["W"] = [w_of(out, i, X[i], demeaned) for i in range(len(X))]
    return out


# ---------------------------------------------------------------------------
# The random orthonormal start of Algorithm 1 when the library draws it.
#
# Algorithm 1 initialises each W_i with "a random orthogonal matrix" without
# saying how (reading R4).  When the caller passes no W0, the library and this
# oracle draw the same one: the polar factor G (G^T G)^-1/2 of a v_i x k matrix
# G of independent N(0, 1) entries, which is Haar distributed on the matrices
# with orthonormal columns (the distribution of G is invariant under
# G -> Q G for orthogonal Q, and polar(Q G) = Q polar(G)).  The Gaussian
# entries come from the counter-based generator Philox4x64-10 (Salmon, Moraes,
# Dror, Shaw, "Parallel random numbers: as easy as 1, 2, 3", SC 2011) and the
# Box-Muller transform; both sides implement them from those definitions and
# share no code.
#
# Element e = r k + b of subject i's G (row-major) is normal number e % 4 of
# the Philox block with counter (e // 4, i, 0, 0) and key (seed, 0): the block's
# 64-bit outputs x0..x3 give u_j = (floor(x_j / 2^11) + 1/2) 2^-53 and
#   z0 = sqrt(-2 ln u0) cos(2 pi u1), z1 = sqrt(-2 ln u0) sin(2 pi u1),
#   z2 = sqrt(-2 ln u2) cos(2 pi u3), z3 = sqrt(-2 ln u2) sin(2 pi u3).
# ---------------------------------------------------------------------------

_PHILOX_M = (np.uint64(0xD2E7470EE14C6C93), np.uint64(0xCA5A826395121157))
_PHILOX_W = (np.uint64(0x9E3779B97F4A7C15), np.uint64(0xBB67AE8584CAA73B))
_LO32 = np.uint64(0xFFFFFFFF)
_S32 = np.uint64(32)


def _mulhilo64(a: np.uint64, b: np.ndarray):
    """High and low 64-bit words of the 128-bit product a * b (elementwise)."""
    b = np.asarray(b, dtype=np.uint64)
    lo = a * b
    a0, a1 = a & _LO32, a >> _S32
    b0, b1 = b & _LO32, b >> _S32
    mid = a1 * b0 + ((a0 * b0) >> _S32)
    mid2 = (mid & _LO32) + a0 * b1
    hi = a1 * b1 + (mid >> _S32) + (mid2 >> _S32)
    return hi, lo


def philox4x64(counter, key):
    """Philox4x64-10: counter = 4 arrays of uint64 words (word 0 least
    significant), key = 2 uint64 words.  Returns the 4 output words."""
    c = [np.asarray(x, dtype=np.uint64) for x in counter]
    k0, k1 = np.uint64(key[0]), np.uint64(key[1])
    with np.errstate(over="ignore"):
        for _ in range(10):
            hi0, lo0 = _mulhilo64(_PHILOX_M[0], c[0])
            hi1, lo1 = _mulhilo64(_PHILOX_M[1], c[2])
            c = [hi1 ^ c[1] ^ k0, lo1, hi0 ^ c[3] ^ k1, lo0]
            k0 = k0 + _PHILOX_W[0]
            k1 = k1 + _PHILOX_W[1]
    return c


def seeded_gaussian(v: int, k: int, seed: int, i: int) -> np.ndarray:
    """Subject i's v x k matrix of N(0, 1) entries (layout above)."""
    n = v * k
    nb = (n + 3) // 4
    b = np.arange(nb, dtype=np.uint64)
    zero = np.zeros(nb, dtype=np.uint64)
    x = philox4x64([b, np.full(nb, i, dtype=np.uint64), zero, zero],
                   (np.uint64(seed), np.uint64(0)))
    u = [((xj >> np.uint64(11)).astype(np.float64) + 0.5) * 2.0 ** -53 for xj in x]
    r0 = np.sqrt(-2.0 * np.log(u[0]))
    r2 = np.sqrt(-2.0 * np.log(u[2]))
    z = np.stack([r0 * np.cos(2.0 * np.pi * u[1]), r0 * np.sin(2.0 * np.pi * u[1]),
                  r2 * np.cos(2.0 * np.pi * u[3]), r2 * np.sin(2.0 * np.pi * u[3])], axis=1)
    return z.reshape(-1)[:n].reshape(v, k)


def seeded_start(v: int, k: int, seed: int, i: int) -> np.ndarray:
    """W0_i = polar factor (Eq. 4's map, here applied to a Gaussian) of
    seeded_gaussian(v, k, seed, i): the library's start when no W0 is given."""
    W, _ = polar_svd(seeded_gaussian(v, k, seed, i))
    return W
