"""Seeded synthetic inputs for the Shared Response Model (SRM) EM sweep.

This module only draws random inputs; it holds none of the SRM method's
arithmetic (no demeaning, no E-step, no M-step).  Its outputs feed both the
FP64 CPU oracle and the HIP library, which is the only thing they share.

The data follow the SRM generative model of Sec. II-A (Eq. 1): every subject
i sees the same shared response ``S`` (k x t, columns s_t ~ N(0, Sigma_s)),
mapped into its own v_i voxels by an orthonormal W_i (W_i^T W_i = I), plus
isotropic noise of standard deviation rho_i.  The generator adds no mean term
(the method removes the per-voxel mean anyway).

Draw order (every draw is deterministic given ``seed``):

* stream ``(0, 0)``: v_i for all subjects, then rho_i for all subjects, then
  diag(Sigma_s) (identity when the workload says so), then the FP64 Gaussian
  k x t matrix that is scaled into S = Sigma_s^{1/2} Z.
* stream ``(0, i + 1)``: subject i's Gaussian v_i x k matrix (its planted W_i
  is the Q factor of its QR, with sign(diag R) > 0), then its v_i x t noise.
* stream ``(1, i)``: subject i's random orthonormal starting map W0_i (the
  "random orthogonal matrix" of Algorithm 1's initialisation), drawn the same
  way as a planted W_i.

Noise is drawn in float32 and X_i is returned in float32, the format the
device library ingests; the oracle upcasts the same values exactly.
An AR(1) temporal noise option (coefficient phi, stationary std rho_i)
deliberately breaks SRM's white-noise assumption for the high-resolution
workload.
"""
from __future__ import annotations

import dataclasses
import os
from concurrent.futures import ThreadPoolExecutor
from typing import Iterator, Optional, Sequence

import numpy as np


@dataclasses.dataclass(frozen=True)
class Workload:
    """One synthetic workload: subject count, voxel range, TRs, features."""

    name: str
    n_subjects: int
    v_lo: int
    v_hi: int  # inclusive; v_lo == v_hi gives equal subjects
    t: int
    k: int
    n_iter: int
    rho_lo: float = 0.5
    rho_hi: float = 1.5
    sigma_lo: Optional[float] = None  # None: Sigma_s = I
    sigma_hi: Optional[float] = None
    ar_phi: float = 0.0
    prec: str = "fp32"  # X storage the workload is quoted on

    def scaled(self, **kw) -> "Workload":
        return dataclasses.replace(self, **kw)


# The five workloads (sizes from the method's target problem statement).
WORKLOADS = {
    # 4 subjects x 500 voxels x 200 TRs, k = 10, Sigma_s = I, 10 iterations.
    "tiny": Workload("tiny", 4, 500, 500, 200, 10, 10),
    # 16 subjects, uneven 40k-60k voxels, 1000 TRs, k = 50, 20 iterations.
    "plain16": Workload("plain16", 16, 40000, 60000, 1000, 50, 20,
                        sigma_lo=0.5, sigma_hi=2.0),
    # 40 subjects, 10k-100k voxels, 2000 TRs, k = 100 (precision study).
    "precision40": Workload("precision40", 40, 10000, 100000, 2000, 100, 20,
                            sigma_lo=0.5, sigma_hi=2.0, prec="bf16x2"),
    # 1024 subjects, 20k-80k voxels, 500 TRs, k = 50 (batched sweep).
    "batch1024": Workload("batch1024", 1024, 20000, 80000, 500, 50, 20,
                          sigma_lo=0.5, sigma_hi=2.0, prec="bf16x2"),
    # 64 subjects, 400k-600k voxels, 1200 TRs, k = 100, AR(1) noise.
    "highres64": Workload("highres64", 64, 400000, 600000, 1200, 100, 30,
                          sigma_lo=0.5, sigma_hi=2.0, ar_phi=0.5,
                          prec="bf16x2"),
}


@dataclasses.dataclass
class Globals:
    v: np.ndarray        # int64 [N]
    rho: np.ndarray      # float64 [N] noise std per subject
    sigma_diag: np.ndarray  # float64 [k]
    S: np.ndarray        # float64 [k, t] planted shared response


def _rng(seed: int, *key: int) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64(
        np.random.SeedSequence(entropy=seed, spawn_key=tuple(key))))


def random_orthonormal(rng: np.random.Generator, v: int, k: int) -> np.ndarray:
    """Haar-distributed v x k matrix with orthonormal columns: the Q factor of
    the QR decomposition (diag(R) > 0) of a v x k N(0,1) matrix.

    Q is formed by two rounds of Cholesky QR (Q = G R^-1 with R^T R = G^T G),
    which gives that same Q for these well-conditioned Gaussian matrices and is
    much faster than Householder QR on tall-skinny shapes."""
    q = rng.standard_normal((v, k))
    for _ in range(2):
        r = np.linalg.cholesky(q.T @ q).T  # upper, positive diagonal
        q = q @ np.linalg.inv(r)
    return q


def draw_globals(w: Workload, seed: int = 0) -> Globals:
    rng = _rng(seed, 0, 0)
    v = rng.integers(w.v_lo, w.v_hi + 1, size=w.n_subjects, dtype=np.int64)
    rho = rng.uniform(w.rho_lo, w.rho_hi, size=w.n_subjects)
    if w.sigma_lo is None:
        sig = np.ones(w.k)
    else:
        sig = rng.uniform(w.sigma_lo, w.sigma_hi, size=w.k)
    z = rng.standard_normal((w.k, w.t))
    S = np.sqrt(sig)[:, None] * z
    return Globals(v=v, rho=rho, sigma_diag=sig, S=S)


def subject(w: Workload, g: Globals, i: int, seed: int = 0,
            want_w: bool = False):
    """X_i (float32, v_i x t, row-major) and optionally the planted W_i."""
    rng = _rng(seed, 0, i + 1)
    vi = int(g.v[i])
    Wp = random_orthonormal(rng, vi, w.k)
    e = rng.standard_normal((vi, w.t), dtype=np.float32)
    if w.ar_phi != 0.0:
        # e_0 = z_0, e_tau = phi e_(tau-1) + sqrt(1 - phi^2) z_tau (stationary
        # unit variance), as one IIR filter along each voxel's time series.
        from scipy.signal import lfilter
        e[:, 1:] *= np.float32(np.sqrt(1.0 - w.ar_phi ** 2))
        e = lfilter([1.0], [1.0, -w.ar_phi], e, axis=1).astype(np.float32, copy=False)
    X = Wp.astype(np.float32) @ g.S.astype(np.float32)
    X += np.float32(g.rho[i]) * e
    return (X, Wp) if want_w else X


def init_map(w: Workload, g: Globals, i: int, seed: int = 0) -> np.ndarray:
    """Random orthonormal starting map W0_i (float64, v_i x k)."""
    return random_orthonormal(_rng(seed, 1, i), int(g.v[i]), w.k)


def _threads() -> int:
    n = os.cpu_count() or 1
    return max(1, min(16, n))


def _blas_single():
    """Context keeping BLAS single-threaded while a thread pool draws subjects."""
    try:
        from threadpoolctl import threadpool_limits
        return threadpool_limits(1)
    except Exception:  # pragma: no cover
        import contextlib
        return contextlib.nullcontext()


def generate(w: Workload, seed: int = 0, subjects: Optional[Sequence[int]] = None,
             want_planted: bool = False, threads: Optional[int] = None):
    """Whole workload in host memory: dict with X, W0, globals (and planted W)."""
    g = draw_globals(w, seed)
    idx = list(range(w.n_subjects)) if subjects is None else list(subjects)

    def one(i):
        X, Wp = subject(w, g, i, seed, want_w=True)
        return X, Wp, init_map(w, g, i, seed)

    with _blas_single(), ThreadPoolExecutor(threads or _threads()) as ex:
        out = list(ex.map(one, idx))
    res = {"globals": g, "subjects": idx, "X": [o[0] for o in out],
           "W0": [o[2] for o in out]}
    if want_planted:
        res["W_planted"] = [o[1] for o in out]
    return res


def iter_subjects(w: Workload, seed: int = 0, threads: Optional[int] = None,
                  with_w0: bool = True) -> Iterator:
    """Yield (i, X_i, W0_i) in subject order, generated ahead on a thread pool."""
    g = draw_globals(w, seed)
    nthr = threads or _threads()

    def one(i):
        X = subject(w, g, i, seed)
        return i, X, (init_map(w, g, i, seed) if with_w0 else None)

    with _blas_single(), ThreadPoolExecutor(nthr) as ex:
        pending = []
        nxt = 0
        while nxt < w.n_subjects and len(pending) < 2 * nthr:
            pending.append(ex.submit(one, nxt))
            nxt += 1
        while pending:
            r = pending.pop(0).result()
            if nxt < w.n_subjects:
                pending.append(ex.submit(one, nxt))
                nxt += 1
            yield r


def to_device(w: Workload, seed: int = 0, device=None, threads: Optional[int] = None,
              with_w0: bool = True):
    """Generate the workload straight into one float32 device buffer.

    Returns (list of per-subject torch views v_i x t, list of W0_i host arrays
    or None, Globals).  Subjects are drawn on a thread pool and copied one by
    one, so host memory holds only a few subjects of X at a time."""
    import torch
    g = draw_globals(w, seed)
    dev = device or torch.device("cuda")
    total = int(g.v.sum())
    buf = torch.empty((total, w.t), dtype=torch.float32, device=dev)
    offs = np.concatenate([[0], np.cumsum(g.v)]).astype(np.int64)
    w0 = [None] * w.n_subjects if with_w0 else None
    for i, X, W0 in iter_subjects(w, seed, threads, with_w0=with_w0):
        buf[offs[i]:offs[i + 1]].copy_(torch.from_numpy(X))
        if with_w0:
            w0[i] = W0
    torch.cuda.synchronize()
    views = [buf[offs[i]:offs[i + 1]] for i in range(w.n_subjects)]
    return views, w0, g
