"""Oracle inputs for workloads too large to hold: each subject is regenerated
from the seed, reduced to what the oracle's t x t Gram form needs
(oracle.gram_summary), and dropped.  Test infrastructure; no SRM arithmetic
here beyond calling the oracle."""
from __future__ import annotations

import os
from concurrent.futures import ThreadPoolExecutor
from typing import Callable, Iterator, Optional

import oracle
from paper_1608_04647_amd import synth


def _threads() -> int:
    return max(1, min(16, os.cpu_count() or 1))


def gram_summaries(w: synth.Workload, seed: int = 0, threads: Optional[int] = None,
                   progress: Optional[Callable[[int], None]] = None) -> Iterator:
    """Yield oracle.gram_summary(X_i, W0_i) for i = 0..N-1 in order.

    Subjects are generated and summarised on a thread pool with BLAS held to
    one thread per worker; at most 2 x threads subjects are in flight, so
    host memory holds a few subjects of X at a time."""
    g = synth.draw_globals(w, seed)
    # each worker holds a subject in float32 and its demeaned float64 copy
    per = float(w.v_hi) * w.t * 16.0
    nthr = threads or max(1, min(_threads(), int(96e9 // per)))

    def one(i):
        X = synth.subject(w, g, i, seed)
        return oracle.gram_summary(X, synth.init_map(w, g, i, seed))

    with synth._blas_single(), ThreadPoolExecutor(nthr) as ex:
        pending = []
        nxt = 0
        while nxt < w.n_subjects and len(pending) < 2 * nthr:
            pending.append(ex.submit(one, nxt))
            nxt += 1
        done = 0
        while pending:
            r = pending.pop(0).result()
            if nxt < w.n_subjects:
                pending.append(ex.submit(one, nxt))
                nxt += 1
            done += 1
            if progress is not None:
                progress(done)
            yield r


def oracle_fit(w: synth.Workload, n_iter: int, seed: int = 0,
               progress: Optional[Callable[[int], None]] = None) -> dict:
    """The oracle's EM iterate after n_iter iterations from the workload's
    W0 (the Gram form, streamed input)."""
    from threadpoolctl import threadpool_limits
    # The per-iteration products are small (k x t by t x t): a few BLAS
    # threads run them faster than many.
    with threadpool_limits(4):
        return oracle.fit_gram_summaries(gram_summaries(w, seed, progress=progress), w.k,
                                         n_iter, final_loglik=True)


def oracle_w(fit: dict, w: synth.Workload, i: int, seed: int = 0):
    """W_i of a streamed oracle fit, its subject regenerated."""
    g = synth.draw_globals(w, seed)
    return oracle.w_of(fit, i, synth.subject(w, g, i, seed))
