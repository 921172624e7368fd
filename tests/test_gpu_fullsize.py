"""Parity at the workloads' full sizes, in the launch configuration bench.py times.

The 16-subject workload (16 x ~50k voxels x 1000 TRs, k = 50) runs its 20
iterations against the complete FP64 oracle.  The 1024-subject batched
workload (51 M voxels x 500 TRs) runs its 20 iterations against the oracle's
t x t Gram form on streamed input: each subject is regenerated from the seed
and reduced to G_i = Xhat_i^T Xhat_i, c_i and W0_i^T Xhat_i, so every result
of the fit (S, Sigma_s, every rho_i^2, every log-likelihood) is compared.
The larger workloads recompute, one subject at a time, the final M-step of
sampled subjects from the device's S and tr(Sigma_s) (Eq. 4 and the rho
update), and check properties that hold at any size: orthonormal maps, a
non-decreasing log-likelihood.
"""
import sys

import numpy as np
import pytest

import oracle
from paper_1608_04647_amd import synth

from _progress import say
from _parity import compare, proj_err

pytestmark = pytest.mark.gpu


def _srm():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1608_04647_amd import srm
    return srm


def _say(*a):
    say(*a)


@pytest.mark.timeout(900)
@pytest.mark.parametrize("prec,bar,gram", [("fp32", 1e-4, False), ("bf16x2", 1e-3, False),
                                           ("fp32", 1e-4, True)])
def test_plain16_full_size_against_complete_oracle(prec, bar, gram):
    srm = _srm()
    w = synth.WORKLOADS["plain16"]
    n_iter = w.n_iter
    d = synth.generate(w, seed=0)
    _say(f"[case] plain16 full size prec={prec} gram={gram} iters={n_iter}")
    g = srm.SRM(d["X"], w.k, prec=prec, W0=d["W0"], gram=gram)
    g.fit(n_iter)
    ora = oracle.em_fit(d["X"], w.k, n_iter, d["W0"], final_loglik=True)
    e = compare(g, ora, w.n_subjects)
    _say(f"[errors] plain16/{prec}: " + ", ".join(
        f"{k}={v:.2e}" for k, v in e.items() if k != "ll_gpu"))
    assert e["S"] <= bar and e["W"] <= bar and e["rho2"] <= bar and e["Sigma_s"] <= bar
    g.close()


def _say_progress(tag, n_total):
    def f(done):
        if done % 128 == 0 or done == n_total:
            _say(f"[oracle] {tag}: {done}/{n_total} subjects summarised")
    return f


@pytest.mark.timeout(1500)
def test_batch1024_full_trajectory_against_oracle():
    """The 1024-subject batched workload (51 M voxels x 500 TRs, k = 50, BF16
    hi+lo) for its 20 iterations, through the one-pass sweep and through the
    sample-space iteration, against the FP64 oracle's Gram form on streamed
    input (every subject regenerated and summarised one at a time): S after
    Procrustes, Sigma_s, all 1024 rho_i^2, the log-likelihood of every
    iteration, and projectors of 8 subjects across the range, each within
    1e-3 (Sec. II-D, Eq. 10-11; Algorithm 1)."""
    import torch
    srm = _srm()
    from _parity import procrustes
    from _streamed import oracle_fit, oracle_w
    w = synth.WORKLOADS["batch1024"]
    n_iter = w.n_iter
    picks = (0, 137, 300, 511, 640, 777, 900, 1023)
    _say("[case] batch1024 full trajectory: generating 1024 subjects on the device")
    X, W0, gl = synth.to_device(w, seed=0)
    fits = {}
    for gram in (False, True):
        g = srm.SRM(X, w.k, prec="bf16x2", W0=W0, flags=srm.SRM_NO_W0_CHECK, gram=gram)
        g.fit(n_iter)
        fits[g.info()["sweep"]] = {
            "S": g.S().cpu().numpy().astype(np.float64), "Sigma_s": g.sigma_s(),
            "rho2": g.rho2(), "ll": g.loglik(),
            "W": {i: g.W(i).cpu().numpy() for i in picks}}
        _say(f"[case] device fit done ({g.info()['sweep']}, graph={g.info()['graph']})")
        g.close()
        del g
        torch.cuda.empty_cache()
    del X, W0
    torch.cuda.empty_cache()
    assert set(fits) == {"one_pass", "gram"}
    ora = oracle_fit(w, n_iter, seed=0, progress=_say_progress("batch1024", w.n_subjects))
    ll_o = np.array(ora["ll"] + [ora["ll_final"]])
    Wo = {i: oracle_w(ora, w, i, seed=0) for i in picks}
    for sweep, f in fits.items():
        Q, eS, _ = procrustes(ora["S"], f["S"])
        eSig = np.linalg.norm(ora["Sigma_s"] - Q @ f["Sigma_s"] @ Q.T) / \
            np.linalg.norm(ora["Sigma_s"])
        eR = float(np.max(np.abs(f["rho2"] / ora["rho2"] - 1)))
        assert len(f["ll"]) == len(ll_o) == n_iter + 1
        eLL = float(np.max(np.abs(f["ll"] - ll_o) / np.abs(ll_o)))
        eW = max(proj_err(Wo[i], f["W"][i]) for i in picks)
        _say(f"[errors] batch1024 full trajectory {sweep}: S={eS:.2e} Sigma_s={eSig:.2e} "
             f"rho2(max of 1024)={eR:.2e} ll(max of {n_iter + 1})={eLL:.2e} "
             f"projector(8)={eW:.2e}")
        assert eS <= 1e-3 and eSig <= 1e-3 and eR <= 1e-3 and eW <= 1e-3
        assert eLL <= 1e-4
        assert np.all(np.diff(f["ll"]) >= -1e-9 * np.abs(f["ll"][:-1])), f["ll"]


def _sampled_m_step(g, w, gl, subjects, seed=0, prec=None):
    S = g.S().cpu().numpy().astype(np.float64)
    sig = g.sigma_s()
    tau = float(np.trace(sig))
    rho = g.rho2()
    out = []
    for i in subjects:
        Xi = synth.subject(w, gl, i, seed=seed)
        _, xh, c = oracle.demean(Xi)
        Wo, r = oracle.m_step_subject(xh, c, S, tau)
        Wg = g.W(i).cpu().numpy().astype(np.float64)
        out.append((proj_err(Wo, Wg), abs(rho[i] / r - 1),
                    float(np.abs(Wg.T @ Wg - np.eye(w.k)).max())))
        _say(f"[errors] {w.name}/{prec} subject {i}: projector {out[-1][0]:.2e}, "
             f"rho2 {out[-1][1]:.2e}, orth {out[-1][2]:.2e}")
    return out


@pytest.mark.timeout(1200)
def test_precision40_full_trajectory_against_oracle():
    """40 subjects x 10k-100k voxels x 2000 TRs, k = 100 (K padding 112, the
    two-pass sweep and the k x k steps outside LDS), 20 iterations in FP32
    and in BF16 hi+lo against the oracle's Gram form on streamed input: S,
    Sigma_s, all 40 rho_i^2, every log-likelihood and 4 projectors."""
    import torch
    srm = _srm()
    from _parity import procrustes
    from _streamed import oracle_fit, oracle_w
    w = synth.WORKLOADS["precision40"]
    picks = (0, 13, 26, 39)
    X, W0, gl = synth.to_device(w, seed=0)
    fits = {}
    for prec in ("fp32", "bf16x2"):
        g = srm.SRM(X, w.k, prec=prec, W0=W0, flags=srm.SRM_NO_W0_CHECK)
        g.fit(w.n_iter)
        fits[prec] = {"S": g.S().cpu().numpy().astype(np.float64), "Sigma_s": g.sigma_s(),
                      "rho2": g.rho2(), "ll": g.loglik(),
                      "W": {i: g.W(i).cpu().numpy() for i in picks}}
        _say(f"[case] precision40 {prec}: device fit done")
        g.close()
        del g
        torch.cuda.empty_cache()
    del X, W0
    torch.cuda.empty_cache()
    ora = oracle_fit(w, w.n_iter, seed=0, progress=_say_progress("precision40", w.n_subjects))
    ll_o = np.array(ora["ll"] + [ora["ll_final"]])
    Wo = {i: oracle_w(ora, w, i, seed=0) for i in picks}
    for prec, f in fits.items():
        bar = 1e-4 if prec == "fp32" else 1e-3
        Q, eS, _ = procrustes(ora["S"], f["S"])
        eSig = np.linalg.norm(ora["Sigma_s"] - Q @ f["Sigma_s"] @ Q.T) / \
            np.linalg.norm(ora["Sigma_s"])
        eR = float(np.max(np.abs(f["rho2"] / ora["rho2"] - 1)))
        eLL = float(np.max(np.abs(f["ll"] - ll_o) / np.abs(ll_o)))
        eW = max(proj_err(Wo[i], f["W"][i]) for i in picks)
        _say(f"[errors] precision40 full trajectory {prec}: S={eS:.2e} Sigma_s={eSig:.2e} "
             f"rho2(max of 40)={eR:.2e} ll(max of {w.n_iter + 1})={eLL:.2e} "
             f"projector(4)={eW:.2e}")
        assert eS <= bar and eSig <= bar and eR <= bar and eW <= bar
        assert eLL <= (1e-6 if prec == "fp32" else 1e-4)


@pytest.mark.timeout(900)
def test_precision40_plain_bf16_sampled():
    """Plain BF16 storage of the 40-subject workload is held to its
    quantisation floor: the oracle's M-step on the original data from the
    device's S (the oracle sees unrounded values)."""
    import torch
    srm = _srm()
    prec, bar = "bf16", 2e-2
    w = synth.WORKLOADS["precision40"]
    X, W0, gl = synth.to_device(w, seed=0)
    g = srm.SRM(X, w.k, prec=prec, W0=W0, flags=srm.SRM_NO_W0_CHECK)
    del X
    torch.cuda.empty_cache()
    g.fit(3)
    ll = g.loglik()
    assert np.all(np.diff(ll) >= -1e-9 * np.abs(ll[:-1])), ll
    for ep, er, orth in _sampled_m_step(g, w, gl, (0, 39), prec=prec):
        assert ep <= bar and er <= bar and orth <= 1e-4
    g.close()


@pytest.mark.timeout(1500)
def test_highres64_full_size_incremental_ingestion():
    """All 64 high-resolution subjects (400k-600k voxels x 1200 TRs, k = 100,
    AR(1) noise; 155 GB of BF16 hi+lo on the device) ingested one at a time
    from host memory through the staging buffers (srm_init_begin /
    srm_ingest / srm_init_end), so the host holds a few subjects at once;
    30 iterations with a non-decreasing log-likelihood, then the oracle's
    M-step for 4 subjects across the range from the device's S and
    tr(Sigma_s) (Sec. IV-A, IV-B per-subject loading; Sec. V)."""
    import time
    srm = _srm()
    w = synth.WORKLOADS["highres64"]
    gl = synth.draw_globals(w, seed=0)
    g = srm.SRM.begin([int(x) for x in gl.v], w.t, w.k, prec="bf16x2", stream_from_host=True,
                      flags=srm.SRM_NO_W0_CHECK)
    t0 = time.perf_counter()
    for i, X, W0 in synth.iter_subjects(w, seed=0, threads=4):
        g.ingest(i, X, W0)
        if i % 8 == 7:
            _say(f"[case] highres64: {i + 1}/64 subjects ingested "
                 f"({time.perf_counter() - t0:.0f} s)")
    g.end()
    g.fit(w.n_iter)
    ll = g.loglik()
    assert len(ll) == w.n_iter + 1
    assert np.all(np.diff(ll) >= -1e-9 * np.abs(ll[:-1])), ll
    for ep, er, orth in _sampled_m_step(g, w, gl, (0, 21, 42, 63), prec="bf16x2"):
        assert ep <= 1e-3 and er <= 1e-3 and orth <= 1e-4
    g.close()
