"""Parity at the workloads' full sizes, in the launch configuration bench.py times.

The 16-subject workload (16 x ~50k voxels x 1000 TRs, k = 50) is small enough
for the complete FP64 oracle over a few iterations.  For the 1024-subject
batched workload (51 M voxels x 500 TRs) the oracle recomputes, one subject
at a time, the final M-step of sampled subjects from the device's S and
tr(Sigma_s) (Eq. 4 and the rho update), and the test checks properties that
hold at any size: orthonormal maps, a non-decreasing log-likelihood, and a
symmetric positive definite Sigma_s.
"""
import sys

import numpy as np
import pytest

import oracle
from paper_1608_04647_amd import synth

from _parity import compare, proj_err

pytestmark = pytest.mark.gpu


def _srm():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1608_04647_amd import srm
    return srm


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.mark.timeout(900)
@pytest.mark.parametrize("prec,bar,gram", [("fp32", 1e-4, False), ("bf16x2", 1e-3, False),
                                           ("fp32", 1e-4, True)])
def test_plain16_full_size_against_complete_oracle(prec, bar, gram):
    srm = _srm()
    w = synth.WORKLOADS["plain16"]
    n_iter = 3
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


@pytest.mark.timeout(900)
@pytest.mark.parametrize("gram", [False, True])
def test_batch1024_full_size_sampled_m_step_and_properties(gram):
    import torch
    srm = _srm()
    w = synth.WORKLOADS["batch1024"]
    n_iter = 5
    _say(f"[case] batch1024 full size gram={gram}: generating 1024 subjects on the device")
    X, W0, gl = synth.to_device(w, seed=0)
    g = srm.SRM(X, w.k, prec="bf16x2", W0=W0, flags=srm.SRM_NO_W0_CHECK, gram=gram)
    del X
    torch.cuda.empty_cache()
    g.fit(n_iter)
    ll = g.loglik()
    assert len(ll) == n_iter + 1
    assert np.all(np.diff(ll) >= -1e-9 * np.abs(ll[:-1])), ll
    sig = g.sigma_s()
    assert np.allclose(sig, sig.T, atol=1e-12)
    assert np.linalg.eigvalsh(sig).min() > 0
    S = g.S().cpu().numpy().astype(np.float64)
    tau = float(np.trace(sig))
    rho = g.rho2()
    assert np.all(rho > 0)
    for i in (0, 511, 1023):
        Xi = synth.subject(w, gl, i, seed=0)
        _, xh, c = oracle.demean(Xi)
        Wo, r = oracle.m_step_subject(xh, c, S, tau)
        Wg = g.W(i).cpu().numpy().astype(np.float64)
        ep = proj_err(Wo, Wg)
        orth = float(np.abs(Wg.T @ Wg - np.eye(w.k)).max())
        er = abs(rho[i] / r - 1)
        _say(f"[errors] batch1024 subject {i}: projector {ep:.2e}, rho2 {er:.2e}, "
             f"orth {orth:.2e}")
        assert ep <= 1e-3 and er <= 1e-3 and orth <= 1e-4
    g.close()


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


@pytest.mark.timeout(900)
@pytest.mark.parametrize("prec,bar", [("fp32", 1e-4), ("bf16x2", 1e-3), ("bf16", 2e-2)])
def test_precision40_full_size_sampled(prec, bar):
    """40 subjects x 10k-100k voxels x 2000 TRs, k = 100 (K padding 112, the
    two-pass sweep and the k x k steps outside LDS).  Plain BF16 is held to
    its quantisation floor (the oracle sees the original data)."""
    import torch
    srm = _srm()
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


@pytest.mark.timeout(900)
def test_highres_subject_shape_streamed_from_host():
    """The high-resolution subjects (400k-600k voxels x 1200 TRs, k = 100,
    AR(1) noise) through streamed ingestion; 8 of the 64 subjects keep host
    memory modest, the per-subject shapes are the workload's own."""
    srm = _srm()
    w = synth.WORKLOADS["highres64"]
    sub = list(range(8))
    d = synth.generate(w, seed=0, subjects=sub, threads=8)
    g = srm.SRM(d["X"], w.k, prec="bf16x2", W0=d["W0"], stream_from_host=True,
                flags=srm.SRM_NO_W0_CHECK)
    g.fit(3)
    ll = g.loglik()
    assert np.all(np.diff(ll) >= -1e-9 * np.abs(ll[:-1])), ll
    w8 = w.scaled(n_subjects=8)
    for ep, er, orth in _sampled_m_step(g, w8, d["globals"], (0, 7), prec="bf16x2"):
        assert ep <= 1e-3 and er <= 1e-3 and orth <= 1e-4
    g.close()
