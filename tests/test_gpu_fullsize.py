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
@pytest.mark.parametrize("prec,bar", [("fp32", 1e-4), ("bf16x2", 1e-3)])
def test_plain16_full_size_against_complete_oracle(prec, bar):
    srm = _srm()
    w = synth.WORKLOADS["plain16"]
    n_iter = 3
    d = synth.generate(w, seed=0)
    _say(f"[case] plain16 full size prec={prec} iters={n_iter}")
    g = srm.SRM(d["X"], w.k, prec=prec, W0=d["W0"])
    g.fit(n_iter)
    ora = oracle.em_fit(d["X"], w.k, n_iter, d["W0"], final_loglik=True)
    e = compare(g, ora, w.n_subjects)
    _say(f"[errors] plain16/{prec}: " + ", ".join(
        f"{k}={v:.2e}" for k, v in e.items() if k != "ll_gpu"))
    assert e["S"] <= bar and e["W"] <= bar and e["rho2"] <= bar and e["Sigma_s"] <= bar
    g.close()


@pytest.mark.timeout(900)
def test_batch1024_full_size_sampled_m_step_and_properties():
    import torch
    srm = _srm()
    w = synth.WORKLOADS["batch1024"]
    n_iter = 5
    _say("[case] batch1024 full size: generating 1024 subjects on the device")
    X, W0, gl = synth.to_device(w, seed=0)
    g = srm.SRM(X, w.k, prec="bf16x2", W0=W0, flags=srm.SRM_NO_W0_CHECK)
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
