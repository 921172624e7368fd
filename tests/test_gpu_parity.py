"""Device path vs the FP64 oracle, element by element on the same seeded inputs.

Bars: relative Frobenius error <= 1e-4 on S (after the Procrustes rotation the
model cannot identify) and on the projectors W_i W_i^T for FP32 storage,
<= 1e-3 for BF16 hi+lo storage; plain BF16 storage is held to 1e-3 against
the oracle fed the same rounded values.  Every test calls the C-ABI through
the Python binding.
"""
import math
import sys

import numpy as np
import pytest

import oracle
from paper_1608_04647_amd import synth

from _progress import say
from _parity import compare, proj_err, stored_values

pytestmark = pytest.mark.gpu

BAR = {"fp32": 1e-4, "bf16x2": 1e-3, "bf16": 1e-3}


def _srm():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1608_04647_amd import srm
    return srm


def _say(*a):
    say(*a)


def _run_case(name, w, prec, seed=0, n_iter=None, **kw):
    srm = _srm()
    n_iter = w.n_iter if n_iter is None else n_iter
    d = synth.generate(w, seed=seed)
    _say(f"[case] {name} prec={prec} N={w.n_subjects} v={[x.shape[0] for x in d['X']][:6]} "
         f"t={w.t} k={w.k} iters={n_iter} {kw}")
    g = srm.SRM(d["X"], w.k, prec=prec, W0=d["W0"], **kw)
    g.fit(n_iter)
    if prec == "bf16":
        Xq = [stored_values(x, prec) for x in d["X"]]
        ora = oracle.em_fit(Xq, w.k, n_iter, d["W0"], final_loglik=True, demeaned=True)
    else:
        ora = oracle.em_fit(d["X"], w.k, n_iter, d["W0"], final_loglik=True)
    e = compare(g, ora, w.n_subjects)
    _say(f"[errors] {name}/{prec}: " + ", ".join(f"{k}={v:.2e}" for k, v in e.items()
                                                 if k != "ll_gpu"))
    return g, ora, e, d


CASES = {
    "tiny": synth.WORKLOADS["tiny"],
    # ragged voxel counts, k not a multiple of 16, t not a multiple of 64
    "ragged": synth.Workload("ragged", 5, 33, 250, 70, 7, 8),
    # many row ranges and slices crossing subjects
    "slices": synth.Workload("slices", 6, 3000, 9000, 300, 20, 6,
                             sigma_lo=0.5, sigma_hi=2.0),
    # k = 100: the k x k work that does not fit in LDS
    "k100": synth.Workload("k100", 3, 300, 420, 150, 100, 4,
                           sigma_lo=0.5, sigma_hi=2.0, rho_lo=0.3, rho_hi=0.6),
    "k128": synth.Workload("k128", 2, 200, 260, 140, 128, 3, rho_lo=0.3, rho_hi=0.6),
    # k = 100 over 700 TRs (ldt 704): the two-pass E-phase with a full and a
    # partial 512-TR panel, and M-phase rounds ending in half-filled tiles
    "k100t700": synth.Workload("k100t700", 3, 1200, 3100, 700, 100, 4,
                               sigma_lo=0.5, sigma_hi=2.0),
    # K padding 48 (three feature blocks) through the one-pass sweep with
    # four waves (t = 180)
    "k40": synth.Workload("k40", 3, 150, 400, 180, 40, 4, sigma_lo=0.5, sigma_hi=2.0),
    # the K paddings at the edges of the polar paths: 80 (the largest held in
    # LDS) and 96 (the smallest with the separate Jacobi launch)
    "k80": synth.Workload("k80", 3, 200, 300, 120, 75, 4, sigma_lo=0.5, sigma_hi=2.0,
                          rho_lo=0.3, rho_hi=0.6),
    "k96": synth.Workload("k96", 3, 200, 300, 130, 90, 4, sigma_lo=0.5, sigma_hi=2.0,
                          rho_lo=0.3, rho_hi=0.6),
    # single subject; smallest k
    "n1k1": synth.Workload("n1k1", 1, 40, 40, 16, 1, 5),
    # 500 TRs and k = 50: the batched workload's shape per subject
    "wide": synth.Workload("wide", 3, 200, 700, 500, 50, 4, sigma_lo=0.5, sigma_hi=2.0),
    # the same shape with several 64-row chunks and slices per row range
    "wide2": synth.Workload("wide2", 3, 20000, 30000, 500, 50, 3, sigma_lo=0.5, sigma_hi=2.0),
    # degenerate shapes: square maps (v_i = k), and the smallest problem
    # (t = 2, one voxel, k = 1)
    "vk": synth.Workload("vk", 3, 6, 6, 40, 6, 5),
    "min": synth.Workload("min", 2, 1, 2, 2, 1, 4),
    # the largest t the boundary accepts
    "tmax": synth.Workload("tmax", 2, 30, 50, 65536, 3, 3),
}


@pytest.mark.parametrize("prec", ["fp32", "bf16x2", "bf16"])
@pytest.mark.parametrize("case", list(CASES))
def test_parity(case, prec):
    g, ora, e, _ = _run_case(case, CASES[case], prec)
    bar = BAR[prec]
    assert e["S"] <= bar and e["W"] <= bar
    assert e["rho2"] <= bar and e["Sigma_s"] <= bar
    assert e["ll"] <= 1e-6 if prec == "fp32" else e["ll"] <= 1e-4
    assert e["orth"] <= (1e-5 if prec == "fp32" else 1e-4)
    ll = e["ll_gpu"]
    assert len(ll) == CASES[case].n_iter + 1
    assert np.all(np.diff(ll) >= -1e-6 * np.abs(ll[:-1]))
    g.close()


@pytest.mark.parametrize("prec", ["fp32", "bf16x2", "bf16"])
@pytest.mark.parametrize("case", ["tiny", "ragged", "slices", "k100", "k128", "k80", "k96",
                                  "n1k1", "wide",
                                  "vk", "min"])
def test_sample_space_iteration_parity(case, prec):
    """The sample-space iteration (G_i = Xhat_i^T Xhat_i formed once, then
    S G_i and S G_i S^T per iteration) reaches the oracle's EM iterate."""
    g, ora, e, _ = _run_case(case, CASES[case], prec, gram=True)
    bar = BAR[prec]
    assert e["S"] <= bar and e["W"] <= bar
    assert e["rho2"] <= bar and e["Sigma_s"] <= bar
    assert e["ll"] <= 1e-6 if prec == "fp32" else e["ll"] <= 1e-4
    assert e["orth"] <= (1e-5 if prec == "fp32" else 1e-4)
    g.close()


def test_sample_space_iteration_tools():
    """Getters, transform, mapping and checkpoints work the same in the
    sample-space iteration; a resumed fit is bitwise identical."""
    srm = _srm()
    w = CASES["slices"]
    d = synth.generate(w, seed=8)
    a = srm.SRM(d["X"], w.k, prec="bf16x2", W0=d["W0"], gram=True)
    a.fit(4)
    b = srm.SRM(d["X"], w.k, prec="bf16x2", W0=d["W0"], gram=True)
    b.fit(2)
    c = srm.SRM(d["X"], w.k, prec="bf16x2", W0=d["W0"], gram=True)
    c.set_state(b.get_state())
    c.fit(2)
    assert np.array_equal(a.S().cpu().numpy(), c.S().cpu().numpy())
    assert np.array_equal(a.loglik(), c.loglik())
    assert np.array_equal(a.W(3).cpu().numpy(), c.W(3).cpu().numpy())
    # a streamed-sweep checkpoint does not fit a sample-space context
    s = srm.SRM(d["X"], w.k, prec="bf16x2", W0=d["W0"])
    s.fit(1)
    with pytest.raises(srm.SRMError):
        c.set_state(s.get_state())
    ora = oracle.em_fit(d["X"], w.k, 4, d["W0"])
    Xn = np.random.default_rng(2).standard_normal((d["X"][1].shape[0], 90)).astype(np.float32)
    out = a.map(1, 4, Xn).cpu().numpy().astype(np.float64)
    ref = ora["W"][4] @ (ora["W"][1].T @ (Xn.astype(np.float64) - ora["mu"][1][:, None]))
    assert np.linalg.norm(out - ref) / np.linalg.norm(ref) <= BAR["bf16x2"]
    prof = a.profile(2)
    assert prof["gram"] > 0 and prof["ephase"] == 0 and prof["mphase"] == 0


def test_bf16_plain_against_original_data_reports_quantisation_error():
    """Plain BF16 storage is within the bar of the oracle fed the rounded data
    and, on the original data, within the rounding floor (~u/sqrt(3))."""
    w = CASES["tiny"]
    g, ora, e, d = _run_case("tiny", w, "bf16")
    ref = oracle.em_fit(d["X"], w.k, w.n_iter, d["W0"])
    eW = max(proj_err(ref["W"][i], g.W(i).cpu().numpy()) for i in range(w.n_subjects))
    _say(f"[errors] bf16 vs oracle on original X: W={eW:.2e}")
    assert eW < 3e-2


def test_fit_is_deterministic_and_resumable():
    srm = _srm()
    w = CASES["slices"]
    d = synth.generate(w, seed=5)
    a = srm.SRM(d["X"], w.k, prec="bf16x2", W0=d["W0"])
    a.fit(6)
    b = srm.SRM(d["X"], w.k, prec="bf16x2", W0=d["W0"])
    b.fit(3)
    b.fit(3)
    c = srm.SRM(d["X"], w.k, prec="bf16x2", W0=d["W0"], flags=srm.SRM_NO_GRAPH)
    for _ in range(6):
        c.em_step()
    for x in (b, c):
        assert np.array_equal(a.S().cpu().numpy(), x.S().cpu().numpy())
        assert np.array_equal(a.rho2(), x.rho2())
        assert np.array_equal(a.loglik(), x.loglik())
        assert np.array_equal(a.W(2).cpu().numpy(), x.W(2).cpu().numpy())
    assert a.iterations() == 6


def test_em_step_returns_entering_loglik():
    srm = _srm()
    w = CASES["tiny"]
    d = synth.generate(w, seed=1)
    g = srm.SRM(d["X"], w.k, prec="fp32", W0=d["W0"])
    ll0 = g.em_step()
    ll1 = g.em_step()
    ora = oracle.em_fit(d["X"], w.k, 2, d["W0"])
    assert abs(ll0 - ora["ll"][0]) <= 1e-7 * abs(ora["ll"][0])
    assert abs(ll1 - ora["ll"][1]) <= 1e-7 * abs(ora["ll"][1])


@pytest.mark.parametrize("prec", ["fp32", "bf16x2"])
def test_transform_matches_oracle_projection(prec):
    """S_new = W_i^T (X_new - mu_i 1^T) (Sec. II-A) for held-out samples."""
    srm = _srm()
    w = CASES["ragged"]
    d = synth.generate(w, seed=2)
    g = srm.SRM(d["X"], w.k, prec=prec, W0=d["W0"])
    g.fit(w.n_iter)
    ora = oracle.em_fit(d["X"], w.k, w.n_iter, d["W0"])
    rng = np.random.default_rng(0)
    for i in (0, 3):
        Xn = rng.standard_normal((d["X"][i].shape[0], 131)).astype(np.float32)
        out = g.transform(i, Xn).cpu().numpy().astype(np.float64)
        ref = ora["W"][i].T @ (Xn.astype(np.float64) - ora["mu"][i][:, None])
        # compare in the rotation-free form W W^T (x - mu)
        lhs = g.W(i).cpu().numpy().astype(np.float64) @ out
        rhs = ora["W"][i] @ ref
        err = np.linalg.norm(lhs - rhs) / np.linalg.norm(rhs)
        _say(f"[errors] transform {prec} subject {i}: {err:.2e}")
        assert err <= BAR[prec]
        mu = g.mu(i).cpu().numpy()
        assert np.allclose(mu, ora["mu"][i], rtol=0, atol=1e-6)


@pytest.mark.parametrize("prec", ["fp32", "bf16x2"])
def test_map_matches_oracle(prec):
    """Subject-to-subject mapping W_j W_i^T (X_new - mu_i 1^T) (Sec. II-A), with
    enough columns to take several scratch chunks, and the i == j case."""
    srm = _srm()
    w = CASES["ragged"]
    d = synth.generate(w, seed=3)
    g = srm.SRM(d["X"], w.k, prec=prec, W0=d["W0"])
    g.fit(w.n_iter)
    ora = oracle.em_fit(d["X"], w.k, w.n_iter, d["W0"])
    rng = np.random.default_rng(1)
    for i, j, tn in ((0, 3, 300), (3, 1, 1), (2, 2, 77)):
        Xn = rng.standard_normal((d["X"][i].shape[0], tn)).astype(np.float32)
        out = g.map(i, j, Xn).cpu().numpy().astype(np.float64)
        assert out.shape == (d["X"][j].shape[0], tn)
        ref = ora["W"][j] @ (ora["W"][i].T @ (Xn.astype(np.float64) - ora["mu"][i][:, None]))
        err = np.linalg.norm(out - ref) / np.linalg.norm(ref)
        _say(f"[errors] map {prec} {i}->{j} t={tn}: {err:.2e}")
        assert err <= BAR[prec]


def test_map_single_subject_full_k():
    """srm_map with one subject and k = 128 (the scratch chunking at its
    tightest) equals the oracle's projection W W^T (X_new - mu)."""
    srm = _srm()
    w = synth.Workload("map1", 1, 200, 200, 160, 128, 2)
    d = synth.generate(w, seed=7)
    g = srm.SRM(d["X"], w.k, prec="fp32", W0=d["W0"])
    g.fit(w.n_iter)
    ora = oracle.em_fit(d["X"], w.k, w.n_iter, d["W0"])
    Xn = np.random.default_rng(3).standard_normal((200, 700)).astype(np.float32)
    out = g.map(0, 0, Xn).cpu().numpy().astype(np.float64)
    ref = ora["W"][0] @ (ora["W"][0].T @ (Xn.astype(np.float64) - ora["mu"][0][:, None]))
    assert np.linalg.norm(out - ref) / np.linalg.norm(ref) <= BAR["fp32"]


@pytest.mark.parametrize("prec", ["fp32", "bf16x2"])
def test_zscore_matches_oracle(prec):
    """Standardised input (Sec. IV-A, reading R14): voxels given very different
    scales and offsets, one constant voxel; the fit, the stored mean and scale
    and the projection of held-out samples follow the oracle on Z."""
    srm = _srm()
    w = CASES["ragged"]
    d = synth.generate(w, seed=4)
    rng = np.random.default_rng(9)
    X = []
    for x in d["X"]:
        a = rng.uniform(0.05, 40.0, (x.shape[0], 1))
        b = rng.normal(0.0, 100.0, (x.shape[0], 1))
        X.append((x * a + b).astype(np.float32))
    X[1][5, :] = np.float32(0.1)
    g = srm.SRM(X, w.k, prec=prec, W0=d["W0"], zscore=True)
    g.fit(w.n_iter)
    zs = [oracle.zscore(x) for x in X]
    ora = oracle.em_fit([z[1] for z in zs], w.k, w.n_iter, d["W0"], final_loglik=True,
                        demeaned=True)
    e = compare(g, ora, w.n_subjects)
    _say(f"[errors] zscore/{prec}: " + ", ".join(f"{k}={v:.2e}" for k, v in e.items()
                                                 if k != "ll_gpu"))
    assert e["S"] <= BAR[prec] and e["W"] <= BAR[prec]
    assert e["rho2"] <= BAR[prec] and e["Sigma_s"] <= BAR[prec]
    for i in range(w.n_subjects):
        assert np.allclose(g.mu(i).cpu().numpy(), zs[i][0], rtol=1e-12, atol=1e-9)
        assert np.allclose(g.scale(i).cpu().numpy(), zs[i][2], rtol=1e-12, atol=0)
    assert g.scale(1).cpu().numpy()[5] == 1.0
    Xn = (rng.standard_normal((X[2].shape[0], 40)) * 10).astype(np.float32)
    out = g.transform(2, Xn).cpu().numpy().astype(np.float64)
    ref = ora["W"][2].T @ ((Xn.astype(np.float64) - zs[2][0][:, None]) * zs[2][2][:, None])
    lhs = g.W(2).cpu().numpy().astype(np.float64) @ out
    err = np.linalg.norm(lhs - ora["W"][2] @ ref) / np.linalg.norm(ora["W"][2] @ ref)
    assert err <= BAR[prec]


@pytest.mark.parametrize("flags", [0, 4])
def test_checkpoint_resume_is_bitwise(flags):
    """A fit stopped after 3 iterations, saved, restored into a fresh context on
    the same data and continued equals the uninterrupted 6-iteration fit."""
    srm = _srm()
    w = CASES["slices"]
    d = synth.generate(w, seed=6)
    a = srm.SRM(d["X"], w.k, prec="bf16x2", W0=d["W0"], flags=flags)
    a.fit(6)
    b = srm.SRM(d["X"], w.k, prec="bf16x2", W0=d["W0"], flags=flags)
    blob0 = b.get_state()  # before the first iteration: resumes from the first E-step
    b.fit(3)
    blob = b.get_state()
    w4 = b.W(4).cpu().numpy()
    b.close()
    c = srm.SRM(d["X"], w.k, prec="bf16x2", W0=d["W0"], flags=flags)
    c.set_state(blob)
    assert c.iterations() == 3
    assert np.array_equal(c.W(4).cpu().numpy(), w4)
    c.fit(3)
    assert c.iterations() == 6
    assert np.array_equal(a.S().cpu().numpy(), c.S().cpu().numpy())
    assert np.array_equal(a.rho2(), c.rho2())
    assert np.array_equal(a.sigma_s(), c.sigma_s())
    assert np.array_equal(a.loglik(), c.loglik())
    for i in (0, 5):
        assert np.array_equal(a.W(i).cpu().numpy(), c.W(i).cpu().numpy())
    # the blob of the freshly initialised context rewinds a fit to its start
    c.set_state(blob0)
    assert c.iterations() == 0
    c.fit(6)
    assert np.array_equal(a.S().cpu().numpy(), c.S().cpu().numpy())
    assert np.array_equal(a.loglik(), c.loglik())
    # a blob is refused by a context on other data, and when truncated
    X2 = [x.copy() for x in d["X"]]
    X2[0][0, 0] += 1.0
    e = srm.SRM(X2, w.k, prec="bf16x2", W0=d["W0"], flags=flags)
    for bad in (blob, blob[:-8]):
        with pytest.raises(srm.SRMError) as ei:
            e.set_state(bad)
        assert ei.value.status == srm.SRM_E_ARG


def test_nonfinite_input_is_rejected():
    srm = _srm()
    w = CASES["tiny"]
    d = synth.generate(w, seed=0)
    d["X"][1][7, 3] = np.nan
    with pytest.raises(srm.SRMError) as ei:
        srm.SRM(d["X"], w.k, prec="fp32", W0=d["W0"])
    assert ei.value.status == srm.SRM_E_NONFINITE


def test_rank_deficient_subject_raises():
    """Reading R10: an all-zero subject gives A_i = 0, which has no polar factor."""
    srm = _srm()
    w = CASES["tiny"]
    d = synth.generate(w, seed=0)
    d["X"][2][:] = 1.0  # constant rows demean to exactly zero
    g = srm.SRM(d["X"], w.k, prec="fp32", W0=d["W0"])
    with pytest.raises(srm.SRMError) as ei:
        g.fit(2)
    assert ei.value.status == srm.SRM_E_RANK


def test_profile_reports_the_sweep_phases():
    """srm_profile times each phase of the sweep that runs: the one-pass sweep
    where it applies, M- and E-phase otherwise; its iterations count like
    srm_fit's and leave the same state as the captured graph."""
    srm = _srm()
    w = CASES["wide"]
    d = synth.generate(w, seed=5)
    for flags, on, off in ((0, ("fused",), ("mphase", "ephase")),
                           (srm.SRM_TWO_PASS, ("mphase", "ephase"), ("fused",))):
        a = srm.SRM(d["X"], w.k, prec="bf16x2", W0=d["W0"], flags=flags)
        b = srm.SRM(d["X"], w.k, prec="bf16x2", W0=d["W0"], flags=flags)
        prof = a.profile(2)
        b.fit(2)
        for ph in on + ("polar", "ereduce", "posterior"):
            assert prof[ph] > 0, (flags, ph, prof)
        for ph in off + ("gram",):
            assert prof[ph] == 0, (flags, ph, prof)
        assert a.iterations() == b.iterations() == 2
        assert np.array_equal(a.S().cpu().numpy(), b.S().cpu().numpy())
        a.close()
        b.close()


def test_getters_before_first_iteration():
    srm = _srm()
    w = CASES["tiny"]
    d = synth.generate(w, seed=0)
    g = srm.SRM(d["X"], w.k, prec="fp32", W0=d["W0"])
    with pytest.raises(srm.SRMError) as ei:
        g.W(0)
    assert ei.value.status == srm.SRM_E_STATE
    assert len(g.loglik()) == 1


@pytest.mark.parametrize("case", ["tiny", "slices", "ragged", "wide", "wide2"])
def test_fused_and_two_pass_sweeps_agree(case):
    """The one-pass sweep (A never stored) and the two-pass sweep (A = Xhat S^T
    written, then A^T Xhat) are the same EM; both meet the BF16 bar against the
    oracle and agree with each other to rounding."""
    srm = _srm()
    w = CASES[case]
    d = synth.generate(w, seed=3)
    ora = oracle.em_fit(d["X"], w.k, w.n_iter, d["W0"], final_loglik=True)
    fits = {}
    for name, flags in (("fused", 0), ("two_pass", srm.SRM_TWO_PASS)):
        g = srm.SRM(d["X"], w.k, prec="bf16x2", W0=d["W0"], flags=flags)
        g.fit(w.n_iter)
        e = compare(g, ora, w.n_subjects)
        _say(f"[errors] {case}/{name}: " + ", ".join(
            f"{k}={v:.2e}" for k, v in e.items() if k != "ll_gpu"))
        assert e["S"] <= 1e-3 and e["W"] <= 1e-3 and e["rho2"] <= 1e-3
        fits[name] = g
    a, b = fits["fused"], fits["two_pass"]
    for i in range(w.n_subjects):
        assert proj_err(a.W(i).cpu().numpy(), b.W(i).cpu().numpy()) <= 1e-4
    assert np.allclose(a.rho2(), b.rho2(), rtol=1e-4)


def test_streamed_host_ingestion_is_bitwise_identical():
    """SRM_X_HOST (each subject staged through the workspace) stores the same
    values and so gives the same fit as converting device-resident X."""
    srm = _srm()
    w = CASES["slices"]
    d = synth.generate(w, seed=6)
    a = srm.SRM(d["X"], w.k, prec="bf16x2", W0=d["W0"])
    b = srm.SRM(d["X"], w.k, prec="bf16x2", W0=d["W0"], stream_from_host=True)
    assert b.workspace_bytes > a.workspace_bytes
    a.fit(3)
    b.fit(3)
    assert np.array_equal(a.S().cpu().numpy(), b.S().cpu().numpy())
    assert np.array_equal(a.loglik(), b.loglik())
    for i in range(w.n_subjects):
        assert np.array_equal(a.mu(i).cpu().numpy(), b.mu(i).cpu().numpy())
