"""Seeded synthetic inputs: determinism, shapes and the planted model's statistics."""
import numpy as np

from paper_1608_04647_amd import synth


def test_deterministic_and_subject_independent():
    w = synth.WORKLOADS["tiny"]
    a = synth.generate(w, seed=0)
    b = synth.generate(w, seed=0, subjects=[2])
    assert np.array_equal(a["X"][2], b["X"][0])
    assert np.array_equal(a["W0"][2], b["W0"][0])
    c = synth.generate(w, seed=1)
    assert not np.array_equal(a["X"][0], c["X"][0])


def test_shapes_and_ranges():
    w = synth.WORKLOADS["plain16"].scaled(v_lo=400, v_hi=600, t=100)
    d = synth.generate(w, seed=0, want_planted=True)
    g = d["globals"]
    assert g.v.min() >= 400 and g.v.max() <= 600 and len(g.v) == 16
    assert np.all((g.rho >= 0.5) & (g.rho <= 1.5))
    assert np.all((g.sigma_diag >= 0.5) & (g.sigma_diag <= 2.0))
    for X, W0, Wp, v in zip(d["X"], d["W0"], d["W_planted"], g.v):
        assert X.shape == (v, 100) and X.dtype == np.float32
        assert np.abs(W0.T @ W0 - np.eye(w.k)).max() < 1e-12
        assert np.abs(Wp.T @ Wp - np.eye(w.k)).max() < 1e-12


def test_planted_statistics():
    w = synth.Workload("stat", 2, 3000, 3000, 4000, 4, 1, rho_lo=0.7, rho_hi=0.7,
                       sigma_lo=0.5, sigma_hi=2.0)
    d = synth.generate(w, seed=5, want_planted=True)
    g = d["globals"]
    emp = g.S @ g.S.T / w.t
    assert np.allclose(np.diag(emp), g.sigma_diag, rtol=0.08)
    X, Wp = d["X"][0].astype(np.float64), d["W_planted"][0]
    resid = X - Wp @ g.S
    assert abs(resid.std() - 0.7) < 0.01


def test_ar1_noise_is_stationary_with_lag_one_correlation():
    w = synth.Workload("ar", 1, 2000, 2000, 400, 2, 1, rho_lo=1.0, rho_hi=1.0,
                       ar_phi=0.5)
    d = synth.generate(w, seed=0, want_planted=True)
    e = d["X"][0].astype(np.float64) - d["W_planted"][0] @ d["globals"].S
    assert abs(e.std() - 1.0) < 0.02
    r1 = np.mean(e[:, 1:] * e[:, :-1]) / np.mean(e * e)
    assert abs(r1 - 0.5) < 0.02
