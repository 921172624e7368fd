"""Host-side study of the Newton-Schulz forms the device's polar step uses
for G^{-1/2} (G = A_i^T A_i, the Gram of Eq. 4's polar factor), in FP64
NumPy with the device's start, stopping and certification rules.

Without a previous P_i to start from, the device runs the coupled form on
Y = G / |G|_F, Z = I: T = (3 I - Z Y) / 2, Y <- Y T, Z <- T Z.  The
uncoupled form X <- X + X E / 2 (E = I - X G X) from the same scaled
identity is the cheaper candidate; these tests show why it is not used, and
that the coupled form's result passes the device's certification
(max |I - X G X| <= 1e-12 and |X|_F^2 |G|_F < 1e13) where it should and fails
it (so the Jacobi eigensolver decides) for a rank-deficient Gram.  The
reference inverse square root comes from NumPy's symmetric eigendecomposition.
"""
import numpy as np
import pytest


def _gram(k, cond, seed):
    rng = np.random.default_rng(seed)
    q, _ = np.linalg.qr(rng.standard_normal((k, k)))
    lam = np.logspace(0.0, -np.log10(cond), k)
    return (q * lam) @ q.T


def _inv_sqrt(g):
    lam, v = np.linalg.eigh(g)
    return (v / np.sqrt(lam)) @ v.T


def _certified(x, g):
    e = np.abs(np.eye(len(g)) - x @ g @ x).max()
    return e <= 1e-12 and np.sum(x * x) * np.linalg.norm(g) < 1e13, e


def coupled(g, max_it=64):
    """The coupled form with the device's exits: converged (1e-14), diverging
    (1.5), or stalled at the rounding floor (below 1e-10, less than 4x
    progress in a step).  Returns X = Z / sqrt(s) and the step count."""
    s = np.linalg.norm(g)
    y, z = g / s, np.eye(len(g))
    prev = np.inf
    for it in range(max_it):
        e = np.abs(np.eye(len(g)) - z @ y).max()
        if e <= 1e-14 or not e < 1.5 or (e < 1e-10 and e > 0.25 * prev):
            break
        prev = e
        t = 1.5 * np.eye(len(g)) - 0.5 * z @ y
        y, z = y @ t, t @ z
    return z / np.sqrt(s), it


def uncoupled(g, max_it=64):
    """X <- X + X E / 2 from X_0 = I / sqrt(|G|_F), with the same exits."""
    x = np.eye(len(g)) / np.sqrt(np.linalg.norm(g))
    prev = np.inf
    for _ in range(max_it):
        e_m = np.eye(len(g)) - x @ g @ x
        e = np.abs(e_m).max()
        if e <= 1e-14 or not e < 1.5 or (e < 1e-10 and e > 0.25 * prev):
            break
        prev = e
        x = x + 0.5 * x @ e_m
        x = 0.5 * (x + x.T)
    return x


@pytest.mark.parametrize("k,cond", [(50, 10.0), (100, 1e2), (100, 1e4), (112, 1e4)])
def test_coupled_form_converges_and_is_certified(k, cond):
    g = _gram(k, cond, seed=k)
    x, steps = coupled(g)
    ok, e = _certified(x, g)
    assert ok, (e, steps)
    assert steps <= 40
    ref = _inv_sqrt(g)
    assert np.abs(x - ref).max() / np.abs(ref).max() < 1e-10


def test_uncoupled_form_from_a_scaled_identity_fails_where_the_coupled_one_holds():
    g = _gram(100, 1e3, seed=7)
    assert not _certified(uncoupled(g), g)[0]
    assert _certified(coupled(g)[0], g)[0]


def test_rank_deficient_gram_is_not_certified():
    g = _gram(60, 10.0, seed=3)
    lam, v = np.linalg.eigh(g)
    lam[:2] = 0.0  # two zero singular values of A_i
    g0 = (v * lam) @ v.T
    x, _ = coupled(g0)
    assert np.all(np.isfinite(x))
    assert not _certified(x, g0)[0]


def test_zero_gram_stays_finite_and_is_not_certified():
    g = np.zeros((20, 20))
    s = np.linalg.norm(g)
    # the device scales by 1 / |G|_F only when it is positive, so Y = 0
    y, z = g * 0.0, np.eye(20)
    for _ in range(64):
        t = 1.5 * np.eye(20) - 0.5 * z @ y
        y, z = y @ t, t @ z
    assert np.all(np.isfinite(z))
    x = z * (0.0 if s == 0.0 else 1.0 / np.sqrt(s))
    assert not _certified(x, g)[0]
