"""Plants plausible mistakes in a copy of the oracle (on the CPU) and checks
that the pins in test_oracle.py catch every one of them: a dropped term, a
wrong sign, a wrong normalisation, a skipped step."""
import os
import shutil
import subprocess
import sys
from concurrent.futures import ThreadPoolExecutor

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
ORACLE = os.path.join(ROOT, "oracle", "srm_oracle.py")

RHO = "(c - 2.0 * tr_wa + t * tau) / (t * v)"
SMEAN = "S = Sigma_s @ (np.eye(k) - rho0 * M) @ Y"
SIGUPD = "Sigma_s = M + (S @ S.T) / t\n        Sigma_s = 0.5 * (Sigma_s + Sigma_s.T)  # R8"
YRED = "Y += (1.0 / rho2[i]) * (W[i].T @ Xh[i])\n        S, M, rho0"
MUTATIONS = {
    "rho: dropped t*tr(Sigma_s) term": (RHO, "(c - 2.0 * tr_wa) / (t * v)"),
    "rho: wrong sign of cross term": (RHO, "(c + 2.0 * tr_wa + t * tau) / (t * v)"),
    "rho: cross term without factor 2": (RHO, "(c - tr_wa + t * tau) / (t * v)"),
    "rho: total V instead of v_i": (RHO, "(c - 2.0 * tr_wa + t * tau) / (t * v * 1.5)"),
    "Eq.10: sign inside bracket": (SMEAN, SMEAN.replace("- rho0", "+ rho0")),
    "Eq.10: Sigma_s factor dropped": (SMEAN, "S = (np.eye(k) - rho0 * M) @ Y"),
    "Eq.8: rho0 sums rho^2": ("rho0 = float(np.sum(1.0 / rho2))", "rho0 = float(np.sum(rho2))"),
    "Eq.7: rho0 dropped from B": ("B = Sinv + rho0 * np.eye(k)", "B = Sinv + np.eye(k)"),
    "Eq.11: posterior covariance dropped": (SIGUPD, SIGUPD.replace("M + (S @ S.T) / t", "(S @ S.T) / t")),
    "Eq.11: 1/T dropped": (SIGUPD, SIGUPD.replace("(S @ S.T) / t", "(S @ S.T)")),
    "Eq.10: rho^-2 weight dropped": (YRED, YRED.replace("(1.0 / rho2[i]) * ", "")),
    "Eq.10: rho^-1 instead of rho^-2": (YRED, YRED.replace("(1.0 / rho2[i])", "(1.0 / np.sqrt(rho2[i]))")),
    "Eq.4: S rows rescaled": ("A = Xh @ S.T\n", "A = Xh @ (S / np.linalg.norm(S, axis=1, keepdims=True)).T\n"),
    "init: no demeaning": ("Xh = X - mu[:, None]", "Xh = X"),
    "loglik: sign of quadratic term": ("float(np.sum(c / rho2)) - float(", "float(np.sum(c / rho2)) + float("),
    "loglik: rho0 dropped in logdet": ("np.eye(k) + rho0 * Sigma_s)", "np.eye(k) + Sigma_s)"),
    "loglik: v_i weight dropped": ("t * float(np.sum(v * np.log(rho2)))", "t * float(np.sum(np.log(rho2)))"),
    "Eq.4: U instead of U V^T": ("return U @ Vt, float(sig.sum())", "return U, float(sig.sum())"),
    "init: Sigma_s starts at 2I": ("Sigma_s = np.eye(k)  # R3", "Sigma_s = 2.0 * np.eye(k)  # R3"),
    "z-score: sample std (1/(t-1))": ("sd = np.sqrt(np.mean(D * D, axis=1))",
                                      "sd = np.sqrt(np.sum(D * D, axis=1) / (X.shape[1] - 1))"),
    "z-score: constant voxels not kept at zero": ("keep = sd > 0", "keep = sd >= 0"),
    "Philox: key not advanced between rounds": ("k0 = k0 + _PHILOX_W[0]", "k0 = k0"),
    "Philox: words of the round swapped": ("c = [hi1 ^ c[1] ^ k0, lo1, hi0 ^ c[3] ^ k1, lo0]",
                                           "c = [hi0 ^ c[1] ^ k0, lo1, hi1 ^ c[3] ^ k1, lo0]"),
    "Box-Muller: one uniform for radius and angle": (
        "r0 * np.cos(2.0 * np.pi * u[1]), r0 * np.sin(2.0 * np.pi * u[1])",
        "r0 * np.cos(2.0 * np.pi * u[0]), r0 * np.sin(2.0 * np.pi * u[0])"),
    "Box-Muller: radius without the factor 2": ("r0 = np.sqrt(-2.0 * np.log(u[0]))",
                                                "r0 = np.sqrt(-np.log(u[0]))"),
    "Gram form: W0 start not applied": ("np.asarray(W0i, dtype=np.float64).T @ xh",
                                        "xh[:W0i.shape[1]]"),
    "Gram form: rho^-2 weight dropped": ("            Y += (1.0 / rho2[i]) * Z[i]\n        S, M",
                                         "            Y += Z[i]\n        S, M"),
}


def _run(item, base):
    name, (a, b) = item
    src = open(ORACLE).read()
    assert a in src, name
    d = os.path.join(base, str(abs(hash(name))))
    os.makedirs(os.path.join(d, "oracle"))
    shutil.copy(os.path.join(ROOT, "oracle", "__init__.py"), os.path.join(d, "oracle"))
    with open(os.path.join(d, "oracle", "srm_oracle.py"), "w") as f:
        f.write(src.replace(a, b))
    os.makedirs(os.path.join(d, "tests"))
    for f in ("conftest.py", "test_oracle.py"):
        shutil.copy(os.path.join(ROOT, "tests", f), os.path.join(d, "tests"))
    os.makedirs(os.path.join(d, "paper_1608_04647_amd"))
    for f in ("__init__.py", "synth.py"):
        shutil.copy(os.path.join(ROOT, "paper_1608_04647_amd", f),
                    os.path.join(d, "paper_1608_04647_amd"))
    env = dict(os.environ, OMP_NUM_THREADS="2", OPENBLAS_NUM_THREADS="2")
    r = subprocess.run([sys.executable, "-m", "pytest", "-q", "-x", "-p", "no:cacheprovider",
                        "tests/test_oracle.py"], cwd=d, capture_output=True, text=True, env=env)
    return name, r.returncode


def test_every_planted_mistake_is_caught(tmp_path):
    with ThreadPoolExecutor(4) as ex:
        res = list(ex.map(lambda it: _run(it, str(tmp_path)), MUTATIONS.items()))
    missed = [n for n, rc in res if rc == 0]
    assert not missed, f"pins missed: {missed}"
