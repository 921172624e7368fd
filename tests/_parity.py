"""Comparison helpers for device-vs-oracle parity (no SRM arithmetic here)."""
import math

import numpy as np


def procrustes(S_ref, S):
    """Q = argmin ||S_ref - Q S|| over orthogonal Q; returns (Q, rel err, raw rel err)."""
    U, _, Vt = np.linalg.svd(S_ref @ S.T)
    Q = U @ Vt
    n = np.linalg.norm(S_ref)
    return Q, np.linalg.norm(S_ref - Q @ S) / n, np.linalg.norm(S_ref - S) / n


def proj_err(W1, W2):
    """||W1 W1^T - W2 W2^T||_F / sqrt(k) without forming v x v matrices."""
    W1 = np.asarray(W1, np.float64)
    W2 = np.asarray(W2, np.float64)
    k = W1.shape[1]
    a = np.linalg.norm(W1.T @ W1, "fro") ** 2 + np.linalg.norm(W2.T @ W2, "fro") ** 2 \
        - 2 * np.linalg.norm(W1.T @ W2, "fro") ** 2
    return math.sqrt(max(a, 0.0)) / math.sqrt(k)


def bf16_round(x32):
    """Round-to-nearest-even float32 -> bfloat16 (returned as float32)."""
    u = np.ascontiguousarray(x32, dtype=np.float32).view(np.uint32).astype(np.uint64)
    u = (u + 0x7FFF + ((u >> 16) & 1)) & 0xFFFF0000
    return u.astype(np.uint32).view(np.float32)


def stored_values(X, prec):
    """The demeaned values the device stores for one subject, as float64."""
    X = np.asarray(X, np.float32)
    mu = X.astype(np.float64).mean(axis=1, keepdims=True)
    f = (X.astype(np.float64) - mu).astype(np.float32)
    if prec == "fp32":
        return f.astype(np.float64)
    hi = bf16_round(f)
    if prec == "bf16":
        return hi.astype(np.float64)
    lo = bf16_round(f - hi)
    return hi.astype(np.float64) + lo.astype(np.float64)


def compare(gpu, ora, N):
    """Errors of a device fit against an oracle fit (dict of floats)."""
    S_g = gpu.S().cpu().numpy().astype(np.float64)
    Q, eS, eS_raw = procrustes(ora["S"], S_g)
    eW = max(proj_err(ora["W"][i], gpu.W(i).cpu().numpy()) for i in range(N))
    rho = gpu.rho2()
    er = float(np.max(np.abs(rho / ora["rho2"] - 1)))
    sig = gpu.sigma_s()
    es = np.linalg.norm(ora["Sigma_s"] - Q @ sig @ Q.T) / np.linalg.norm(ora["Sigma_s"])
    ll_g = gpu.loglik()
    ll_o = np.array(ora["ll"] + ([ora["ll_final"]] if "ll_final" in ora else []))
    n = min(len(ll_g), len(ll_o))
    ell = float(np.max(np.abs(ll_g[:n] - ll_o[:n]) / np.abs(ll_o[:n])))
    orth = max(float(np.abs(gpu.W(i).cpu().numpy().astype(np.float64).T
                            @ gpu.W(i).cpu().numpy().astype(np.float64)
                            - np.eye(ora["S"].shape[0])).max()) for i in range(N))
    return {"S": eS, "S_raw": eS_raw, "W": eW, "rho2": er, "Sigma_s": es, "ll": ell,
            "orth": orth, "ll_gpu": ll_g}
