"""Benchmark of the SRM EM sweep on one MI355X: EM iterations per second.

The headline number is the BF16 hi+lo storage form (the BF16 form that meets
the 1e-3 error bar against the FP64 oracle) on the 1024-subject batched
workload; the plain FP32 form runs beside it on the same data.  One step is
one EM iteration (M-step on the current posterior, then the next E-step)
over all subjects, replayed as one captured hipGraph; inputs are resident in
HBM before the timed region starts.

Prints one JSON line.  --gpus N with N > 1 is refused: the sweep is measured
on one GPU (across GPUs it would shard by subject, with one all-reduce of the
k x t E-step sum per iteration, which is not implemented).
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "SRM EM iters/s + HBM GB/s, BF16-batched vs FP32 plain at fixed oracle error"
HBM_PEAK_GBS = 8000.0
MFMA_PEAK = {"bf16": 2500.0, "fp32": 157.3}  # dense TFLOP/s


def log(*a):
    print(*a, file=sys.stderr, flush=True)


KERNEL_SRC = os.path.join(ROOT, "paper_1608_04647_amd", "csrc", "srm_kernels.hip")


def kernel_source_hash(kernel: str) -> str:
    """SHA-256 (16 hex digits) of one kernel's own source text: from its
    template line (or __global__ line) to its closing brace."""
    import hashlib
    import re
    src = open(KERNEL_SRC).read()
    m = (re.search(r"^template <[^\n]*>\n__global__[^\n]*\b" + kernel + r"\(", src, re.M) or
         re.search(r"^__global__[^\n]*\b" + kernel + r"\(", src, re.M))
    if m is None:
        return "absent"
    end = src.index("\n}\n", m.start()) + 3
    return hashlib.sha256(src[m.start():end].encode()).hexdigest()[:16]


def committed_traffic(kernel: str, workload: str, prec: str):
    """HBM bytes per launch of `kernel` from the committed counter summary
    (profiles/<kernel>_<workload>_<prec>_traffic.md), or None when absent or
    taken on a different source of that kernel."""
    path = os.path.join(ROOT, "profiles", f"{kernel}_{workload}_{prec}_traffic.md")
    if not os.path.exists(path):
        return None
    vals = {}
    for line in open(path):
        if line.startswith("traffic:"):
            for kv in line.split(":", 1)[1].split():
                k_, v_ = kv.split("=")
                vals[k_] = v_
    if vals.get("source_sha256_16") != kernel_source_hash(kernel):
        return None
    try:
        return float(vals["bytes_per_launch"])
    except (KeyError, ValueError):
        return None


def algorithmic(w, v, prec):
    """Bytes and flops one EM iteration must move and compute (unpadded sizes).

    Per subject: the M-phase reads Xhat_i and writes A_i = Xhat_i S^T; the
    E-phase reads Xhat_i and A_i again (Z = A^T Xhat, G = A^T A).  A_i is kept
    as FP32 or as a BF16 hi+lo pair: 4 bytes per element either way."""
    V = float(np.sum(v))
    bx = {"fp32": 4, "bf16": 2, "bf16x2": 4}[prec]
    x_bytes = V * w.t * bx
    a_bytes = V * w.k * 4
    mph = {"bytes": x_bytes + a_bytes, "flops": 2.0 * V * w.t * w.k}
    eph = {"bytes": x_bytes + a_bytes, "flops": 2.0 * V * w.t * w.k + 2.0 * V * w.k * w.k}
    # The fused sweep reads Xhat once and never stores A.
    fus = {"bytes": x_bytes, "flops": mph["flops"] + eph["flops"]}
    return {"mphase": mph, "ephase": eph, "fused": fus,
            "iter_bytes": mph["bytes"] + eph["bytes"],
            "iter_flops": mph["flops"] + eph["flops"]}


def paper_flop_model(v, t, k):
    """Floating-point operations of one EM iteration by the count the paper
    uses for its Gflop/s figures (Sec. V-A): per subject, two v_i x t x k
    matrix products, one v_i x k x k product, and an economy SVD of the
    v_i x k matrix counted as Householder QR, 2 m n^2 - 2 n^3 / 3."""
    v = np.asarray(v, dtype=np.float64)
    return float(np.sum(2.0 * 2.0 * v * t * k + 2.0 * v * k * k
                        + 2.0 * v * k * k - 2.0 * k ** 3 / 3.0))


def copy_stream_GBps(nbytes=4_000_000_000, reps=5):
    """Best-of-reps rate of a plain device-to-device copy of nbytes (bytes
    read plus bytes written, per second)."""
    import torch
    src = torch.ones(nbytes // 4, dtype=torch.float32, device="cuda")
    dst = torch.empty_like(src)
    best = float("inf")
    for _ in range(reps + 1):  # the first call warms up
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        dst.copy_(src)
        torch.cuda.synchronize()
        best = min(best, time.perf_counter() - t0)
    del src, dst
    torch.cuda.empty_cache()
    return 2 * nbytes / best / 1e9


def time_fit(g, steps):
    import torch
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    ll = g.fit(steps)  # synchronises the library's stream at the end
    torch.cuda.synchronize()
    return time.perf_counter() - t0, ll


def open_fit(srm, X, W0, w, v, prec, gram, seed):
    """The fit of one form: from the device-resident data, or (X is None)
    ingested one subject at a time from host memory as the subjects are
    generated, through the library's staging buffers."""
    from paper_1608_04647_amd import synth
    if X is not None:
        return srm.SRM(X, w.k, prec=prec, W0=W0, flags=srm.SRM_NO_W0_CHECK, gram=gram)
    t0 = time.perf_counter()
    g = srm.SRM.begin([int(x) for x in v], w.t, w.k, prec=prec, stream_from_host=True,
                      flags=srm.SRM_NO_W0_CHECK, gram=gram)
    ingest_s = 0.0
    last = None
    for i, Xi, W0i in synth.iter_subjects(w, seed, threads=4):
        t1 = time.perf_counter()
        g.ingest(i, Xi, W0i)
        ingest_s += time.perf_counter() - t1
        last = Xi
        if i % 16 == 15:
            log(f"[bench] {i + 1}/{w.n_subjects} subjects ingested")
    g.end()
    g.ingest_seconds = ingest_s
    g.gen_and_ingest_seconds = time.perf_counter() - t0
    # For comparison: a plain host-to-device copy of one subject's FP32 rows
    # from the same kind of (pageable) host memory, no conversion.
    import torch
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    dev = torch.from_numpy(last).to("cuda")
    torch.cuda.synchronize()
    g.plain_copy_GBps = last.nbytes / (time.perf_counter() - t1) / 1e9
    del dev
    return g


def run_form(srm, X, W0, w, v, prec, steps, warmup, prof_steps, gram=False, tune=True,
             table=False, seed=0):
    log(f"[bench] init {prec}{' sample-space' if gram else ''}")
    g = open_fit(srm, X, W0, w, v, prec, gram, seed)
    # the library's own initialisation (W0 upload, conversion, G_i for the
    # sample-space variant, first E-step; with host ingestion its ingest calls
    # and srm_init_end, not the generation of the data); the caller's
    # workspace allocation is not part of it
    init_s = g.init_seconds if X is not None else g.ingest_seconds + g.end_seconds
    ingest = None
    if X is None:
        fp32 = float(np.sum(v)) * w.t * 4
        ingest = {"host_ingest_s": g.ingest_seconds, "generate_and_ingest_s":
                  g.gen_and_ingest_seconds, "end_s": g.end_seconds,
                  "ingest_GBps": fp32 / g.ingest_seconds / 1e9,
                  "plain_h2d_copy_GBps": g.plain_copy_GBps,
                  "note": "srm_ingest of host rows (upload through two staging buffers on a "
                          "second stream, conversion to the stored format on the compute "
                          "stream) against a plain pageable copy of one subject"}
    default_shape = g.tuning()
    tuning = {"default": default_shape}
    if table:  # every sweep shape at the default reduction, timed alike
        rows = []
        for t in g.tuning_candidates():
            if t["reduce_wgs"] != default_shape["reduce_wgs"]:
                continue
            g.set_tuning(t)
            g.fit(1)
            dt_, _ = time_fit(g, 5)
            rows.append(dict(t, ms=1e3 * dt_ / 5))
            log(f"[bench] shape {t}: {rows[-1]['ms']:.3f} ms/iter")
        tuning["table"] = rows
        g.set_tuning(default_shape)
    if tune:
        t0 = time.perf_counter()
        best, best_ms = g.autotune(trials=2)
        tuning.update(chosen=best, autotune_ms_per_iter=best_ms,
                      autotune_s=time.perf_counter() - t0)
        log(f"[bench] autotuned {prec}: {best} ({best_ms:.3f} ms/iter in its trials)")
    # the first iteration of the fit, phase by phase (its polar step has no
    # previous P_i to start from), then the state it started from again
    st0 = g.get_state()
    first_ph = g.profile(1)
    g.set_state(st0)
    log(f"[bench] first iteration ({prec}): polar {first_ph.get('polar', 0.0):.3f} ms")
    log(f"[bench] init {prec} done in {init_s:.2f}s; warmup {warmup}")
    if warmup:
        g.fit(warmup)
    compare = tune and tuning["chosen"] != default_shape
    st_w = g.get_state() if compare else None
    log(f"[bench] timing {steps} iterations ({prec})")
    dt, ll = time_fit(g, steps)
    log(f"[bench] {prec}: {steps / dt:.2f} iters/s; profiling {prof_steps} iterations")
    if compare:
        # the default shape over the same iterations from the same state (the
        # first iterations of a fit can carry cold polar solves), for
        # comparison; then the tuned fit's state again
        st_t = g.get_state()
        cur = g.tuning()
        g.set_tuning(default_shape)
        g.fit(1)  # captures the default shape's graph
        g.set_state(st_w)
        dt_d, _ = time_fit(g, steps)
        tuning["default_ms_per_step"] = 1e3 * dt_d / steps
        g.set_tuning(cur)
        g.set_state(st_t)
        log(f"[bench] default shape: {steps / dt_d:.2f} iters/s")
    info = g.info()  # after the timed srm_fit: which sweep ran, and whether it
    # replayed the captured graph
    ph = g.profile(prof_steps)
    ph = {k: v_ / prof_steps for k, v_ in ph.items()}
    alg = algorithmic(w, v, prec)
    if ph.get("fused", 0.0) > 0.0:  # one-pass sweep: Xhat read once, A never stored
        alg["iter_bytes"] = alg["fused"]["bytes"]
    if gram:  # per iteration: G_i (t x t; FP32 for the BF16 forms, FP64 for FP32
        # storage) read once, S G_i and S G_i S^T
        Nn, t, k = float(len(v)), float(w.t), float(w.k)
        gb = 8 if prec == "fp32" else 4
        alg["gram"] = {"bytes": Nn * t * t * gb, "flops": 2.0 * Nn * k * t * t + 2.0 * Nn * k * k * t}
        alg["iter_bytes"], alg["iter_flops"] = alg["gram"]["bytes"], alg["gram"]["flops"]
    res = {"iters_per_s": steps / dt, "ms_per_step": 1e3 * dt / steps, "init_s": init_s,
           "tuning": tuning, "ingest": ingest,
           "sweep": info["sweep"], "graph_replayed": info["graph"],
           "hbm_GBps": alg["iter_bytes"] / (dt / steps) / 1e9,
           "phase_ms": ph, "first_iteration_phase_ms": first_ph, "alg": alg,
           "ll_last": float(ll[-1]) if len(ll) else None}
    return g, res


def snapshot(g, picks):
    """Host copies of a device fit's results for the oracle comparison."""
    return {"S": g.S().cpu().numpy().astype(np.float64), "Sigma_s": g.sigma_s(),
            "rho2": g.rho2(), "ll": g.loglik(), "iters": g.iterations(),
            "W": {i: g.W(i).cpu().numpy() for i in picks}}


def oracle_check(w, seed, snap):
    """Errors of the device fit against the FP64 oracle run for the same
    number of iterations on every subject (its Gram form, each subject
    regenerated from the seed and summarised one at a time): S after the
    Procrustes rotation, Sigma_s, every rho_i^2, every log-likelihood, and the
    projectors of the sampled subjects."""
    sys.path.insert(0, os.path.join(ROOT, "tests"))
    from _parity import procrustes, proj_err
    from _streamed import oracle_fit, oracle_w
    n = snap["iters"]
    t0 = time.perf_counter()
    step = max(1, w.n_subjects // 16)

    def progress(done):
        if done % step == 0 or done == w.n_subjects:
            log(f"[oracle] {done}/{w.n_subjects} subjects summarised "
                f"({time.perf_counter() - t0:.0f} s)")

    ora = oracle_fit(w, n, seed, progress=progress)
    log(f"[oracle] {n} iterations done ({time.perf_counter() - t0:.0f} s)")
    Q, eS, _ = procrustes(ora["S"], snap["S"])
    eSig = float(np.linalg.norm(ora["Sigma_s"] - Q @ snap["Sigma_s"] @ Q.T)
                 / np.linalg.norm(ora["Sigma_s"]))
    ll_o = np.array(ora["ll"] + [ora["ll_final"]])
    ll_g = snap["ll"][:len(ll_o)]
    eW = 0.0
    for i, Wg in snap["W"].items():
        eW = max(eW, proj_err(oracle_w(ora, w, i, seed), Wg))
        log(f"[oracle] projector of subject {i} checked ({time.perf_counter() - t0:.0f} s)")
    return {"oracle": f"FP64 Gram form on streamed input, all {w.n_subjects} subjects, "
                      f"{n} iterations from the same W0",
            "S": float(eS), "Sigma_s": eSig,
            "rho2_max": float(np.max(np.abs(snap["rho2"] / ora["rho2"] - 1))),
            "loglik_max": float(np.max(np.abs(ll_g - ll_o) / np.abs(ll_o))),
            "projector_max": float(eW), "projector_subjects": sorted(snap["W"]),
            "oracle_s": time.perf_counter() - t0}


def cpu_baseline(w, seed, n_sub):
    """The FP64 oracle as it stands, timed on a sample of the workload's subjects;
    seconds per EM iteration scaled linearly by total voxels."""
    import oracle
    from paper_1608_04647_amd import synth
    try:
        from threadpoolctl import threadpool_info
        cores = max([d.get("num_threads", 1) for d in threadpool_info()] + [1])
    except Exception:
        cores = os.cpu_count() or 1
    sub = list(range(n_sub))
    d = synth.generate(w, seed=seed, subjects=sub)
    t0 = time.perf_counter()
    oracle.em_fit(d["X"], w.k, 1, d["W0"])
    t1 = time.perf_counter()
    oracle.em_fit(d["X"], w.k, 3, d["W0"])
    t2 = time.perf_counter()
    per_iter = ((t2 - t1) - (t1 - t0)) / 2.0
    v_all = synth.draw_globals(w, seed).v
    scale = float(np.sum(v_all)) / float(sum(x.shape[0] for x in d["X"]))
    return {"value": 1.0 / (per_iter * scale), "unit": "iters/s", "cores": int(cores),
            "kind": "oracle",
            "sample": f"NumPy FP64 oracle, {n_sub} of {w.n_subjects} subjects, "
                      f"2 EM iterations timed ({per_iter:.2f} s/iter), scaled by total "
                      f"voxels x{scale:.1f} (extrapolated)"}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--workload", default="batch1024")
    ap.add_argument("--seed", type=int, default=0)
    ap.add_argument("--forms", default="bf16x2,fp32")
    ap.add_argument("--profile-steps", type=int, default=5)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-check", action="store_true")
    ap.add_argument("--no-stream", action="store_true",
                    help="skip the plain copy-stream rate measured after the fits")
    ap.add_argument("--cpu-subjects", type=int, default=24)
    ap.add_argument("--subjects", type=int, default=0,
                    help="development only: fewer subjects of the same shape")
    ap.add_argument("--no-gram", action="store_true",
                    help="skip the sample-space (G_i = Xhat_i^T Xhat_i) variant")
    ap.add_argument("--no-autotune", action="store_true",
                    help="keep the library's default launch shapes")
    ap.add_argument("--tuning-table", action="store_true",
                    help="also time every sweep shape of the headline form")
    ap.add_argument("--copy-probe", type=float, default=0.0,
                    help="GB: also run one plain device copy of this size "
                         "(calibrates FETCH_SIZE / WRITE_SIZE counters)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py runs on exactly one GPU; --gpus {args.gpus} is not supported "
              "(sharding subjects across GPUs is not implemented)", file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_1608_04647_amd import srm, synth
    w = synth.WORKLOADS[args.workload]
    if args.subjects:
        w = w.scaled(n_subjects=args.subjects)
    forms = args.forms.split(",")
    log(f"[bench] generating {w.name}: {w.n_subjects} subjects, v {w.v_lo}-{w.v_hi}, "
        f"t={w.t}, k={w.k}")
    t0 = time.time()
    gl = synth.draw_globals(w, args.seed)
    v = gl.v
    fp32_bytes = float(np.sum(v)) * w.t * 4
    ws_max = max(srm.workspace_size(v, w.t, w.k, p) for p in forms)
    if fp32_bytes + ws_max > 0.9 * torch.cuda.get_device_properties(0).total_memory:
        # FP32 data and the workspace do not fit together: each form ingests
        # the subjects one at a time from host memory
        X = W0 = None
        log(f"[bench] {fp32_bytes / 1e9:.1f} GB FP32 + {ws_max / 1e9:.1f} GB workspace exceed "
            f"the device: subjects are ingested from host memory one at a time")
    else:
        X, W0, gl = synth.to_device(w, args.seed)
        log(f"[bench] data on device in {time.time() - t0:.1f}s ({fp32_bytes / 1e9:.1f} GB FP32)")

    results = {}
    snap = None
    for prec in forms:
        g, res = run_form(srm, X, W0, w, v, prec, args.steps, args.warmup, args.profile_steps,
                          tune=not args.no_autotune,
                          table=args.tuning_table and prec == forms[0], seed=args.seed)
        if prec == forms[0] and not args.no_check:
            picks = sorted({int(round(x)) for x in np.linspace(0, w.n_subjects - 1, 8)})
            snap = snapshot(g, picks)
        results[prec] = res
        g.close()
        del g
        torch.cuda.empty_cache()
    gram_res = None
    if not args.no_gram:
        g, gram_res = run_form(srm, X, W0, w, v, forms[0], args.steps, args.warmup,
                               args.profile_steps, gram=True, tune=not args.no_autotune,
                               seed=args.seed)
        g.close()
        del g
        torch.cuda.empty_cache()
    del X, W0
    torch.cuda.empty_cache()

    head = results[forms[0]]
    ph = head["phase_ms"]
    dom = max(("fused", "ephase", "mphase"), key=lambda k_: ph.get(k_, 0.0))
    alg = head["alg"][dom]
    dur = ph[dom] / 1e3
    hp = forms[0]
    if hp == "fp32":
        roof = {"bound": "mfma", "achieved": alg["flops"] / dur / 1e12,
                "peak": MFMA_PEAK["fp32"], "unit": "TFLOP/s"}
    else:
        roof = {"bound": "hbm", "achieved": alg["bytes"] / dur / 1e9,
                "peak": HBM_PEAK_GBS, "unit": "GB/s"}
    roof["frac"] = roof["achieved"] / roof["peak"]
    shape = head["tuning"].get("chosen", head["tuning"]["default"])
    if dom == "fused":
        kname = "k_staged" if shape["sweep_kernel"] == 1 else "k_fused"
    else:  # the two-pass kernels of the BF16 forms stage their shared operand in LDS
        kname = f"k_{dom}" if hp == "fp32" else f"k_{dom}_s"
    roof["traffic"] = committed_traffic(kname, w.name if not args.subjects else
                                        f"{w.name}-{args.subjects}", hp)
    roof["kernel"] = kname
    roof["kernel_ms"] = ph[dom]

    out = {"metric": METRIC, "value": head["iters_per_s"], "unit": "iters/s", "n_gpus": 1,
           "steps": args.steps, "warmup": args.warmup, "ms_per_step": head["ms_per_step"],
           "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
           "dtype": "bf16" if hp != "fp32" else "fp32",
           "data": "synthetic (planted SRM model, seeded)",
           "config": {"workload": w.name, "subjects": w.n_subjects,
                      "voxels": [w.v_lo, w.v_hi], "total_voxels": int(np.sum(v)),
                      "trs": w.t, "features": w.k, "storage": hp},
           "hbm_GBps": head["hbm_GBps"],
           "hbm_frac": head["hbm_GBps"] / HBM_PEAK_GBS,
           "phase_ms": ph,
           "first_iteration_phase_ms": head["first_iteration_phase_ms"],
           "tuning": head["tuning"],
           "sweep": head["sweep"], "graph_replayed": head["graph_replayed"],
           "paper_model_GFLOPs": paper_flop_model(v, w.t, w.k) / (head["ms_per_step"] / 1e3) / 1e9,
           "roofline": roof}
    if head["ingest"] is not None:
        out["ingest"] = head["ingest"]
    for prec in forms[1:]:
        r = results[prec]
        out[f"{prec}_plain" if prec == "fp32" else prec] = {
            "iters_per_s": r["iters_per_s"], "ms_per_step": r["ms_per_step"],
            "hbm_GBps": r["hbm_GBps"], "phase_ms": r["phase_ms"], "tuning": r["tuning"],
            "sweep": r["sweep"], "graph_replayed": r["graph_replayed"],
            "mfma_TFLOPs": r["alg"]["iter_flops"] / (r["ms_per_step"] / 1e3) / 1e12,
            "paper_model_GFLOPs": paper_flop_model(v, w.t, w.k) / (r["ms_per_step"] / 1e3) / 1e9}
        out[f"speedup_vs_{prec}"] = head["iters_per_s"] / r["iters_per_s"]
    if gram_res is not None:
        ga = gram_res["alg"]["gram"]
        gms = gram_res["phase_ms"].get("gram", 0.0)
        n_fit = w.n_iter
        out["sample_space_variant"] = {
            "note": "separate variant, not the headline: G_i = Xhat_i^T Xhat_i formed once "
                    "in init, iterations read no voxel data",
            "storage": forms[0], "iters_per_s": gram_res["iters_per_s"],
            "ms_per_step": gram_res["ms_per_step"], "phase_ms": gram_res["phase_ms"],
            "init_s": gram_res["init_s"], "streamed_init_s": head["init_s"],
            "fit_s_at_workload_iters": {
                "iters": n_fit,
                "sample_space": gram_res["init_s"] + n_fit * gram_res["ms_per_step"] / 1e3,
                "streamed": head["init_s"] + n_fit * head["ms_per_step"] / 1e3},
            "k_gram_z_TFLOPs": ga["flops"] / (gms / 1e3) / 1e12 if gms > 0 else None,
            "k_gram_z_GBps": ga["bytes"] / (gms / 1e3) / 1e9 if gms > 0 else None}
    if snap is not None:
        log(f"[bench] oracle check: {snap['iters']} iterations on all {w.n_subjects} subjects")
        out["error_vs_oracle"] = oracle_check(w, args.seed, snap)
        log(f"[bench] oracle check {out['error_vs_oracle']}")
    if not args.no_stream:
        # What a plain streaming copy reaches on this device (bytes read and
        # written), as the practical counterpart of the 8 TB/s peak; measured
        # after the fits, outside any timed region.
        cs = copy_stream_GBps()
        out["copy_stream"] = {"GBps": cs, "method": "device-to-device copy of 4 GB "
                              "(torch), best of 5; bytes read plus bytes written"}
        if roof["unit"] == "GB/s":
            roof["frac_of_copy_stream"] = roof["achieved"] / cs
            log(f"[bench] copy stream: {cs:.0f} GB/s; the dominant kernel reaches "
                f"{100 * roof['achieved'] / cs:.0f}% of it")
    if args.copy_probe > 0:
        nbytes = int(args.copy_probe * 1e9) // 4 * 4
        src = torch.ones(nbytes // 4, dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        dst.copy_(src)
        torch.cuda.synchronize()
        out["copy_probe_bytes"] = nbytes
        del src, dst
        log(f"[bench] copy probe: {nbytes} bytes read and written")
    if not args.no_cpu_baseline:
        log("[bench] CPU baseline (oracle)")
        out["cpu_baseline"] = cpu_baseline(w, args.seed, min(args.cpu_subjects, w.n_subjects))
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
