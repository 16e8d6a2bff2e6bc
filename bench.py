"""Benchmark: rank-k PCA solves/s on one MI355X, plus HBM GB/s per pass over A.

Workload (one step = one whole solve): dense float32 A of 100000 x 4000 built
as U diag(sigma) V^T with Haar U, V and sigma_j = 1/j (j <= 50), then
1e-3 exp(-(j-51)/200); PCA of the column-centered matrix with k = 50,
l = 60, its = 2 (six passes over A).  A is generated on the device and is
resident in HBM before timing starts.

Prints one JSON line.  ``roofline`` is for the dominant kernel (the product
pass that takes the most time): algorithmic bytes per launch divided by the
average launch duration, measured with HIP events recorded by the library on
its stream over the timed region.  ``cpu_baseline`` times the FP64 oracle on
this host's cores on a bounded sample of the same workload.
"""

import argparse
import json
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, HERE)

METRIC = "rank-k PCA solves/s + HBM GB/s per A-pass; BF16 vs FP32 at err≤1.1·σ_{k+1}"
HBM_PEAK_GBS = 8000.0


def parse():
    p = argparse.ArgumentParser()
    p.add_argument("--gpus", type=int, default=1)
    p.add_argument("--steps", type=int, default=20)
    p.add_argument("--warmup", type=int, default=3)
    p.add_argument("--m", type=int, default=100000)
    p.add_argument("--n", type=int, default=4000)
    p.add_argument("--k", type=int, default=50)
    p.add_argument("--l", type=int, default=60)
    p.add_argument("--its", type=int, default=2)
    p.add_argument("--seed", type=int, default=2002)
    p.add_argument("--no-cpu-baseline", action="store_true",
                   help="skip the oracle leg (profiling runs)")
    p.add_argument("--cpu-sample-solves", type=int, default=3)
    p.add_argument("--no-precision", action="store_true",
                   help="skip the bfloat16 / E4M3 precision-form measurement")
    p.add_argument("--precision-steps", type=int, default=10)
    p.add_argument("--no-batched", action="store_true",
                   help="skip the 512-problem batched workload report")
    p.add_argument("--precision-only", action="store_true",
                   help="run only the precision-form configuration (200000x8000, k=100, l=120, "
                        "its=3) and print its report")
    p.add_argument("--batched-only", action="store_true",
                   help="run only the 512-problem batched workload (for profiling it) and print "
                        "its report")
    p.add_argument("--no-tune", action="store_true",
                   help="skip the autotuner (built-in tile configurations)")
    p.add_argument("--passes-only", action="store_true",
                   help="time the solves of the main workload and report the passes only: "
                        "no other workload, no cpu baseline and no exact error norm (for "
                        "counter-collecting profiler runs: the norm's torch.linalg.eigvalsh "
                        "does not survive rocprofv3 --pmc); err_over_sigma_k1 is null.  With "
                        "--precision-only: that workload without its exact norms")
    p.add_argument("--no-sparse", action="store_true",
                   help="skip the 10^6 x 10^6 sparse workload report")
    p.add_argument("--sparse-only", action="store_true",
                   help="run only the 10^6 x 10^6 sparse workload (for profiling it) and print "
                        "its report")
    p.add_argument("--no-noisy", action="store_true",
                   help="skip the rank-4 noisy Gaussian workload (n = 10^5, its = 0, 2, 4)")
    p.add_argument("--noisy-n", type=int, default=100000)
    p.add_argument("--no-fused", action="store_true",
                   help="skip the schedule that renormalizes every second application")
    p.add_argument("--no-fused-bf16-oracle", action="store_true",
                   help="skip the oracle's bfloat16-copy solve of the fused schedule "
                        "(about 20 s of host time)")
    p.add_argument("--renorm", choices=("chol", "lu", "orth"), default="chol",
                   help="renormalization between applications: one Cholesky QR pass (the "
                        "library's default), pivoted LU (the paper's) "
                        "or Cholesky QR")
    p.add_argument("--traffic-json", default=os.path.join(HERE, "profiles", "traffic.json"),
                   help="HBM bytes per launch measured by rocprofv3 counters")
    p.add_argument("--traffic-from-pmc", nargs=5, metavar=("FETCH_DIR", "WRITE_DIR",
                                                           "CAL_FETCH_DIR", "CAL_WRITE_DIR",
                                                           "COPY_BYTES"),
                   help="write --traffic-json from rocprofv3 --pmc FETCH_SIZE / WRITE_SIZE "
                        "runs of this bench and of a plain copy of COPY_BYTES bytes, then exit")
    return p.parse_args()


# Kernel sources whose change invalidates stored counter readings.
TRAFFIC_SOURCES = ("paper_1412_3510_amd/csrc/ax_tall.hip", "paper_1412_3510_amd/csrc/atx_wide.hip",
                   "paper_1412_3510_amd/csrc/gemm.hip", "paper_1412_3510_amd/csrc/dma.h",
                   "paper_1412_3510_amd/csrc/common.h")
PASS_KERNELS = {"ax": "rpca::ax_tall_kernel", "atx": "rpca::atx_wide_kernel"}


def _sources_digest():
    import hashlib
    h = hashlib.sha256()
    for rel in TRAFFIC_SOURCES:
        with open(os.path.join(HERE, rel), "rb") as f:
            h.update(f.read())
    return h.hexdigest()


def _counter_rows(d):
    import csv
    with open(os.path.join(d, "run_counter_collection.csv")) as f:
        return list(csv.DictReader(f))


def traffic_from_pmc(args):
    """HBM bytes per pass launch from rocprofv3 counters (KiB per dispatch).

    Each counter is scaled by copy_bytes / (what it reads for the plain copy),
    so FETCH_SIZE and WRITE_SIZE both report the copy's true size.
    """
    fetch_dir, write_dir, cal_f, cal_w, copy_bytes = args.traffic_from_pmc
    copy_bytes = float(copy_bytes)

    def copy_kib(d):
        vals = [float(r["Counter_Value"]) for r in _counter_rows(d)
                if "copyBuffer" in r["Kernel_Name"]]
        return max(vals)

    sf = copy_bytes / (1024.0 * copy_kib(cal_f))
    sw = copy_bytes / (1024.0 * copy_kib(cal_w))
    out = {"m": args.m, "n": args.n, "l": args.l, "sources_sha256": _sources_digest(),
           "fetch_scale": sf, "write_scale": sw, "copy_bytes": copy_bytes}
    for q, name in PASS_KERNELS.items():
        fk = [float(r["Counter_Value"]) for r in _counter_rows(fetch_dir) if name in r["Kernel_Name"]]
        wk = [float(r["Counter_Value"]) for r in _counter_rows(write_dir) if name in r["Kernel_Name"]]
        if not fk or not wk:
            continue
        fb = 1024.0 * sf * sum(fk) / len(fk)
        wb = 1024.0 * sw * sum(wk) / len(wk)
        out[q] = {"fetch_bytes": fb, "write_bytes": wb, "bytes_per_launch": fb + wb,
                  "dispatches": [len(fk), len(wk)]}
    with open(args.traffic_json, "w") as f:
        json.dump(out, f, indent=1)
    print(json.dumps(out))


def exact_residual_norm(A, U, S, V=None, center=False, chunk=8192):
    """||E||_2 for E = A - U diag(S) V^T (A - 1 c with centering, c the column
    means; V None: E = A - U diag(S) U^T, A symmetric), exactly in float64.

    Section 4 measures accuracy by this spectral norm.  E is formed in row (or
    column) blocks of float64 where A lives (the GPU, through PyTorch's
    float64 products, or the host), its smaller Gram matrix accumulated, and
    ||E||_2^2 is that matrix's largest eigenvalue (for symmetric E, ||E||_2
    is the largest |eigenvalue| of E itself).  Not a step of the method: the
    library's kernels take no part in it.
    """
    import torch
    f64 = torch.float64
    dev = A.device
    m, n = A.shape
    U = U.to(dev, f64)
    S = torch.as_tensor(np.array(S.detach().cpu().numpy() if hasattr(S, "cpu") else S,
                                 dtype=np.float64)).to(dev)
    sym = V is None
    V = U if sym else V.to(dev, f64)
    W = (V * S).T.contiguous()  # k x n
    c = None
    if center:
        c = torch.zeros(n, dtype=f64, device=dev)
        for i in range(0, m, chunk):
            c += A[i:i + chunk].to(f64).sum(dim=0)
        c /= m
    if sym:
        E = A.to(f64) - U @ W
        ev = torch.linalg.eigvalsh(0.5 * (E + E.T))
        return float(ev.abs().max())
    if n <= m:
        G = torch.zeros(n, n, dtype=f64, device=dev)
        for i in range(0, m, chunk):
            E = A[i:i + chunk].to(f64) - U[i:i + chunk] @ W
            if c is not None:
                E -= c
            G += E.T @ E
    else:
        G = torch.zeros(m, m, dtype=f64, device=dev)
        for j in range(0, n, chunk):
            E = A[:, j:j + chunk].to(f64) - U @ W[:, j:j + chunk]
            if c is not None:
                E -= c[j:j + chunk]
            G += E @ E.T
    lam = float(torch.linalg.eigvalsh(0.5 * (G + G.T))[-1])
    return float(np.sqrt(max(lam, 0.0)))


def _host_info():
    """(BLAS threads, BLAS name and version, CPU model) of this host."""
    threads, blas, cpu = len(os.sched_getaffinity(0)), "unknown", "unknown"
    try:
        from threadpoolctl import threadpool_info
        libs = [d for d in threadpool_info() if d.get("user_api") == "blas"]
        if libs:
            threads = max(d.get("num_threads", 1) for d in libs)
            blas = "%s %s" % (libs[0].get("internal_api"), libs[0].get("version"))
    except Exception:
        pass
    try:
        with open("/proc/cpuinfo") as f:
            for ln in f:
                if ln.startswith("model name"):
                    cpu = ln.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    return threads, blas, cpu


def cpu_oracle_worst(batched, probs):
    """The FP64 oracle (host) on the batch's worst problems: its exact error
    against the same sigma_{k+1}, beside the device's."""
    from oracle import nystrom, philox, rsvd, spectral
    from synth import dense
    params = dense.batch_params()
    out = []
    for w in batched["worst_problems"]:
        i = w["index"]
        q, A = params[i], probs[i]["A"].cpu().numpy()
        om = philox.omega(q["seed"], A.shape[1], q["l"])
        t0 = time.perf_counter()
        if q["kind"] == "svd":
            U0, S0, V0 = rsvd.rsvd(A, q["k"], q["l"], q["its"], om)
            err = spectral.spectral_err_exact(A, U0, S0, V0)
            sk1 = (q["k"] + 1) ** -1.5
        else:
            U0, S0, _, _ = nystrom.eig_psd(A, q["k"], q["l"], q["its"], om, u_A=2.0 ** -16)
            err = spectral.spectral_err_exact(A, U0, S0, None)
            sk1 = float(np.exp(-(q["k"] + 1) / 10.0))
        out.append(dict(index=i, device=w["err_over_sigma_k1"],
                        oracle=round(float(err / sk1), 4),
                        oracle_s=round(time.perf_counter() - t0, 2)))
    return out


def cpu_baseline(A_gpu, k, l, its, seed, center, nsolves, S_gpu):
    """Time the FP64 oracle on the host: ``nsolves`` whole solves of the same A
    (the median is reported)."""
    from oracle import philox, rsvd
    threads, blas, cpu = _host_info()
    A = A_gpu.cpu().numpy()
    n = A.shape[1]
    om = philox.omega(seed, n, l)
    times = []
    S0 = None
    for _ in range(nsolves):
        t0 = time.perf_counter()
        _, S0, _ = rsvd.rsvd(A, k, l, its, om, center=center)
        times.append(time.perf_counter() - t0)
    med = float(np.median(times))
    rel = float(np.max(np.abs(S_gpu - S0) / S0))
    return {"value": 1.0 / med, "unit": "solves/s", "cores": int(threads), "kind": "oracle",
            "cpu": cpu, "blas": blas,
            "sample": "%d whole solves of the same %dx%d centered workload (float64, "
                      "NumPy + %s), median %.2f s" % (nsolves, A.shape[0], n, blas, med)}, rel


def time_solves(ctx, A, k, l, its, seed, out, mat, steps, warmup, renorm="chol", center=True,
                fused=False):
    """Warm up, then time ``steps`` solves on the stream with events; returns
    (ms per solve, library stats over the timed solves)."""
    import torch
    for _ in range(warmup):
        ctx.svd(A, k, l, its, seed, center=center, out=out, mat=mat, renorm=renorm, fused=fused)
    torch.cuda.synchronize()
    ctx.reset_stats()
    ctx.set_timing(True)
    stream = torch.cuda.current_stream()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    e0.record(stream)
    for _ in range(steps):
        ctx.svd(A, k, l, its, seed, center=center, out=out, mat=mat, renorm=renorm, fused=fused)
    e1.record(stream)
    torch.cuda.synchronize()
    ctx.set_timing(False)
    return e0.elapsed_time(e1) / steps, ctx.stats()


def fused_schedule(ctx, A, k, l, its, seed, sk1, ms_std, steps, renorm):
    """The schedule that renormalizes only after every second application
    (RPCA_FUSED_ATA) on the timed workload, with the float32 A and with a
    bfloat16 copy in the range finder: ms per solve, the exact err /
    sigma_{k+1}, A-passes per solve.  The oracle's errors for the same
    schedule are added by the cpu_baseline leg."""
    import torch
    import paper_1412_3510_amd as rp
    m, n = A.shape
    U = torch.empty(m, k, device=A.device, dtype=torch.float32)
    S = torch.empty(k, device=A.device, dtype=torch.float64)
    V = torch.empty(n, k, device=A.device, dtype=torch.float32)
    res = {"schedule": "its x (Z = A_c^T (A_c Z), renormalized), then Y = A_c Z "
                       "orthonormalized; A^T A Z as two reads of A"}
    for kind in ("f32", "bf16"):
        if kind == "f32":
            X, mat = A, rp.dense(A)
        else:
            X, sc = ctx.quantize(A, "bf16")
            mat = rp.dense(X, col_scale=sc, A_f32=A)
        ms, st = time_solves(ctx, X, k, l, its, seed, (U, S, V), mat, steps, 2, renorm,
                             fused=True)
        err = exact_residual_norm(A, U, S, V, center=True)
        res[kind] = {"ms_per_step": round(ms, 4), "solves_per_s": round(1e3 / ms, 3),
                     "speedup_vs_standard_f32": round(ms_std / ms, 3),
                     "err_over_sigma_k1": round(err / sk1, 7),
                     "a_passes_per_solve": round(st["a_passes"] / max(1, steps), 2)}
    return res


def oracle_fused(A_gpu, k, l, its, seed, sk1, with_bf16):
    """The oracle's own error for the fused schedule on the timed workload (one
    float64 solve each for the float32 A and, with ``with_bf16``, for the
    bfloat16 copy as the precision form defines it), measured with the same
    exact residual norm as the device's results."""
    import torch
    from oracle import philox, precision, rsvd
    A = A_gpu.cpu().numpy()
    n = A.shape[1]
    om = philox.omega(seed, n, l)
    out = {}
    runs = [("f32", None)]
    if with_bf16:
        runs.append(("bf16", precision.LowPrecisionA(precision.to_bf16(A), None)))
    for kind, op in runs:
        t0 = time.perf_counter()
        U0, S0, V0 = rsvd.rsvd(A, k, l, its, om, center=True, A_range=op, fused=True)
        dt = time.perf_counter() - t0
        dev = A_gpu.device
        err = exact_residual_norm(A_gpu, torch.from_numpy(U0).to(dev),
                                  torch.from_numpy(S0).to(dev), torch.from_numpy(V0).to(dev),
                                  center=True)
        out[kind] = {"err_over_sigma_k1": round(float(err) / sk1, 7), "seconds": round(dt, 1)}
        del op
    return out


def pass_rates(st, suffix=""):
    out = {}
    for q in ("ax", "atx"):
        n_ = st["n_" + q + suffix]
        if n_:
            ms = st["ms_" + q + suffix] / n_
            b = st["bytes_" + q + suffix] / n_
            out[q] = {"avg_ms": round(ms, 4), "GB/s": round(b / (ms * 1e-3) / 1e9, 1)}
    return out


def precision_form(ctx, A, k, l, its, seed, sk1, ms_f32, err_f32, steps, renorm):
    """bfloat16 and E4M3 copies of A for the range finder, float32 A for the
    Rayleigh-Ritz product: solves/s, pass rates and err / sigma_{k+1}."""
    import torch
    import paper_1412_3510_amd as rp
    m, n = A.shape
    res = {"f32": {"ms_per_step": round(ms_f32, 4), "err_over_sigma_k1": round(err_f32 / sk1, 5)}}
    for kind in ("bf16", "fp8"):
        q, sc = ctx.quantize(A, kind)
        mat = rp.dense(q, col_scale=sc, A_f32=A)
        ctx.tune(q, l, reps=2, mat=mat)   # the tournament of this class
        U = torch.empty(m, k, device=A.device, dtype=torch.float32)
        S = torch.empty(k, device=A.device, dtype=torch.float64)
        V = torch.empty(n, k, device=A.device, dtype=torch.float32)
        ms, st = time_solves(ctx, q, k, l, its, seed, (U, S, V), mat, steps, 2, renorm)
        err = exact_residual_norm(A, U, S, V, center=True)
        res[kind] = {"solves_per_s": round(1e3 / ms, 3), "ms_per_step": round(ms, 4),
                     "speedup_vs_f32": round(ms_f32 / ms, 3),
                     "err_over_sigma_k1": round(err / sk1, 5),
                     "meets_1.1_bound": bool(err <= 1.1 * sk1),
                     "passes_low_precision": pass_rates(st, "_lp"),
                     "passes_f32_rayleigh_ritz": pass_rates(st)}
        del q, sc, mat
    return res


def sigma_errors(S, sig):
    """Relative error of each returned singular value against the construction's
    exact sigma_j: the largest over the converged j <= 50 (sigma_j = 1/j) and
    over the tail, and the error of every tenth value."""
    rel = np.abs(np.asarray(S) - sig) / sig
    lead = sig > 1e-2
    return {"max_j_le_50": float(rel[lead].max()), "max_tail": float(rel[~lead].max()),
            "every_10th": [float("%.3g" % r) for r in rel[9::10]]}


def _ratio(err, ref, nd):
    return None if err is None else round(err / ref, nd)


def precision_form_full(ctx, steps, renorm, exact=True):
    """The precision form's own configuration: 200000 x 8000 (the same spectral
    law, not centered), k = 100, l = 120, its = 3; float32, bfloat16 and E4M3
    range finders (float32 Rayleigh-Ritz product in all three): solves/s,
    pass rates, speedup over float32 and err / sigma_{k+1} (FP64 power
    estimate on the device).  exact=False skips the exact norms (their
    ratios are then null), for counter-collecting profiler runs."""
    import torch
    import paper_1412_3510_amd as rp
    from synth import dense
    m, n, k, l, its, seed = 200000, 8000, 100, 120, 3, 2003
    sig = dense.spectrum_tall(n)
    t0 = time.perf_counter()
    A, _, _ = dense.dense_torch(m, n, sig, seed=1003, device="cuda")
    torch.cuda.synchronize()
    gen_s = time.perf_counter() - t0
    sk1 = float(sig[k])
    U = torch.empty(m, k, device="cuda", dtype=torch.float32)
    S = torch.empty(k, device="cuda", dtype=torch.float64)
    V = torch.empty(n, k, device="cuda", dtype=torch.float32)
    res = {"workload": "dense %dx%d, sigma_j=1/j (j<=50) then 1e-3*exp(-(j-51)/200), not "
                       "centered; k=%d l=%d its=%d" % (m, n, k, l, its),
           "sigma_k_plus_1": sk1, "generation_s": round(gen_s, 1)}
    norm = exact_residual_norm if exact else (lambda *a, **kw: None)
    mat = rp.dense(A)
    ms32, st = time_solves(ctx, A, k, l, its, seed, (U, S, V), mat, steps, 2, renorm, center=False)
    err = norm(A, U, S, V)
    S32 = S.cpu().numpy().copy()
    res["f32"] = {"solves_per_s": round(1e3 / ms32, 3), "ms_per_step": round(ms32, 4),
                  "err_over_sigma_k1": _ratio(err, sk1, 5),
                  "sigma_rel_err": sigma_errors(S32, sig[:k]), "passes": pass_rates(st)}
    for kind in ("bf16", "fp8"):
        q, sc = ctx.quantize(A, kind)
        mat = rp.dense(q, col_scale=sc, A_f32=A)
        ms, st = time_solves(ctx, q, k, l, its, seed, (U, S, V), mat, steps, 2, renorm,
                             center=False)
        err = norm(A, U, S, V)
        Sk = S.cpu().numpy()
        res[kind] = {"solves_per_s": round(1e3 / ms, 3), "ms_per_step": round(ms, 4),
                     "speedup_vs_f32": round(ms32 / ms, 3),
                     "err_over_sigma_k1": _ratio(err, sk1, 5),
                     "meets_1.1_bound": None if err is None else bool(err <= 1.1 * sk1),
                     "sigma_rel_err": sigma_errors(Sk, sig[:k]),
                     "sigma_rel_diff_vs_f32": round(float(np.max(np.abs(Sk - S32) / S32)), 7),
                     "passes_low_precision": pass_rates(st, "_lp"),
                     "passes_f32_rayleigh_ritz": pass_rates(st)}
        if kind == "bf16":
            msf, stf = time_solves(ctx, q, k, l, its, seed, (U, S, V), mat, steps, 1, renorm,
                                   center=False, fused=True)
            errf = norm(A, U, S, V)
            res["bf16_fused"] = {"ms_per_step": round(msf, 4),
                                 "speedup_vs_f32": round(ms32 / msf, 3),
                                 "err_over_sigma_k1": _ratio(errf, sk1, 5),
                                 "sigma_rel_err": sigma_errors(S.cpu().numpy(), sig[:k])}
        del q, sc, mat
    mat = rp.dense(A)
    msf, stf = time_solves(ctx, A, k, l, its, seed, (U, S, V), mat, steps, 1, renorm,
                           center=False, fused=True)
    errf = norm(A, U, S, V)
    res["f32_fused"] = {"ms_per_step": round(msf, 4), "speedup_vs_f32": round(ms32 / msf, 3),
                        "err_over_sigma_k1": _ratio(errf, sk1, 5),
                        "sigma_rel_err": sigma_errors(S.cpu().numpy(), sig[:k])}
    del A, U, S, V, mat
    torch.cuda.empty_cache()
    return res


def sparse_workload(ctx, steps, renorm):
    """The 10^6 x 10^6 sparse workload (10 entries per row, k = 20, l = 30,
    its = 4): solves/s, compulsory GB/s per pass, err / sigma_{k+1}."""
    import torch
    import paper_1412_3510_amd as rp
    from synth import sparse
    m = n = 1000000
    k, l, its, seed = 20, 30, 4, 2004
    t0 = time.perf_counter()
    rptr, ci, va = sparse.random_rows(m, n, 10, 1004)
    cptr, ri, vt = sparse.transpose(m, n, rptr, ci, va)
    dev = [torch.from_numpy(a).cuda() for a in (rptr, ci, va, cptr, ri, vt)]
    S = rp.csr(m, n, *dev)
    gen_s = time.perf_counter() - t0
    U = torch.empty(m, k, device="cuda", dtype=torch.float32)
    Sv = torch.empty(k, device="cuda", dtype=torch.float64)
    V = torch.empty(n, k, device="cuda", dtype=torch.float32)
    ms, st = time_solves(ctx, S, k, l, its, seed, (U, Sv, V), None, steps, 2, renorm,
                         center=False)
    try:
        with open(os.path.join(HERE, "tests", "golden", "sparse_1e6_sigma.json")) as f:
            sk1 = json.load(f)["sigma_k_plus_1"]
    except (OSError, ValueError, KeyError):
        sk1 = None
    err = ctx.spectral_err(S, U, Sv, V, iters=20, seed=7)
    out = {"workload": "CSR %dx%d, 10 distinct uniform columns per row, N(0,1) i^-1/2 values; "
                       "k=%d l=%d its=%d" % (m, n, k, l, its),
           "solves_per_s": round(1e3 / ms, 3), "ms_per_step": round(ms, 4),
           "passes": pass_rates(st), "err_estimate": err,
           "err_over_sigma_k1": round(err / sk1, 5) if sk1 else None,
           "err_note": "FP64 power estimate (20 iterations, a lower bound) over sigma_{k+1} "
                       "of the oracle run at l=60, its=8",
           "generation_s": round(gen_s, 1)}
    # the same matrix with bfloat16 values (half the value bytes per pass)
    Sb = rp.csr(m, n, dev[0], dev[1], dev[2].to(torch.bfloat16), dev[3], dev[4],
                dev[5].to(torch.bfloat16))
    msb, stb = time_solves(ctx, Sb, k, l, its, seed, (U, Sv, V), None, steps, 2, renorm,
                           center=False)
    errb = ctx.spectral_err(Sb, U, Sv, V, iters=20, seed=7)
    out["bf16_values"] = {"solves_per_s": round(1e3 / msb, 3), "ms_per_step": round(msb, 4),
                          "speedup_vs_f32_values": round(ms / msb, 3),
                          "passes": pass_rates(stb), "err_estimate": errb,
                          "err_over_sigma_k1": round(errb / sk1, 5) if sk1 else None}
    return out


def noisy_workload(ctx, n, steps):
    """The paper's second dense experiment (Section 7) at its largest size: an
    n x n matrix of i.i.d. N(sqrt(30/n), 1) entries with signs flipped where
    i*j is odd, rank-4 approximations with l = k + 2 and its = 0, 2, 4.  The
    best rank-4 error is about ||A|| / 2; the library's FP64 power estimate
    (a lower bound) of each error is reported over the largest computed
    singular value."""
    import torch
    from synth import dense
    t0 = time.perf_counter()
    A = dense.noisy_gaussian_torch(n, seed=7000 + n, device="cuda")
    torch.cuda.synchronize()
    gen_s = time.perf_counter() - t0
    k, l = 4, 6
    U = torch.empty(n, k, device="cuda", dtype=torch.float32)
    S = torch.empty(k, device="cuda", dtype=torch.float64)
    V = torch.empty(n, k, device="cuda", dtype=torch.float32)
    res = {"workload": "%dx%d N(sqrt(30/n),1), signs flipped where i*j is odd; k=4 l=6" % (n, n),
           "generation_s": round(gen_s, 1)}
    runs = {}
    for its in (4, 2, 0):
        ms, _ = time_solves(ctx, A, k, l, its, 100 + its, (U, S, V), None, steps, 1,
                            center=False)
        err = ctx.spectral_err(A, U, S, V, iters=20, seed=7)
        runs[its] = (ms, err, float(S[0].item()), float(S[3].item()))
    s1 = runs[4][2]
    for its in (0, 2, 4):
        ms, err, _, s4 = runs[its]
        res["its=%d" % its] = {"ms_per_step": round(ms, 3), "err_estimate": round(err, 4),
                               "err_over_sigma1": round(err / s1, 4),
                               "err_over_its4": round(err / runs[4][1], 4),
                               "sigma4": round(s4, 4)}
    res["note"] = ("err_estimate: FP64 power method, 20 iterations (a lower bound); sigma1 "
                   "from the its=4 solve; the best possible error is sigma_5, about sigma1/2")
    del A, U, S, V
    torch.cuda.empty_cache()
    return res


def batched_workload(ctx, steps):
    """512 small problems (256 dense, 256 PSD) in one rpca_svd_batched call:
    the persistent launch, eager and replayed from a captured graph, and the
    same batch on streams for comparison; problems/s and err / sigma_{k+1}."""
    import torch
    from synth import dense
    t0 = time.perf_counter()
    params = dense.batch_params()
    probs = []
    for q in params:
        if q["kind"] == "svd":
            r = min(q["m"], q["n"])
            A, _, _ = dense.dense_torch(q["m"], q["n"], dense.spectrum_power(r), q["seed_A"], "cuda")
            probs.append(dict(A=A, k=q["k"], l=q["l"], its=q["its"], seed=q["seed"]))
        else:
            A = dense.psd_torch(q["n"], dense.spectrum_exp(q["n"]), q["seed_A"], "cuda")
            probs.append(dict(A=A, k=q["k"], l=q["l"], its=q["its"], seed=q["seed"], kind="psd"))
    torch.cuda.synchronize()
    gen_s = time.perf_counter() - t0
    s = torch.cuda.Stream()
    ctx.set_stream(s)
    try:
        with torch.cuda.stream(s):
            outs = ctx.svd_batched(probs)   # sizes the persistent working memory
            s.synchronize()
            e0 = torch.cuda.Event(enable_timing=True)
            e1 = torch.cuda.Event(enable_timing=True)
            e0.record(s)
            for _ in range(steps):
                outs = ctx.svd_batched(probs)
            e1.record(s)
            s.synchronize()
            ms_eager = e0.elapsed_time(e1) / steps
            g = torch.cuda.CUDAGraph()
            with torch.cuda.graph(g, stream=s):
                gouts = ctx.svd_batched(probs)
            g.replay()
            s.synchronize()
            e0.record(s)
            for _ in range(steps):
                g.replay()
            e1.record(s)
            s.synchronize()
            ms_graph = e0.elapsed_time(e1) / steps
            # the same batch on streams (single-problem kernels)
            ctx.set_batch_mode(1)
            ctx.svd_batched(probs)
            s.synchronize()
            e0.record(s)
            for _ in range(steps):
                ctx.svd_batched(probs)
            e1.record(s)
            s.synchronize()
            ms_streams = e0.elapsed_time(e1) / steps
    finally:
        ctx.set_batch_mode(0)
        ctx.set_stream(torch.cuda.current_stream())
    ratios = []
    t1 = time.perf_counter()
    for q, pr, o in zip(params, probs, gouts):
        if q["kind"] == "svd":
            err = exact_residual_norm(pr["A"], o[0], o[1], o[2])
            sk1 = (q["k"] + 1) ** -1.5
        else:
            err = exact_residual_norm(pr["A"], o[0], o[1], None)
            sk1 = float(np.exp(-(q["k"] + 1) / 10.0))
        ratios.append(err / sk1)
    norm_s = time.perf_counter() - t1
    r = np.array(ratios)
    worst = [int(i) for i in np.argsort(r)[::-1][:4]]
    return {"workload": "512 problems: 256 dense (m~logU[256,8192], n~logU[64,2048], "
                        "sigma_j=j^-1.5) + 256 PSD Nystrom (n~logU[128,4096], lambda_j=e^-j/10); "
                        "k~U{5..40}, l=k+5, its=2",
            "mode": "persistent launch (one workgroup per problem)",
            "ms_per_batch_eager": round(ms_eager, 3), "ms_per_batch_graph": round(ms_graph, 3),
            "ms_per_batch_streams": round(ms_streams, 3),
            "problems_per_s": round(512 * 1e3 / ms_graph, 1),
            "err_over_sigma_k1": {"p50": round(float(np.median(r)), 4),
                                  "p99": round(float(np.quantile(r, 0.99)), 4),
                                  "max": round(float(r.max()), 4),
                                  "norm": "exact ||E||_2 per problem (float64, %.0f s)" % norm_s},
            "worst_problems": [dict(index=i, kind=params[i]["kind"], m=params[i]["m"],
                                    n=params[i]["n"], k=params[i]["k"],
                                    err_over_sigma_k1=round(float(r[i]), 4)) for i in worst],
            "generation_s": round(gen_s, 1)}, probs


def main():
    args = parse()
    if args.passes_only:
        args.no_fused = args.no_precision = args.no_sparse = args.no_batched = True
        args.no_noisy = args.no_cpu_baseline = True
    if args.traffic_from_pmc:
        traffic_from_pmc(args)
        return
    if args.gpus != 1:
        print("bench.py runs on one GPU only: the library has no multi-GPU path "
              "(--gpus must be 1)", file=sys.stderr)
        sys.exit(2)
    import torch
    import paper_1412_3510_amd as rp
    from synth import dense

    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    if args.batched_only:
        print(json.dumps(batched_workload(rp.Context(), args.steps)[0]), flush=True)
        return
    if args.precision_only:
        print(json.dumps(precision_form_full(rp.Context(), args.steps, args.renorm,
                                             exact=not args.passes_only)), flush=True)
        return
    if args.sparse_only:
        print(json.dumps(sparse_workload(rp.Context(), args.steps, args.renorm)), flush=True)
        return
    m, n, k, l, its = args.m, args.n, args.k, args.l, args.its
    sigma = dense.spectrum_tall(min(m, n))
    t0 = time.perf_counter()
    A, _, csig = dense.dense_torch(m, n, sigma, seed=1002, device=dev, center_spectrum=True)
    torch.cuda.synchronize()
    gen_s = time.perf_counter() - t0
    print("generated A %dx%d in %.1f s" % (m, n, gen_s), file=sys.stderr, flush=True)

    ctx = rp.Context()
    U = torch.empty(m, k, device=dev, dtype=torch.float32)
    S = torch.empty(k, device=dev, dtype=torch.float64)
    V = torch.empty(n, k, device=dev, dtype=torch.float32)
    mat = rp.dense(A)
    tuned = None
    if not args.no_tune:
        # the autotuner picks the tile configurations of this shape class
        tuned = ctx.tune(A, l, reps=3, mat=mat)
        print("autotune: %s" % tuned, file=sys.stderr, flush=True)
    for _ in range(args.warmup):
        ctx.svd(A, k, l, its, args.seed, center=True, out=(U, S, V), mat=mat, renorm=args.renorm)
    torch.cuda.synchronize()
    print("warmup done", file=sys.stderr, flush=True)

    ctx.reset_stats()
    ctx.set_timing(True)
    stream = torch.cuda.current_stream()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    e0.record(stream)
    w0 = time.perf_counter()
    for _ in range(args.steps):
        ctx.svd(A, k, l, its, args.seed, center=True, out=(U, S, V), mat=mat, renorm=args.renorm)
    e1.record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - w0
    ctx.set_timing(False)
    ms_total = e0.elapsed_time(e1)
    st = ctx.stats()
    ms_per_step = ms_total / args.steps
    print("timed %d solves: %.3f ms/solve (wall %.3f ms)" % (args.steps, ms_per_step,
                                                             1e3 * wall / args.steps),
          file=sys.stderr, flush=True)

    kernels = {}
    if st["n_ax"]:
        kernels["ax"] = (st["ms_ax"] / st["n_ax"], st["bytes_ax"] / st["n_ax"], st["ms_ax"])
    if st["n_atx"]:
        kernels["atx"] = (st["ms_atx"] / st["n_atx"], st["bytes_atx"] / st["n_atx"], st["ms_atx"])
    dom = max(kernels, key=lambda q: kernels[q][2])
    avg_ms, bytes_per, _ = kernels[dom]
    achieved = bytes_per / (avg_ms * 1e-3) / 1e9
    traffic = None
    try:
        with open(args.traffic_json) as f:
            tj = json.load(f)
        ent = tj.get(dom)
        if (ent and tj.get("m") == m and tj.get("n") == n and tj.get("l") == l
                and tj.get("sources_sha256") == _sources_digest()):
            traffic = round(ent["bytes_per_launch"])
    except (OSError, ValueError, KeyError):
        pass
    roofline = {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS,
                "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": traffic,
                "kernel": {"ax": "ax_tall_kernel (Y = A X)",
                           "atx": "atx_wide_kernel (A^T X, split over rows)"}[dom],
                "avg_launch_ms": round(avg_ms, 4), "algorithmic_bytes": bytes_per}
    passes = {q: {"avg_ms": round(v[0], 4), "GB/s": round(v[1] / (v[0] * 1e-3) / 1e9, 1)}
              for q, v in kernels.items()}

    S_host = S.cpu().numpy()
    sk1 = float(csig[k])
    err_f32 = None if args.passes_only else exact_residual_norm(A, U, S, V, center=True)
    est_f32 = ctx.spectral_err(A, U, S, V, iters=30, seed=7, center=True)
    fused = None
    if not args.no_fused:
        fused = fused_schedule(ctx, A, k, l, its, args.seed, sk1, ms_per_step,
                               args.precision_steps, args.renorm)
    prec = None
    if not args.no_precision:
        prec = precision_form(ctx, A, k, l, its, args.seed, sk1, ms_per_step, err_f32,
                              args.precision_steps, args.renorm)
    out = {
        "metric": METRIC,
        "value": round(1e3 / ms_per_step, 3),
        "unit": "solves/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_per_step, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32 (products as 3 bf16 MFMA terms, f32 accumulation)",
        "data": "synthetic",
        "config": {"workload": "dense %dx%d float32, centered, sigma_j=1/j (j<=50) then "
                               "1e-3*exp(-(j-51)/200); k=%d l=%d its=%d" % (m, n, k, l, its),
                   "m": m, "n": n, "k": k, "l": l, "its": its, "center": True, "renorm": args.renorm},
        "passes": passes,
        "autotune": ({kk: (round(v, 4) if isinstance(v, float) else v) for kk, v in tuned.items()}
                     if tuned else None),
        "roofline": roofline,
        "sigma_k_plus_1": sk1,
        "err_over_sigma_k1": None if err_f32 is None else round(err_f32 / sk1, 6),
        "err_note": "||A_c - U S V^T||_2 exact (float64 Gram on the device); the library's "
                    "FP64 power estimate (30 iterations, a lower bound) gives %.6f"
                    % (est_f32 / sk1),
    }
    if fused is not None:
        out["fused_ata"] = fused
    if prec is not None:
        out["precision_form"] = precision_form_full(ctx, args.precision_steps, args.renorm)
        out["precision_form_on_timed_workload"] = prec
    if not args.no_sparse:
        out["sparse"] = sparse_workload(ctx, args.precision_steps, args.renorm)
    if not args.no_noisy:
        out["noisy_gaussian"] = noisy_workload(ctx, args.noisy_n, 3)
    bprobs = None
    if not args.no_batched:
        out["batched"], bprobs = batched_workload(ctx, 5)
    if not args.no_cpu_baseline:
        cb, rel = cpu_baseline(A, k, l, its, args.seed, True, args.cpu_sample_solves, S_host)
        out["cpu_baseline"] = cb
        out["parity_max_rel_sigma"] = rel
        if bprobs is not None:
            # the oracle on the batch's worst problems: its own error, for comparison
            out["batched"]["oracle_on_worst"] = cpu_oracle_worst(out["batched"], bprobs)
        if fused is not None:
            out["fused_ata"]["oracle"] = oracle_fused(A, k, l, its, args.seed, sk1,
                                                      not args.no_fused_bf16_oracle)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
