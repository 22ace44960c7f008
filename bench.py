#!/usr/bin/env python3
"""Benchmark: effective TFLOP/s (n^3/3 flops per inverse) of the lower-triangular
inverse at n = 16384, BF16-MFMA + Newton-Schulz refinement vs the plain FP64
GPU path, both certified to a relative residual <= 1e-12.

One step = one full inversion of the n = 16384 matrix (staging casts, leaf
inversion, every recursion level, and for the refine path the residual and
correction products until the tolerance is met). Inputs are seeded synthetic
matrices (see the synth package) resident in HBM before timing starts.

Prints one JSON line (see the repository documentation for the fields).
"""

from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "TFLOP/s (n^3/3) tril inverse n=16384: BF16+refine vs FP64, equal residual"
PEAK_TFLOPS = {"f64": 78.6, "f32": 157.3, "bf16": 2500.0, "f16": 2500.0}
HBM_PEAK_GBS = 8000.0
# Library profile classes that are matrix-core products (one class = one kernel
# instantiation); the leading token is the operand precision.
MFMA_KINDS = ("level_T", "level_X21", "residual", "residual2", "correction")
# HBM traffic per launch measured with hardware counters, keyed by profile class
# and by a hash of the kernel sources at the time of the measurement.
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "hbm_traffic_n16384.md")
_LP_SOURCES = ["paper_2307_07611_amd/csrc/gemm_lp.hip", "paper_2307_07611_amd/csrc/lowp.h",
               "paper_2307_07611_amd/csrc/common.h", "paper_2307_07611_amd/csrc/refine.cpp",
               "paper_2307_07611_amd/csrc/split.hip", "paper_2307_07611_amd/csrc/launch.h"]
KERNEL_SOURCES = {
    "bf16": _LP_SOURCES,
    "f16": _LP_SOURCES,
    "f64": ["paper_2307_07611_amd/csrc/gemm_fp.hip", "paper_2307_07611_amd/csrc/launch.h",
            "paper_2307_07611_amd/csrc/common.h", "paper_2307_07611_amd/csrc/api.cpp",
            "paper_2307_07611_amd/csrc/leaf.hip"],
}


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def time_path(P, torch, Ld, mode, steps, warmup, leaf):
    """Warm-up steps; then `steps` untimed steps with every kernel class timed
    (the per-class breakdown); then the `steps` timed steps, in which only the
    dominant product class carries timing events (a timed kernel ends with a
    flush that its completion event needs, a few microseconds that the other
    kernels are spared)."""
    n = Ld.shape[0]
    X = torch.empty_like(Ld)
    ws = torch.empty(max(P.workspace_bytes(n, mode, leaf=leaf), 1), dtype=torch.uint8, device=Ld.device)
    kw = dict(leaf=leaf, out=X, workspace=ws, blocking=False, return_info=True)
    infos = []
    for _ in range(warmup):
        _, info = P.tril_inverse(Ld, mode, **kw)
        infos.append(info)
    torch.cuda.synchronize()
    P.profile_select(None)
    P.profile_enable(True)
    for _ in range(steps):
        P.tril_inverse(Ld, mode, **kw)
    torch.cuda.synchronize()
    breakdown = P.profile_read()
    P.profile_enable(False)
    dom = dominant_class(breakdown)
    P.profile_select([dom] if dom else None)
    P.profile_enable(True)
    start, stop = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    start.record()
    for _ in range(steps):
        _, info = P.tril_inverse(Ld, mode, **kw)
        infos.append(info)
    stop.record()
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    prof = P.profile_read()
    P.profile_enable(False)
    P.profile_select(None)
    ms = start.elapsed_time(stop) / steps
    return X, ms, wall, prof, breakdown, infos[-1]


def sources_hash(dtype):
    import hashlib

    h = hashlib.sha256()
    for rel in KERNEL_SOURCES.get(dtype, []):
        with open(os.path.join(ROOT, rel), "rb") as f:
            h.update(f.read())
    return h.hexdigest()[:16]


def measured_traffic(cls, dtype):
    """HBM bytes per launch of `cls` from the committed counter summary, or None
    when there is none or the kernel sources changed since it was taken.
    Table rows: | class | sources hash | fetch bytes | write bytes | total bytes |"""
    if not os.path.exists(TRAFFIC_FILE):
        return None
    want = sources_hash(dtype)
    with open(TRAFFIC_FILE) as f:
        for line in f:
            cells = [c.strip() for c in line.strip().strip("|").split("|")]
            if len(cells) >= 5 and cells[0] == cls and cells[1] == want:
                try:
                    return float(cells[4])
                except ValueError:
                    return None
    return None


def dominant_class(prof):
    """The matrix-core product class with the largest total time."""
    mm = {k: v for k, v in prof.items() if k.split("_", 1)[-1] in MFMA_KINDS and v["launches"]}
    return max(mm.items(), key=lambda kv: kv[1]["total_ms"])[0] if mm else None


def roofline(prof):
    name = dominant_class(prof)
    if name is None:
        return None
    e = prof[name]
    dtype = name.split("_", 1)[0]
    avg_ms = e["total_ms"] / e["launches"]
    achieved = (e["flops"] / e["launches"]) / (avg_ms * 1e-3) / 1e12
    peak = PEAK_TFLOPS[dtype]
    return {"bound": "mfma", "achieved": round(achieved, 3), "peak": peak, "unit": "TFLOP/s",
            "frac": round(achieved / peak, 4), "traffic": measured_traffic(name, dtype),
            "kernel_class": name, "launches": e["launches"], "avg_launch_ms": round(avg_ms, 4),
            "flops_per_launch": e["flops"] / e["launches"], "sources_hash": sources_hash(dtype)}


def copy_calibration(mib, reps):
    """Plain copy kernel of known size (elementwise negate, fp32) to scale the
    hardware byte counters: each launch reads and writes exactly `mib` MiB."""
    import torch

    src = torch.ones(mib * (1 << 20) // 4, dtype=torch.float32, device="cuda")
    dst = torch.empty_like(src)
    torch.cuda.synchronize()
    for _ in range(reps):
        torch.neg(src, out=dst)
    torch.cuda.synchronize()
    print(json.dumps({"copy_calibration_mib": mib, "launches": reps,
                      "bytes_read_per_launch": src.numel() * 4, "bytes_written_per_launch": dst.numel() * 4}),
          flush=True)


def time_events(torch, fn, reps):
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    e0.record()
    for _ in range(reps):
        fn()
    e1.record()
    torch.cuda.synchronize()
    return e0.elapsed_time(e1) / reps


def plain_config_secondary(P, torch, n, seed, leaf, reps):
    """The plain FP64 path on its own configurations: n = 256, leaf 32 (a
    latency case) and n = 8192, leaf 64 (FP64-MFMA bound, 50% gate)."""
    import oracle
    import synth

    L = synth.lower_triangular(n, seed)
    Ld = torch.from_numpy(L).cuda()
    X = torch.empty_like(Ld)
    ws = torch.empty(max(P.workspace_bytes(n, "f64", leaf=leaf), 1), dtype=torch.uint8, device=Ld.device)
    run = lambda: P.tril_inverse(Ld, "f64", leaf=leaf, out=X, workspace=ws, blocking=False)  # noqa: E731
    for _ in range(3):
        run()
    ms = time_events(torch, run, reps)
    fl = n ** 3 / 3.0
    out = {"workload": f"plain FP64 lower-triangular inverse n={n} seed={seed} leaf={leaf}", "ms": round(ms, 5),
           "tflops": round(fl / ms / 1e9, 4), "frac_fp64_mfma": round(fl / ms / 1e9 / PEAK_TFLOPS["f64"], 4),
           "reps": reps}
    r = P.residual(Ld, X)
    out["rel_residual"] = r["rel"]
    cols = np.unique(np.linspace(0, n - 2, 6).astype(np.int64))
    Xo = oracle.tril_inverse_columns(L, cols)
    Xg = X[:, torch.from_numpy(cols).cuda()].cpu().numpy()
    out.update(fwd_errors(Xg, Xo, cols))
    if n >= 4096:
        out["meets_50pct_fp64_peak"] = bool(out["frac_fp64_mfma"] >= 0.5)
    return out


def fwd_errors(Xg, Xo, cols):
    """Relative forward errors on sampled columns: all entries, and the
    strictly lower part alone (the entries the products compute; the
    diagonal is 1 / L_ii on every path)."""
    n = Xo.shape[0]
    strict = np.arange(n)[:, None] > np.asarray(cols)[None, :]
    return {"fwd_err_sampled_cols": float(np.linalg.norm(Xg - Xo) / np.linalg.norm(Xo)),
            "fwd_err_strict": float(np.linalg.norm((Xg - Xo)[strict]) / np.linalg.norm(Xo[strict]))}


def batched_secondary(P, torch, reps):
    """4096 FP32 matrices of order n_i = 16 + (splitmix(6, i) mod 497) in one
    persistent launch (configuration chosen by the autotuner), captured in a
    graph and replayed."""
    import synth

    sizes = synth.batch_sizes(4096)
    g = P.BatchedGraph(sizes, dtype=torch.float32)
    host = np.zeros(g.L.numel(), dtype=np.float32)
    for i, n in enumerate(sizes):
        o = int(g.offsets[i])
        host[o:o + n * n] = synth.lower_triangular(int(n), 1000 + i, dtype=np.float32).ravel()
    g.L.copy_(torch.from_numpy(host).cuda())
    g.capture()  # autotunes the persistent launch on this batch first
    for _ in range(3):
        g.replay()
    ms = time_events(torch, g.replay, reps)
    nn = sizes.astype(np.float64)
    flops = float(np.sum(nn ** 3) / 3)
    byts = float(np.sum(4 * (nn * (nn + 1) / 2 + nn * nn)))  # lower triangle in, full X out
    st = g.status.cpu().numpy()
    return {"workload": "batched: 4096 FP32 lower-triangular matrices, n_i = 16 + (splitmix64(6, i) mod 497), "
                        "one persistent launch (graph replay)",
            "ms": round(ms, 4), "tflops": round(flops / ms / 1e9, 3), "hbm_GBs": round(byts / ms / 1e6, 1),
            "frac_fp32_mfma": round(flops / ms / 1e9 / PEAK_TFLOPS["f32"], 4),
            "frac_hbm": round(byts / ms / 1e6 / HBM_PEAK_GBS, 4), "sum_n3_over_3": flops,
            "algorithmic_bytes": byts, "all_status_ok": bool(np.all(st == 0)), "reps": reps,
            "autotuned": g.config}


def backward_secondary(P, torch, reps):
    """64 FP32 matrices of order 1024: forward (batched path) and the adjoint
    gradL = -tril(X^T G X^T) (two MFMA products per matrix)."""
    import synth

    batch, n = 64, 1024
    L = torch.from_numpy(np.stack([synth.lower_triangular(n, 2000 + b, dtype=np.float32)
                                   for b in range(batch)])).cuda()
    G = torch.from_numpy(np.stack([synth.normal(n, n, 3000 + b, dtype=np.float32) for b in range(batch)])).cuda()
    X = P.batched_uniform_inverse(L)
    fwd = lambda: P.batched_uniform_inverse(L)  # noqa: E731
    bwd = lambda: P.tril_inverse_backward(X, G)  # noqa: E731
    for _ in range(2):
        fwd()
        bwd()
    ms_f = time_events(torch, fwd, reps)
    ms_b = time_events(torch, bwd, reps)
    ff = batch * n ** 3 / 3.0
    fb = batch * 2.0 * n ** 3 / 3.0
    return {"workload": "backward: 64 FP32 lower-triangular matrices of order 1024, forward + adjoint",
            "forward_ms": round(ms_f, 4), "forward_tflops": round(ff / ms_f / 1e9, 3),
            "backward_ms": round(ms_b, 4), "backward_tflops": round(fb / ms_b / 1e9, 3),
            "backward_frac_fp32_mfma": round(fb / ms_b / 1e9 / PEAK_TFLOPS["f32"], 4), "reps": reps}


def combrit_secondary(P, torch, Ld, reps):
    """Top level of algorithm COMBRIT on a beta x beta block grid (FP64), on
    the same n = 16384 matrix: effective TFLOP/s (n^3/3) and the residual."""
    n = Ld.shape[0]
    out = {"workload": f"COMBRIT top level, FP64, n={n} (same matrix as the headline)"}
    for beta in (4, 8):
        X = torch.empty_like(Ld)
        ws = torch.empty(max(P.workspace_bytes(n, "f64", beta=beta, leaf=128), 1), dtype=torch.uint8,
                         device=Ld.device)
        run = lambda: P.tril_inverse(Ld, "f64", beta=beta, leaf=128, out=X, workspace=ws, blocking=False)  # noqa
        run()
        ms = time_events(torch, run, reps)
        r = P.residual(Ld, X)
        out[f"beta{beta}"] = {"ms": round(ms, 4), "tflops": round(n ** 3 / 3 / ms / 1e9, 3),
                              "rel_residual": r["rel"]}
        del X, ws
        torch.cuda.empty_cache()
    return out


def factored_secondary(P, torch, reps):
    """Factored inverse at n = 4096, FP64: L unit lower (seed 3), U upper
    (seed 4); L^-1 and U^-1 (n^3/3 flops each) and Ainv = U^-1 L^-1
    (2 n^3/3 flops over the two triangles)."""
    import synth

    n = 4096
    L = torch.from_numpy(synth.lower_triangular(n, 3, unit=True)).cuda()
    U = torch.from_numpy(synth.upper_triangular(n, 4)).cuda()
    out = {"workload": f"factored inverse A^-1 = U^-1 L^-1 from given factors, FP64 n={n}"}
    for want in (False, True):
        run = lambda: P.factored_inverse(L, U, l_unit=True, want_ainv=want, leaf=64, blocking=False)  # noqa: E731
        run()
        ms = time_events(torch, run, reps)
        fl = 2 * n ** 3 / 3 + (2 * n ** 3 / 3 if want else 0.0)
        out["with_ainv" if want else "factors_only"] = {"ms": round(ms, 4), "tflops": round(fl / ms / 1e9, 3),
                                                        "frac_fp64_mfma": round(fl / ms / 1e9 / PEAK_TFLOPS["f64"], 4)}
    Linv, Uinv, Ainv = P.factored_inverse(L, U, l_unit=True, leaf=64)
    A = L @ U
    eye = torch.eye(n, dtype=A.dtype, device=A.device)
    out["rel_inverse_residual"] = float(torch.linalg.norm(Ainv @ A - eye) / n ** 0.5)
    out["reps"] = reps
    return out


def skul_secondary(P, torch, reps):
    """Algorithm SKUL at n = 4096, FP64: Crout factorization plus S = U^-1,
    K = L^-1 and Ainv = S K; effective rate over 2 n^3 flops (2n^3/3 for the
    factorization, n^3/3 per triangular inverse, 2n^3/3 for S K)."""
    import synth

    n = 4096
    A = torch.from_numpy(synth.diag_dominant(n, 77)).cuda()
    P.skul(A)
    ms = time_events(torch, lambda: P.skul(A, blocking=False), reps)
    L, U, S, K, Ainv = P.skul(A)
    lu = float(torch.linalg.norm(L @ U - A) / torch.linalg.norm(A))
    return {"workload": f"SKUL: Crout A = L U with S = U^-1, K = L^-1, Ainv = S K; FP64 n={n}, diagonally dominant",
            "ms": round(ms, 3), "tflops_2n3": round(2.0 * n ** 3 / ms / 1e9, 3), "rel_lu_residual": lu,
            "reps": reps}


def sqr_secondary(P, torch, reps):
    """Algorithm SQR at n = 4096, FP64: modified Gram-Schmidt A = Q R, S = R^-1
    and Ainv = S Q^T; effective rate over 3 n^3 flops (2 n^3 for Gram-Schmidt,
    n^3 / 3 for the triangular inverse, 2 n^3 / 3 for S Q^T)."""
    import synth

    n = 4096
    A = torch.from_numpy(synth.diag_dominant(n, 22)).cuda()
    P.sqr(A)
    ms = time_events(torch, lambda: P.sqr(A, blocking=False), reps)
    Q, R, S, Ainv = P.sqr(A)
    eye = torch.eye(n, dtype=A.dtype, device=A.device)
    orth = float(torch.linalg.norm(Q.T @ Q - eye) / n ** 0.5)
    res = float(torch.linalg.norm(A @ Ainv - eye) / n ** 0.5)
    return {"workload": f"SQR: Gram-Schmidt A = Q R with S = R^-1, Ainv = S Q^T; FP64 n={n}, diagonally dominant",
            "ms": round(ms, 3), "tflops_3n3": round(3.0 * n ** 3 / ms / 1e9, 3), "orthogonality": orth,
            "rel_inverse_residual": res, "reps": reps}


def brsi_secondary(P, torch, reps):
    """General inverse by BRSI (gamma = 2) at n = 4096, FP64; effective rate
    over 2 n^3 flops (the Gauss-Jordan count of a general inverse; the
    recursion itself executes about 3.2 n^3)."""
    import synth

    n = 4096
    A = torch.from_numpy(synth.diag_dominant(n, 16)).cuda()
    P.brsi(A)
    ms = time_events(torch, lambda: P.brsi(A, blocking=False), reps)
    X = P.brsi(A)
    eye = torch.eye(n, dtype=A.dtype, device=A.device)
    res = float(torch.linalg.norm(A @ X - eye) / n ** 0.5)
    return {"workload": f"BRSI gamma=2: general inverse, FP64 n={n}, diagonally dominant",
            "ms": round(ms, 3), "tflops_2n3": round(2.0 * n ** 3 / ms / 1e9, 3), "rel_inverse_residual": res,
            "reps": reps}


# The paper's own timing of this method (Table tab:combrit: COMBRIT, MATLAB
# R2021b, sequential, on an Intel i7 machine; seconds, mean of 10 runs) at
# its largest order, with the effective rate n^3/3 / t. Another machine and
# a 16x smaller order: context only, not a baseline for this measurement.
PAPER_CONTEXT = {
    "source": "Table tab:combrit (COMBRIT; MATLAB R2021b, sequential, Intel i7)",
    "n": 1024,
    "seconds": {"beta2": 4.15e-2, "beta4": 3.06e-2, "crit": 3.33},
    "effective_gflops": {"beta2": round(1024 ** 3 / 3 / 4.15e-2 / 1e9, 2),
                         "beta4": round(1024 ** 3 / 3 / 3.06e-2 / 1e9, 2),
                         "crit": round(1024 ** 3 / 3 / 3.33 / 1e9, 4)},
}


def cpu_baseline(L, seconds):
    """The oracle (column recurrence, all host cores via OpenMP) on a bounded
    sample of the same matrix: evenly spaced columns of L^-1."""
    import oracle

    n = L.shape[0]

    def col_flops(cols):
        c = np.asarray(cols, dtype=np.float64)
        return float(np.sum((n - c) * (n - c - 1)))  # sum_{i>j} 2 (i - j)

    threads = oracle.num_threads()
    probe = np.linspace(0, n - 1, 4 * threads).astype(np.int64)
    t0 = time.perf_counter()
    oracle.tril_inverse_columns(L, probe)
    dt = time.perf_counter() - t0
    rate = col_flops(probe) / max(dt, 1e-9)
    per_col = n * n / 3.0  # average cost of one column
    count = int(min(n, max(threads, seconds * rate / per_col)))
    cols = np.linspace(0, n - 1, count).astype(np.int64)
    t0 = time.perf_counter()
    oracle.tril_inverse_columns(L, cols)
    dt = time.perf_counter() - t0
    fl = col_flops(cols)
    cpu = "unknown"
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    cpu = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    return {"value": round(fl / dt / 1e12, 6), "unit": "TFLOP/s", "cores": threads, "kind": "oracle",
            "sample": f"{count} evenly spaced columns of L^-1 (n={n}), {fl:.3e} flops in {dt:.1f} s",
            "seconds": round(dt, 2), "cpu_model": cpu}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--n", type=int, default=16384)
    ap.add_argument("--seed", type=int, default=5)
    ap.add_argument("--paths", default="bf16_refine,f16_refine,f64", help="comma list, or none")
    ap.add_argument("--cpu-seconds", type=float, default=20.0)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-secondary", action="store_true",
                    help="skip the secondary measurements")
    ap.add_argument("--secondary", default="all",
                    help="comma list of secondary measurements to run (plain, batched, backward, factored, "
                         "skul, sqr, brsi, combrit) or 'all'")
    ap.add_argument("--copy-calibration-mib", type=int, default=0,
                    help="only run a plain copy kernel of this size (counter calibration) and exit")
    args = ap.parse_args()
    if args.gpus != 1:
        print(json.dumps({"error": "runs on one GPU: --gpus must be 1 "
                                   "(the multi-GPU sharding is a design note, not code)"}), flush=True)
        sys.exit(2)

    if args.copy_calibration_mib:
        copy_calibration(args.copy_calibration_mib, max(args.steps, 1))
        return

    import torch

    import paper_2307_07611_amd as P
    import synth

    P.load()
    n = args.n
    log(f"generating L n={n} seed={args.seed}")
    L = synth.lower_triangular(n, args.seed)
    Ld = torch.from_numpy(L).cuda()
    torch.cuda.synchronize()
    flops = n ** 3 / 3.0
    results = {}
    for path in [p for p in args.paths.split(",") if p and p != "none"]:
        leaf = 128 if n >= 4096 else 64
        log(f"path {path}: warmup {args.warmup}, steps {args.steps}")
        try:
            X, ms, wall, prof, breakdown, info = time_path(P, torch, Ld, path, args.steps, args.warmup, leaf)
        except P.TrinvError as e:
            log(f"path {path} unavailable: {e}")
            continue
        r = P.residual(Ld, X)
        cols = np.array([0, n // 3, n // 2, n - 2])
        import oracle

        Xo = oracle.tril_inverse_columns(L, cols)
        Xg = X[:, torch.from_numpy(cols).cuda()].cpu().numpy()
        fe = fwd_errors(Xg, Xo, cols)
        results[path] = {"ms": ms, "tflops": flops / (ms * 1e-3) / 1e12, "rel_residual": r["rel"],
                         "rel_residual_in_loop": info.get("rel_residual"),
                         "resid_error_est": info.get("resid_error_est"),
                         "resid_error_bound": info.get("resid_error_bound"), **fe, "profile": breakdown,
                         "iterations": info.get("iterations"), "roofline": roofline(prof), "wall_s": wall}
        log(f"path {path}: {ms:.3f} ms/step, {results[path]['tflops']:.2f} TFLOP/s, rel residual {r['rel']:.3e}, "
            f"fwd err {fe['fwd_err_sampled_cols']:.3e}, strictly lower {fe['fwd_err_strict']:.3e}")
        del X
        torch.cuda.empty_cache()

    head = "bf16_refine" if "bf16_refine" in results else ("f64" if "f64" in results else None)
    h = results[head] if head else {"tflops": 0.0, "ms": 0.0, "roofline": None, "rel_residual": None,
                                    "fwd_err_sampled_cols": None, "fwd_err_strict": None}
    out = {
        "metric": METRIC, "value": round(h["tflops"], 3), "unit": "TFLOP/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": round(h["ms"], 4), "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None,
        "dtype": "bf16" if head == "bf16_refine" else "f64",
        "data": "synthetic",
        "config": {"workload": f"lower-triangular inverse n={n} seed={args.seed} (diag +-U[1,2], strict lower "
                               f"U[-1,1]/n), path={head}, certified rel. residual <= 1e-12",
                   "n": n, "path": head},
        "roofline": h["roofline"],
        "rel_residual": h["rel_residual"],
        "fwd_err_sampled_cols": h["fwd_err_sampled_cols"],
        "fwd_err_strict": h["fwd_err_strict"],
        "paths": {k: {kk: vv for kk, vv in v.items() if kk != "profile"} for k, v in results.items()},
        "kernel_profile": {k: v["profile"] for k, v in results.items()},
        "paper_context": PAPER_CONTEXT,
    }
    if "bf16_refine" in results and "f64" in results:
        out["speedup_vs_f64_path"] = round(results["f64"]["ms"] / results["bf16_refine"]["ms"], 3)
    if not args.no_secondary:
        want = set(args.secondary.split(",")) if args.secondary != "all" else None
        run = lambda name: want is None or name in want  # noqa: E731
        out["secondary"] = {}
        if run("plain"):
            log("plain FP64 n=256 leaf 32 and n=8192 leaf 64")
            out["secondary"]["plain_n256"] = plain_config_secondary(P, torch, 256, 1, 32, 50)
            out["secondary"]["plain_n8192"] = plain_config_secondary(P, torch, 8192, 2, 64, 5)
            log(f"plain: {out['secondary']['plain_n256']['ms']} ms (n=256), "
                f"{out['secondary']['plain_n8192']['ms']} ms (n=8192)")
        if run("batched"):
            log("batched 4096 FP32 (graph replay)")
            out["secondary"]["batched"] = batched_secondary(P, torch, 20)
            log(f"batched: {out['secondary']['batched']['ms']} ms")
        if run("backward"):
            log("backward 64 x 1024 FP32")
            out["secondary"]["backward"] = backward_secondary(P, torch, 10)
            log(f"backward: {out['secondary']['backward']['backward_ms']} ms")
        if run("factored"):
            log("factored inverse n=4096 FP64")
            out["secondary"]["factored"] = factored_secondary(P, torch, 5)
            log(f"factored: {out['secondary']['factored']}")
        if run("skul"):
            log("SKUL n=4096 FP64")
            out["secondary"]["skul"] = skul_secondary(P, torch, 3)
            log(f"skul: {out['secondary']['skul']}")
        if run("sqr"):
            log("SQR n=4096 FP64")
            out["secondary"]["sqr"] = sqr_secondary(P, torch, 3)
            log(f"sqr: {out['secondary']['sqr']}")
        if run("brsi"):
            log("BRSI n=4096 FP64")
            out["secondary"]["brsi"] = brsi_secondary(P, torch, 3)
            log(f"brsi: {out['secondary']['brsi']}")
        if n == 16384 and run("combrit"):
            log("COMBRIT beta = 4, 8 (FP64)")
            out["secondary"]["combrit"] = combrit_secondary(P, torch, Ld, 3)
            log(f"combrit: {out['secondary']['combrit']}")
    if not args.no_cpu_baseline:
        log("timing the CPU oracle on a bounded sample")
        out["cpu_baseline"] = cpu_baseline(L, args.cpu_seconds)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
