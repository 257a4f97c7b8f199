#!/usr/bin/env python3
"""Throughput of the stochastic gamma-EigenGame step on one MI355X.

A step is one full iteration of Alg. 2 (forward products, k x k terms,
backward products, update, auxiliary update) on one minibatch that is already
resident in HBM.  Default workload: CCA in FP32 with two views of width 512
(d = 1024), k = 16 players, minibatch 1024, Adam with the inverse-time
schedule; a ring of pre-generated synthetic minibatches is replayed through
a hipGraph that holds one pass over the ring.

Prints ONE JSON line (rank 0).  Usage:
    python bench.py [--gpus 1] [--steps K] [--warmup W] [--workload NAME]
                    [--no-cpu-baseline]
"""
from __future__ import annotations

import argparse
import ctypes
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

PEAK_FP32_MFMA_TFLOPS = 157.3
PEAK_FP64_MFMA_TFLOPS = 78.6
PEAK_HBM_GBS = 8000.0

# (name) -> workload description
WORKLOADS = {
    "cca_d1024_k16_b1024_fp32": dict(
        kind="cca", dtype="f32", dx=512, dy=512, k=16, b=1024, ring=128,
        optimizer="adam", schedule="inv", eta0=2e-3, t0=3000.0, gamma=0.3, rho=1e-6,
        generator="medium_cca",
        describe="CCA FP32: views 512+512 (d=1024), k=16, minibatch 1024; planted "
                 "correlations linspace(0.95,0.2,16), per-view condition 100"),
    "cca_d16_k4_b128_fp64": dict(
        kind="cca", dtype="f64", dx=8, dy=8, k=4, b=128, ring=128,
        optimizer="sgd", schedule="inv", eta0=1.0, t0=200.0, gamma=1.0, rho=1e-6,
        generator="tiny_cca",
        describe="CCA FP64: views 8+8 (d=16), k=4, minibatch 128; planted "
                 "correlations 0.9,0.7,0.5,0.3"),
}
DEFAULT = "cca_d1024_k16_b1024_fp32"


def hip_runtime():
    """The HIP runtime torch already loaded (same soname as ROCm's)."""
    lib = ctypes.CDLL("libamdhip64.so.7", mode=os.RTLD_NOLOAD | os.RTLD_GLOBAL)
    lib.hipEventCreate.argtypes = [ctypes.POINTER(ctypes.c_void_p)]
    lib.hipEventElapsedTime.argtypes = [ctypes.POINTER(ctypes.c_float), ctypes.c_void_p,
                                        ctypes.c_void_p]
    lib.hipEventSynchronize.argtypes = [ctypes.c_void_p]
    lib.hipEventDestroy.argtypes = [ctypes.c_void_p]
    return lib


def make_batches(w, ring):
    import synth
    if w["generator"] == "medium_cca":
        gen = synth.medium_cca(0)
        X, Y = gen.sample(ring * w["b"], np.random.default_rng([1, 0]))
    else:
        gen, pool = synth.tiny_cca_pool(0)
        idx = np.concatenate([pool.indices(t, w["b"]) for t in range(1, ring + 1)])
        X, Y = pool.X[idx], pool.Y[idx]
    npdt = np.float32 if w["dtype"] == "f32" else np.float64
    X = X.astype(npdt).reshape(ring, w["b"], w["dx"])
    Y = Y.astype(npdt).reshape(ring, w["b"], w["dy"])
    return X, Y


def config_for(sg, w):
    return sg.make_config(
        sg.SGEP_KIND_CCA if w["kind"] == "cca" else sg.SGEP_KIND_GENERAL,
        sg.SGEP_F32 if w["dtype"] == "f32" else sg.SGEP_F64,
        w["k"], w["dx"], w["dy"], w["b"],
        optimizer=sg.SGEP_ADAM if w["optimizer"] == "adam" else sg.SGEP_SGD,
        schedule={"const": sg.SGEP_SCHED_CONST, "inv": sg.SGEP_SCHED_INV}[w["schedule"]],
        eta0=w["eta0"], t0=w.get("t0", 1.0), gamma=w["gamma"], rho=w["rho"])


def kernel_source_hash(header: str = "sgep_kernels.hpp") -> str:
    """Hash of the device code of one kernel family (its header under csrc/);
    the launch grids the counters were taken with are in the same summary."""
    import hashlib
    h = hashlib.sha256()
    h.update(open(os.path.join(ROOT, "paper_2206_04993_amd", "csrc", header), "rb").read())
    return h.hexdigest()[:16]


def measured_traffic(workload: str, kernel: str):
    """HBM bytes per launch of `kernel` from the committed rocprofv3
    FETCH_SIZE / WRITE_SIZE summary (calibrated against a plain copy), or
    None when no summary exists or the kernel sources changed since."""
    path = os.path.join(ROOT, "profiles", f"traffic_{workload}.txt")
    if not os.path.exists(path):
        return None
    rec = {}
    for line in open(path):
        if line.startswith("json: "):
            rec = json.loads(line[6:])
    if rec.get("source_hash") != kernel_source_hash() or kernel not in rec.get("kernels", {}):
        return None
    k = rec["kernels"][kernel]
    return {"read_bytes": k["read_bytes"], "write_bytes": k["write_bytes"],
            "total_bytes": k["read_bytes"] + k["write_bytes"], "source": os.path.basename(path)}


def cpu_baseline(w, budget_s: float):
    """The FP64 oracle (Alg. 2 per player, OpenMP over players) on a bounded
    sample of the same workload: consecutive minibatches until budget_s of
    wall time is spent (at least 3)."""
    import oracle
    import synth
    if w["generator"] == "medium_cca":
        gen = synth.medium_cca(0)
        batch = lambda t: gen.batch(t, w["b"])
    else:
        _, pool = synth.tiny_cca_pool(0)
        batch = lambda t: pool.batch(t, w["b"])
    npdt = np.float32 if w["dtype"] == "f32" else np.float64
    pre = [tuple(a.astype(npdt).astype(np.float64) for a in batch(t)) for t in range(1, 9)]
    pb = oracle.Problem(oracle.KIND_CCA, w["k"], w["dx"], w["dy"], rho=w["rho"],
                        optimizer=oracle.OPT_ADAM if w["optimizer"] == "adam" else oracle.OPT_SGD)
    st = oracle.State.init(synth.initial_players(w["dx"] + w["dy"], w["k"], 0),
                           adam=w["optimizer"] == "adam")
    n = 0
    t0 = time.perf_counter()
    while True:
        X, Y = pre[n % len(pre)]
        oracle.gamma_step(pb, st, X, Y, oracle.eta(oracle.SCHED_INV, n + 1, w["eta0"],
                                                   t0=w.get("t0", 1.0)), w["gamma"])
        n += 1
        el = time.perf_counter() - t0
        if n >= 3 and el >= budget_s:
            break
    return {"value": n * w["b"] / el, "unit": "samples/s", "cores": oracle.threads(),
            "kind": "oracle",
            "sample": f"{n} consecutive iterations ({n * w['b']} samples) of the same workload, "
                      f"FP64 oracle, {el:.1f} s wall"}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=2048)
    ap.add_argument("--warmup", type=int, default=64)
    ap.add_argument("--workload", default=DEFAULT, choices=sorted(WORKLOADS))
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-budget", type=float, default=15.0)
    ap.add_argument("--calibrate-copy-mb", type=int, default=0,
                    help="also run a plain device copy of this many MiB (counter calibration)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py: this build measures one GPU only (asked for --gpus {args.gpus}); "
              "the multi-GPU sharding is described in DESIGN.md and not built.", file=sys.stderr)
        sys.exit(2)

    import torch
    import paper_2206_04993_amd as sg
    import synth

    sg.load()
    assert torch.cuda.is_available(), "bench.py needs a GPU"
    w = WORKLOADS[args.workload]
    K, W, R = args.steps, args.warmup, w["ring"]
    tdt = torch.float32 if w["dtype"] == "f32" else torch.float64
    Xh, Yh = make_batches(w, R)
    X = torch.from_numpy(Xh).to("cuda", dtype=tdt).contiguous()
    Y = torch.from_numpy(Yh).to("cuda", dtype=tdt).contiguous()
    del Xh, Yh
    torch.cuda.synchronize()
    d, k, b = w["dx"] + w["dy"], w["k"], w["b"]
    stream = torch.cuda.Stream()
    solver = sg.Solver(config_for(sg, w), synth.initial_players(d, k, 0), stream=stream)

    def step(t):
        s = t % R
        solver.step(X[s], Y[s])

    for t in range(W):
        step(t)
    torch.cuda.synchronize()

    # one hipGraph per pass over (a prefix of) the ring
    chunk = min(K, R)
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g, stream=stream):
        for t in range(chunk):
            step(t)
    torch.cuda.synchronize()
    n_rep, rem = divmod(K, chunk)

    if args.calibrate_copy_mb:
        # a plain copy of known size: FETCH_SIZE / WRITE_SIZE of this kernel
        # calibrate the per-dispatch counters of the step kernels
        src = torch.ones(args.calibrate_copy_mb << 18, device="cuda", dtype=torch.float32)
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst

    # ---- timed region: exactly K steps ----
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(n_rep):
        g.replay()
    with torch.cuda.stream(stream):
        for t in range(rem):
            step(t)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    ms_per_step = (t1 - t0) * 1e3 / K
    value = b / (ms_per_step * 1e-3)

    # ---- per-kernel durations: the same K steps again, each kernel launched
    # with a start/stop HIP event pair stamped by its own dispatch ----
    hip = hip_runtime()
    nev = 4 * K
    evs = [ctypes.c_void_p() for _ in range(nev)]
    for e in evs:
        assert hip.hipEventCreate(ctypes.byref(e)) == 0
    torch.cuda.synchronize()
    for t in range(K):
        s = t % R
        sg.sgep_step_profiled(solver.h, X[s], X[s].stride(0), Y[s], Y[s].stride(0), None, b,
                              [evs[4 * t + i].value for i in range(4)])
    torch.cuda.synchronize()
    ms = ctypes.c_float()
    fwd_us, bwd_us = [], []
    for t in range(K):
        assert hip.hipEventElapsedTime(ctypes.byref(ms), evs[4 * t], evs[4 * t + 1]) == 0
        fwd_us.append(ms.value * 1e3)
        assert hip.hipEventElapsedTime(ctypes.byref(ms), evs[4 * t + 2], evs[4 * t + 3]) == 0
        bwd_us.append(ms.value * 1e3)
    for e in evs:
        hip.hipEventDestroy(e)
    solver.sync()
    fwd_avg, bwd_avg = float(np.mean(fwd_us)), float(np.mean(bwd_us))

    # algorithmic work per launch (CCA): forward 2 b d k FLOPs, backward 4 b d k
    # FLOPs; bytes: one read of the minibatch (b d e) + state traffic
    e = 4 if w["dtype"] == "f32" else 8
    flops = {"k_fwd": 2.0 * b * d * k, "k_bwd": 4.0 * b * d * k}
    dom = "k_bwd" if bwd_avg >= fwd_avg else "k_fwd"
    dom_us = bwd_avg if dom == "k_bwd" else fwd_avg
    peak = PEAK_FP32_MFMA_TFLOPS if w["dtype"] == "f32" else PEAK_FP64_MFMA_TFLOPS
    achieved = flops[dom] / (dom_us * 1e-6) / 1e12
    roofline = {"bound": "mfma", "achieved": round(achieved, 3), "peak": peak,
                "unit": "TFLOP/s", "frac": round(achieved / peak, 5),
                "traffic": measured_traffic(args.workload, dom),
                "kernel": dom, "kernel_avg_us": round(dom_us, 3),
                "k_fwd_avg_us": round(fwd_avg, 3), "k_bwd_avg_us": round(bwd_avg, 3),
                "algorithmic_flops_per_launch": flops[dom],
                "algorithmic_hbm_bytes_per_step": float(
                    b * d * e + (8 if w["optimizer"] == "adam" else 4) * d * k * e)}

    out = {
        "metric": "samples/s per gamma-EigenGame step",
        "value": round(value, 1),
        "unit": "samples/s",
        "n_gpus": 1,
        "steps": K,
        "warmup": W,
        "ms_per_step": round(ms_per_step, 6),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": w["dtype"],
        "data": f"synthetic: ring of {R} pre-generated minibatches resident in HBM",
        "config": {"workload": args.workload, "description": w["describe"], "d": d, "k": k,
                   "minibatch": b, "optimizer": w["optimizer"], "graph_steps": chunk,
                   "parallelism": "single GPU"},
        "roofline": roofline,
    }
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(w, args.cpu_budget)
    solver.close()
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
