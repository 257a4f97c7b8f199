#!/usr/bin/env python3
"""Throughput of the stochastic gamma-EigenGame step on one MI355X.

A step is one full iteration of Alg. 2 (forward products, k x k terms,
backward products, update, auxiliary update) on one minibatch that is already
resident in HBM.  Default workload: CCA in FP32 with two views of width 512
(d = 1024), k = 16 players, minibatch 1024, Adam with the inverse-time
schedule.  A ring of pre-generated synthetic minibatches is replayed through a
hipGraph that holds one pass over the ring.

Other workloads (``--workload``): the FP64 tiny CCA, the large CCA
(8192 + 8192 activation-like views, k = 32, b = 4096) in BF16, FP8-e4m3 and
FP32, and the large LDA (d = 65536, 10 classes, k = 64, b = 2048) in BF16.

Prints ONE JSON line.  Usage:
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
PEAK_BF16_MFMA_TFLOPS = 2500.0
PEAK_HBM_GBS = 8000.0

_C3 = dict(kind="cca", dx=8192, dy=8192, k=32, b=4096, ring=4, optimizer="adam",
           schedule="inv", eta0=1e-3, t0=3000.0, gamma=0.3, rho=1e-6,
           generator="cca_activation")
_C5 = dict(kind="lda", dx=65536, dy=0, k=64, b=2048, ring=4, optimizer="adam",
           schedule="inv", eta0=1e-3, t0=3000.0, gamma=0.3, rho=1e-6, eps_reg=1e-4,
           n_classes=10, generator="lda_classes")

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
    "cca_d16384_k32_b4096_bf16": dict(
        _C3, dtype="bf16",
        describe="CCA BF16: activation-like views 8192+8192 (d=16384), k=32, minibatch 4096; "
                 "ReLU of a shared 64-dim Gaussian latent, log-normal feature scales"),
    "cca_d16384_k32_b4096_fp8": dict(
        _C3, dtype="fp8",
        describe="CCA FP8-e4m3 with per-column scales: activation-like views 8192+8192 "
                 "(d=16384), k=32, minibatch 4096"),
    "cca_d16384_k32_b4096_fp32": dict(
        _C3, dtype="f32",
        describe="CCA FP32 reference of the activation-like views 8192+8192 (d=16384), k=32, "
                 "minibatch 4096"),
    "lda_d65536_k64_b2048_bf16": dict(
        _C5, dtype="bf16",
        describe="LDA BF16: d=65536, 10 Gaussian classes with means on a random 64-dim "
                 "subspace, within-class B + 1e-4 I, k=64, minibatch 2048"),
}
DEFAULT = "cca_d1024_k16_b1024_fp32"

# kernels of one iteration, in launch order, and the header holding their code
KERNELS = {False: ("k_fwd", "k_bwd"), True: ("k_wfwd", "k_wmid", "k_wbwd")}
KERNEL_HEADER = {"k_fwd": "sgep_kernels.hpp", "k_bwd": "sgep_kernels.hpp",
                 "k_wfwd": "sgep_wide.hpp", "k_wmid": "sgep_wide.hpp", "k_wbwd": "sgep_wide.hpp"}


def hip_runtime():
    """The HIP runtime torch already loaded (same soname as ROCm's)."""
    lib = ctypes.CDLL("libamdhip64.so.7", mode=os.RTLD_NOLOAD | os.RTLD_GLOBAL)
    lib.hipEventCreate.argtypes = [ctypes.POINTER(ctypes.c_void_p)]
    lib.hipEventElapsedTime.argtypes = [ctypes.POINTER(ctypes.c_float), ctypes.c_void_p,
                                        ctypes.c_void_p]
    lib.hipEventSynchronize.argtypes = [ctypes.c_void_p]
    lib.hipEventDestroy.argtypes = [ctypes.c_void_p]
    return lib


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
    None when no summary exists or the kernel's code changed since."""
    path = os.path.join(ROOT, "profiles", f"traffic_{workload}.txt")
    if not os.path.exists(path):
        return None
    rec = {}
    for line in open(path):
        if line.startswith("json: "):
            rec = json.loads(line[6:])
    k = rec.get("kernels", {}).get(kernel)
    if k is None:
        return None
    if k.get("source_hash", rec.get("source_hash")) != kernel_source_hash(KERNEL_HEADER[kernel]):
        return None
    return {"read_bytes": k["read_bytes"], "write_bytes": k["write_bytes"],
            "total_bytes": k["read_bytes"] + k["write_bytes"], "source": os.path.basename(path)}


def _generator(w):
    import synth
    g = w["generator"]
    if g == "medium_cca":
        return synth.medium_cca(0)
    if g == "cca_activation":
        return synth.CCAActivation(dx=w["dx"], dy=w["dy"], seed=0)
    if g == "lda_classes":
        return synth.LDAClasses(d=w["dx"], c=w["n_classes"], seed=0)
    return synth.tiny_cca_pool(0)[1]


def host_batches(w, n):
    """The first n minibatches of the workload's seeded stream (host arrays;
    LDA: data and int32 labels)."""
    gen = _generator(w)
    b = w["b"]
    if w["generator"] == "medium_cca":
        X, Y = gen.sample(n * b, np.random.default_rng([1, 0]))
        return [(X[i * b:(i + 1) * b], Y[i * b:(i + 1) * b]) for i in range(n)]
    return [gen.batch(t, b) for t in range(1, n + 1)]


def encode(w, X, scales=None):
    """Storage format of the workload for host float data: a torch CPU tensor
    (FP32, FP64, BF16, or the uint8 e4m3 codes of X / scales, saturating) and
    the float64 values the device will see.  torch's conversions round to
    nearest even: the encoding of synth.bf16_bits and synth.e4m3_encode."""
    import torch
    dt = w["dtype"]
    if dt == "f64":
        t = torch.from_numpy(np.ascontiguousarray(X, dtype=np.float64))
        return t, t.numpy()
    if dt == "f32":
        t = torch.from_numpy(np.ascontiguousarray(X, dtype=np.float32))
        return t, t.numpy().astype(np.float64)
    x = torch.from_numpy(np.ascontiguousarray(X, dtype=np.float32))
    if dt == "bf16":
        t = x.to(torch.bfloat16)
        return t, t.to(torch.float64).numpy()
    s = torch.from_numpy(scales)
    t = torch.clamp(x / s, -448.0, 448.0).to(torch.float8_e4m3fn)
    return t.view(torch.uint8), (t.to(torch.float64) * s.to(torch.float64)).numpy()


def config_for(sg, w):
    dtype = {"f64": sg.SGEP_F64, "f32": sg.SGEP_F32, "bf16": sg.SGEP_BF16,
             "fp8": sg.SGEP_FP8_E4M3}[w["dtype"]]
    kind = {"cca": sg.SGEP_KIND_CCA, "lda": sg.SGEP_KIND_LDA}[w["kind"]]
    return sg.make_config(
        kind, dtype, w["k"], w["dx"], w["dy"], w["b"],
        optimizer=sg.SGEP_ADAM if w["optimizer"] == "adam" else sg.SGEP_SGD,
        schedule={"const": sg.SGEP_SCHED_CONST, "inv": sg.SGEP_SCHED_INV}[w["schedule"]],
        eta0=w["eta0"], t0=w.get("t0", 1.0), gamma=w["gamma"], rho=w["rho"],
        eps_reg=w.get("eps_reg", 0.0), n_classes=w.get("n_classes", 0))


def algorithmic_work(w, kernel):
    """(FLOPs, HBM bytes) one launch of `kernel` must do at minimum: one read
    of the minibatch, its products once, the O(d k) state it touches."""
    b, k = w["b"], w["k"]
    d = w["dx"] + w["dy"]
    e = {"f64": 8, "f32": 4, "bf16": 2, "fp8": 1}[w["dtype"]]
    adam = w["optimizer"] == "adam"
    lda = w["kind"] == "lda"
    c = w.get("n_classes", 0)
    data = b * d * e + (4 * b if lda else 0)
    se = 8 if w["dtype"] == "f64" else 4                       # state element
    state = (4 + (4 if adam else 0)) * se * d * k               # V, G (+ moments) read + written
    if kernel == "k_fwd":
        return 2.0 * b * d * k, float(data + se * d * k + se * 2 * b * k)
    if kernel == "k_bwd":
        return 4.0 * b * d * k, float(data + se * 2 * b * k + state)
    mw = k + c if lda else 2 * k                                # rows of the backward operand W
    if kernel == "k_wfwd":
        return 2.0 * b * d * k, float(data + 4 * d * k + 4 * b * k * (1 if lda else 2))
    if kernel == "k_wmid":
        return 0.0, float(4 * b * k * (1 if lda else 2) + 4 * b * mw)
    extra = (4 * c * d + 4 * d) if lda else 0                   # class means, their mean
    return 2.0 * b * d * mw, float(data + 4 * b * mw + state + 4 * d * k + extra)


def cpu_baseline(w, budget_s: float, host):
    """The FP64 oracle (Alg. 2 per player, OpenMP over players) on a bounded
    sample of the same workload: consecutive minibatches (the values the GPU
    receives) until budget_s of wall time is spent (at least 2)."""
    import oracle
    import synth
    lda = w["kind"] == "lda"
    extra = {}
    if lda:
        gen = _generator(w)
        extra = dict(class_means=gen.means,
                     class_priors=np.full(w["n_classes"], 1.0 / w["n_classes"]))
    pb = oracle.Problem(oracle.KIND_LDA if lda else oracle.KIND_CCA, w["k"], w["dx"], w["dy"],
                        rho=w["rho"], eps_reg=w.get("eps_reg", 0.0),
                        optimizer=oracle.OPT_ADAM if w["optimizer"] == "adam" else oracle.OPT_SGD,
                        **extra)
    st = oracle.State.init(synth.initial_players(w["dx"] + w["dy"], w["k"], 0),
                           adam=w["optimizer"] == "adam")
    n = 0
    t0 = time.perf_counter()
    while True:
        X, Y = host[n % len(host)]
        eta = oracle.eta(oracle.SCHED_INV, n + 1, w["eta0"], t0=w.get("t0", 1.0))
        if lda:
            oracle.gamma_step(pb, st, X, None, eta, w["gamma"], labels=Y)
        else:
            oracle.gamma_step(pb, st, X, Y, eta, w["gamma"])
        n += 1
        el = time.perf_counter() - t0
        if n >= 2 and el >= budget_s:
            break
    return {"value": n * w["b"] / el, "unit": "samples/s", "cores": oracle.threads(),
            "kind": "oracle",
            "sample": f"{n} consecutive iterations ({n * w['b']} samples) of the same workload "
                      f"on the values the GPU receives, FP64 oracle, {el:.1f} s wall"}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=None, help="timed steps (default per workload)")
    ap.add_argument("--warmup", type=int, default=None)
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
    big = w["b"] * (w["dx"] + w["dy"]) > 1 << 24
    K = args.steps if args.steps is not None else (256 if big else 2048)
    W = args.warmup if args.warmup is not None else (8 if big else 64)
    R = w["ring"]
    lda = w["kind"] == "lda"
    d, k, b = w["dx"] + w["dy"], w["k"], w["b"]

    # ---- the ring of minibatches, resident in HBM ----
    print(f"bench: generating {R} minibatches of {args.workload}", file=sys.stderr, flush=True)
    raw = host_batches(w, R)
    aux, scales = {}, None
    if w["dtype"] == "fp8":
        # per-column scales calibrated on the resident ring (all R minibatches)
        scales = (synth.fp8_column_scales(np.concatenate([r[0] for r in raw])),
                  synth.fp8_column_scales(np.concatenate([r[1] for r in raw])))
        aux = dict(x_col_scale=scales[0], y_col_scale=scales[1])
    if lda:
        gen = _generator(w)
        aux = dict(class_means=gen.means,
                   class_priors=np.full(w["n_classes"], 1.0 / w["n_classes"]))
    Xs, Ys, host = [], [], []
    for i, (Xr, Yr) in enumerate(raw):
        tx, vx = encode(w, Xr, scales[0] if scales else None)
        if lda:
            ty = torch.from_numpy(np.ascontiguousarray(Yr, dtype=np.int32))
            vy = ty.numpy()
        else:
            ty, vy = encode(w, Yr, scales[1] if scales else None)
        Xs.append(tx)
        Ys.append(ty)
        if i < 3:
            host.append((vx, vy))
    del raw
    X = torch.stack(Xs).to("cuda").contiguous()
    Y = torch.stack(Ys).to("cuda").contiguous()
    del Xs, Ys
    torch.cuda.synchronize()
    stream = torch.cuda.Stream()
    solver = sg.Solver(config_for(sg, w), synth.initial_players(d, k, 0), stream=stream, **aux)
    wide = solver.kernels_per_step() == 3

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

    # ---- per-kernel durations: the same steps again, each kernel launched
    # with a start/stop HIP event pair stamped by its own dispatch ----
    names = KERNELS[wide]
    nk = len(names)
    hip = hip_runtime()
    Kp = min(K, 512)
    evs = [ctypes.c_void_p() for _ in range(2 * nk * Kp)]
    for e in evs:
        assert hip.hipEventCreate(ctypes.byref(e)) == 0
    torch.cuda.synchronize()
    for t in range(Kp):
        s = t % R
        ev = [evs[2 * nk * t + i].value for i in range(2 * nk)]
        if lda:
            sg.sgep_step_profiled(solver.h, X[s], X[s].stride(0), None, 0, Y[s], b, ev)
        else:
            sg.sgep_step_profiled(solver.h, X[s], X[s].stride(0), Y[s], Y[s].stride(0), None, b,
                                  ev)
    torch.cuda.synchronize()
    ms = ctypes.c_float()
    dur = {n: [] for n in names}
    for t in range(Kp):
        for i, n in enumerate(names):
            assert hip.hipEventElapsedTime(ctypes.byref(ms), evs[2 * nk * t + 2 * i],
                                           evs[2 * nk * t + 2 * i + 1]) == 0
            dur[n].append(ms.value * 1e3)
    for e in evs:
        hip.hipEventDestroy(e)
    solver.sync()
    avg = {n: float(np.mean(v)) for n, v in dur.items()}
    dom = max(avg, key=avg.get)
    flops, nbytes = algorithmic_work(w, dom)
    if w["dtype"] in ("bf16", "fp8"):
        achieved = nbytes / (avg[dom] * 1e-6) / 1e9
        roofline = {"bound": "hbm", "achieved": round(achieved, 1), "peak": PEAK_HBM_GBS,
                    "unit": "GB/s", "frac": round(achieved / PEAK_HBM_GBS, 5)}
    else:
        peak = PEAK_FP32_MFMA_TFLOPS if w["dtype"] == "f32" else PEAK_FP64_MFMA_TFLOPS
        achieved = flops / (avg[dom] * 1e-6) / 1e12
        roofline = {"bound": "mfma", "achieved": round(achieved, 3), "peak": peak,
                    "unit": "TFLOP/s", "frac": round(achieved / peak, 5)}
    roofline.update({
        "traffic": measured_traffic(args.workload, dom),
        "kernel": dom, "kernel_avg_us": round(avg[dom], 3),
        "kernels_avg_us": {n: round(v, 3) for n, v in avg.items()},
        "algorithmic_flops_per_launch": flops,
        "algorithmic_hbm_bytes_per_launch": nbytes,
    })

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
        out["cpu_baseline"] = cpu_baseline(w, args.cpu_budget, host)
    solver.close()
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
