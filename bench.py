#!/usr/bin/env python3
"""Throughput and time to accuracy of the stochastic gamma-EigenGame step on
one MI355X.

A step is one full iteration of Alg. 2 (forward products, k x k terms,
backward products, update, auxiliary update) on one minibatch that is already
resident in HBM.  Default workload: the large LDA-form problem (d = 65536,
10 Gaussian classes with means on a random 64-dim subspace, diagonal
within-class covariance + 1e-4 I, k = 64 players, minibatch 2048) with the
minibatch stored in BF16 -- the line's value -- and, beside it, the same
problem with FP32 minibatches (``fp32_reference``).  A ring of pre-generated
synthetic minibatches is replayed through a hipGraph that holds one pass over
the ring.  Both dtypes also run a time-to-accuracy leg on fresh minibatches
drawn on the device, graded against the exact population solution (the top
c - 1 = 9 generalized eigenvectors, from the reduced c x c problem), within a
bounded number of steps.

Other workloads (``--workload``): the FP64 tiny CCA, the medium FP32 CCA
(d = 1024, k = 16, b = 1024; BF16 / FP8 ingest, Alg. 3, centring variants),
the ICA problem, the large CCA (8192 + 8192 activation-like views, k = 32,
b = 4096) in BF16, FP8-e4m3 and FP32, and 256 independent general instances
(d uniform in [64, 2048], k = 8, b = 512) advanced together in FP32.

Prints ONE JSON line.  Usage:
    python bench.py [--gpus 1] [--steps K] [--warmup W] [--workload NAME]
                    [--no-cpu-baseline] [--no-tta] [--tta-steps N]
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
           generator="cca_activation",
           tta=dict(targets=(5e-3, 2e-3, 1e-3, 5e-4), every=500, max_steps=30_000, chunk=25))
# the large LDA problem: plain ascent (Alg. 2) with the inverse-time
# schedule, which reaches a given subspace error in fewer steps than Adam on
# this problem (d / b = 32: the minibatch within-class covariance is noisy,
# and Adam's per-coordinate steps follow the noise); a slow auxiliary rate
# gamma averages the noise of [Bv]
_C5 = dict(kind="lda", dx=65536, dy=0, k=64, b=2048, ring=4, optimizer="sgd",
           schedule="inv", eta0=4e-3, t0=250.0, gamma=0.015, rho=1e-6, eps_reg=1e-4,
           n_classes=10, generator="lda_classes")
# time to accuracy: graded on the top c - 1 = 9 players (rank of the
# between-class A), within a bounded number of steps
_C5_TTA = dict(targets=(1e-1, 5e-2, 2e-2, 1e-2, 5e-3, 2e-3, 1e-3), every=8000,
               max_steps=96_000, chunk=50)

# (name) -> workload description
WORKLOADS = {
    "cca_d1024_k16_b1024_fp32": dict(
        kind="cca", dtype="f32", dx=512, dy=512, k=16, b=1024, ring=128,
        optimizer="adam", schedule="inv", eta0=4e-3, t0=100.0, gamma=0.3, rho=1e-6,
        generator="medium_cca", tta=dict(targets=(5e-3, 1e-3), max_steps=100_000, every=1000),
        describe="CCA FP32: views 512+512 (d=1024), k=16, minibatch 1024; planted "
                 "correlations linspace(0.95,0.2,16), per-view condition 100"),
    "cca_d1024_k16_b1024_fp32_alg3": dict(
        kind="cca", dtype="f32", dx=512, dy=512, k=16, b=1024, ring=128,
        optimizer="adam", schedule="inv", eta0=4e-3, t0=100.0, gamma=0.3, rho=1e-3,
        smooth=1, nu=4.0,
        generator="medium_cca", tta=dict(targets=(5e-3, 1e-3), max_steps=100_000, every=1000),
        describe="the medium FP32 CCA (views 512+512, k=16, minibatch 1024) with Alg. 3: "
                 "parents' B-norms estimated in log space between rho=1e-3 and nu=4"),
    "cca_d1024_k16_b1024_fp32_center": dict(
        kind="cca", dtype="f32", dx=512, dy=512, k=16, b=1024, ring=128,
        optimizer="adam", schedule="warmup", eta0=4e-3, t_c=100.0, eta_T=4e-6, T=100_000.0,
        gamma=0.3, rho=1e-6, center=1, offset=1.0,
        generator="medium_cca", tta=dict(targets=(5e-3, 1e-3), max_steps=100_000, every=1000),
        describe="the medium FP32 CCA (views 512+512, k=16, minibatch 1024) shifted by fixed "
                 "per-feature offsets N(0, 1), centred by running means of the views; "
                 "eta warms up over 100 steps while the means settle, then decays "
                 "harmonically"),
    "ica_d1024_k16_b1024_fp32": dict(
        kind="ica", dtype="f32", dx=1024, dy=0, k=16, b=1024, ring=128,
        optimizer="adam", schedule="inv", eta0=1e-3, t0=1000.0, gamma=0.3, rho=1e-6,
        eps_reg=1e-4, generator="ica_mixed",
        tta=dict(targets=(1e-1, 7e-2), max_steps=60_000, every=1000),
        describe="ICA (kurtosis form): d=1024 orthogonal mixtures of 16 Bernoulli-Gaussian "
                 "sources with excess kurtosis linspace(20, 2, 16) and 1008 Gaussian ones, "
                 "k=16, minibatch 1024, B ridge 1e-4"),
    "cca_d16_k4_b128_fp64": dict(
        kind="cca", dtype="f64", dx=8, dy=8, k=4, b=128, ring=128,
        optimizer="sgd", schedule="inv", eta0=1.0, t0=200.0, gamma=1.0, rho=1e-6,
        generator="tiny_cca", tta=dict(targets=(1e-3,), max_steps=6000, every=100),
        describe="CCA FP64: views 8+8 (d=16), k=4, minibatch 128; planted "
                 "correlations 0.9,0.7,0.5,0.3"),
    "cca_d1024_k16_b1024_bf16": dict(
        kind="cca", dtype="bf16", dx=512, dy=512, k=16, b=1024, ring=128,
        optimizer="adam", schedule="inv", eta0=4e-3, t0=100.0, gamma=0.3, rho=1e-6,
        generator="medium_cca", tta=dict(targets=(5e-3, 1e-3), max_steps=100_000, every=1000),
        describe="CCA BF16 ingest of the medium problem: views 512+512 (d=1024), k=16, "
                 "minibatch 1024 (same generator and target as the FP32 workload)"),
    "cca_d1024_k16_b1024_fp8": dict(
        kind="cca", dtype="fp8", dx=512, dy=512, k=16, b=1024, ring=128,
        optimizer="adam", schedule="inv", eta0=4e-3, t0=100.0, gamma=0.3, rho=1e-6,
        generator="medium_cca", tta=dict(targets=(5e-3, 1e-3), max_steps=100_000, every=1000),
        describe="CCA FP8-e4m3 ingest (per-column scales) of the medium problem: views 512+512 "
                 "(d=1024), k=16, minibatch 1024"),
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
        _C5, dtype="bf16", twin="lda_d65536_k64_b2048_fp32", tta=_C5_TTA,
        describe="LDA BF16: d=65536, 10 Gaussian classes with means on a random 64-dim "
                 "subspace, within-class B + 1e-4 I, k=64, minibatch 2048"),
    "lda_d65536_k64_b2048_fp32": dict(
        _C5, dtype="f32", tta=_C5_TTA,
        describe="LDA FP32 reference: d=65536, 10 Gaussian classes with means on a random "
                 "64-dim subspace, within-class B + 1e-4 I, k=64, minibatch 2048"),
}
# many independent GENERAL instances advanced together (widths uniform in
# [64, 2048], planted generalized eigenvalues geomspace(10, 0.1, 8), B ridge
# 1e-3); minibatches drawn on the device
BATCH_WORKLOADS = {
    "batch256_general_d64-2048_k8_b512_fp32": dict(
        kind="batch", dtype="f32", n=256, lo=64, hi=2048, k=8, b=512, ring=2,
        optimizer="adam", schedule="inv", eta0=1e-3, t0=3000.0, gamma=0.3, rho=1e-6,
        eps_reg=1e-3,
        tta=dict(targets=(1e-1, 5e-2, 2e-2, 1e-2, 5e-3), every=1000, max_steps=12_000, chunk=8),
        describe="256 independent general SGEP instances (A = E[yy^T], B = E[xx^T] + 1e-3 I), "
                 "d uniform in [64, 2048], k=8, minibatch 512, FP32, one batched iteration "
                 "per step in the autotuned launch plan"),
}
DEFAULT = "lda_d65536_k64_b2048_bf16"

# the header holding each kernel's code
KERNEL_HEADER = {"k_fwd": "sgep_kernels.hpp", "k_fwds": "sgep_kernels.hpp",
                 "k_bwd": "sgep_kernels.hpp",
                 "k_coef": "sgep_kernels.hpp", "k_bwdp": "sgep_kernels.hpp",
                 "k_bwd1": "sgep_kernels.hpp", "k_fwd2": "sgep_kernels.hpp",
                 "k_coefa": "sgep_kernels.hpp", "k_coefb": "sgep_kernels.hpp",
                 "k_wfwd": "sgep_wide.hpp", "k_wmid": "sgep_wide.hpp", "k_wbwd": "sgep_wide.hpp",
                 "k_wprod": "sgep_wide.hpp", "k_wepi": "sgep_wide.hpp",
                 "k_bfwd": ("sgep_kernels.hpp", "sgep_batch.hpp"),
                 "k_bcoef": ("sgep_kernels.hpp", "sgep_batch.hpp"),
                 "k_bbwd": ("sgep_kernels.hpp", "sgep_batch.hpp"),
                 "k_bpers": ("sgep_kernels.hpp", "sgep_batch.hpp")}


def hip_runtime():
    """The HIP runtime torch already loaded (same soname as ROCm's)."""
    lib = ctypes.CDLL("libamdhip64.so.7", mode=os.RTLD_NOLOAD | os.RTLD_GLOBAL)
    lib.hipEventCreate.argtypes = [ctypes.POINTER(ctypes.c_void_p)]
    lib.hipEventElapsedTime.argtypes = [ctypes.POINTER(ctypes.c_float), ctypes.c_void_p,
                                        ctypes.c_void_p]
    lib.hipEventSynchronize.argtypes = [ctypes.c_void_p]
    lib.hipEventDestroy.argtypes = [ctypes.c_void_p]
    return lib


def kernel_source_hash(header="sgep_kernels.hpp") -> str:
    """Hash of the device code of one kernel family (its header, or headers,
    under csrc/); the launch grids the counters were taken with are in the
    same summary."""
    import hashlib
    h = hashlib.sha256()
    for name in ((header,) if isinstance(header, str) else header):
        h.update(open(os.path.join(ROOT, "paper_2206_04993_amd", "csrc", name), "rb").read())
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
    if g == "ica_mixed":
        return synth.ICAMixed(d=w["dx"], kurtosis=tuple(np.linspace(20.0, 2.0, 16)), seed=0)
    return synth.tiny_cca_pool(0)[1]


def offsets(w):
    """Fixed per-feature offsets of a non-zero-mean stream (None: zero-mean)."""
    if not w.get("offset"):
        return None
    rng = np.random.default_rng([7, 0])
    return rng.normal(0.0, w["offset"], w["dx"]), rng.normal(0.0, w["offset"], w["dy"])


def _eta(w, t):
    """eta_t of the workload's schedule (the oracle's definition)."""
    import oracle
    sched = {"const": oracle.SCHED_CONST, "inv": oracle.SCHED_INV,
             "warmup": oracle.SCHED_WARMUP_HARMONIC}[w["schedule"]]
    return oracle.eta(sched, t, w["eta0"], eta_T=w.get("eta_T", 0.0), t0=w.get("t0", 1.0),
                      t_c=w.get("t_c", 1.0), T=w.get("T", 1.0))


def host_batches(w, n):
    """The first n minibatches of the workload's seeded stream (host arrays;
    LDA: data and int32 labels)."""
    gen = _generator(w)
    b = w["b"]
    if w["generator"] == "medium_cca":
        X, Y = gen.sample(n * b, np.random.default_rng([1, 0]))
        off = offsets(w)
        if off is not None:
            X, Y = X + off[0], Y + off[1]
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
    kind = {"cca": sg.SGEP_KIND_CCA, "lda": sg.SGEP_KIND_LDA, "ica": sg.SGEP_KIND_ICA}[w["kind"]]
    return sg.make_config(
        kind, dtype, w["k"], w["dx"], w["dy"], w["b"],
        optimizer=sg.SGEP_ADAM if w["optimizer"] == "adam" else sg.SGEP_SGD,
        schedule={"const": sg.SGEP_SCHED_CONST, "inv": sg.SGEP_SCHED_INV,
                  "warmup": sg.SGEP_SCHED_WARMUP_HARMONIC}[w["schedule"]],
        eta0=w["eta0"], t0=w.get("t0", 1.0), t_c=w.get("t_c", 1.0), eta_T=w.get("eta_T", 0.0),
        T=w.get("T", 1.0), gamma=w["gamma"], rho=w["rho"],
        eps_reg=w.get("eps_reg", 0.0), n_classes=w.get("n_classes", 0),
        smooth=w.get("smooth", 0), nu=w.get("nu", 0.0), center=w.get("center", 0))


def algorithmic_work(w, kernel, names=()):
    """(FLOPs, HBM bytes) one launch of `kernel` must do at minimum: one read
    of the minibatch, its products once, the O(d k) state it touches.  names:
    the kernels of the iteration (with k_bwdp, k_bwd is the finishing pass:
    the update alone)."""
    b, k = w["b"], w["k"]
    d = w["dx"] + w["dy"]
    e = {"f64": 8, "f32": 4, "bf16": 2, "fp8": 1}[w["dtype"]]
    adam = w["optimizer"] == "adam"
    lda = w["kind"] == "lda"
    c = w.get("n_classes", 0)
    data = b * d * e + (4 * b if lda else 0)
    se = 8 if w["dtype"] == "f64" else 4                       # state element
    state = (4 + (4 if adam else 0)) * se * d * k               # V, G (+ moments) read + written
    if w["kind"] == "ica":  # four passes: P; X^T [P|Q]; X C V; X^T X C V + update
        if kernel == "k_fwd":
            return 2.0 * b * d * k, float(data + se * d * k + se * 2 * b * k)
        if kernel == "k_bwd1":
            return 4.0 * b * d * k, float(data + se * 2 * b * k + se * 2 * d * k)
        if kernel == "k_fwd2":
            return 2.0 * b * d * k, float(data + se * d * k + se * b * k)
        return 2.0 * b * d * k, float(data + se * b * k + se * 2 * d * k + state)
    if kernel in ("k_fwd", "k_fwds"):
        return 2.0 * b * d * k, float(data + se * d * k + se * 2 * b * k)
    if kernel == "k_coefb":  # the column totals of k_coefa
        kp = 16 if k <= 16 else (32 if k <= 32 else 64)
        return 0.0, float(8 * (kp * (kp + 1) // 2 + kp))
    if kernel in ("k_coef", "k_coefa"):  # the Gram partials of the forward row tiles, once
        kp = 16 if k <= 16 else (32 if k <= 32 else 64)
        return 0.0, float(8 * (kp * (kp + 1) // 2 + kp) * ((b + 15) // 16))
    if kernel == "k_bwdp":  # without a finishing pass it also runs the update
        return 4.0 * b * d * k, float(data + se * 2 * b * k + (0 if "k_bwd" in names else state))
    if kernel == "k_bwd" and "k_bwdp" in names:
        return 0.0, float(state)
    if kernel == "k_bwd":
        return 4.0 * b * d * k, float(data + se * 2 * b * k + state)
    mw = k + c if lda else 2 * k                                # rows of the backward operand W
    mp = k if lda else 2 * k                                    # of them, rows multiplied by X^T
    if kernel == "k_wfwd":
        return 2.0 * b * d * k, float(data + 4 * d * k + 4 * b * k * (1 if lda else 2))
    if kernel == "k_wmid":
        return 0.0, float(4 * b * k * (1 if lda else 2) + 4 * b * mw)
    extra = (4 * c * d + 4 * d) if lda else 0                   # class means, their mean
    if kernel == "k_wprod":  # X^T W of the split backward: products to memory
        return 2.0 * b * d * mp, float(data + 4 * b * mw + 4 * d * mp)
    if kernel == "k_wepi":   # its epilogue: products in, state, next V operand out
        return 0.0, float(4 * d * mp + state + 4 * d * k + extra)
    return 2.0 * b * d * mp, float(data + 4 * b * mw + state + 4 * d * k + extra)


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
    okind = {"cca": oracle.KIND_CCA, "lda": oracle.KIND_LDA, "ica": oracle.KIND_ICA}[w["kind"]]
    pb = oracle.Problem(okind, w["k"], w["dx"], w["dy"],
                        rho=w["rho"], eps_reg=w.get("eps_reg", 0.0),
                        optimizer=oracle.OPT_ADAM if w["optimizer"] == "adam" else oracle.OPT_SGD,
                        smooth=bool(w.get("smooth", 0)), nu=w.get("nu", 0.0),
                        center=bool(w.get("center", 0)), **extra)
    st = oracle.State.init(synth.initial_players(w["dx"] + w["dy"], w["k"], 0),
                           adam=w["optimizer"] == "adam")
    n = 0
    t0 = time.perf_counter()
    while True:
        X, Y = host[n % len(host)]
        eta = _eta(w, n + 1)
        if lda:
            oracle.gamma_step(pb, st, X, None, eta, w["gamma"], labels=Y)
        else:
            oracle.gamma_step(pb, st, X, Y, eta, w["gamma"])
        n += 1
        el = time.perf_counter() - t0
        if n >= 2 and el >= budget_s:
            break
    thr = oracle.threads()
    return {"value": n * w["b"] / el, "unit": "samples/s", "cores": min(thr, w["k"]),
            "kind": "oracle", "omp_threads": thr, **host_info(),
            "parallelism": "OpenMP over the k players (at most k threads busy)",
            "sample": f"{n} consecutive iterations ({n * w['b']} samples) of the same workload "
                      f"on the values the GPU receives, FP64 oracle, {el:.1f} s wall"}


def calibration_copy(mib: int):
    """A plain device copy of known size: its FETCH_SIZE / WRITE_SIZE counters
    calibrate the per-dispatch counters of the step kernels."""
    import torch
    src = torch.ones(mib << 18, device="cuda", dtype=torch.float32)
    dst = torch.empty_like(src)
    for _ in range(3):
        dst.copy_(src)
    torch.cuda.synchronize()
    del src, dst


def time_to_accuracy(w, targets, max_steps: int, every: int, hyper=None, log=None):
    """Time to each subspace error in `targets` (normalised, Gram form of
    App. A) for a single-handle workload, by the rule: summed step time (HIP
    events around hipGraph replays of `every` steps) up to the first
    evaluation at or below the target whose next evaluation also is.
    Minibatches are refilled and the error evaluated outside the timed region;
    the run stops when the smallest target is met or after max_steps.
      medium CCA: fresh pairs drawn on the device from the same generator
                  each chunk (stored in the workload's format: FP32, BF16, or
                  FP8-e4m3 with per-column scales fixed from a 65,536-pair
                  prefix); target the population solution (planted
                  correlations, closed form)
      tiny CCA:   i.i.d. minibatches of the fixed 10,000-pair pool; target
                  the pool's exact FP64 solution (oracle)
      large CCA:  fresh activation-like pairs drawn on the device each chunk
                  (FP32, BF16, or FP8-e4m3 with per-column scales fixed from a
                  65,536-pair prefix); target the population solution from the
                  arc-cosine-kernel covariances: the players' subspace graded
                  by its containment in the leading block of r near-equal
                  canonical correlations (r = 64, the latent width; the block
                  is separated from the next correlation by 0.06, while its
                  own correlations differ by less than 1e-4)
      LDA:        fresh labelled rows drawn on the device each chunk (stored
                  in the workload's format); target the exact population
                  solution from the reduced c x c problem, graded on the top
                  c - 1 players (the rank of the between-class A)
    Steps run in hipGraph replays of the workload's `chunk` steps (default
    `every`)."""
    import torch
    import oracle
    import paper_2206_04993_amd as sg
    import synth
    from oracle import targets as otargets

    w = dict(w, **(hyper or {}))
    targets = sorted(targets, reverse=True)
    d, k, b = w["dx"] + w["dy"], w["k"], w["b"]
    E = w.get("tta", {}).get("chunk", every)  # steps per hipGraph replay
    assert every % E == 0
    fmt = w["dtype"]
    store = {"f64": torch.float64, "f32": torch.float32, "bf16": torch.bfloat16,
             "fp8": torch.uint8}[fmt]
    aux = {}
    graded = k  # players graded (LDA: the top c - 1)
    metric = oracle.subspace_error
    lda = w["kind"] == "lda"
    if lda:
        gen = _generator(w)
        graded = w["n_classes"] - 1
        _, Vs = otargets.lda_reduced_topk(gen, graded, w["eps_reg"])
        B = gen.sigma ** 2 + w["eps_reg"]  # the diagonal of B
        ref = (f"exact population solution, top {graded} generalized eigenvectors (rank of the "
               "between-class A) from the reduced c x c problem")
        aux = dict(class_means=gen.means, class_priors=np.full(w["n_classes"], 1.0 / w["n_classes"]))
        tables = gen.device_tables("cuda")

        def fill(c, Xb, Lb):
            for j in range(E):
                _, lab = gen.sample_torch(b, 1_000_000 + c * E + j, "cuda", store, tables=tables,
                                          out=Xb[j])
                Lb[j].copy_(lab)
    elif w["generator"] == "cca_activation":
        gen = _generator(w)
        Sxx, Syy, Sxy = otargets.cca_activation_population(gen)
        # the leading r canonical correlations (r the latent width) form a
        # near-degenerate block well separated from the rest: the players are
        # graded by the containment of their subspace in that block
        nblk = gen.r
        _, Vs = otargets.cca_topk_subspace(Sxx, Syy, Sxy, nblk, p=nblk + 16)
        dxv = w["dx"]

        def B(M):
            return np.vstack([Sxx @ M[:dxv], Syy @ M[dxv:]])

        metric = oracle.subspace_containment_error
        ref = (f"exact population solution (arc-cosine-kernel covariances): the leading block "
               f"of {nblk} canonical correlations, players graded by containment in it")
        tables = gen.device_tables("cuda")
        scales = None
        if fmt == "fp8":
            px, py = gen.sample_torch(65536, 999_999, "cuda", torch.float32, tables=tables)
            scales = (synth.fp8_column_scales(px.cpu().numpy()),
                      synth.fp8_column_scales(py.cpu().numpy()))
            aux = dict(x_col_scale=scales[0], y_col_scale=scales[1])
            sxa = torch.from_numpy(scales[0]).cuda()
            sya = torch.from_numpy(scales[1]).cuda()
            del px, py

        def fill(c, Xb, Yb):
            for j in range(E):
                x, y = gen.sample_torch(b, 1_000_000 + c * E + j, "cuda", torch.float32,
                                        tables=tables)
                if fmt == "fp8":
                    Xb[j].copy_(torch.clamp(x / sxa, -448.0, 448.0).to(torch.float8_e4m3fn)
                                .view(torch.uint8))
                    Yb[j].copy_(torch.clamp(y / sya, -448.0, 448.0).to(torch.float8_e4m3fn)
                                .view(torch.uint8))
                else:
                    Xb[j].copy_(x)
                    Yb[j].copy_(y)
    elif w["generator"] == "ica_mixed":
        gen = _generator(w)
        _, Vs = otargets.ica_planted_topk(gen, k)
        A_, B = otargets.ica_population_AB(gen)
        B = B + w.get("eps_reg", 0.0) * np.eye(d)
        ref = "population solution of the generator (mixing columns of the most kurtotic sources)"

        def fill(c, Xb, Yb):
            Xb.copy_(gen.sample_torch(E * b, 1_000_000 + c, "cuda", torch.float32)
                     .to(store).view(E, b, -1))
    elif w["generator"] == "medium_cca":
        gen = synth.medium_cca(0)
        _, Vs = otargets.cca_planted_topk(gen, k)
        _, B = otargets.cca_population_AB(gen)
        ref = "population solution of the generator (planted correlations, closed form)"
        scales = None
        if fmt == "fp8":
            px, py = gen.sample_torch(65536, 999_999, "cuda", torch.float32)
            scales = (synth.fp8_column_scales(px.cpu().numpy()),
                      synth.fp8_column_scales(py.cpu().numpy()))
            aux = dict(x_col_scale=scales[0], y_col_scale=scales[1])
            sx = torch.from_numpy(scales[0]).cuda()
            sy = torch.from_numpy(scales[1]).cuda()

        def conv(v, sc):
            if fmt == "fp8":  # e4m3 codes of v / s, saturating, nearest even
                return torch.clamp(v / sc, -448.0, 448.0).to(torch.float8_e4m3fn).view(torch.uint8)
            return v.to(store)

        off = offsets(w)
        if off is not None:
            off = tuple(torch.from_numpy(o).to("cuda", torch.float32) for o in off)

        def fill(c, Xb, Yb):
            x, y = gen.sample_torch(E * b, 1_000_000 + c, "cuda", torch.float32)
            if off is not None:
                x, y = x + off[0], y + off[1]
            Xb.copy_(conv(x, sx if fmt == "fp8" else None).view(E, b, -1))
            Yb.copy_(conv(y, sy if fmt == "fp8" else None).view(E, b, -1))
    else:
        gen, pool = synth.tiny_cca_pool(0)
        pb = oracle.Problem(oracle.KIND_CCA, k, w["dx"], w["dy"])
        A, B = oracle.problem_matrices(pb, pool.X, pool.Y)
        _, Vs = oracle.gep_topk(A, B, k)
        ref = "exact FP64 solution of the 10,000-pair pool (oracle)"
        PX = torch.from_numpy(pool.X).to("cuda", store)
        PY = torch.from_numpy(pool.Y).to("cuda", store)

        def fill(c, Xb, Yb):
            idx = np.concatenate([pool.indices(c * E + j + 1, b) for j in range(E)])
            it = torch.from_numpy(idx).cuda()
            Xb.copy_(PX.index_select(0, it).view(E, b, -1))
            Yb.copy_(PY.index_select(0, it).view(E, b, -1))
    Xb = torch.empty((E, b, w["dx"]), device="cuda", dtype=store)
    if lda:
        Yb = torch.empty((E, b), device="cuda", dtype=torch.int32)
    else:
        Yb = (torch.empty((E, b, w["dy"]), device="cuda", dtype=store) if w["dy"] else
              [None] * E)
    stream = torch.cuda.Stream()
    solver = sg.Solver(config_for(sg, w), synth.initial_players(d, k, 0), stream=stream, **aux)
    fill(0, Xb, Yb)
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g, stream=stream):
        for j in range(E):
            solver.step(Xb[j], Yb[j])
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    t_gpu, steps, hist, hits = 0.0, 0, [], {}
    c = 0
    while steps < max_steps:
        if c > 0:
            fill(c, Xb, Yb)
            torch.cuda.synchronize()
        with torch.cuda.stream(stream):  # a graph replays on the current stream
            e0.record(stream)
            g.replay()
            e1.record(stream)
        e1.synchronize()
        t_gpu += e0.elapsed_time(e1) * 1e-3
        steps += E
        c += 1
        if steps % every:
            continue
        err = metric(solver.vectors()[:, :graded], Vs, B)
        hist.append((steps, t_gpu, err))
        if log:
            log(f"tta {fmt} steps {steps} gpu {t_gpu:.3f}s err {err:.3e}")
        for tg in targets:
            if tg not in hits and len(hist) >= 2 and hist[-2][2] <= tg and err <= tg:
                hits[tg] = hist[-2]
        if targets[-1] in hits:
            break
    solver.close()
    out = {"targets": {}, "eval_every_steps": every, "reference": ref,
           "stream": ("fresh device-drawn samples"
                      if w["generator"] in ("medium_cca", "ica_mixed", "lda_classes",
                                            "cca_activation")
                      else "i.i.d. minibatches of the pool") + f", stored as {fmt}",
           "graded_players": graded, "max_steps": max_steps,
           "final_error": hist[-1][2] if hist else None, "steps_run": steps,
           "gpu_seconds_run": round(t_gpu, 4),
           "trajectory": [(h[0], round(h[1], 4), h[2]) for h in hist]}
    for tg in targets:
        h = hits.get(tg)
        out["targets"][f"{tg:g}"] = ({"reached": True, "seconds": round(h[1], 4), "steps": h[0],
                                      "samples": h[0] * b} if h else {"reached": False})
    return out


def run_batch(args, w):
    """The many-instance workload: value = instance-samples/s (n b per step)."""
    import torch
    import paper_2206_04993_amd as sg
    import synth

    sg.load()
    n, k, b, R = w["n"], w["k"], w["b"], w["ring"]
    K = args.steps if args.steps is not None else 128
    W = args.warmup if args.warmup is not None else 8
    gens = synth.batched_general(n, w["lo"], w["hi"], k, w["eps_reg"], seed=0)
    dims = [g.d for g in gens]
    print(f"bench: drawing {R} minibatches of {n} instances on the device", file=sys.stderr,
          flush=True)
    ring = []
    for t in range(1, R + 1):
        xs, ys = [], []
        for g in gens:
            x, y = g.sample_torch(b, t, "cuda", torch.float32)
            xs.append(x.contiguous())
            ys.append(y.contiguous())
        ring.append((xs, ys, sg.BatchSolver.pointers(xs, "cuda"),
                     sg.BatchSolver.pointers(ys, "cuda")))
    torch.cuda.synchronize()
    cfg = sg.make_config(sg.SGEP_KIND_GENERAL, sg.SGEP_F32, k, 0, 0, b,
                         optimizer=sg.SGEP_ADAM if w["optimizer"] == "adam" else sg.SGEP_SGD,
                         schedule=sg.SGEP_SCHED_INV, eta0=w["eta0"], t0=w["t0"],
                         gamma=w["gamma"], rho=w["rho"], eps_reg=w["eps_reg"])
    stream = torch.cuda.Stream()
    V0s = [synth.initial_players(d, k, 1000 + i) for i, d in enumerate(dims)]
    bat = sg.BatchSolver(dims, cfg, V0s, stream=stream)
    if args.batch_plan:
        g_, *mb_ = [int(x) for x in args.batch_plan.split(",")]
        bat.set_plan(g_, mb_)
        plan_src = "set"
    else:
        tune_us = bat.tune(ring[0][2], ring[0][3], b, reps=3)
        plan_src = f"autotuned ({tune_us:.1f} us per iteration)"
    groups, mb = bat.plan()
    print(f"bench: plan groups={groups} tile heights={mb}, {plan_src}", file=sys.stderr, flush=True)

    def step(t):
        bat.step(ring[t % R][2], ring[t % R][3], b)

    with torch.cuda.stream(stream):
        for t in range(W):
            step(t)
    torch.cuda.synchronize()
    chunk = min(K, R)
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g, stream=stream):
        for t in range(chunk):
            step(t)
    torch.cuda.synchronize()
    n_rep, rem = divmod(K, chunk)
    if args.calibrate_copy_mb:
        calibration_copy(args.calibrate_copy_mb)
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
    value = n * b / (ms_per_step * 1e-3)

    # per-launch durations (events stamped by each kernel's dispatch)
    kinds = bat.launches()
    hip = hip_runtime()
    Kp = min(K, 64)
    ne = 2 * len(kinds)
    evs = [ctypes.c_void_p() for _ in range(ne * Kp)]
    for e in evs:
        assert hip.hipEventCreate(ctypes.byref(e)) == 0
    torch.cuda.synchronize()
    for t in range(Kp):
        sg.sgep_batch_step_profiled(bat.bt, ring[t % R][2], ring[t % R][3], b,
                                    [evs[ne * t + i].value for i in range(ne)])
    torch.cuda.synchronize()
    ms = ctypes.c_float()
    fwd_us, coef_us, bwd_us, pers_us = [], [], [], []
    for t in range(Kp):
        f = cc = bb = pp = 0.0
        for i, kd in enumerate(kinds):
            assert hip.hipEventElapsedTime(ctypes.byref(ms), evs[ne * t + 2 * i],
                                           evs[ne * t + 2 * i + 1]) == 0
            if kd == 0:
                f += ms.value * 1e3
            elif kd == -2:
                pp += ms.value * 1e3
            elif kd < 0:
                cc += ms.value * 1e3
            else:
                bb += ms.value * 1e3
        fwd_us.append(f)
        coef_us.append(cc)
        bwd_us.append(bb)
        pers_us.append(pp)
    for e in evs:
        hip.hipEventDestroy(e)
    bat.sync()
    # algorithmic HBM bytes: one read of both minibatch views of every
    # instance, plus the FP32 state each kernel must touch
    D = float(sum(dims))
    adam = w["optimizer"] == "adam"
    data = 2.0 * b * D * 4
    fwd_bytes = data + 4 * D * 16 + 2 * 4 * b * 16 * n          # X, Y; V (KP = 16); P, Q out
    bwd_bytes = data + (4 + (4 if adam else 0)) * 4 * D * 16 + 2 * 4 * b * 16 * n
    step_bytes = data + (4 + (4 if adam else 0)) * 4 * D * k
    # the persistent launch: one read of the minibatch, V, the state read and
    # written, P and Q written and read back
    pers_bytes = (data + 4 * D * 16 + (4 + (4 if adam else 0)) * 4 * D * 16
                  + 2 * 2 * 4 * b * 16 * n)
    avg_f, avg_b, avg_p = (float(np.mean(fwd_us)), float(np.mean(bwd_us)),
                           float(np.mean(pers_us)))
    if avg_p > 0:
        dom, dom_us, dom_bytes = "k_bpers", avg_p, pers_bytes
    else:
        dom, dom_us, dom_bytes = ("k_bbwd", avg_b, bwd_bytes) if avg_b >= avg_f else (
            "k_bfwd", avg_f, fwd_bytes)
    achieved = dom_bytes / (dom_us * 1e-6) / 1e9
    roofline = {"bound": "hbm", "achieved": round(achieved, 1), "peak": PEAK_HBM_GBS,
                "unit": "GB/s", "frac": round(achieved / PEAK_HBM_GBS, 5),
                "traffic": measured_traffic(args.workload, dom),
                "kernel": dom, "kernel_avg_us": round(dom_us, 3),
                "kernel_note": "sum over the step's launches of this kernel",
                "kernels_avg_us": ({"k_bpers": round(avg_p, 3)} if avg_p > 0 else
                                   {"k_bfwd": round(avg_f, 3),
                                    "k_bcoef": round(float(np.mean(coef_us)), 3),
                                    "k_bbwd": round(avg_b, 3)}),
                "algorithmic_hbm_bytes_per_launch": dom_bytes,
                "step_algorithmic_hbm_bytes": step_bytes,
                "step_hbm_frac": round(step_bytes / (ms_per_step * 1e-3) / 1e9 / PEAK_HBM_GBS, 5)}
    out = {
        "metric": "samples/s per gamma-EigenGame step",
        "value": round(value, 1),
        "unit": "instance-samples/s",
        "n_gpus": 1,
        "steps": K,
        "warmup": W,
        "ms_per_step": round(ms_per_step, 6),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": f"synthetic: ring of {R} minibatches per instance drawn on the device",
        "config": {"workload": args.workload, "description": w["describe"], "instances": n,
                   "sum_d": int(D), "k": k, "minibatch": b, "optimizer": w["optimizer"],
                   "plan": {"groups": groups, "tile_heights": mb, "launches": len(kinds),
                            "source": plan_src},
                   "graph_steps": chunk, "parallelism": "single GPU"},
        "roofline": roofline,
    }
    bat.close()
    if "tta" in w and not args.no_tta:
        tt = w["tta"]
        mx = args.tta_steps if args.tta_steps is not None else tt["max_steps"]
        print(f"bench: time to subspace error {tt['targets']} (every instance)", file=sys.stderr,
              flush=True)
        out["time_to_accuracy"] = batch_time_to_accuracy(
            w, gens, dims, cfg, (groups, mb), tt["targets"], mx, tt["every"], tt["chunk"],
            log=lambda m: print("bench: " + m, file=sys.stderr, flush=True))
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline_batch(w, gens, dims, V0s, ring, args.cpu_budget)
    print(json.dumps(out), flush=True)


def batch_time_to_accuracy(w, gens, dims, cfg, plan, targets, max_steps, every, E, log=None):
    """Time to each subspace error in `targets` for the many-instance
    workload, reached by every instance (the worst of the n errors), by the
    rule of time_to_accuracy: summed step time (HIP events around hipGraph
    replays of E batched iterations) up to the first evaluation at or below
    the target whose next evaluation also is.  Fresh minibatches of every
    instance are drawn on the device between replays (outside the timed
    region); the target of instance i is its planted solution
    V* = Qx diag(ax + eps)^-1/2 O[:, top k] (the closed form of
    oracle.targets.general_planted_topk for the fast mixing), graded with the
    oracle's normalised subspace error under B = Qx diag(ax + eps) Qx^T."""
    import torch
    import oracle
    import paper_2206_04993_amd as sg
    import synth

    n, k, b = len(gens), w["k"], w["b"]
    targets = sorted(targets, reverse=True)
    Vs, Bops = [], []
    for g in gens:
        Q = g._fx.dense()
        order = np.argsort(-g.lam)[:k]
        s = g.ax + g.eps
        Vs.append(Q @ (g._fo.dense()[:, order] / np.sqrt(s)[:, None]))
        Bops.append(lambda M, Q=Q, s=s: Q @ (s[:, None] * (Q.T @ M)))
    tables = [g.device_tables("cuda") for g in gens]
    xs = [torch.empty((E, b, d), device="cuda", dtype=torch.float32) for d in dims]
    ys = [torch.empty((E, b, d), device="cuda", dtype=torch.float32) for d in dims]

    def fill(c):
        for i, g in enumerate(gens):
            x, y = g.sample_torch(E * b, 2_000_000 + c, "cuda", torch.float32, tables=tables[i])
            xs[i].copy_(x.view(E, b, -1))
            ys[i].copy_(y.view(E, b, -1))

    ptrs = [(sg.BatchSolver.pointers([x[j] for x in xs], "cuda"),
             sg.BatchSolver.pointers([y[j] for y in ys], "cuda")) for j in range(E)]
    stream = torch.cuda.Stream()
    V0s = [synth.initial_players(d, k, 1000 + i) for i, d in enumerate(dims)]
    bat = sg.BatchSolver(dims, cfg, V0s, stream=stream)
    bat.set_plan(plan[0], plan[1])
    fill(0)
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g, stream=stream):
        for j in range(E):
            bat.step(ptrs[j][0], ptrs[j][1], b)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    t_gpu, steps, hist, hits, c = 0.0, 0, [], {}, 0
    while steps < max_steps:
        if c > 0:
            fill(c)
            torch.cuda.synchronize()
        with torch.cuda.stream(stream):
            e0.record(stream)
            g.replay()
            e1.record(stream)
        e1.synchronize()
        t_gpu += e0.elapsed_time(e1) * 1e-3
        steps += E
        c += 1
        if steps % every:
            continue
        errs = [oracle.subspace_containment_error(bat.vectors(i), Vs[i], Bops[i])
                for i in range(n)]
        worst = float(max(errs))
        hist.append((steps, t_gpu, worst, float(np.median(errs))))
        if log:
            log(f"tta batch steps {steps} gpu {t_gpu:.3f}s worst {worst:.3e} "
                f"median {hist[-1][3]:.3e}")
        for tg in targets:
            if tg not in hits and len(hist) >= 2 and hist[-2][2] <= tg and worst <= tg:
                hits[tg] = hist[-2]
        if targets[-1] in hits:
            break
    bat.close()
    res = {"targets": {}, "eval_every_steps": every, "graded": "every instance (worst error)",
           "reference": "planted solution of each instance (closed form)",
           "stream": "fresh device-drawn minibatches of every instance",
           "max_steps": max_steps, "steps_run": steps, "gpu_seconds_run": round(t_gpu, 4),
           "final_worst_error": hist[-1][2] if hist else None,
           "final_median_error": hist[-1][3] if hist else None,
           "trajectory": [(h[0], round(h[1], 4), h[2], h[3]) for h in hist]}
    for tg in targets:
        h = hits.get(tg)
        res["targets"][f"{tg:g}"] = ({"reached": True, "seconds": round(h[1], 4), "steps": h[0],
                                      "instance_samples": h[0] * b * n} if h else {"reached": False})
    return res


def cpu_baseline_batch(w, gens, dims, V0s, ring, budget_s):
    """The FP64 oracle on the many-instance workload: whole iterations over
    every instance (the values the GPU received) until budget_s is spent."""
    import oracle
    pbs = {}
    states = [oracle.State.init(V0, adam=w["optimizer"] == "adam") for V0 in V0s]
    host = [[(x.double().cpu().numpy(), y.double().cpu().numpy()) for x, y in zip(r[0], r[1])]
            for r in ring]
    n_it = 0
    t0 = time.perf_counter()
    while True:
        eta = oracle.eta(oracle.SCHED_INV, n_it + 1, w["eta0"], t0=w["t0"])
        for i, d in enumerate(dims):
            pb = pbs.get(d)
            if pb is None:
                pb = pbs[d] = oracle.Problem(
                    oracle.KIND_GENERAL, w["k"], d, d, rho=w["rho"], eps_reg=w["eps_reg"],
                    optimizer=oracle.OPT_ADAM if w["optimizer"] == "adam" else oracle.OPT_SGD)
            X, Y = host[n_it % len(host)][i]
            oracle.gamma_step(pb, states[i], X, Y, eta, w["gamma"])
        n_it += 1
        el = time.perf_counter() - t0
        if el >= budget_s:
            break
    n = len(dims)
    return {"value": n_it * n * w["b"] / el, "unit": "instance-samples/s",
            "cores": min(oracle.threads(), w["k"]), "kind": "oracle",
            "omp_threads": oracle.threads(), **host_info(),
            "parallelism": "OpenMP over the k players of each instance",
            "sample": f"{n_it} whole iteration(s) of all {n} instances ({n_it * n * w['b']} "
                      f"instance-samples) on the values the GPU received, FP64 oracle, "
                      f"{el:.1f} s wall"}


def host_info():
    """The host's CPU model and logical core count."""
    model = None
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                model = line.split(":", 1)[1].strip()
                break
    except OSError:
        pass
    return {"nproc": os.cpu_count(), "cpu_model": model}


def measure_hbm_stream():
    """Achievable HBM bandwidth on this GPU, measured with torch's own
    kernels on 4 GiB: a device copy (bytes read + written) and a full
    reduction (bytes read); the larger of the two rates."""
    import torch
    n = 1 << 30
    x = torch.ones(n, device="cuda", dtype=torch.float32)
    y = torch.empty_like(x)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    best = {}
    for name, fn, nbytes in (("copy", lambda: y.copy_(x), 8.0 * n),
                             ("sum", lambda: x.sum(), 4.0 * n)):
        fn()
        torch.cuda.synchronize()
        e0.record()
        for _ in range(5):
            fn()
        e1.record()
        e1.synchronize()
        best[name] = nbytes * 5 / (e0.elapsed_time(e1) * 1e-3) / 1e9
    del x, y
    torch.cuda.empty_cache()
    return {"GB_per_s": round(max(best.values()), 1),
            "by_kernel_GB_per_s": {k: round(v, 1) for k, v in best.items()},
            "method": "torch device copy (read + write bytes) and full sum (read bytes) of 4 GiB"}


def measure(args, wname, w, K, W, hbm_meas=None):
    """Throughput of one single-handle workload: value, step time, per-kernel
    durations and the roofline of the dominant kernel.  Returns (record,
    host sample of the first minibatches for the CPU baseline)."""
    import torch
    import paper_2206_04993_amd as sg
    import synth

    R = w["ring"]
    lda = w["kind"] == "lda"
    d, k, b = w["dx"] + w["dy"], w["k"], w["b"]

    # ---- the ring of minibatches, resident in HBM ----
    print(f"bench: generating {R} minibatches of {wname}", file=sys.stderr, flush=True)
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
        elif Yr is None:  # one stream (ICA)
            ty, vy = None, None
        else:
            ty, vy = encode(w, Yr, scales[1] if scales else None)
        Xs.append(tx)
        Ys.append(ty)
        if i < 3:
            host.append((vx, vy))
    del raw
    X = torch.stack(Xs).to("cuda").contiguous()
    Y = torch.stack(Ys).to("cuda").contiguous() if Ys[0] is not None else [None] * R
    del Xs, Ys
    torch.cuda.synchronize()
    stream = torch.cuda.Stream()
    solver = sg.Solver(config_for(sg, w), synth.initial_players(d, k, 0), stream=stream, **aux)
    nk = solver.kernels_per_step()
    names = solver.kernel_names()

    def step(t):
        s_ = t % R
        solver.step(X[s_], Y[s_])

    with torch.cuda.stream(stream):
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
        calibration_copy(args.calibrate_copy_mb)

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
    del g

    # ---- per-kernel durations: the same steps again, each kernel launched
    # with a start/stop HIP event pair stamped by its own dispatch, on the
    # solver's stream ----
    hip = hip_runtime()
    Kp = min(K, 512)
    evs = [ctypes.c_void_p() for _ in range(2 * nk * Kp)]
    for e in evs:
        assert hip.hipEventCreate(ctypes.byref(e)) == 0
    torch.cuda.synchronize()
    for t in range(Kp):
        s_ = t % R
        ev = [evs[2 * nk * t + i].value for i in range(2 * nk)]
        if lda:
            sg.sgep_step_profiled(solver.h, X[s_], X[s_].stride(0), None, 0, Y[s_], b, ev)
        elif Y[s_] is None:
            sg.sgep_step_profiled(solver.h, X[s_], X[s_].stride(0), None, 0, None, b, ev)
        else:
            sg.sgep_step_profiled(solver.h, X[s_], X[s_].stride(0), Y[s_], Y[s_].stride(0), None,
                                  b, ev)
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
    solver.close()
    del X, Y
    torch.cuda.empty_cache()
    avg = {n: float(np.mean(v)) for n, v in dur.items()}
    dom = max(avg, key=avg.get)
    flops, nbytes = algorithmic_work(w, dom, names)
    if w["dtype"] in ("bf16", "fp8") or flops == 0.0:
        achieved = nbytes / (avg[dom] * 1e-6) / 1e9
        roofline = {"bound": "hbm", "achieved": round(achieved, 1), "peak": PEAK_HBM_GBS,
                    "unit": "GB/s", "frac": round(achieved / PEAK_HBM_GBS, 5)}
        if hbm_meas:
            roofline["measured_peak"] = hbm_meas["GB_per_s"]
            roofline["frac_of_measured_peak"] = round(achieved / hbm_meas["GB_per_s"], 5)
    else:
        peak = PEAK_FP32_MFMA_TFLOPS if w["dtype"] == "f32" else PEAK_FP64_MFMA_TFLOPS
        achieved = flops / (avg[dom] * 1e-6) / 1e12
        roofline = {"bound": "mfma", "achieved": round(achieved, 3), "peak": peak,
                    "unit": "TFLOP/s", "frac": round(achieved / peak, 5)}
    # the whole step against the roofline of its algorithmic work (the sum
    # over its kernels)
    step_flops = sum(algorithmic_work(w, n, names)[0] for n in names)
    step_bytes = step_work_bytes(w)
    roofline.update({
        "traffic": measured_traffic(wname, dom),
        "kernel": dom, "kernel_avg_us": round(avg[dom], 3),
        "kernels_avg_us": {n: round(v, 3) for n, v in avg.items()},
        "algorithmic_flops_per_launch": flops,
        "algorithmic_hbm_bytes_per_launch": nbytes,
        "step_algorithmic_flops": step_flops,
        "step_algorithmic_hbm_bytes": step_bytes,
        "step_tflops": round(step_flops / (ms_per_step * 1e-3) / 1e12, 3),
        "step_hbm_GB_per_s": round(step_bytes / (ms_per_step * 1e-3) / 1e9, 1),
    })
    rec = {"value": round(value, 1), "unit": "samples/s", "steps": K, "warmup": W,
           "ms_per_step": round(ms_per_step, 6), "dtype": w["dtype"],
           "data": f"synthetic: ring of {R} pre-generated minibatches resident in HBM",
           "config": {"workload": wname, "description": w["describe"], "d": d, "k": k,
                      "minibatch": b, "optimizer": w["optimizer"], "graph_steps": chunk,
                      "parallelism": "single GPU"},
           "roofline": roofline}
    return rec, host


def step_work_bytes(w):
    """Algorithmic HBM bytes of one whole step: one read of the minibatch
    (LDA: and its labels) plus the FP32 (FP64) state read and written once."""
    b, k = w["b"], w["k"]
    d = w["dx"] + w["dy"]
    e = {"f64": 8, "f32": 4, "bf16": 2, "fp8": 1}[w["dtype"]]
    se = 8 if w["dtype"] == "f64" else 4
    mult = (2 if w["kind"] == "general" else 1)
    data = mult * b * d * e + (4 * b if w["kind"] == "lda" else 0)
    return float(data + (4 + (4 if w["optimizer"] == "adam" else 0)) * se * d * k)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=None, help="timed steps (default per workload)")
    ap.add_argument("--warmup", type=int, default=None)
    ap.add_argument("--workload", default=DEFAULT, choices=sorted(WORKLOADS) +
                    sorted(BATCH_WORKLOADS))
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-tta", action="store_true", help="skip the time-to-accuracy run")
    ap.add_argument("--no-twin", action="store_true",
                    help="skip the FP32 reference of a reduced-precision workload")
    ap.add_argument("--tta-only", action="store_true",
                    help="run only the time-to-accuracy leg of --workload (no throughput, twin "
                         "or CPU baseline) and print its record with the error trajectory")
    ap.add_argument("--tta-steps", type=int, default=None,
                    help="step limit of each time-to-accuracy run (default per workload)")
    ap.add_argument("--batch-plan", default="",
                    help="batched workloads: 'groups,mb0,mb1,mb2' instead of autotuning")
    ap.add_argument("--cpu-budget", type=float, default=15.0)
    ap.add_argument("--calibrate-copy-mb", type=int, default=0,
                    help="also run a plain device copy of this many MiB (counter calibration)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py: measures one GPU only (asked for --gpus {args.gpus}); the step has "
              "no multi-GPU path.", file=sys.stderr)
        sys.exit(2)

    import torch
    import paper_2206_04993_amd as sg

    sg.load()
    assert torch.cuda.is_available(), "bench.py needs a GPU"
    if args.workload in BATCH_WORKLOADS:
        run_batch(args, BATCH_WORKLOADS[args.workload])
        return
    w = WORKLOADS[args.workload]
    if args.tta_only:
        tt = w["tta"]
        mx = args.tta_steps if args.tta_steps is not None else tt["max_steps"]
        log = (lambda m: print("bench: " + m, file=sys.stderr, flush=True))
        res = time_to_accuracy(w, tt["targets"], mx, tt["every"], log=log)
        print(json.dumps({"workload": args.workload, "dtype": w["dtype"],
                          "config": {kk: w[kk] for kk in sorted(w)
                                     if kk not in ("tta", "twin", "describe")},
                          "time_to_accuracy": res}), flush=True)
        return
    big = w["b"] * (w["dx"] + w["dy"]) > 1 << 24
    K = args.steps if args.steps is not None else (256 if big else 2048)
    W = args.warmup if args.warmup is not None else (8 if big else 64)
    # (not in counter runs: its large copies would be taken for the calibration copy)
    hbm_meas = (measure_hbm_stream() if w["dtype"] in ("bf16", "fp8")
                and not args.calibrate_copy_mb else None)
    rec, host = measure(args, args.workload, w, K, W, hbm_meas)
    out = {"metric": "samples/s per gamma-EigenGame step", "value": rec["value"],
           "unit": "samples/s", "n_gpus": 1, "steps": K, "warmup": W,
           "ms_per_step": rec["ms_per_step"], "higher_is_better": True, "scaling": "weak",
           "vs_baseline": None, "dtype": w["dtype"], "data": rec["data"],
           "config": rec["config"], "roofline": rec["roofline"]}
    if hbm_meas:
        out["hbm_stream_measured"] = hbm_meas
    twin = w.get("twin")
    if twin and not args.no_twin:
        # the same problem with FP32 minibatches: throughput beside the value
        tw = WORKLOADS[twin]
        trec, _ = measure(args, twin, tw, K, W)
        out["fp32_reference"] = {key: trec[key] for key in
                                 ("value", "unit", "ms_per_step", "dtype", "config", "roofline")}
        out["fp32_reference"]["speedup_of_value"] = round(rec["value"] / trec["value"], 3)
    if "tta" in w and not args.no_tta:
        tt = w["tta"]
        mx = args.tta_steps if args.tta_steps is not None else tt["max_steps"]
        log = (lambda m: print("bench: " + m, file=sys.stderr, flush=True))
        print(f"bench: time to subspace error {tt['targets']}", file=sys.stderr, flush=True)
        res = {w["dtype"]: time_to_accuracy(w, tt["targets"], mx, tt["every"], log=log)}
        if twin and not args.no_twin:
            res[WORKLOADS[twin]["dtype"]] = time_to_accuracy(WORKLOADS[twin], tt["targets"], mx,
                                                             tt["every"], log=log)
            out["time_to_accuracy"] = res
        else:
            out["time_to_accuracy"] = res[w["dtype"]]
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(w, args.cpu_budget, host)
        tta = out.get("time_to_accuracy")
        if tta:
            # the oracle follows the same iteration: its time per step times
            # the GPU's step count (an extrapolation, not a run to target)
            first = tta.get(w["dtype"], tta)
            sps = out["cpu_baseline"]["value"] / w["b"]
            out["cpu_baseline"]["time_to_accuracy_extrapolated_s"] = {
                tg: round(h["steps"] / sps, 3) for tg, h in first["targets"].items()
                if h["reached"]}
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
