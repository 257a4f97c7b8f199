"""GPU parity of the BF16 / FP8 path (CCA and LDA) against the FP64 oracle,
through the C ABI.

The oracle is fed the exact values the GPU receives: BF16 inputs decoded to
float64, FP8 codes times their column scales (exact in float64).  The
difference that remains is the GPU's own arithmetic: the FP32 right-hand
operands (players V, projections P and Q) are split into BF16 hi + lo (16
significand bits, relative error <= 2^-17 per element), products accumulate
in FP32, the state is FP32: the FP32 path's error budget with the operand
rounding 2^-24 replaced by about 2^-17 on one factor.  Bars (TOLW_1 after
one iteration, TOLW_N after N) are 5-20x the differences observed with plain
ascent; with Adam (TOLW_ADAM_1, TOLW_ADAM_N) the renormalisation spreads the
steps of rounding-level-gradient elements, which may go either way, over
their column.  Sizes span several 64-feature subtiles, several forward
splits and ragged row blocks."""
import ctypes

import numpy as np
import pytest

import oracle
import synth
from parity_bars import assert_players_close

pytestmark = pytest.mark.gpu

# BF16 / FP8 minibatches (the FP32 operands enter the MFMA as BF16 hi + lo):
# about 5-20x the largest plain-ascent differences observed on MI355X
# (players 1.8e-6, relative [Bv] 1.1e-5); with Adam, elements of
# rounding-level gradient may step either way (tests/parity_bars.py)
TOLW_1 = 5e-5
TOLW_N = 2e-4
TOLW_ADAM_1 = 8e-5   # Adam: observed up to 6e-5 after one iteration
TOLW_ADAM_N = 1.2e-3  # and 2.4e-4 ([Bv]) after 40


def _torch():
    import torch
    return torch


def _sg():
    import paper_2206_04993_amd as sg
    sg.load()
    return sg


def _bf16_dev(bits):
    torch = _torch()
    t = torch.from_numpy(np.ascontiguousarray(bits).view(np.int16))
    return t.to("cuda").view(torch.bfloat16).contiguous()


def _u8_dev(codes):
    torch = _torch()
    return torch.from_numpy(np.ascontiguousarray(codes, dtype=np.uint8)).to("cuda").contiguous()


def _i32_dev(lab):
    torch = _torch()
    return torch.from_numpy(np.ascontiguousarray(lab, dtype=np.int32)).to("cuda").contiguous()


def _maxdiff(a, b):
    return float(np.abs(np.asarray(a) - np.asarray(b)).max())


def _cca_inputs(gen, n, b, fmt, scales=None):
    """Minibatches as (device X, device Y, float64 X, float64 Y) in the given
    storage format."""
    out = []
    for t in range(1, n + 1):
        X, Y = gen.batch(t, b)
        if fmt == "bf16":
            bx, by = synth.bf16_bits(X), synth.bf16_bits(Y)
            out.append((_bf16_dev(bx), _bf16_dev(by), synth.bf16_value(bx), synth.bf16_value(by)))
        else:
            sx, sy = scales
            cx, cy = synth.fp8_quantize(X, sx), synth.fp8_quantize(Y, sy)
            out.append((_u8_dev(cx), _u8_dev(cy), synth.fp8_dequantize(cx, sx),
                        synth.fp8_dequantize(cy, sy)))
    return out


def _eta(cfg, t):
    return oracle.eta(cfg.schedule, t, cfg.eta0, eta_T=cfg.eta_T, t0=cfg.t0, t_c=cfg.t_c, T=cfg.T)


def _run_cca(cfg, batches, V0, checkpoints, aux=None):
    sg = _sg()
    s = sg.Solver(cfg, V0, **(aux or {}))
    pb = oracle.Problem(oracle.KIND_CCA, cfg.k, cfg.dx, cfg.dy, rho=cfg.rho,
                        optimizer=cfg.optimizer, adam_b1=cfg.adam_b1, adam_b2=cfg.adam_b2,
                        adam_eps=cfg.adam_eps)
    st = oracle.State.init(V0, adam=cfg.optimizer == sg.SGEP_ADAM)
    res = []
    for t, (Xd, Yd, X, Y) in enumerate(batches, start=1):
        s.step(Xd, Yd)
        oracle.gamma_step(pb, st, X, Y, _eta(cfg, t), cfg.gamma)
        if t in checkpoints:
            snap = oracle.State(V=st.V.copy(), G=st.G.copy(), t=st.t,
                                s2=None if st.s2 is None else st.s2.copy())
            res.append((t, s.vectors(), snap, s.auxiliary(), st.G.copy(), s.eigvals(),
                        st.eigvals()))
    s.close()
    return res


@pytest.mark.parametrize("fmt,dx,dy,k,b,opt", [
    ("bf16", 200, 136, 13, 100, "sgd"),     # ragged rows, 4 + 3 subtiles, KP 16
    ("bf16", 520, 264, 32, 130, "adam"),    # KP 32, several forward splits
    ("bf16", 64, 64, 1, 1, "sgd"),          # one player, one row
    ("fp8", 200, 136, 13, 100, "sgd"),
    ("fp8", 520, 264, 32, 130, "adam"),
    # views wide enough for the split backward (128-feature products, then
    # the epilogue per 64-feature tile); ragged last subtile of view x
    ("bf16", 16392, 16384, 20, 300, "sgd"),  # with the four-wave forward (b >= 256)
    ("fp8", 16392, 16384, 20, 64, "adam"),
    ("fp8", 520, 264, 32, 300, "adam"),       # four-wave forward, KP 32, FP8 codes
    # 512-row forward workgroups sharing V through LDS at KP 32 (b >= 1024), ragged rows
    ("bf16", 520, 264, 32, 1100, "adam"),
    ("bf16", 4104, 2056, 20, 1030, "sgd"),
    ("fp8", 520, 264, 32, 1100, "sgd"),
    ("fp8", 4104, 2056, 20, 1030, "adam"),
])
def test_wide_cca_parity(fmt, dx, dy, k, b, opt):
    sg = _sg()
    print(f"wide CCA {fmt} dx={dx} dy={dy} k={k} b={b} {opt}", flush=True)
    gen = synth.CCAPlanted(dx, dy, np.linspace(0.9, 0.3, min(k, 6)), sigma=0.5, seed=3)
    dtype = sg.SGEP_BF16 if fmt == "bf16" else sg.SGEP_FP8_E4M3
    adam = opt == "adam"
    cfg = sg.make_config(sg.SGEP_KIND_CCA, dtype, k, dx, dy, b,
                         optimizer=sg.SGEP_ADAM if adam else sg.SGEP_SGD,
                         schedule=sg.SGEP_SCHED_INV, eta0=2e-3 if adam else 0.05, t0=100.0,
                         gamma=0.5, rho=1e-6)
    aux, scales = None, None
    if fmt == "fp8":
        Xc, Yc = gen.sample(4096, np.random.default_rng([3, 99]))
        scales = (synth.fp8_column_scales(Xc), synth.fp8_column_scales(Yc))
        aux = dict(x_col_scale=scales[0], y_col_scale=scales[1])
    N = 40
    batches = _cca_inputs(gen, N, b, fmt, scales)
    V0 = synth.initial_players(dx + dy, k, 4)
    res = _run_cca(cfg, batches, V0, {1, N}, aux)
    for t, Vg, so, Gg, Go, lg, lo in res:
        tol = (TOLW_ADAM_1 if t == 1 else TOLW_ADAM_N) if adam else (TOLW_1 if t == 1 else TOLW_N)
        dv, dg = _maxdiff(Vg, so.V), _maxdiff(Gg, Go)
        print(f"  t={t}: max|dV|={dv:.2e} max|dG|={dg:.2e}", flush=True)
        assert_players_close(Vg, so, tol, adam, sum(_eta(cfg, i) for i in range(1, t + 1)))
        assert dg < tol, (t, dg)
        assert np.allclose(lg, lo, rtol=10 * tol, atol=10 * tol), (t, lg, lo)
        # unit players (Alg. 2 output)
        assert np.allclose((Vg * Vg).sum(axis=0), 1.0, atol=1e-5)


def _lda_problem(d, c, k, seed=5):
    gen = synth.LDAClasses(d=d, c=c, r=min(16, d), seed=seed)
    priors = np.full(c, 1.0 / c)
    return gen, priors


# FP32 minibatches on the large-d path: FP32 operands and FP32 MFMA (observed
# at most 4.2e-6 after one iteration, with Adam, and 4.1e-6 after 30)
TOLF_1 = 2e-5
TOLF_N = 5e-5


@pytest.mark.parametrize("fmt", ["bf16", "f32"])
@pytest.mark.parametrize("d,c,k,b,opt", [
    (200, 10, 9, 300, "sgd"),     # KP 16, 4 subtiles, ragged rows
    (520, 6, 20, 130, "adam"),    # KP 32
    (136, 10, 64, 77, "sgd"),     # KP 64, k > classes (zero eigenvalues beyond c - 1)
    (4104, 5, 40, 200, "adam"),   # KP 64, several forward slices, ragged last subtile
    (32776, 5, 40, 300, "adam"),  # BF16: four-wave forward, split backward, ragged subtile
    (4104, 5, 40, 300, "sgd"),    # BF16: four-wave forward (128 rows per wave at KP 64)
    # BF16: 512-row forward workgroups sharing V through LDS (b >= 1024), ragged
    # last row block; with the split backward at the wider view
    (4104, 5, 40, 1100, "sgd"),
    (32776, 5, 40, 1030, "adam"),
])
def test_wide_lda_parity(d, c, k, b, opt, fmt):
    sg = _sg()
    torch = _torch()
    print(f"wide LDA {fmt} d={d} c={c} k={k} b={b} {opt}", flush=True)
    gen, priors = _lda_problem(d, c, k)
    adam = opt == "adam"
    eps = 1e-3
    dt = sg.SGEP_BF16 if fmt == "bf16" else sg.SGEP_F32
    tol1, tolN = (TOLW_1, TOLW_N) if fmt == "bf16" else (TOLF_1, TOLF_N)
    if adam and fmt == "bf16":
        tol1, tolN = TOLW_ADAM_1, TOLW_ADAM_N
    cfg = sg.make_config(sg.SGEP_KIND_LDA, dt, k, d, 0, b,
                         optimizer=sg.SGEP_ADAM if adam else sg.SGEP_SGD,
                         schedule=sg.SGEP_SCHED_INV, eta0=1e-3 if adam else 0.01, t0=100.0,
                         gamma=0.5, rho=1e-6, eps_reg=eps, n_classes=c)
    V0 = synth.initial_players(d, k, 6)
    s = sg.Solver(cfg, V0, class_means=gen.means, class_priors=priors)
    pb = oracle.Problem(oracle.KIND_LDA, k, d, 0, eps_reg=eps, rho=1e-6, optimizer=cfg.optimizer,
                        class_means=gen.means, class_priors=priors)
    st = oracle.State.init(V0, adam=adam)
    N = 30
    for t in range(1, N + 1):
        X, lab = gen.batch(t, b)
        if fmt == "bf16":
            bits = synth.bf16_bits(X)
            s.step(_bf16_dev(bits), _i32_dev(lab))
            Xo = synth.bf16_value(bits)
        else:
            X32 = np.ascontiguousarray(X, dtype=np.float32)
            s.step(torch.from_numpy(X32).cuda(), _i32_dev(lab))
            Xo = X32.astype(np.float64)
        oracle.gamma_step(pb, st, Xo, None, _eta(cfg, t), cfg.gamma, labels=lab)
        if t in (1, N):
            tol = tol1 if t == 1 else tolN
            Vg, Gg = s.vectors(), s.auxiliary()
            # players beyond the rank c - 1 of the between-class A have no
            # signal (eigenvalue 0): both sides follow the same dynamics, which
            # amplifies rounding-level differences (1e-8 -> 1e-3 over 30 steps
            # observed), so after the first iteration only the leading c - 1
            # players are compared element by element
            m = k if t == 1 else min(k, c - 1)
            sv = oracle.State(V=st.V[:, :m], G=st.G[:, :m], t=st.t,
                              s2=None if st.s2 is None else st.s2[:, :m])
            dv, dg = _maxdiff(Vg[:, :m], sv.V), _maxdiff(Gg[:, :m], sv.G)
            print(f"  t={t}: players 0..{m - 1}: max|dV|={dv:.2e} max|dG|={dg:.2e}", flush=True)
            assert_players_close(Vg[:, :m], sv, tol, adam,
                                 sum(_eta(cfg, i) for i in range(1, t + 1)))
            assert dg < tol * max(1.0, float(np.abs(sv.G).max())), (t, dg)
            lg, lo = s.eigvals()[:m], st.eigvals()[:m]
            assert np.allclose(lg, lo, rtol=10 * tol, atol=10 * tol), (t, lg, lo)
            assert np.all(np.isfinite(Vg)) and np.allclose(np.linalg.norm(Vg, axis=0), 1.0,
                                                           atol=1e-5)
    s.close()


@pytest.mark.parametrize("dx,dy", [(136, 72), (16392, 16384)])
def test_wide_determinism_resume_and_graph(dx, dy):
    """Bitwise-identical reruns, checkpoint / resume in a fresh handle, and
    hipGraph replay equal to eager steps (BF16 CCA with Adam; one backward
    kernel, and the split backward at the wider views)."""
    torch = _torch()
    sg = _sg()
    gen = synth.CCAPlanted(dx, dy, np.linspace(0.9, 0.3, 4), sigma=0.5, seed=8)
    cfg = sg.make_config(sg.SGEP_KIND_CCA, sg.SGEP_BF16, 8, dx, dy, 96,
                         optimizer=sg.SGEP_ADAM, eta0=1e-3, gamma=0.3)
    batches = _cca_inputs(gen, 8, 96, "bf16")
    V0 = synth.initial_players(dx + dy, 8, 1)
    probe = sg.Solver(cfg, V0)
    nk = probe.kernels_per_step()
    probe.close()
    assert nk == (4 if dx > 10_000 else 3)

    def run(bs, solver=None):
        s = solver or sg.Solver(cfg, V0)
        for Xd, Yd, _, _ in bs:
            s.step(Xd, Yd)
        return s

    a, b = run(batches), run(batches)
    assert np.array_equal(a.vectors(), b.vectors())
    assert np.array_equal(a.auxiliary(), b.auxiliary())
    c = run(batches[:4])
    blob = c.get_state()
    d = sg.Solver(cfg, synth.initial_players(dx + dy, 8, 7))
    d.set_state(blob)
    assert d.step_count() == 4
    run(batches[4:], solver=d)
    assert np.array_equal(a.vectors(), d.vectors())
    assert np.array_equal(a.eigvals(), d.eigvals())
    # graph: the same 8 steps captured once, replayed twice, against eager
    stream = torch.cuda.Stream()
    g_s = sg.Solver(cfg, V0, stream=stream)
    e_s = sg.Solver(cfg, V0)
    graph = torch.cuda.CUDAGraph()
    torch.cuda.synchronize()
    with torch.cuda.graph(graph, stream=stream):
        for Xd, Yd, _, _ in batches:
            g_s.step(Xd, Yd)
    for rep in range(2):
        run(batches, solver=e_s)
        e_s.sync()
        graph.replay()
        torch.cuda.synchronize()
        assert g_s.step_count() == 8 * (rep + 1)
        assert np.array_equal(e_s.vectors(), g_s.vectors()), rep
    for s in (a, b, c, d, e_s, g_s):
        s.close()


def test_wide_step_errors_and_bad_label():
    torch = _torch()
    sg = _sg()
    gen, priors = _lda_problem(64, 4, 4)
    cfg = sg.make_config(sg.SGEP_KIND_LDA, sg.SGEP_BF16, 4, 64, 0, 32, eta0=0.01,
                         eps_reg=1e-3, n_classes=4)
    s = sg.Solver(cfg, synth.initial_players(64, 4, 0), class_means=gen.means,
                  class_priors=priors)
    X, lab = gen.batch(1, 32)
    Xd = _bf16_dev(synth.bf16_bits(X))
    with pytest.raises(sg.SgepError) as e:           # LDA needs labels
        sg.sgep_step(s.h, Xd, 64, Xd, 64, 32)
    assert e.value.status == sg.SGEP_EINVAL
    with pytest.raises(sg.SgepError) as e:           # b > b_max
        sg.sgep_step_lda(s.h, Xd, 64, _i32_dev(lab), 33)
    assert e.value.status == sg.SGEP_ESHAPE
    with pytest.raises(sg.SgepError) as e:           # ldx not a multiple of 8
        sg.sgep_step_lda(s.h, Xd, 66, _i32_dev(lab), 16)
    assert e.value.status == sg.SGEP_ESHAPE
    assert s.kernels_per_step() == 3
    s.step(Xd, _i32_dev(lab))
    s.sync()
    bad = lab.copy()
    bad[5] = 4                                        # class index out of range
    s.step(Xd, _i32_dev(bad))
    with pytest.raises(sg.SgepError) as e:
        s.sync()
    assert e.value.status == sg.SGEP_ELABEL
    with pytest.raises(sg.SgepError) as e:
        s.step(Xd, _i32_dev(lab))
    assert e.value.status == sg.SGEP_EPOISONED
    s.close()


def test_wide_profiled_step_matches_plain():
    sg = _sg()
    import bench
    gen = synth.CCAPlanted(136, 72, np.linspace(0.9, 0.3, 4), sigma=0.5, seed=2)
    cfg = sg.make_config(sg.SGEP_KIND_CCA, sg.SGEP_BF16, 8, 136, 72, 96, eta0=0.05, gamma=0.5)
    batches = _cca_inputs(gen, 3, 96, "bf16")
    V0 = synth.initial_players(208, 8, 3)
    plain, timed = sg.Solver(cfg, V0), sg.Solver(cfg, V0)
    hip = bench.hip_runtime()
    evs = [ctypes.c_void_p() for _ in range(6)]
    for e in evs:
        assert hip.hipEventCreate(ctypes.byref(e)) == 0
    for Xd, Yd, _, _ in batches:
        plain.step(Xd, Yd)
        sg.sgep_step_profiled(timed.h, Xd, 136, Yd, 72, None, 96, [e.value for e in evs])
    timed.sync()
    assert np.array_equal(plain.vectors(), timed.vectors())
    ms = ctypes.c_float()
    for i in range(3):
        assert hip.hipEventElapsedTime(ctypes.byref(ms), evs[2 * i], evs[2 * i + 1]) == 0
        assert 0.0 < ms.value < 100.0
    Xd, Yd, _, _ = batches[0]
    with pytest.raises(sg.SgepError):                 # four events for three kernels
        sg.sgep_step_profiled(timed.h, Xd, 136, Yd, 72, None, 96, [e.value for e in evs[:4]])
    for e in evs:
        hip.hipEventDestroy(e)
    plain.close()
    timed.close()


@pytest.mark.parametrize("path", ["narrow_f32_cca", "wide_bf16_lda", "wide_f32_lda"])
def test_vectors_sign_convention(path):
    """SGEP_VEC_CANONICAL: each column of the read-out is negated exactly when
    its largest-magnitude component (lowest index on ties) is negative; with
    and without B-normalisation; unknown flag bits are rejected."""
    torch = _torch()
    sg = _sg()
    if path == "narrow_f32_cca":
        gen = synth.CCAPlanted(40, 24, np.linspace(0.9, 0.3, 4), sigma=0.5, seed=3)
        cfg = sg.make_config(sg.SGEP_KIND_CCA, sg.SGEP_F32, 6, 40, 24, 64, eta0=0.05, gamma=0.5)
        s = sg.Solver(cfg, synth.initial_players(64, 6, 2))
        for t in range(1, 4):
            X, Y = gen.batch(t, 64)
            s.step(torch.from_numpy(X.astype(np.float32)).cuda(),
                   torch.from_numpy(Y.astype(np.float32)).cuda())
    else:
        fmt = "bf16" if path == "wide_bf16_lda" else "f32"
        gen, priors = _lda_problem(136, 5, 12)
        cfg = sg.make_config(sg.SGEP_KIND_LDA, sg.SGEP_BF16 if fmt == "bf16" else sg.SGEP_F32,
                             12, 136, 0, 64, eta0=0.01, eps_reg=1e-3, n_classes=5)
        s = sg.Solver(cfg, synth.initial_players(136, 12, 2), class_means=gen.means,
                      class_priors=priors)
        for t in range(1, 4):
            X, lab = gen.batch(t, 64)
            Xd = (_bf16_dev(synth.bf16_bits(X)) if fmt == "bf16"
                  else torch.from_numpy(np.ascontiguousarray(X, dtype=np.float32)).cuda())
            s.step(Xd, _i32_dev(lab))
    for base in (0, sg.SGEP_VEC_BNORM):
        V = s.vectors(base)
        C = s.vectors(base | sg.SGEP_VEC_CANONICAL)
        idx = np.argmax(np.abs(V), axis=0)
        sign = np.sign(V[idx, np.arange(V.shape[1])])
        assert np.array_equal(C, V * sign[None, :])
        assert np.all(C[idx, np.arange(V.shape[1])] > 0)
    with pytest.raises(sg.SgepError) as e:
        s.vectors(4)
    assert e.value.status == sg.SGEP_EINVAL
    s.close()


class _Shifted:
    """A generator's minibatches shifted by fixed per-feature offsets N(0, s^2)
    (non-zero-mean views for the running-mean centring)."""

    def __init__(self, gen, dx, dy, seed, scale):
        rng = np.random.default_rng(seed)
        self.gen = gen
        self.ox, self.oy = rng.normal(0.0, scale, dx), rng.normal(0.0, scale, dy)

    def batch(self, t, b):
        X, Y = self.gen.batch(t, b)
        return X + self.ox, Y + self.oy

    def sample(self, n, rng):
        X, Y = self.gen.sample(n, rng)
        return X + self.ox, Y + self.oy


@pytest.mark.parametrize("fmt,dx,dy,k,b,opt", [
    ("bf16", 520, 264, 20, 300, "sgd"),      # one backward kernel, several subtiles
    ("bf16", 520, 264, 20, 1100, "adam"),    # the LDS-shared forward at KP 32
    ("fp8", 520, 264, 20, 1100, "sgd"),
    ("fp8", 200, 136, 13, 100, "adam"),      # column scales, ragged rows
    # split backward (k_wprod, k_wepi), offsets of scale 0.1: while the
    # running mean is still far from the offsets, the products carry the mean
    # component, whose size grows with d (|mu|^2 ~ d s^2), and the FP32
    # operands' BF16 hi/lo rounding (2^-17) scales with it -- at d = 32776
    # with s = 0.5 that is 1e-4 of [Bv] with or without centring
    ("bf16", 16392, 16384, 4, 512, "sgd"),
    ("fp8", 16392, 16384, 4, 256, "adam"),
])
def test_wide_cca_centring(fmt, dx, dy, k, b, opt):
    """Running-mean centring on the BF16 / FP8 path (rank-one corrections of
    the products, the minibatch column sums from the backward stream) against
    the oracle's centring (Sec. 1 zero-mean assumption; the mean learnt at
    rate gamma): players, [Bv], eigenvalues and the means themselves."""
    sg = _sg()
    print(f"wide CCA centred {fmt} dx={dx} dy={dy} k={k} b={b} {opt}", flush=True)
    adam = opt == "adam"
    gen = _Shifted(synth.CCAPlanted(dx, dy, np.linspace(0.9, 0.3, 4), sigma=0.5, seed=dx + 7),
                   dx, dy, seed=dy + 11, scale=0.5 if dx < 8192 else 0.1)
    cfg = sg.make_config(sg.SGEP_KIND_CCA, sg.SGEP_BF16 if fmt == "bf16" else sg.SGEP_FP8_E4M3, k,
                         dx, dy, b, optimizer=sg.SGEP_ADAM if adam else sg.SGEP_SGD,
                         schedule=sg.SGEP_SCHED_INV, eta0=2e-3 if adam else 0.05, t0=100.0,
                         gamma=0.3, rho=1e-6, center=1)
    aux, scales = None, None
    if fmt == "fp8":
        Xc, Yc = gen.sample(4096, np.random.default_rng([5, 99]))
        scales = (synth.fp8_column_scales(Xc), synth.fp8_column_scales(Yc))
        aux = dict(x_col_scale=scales[0], y_col_scale=scales[1])
    N = 20
    batches = _cca_inputs(gen, N, b, fmt, scales)
    V0 = synth.initial_players(dx + dy, k, 5)
    s = sg.Solver(cfg, V0, **(aux or {}))
    pb = oracle.Problem(oracle.KIND_CCA, k, dx, dy, rho=cfg.rho, optimizer=cfg.optimizer,
                        center=True)
    st = oracle.State.init(V0, adam=adam)
    for t, (Xd, Yd, X, Y) in enumerate(batches, start=1):
        s.step(Xd, Yd)
        oracle.gamma_step(pb, st, X, Y, _eta(cfg, t), cfg.gamma)
        if t in (1, N):
            tol = (TOLW_ADAM_1 if t == 1 else TOLW_ADAM_N) if adam else (TOLW_1 if t == 1 else TOLW_N)
            Vg, Gg = s.vectors(), s.auxiliary()
            mx, my = s.means()
            dm = _maxdiff(np.concatenate([mx, my]), np.concatenate([st.mu_x, st.mu_y]))
            dv, dg = _maxdiff(Vg, st.V), _maxdiff(Gg, st.G)
            print(f"  t={t}: max|dV|={dv:.2e} max|dG|={dg:.2e} max|dmu|={dm:.2e}; per player "
                  + " ".join(f"{x:.1e}" for x in np.abs(Vg - st.V).max(axis=0)[:8]), flush=True)
            snap = oracle.State(V=st.V.copy(), G=st.G.copy(), t=st.t,
                                s2=None if st.s2 is None else st.s2.copy())
            assert_players_close(Vg, snap, tol, adam, sum(_eta(cfg, i) for i in range(1, t + 1)))
            assert dg < tol, (t, dg)
            # the means: FP32 running means of sums over b rows
            assert dm < 1e-5 * max(1.0, float(np.abs(st.mu_x).max())), (t, dm)
            assert np.allclose(s.eigvals(), st.eigvals(), rtol=10 * tol, atol=10 * tol)
    # the centring changes the iterate: the uncentred oracle is far away
    pb0 = oracle.Problem(oracle.KIND_CCA, k, dx, dy, rho=cfg.rho, optimizer=cfg.optimizer)
    st0 = oracle.State.init(V0, adam=adam)
    for t, (_, _, X, Y) in enumerate(batches, start=1):
        oracle.gamma_step(pb0, st0, X, Y, _eta(cfg, t), cfg.gamma)
    assert _maxdiff(s.vectors(), st0.V) > 100 * TOLW_N
    s.close()
