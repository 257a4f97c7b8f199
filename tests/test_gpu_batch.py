"""GPU tests of batched execution (many GENERAL instances per launch),
through the C ABI.

* Every instance advanced by the batch holds the same bits as the same
  instance advanced alone (sgep_step on its borrowed handle) with the same
  feature-tile height, whatever the group count.
* Every instance agrees with the FP64 oracle run on the same minibatches
  (FP64: 1e-11 on unit players; FP32: the single-handle bars).
* Row padding beyond d_i (filled with NaN) is never read.
* The autotuner leaves the initial state untouched; hipGraph replay equals
  eager stepping bitwise.
* Full size: 256 instances with widths uniform in [64, 2048], k = 8, b = 512,
  FP32 with Adam, sampled instances against the oracle."""
import ctypes

import numpy as np
import pytest

import oracle
import synth

pytestmark = pytest.mark.gpu

TOL64 = 1e-12
TOL32_N = 3e-4


def _torch():
    import torch
    return torch


def _sg():
    import paper_2206_04993_amd as sg
    sg.load()
    return sg


def _cfg(sg, dtype, k, b_max, adam=False):
    return sg.make_config(sg.SGEP_KIND_GENERAL, dtype, k, 0, 0, b_max,
                          optimizer=sg.SGEP_ADAM if adam else sg.SGEP_SGD,
                          schedule=sg.SGEP_SCHED_INV, eta0=2e-3 if adam else 0.05, t0=50.0,
                          gamma=0.5, rho=1e-6, eps_reg=1e-3)


def _padded(A, ld, fill=np.nan):
    out = np.full((A.shape[0], ld), fill, dtype=A.dtype)
    out[:, :A.shape[1]] = A
    return out


class _Data:
    """Host minibatches per (step, instance), rounded to the element type, and
    their device copies with rows padded to ld_i (padding NaN)."""

    def __init__(self, gens, lds, T, b, ndt, tdt):
        torch = _torch()
        self.host = []
        self.dev = []
        self.ptrs = []
        for t in range(1, T + 1):
            hs, xs, ys = [], [], []
            for g, ld in zip(gens, lds):
                X, Y = g.batch(t, b)
                X = X.astype(ndt).astype(np.float64)
                Y = Y.astype(ndt).astype(np.float64)
                hs.append((X, Y))
                xs.append(torch.from_numpy(_padded(X.astype(ndt), ld)).to("cuda", tdt))
                ys.append(torch.from_numpy(_padded(Y.astype(ndt), ld)).to("cuda", tdt))
            self.host.append(hs)
            self.dev.append((xs, ys))
            self.ptrs.append((torch.tensor([x.data_ptr() for x in xs], dtype=torch.int64,
                                           device="cuda"),
                              torch.tensor([y.data_ptr() for y in ys], dtype=torch.int64,
                                           device="cuda")))


def _oracle_run(cfg, gen_d, V0, host_steps, i):
    pb = oracle.Problem(oracle.KIND_GENERAL, cfg.k, gen_d, gen_d, eps_reg=cfg.eps_reg,
                        rho=cfg.rho, optimizer=cfg.optimizer)
    st = oracle.State.init(V0, adam=cfg.optimizer == 1)
    for t, hs in enumerate(host_steps, start=1):
        X, Y = hs[i]
        oracle.gamma_step(pb, st, X, Y, oracle.eta(cfg.schedule, t, cfg.eta0, t0=cfg.t0),
                          cfg.gamma)
    return st


DIMS = [64, 67, 130, 13, 257, 300, 513, 1000, 1030, 9]


@pytest.mark.parametrize("dtype,adam", [("f64", False), ("f32", False), ("f32", True)])
def test_batch_matches_single_handles_and_oracle(dtype, adam):
    torch = _torch()
    sg = _sg()
    f64 = dtype == "f64"
    sdt = sg.SGEP_F64 if f64 else sg.SGEP_F32
    ndt, tdt = (np.float64, torch.float64) if f64 else (np.float32, torch.float32)
    k, b, T = 8, 100, 4
    vec = 2 if f64 else 4
    lds = [d if i % 2 else (d + vec - 1) // vec * vec + vec for i, d in enumerate(DIMS)]
    gens = [synth.GeneralPlanted(d, k=min(k, d), seed=50 + i) for i, d in enumerate(DIMS)]
    V0s = [synth.initial_players(d, k, i) for i, d in enumerate(DIMS)]
    cfg = _cfg(sg, sdt, k, 128, adam)
    data = _Data(gens, lds, T, b, ndt, tdt)
    for groups, mb in [(1, [1, 1, 1]), (3, [1, 4, 4])]:
        bat = sg.BatchSolver(DIMS, cfg, V0s, ld=lds)
        bat.set_plan(groups, mb)
        ref = sg.BatchSolver(DIMS, cfg, V0s, ld=lds)
        ref.set_plan(groups, mb)
        kinds = bat.launches()
        print(f"{dtype} adam={adam} plan={bat.plan()} launches={kinds}")
        assert kinds.count(0) == bat.plan()[0] and kinds.count(-1) == bat.plan()[0]
        for t in range(T):
            bat.step(*data.ptrs[t], b)
            xs, ys = data.dev[t]
            for i, d in enumerate(DIMS):  # the same instance stepped alone
                sg.sgep_step(ref.instance(i), xs[i], lds[i], ys[i], lds[i], b)
        bat.sync()
        ref.sync()
        for i, d in enumerate(DIMS):
            vb, vr = bat.vectors(i), ref.vectors(i)
            assert np.array_equal(vb, vr), (i, d)
            assert np.array_equal(bat.auxiliary(i), ref.auxiliary(i)), (i, d)
            assert np.array_equal(bat.eigvals(i), ref.eigvals(i)), (i, d)
            assert bat.step_count(i) == T
            st = _oracle_run(cfg, d, V0s[i], data.host, i)
            dv = float(np.abs(vb - st.V).max())
            dg = float(np.abs(bat.auxiliary(i) - st.G).max()) / max(1.0, np.abs(st.G).max())
            tol = TOL64 if f64 else TOL32_N * (5 if adam else 1)
            print(f"  d={d} ld={lds[i]} max|dV|={dv:.2e} rel|dG|={dg:.2e}")
            assert dv < tol and dg < tol, (i, d, dv, dg)
        bat.close()
        ref.close()


def test_batch_groups_do_not_change_bits():
    torch = _torch()
    sg = _sg()
    k, b, T = 8, 128, 3
    gens = [synth.GeneralPlanted(d, k=k, seed=80 + i) for i, d in enumerate(DIMS[:8])]
    dims = [g.d for g in gens]
    V0s = [synth.initial_players(d, k, 7 + i) for i, d in enumerate(dims)]
    cfg = _cfg(sg, sg.SGEP_F32, k, b, adam=True)
    data = _Data(gens, dims, T, b, np.float32, torch.float32)
    res = []
    for groups in (1, 2, 8):
        bat = sg.BatchSolver(dims, cfg, V0s)
        bat.set_plan(groups, [4, 4, 4])
        for t in range(T):
            bat.step(*data.ptrs[t], b)
        res.append([bat.vectors(i) for i in range(len(dims))])
        print("groups", bat.plan(), "launches", bat.launches())
        bat.close()
    for r in res[1:]:
        for a, c in zip(res[0], r):
            assert np.array_equal(a, c)


@pytest.mark.parametrize("dtype,adam", [("f64", False), ("f32", False), ("f32", True)])
def test_batch_persistent_matches_single_handles(dtype, adam):
    """The persistent plan (one launch per iteration over per-XCC work
    queues) with look-aheads 1 and 3: every instance bitwise equal to the
    same instance stepped alone, over minibatches of varying length (row
    tiles past b do nothing but count), and to the oracle at the
    single-handle bars; a hipGraph of the persistent step replayed several
    times, with eager work in between, equals eager stepping bitwise."""
    torch = _torch()
    sg = _sg()
    f64 = dtype == "f64"
    sdt = sg.SGEP_F64 if f64 else sg.SGEP_F32
    ndt, tdt = (np.float64, torch.float64) if f64 else (np.float32, torch.float32)
    k, b_max = 8, 128
    sizes = [128, 100, 128, 37, 1]
    T = len(sizes)
    vec = 2 if f64 else 4
    lds = [d if i % 2 else (d + vec - 1) // vec * vec + vec for i, d in enumerate(DIMS)]
    gens = [synth.GeneralPlanted(d, k=min(k, d), seed=60 + i) for i, d in enumerate(DIMS)]
    V0s = [synth.initial_players(d, k, 20 + i) for i, d in enumerate(DIMS)]
    cfg = _cfg(sg, sdt, k, b_max, adam)
    data = _Data(gens, lds, T, b_max, ndt, tdt)
    for lag in (1, 3):
        bat = sg.BatchSolver(DIMS, cfg, V0s, ld=lds)
        bat.set_plan(-lag, [1, 1, 1])
        assert bat.plan()[0] == -lag and bat.launches() == [-2]
        ref = sg.BatchSolver(DIMS, cfg, V0s, ld=lds)
        print(f"{dtype} adam={adam} lag={lag} plan={bat.plan()}", flush=True)
        for t, b in enumerate(sizes):
            bat.step(*data.ptrs[t], b)
            xs, ys = data.dev[t]
            for i in range(len(DIMS)):
                sg.sgep_step(ref.instance(i), xs[i], lds[i], ys[i], lds[i], b)
        bat.sync()
        ref.sync()
        for i, d in enumerate(DIMS):
            assert np.array_equal(bat.vectors(i), ref.vectors(i)), (lag, i, d)
            assert np.array_equal(bat.auxiliary(i), ref.auxiliary(i)), (lag, i, d)
            assert bat.step_count(i) == T
        if lag == 1:
            host = [[(X[:b], Y[:b]) for X, Y in hs] for hs, b in zip(data.host, sizes)]
            for i, d in enumerate(DIMS):
                st = _oracle_run(cfg, d, V0s[i], host, i)
                dv = float(np.abs(bat.vectors(i) - st.V).max())
                dg = float(np.abs(bat.auxiliary(i) - st.G).max()) / max(1.0, np.abs(st.G).max())
                tol = TOL64 if f64 else TOL32_N * (5 if adam else 1)
                print(f"  d={d} max|dV|={dv:.2e} rel|dG|={dg:.2e}")
                assert dv < tol and dg < tol, (i, d, dv, dg)
        bat.close()
        ref.close()
    # graph replays of the persistent step against eager persistent steps
    stream = torch.cuda.Stream()
    gb = sg.BatchSolver(DIMS, cfg, V0s, ld=lds, stream=stream)
    gb.set_plan(-2, [1, 1, 1])
    eb = sg.BatchSolver(DIMS, cfg, V0s, ld=lds)
    eb.set_plan(-2, [1, 1, 1])
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g, stream=stream):
        gb.step(*data.ptrs[0], b_max)
    torch.cuda.synchronize()
    for r in range(4):
        g.replay()
        torch.cuda.synchronize()
        eb.step(*data.ptrs[0], b_max)
        eb.sync()
        for i in range(len(DIMS)):
            assert gb.step_count(i) == r + 1
            assert np.array_equal(gb.vectors(i), eb.vectors(i)), (r, i)
    gb.close()
    eb.close()


class _ShiftedGen:
    """A generator whose views carry per-feature offsets of order 1 (so an
    uncentred step differs at O(1))."""

    def __init__(self, gen, d, seed):
        rng = np.random.default_rng(seed)
        self.gen, self.ox, self.oy = gen, rng.normal(0.0, 1.0, d), rng.normal(0.0, 1.0, d)

    def batch(self, t, n):
        X, Y = self.gen.batch(t, n)
        return X + self.ox, Y + self.oy


@pytest.mark.parametrize("dtype,groups", [("f64", 1), ("f64", -2), ("f32", 3), ("f32", -1)])
def test_batch_centring_matches_single_handles_and_oracle(dtype, groups):
    """Running-mean centring in the batch (grouped and persistent plans):
    every instance bitwise equal to the same centred instance stepped alone,
    and to the oracle's centring (Sec. 1 zero-mean assumption, the means
    learnt at rate gamma) at the single-handle bars, the means included."""
    torch = _torch()
    sg = _sg()
    f64 = dtype == "f64"
    sdt = sg.SGEP_F64 if f64 else sg.SGEP_F32
    ndt, tdt = (np.float64, torch.float64) if f64 else (np.float32, torch.float32)
    k, b_max = 8, 128
    sizes = [128, 100, 128, 37]
    gens = [_ShiftedGen(synth.GeneralPlanted(d, k=min(k, d), seed=70 + i), d, 170 + i)
            for i, d in enumerate(DIMS)]
    V0s = [synth.initial_players(d, k, 30 + i) for i, d in enumerate(DIMS)]
    cfg = sg.make_config(sg.SGEP_KIND_GENERAL, sdt, k, 0, 0, b_max, optimizer=sg.SGEP_SGD,
                         schedule=sg.SGEP_SCHED_INV, eta0=0.05, t0=50.0, gamma=0.5, rho=1e-4,
                         eps_reg=1e-3, center=1)
    data = _Data(gens, DIMS, len(sizes), b_max, ndt, tdt)
    bat = sg.BatchSolver(DIMS, cfg, V0s)
    bat.set_plan(groups, [1, 1, 1])
    ref = sg.BatchSolver(DIMS, cfg, V0s)
    print(f"{dtype} centred batch plan={bat.plan()} launches={bat.launches()}", flush=True)
    for t, b in enumerate(sizes):
        bat.step(*data.ptrs[t], b)
        xs, ys = data.dev[t]
        for i, d in enumerate(DIMS):
            sg.sgep_step(ref.instance(i), xs[i], d, ys[i], d, b)
    bat.sync()
    ref.sync()
    host = [[(X[:b], Y[:b]) for X, Y in hs] for hs, b in zip(data.host, sizes)]
    tol = TOL64 if f64 else TOL32_N
    for i, d in enumerate(DIMS):
        mb_ = sg.sgep_means(bat.instance(i), 2 * d)
        assert np.array_equal(bat.vectors(i), ref.vectors(i)), (i, d)
        assert np.array_equal(mb_, sg.sgep_means(ref.instance(i), 2 * d)), (i, d)
        pb = oracle.Problem(oracle.KIND_GENERAL, cfg.k, d, d, eps_reg=cfg.eps_reg, rho=cfg.rho,
                            optimizer=cfg.optimizer, center=True)
        st = oracle.State.init(V0s[i], adam=False)
        for t, hs in enumerate(host, start=1):
            X, Y = hs[i]
            oracle.gamma_step(pb, st, X, Y, oracle.eta(cfg.schedule, t, cfg.eta0, t0=cfg.t0),
                              cfg.gamma)
        dv = float(np.abs(bat.vectors(i) - st.V).max())
        dg = float(np.abs(bat.auxiliary(i) - st.G).max()) / max(1.0, np.abs(st.G).max())
        mo = np.concatenate([st.mu_x, st.mu_y])
        dm = float(np.abs(mb_ - mo).max()) / max(1.0, float(np.abs(mo).max()))
        print(f"  d={d} max|dV|={dv:.2e} rel|dG|={dg:.2e} rel|dmu|={dm:.2e}")
        assert dv < tol and dg < tol, (i, d, dv, dg)
        assert dm < (1e-12 if f64 else 1e-6), (i, d, dm)
    bat.close()
    ref.close()


def test_batch_tune_keeps_initial_state_and_graph_replay_matches_eager():
    torch = _torch()
    sg = _sg()
    k, b, T = 8, 64, 4
    gens = [synth.GeneralPlanted(d, k=k, seed=90 + i, mixing="fast")
            for i, d in enumerate([100, 700, 1500, 40, 2048, 333])]
    dims = [g.d for g in gens]
    V0s = [synth.initial_players(d, k, 3 + i) for i, d in enumerate(dims)]
    cfg = _cfg(sg, sg.SGEP_F32, k, b, adam=True)
    data = _Data(gens, dims, T, b, np.float32, torch.float32)
    torch.cuda.synchronize()
    fresh = sg.BatchSolver(dims, cfg, V0s)
    stream = torch.cuda.Stream()
    tuned = sg.BatchSolver(dims, cfg, V0s, stream=stream)
    us = tuned.tune(*data.ptrs[0], b, reps=2)
    groups, mb = tuned.plan()
    print(f"tuned plan groups={groups} mb={mb} {us:.1f} us/iteration")
    assert us > 0 and groups != 0 and all(m in (1, 4) for m in mb)
    for i in range(len(dims)):
        assert tuned.step_count(i) == 0
        assert np.array_equal(tuned.vectors(i), fresh.vectors(i))
        assert np.array_equal(tuned.auxiliary(i), fresh.auxiliary(i))
    # eager reference with the tuned plan on a separate batch
    eager = sg.BatchSolver(dims, cfg, V0s)
    eager.set_plan(groups, mb)
    for t in range(T):
        eager.step(*data.ptrs[t], b)
    eager.sync()
    # graph: the same T iterations captured once, replayed once
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g, stream=stream):
        for t in range(T):
            tuned.step(*data.ptrs[t], b)
    torch.cuda.synchronize()
    for i in range(len(dims)):  # capture ran nothing
        assert tuned.step_count(i) == 0
    g.replay()
    torch.cuda.synchronize()
    for i in range(len(dims)):
        assert tuned.step_count(i) == T
        assert np.array_equal(tuned.vectors(i), eager.vectors(i))
    with pytest.raises(sg.SgepError) as ei:  # tuning only before the first iteration
        tuned.tune(*data.ptrs[0], b)
    assert ei.value.status == sg.SGEP_EINVAL
    with pytest.raises(sg.SgepError) as ei:
        tuned.set_plan(1, [1, 1, 1])
    assert ei.value.status == sg.SGEP_EINVAL
    for s in (fresh, tuned, eager):
        s.close()


def test_batch_argument_errors():
    torch = _torch()
    sg = _sg()
    lib = sg.load()
    dims = [32, 48]
    V0s = [synth.initial_players(d, 4, i) for i, d in enumerate(dims)]
    cfg = _cfg(sg, sg.SGEP_F32, 4, 16)
    bat = sg.BatchSolver(dims, cfg, V0s)
    xs = [torch.zeros((16, d), device="cuda") for d in dims]
    p = sg.BatchSolver.pointers(xs, "cuda")
    assert lib.sgep_batch_step(bat.bt, p.data_ptr(), p.data_ptr(), 17) == sg.SGEP_ESHAPE
    assert lib.sgep_batch_step(bat.bt, p.data_ptr(), p.data_ptr(), 0) == sg.SGEP_ESHAPE
    assert lib.sgep_batch_step(bat.bt, None, p.data_ptr(), 4) == sg.SGEP_EINVAL
    mb = (ctypes.c_int32 * 3)(1, 3, 1)
    assert lib.sgep_batch_set_plan(bat.bt, 1, mb) == sg.SGEP_EINVAL
    h = ctypes.c_void_p()
    assert lib.sgep_batch_instance(bat.bt, 2, ctypes.byref(h)) == sg.SGEP_EINVAL
    n = ctypes.c_int32()
    kinds = (ctypes.c_int32 * 1)()
    assert lib.sgep_batch_launches(bat.bt, ctypes.byref(n), kinds, 1) == sg.SGEP_ESHAPE
    ev = (ctypes.c_void_p * 1)()
    assert lib.sgep_batch_step_profiled(bat.bt, p.data_ptr(), p.data_ptr(), 4, ev,
                                        1) == sg.SGEP_EINVAL
    for x in xs:
        x.fill_(float("nan"))
    bat.step(p, p, 16)  # non-finite data: a non-finite Gram term poisons the instances
    with pytest.raises(sg.SgepError) as ei:
        bat.sync()
    assert ei.value.status == sg.SGEP_ENONFINITE
    assert lib.sgep_batch_step(bat.bt, p.data_ptr(), p.data_ptr(), 4) == sg.SGEP_EPOISONED
    bat.close()


def test_batch_full_size_against_oracle():
    """256 instances, d uniform in [64, 2048], k = 8, b = 512, FP32, Adam, in
    the tuned launch plan; 2 iterations; 8 instances checked against the
    oracle on the same (device-drawn) data, every instance for unit norm."""
    torch = _torch()
    sg = _sg()
    k, b, T = 8, 512, 2
    gens = synth.batched_general()
    dims = [g.d for g in gens]
    V0s = [synth.initial_players(d, k, 1000 + i) for i, d in enumerate(dims)]
    cfg = sg.make_config(sg.SGEP_KIND_GENERAL, sg.SGEP_F32, k, 0, 0, b,
                         optimizer=sg.SGEP_ADAM, schedule=sg.SGEP_SCHED_INV, eta0=1e-3,
                         t0=3000.0, gamma=0.3, rho=1e-6, eps_reg=1e-3)
    steps = []
    for t in range(1, T + 1):
        xs, ys = [], []
        for g in gens:
            x, y = g.sample_torch(b, t, "cuda", torch.float32)
            xs.append(x.contiguous())
            ys.append(y.contiguous())
        steps.append((xs, ys, sg.BatchSolver.pointers(xs, "cuda"),
                      sg.BatchSolver.pointers(ys, "cuda")))
    bat = sg.BatchSolver(dims, cfg, V0s)
    us = bat.tune(steps[0][2], steps[0][3], b, reps=2)
    print(f"full size: plan {bat.plan()} {us:.1f} us/iteration, launches {bat.launches()}")
    for xs, ys, px, py in steps:
        bat.step(px, py, b)
    bat.sync()
    order = np.argsort(dims)
    check = sorted(set([int(order[0]), int(order[1]), int(order[-1]), int(order[-2]), 0, 17,
                        100, 255]))
    for i in range(len(dims)):
        V = bat.vectors(i)
        assert np.allclose(np.linalg.norm(V, axis=0), 1.0, atol=1e-5), i
        if i not in check:
            continue
        host = [[(s[0][i].double().cpu().numpy(), s[1][i].double().cpu().numpy())]
                for s in steps]
        st = _oracle_run(cfg, dims[i], V0s[i], host, 0)
        dv = float(np.abs(V - st.V).max())
        dg = float(np.abs(bat.auxiliary(i) - st.G).max()) / max(1.0, np.abs(st.G).max())
        print(f"  instance {i} d={dims[i]} max|dV|={dv:.2e} rel|dG|={dg:.2e}")
        assert dv < 5 * TOL32_N and dg < 5 * TOL32_N, (i, dv, dg)
    # the persistent plan over the same steps: every instance bit for bit as
    # under the tuned plan (16-feature tiles in both)
    if all(m == 1 for m in bat.plan()[1]):
        per = sg.BatchSolver(dims, cfg, V0s)
        per.set_plan(-1, [1, 1, 1])
        for xs, ys, px, py in steps:
            per.step(px, py, b)
        per.sync()
        for i in range(len(dims)):
            assert np.array_equal(per.vectors(i), bat.vectors(i)), i
            assert np.array_equal(per.auxiliary(i), bat.auxiliary(i)), i
        per.close()
    bat.close()
