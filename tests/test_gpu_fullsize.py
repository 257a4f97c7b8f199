"""Full-size parity of the large workloads, in the launch configuration the
benchmark times (bench.py's workload definitions, encodings and solver
configuration), against the FP64 oracle fed the exact values the GPU
receives.  Eight iterations with plain ascent (SGD), two with Adam; every
output compared.

* activation-like CCA, d = 8192 + 8192, k = 32, b = 4096: BF16, FP8-e4m3 with
  per-column scales (BF16 / FP8 path), FP32 (narrow path, 64-feature tiles,
  coefficients in k_coef)
* LDA, d = 65536, 10 classes, k = 64, b = 2048, BF16 and FP32 (both on the
  large-d path)

Bars, on unit players and relative on [Bv] and the eigenvalue estimates.
Adam: the N-iteration bars of the small-size tests (BF16 / FP8: 1.2e-3; FP32:
3e-4) after two iterations.  Plain ascent: after the first iteration 1e-6
(BF16 / FP8) and 2e-7 (FP32), about ten times the observed 1.1e-7 and 1.2e-8;
after eight, 5e-3 (BF16 / FP8) and 3e-4 (FP32): the activation-like CCA's
first iterations amplify a difference at the rounding level by about 10^4 in
every precision (FP32: 1.2e-8 -> 5e-5; FP8: 1.1e-7 -> 2.2e-3), while LDA
stays near the first iteration's 2e-9 (bar 1e-7 at every iteration, BF16 and
FP32).  With Adam an element's step is about eta_t sign(g) while its
second moment is g^2 (the first iterations), so an element whose gradient g
is at the rounding level may step either way: such elements can differ by up
to 2 sum_t eta_t: checked as that bound on every element, at most 1e-4 of
the elements (at least 4) above the plain bar -- printed with their smallest
gradient over the iterations, e.g. 1.2e-7 against a column median of 0.11 for
the one such element of the large CCA in BF16 -- and a relative Frobenius
difference below the plain bar.  The same workloads with plain ascent (SGD)
meet the plain bars on every element, after one and after eight iterations."""
import numpy as np
import pytest

import oracle
import synth
from parity_bars import assert_players_close

pytestmark = pytest.mark.gpu

TOL = {"bf16": 1.2e-3, "fp8": 1.2e-3, "f32": 3e-4}   # Adam, two iterations
TOL1 = {"bf16": 1e-6, "fp8": 1e-6, "f32": 2e-7}       # plain ascent, first iteration
TOL8 = {"bf16": 5e-3, "fp8": 5e-3, "f32": 3e-4}       # plain ascent, eight iterations
TOL_LDA_SGD = 1e-7  # LDA with plain ascent, every iteration (observed <= 6.1e-9)

WORKLOADS = ["cca_d16384_k32_b4096_bf16", "cca_d16384_k32_b4096_fp8",
             "cca_d16384_k32_b4096_fp32", "lda_d65536_k64_b2048_bf16",
             "lda_d65536_k64_b2048_fp32"]


@pytest.mark.parametrize("opt", ["adam", "sgd"])
@pytest.mark.parametrize("wname", WORKLOADS)
def test_full_size_against_oracle(wname, opt):
    import torch

    import bench
    import paper_2206_04993_amd as sg
    sg.load()
    w = dict(bench.WORKLOADS[wname], optimizer=opt)
    lda = w["kind"] == "lda"
    d, k, b = w["dx"] + w["dy"], w["k"], w["b"]
    T = 8 if opt == "sgd" else 2
    print(f"full size {wname}: generating {T} minibatches", flush=True)
    raw = bench.host_batches(w, T)
    aux, scales, extra = {}, None, {}
    if w["dtype"] == "fp8":
        scales = (synth.fp8_column_scales(np.concatenate([r[0] for r in raw])),
                  synth.fp8_column_scales(np.concatenate([r[1] for r in raw])))
        aux = dict(x_col_scale=scales[0], y_col_scale=scales[1])
    if lda:
        gen = bench._generator(w)
        priors = np.full(w["n_classes"], 1.0 / w["n_classes"])
        aux = dict(class_means=gen.means, class_priors=priors)
        extra = dict(class_means=gen.means, class_priors=priors)
    V0 = synth.initial_players(d, k, 0)
    solver = sg.Solver(bench.config_for(sg, w), V0, **aux)
    pb = oracle.Problem(oracle.KIND_LDA if lda else oracle.KIND_CCA, k, w["dx"], w["dy"],
                        rho=w["rho"], eps_reg=w.get("eps_reg", 0.0),
                        optimizer=oracle.OPT_ADAM if w["optimizer"] == "adam" else oracle.OPT_SGD,
                        **extra)
    st = oracle.State.init(V0, adam=w["optimizer"] == "adam")
    gmin = None  # Adam: the smallest |gradient| of each element over the iterations
    for t, (Xr, Yr) in enumerate(raw, start=1):
        m_prev = None if st.m is None else st.m.copy()
        tx, vx = bench.encode(w, Xr, scales[0] if scales else None)
        if lda:
            ty = torch.from_numpy(np.ascontiguousarray(Yr, dtype=np.int32))
            vy = None
        else:
            ty, vy = bench.encode(w, Yr, scales[1] if scales else None)
        solver.step(tx.cuda(), ty.cuda())
        eta = oracle.eta(oracle.SCHED_INV, t, w["eta0"], t0=w["t0"])
        if lda:
            oracle.gamma_step(pb, st, vx, None, eta, w["gamma"], labels=Yr.astype(np.int32))
        else:
            oracle.gamma_step(pb, st, vx, vy, eta, w["gamma"])
        if opt == "sgd":  # the growth of the difference over the iterations
            dvt = float(np.abs(solver.vectors() - st.V).max())
            print(f"    t={t}: max|dV| = {dvt:.2e}", flush=True)
            if lda:
                assert dvt < TOL_LDA_SGD, (t, dvt)
            elif t == 1:
                assert dvt < TOL1[w["dtype"]], dvt
        if m_prev is not None:  # g_t from m_t = b1 m_(t-1) + (1 - b1) g_t
            g = np.abs(st.m - 0.9 * m_prev) / 0.1
            gmin = g if gmin is None else np.minimum(gmin, g)
    V, G, lam = solver.vectors(), solver.auxiliary(), solver.eigvals()
    solver.close()
    dV = np.abs(V - st.V)
    dv = float(dV.max())
    dg = float(np.abs(G - st.G).max()) / max(1.0, float(np.abs(st.G).max()))
    dl = float(np.abs(lam - st.eigvals()).max()) / max(1.0, float(np.abs(st.eigvals()).max()))
    tol = TOL[w["dtype"]] if opt == "adam" else (TOL_LDA_SGD if lda else TOL8[w["dtype"]])
    over = int((dV > tol).sum())
    fro = float(np.linalg.norm(V - st.V) / np.linalg.norm(st.V))
    print(f"  {wname} {opt}: max|dV| = {dv:.2e} ({over} of {dV.size} above {tol:g}), "
          f"rel F |dV| = {fro:.2e}, rel|dG| = {dg:.2e}, rel|dlam| = {dl:.2e}", flush=True)
    assert dg < tol and dl < tol, (dg, dl)
    eta_sum = sum(oracle.eta(oracle.SCHED_INV, t, w["eta0"], t0=w["t0"]) for t in range(1, T + 1))
    if opt == "sgd":  # the plain bar on every element
        assert_players_close(V, st, tol)
    else:
        # Adam: every element within 2 sum_t eta_t + tol of the oracle; above
        # the plain bar only a few elements, those whose gradient came close
        # to the rounding of its terms at some iteration (printed with their
        # smallest gradient against the column median); for LDA the leading
        # c - 1 players (beyond the rank of the between-class A the players
        # carry no signal and are only required to be finite unit vectors)
        c1 = w["n_classes"] - 1 if lda else V.shape[1]
        Dc = dV[:, :c1]
        big = Dc > tol
        for jj in zip(*np.nonzero(big)):
            print(f"      element {jj}: |dV| {float(Dc[jj]):.2e}, smallest |g| "
                  f"{float(gmin[jj]):.2e}, column median {float(np.median(gmin[:, jj[1]])):.2e}",
                  flush=True)
        assert float(Dc.max()) <= 2.0 * eta_sum + tol, float(Dc.max())
        assert int(big.sum()) <= max(4, 1e-4 * Dc.size), int(big.sum())
        assert fro < tol, fro
        assert np.isfinite(V).all()
    assert np.allclose(np.linalg.norm(V, axis=0), 1.0, atol=1e-5)
