"""Pins of the FP64 oracle against facts the paper and the mathematics fix.

None of these retypes the oracle's own formula: each compares it with a value
the paper prints, a closed form, an invariant, a library routine the paper
itself names as ground truth (scipy.linalg.eigh), or brute force."""
import json
import os

import numpy as np
import pytest
import scipy.linalg as sla

import oracle
from oracle import targets
import synth

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _rand_spd(rng, d, shift=1.0):
    M = rng.standard_normal((d, d))
    return M @ M.T / d + shift * np.eye(d)


def _rand_sym(rng, d):
    M = rng.standard_normal((d, d))
    return (M + M.T) / 2


def _unit(V):
    return V / np.linalg.norm(V, axis=0, keepdims=True)


# --------------------------------------------------------------------------- #
# Exact solver                                                                 #
# --------------------------------------------------------------------------- #

def test_worked_example_2x2_angle_and_utilities():
    """App. B example matrices; Fig. 1: eigenvectors ~71 deg (109 deg) apart,
    u_2 = 0 when player 2 copies v_1 and u_2 = lambda_2 at v_2."""
    g = json.load(open(os.path.join(GOLDEN, "warped_sinusoid_2x2.json")))
    A, B = np.array(g["A"]), np.array(g["B"])
    lam, V = oracle.gep_topk(A, B, 2)
    U = _unit(V)
    ang = np.degrees(np.arccos(U[:, 0] @ U[:, 1]))
    folded = min(ang, 180 - ang)
    assert abs(folded - g["angle_deg"]) < g["angle_tolerance_deg"]
    assert abs(max(ang, 180 - ang) - g["angle_deg_supplement"]) < g["angle_tolerance_deg"]
    W = np.stack([U[:, 0], U[:, 0]], axis=1)
    assert abs(oracle.utility(A, B, W, 1)) < 1e-12
    W = np.stack([U[:, 0], U[:, 1]], axis=1)
    assert abs(oracle.utility(A, B, W, 1) - lam[1]) < 1e-10 * lam[0]


@pytest.mark.parametrize("d,k", [(2, 1), (7, 3), (16, 4), (40, 8)])
def test_gep_matches_scipy_and_is_b_orthonormal(d, k):
    """scipy.linalg.eigh(A, B) is the ground truth the paper uses; V^T B V = I
    (B-orthogonality lemma) and A v = lambda B v."""
    rng = np.random.default_rng(d)
    A, B = _rand_sym(rng, d), _rand_spd(rng, d)
    lam, V = oracle.gep_topk(A, B, k)
    ref = sla.eigh(A, B, eigvals_only=True)[::-1][:k]
    assert np.allclose(lam, ref, rtol=0, atol=1e-12 * abs(ref).max())
    assert np.abs(V.T @ B @ V - np.eye(k)).max() < 1e-12
    res = A @ V - (B @ V) * lam[None, :]
    assert np.abs(res).max() < 1e-12 * np.abs(A).max() * max(1, np.abs(V).max())
    # vectors agree with scipy's up to sign
    w, Z = sla.eigh(A, B)
    Z = Z[:, ::-1][:, :k]
    for i in range(k):
        assert min(np.abs(V[:, i] - Z[:, i]).max(), np.abs(V[:, i] + Z[:, i]).max()) < 1e-9


def test_cholesky_and_jacobi_against_definitions():
    rng = np.random.default_rng(3)
    B = _rand_spd(rng, 12)
    L = oracle.cholesky(B)
    assert np.allclose(np.triu(L, 1), 0) and np.all(np.diag(L) > 0)
    assert np.abs(L @ L.T - B).max() < 1e-13
    with pytest.raises(np.linalg.LinAlgError):
        oracle.cholesky(-B)
    C = _rand_sym(rng, 12)
    w, Z = oracle.jacobi_eigh(C)
    assert np.abs(Z.T @ Z - np.eye(12)).max() < 1e-13
    assert np.abs(C @ Z - Z * w[None, :]).max() < 1e-12
    assert np.allclose(np.sort(w), np.linalg.eigvalsh(C), atol=1e-12)


def _count_below(A, B, sigma):
    """Sylvester inertia: number of eigenvalues of (A, B) below sigma equals
    the number of negative pivots of symmetric elimination of A - sigma B."""
    M = (A - sigma * B).copy()
    n = M.shape[0]
    neg = 0
    for p in range(n):
        piv = M[p, p]
        if piv < 0:
            neg += 1
        for i in range(p + 1, n):
            f = M[i, p] / piv
            for j in range(p + 1, n):
                M[i, j] -= f * M[p, j]
    return neg


def test_brute_force_bisection_d16():
    """Eigenvalues by bisection on inertia counts and vectors by inverse
    iteration, on a d = 16 instance (the tiny CCA width)."""
    rng = np.random.default_rng(16)
    d, k = 16, 4
    A, B = _rand_sym(rng, d), _rand_spd(rng, d)
    lam, V = oracle.gep_topk(A, B, k)
    R = 1e3
    for i in range(k):
        target = d - 1 - i  # index in ascending order
        lo, hi = -R, R
        for _ in range(80):
            mid = 0.5 * (lo + hi)
            if _count_below(A, B, mid) > target:
                hi = mid
            else:
                lo = mid
        lam_bf = 0.5 * (lo + hi)
        assert abs(lam_bf - lam[i]) < 1e-11
        v = rng.standard_normal(d)
        for _ in range(3):
            v = np.linalg.solve(A - (lam_bf + 1e-9) * B, B @ v)
            v /= np.sqrt(v @ B @ v)
        assert min(np.abs(v - V[:, i]).max(), np.abs(v + V[:, i]).max()) < 1e-7


def test_planted_cca_spectrum_tiny():
    """Orthonormal mixing with 0.1 noise: canonical correlations rho/(1+0.1^2)."""
    gen = synth.tiny_cca(0)
    A, B = targets.cca_population_AB(gen)
    lam, V = oracle.gep_topk(A, B, 4)
    assert np.allclose(lam, gen.rho / 1.01, atol=1e-12)
    # the spectrum of the CCA pencil is symmetric: -rho/1.01 are eigenvalues too
    lam_all, _ = oracle.gep_topk(A, B, 16)
    assert np.allclose(np.sort(lam_all)[:4], -gen.rho / 1.01, atol=1e-12)


def test_planted_cca_closed_form_matches_exact_solver():
    """Noiseless square mixing: the planted correlations exactly, with
    v_i = [Wx^{-T} e_i; Wy^{-T} e_i]/sqrt(2) (per-view invariance of CCA)."""
    gen = synth.CCAPlanted(32, 32, np.linspace(0.95, 0.2, 4), n_free=28, spread=0.1, seed=5)
    A, B = targets.cca_population_AB(gen)
    lam, V = oracle.gep_topk(A, B, 4)
    lam_c, V_c = targets.cca_planted_topk(gen, 4)
    assert np.allclose(lam, lam_c, atol=1e-11)
    assert oracle.subspace_error(V_c, V, B) < 1e-12
    assert np.abs(V_c.T @ B @ V_c - np.eye(4)).max() < 1e-10


def test_general_planted_matches_exact_solver():
    gen = synth.GeneralPlanted(40, k=8, seed=2)
    A, B = targets.general_population_AB(gen)
    lam, V = oracle.gep_topk(A, B, 8)
    lam_c, V_c = targets.general_planted_topk(gen, 8)
    assert np.allclose(lam, np.geomspace(10, 0.1, 8), rtol=1e-10)
    assert np.allclose(lam_c, lam, rtol=1e-10)
    assert oracle.subspace_error(V_c, V, B) < 1e-12


# --------------------------------------------------------------------------- #
# Metric                                                                       #
# --------------------------------------------------------------------------- #

def test_subspace_error_gram_form_equals_definition():
    rng = np.random.default_rng(4)
    d, k = 12, 3
    A, B = _rand_sym(rng, d), _rand_spd(rng, d)
    lam, Vs = oracle.gep_topk(A, B, k)
    for _ in range(5):
        Vh = rng.standard_normal((d, k))
        e1 = oracle.subspace_error(Vh, Vs, B)
        e2 = oracle.subspace_error_definition(Vh, Vs, B)
        assert abs(e1 - e2) < 1e-12 and 0 <= e1 <= 1
    # exact subspace (any scaling / sign / order) -> 0
    assert abs(oracle.subspace_error(Vs[:, ::-1] * np.array([2.0, -1.0, 0.5]), Vs, B)) < 1e-12
    # B-orthogonal complement -> 1
    _, Vall = oracle.gep_topk(A, B, d)
    assert abs(oracle.subspace_error(Vall[:, k:2 * k], Vs, B) - 1.0) < 1e-12


# --------------------------------------------------------------------------- #
# Update direction and Alg. 2                                                  #
# --------------------------------------------------------------------------- #

def _cca_data(rng, b=64, dx=5, dy=7):
    Z = rng.standard_normal((b, 3))
    X = Z @ rng.standard_normal((3, dx)) + 0.3 * rng.standard_normal((b, dx))
    Y = Z @ rng.standard_normal((3, dy)) + 0.3 * rng.standard_normal((b, dy))
    return X, Y


@pytest.mark.parametrize("kind", [oracle.KIND_CCA, oracle.KIND_GENERAL, oracle.KIND_LDA,
                                  oracle.KIND_ICA])
def test_minibatch_products_equal_dense_matrices(kind):
    """The per-row sums of the minibatch step equal the step taken with the
    minibatch's A and B formed explicitly (Sec. 1 definitions)."""
    rng = np.random.default_rng(10 + kind)
    k = 3
    labels = None
    if kind == oracle.KIND_CCA:
        X, Y = _cca_data(rng)
        pb = oracle.Problem(kind, k, 5, 7, rho=1e-6)
    elif kind == oracle.KIND_GENERAL:
        X, Y = rng.standard_normal((50, 9)), rng.standard_normal((50, 9)) * 2
        pb = oracle.Problem(kind, k, 9, 9, eps_reg=1e-2)
    elif kind == oracle.KIND_ICA:
        X, Y = rng.laplace(size=(50, 9)) @ rng.standard_normal((9, 9)), None
        pb = oracle.Problem(kind, k, 9, 0, eps_reg=1e-2)
    else:
        means = rng.standard_normal((4, 9))
        labels = rng.integers(0, 4, size=50)
        X, Y = means[labels] + 0.5 * rng.standard_normal((50, 9)), None
        pb = oracle.Problem(kind, k, 9, eps_reg=1e-2, class_means=means,
                            class_priors=np.array([0.1, 0.2, 0.3, 0.4]))
    A, B = oracle.problem_matrices(pb, X, Y, labels)
    V0 = rng.standard_normal((pb.d, k))
    s1 = oracle.State.init(V0)
    s1.G = s1.G + 0.1 * rng.standard_normal(s1.G.shape)
    s2 = oracle.State(V=s1.V.copy(), G=s1.G.copy(), ema_a=np.zeros(k), ema_b=np.zeros(k))
    _, g1 = oracle.gamma_step(pb, s1, X, Y, 0.1, 0.3, labels=labels, return_grad=True)
    _, g2 = oracle.gamma_step_dense(pb, s2, A, B, 0.1, 0.3, return_grad=True)
    assert np.abs(g1 - g2).max() < 1e-12 * np.abs(g2).max()
    assert np.abs(s1.V - s2.V).max() < 1e-13
    assert np.abs(s1.G - s2.G).max() < 1e-13


def test_tangency_of_update_direction():
    """With one minibatch for every term, v_i^T grad_i = 0 for any V, G."""
    rng = np.random.default_rng(5)
    X, Y = _cca_data(rng)
    pb = oracle.Problem(oracle.KIND_CCA, 4, 5, 7, rho=1e-6)
    st = oracle.State.init(rng.standard_normal((12, 4)))
    st.G = rng.standard_normal(st.G.shape)
    V = st.V.copy()
    _, g = oracle.gamma_step(pb, st, X, Y, 0.1, 0.5, return_grad=True)
    for i in range(4):
        assert abs(V[:, i] @ g[:, i]) <= 1e-13 * np.linalg.norm(g[:, i])


def test_fixed_point_at_exact_solution():
    """Lemma (right fixed point): with exact expectations, unit-norm exact
    eigenvectors and [Bv] = Bv, the update direction vanishes."""
    rng = np.random.default_rng(6)
    d, k = 10, 4
    A, B = _rand_sym(rng, d) + 3 * np.eye(d), _rand_spd(rng, d)
    lam, Vs = oracle.gep_topk(A, B, k)
    pb = oracle.Problem(oracle.KIND_GENERAL, k, d, d, rho=0.0)
    st = oracle.State.init(Vs)
    st.G = B @ st.V
    V0 = st.V.copy()
    _, g = oracle.gamma_step_dense(pb, st, A, B, 0.5, 1.0, return_grad=True)
    assert np.abs(g).max() < 1e-13 * np.abs(A).max()
    assert np.abs(st.V - V0).max() < 1e-13


def test_reduces_to_mu_eigengame_when_b_is_identity():
    """Proposition (equivalence when B = I): with G = V the direction is
    (I - v_i v_i^T)[A v_i - sum_{j<i} (v_i^T A v_j) v_j]."""
    rng = np.random.default_rng(7)
    d, k = 9, 4
    A = _rand_sym(rng, d)
    pb = oracle.Problem(oracle.KIND_GENERAL, k, d, d, rho=0.0)
    st = oracle.State.init(rng.standard_normal((d, k)))
    V = st.V.copy()
    _, g = oracle.gamma_step_dense(pb, st, A, np.eye(d), 0.1, 1.0, return_grad=True)
    for i in range(k):
        vi = V[:, i]
        u = A @ vi - sum((vi @ A @ V[:, j]) * V[:, j] for j in range(i))
        ref = u - vi * (vi @ u)
        assert np.abs(g[:, i] - ref).max() < 1e-13 * max(1, np.abs(ref).max())


def test_utility_gradient_finite_differences_and_steepest_ascent():
    """Gradient lemma against central differences of the utility; with exact
    parents and [Bv] = Bv the update direction equals <v_i,Bv_i>^2/2 times
    the utility gradient (steepest-ascent lemma)."""
    rng = np.random.default_rng(8)
    d, k = 8, 3
    A, B = _rand_sym(rng, d) + 2 * np.eye(d), _rand_spd(rng, d)
    lam, Vs = oracle.gep_topk(A, B, k)
    V = _unit(Vs.copy())
    V[:, k - 1] = _unit(rng.standard_normal((d, 1)))[:, 0]  # last player arbitrary
    i = k - 1
    g = oracle.utility_grad(A, B, V, i)
    h = 1e-6
    fd = np.zeros(d)
    for f in range(d):
        Vp, Vm = V.copy(), V.copy()
        Vp[f, i] += h
        Vm[f, i] -= h
        fd[f] = (oracle.utility(A, B, Vp, i) - oracle.utility(A, B, Vm, i)) / (2 * h)
    assert np.abs(fd - g).max() < 1e-6 * np.abs(g).max()
    pb = oracle.Problem(oracle.KIND_GENERAL, k, d, d, rho=0.0)
    st = oracle.State(V=V.copy(), G=B @ V, ema_a=np.zeros(k), ema_b=np.zeros(k))
    _, gt = oracle.gamma_step_dense(pb, st, A, B, 0.0, 0.0, return_grad=True)
    vi = V[:, i]
    scale = (vi @ B @ vi) ** 2 / 2
    assert np.abs(gt[:, i] - scale * g).max() < 1e-12 * np.abs(gt[:, i]).max()


def test_utility_equals_deflated_rayleigh_quotient():
    """Deflation proposition: with exact parents u_i equals the Rayleigh
    quotient of (I - sum_{j<i} B v_j v_j^T / ||v_j||_B^2) A."""
    rng = np.random.default_rng(9)
    d, k = 8, 3
    A, B = _rand_sym(rng, d), _rand_spd(rng, d)
    lam, Vs = oracle.gep_topk(A, B, k)
    V = _unit(Vs.copy())
    for _ in range(3):
        V[:, k - 1] = rng.standard_normal(d)
        D = np.eye(d)
        for j in range(k - 1):
            vj = Vs[:, j]
            D -= np.outer(B @ vj, vj) / (vj @ B @ vj)
        At = D @ A
        vi = V[:, k - 1]
        assert abs(oracle.utility(A, B, V, k - 1) - (vi @ At @ vi) / (vi @ B @ vi)) < 1e-12


def test_alg2_with_exact_auxiliary_equals_alg1():
    """With [Bv] reset to the exact B v before each iteration and rho = 0,
    Alg. 2 on exact matrices takes exactly Alg. 1's step."""
    rng = np.random.default_rng(11)
    d, k = 10, 4
    A, B = _rand_sym(rng, d), _rand_spd(rng, d)
    pb = oracle.Problem(oracle.KIND_GENERAL, k, d, d, rho=0.0)
    st = oracle.State.init(rng.standard_normal((d, k)))
    V1 = st.V.copy()
    for t in range(1, 6):
        st.G = B @ st.V
        oracle.gamma_step_dense(pb, st, A, B, 0.05, 1.0)
        V1 = oracle.alg1_step(A, B, V1, 0.05)
        assert np.abs(st.V - V1).max() < 1e-13


def _problem_with_gap(rng, d):
    A = _rand_sym(rng, d)
    B = _rand_spd(rng, d)
    return A, B


def test_full_batch_convergence_alg1_and_alg2():
    """Convergence theorem (deterministic case): Alg. 1, and Alg. 2 on exact
    matrices, reach the exact top-k to 1e-10 subspace error."""
    rng = np.random.default_rng(12)
    d, k = 8, 3
    lam_p = np.array([5.0, 3.0, 2.0, 0.5, 0.3, 0.2, 0.1, 0.05])
    B = _rand_spd(rng, d)
    L = np.linalg.cholesky(B)
    Q, _ = np.linalg.qr(rng.standard_normal((d, d)))
    A = L @ Q @ np.diag(lam_p) @ Q.T @ L.T
    lam, Vs = oracle.gep_topk(A, B, k)
    assert np.allclose(lam, lam_p[:k])
    V = _unit(rng.standard_normal((d, k)))
    for t in range(1, 4001):
        V = oracle.alg1_step(A, B, V, 0.05)
    assert oracle.subspace_error(V, Vs, B) < 1e-10
    pb = oracle.Problem(oracle.KIND_GENERAL, k, d, d, rho=0.0)
    st = oracle.State.init(rng.standard_normal((d, k)))
    for t in range(1, 4001):
        oracle.gamma_step_dense(pb, st, A, B, 0.05, 0.5)
    assert oracle.subspace_error(st.V, Vs, B) < 1e-10
    # the Rayleigh-quotient readout converges to the eigenvalues
    assert np.allclose(st.eigvals(), lam, rtol=1e-8)


def test_stochastic_tiny_cca_reaches_1e3():
    """Alg. 2 on the tiny CCA pool (n = 10,000, b = 128, 2000 steps) reaches
    1e-3 subspace error against the pool's exact solution."""
    gen, pool = synth.tiny_cca_pool(0)
    pb = oracle.Problem(oracle.KIND_CCA, 4, 8, 8, rho=1e-6)
    A, B = oracle.problem_matrices(pb, pool.X, pool.Y)
    lam, Vs = oracle.gep_topk(A, B, 4)
    # empirical correlations close to the population ones rho/1.01
    assert np.abs(lam - gen.rho / 1.01).max() < 0.03
    st = oracle.State.init(synth.initial_players(16, 4, 0))
    for t in range(1, 2001):
        X, Y = pool.batch(t, 128)
        oracle.gamma_step(pb, st, X, Y, oracle.eta(oracle.SCHED_INV, t, 1.0, t0=200.0), 1.0)
    assert oracle.subspace_error(st.V, Vs, B) < 1e-3


def test_clip_counts_and_guards():
    """<v_j, [Bv]_j> below rho is clipped (Alg. 2): with G = -V every player
    is clipped and the step stays finite."""
    rng = np.random.default_rng(13)
    X, Y = _cca_data(rng)
    pb = oracle.Problem(oracle.KIND_CCA, 3, 5, 7, rho=1e-3)
    st = oracle.State.init(rng.standard_normal((12, 3)))
    st.G = -st.V
    n = oracle.gamma_step(pb, st, X, Y, 0.1, 0.5)
    assert n == 3
    assert np.all(np.isfinite(st.V))
    assert np.allclose(np.linalg.norm(st.V, axis=0), 1.0)


def test_adam_first_step_closed_form():
    """First Adam step: bias-corrected moments are g and g^2, so the step is
    eta * g / (|g| + eps) before the retraction."""
    rng = np.random.default_rng(14)
    X, Y = _cca_data(rng)
    pb = oracle.Problem(oracle.KIND_CCA, 3, 5, 7, rho=1e-6, optimizer=oracle.OPT_ADAM)
    st = oracle.State.init(rng.standard_normal((12, 3)), adam=True)
    V = st.V.copy()
    pb_sgd = oracle.Problem(oracle.KIND_CCA, 3, 5, 7, rho=1e-6)
    st2 = oracle.State.init(V)
    _, g = oracle.gamma_step(pb_sgd, st2, X, Y, 0.0, 0.5, return_grad=True)
    oracle.gamma_step(pb, st, X, Y, 0.01, 0.5)
    ref = _unit(V + 0.01 * g / (np.abs(g) + 1e-8))
    assert np.abs(st.V - ref).max() < 1e-12


def test_schedules_closed_forms():
    e = oracle.eta
    assert e(oracle.SCHED_CONST, 17, 0.3) == 0.3
    assert abs(e(oracle.SCHED_INV, 200, 1.0, t0=200) - 0.5) < 1e-15
    # warmup + harmonic decay with the neural-CCA table's values: Delta = 0
    kw = dict(eta0=1e-4, eta_T=1e-6, t_c=1e5, T=1e7)
    assert abs(e(oracle.SCHED_WARMUP_HARMONIC, 5e4, **kw) - 0.5e-4) < 1e-18
    assert abs(e(oracle.SCHED_WARMUP_HARMONIC, 1e5, **kw) - 1e-4) < 1e-18
    assert abs(e(oracle.SCHED_WARMUP_HARMONIC, 1e7, **kw) - 1e-6) < 1e-18
    assert abs(e(oracle.SCHED_WARMUP_HARMONIC, 2e5, **kw) - 0.5e-4) < 1e-18
    # a case with nonzero Delta still hits both ends
    kw = dict(eta0=1e-2, eta_T=1e-3, t_c=100, T=1000)
    assert abs(e(oracle.SCHED_WARMUP_HARMONIC, 100, **kw) - 1e-2) < 1e-15
    assert abs(e(oracle.SCHED_WARMUP_HARMONIC, 1000, **kw) - 1e-3) < 1e-15


# --------------------------------------------------------------------------- #
# Alg. 3 (smooth stochastic gamma-EigenGame, App. G)                          #
# --------------------------------------------------------------------------- #

def _z_for(pb, s):
    """z with exp(log rho + (log nu - log rho) sigmoid(z)) = s, rho < s < nu."""
    f = (np.log(s) - np.log(pb.rho)) / (np.log(pb.nu) - np.log(pb.rho))
    return np.log(f / (1.0 - f))


def test_smooth_estimate_closed_forms():
    """The log-space estimate lies strictly between rho and nu, equals their
    geometric mean at z = 0 (the initial value), tends to rho and nu at the
    ends, and its logarithm is affine in sigmoid(z)."""
    pb = oracle.Problem(oracle.KIND_CCA, 3, 5, 7, rho=1e-4, nu=25.0, smooth=True)
    assert np.isclose(oracle.smooth_estimate(pb, [0.0])[0], np.sqrt(1e-4 * 25.0), rtol=1e-14)
    z = np.linspace(-30, 30, 61)
    s = oracle.smooth_estimate(pb, z)
    assert np.all(s > pb.rho * (1 - 1e-12)) and np.all(s < pb.nu * (1 + 1e-12))
    assert np.all(np.diff(s) > 0)
    assert np.isclose(s[0], pb.rho, rtol=1e-9) and np.isclose(s[-1], pb.nu, rtol=1e-9)
    sg = 1 / (1 + np.exp(-z))
    assert np.allclose(np.log(s), np.log(1e-4) + np.log(25.0 / 1e-4) * sg, atol=1e-12)
    # the inverse used by the tests below
    assert np.allclose(oracle.smooth_estimate(pb, _z_for(pb, np.array([0.01, 0.3, 7.0]))),
                       [0.01, 0.3, 7.0], rtol=1e-12)


def test_smooth_z_step_is_descent_on_squared_mismatch():
    """One Alg. 3 iteration with eta = 0 moves z_i by gamma times minus the
    derivative of (c_i - s(z_i))^2 / 2, c_i = <v_i, [Bv]_i> of the iteration:
    checked against central finite differences of that loss (which also
    fixes the sign: the estimate moves toward c_i)."""
    rng = np.random.default_rng(21)
    d, k = 9, 4
    A, B = _rand_sym(rng, d), _rand_spd(rng, d)
    pb = oracle.Problem(oracle.KIND_GENERAL, k, d, d, rho=1e-3, nu=50.0, smooth=True)
    st = oracle.State.init(rng.standard_normal((d, k)))
    st.G = B @ st.V + 0.1 * rng.standard_normal((d, k))
    st.z = rng.uniform(-2, 2, k)
    c = np.einsum("fi,fi->i", st.V, st.G)
    z0 = st.z.copy()
    gamma = 0.3
    oracle.gamma_step_dense(pb, st, A, B, 0.0, gamma)
    h = 1e-6

    def loss(z):
        return 0.5 * (c - oracle.smooth_estimate(pb, z)) ** 2

    fd = (loss(z0 + h) - loss(z0 - h)) / (2 * h)
    assert np.allclose(st.z - z0, -gamma * fd, rtol=1e-6, atol=1e-12)
    assert np.all(np.sign(st.z - z0) == np.sign(c - oracle.smooth_estimate(pb, z0)))


def test_smooth_reduces_to_clip_when_estimate_matches():
    """When z_j gives s_j = <v_j, [Bv]_j> (inside (rho, nu)), Alg. 3 takes
    exactly Alg. 2's step and z stays put (its gradient vanishes)."""
    rng = np.random.default_rng(22)
    X, Y = _cca_data(rng, b=96)
    p2 = oracle.Problem(oracle.KIND_CCA, 4, 5, 7, rho=1e-6)
    p3 = oracle.Problem(oracle.KIND_CCA, 4, 5, 7, rho=1e-6, nu=100.0, smooth=True)
    V0 = rng.standard_normal((12, 4))
    s2, s3 = oracle.State.init(V0), oracle.State.init(V0)
    G = s2.V * rng.uniform(0.5, 2.0, 4) + 0.05 * rng.standard_normal((12, 4))
    s2.G, s3.G = G.copy(), G.copy()
    c = np.einsum("fi,fi->i", s3.V, s3.G)
    assert np.all(c > 1e-6)
    s3.z = _z_for(p3, c)
    z0 = s3.z.copy()
    _, g2 = oracle.gamma_step(p2, s2, X, Y, 0.2, 0.5, return_grad=True)
    _, g3 = oracle.gamma_step(p3, s3, X, Y, 0.2, 0.5, return_grad=True)
    assert np.abs(g2 - g3).max() < 1e-12 * np.abs(g2).max()
    assert np.abs(s2.V - s3.V).max() < 1e-13 and np.abs(s2.G - s3.G).max() < 1e-13
    assert np.abs(s3.z - z0).max() < 1e-12


def test_smooth_tangency_and_fixed_point():
    """The smooth estimate changes only the parents' scaling: v_i^T grad_i = 0
    for any z, and at the exact solution with [Bv] = Bv and s_j = v_j^T B v_j
    the direction and the z step vanish."""
    rng = np.random.default_rng(23)
    X, Y = _cca_data(rng)
    pb = oracle.Problem(oracle.KIND_CCA, 4, 5, 7, rho=1e-6, nu=10.0, smooth=True)
    st = oracle.State.init(rng.standard_normal((12, 4)))
    st.G = rng.standard_normal(st.G.shape)
    st.z = rng.uniform(-3, 3, 4)
    V = st.V.copy()
    _, g = oracle.gamma_step(pb, st, X, Y, 0.1, 0.5, return_grad=True)
    for i in range(4):
        assert abs(V[:, i] @ g[:, i]) <= 1e-13 * np.linalg.norm(g[:, i])
    d, k = 10, 4
    A, B = _rand_sym(rng, d) + 3 * np.eye(d), _rand_spd(rng, d)
    lam, Vs = oracle.gep_topk(A, B, k)
    pb = oracle.Problem(oracle.KIND_GENERAL, k, d, d, rho=1e-6, nu=1e3, smooth=True)
    st = oracle.State.init(Vs)
    st.G = B @ st.V
    st.z = _z_for(pb, np.einsum("fi,fi->i", st.V, st.G))
    z0, V0 = st.z.copy(), st.V.copy()
    _, g = oracle.gamma_step_dense(pb, st, A, B, 0.5, 1.0, return_grad=True)
    assert np.abs(g).max() < 1e-13 * np.abs(A).max()
    assert np.abs(st.V - V0).max() < 1e-13 and np.abs(st.z - z0).max() < 1e-10


def test_smooth_estimate_tracks_b_norm_and_alg3_converges():
    """With eta = 0 on exact matrices, [Bv] -> B v and the estimate s_j ->
    v_j^T B v_j (the stationary point of the z dynamics); with a decaying
    eta, Alg. 3 on exact matrices reaches the exact top-k (the convergence
    the paper conjectures) to 1e-9 subspace error.  The z step is gradient
    descent on (c - s(z))^2 / 2 at rate gamma, stable only while
    gamma s'(z)^2 < 2 near the target; (rho, nu) = (0.1, 10) with gamma = 0.1
    keeps it there (gamma = 0.5 with (1e-3, 1e2) overshoots into the flat
    tail at rho)."""
    rng = np.random.default_rng(24)
    d, k = 8, 3
    lam_p = np.array([5.0, 3.0, 2.0, 0.5, 0.3, 0.2, 0.1, 0.05])
    B = _rand_spd(rng, d)
    L = np.linalg.cholesky(B)
    Q, _ = np.linalg.qr(rng.standard_normal((d, d)))
    A = L @ Q @ np.diag(lam_p) @ Q.T @ L.T
    lam, Vs = oracle.gep_topk(A, B, k)
    pb = oracle.Problem(oracle.KIND_GENERAL, k, d, d, rho=0.1, nu=10.0, smooth=True)
    st = oracle.State.init(rng.standard_normal((d, k)))
    for t in range(1, 3001):
        oracle.gamma_step_dense(pb, st, A, B, 0.0, 0.1)
    bnorm = np.einsum("fi,fg,gi->i", st.V, B, st.V)
    assert np.allclose(oracle.smooth_estimate(pb, st.z), bnorm, rtol=1e-9)
    st = oracle.State.init(rng.standard_normal((d, k)))
    for t in range(1, 6001):
        oracle.gamma_step_dense(pb, st, A, B, 0.05, 0.1)
    assert oracle.subspace_error(st.V, Vs, B) < 1e-9


# --------------------------------------------------------------------------- #
# Running-mean centring of non-zero-mean streams                              #
# --------------------------------------------------------------------------- #

def test_centering_removes_a_known_offset_and_tracks_the_mean():
    """With the running means equal to the streams' offsets, a shifted stream
    takes exactly the step of the unshifted one without centring (shift
    invariance of the covariances); the means move toward the minibatch
    means at rate gamma (closed form after n identical minibatches)."""
    rng = np.random.default_rng(31)
    X, Y = _cca_data(rng, b=80)
    mx, my = rng.normal(3.0, 1.0, 5), rng.normal(-2.0, 1.0, 7)
    p0 = oracle.Problem(oracle.KIND_CCA, 3, 5, 7, rho=1e-6)
    p1 = oracle.Problem(oracle.KIND_CCA, 3, 5, 7, rho=1e-6, center=True)
    V0 = rng.standard_normal((12, 3))
    s0, s1 = oracle.State.init(V0), oracle.State.init(V0)
    s1.mu_x, s1.mu_y = mx.copy(), my.copy()
    _, g0 = oracle.gamma_step(p0, s0, X, Y, 0.2, 0.5, return_grad=True)
    _, g1 = oracle.gamma_step(p1, s1, X + mx, Y + my, 0.2, 0.5, return_grad=True)
    assert np.abs(g0 - g1).max() < 1e-12 * np.abs(g0).max()
    assert np.abs(s0.V - s1.V).max() < 1e-13 and np.abs(s0.G - s1.G).max() < 1e-13
    # mean update: mu <- mu + gamma (xbar - mu), xbar of the shifted minibatch
    assert np.allclose(s1.mu_x, mx + 0.5 * (X.mean(0) + mx - mx), atol=1e-14)
    st = oracle.State.init(V0)
    xbar = (X + mx).mean(0)
    for n in range(1, 6):
        oracle.gamma_step(p1, st, X + mx, Y + my, 0.0, 0.3)
        assert np.allclose(st.mu_x, (1 - 0.7 ** n) * xbar, atol=1e-13)


def test_centered_stochastic_cca_reaches_centered_solution():
    """A tiny CCA pool shifted by large per-feature offsets: with centring,
    Alg. 2 reaches 1e-3 subspace error against the exact solution of the
    pool's covariances (centred); without it the offsets dominate the
    uncentred second moments and the run misses that solution by far."""
    gen, pool = synth.tiny_cca_pool(0)
    rng = np.random.default_rng(32)
    off_x, off_y = rng.normal(0, 2.0, 8), rng.normal(0, 2.0, 8)
    PX, PY = pool.X + off_x, pool.Y + off_y
    Xc, Yc = PX - PX.mean(0), PY - PY.mean(0)
    pb = oracle.Problem(oracle.KIND_CCA, 4, 8, 8, rho=1e-6, center=True)
    A, B = oracle.problem_matrices(pb, Xc, Yc)
    lam, Vs = oracle.gep_topk(A, B, 4)
    st = oracle.State.init(synth.initial_players(16, 4, 0))
    plain = oracle.State.init(synth.initial_players(16, 4, 0))
    p0 = oracle.Problem(oracle.KIND_CCA, 4, 8, 8, rho=1e-6)
    for t in range(1, 3001):
        idx = pool.indices(t, 128)
        eta = oracle.eta(oracle.SCHED_INV, t, 1.0, t0=200.0)
        oracle.gamma_step(pb, st, PX[idx], PY[idx], eta, 0.5)
        if t <= 1000:
            oracle.gamma_step(p0, plain, PX[idx], PY[idx], eta, 0.5)
    assert oracle.subspace_error(st.V, Vs, B) < 1e-3
    assert oracle.subspace_error(plain.V, Vs, B) > 1e-2
    assert np.abs(st.mu_x - PX.mean(0)).max() < 0.1



# --------------------------------------------------------------------------- #
# ICA (kurtosis form of Sec. 1)                                               #
# --------------------------------------------------------------------------- #

def test_ica_moments_match_the_kurtosis_closed_form():
    """For an orthogonal mixing of independent unit-variance sources with
    excess kurtoses kappa, E[<x, x> x x^T] - tr(C) C - 2 C^2 = M diag(kappa) M^T
    and C = I (fourth moments of independent sources); the empirical matrices
    of 400,000 samples agree within sampling error (0.04 observed; dropping
    any one of the three terms moves them by >= 2), and the exact top-3 are
    the three kurtoses."""
    g = synth.ICAMixed(d=8, kurtosis=(9.0, 4.0, 1.0), seed=3)
    X = g.sample(400_000, np.random.default_rng(1))
    pb = oracle.Problem(oracle.KIND_ICA, 3, 8, 0)
    A, B = oracle.problem_matrices(pb, X)
    A0, B0 = targets.ica_population_AB(g)
    assert np.abs(A - A0).max() < 0.15 and np.abs(B - B0).max() < 0.02
    lam, Vs = oracle.gep_topk(A, B, 3)
    assert np.allclose(lam, [9.0, 4.0, 1.0], atol=0.15)
    lam0, V0 = targets.ica_planted_topk(g, 3)
    assert oracle.subspace_error(Vs, V0, B0) < 1e-3


def test_ica_stochastic_recovers_the_most_kurtotic_sources():
    """Alg. 2 on minibatches of the ICA stream (one minibatch for every
    term) finds the mixing columns of the three most kurtotic sources."""
    g = synth.ICAMixed(d=8, kurtosis=(9.0, 4.0, 1.0), seed=3)
    lam0, V0 = targets.ica_planted_topk(g, 3)
    pb = oracle.Problem(oracle.KIND_ICA, 3, 8, 0, rho=1e-6)
    st = oracle.State.init(synth.initial_players(8, 3, 0))
    for t in range(1, 3001):
        X, _ = g.batch(t, 512)
        oracle.gamma_step(pb, st, X, None, oracle.eta(oracle.SCHED_INV, t, 0.05, t0=300.0), 0.5)
    err = oracle.subspace_error(st.V, V0, np.eye(8))
    assert err < 1e-2, err


def test_fixed_point_does_not_depend_on_the_minibatch_size():
    """Minibatches of 32, 128 and 512 rows of the same pool lead Alg. 2 to
    the same solution (the pool's exact one), only with different noise: the
    one-minibatch estimate of the products does not move the fixed point."""
    gen, pool = synth.tiny_cca_pool(0)
    pb = oracle.Problem(oracle.KIND_CCA, 4, 8, 8, rho=1e-6)
    A, B = oracle.problem_matrices(pb, pool.X, pool.Y)
    lam, Vs = oracle.gep_topk(A, B, 4)
    finals = []
    for b in (32, 128, 512):
        st = oracle.State.init(synth.initial_players(16, 4, 0))
        for t in range(1, 4001):
            X, Y = pool.batch(t, b)
            oracle.gamma_step(pb, st, X, Y, oracle.eta(oracle.SCHED_INV, t, 1.0, t0=200.0), 1.0)
        err = oracle.subspace_error(st.V, Vs, B)
        assert err < 5e-3, (b, err)
        finals.append(err)
    # the noise, not the limit, depends on b: larger minibatches end closer
    assert finals[2] < finals[0]


# --------------------------------------------------------------------------- #
# LDA (Sec. 1): the reduced c x c route and the stochastic step              #
# --------------------------------------------------------------------------- #

@pytest.mark.parametrize("priors", [None, (0.1, 0.15, 0.2, 0.25, 0.3)])
def test_lda_reduced_solve_equals_dense_exact_solver(priors):
    """The c x c reduced route (A = N^T N has rank <= c - 1, so v lies in
    B^{-1} N^T) gives the same top c - 1 pairs as the dense Cholesky + Jacobi
    route and scipy's generalized eigh on the population matrices, with
    v^T B v = I and A v = lambda B v; the c-th eigenvalue of the dense problem
    is zero (rank c - 1)."""
    g = synth.LDAClasses(d=40, c=5, r=7, seed=3)
    eps = 1e-4
    A, B = targets.lda_population_AB(g, eps, priors)
    lam, V = targets.lda_reduced_topk(g, 4, eps, priors)
    lam_d, Vd = oracle.gep_topk(A, B, 5)
    assert np.allclose(lam, lam_d[:4], rtol=1e-11, atol=0)
    assert abs(lam_d[4]) < 1e-10 * lam_d[0]
    assert oracle.subspace_error(V, Vd[:, :4], B) < 1e-13
    for i in range(4):  # distinct eigenvalues: the vectors agree up to sign
        s = np.sign(V[:, i] @ B @ Vd[:, i])
        assert np.abs(V[:, i] - s * Vd[:, i]).max() < 1e-10 * np.abs(V[:, i]).max()
    assert np.abs(V.T @ B @ V - np.eye(4)).max() < 1e-12
    assert np.abs(A @ V - (B @ V) * lam[None, :]).max() < 1e-11 * np.abs(A).max()
    w = sla.eigh(A, B, eigvals_only=True)[::-1]
    assert np.allclose(lam, w[:4], rtol=1e-10, atol=0)


def test_lda_reduced_solve_at_the_benchmark_width():
    """At d = 65536 the reduced route still satisfies A v = lambda B v and
    v^T B v = I, checked through products with the class means only (A is
    never formed): A v = N^T (N v)."""
    g = synth.LDAClasses()
    eps = 1e-4
    lam, V = targets.lda_reduced_topk(g, 9, eps)
    pri = np.full(g.c, 1.0 / g.c)
    N = np.sqrt(pri)[:, None] * (g.means - pri @ g.means)
    Bd = g.sigma ** 2 + eps
    AV = N.T @ (N @ V)
    BV = Bd[:, None] * V
    assert np.abs(AV - BV * lam[None, :]).max() < 1e-10 * np.abs(AV).max()
    assert np.abs(V.T @ BV - np.eye(9)).max() < 1e-11
    assert np.all(np.diff(lam) < 0) and lam[-1] > 1.0


def test_lda_stochastic_alg2_reaches_the_reduced_solution():
    """Alg. 2 on fresh labelled minibatches of the Gaussian classes, with the
    oracle's minibatch within-class B (samples minus their class mean) and
    between-class A (given means and priors), converges to the exact top
    c - 1 subspace of the population problem.  A wrong reading of either
    matrix (e.g. B from uncentred samples) converges elsewhere."""
    g = synth.LDAClasses(d=24, c=4, r=6, seed=5)
    eps = 1e-4
    lam, Vs = targets.lda_reduced_topk(g, 3, eps)
    A, B = targets.lda_population_AB(g, eps)
    pb = oracle.Problem(oracle.KIND_LDA, 3, 24, eps_reg=eps, class_means=g.means, rho=1e-6)
    st = oracle.State.init(synth.initial_players(24, 3, 5))
    for t in range(1, 2501):
        X, lab = g.batch(t, 256, dtype=np.float64)
        oracle.gamma_step(pb, st, X, None, oracle.eta(oracle.SCHED_INV, t, 0.05, t0=200.0), 0.5,
                          labels=lab)
    err = oracle.subspace_error(st.V, Vs, B)
    assert err < 3e-3, err
    # the same run with B taken from the raw (uncentred) samples: the class
    # means enter B and the top subspace changes
    Xs, _ = g.batch(0, 4096, dtype=np.float64)
    Bw = Xs.T @ Xs / 4096 + eps * np.eye(24)
    assert oracle.subspace_error(oracle.gep_topk(A, Bw, 3)[1], Vs, B) > 10 * err


def test_subspace_error_diagonal_b_equals_dense_diagonal():
    """The diagonal form of the metric (B given by its diagonal) equals the
    dense form with np.diag(B), and App. A's definition."""
    rng = np.random.default_rng(21)
    d, k = 30, 4
    bd = np.exp(rng.uniform(-2, 2, d))
    Vs = rng.standard_normal((d, k))
    L = np.linalg.cholesky(Vs.T @ (bd[:, None] * Vs))
    Vs = Vs @ np.linalg.inv(L).T  # B-orthonormal
    Vh = Vs + 0.1 * rng.standard_normal((d, k))
    e1 = oracle.subspace_error(Vh, Vs, bd)
    e2 = oracle.subspace_error(Vh, Vs, np.diag(bd))
    e3 = oracle.subspace_error_definition(Vh, Vs, np.diag(bd))
    assert abs(e1 - e2) < 1e-14 and abs(e1 - e3) < 1e-12 and 0.0 < e1 < 1.0



# --------------------------------------------------------------------------- #
# The activation-like CCA: population covariances and the top-k route        #
# --------------------------------------------------------------------------- #

def test_relu_pair_cov_special_cases_and_quadrature():
    """Covariance of relu of jointly Gaussian pairs: E[relu(a)^2] = s^2/2
    (so the variance is s^2 (1/2 - 1/(2 pi))); independent pairs have zero
    covariance; relu(a) relu(-a) = 0, so a perfectly anti-correlated pair
    has covariance -E relu(a) E relu(-a); a generic pair agrees with direct
    numerical integration of the bivariate normal density."""
    from scipy import integrate
    sa, sb = np.array([1.3]), np.array([0.7])
    v = targets.relu_pair_cov(np.array([[1.3 * 1.3]]), sa, sa)[0, 0]
    assert abs(v - 1.69 * (0.5 - 0.5 / np.pi)) < 1e-14
    assert abs(targets.relu_pair_cov(np.array([[0.0]]), sa, sb)[0, 0]) < 1e-15
    anti = targets.relu_pair_cov(np.array([[-1.3 * 0.7]]), sa, sb)[0, 0]
    assert abs(anti + 1.3 * 0.7 / (2 * np.pi)) < 1e-14
    for c in (0.35, -0.6, 0.9):
        cab = c * 1.3 * 0.7

        q = np.sqrt(1 - c * c)

        def f(z2, z1):  # on the region a > 0, b > 0 the integrand is smooth
            a = 1.3 * z1
            b = 0.7 * (c * z1 + q * z2)
            return a * b * np.exp(-0.5 * (z1 * z1 + z2 * z2)) / (2 * np.pi)

        e_ab, _ = integrate.dblquad(f, 0.0, 12.0, lambda z1: -c * z1 / q, 12.0,
                                    epsabs=1e-13, epsrel=1e-12)
        ref = e_ab - (1.3 / np.sqrt(2 * np.pi)) * (0.7 / np.sqrt(2 * np.pi))
        got = targets.relu_pair_cov(np.array([[cab]]), sa, sb)[0, 0]
        assert abs(got - ref) < 1e-11, (c, got, ref)


def test_activation_cca_population_matches_a_large_sample():
    """The closed-form covariances of the activation-like views agree with
    the empirical covariances of 400,000 drawn pairs (statistical, 5 sigma
    of the sampling error) and the views have mean zero."""
    g = synth.CCAActivation(dx=6, dy=5, r=4, seed=2)
    Sxx, Syy, Sxy = targets.cca_activation_population(g)
    X, Y = g.sample(400_000, np.random.default_rng(9), dtype=np.float64)
    n = X.shape[0]
    for M, E in ((Sxx, X.T @ X / n), (Syy, Y.T @ Y / n), (Sxy, X.T @ Y / n)):
        scale = np.sqrt(np.outer(np.diag(Sxx if M is not Syy else Syy),
                                 np.diag(Syy if M is not Sxx else Sxx)))
        assert np.abs(E - M).max() < 5 * 3 * scale.max() / np.sqrt(n)
    assert np.abs(X.mean(axis=0)).max() < 5 * np.sqrt(np.diag(Sxx).max() / n)


@pytest.mark.parametrize("dxy", [64, 256])
def test_activation_cca_topk_route_equals_dense_solver(dxy):
    """The singular-pair route (block subspace iteration on K K^T with a
    Jacobi Rayleigh-Ritz step) gives the top canonical correlations and
    B-orthonormal vectors of the dense Cholesky + Jacobi solve of the same
    population problem: eigenvalues to 1e-10, subspaces to 1e-10."""
    g = synth.CCAActivation(dx=dxy, dy=dxy, r=16, seed=1)
    Sxx, Syy, Sxy = targets.cca_activation_population(g)
    k = 8
    sig, V = targets.cca_topk_subspace(Sxx, Syy, Sxy, k, tol=1e-12)
    A, B = oracle.cca_matrices(Sxx, Syy, Sxy)
    lam, Vd = oracle.gep_topk(A, B, k)
    assert np.abs(sig - lam).max() < 1e-10
    assert abs(oracle.subspace_error(V, Vd, B)) < 1e-10
    assert np.abs(V.T @ B @ V - np.eye(k)).max() < 1e-10
    assert np.abs(A @ V - (B @ V) * sig[None, :]).max() < 1e-9 * np.abs(A).max()


@pytest.mark.slow
def test_activation_cca_topk_route_at_d1024_equals_dense_jacobi():
    """The same check on a d = 512 + 512 instance of the benchmark's
    activation-like generator (r = 64), the top 64-block included (about
    two minutes of dense Jacobi)."""
    g = synth.CCAActivation(dx=512, dy=512, seed=0)
    Sxx, Syy, Sxy = targets.cca_activation_population(g)
    sig, V = targets.cca_topk_subspace(Sxx, Syy, Sxy, 66, p=132, tol=1e-11)
    A, B = oracle.cca_matrices(Sxx, Syy, Sxy)
    lam, Vd = oracle.gep_topk(A, B, 66)
    assert np.abs(sig - lam).max() < 1e-10
    assert abs(oracle.subspace_error(V[:, :64], Vd[:, :64], B)) < 1e-10


def test_subspace_containment_error_properties():
    """Players inside the exact block give 0, players B-orthogonal to it 1,
    a block of the players' own size reduces to subspace_error, and a
    rotation of the players does not change it."""
    rng = np.random.default_rng(4)
    d, m, k = 20, 6, 3
    B = _rand_spd(rng, d)
    W = rng.standard_normal((d, d))
    L = np.linalg.cholesky(B)
    Q, _ = np.linalg.qr(W)
    Vall = np.linalg.solve(L.T, Q)  # B-orthonormal basis of R^d
    Vs = Vall[:, :m]
    inside = Vs @ rng.standard_normal((m, k))
    assert abs(oracle.subspace_containment_error(inside, Vs, B)) < 1e-13
    outside = Vall[:, m:m + k] @ rng.standard_normal((k, k))
    assert abs(oracle.subspace_containment_error(outside, Vs, B) - 1.0) < 1e-13
    Vh = rng.standard_normal((d, k))
    assert abs(oracle.subspace_containment_error(Vh, Vs[:, :k], B)
               - oracle.subspace_error(Vh, Vs[:, :k], B)) < 1e-13
    R = rng.standard_normal((k, k))
    assert abs(oracle.subspace_containment_error(Vh @ R, Vs, B)
               - oracle.subspace_containment_error(Vh, Vs, B)) < 1e-12
