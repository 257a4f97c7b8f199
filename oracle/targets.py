"""Exact targets of the synthetic workloads -- TEST INFRASTRUCTURE.

Population matrices A and B of each generator in ``synth`` (derived from the
generator's definition), and closed-form top-k solutions where the
construction plants them.  The generic route is ``oracle.gep_topk``."""
from __future__ import annotations

import numpy as np

from . import cca_matrices, jacobi_eigh


def cca_population(gen):
    """Population covariances of ``synth.CCAPlanted``:
    Sxx = Wx Wx^T + sigma^2 I, Syy likewise, Sxy = Wx[:, :r] diag(rho) Wy[:, :r]^T."""
    r = len(gen.rho)
    Sxx = gen.Wx @ gen.Wx.T + gen.sigma ** 2 * np.eye(gen.dx)
    Syy = gen.Wy @ gen.Wy.T + gen.sigma ** 2 * np.eye(gen.dy)
    Sxy = (gen.Wx[:, :r] * gen.rho[None, :]) @ gen.Wy[:, :r].T
    return Sxx, Syy, Sxy


def cca_population_AB(gen):
    return cca_matrices(*cca_population(gen))


def cca_planted_topk(gen, k: int):
    """Closed-form top-k of the noiseless square-mixing CCA generator
    (sigma = 0, Wx and Wy square and invertible): the canonical correlations
    are the planted rho (descending) with B-orthonormal vectors
    v_i = [Wx^{-T} e_i ; Wy^{-T} e_i] / sqrt(2)."""
    assert gen.sigma == 0.0 and gen.Wx.shape[0] == gen.Wx.shape[1]
    order = np.argsort(-gen.rho)[:k]
    E = np.eye(gen.dx)[:, order]
    Vx = np.linalg.solve(gen.Wx.T, E)
    Vy = np.linalg.solve(gen.Wy.T, E)
    return gen.rho[order].copy(), np.vstack([Vx, Vy]) / np.sqrt(2.0)


def general_population_AB(gen):
    """A = E[y y^T] = Ymap Ymap^T and B = E[x x^T] + eps I of ``synth.GeneralPlanted``."""
    A = gen.Y_map @ gen.Y_map.T
    B = gen.Sx_half @ gen.Sx_half.T + gen.eps * np.eye(gen.d)
    return A, B


def general_planted_topk(gen, k: int):
    """Planted top-k: with L O = Ymap diag(lam^{-1/2}), v_i = (L O)^{-T} e_i,
    which is B-orthonormal and satisfies A v_i = lam_i B v_i."""
    LO = gen.Y_map / np.sqrt(gen.lam)[None, :]
    order = np.argsort(-gen.lam)[:k]
    E = np.eye(gen.d)[:, order]
    return gen.lam[order].copy(), np.linalg.solve(LO.T, E)


def ica_population_AB(gen):
    """Kurtosis-form ICA matrices of ``synth.ICAMixed`` (orthogonal mixing,
    independent unit-variance sources with excess kurtosis kappa_i):
    E[||s||^2 s s^T] = diag(kappa) + (d + 2) I, so with C = M M^T = I,
    A = M (diag(kappa) + (d + 2) I) M^T - d I - 2 I = M diag(kappa) M^T and
    B = I."""
    kap = np.zeros(gen.d)
    kap[:len(gen.kurtosis)] = gen.kurtosis
    return (gen.M * kap[None, :]) @ gen.M.T, np.eye(gen.d)


def ica_planted_topk(gen, k: int):
    """Top-k of the population ICA problem: the mixing columns of the k most
    kurtotic sources, eigenvalues their excess kurtoses (unit vectors; B = I)."""
    kap = np.asarray(gen.kurtosis, dtype=np.float64)
    order = np.argsort(-kap)[:k]
    return kap[order].copy(), gen.M[:, order].copy()


def lda_population_AB(gen, eps: float, priors=None):
    """Population matrices of ``synth.LDAClasses`` (Sec. 1, LDA as a GEP):
    A = sum_c pi_c (mu_c - mubar)(mu_c - mubar)^T with mubar = sum_c pi_c mu_c
    (between-class), B = diag(sigma_f^2) + eps I (within-class covariance of
    the generator plus the ridge).  Dense d x d: small d only."""
    pri = _lda_priors(gen, priors)
    Mt = gen.means - pri @ gen.means
    A = Mt.T @ (pri[:, None] * Mt)
    B = np.diag(gen.sigma ** 2 + eps)
    return A, B


def _lda_priors(gen, priors):
    if priors is None:
        return np.full(gen.c, 1.0 / gen.c)
    p = np.asarray(priors, dtype=np.float64)
    assert p.shape == (gen.c,) and np.all(p > 0)
    return p


def lda_reduced_topk(gen, k: int, eps: float, priors=None):
    """Exact top-k (k <= c - 1) generalized eigenpairs of the population LDA
    problem of ``synth.LDAClasses`` through its c x c reduced form.

    With N = diag(pi)^{1/2} (M - 1 mubar^T) (c x d), A = N^T N has rank at
    most c - 1, so every eigenvector of A v = lambda B v with lambda != 0 lies
    in B^{-1} N^T (the span of the class-mean directions after B^{-1}).
    Writing v = B^{-1} N^T u / sqrt(lambda) turns the problem into the
    symmetric c x c eigenproblem K u = lambda u with K = N B^{-1} N^T, and
    then A v = N^T K u / sqrt(lambda) = lambda B v and v^T B v = u^T K u /
    lambda = 1 (B-orthonormal).  B is diagonal for this generator, so the
    route costs O(c^2 d) and K's eigenproblem is solved by the oracle's
    cyclic Jacobi.  Returns (lam descending, V (d, k)), signs canonical
    (largest-magnitude component positive)."""
    pri = _lda_priors(gen, priors)
    if not 1 <= k <= gen.c - 1:
        raise ValueError("the between-class matrix has rank <= c - 1")
    Binv = 1.0 / (gen.sigma ** 2 + eps)
    N = np.sqrt(pri)[:, None] * (gen.means - pri @ gen.means)
    K = (N * Binv[None, :]) @ N.T
    K = 0.5 * (K + K.T)
    w, U = jacobi_eigh(K)
    order = np.argsort(-w, kind="stable")[:k]
    lam = w[order]
    if not np.all(lam > 0):
        raise ValueError("fewer than k positive between-class eigenvalues")
    V = (Binv[:, None] * (N.T @ U[:, order])) / np.sqrt(lam)[None, :]
    return lam.copy(), _canon(V)


def _canon(V):
    """Each column's largest-magnitude component made positive (lowest index
    on ties)."""
    V = np.array(V, dtype=np.float64, copy=True)
    for i in range(V.shape[1]):
        j = int(np.argmax(np.abs(V[:, i])))
        if V[j, i] < 0:
            V[:, i] = -V[:, i]
    return V


def relu_pair_cov(C, sa, sb):
    """Covariance of relu(a) and relu(b) for zero-mean jointly Gaussian (a, b)
    with standard deviations sa, sb and covariance C (arrays broadcast as
    C[i, j], sa[i], sb[j]): E[relu(a) relu(b)] is the degree-1 arc-cosine
    kernel (Cho and Saul, 2009), sa sb (sin t + (pi - t) cos t) / (2 pi) with
    cos t = C / (sa sb), and E[relu(a)] = sa / sqrt(2 pi)."""
    S = np.outer(sa, sb)
    cos = np.clip(C / S, -1.0, 1.0)
    th = np.arccos(cos)
    K = S * (np.sin(th) + (np.pi - th) * cos) / (2.0 * np.pi)
    return K - S / (2.0 * np.pi)


def cca_activation_population(gen):
    """Population covariances of ``synth.CCAActivation``: with
    u_x = Wx h + xi (covariance Wx Wx^T + I), u_y = Wy h + xi' and
    cov(u_x, u_y) = Wx Wy^T, the views x = Dx (relu(u_x) - mu_x) and
    y = Dy (relu(u_y) - mu_y) have Sxx = Dx cov(relu(u_x)) Dx,
    Syy = Dy cov(relu(u_y)) Dy and Sxy = Dx cov(relu(u_x), relu(u_y)) Dy,
    each entry from ``relu_pair_cov``."""
    sx = np.sqrt((gen.Wx ** 2).sum(axis=1) + 1.0)
    sy = np.sqrt((gen.Wy ** 2).sum(axis=1) + 1.0)
    Cxx = gen.Wx @ gen.Wx.T
    Cxx[np.diag_indices_from(Cxx)] += 1.0
    Cyy = gen.Wy @ gen.Wy.T
    Cyy[np.diag_indices_from(Cyy)] += 1.0
    Sxx = relu_pair_cov(Cxx, sx, sx) * np.outer(gen.Dx, gen.Dx)
    Syy = relu_pair_cov(Cyy, sy, sy) * np.outer(gen.Dy, gen.Dy)
    Sxy = relu_pair_cov(gen.Wx @ gen.Wy.T, sx, sy) * np.outer(gen.Dx, gen.Dy)
    return Sxx, Syy, Sxy


def cca_topk_subspace(Sxx, Syy, Sxy, k: int, p: int = None, tol: float = 1e-10,
                      max_iter: int = 5000, seed: int = 0):
    """Exact top-k of the CCA problem (Sec. 1) through the singular pairs of
    K = Lx^{-1} Sxy Ly^{-T} (Lx Lx^T = Sxx, Ly Ly^T = Syy): the generalized
    eigenvalues of A v = lambda B v are +-sigma_i, and the B-orthonormal
    vectors of +sigma_i are v_i = [Lx^{-T} u_i; Ly^{-T} w_i] / sqrt(2) for the
    singular pair (u_i, w_i).  The top-k left singular vectors come from
    block subspace iteration on K K^T (block of p >= k columns, a QR
    re-orthonormalisation per iteration) with a Rayleigh-Ritz step by the
    oracle's cyclic Jacobi, until every leading residual
    ||K K^T u_i - sigma_i^2 u_i|| <= tol sigma_1^2.  Cholesky factors,
    triangular solves, QR and matrix products are library routines.
    Returns (sigma descending (k,), V (dx + dy, k)), signs canonical."""
    import scipy.linalg as sla
    dx = Sxx.shape[0]
    p = p or min(dx, 2 * k)
    Lx = np.linalg.cholesky(Sxx)
    Ly = np.linalg.cholesky(Syy)
    K = sla.solve_triangular(Lx, Sxy, lower=True)
    K = sla.solve_triangular(Ly, K.T, lower=True).T
    rng = np.random.default_rng(seed)
    Q, _ = np.linalg.qr(rng.standard_normal((dx, p)))
    it = 0
    while True:
        Z = K @ (K.T @ Q)
        Q, _ = np.linalg.qr(Z)
        KtQ = K.T @ Q
        M = KtQ.T @ KtQ
        w, U = jacobi_eigh(0.5 * (M + M.T))
        order = np.argsort(-w, kind="stable")
        w, U = w[order], U[:, order]
        Q = Q @ U
        KtQ = KtQ @ U
        R = K @ KtQ[:, :k] - Q[:, :k] * w[None, :k]
        it += 1
        if np.linalg.norm(R, axis=0).max() <= tol * w[0]:
            break
        if it >= max_iter:
            raise RuntimeError("subspace iteration did not converge")
    sig = np.sqrt(w[:k])
    Uk = Q[:, :k]
    Wk = KtQ[:, :k] / sig[None, :]
    Vx = sla.solve_triangular(Lx.T, Uk, lower=False)
    Vy = sla.solve_triangular(Ly.T, Wk, lower=False)
    return sig.copy(), _canon(np.vstack([Vx, Vy]) / np.sqrt(2.0))
