"""FP64 CPU oracle for the gamma-EigenGame hot path -- TEST INFRASTRUCTURE.

Only ``tests/``, ``__graft_entry__.smoke()`` and the CPU-baseline leg of
``bench.py`` may import this package.  The product library never imports,
links or calls it, and the two share no code: the oracle is plain C
(``sgep_oracle.c``, double precision throughout) plus the numpy helpers below,
each written from the paper (Gemp, Chen, McWilliams, ICLR 2023,
arXiv 2206.04993):

* ``gep_topk``       exact top-k of A v = lambda B v (Sec. 1 problem; App. A
                     reduction through a Cholesky factor of B and a cyclic
                     Jacobi eigensolve of L^{-1} A L^{-T}).
* ``gamma_step``     one iteration of Alg. 2 with M = 1, per player, with
                     explicit sums over the minibatch rows; Alg. 3 (smooth
                     estimate of <v_j, B v_j>, App. G) with Problem.smooth;
                     with Problem.center the minibatch is first centred by
                     running means of the views (Sec. 1 assumes zero-mean
                     data; App. H learns mean estimates beside the players).
* ``alg1_step``      one iteration of Alg. 1 (full batch, exact B y_j).
* ``utility``        the player utility of Sec. 2 (eq. util_new).
* ``utility_grad``   its gradient (App. B, gradient lemma).
* ``subspace_error`` the normalised subspace error of App. A.
* ``eta``            the step-size schedules.

Arrays of player vectors are numpy (d, k) arrays whose column i is player i.
"""
from __future__ import annotations

import ctypes
import os
from dataclasses import dataclass
from typing import Optional

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "liboracle.so")

KIND_CCA, KIND_GENERAL, KIND_LDA, KIND_ICA = 0, 1, 2, 3
OPT_SGD, OPT_ADAM = 0, 1
SCHED_CONST, SCHED_INV, SCHED_WARMUP_HARMONIC = 0, 1, 2

_lib = None


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            from . import build as _b
            _b.build()
        lib = ctypes.CDLL(LIB_PATH)
        D = ctypes.POINTER(ctypes.c_double)
        I32 = ctypes.POINTER(ctypes.c_int32)
        lib.oracle_cholesky.argtypes = [ctypes.c_int, D]
        lib.oracle_cholesky.restype = ctypes.c_int
        lib.oracle_jacobi_eigh.argtypes = [ctypes.c_int, D, D, D, ctypes.c_double, ctypes.c_int]
        lib.oracle_jacobi_eigh.restype = ctypes.c_int
        lib.oracle_gep_topk.argtypes = [ctypes.c_int, D, D, ctypes.c_int, D, D, ctypes.c_int]
        lib.oracle_gep_topk.restype = ctypes.c_int
        lib.oracle_eta.argtypes = [ctypes.c_int] + [ctypes.c_double] * 6
        lib.oracle_eta.restype = ctypes.c_double
        P = ctypes.POINTER(_Problem)
        lib.oracle_gamma_step.argtypes = [P, ctypes.c_int64, D, ctypes.c_int64, D, ctypes.c_int64,
                                          I32, D, D, ctypes.c_double, ctypes.c_double,
                                          ctypes.c_double, D, D, D, D, D, D]
        lib.oracle_gamma_step.restype = ctypes.c_int
        lib.oracle_gamma_step_dense.argtypes = [P, ctypes.c_int64, D, D, D, D, ctypes.c_double,
                                                ctypes.c_double, ctypes.c_double, D, D, D, D, D,
                                                D]
        lib.oracle_gamma_step_dense.restype = ctypes.c_int
        lib.oracle_alg1_step.argtypes = [ctypes.c_int64, ctypes.c_int, D, D, D, ctypes.c_double, D]
        lib.oracle_alg1_step.restype = ctypes.c_int
        lib.oracle_threads.argtypes = []
        lib.oracle_threads.restype = ctypes.c_int
        _lib = lib
    return _lib


class _Problem(ctypes.Structure):
    _fields_ = [
        ("kind", ctypes.c_int32), ("k", ctypes.c_int32), ("n_classes", ctypes.c_int32),
        ("optimizer", ctypes.c_int32), ("dx", ctypes.c_int64), ("dy", ctypes.c_int64),
        ("eps_reg", ctypes.c_double), ("rho", ctypes.c_double), ("adam_b1", ctypes.c_double),
        ("adam_b2", ctypes.c_double), ("adam_eps", ctypes.c_double),
        ("class_means", ctypes.POINTER(ctypes.c_double)),
        ("class_priors", ctypes.POINTER(ctypes.c_double)),
        ("smooth", ctypes.c_int32), ("pad", ctypes.c_int32), ("nu", ctypes.c_double),
    ]


def _dp(a: Optional[np.ndarray]):
    if a is None:
        return None
    assert a.dtype == np.float64 and a.flags["C_CONTIGUOUS"], "oracle arrays must be C-contiguous float64"
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


# --------------------------------------------------------------------------- #
# Dense linear algebra                                                        #
# --------------------------------------------------------------------------- #

def cholesky(B: np.ndarray) -> np.ndarray:
    """Lower Cholesky factor L of the SPD matrix B (B = L L^T)."""
    a = np.ascontiguousarray(B, dtype=np.float64).copy()
    rc = _load().oracle_cholesky(a.shape[0], _dp(a))
    if rc != 0:
        raise np.linalg.LinAlgError("matrix is not positive definite")
    return a


def jacobi_eigh(C: np.ndarray, tol: float = 1e-15, max_sweeps: int = 100):
    """Eigen-decomposition of the symmetric C by cyclic Jacobi.

    Returns (w, Z) unsorted, with C Z[:, c] = w[c] Z[:, c]."""
    n = C.shape[0]
    a = np.ascontiguousarray(C, dtype=np.float64).copy()
    w = np.zeros(n)
    z = np.zeros((n, n))
    rc = _load().oracle_jacobi_eigh(n, _dp(a), _dp(w), _dp(z), tol, max_sweeps)
    if rc < 0:
        raise RuntimeError("Jacobi did not converge")
    return w, z


def gep_topk(A: np.ndarray, B: np.ndarray, k: int, canon: bool = True):
    """Top-k generalized eigenpairs of A v = lambda B v (Sec. 1).

    Returns (lam, V): lam descending (k,), V (d, k) B-orthonormal
    (V^T B V = I, App. A B-orthogonality lemma)."""
    d = A.shape[0]
    A = np.ascontiguousarray(A, dtype=np.float64)
    B = np.ascontiguousarray(B, dtype=np.float64)
    lam = np.zeros(k)
    Vc = np.zeros((k, d))  # column-major d x k == row-major k x d
    rc = _load().oracle_gep_topk(d, _dp(A), _dp(B), k, _dp(lam), _dp(Vc), 1 if canon else 0)
    if rc == -1:
        raise np.linalg.LinAlgError("B is not positive definite")
    if rc != 0:
        raise RuntimeError(f"oracle_gep_topk failed ({rc})")
    return lam, Vc.T.copy()


def threads() -> int:
    """OpenMP threads the oracle's parallel regions use."""
    return int(_load().oracle_threads())


def eta(schedule: int, t: float, eta0: float, eta_T: float = 0.0, t0: float = 1.0,
        t_c: float = 1.0, T: float = 1.0) -> float:
    """Step size eta_t for iteration t = 1, 2, ... (see sgep_oracle.c)."""
    return float(_load().oracle_eta(schedule, float(t), eta0, eta_T, t0, t_c, T))


# --------------------------------------------------------------------------- #
# Alg. 2 / Alg. 1                                                              #
# --------------------------------------------------------------------------- #

@dataclass
class Problem:
    """Problem description shared by the step functions.

    kind: KIND_CCA (A, B the block matrices of Sec. 1), KIND_GENERAL
    (A = E[y y^T], B = E[x x^T] + eps I), KIND_LDA (A between-class,
    B within-class covariance + eps I) or KIND_ICA (the kurtosis form of
    Sec. 1: A = E[<x, x> x x^T] - tr(C) C - 2 C^2, B = C + eps I with
    C = E[x x^T]; data X only, dy = 0).  smooth: Alg. 3 instead of Alg. 2
    (the denominator <v_j, [Bv]_j> clipped at rho is replaced by
    exp(log rho + (log nu - log rho) sigmoid(z_j)), z_j updated at rate
    gamma toward <v_j, [Bv]_j>); nu bounds lambda_max(B) from above.
    center (CCA, GENERAL): each view is centred by its running mean before the
    iteration, and the mean moves toward the minibatch mean at rate gamma
    afterwards (State.mu_x, State.mu_y, zero at the start)."""
    kind: int
    k: int
    dx: int
    dy: int = 0
    eps_reg: float = 0.0
    rho: float = 1e-6
    optimizer: int = OPT_SGD
    adam_b1: float = 0.9
    adam_b2: float = 0.999
    adam_eps: float = 1e-8
    class_means: Optional[np.ndarray] = None   # (c, d)
    class_priors: Optional[np.ndarray] = None  # (c,)
    smooth: bool = False
    nu: float = 0.0
    center: bool = False

    @property
    def d(self) -> int:
        return self.dx + self.dy if self.kind == KIND_CCA else self.dx

    def _c(self):
        self._keep = []
        means = priors = None
        nc = 0
        if self.kind == KIND_LDA:
            m = np.ascontiguousarray(self.class_means, dtype=np.float64)
            nc = m.shape[0]
            p = (np.full(nc, 1.0 / nc) if self.class_priors is None
                 else np.ascontiguousarray(self.class_priors, dtype=np.float64))
            self._keep += [m, p]
            means, priors = _dp(m), _dp(p)
        return _Problem(self.kind, self.k, nc, self.optimizer, self.dx, self.dy, self.eps_reg,
                        self.rho, self.adam_b1, self.adam_b2, self.adam_eps, means, priors,
                        1 if self.smooth else 0, 0, self.nu)


@dataclass
class State:
    """Iterate of Alg. 2: V (unit columns), the auxiliary G = [Bv], the Adam
    moments, the iteration counter, the Rayleigh-quotient running means and
    the log-space variables z of Alg. 3 (zero at the start)."""
    V: np.ndarray
    G: np.ndarray
    m: Optional[np.ndarray] = None
    s2: Optional[np.ndarray] = None
    t: int = 0
    ema_a: Optional[np.ndarray] = None
    ema_b: Optional[np.ndarray] = None
    z: Optional[np.ndarray] = None
    mu_x: Optional[np.ndarray] = None
    mu_y: Optional[np.ndarray] = None

    @staticmethod
    def init(V0: np.ndarray, adam: bool = False) -> "State":
        """Alg. 2 initialisation: columns of V0 normalised to the unit sphere,
        [Bv]_i <- v_i."""
        V = np.asarray(V0, dtype=np.float64)
        V = V / np.sqrt((V * V).sum(axis=0, keepdims=True))
        k = V.shape[1]
        return State(V=V.copy(), G=V.copy(),
                     m=np.zeros_like(V) if adam else None,
                     s2=np.zeros_like(V) if adam else None,
                     t=0, ema_a=np.zeros(k), ema_b=np.zeros(k), z=np.zeros(k))

    def eigvals(self) -> np.ndarray:
        return self.ema_a / self.ema_b


def _colmajor(M: np.ndarray) -> np.ndarray:
    """(d, k) array -> contiguous buffer laid out d x k column-major."""
    return np.ascontiguousarray(M.T, dtype=np.float64)


def _z(pb: Problem, st: State) -> Optional[np.ndarray]:
    """The Alg. 3 variables, updated in place by the C step (None for Alg. 2)."""
    if not pb.smooth:
        return None
    if st.z is None:
        st.z = np.zeros(pb.k)
    st.z = np.ascontiguousarray(st.z, dtype=np.float64)
    return st.z


def smooth_estimate(pb: Problem, z: np.ndarray) -> np.ndarray:
    """Alg. 3's estimate of <v_j, B v_j>: exp(log rho + (log nu - log rho) sigmoid(z_j))."""
    sg = 1.0 / (1.0 + np.exp(-np.asarray(z, dtype=np.float64)))
    return np.exp(np.log(pb.rho) + (np.log(pb.nu) - np.log(pb.rho)) * sg)


def gamma_step(pb: Problem, st: State, X: np.ndarray, Y: Optional[np.ndarray], eta_t: float,
               gamma_t: float, labels: Optional[np.ndarray] = None, return_grad: bool = False):
    """One iteration of Alg. 2 (M = 1) on the minibatch (X, Y). Updates st in
    place; returns the number of clipped parents (and the update direction
    as a (d, k) array when return_grad)."""
    X = np.ascontiguousarray(X, dtype=np.float64)
    b = X.shape[0]
    Yc = np.ascontiguousarray(Y if Y is not None else X, dtype=np.float64)
    if pb.center:
        # centre each view by the running mean of the iteration's start, then
        # move the mean toward this minibatch's mean at rate gamma
        if pb.kind == KIND_LDA:
            raise NotImplementedError("centring applies to CCA and GENERAL")
        if st.mu_x is None:
            st.mu_x = np.zeros(X.shape[1])
        if st.mu_y is None:
            st.mu_y = np.zeros(Yc.shape[1])
        mx, my = st.mu_x, st.mu_y
        st.mu_x = mx + gamma_t * (X.mean(axis=0) - mx)
        st.mu_y = my + gamma_t * (Yc.mean(axis=0) - my)
        X = np.ascontiguousarray(X - mx[None, :])
        Yc = np.ascontiguousarray(Yc - my[None, :])
    lab = None
    if labels is not None:
        lab_arr = np.ascontiguousarray(labels, dtype=np.int32)
        lab = lab_arr.ctypes.data_as(ctypes.POINTER(ctypes.c_int32))
    V, G = _colmajor(st.V), _colmajor(st.G)
    adam = pb.optimizer == OPT_ADAM
    m = _colmajor(st.m) if adam else None
    s2 = _colmajor(st.s2) if adam else None
    ga = np.ascontiguousarray(st.ema_a, dtype=np.float64)
    gb = np.ascontiguousarray(st.ema_b, dtype=np.float64)
    grad = np.zeros((pb.k, pb.d)) if return_grad else None
    z = _z(pb, st)
    st.t += 1
    cp = pb._c()
    rc = _load().oracle_gamma_step(ctypes.byref(cp), b, _dp(X), X.shape[1], _dp(Yc), Yc.shape[1],
                                   lab, _dp(V), _dp(G), eta_t, gamma_t, float(st.t),
                                   _dp(m), _dp(s2), _dp(ga), _dp(gb), _dp(grad), _dp(z))
    if rc < 0:
        raise MemoryError("oracle_gamma_step")
    st.V, st.G, st.ema_a, st.ema_b = V.T.copy(), G.T.copy(), ga, gb
    if adam:
        st.m, st.s2 = m.T.copy(), s2.T.copy()
    return (rc, grad.T.copy()) if return_grad else rc


def gamma_step_dense(pb: Problem, st: State, A: np.ndarray, B: np.ndarray, eta_t: float,
                     gamma_t: float, return_grad: bool = False):
    """Alg. 2 iteration with exact A and B (full batch)."""
    A = np.ascontiguousarray(A, dtype=np.float64)
    B = np.ascontiguousarray(B, dtype=np.float64)
    V, G = _colmajor(st.V), _colmajor(st.G)
    adam = pb.optimizer == OPT_ADAM
    m = _colmajor(st.m) if adam else None
    s2 = _colmajor(st.s2) if adam else None
    ga = np.ascontiguousarray(st.ema_a, dtype=np.float64)
    gb = np.ascontiguousarray(st.ema_b, dtype=np.float64)
    grad = np.zeros((pb.k, A.shape[0])) if return_grad else None
    z = _z(pb, st)
    st.t += 1
    cp = pb._c()
    rc = _load().oracle_gamma_step_dense(ctypes.byref(cp), A.shape[0], _dp(A), _dp(B), _dp(V),
                                         _dp(G), eta_t, gamma_t, float(st.t), _dp(m), _dp(s2),
                                         _dp(ga), _dp(gb), _dp(grad), _dp(z))
    if rc < 0:
        raise MemoryError("oracle_gamma_step_dense")
    st.V, st.G, st.ema_a, st.ema_b = V.T.copy(), G.T.copy(), ga, gb
    if adam:
        st.m, st.s2 = m.T.copy(), s2.T.copy()
    return (rc, grad.T.copy()) if return_grad else rc


def alg1_step(A: np.ndarray, B: np.ndarray, V: np.ndarray, eta_t: float, return_grad: bool = False):
    """One iteration of Alg. 1; returns the new V (and the direction)."""
    A = np.ascontiguousarray(A, dtype=np.float64)
    B = np.ascontiguousarray(B, dtype=np.float64)
    d, k = V.shape
    Vc = _colmajor(V)
    grad = np.zeros((k, d)) if return_grad else None
    _load().oracle_alg1_step(d, k, _dp(A), _dp(B), _dp(Vc), eta_t, _dp(grad))
    return (Vc.T.copy(), grad.T.copy()) if return_grad else Vc.T.copy()


# --------------------------------------------------------------------------- #
# Utilities, gradient and metrics (numpy, written from the formulas)         #
# --------------------------------------------------------------------------- #

def utility(A: np.ndarray, B: np.ndarray, V: np.ndarray, i: int) -> float:
    """Player i's utility u_i(v_i | v_{j<i}) (Sec. 2, eq. util_new):
    generalized Rayleigh quotient minus sum_{j<i} <v_j,Av_j> <v_i,Bv_j>^2 /
    (<v_j,Bv_j>^2 <v_i,Bv_i>)."""
    vi = V[:, i]
    vBv = vi @ B @ vi
    u = (vi @ A @ vi) / vBv
    for j in range(i):
        vj = V[:, j]
        u -= (vj @ A @ vj) * (vi @ B @ vj) ** 2 / ((vj @ B @ vj) ** 2 * vBv)
    return float(u)


def utility_grad(A: np.ndarray, B: np.ndarray, V: np.ndarray, i: int) -> np.ndarray:
    """Gradient of u_i with respect to v_i (App. B gradient lemma, including
    the factor 2 and the common 1/<v_i,Bv_i>^2)."""
    vi = V[:, i]
    Avi, Bvi = A @ vi, B @ vi
    vBv, vAv = vi @ Bvi, vi @ Avi
    g = (vBv * Avi - vAv * Bvi) / vBv ** 2
    for j in range(i):
        vj = V[:, j]
        Bvj = B @ vj
        lam_j = (vj @ A @ vj) / (vj @ Bvj)
        g -= lam_j / (vj @ Bvj) * (vi @ Bvj) * (vBv * Bvj - (vi @ Bvj) * Bvi) / vBv ** 2
    return 2.0 * g


def subspace_error(Vhat: np.ndarray, Vstar: np.ndarray, B: np.ndarray) -> float:
    """Normalised subspace error of App. A in its Gram form.

    With Vstar B-orthonormal (Vstar^T B Vstar = I), W = B^{1/2} Vstar is
    orthonormal and 1 - tr(U* P)/k = 1 - tr(C^T G^{-1} C)/k where
    C = Vhat^T B Vstar and G = Vhat^T B Vhat.  The sign and scale of each
    column of Vhat do not matter.  A one-dimensional B is the diagonal of a
    diagonal B (large d)."""
    k = Vstar.shape[1]
    B = np.asarray(B)

    def mulB(M):
        return B[:, None] * M if B.ndim == 1 else B @ M

    C = Vhat.T @ mulB(Vstar)
    G = Vhat.T @ mulB(Vhat)
    return float(1.0 - np.trace(C.T @ np.linalg.solve(G, C)) / k)


def subspace_containment_error(Vhat: np.ndarray, Vstar: np.ndarray, B: np.ndarray) -> float:
    """App. A's normalised subspace error when the exact subspace is larger
    than the players' (Vstar: the m >= k columns of a B-orthonormal
    eigenspace block whose eigenvalues are separated from the rest, Vhat: k
    players): 1 - tr(U* P)/k with U* the B-projector on span(Vstar) and P the
    one on span(Vhat), i.e. the mean sin^2 of the angles between the players'
    subspace and the block in the B-inner product.  0 when span(Vhat) lies in
    span(Vstar), 1 when it is B-orthogonal to it; equal to subspace_error when
    m = k.  With C = Vhat^T B Vstar and G = Vhat^T B Vhat this is
    1 - tr(G^{-1} C C^T)/k.  B: a matrix, its diagonal (1-D), or a function
    applying B to a block of columns."""
    k = Vhat.shape[1]
    if callable(B):
        mulB = B
    else:
        B = np.asarray(B)

        def mulB(M):
            return B[:, None] * M if B.ndim == 1 else B @ M

    C = Vhat.T @ mulB(Vstar)
    G = Vhat.T @ mulB(Vhat)
    return float(1.0 - np.trace(np.linalg.solve(G, C @ C.T)) / k)


def subspace_error_definition(Vhat: np.ndarray, Vstar: np.ndarray, B: np.ndarray) -> float:
    """The same error written as App. A defines it: W holds the top-k
    eigenvectors of B^{-1/2} A B^{-1/2} (= B^{1/2} Vstar), What = B^{1/2} Vhat,
    U* = W W^+, P = What What^+, error = 1 - tr(U* P)/k.  Uses the symmetric
    square root of B from its eigen-decomposition."""
    w, Q = np.linalg.eigh(B)
    Bh = (Q * np.sqrt(w)) @ Q.T
    W = Bh @ Vstar
    Wh = Bh @ Vhat
    U = W @ np.linalg.pinv(W)
    P = Wh @ np.linalg.pinv(Wh)
    return float(1.0 - np.trace(U @ P) / Vstar.shape[1])


def cca_matrices(Sxx: np.ndarray, Syy: np.ndarray, Sxy: np.ndarray):
    """A and B of CCA (Sec. 1): A = [[0, Sxy], [Sxy^T, 0]], B = diag(Sxx, Syy)."""
    dx, dy = Sxx.shape[0], Syy.shape[0]
    A = np.zeros((dx + dy, dx + dy))
    A[:dx, dx:] = Sxy
    A[dx:, :dx] = Sxy.T
    B = np.zeros_like(A)
    B[:dx, :dx] = Sxx
    B[dx:, dx:] = Syy
    return A, B


def problem_matrices(pb: Problem, X: np.ndarray, Y: Optional[np.ndarray] = None,
                     labels: Optional[np.ndarray] = None):
    """Empirical A and B of a finite dataset (uncentred means, Sec. 1)."""
    X = np.asarray(X, dtype=np.float64)
    n = X.shape[0]
    if pb.kind == KIND_CCA:
        Y = np.asarray(Y, dtype=np.float64)
        return cca_matrices(X.T @ X / n, Y.T @ Y / n, X.T @ Y / n)
    if pb.kind == KIND_GENERAL:
        Y = np.asarray(Y, dtype=np.float64)
        return Y.T @ Y / n, X.T @ X / n + pb.eps_reg * np.eye(X.shape[1])
    if pb.kind == KIND_ICA:
        # kurtosis form of Sec. 1 with the empirical moments of the dataset
        C = X.T @ X / n
        nr = (X * X).sum(axis=1)
        K = (X * nr[:, None]).T @ X / n
        return K - np.trace(C) * C - 2.0 * C @ C, C + pb.eps_reg * np.eye(X.shape[1])
    means = np.asarray(pb.class_means, dtype=np.float64)
    c = means.shape[0]
    pri = np.full(c, 1.0 / c) if pb.class_priors is None else np.asarray(pb.class_priors)
    E = X - means[np.asarray(labels)]
    B = E.T @ E / n + pb.eps_reg * np.eye(X.shape[1])
    Mt = means - pri @ means
    A = Mt.T @ (pri[:, None] * Mt)
    return A, B
