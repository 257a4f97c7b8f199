"""Seeded synthetic workloads for the five benchmark shapes.

This module only DRAWS data: it holds none of the gamma-EigenGame
arithmetic and is imported by both the tests/oracle side and the benchmark.
Every array is a deterministic function of (seed, batch index).

Workloads (the paper's datasets are not available; these stand in with the
shapes of the benchmark configurations):

* ``CCAPlanted``   paired views with planted canonical correlations
                   (tiny CCA: d = 8 + 8, k = 4; medium CCA: d = 512 + 512,
                   k = 16, condition number 100 per view).
* ``CCAActivation`` activation-like paired views: ReLU of a shared Gaussian
                   latent through dense maps with log-normal feature scales
                   (d = 8192 + 8192).
* ``GeneralPlanted`` general SGEP instance with A = E[y y^T],
                   B = E[x x^T] + eps I and planted generalized eigenvalues.
* ``LDAClasses``   Gaussian classes with means on a random low-dimensional
                   subspace and diagonal within-class covariance.
* ``ICAMixed``     independent sources (Bernoulli-Gaussian with chosen
                   excess kurtosis, the rest Gaussian) under an orthogonal
                   mixing map (pre-whitened mixtures, the ICA problem).

Generator seeds: parameters use ``seed``, the minibatch stream uses
``(seed + 1, t)`` and the initial players ``seed + 2``.
"""
from __future__ import annotations

from dataclasses import dataclass, field
from typing import Optional, Tuple

import numpy as np


def _orth(rng: np.random.Generator, n: int, m: int) -> np.ndarray:
    """n x m matrix with orthonormal columns (QR of a Gaussian, signs fixed)."""
    q, r = np.linalg.qr(rng.standard_normal((n, m)))
    return q * np.sign(np.diag(r))[None, :]


def initial_players(d: int, k: int, seed: int) -> np.ndarray:
    """Gaussian draws for the players' starting points, (d, k), NOT normalised
    (each side normalises them itself)."""
    return np.random.default_rng(seed + 2).standard_normal((d, k))


@dataclass
class CCAPlanted:
    """x = Wx [z; e_x] + sigma n_x and y = Wy [z'; e_y] + sigma n_y, where the
    r latent pairs (z_i, z'_i) are standard normal with correlation rho_i and
    e, n are independent standard normal.  ``n_free`` extra latent noise
    dimensions per view; ``spread`` gives the singular values of the mixing
    maps as geomspace(1, spread, dx) (None: orthonormal columns)."""
    dx: int
    dy: int
    rho: np.ndarray
    sigma: float = 0.0
    n_free: int = 0
    spread: Optional[float] = None
    seed: int = 0
    Wx: np.ndarray = field(init=False, repr=False)
    Wy: np.ndarray = field(init=False, repr=False)

    def __post_init__(self):
        rng = np.random.default_rng(self.seed)
        self.rho = np.asarray(self.rho, dtype=np.float64)
        r = len(self.rho)
        cols = r + self.n_free
        assert cols <= min(self.dx, self.dy)
        self.Wx = _orth(rng, self.dx, cols)
        self.Wy = _orth(rng, self.dy, cols)
        if self.spread is not None:
            assert cols == self.dx == self.dy
            self.Wx = self.Wx * np.geomspace(1.0, self.spread, cols)[None, :]
            self.Wy = self.Wy * np.geomspace(1.0, self.spread, cols)[None, :]

    @property
    def d(self) -> int:
        return self.dx + self.dy

    def sample(self, n: int, rng: np.random.Generator) -> Tuple[np.ndarray, np.ndarray]:
        r = len(self.rho)
        z = rng.standard_normal((n, r))
        xi = rng.standard_normal((n, r))
        z2 = z * self.rho + xi * np.sqrt(1.0 - self.rho ** 2)
        ux = np.concatenate([z, rng.standard_normal((n, self.n_free))], axis=1)
        uy = np.concatenate([z2, rng.standard_normal((n, self.n_free))], axis=1)
        x = ux @ self.Wx.T
        y = uy @ self.Wy.T
        if self.sigma:
            x += self.sigma * rng.standard_normal((n, self.dx))
            y += self.sigma * rng.standard_normal((n, self.dy))
        return x, y

    def batch(self, t: int, b: int) -> Tuple[np.ndarray, np.ndarray]:
        """Fresh minibatch number t (float64)."""
        return self.sample(b, np.random.default_rng([self.seed + 1, t]))

    def sample_torch(self, n: int, t: int, device, dtype):
        """n fresh pairs drawn on `device` from a torch generator seeded by
        (seed, t), with the mixing maps in FP32 (same distribution as
        ``sample``, different values)."""
        import torch
        g = torch.Generator(device=device)
        g.manual_seed((int(self.seed) * 1_000_003 + 7919 * int(t) + 1) & ((1 << 63) - 1))
        f32 = torch.float32
        r = len(self.rho)
        rho = torch.from_numpy(self.rho).to(device=device, dtype=f32)
        z = torch.randn((n, r), generator=g, device=device, dtype=f32)
        xi = torch.randn((n, r), generator=g, device=device, dtype=f32)
        z2 = z * rho + xi * torch.sqrt(1.0 - rho * rho)
        ux = torch.cat([z, torch.randn((n, self.n_free), generator=g, device=device, dtype=f32)], 1)
        uy = torch.cat([z2, torch.randn((n, self.n_free), generator=g, device=device, dtype=f32)], 1)
        x = ux @ torch.from_numpy(self.Wx.T).to(device=device, dtype=f32)
        y = uy @ torch.from_numpy(self.Wy.T).to(device=device, dtype=f32)
        if self.sigma:
            x += self.sigma * torch.randn((n, self.dx), generator=g, device=device, dtype=f32)
            y += self.sigma * torch.randn((n, self.dy), generator=g, device=device, dtype=f32)
        return x.to(dtype), y.to(dtype)


def tiny_cca(seed: int = 0) -> CCAPlanted:
    """Two views of width 8 from 4 latent pairs with correlations
    0.9, 0.7, 0.5, 0.3, orthonormal mixing and 0.1 isotropic noise."""
    return CCAPlanted(8, 8, np.array([0.9, 0.7, 0.5, 0.3]), sigma=0.1, seed=seed)


def medium_cca(seed: int = 0) -> CCAPlanted:
    """Two views of width 512; 16 latent pairs with correlations linearly
    spaced 0.95 -> 0.2, the other 496 latent dimensions independent noise,
    mixing maps Q diag(geomspace(1, 0.1, 512)) (per-view condition 100)."""
    return CCAPlanted(512, 512, np.linspace(0.95, 0.2, 16), sigma=0.0, n_free=496, spread=0.1,
                      seed=seed)


@dataclass
class Pool:
    """A fixed finite dataset with i.i.d. minibatch indices drawn with
    replacement (used for the tiny CCA case: n = 10,000 pairs)."""
    X: np.ndarray
    Y: Optional[np.ndarray]
    seed: int
    labels: Optional[np.ndarray] = None

    def indices(self, t: int, b: int) -> np.ndarray:
        return np.random.default_rng([self.seed + 1, t]).integers(0, self.X.shape[0], size=b)

    def batch(self, t: int, b: int):
        idx = self.indices(t, b)
        Y = None if self.Y is None else self.Y[idx]
        return self.X[idx], Y


def tiny_cca_pool(seed: int = 0, n: int = 10_000) -> Tuple[CCAPlanted, Pool]:
    gen = tiny_cca(seed)
    X, Y = gen.sample(n, np.random.default_rng([seed, 7]))
    return gen, Pool(X, Y, seed)


@dataclass
class CCAActivation:
    """Activation-like paired views: a shared latent h ~ N(0, I_r), then
    x = Dx (relu(Wx h + xi) - mu_x), y = Dy (relu(Wy h + xi') - mu_y) with
    W Gaussian / sqrt(r), xi standard normal noise, D = diag(exp(N(0, 1)))
    (log-normal feature scales, sigma = 1) and mu the exact mean of the
    ReLU of a centred Gaussian of standard deviation s (mu = s / sqrt(2 pi)),
    so the views have mean zero."""
    dx: int = 8192
    dy: int = 8192
    r: int = 64
    seed: int = 0
    Wx: np.ndarray = field(init=False, repr=False)
    Wy: np.ndarray = field(init=False, repr=False)
    Dx: np.ndarray = field(init=False, repr=False)
    Dy: np.ndarray = field(init=False, repr=False)

    def __post_init__(self):
        rng = np.random.default_rng(self.seed)
        self.Wx = rng.standard_normal((self.dx, self.r)) / np.sqrt(self.r)
        self.Wy = rng.standard_normal((self.dy, self.r)) / np.sqrt(self.r)
        self.Dx = np.exp(rng.standard_normal(self.dx))
        self.Dy = np.exp(rng.standard_normal(self.dy))

    @property
    def d(self) -> int:
        return self.dx + self.dy

    def relu_means(self):
        sx = np.sqrt((self.Wx ** 2).sum(axis=1) + 1.0)
        sy = np.sqrt((self.Wy ** 2).sum(axis=1) + 1.0)
        return sx / np.sqrt(2 * np.pi), sy / np.sqrt(2 * np.pi)

    def sample(self, n: int, rng: np.random.Generator, dtype=np.float32):
        h = rng.standard_normal((n, self.r)).astype(np.float32)
        mx, my = self.relu_means()
        ux = h @ self.Wx.T.astype(np.float32) + rng.standard_normal((n, self.dx), dtype=np.float32)
        uy = h @ self.Wy.T.astype(np.float32) + rng.standard_normal((n, self.dy), dtype=np.float32)
        x = (np.maximum(ux, 0) - mx.astype(np.float32)) * self.Dx.astype(np.float32)
        y = (np.maximum(uy, 0) - my.astype(np.float32)) * self.Dy.astype(np.float32)
        return x.astype(dtype, copy=False), y.astype(dtype, copy=False)

    def batch(self, t: int, b: int, dtype=np.float32):
        return self.sample(b, np.random.default_rng([self.seed + 1, t]), dtype)

    def device_tables(self, device):
        """Maps, feature scales and ReLU means as FP32 device tensors (kept
        by the caller across calls of sample_torch)."""
        import torch
        f32 = torch.float32
        mx, my = self.relu_means()
        return tuple(torch.from_numpy(np.ascontiguousarray(a)).to(device=device, dtype=f32)
                     for a in (self.Wx.T, self.Wy.T, self.Dx, self.Dy, mx, my))

    def sample_torch(self, n: int, t: int, device, dtype, tables=None):
        """n fresh pairs drawn on `device` from a torch generator seeded by
        (seed, t), in FP32 (same distribution as ``sample``, different
        values), returned in `dtype`."""
        import torch
        g = torch.Generator(device=device)
        g.manual_seed((int(self.seed) * 1_000_003 + 7919 * int(t) + 3) & ((1 << 63) - 1))
        WxT, WyT, Dx, Dy, mx, my = tables if tables is not None else self.device_tables(device)
        f32 = torch.float32
        h = torch.randn((n, self.r), generator=g, device=device, dtype=f32)
        x = torch.randn((n, self.dx), generator=g, device=device, dtype=f32)
        x.addmm_(h, WxT).clamp_(min=0.0).sub_(mx).mul_(Dx)
        y = torch.randn((n, self.dy), generator=g, device=device, dtype=f32)
        y.addmm_(h, WyT).clamp_(min=0.0).sub_(my).mul_(Dy)
        return x.to(dtype), y.to(dtype)


class _FastOrth:
    """Dense random orthogonal d x d matrix Q = H2 H1 C Pi: Pi a signed random
    permutation (Pi[perm[j], j] = sign[j]), C the orthonormal DCT-II matrix
    C[i, j] = c_i cos(pi i (2 j + 1) / (2 d)) with c_0 = sqrt(1/d) and
    c_i = sqrt(2/d) otherwise, and H = I - 2 u u^T two random Householder
    reflections.  Every factor is orthogonal, so Q is; building it costs
    O(d^2) instead of the O(d^3) of a QR."""

    def __init__(self, rng: np.random.Generator, d: int):
        self.d = d
        self.perm = rng.permutation(d)
        self.sign = rng.choice([-1.0, 1.0], size=d)
        self.u = []
        for _ in range(2):
            u = rng.standard_normal(d)
            self.u.append(u / np.linalg.norm(u))

    def dense(self) -> np.ndarray:
        d = self.d
        i = np.arange(d)[:, None]
        j = self.perm[None, :]                    # column j of C Pi is C[:, perm[j]] sign[j]
        M = np.cos(np.pi * i * (2 * j + 1) / (2 * d)) * self.sign[None, :]
        M *= np.where(np.arange(d) == 0, np.sqrt(1.0 / d), np.sqrt(2.0 / d))[:, None]
        for u in self.u:
            M -= 2.0 * np.outer(u, u @ M)
        return M

    def dense_torch(self, device, dtype):
        """The same matrix built with torch on `device` (rounded to dtype)."""
        import torch
        d = self.d
        i = torch.arange(d, device=device, dtype=torch.float64)[:, None]
        j = torch.from_numpy(self.perm).to(device=device, dtype=torch.float64)[None, :]
        M = torch.cos(np.pi * i * (2 * j + 1) / (2 * d))
        M *= torch.from_numpy(self.sign).to(device)[None, :]
        c = torch.full((d, 1), np.sqrt(2.0 / d), dtype=torch.float64, device=device)
        c[0, 0] = np.sqrt(1.0 / d)
        M *= c
        for u in self.u:
            ut = torch.from_numpy(u).to(device)
            M -= 2.0 * torch.outer(ut, ut @ M)
        return M.to(dtype)


@dataclass
class GeneralPlanted:
    """General SGEP instance of width d: x = Qx diag(sqrt(ax)) g with ax
    log-uniform in [0.1, 1]; B = E[x x^T] + eps I = L L^T; y = L O diag(sqrt(lam)) g'
    with O random orthogonal, so that A = E[y y^T] = L O diag(lam) O^T L^T and
    A v = lam B v holds exactly for v = L^{-T} O e_i.  The top ``k`` planted
    values are geomspace(10, 0.1, k), the rest uniform in [0.01, 0.05].

    ``mixing="haar"``: Qx and O Haar-distributed (QR of Gaussians), L the
    Cholesky factor of B (O(d^3)).  ``mixing="fast"``: Qx and O from
    ``_fast_orth`` and L = Qx diag(sqrt(ax + eps)), another square root of
    the same B (O(d^2 log d); used for the many-instance workload)."""
    d: int
    k: int = 8
    eps: float = 1e-3
    seed: int = 0
    mixing: str = "haar"
    Sx_half: np.ndarray = field(init=False, repr=False)
    lam: np.ndarray = field(init=False, repr=False)
    ax: np.ndarray = field(init=False, repr=False)
    Qx: np.ndarray = field(init=False, repr=False)

    def __post_init__(self):
        rng = np.random.default_rng(self.seed)
        d = self.d
        self._fx = self._fo = None
        if self.mixing == "fast":
            self._fx = _FastOrth(rng, d)
        else:
            self.Qx = _orth(rng, d, d)
        self.ax = np.exp(rng.uniform(np.log(0.1), np.log(1.0), size=d))
        if self.mixing == "fast":
            self._fo = _FastOrth(rng, d)
            self._Y_map = None
        else:
            self.Sx_half = self.Qx * np.sqrt(self.ax)[None, :]
            Bfull = (self.Qx * self.ax[None, :]) @ self.Qx.T + self.eps * np.eye(d)
            L = np.linalg.cholesky(Bfull)
            O = _orth(rng, d, d)
        lam = np.empty(d)
        lam[: self.k] = np.geomspace(10.0, 0.1, self.k)
        lam[self.k:] = rng.uniform(0.01, 0.05, size=d - self.k)
        self.lam = lam
        if self.mixing != "fast":
            self._Y_map = (L @ O) * np.sqrt(lam)[None, :]

    def __getattr__(self, name):
        # dense factors of the fast construction, formed on first use
        if name in ("Qx", "Sx_half") and self.__dict__.get("_fx") is not None:
            Q = self._fx.dense()
            self.__dict__["Qx"] = Q
            self.__dict__["Sx_half"] = Q * np.sqrt(self.ax)[None, :]
            return self.__dict__[name]
        raise AttributeError(name)

    @property
    def Y_map(self) -> np.ndarray:
        """L O diag(sqrt(lam)); for fast mixing L = Qx diag(sqrt(ax + eps)),
        formed on first use."""
        if self._Y_map is None:
            L = self.Qx * np.sqrt(self.ax + self.eps)[None, :]
            self._Y_map = (L @ self._fo.dense()) * np.sqrt(self.lam)[None, :]
        return self._Y_map

    def sample(self, n: int, rng: np.random.Generator, dtype=np.float64):
        x = rng.standard_normal((n, self.d)) @ self.Sx_half.T
        y = rng.standard_normal((n, self.d)) @ self.Y_map.T
        return x.astype(dtype, copy=False), y.astype(dtype, copy=False)

    def device_tables(self, device):
        """The dense factors Qx, O and the vectors ax, lam as FP32 device
        tensors (fast mixing; kept by the caller across calls of
        sample_torch)."""
        import torch
        assert self._fx is not None, "device tables need mixing='fast'"
        f32 = torch.float32
        return (self._fx.dense_torch(device, f32), self._fo.dense_torch(device, f32),
                torch.from_numpy(self.ax).to(device=device, dtype=f32),
                torch.from_numpy(self.lam).to(device=device, dtype=f32))

    def sample_torch(self, n: int, t: int, device, dtype, tables=None):
        """n fresh rows of x and y drawn on `device` (fast mixing only), from
        a torch generator seeded by (seed, t): x = Qx diag(sqrt(ax)) g and
        y = Qx diag(sqrt(ax + eps)) O diag(sqrt(lam)) g' with the dense
        factors built in FP32 on the device (``device_tables``).  Values
        differ from ``sample``, which uses numpy's generator."""
        import torch
        assert self._fx is not None, "sample_torch needs mixing='fast'"
        g = torch.Generator(device=device)
        g.manual_seed((int(self.seed) * 1_000_003 + int(t)) & ((1 << 63) - 1))
        f32 = torch.float32
        Q, O, ax, lam = tables if tables is not None else self.device_tables(device)
        gx = torch.randn((n, self.d), generator=g, device=device, dtype=f32)
        gy = torch.randn((n, self.d), generator=g, device=device, dtype=f32)
        x = (gx * ax.sqrt()) @ Q.T
        y = (((gy * lam.sqrt()) @ O.T) * (ax + self.eps).sqrt()) @ Q.T
        return x.to(dtype), y.to(dtype)

    def batch(self, t: int, b: int, dtype=np.float64):
        return self.sample(b, np.random.default_rng([self.seed + 1, t]), dtype)


def batched_dims(n: int = 256, lo: int = 64, hi: int = 2048, seed: int = 0) -> np.ndarray:
    """Instance widths d_i uniform on {lo..hi} for the batched workload."""
    return np.random.default_rng([seed, 11]).integers(lo, hi + 1, size=n)


def batched_general(n: int = 256, lo: int = 64, hi: int = 2048, k: int = 8, eps: float = 1e-3,
                    seed: int = 0, dims=None):
    """The many-instance workload: n ``GeneralPlanted`` instances with widths
    ``batched_dims`` (or ``dims``), fast mixing, instance i seeded
    (seed, 100 + i)."""
    dims = batched_dims(n, lo, hi, seed) if dims is None else np.asarray(dims)
    return [GeneralPlanted(int(di), k=k, eps=eps, seed=(seed << 16) + 100 + 2 * i, mixing="fast")
            for i, di in enumerate(dims)]


@dataclass
class LDAClasses:
    """c Gaussian classes in R^d with equal priors: means mu_c = U a_c with U
    (d x r) orthonormal and a_c ~ N(0, 4 I_r); within-class covariance
    diag(sigma_f^2) with sigma_f log-uniform in [0.3, 3]; labels uniform."""
    d: int = 65536
    c: int = 10
    r: int = 64
    seed: int = 0
    means: np.ndarray = field(init=False, repr=False)
    sigma: np.ndarray = field(init=False, repr=False)

    def __post_init__(self):
        rng = np.random.default_rng(self.seed)
        U = _orth(rng, self.d, self.r)
        a = 2.0 * rng.standard_normal((self.c, self.r))
        self.means = a @ U.T
        self.sigma = np.exp(rng.uniform(np.log(0.3), np.log(3.0), size=self.d))

    def sample(self, n: int, rng: np.random.Generator, dtype=np.float32):
        lab = rng.integers(0, self.c, size=n).astype(np.int32)
        x = self.means[lab].astype(np.float32) + (
            rng.standard_normal((n, self.d), dtype=np.float32) * self.sigma.astype(np.float32))
        return x.astype(dtype, copy=False), lab

    def batch(self, t: int, b: int, dtype=np.float32):
        return self.sample(b, np.random.default_rng([self.seed + 1, t]), dtype)

    def device_tables(self, device):
        """The class means and per-feature standard deviations as FP32
        device tensors (kept by the caller across calls of sample_torch)."""
        import torch
        return (torch.from_numpy(self.means).to(device=device, dtype=torch.float32),
                torch.from_numpy(self.sigma).to(device=device, dtype=torch.float32))

    def sample_torch(self, n: int, t: int, device, dtype, tables=None, out=None):
        """n fresh labelled rows drawn on `device`, seeded by (seed, t): the
        class counts are multinomial(n, uniform) (host generator), the rows
        come grouped by class (a minibatch is an unordered sample, so this is
        the distribution of n i.i.d. uniform labels), and each row is
        mu_label + sigma * g with g from a torch generator, formed in FP32 and
        rounded once to `dtype` (same distribution as ``sample``, different
        values).  Returns (x in `dtype`, int32 labels on `device`); `out`
        (n x d, `dtype`) receives x when given."""
        import torch
        g = torch.Generator(device=device)
        g.manual_seed((int(self.seed) * 1_000_003 + 7919 * int(t) + 5) & ((1 << 63) - 1))
        means, sig = tables if tables is not None else self.device_tables(device)
        counts = np.random.default_rng([self.seed + 3, int(t)]).multinomial(
            n, np.full(self.c, 1.0 / self.c))
        noise = torch.randn((n, self.d), generator=g, device=device, dtype=torch.float32)
        x = out if out is not None else torch.empty((n, self.d), device=device, dtype=dtype)
        lab = torch.empty((n,), device=device, dtype=torch.int32)
        r0 = 0
        for cls, m in enumerate(counts.tolist()):
            if m:
                torch.addcmul(means[cls:cls + 1], noise[r0:r0 + m], sig, out=x[r0:r0 + m])
                lab[r0:r0 + m].fill_(cls)
                r0 += m
        return x, lab


@dataclass
class ICAMixed:
    """x = M s with M (d x d) orthogonal and independent unit-variance sources
    s: source i < len(kurtosis) is Bernoulli-Gaussian, g * z / sqrt(p_i) with
    g ~ N(0, 1), z ~ Bernoulli(p_i), p_i = 3 / (kurtosis_i + 3), whose excess
    kurtosis is kurtosis_i; the other sources are N(0, 1)."""
    d: int = 1024
    kurtosis: Tuple[float, ...] = tuple(np.linspace(20.0, 2.0, 16))
    seed: int = 0
    M: np.ndarray = field(init=False, repr=False)
    p: np.ndarray = field(init=False, repr=False)

    def __post_init__(self):
        rng = np.random.default_rng(self.seed)
        self.M = _orth(rng, self.d, self.d)
        self.p = 3.0 / (np.asarray(self.kurtosis, dtype=np.float64) + 3.0)

    def sample(self, n: int, rng: np.random.Generator, dtype=np.float64):
        m = len(self.p)
        S = rng.standard_normal((n, self.d))
        z = rng.random((n, m)) < self.p[None, :]
        S[:, :m] = S[:, :m] * z / np.sqrt(self.p)[None, :]
        return (S @ self.M.T).astype(dtype, copy=False)

    def batch(self, t: int, b: int, dtype=np.float64):
        X = self.sample(b, np.random.default_rng([self.seed + 1, t]), dtype)
        return X, None

    def sample_torch(self, n: int, t: int, device, dtype):
        """n fresh rows drawn on `device` from a torch generator seeded by
        (seed, t), M in FP32 (same distribution as ``sample``)."""
        import torch
        g = torch.Generator(device=device)
        g.manual_seed((int(self.seed) * 1_000_003 + 7919 * int(t) + 5) & ((1 << 63) - 1))
        f32 = torch.float32
        m = len(self.p)
        S = torch.randn((n, self.d), generator=g, device=device, dtype=f32)
        p = torch.from_numpy(self.p).to(device=device, dtype=f32)
        z = (torch.rand((n, m), generator=g, device=device, dtype=f32) < p).to(f32)
        S[:, :m] = S[:, :m] * z / torch.sqrt(p)
        return (S @ torch.from_numpy(self.M.T).to(device=device, dtype=f32)).to(dtype)


# ---------------------------------------------------------------------------
# Narrow storage formats of the minibatch (input preparation, shared by the
# tests, the oracle's inputs and the benchmark; no method arithmetic).
# ---------------------------------------------------------------------------

def bf16_bits(x: np.ndarray) -> np.ndarray:
    """BF16 encoding (round to nearest, ties to even) of float32 values, as
    uint16 bit patterns.  Inputs are finite."""
    u = np.ascontiguousarray(x, dtype=np.float32).view(np.uint32).astype(np.uint64)
    return ((u + 0x7FFF + ((u >> 16) & 1)) >> 16).astype(np.uint16)


def bf16_value(bits: np.ndarray) -> np.ndarray:
    """Exact float64 value of BF16 bit patterns."""
    u = (np.asarray(bits, dtype=np.uint16).astype(np.uint32) << 16)
    return u.view(np.float32).astype(np.float64)


def _e4m3_table() -> np.ndarray:
    """Values of the OCP FP8 e4m3 codes 0x00 .. 0x7E (sign bit clear): 4-bit
    exponent with bias 7, 3-bit mantissa, subnormals at exponent 0; 0x7F is
    NaN and there is no infinity."""
    codes = np.arange(0x7F)
    e, m = codes >> 3, codes & 7
    return np.where(e == 0, m / 8.0 * 2.0 ** -6, (1.0 + m / 8.0) * 2.0 ** (e - 7.0))


E4M3_VALUES = _e4m3_table()
E4M3_MAX = float(E4M3_VALUES[-1])  # 448


def e4m3_encode(y: np.ndarray) -> np.ndarray:
    """OCP e4m3 codes of y: round to nearest (ties to the even code),
    saturating at +-448."""
    y = np.asarray(y, dtype=np.float64)
    a = np.minimum(np.abs(y), E4M3_MAX)
    hi = np.clip(np.searchsorted(E4M3_VALUES, a), 1, len(E4M3_VALUES) - 1)
    lo = hi - 1
    dlo, dhi = a - E4M3_VALUES[lo], E4M3_VALUES[hi] - a
    pick_hi = (dhi < dlo) | ((dhi == dlo) & (hi % 2 == 0))
    code = np.where(pick_hi, hi, lo).astype(np.uint8)
    return np.where(y < 0, code | 0x80, code).astype(np.uint8)


def e4m3_value(codes: np.ndarray) -> np.ndarray:
    """Exact float64 value of e4m3 codes (0x7F / 0xFF are NaN)."""
    c = np.asarray(codes, dtype=np.uint8)
    mag = c & 0x7F
    v = np.where(mag == 0x7F, np.nan, E4M3_VALUES[np.minimum(mag, 0x7E)])
    return np.where(c & 0x80, -v, v)


def fp8_column_scales(X: np.ndarray) -> np.ndarray:
    """Per-column scales s_c = max_r |X[r, c]| / 448 (float32) from a
    calibration prefix, so X / s maps onto the full e4m3 range; an all-zero
    column gets scale 1."""
    amax = np.abs(np.asarray(X, dtype=np.float64)).max(axis=0)
    s = np.where(amax > 0, amax / E4M3_MAX, 1.0).astype(np.float32)
    return s


def fp8_quantize(X: np.ndarray, scales: np.ndarray) -> np.ndarray:
    """e4m3 codes of X / scales (column-wise), saturating."""
    return e4m3_encode(np.asarray(X, dtype=np.float64) / scales.astype(np.float64)[None, :])


def fp8_dequantize(codes: np.ndarray, scales: np.ndarray) -> np.ndarray:
    """Exact float64 values code * scale (products of a 4-bit and a 24-bit
    significand are exact in float64)."""
    return e4m3_value(codes) * scales.astype(np.float64)[None, :]
