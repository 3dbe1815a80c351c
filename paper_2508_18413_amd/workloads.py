"""Seeded synthetic inputs for the parallel-in-sequence MCMC workloads.

This module draws random numbers and target parameters only; it contains no
step of the sampler or of the Newton solver, so both the HIP path and the FP64
oracle can consume its arrays without sharing any of the method's arithmetic.

Recipe (one ``SeedSequence([seed, stream])`` per independent stream, so the
target does not change with T and every chain of a batch can be regenerated
on its own):

* stream 0 -- target parameters (logistic-regression design, Gaussian
  precision, funnel log-scale);
* stream 1 -- initial states;
* stream 2 -- burn-in noise and uniforms (3 MALA steps, Appendix B.1);
* stream 3 (+chain index * 16) -- per-step Gaussian noise xi_t, row-major [T, D];
* stream 4 (+chain index * 16) -- per-step uniforms u_t.

Uniforms are u = (k + 1/2) 2^-23 with k a uniform 23-bit integer (52-bit and
2^-52 for FP64): exactly representable in the storage type, never 0 or 1, so
log u is finite and identical on every side.  Normals are drawn directly in
the storage precision and promoted exactly by consumers that work in FP64.
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np


def _rng(seed: int, stream: int) -> np.random.Generator:
    return np.random.default_rng(np.random.SeedSequence([int(seed), int(stream)]))


def uniforms(rng: np.random.Generator, n, dtype=np.float32) -> np.ndarray:
    if dtype == np.float64:
        k = rng.integers(0, 2 ** 52, size=n, dtype=np.int64).astype(np.float64)
        return (k + 0.5) * 2.0 ** -52
    k = rng.integers(0, 2 ** 23, size=n, dtype=np.int64).astype(np.float64)
    return ((k + 0.5) * 2.0 ** -23).astype(np.float32)


def normals(rng: np.random.Generator, shape, dtype=np.float32) -> np.ndarray:
    return rng.standard_normal(size=shape, dtype=dtype)


@dataclass
class Chain:
    """One MALA/ULA chain problem: target, step size, s0, noise and uniforms."""
    target: dict
    eps: float
    x0: np.ndarray
    xi: np.ndarray          # [T, D]
    u: np.ndarray           # [T]
    dtype: type = np.float32
    burn_xi: np.ndarray | None = None   # [3, D] burn-in noise, applied to x0 before use
    burn_u: np.ndarray | None = None
    meta: dict = field(default_factory=dict)

    @property
    def T(self):
        return self.xi.shape[0]

    @property
    def D(self):
        return self.xi.shape[1]


# --------------------------------------------------------------- targets

def banana_target() -> dict:
    """log p(x) = -x1^2/2 - (x2 - x1^2)^2/2, D = 2."""
    return dict(kind="banana", dim=2)


def logreg_target(seed: int = 0, n_data: int = 1000, dim: int = 25, dtype=np.float32) -> dict:
    """Synthetic Bayesian logistic regression: X ~ N(0,1) [N, D], w* ~ N(0, I),
    y ~ Bernoulli(sigmoid(X w*)), prior N(0, I).  Stands in for the paper's
    German-Credit design, which is not available here."""
    r = _rng(seed, 0)
    X = normals(r, (n_data, dim), np.float64)
    w = r.standard_normal(dim)
    p = 1.0 / (1.0 + np.exp(-(X @ w)))
    y = (r.random(n_data) < p).astype(np.float64)
    return dict(kind="logreg", dim=dim, X=X.astype(dtype), y=y.astype(dtype), prior_var=1.0,
                w_true=w)


def gaussian_target(seed: int = 0, dim: int = 100, lam_lo: float = 1e-2, lam_hi: float = 1.0,
                    dtype=np.float32) -> dict:
    """N(0, Q diag(lam) Q^T): Q from the QR factorisation of a Gaussian matrix
    with the signs of diag(R) folded in, lam log-uniform in [lam_lo, lam_hi].
    The precision P = Q diag(1/lam) Q^T is built in FP64, then rounded."""
    r = _rng(seed, 0)
    G = r.standard_normal((dim, dim))
    Q, R = np.linalg.qr(G)
    Q = Q * np.sign(np.diag(R))[None, :]
    lam = 10.0 ** r.uniform(np.log10(lam_lo), np.log10(lam_hi), size=dim)
    P = (Q * (1.0 / lam)[None, :]) @ Q.T
    P = 0.5 * (P + P.T)
    Sigma = (Q * lam[None, :]) @ Q.T
    return dict(kind="gaussian", dim=dim, mean=np.zeros(dim, dtype=dtype), prec=P.astype(dtype),
                Q=Q, lam=lam, Sigma=Sigma)


def funnel_target(seed: int = 0, dim: int = 32, theta: float | None = None) -> dict:
    """Neal-style funnel with neck log-scale theta: x1 ~ N(0, e^{2 theta}),
    x_d | x1 ~ N(0, e^{x1}) for d >= 2.  theta ~ N(0, 1) from the seed unless given."""
    if theta is None:
        theta = float(_rng(seed, 0).standard_normal())
    return dict(kind="funnel", dim=dim, theta=float(theta))


# --------------------------------------------------------------- chains

def banana_chain(T: int = 1024, seed: int = 0, eps: float = 0.1) -> Chain:
    """MALA on the banana in FP64, x0 = 0, T steps."""
    return Chain(target=banana_target(), eps=eps, x0=np.zeros(2), dtype=np.float64,
                 xi=normals(_rng(seed, 3), (T, 2), np.float64),
                 u=uniforms(_rng(seed, 4), T, np.float64),
                 meta=dict(workload="mala-banana-d2-fp64", T=T, seed=seed))


def logreg_chain(T: int = 65536, seed: int = 0, eps: float = 0.02, n_data: int = 1000,
                 dim: int = 25, chain: int = 0) -> Chain:
    """MALA on the synthetic logistic-regression posterior, FP32 states.
    x0 ~ N(0, I) followed by 3 burn-in MALA steps (Appendix B.1) whose noise is
    given in burn_xi / burn_u; the sampler that consumes the chain runs them."""
    tg = logreg_target(seed, n_data, dim)
    r1 = _rng(seed, 1 + 16 * chain)
    r2 = _rng(seed, 2 + 16 * chain)
    return Chain(target=tg, eps=eps, x0=normals(r1, dim, np.float32),
                 xi=normals(_rng(seed, 3 + 16 * chain), (T, dim), np.float32),
                 u=uniforms(_rng(seed, 4 + 16 * chain), T, np.float32),
                 burn_xi=normals(r2, (3, dim), np.float32), burn_u=uniforms(r2, 3, np.float32),
                 meta=dict(workload=f"mala-logreg-d{dim}-n{n_data}", T=T, seed=seed, chain=chain))


def embedding_logreg_target(seed: int = 0, n_data: int = 1024, dim: int = 768, decay: float = 0.75,
                            dtype=np.float32) -> dict:
    """Synthetic stand-in for a logistic regression on sentence embeddings
    (Sec. 5.5 uses 768-D text embeddings of 1024 reviews, which are not
    available here): rows are unit vectors whose covariance has a power-law
    spectrum (the k-th principal direction carries weight (1 + k)^-decay
    before normalisation, in a random orthogonal basis V), labels follow a
    logistic model on w* ~ N(0, I), prior N(0, I).  Also returns the
    orthogonal basis the paper uses for this model: the left singular
    vectors of the feature covariance X^T X / N (computed in FP64), as
    `basis` [D, D] with columns ordered by decreasing singular value."""
    r = _rng(seed, 0)
    G = r.standard_normal((dim, dim))
    V, R = np.linalg.qr(G)
    V = V * np.sign(np.diag(R))[None, :]
    scale = (1.0 + np.arange(dim)) ** (-decay)
    Z = normals(r, (n_data, dim), np.float64)
    X = (Z * scale[None, :]) @ V.T
    X /= np.linalg.norm(X, axis=1, keepdims=True)
    w = r.standard_normal(dim)
    p = 1.0 / (1.0 + np.exp(-(X @ w)))
    y = (r.random(n_data) < p).astype(np.float64)
    Xr = X.astype(dtype).astype(np.float64)
    U, _, _ = np.linalg.svd(Xr.T @ Xr / n_data)
    return dict(kind="logreg", dim=dim, X=X.astype(dtype), y=y.astype(dtype), prior_var=1.0, w_true=w,
                basis=np.ascontiguousarray(U.astype(dtype)))


def embedding_logreg_batch(seed: int = 0, n_chains: int = 4, T: int = 4096, eps: float = 0.015,
                           n_data: int = 1024, dim: int = 768) -> "Batch":
    """B chains of MALA on the embedding stand-in (Sec. 5.5: B = 4, 4096
    samples, step size 0.015), x0 = 0, laid end to end (CSR offsets).  No
    burn-in steps (burn_xi and burn_u are empty)."""
    tg = embedding_logreg_target(seed, n_data, dim)
    offsets = np.arange(n_chains + 1, dtype=np.int64) * T
    return Batch(target=tg, eps=eps, offsets=offsets, x0=np.zeros((n_chains, dim), dtype=np.float32),
                 xi=normals(_rng(seed, 3), (n_chains * T, dim), np.float32),
                 u=uniforms(_rng(seed, 4), n_chains * T, np.float32),
                 burn_xi=np.zeros((n_chains, 0, dim), dtype=np.float32),
                 burn_u=np.zeros((n_chains, 0), dtype=np.float32))


def funnel_chain(T: int = 16384, seed: int = 0, eps: float = 0.05, theta: float | None = None,
                 dim: int = 32) -> Chain:
    """MALA on the funnel, FP32, x0 = 0."""
    tg = funnel_target(seed, dim, theta)
    return Chain(target=tg, eps=eps, x0=np.zeros(dim, dtype=np.float32),
                 xi=normals(_rng(seed, 3), (T, dim), np.float32),
                 u=uniforms(_rng(seed, 4), T, np.float32),
                 meta=dict(workload=f"mala-funnel-d{dim}", T=T, seed=seed))


def gaussian_chain(T: int, seed: int = 0, eps: float = 0.05, dim: int = 8,
                   dtype=np.float64, lam_lo: float = 0.1) -> Chain:
    """MALA/ULA on a correlated Gaussian; x0 = 0."""
    tg = gaussian_target(seed, dim, lam_lo=lam_lo, dtype=dtype)
    return Chain(target=tg, eps=eps, x0=np.zeros(dim, dtype=dtype), dtype=dtype,
                 xi=normals(_rng(seed, 3), (T, dim), dtype), u=uniforms(_rng(seed, 4), T, dtype),
                 meta=dict(workload=f"mala-gaussian-d{dim}", T=T, seed=seed))


@dataclass
class HMCProblem:
    target: dict
    eps: float
    L: int
    x0: np.ndarray
    momenta: np.ndarray     # [n_prop, D]
    U: np.ndarray           # [n_prop]


def hmc_gaussian(seed: int = 0, dim: int = 100, L: int = 64, eps: float = 0.05,
                 n_prop: int = 2000) -> HMCProblem:
    """HMC on N(0, Q diag(lam) Q^T), lam log-uniform in [1e-2, 1]; x0 is an
    exact stationary draw Q diag(sqrt(lam)) z; momenta N(0, I); FP32."""
    tg = gaussian_target(seed, dim, 1e-2, 1.0, np.float32)
    z = _rng(seed, 1).standard_normal(dim)
    x0 = (tg["Q"] @ (np.sqrt(tg["lam"]) * z)).astype(np.float32)
    return HMCProblem(target=tg, eps=eps, L=L, x0=x0,
                      momenta=normals(_rng(seed, 3), (n_prop, dim), np.float32),
                      U=uniforms(_rng(seed, 4), n_prop, np.float32))


@dataclass
class Batch:
    """Uneven-length chains on one target, concatenated (CSR offsets)."""
    target: dict
    eps: float
    offsets: np.ndarray     # [B+1] int64
    x0: np.ndarray          # [B, D]
    xi: np.ndarray          # [sum T, D]
    u: np.ndarray           # [sum T]
    burn_xi: np.ndarray     # [B, n_burn, D] (3 MALA steps, or 5 HMC steps)
    burn_u: np.ndarray      # [B, n_burn]
    L: int = 0              # HMC transitions: leapfrog steps per transition

    @property
    def n_chains(self):
        return len(self.offsets) - 1


def batch_lengths(seed: int, n_chains: int, lo: int, hi: int) -> np.ndarray:
    r = _rng(seed, 5)
    return np.floor(np.exp(r.uniform(np.log(lo), np.log(hi), size=n_chains))).astype(np.int64)


def logreg_batch(seed: int = 0, n_chains: int = 512, lo: int = 4096, hi: int = 131072,
                 eps: float = 0.02, n_data: int = 1000, dim: int = 25) -> Batch:
    """n_chains independent chains on the logistic posterior, lengths
    log-uniform in [lo, hi]; chain c reuses logreg_chain(..., chain=c)'s streams."""
    tg = logreg_target(seed, n_data, dim)
    lens = batch_lengths(seed, n_chains, lo, hi)
    off = np.zeros(n_chains + 1, dtype=np.int64)
    off[1:] = np.cumsum(lens)
    xi = np.empty((off[-1], dim), dtype=np.float32)
    u = np.empty(off[-1], dtype=np.float32)
    x0 = np.empty((n_chains, dim), dtype=np.float32)
    bxi = np.empty((n_chains, 3, dim), dtype=np.float32)
    bu = np.empty((n_chains, 3), dtype=np.float32)
    for c in range(n_chains):
        T = int(lens[c])
        r1 = _rng(seed, 1 + 16 * c)
        r2 = _rng(seed, 2 + 16 * c)
        x0[c] = normals(r1, dim, np.float32)
        bxi[c] = normals(r2, (3, dim), np.float32)
        bu[c] = uniforms(r2, 3, np.float32)
        xi[off[c]:off[c + 1]] = normals(_rng(seed, 3 + 16 * c), (T, dim), np.float32)
        u[off[c]:off[c + 1]] = uniforms(_rng(seed, 4 + 16 * c), T, np.float32)
    return Batch(target=tg, eps=eps, offsets=off, x0=x0, xi=xi, u=u, burn_xi=bxi, burn_u=bu)


def logreg_hmc_batch(seed: int = 0, n_chains: int = 4, T: int = 1000, eps: float = 0.04, L: int = 4,
                     n_data: int = 1000, dim: int = 25, n_burn: int = 5) -> Batch:
    """HMC across the sequence on the logistic posterior with the settings of
    App. B.4: n_chains chains of T whole HMC transitions (L leapfrog steps of
    size eps), momentum draws xi_t ~ N(0, I) and uniforms u_t per transition,
    each chain started after n_burn sequential transitions from x0 ~ N(0, I)
    (their draws in burn_xi / burn_u; the consumer runs them)."""
    tg = logreg_target(seed, n_data, dim)
    off = np.arange(n_chains + 1, dtype=np.int64) * T
    xi = np.empty((off[-1], dim), dtype=np.float32)
    u = np.empty(off[-1], dtype=np.float32)
    x0 = np.empty((n_chains, dim), dtype=np.float32)
    bxi = np.empty((n_chains, n_burn, dim), dtype=np.float32)
    bu = np.empty((n_chains, n_burn), dtype=np.float32)
    for c in range(n_chains):
        r1 = _rng(seed, 1 + 16 * c)
        r2 = _rng(seed, 2 + 16 * c)
        x0[c] = normals(r1, dim, np.float32)
        bxi[c] = normals(r2, (n_burn, dim), np.float32)
        bu[c] = uniforms(r2, n_burn, np.float32)
        xi[off[c]:off[c + 1]] = normals(_rng(seed, 3 + 16 * c), (T, dim), np.float32)
        u[off[c]:off[c + 1]] = uniforms(_rng(seed, 4 + 16 * c), T, np.float32)
    return Batch(target=tg, eps=eps, offsets=off, x0=x0, xi=xi, u=u, burn_xi=bxi, burn_u=bu, L=L)
