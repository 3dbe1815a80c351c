"""Pins of the oracle's sequential chains against closed forms and invariants.

* MALA and HMC are exact Metropolis-Hastings samplers: long chains on a
  Gaussian target reproduce its mean and covariance (batch-means error bars).
  A dropped or mis-signed term of the proposal density or of the energy would
  bias these moments far beyond the error bars at the step sizes used.
* ULA (MALA without the accept step) on N(0, P^-1) is the linear recursion
  x' = (I - eps P) x + sqrt(2 eps) xi; its stationary covariance has
  eigenvalues 1 / (p (1 - eps p / 2)) in the eigenbasis of P.
* Leapfrog on a Gaussian is linear with unit determinant per eigen-mode; the
  L-step map follows from the Cayley-Hamilton / Chebyshev closed form
  M^L = (sin(L phi) M - sin((L-1) phi) I) / sin(phi), cos(phi) = 1 - eps^2 p / 2.
"""
import numpy as np
import pytest

from conftest import oracle_target
from paper_2508_18413_amd import workloads as W


def _gauss(dim, seed=0, lam_lo=0.25):
    return W.gaussian_target(seed, dim=dim, lam_lo=lam_lo, lam_hi=1.0, dtype=np.float64)


def _batch_means(x, nb=64):
    """Mean and standard error per column by non-overlapping batch means."""
    n = (x.shape[0] // nb) * nb
    b = x[:n].reshape(nb, -1, *x.shape[1:]).mean(axis=1)
    return b.mean(axis=0), b.std(axis=0, ddof=1) / np.sqrt(nb)


def _moment_check(samples, Sigma, z=5.0):
    m, se = _batch_means(samples)
    assert np.all(np.abs(m) < z * se + 1e-3), (m, se)
    D = samples.shape[1]
    outer = (samples[:, :, None] * samples[:, None, :]).reshape(len(samples), D * D)
    c, cse = _batch_means(outer)
    c = c.reshape(D, D)
    cse = cse.reshape(D, D)
    assert np.all(np.abs(c - Sigma) < z * cse + 2e-3), np.max(np.abs(c - Sigma) / cse)


def test_mala_gaussian_moments(orc):
    gt = _gauss(4, seed=1)
    tg = oracle_target(gt)
    T = 1 << 18
    rng = np.random.default_rng(11)
    xi = rng.normal(size=(T, 4))
    u = rng.uniform(size=T)
    eps = 0.35  # large step: without the Metropolis correction the covariance is badly off
    st, acc, _ = orc.mala_chain(tg, eps, np.zeros(4), xi, u)
    assert 0.25 < acc.mean() < 0.95
    _moment_check(st[1000:], gt["Sigma"])


def test_ula_stationary_covariance_closed_form(orc):
    gt = _gauss(3, seed=2)
    tg = oracle_target(gt)
    P = gt["prec"]
    T = 1 << 18
    eps = 0.4
    rng = np.random.default_rng(12)
    st, acc, _ = orc.mala_chain(tg, eps, np.zeros(3), rng.normal(size=(T, 3)), None, ula=True)
    assert acc.all()
    p, V = np.linalg.eigh(P)
    assert np.all(eps * p < 2)
    C = (V * (1.0 / (p * (1 - eps * p / 2)))[None, :]) @ V.T
    _moment_check(st[1000:], C)
    # and it is measurably different from the target covariance
    assert np.max(np.abs(C - gt["Sigma"])) > 0.05


def test_hmc_gaussian_moments(orc):
    gt = _gauss(4, seed=3)
    tg = oracle_target(gt)
    n = 1 << 15
    rng = np.random.default_rng(13)
    r = orc.hmc_chain(tg, 0.45, 6, np.zeros(4), rng.normal(size=(n, 4)), rng.uniform(size=n))
    assert 0.4 < r["accept"].mean() < 0.99
    _moment_check(r["chain"][100:], gt["Sigma"])


def test_leapfrog_gaussian_closed_form(orc):
    gt = _gauss(5, seed=4)
    tg = oracle_target(gt)
    L, eps = 17, 0.3
    rng = np.random.default_rng(14)
    r = orc.hmc_chain(tg, eps, L, rng.normal(size=5), rng.normal(size=(3, 5)), np.full(3, 0.5),
                      want_traj=True)
    p, V = np.linalg.eigh(gt["prec"])
    for k in range(3):
        x0, v0 = r["s0"][k, :5], r["s0"][k, 5:]
        a, b = V.T @ x0, V.T @ v0
        for l in range(1, L + 1):
            phi = np.arccos(1 - eps * eps * p / 2)
            M = np.array([[np.ones_like(p), eps * np.ones_like(p)], [-eps * p, 1 - eps * eps * p]])
            c1 = np.sin(l * phi) / np.sin(phi)
            c0 = np.sin((l - 1) * phi) / np.sin(phi)
            xl = c1 * (M[0, 0] * a + M[0, 1] * b) - c0 * a
            vl = c1 * (M[1, 0] * a + M[1, 1] * b) - c0 * b
            np.testing.assert_allclose(V @ xl, r["traj"][k, l - 1, :5], atol=1e-12)
            np.testing.assert_allclose(V @ vl, r["traj"][k, l - 1, 5:], atol=1e-12)


def test_hmc_half_steps_and_accept_rule(orc):
    """s0 = [x0, v0 + eps/2 grad log p(x0)] and accept iff log U < H0 - HL."""
    gt = _gauss(3, seed=5)
    tg = oracle_target(gt)
    rng = np.random.default_rng(15)
    x0 = rng.normal(size=3)
    mom = rng.normal(size=(40, 3))
    U = rng.uniform(size=40)
    eps, L = 0.9, 5
    r = orc.hmc_chain(tg, eps, L, x0, mom, U, want_traj=True)
    x = x0
    for k in range(40):
        np.testing.assert_allclose(r["s0"][k, :3], x, atol=0)
        np.testing.assert_allclose(r["s0"][k, 3:], mom[k] + 0.5 * eps * tg.grad(x), atol=1e-14)
        xL, vL = r["traj"][k, -1, :3], r["traj"][k, -1, 3:] - 0.5 * eps * tg.grad(r["traj"][k, -1, :3])
        H0 = 0.5 * mom[k] @ mom[k] - tg.logp(x)
        HL = 0.5 * vL @ vL - tg.logp(xL)
        assert abs(r["logr"][k] - (H0 - HL - np.log(U[k]))) < 1e-10
        assert r["accept"][k] == (np.log(U[k]) < H0 - HL)
        x = xL if r["accept"][k] else x
        np.testing.assert_array_equal(r["chain"][k + 1], x)
    assert 0 < r["accept"].mean() < 1


def test_forced_decisions(orc):
    ch = W.banana_chain(256, seed=3)
    tg = oracle_target(ch.target)
    st, acc, gt = orc.mala_chain(tg, ch.eps, ch.x0, ch.xi, ch.u)
    st2, acc2, _ = orc.mala_chain(tg, ch.eps, ch.x0, ch.xi, ch.u, force=acc)
    np.testing.assert_array_equal(st, st2)
    f = np.full(256, -1, dtype=np.int8)
    k = int(np.argmax(acc == 1))
    f[k] = 0
    st3, acc3, _ = orc.mala_chain(tg, ch.eps, ch.x0, ch.xi, ch.u, force=f)
    np.testing.assert_array_equal(st3[:k], st[:k])
    np.testing.assert_array_equal(st3[k], st3[k - 1] if k else ch.x0)
    assert acc3[k] == 0


def test_logreg_step_matches_plain_definition(orc):
    """One MALA step on the logistic posterior against the definition written
    with scipy's Bernoulli/normal log-densities and numpy."""
    from scipy import stats
    tgd = W.logreg_target(5, n_data=30, dim=4)
    tg = oracle_target(tgd)
    X = tgd["X"].astype(np.float64)
    y = tgd["y"].astype(np.float64)

    def logp(w):
        return stats.bernoulli.logpmf(y, 1 / (1 + np.exp(-(X @ w)))).sum() + stats.norm.logpdf(w).sum()

    rng = np.random.default_rng(16)
    for _ in range(5):
        x = rng.normal(size=4) * 0.3
        xi = rng.normal(size=4)
        u = rng.uniform()
        eps = 0.01
        _, a, gt, ell, xp = orc.mala_step(tg, eps, x, xi, u)
        cov = 2 * eps * np.eye(4)
        ref = (logp(xp) - logp(x) + stats.multivariate_normal(xp + eps * tg.grad(xp), cov).logpdf(x)
               - stats.multivariate_normal(x + eps * tg.grad(x), cov).logpdf(xp))
        assert abs(ell - ref) < 1e-9


def test_golden_banana_fixture(orc):
    """Regression fixture written by tests/golden/make_golden.py (oracle only)."""
    import json
    import os
    with open(os.path.join(os.path.dirname(__file__), "golden", "banana_mala_t32.json")) as f:
        g = json.load(f)
    tg = orc.Target(orc.BANANA, 2)
    st, acc, gt = orc.mala_chain(tg, g["eps"], np.array(g["x0"]), np.array(g["xi"]), np.array(g["u"]))
    np.testing.assert_array_equal(st, np.array(g["states"]))
    np.testing.assert_array_equal(acc, np.array(g["accept"]))
    # the inputs are those of the seeded workload
    ch = W.banana_chain(32, seed=0)
    np.testing.assert_array_equal(ch.xi, np.array(g["xi"]))
