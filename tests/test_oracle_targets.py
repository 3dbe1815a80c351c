"""Pins of the oracle's targets and step Jacobians against finite differences
and library densities (scipy), independent of the oracle's own formulas."""
import numpy as np
import pytest
from scipy import stats

from conftest import oracle_target
from paper_2508_18413_amd import workloads as W


def _targets():
    lt = W.logreg_target(3, n_data=40, dim=5)
    gt = W.gaussian_target(3, dim=6, lam_lo=0.1)
    return {
        "banana": W.banana_target(),
        "gaussian": gt,
        "logreg": lt,
        "funnel": W.funnel_target(3, dim=7, theta=-0.4),
    }


def _fd_grad(f, x, h=1e-5):
    g = np.empty_like(x)
    for i in range(len(x)):
        e = np.zeros_like(x)
        e[i] = h
        g[i] = (f(x + e) - f(x - e)) / (2 * h)
    return g


@pytest.mark.parametrize("name", ["banana", "gaussian", "logreg", "funnel"])
def test_grad_hess_fd(orc, name):
    tg = oracle_target(_targets()[name])
    rng = np.random.default_rng(1)
    for _ in range(4):
        x = rng.normal(size=tg.dim) * 0.7
        g = tg.grad(x)
        np.testing.assert_allclose(g, _fd_grad(tg.logp, x), rtol=1e-7, atol=1e-7)
        H = tg.hess(x)
        Hfd = np.stack([_fd_grad(lambda z: tg.grad(z)[i], x) for i in range(tg.dim)])
        np.testing.assert_allclose(H, Hfd, rtol=1e-6, atol=1e-6)
        np.testing.assert_allclose(H, H.T, atol=0)


def test_theta_derivatives_fd(orc):
    base = _targets()["funnel"]
    rng = np.random.default_rng(2)
    x = rng.normal(size=base["dim"])
    h = 1e-6
    tp = oracle_target(dict(base, theta=base["theta"] + h))
    tm = oracle_target(dict(base, theta=base["theta"] - h))
    t0 = oracle_target(base)
    np.testing.assert_allclose(t0.dgrad_dtheta(x), (tp.grad(x) - tm.grad(x)) / (2 * h), atol=1e-7)
    assert abs(t0.dlogp_dtheta(x) - (tp.logp(x) - tm.logp(x)) / (2 * h)) < 1e-7
    # other targets do not depend on theta
    for nm in ("banana", "gaussian", "logreg"):
        assert np.all(oracle_target(_targets()[nm]).dgrad_dtheta(x[:_targets()[nm]["dim"]]) == 0)


def test_logdensities_match_library(orc):
    """Gaussian and banana log-densities against scipy.stats, up to a constant."""
    gt = _targets()["gaussian"]
    tg = oracle_target(gt)
    cov = np.linalg.inv(gt["prec"].astype(np.float64))
    mvn = stats.multivariate_normal(mean=gt["mean"].astype(np.float64), cov=cov)
    rng = np.random.default_rng(3)
    xs = rng.normal(size=(5, gt["dim"]))
    d = [tg.logp(x) - mvn.logpdf(x) for x in xs]
    assert np.ptp(d) < 1e-10
    # banana: x1 ~ N(0,1), x2 | x1 ~ N(x1^2, 1)
    bn = oracle_target(_targets()["banana"])
    d = [bn.logp(x) - (stats.norm.logpdf(x[0]) + stats.norm.logpdf(x[1] - x[0] ** 2)) for x in
         rng.normal(size=(5, 2)) * 1.5]
    assert np.ptp(d) < 1e-12
    # funnel: x1 ~ N(0, e^{2 theta}), x_d | x1 ~ N(0, e^{x1})
    ft = _targets()["funnel"]
    fn = oracle_target(ft)
    th = ft["theta"]
    d = []
    for x in rng.normal(size=(5, ft["dim"])):
        ref = stats.norm.logpdf(x[0], scale=np.exp(th)) + stats.norm.logpdf(
            x[1:], scale=np.exp(x[0] / 2)).sum()
        d.append(fn.logp(x) - ref)
    assert np.ptp(d) < 1e-10


def test_mala_ratio_matches_library_densities(orc):
    """The log Metropolis ratio of one MALA step, rebuilt from scipy's normal
    densities: log p(x~) - log p(x) + log q(x|x~) - log q(x~|x) with
    q(a|b) = N(a; b + eps grad log p(b), 2 eps I)  (Sec. 3.2)."""
    rng = np.random.default_rng(4)
    for name in ("banana", "gaussian", "funnel"):
        tgd = _targets()[name]
        tg = oracle_target(tgd)
        D = tg.dim
        eps = 0.07
        for _ in range(5):
            x = rng.normal(size=D) * 0.5
            xi = rng.normal(size=D)
            u = rng.uniform()
            xn, a, gt, ell, xp = orc.mala_step(tg, eps, x, xi, u)
            np.testing.assert_allclose(xp, x + eps * tg.grad(x) + np.sqrt(2 * eps) * xi, atol=1e-14)
            cov = 2 * eps * np.eye(D)
            lq_rev = stats.multivariate_normal(xp + eps * tg.grad(xp), cov).logpdf(x)
            lq_fwd = stats.multivariate_normal(x + eps * tg.grad(x), cov).logpdf(xp)
            ref = tg.logp(xp) - tg.logp(x) + lq_rev - lq_fwd
            assert abs(ell - ref) < 1e-9 * max(1, abs(ref))
            assert abs(gt - (min(0.0, ref) - np.log(u))) < 1e-9
            assert a == (gt > 0)
            np.testing.assert_array_equal(xn, xp if a else x)


def _fd_jac(f, x, h=1e-6):
    cols = []
    for i in range(len(x)):
        e = np.zeros_like(x)
        e[i] = h
        cols.append((f(x + e) - f(x - e)) / (2 * h))
    return np.stack(cols, axis=1)


@pytest.mark.parametrize("name", ["banana", "gaussian", "logreg", "funnel"])
def test_mala_jacobian_frozen_fd(orc, name):
    """Frozen-gate Jacobian = FD of the step with the decision held fixed."""
    tg = oracle_target(_targets()[name])
    rng = np.random.default_rng(5)
    eps = 0.03
    for _ in range(4):
        x = rng.normal(size=tg.dim) * 0.5
        xi = rng.normal(size=tg.dim)
        u = rng.uniform()
        F, J, a = orc.mala_jac(tg, eps, x, xi, u, gate=0)
        Jfd = _fd_jac(lambda z: orc.mala_step(tg, eps, z, xi, u, force=a)[0], x)
        np.testing.assert_allclose(J, Jfd, rtol=1e-6, atol=1e-7)
        np.testing.assert_array_equal(F, orc.mala_step(tg, eps, x, xi, u)[0])
        Fu, Ju, _ = orc.mala_jac(tg, eps, x, xi, u, ula=True)
        Jfd = _fd_jac(lambda z: orc.mala_step(tg, eps, z, xi, u, ula=True)[0], x)
        np.testing.assert_allclose(Ju, Jfd, rtol=1e-6, atol=1e-7)


@pytest.mark.parametrize("name", ["banana", "gaussian", "logreg", "funnel"])
def test_mala_jacobian_surrogate_fd(orc, name):
    """The stop-gradient gate adds sigma'(g~)(x~ - x) dg~/dx^T (Sec. 3.2).
    The same rank-one term is the derivative of the sigma-smoothed step minus
    its smooth part sigma(g~) M + (1 - sigma(g~)) I; pin it by FD."""
    tg = oracle_target(_targets()[name])
    rng = np.random.default_rng(6)
    eps = 0.03
    n_checked = 0
    for _ in range(12):
        x = rng.normal(size=tg.dim) * 0.5
        xi = rng.normal(size=tg.dim) * 2.0
        u = rng.uniform(0.2, 0.9)
        _, J0, a = orc.mala_jac(tg, eps, x, xi, u, gate=0)
        _, J1, _ = orc.mala_jac(tg, eps, x, xi, u, gate=1)
        _, _, gt, ell, xp = orc.mala_step(tg, eps, x, xi, u)
        if ell >= 0:
            np.testing.assert_array_equal(J0, J1)
            continue
        s = 1 / (1 + np.exp(-gt))
        M = np.eye(tg.dim) + eps * tg.hess(x)
        Jsm = _fd_jac(lambda z: orc.mala_smoothed_step(tg, eps, z, xi, u), x)
        rank1_fd = Jsm - (s * M + (1 - s) * np.eye(tg.dim))
        rank1 = J1 - (a * M + (1 - a) * np.eye(tg.dim))
        np.testing.assert_allclose(rank1, rank1_fd, rtol=1e-5, atol=1e-7)
        n_checked += 1
    assert n_checked >= 3


def test_leapfrog_jacobian_fd(orc):
    """Leapfrog Jacobian [[I, eps I], [eps H(x'), I + eps^2 H(x')]] (Sec. 3.3)."""
    rng = np.random.default_rng(7)
    for name in ("banana", "gaussian", "logreg", "funnel"):
        tg = oracle_target(_targets()[name])
        D = tg.dim
        s = rng.normal(size=2 * D) * 0.5
        out, J = orc.leapfrog_step(tg, 0.05, s, with_jac=True)
        Jfd = _fd_jac(lambda z: orc.leapfrog_step(tg, 0.05, z), s)
        np.testing.assert_allclose(J, Jfd, rtol=1e-6, atol=1e-8)
        np.testing.assert_array_equal(J[:D, :D], np.eye(D))
        np.testing.assert_array_equal(J[:D, D:], 0.05 * np.eye(D))
