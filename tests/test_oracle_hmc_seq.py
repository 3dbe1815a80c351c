"""Pins of the oracle's whole-HMC-transition step (Sec. 3.3, parallel HMC
across the sequence: f_t runs a sequential leapfrog integrator and the
relaxed accept gate) and of its Jacobian.

* With the identity mass matrix the chain of transitions equals the oracle's
  HMC chain of Appendix A.2 (a separate implementation, itself pinned by
  Gaussian moments and the leapfrog closed form in test_oracle_chains.py).
* With a diagonal mass matrix (Appendix A.2 remarks, App. B.3) HMC is still
  exact Metropolis-Hastings: long chains on a Gaussian reproduce its mean and
  covariance.  A mass matrix applied in the wrong place (kinetic energy,
  position update or momentum draw) biases them.
* Frozen-gate Jacobian: central finite differences of the transition with
  the accept decision held fixed.  Relaxed gate: central differences of the
  sigma-smoothed transition (whose derivative the stop-gradient construction
  returns).
* Closed form on a Gaussian with identity mass: the accepted transition maps
  x0 to x_L linearly with dx_L/dx0 = Q diag(cos(L phi_k)) Q^T,
  cos(phi_k) = 1 - eps^2 p_k / 2, in the eigenbasis (Q, p) of the precision
  (Chebyshev form of the leapfrog powers after the half step).
* Newton reference on this step: causal exactness (after sweep i the first i
  states equal the sequential chain bitwise) for the dense, diagonal and
  probed-diagonal updates, and the fixed point is the sequential chain.
"""
import numpy as np
import pytest

from conftest import oracle_target
from paper_2508_18413_amd import workloads as W


def _gauss(dim, seed=0, lam_lo=0.25):
    return W.gaussian_target(seed, dim=dim, lam_lo=lam_lo, lam_hi=1.0, dtype=np.float64)


def _targets(orc):
    lt = W.logreg_target(seed=2, n_data=60, dim=5, dtype=np.float64)
    return {
        "banana": (orc.Target(orc.BANANA, 2), 0.5, 8),
        "funnel": (oracle_target(W.funnel_target(seed=1, dim=6, theta=0.3)), 0.1, 5),
        "logreg": (oracle_target(lt), 0.04, 4),
        "gaussian": (oracle_target(_gauss(4, seed=7)), 0.3, 6),
    }


def test_identity_mass_chain_equals_appendix_chain(orc):
    gt = _gauss(5, seed=2)
    tg = oracle_target(gt)
    rng = np.random.default_rng(21)
    n = 400
    x0 = rng.normal(size=5)
    mom = rng.normal(size=(n, 5))
    U = rng.uniform(size=n)
    ref = orc.hmc_chain(tg, 0.35, 7, x0, mom, U)
    st, acc, gtl = orc.hmc_seq_chain(tg, 0.35, 7, x0, mom, U)
    assert np.array_equal(acc, ref["accept"])
    np.testing.assert_allclose(st, ref["chain"][1:], rtol=0, atol=1e-13)
    # the gate g~ = min(0, H0 - HL) - log U has the decision's sign and equals
    # the Appendix margin (H0 - HL) - log U wherever H0 < HL
    assert np.array_equal(gtl > 0, ref["logr"] > 0)
    lower = ref["logr"] < -np.log(U)
    np.testing.assert_allclose(gtl[lower], ref["logr"][lower], rtol=0, atol=1e-12)


@pytest.mark.slow
def test_diagonal_mass_gaussian_moments(orc):
    gt = _gauss(3, seed=9, lam_lo=0.05)
    tg = oracle_target(gt)
    inv_mass = 1.0 / np.array([0.3, 1.5, 4.0])
    T = 1 << 16
    rng = np.random.default_rng(22)
    st, acc, _ = orc.hmc_seq_chain(tg, 0.3, 5, np.zeros(3), rng.normal(size=(T, 3)), rng.uniform(size=T),
                                   inv_mass=inv_mass)
    assert 0.4 < acc.mean() < 0.99
    from test_oracle_chains import _moment_check
    _moment_check(st[200:], gt["Sigma"])


def test_mass_matrix_enters_the_transition(orc):
    """A non-identity mass matrix changes the transition (and the identity one
    reproduces the default)."""
    tg = oracle_target(_gauss(3, seed=3))
    x, xi = np.array([0.2, -0.5, 0.9]), np.array([0.3, 1.1, -0.7])
    a = orc.hmc_step(tg, 0.3, 5, x, xi, 0.5)
    b = orc.hmc_step(tg, 0.3, 5, x, xi, 0.5, inv_mass=np.ones(3))
    c = orc.hmc_step(tg, 0.3, 5, x, xi, 0.5, inv_mass=np.array([0.5, 2.0, 1.0]))
    np.testing.assert_array_equal(a[4], b[4])
    assert np.max(np.abs(a[4] - c[4])) > 1e-3


@pytest.mark.parametrize("kind", ["banana", "funnel", "logreg", "gaussian"])
@pytest.mark.parametrize("mass", [False, True])
def test_frozen_jacobian_fd(orc, kind, mass):
    tg, eps, L = _targets(orc)[kind]
    D = tg.dim
    rng = np.random.default_rng(31)
    im = rng.uniform(0.5, 2.0, size=D) if mass else None
    for _ in range(3):
        x = rng.normal(size=D) * 0.5
        xi = rng.normal(size=D)
        u = rng.uniform()
        for force in (0, 1):
            F, J = orc.hmc_step_jac(tg, eps, L, x, xi, u, gate=0, force=force, inv_mass=im)
            h = 1e-6
            Jfd = np.empty((D, D))
            for j in range(D):
                e = np.zeros(D)
                e[j] = h
                fp = orc.hmc_step(tg, eps, L, x + e, xi, u, force=force, inv_mass=im)[0]
                fm = orc.hmc_step(tg, eps, L, x - e, xi, u, force=force, inv_mass=im)[0]
                Jfd[:, j] = (fp - fm) / (2 * h)
            np.testing.assert_allclose(J, Jfd, rtol=1e-6, atol=1e-7)
            if force == 0:
                np.testing.assert_array_equal(J, np.eye(D))


@pytest.mark.parametrize("kind", ["banana", "funnel", "logreg", "gaussian"])
def test_relaxed_jacobian_fd_of_smoothed_step(orc, kind):
    """The relaxed gate's Jacobian at the accepted and at the rejected value
    equals the FD derivative of the sigma-smoothed step minus the derivative
    the forward select does not have: J_relaxed - J_frozen is the rank-one
    term sigma'(g~) (x_L - x) (dg~/dx)^T, which the smoothed step's FD sees
    (with the smoothed gate's own a-weighted path derivative removed)."""
    tg, eps, L = _targets(orc)[kind]
    D = tg.dim
    rng = np.random.default_rng(41)
    checked = 0
    for _ in range(400):
        if checked >= 5:
            break
        x = rng.normal(size=D) * 0.5
        xi = rng.normal(size=D)
        u = rng.uniform()
        _, _, gt, dh, xl = orc.hmc_step(tg, eps, L, x, xi, u)
        if not dh < 0:
            continue  # where H0 >= HL the gate is the constant min(0, .) = 0 branch
        s = 1.0 / (1.0 + np.exp(-gt))
        _, J1 = orc.hmc_step_jac(tg, eps, L, x, xi, u, gate=1)
        _, Ja = orc.hmc_step_jac(tg, eps, L, x, xi, u, gate=0, force=1)  # dx_L/dx
        h = 1e-6
        Jfd = np.empty((D, D))
        for j in range(D):
            e = np.zeros(D)
            e[j] = h
            Jfd[:, j] = (orc.hmc_smoothed_step(tg, eps, L, x + e, xi, u)
                         - orc.hmc_smoothed_step(tg, eps, L, x - e, xi, u)) / (2 * h)
        # smoothed step: s dx_L/dx + (1 - s) I + s'(g~) (x_L - x) dg~/dx
        rank1 = Jfd - (s * Ja + (1 - s) * np.eye(D))
        a = int(gt > 0)
        frozen = a * Ja + (1 - a) * np.eye(D)
        np.testing.assert_allclose(J1 - frozen, rank1, rtol=2e-5, atol=2e-7)
        checked += 1
    assert checked >= 3


def test_gaussian_jacobian_closed_form(orc):
    gt = _gauss(4, seed=11)
    tg = oracle_target(gt)
    p, Q = np.linalg.eigh(gt["prec"])
    rng = np.random.default_rng(51)
    for L, eps in ((1, 0.4), (6, 0.3), (13, 0.2)):
        x, xi = rng.normal(size=4), rng.normal(size=4)
        _, J = orc.hmc_step_jac(tg, eps, L, x, xi, 0.5, gate=0, force=1)
        phi = np.arccos(1 - eps * eps * p / 2)
        np.testing.assert_allclose(J, (Q * np.cos(L * phi)[None, :]) @ Q.T, atol=1e-12)


def _provider(orc, tg, eps, L, xi, u, gate=0, inv_mass=None):
    def sj(t, s_prev):
        return orc.hmc_step_jac(tg, eps, L, s_prev, xi[t], u[t], gate=gate, inv_mass=inv_mass)
    return sj


@pytest.mark.parametrize("kind", ["banana", "logreg"])
@pytest.mark.parametrize("variant", ["dense", "diag", "hutchinson", "picard"])
def test_newton_causal_exactness_hmc(orc, kind, variant):
    tg, eps, L = _targets(orc)[kind]
    D = tg.dim
    T = 12
    rng = np.random.default_rng(61)
    x0 = rng.normal(size=D) * 0.3
    xi = rng.normal(size=(T, D))
    u = rng.uniform(size=T)
    ref, _, _ = orc.hmc_seq_chain(tg, eps, L, x0, xi, u)
    S, trace, sweeps = orc.newton_reference(_provider(orc, tg, eps, L, xi, u, gate=1), x0, T, variant=variant,
                                            probe_seed=5)
    for i in range(1, len(trace)):
        assert np.array_equal(trace[i][:i], ref[:i]), (variant, i)
    np.testing.assert_array_equal(S, ref)
    assert sweeps <= T + 1


def test_diverged_trajectory_rejects(orc):
    """A trajectory that overflows (banana from a far-out start) gives a NaN
    energy difference, and the transition rejects it (the reading for a NaN
    Metropolis ratio); an infinite energy error rejects by the ratio itself."""
    tg = orc.Target(orc.BANANA, 2)
    x = np.array([1e120, 0.0])
    xn, a, gt, dh, xl = orc.hmc_step(tg, 0.5, 8, x, np.array([0.3, -0.2]), 0.5)
    assert not np.isfinite(dh) and a == 0
    np.testing.assert_array_equal(xn, x)
    for force in (-1,):
        F, J = orc.hmc_step_jac(tg, 0.5, 8, x, np.array([0.3, -0.2]), 0.5, gate=1, force=force)
        np.testing.assert_array_equal(J, np.eye(2))
