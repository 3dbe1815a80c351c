"""Pins of the oracle's trajectory derivatives.

The functional is F = (1/T) sum_t |x_t|^2 (the trajectory mean of the squared
norm).  Two different algorithms -- forward-mode tangent propagation and the
reverse-mode adjoint recursion -- must agree to rounding, and both must agree
with central finite differences of the sequential FP64 chain in which every
accept decision is held at the base run's pattern (the frozen-gate derivative
is the exact derivative of that piecewise-smooth map).
"""
import numpy as np
import pytest

from conftest import oracle_target
from paper_2508_18413_amd import workloads as W


def _F(states):
    return (states ** 2).sum() / states.shape[0]


def _dF(states):
    return 2 * states / states.shape[0]


@pytest.mark.parametrize("case", ["funnel", "banana", "logreg"])
def test_tangent_adjoint_fd(orc, case):
    if case == "funnel":
        ch = W.funnel_chain(400, seed=2, dim=8, eps=0.05, theta=-0.3)
    elif case == "banana":
        ch = W.banana_chain(400, seed=2)
    else:
        ch = W.logreg_chain(200, seed=2, eps=0.004, n_data=50, dim=5)
    tg = oracle_target(ch.target)
    x0 = np.asarray(ch.x0, dtype=np.float64)
    st, acc, _ = orc.mala_chain(tg, ch.eps, x0, ch.xi, ch.u)
    assert 0 < acc.mean() < 1
    tan = orc.mala_tangent(tg, ch.eps, x0, ch.xi, st, acc, _dF(st))
    adj = orc.mala_adjoint(tg, ch.eps, x0, ch.xi, st, acc, _dF(st))
    np.testing.assert_allclose(tan, adj, rtol=1e-10, atol=1e-12)

    def fd_eps(h):
        Fp = _F(orc.mala_chain(tg, ch.eps + h, x0, ch.xi, ch.u, force=acc)[0])
        Fm = _F(orc.mala_chain(tg, ch.eps - h, x0, ch.xi, ch.u, force=acc)[0])
        return (Fp - Fm) / (2 * h)

    def fd_theta(h):
        tp = oracle_target(dict(ch.target, theta=ch.target["theta"] + h))
        tm = oracle_target(dict(ch.target, theta=ch.target["theta"] - h))
        return (_F(orc.mala_chain(tp, ch.eps, x0, ch.xi, ch.u, force=acc)[0])
                - _F(orc.mala_chain(tm, ch.eps, x0, ch.xi, ch.u, force=acc)[0])) / (2 * h)

    # central differences converge to the adjoint at second order: the error
    # at h (1e-3, or eps/50 for small steps) is small and shrinks ~16x at h / 4
    h = min(1e-3, ch.eps / 50)
    checks = [(fd_eps, 1)] + ([(fd_theta, 0)] if case == "funnel" else [])
    for fd, k in checks:
        e1 = abs(fd(h) - adj[k])
        e2 = abs(fd(h / 4) - adj[k])
        assert e1 < 2e-3 * max(1.0, abs(adj[k])), (fd(h), adj[k])
        assert e2 < e1 / 8 + 1e-9 * max(1.0, abs(adj[k])), (e1, e2)
    if case == "funnel":
        assert abs(adj[0]) > 1e-3
    else:
        assert adj[0] == 0


def test_adjoint_states_are_reverse_recursion(orc):
    """lambda_t = dF/ds_t + J_{t+1}^T lambda_{t+1}, with J from the step Jacobian."""
    ch = W.funnel_chain(30, seed=5, dim=4, eps=0.1, theta=0.2)
    tg = oracle_target(ch.target)
    x0 = np.asarray(ch.x0, dtype=np.float64)
    st, acc, _ = orc.mala_chain(tg, ch.eps, x0, ch.xi, ch.u)
    g = _dF(st)
    _, lam = orc.mala_adjoint(tg, ch.eps, x0, ch.xi, st, acc, g, want_lambda=True)
    T = st.shape[0]
    ref = np.zeros_like(st)
    ref[T - 1] = g[T - 1]
    for t in range(T - 2, -1, -1):
        _, J, _ = orc.mala_jac(tg, ch.eps, st[t], ch.xi[t + 1], ch.u[t + 1], force=acc[t + 1])
        ref[t] = g[t] + J.T @ ref[t + 1]
    np.testing.assert_allclose(lam, ref, rtol=1e-12, atol=1e-14)
