"""Pins of the oracle on the 768-dimensional logistic-regression stand-in
(Sec. 5.5): the same density and gradient code as the small-D pins, now at
the dimension that sizes its per-call arrays.

* Central finite differences of log p reproduce the gradient on sampled
  coordinates of a D = 768, N = 1024 posterior (the arrays of one call
  hold the whole state, so a capacity error would show as a wrong or
  truncated gradient).
* At D = 1024 (the capacity) the gradient still agrees; D = 1025 is refused
  by the wrapper.
* The orthogonal basis the workload supplies is orthonormal and
  diagonalises the feature covariance (left singular vectors, Sec. 5.5).
* A MALA step in the rotated coordinates z = Q^T s (eq. 11: design X Q,
  noise Q^T xi) is the rotated MALA step in s, to rounding.
"""
import numpy as np
import pytest

from conftest import oracle_target
from paper_2508_18413_amd import workloads as W


def _fd_check(tg, x, coords, h=1e-5):
    g = tg.grad(x)
    for d in coords:
        e = np.zeros_like(x)
        e[d] = h
        fd = (tg.logp(x + e) - tg.logp(x - e)) / (2 * h)
        assert abs(fd - g[d]) <= 1e-5 * max(1.0, abs(g[d])), (d, fd, g[d])
    return g


def test_wide_gradient_fd(orc):
    t = W.embedding_logreg_target(seed=1)
    tg = oracle_target(t)
    rng = np.random.default_rng(3)
    x = rng.normal(size=768) * 0.3
    g = _fd_check(tg, x, [0, 1, 255, 256, 511, 512, 700, 767])
    assert np.all(np.isfinite(g)) and np.count_nonzero(g) == 768


def test_capacity(orc):
    rng = np.random.default_rng(4)
    X = rng.normal(size=(64, 1024)) / 32.0
    y = (rng.random(64) < 0.5).astype(np.float64)
    tg = orc.Target(orc.LOGREG, 1024, X=X, y=y, prior_var=1.0)
    _fd_check(tg, rng.normal(size=1024) * 0.2, [0, 511, 1023])
    with pytest.raises(ValueError):
        orc.Target(orc.LOGREG, 1025, X=np.zeros((4, 1025)), y=np.zeros(4), prior_var=1.0)


def test_basis_diagonalises_covariance():
    t = W.embedding_logreg_target(seed=2)
    Q = t["basis"].astype(np.float64)
    X = t["X"].astype(np.float64)
    np.testing.assert_allclose(Q.T @ Q, np.eye(768), atol=2e-5)
    C = Q.T @ (X.T @ X / X.shape[0]) @ Q
    off = C - np.diag(np.diag(C))
    assert np.max(np.abs(off)) <= 1e-5 * np.max(np.abs(np.diag(C)))
    assert np.all(np.diff(np.diag(C)) <= 1e-9)  # decreasing


def test_rotated_step_is_rotated_mala(orc):
    t = W.embedding_logreg_target(seed=3)
    # the FP32 basis made exactly orthogonal in FP64 (the identity is exact
    # for an orthogonal Q; rounding of Q itself is not what is tested here)
    Q, R = np.linalg.qr(t["basis"].astype(np.float64))
    Q = Q * np.sign(np.diag(R))[None, :]
    tg = oracle_target(t)
    rot = dict(t, X=(t["X"].astype(np.float64) @ Q))
    tr = oracle_target(rot)
    rng = np.random.default_rng(5)
    x, xi = rng.normal(size=768) * 0.2, rng.normal(size=768)
    for u in (0.3, 0.999):
        xn, a, gt, ell, xp = orc.mala_step(tg, 0.015, x, xi, u)
        zn, az, gz, ellz, zp = orc.mala_step(tr, 0.015, Q.T @ x, Q.T @ xi, u)
        np.testing.assert_allclose(Q @ zp, xp, atol=1e-9)
        assert abs(ell - ellz) <= 1e-9 * max(1.0, abs(ell))
        assert a == az
