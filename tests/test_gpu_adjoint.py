"""GPU adjoint (reverse scan over transposed Jacobians) against the FP64
oracle's adjoint and tangent through the same trajectory, and against central
finite differences of the oracle chain with the accept pattern held fixed.
F = (1/T) sum_t |x_t|^2; parameters: the funnel log-scale theta and eps."""
import numpy as np
import pytest

from conftest import oracle_target
from paper_2508_18413_amd import workloads as W

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")
DEV = "cuda:0"


def _t(x):
    return torch.tensor(np.ascontiguousarray(x), device=DEV)


@pytest.fixture(scope="module")
def pm():
    import paper_2508_18413_amd as pm
    return pm


@pytest.fixture(scope="module")
def ctx(pm):
    c = pm.Context(0)
    yield c
    c.close()


@pytest.mark.parametrize("T,theta", [(2048, 0.0), (16384, None)])
def test_adjoint_funnel(pm, ctx, orc, T, theta):
    print(f"adjoint funnel T={T} theta={theta}", flush=True)
    ch = W.funnel_chain(T=T, seed=0, theta=theta)
    tg = oracle_target(ch.target)
    g = pm.Target(ctx, ch.target)
    r = pm.solve(ctx, g, ch.eps, _t(ch.x0), _t(ch.xi), _t(ch.u), variant="diag", max_iter=T + 1)
    assert r.status == 0
    st = r.states
    dF = (2.0 / T) * st
    dth, deps = pm.adjoint(ctx, g, ch.eps, _t(ch.x0), _t(ch.xi), _t(ch.u), st, r.accept, dF.contiguous())
    s64 = st.cpu().numpy().astype(np.float64)
    acc = r.accept.cpu().numpy()
    ref = orc.mala_adjoint(tg, ch.eps, ch.x0.astype(np.float64), ch.xi, s64, acc, 2.0 * s64 / T)
    tan = orc.mala_tangent(tg, ch.eps, ch.x0.astype(np.float64), ch.xi, s64, acc, 2.0 * s64 / T)
    print(f"  gpu=({dth:.6g}, {deps:.6g}) oracle adjoint=({ref[0]:.6g}, {ref[1]:.6g}) "
          f"tangent=({tan[0]:.6g}, {tan[1]:.6g})", flush=True)
    np.testing.assert_allclose([dth, deps], ref, rtol=1e-4, atol=1e-6)
    np.testing.assert_allclose(ref, tan, rtol=1e-9, atol=1e-12)
    # central differences (h = 1e-3) of the FP64 chain with the accept pattern frozen
    x0 = ch.x0.astype(np.float64)

    def F_of(th, ep):
        t2 = oracle_target(dict(ch.target, theta=th))
        s, _, _ = orc.mala_chain(t2, ep, x0, ch.xi, ch.u, force=acc)
        return (s ** 2).sum() / T

    h = 1e-3
    th0 = ch.target["theta"]
    fd_th = (F_of(th0 + h, ch.eps) - F_of(th0 - h, ch.eps)) / (2 * h)
    fd_ep = (F_of(th0, ch.eps + h) - F_of(th0, ch.eps - h)) / (2 * h)
    print(f"  fd=({fd_th:.6g}, {fd_ep:.6g})", flush=True)
    assert abs(fd_th - dth) <= 2e-3 * max(1.0, abs(dth))
    assert abs(fd_ep - deps) <= 2e-2 * max(1.0, abs(deps))


def test_autograd_function(pm, ctx, orc):
    print("autograd function", flush=True)
    ch = W.funnel_chain(T=1024, seed=2, theta=-0.3)
    theta = torch.tensor(-0.3, dtype=torch.float64, requires_grad=True)
    eps = torch.tensor(ch.eps, dtype=torch.float64, requires_grad=True)
    st = pm.ParallelMALA.apply(theta, eps, ctx, ch.target, _t(ch.x0), _t(ch.xi), _t(ch.u),
                               dict(variant="diag", max_iter=1025))
    F = (st.double() ** 2).sum() / st.shape[0]
    F.backward()
    g = pm.Target(ctx, ch.target)
    r = pm.solve(ctx, g, ch.eps, _t(ch.x0), _t(ch.xi), _t(ch.u), variant="diag", max_iter=1025)
    dth, deps = pm.adjoint(ctx, g, ch.eps, _t(ch.x0), _t(ch.xi), _t(ch.u), r.states, r.accept,
                           ((2.0 / st.shape[0]) * r.states).contiguous())
    assert abs(theta.grad.item() - dth) <= 1e-4 * max(1.0, abs(dth))
    assert abs(eps.grad.item() - deps) <= 1e-4 * max(1.0, abs(deps))


def test_adjoint_unsupported(pm, ctx):
    from paper_2508_18413_amd import _binding as B
    ch = W.logreg_chain(T=64, eps=0.001, n_data=40, dim=4)
    g = pm.Target(ctx, ch.target)
    st = torch.zeros((64, 4), device=DEV)
    with pytest.raises(B.PMCError) as e:
        pm.adjoint(ctx, g, ch.eps, _t(ch.x0), _t(ch.xi), _t(ch.u), st,
                   torch.zeros(64, dtype=torch.uint8, device=DEV), st)
    assert e.value.status == B.PMC_ERR_UNSUPPORTED
