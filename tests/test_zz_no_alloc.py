"""pmc_solve_noalloc (through the C ABI) against pmc_solve: the same kernels on
a workspace taken from the library's static per-device scratch array, so the
results must be identical bit for bit.  Two calls in a row, the second on a
smaller problem, reuse the scratch the first one left behind."""
import numpy as np
import pytest

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


def _same(a, b):
    assert a.status == b.status
    assert a.sweeps == b.sweeps and a.sweeps_per_chain == b.sweeps_per_chain
    assert torch.equal(a.states, b.states)
    assert torch.equal(a.accept, b.accept)
    assert torch.equal(a.gtilde, b.gtilde)


def test_noalloc_matches_solve_two_calls(pm):
    print("noalloc: logistic T=65536 then T=4096", flush=True)
    # load the library's code objects and let the runtime size its per-device
    # scratch backing for these kernels (both happen at a kernel's first
    # launch in the process, outside the library's control), in a context of
    # its own that is then destroyed
    warm = pm.Context(0)
    ch0 = W.logreg_chain(T=65536, seed=1, eps=0.0015)
    g0 = pm.Target(warm, ch0.target)
    pm.solve(warm, g0, ch0.eps, _t(ch0.x0), _t(ch0.xi), _t(ch0.u), variant="diag", max_iter=65537)
    # and one allocation-free call: the first one in a process lets the HIP
    # runtime set up its own buffers (2 MiB of device memory measured once per
    # process, none on later calls)
    pm.solve_noalloc(warm, g0, ch0.eps, _t(ch0.x0), _t(ch0.xi), _t(ch0.u), variant="diag", max_iter=65537)
    del g0
    warm.close()
    torch.cuda.synchronize()

    ctx = pm.Context(0)
    big = W.logreg_chain(T=65536, seed=0, eps=0.0015)
    small = W.logreg_chain(T=4096, seed=7, eps=0.0015)
    g = pm.Target(ctx, big.target)
    g2 = pm.Target(ctx, small.target)
    for ch, tg in ((big, g), (small, g2)):
        s0, xi, u = _t(ch.x0), _t(ch.xi), _t(ch.u)
        n, D = xi.shape
        outs = (torch.empty((n, D), dtype=xi.dtype, device=DEV), torch.empty(n, dtype=torch.uint8, device=DEV),
                torch.empty(n, dtype=torch.float32, device=DEV))
        # An allocation shows as free memory shrinking across the call.  The
        # HIP runtime may hand scratch backing that earlier kernels of the
        # process used back to the device at any moment, which shows as free
        # memory growing; such a call is repeated (at most three times) until
        # one leaves the free memory exactly unchanged, and no call may shrink it.
        used = []
        for _ in range(3):
            torch.cuda.synchronize()
            free0 = torch.cuda.mem_get_info()[0]
            rn = pm.solve_noalloc(ctx, tg, ch.eps, s0, xi, u, variant="diag", max_iter=n + 1, out=outs)
            torch.cuda.synchronize()
            used.append(free0 - torch.cuda.mem_get_info()[0])
            if used[-1] == 0:
                break
        r = pm.solve(ctx, tg, ch.eps, s0, xi, u, variant="diag", max_iter=n + 1)
        print(f"  T={n}: sweeps {rn.sweeps} / {r.sweeps}, device memory taken per call {used} bytes", flush=True)
        assert max(used) <= 0 and used[-1] == 0, "the allocation-free call changed the device's free memory"
        assert rn.status == 0
        _same(rn, r)
    ctx.close()


def test_noalloc_limits(pm):
    print("noalloc: refusals", flush=True)
    from paper_2508_18413_amd import _binding as B
    ctx = pm.Context(0)
    ch = W.funnel_chain(T=3000, seed=5)
    g = pm.Target(ctx, ch.target)
    args = (ctx, g, ch.eps, _t(ch.x0), _t(ch.xi), _t(ch.u))
    with pytest.raises(B.PMCError) as e:
        pm.solve_noalloc(*args, variant="diag", max_iter=3001, graph_sweeps=4)
    assert e.value.status == B.PMC_ERR_UNSUPPORTED
    # 32 x 2^20 FP32 steps need 3 x 128 MiB of planes: more than the scratch
    big = W.funnel_chain(T=1 << 20, seed=5)
    gb = pm.Target(ctx, big.target)
    with pytest.raises(B.PMCError) as e:
        pm.solve_noalloc(ctx, gb, big.eps, _t(big.x0), _t(big.xi), _t(big.u), variant="diag", max_iter=4)
    assert e.value.status == B.PMC_ERR_INVALID
    # a problem that fits after the refusals still matches pmc_solve
    rn = pm.solve_noalloc(*args, variant="diag", max_iter=3001)
    r = pm.solve(*args, variant="diag", max_iter=3001)
    _same(rn, r)
    ctx.close()
