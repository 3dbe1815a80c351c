"""GPU parity of the parallel Newton path (through the C ABI) against the FP64
oracle, on seeded synthetic inputs.

Bars: FP64 state error <= 1e-10; FP32 state error <= 1e-5 (mixed
absolute/relative per step).  Accept patterns identical except for two
classes of resynchronised decisions (tests/parity.py), both recorded per
comparison: near-ties, |g~*| < 1e-6 (FP64 chains admit only these), and
FP32-floor ties, 1e-6 <= |g~*| < F32_GATE_ERR = 2e-5 (the pinned bound on the
FP32 error of g~, test_logreg_gate_precision), capped at one per 16384 steps
compared.  Scans: relative error <= 1e-12 (FP64) / 2e-5 (FP32) against the
sequential recursion.
"""
import numpy as np
import pytest

from conftest import oracle_burnin, oracle_target
from parity import compare_with_resync, floor_cap, record, state_error
from paper_2508_18413_amd import workloads as W

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
DEV = "cuda:0"


def _t(x, dtype=None):
    return torch.tensor(np.ascontiguousarray(x), dtype=dtype, device=DEV)


@pytest.fixture(scope="module")
def pm():
    import paper_2508_18413_amd as pm
    return pm


@pytest.fixture(scope="module")
def ctx(pm):
    c = pm.Context(0)
    yield c
    c.close()


def _say(*a):
    print(*a, flush=True)


# ------------------------------------------------------------- scans

@pytest.mark.parametrize("dtype", ["f32", "f64"])
@pytest.mark.parametrize("T", [1, 63, 64, 65, 2047, 4096, 4097, 100003])
def test_linrec_diag(ctx, pm, orc, dtype, T):
    _say(f"linrec_diag dtype={dtype} T={T}")
    rng = np.random.default_rng(T)
    lanes = 3
    a = rng.uniform(-0.98, 0.98, size=(lanes, T))
    b = rng.normal(size=(lanes, T))
    td = torch.float32 if dtype == "f32" else torch.float64
    ga, gb = _t(a, td), _t(b, td)
    out = pm.linrec_diag(ctx, ga, gb).cpu().numpy().astype(np.float64)
    ref = orc.linrec_diag(ga.cpu().numpy().T, gb.cpu().numpy().T).T
    tol = 2e-5 if dtype == "f32" else 1e-12
    assert np.max(np.abs(out - ref)) <= tol * max(1.0, np.max(np.abs(ref)))


def test_linrec_diag_exact_carries(ctx, pm):
    """a = 1, b = 1: delta_t = t + 1, exact in FP32 below 2^24 -- every carry
    across ~260 tiles must be exact; a = 0 returns b."""
    _say("linrec_diag exact carries T=2^20+17")
    T = (1 << 20) + 17
    ones = torch.ones((2, T), device=DEV)
    out = pm.linrec_diag(ctx, ones, ones)
    ref = torch.arange(1, T + 1, device=DEV, dtype=torch.float32)
    assert torch.equal(out[0], ref) and torch.equal(out[1], ref)
    b = torch.randn((4, 5000), device=DEV)
    assert torch.equal(pm.linrec_diag(ctx, torch.zeros_like(b), b), b)


def test_linrec_diag_large(ctx, pm, orc):
    _say("linrec_diag large T=2^20+17")
    T = (1 << 20) + 17
    rng = np.random.default_rng(5)
    a = rng.uniform(-0.99, 0.99, size=(2, T)).astype(np.float32)
    b = rng.normal(size=(2, T)).astype(np.float32)
    out = pm.linrec_diag(ctx, _t(a), _t(b)).cpu().numpy().astype(np.float64)
    ref = orc.linrec_diag(a.T, b.T).T
    assert np.max(np.abs(out - ref)) <= 2e-5 * max(1.0, np.max(np.abs(ref)))


def test_linrec_diag_large_vector_tiles(ctx, pm, orc):
    """8 lanes x 2^20 steps (the chunked scan): exact carries (a = 1, b = 1,
    where the correction covers every chunk in full) and a random recursion
    against the oracle."""
    _say("linrec_diag 8 x 2^20 (large tiles, vector path)")
    L, T = 8, 1 << 20
    ones = torch.ones((L, T), device=DEV)
    out = pm.linrec_diag(ctx, ones, ones)
    ref = torch.arange(1, T + 1, device=DEV, dtype=torch.float32)
    assert all(torch.equal(out[k], ref) for k in range(L))
    rng = np.random.default_rng(11)
    a = rng.uniform(-0.99, 0.99, size=(L, T)).astype(np.float32)
    b = rng.normal(size=(L, T)).astype(np.float32)
    out = pm.linrec_diag(ctx, _t(a), _t(b)).cpu().numpy().astype(np.float64)
    ref = orc.linrec_diag(a.T, b.T).T
    assert np.max(np.abs(out - ref)) <= 2e-5 * max(1.0, np.max(np.abs(ref)))


@pytest.mark.parametrize("L,T,lo,hi,zeros", [(5, (1 << 21) + 8192 * 3, -0.99, 0.99, True),
                                             (3, (1 << 22) - 8192, 0.999, 1.0, False),
                                             (300, 1 << 15, -0.9, 0.9, False)])
def test_linrec_diag_chunked(ctx, pm, orc, L, T, lo, hi, zeros):
    """Long recursions whose length is a multiple of the 8192-step tile take
    the chunked scan (each workgroup scans its chunk from a zero carry, then
    corrects the chunk's head with the true carry): chunk counts off the
    powers of two (a short last chunk), exact zeros in a (a correction ends
    at once), slowly decaying products (the correction runs over many tiles),
    and more lanes than compute units (one chunk per lane)."""
    _say(f"linrec_diag chunked L={L} T={T} a in [{lo}, {hi}] zeros={zeros}")
    rng = np.random.default_rng(L + T)
    a = rng.uniform(lo, hi, size=(L, T)).astype(np.float32)
    if zeros:
        a[:, ::4099] = 0.0
    b = rng.normal(size=(L, T)).astype(np.float32)
    out = pm.linrec_diag(ctx, _t(a), _t(b)).cpu().numpy().astype(np.float64)
    ref = orc.linrec_diag(a.T, b.T).T
    err = np.max(np.abs(out - ref)) / max(1.0, np.max(np.abs(ref)))
    _say(f"  max error / scale = {err:.3e}")
    assert err <= 2e-5


def test_linrec_block2_chunked(ctx, pm, orc):
    """2 x 2 blocks through the chunked scan: 5 lanes x (2^20 + 7 x 4096) steps."""
    _say("linrec_block2 chunked 5 x (2^20 + 7 x 4096)")
    L, T = 5, (1 << 20) + 7 * 4096
    rng = np.random.default_rng(13)
    coef = rng.uniform(-0.6, 0.6, size=(4, L, T)).astype(np.float32)
    rhs = rng.normal(size=(2, L, T)).astype(np.float32)
    out = pm.linrec_block2(ctx, _t(coef), _t(rhs)).cpu().numpy().astype(np.float64)
    c = coef.astype(np.float64)
    r = rhs.astype(np.float64)
    p, q = orc.linrec_block2(c[0].T, c[1].T, c[2].T, c[3].T, r[0].T, r[1].T)
    ref = np.stack([p.T, q.T])
    assert np.max(np.abs(out - ref)) <= 2e-5 * max(1.0, np.max(np.abs(ref)))


def test_scan_timing(pm):
    """pmc_set_scan_timing / pmc_last_scan_ms: off by default (0), then the
    scan kernel's own duration, shorter than the synchronising call."""
    import time
    c = pm.Context(0)
    try:
        a = torch.full((16, 1 << 20), 0.5, device=DEV)
        b = torch.ones((16, 1 << 20), device=DEV)
        pm.linrec_diag(c, a, b)
        assert c.last_scan_ms() == 0.0
        c.set_scan_timing(True)
        t0 = time.perf_counter()
        out = pm.linrec_diag(c, a, b)
        call_ms = 1e3 * (time.perf_counter() - t0)
        ms = c.last_scan_ms()
        _say(f"  scan kernel {ms:.4f} ms, call {call_ms:.4f} ms")
        assert 0.0 < ms < call_ms
        assert torch.allclose(out[:, -1], torch.full((16,), 2.0, device=DEV))
    finally:
        c.close()


def test_linrec_block2_large_vector_tiles(ctx, pm, orc):
    """2 lanes x 2^21 steps (the chunked scan for 2 x 2 blocks)."""
    _say("linrec_block2 2 x 2^21 (large tiles, vector path)")
    L, T = 2, 1 << 21
    rng = np.random.default_rng(12)
    coef = rng.uniform(-0.6, 0.6, size=(4, L, T)).astype(np.float32)
    rhs = rng.normal(size=(2, L, T)).astype(np.float32)
    out = pm.linrec_block2(ctx, _t(coef), _t(rhs)).cpu().numpy().astype(np.float64)
    c = coef.astype(np.float64)
    r = rhs.astype(np.float64)
    p, q = orc.linrec_block2(c[0].T, c[1].T, c[2].T, c[3].T, r[0].T, r[1].T)
    ref = np.stack([p.T, q.T])
    assert np.max(np.abs(out - ref)) <= 2e-5 * max(1.0, np.max(np.abs(ref)))


@pytest.mark.parametrize("T", [1, 1000, 5001])
def test_linrec_block2(ctx, pm, orc, T):
    _say(f"linrec_block2 T={T}")
    rng = np.random.default_rng(T + 7)
    lanes = 5
    coef = rng.uniform(-0.6, 0.6, size=(4, lanes, T)).astype(np.float32)
    rhs = rng.normal(size=(2, lanes, T)).astype(np.float32)
    out = pm.linrec_block2(ctx, _t(coef), _t(rhs)).cpu().numpy().astype(np.float64)
    c = coef.astype(np.float64)
    r = rhs.astype(np.float64)
    p, q = orc.linrec_block2(c[0].T, c[1].T, c[2].T, c[3].T, r[0].T, r[1].T)
    ref = np.stack([p.T, q.T])
    assert np.max(np.abs(out - ref)) <= 2e-5 * max(1.0, np.max(np.abs(ref)))


@pytest.mark.parametrize("D", [2, 3, 4])
@pytest.mark.parametrize("T", [1, 1000, 3001])
def test_linrec_dense_f64(ctx, pm, orc, D, T):
    _say(f"linrec_dense f64 D={D} T={T}")
    rng = np.random.default_rng(D * 1000 + T)
    A = rng.normal(size=(T, D, D)) / (1.2 * D)
    b = rng.normal(size=(T, D))
    out = pm.linrec_dense(ctx, _t(A), _t(b)).cpu().numpy()
    ref = orc.linrec_dense(A, b)
    assert np.max(np.abs(out - ref)) <= 1e-12 * max(1.0, np.max(np.abs(ref)))


# -------------------------------------------------------- Newton solves

def _banana(orc, T=1024, seed=0):
    ch = W.banana_chain(T=T, seed=seed)
    tg = oracle_target(ch.target)
    return ch, tg


@pytest.mark.parametrize("variant,kw", [("diag", {}), ("picard", {}),
                                        ("dense", dict(clip=1.0, clip_inf_norm=True)),
                                        ("dense", {})])
def test_banana_fp64(ctx, pm, orc, variant, kw):
    _say(f"banana fp64 variant={variant} {kw}")
    ch, tg = _banana(orc)
    g = pm.Target(ctx, ch.target, dtype=torch.float64)
    r = pm.solve(ctx, g, ch.eps, _t(ch.x0), _t(ch.xi), _t(ch.u), variant=variant,
                 max_iter=ch.T + 1, **kw)
    _say(f"  sweeps={r.sweeps} status={r.status} ratio={r.max_ratio:.3g}")
    assert r.status == 0
    gacc = r.accept.cpu().numpy()
    st, acc, rep = compare_with_resync(
        lambda f: orc.mala_chain(tg, ch.eps, ch.x0, ch.xi, ch.u, force=f), gacc)
    err = state_error(r.states.cpu().numpy(), st)
    record(f"banana T={ch.T} fp64", ch.T, err, rep)
    assert not [x for x in rep if x[2] == "failure"], rep
    assert err <= 1e-10
    assert r.n_accept == int(acc.sum())


def test_banana_golden_fixture(ctx, pm):
    """The first 32 steps against the stored oracle fixture (tests/golden)."""
    import json
    import os
    with open(os.path.join(os.path.dirname(__file__), "golden", "banana_mala_t32.json")) as f:
        gd = json.load(f)
    g = pm.Target(ctx, W.banana_target(), dtype=torch.float64)
    r = pm.solve(ctx, g, gd["eps"], _t(gd["x0"], torch.float64), _t(gd["xi"], torch.float64),
                 _t(gd["u"], torch.float64), variant="diag", max_iter=40)
    assert state_error(r.states.cpu().numpy(), np.array(gd["states"])) <= 1e-10
    assert np.array_equal(r.accept.cpu().numpy(), np.array(gd["accept"]))


def test_causal_exactness_trace(ctx, pm, orc):
    """After sweep i the first i states equal the sequential trace (FP64)."""
    _say("causal exactness trace")
    ch, tg = _banana(orc, T=48, seed=4)
    g = pm.Target(ctx, ch.target, dtype=torch.float64)
    for variant in ("diag", "picard"):
        r = pm.solve(ctx, g, ch.eps, _t(ch.x0), _t(ch.xi), _t(ch.u), variant=variant, max_iter=49,
                     want_trace=True, skip_converged_prefix=False)
        ref, _, _ = orc.mala_chain(tg, ch.eps, ch.x0, ch.xi, ch.u)
        tr = r.trace.cpu().numpy()
        for i in range(r.sweeps):
            k = i + 1
            assert np.max(np.abs(tr[i, :k] - ref[:k])) <= 1e-13, (variant, i)


@pytest.mark.parametrize("dtype", ["f64", "f32"])
def test_ula_gaussian_one_solve(ctx, pm, orc, dtype):
    """ULA on a Gaussian is affine: the first dense Newton solve is already the
    chain; Algorithm 1 stops after the confirming sweep."""
    _say(f"ula gaussian one solve {dtype}")
    td = torch.float64 if dtype == "f64" else torch.float32
    npd = np.float64 if dtype == "f64" else np.float32
    ch = W.gaussian_chain(3000, seed=2, eps=0.2, dim=4, dtype=npd, lam_lo=0.3)
    tg = oracle_target(ch.target)
    g = pm.Target(ctx, ch.target, dtype=td)
    r = pm.solve(ctx, g, ch.eps, _t(ch.x0, td), _t(ch.xi, td), None, sampler="ula",
                 variant="dense", max_iter=5, want_trace=True)
    ref, _, _ = orc.mala_chain(tg, ch.eps, ch.x0, ch.xi, None, ula=True)
    first = r.trace[0].cpu().numpy()
    tol = 1e-12 if dtype == "f64" else 1e-5
    assert state_error(first, ref) <= tol
    # the confirming sweep moves FP32 states by rounding only (a few ulps),
    # which the default 5e-7 stop may count as one more change
    assert r.sweeps == 2 if dtype == "f64" else r.sweeps <= 3
    assert r.status == 0


def test_newton_chunked_scan_ula_gaussian(ctx, pm, orc):
    """A single chain of 16 x 2^19 steps takes the chunked Newton scan (the
    scan tile divides T and the scan is large): ULA on a correlated Gaussian,
    quasi-DEER to the tolerance, against the FP64 oracle."""
    _say("chunked Newton scan: ULA Gaussian D=16 T=2^19")
    T = 1 << 19
    ch = W.gaussian_chain(T, seed=5, eps=0.1, dim=16, dtype=np.float32, lam_lo=0.3)
    tg = oracle_target(ch.target)
    g = pm.Target(ctx, ch.target)
    r = pm.solve(ctx, g, ch.eps, _t(ch.x0), _t(ch.xi), None, sampler="ula", variant="diag", max_iter=200)
    _say(f"  sweeps={r.sweeps} status={r.status} ratio={r.max_ratio:.3g}")
    assert r.status == 0
    ref, _, _ = orc.mala_chain(tg, ch.eps, ch.x0.astype(np.float64), ch.xi, None, ula=True)
    err = state_error(r.states.cpu().numpy(), ref)
    _say(f"  state_error={err:.3e}")
    assert err <= 1e-5


def test_newton_chunked_scan_logreg(ctx, pm, orc):
    """MALA on a logistic posterior (200 x 32 data, T = 2^18): the chunked
    Newton scan under the sliding window (the window start moves into the
    chunks' tiles) against the FP64 oracle."""
    _say("chunked Newton scan: MALA logreg D=32 N=200 T=2^18")
    T = 1 << 18
    ch = W.logreg_chain(T=T, seed=7, eps=0.002, n_data=200, dim=32)
    tg = oracle_target(ch.target)
    s0 = oracle_burnin(tg, ch).astype(np.float32)
    g = pm.Target(ctx, ch.target)
    r = pm.solve(ctx, g, ch.eps, _t(s0), _t(ch.xi), _t(ch.u), variant="diag", max_iter=T + 1)
    _say(f"  sweeps={r.sweeps} status={r.status} ratio={r.max_ratio:.3g} acceptance={r.n_accept / T:.3f}")
    assert r.status == 0
    _check_mala(orc, tg, ch, s0, r.states.cpu().numpy(), r.accept.cpu().numpy())


def test_probed_diagonal_trace_banana_fp64(ctx, pm, orc):
    """Stochastic diagonal (Sec. 3.4 eq. 10, one Rademacher probe per step and
    sweep): every sweep's iterate against the oracle's Newton reference with
    the same counter-based signs (FP64, no sliding window)."""
    _say("probed diagonal: banana FP64 trace")
    ch, tg = _banana(orc, T=48, seed=6)
    g = pm.Target(ctx, ch.target, dtype=torch.float64)
    r = pm.solve(ctx, g, ch.eps, _t(ch.x0), _t(ch.xi), _t(ch.u), variant="diag", max_iter=49,
                 want_trace=True, skip_converged_prefix=False, jac_probes=1, probe_seed=9)
    xi, u = np.asarray(ch.xi, dtype=np.float64), np.asarray(ch.u, dtype=np.float64)

    def sj(t, s):
        F, J, _ = orc.mala_jac(tg, ch.eps, s, xi[t], u[t])
        return F, J
    _, ref_trace, _ = orc.newton_reference(sj, np.asarray(ch.x0, dtype=np.float64), ch.T,
                                           variant="hutchinson", max_iter=r.sweeps, tol=-1.0, probe_seed=9)
    tr = r.trace.cpu().numpy()
    _say(f"  sweeps={r.sweeps} status={r.status}")
    assert r.status == 0
    for i in range(r.sweeps):
        assert np.max(np.abs(tr[i] - ref_trace[i + 1])) <= 1e-11, i


@pytest.mark.parametrize("case", ["banana_f64", "gaussian_f32"])
def test_probed_diagonal_converges_to_sequential(ctx, pm, orc, case):
    """The probed diagonal changes the sweeps, not the fixed point."""
    _say(f"probed diagonal: {case}")
    if case == "banana_f64":
        ch, tg = _banana(orc, T=1024, seed=8)
        g = pm.Target(ctx, ch.target, dtype=torch.float64)
        r = pm.solve(ctx, g, ch.eps, _t(ch.x0), _t(ch.xi), _t(ch.u), variant="diag", max_iter=ch.T + 1,
                     jac_probes=1, probe_seed=4)
        ref, _, _ = orc.mala_chain(tg, ch.eps, ch.x0, ch.xi, ch.u)
        tol = 1e-10
    else:
        ch = W.gaussian_chain(4096, seed=9, eps=0.1, dim=8, dtype=np.float32, lam_lo=0.3)
        tg = oracle_target(ch.target)
        g = pm.Target(ctx, ch.target)
        r = pm.solve(ctx, g, ch.eps, _t(ch.x0), _t(ch.xi), None, sampler="ula", variant="diag",
                     max_iter=400, jac_probes=1, probe_seed=4)
        ref, _, _ = orc.mala_chain(tg, ch.eps, ch.x0.astype(np.float64), ch.xi, None, ula=True)
        tol = 1e-5
    err = state_error(r.states.cpu().numpy(), ref)
    _say(f"  sweeps={r.sweeps} status={r.status} state_error={err:.3e}")
    assert r.status == 0
    assert err <= tol


def test_logreg_probed_diagonal_batch_one_sweep(ctx, pm, orc):
    """The probed logistic diagonal for chains laid end to end (lengths not
    multiples of 32, so 32-step groups straddle chains): one ULA sweep from a
    perturbed guess, each chain against the oracle's FP64 Hutchinson sweep
    drawn at the chain's global steps and started from its own s0."""
    _say("logreg probed diagonal batch one sweep")
    b = W.logreg_batch(seed=6, n_chains=3, lo=200, hi=700, eps=0.0015)
    tg = oracle_target(b.target)
    rng = np.random.default_rng(9)
    guess = np.empty_like(b.xi)
    refs = []
    for c in range(b.n_chains):
        o0, o1 = b.offsets[c], b.offsets[c + 1]
        ref, _, _ = orc.mala_chain(tg, b.eps, b.x0[c].astype(np.float64), b.xi[o0:o1].astype(np.float64), None,
                                   ula=True)
        guess[o0:o1] = ref + 0.05 * rng.standard_normal(ref.shape)
        refs.append(ref)
    g = pm.Target(ctx, b.target)
    r = pm.solve(ctx, g, b.eps, _t(b.x0), _t(b.xi), None, sampler="ula", offsets=list(b.offsets), variant="diag",
                 jac_probes=1, probe_seed=77, init_guess=_t(guess), max_iter=1, want_trace=True)
    got = r.trace[0].cpu().numpy().astype(np.float64)
    _say(f"  lens={np.diff(b.offsets).tolist()}")
    for c in range(b.n_chains):
        o0, o1 = int(b.offsets[c]), int(b.offsets[c + 1])
        x0 = b.x0[c].astype(np.float64)
        xi = b.xi[o0:o1].astype(np.float64)
        g64 = guess[o0:o1].astype(np.float64)

        def sj(t, s):
            F, J, _ = orc.mala_jac(tg, b.eps, s, xi[t], 0.5, ula=True)
            return F, J
        want, _, _ = orc.newton_reference(sj, x0, o1 - o0, variant="hutchinson", init=g64, max_iter=1,
                                          full_trace=False, probe_seed=77, step0=o0)
        F = np.array([sj(t, x0 if t == 0 else g64[t - 1])[0] for t in range(o1 - o0)])
        jterm = np.max(np.abs(want - F))
        err = np.max(np.abs(got[o0:o1] - want))
        _say(f"  chain {c}: |J part| {jterm:.3e}  gpu error {err:.3e}")
        assert err <= 0.02 * jterm


def test_logreg_probed_diagonal_batch_mala(ctx, pm, orc):
    """Batched uneven chains with the probed diagonal converge, each to its
    FP64 sequential chain."""
    _say("logreg probed diagonal batch mala")
    b = W.logreg_batch(seed=3, n_chains=6, lo=1, hi=9000, eps=0.0015)
    lens = np.diff(b.offsets)
    tg = oracle_target(b.target)
    s0 = np.stack([oracle_burnin(tg, _as_chain(b, c)) for c in range(b.n_chains)]).astype(np.float32)
    g = pm.Target(ctx, b.target)
    r = pm.solve(ctx, g, b.eps, _t(s0), _t(b.xi), _t(b.u), offsets=list(b.offsets), variant="diag", jac_probes=1,
                 probe_seed=5, max_iter=int(lens.max()) + 1)
    _say(f"  lens={lens.tolist()} sweeps/chain={r.sweeps_per_chain}")
    assert r.status == 0 and r.n_converged == b.n_chains
    st = r.states.cpu().numpy()
    acc = r.accept.cpu().numpy()
    for c in range(b.n_chains):
        o0, o1 = b.offsets[c], b.offsets[c + 1]
        _check_mala(orc, tg, _as_chain(b, c), s0[c], st[o0:o1], acc[o0:o1])


@pytest.mark.parametrize("shape", ["d25n1000", "d5n50", "d32n300"])
def test_logreg_probed_diagonal_one_sweep(ctx, pm, orc, shape):
    """One-probe diagonal z o (J z) of the logistic posterior (matrix-core
    J z): one ULA sweep from a perturbed guess against the oracle's FP64
    sweep with the same counter-based probe.  The Jacobian's part of the
    update is matched to 2 % (BF16 operands); the sweep with the exact
    diagonal misses it by far more, so the probe's off-diagonal terms (and
    its signs) are checked."""
    dim, n_data, eps = DENSE_SHAPES[shape]
    _say(f"logreg probed diagonal one sweep D={dim} N={n_data}")
    T, seed = 1024, 1234
    ch = W.logreg_chain(T=T, seed=4, eps=eps, n_data=n_data, dim=dim)
    tg = oracle_target(ch.target)
    x0 = ch.x0.astype(np.float64)
    xi = ch.xi.astype(np.float64)
    ref, _, _ = orc.mala_chain(tg, ch.eps, x0, xi, None, ula=True)
    guess = (ref + 0.05 * np.random.default_rng(8).standard_normal(ref.shape)).astype(np.float32)
    g64 = guess.astype(np.float64)
    g = pm.Target(ctx, ch.target)
    r = pm.solve(ctx, g, ch.eps, _t(ch.x0), _t(ch.xi), None, sampler="ula", variant="diag", jac_probes=1,
                 probe_seed=seed, init_guess=_t(guess), max_iter=1, want_trace=True)
    got = r.trace[0].cpu().numpy().astype(np.float64)

    def sj(t, s):
        F, J, _ = orc.mala_jac(tg, ch.eps, s, xi[t], 0.5, ula=True)
        return F, J
    want, _, _ = orc.newton_reference(sj, x0, T, variant="hutchinson", init=g64, max_iter=1, full_trace=False,
                                      probe_seed=seed)
    exact, _, _ = orc.newton_reference(sj, x0, T, variant="diag", init=g64, max_iter=1, full_trace=False)
    F = np.array([sj(t, x0 if t == 0 else g64[t - 1])[0] for t in range(T)])
    jterm = np.max(np.abs(want - F))
    err = np.max(np.abs(got - want))
    miss = np.max(np.abs(exact - want))
    _say(f"  |J part| {jterm:.3e}  gpu error {err:.3e}  exact-diagonal miss {miss:.3e}")
    assert jterm > 1e-2
    assert err <= 0.02 * jterm
    assert miss >= 5 * err


def test_logreg_probed_diagonal_mala(ctx, pm, orc):
    """Quasi-DEER with the one-probe diagonal (a fresh probe every sweep) on
    the logistic posterior converges to the FP64 sequential chain."""
    _say("logreg probed diagonal mala")
    ch, tg, s0 = _logreg_case(orc, 4096, 0.0015)
    g = pm.Target(ctx, ch.target)
    r = pm.solve(ctx, g, ch.eps, _t(s0), _t(ch.xi), _t(ch.u), variant="diag", jac_probes=1, probe_seed=7,
                 max_iter=ch.T + 1)
    rd = pm.solve(ctx, g, ch.eps, _t(s0), _t(ch.xi), _t(ch.u), variant="diag", max_iter=ch.T + 1)
    _say(f"  probed sweeps={r.sweeps} (exact diagonal {rd.sweeps}) status={r.status} floor={r.n_floor}")
    assert r.status == 0
    _check_mala(orc, tg, ch, s0, r.states.cpu().numpy(), r.accept.cpu().numpy())


def _logreg_case(orc, T, eps, seed=0):
    ch = W.logreg_chain(T=T, seed=seed, eps=eps)
    tg = oracle_target(ch.target)
    s0 = oracle_burnin(tg, ch).astype(np.float32)
    return ch, tg, s0


# Near-tie band of FP32 chains: the bound on |g~ - g~*| that
# test_logreg_gate_precision pins for one FP32 evaluation at given states.
# On the logistic posterior the log ratio's terms reach ~1e2 and cancel to
# O(1), so FP32 predictors and gradient sums leave errors of several 1e-6 in
# g~; a decision flip closer to the threshold than that is a tie in FP32.
F32_GATE_ERR = 2e-5


def _check_mala(orc, tg, ch, s0, got_states, got_acc, tol=1e-5, label=None):
    """State error and accept pattern of one chain against the oracle; both
    tie classes are recorded, and the FP32-floor class is capped."""
    x0 = s0.astype(np.float64)
    fp32 = np.asarray(got_states).dtype == np.float32
    st, acc, rep = compare_with_resync(
        lambda f: orc.mala_chain(tg, ch.eps, x0, ch.xi, ch.u, force=f), got_acc,
        floor_band=F32_GATE_ERR if fp32 else None)
    err = state_error(got_states, st)
    n = len(got_acc)
    n_tie, n_floor = record(label or f"T={n} {'fp32' if fp32 else 'fp64'}", n, err, rep)
    _say(f"  state_error={err:.3e} near-ties={n_tie} fp32-floor={n_floor} mismatches={rep}")
    assert not [x for x in rep if x[2] == "failure"], rep
    assert n_floor <= floor_cap(n), (n_floor, rep)
    assert err <= tol
    return err, rep


@pytest.mark.parametrize("products", ["split16", "f32", "refine"])
@pytest.mark.parametrize("T", [4096, 5000])
def test_logreg_diag_fp32(ctx, pm, orc, T, products):
    _say(f"logreg diag fp32 T={T} products={products}")
    ch, tg, s0 = _logreg_case(orc, T, 0.0015)
    g = pm.Target(ctx, dict(ch.target, products=products))
    r = pm.solve(ctx, g, ch.eps, _t(s0), _t(ch.xi), _t(ch.u), variant="diag", max_iter=T + 1)
    _say(f"  sweeps={r.sweeps} status={r.status} ratio={r.max_ratio:.3g}")
    assert r.status == 0
    _check_mala(orc, tg, ch, s0, r.states.cpu().numpy(), r.accept.cpu().numpy())


def _gate_at(orc, tg, ch, s0, states):
    """The oracle's g~* of every step taken from the given (FP32) states."""
    prev = np.concatenate([np.asarray(s0)[None, :], np.asarray(states)[:-1]]).astype(np.float64)
    return np.array([orc.mala_step(tg, ch.eps, prev[t], ch.xi[t], ch.u[t])[2] for t in range(prev.shape[0])])


def test_logreg_gate_precision(ctx, pm, orc):
    """One parallel evaluation at the oracle's trajectory (rounded to FP32),
    with either product arithmetic, and the sequential sampler along its own
    trajectory: each step's g~ against the oracle's g~* from the same FP32
    states, and the decisions wherever |g~*| exceeds that error."""
    T = 2048
    for seed in (0, 1):
        ch, tg, s0 = _logreg_case(orc, T, 0.0015, seed=seed)
        st, _, _ = orc.mala_chain(tg, ch.eps, s0.astype(np.float64), ch.xi, ch.u)
        init = st.astype(np.float32)
        ref = _gate_at(orc, tg, ch, s0, init)
        for products in ("split16", "f32"):
            g = pm.Target(ctx, dict(ch.target, products=products))
            r = pm.solve(ctx, g, ch.eps, _t(s0), _t(ch.xi), _t(ch.u), variant="diag", max_iter=1,
                         init_guess=_t(init))
            got = r.gtilde.cpu().numpy().astype(np.float64)
            err = np.abs(got - ref)
            _say(f"  seed {seed} parallel eval ({products}): max |g~ - g~*| = {err.max():.3e}, "
                 f"p99 {np.quantile(err, 0.99):.3e}")
            assert err.max() <= F32_GATE_ERR
            clear = np.abs(ref) > F32_GATE_ERR
            assert np.array_equal(r.accept.cpu().numpy()[clear].astype(bool), ref[clear] > 0)

        rs = pm.sample_sequential(ctx, g, ch.eps, _t(s0), _t(ch.xi), _t(ch.u))
        sst = rs.states.cpu().numpy()
        ref = _gate_at(orc, tg, ch, s0, sst)
        err = np.abs(rs.gtilde.cpu().numpy().astype(np.float64) - ref)
        _say(f"  seed {seed} sequential: max |g~ - g~*| = {err.max():.3e}, p99 {np.quantile(err, 0.99):.3e}")
        assert err.max() <= F32_GATE_ERR


def test_logreg_refined_products(ctx, pm, orc):
    """Refined products: split-FP16 sweeps until the chain meets the tolerance,
    then FP32-product sweeps from its first step until it meets it again.
    The result is a converged point of the FP32-product iteration: one more
    FP32-product sweep started from it moves no step by more than the
    tolerance (this chain has no decision within the FP32 error of g~ of its
    threshold, where a further sweep could take the other side).  With a fixed-width window the chains use FP32 products
    throughout, bit for bit what FP32 products give; more data points than
    the FP32 image holds are refused at target creation."""
    _say("logreg refined products")
    from paper_2508_18413_amd._binding import PMCError
    T = 8192
    ch, tg, s0 = _logreg_case(orc, T, 0.0015, seed=2)
    gr = pm.Target(ctx, dict(ch.target, products="refine"))
    gf = pm.Target(ctx, dict(ch.target, products="f32"))
    gs = pm.Target(ctx, dict(ch.target, products="split16"))
    a = (_t(s0), _t(ch.xi), _t(ch.u))
    kw = dict(variant="diag", max_iter=T + 1)
    rr = pm.solve(ctx, gr, ch.eps, *a, **kw)
    rf = pm.solve(ctx, gf, ch.eps, *a, **kw)
    rs = pm.solve(ctx, gs, ch.eps, *a, **kw)
    _say(f"  sweeps refine {rr.sweeps} (split16 alone {rs.sweeps}, f32 alone {rf.sweeps}); "
         f"max |refine - f32| {(rr.states - rf.states).abs().max().item():.3e}")
    assert rr.status == 0 and rr.sweeps > rs.sweeps
    one = pm.solve(ctx, gf, ch.eps, *a, **dict(kw, max_iter=1), init_guess=rr.states)
    _say(f"  one FP32 sweep from the refined result: ratio {one.max_ratio:.3g}")
    assert one.status == 0 and one.max_ratio <= 1.0
    clear = one.gtilde.abs() > F32_GATE_ERR
    assert torch.equal(one.accept[clear], rr.accept[clear])
    _check_mala(orc, tg, ch, s0, rr.states.cpu().numpy(), rr.accept.cpu().numpy())
    # the same solve from a graph of 8 sweeps: the phase switch happens on
    # the device, so the replays give the eager result bit for bit
    rg = pm.solve(ctx, gr, ch.eps, *a, **dict(kw, graph_sweeps=8))
    assert rg.sweeps == rr.sweeps and torch.equal(rg.states, rr.states) and torch.equal(rg.accept, rr.accept)
    # max_iter reached by the split-FP16 phase itself: no FP32-product sweep
    # is left, so the chain is reported not converged after exactly max_iter
    short = pm.solve(ctx, gr, ch.eps, *a, **dict(kw, max_iter=rs.sweeps))
    assert short.sweeps == rs.sweeps and short.status == pm.B.PMC_NOT_CONVERGED
    assert list(short.chain_state) == [2]
    # fixed-width windows: FP32 products from the start
    wkw = dict(kw, window_width=1024)
    w1 = pm.solve(ctx, gr, ch.eps, *a, **wkw)
    w2 = pm.solve(ctx, gf, ch.eps, *a, **wkw)
    assert torch.equal(w1.states, w2.states) and w1.sweeps == w2.sweeps
    big = W.logreg_chain(T=64, seed=5, eps=0.001, n_data=1200, dim=8)
    with pytest.raises(PMCError, match="refined products"):
        pm.Target(ctx, dict(big.target, products="refine"))


def test_logreg_products_routing(ctx, pm):
    """Split-FP16 products need the LDS image (n_data <= 1216): asked for with
    more data points they are refused at target creation, and AUTO then runs
    the FP32-product kernels, bit for bit what asking for FP32 products gives."""
    _say("logreg products routing")
    from paper_2508_18413_amd._binding import PMCError
    ch = W.logreg_chain(T=1024, seed=5, eps=0.001, n_data=1300, dim=8)
    with pytest.raises(PMCError, match="split-FP16"):
        pm.Target(ctx, dict(ch.target, products="split16"))
    outs = []
    for products in ("auto", "f32"):
        g = pm.Target(ctx, dict(ch.target, products=products))
        outs.append(pm.solve(ctx, g, ch.eps, _t(ch.x0), _t(ch.xi), _t(ch.u), variant="diag",
                             max_iter=60))
    assert torch.equal(outs[0].states, outs[1].states)
    assert torch.equal(outs[0].accept, outs[1].accept)


@pytest.mark.parametrize("x_scale,w_scale,prior_var", [(1e-4, 2e4, 1e10), (100.0, 1e-2, 1.0),
                                                       (1.0, 1e-3, 1e-6)])
def test_logreg_split16_scaled_data(ctx, pm, orc, x_scale, w_scale, prior_var):
    """Data and coefficients far from unit scale: columns of X of order 1e-4 or
    1e2, iterates of order 1e4 or 1e-3.  The split-FP16 path brings every
    operand to FP16's range with power-of-two scalings (per column of X, and
    per 32-step tile for the iterate and the increment); parity with the
    oracle as for any FP32 chain."""
    _say(f"logreg split16 scaled data X*{x_scale} w*{w_scale} prior_var={prior_var}")
    r = np.random.default_rng(11)
    N, D, T = 256, 8, 2048
    X = (r.standard_normal((N, D)) * x_scale).astype(np.float32)
    w = r.standard_normal(D) * w_scale
    p = 1.0 / (1.0 + np.exp(-(X.astype(np.float64) @ w)))
    y = (r.random(N) < p).astype(np.float32)
    # step size from the curvature at w: proposal variance 2 eps = 0.5 / max_d H_dd
    h = (X.astype(np.float64) ** 2 * (p * (1 - p))[:, None]).sum(axis=0) + 1.0 / prior_var
    eps = 0.25 / h.max()
    target = dict(kind="logreg", dim=D, X=X, y=y, prior_var=prior_var)
    ch = W.Chain(target=target, eps=eps, x0=w.astype(np.float32),
                 xi=r.standard_normal((T, D)).astype(np.float32), u=r.random(T).astype(np.float32))
    tg = oracle_target(target)
    g = pm.Target(ctx, dict(target, products="split16"))
    res = pm.solve(ctx, g, ch.eps, _t(ch.x0), _t(ch.xi), _t(ch.u), variant="diag", max_iter=T + 1)
    _say(f"  eps={eps:.3g} sweeps={res.sweeps} status={res.status} acceptance={res.n_accept / T:.3f}")
    assert res.status == 0
    _check_mala(orc, tg, ch, ch.x0, res.states.cpu().numpy(), res.accept.cpu().numpy())


def test_logreg_large_n_fallback_fp32(ctx, pm, orc):
    """N = 1300 data points, more 32-row tiles than the LDS image holds: the
    evaluation takes its operands from global memory instead."""
    _say("logreg N=1300 D=8 fp32 (global-memory evaluation)")
    ch = W.logreg_chain(T=2048, seed=3, eps=0.001, n_data=1300, dim=8)
    tg = oracle_target(ch.target)
    s0 = oracle_burnin(tg, ch).astype(np.float32)
    g = pm.Target(ctx, ch.target)
    r = pm.solve(ctx, g, ch.eps, _t(s0), _t(ch.xi), _t(ch.u), variant="diag", max_iter=2049)
    _say(f"  sweeps={r.sweeps} status={r.status} acceptance={r.n_accept / 2048:.3f}")
    assert r.status == 0
    _check_mala(orc, tg, ch, s0, r.states.cpu().numpy(), r.accept.cpu().numpy())
    rs = pm.sample_sequential(ctx, g, ch.eps, _t(s0), _t(ch.xi), _t(ch.u))
    _check_mala(orc, tg, ch, s0, rs.states.cpu().numpy(), rs.accept.cpu().numpy())


def test_logreg_sequential_fp32(ctx, pm, orc):
    _say("logreg sequential fp32")
    ch, tg, s0 = _logreg_case(orc, 4096, 0.0015)
    g = pm.Target(ctx, ch.target)
    r = pm.sample_sequential(ctx, g, ch.eps, _t(s0), _t(ch.xi), _t(ch.u))
    _check_mala(orc, tg, ch, s0, r.states.cpu().numpy(), r.accept.cpu().numpy())


@pytest.mark.parametrize("variant", ["diag", "picard"])
def test_funnel_fp32(ctx, pm, orc, variant):
    _say(f"funnel fp32 {variant}")
    ch = W.funnel_chain(T=2048, seed=1)
    tg = oracle_target(ch.target)
    g = pm.Target(ctx, ch.target)
    r = pm.solve(ctx, g, ch.eps, _t(ch.x0), _t(ch.xi), _t(ch.u), variant=variant,
                 max_iter=ch.T + 1)
    _say(f"  sweeps={r.sweeps} status={r.status}")
    _check_mala(orc, tg, ch, ch.x0, r.states.cpu().numpy(), r.accept.cpu().numpy())


@pytest.mark.parametrize("kind", ["banana", "funnel"])
def test_surrogate_gate(ctx, pm, orc, kind):
    """The stop-gradient Jacobian changes sweep counts, never the fixed point."""
    _say(f"surrogate gate {kind}")
    if kind == "banana":
        ch = W.banana_chain(1024, seed=2)
        td, x0 = torch.float64, ch.x0
        tol = 1e-10
    else:
        ch = W.funnel_chain(T=1024, seed=3)
        td, x0 = torch.float32, ch.x0
        tol = 1e-5
    tg = oracle_target(ch.target)
    g = pm.Target(ctx, ch.target, dtype=td)
    r = pm.solve(ctx, g, ch.eps, _t(x0, td), _t(ch.xi, td), _t(ch.u, td), variant="diag",
                 gate="surrogate", max_iter=ch.T + 1)
    _say(f"  sweeps={r.sweeps}")
    _check_mala(orc, tg, ch, np.asarray(x0), r.states.cpu().numpy(), r.accept.cpu().numpy(), tol)


@pytest.mark.parametrize("products", ["auto", "refine"])
def test_batched_uneven_chains(ctx, pm, orc, products):
    _say(f"batched uneven chains products={products}")
    b = W.logreg_batch(seed=3, n_chains=6, lo=1, hi=9000, eps=0.0015)
    lens = np.diff(b.offsets)
    tg = oracle_target(b.target)
    s0 = np.stack([oracle_burnin(tg, _as_chain(b, c)) for c in range(b.n_chains)]).astype(np.float32)
    g = pm.Target(ctx, dict(b.target, products=products))
    r = pm.solve(ctx, g, b.eps, _t(s0), _t(b.xi), _t(b.u), offsets=list(b.offsets),
                 variant="diag", max_iter=int(lens.max()) + 1)
    _say(f"  lens={lens.tolist()} sweeps/chain={r.sweeps_per_chain}")
    assert r.status == 0 and r.n_converged == b.n_chains
    st = r.states.cpu().numpy()
    acc = r.accept.cpu().numpy()
    for c in range(b.n_chains):
        o0, o1 = b.offsets[c], b.offsets[c + 1]
        ch = _as_chain(b, c)
        _check_mala(orc, tg, ch, s0[c], st[o0:o1], acc[o0:o1])


def _as_chain(b, c):
    o0, o1 = b.offsets[c], b.offsets[c + 1]
    return W.Chain(target=b.target, eps=b.eps, x0=b.x0[c], xi=b.xi[o0:o1], u=b.u[o0:o1],
                   burn_xi=b.burn_xi[c], burn_u=b.burn_u[c])


def test_graph_mode_matches_eager(ctx, pm):
    _say("graph mode vs eager")
    ch = W.funnel_chain(T=3000, seed=5)
    g = pm.Target(ctx, ch.target)
    args = (ctx, g, ch.eps, _t(ch.x0), _t(ch.xi), _t(ch.u))
    r0 = pm.solve(*args, variant="diag", max_iter=3001)
    for m in (1, 3, 8):
        r1 = pm.solve(*args, variant="diag", max_iter=3001, graph_sweeps=m)
        assert torch.equal(r0.states, r1.states), m
        assert torch.equal(r0.accept, r1.accept), m
        assert r1.sweeps == r0.sweeps


def test_sweep_batches_and_max_iter(ctx, pm):
    """Sweeps are enqueued several at a time between status reads: a solve
    capped by max_iter runs exactly max_iter sweeps, a solve capped at its own
    sweep count equals the uncapped one (sweeps queued after convergence change
    nothing), and the profiled step count covers the executed sweeps only."""
    _say("sweep batches and max_iter")
    ch = W.funnel_chain(T=3000, seed=5)
    g = pm.Target(ctx, ch.target)
    args = (ctx, g, ch.eps, _t(ch.x0), _t(ch.xi), _t(ch.u))
    r = pm.solve(*args, variant="diag", max_iter=3001)
    assert r.status == 0
    for cap in (1, 7, 8, 13):
        if cap >= r.sweeps:
            continue
        rc = pm.solve(*args, variant="diag", max_iter=cap)
        assert rc.status == pm.B.PMC_NOT_CONVERGED, cap
        assert rc.sweeps == cap and rc.sweeps_per_chain == [cap], (cap, rc.sweeps)
    rx = pm.solve(*args, variant="diag", max_iter=r.sweeps)
    assert rx.status == 0 and rx.sweeps == r.sweeps
    assert torch.equal(rx.states, r.states) and torch.equal(rx.accept, r.accept)
    rp = pm.solve(*args, variant="diag", max_iter=3001, profile_kernels=True)
    assert torch.equal(rp.states, r.states) and rp.sweeps == r.sweeps
    assert 0 < rp.eval_steps <= r.sweeps * 3000
    assert rp.eval_steps >= 3000  # the first sweep evaluates every step


def test_max_iter_counts_with_fixed_windows(ctx, pm):
    """A solve stopped by max_iter runs exactly max_iter sweeps on every chain
    that was still iterating, also when the last sweep moved a fixed-width
    window on; such a chain is reported as not converged."""
    _say("max_iter with fixed-width windows")
    b = W.logreg_batch(seed=4, n_chains=3, lo=600, hi=1500, eps=0.0015)
    g = pm.Target(ctx, b.target)
    args = (_t(b.x0), _t(b.xi), _t(b.u))
    full = pm.solve(ctx, g, b.eps, *args, offsets=list(b.offsets), variant="diag", window_width=128,
                    max_iter=20000)
    assert full.status == 0
    for m in range(3, 40, 3):
        r = pm.solve(ctx, g, b.eps, *args, offsets=list(b.offsets), variant="diag", window_width=128, max_iter=m)
        spc, cst = list(r.sweeps_per_chain), list(r.chain_state)
        assert max(spc) <= m, (m, spc)
        for c in range(b.n_chains):
            if cst[c] == 0:  # converged: its count is the unlimited solve's
                assert spc[c] == full.sweeps_per_chain[c], (m, c, spc, full.sweeps_per_chain)
            elif cst[c] == 2:  # stopped by max_iter
                assert spc[c] == m, (m, c, spc, cst)


def test_sliding_window_prefix_skip(ctx, pm, orc):
    _say("sliding window")
    ch, tg, s0 = _logreg_case(orc, 4096, 0.0015, seed=1)
    g = pm.Target(ctx, ch.target)
    r = pm.solve(ctx, g, ch.eps, _t(s0), _t(ch.xi), _t(ch.u), variant="diag", max_iter=4097,
                 skip_converged_prefix=True)
    _say(f"  sweeps={r.sweeps} status={r.status}")
    assert r.status == 0
    _check_mala(orc, tg, ch, s0, r.states.cpu().numpy(), r.accept.cpu().numpy())


def test_invalid_arguments(ctx, pm):
    from paper_2508_18413_amd import _binding as B
    ch = W.funnel_chain(T=100, seed=1, dim=8)
    g = pm.Target(ctx, ch.target)
    with pytest.raises(B.PMCError) as e:
        pm.solve(ctx, g, ch.eps, _t(ch.x0), _t(ch.xi), _t(ch.u), offsets=[0, 50])
    assert e.value.status == B.PMC_ERR_INVALID
    with pytest.raises(B.PMCError) as e:
        pm.solve(ctx, g, ch.eps, _t(ch.x0), _t(ch.xi), _t(ch.u), variant="block2")
    assert e.value.status == B.PMC_ERR_UNSUPPORTED
    # per-lane Gaussian evaluation stops at D = 16 (its private arrays beyond
    # that would not fit the per-lane stack); the solve and the sequential
    # sampler both refuse D = 20 before any launch
    gc = W.gaussian_chain(64, seed=1, eps=0.1, dim=20, dtype=np.float32, lam_lo=0.3)
    gg = pm.Target(ctx, gc.target)
    for call in (pm.solve, pm.sample_sequential):
        with pytest.raises(B.PMCError) as e:
            call(ctx, gg, gc.eps, _t(gc.x0), _t(gc.xi), _t(gc.u))
        assert e.value.status == B.PMC_ERR_UNSUPPORTED


def test_empty_and_length_one(ctx, pm, orc):
    ch = W.banana_chain(1, seed=9)
    g = pm.Target(ctx, ch.target, dtype=torch.float64)
    r = pm.solve(ctx, g, ch.eps, _t(ch.x0), _t(ch.xi), _t(ch.u), variant="diag")
    ref, _, _ = orc.mala_chain(orc.Target(orc.BANANA, 2), ch.eps, ch.x0, ch.xi, ch.u)
    assert state_error(r.states.cpu().numpy(), ref) <= 1e-12 and r.sweeps == 2
    e = pm.solve(ctx, g, ch.eps, _t(ch.x0), _t(ch.xi[:0].reshape(0, 2)), _t(ch.u[:0]))
    assert e.states.shape == (0, 2) and e.status == 0


# ------------------------------------------------ matrix-core dense DEER

@pytest.mark.parametrize("jac", ["f32", "bf16"])
@pytest.mark.parametrize("D,T", [(32, 1), (32, 31), (32, 33), (25, 1000), (7, 4097), (32, 40000)])
def test_linrec_dense_mfma(ctx, pm, orc, jac, D, T):
    """F32 compositions match the sequential recursion to FP32 accuracy; BF16
    compositions (one solve, no refinement) to the BF16 product bound."""
    _say(f"linrec_dense mfma {jac} D={D} T={T}")
    rng = np.random.default_rng(D * 7 + T)
    A = (rng.normal(size=(T, D, D)) / (1.6 * np.sqrt(D))).astype(np.float32)
    b = rng.normal(size=(T, D)).astype(np.float32)
    out = pm.linrec_dense(ctx, _t(A), _t(b), jac_prec=jac).cpu().numpy().astype(np.float64)
    ref = orc.linrec_dense(A.astype(np.float64), b.astype(np.float64))
    rel = np.max(np.abs(out - ref)) / max(1.0, np.max(np.abs(ref)))
    _say(f"  rel={rel:.3e}")
    assert rel <= (2e-5 if jac == "f32" else 4e-2)


@pytest.mark.parametrize("jac", ["f32", "bf16"])
def test_funnel_dense_deer(ctx, pm, orc, jac):
    _say(f"funnel dense DEER {jac}")
    ch = W.funnel_chain(T=4096, seed=1)
    tg = oracle_target(ch.target)
    g = pm.Target(ctx, ch.target)
    r = pm.solve(ctx, g, ch.eps, _t(ch.x0), _t(ch.xi), _t(ch.u), variant="dense", jac_prec=jac,
                 max_iter=ch.T + 1)
    rd = pm.solve(ctx, g, ch.eps, _t(ch.x0), _t(ch.xi), _t(ch.u), variant="diag", max_iter=ch.T + 1)
    _say(f"  dense sweeps={r.sweeps} (diag {rd.sweeps}) status={r.status} floor={r.n_floor}")
    assert r.status == 0
    _check_mala(orc, tg, ch, ch.x0, r.states.cpu().numpy(), r.accept.cpu().numpy())


@pytest.mark.parametrize("jac", ["bf16", "f32"])
def test_funnel_dense_deer_full_length(ctx, pm, orc, jac):
    """The funnel at its full length, D = 32, T = 16384: full DEER on the
    matrix-core dense scan against the FP64 chain."""
    _say(f"funnel dense DEER T=16384 {jac}")
    ch = W.funnel_chain(T=16384, seed=4)
    tg = oracle_target(ch.target)
    g = pm.Target(ctx, ch.target)
    r = pm.solve(ctx, g, ch.eps, _t(ch.x0), _t(ch.xi), _t(ch.u), variant="dense", jac_prec=jac,
                 max_iter=ch.T + 1)
    _say(f"  dense sweeps={r.sweeps} status={r.status} floor={r.n_floor} {r.elapsed_ms:.1f} ms")
    assert r.status == 0
    _check_mala(orc, tg, ch, ch.x0, r.states.cpu().numpy(), r.accept.cpu().numpy(),
                label=f"funnel dense {jac} T=16384")


@pytest.mark.parametrize("jac", ["bf16", "f32"])
def test_batched_dense_deer_logreg(ctx, pm, orc, jac):
    """Full DEER on uneven logistic chains laid end to end in one solve (chain
    lengths not multiples of the 32-step tile, from 1 step to several levels
    of the matrix-core hierarchy): each chain against its FP64 sequential
    chain from its own burned-in start."""
    _say(f"batched dense DEER logreg {jac}")
    b = W.logreg_batch(seed=3, n_chains=6, lo=1, hi=9000, eps=0.0015)
    lens = np.diff(b.offsets)
    tg = oracle_target(b.target)
    s0 = np.stack([oracle_burnin(tg, _as_chain(b, c)) for c in range(b.n_chains)]).astype(np.float32)
    g = pm.Target(ctx, b.target)
    r = pm.solve(ctx, g, b.eps, _t(s0), _t(b.xi), _t(b.u), offsets=list(b.offsets), variant="dense",
                 jac_prec=jac, clip=1.0, clip_inf_norm=True, max_iter=int(lens.max()) + 1)
    _say(f"  lens={lens.tolist()} sweeps/chain={r.sweeps_per_chain} status={r.status}")
    assert r.status == 0 and r.n_converged == b.n_chains
    st = r.states.cpu().numpy()
    acc = r.accept.cpu().numpy()
    for c in range(b.n_chains):
        o0, o1 = b.offsets[c], b.offsets[c + 1]
        _check_mala(orc, tg, _as_chain(b, c), s0[c], st[o0:o1], acc[o0:o1], label=f"batched dense {jac} chain {c}")


def test_batched_dense_deer_funnel(ctx, pm, orc):
    """Full DEER on three funnel chains of one target (D = 32, per-step
    Jacobians of the evaluation kernel), lengths 300, 2000 and 4097, solved
    together and each compared with its FP64 chain."""
    _say("batched dense DEER funnel")
    lens = (300, 2000, 4097)
    chs = [W.funnel_chain(T=n, seed=1) for n in lens]
    # one target: the chains differ in their noise streams
    chs = [W.Chain(target=chs[0].target, eps=c.eps, x0=c.x0, xi=W.normals(np.random.default_rng(40 + k), (n, 32),
                                                                           np.float32),
                   u=W.uniforms(np.random.default_rng(50 + k), n, np.float32))
           for k, (c, n) in enumerate(zip(chs, lens))]
    offs = np.concatenate([[0], np.cumsum(lens)]).astype(np.int64)
    tg = oracle_target(chs[0].target)
    g = pm.Target(ctx, chs[0].target)
    x0 = np.stack([c.x0 for c in chs])
    xi = np.concatenate([c.xi for c in chs])
    u = np.concatenate([c.u for c in chs])
    r = pm.solve(ctx, g, chs[0].eps, _t(x0), _t(xi), _t(u), offsets=list(offs), variant="dense", jac_prec="bf16",
                 max_iter=max(lens) + 1)
    _say(f"  sweeps/chain={r.sweeps_per_chain} status={r.status}")
    assert r.status == 0
    st = r.states.cpu().numpy()
    acc = r.accept.cpu().numpy()
    for c, ch in enumerate(chs):
        _check_mala(orc, tg, ch, ch.x0, st[offs[c]:offs[c + 1]], acc[offs[c]:offs[c + 1]],
                    label=f"batched dense funnel chain {c}")


def test_ula_gaussian_one_solve_mfma(ctx, pm, orc):
    """Affine f: the first matrix-core (F32) dense solve already gives the chain."""
    _say("ula gaussian one solve mfma D=16")
    ch = W.gaussian_chain(5000, seed=6, eps=0.2, dim=16, dtype=np.float32, lam_lo=0.3)
    tg = oracle_target(ch.target)
    g = pm.Target(ctx, ch.target)
    r = pm.solve(ctx, g, ch.eps, _t(ch.x0), _t(ch.xi), None, sampler="ula", variant="dense",
                 jac_prec="f32", max_iter=5, want_trace=True)
    ref, _, _ = orc.mala_chain(tg, ch.eps, ch.x0, ch.xi, None, ula=True)
    assert state_error(r.trace[0].cpu().numpy(), ref) <= 1e-5
    assert r.sweeps <= 3


def test_autotune_and_cache(ctx, pm, orc, tmp_path):
    """The tuner picks a tile configuration, caches it by architecture and
    shape, and the solve with the tuned tiles still matches the oracle."""
    _say("autotune")
    ch, tg, s0 = _logreg_case(orc, 4096, 0.0015, seed=2)
    g = pm.Target(ctx, ch.target)
    cache = tmp_path / "tune.json"
    pm.autotune(ctx, g, ch.eps, _t(s0), _t(ch.xi), _t(ch.u), cache_path=str(cache))
    txt = cache.read_text()
    assert "gfx950" in txt and '"items"' in txt
    pm.autotune(ctx, g, ch.eps, _t(s0), _t(ch.xi), _t(ch.u), cache_path=str(cache))  # cached
    r = pm.solve(ctx, g, ch.eps, _t(s0), _t(ch.xi), _t(ch.u), variant="diag", max_iter=4097)
    assert r.status == 0
    _check_mala(orc, tg, ch, s0, r.states.cpu().numpy(), r.accept.cpu().numpy())


@pytest.mark.parametrize("products", ["auto", "refine"])
def test_batched_full_size_sampled(ctx, pm, orc, products):
    """512 burned-in chains, lengths log-uniform in [4096, 131072] (sum ~ 1.9e7
    steps) in one graph-replayed solve.  Compared step by step with the
    oracle: the three shortest chains, the three longest (~131072 steps) and
    every chain that stopped at its rounding floor (reported as not converged,
    so the call's status is PMC_NOT_CONVERGED exactly when such a chain
    exists); with the default (split-FP16) and the refined products.  Every chain starts from its 3 burn-in steps run by the GPU
    sequential sampler; the oracle runs each compared chain from that same
    FP32 start."""
    import concurrent.futures as cf
    _say(f"batched full size (512 chains) products={products}")
    b = W.logreg_batch(seed=0, n_chains=512, lo=4096, hi=131072, eps=0.0015)
    lens = np.diff(b.offsets)
    tg = oracle_target(b.target)
    g = pm.Target(ctx, dict(b.target, products=products))
    D = b.x0.shape[1]
    bx = pm.sample_sequential(ctx, g, b.eps, _t(b.x0), _t(b.burn_xi.reshape(-1, D)),
                              _t(b.burn_u.reshape(-1)), offsets=list(range(0, 3 * b.n_chains + 1, 3)))
    s0 = bx.states.reshape(b.n_chains, 3, D)[:, -1].cpu().numpy().copy()
    r = pm.solve(ctx, g, b.eps, _t(s0), _t(b.xi), _t(b.u), offsets=list(b.offsets), variant="diag",
                 max_iter=400, graph_sweeps=8, skip_converged_prefix=True)
    spc = np.array(r.sweeps_per_chain)
    cst = np.array(r.chain_state)
    floors = np.nonzero(cst == 1)[0]
    _say(f"  n={int(b.offsets[-1])} status={r.status} converged={r.n_converged} floor={r.n_floor} "
         f"sweeps median={np.median(spc)} max={spc.max()} ms={r.elapsed_ms:.1f} floor chains={floors.tolist()}")
    assert not np.any(cst == 2), "a chain reached max_iter"
    assert r.n_converged == int(np.sum(cst == 0)) and r.n_floor == len(floors)
    assert r.status == (pm.B.PMC_NOT_CONVERGED if len(floors) else 0)
    order = np.argsort(lens)
    pick = sorted(set(order[:3].tolist()) | set(order[-3:].tolist()) | set(floors.tolist()))
    st = r.states.cpu().numpy()
    acc = r.accept.cpu().numpy()

    def one(c):
        o0, o1 = int(b.offsets[c]), int(b.offsets[c + 1])
        kind = "floor" if c in floors else "converged"
        return _check_mala(orc, tg, _as_chain(b, c), s0[c], st[o0:o1], acc[o0:o1],
                           label=f"batch chain {c} T={o1 - o0} ({kind}, {spc[c]} sweeps)")

    with cf.ThreadPoolExecutor(max_workers=8) as ex:
        for c, res in zip(pick, ex.map(one, pick)):
            _say(f"  chain {c}: T={lens[c]} state error {res[0]:.3e}")


# (dim, n_data, eps): 11 pair tiles in 4 passes over 32 full data tiles; one
# pair tile and a padded second data tile; 17 pair tiles (the last ragged) in
# 6 passes over 10 data tiles (the last ragged)
DENSE_SHAPES = {"d25n1000": (25, 1000, 0.0015), "d5n50": (5, 50, 0.02), "d32n300": (32, 300, 0.003)}


@pytest.mark.parametrize("shape", list(DENSE_SHAPES))
@pytest.mark.parametrize("clip", [False, True])
@pytest.mark.parametrize("jac", ["bf16", "f32"])
def test_logreg_dense_jacobian_one_sweep(ctx, pm, orc, jac, clip, shape):
    """Full-DEER Jacobians of the logistic posterior (pair-sum kernels): one
    ULA sweep (no accept decisions) from a perturbed guess against the
    oracle's FP64 sweep with the exact, damped and clipped Jacobians.  The
    Jacobian's part of the update, S1 - F, is matched to 2 % (BF16 operands);
    at D = 25 the sweep with the diagonal alone misses it by far more, so the
    off-diagonal entries are checked too."""
    dim, n_data, eps = DENSE_SHAPES[shape]
    _say(f"logreg dense J one sweep jac={jac} clip={clip} D={dim} N={n_data}")
    T = 1024
    ch = W.logreg_chain(T=T, seed=3, eps=eps, n_data=n_data, dim=dim)
    tg = oracle_target(ch.target)
    x0 = ch.x0.astype(np.float64)
    xi = ch.xi.astype(np.float64)
    ref, _, _ = orc.mala_chain(tg, ch.eps, x0, xi, None, ula=True)
    guess = (ref + 0.05 * np.random.default_rng(7).standard_normal(ref.shape)).astype(np.float32)
    g64 = guess.astype(np.float64)
    g = pm.Target(ctx, ch.target)
    kw = dict(clip=1.0, clip_inf_norm=True) if clip else {}
    r = pm.solve(ctx, g, ch.eps, _t(ch.x0), _t(ch.xi), None, sampler="ula", variant="dense", jac_prec=jac,
                 init_guess=_t(guess), max_iter=1, want_trace=True, **kw)
    got = r.trace[0].cpu().numpy().astype(np.float64)

    def sj(t, s):
        F, J, _ = orc.mala_jac(tg, ch.eps, s, xi[t], 0.5, ula=True)
        return F, orc.damp_and_clip(J, 1.0, clip=1.0 if clip else 0.0, inf_norm=clip)
    want, _, _ = orc.newton_reference(sj, x0, T, variant="dense", init=g64, max_iter=1, full_trace=False)
    diag, _, _ = orc.newton_reference(sj, x0, T, variant="diag", init=g64, max_iter=1, full_trace=False)
    F = np.array([sj(t, x0 if t == 0 else g64[t - 1])[0] for t in range(T)])
    jterm = np.max(np.abs(want - F))
    err = np.max(np.abs(got - want))
    miss = np.max(np.abs(diag - want))
    _say(f"  |J part| {jterm:.3e}  gpu error {err:.3e}  diagonal-only miss {miss:.3e}")
    assert jterm > 1e-2
    assert err <= 0.02 * jterm
    if dim == 25:
        assert miss >= 5 * err


@pytest.mark.parametrize("jac", ["bf16", "f32"])
def test_logreg_dense_deer_mala(ctx, pm, orc, jac):
    """Full DEER with the infinity-norm clip on the logistic posterior (MALA,
    frozen gate) converges to the FP64 sequential chain."""
    _say(f"logreg dense DEER mala jac={jac}")
    ch, tg, s0 = _logreg_case(orc, 4096, 0.0015)
    g = pm.Target(ctx, ch.target)
    r = pm.solve(ctx, g, ch.eps, _t(s0), _t(ch.xi), _t(ch.u), variant="dense", jac_prec=jac, clip=1.0,
                 clip_inf_norm=True, max_iter=ch.T + 1)
    rd = pm.solve(ctx, g, ch.eps, _t(s0), _t(ch.xi), _t(ch.u), variant="diag", max_iter=ch.T + 1)
    _say(f"  dense sweeps={r.sweeps} (diag {rd.sweeps}) status={r.status} floor={r.n_floor}")
    assert r.status == 0
    _check_mala(orc, tg, ch, s0, r.states.cpu().numpy(), r.accept.cpu().numpy())


def _residual_ratio(orc, tg, eps, s0, xi, u, states, atol=5e-7, rtol=5e-7):
    """max_t |S_t - f_t(S_{t-1})|_inf / (atol + rtol |S_t|) with f evaluated
    by the oracle in FP64 at the GPU's own states (decision of each step as
    the oracle takes it there; steps whose gate lies within the FP32 tie band
    are skipped, their decision is not fixed by the states)."""
    S = np.asarray(states, dtype=np.float64)
    prev = np.concatenate([np.asarray(s0, dtype=np.float64)[None, :], S[:-1]])
    worst = 0.0
    for t in range(S.shape[0]):
        f, _, gt, _, _ = orc.mala_step(tg, eps, prev[t], xi[t], u[t])
        if abs(gt) < F32_GATE_ERR:
            continue
        worst = max(worst, float(np.max(np.abs(S[t] - f) / (atol + rtol * np.abs(S[t])))))
    return worst


@pytest.mark.parametrize("jac", ["bf16", "f32"])
def test_dense_sliding_window(ctx, pm, orc, jac):
    """The matrix-core dense scan with the sliding window on (the default):
    steps before a chain's window start are frozen (S kept, delta = 0 carried
    into the window), so the converged trajectory satisfies S_t = f_t(S_{t-1})
    over the whole chain to the tolerance, as the solve without the window
    does, and both match the FP64 chain."""
    _say(f"dense sliding window jac={jac}")
    ch, tg, s0 = _logreg_case(orc, 4096, 0.0015, seed=3)
    g = pm.Target(ctx, ch.target)
    out = {}
    for win in (True, False):
        r = pm.solve(ctx, g, ch.eps, _t(s0), _t(ch.xi), _t(ch.u), variant="dense", jac_prec=jac, clip=1.0,
                     clip_inf_norm=True, max_iter=ch.T + 1, skip_converged_prefix=win)
        st = r.states.cpu().numpy()
        rr = _residual_ratio(orc, tg, ch.eps, s0, ch.xi, ch.u, st)
        _say(f"  window={win} sweeps={r.sweeps} status={r.status} max residual / tolerance = {rr:.2f}")
        assert r.status == 0
        assert rr <= 8.0
        _check_mala(orc, tg, ch, s0, st, r.accept.cpu().numpy(), label=f"dense {jac} window={win}")
        out[win] = st
    assert np.max(np.abs(out[True] - out[False])) <= 2e-5


@pytest.mark.parametrize("jac", ["bf16", "f32"])
def test_dense_batched_sweeps_match_single_sweeps(ctx, pm, jac):
    """Sweeps are queued 8 at a time between status reads; once a chain
    stops, the queued sweeps must leave its states alone.  A dense solve with
    a trace (one sweep per status read) and one without give the same states
    bit for bit (a 32-dimensional funnel chain and a 25-dimensional logistic
    chain, matrix-core dense scan)."""
    _say(f"dense batched vs single sweeps {jac}")
    # both solves run to convergence (unconverged funnel iterates can be
    # non-finite, which no comparison can call equal)
    for ch, kw in ((W.funnel_chain(T=512, seed=2), {}),
                   (W.logreg_chain(T=2048, seed=5, eps=0.0015), dict(clip=1.0, clip_inf_norm=True))):
        g = pm.Target(ctx, ch.target)
        args = (ctx, g, ch.eps, _t(ch.x0), _t(ch.xi), _t(ch.u))
        a = pm.solve(*args, variant="dense", jac_prec=jac, max_iter=ch.T + 1, **kw)
        b = pm.solve(*args, variant="dense", jac_prec=jac, max_iter=ch.T + 1, want_trace=True, **kw)
        _say(f"  {ch.meta['workload']}: sweeps {a.sweeps} / {b.sweeps} status {a.status} / {b.status}")
        assert a.status == 0 and b.status == 0
        assert a.sweeps == b.sweeps
        assert bool(torch.isfinite(a.states).all())
        assert torch.equal(a.states, b.states)


@pytest.mark.parametrize("jac", ["bf16", "f32"])
def test_logreg_dense_jacobian_ragged_entry_clip(ctx, pm, orc, jac):
    """Full-DEER Jacobians with the entrywise clip (every entry clamped to
    [-0.5, 0.5], the diagonal included) on a chain whose length is not a
    multiple of the 32-step groups: one ULA sweep against the oracle's FP64
    sweep with the same clip."""
    _say(f"logreg dense J ragged entry clip jac={jac}")
    T = 1000
    ch = W.logreg_chain(T=T, seed=7, eps=0.0015)
    tg = oracle_target(ch.target)
    x0 = ch.x0.astype(np.float64)
    xi = ch.xi.astype(np.float64)
    ref, _, _ = orc.mala_chain(tg, ch.eps, x0, xi, None, ula=True)
    guess = (ref + 0.05 * np.random.default_rng(10).standard_normal(ref.shape)).astype(np.float32)
    g64 = guess.astype(np.float64)
    g = pm.Target(ctx, ch.target)
    r = pm.solve(ctx, g, ch.eps, _t(ch.x0), _t(ch.xi), None, sampler="ula", variant="dense", jac_prec=jac,
                 clip=0.5, init_guess=_t(guess), max_iter=1, want_trace=True)
    got = r.trace[0].cpu().numpy().astype(np.float64)

    def sj(t, s):
        F, J, _ = orc.mala_jac(tg, ch.eps, s, xi[t], 0.5, ula=True)
        return F, orc.damp_and_clip(J, 1.0, clip=0.5)
    want, _, _ = orc.newton_reference(sj, x0, T, variant="dense", init=g64, max_iter=1, full_trace=False)
    F = np.array([sj(t, x0 if t == 0 else g64[t - 1])[0] for t in range(T)])
    jterm = np.max(np.abs(want - F))
    err = np.max(np.abs(got - want))
    _say(f"  |J part| {jterm:.3e}  gpu error {err:.3e}")
    assert jterm > 1e-2
    assert err <= 0.02 * jterm


def _orthogonal(D, seed):
    q, r = np.linalg.qr(np.random.default_rng(seed).standard_normal((D, D)))
    return q * np.sign(np.diag(r))


def test_basis_eigenbasis_ula_gaussian(ctx, pm, orc):
    """Orthogonal reparameterisation (Sec. 3.4 eq. 11): ULA on a Gaussian in
    the eigenbasis of its precision has a diagonal Jacobian, so the first
    quasi-DEER sweep there is exact Newton and already gives the chain (to
    FP32 rounding), while the first sweep in the original coordinates is far
    off.  The tolerance-based stop then takes a few more sweeps in FP32:
    rounding moves the iterate by about the tolerance, amplified by the
    recursion's coefficients near 1; it still stops sooner than the plain
    iteration."""
    _say("basis: eigenbasis ULA gaussian D=16")
    ch = W.gaussian_chain(5000, seed=6, eps=0.2, dim=16, dtype=np.float32, lam_lo=0.3)
    tg = oracle_target(ch.target)
    _, Q = np.linalg.eigh(np.asarray(ch.target["prec"], dtype=np.float64))
    g = pm.Target(ctx, ch.target)
    q = _t(Q.astype(np.float32))
    args = (ctx, g, ch.eps, _t(ch.x0), _t(ch.xi), None)
    r = pm.solve(*args, sampler="ula", variant="diag", basis=q, max_iter=200, want_trace=True)
    r0 = pm.solve(*args, sampler="ula", variant="diag", max_iter=200, want_trace=True)
    ref, _, _ = orc.mala_chain(tg, ch.eps, ch.x0, ch.xi, None, ula=True)
    e1 = state_error(r.trace[0].cpu().numpy(), ref)
    e1_plain = state_error(r0.trace[0].cpu().numpy(), ref)
    _say(f"  first sweep error {e1:.2e} (plain {e1_plain:.2e}); sweeps {r.sweeps} (plain {r0.sweeps})")
    assert e1 <= 1e-5 and e1_plain > 1e-3
    assert r.status == 0 and r.sweeps < r0.sweeps
    assert state_error(r.states.cpu().numpy(), ref) <= 1e-5


@pytest.mark.parametrize("kind", ["banana_f64", "funnel_f32"])
def test_basis_random_rotation_mala(ctx, pm, orc, kind):
    """Quasi-DEER in randomly rotated coordinates (diag of Q^T J Q, states
    rotated in and out) converges to the FP64 sequential chain."""
    _say(f"basis: random rotation {kind}")
    if kind == "banana_f64":
        ch, td, tol = W.banana_chain(1024, seed=2), torch.float64, 1e-10
    else:
        ch, td, tol = W.funnel_chain(T=1024, seed=3), torch.float32, 1e-5
    tg = oracle_target(ch.target)
    D = ch.x0.shape[0]
    q = _t(_orthogonal(D, 11), td)
    g = pm.Target(ctx, ch.target, dtype=td)
    r = pm.solve(ctx, g, ch.eps, _t(ch.x0, td), _t(ch.xi, td), _t(ch.u, td), variant="diag", basis=q,
                 max_iter=ch.T + 1)
    r0 = pm.solve(ctx, g, ch.eps, _t(ch.x0, td), _t(ch.xi, td), _t(ch.u, td), variant="diag", max_iter=ch.T + 1)
    _say(f"  rotated sweeps={r.sweeps} plain sweeps={r0.sweeps} status={r.status}")
    assert r.status == 0
    _check_mala(orc, tg, ch, np.asarray(ch.x0), r.states.cpu().numpy(), r.accept.cpu().numpy(), tol)


def test_basis_is_refused_where_it_does_not_apply(ctx, pm):
    from paper_2508_18413_amd._binding import PMCError
    fch = W.funnel_chain(T=256, seed=1)
    fg = pm.Target(ctx, fch.target)
    with pytest.raises(PMCError, match="basis"):
        pm.solve(ctx, fg, fch.eps, _t(fch.x0), _t(fch.xi), _t(fch.u), variant="dense",
                 basis=_t(np.eye(32, dtype=np.float32)))


@pytest.mark.parametrize("probes", [0, 1])
def test_basis_logreg_rotated_model(ctx, pm, orc, probes):
    """The logistic posterior with an orthogonal basis is solved as the
    rotated model (design X Q, noise Q^T xi) and rotated back: it converges
    to the FP64 chain in the original coordinates, with the exact or the
    probed diagonal, and its trace comes back in s."""
    _say(f"basis: logistic posterior, random rotation, probes={probes}")
    ch, tg, s0 = _logreg_case(orc, 4096, 0.0015)
    g = pm.Target(ctx, ch.target)
    q = _t(_orthogonal(25, 12).astype(np.float32))
    r = pm.solve(ctx, g, ch.eps, _t(s0), _t(ch.xi), _t(ch.u), variant="diag", basis=q, jac_probes=probes,
                 max_iter=ch.T + 1)
    r0 = pm.solve(ctx, g, ch.eps, _t(s0), _t(ch.xi), _t(ch.u), variant="diag", max_iter=ch.T + 1)
    _say(f"  rotated sweeps={r.sweeps} plain sweeps={r0.sweeps} status={r.status}")
    assert r.status == 0
    _check_mala(orc, tg, ch, s0, r.states.cpu().numpy(), r.accept.cpu().numpy())
    rt = pm.solve(ctx, g, ch.eps, _t(s0), _t(ch.xi), _t(ch.u), variant="diag", basis=q, jac_probes=probes,
                  max_iter=r.sweeps + 3, want_trace=True)
    last = rt.trace[rt.sweeps - 1]
    assert (last - rt.states).abs().max().item() <= 1e-5
    assert bool(torch.isnan(rt.trace[rt.sweeps:]).all())


@pytest.mark.parametrize("width", [128, 512, 1024])
def test_fixed_width_window(ctx, pm, orc, width):
    """Sec. 3.4 sliding window of a fixed width (the widths of Sec. 5.5): each
    sweep updates at most `width` steps from the chain's first unconverged
    one, and the solve still reaches the FP64 chain; a batch of uneven chains
    too.  The sweep counts are reported beside the unlimited window's."""
    _say(f"fixed-width window {width}")
    ch, tg, s0 = _logreg_case(orc, 4096, 0.0015, seed=4)
    g = pm.Target(ctx, ch.target)
    r = pm.solve(ctx, g, ch.eps, _t(s0), _t(ch.xi), _t(ch.u), variant="diag", max_iter=20000,
                 window_width=width)
    r0 = pm.solve(ctx, g, ch.eps, _t(s0), _t(ch.xi), _t(ch.u), variant="diag", max_iter=4097)
    _say(f"  width {width}: sweeps={r.sweeps} (unlimited window {r0.sweeps}) status={r.status}")
    assert r.status == 0
    _check_mala(orc, tg, ch, s0, r.states.cpu().numpy(), r.accept.cpu().numpy(), label=f"window {width}")
    if width == 512:
        b = W.logreg_batch(seed=6, n_chains=3, lo=300, hi=3000, eps=0.0015)
        bt = oracle_target(b.target)
        s0b = np.stack([oracle_burnin(bt, _as_chain(b, c)) for c in range(b.n_chains)]).astype(np.float32)
        gb = pm.Target(ctx, b.target)
        rb = pm.solve(ctx, gb, b.eps, _t(s0b), _t(b.xi), _t(b.u), offsets=list(b.offsets), variant="diag",
                      max_iter=20000, window_width=width)
        assert rb.status == 0
        st, acc = rb.states.cpu().numpy(), rb.accept.cpu().numpy()
        for c in range(b.n_chains):
            o0, o1 = b.offsets[c], b.offsets[c + 1]
            _check_mala(orc, bt, _as_chain(b, c), s0b[c], st[o0:o1], acc[o0:o1], label=f"window {width} chain {c}")


def test_fixed_width_window_dense(ctx, pm, orc):
    """The fixed-width window with the matrix-core dense scan (full DEER on the
    logistic posterior, BF16 Jacobians, infinity-norm clip)."""
    _say("fixed-width window, dense")
    ch, tg, s0 = _logreg_case(orc, 2048, 0.0015, seed=5)
    g = pm.Target(ctx, ch.target)
    r = pm.solve(ctx, g, ch.eps, _t(s0), _t(ch.xi), _t(ch.u), variant="dense", jac_prec="bf16", clip=1.0,
                 clip_inf_norm=True, max_iter=20000, window_width=256)
    _say(f"  sweeps={r.sweeps} status={r.status}")
    assert r.status == 0
    _check_mala(orc, tg, ch, s0, r.states.cpu().numpy(), r.accept.cpu().numpy(), label="dense window 256")


@pytest.mark.parametrize("probes", [0, 1])
@pytest.mark.parametrize("kw", [{}, dict(damping=0.4, clip=1.0)])
def test_logreg_surrogate_gate_one_sweep(ctx, pm, orc, probes, kw):
    """The relaxed (stop-gradient) gate of Sec. 3.2 on the logistic
    posterior: one quasi-DEER sweep from a perturbed guess against the
    oracle's FP64 sweep with the diagonal of the relaxed-gate Jacobian (or its
    one-probe estimate with the same signs), damped and clipped.  The part of
    the update the relaxed term changes is matched to 2 %."""
    _say(f"logreg relaxed gate one sweep probes={probes} {kw}")
    T = 1024
    ch, tg, s0 = _logreg_case(orc, T, 0.0015, seed=8)
    x0 = s0.astype(np.float64)
    ref, _, _ = orc.mala_chain(tg, ch.eps, x0, ch.xi, ch.u)
    guess = (ref + 2e-3 * np.random.default_rng(9).standard_normal(ref.shape)).astype(np.float32)
    g64 = guess.astype(np.float64)
    g = pm.Target(ctx, ch.target)
    r = pm.solve(ctx, g, ch.eps, _t(s0), _t(ch.xi), _t(ch.u), variant="diag", gate="surrogate", jac_probes=probes,
                 probe_seed=21, init_guess=_t(guess), max_iter=1, want_trace=True, **kw)
    got = r.trace[0].cpu().numpy().astype(np.float64)

    def sj(gate):
        def f(t, s):
            F, J, _ = orc.mala_jac(tg, ch.eps, s, ch.xi[t], ch.u[t], gate=gate)
            return F, J
        return f

    def sweep(gate):
        variant = "hutchinson" if probes else "diag"
        want, _, _ = orc.newton_reference(sj(gate), x0, T, variant=variant, init=g64, max_iter=1,
                                          full_trace=False, probe_seed=21)
        if kw:  # damping and clip act on the (structured) diagonal: redo the sweep with them
            F = np.array([sj(gate)(t, x0 if t == 0 else g64[t - 1])[0] for t in range(T)])
            jd = np.empty((T, ch.D))
            for t in range(T):
                _, J = sj(gate)(t, x0 if t == 0 else g64[t - 1])
                if probes:
                    z = np.array([orc.probe_sign(21, 0, t, d) for d in range(ch.D)])
                    d = orc.hutchinson_diag(J, z)
                else:
                    d = np.diag(J)
                jd[t] = np.clip(kw["damping"] * d, -kw["clip"], kw["clip"])
            want = np.empty((T, ch.D))
            for t in range(T):
                want[t] = F[t] if t == 0 else F[t] + jd[t] * (want[t - 1] - g64[t - 1])
        return want
    want = sweep(1)
    frozen = sweep(0)
    effect = np.max(np.abs(want - frozen))
    err = np.max(np.abs(got - want))
    _say(f"  relaxed-gate effect {effect:.3e}  gpu error {err:.3e}")
    assert effect > 1e-5
    assert err <= 0.02 * effect + 2e-6


@pytest.mark.parametrize("probes", [0, 1])
def test_logreg_surrogate_gate_mala(ctx, pm, orc, probes):
    """The relaxed gate changes sweep counts, never the fixed point: the
    logistic chain still reaches the FP64 sequential chain."""
    _say(f"logreg relaxed gate mala probes={probes}")
    ch, tg, s0 = _logreg_case(orc, 4096, 0.0015, seed=2)
    g = pm.Target(ctx, ch.target)
    r = pm.solve(ctx, g, ch.eps, _t(s0), _t(ch.xi), _t(ch.u), variant="diag", gate="surrogate", jac_probes=probes,
                 probe_seed=5, max_iter=4097)
    rf = pm.solve(ctx, g, ch.eps, _t(s0), _t(ch.xi), _t(ch.u), variant="diag", jac_probes=probes, probe_seed=5,
                  max_iter=4097)
    _say(f"  sweeps relaxed {r.sweeps} frozen {rf.sweeps} status {r.status}")
    assert r.status == 0
    _check_mala(orc, tg, ch, s0, r.states.cpu().numpy(), r.accept.cpu().numpy(), label=f"relaxed gate probes={probes}")
