"""GPU parity of MALA on the 768-dimensional logistic-regression stand-in of
Sec. 5.5 (1024 unit-norm rows, step size 0.015), evaluated by the
matrix-core GEMM path, against the FP64 oracle.

* Gate precision: one parallel evaluation at the oracle's own trajectory
  (rounded to FP32): every step's g~ against the oracle's g~* from the same
  states.  Its maximum pins WIDE_GATE_ERR, the FP32-floor tie band of the
  chain comparisons below.
* Chains: two chains of uneven length (ragged against the 128-step tile),
  quasi-DEER with and without the orthogonal basis of Sec. 5.5 (left
  singular vectors of the feature covariance) and with fixed-width windows
  (Sec. 3.4), Picard, ULA, and the same-GPU sequential sampler, each
  compared chain by chain with the oracle (both tie classes recorded, the
  FP32-floor class capped).
* What the path does not take is refused before launch.
"""
import numpy as np
import pytest

from conftest import oracle_target
from parity import compare_with_resync, floor_cap, record, state_error
from paper_2508_18413_amd import workloads as W

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")
DEV = "cuda:0"

# Pinned bound on |g~ - g~*| of one step computed in FP32 from the oracle's
# states (test_wide_gate_precision): the log ratio sums 1024 softplus
# increments and 768-term products, each with FP32 rounding.
WIDE_GATE_ERR = 2e-5
LENS = (256, 200)


def _t(x, dtype=None):
    return torch.tensor(np.ascontiguousarray(x), dtype=dtype, device=DEV)


def _say(*a):
    print(*a, flush=True)


@pytest.fixture(scope="module")
def pm():
    import paper_2508_18413_amd as pm
    return pm


@pytest.fixture(scope="module")
def ctx(pm):
    c = pm.Context(0)
    yield c
    c.close()


@pytest.fixture(scope="module")
def case(orc):
    """Two chains (lengths 256 and 200) laid end to end, and their FP64 oracle
    chains."""
    b = W.embedding_logreg_batch(seed=0, n_chains=2, T=max(LENS))
    offs = np.concatenate([[0], np.cumsum(LENS)]).astype(np.int64)
    xi = np.concatenate([b.xi[c * max(LENS):c * max(LENS) + n] for c, n in enumerate(LENS)])
    u = np.concatenate([b.u[c * max(LENS):c * max(LENS) + n] for c, n in enumerate(LENS)])
    tg = oracle_target(b.target)
    chains = []
    for c in range(2):
        o0, o1 = offs[c], offs[c + 1]
        chains.append(W.Chain(target=b.target, eps=b.eps, x0=b.x0[c], xi=xi[o0:o1], u=u[o0:o1]))
    return dict(b=b, offs=offs, xi=xi, u=u, tg=tg, chains=chains)


def _check(orc, case, states, acc, label, ula=False):
    errs = []
    for c, ch in enumerate(case["chains"]):
        o0, o1 = case["offs"][c], case["offs"][c + 1]
        x0 = ch.x0.astype(np.float64)
        st, oacc, rep = compare_with_resync(
            lambda f: orc.mala_chain(case["tg"], ch.eps, x0, ch.xi, ch.u, ula=ula, force=f), acc[o0:o1],
            floor_band=WIDE_GATE_ERR)
        err = state_error(states[o0:o1], st)
        n_tie, n_floor = record(f"{label} chain {c}", o1 - o0, err, rep)
        _say(f"  {label} chain {c}: state_error={err:.3e} near-ties={n_tie} fp32-floor={n_floor} {rep}")
        assert not [x for x in rep if x[2] == "failure"], rep
        assert n_floor <= floor_cap(o1 - o0), rep
        assert err <= 1e-5
        errs.append(err)
    return errs


def _solve(pm, ctx, case, **kw):
    b = case["b"]
    g = pm.Target(ctx, b.target)
    kw.setdefault("max_iter", max(LENS) + 1)
    return pm.solve(ctx, g, b.eps, _t(b.x0), _t(case["xi"]), _t(case["u"]), offsets=list(case["offs"]), **kw)


def test_wide_gate_precision(pm, ctx, orc, case):
    _say("wide gate precision")
    b, offs = case["b"], case["offs"]
    init, ref = [], []
    for c, ch in enumerate(case["chains"]):
        st, _, _ = orc.mala_chain(case["tg"], ch.eps, ch.x0.astype(np.float64), ch.xi, ch.u)
        s32 = st.astype(np.float32)
        init.append(s32)
        prev = np.concatenate([ch.x0[None, :].astype(np.float64), s32[:-1].astype(np.float64)])
        ref.append(np.array([orc.mala_step(case["tg"], ch.eps, prev[t], ch.xi[t], ch.u[t])[2]
                             for t in range(prev.shape[0])]))
    init, ref = np.concatenate(init), np.concatenate(ref)
    r = _solve(pm, ctx, case, variant="diag", max_iter=1, init_guess=_t(init))
    got = r.gtilde.cpu().numpy().astype(np.float64)
    err = np.abs(got - ref)
    _say(f"  max |g~ - g~*| = {err.max():.3e}, p99 {np.quantile(err, 0.99):.3e}, "
         f"median |g~*| {np.median(np.abs(ref)):.3g}, acceptance {np.mean(ref > 0):.3f}")
    assert err.max() <= WIDE_GATE_ERR
    clear = np.abs(ref) > WIDE_GATE_ERR
    assert np.array_equal(r.accept.cpu().numpy()[clear].astype(bool), ref[clear] > 0)
    # from exact states one sweep returns f(s_{t-1}): the oracle's step, to FP32
    for c, ch in enumerate(case["chains"]):
        o0, o1 = offs[c], offs[c + 1]
        prev = np.concatenate([ch.x0[None, :], init[o0:o1 - 1]]).astype(np.float64)
        acc = r.accept.cpu().numpy()[o0:o1]
        want = np.array([orc.mala_step(case["tg"], ch.eps, prev[t], ch.xi[t], ch.u[t], force=int(acc[t]))[0]
                         for t in range(o1 - o0)])
        assert state_error(r.states.cpu().numpy()[o0:o1], want) <= 1e-5


@pytest.mark.parametrize("basis", [False, True])
@pytest.mark.parametrize("window", [0, 128])
def test_wide_mala_diag(pm, ctx, orc, case, basis, window):
    _say(f"wide MALA quasi-DEER basis={basis} window={window}")
    kw = {}
    if basis:
        kw["basis"] = _t(case["b"].target["basis"])
    r = _solve(pm, ctx, case, variant="diag", window_width=window, **kw)
    _say(f"  sweeps per chain {r.sweeps_per_chain} status {r.status}")
    assert r.status == 0
    _check(orc, case, r.states.cpu().numpy(), r.accept.cpu().numpy(),
           f"wide D=768 diag basis={basis} window={window}")


def test_wide_picard(pm, ctx, orc, case):
    _say("wide MALA Picard")
    r = _solve(pm, ctx, case, variant="picard")
    _say(f"  sweeps per chain {r.sweeps_per_chain} status {r.status}")
    assert r.status == 0
    _check(orc, case, r.states.cpu().numpy(), r.accept.cpu().numpy(), "wide D=768 picard")


def test_wide_ula(pm, ctx, orc, case):
    _say("wide ULA quasi-DEER")
    b = case["b"]
    g = pm.Target(ctx, b.target)
    r = pm.solve(ctx, g, b.eps, _t(b.x0), _t(case["xi"]), None, sampler="ula", offsets=list(case["offs"]),
                 variant="diag", max_iter=max(LENS) + 1)
    assert r.status == 0
    for c, ch in enumerate(case["chains"]):
        o0, o1 = case["offs"][c], case["offs"][c + 1]
        st, _, _ = orc.mala_chain(case["tg"], ch.eps, ch.x0.astype(np.float64), ch.xi, None, ula=True)
        err = state_error(r.states.cpu().numpy()[o0:o1], st)
        _say(f"  chain {c}: state_error={err:.3e}")
        assert err <= 1e-5


def test_wide_sequential(pm, ctx, orc, case):
    _say("wide sequential sampler")
    b = case["b"]
    g = pm.Target(ctx, b.target)
    r = pm.sample_sequential(ctx, g, b.eps, _t(b.x0), _t(case["xi"]), _t(case["u"]), offsets=list(case["offs"]))
    _check(orc, case, r.states.cpu().numpy(), r.accept.cpu().numpy(), "wide D=768 sequential")


def test_wide_jacobian_one_sweep(pm, ctx, orc, case):
    """One ULA quasi-DEER sweep from a perturbed guess (first 16 steps of the
    first chain): S1 = F + J d with the Jacobian diagonal that the path forms
    from (X o X)^T W on BF16 matrix instructions, against the oracle's FP64
    sweep with the exact diagonal.  The Jacobian's part of the update,
    S1 - F, is matched to 1 %."""
    _say("wide Jacobian diagonal, one sweep")
    T = 16
    ch = case["chains"][0]
    tg = case["tg"]
    x0 = ch.x0.astype(np.float64)
    xi = ch.xi[:T].astype(np.float64)
    ref, _, _ = orc.mala_chain(tg, ch.eps, x0, xi, None, ula=True)
    guess = (ref + 0.02 * np.random.default_rng(3).standard_normal(ref.shape)).astype(np.float32)
    g64 = guess.astype(np.float64)
    g = pm.Target(ctx, case["b"].target)
    r = pm.solve(ctx, g, ch.eps, _t(ch.x0[None, :]), _t(ch.xi[:T]), None, sampler="ula", variant="diag",
                 init_guess=_t(guess), max_iter=1)
    got = r.states.cpu().numpy().astype(np.float64)

    def sj(t, s):
        F, J, _ = orc.mala_jac(tg, ch.eps, s, xi[t], 0.5, ula=True)
        return F, J
    want, _, _ = orc.newton_reference(sj, x0, T, variant="diag", init=g64, max_iter=1, full_trace=False)
    F = np.array([orc.mala_step(tg, ch.eps, x0 if t == 0 else g64[t - 1], xi[t], 0.5, ula=True)[0]
                  for t in range(T)])
    jterm = np.max(np.abs(want - F))
    err = np.max(np.abs(got - want))
    _say(f"  |J part| {jterm:.3e}  gpu error {err:.3e}")
    assert jterm > 1e-3
    assert err <= 0.01 * jterm


def test_wide_refusals(pm, ctx, case):
    from paper_2508_18413_amd import _binding as B
    b = case["b"]
    g = pm.Target(ctx, b.target)
    args = (ctx, g, b.eps, _t(b.x0), _t(case["xi"]), _t(case["u"]))
    for kw in (dict(variant="dense"), dict(variant="diag", jac_probes=1), dict(variant="diag", gate="surrogate"),
               dict(variant="diag", sampler="hmc", n_leapfrog=4)):
        with pytest.raises(B.PMCError) as e:
            pm.solve(*args, offsets=list(case["offs"]), **kw)
        assert e.value.status == B.PMC_ERR_UNSUPPORTED, kw
    rng = np.random.default_rng(0)
    big = dict(kind="logreg", dim=1025, X=rng.normal(size=(64, 1025)).astype(np.float32),
               y=np.zeros(64, dtype=np.float32), prior_var=1.0)
    with pytest.raises(B.PMCError) as e:
        pm.Target(ctx, big)
    assert e.value.status == B.PMC_ERR_UNSUPPORTED
