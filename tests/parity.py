"""Parity helpers shared by the GPU tests: the state-error metric, the
accept-pattern comparison with near-tie resynchronisation, and the record of
every resynchronised decision.

State error (mixed absolute/relative, per step):
    e = max_t |s_t - s*_t|_inf / max(1, |s*_t|_inf).
Accept patterns: at the first step where the GPU's decision differs from the
oracle's, the oracle's gate g~* = log alpha - log u is inspected and the
mismatch falls in one of three classes:
  * "near-tie"   |g~*| < 1e-6 (the bound the parity contract names): a tie;
  * "fp32-floor" 1e-6 <= |g~*| < floor_band, for chains computed in FP32,
                 where floor_band is the pinned bound on the FP32 error of g~
                 (test_logreg_gate_precision for MALA, test_hmc_energy_precision
                 for HMC): a decision inside the arithmetic's own error;
  * "failure"    anything else.
Ties of both kinds are resynchronised (the oracle is re-run with the GPU's
decision imposed at that step) and the comparison continues; each test then
asserts a cap on the fp32-floor class.  Every comparison is appended to
RECORD, which conftest writes out at the end of the session, so that the
counts of both classes are visible per test rather than absorbed.
"""
import math

import numpy as np

CONTRACT_TIE = 1e-6

# (test id, chain label, steps compared, state error, near-tie count,
#  fp32-floor count, [(t, g~*, kind), ...])
RECORD = []
_current_test = ["?"]


def set_current_test(nodeid):
    _current_test[0] = nodeid


def state_error(got, ref):
    got = np.asarray(got, dtype=np.float64)
    ref = np.asarray(ref, dtype=np.float64)
    if got.size == 0:
        return 0.0
    den = np.maximum(1.0, np.abs(ref).max(axis=1))
    return float(np.max(np.abs(got - ref).max(axis=1) / den))


def classify(gt_star, floor_band):
    a = abs(gt_star)
    if a < CONTRACT_TIE:
        return "near-tie"
    if floor_band is not None and a < floor_band:
        return "fp32-floor"
    return "failure"


def compare_with_resync(run_oracle, gpu_accept, floor_band=None, max_resync=64):
    """run_oracle(force) -> (states, accept, gtilde) in FP64, force an int8 array
    of -1/0/1.  Returns (states, accept, report) where report lists
    (t, gtilde*, kind) for every mismatch, kind in {"near-tie", "fp32-floor",
    "failure"}.  floor_band=None (FP64 chains) admits contract ties only."""
    gpu_accept = np.asarray(gpu_accept).astype(np.int8)
    T = gpu_accept.shape[0]
    force = np.full(T, -1, dtype=np.int8)
    report = []
    for _ in range(max_resync + 1):
        st, acc, gt = run_oracle(force)
        mism = np.nonzero((acc != gpu_accept) & (force < 0))[0]
        if mism.size == 0:
            return st, acc, report
        t = int(mism[0])
        kind = classify(gt[t], floor_band)
        report.append((t, float(gt[t]), kind))
        if kind == "failure":
            return st, acc, report
        force[t] = gpu_accept[t]
    report.append((-1, float("nan"), "failure"))
    return st, acc, report


def floor_cap(n_steps):
    """Largest number of fp32-floor ties a comparison of n_steps decisions may
    show: one per 16384 steps, rounded up.  A decision lands in the band with
    probability about 2 * floor_band * (density of g~ at 0) <= 2 * 2e-5 per
    step, and flips only if the FP32 error (a few 1e-6) crosses it, so the
    expected count is well below one per 16384 steps."""
    return max(1, math.ceil(n_steps / 16384))


def record(label, n_steps, err, report):
    n_tie = sum(1 for r in report if r[2] == "near-tie")
    n_floor = sum(1 for r in report if r[2] == "fp32-floor")
    RECORD.append((_current_test[0], label, int(n_steps), float(err), n_tie, n_floor,
                   [(int(t), float(g), k) for t, g, k in report]))
    return n_tie, n_floor
