"""Parity helpers shared by the GPU tests: the state-error metric and the
accept-pattern comparison with near-tie resynchronisation.

State error (mixed absolute/relative, per step):
    e = max_t |s_t - s*_t|_inf / max(1, |s*_t|_inf).
Accept patterns: at the first step where the GPU's decision differs from the
oracle's, the oracle's gate g~* = log alpha - log u is inspected.  If
|g~*| < tie_band the mismatch is a near-tie: it is recorded, the oracle is
re-run with the GPU's decision imposed at that step, and the comparison
continues.  A mismatch outside the band is a failure.
"""
import numpy as np


def state_error(got, ref):
    got = np.asarray(got, dtype=np.float64)
    ref = np.asarray(ref, dtype=np.float64)
    if got.size == 0:
        return 0.0
    den = np.maximum(1.0, np.abs(ref).max(axis=1))
    return float(np.max(np.abs(got - ref).max(axis=1) / den))


def compare_with_resync(run_oracle, gpu_accept, tie_band=1e-6, max_resync=64):
    """run_oracle(force) -> (states, accept, gtilde) in FP64, force an int8 array
    of -1/0/1.  Returns (states, accept, report) where report lists
    (t, gtilde*, kind) for every mismatch, kind in {"near-tie", "failure"}."""
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
        kind = "near-tie" if abs(gt[t]) < tie_band else "failure"
        report.append((t, float(gt[t]), kind))
        if kind == "failure":
            return st, acc, report
        force[t] = gpu_accept[t]
    report.append((-1, float("nan"), "failure"))
    return st, acc, report
