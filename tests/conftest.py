import os
import sys

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (runs through the C-ABI library)")
    config.addinivalue_line("markers", "slow: long-running CPU statistics test")


def pytest_runtest_setup(item):
    import parity
    parity.set_current_test(item.nodeid)


def pytest_sessionfinish(session, exitstatus):
    """With PMC_PARITY_RECORD=<path>, writes every accept-pattern comparison of
    the session (steps compared, state error, near-tie and fp32-floor counts,
    and each resynchronised step) as JSON to <path> and a table to <path>.md."""
    import json

    import parity
    path = os.environ.get("PMC_PARITY_RECORD")
    if not path or not parity.RECORD:
        return
    rows = [dict(test=r[0], chain=r[1], steps=r[2], state_error=r[3], near_ties=r[4], fp32_floor_ties=r[5],
                 resync=r[6]) for r in parity.RECORD]
    with open(path, "w") as f:
        json.dump(rows, f, indent=1)
    tot = sum(r["steps"] for r in rows)
    lines = ["| test | chain | steps | state error | near-ties (<1e-6) | fp32-floor ties | resynchronised (t, g~*) |",
             "|---|---|---|---|---|---|---|"]
    for r in rows:
        rs = "; ".join(f"{t}: {g:.2e}" for t, g, _ in r["resync"]) or "-"
        lines.append(f"| {r['test'].split('::')[-1]} | {r['chain']} | {r['steps']} | {r['state_error']:.2e} | "
                     f"{r['near_ties']} | {r['fp32_floor_ties']} | {rs} |")
    lines.append(f"| total | {len(rows)} comparisons | {tot} | | {sum(r['near_ties'] for r in rows)} | "
                 f"{sum(r['fp32_floor_ties'] for r in rows)} | |")
    with open(path + ".md", "w") as f:
        f.write("\n".join(lines) + "\n")


def oracle_target(tg: dict):
    """Build an oracle Target from a workload's target dictionary."""
    import oracle
    kind = tg["kind"]
    if kind == "banana":
        return oracle.Target(oracle.BANANA, 2)
    if kind == "gaussian":
        return oracle.Target(oracle.GAUSSIAN, tg["dim"], mean=tg["mean"], prec=tg["prec"])
    if kind == "logreg":
        return oracle.Target(oracle.LOGREG, tg["dim"], X=tg["X"], y=tg["y"],
                             prior_var=tg.get("prior_var", 1.0))
    if kind == "funnel":
        return oracle.Target(oracle.FUNNEL, tg["dim"], theta=tg["theta"])
    raise ValueError(kind)


def oracle_burnin(tg, chain):
    """s0 = x0 advanced by the chain's 3 burn-in MALA steps, in FP64 (Appendix B.1)."""
    import oracle
    x0 = np.asarray(chain.x0, dtype=np.float64)
    if chain.burn_xi is None:
        return x0
    st, _, _ = oracle.mala_chain(tg, chain.eps, x0, chain.burn_xi, chain.burn_u)
    return st[-1]


@pytest.fixture(scope="session")
def orc():
    import oracle
    oracle.lib()
    return oracle
