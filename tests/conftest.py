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
