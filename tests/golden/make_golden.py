"""Writes tests/golden/*.json from the FP64 oracle only (no GPU code involved).

banana_mala_t32.json: MALA on log p(x) = -x1^2/2 - (x2 - x1^2)^2/2 with step
size 0.1, x0 = 0, the first 32 steps of workloads.banana_chain(seed=0): the
trajectory, accept pattern and gates g~.  Used as a regression fixture for
the oracle and as a small exact parity case for the FP64 GPU path.
"""
import json
import os
import sys

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import oracle  # noqa: E402
from paper_2508_18413_amd import workloads as W  # noqa: E402


def main():
    ch = W.banana_chain(32, seed=0)
    tg = oracle.Target(oracle.BANANA, 2)
    st, acc, gt = oracle.mala_chain(tg, ch.eps, ch.x0, ch.xi, ch.u)
    out = dict(source="oracle.mala_chain, FP64", eps=ch.eps, x0=ch.x0.tolist(), xi=ch.xi.tolist(),
               u=ch.u.tolist(), states=st.tolist(), accept=acc.tolist(), gtilde=gt.tolist())
    with open(os.path.join(HERE, "banana_mala_t32.json"), "w") as f:
        json.dump(out, f, indent=1)


if __name__ == "__main__":
    main()
