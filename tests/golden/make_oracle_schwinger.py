"""Writes ``tests/golden/oracle_schwinger.json``: the oracle's Schwinger
function of the gluon propagator at the full workload size, with the solution
it is computed on.

Calls only ``oracle/``.  The scaling solution at the paper's parameters
(Lambda^2 = 5e4, eps^2 = 1e-6, Z(Lambda^2) = 0.256, alpha(mu^2) = 1; Sec. 2.1)
from the oracle's Newton iteration (two full steps after convergence), then
Delta(t) = (1/pi) int_0^p_max dp cos(t p) Z(p^2)/p^2 (Sec. 2.2) with the
2^17-node mapped Gauss-Legendre rule (Sec. 5), p_max = 1e3 GeV, at 48 times
t = 0.25 k GeV^-1; also mu^2 (G^2 Z = 1, Sec. 2.1 footnote).

Run from the repository root:  python tests/golden/make_oracle_schwinger.py
(about a minute on eight host threads: the 2^17-node rule is O(n^2)).
"""
from __future__ import annotations

import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import oracle  # noqa: E402
import workloads  # noqa: E402

OUT = os.path.join(ROOT, "tests", "golden", "oracle_schwinger.json")


def main() -> None:
    cfg = workloads.config("paper")
    p = oracle.params(**cfg)
    c, rep = oracle.newton(p, extra_iters=2)
    assert rep["status"] == 0
    n, p_max = workloads.SCHWINGER["n_nodes"], workloads.SCHWINGER["p_max"]
    t = 0.25 * np.arange(48)
    t0 = time.time()
    delta = oracle.schwinger(p, c, t, n=n, p_max=p_max)
    secs = time.time() - t0
    out = {"workload": workloads.WORKLOAD_NAMES["paper"], "config": cfg, "c": c.tolist(),
           "n_nodes": n, "p_max": p_max, "t": t.tolist(), "delta": delta.tolist(),
           "mu2": oracle.renorm_scale(p, c), "oracle_seconds": secs,
           "oracle_threads": oracle.get_threads()}
    with open(OUT, "w") as f:
        json.dump(out, f, indent=1)
    print("wrote %s (%.1f s)" % (OUT, secs))


if __name__ == "__main__":
    main()
