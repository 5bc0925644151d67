"""Writes ``tests/golden/oracle_roots.json``: the oracle's converged Chebyshev
coefficients of the N = 16, N = 64 and N = 128 workloads, with the numbers the
GPU parity tests judge them by.

Calls only ``oracle/``.  For each workload:
  c      the root of the oracle's Newton iteration from its asymptotic start,
         with two full steps after convergence (Sec. 3 Newton-Raphson);
  bound  u || |J^{-1}| S ||_inf at the root (u = 2^-53): how far the root can
         move when every term of every row changes by one unit roundoff;
  floor  the largest shift of the root when every quadrature weight of the
         oracle is moved by one ulp (both sign patterns), i.e. the rounding
         floor of the discrete problem itself;
  iters  oracle Newton iterations.

Run from the repository root:  python tests/golden/make_oracle_roots.py [names]
(N = 128 takes several minutes on eight host threads).
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

OUT = os.path.join(ROOT, "tests", "golden", "oracle_roots.json")


def solve(name: str) -> dict:
    cfg = workloads.config(name)
    p = oracle.params(**cfg)
    t0 = time.time()
    c, rep = oracle.newton(p, extra_iters=2)
    assert rep["status"] == 0, rep
    J = oracle.jacobian(p, c)
    S = oracle.residual_scale(p, c)
    bound = 2.0 ** -53 * float(np.max(np.abs(np.linalg.inv(J)) @ S))
    shifts = []
    for sign in (1.0, -1.0):
        try:
            oracle.set_jitter(sign * 2.0 ** -52)
            cj, rj = oracle.newton(p, c0=c, extra_iters=2)
        finally:
            oracle.set_jitter(0.0)
        assert rj["status"] == 0, rj
        shifts.append(float(np.max(np.abs(cj - c))))
    print("%s: %d iterations, bound %.3e, floor %.3e, %.0f s"
          % (name, rep["iters"], bound, max(shifts), time.time() - t0), flush=True)
    return {"workload": workloads.WORKLOAD_NAMES[name], "config": cfg,
            "c": [float(v) for v in c], "iters": int(rep["iters"]),
            "bound": bound, "floor": max(shifts),
            "scaled_residual": float(rep["fnorm"])}


def main(names):
    data = {}
    if os.path.exists(OUT):
        with open(OUT) as f:
            data = json.load(f)
    for name in names:
        data[name] = solve(name)
        with open(OUT, "w") as f:
            json.dump(data, f, indent=1)
            f.write("\n")


if __name__ == "__main__":
    main(sys.argv[1:] or ["cfg1", "cfg2", "cfg3"])
