#!/usr/bin/env python3
"""Write the converged FP64 oracle solutions of the benchmarked feeders.

Runs the CPU oracle (Algorithm 1 with the termination test of Section III-C,
rho = 100, eps_rel = 1e-4, the literal residual form) from the initial point
of Section V-A until the test holds, and stores what the GPU parity tests
compare against: the stopping sweep T_stop, the residual history (every row
near the stop and a thinned trace before it), the objective c'x, and the
final x, x_s and lambda.

Only ``oracle`` and the seeded input generator ``synth`` are used; nothing
here reads anything the GPU library computed.

Usage: python tests/golden/make_converged.py [8500] [2500] ...
(about 9 minutes for the 8500-bus feeder on one core).
"""
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

from oracle import admm, model  # noqa: E402
from synth import DEFAULT_SEEDS, make_feeder  # noqa: E402

TAIL = 64      # history rows kept in full before the stop
THIN = 1000    # and every THIN-th row before that


def path(name: str) -> str:
    return os.path.join(HERE, f"converged_{name}.npz")


def make(name: str) -> str:
    seed = DEFAULT_SEEDS[name]
    net = make_feeder(name, seed)
    t0 = time.perf_counter()
    prep = admm.prepare(model.decompose(net))
    res = admm.solve(prep, rho=100.0, eps_rel=1e-4, eps_abs=0.0, max_iter=1_000_000, form="paper")
    dt = time.perf_counter() - t0
    if not res.converged:
        raise RuntimeError(f"{name}: the oracle did not converge")
    H = res.history
    T = res.iters
    thin_rows = np.arange(THIN, max(T - TAIL, 0), THIN)
    tail_rows = np.arange(max(T - TAIL, 0) + 1, T + 1)
    out = path(name)
    np.savez_compressed(
        out, name=name, seed=seed, rho=100.0, eps_rel=1e-4, t_stop=T, objective=res.objective,
        x=res.x, xs=res.xs, lam=res.lam,
        hist_thin_sweeps=thin_rows, hist_thin=H[thin_rows - 1],
        hist_tail_sweeps=tail_rows, hist_tail=H[tail_rows - 1],
        oracle_seconds=dt)
    print(f"{name}: T_stop = {T}, objective = {res.objective:.15g}, {dt:.0f} s -> {out}", flush=True)
    return out


if __name__ == "__main__":
    for nm in (sys.argv[1:] or ["2500", "8500"]):
        make(nm)
