#!/usr/bin/env python3
"""ADMM iter/s and time to the 1e-4 residual on the 8500-bus synthetic feeder.

One step = one full solve of the closed-form ADMM (Algorithm 1: global
update, local update, dual update, termination test at eps_rel = 1e-4, rho =
100) from the initial point, on the seed-8500 synthetic radial three-phase
feeder with about 8500 buses, 70% single-phase laterals and lognormal loads.
The network is assembled, decomposed, uploaded and its operators precomputed
on the GPU before timing (the precompute time is reported beside the result);
the timed region is the solve itself with every input resident in HBM.

Prints one JSON line. ``--gpus N`` with N > 1 is refused: the solver runs on
one GPU.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import re
import subprocess
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0  # MI355X HBM3E
PROFILE_MD = os.path.join(ROOT, "profiles", "sweep_fp64_8500bus_counters.md")
KERNEL_SRC = os.path.join(ROOT, "paper_2310_09410_amd", "csrc", "device.hip")
WORKLOAD = ("8500-bus synthetic radial 3-phase feeder (seed 8500; 20/10/70% three/two/single-phase lines; "
            "lognormal(ln 5 kW, 0.8) per-phase loads, Q = 0.3 P; one substation generator), "
            "plain FP64 ADMM to eps_rel = 1e-4, rho = 100")


def progress(msg: str) -> None:
    """One line on stderr per finished part of the run (stdout carries only the result)."""
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def algorithmic_bytes_per_sweep(sizes, w: int) -> float:
    """Compulsory bytes of one sweep: the rank-form operators and bbar, the
    local copies' x_s and lambda read and written plus their int32 global
    index, and the global x written and gathered with its lo, hi and c."""
    return (w * (sizes.rank_words + sizes.n_local) + sizes.n_local * (4 * w + 4) + sizes.n * 5 * w)


def kernel_sha() -> str:
    """Hash of the sweep kernel's source with comments and whitespace removed,
    so that the stored counters stay valid across comment-only edits and
    lapse with any change of code."""
    src = open(KERNEL_SRC, encoding="utf-8").read()
    src = re.sub(r"/\*.*?\*/", " ", src, flags=re.S)
    src = re.sub(r"//[^\n]*", " ", src)
    src = re.sub(r"\s+", "", src)
    return hashlib.sha256(src.encode()).hexdigest()


def stored_traffic():
    """HBM bytes per sweep-kernel launch from the committed counter summary,
    or None when it is missing or was taken on a different kernel source."""
    if not os.path.exists(PROFILE_MD):
        return None
    text = open(PROFILE_MD).read()
    m_sha = re.search(r"kernel_source_sha256:\s*([0-9a-f]{64})", text)
    m_t = re.search(r"traffic_bytes_per_launch:\s*([0-9.eE+]+)", text)
    if not m_sha or not m_t or m_sha.group(1) != kernel_sha():
        return None
    return float(m_t.group(1))


def batched_bytes_per_sweep(bs) -> float:
    """Compulsory bytes of one batched sweep (FP32): shared and per-scenario
    operators once, and per scenario bbar, x_s and lambda read and written,
    the gather of B_s x and the global x written."""
    per_scen = 4 * (bs.n_local * (1 + 4 + 1) + bs.n)
    return 4 * (bs.shared_operator_words + bs.scenario_operator_words) + bs.n_scen * per_scen


def run_batched(P, L, make_feeder, scenario_factors, stream):
    """2500-bus feeder x 256 load scenarios (FP32-mixed, MFMA) against plain
    FP64 solves of the same feeder, both to eps_rel 1e-4."""
    net = make_feeder("2500", 2500)
    f = scenario_factors(net, 256)
    b = P.ldopf_batch_create(net, f, stream=stream)
    b.tune(None)
    b.set_options(P.ldopf_default_options(precision=L.LDOPF_FP32_MIXED, max_iter=64, check_termination=0))
    b.reset()
    b.solve()  # warm: graph instantiation
    b.set_options(P.ldopf_default_options(precision=L.LDOPF_FP32_MIXED))
    b.reset()
    t0 = time.perf_counter()
    st = b.solve()
    dt = time.perf_counter() - t0
    bs = b.sizes()
    it = sorted(b.scenario(k).iterations for k in range(256))
    plain = P.ldopf_create(net, P.ldopf_default_options(), stream=stream)
    plain.solve()
    plain.reset()
    t1 = time.perf_counter()
    ps = plain.solve()
    dp = time.perf_counter() - t1
    us = 1e3 * st.solve_ms / max(1, st.sweeps)
    rec = {"workload": "2500-bus feeder (seed 2500) x 256 load scenarios (per-bus factors U[0.7, 1.3]), "
                       "FP32-mixed, each scenario to eps_rel 1e-4",
           "solves_per_s": 256 / dt, "batch_time_s": dt, "converged": st.n_converged, "sweeps": st.sweeps,
           "iterations_min_median_max": [it[0], it[128], it[-1]], "us_per_batched_sweep": us,
           "achieved_GBs": batched_bytes_per_sweep(bs) / (us * 1e-6) / 1e9,
           "bytes_per_batched_sweep": batched_bytes_per_sweep(bs),
           "mfma_subsystems": bs.n_mfma_subsystems, "vector_subsystems": bs.n_vector_subsystems,
           "precompute_ms": st.precompute_ms,
           "plain_fp64_solves_per_s": 1.0 / dp, "plain_fp64_iterations": ps.iterations,
           "speedup_vs_plain_fp64": (256 / dt) * dp}
    b.close()
    plain.close()
    return rec


def run_serving(P, make_feeder, n_req: int, seed: int = 7):
    """Poisson arrivals of solve requests on fresh feeders sized uniformly
    from {13, 123, 2500, 8500} buses, FP32-mixed or FP64 with probability
    1/2 each, at about 0.9 of a serial server's throughput."""
    import numpy as np
    rng = np.random.default_rng(seed)
    sizes = ["13", "123", "2500", "8500"]
    est_s = {"13": 0.005, "123": 0.05, "2500": 1.1, "8500": 2.0}  # serial solve times, measured before
    rate = 0.9 / (sum(est_s.values()) / 4)
    plan = []
    t = 0.0
    for i in range(n_req):
        t += rng.exponential(1.0 / rate)
        plan.append((t, sizes[int(rng.integers(0, 4))], int(rng.integers(0, 2)), 50000 + i))
    nets = [(at, make_feeder(sz, sd), prec) for at, sz, prec, sd in plan]
    srv = P.Server(max_slots=8)
    start = time.perf_counter()
    ids = []
    for at, net, prec in nets:
        while time.perf_counter() - start < at:
            time.sleep(0.001)
        ids.append(srv.submit(net, P.ldopf_default_options(precision=prec)))
    for rid in ids:
        srv.wait(rid, 600)
    st = srv.stats()
    srv.close()
    return {"workload": f"{n_req} Poisson requests (rate {rate:.2f}/s) on fresh 13/123/2500/8500-bus feeders, "
                        "FP32-mixed or FP64 at random, to eps_rel 1e-4",
            "solves_per_s": st.solves_per_s, "p50_ms": st.p50_ms, "p99_ms": st.p99_ms, "mean_ms": st.mean_ms,
            "completed": st.completed, "failed": st.failed, "peak_in_flight": st.peak_running,
            "peak_bytes": st.peak_bytes_in_use, "sizes": [p_[1] for p_ in plan]}


def cpu_baseline(sweeps: int) -> dict:
    """The FP64 oracle timed on this host: a bounded sample of sweeps of the
    same feeder after its precompute. Runs in a child process pinned to one
    BLAS/OpenMP thread so the core count is exact."""
    env = dict(os.environ, OMP_NUM_THREADS="1", OPENBLAS_NUM_THREADS="1", MKL_NUM_THREADS="1")
    out = subprocess.run([sys.executable, os.path.abspath(__file__), "--cpu-baseline-only", str(sweeps)],
                         env=env, capture_output=True, text=True, check=True)
    return json.loads(out.stdout.strip().splitlines()[-1])


def _cpu_baseline_child(sweeps: int):
    from oracle import admm, model
    from synth import make_feeder
    net = make_feeder("8500", 8500)
    prep = admm.prepare(model.decompose(net))
    t0 = time.perf_counter()
    admm.solve(prep, max_iter=sweeps, check=False)
    dt = time.perf_counter() - t0
    print(json.dumps({"value": sweeps / dt, "unit": "iter/s", "cores": 1, "kind": "oracle",
                      "sample": f"{sweeps} FP64 oracle sweeps (global, local, dual update and residuals) of the "
                                f"same 8500-bus feeder after its precompute, {dt:.1f} s, one thread"}))


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--cpu-sweeps", type=int, default=6000, help="oracle sweeps timed for the CPU baseline (about 13 s)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-fp32", action="store_true")
    ap.add_argument("--no-batched", action="store_true")
    ap.add_argument("--no-serving", action="store_true")
    ap.add_argument("--serving-requests", type=int, default=12)
    ap.add_argument("--profile-pass", action="store_true",
                    help="one copy of known size and one solve, for rocprofv3 counter runs")
    ap.add_argument("--profile-batched", type=int, default=0, metavar="SWEEPS",
                    help="only the batched workload: tune, then SWEEPS fixed sweeps, for rocprofv3 runs")
    ap.add_argument("--cpu-baseline-only", type=int, default=0, help=argparse.SUPPRESS)
    args = ap.parse_args()
    if args.cpu_baseline_only:
        _cpu_baseline_child(args.cpu_baseline_only)
        return
    if args.gpus != 1:
        print(f"bench.py runs on one GPU; --gpus {args.gpus} is not supported "
              "(independent solves shard across GPUs without communication)", file=sys.stderr)
        sys.exit(2)

    import torch
    import paper_2310_09410_amd as P
    from paper_2310_09410_amd import ldopf as L
    from synth import make_feeder, scenario_factors

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    torch.cuda.set_device(0)
    stream = torch.cuda.current_stream()
    net = make_feeder("8500", 8500)

    if args.profile_batched:
        bnet = make_feeder("2500", 2500)
        b = P.ldopf_batch_create(bnet, scenario_factors(bnet, 256), stream=stream)
        r, w = b.tune(None)
        b.set_options(P.ldopf_default_options(precision=L.LDOPF_FP32_MIXED, max_iter=args.profile_batched,
                                              check_termination=0))
        b.reset()
        st = b.solve()
        bs = b.sizes()
        us = 1e3 * st.solve_ms / max(1, st.sweeps)
        print(json.dumps({"sweeps": st.sweeps, "us_per_batched_sweep": us, "rows_per_chunk": r, "blocks_per_tile": w,
                          "bytes_per_batched_sweep": batched_bytes_per_sweep(bs),
                          "achieved_GBs": batched_bytes_per_sweep(bs) / (us * 1e-6) / 1e9}))
        b.close()
        return

    if args.profile_pass:
        n = 256 << 20  # 1 GiB of float32 read and 1 GiB written: past the 256 MB cache
        x = torch.empty(n, dtype=torch.float32, device="cuda").uniform_()
        y = torch.empty_like(x)
        y.copy_(x)
        prob = P.ldopf_create(net, P.ldopf_default_options(), stream=stream)
        st = prob.solve()
        torch.cuda.synchronize()
        prob.close()
        print(json.dumps({"copy_bytes_each_way": 4 * n, "sweeps_computed": st.sweeps_computed,
                          "sweep_ms": st.sweep_ms, "kernel_source_sha256": kernel_sha()}))
        return

    def run(precision):
        prob = P.ldopf_create(net, P.ldopf_default_options(precision=precision), stream=stream)
        for _ in range(args.warmup):
            prob.reset()
            prob.solve()
        torch.cuda.synchronize()
        iters = computed = 0
        kms = []
        t0 = time.perf_counter()
        for _ in range(args.steps):
            prob.reset()
            st = prob.solve()
            iters += st.iterations
            computed += st.sweeps_computed
            kms.append(st.sweep_ms)
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        return prob, st, iters, computed, kms, dt

    prob, st, iters, computed, kms, dt = run(L.LDOPF_FP64)
    progress(f"fp64: {args.steps} solves in {dt:.2f} s")
    sizes = prob.sizes()
    obj = prob.objective()
    b_sweep = algorithmic_bytes_per_sweep(sizes, 8)
    launch_ms = sum(kms) / len(kms)
    sweeps_per_launch = computed / args.steps
    achieved = b_sweep * sweeps_per_launch / (launch_ms * 1e-3) / 1e9
    rec = {
        "metric": "ADMM iter/s + time to 1e-4 residual, 8500-bus-shaped feeder; batched solves/s",
        "value": iters / dt,
        "unit": "iter/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": 1e3 * dt / args.steps,
        "higher_is_better": True,
        "scaling": "strong",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": WORKLOAD, "buses": net["n_bus"], "subsystems": sizes.n_sub,
                   "global_vars": sizes.n, "local_copies": sizes.n_local, "workgroups": sizes.n_parts,
                   "block_threads": sizes.block_threads, "lds_bytes_per_workgroup": sizes.lds_bytes},
        "iterations_to_tol": st.iterations,
        "time_to_tol_s": 1e-3 * launch_ms,
        "us_per_sweep": 1e3 * launch_ms / sweeps_per_launch,
        "precompute_ms": st.precompute_ms,
        "objective": obj,
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS, "traffic": stored_traffic(),
                     "kernel": "sweep_kernel<double> (one persistent launch per solve)",
                     "bytes_per_sweep": b_sweep, "sweeps_per_launch": sweeps_per_launch,
                     "launch_ms": launch_ms},
    }
    prob.close()
    if not args.no_fp32:
        p32, st32, it32, c32, k32, dt32 = run(L.LDOPF_FP32_MIXED)
        progress(f"fp32-mixed: {args.steps} solves in {dt32:.2f} s")
        s32 = p32.sizes()
        rec["fp32_mixed"] = {"iter_per_s": it32 / dt32, "iterations_to_tol": st32.iterations,
                             "time_to_tol_s": 1e-3 * sum(k32) / len(k32),
                             "us_per_sweep": 1e3 * sum(k32) / c32,
                             "achieved_GBs": algorithmic_bytes_per_sweep(s32, 4) * c32 / (1e-3 * sum(k32)) / 1e9,
                             "objective": p32.objective(), "objective_rel_diff_vs_fp64":
                                 abs(p32.objective() - obj) / max(1.0, abs(obj))}
        p32.close()
    if not args.no_batched:
        rec["batched"] = run_batched(P, L, make_feeder, scenario_factors, stream)
        progress(f"batched: {rec['batched']['solves_per_s']:.2f} solves/s")
    if not args.no_serving:
        rec["serving"] = run_serving(P, make_feeder, args.serving_requests)
        progress("serving done")
    if not args.no_cpu_baseline:
        rec["cpu_baseline"] = cpu_baseline(args.cpu_sweeps)
        progress("cpu baseline done")
    print(json.dumps(rec))


if __name__ == "__main__":
    main()
