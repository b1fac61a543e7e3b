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


def dense_equivalent_bytes_per_sweep(sizes, w: int) -> float:
    """The same compulsory traffic with the dense n_s x n_s operator Abar_s in
    place of its rank form (the accounting of a dense matvec per subsystem)."""
    return (w * (sizes.op_words + sizes.n_local) + sizes.n_local * (4 * w + 4) + sizes.n * 5 * w)


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
    operators once, and per scenario bbar, x_s and lambda read and written
    (stored as x_s - lambda / rho and lambda), the gather of B_s x and the
    global x written."""
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


def run_many(P, make_feeder, stream, n13: int = 64, n123: int = 16) -> dict:
    """Several feeders in one persistent launch (ldopf_solve_many) against
    the same solves one after another, FP64, each to eps_rel 1e-4."""
    nets = [make_feeder("13", 54000 + i) for i in range(n13)] + [make_feeder("123", 54500 + i) for i in range(n123)]
    hs = [P.ldopf_create(n, P.ldopf_default_options(), stream=stream) for n in nets]
    for h in hs:  # warm: kernels loaded, history buffers allocated
        h.solve()
        h.reset()
    t0 = time.perf_counter()
    for h in hs:
        h.solve()
    t_seq = time.perf_counter() - t0
    for h in hs:
        h.reset()
    t0 = time.perf_counter()
    sts = P.ldopf_solve_many(hs)
    t_many = time.perf_counter() - t0
    out = {"workload": f"{n13} fresh 13-bus and {n123} fresh 123-bus feeders (seeds 54000+, 54500+), FP64, "
                       "each to eps_rel 1e-4",
           "workgroups": int(sum(h.sizes().n_parts for h in hs)),
           "converged": int(sum(s.converged for s in sts)),
           "one_launch_s": t_many, "one_launch_solves_per_s": len(hs) / t_many,
           "one_by_one_s": t_seq, "one_by_one_solves_per_s": len(hs) / t_seq,
           "speedup": t_seq / t_many, "max_iterations": int(max(s.iterations for s in sts))}
    for h in hs:
        h.close()
    return out


def run_streamed(P, L, make_feeder, net8500, iters_persistent: int, us_persistent: float, stream) -> dict:
    """The streamed sweep (operators and state in HBM, three launches per
    sweep replayed as HIP graphs): on the 8500-bus feeder beside the
    persistent sweep, and on a 12,000-bus feeder (the 8500-bus recipe with
    more buses), which the persistent sweep cannot hold in FP64 and the
    automatic choice streams; FP64, each to eps_rel 1e-4."""
    import dataclasses
    from synth import SPECS
    out = {}

    def solve(net, opts):
        p = P.ldopf_create(net, opts, stream=stream)
        warm = P.ldopf_default_options(max_iter=64, check_termination=0, sweep_path=opts.sweep_path)
        keep = P.ldopf_default_options(sweep_path=opts.sweep_path)
        p.set_options(warm)
        p.solve()  # warm: kernels loaded, graph path exercised
        p.reset()
        p.set_options(keep)
        t0 = time.perf_counter()
        st = p.solve()
        dt = time.perf_counter() - t0
        s = p.sizes()
        us = 1e3 * st.sweep_ms / max(1, st.sweeps_computed)
        rec = {"path": "streamed" if s.sweep_path == L.LDOPF_PATH_STREAMED else "persistent",
               "iterations_to_tol": st.iterations, "converged": bool(st.converged), "time_to_tol_s": dt,
               "us_per_sweep": us, "subsystems": s.n_sub, "local_copies": s.n_local,
               "bytes_per_sweep": algorithmic_bytes_per_sweep(s, 8),
               "achieved_GBs": algorithmic_bytes_per_sweep(s, 8) / (us * 1e-6) / 1e9, "objective": p.objective()}
        rec["frac_of_hbm_peak"] = rec["achieved_GBs"] / HBM_PEAK_GBS
        p.close()
        return rec

    out["8500"] = solve(net8500, P.ldopf_default_options(sweep_path=L.LDOPF_PATH_STREAMED))
    out["8500"]["persistent_iterations_to_tol"] = iters_persistent
    out["8500"]["persistent_us_per_sweep"] = us_persistent
    big = make_feeder(dataclasses.replace(SPECS["8500"], n_bus=12000), 12000)
    out["12000"] = solve(big, P.ldopf_default_options())
    out["12000"]["workload"] = ("12,000-bus synthetic feeder (the 8500-bus recipe, seed 12000), FP64 to eps_rel 1e-4: "
                                "too large for the LDS-resident sweep, run on the streamed one")
    return out


def _serving_requests(make_feeder, n_req: int, seed: int, id0: int):
    """n_req requests: feeder size uniform over {13, 123, 2500, 8500} buses,
    a fresh feeder seed each (id0 + i), FP32-mixed or FP64 with probability
    1/2 each."""
    import numpy as np
    rng = np.random.default_rng(seed)
    sizes = ["13", "123", "2500", "8500"]
    out = []
    for i in range(n_req):
        sz = sizes[int(rng.integers(0, 4))]
        out.append((sz, int(rng.integers(0, 2)), make_feeder(sz, id0 + i)))
    return out


def _serve(P, reqs, arrivals):
    """Submit reqs at the given arrival times (seconds from the start; None:
    all at once), wait for all, return the server's statistics."""
    srv = P.Server(max_slots=8)
    start = time.perf_counter()
    ids = []
    for k, (_, prec, net) in enumerate(reqs):
        if arrivals is not None:
            while time.perf_counter() - start < arrivals[k]:
                time.sleep(0.0005)
        ids.append(srv.submit(net, P.ldopf_default_options(precision=prec)))
        if arrivals is not None and (k + 1) % 25 == 0:
            progress(f"serving: {k + 1} of {len(reqs)} requests submitted")
    for k, rid in enumerate(ids):
        srv.wait(rid, 1200)
        if (k + 1) % 25 == 0:
            progress(f"serving: {k + 1} of {len(ids)} requests done")
    st = srv.stats()
    srv.close()
    return st


def run_serving(P, make_feeder, n_req: int, rate_fracs=(0.5, 0.9), seed: int = 7):
    """The serving stream: first the saturated throughput (n_req requests
    submitted at once), then Poisson arrivals of n_req fresh requests at each
    fraction of that throughput; latency = completion - submit."""
    import numpy as np

    def stats(st):
        return {"solves_per_s": st.solves_per_s, "p50_ms": st.p50_ms, "p99_ms": st.p99_ms, "mean_ms": st.mean_ms,
                "max_ms": st.max_ms, "completed": st.completed, "failed": st.failed,
                "peak_in_flight": st.peak_running, "peak_bytes": st.peak_bytes_in_use}

    reqs = _serving_requests(make_feeder, n_req, seed, 50000)
    sat = _serve(P, reqs, None)
    mu = sat.completed / max(sat.wall_s, 1e-9)
    progress(f"serving: saturated {mu:.2f} solves/s over {n_req} requests")
    out = {"workload": f"{n_req} requests per phase on fresh 13/123/2500/8500-bus feeders (size uniform), "
                       "FP32-mixed or FP64 at random, each to eps_rel 1e-4",
           "sizes": {z: sum(1 for r in reqs if r[0] == z) for z in ("13", "123", "2500", "8500")},
           "saturated": dict(stats(sat), arrivals="all at once"), "poisson": []}
    for j, frac in enumerate(rate_fracs):
        rate = frac * mu
        rng = np.random.default_rng(seed + 1 + j)
        arr = np.cumsum(rng.exponential(1.0 / rate, n_req))
        reqs = _serving_requests(make_feeder, n_req, seed + 100 + j, 60000 + 10000 * j)
        st = _serve(P, reqs, arr)
        out["poisson"].append(dict(stats(st), rate_fraction_of_saturated=frac, rate_per_s=rate))
        progress(f"serving: Poisson at {frac} x saturated done (p99 {st.p99_ms:.0f} ms)")
    return out


def _cpu_model() -> str:
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def _host_cores() -> int:
    try:
        return len(os.sched_getaffinity(0))
    except AttributeError:
        return os.cpu_count() or 1


def cpu_baseline(sweeps: int) -> dict:
    """The FP64 oracle timed on this host: a bounded sample of sweeps of the
    same feeder after its precompute, in a child process, once with one
    BLAS/OpenMP thread (the reported value) and once with every host core
    this process may run on available to BLAS/OpenMP."""
    def child(threads: int) -> dict:
        env = dict(os.environ, OMP_NUM_THREADS=str(threads), OPENBLAS_NUM_THREADS=str(threads),
                   MKL_NUM_THREADS=str(threads))
        out = subprocess.run([sys.executable, os.path.abspath(__file__), "--cpu-baseline-only", str(sweeps),
                              "--cpu-threads", str(threads)], env=env, capture_output=True, text=True, check=True)
        return json.loads(out.stdout.strip().splitlines()[-1])
    one = child(1)
    cores = _host_cores()
    allc = child(cores)
    one["cpu_model"] = _cpu_model()
    one["nproc"] = cores
    one["all_cores"] = {"value": allc["value"], "unit": allc["unit"], "cores": cores, "sample": allc["sample"]}
    return one


def _cpu_baseline_child(sweeps: int, threads: int):
    from oracle import admm, model
    from synth import make_feeder
    net = make_feeder("8500", 8500)
    prep = admm.prepare(model.decompose(net))
    t0 = time.perf_counter()
    admm.solve(prep, max_iter=sweeps, check=False)
    dt = time.perf_counter() - t0
    what = "one thread" if threads == 1 else f"{threads} BLAS/OpenMP threads allowed"
    print(json.dumps({"value": sweeps / dt, "unit": "iter/s", "cores": threads, "kind": "oracle",
                      "sample": f"{sweeps} FP64 oracle sweeps (global, local, dual update and residuals) of the "
                                f"same 8500-bus feeder after its precompute, {dt:.1f} s, {what}"}))


def run_small(P, L, make_feeder, stream, steps: int = 5) -> dict:
    """The 13- and 123-bus feeders to eps_rel 1e-4 in FP64: iterations, time
    to tolerance and time per sweep. The 13-bus plan is one workgroup with no
    exchange between workgroups, so its time per sweep is the floor that the
    sweep's block barriers and residual-sum round trip set."""
    out = {}
    for name in ("13", "123"):
        net = make_feeder(name, int(name))
        prob = P.ldopf_create(net, P.ldopf_default_options(), stream=stream)
        prob.solve()
        kms, comp = [], 0
        for _ in range(steps):
            prob.reset()
            st = prob.solve()
            kms.append(st.sweep_ms)
            comp += st.sweeps_computed
        sz = prob.sizes()
        out[name] = {"iterations_to_tol": st.iterations, "time_to_tol_ms": sum(kms) / len(kms),
                     "us_per_sweep": 1e3 * sum(kms) / comp, "workgroups": sz.n_parts,
                     "block_threads": sz.block_threads, "objective": prob.objective()}
        prob.close()
    return out


def exchange_floor(P, make_feeder, stream, sweeps: int = 20000) -> dict:
    """Time per sweep with the neighbour exchange and the grid-wide test over
    many workgroups but little work in each (fixed sweeps, FP64): the
    123-bus feeder cut into about 24 copies per workgroup (186 workgroups,
    one per subsystem), and the 2500-bus feeder on 256 workgroups of about 220
    copies; beside the 8500-bus sweep (256 workgroups of about 700 copies) and
    the 13-bus sweep (one workgroup, no exchange), they show how much of a
    sweep is the exchange floor and how much the work of a part."""
    out = {}
    for name, rows in (("123", 16), ("2500", 1)):
        net = make_feeder(name, int(name))
        prob = P.ldopf_create(net, P.ldopf_default_options(max_iter=sweeps, check_termination=0, rows_per_part=rows),
                              stream=stream)
        prob.solve()
        prob.reset()
        st = prob.solve()
        sz = prob.sizes()
        out[f"{name}bus"] = {"workgroups": sz.n_parts, "block_threads": sz.block_threads,
                             "local_copies_per_workgroup": sz.n_local / max(1, sz.n_parts),
                             "us_per_sweep": 1e3 * st.sweep_ms / max(1, st.sweeps_computed)}
        prob.close()
    return out


def phase_profile(P, net, stream, sweeps: int = 20000) -> dict:
    """Per-phase wall-clock time of one workgroup of the 8500-bus sweep
    (profiled build of the kernel, fixed sweeps), in us per sweep."""
    prob = P.ldopf_create(net, P.ldopf_default_options(max_iter=sweeps, check_termination=0, profile=1),
                          stream=stream)
    st = prob.solve()
    ms = prob.get_phase_times(0)
    prob.close()
    k = 1e3 / max(1, st.sweeps_computed)
    return {"sweeps": st.sweeps_computed, "us_per_sweep_profiled": 1e3 * st.sweep_ms / max(1, st.sweeps_computed),
            "global_update_and_exchange_wait": ms[0] * k, "own_global_update": ms[7] * k,
            "gather": ms[1] * k, "t_eq_W_v": ms[2] * k, "local_dual_residual_sums": ms[3] * k,
            "publish": ms[4] * k, "termination_test_wave": ms[6] * k}


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
    ap.add_argument("--serving-requests", type=int, default=16, help="requests per serving phase")
    ap.add_argument("--serving-only", action="store_true",
                    help="only the serving stream (saturated, then Poisson at 0.5 and 0.9 of it)")
    ap.add_argument("--profile-pass", action="store_true",
                    help="one copy of known size and one solve, for rocprofv3 counter runs")
    ap.add_argument("--profile-batched", type=int, default=0, metavar="SWEEPS",
                    help="only the batched workload: tune, then SWEEPS fixed sweeps, for rocprofv3 runs")
    ap.add_argument("--cpu-baseline-only", type=int, default=0, help=argparse.SUPPRESS)
    ap.add_argument("--cpu-threads", type=int, default=1, help=argparse.SUPPRESS)
    ap.add_argument("--no-small", action="store_true")
    ap.add_argument("--no-rho-balance", action="store_true")
    ap.add_argument("--no-many", action="store_true")
    ap.add_argument("--no-streamed", action="store_true")
    ap.add_argument("--profile-streamed", type=int, default=0, metavar="SWEEPS",
                    help="only the 8500-bus feeder on the streamed sweep, SWEEPS fixed sweeps, for rocprofv3 runs")
    args = ap.parse_args()
    if args.cpu_baseline_only:
        _cpu_baseline_child(args.cpu_baseline_only, args.cpu_threads)
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

    if args.profile_streamed:
        pnet = make_feeder("8500", 8500)
        ps = P.ldopf_create(pnet, P.ldopf_default_options(sweep_path=L.LDOPF_PATH_STREAMED,
                                                          max_iter=args.profile_streamed, check_termination=0),
                            stream=stream)
        st = ps.solve()
        sz = ps.sizes()
        us = 1e3 * st.sweep_ms / max(1, st.sweeps_computed)
        print(json.dumps({"sweeps": st.sweeps_computed, "us_per_sweep": us,
                          "bytes_per_sweep": algorithmic_bytes_per_sweep(sz, 8),
                          "achieved_GBs": algorithmic_bytes_per_sweep(sz, 8) / (us * 1e-6) / 1e9}))
        ps.close()
        return

    if args.serving_only:
        print(json.dumps({"serving": run_serving(P, make_feeder, args.serving_requests)}))
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
                     "launch_ms": launch_ms,
                     "achieved_is": "algorithmic bytes per sweep / time per sweep (operators and state stay in LDS)",
                     "measured_hbm_GBs": None, "limiter": "exchange latency between workgroups, block barriers "
                                                          "and dependent LDS reads, not HBM bandwidth",
                     "dense_equivalent_bytes_per_sweep": dense_equivalent_bytes_per_sweep(sizes, 8),
                     "dense_equivalent_GBs": dense_equivalent_bytes_per_sweep(sizes, 8) * sweeps_per_launch
                                             / (launch_ms * 1e-3) / 1e9},
    }
    if rec["roofline"]["traffic"] is not None:
        rec["roofline"]["measured_hbm_GBs"] = rec["roofline"]["traffic"] / (launch_ms * 1e-3) / 1e9
    prob.close()
    if not args.no_small:
        rec["small_feeders"] = run_small(P, L, make_feeder, stream)
        rec["sync_floor"] = {"us_per_sweep_13bus_one_workgroup": rec["small_feeders"]["13"]["us_per_sweep"],
                             "us_per_sweep_8500bus": rec["us_per_sweep"],
                             "many_workgroups_little_work": exchange_floor(P, make_feeder, stream),
                             "phase_us_8500bus_workgroup0": phase_profile(P, net, stream)}
        progress("small feeders and phase profile done")
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
    if not args.no_rho_balance:
        # residual balancing of rho (default rule: every 100 sweeps, mu 10,
        # tau 2, at most 16 changes) on the same feeder, capped at 500,000 sweeps
        pr = P.ldopf_create(net, P.ldopf_default_options(rho_update=L.LDOPF_RHO_BALANCE, max_iter=500000),
                            stream=stream)
        srb = pr.solve()
        rec["rho_balance"] = {"rule": "rho x/÷ 2 when pres/eps_prim and dres/eps_dual differ by more than 10x, "
                                      "checked every 100 sweeps, effective 4 sweeps later, at most 16 changes",
                              "iterations": srb.iterations, "converged": bool(srb.converged),
                              "time_s": 1e-3 * srb.sweep_ms, "rho_final": srb.rho, "rho_changes": srb.rho_changes,
                              "objective_rel_diff_vs_fixed_rho": (pr.objective() - obj) / max(1.0, abs(obj))}
        pr.close()
        progress(f"rho balancing: {srb.iterations} sweeps, converged {bool(srb.converged)}")
    if not args.no_many:
        rec["feeders_one_launch"] = run_many(P, make_feeder, stream)
        progress(f"feeders in one launch: {rec['feeders_one_launch']['speedup']:.1f}x one by one")
    if not args.no_streamed:
        rec["streamed"] = run_streamed(P, L, make_feeder, net, rec["iterations_to_tol"], rec["us_per_sweep"], stream)
        progress(f"streamed: 12000-bus in {rec['streamed']['12000']['time_to_tol_s']:.1f} s")
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
