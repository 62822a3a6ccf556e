#!/usr/bin/env python3
"""Benchmark: PBN node-updates/s, batched vs plain, plus p50/p99 query latency.

One step = one end-to-end solve of the batched workload: 512 random PBNs
(n log-uniform in 20..2000, 1-3 predictors per node, 1-5 parents, p in
{1e-3, 1e-4}, 64-1024 chains each), every network estimating P(2-node state
set) by Gelman-Rubin (R < 1.1) then the parallel two-state method at r = 0.01,
95% confidence; all networks advance together (one trajectory launch and one
reduction launch per round).  Inputs (compiled networks, device buffers) are
resident before the timed region.

Beside the timed line it measures, outside the timed region:
  * plain: the same solves one network at a time (own launches per network) on a
    fixed sample of the networks, as node-updates/s;
  * serving: a Poisson stream (200 requests/s) of queries on PBNs with n
    log-uniform in 50..5000 through the continuous-batching server, p50/p99
    latency from arrival to result, and a serial-solve baseline on the first
    requests of the same trace;
  * roofline of the trajectory kernel from HIP-event-timed launches;
  * cpu_baseline: the oracle's simulator on the host cores on a bounded sample.
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

import numpy as np  # noqa: E402

import pbnsynth as ps  # noqa: E402

METRIC = "PBN node-updates/s (batched vs plain) + p50/p99 query latency at r=0.01"
# MI355X: 256 CUs x 4 SIMDs x 16 lanes at 2.4 GHz, one 32-bit integer op per lane per clock
PEAK_INT32_OPS = 256 * 4 * 16 * 2.4e9
MAX_LEN = 1 << 17


def log(msg: str) -> None:
    print(msg, file=sys.stderr, flush=True)


def make_sims(pkg, jobs, max_len=MAX_LEN):
    nets = [pkg.Network(ps.to_text(j.net)) for j in jobs]
    sims = [pkg.Simulation(nt, j.chains, j.seed, max_props=len(j.patterns), max_len=max_len)
            for nt, j in zip(nets, jobs)]
    return nets, sims


def batched_step(pkg, sims, jobs):
    return pkg.batch_estimate(sims, [j.patterns for j in jobs], [j.r for j in jobs],
                              [j.confidence for j in jobs], psrf_max=1.1)


def node_updates_of(sims, jobs):
    return float(sum(s.position()[1] * j.chains * j.net.n for s, j in zip(sims, jobs)))


def run_serving(pkg, torch, seconds, rate, arena_bytes, serial_budget_s=20.0, sched=None, workers=None):
    jobs = ps.serving(duration_s=seconds, rate=rate, workers=cpu_threads() if workers is None else workers)
    log("serving: {} requests over {:.1f} s".format(len(jobs), seconds))
    nets = [pkg.Network(j.text) for j in jobs]
    srv = pkg.Server(arena_bytes)
    srv.configure(**(sched or {}))
    t0 = time.perf_counter()
    nxt, ids, finish = 0, {}, {}
    pkg.profile_enable(True)
    pkg.profile_reset()
    rounds = 0
    pending = set()                   # submitted, not yet answered
    while len(finish) < len(jobs):
        now = time.perf_counter() - t0
        while nxt < len(jobs) and jobs[nxt].arrival <= now:
            j = jobs[nxt]
            ids[nxt] = srv.submit(nets[nxt], j.chains, j.seed, j.patterns, j.r, j.confidence,
                                  max_len=MAX_LEN, psrf_max=1.1)
            pending.add(nxt)
            nxt += 1
        active, waiting, done = srv.step()
        rounds += 1
        if rounds % 50 == 0:
            log("  round {}: t={:.1f}s submitted {} active {} waiting {} done {}".format(
                rounds, time.perf_counter() - t0, nxt, active, waiting, done))
        if done > len(finish):
            t_now = time.perf_counter() - t0
            for i in [i for i in pending if srv.poll(ids[i]) is not None]:
                finish[i] = t_now
                pending.discard(i)
        if active == 0 and waiting == 0 and nxt < len(jobs):
            time.sleep(max(0.0, jobs[nxt].arrival - (time.perf_counter() - t0)))
    wall = time.perf_counter() - t0
    prof = pkg.profile_read()
    pkg.profile_enable(False)
    long_moved, long_rounds = srv.lane_stats()
    lat = np.array([finish[i] - jobs[i].arrival for i in range(len(jobs))])
    results = [srv.poll(ids[i]) for i in range(len(jobs))]
    _, peak_mem = srv.memory()
    # serial baseline: the first requests solved one at a time in arrival order
    # (as many as fit in the time budget)
    k = 0
    t_free, serial_lat = 0.0, []
    t_serial = time.perf_counter()
    for i in range(len(jobs)):
        if time.perf_counter() - t_serial > serial_budget_s:
            break
        k += 1
        j = jobs[i]
        sim = pkg.Simulation(nets[i], j.chains, j.seed, max_props=1, max_len=MAX_LEN)
        a = time.perf_counter()
        sim.estimate(j.patterns, j.r, j.confidence, psrf_max=1.1)
        service = time.perf_counter() - a
        start = max(j.arrival, t_free)
        t_free = start + service
        serial_lat.append(t_free - j.arrival)
        log("  serial {}: n={} {:.1f} ms".format(i, j.net.n, service * 1e3))
        del sim
    serial_lat = np.array(serial_lat)
    return dict(
        requests=len(jobs), arrival_rate_per_s=rate, arrival_seconds=seconds, wall_s=wall, rounds=rounds,
        p50_ms=float(np.percentile(lat, 50) * 1e3), p99_ms=float(np.percentile(lat, 99) * 1e3),
        queries_per_s=len(jobs) / wall, node_updates_per_s=prof["node_updates"] / wall,
        # the trajectory kernels' algorithmic operations over the serving wall time
        roofline={"bound": "alu", "achieved": prof["alg_ops"] / wall / 1e12, "peak": PEAK_INT32_OPS / 1e12,
                  "unit": "Tops/s", "frac": prof["alg_ops"] / wall / PEAK_INT32_OPS,
                  "kernel_frac": prof["alg_ops"] / max(prof["kernel_ms"] / 1e3, 1e-12) / PEAK_INT32_OPS,
                  "launches": int(prof["launches"]), "split_launches": int(prof["split_launches"])},
        not_converged=int(sum(r[0]["status"] != 0 for r in results)),
        long_lane_requests=long_moved, long_lane_rounds=long_rounds,
        split_fallbacks=int(prof["split_fallbacks"]),
        arena_bytes=arena_bytes, arena_peak_bytes=peak_mem,
        serial_first_k=k,
        serial_p50_ms=float(np.percentile(serial_lat, 50) * 1e3) if k else None,
        serial_p99_ms=float(np.percentile(serial_lat, 99) * 1e3) if k else None,
    )


def run_saturated(pkg, count, arena_bytes):
    """Capacity: the first `count` requests of the serving trace all queued at
    once, the server stepped until every one is answered; queries/s and
    node-updates/s over that wall time, and queries/s up to the answer that
    completes 99% of them (the last ones are bound by their own chain length,
    with the device nearly idle)."""
    jobs = ps.serving(duration_s=1e9, rate=200.0, limit=count, workers=cpu_threads())
    nets = [pkg.Network(j.text) for j in jobs]
    srv = pkg.Server(arena_bytes)
    pkg.profile_enable(True)
    pkg.profile_reset()
    t0 = time.perf_counter()
    ids = [srv.submit(nt, j.chains, j.seed, j.patterns, j.r, j.confidence, max_len=MAX_LEN, psrf_max=1.1)
           for nt, j in zip(nets, jobs)]
    rounds = 0
    t99 = None
    while True:
        active, waiting, done = srv.step()
        rounds += 1
        if rounds % 100 == 0:
            log("  saturated round {}: active {} waiting {} done {}".format(rounds, active, waiting, done))
        if t99 is None and 100 * done >= 99 * len(jobs):
            t99 = time.perf_counter() - t0
        if done == len(jobs):
            break
    wall = time.perf_counter() - t0
    prof = pkg.profile_read()
    pkg.profile_enable(False)
    nconv = sum(srv.poll(i)[0]["status"] != 0 for i in ids)
    _, peak_mem = srv.memory()
    n99 = -(-99 * len(jobs) // 100)
    return dict(requests=len(jobs), wall_s=wall, rounds=rounds, queries_per_s=len(jobs) / wall,
                wall_99_s=t99, queries_per_s_99=n99 / t99,
                node_updates_per_s=prof["node_updates"] / wall,
                roofline_frac=prof["alg_ops"] / wall / PEAK_INT32_OPS, not_converged=int(nconv),
                arena_peak_bytes=peak_mem)


def single_workload(pkg, torch, name: str, steps: int, warmup: int, cpu_s: float, no_cpu: bool) -> dict:
    """One network of a plain configuration (tiny, medium or large), solved end
    to end by estimate_prob per step; every step restarts the same chains."""
    job = getattr(ps, name)()
    net = pkg.Network(ps.to_text(job.net))
    sim = pkg.Simulation(net, job.chains, job.seed, max_props=len(job.patterns), max_len=MAX_LEN)
    kw = dict(method=job.method, psrf_max=job.psrf_max)
    for w in range(warmup):
        log("warmup {}".format(w))
        sim.estimate(job.patterns, job.r, job.confidence, **kw)
    torch.cuda.synchronize()
    pkg.profile_enable(True)
    pkg.profile_reset()
    times, nus, res = [], [], None
    for k in range(steps):
        torch.cuda.synchronize()
        a = time.perf_counter()
        res = sim.estimate(job.patterns, job.r, job.confidence, **kw)
        torch.cuda.synchronize()
        times.append(time.perf_counter() - a)
        nus.append(float(sim.position()[1]) * job.chains * job.net.n)
        log("step {}: {:.3f} s, {:.3e} node-updates".format(k, times[-1], nus[-1]))
    prof = pkg.profile_read()
    pkg.profile_enable(False)
    total_t = sum(times)
    line = {
        "metric": METRIC, "value": sum(nus) / total_t, "unit": "node-updates/s", "n_gpus": 1, "steps": steps,
        "warmup": warmup, "ms_per_step": total_t / steps * 1e3, "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "u32", "data": "synthetic",
        "config": {"workload": "{}: one random PBN, n={}, {} chains, {} state set(s), {} r={} s={}, psrf {}".format(
            name, job.net.n, job.chains, len(job.patterns), job.method, job.r, job.confidence, job.psrf_max),
            "chain_len": int(sim.position()[0]), "transitions": int(sim.position()[1])},
        "roofline": roofline_of(prof, total_t, batched=False),
        "results": [{k: r[k] for k in ("prob", "ci_lo", "ci_hi", "psi", "n", "N", "M", "kappa", "batches")} for r in res],
        "cpu_baseline": None if no_cpu else cpu_baseline([job], cpu_s, "the {} configuration".format(name)),
    }
    return line


def multiprop_workload(pkg, torch, steps: int, warmup: int, cpu_s: float, no_cpu: bool) -> dict:
    """The paper's multi-property experiment shape (Sec. 5.2, Table 2) on a
    synthetic 96-node network: 7 state sets estimated together (one run whose
    chains serve every property) against one by one (a run per property), both
    on the GPU.  Reports the speed-up sum(t_i)/t_multi and the sample-size
    reduction; each property's result must be identical in both."""
    job = ps.multiprop()
    net = pkg.Network(ps.to_text(job.net))
    max_len = 1 << 15
    kw = dict(psrf_max=job.psrf_max)

    def solve(pats):
        sim = pkg.Simulation(net, job.chains, job.seed, max_props=len(pats), max_len=max_len)
        torch.cuda.synchronize()
        a = time.perf_counter()
        res = sim.estimate(pats, job.r, job.confidence, **kw)
        torch.cuda.synchronize()
        t = time.perf_counter() - a
        nu = float(sim.position()[1]) * job.chains * job.net.n
        del sim
        return t, nu, res

    for w in range(warmup):
        log("warmup {}".format(w))
        solve(job.patterns)
    pkg.profile_enable(True)
    pkg.profile_reset()
    t_multi, nus, res_multi = [], [], None
    for k in range(steps):
        t, nu, res_multi = solve(job.patterns)
        t_multi.append(t)
        nus.append(nu)
        log("simultaneous {}: {:.1f} ms".format(k, t * 1e3))
    prof = pkg.profile_read()
    pkg.profile_enable(False)
    t_one, res_one = [], []
    for q, pat in enumerate(job.patterns):
        t, _, r = solve([pat])
        t_one.append(t)
        res_one.append(r[0])
        log("property {} alone: {:.1f} ms".format(q, t * 1e3))
    same = all(res_one[q][key] == res_multi[q][key] for q in range(len(job.patterns))
               for key in ("prob", "psi", "n", "N", "M", "chain_len", "status"))
    t_m = sum(t_multi) / len(t_multi)
    samples_multi = job.chains * max(r["chain_len"] for r in res_multi)
    samples_one = sum(job.chains * r["chain_len"] for r in res_one)
    return {
        "metric": METRIC, "value": sum(nus) / sum(t_multi), "unit": "node-updates/s", "n_gpus": 1, "steps": steps,
        "warmup": warmup, "ms_per_step": t_m * 1e3, "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "u32", "data": "synthetic",
        "config": {"workload": "multiprop: 96-node synthetic PBN (107 functions), {} chains, 7 state sets, "
                               "two-state r={} s={}, psrf {}".format(job.chains, job.r, job.confidence, job.psrf_max)},
        "multiprop": {"t_multi_ms": t_m * 1e3, "t_one_by_one_ms": [t * 1e3 for t in t_one],
                      "speedup_sum_ti_over_tmulti": sum(t_one) / t_m,
                      "samples_multi": samples_multi, "samples_one_by_one": samples_one,
                      "sample_reduction": samples_one / samples_multi, "results_identical": bool(same),
                      "N": [int(r["N"]) for r in res_multi], "prob": [r["prob"] for r in res_multi]},
        "roofline": roofline_of(prof, sum(t_multi), batched=False),
        "cpu_baseline": None if no_cpu else cpu_baseline([job], cpu_s, "the multiprop configuration"),
    }


R_SEQ = 2e-3      # the paper's 1e-4 would take minutes for one chain
SEQ_LEN = 1 << 22  # positions of the one sequential chain


def sequential_workload(pkg, torch, cpu_s: float, no_cpu: bool) -> dict:
    """The paper's sequential-versus-parallel comparison (Sec. 5.1, Table 1): for each
    network, the sequential method on one chain against the parallel method on
    the configuration's chains, both on the GPU, for the two-state pair (Alg. 1
    against Alg. 4) and the Skart pair (Alg. 2 against Alg. 5).  Reports
    t_sequential/t_parallel, the speed-up corrected for the sample sizes (sp *
    size_p / size_s), and the paired agreement |p_seq - p_par| < 2r of the
    paper's check; optionally the oracle's sequential method on one host thread
    (the paper's sequential baseline runs on one core)."""
    from oracle import drivers
    batched = ps.batched(512)
    jobs = [ps.medium()] + [min(batched, key=lambda j: abs(j.net.n - target)) for target in (200, 1000)]
    rows = []
    for job in jobs:
        net = pkg.Network(ps.to_text(job.net))
        pat = job.patterns[:1]
        job.r = R_SEQ

        def timed(omega, method):
            sim = pkg.Simulation(net, omega, job.seed, max_props=1, max_len=MAX_LEN if omega > 1 else SEQ_LEN)
            sim.estimate(pat, job.r, job.confidence, method=method, psrf_max=job.psrf_max)   # warm-up
            torch.cuda.synchronize()
            a = time.perf_counter()
            res = sim.estimate(pat, job.r, job.confidence, method=method, psrf_max=job.psrf_max)[0]
            torch.cuda.synchronize()
            return time.perf_counter() - a, res

        for par, seq in (("two_state", "sequential"), ("skart", "sequential_skart")):
            t_par, rp = timed(job.chains, par)
            t_seq, rs = timed(1, seq)
            # sample sizes without burn-in: omega n for the parallel methods,
            # N (Alg. 1) or the CI batches' positions (Alg. 2) for the sequential ones
            size_p = job.chains * rp["n"]
            size_s = rs["N"] if seq == "sequential" else rs["n"]
            sp = t_seq / t_par
            row = {"method": par, "n": job.net.n, "chains": job.chains, "r": job.r,
                   "p_parallel": rp["prob"], "p_sequential": rs["prob"],
                   "agree_2r": abs(rp["prob"] - rs["prob"]) < 2 * job.r, "t_parallel_ms": t_par * 1e3,
                   "t_sequential_ms": t_seq * 1e3, "speedup": sp, "speedup_E": sp * size_p / max(size_s, 1),
                   "size_parallel": size_p, "size_sequential": size_s,
                   "status_parallel": rp["status"], "status_sequential": rs["status"]}
            if not no_cpu:
                a = time.perf_counter()
                ro = drivers.solve(ps.to_text(job.net), 1, job.seed, pat, job.r, job.confidence, job.psrf_max,
                                   method=seq, cap=SEQ_LEN, threads=1)[0]
                row["t_sequential_oracle_1thread_ms"] = (time.perf_counter() - a) * 1e3
                row["speedup_vs_oracle_sequential"] = row["t_sequential_oracle_1thread_ms"] / row["t_parallel_ms"]
                # integers identical; the Skart mean sums batch means in another order (1e-12 relative)
                row["oracle_identical"] = (abs(ro["prob"] - rs["prob"]) <= 1e-12 * max(1.0, abs(ro["prob"]))
                                           and ro["n"] == rs["n"] and ro["chain_len"] == rs["chain_len"])
            log("n={} {}: parallel {:.1f} ms, sequential {:.1f} ms".format(job.net.n, par, t_par * 1e3, t_seq * 1e3))
            rows.append(row)
    return {"workload": "sequential (one chain: Alg. 1, Alg. 2) vs parallel (Alg. 4, Alg. 5), r={}, s=0.95".format(
                R_SEQ),
            "pairs": rows, "all_agree_2r": all(r["agree_2r"] for r in rows)}


def isolated_kernel(pkg, torch, jobs, steps: int = 256, chains: int = 65536, target_n: int = 803) -> dict:
    """The dominant kernel alone on the chip: the batched network nearest
    target_n nodes with 65536 chains (1024 blocks, every CU busy), extended on
    one stream, so each launch's event-timed duration is not shared with the
    other lanes' launches as it is in the batched solve."""
    job = min(jobs, key=lambda j: abs(j.net.n - target_n))
    sim = pkg.Simulation(pkg.Network(ps.to_text(job.net)), chains, job.seed, max_props=1, max_len=steps + 64)
    sim.reset(job.patterns)
    sim.run(16)
    sim.sync()
    pkg.profile_enable(True)
    pkg.profile_reset()
    torch.cuda.synchronize()
    a = time.perf_counter()
    sim.run(steps)
    sim.sync()
    t = time.perf_counter() - a
    prof = pkg.profile_read()
    pkg.profile_enable(False)
    r = roofline_of(prof, t, batched=False)
    return {"network_nodes": job.net.n, "chains": chains, "transitions": steps, "kernel": r["kernel"],
            "launches": r["launches"], "avg_launch_ms": r["avg_launch_ms"], "achieved": r["achieved"],
            "frac": r["frac"], "node_updates_per_s": r["kernel_node_updates_per_s"]}


def roofline_of(prof: dict, total_t: float, batched: bool = True) -> dict:
    launches = max(1, prof["launches"])
    avg_launch_s = prof["kernel_ms"] / launches / 1e3
    ops_per_launch = prof["alg_ops"] / launches
    achieved = ops_per_launch / max(avg_launch_s, 1e-12)
    roofline = {"bound": "alu", "achieved": achieved / 1e12, "peak": PEAK_INT32_OPS / 1e12, "unit": "Tops/s",
                "frac": achieved / PEAK_INT32_OPS, "traffic": None,
                # the node-split form when most dispatches used it (latency-bound plain solves)
                "kernel": "k_step_split" if 2 * prof["split_launches"] > prof["launches"] else "k_step_bs",
                "launches": int(prof["launches"]), "split_launches": int(prof["split_launches"]),
                "avg_launch_ms": avg_launch_s * 1e3,
                "alg_ops_per_launch": ops_per_launch,
                "kernel_node_updates_per_s": prof["node_updates"] / max(prof["kernel_ms"] / 1e3, 1e-12),
                "philox_evals_per_s": prof["philox_evals"] / max(prof["kernel_ms"] / 1e3, 1e-12),
                # launches of the lanes overlap: the chip-wide rate over the timed region
                "aggregate_tops": prof["alg_ops"] / total_t / 1e12,
                "aggregate_frac": prof["alg_ops"] / total_t / PEAK_INT32_OPS}
    # counter traffic recorded on the batched workload's k_step_bs dispatches
    tr = os.path.join(ROOT, "profiles", "k_step_bs_traffic.json")
    if batched and roofline["kernel"] == "k_step_bs" and os.path.exists(tr):
        info = json.load(open(tr))
        if info.get("kernel_source_sha") == kernel_sha():
            roofline["traffic"] = info.get("bytes_per_launch")
    return roofline


def cpu_threads() -> int:
    """Host threads for the oracle: every core this process may run on, within
    the host's stated thread budget (OMP_NUM_THREADS, the CPU share of one GPU
    on a shared host) when one is set."""
    cores = len(os.sched_getaffinity(0))
    budget = os.environ.get("OMP_NUM_THREADS", "")
    return max(1, min(cores, int(budget))) if budget.isdigit() else max(1, cores)


def cpu_baseline(jobs, budget_s: float, label: str = "the batched workload"):
    """The oracle's simulator on the host cores: 256-step extensions of every
    chain of each job in turn until the time budget is spent (a single job is
    extended repeatedly)."""
    import oracle
    threads = cpu_threads()
    done_nu, t_used, used, chunks = 0.0, 0.0, 0, 0
    steps = 256
    for j in jobs:
        if t_used >= budget_s:
            break
        ch = oracle.Chains(oracle.Net(ps.to_text(j.net)), j.chains, j.seed, j.patterns, threads=threads)
        used += 1
        while True:
            a = time.perf_counter()
            ch.extend(steps)
            t_used += time.perf_counter() - a
            done_nu += float(steps) * j.chains * j.net.n
            chunks += 1
            if len(jobs) > 1 or t_used >= budget_s or chunks >= 64:
                break
    return dict(value=done_nu / t_used, unit="node-updates/s", cores=threads, kind="oracle",
                nproc=os.cpu_count(), affinity=len(os.sched_getaffinity(0)),
                sample="{} network(s) of {}, all their chains, {} extension(s) of {} recorded steps "
                       "(CPU simulator with indicator recording, {} threads over chains, {:.1f} s)".format(
                           used, label, chunks, steps, threads, t_used))


def main() -> int:
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--count", type=int, default=512)
    ap.add_argument("--plain-sample", type=int, default=0, help="networks of the plain leg (0 = all)")
    ap.add_argument("--serve-seconds", type=float, default=30.0)
    ap.add_argument("--serve-workers", type=int, default=-1,
                    help="processes drawing the serving trace (-1: the host threads; 0: this process, as under a profiler)")
    ap.add_argument("--long-lane-us", type=float, default=0.0,
                    help="server long-request lane threshold in us of kernel time (0 = no long lane)")
    ap.add_argument("--ahead-us", type=float, default=0.0,
                    help="server ahead slice in us of kernel time (0 = none)")
    ap.add_argument("--long-lane-quarters", type=int, default=0,
                    help="CU share of the server's long-request lane in quarters (0 = default)")
    ap.add_argument("--saturate", type=int, default=1000,
                    help="requests of the serving trace queued at once for the capacity figure (0 = skip)")
    ap.add_argument("--serial-seconds", type=float, default=20.0,
                    help="time budget of the serving leg's serial-solve baseline")
    ap.add_argument("--cpu-seconds", type=float, default=12.0)
    ap.add_argument("--no-serve", action="store_true")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-plain", action="store_true")
    ap.add_argument("--no-isolated", action="store_true", help="skip the single-network kernel measurement")
    ap.add_argument("--waves", type=int, default=0, help="bit-sliced waves per block (0 = by n)")
    ap.add_argument("--tune", action="store_true",
                    help="measure the kernel shapes per network size first (untimed) and use them")
    ap.add_argument("--workload", default="batched", choices=["batched", "tiny", "medium", "large", "multiprop", "sequential",
                                                         "isolated"],
                    help="batched (default, the headline) or one plain configuration")
    ap.add_argument("--copy-probe", action="store_true", help="only run a 1 GiB device copy (counter scale)")
    ap.add_argument("--trace-union", nargs=4, metavar=("TRACE_CSV", "KERNEL", "SOLVES", "OUT"),
                    help="busy time of a kernel's dispatches in a rocprofv3 kernel trace, per solve")
    ap.add_argument("--traffic-from", nargs=5, metavar=("FETCH", "WRITE", "COPY_FETCH", "COPY_WRITE", "OUT"),
                    help="turn rocprofv3 FETCH_SIZE/WRITE_SIZE runs into bytes per k_step_bs launch")
    args = ap.parse_args()
    if args.traffic_from:
        return traffic_from(*args.traffic_from)
    if args.trace_union:
        f, k, n, o = args.trace_union
        return trace_union(f, k, int(n), o)
    if args.copy_probe:
        return copy_probe()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) > 1:
        print("bench.py measures one GPU only: this build runs every simulation on a single MI355X "
              "(chains shard by id across GPUs by design, but no multi-GPU path is built)", file=sys.stderr)
        return 2
    import torch
    import paper_1508_07828_amd as pkg
    if not torch.cuda.is_available():
        print("no GPU visible", file=sys.stderr)
        return 1
    torch.cuda.set_device(0)
    pkg.lib()
    if args.waves:
        pkg.set_kernel("bitsliced", args.waves)
    tune = None
    if args.tune:
        log("autotune")
        tune = pkg.autotune()
        for r in tune:
            log("  n={n}: throughput {waves_throughput} waves ({node_updates_per_s:.3e}/s), "
                "latency {waves_latency} waves ({transition_us:.2f} us)".format(**r))
    if args.workload == "sequential":
        print(json.dumps(sequential_workload(pkg, torch, args.cpu_seconds, args.no_cpu)))
        return 0
    if args.workload == "isolated":
        print(json.dumps(isolated_kernel(pkg, torch, ps.batched(args.count))))
        return 0
    if args.workload == "multiprop":
        print(json.dumps(multiprop_workload(pkg, torch, args.steps, args.warmup, args.cpu_seconds, args.no_cpu)))
        return 0
    if args.workload != "batched":
        print(json.dumps(single_workload(pkg, torch, args.workload, args.steps, args.warmup, args.cpu_seconds,
                                         args.no_cpu)))
        return 0

    jobs = ps.batched(args.count)
    log("setting up {} networks".format(len(jobs)))
    nets, sims = make_sims(pkg, jobs)
    torch.cuda.synchronize()

    for w in range(args.warmup):
        log("warmup {}".format(w))
        batched_step(pkg, sims, jobs)
    torch.cuda.synchronize()

    pkg.profile_enable(True)
    pkg.profile_reset()
    times, nus = [], []
    for k in range(args.steps):
        torch.cuda.synchronize()
        a = time.perf_counter()
        res = batched_step(pkg, sims, jobs)
        torch.cuda.synchronize()
        times.append(time.perf_counter() - a)
        nus.append(node_updates_of(sims, jobs))
        log("step {}: {:.3f} s, {:.3e} node-updates".format(k, times[-1], nus[-1]))
    prof = pkg.profile_read()
    pkg.profile_enable(False)
    total_t = sum(times)
    dump = os.environ.get("PBN_BENCH_DUMP")
    if dump:
        with open(dump, "w") as fh:
            json.dump([dict(nodes=j.net.n, chains=j.chains, p=j.net.p, **{k: r[0][k] for k in
                       ("psi_gr", "psi", "n", "N", "M", "chain_len", "prob")}) for j, r in zip(jobs, res)], fh)
    value = sum(nus) / total_t
    nconv = sum(r[0]["status"] != 0 for r in res)

    roofline = roofline_of(prof, total_t)
    if not args.no_isolated:
        # the same kernel without the lanes' concurrency (untimed for the bench value)
        roofline["isolated"] = isolated_kernel(pkg, torch, jobs)
        log("isolated kernel: {:.3f} of the ALU peak".format(roofline["isolated"]["frac"]))

    plain = None
    if not args.no_plain:
        n_plain = len(jobs) if args.plain_sample <= 0 else min(args.plain_sample, len(jobs))
        idx = np.random.default_rng(1).choice(len(jobs), size=n_plain, replace=False)
        sub = [jobs[i] for i in sorted(idx)]
        _, psims = make_sims(pkg, sub)
        # warm every simulation (its workspace, kernels, tables) with one
        # untimed estimate; each estimate restarts the chains from s(0)
        for s, j in zip(psims, sub):
            s.estimate(j.patterns, j.r, j.confidence, psrf_max=1.1)
        torch.cuda.synchronize()
        a = time.perf_counter()
        for s, j in zip(psims, sub):
            s.estimate(j.patterns, j.r, j.confidence, psrf_max=1.1)
        torch.cuda.synchronize()
        tp = time.perf_counter() - a
        nu = node_updates_of(psims, sub)
        plain = {"value": nu / tp, "unit": "node-updates/s", "networks": len(sub), "seconds": tp,
                 "note": "one estimate per network, its own launches and synchronisations per round; "
                         "each simulation warmed by one untimed estimate"}
        del psims
        log("plain: {:.3e} node-updates/s over {} networks".format(plain["value"], len(sub)))

    serving = None
    if not args.no_serve:
        log("serving")
        sched = dict(ahead_us=args.ahead_us, long_lane_us=args.long_lane_us, long_quarters=args.long_lane_quarters)
        serving = run_serving(pkg, torch, args.serve_seconds, 200.0, 16 << 30, args.serial_seconds, sched,
                              None if args.serve_workers < 0 else args.serve_workers)
        serving["schedule"] = sched
        log("serving: p50 {:.1f} ms p99 {:.1f} ms".format(serving["p50_ms"], serving["p99_ms"]))
        if args.saturate > 0:
            log("serving, saturated: {} requests at once".format(args.saturate))
            serving["saturated"] = run_saturated(pkg, args.saturate, 16 << 30)
            log("saturated: {:.1f} queries/s ({:.1f} up to 99% answered)".format(
                serving["saturated"]["queries_per_s"], serving["saturated"]["queries_per_s_99"]))

    cpu = None if args.no_cpu else cpu_baseline(jobs, args.cpu_seconds)

    line = {
        "metric": METRIC, "value": value, "unit": "node-updates/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": total_t / args.steps * 1e3, "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "u32", "data": "synthetic",
        "config": {"workload": "batched: {} random PBNs, n log-uniform 20..2000, 1-3 predictors/node, "
                               "1-5 parents, p in {{1e-3,1e-4}}, 64-1024 chains each; GR R<1.1 then "
                               "two-state r=0.01 s=0.95 on a 2-node state set".format(len(jobs)),
                   "networks": len(jobs), "chains_total": int(sum(j.chains for j in jobs)),
                   "not_converged": int(nconv)},
        "roofline": roofline,
        "plain": plain,
        "batched_vs_plain": (value / plain["value"]) if plain else None,
        "serving": serving,
        "cpu_baseline": cpu,
        "autotune": tune,
    }
    print(json.dumps(line))
    return 0


def kernel_sha() -> str:
    """Hash of the sources the step kernel is compiled from (kernel file and the
    headers it includes), comments and whitespace left out, so recorded counter
    traffic is used only while it still describes the same kernel."""
    import hashlib
    import re
    h = hashlib.sha256()
    for f in ("pbn_step_bs.hip", "pbn_device.h", "pbn_internal.h"):
        text = open(os.path.join(ROOT, "paper_1508_07828_amd", "csrc", f)).read()
        text = re.sub(r"/\*.*?\*/", " ", text, flags=re.S)     # block comments
        text = re.sub(r"//[^\n]*", " ", text)                   # line comments
        h.update(" ".join(text.split()).encode())
    return h.hexdigest()[:16]


def copy_probe(mib: int = 1024, reps: int = 4) -> int:
    """A plain device copy of known size, for scaling the HBM byte counters."""
    import torch
    src = torch.ones(mib << 18, dtype=torch.int32, device="cuda")
    dst = torch.empty_like(src)
    torch.cuda.synchronize()
    for _ in range(reps):
        dst.copy_(src)
    torch.cuda.synchronize()
    print(json.dumps({"copy_bytes_per_launch": mib << 20, "launches": reps}))
    return 0


def trace_union(trace_csv: str, kernel: str, solves: int, out: str) -> int:
    """From a rocprofv3 kernel-trace CSV of a run of `solves` batched solves
    (one warm-up, then the timed ones; no other legs): the wall time with at
    least one `kernel` dispatch in flight, and the summed dispatch time.  The
    solves run one after another with host work between them, so the merged
    busy intervals split into solves at their `solves` - 1 widest gaps; the
    union per timed solve (the warm-up left out) against a solve's algorithmic
    operations gives the chip-wide fraction of the ALU peak, and the summed
    dispatch time over the union the mean number of dispatches in flight (the
    lanes' launches overlap)."""
    import csv
    spans = sorted((int(r["Start_Timestamp"]), int(r["End_Timestamp"]))
                   for r in csv.DictReader(open(trace_csv)) if kernel in r["Kernel_Name"])
    merged = []
    for a, b in spans:
        if merged and a <= merged[-1][1]:
            merged[-1][1] = max(merged[-1][1], b)
        else:
            merged.append([a, b])
    solves = max(1, min(solves, len(merged)))
    gaps = sorted(range(len(merged) - 1), key=lambda i: merged[i + 1][0] - merged[i][1], reverse=True)
    cuts = sorted(gaps[: solves - 1]) + [len(merged) - 1]
    per_solve, lo = [], 0
    for c in cuts:
        group = merged[lo: c + 1]
        g_lo, g_hi = group[0][0], group[-1][1]
        busy = sum(b - a for a, b in group)
        summed = sum(min(b, g_hi) - max(a, g_lo) for a, b in spans if a < g_hi and b > g_lo)
        per_solve.append({"union_ms": busy / 1e6, "first_to_last_ms": (g_hi - g_lo) / 1e6,
                          "summed_dispatch_ms": summed / 1e6})
        lo = c + 1
    timed = per_solve[1:] or per_solve
    union_ns = sum(b - a for a, b in merged)
    summed_ns = sum(b - a for a, b in spans)
    t_union = sum(p["union_ms"] for p in timed) / len(timed)
    t_summed = sum(p["summed_dispatch_ms"] for p in timed) / len(timed)
    info = {"kernel": kernel, "dispatches": len(spans), "solves": solves,
            "union_ms": union_ns / 1e6, "summed_dispatch_ms": summed_ns / 1e6,
            "per_solve": per_solve,
            "timed_union_ms_per_solve": t_union, "timed_summed_ms_per_solve": t_summed,
            "timed_mean_in_flight": t_summed / max(t_union, 1e-9)}
    with open(out, "w") as fh:
        json.dump(info, fh, indent=1)
    print(json.dumps(info))
    return 0


def _counter_sum(csv_dir: str, kernel: str, counter: str):
    import csv
    import glob
    total, n = 0.0, 0
    for f in glob.glob(os.path.join(csv_dir, "**", "*counter_collection.csv"), recursive=True):
        for r in csv.DictReader(open(f)):
            if kernel in r["Kernel_Name"] and r["Counter_Name"] == counter:
                total += float(r["Counter_Value"])
                n += 1
    return total, n


def traffic_from(fetch_dir: str, write_dir: str, copy_fetch_dir: str, copy_write_dir: str, out: str) -> int:
    """HBM bytes per k_step_bs launch from FETCH_SIZE / WRITE_SIZE runs (KiB per
    dispatch), each scaled so that the plain copy reads and writes its size."""
    f_k, n_kf = _counter_sum(fetch_dir, "k_step_bs", "FETCH_SIZE")
    w_k, n_kw = _counter_sum(write_dir, "k_step_bs", "WRITE_SIZE")
    # the probe's copies only: the fill that makes its source reads nothing
    f_c, n_cf = _counter_sum(copy_fetch_dir, "copyBuffer", "FETCH_SIZE")
    w_c, n_cw = _counter_sum(copy_write_dir, "copyBuffer", "WRITE_SIZE")
    copy_bytes = float(1024 << 20)
    f_scale = copy_bytes / (f_c / n_cf * 1024.0)
    w_scale = copy_bytes / (w_c / n_cw * 1024.0)
    fetch = f_k / n_kf * 1024.0 * f_scale
    write = w_k / n_kw * 1024.0 * w_scale
    info = {"kernel": "k_step_bs", "kernel_source_sha": kernel_sha(), "dispatches": n_kf,
            "fetch_bytes_per_launch": fetch, "write_bytes_per_launch": write,
            "bytes_per_launch": fetch + write, "fetch_scale": f_scale, "write_scale": w_scale}
    with open(out, "w") as fh:
        json.dump(info, fh, indent=1)
    print(json.dumps(info))
    return 0


if __name__ == "__main__":
    sys.exit(main())
