#!/usr/bin/env python3
"""Throughput benchmark of the batched SQA path on one MI355X.

Workload (one step): 512 synthetic SK instances (J_ij = +-1, h = 0), instance
i embedded as ME (even i) or LHZ (odd i) with N = 12, 16, 20, 24 in turn, 64
replicas each, L = 64 Trotter slices, 10^4 sweeps, beta = 10, Gamma linear
3 -> 0.01, penalty -2.  A step is the whole hot path on the device: lattice
initialisation, all sweeps, per-slice energies (one persistent launch replayed
from a HIP graph) and majority-vote decoding of the ME replicas.  Inputs
(tables, site records) are resident in HBM before timing starts.

Prints one JSON line.  Also reports the same instances launched one per
instance (at a reduced sweep count, both ways), serving latency percentiles on
a short Poisson job stream, the roofline of the sweep kernel and the CPU
oracle on a bounded sample of the workload.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

PEAK_INT32_OPS = 256 * 64 * 2.4e9      # VALU lane-ops/s: 256 CUs x 64 lanes x 2.4 GHz
PHILOX_OPS_PER_WORD = 25.0             # 10 rounds x (4 multiply halves + 4 xor + 2 key adds) / 4 words
DECISION_OPS = 6.0                     # time-neighbour sum (2), table index (2), compare (1), flip (1)


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--instances", type=int, default=512)
    ap.add_argument("--sweeps", type=int, default=10_000)
    ap.add_argument("--no-extras", action="store_true", help="only the timed batched steps")
    ap.add_argument("--cpu-seconds", type=float, default=15.0)
    return ap.parse_args()


def algorithmic_ops_per_attempt(jobs, O) -> float:
    """Method arithmetic per attempt averaged over the workload's sites: the
    Philox share, one product and one accumulate per partner spin of each
    incident term (plus the site field), and the Metropolis decision."""
    tot_ops, tot_w = 0.0, 0.0
    seen = {}
    for j in jobs:
        key = (j.kind, j.n)
        if key not in seen:
            emb = O.Embedding(j.kind, j.J, j.penalty)
            partners = np.zeros(emb.n_sites)
            for t in range(emb.n_terms):
                for k in emb.tsite[t][:emb.arity[t]]:
                    partners[k] += emb.arity[t] - 1
            fields = (emb.h != 0).astype(float)
            seen[key] = float(np.mean(PHILOX_OPS_PER_WORD + 2 * partners + 2 * fields + DECISION_OPS))
        w = j.sites * j.slices * j.replicas * j.sweeps
        tot_ops += seen[key] * w
        tot_w += w
    return tot_ops / tot_w


def cpu_baseline(jobs, seconds: float):
    """The oracle on a stratified sample: for every (embedding, N) stratum one
    instance, 2 replicas, a sweep count sized to about `seconds` of total CPU work."""
    import oracle as O
    cores = min(os.cpu_count() or 1, 16)
    strata = {}
    for j in jobs:
        strata.setdefault((j.kind, j.n), j)
    sample = list(strata.values())
    # calibrate on the smallest stratum
    probe = min(sample, key=lambda j: j.sites)
    t0 = time.perf_counter()
    O.sqa_anneal(probe.kind, probe.J, probe.penalty, probe.beta, probe.slices, 20, 2, probe.gamma0,
                 probe.gamma1, probe.seed, nthreads=2)
    rate1 = probe.sites * probe.slices * 2 * 20 / max(time.perf_counter() - t0, 1e-6)
    per_sweep = sum(j.sites * j.slices * 2 for j in sample)
    sweeps = int(max(5, min(2000, seconds * rate1 * min(cores, 2 * len(sample)) / 2 / per_sweep)))
    t0 = time.perf_counter()
    attempts = 0
    # replicas of all strata spread over the cores: run strata concurrently via threads in C
    from concurrent.futures import ThreadPoolExecutor

    def run(j):
        O.sqa_anneal(j.kind, j.J, j.penalty, j.beta, j.slices, sweeps, 2, j.gamma0, j.gamma1, j.seed,
                     nthreads=2)
        return j.sites * j.slices * 2 * sweeps

    with ThreadPoolExecutor(max_workers=max(1, cores // 2)) as ex:
        for a in ex.map(run, sample):
            attempts += a
    dt = time.perf_counter() - t0
    return {"value": attempts / dt, "unit": "spin-flip attempts/s", "cores": min(cores, 2 * len(sample)),
            "kind": "oracle",
            "sample": f"{len(sample)} instances (one per embedding x N stratum), 2 replicas each, L=64, "
                      f"{sweeps} sweeps of the 10^4-sweep schedule's table prefix; {attempts:.3e} attempts in "
                      f"{dt:.1f} s"}


def main():
    args = parse()
    if args.gpus != 1:
        print(f"bench.py measures one GPU only; --gpus {args.gpus} is not supported (instances and replicas are "
              f"independent, see DESIGN.md for how the batch would shard).", file=sys.stderr)
        sys.exit(2)
    import torch

    assert torch.cuda.is_available(), "needs a GPU"
    torch.cuda.set_device(0)
    import oracle as O
    from paper_1603_03755_amd import sqa
    from paper_1603_03755_amd.workloads import LHZ, ME, batch_jobs, serving_stream

    jobs = batch_jobs(count=args.instances, sweeps=args.sweeps)
    t_setup = time.perf_counter()
    handles = [sqa.SQA(j.kind, j.J, j.penalty, j.beta, j.slices, j.sweeps, j.replicas, j.gamma0, j.gamma1, j.seed)
               for j in jobs]
    batch = sqa.Batch(handles)
    waves, gpc = batch.config()
    setup_s = time.perf_counter() - t_setup
    attempts_per_step = sum(j.attempts for j in jobs)
    me_handles = [h for h, j in zip(handles, jobs) if j.kind == ME]

    stream = torch.cuda.Stream()
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(4)]

    def step(timed_kernel):
        with torch.cuda.stream(stream):
            if timed_kernel:
                ev[0].record(stream)
            batch.run(stream)
            if timed_kernel:
                ev[1].record(stream)
        stream.synchronize()
        for h in me_handles:
            h.decode(sqa.SQA_DEC_ME_MAJORITY, 0)

    for _ in range(args.warmup):
        step(False)
    torch.cuda.synchronize()
    kernel_ms = []
    t0 = time.perf_counter()
    for _ in range(args.steps):
        step(True)
        kernel_ms.append(ev[0].elapsed_time(ev[1]))
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    value = attempts_per_step * args.steps / wall
    kernel_s = float(np.mean(kernel_ms)) / 1e3

    ops = algorithmic_ops_per_attempt(jobs, O)
    achieved = ops * attempts_per_step / kernel_s
    out = {
        "metric": "spin-flip attempts/s (batched vs per-instance launch) + p50/p99 anneal latency",
        "value": value,
        "unit": "spin-flip attempts/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": wall / args.steps * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "int8 spins / int32 energies / uint32 Philox thresholds",
        "data": "synthetic: seeded SK instances J=+-1 standing in for the paper's K8/K16 sets",
        "config": {"workload": f"batched SQA, {args.instances} instances N in {{12,16,20,24}}, half ME half LHZ, "
                               f"64 replicas, L=64, {args.sweeps} sweeps, beta=10, Gamma 3->0.01, penalty -2",
                   "attempts_per_step": attempts_per_step, "launch": {"waves_per_group": waves,
                                                                      "groups_per_cu": gpc},
                   "parallelism": "single GPU, one persistent launch"},
        "roofline": {"bound": "alu", "achieved": achieved / 1e12, "peak": PEAK_INT32_OPS / 1e12,
                     "unit": "TOP/s (int32 VALU lane-ops)", "frac": achieved / PEAK_INT32_OPS,
                     "traffic": None, "kernel": "sqa_anneal_kernel", "kernel_ms": kernel_s * 1e3,
                     "ops_per_attempt": ops},
        "kernel_attempts_per_s": attempts_per_step / kernel_s,
        "setup_s": setup_s,
    }
    if not args.no_extras:
        # one launch per instance vs one batched launch, same instances, reduced sweeps
        short = 200
        hs2 = [sqa.SQA(j.kind, j.J, j.penalty, j.beta, j.slices, short, j.replicas, j.gamma0, j.gamma1, j.seed)
               for j in jobs]
        b2 = sqa.Batch(hs2)
        b2.run(stream)
        stream.synchronize()
        t0 = time.perf_counter()
        b2.run(stream)
        stream.synchronize()
        t_batch = time.perf_counter() - t0
        t0 = time.perf_counter()
        for h in hs2:
            h.anneal(stream)
        stream.synchronize()
        t_single = time.perf_counter() - t0
        att2 = sum(j.sites * j.slices * j.replicas * short for j in jobs)
        out["batched_vs_per_instance"] = {"sweeps": short, "batched_attempts_per_s": att2 / t_batch,
                                          "per_instance_attempts_per_s": att2 / t_single,
                                          "speedup": t_single / t_batch}
        b2.close()
        for h in hs2:
            h.close()
        # serving: a Poisson stream of mixed jobs through the continuous-batching server
        stream_jobs = serving_stream(count=48, rate_per_s=12.0)
        srv = sqa.Server(hbm_budget_bytes=64 << 20, max_slots=32, chunk_sweeps=500)
        t0 = time.perf_counter()
        tickets = []
        for arr, j in stream_jobs:
            now = time.perf_counter() - t0
            if arr > now:
                time.sleep(arr - now)
            tickets.append((srv.submit(j.kind, j.J, j.penalty, j.beta, j.slices, j.sweeps, j.replicas, j.gamma0,
                                       j.gamma1, j.seed), j))
        lats, att3 = [], 0
        for t, j in tickets:
            srv.wait(t)
            _, _, lat = srv.result(t)
            lats.append(lat)
            att3 += j.attempts
        span = time.perf_counter() - t0
        completed, launches, peak = srv.stats()
        srv.close()
        out["serving"] = {"jobs": len(tickets), "p50_latency_s": float(np.percentile(lats, 50)),
                          "p99_latency_s": float(np.percentile(lats, 99)), "jobs_per_s": len(tickets) / span,
                          "attempts_per_s": att3 / span, "launches": launches, "peak_resident_bytes": peak,
                          "budget_bytes": 64 << 20, "arrival_rate_per_s": 12.0}
        out["cpu_baseline"] = cpu_baseline(jobs, args.cpu_seconds)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
