#!/usr/bin/env python3
"""Throughput benchmark of the batched SQA path on one MI355X.

Workload (one step): 512 synthetic SK instances (J_ij = +-1, h = 0), instance
i embedded as ME (even i) or LHZ (odd i) with N = 12, 16, 20, 24 in turn, 64
replicas each, L = 64 Trotter slices, 10^4 sweeps, beta = 10, Gamma linear
3 -> 0.01, penalty -2.  A step is the whole hot path on the device: lattice
initialisation, all sweeps, per-slice energies (one persistent launch replayed
from a HIP graph), then decoding of every replica's slice 0 on the device:
majority vote of the ME chains and exhaustive minimum-weight decoding of the
LHZ states.  Inputs (tables, site records) are resident in HBM before timing
starts.

Prints one JSON line.  Also reports the same instances launched one per
instance (at a reduced sweep count, both ways), serving latency percentiles on
a short Poisson job stream, parallel tempering, the same batch with the
paper's time-like Wolff cluster moves, each LHZ decoder alone, the penalty
scans, the roofline of the sweep kernels and the CPU oracle on a bounded
sample of the workload.

`--copy-calibration` instead runs only a cold 2 GiB device-to-device copy, the
reference for scaling the FETCH_SIZE / WRITE_SIZE counters to bytes;
`--valu-calibration` measures the issue rate of the three VALU instruction
kinds the sweep loops are built from (three-input XOR, widening multiply-add,
packed 16-bit multiply-add) against the integer-ALU peak used by the roofline.
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

# Integer VALU peak in 32-bit lane-op slots: 256 CUs x 4 SIMDs x 16 lanes x 2.4 GHz =
# 39.3e12/s, one wave64 instruction per SIMD every 4 clocks.  (The fp32 vector rate of
# 157.3 TFLOP/s is this x 2 flops per FMA x 2 for packed FP32, which 32-bit integer
# code has no form of.)  `--valu-calibration` measures the instruction kinds of the
# sweep loops at this issue rate, the widening multiply included.
PEAK_LANE_OPS = 256 * 64 * 2.4e9
# Philox4x32-10 per call: 10 rounds x (2 widening 32x32 multiplies, one full-rate slot
# each on gfx950, + 2 three-input XORs).  An attempt (a Wolff bond) consumes one 16-bit
# half of a word, i.e. 1/8 of a call; the second call that supplies the low halves is
# drawn only on a tie of the high half with the threshold (probability 2^-16 each).
PHILOX_OPS_PER_CALL = 10 * (2 + 2)
PHILOX_OPS_PER_HALF = PHILOX_OPS_PER_CALL / 8
DECISION_OPS = 4.0   # compare, tie test and select of the Metropolis test, time-neighbour term, table index
# Wolff moves, per site-slice: bond test (equality, compare, select) and the masked cluster sum;
# per site and sweep, amortised over the L slices: one Philox call (seed slice and acceptance
# words), the run search on the ring and the acceptance decision.
WOLFF_BOND_OPS = 4.0
WOLFF_SITE_OPS = PHILOX_OPS_PER_CALL + 24.0

# HBM bytes of one launch of the sweep kernel on this workload, from rocprofv3 --pmc FETCH_SIZE and
# WRITE_SIZE passes (KiB per dispatch) scaled by the same counters on a cold 2 GiB copy
# (profiles/sqa_anneal_kernel_batched512_L64.md).  Valid only for the kernel sources it was taken on.
TRAFFIC_PROFILE = {"kernel_sha256_prefix": "f0ebdb131c2a1443", "instances": 512, "sweeps": 10_000,
                   "fetch_kib": 1087481.5, "write_kib": 509217.6, "fetch_scale": 2.0, "write_scale": 1.0,
                   "wolff_fetch_kib": 29838.2, "wolff_write_kib": 509208.0}


# Sources the sweep kernels are compiled from; the traffic figures hold for one hash of them.
KERNEL_SOURCES = ("sqa_kernels.hip", "sqa_sweep.h", "device_common.h", "device_types.h")


def kernel_sources_sha256() -> str:
    import hashlib
    h = hashlib.sha256()
    for name in KERNEL_SOURCES:
        h.update(open(os.path.join(ROOT, "paper_1603_03755_amd", "csrc", name), "rb").read())
    return h.hexdigest()


def measured_traffic(args, wolff=False):
    sha = kernel_sources_sha256()
    t = TRAFFIC_PROFILE
    if not sha.startswith(t["kernel_sha256_prefix"]) or args.instances != t["instances"] or args.sweeps != t["sweeps"]:
        return None
    f, w = (t["wolff_fetch_kib"], t["wolff_write_kib"]) if wolff else (t["fetch_kib"], t["write_kib"])
    return (f * t["fetch_scale"] + w * t["write_scale"]) * 1024


def log(msg: str):
    """Progress on stderr (the JSON result line is the only stdout output)."""
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--instances", type=int, default=512)
    ap.add_argument("--sweeps", type=int, default=10_000)
    ap.add_argument("--no-extras", action="store_true", help="only the timed batched steps")
    ap.add_argument("--valu-calibration", action="store_true",
                    help="only measure the VALU issue rate of the sweep loops' instruction kinds")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="only copy 2 GiB device to device, source evicted from the last-level cache first")
    ap.add_argument("--legs", default="single,per_instance,serving,pt,wolff,decoders,scan,ptscan,cpu",
                    help="comma list of the extra legs to run after the timed steps")
    ap.add_argument("--pt-sweeps", type=int, default=100_000, help="sweeps of the parallel-tempering leg")
    return ap.parse_args()


def algorithmic_ops_per_attempt(jobs, O) -> float:
    """Method arithmetic per attempt (full-rate lane-op slots), averaged over the
    workload's sites: the Philox share of the random half word, one multiply-add per
    incident term and per nonzero field in the local field, and the decision."""
    tot_ops, tot_w = 0.0, 0.0
    seen = {}
    for j in jobs:
        key = (j.kind, j.n)
        if key not in seen:
            emb = O.Embedding(j.kind, j.J, j.penalty)
            terms = np.diff(emb.row).astype(float)
            fields = (emb.h != 0).astype(float)
            seen[key] = float(np.mean(PHILOX_OPS_PER_HALF + terms + fields + DECISION_OPS))
        w = j.sites * j.slices * j.replicas * j.sweeps
        tot_ops += seen[key] * w
        tot_w += w
    return tot_ops / tot_w


def wolff_ops_per_site_slice(jobs, O) -> float:
    """Method arithmetic of a Wolff sweep per site-slice (full-rate lane-op slots): the
    Philox share of the bond's random half word, the local-field terms, the bond test and cluster sum,
    and the per-site work spread over the ring."""
    tot_ops, tot_w = 0.0, 0.0
    seen = {}
    for j in jobs:
        key = (j.kind, j.n)
        if key not in seen:
            emb = O.Embedding(j.kind, j.J, j.penalty)
            terms = np.diff(emb.row).astype(float)
            fields = (emb.h != 0).astype(float)
            seen[key] = float(np.mean(PHILOX_OPS_PER_HALF + terms + fields + WOLFF_BOND_OPS
                                      + WOLFF_SITE_OPS / j.slices))
        w = j.sites * j.slices * j.replicas * j.sweeps
        tot_ops += seen[key] * w
        tot_w += w
    return tot_ops / tot_w


def wolff_leg(sqa, O, jobs, stream, metropolis_kernel_s, traffic):
    """The same batch with the paper's move (one time-like Wolff cluster per site and
    sweep) in one persistent launch replayed from its graph; kernel time from events on
    the launch stream; the oracle on one replica lattice per stratum beside it."""
    import torch
    from concurrent.futures import ThreadPoolExecutor
    hs = [sqa.SQA(j.kind, j.J, j.penalty, j.beta, j.slices, j.sweeps, j.replicas, j.gamma0, j.gamma1, j.seed,
                  move=sqa.SQA_MOVE_WOLFF) for j in jobs]
    b = sqa.Batch(hs)
    waves, gpc = b.config()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    b.run(stream)
    stream.synchronize()
    with torch.cuda.stream(stream):
        e0.record(stream)
        b.run(stream)
        e1.record(stream)
    stream.synchronize()
    kernel_s = e0.elapsed_time(e1) / 1e3
    moves = sum(j.sites * j.replicas * j.sweeps for j in jobs)
    cells = sum(j.sites * j.slices * j.replicas * j.sweeps for j in jobs)
    ops = wolff_ops_per_site_slice(jobs, O)
    b.close()
    for h in hs:
        h.close()
    threads = oracle_threads()
    sample = stratified_lattices(jobs, threads)

    def run(jr):
        j, r = jr
        O.sqa_anneal_wolff(j.kind, j.J, j.penalty, j.beta, j.slices, j.sweeps, 1, j.gamma0, j.gamma1, j.seed,
                           nthreads=1, r0=r)
        return j.sites * j.slices * j.sweeps

    t0 = time.perf_counter()
    with ThreadPoolExecutor(max_workers=threads) as ex:
        ocells = sum(ex.map(run, sample))
    odt = time.perf_counter() - t0
    return {"kernel": "sqa_anneal_kernel<Wolff>", "kernel_ms": kernel_s * 1e3,
            "cluster_moves_per_s": moves / kernel_s, "site_slices_per_s": cells / kernel_s,
            "launch": {"waves_per_group": waves, "groups_per_cu": gpc},
            "vs_metropolis_sweep_time": metropolis_kernel_s / kernel_s,
            "roofline": {"bound": "alu", "achieved": ops * cells / kernel_s / 1e12, "peak": PEAK_LANE_OPS / 1e12,
                         "unit": "TOP/s (32-bit VALU lane-op slots)", "frac": ops * cells / kernel_s / PEAK_LANE_OPS,
                         "traffic": traffic, "ops_per_site_slice": ops},
            "oracle": {"site_slices_per_s": ocells / odt, "cores": threads,
                       "sample": f"{len(sample)} replica lattices, one per thread, dealt over the embedding x N "
                                 f"strata, full schedule"}}


def scan_leg(sqa):
    """The paper's experiment shape on synthetic K8 instances (J in {+-0.1..+-1}, times 10):
    8 instances x 6 penalty strengths x {ME on Chimera, clique-chain ME, LHZ}, 1000 reads
    each, L = 64, 10^4 sweeps, Wolff moves, one batched launch; p_s from device decoding
    against device ground states."""
    from paper_1603_03755_amd import harness as H
    from paper_1603_03755_amd.workloads import SEED_BATCH
    instances = [H.paper_instance(8, SEED_BATCH + 7000 + i) for i in range(8)]
    penalties = [0.5, 1.0, 1.5, 2.0, 2.5, 3.0]
    t0 = time.perf_counter()
    res = H.penalty_scan(instances, penalties, H.ScanConfig(schemes=("mec", "me", "lhz")))
    total = time.perf_counter() - t0
    summary = {}
    for scheme in res.p_s:
        pen, ps = res.optimal(scheme)
        summary[scheme] = {"p_s_at_optimal_penalty_mean": float(np.mean(ps)),
                           "optimal_penalty_mean": float(np.mean(pen))}
    return {"instances": len(instances), "n": 8, "penalties": penalties, "reads": 1000, "slices": 64,
            "sweeps": 10_000, "move": "wolff", "anneal_seconds": res.seconds_anneal, "total_seconds": total,
            "site_slices_per_s": res.site_slices / res.seconds_anneal, "schemes": summary}


def host_info():
    """The host the oracle is timed on: logical CPUs, those this process may use, CPU
    model, C library."""
    import platform
    model = ""
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    usable = len(os.sched_getaffinity(0)) if hasattr(os, "sched_getaffinity") else (os.cpu_count() or 1)
    return {"nproc": os.cpu_count(), "usable_cpus": usable, "cpu_model": model,
            "libc": " ".join(x for x in platform.libc_ver() if x)}


def oracle_threads() -> int:
    """One oracle thread per usable host CPU, at most 16 (the CPU share of one GPU)."""
    return max(1, min(host_info()["usable_cpus"], 16))


def stratified_lattices(jobs, count):
    """`count` (job, replica) lattices dealt round-robin over the workload's (embedding, N)
    strata: lattice q is replica q // strata of the stratum's first instance."""
    strata = {}
    for j in jobs:
        strata.setdefault((j.kind, j.n), j)
    first = list(strata.values())
    return [(first[q % len(first)], q // len(first)) for q in range(count)]


def pt_scan_leg(sqa, scan):
    """The paper's PT experiment shape (Sec. III, Figs. 5-7, Appendix B) on the scan's 8
    synthetic K8 instances: 6 penalty strengths x {ME on Chimera, clique-chain ME, LHZ},
    32 independent ladders each of 64 temperatures (beta 20 -> 0.1, paper units), 10
    sweeps per swap, 10^4 swaps, all in one batched launch; every ladder's final states
    decoded on the device (chain majority, three-tree majority for LHZ).  Reports p_s at
    beta = 20 and the critical penalty (p_s = 0.5 crossing, Fig. 7) beside the SQA scan's
    optimal penalty (Fig. 5)."""
    from paper_1603_03755_amd import harness as H
    from paper_1603_03755_amd.workloads import SEED_BATCH
    instances = [H.paper_instance(8, SEED_BATCH + 7000 + i) for i in range(8)]
    penalties = [0.5, 1.0, 1.5, 2.0, 2.5, 3.0]
    cfg = H.PTScanConfig(schemes=("mec", "me", "lhz"))
    t0 = time.perf_counter()
    res = H.pt_penalty_scan(instances, penalties, cfg)
    total = time.perf_counter() - t0
    schemes = {}
    for x in cfg.schemes:
        crit = res.critical(x)
        ok = [c for c in crit if c == c]
        schemes[x] = {"p_s_beta20_by_penalty": [float(v) for v in np.mean(res.p_s[x][:, :, 0], axis=0)],
                      "critical_penalty_mean": float(np.mean(ok)) if ok else None,
                      "critical_penalty_found": len(ok)}
        sq = (scan or {}).get("schemes", {}).get("lhz_mvd" if x == "lhz" else x)
        if sq:
            schemes[x]["sqa_optimal_penalty_mean"] = sq["optimal_penalty_mean"]
    return {"instances": len(instances), "n": 8, "penalties": penalties, "runs": cfg.runs, "temps": cfg.temps,
            "beta": [cfg.beta_max, cfg.beta_min], "sweeps_per_swap": cfg.sweeps_per_swap, "swaps": cfg.swaps,
            "pt_seconds": res.seconds_pt, "total_seconds": total, "attempts_per_s": res.attempts / res.seconds_pt,
            "schemes": schemes}


def cpu_baseline(jobs):
    """The oracle, as it stands, on a bounded sample of the same workload: one replica
    lattice per host thread (one thread per usable CPU, at most 16), dealt over the
    (embedding, N) strata, each over the full sweep schedule."""
    import oracle as O
    from concurrent.futures import ThreadPoolExecutor
    threads = oracle_threads()
    lattices = stratified_lattices(jobs, threads)

    def run(jr):
        j, r = jr
        O.sqa_anneal(j.kind, j.J, j.penalty, j.beta, j.slices, j.sweeps, 1, j.gamma0, j.gamma1, j.seed,
                     nthreads=1, r0=r)
        return j.sites * j.slices * j.sweeps

    t0 = time.perf_counter()
    with ThreadPoolExecutor(max_workers=threads) as ex:
        attempts = sum(ex.map(run, lattices))
    dt = time.perf_counter() - t0
    return {"value": attempts / dt, "unit": "spin-flip attempts/s", "cores": threads, "kind": "oracle",
            "host": host_info(),
            "sample": f"{len(lattices)} of the workload's replica lattices, one per thread, dealt over the 8 "
                      f"embedding x N strata, full {jobs[0].sweeps}-sweep schedule: {attempts:.3e} attempts "
                      f"in {dt:.1f} s"}


def serve_run(sqa, stream_jobs, budget, slots, chunk):
    """Pushes (arrival_time, job) pairs through a continuous-batching server; returns
    per-job latencies and totals."""
    srv = sqa.Server(hbm_budget_bytes=budget, max_slots=slots, chunk_sweeps=chunk)
    t0 = time.perf_counter()
    tickets = []
    for arr, j in stream_jobs:
        now = time.perf_counter() - t0
        if arr > now:
            time.sleep(arr - now)
        tickets.append((srv.submit(j.kind, j.J, j.penalty, j.beta, j.slices, j.sweeps, j.replicas, j.gamma0,
                                   j.gamma1, j.seed), j))
    lats, att = [], 0
    for t, j in tickets:
        srv.wait(t)
        _, _, _, _, lat = srv.result(t, logical=True)      # spins, energies, decoded states and their energies
        lats.append(lat)
        att += j.attempts
    span = time.perf_counter() - t0
    completed, launches, peak = srv.stats()
    srv.close()
    return {"jobs": len(tickets), "p50_latency_s": float(np.percentile(lats, 50)),
            "p99_latency_s": float(np.percentile(lats, 99)), "jobs_per_s": len(tickets) / span,
            "attempts_per_s": att / span, "launches": int(launches), "peak_resident_bytes": int(peak)}


def serving_leg(sqa):
    """Continuous batching under a 64 MB device budget and 32 slots, each job decoded on
    the device when it finishes (majority vote for ME, minimum-weight decoding for LHZ)
    and returned with its logical states: capacity from a
    burst of 48 mixed jobs (N 8..32, ME/LHZ, L 32/64, 10^3-10^4 sweeps, 16 replicas),
    then Poisson arrivals of the same jobs at 0.25, 0.5, 0.75 and 0.9 of capacity."""
    from paper_1603_03755_amd.workloads import serving_stream
    budget, slots, chunk, count = 64 << 20, 32, 500, 48
    burst = [(0.0, j) for _, j in serving_stream(count=count, rate_per_s=1.0)]
    cap = serve_run(sqa, burst, budget, slots, chunk)
    capacity = cap["jobs_per_s"]
    rates = []
    for f in (0.25, 0.5, 0.75, 0.9):
        r = serve_run(sqa, serving_stream(count=count, rate_per_s=f * capacity), budget, slots, chunk)
        r.update({"fraction_of_capacity": f, "arrival_rate_per_s": f * capacity})
        rates.append(r)
    head = rates[2]
    import oracle as O
    jobs = [j for _, j in burst]
    ops = algorithmic_ops_per_attempt(jobs, O)
    roof = {"bound": "alu", "achieved": ops * cap["attempts_per_s"] / 1e12, "peak": PEAK_LANE_OPS / 1e12,
            "unit": "TOP/s (32-bit VALU lane-op slots)", "frac": ops * cap["attempts_per_s"] / PEAK_LANE_OPS,
            "traffic": None, "ops_per_attempt": ops,
            "over": "the capacity burst's whole span (admission, launches, decoding, copies to the host)"}
    return {"capacity_jobs_per_s": capacity, "burst": cap, "rates": rates, "roofline": roof,
            "p50_latency_s": head["p50_latency_s"], "p99_latency_s": head["p99_latency_s"],
            "at_fraction_of_capacity": 0.75, "budget_bytes": budget, "slots": slots, "chunk_sweeps": chunk}


def decoders_leg(sqa):
    """The LHZ decoders on the device: minimum-weight (exhaustive over 2^(N-1) logical states),
    maximum-likelihood at the Nishimori temperature of error rate 0.2 (the same walk with a
    weight per state; N <= 24), belief propagation on the weight-3 parity checks (10 rounds, then one
    random spanning tree) and majority over three random spanning trees.  Each at N = 24 with
    64 replicas (the benchmark's largest LHZ handles) and N = 32 with 16 replicas (the serving
    leg's largest), on the readout slice of a short anneal; a decode is queued on a stream and
    timed with HIP events there (median of 5 after one warm-up)."""
    import torch
    from paper_1603_03755_amd.workloads import LHZ, sk_instance
    stream = torch.cuda.Stream()
    out = {}
    for N, R in ((24, 64), (32, 16)):
        h = sqa.SQA(LHZ, sk_instance(N, 1603 + N), -2, 10.0, 64, 50, R, 3.0, 0.01, 0x5EED + N)
        h.anneal(stream)
        stream.synchronize()
        trees1 = sqa.sqa_random_trees(0x7EE + N, N, 1)
        trees3 = sqa.sqa_random_trees(0x7EF + N, N, 3)
        res = {}
        for name, dec, kw in (("mwd", sqa.SQA_DEC_LHZ_MWD, {}),
                              ("mld", sqa.SQA_DEC_LHZ_MLD, {"error_rate": 0.2}),
                              ("bp", sqa.SQA_DEC_LHZ_BP, {"error_rate": 0.2, "iterations": 10, "trees": trees1}),
                              ("trees", sqa.SQA_DEC_LHZ_TREES, {"trees": trees3})):
            if name == "mld" and N > 24:     # the library's exhaustive MLD stops at N = 24
                continue
            ts = []
            for rep in range(6):
                e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
                e0.record(stream)
                h.decode(dec, 0, stream=stream, host=False, **kw)
                e1.record(stream)
                stream.synchronize()
                if rep:
                    ts.append(e0.elapsed_time(e1))
            ms = float(np.median(ts))
            r = {"ms": ms}
            if name in ("mwd", "mld"):
                r["candidates_per_s"] = R * float(2 ** (N - 1)) / (ms / 1e3)
            res[name] = r
        h.close()
        out[f"lhz_n{N}_r{R}"] = res
    return out


def single_leg(sqa):
    """The two single-instance configurations: the N = 8 instance as clique-chain ME (56
    sites) and as LHZ (28 sites), 16 replicas, L = 32, 10^3 sweeps, one handle each; a
    call is sqa_anneal (init, sweeps, energies) on a stream, timed with HIP events there
    and on the host clock around launch and synchronisation; median of 20 calls."""
    import torch
    from paper_1603_03755_amd.workloads import LHZ, ME, single_job
    out = {}
    stream = torch.cuda.Stream()
    for kind, name in ((ME, "me_n8"), (LHZ, "lhz_n8")):
        j = single_job(kind)
        h = sqa.SQA(j.kind, j.J, j.penalty, j.beta, j.slices, j.sweeps, j.replicas, j.gamma0, j.gamma1, j.seed)
        dev_ms, host_ms = [], []
        for rep in range(21):
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            t0 = time.perf_counter()
            e0.record(stream)
            h.anneal(stream)
            e1.record(stream)
            stream.synchronize()
            if rep:                                  # the first call loads code and sets up
                host_ms.append((time.perf_counter() - t0) * 1e3)
                dev_ms.append(e0.elapsed_time(e1))
        h.close()
        med_dev, med_host = float(np.median(dev_ms)), float(np.median(host_ms))
        out[name] = {"sites": j.sites, "attempts": j.attempts, "device_ms": med_dev, "host_ms": med_host,
                     "attempts_per_s": j.attempts / (med_dev / 1e3),
                     "attempts_per_s_incl_launch": j.attempts / (med_host / 1e3)}
    return out


def pt_ops_per_attempt(jobs, O) -> float:
    """Method arithmetic of a PT attempt (full-rate lane-op slots), averaged over the
    ladders' sites: the Philox share of the random half word, one multiply-add per
    incident term and per nonzero field, and the decision (compare, tie test, select,
    table index).  The swap phases are counted apart (per swap attempt, not here)."""
    tot_ops, tot_w, seen = 0.0, 0.0, {}
    for j in jobs:
        key = (j.kind, j.n)
        if key not in seen:
            emb = O.Embedding(j.kind, j.J, j.penalty)
            terms = np.diff(emb.row).astype(float)
            fields = (emb.h != 0).astype(float)
            seen[key] = float(np.mean(PHILOX_OPS_PER_HALF + terms + fields + DECISION_OPS))
        w = j.sites * j.temps * j.sweeps
        tot_ops += seen[key] * w
        tot_w += w
    return tot_ops / tot_w


def pt_leg(sqa, O, sweeps: int):
    """Parallel tempering over 128 N = 24 instances embedded both ways (256 ladders of 32
    temperatures, beta geometric in [0.1, 5], a swap phase after every sweep), one launch;
    its duration from HIP events on the launch stream."""
    import torch
    from paper_1603_03755_amd.workloads import pt_jobs
    jobs = pt_jobs(sweeps=sweeps)
    hs = [sqa.PT(j.kind, j.J, j.penalty, j.beta_min, j.beta_max, j.temps, j.sweeps, j.sweeps_per_swap, j.seed)
          for j in jobs]
    stream = torch.cuda.Stream()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    t0 = time.perf_counter()
    e0.record(stream)
    sqa.pt_run_batch(hs, stream)
    e1.record(stream)
    stream.synchronize()
    wall = time.perf_counter() - t0
    dt = e0.elapsed_time(e1) / 1e3
    attempts = sum(j.sites * j.temps * j.sweeps for j in jobs)
    swaps = sum((j.temps - 1) * (j.sweeps // j.sweeps_per_swap) for j in jobs)
    ops = pt_ops_per_attempt(jobs, O)
    for h in hs:
        h.close()
    return {"kernel": "pt_kernel", "ladders": len(jobs), "temps": 32, "sweeps": sweeps, "attempts": attempts,
            "attempts_per_s": attempts / dt, "swap_attempts_per_s": swaps / dt, "kernel_seconds": dt,
            "wall_seconds": wall, "hbm_yardstick_frac": attempts / dt / 4.0e12,
            "roofline": {"bound": "alu", "achieved": ops * attempts / dt / 1e12, "peak": PEAK_LANE_OPS / 1e12,
                         "unit": "TOP/s (32-bit VALU lane-op slots)", "frac": ops * attempts / dt / PEAK_LANE_OPS,
                         "traffic": None, "ops_per_attempt": ops}}


def copy_calibration():
    import torch
    torch.cuda.set_device(0)
    n = 2 << 30
    a = torch.empty(n, dtype=torch.uint8, device="cuda")
    a.fill_(1)
    junk = torch.empty(1 << 30, dtype=torch.uint8, device="cuda")
    junk.fill_(2)            # 1 GiB written after the source: evicts it from the 256 MB last-level cache
    b = torch.empty_like(a)
    torch.cuda.synchronize()
    b.copy_(a)
    torch.cuda.synchronize()
    print(json.dumps({"copy_calibration_bytes": n}), flush=True)


VALU_CALIB_OPS = {0: "v_bitop3_b32", 1: "v_mad_u64_u32", 2: "v_pk_mad_u16"}


def calib_lib():
    """The VALU issue-rate probe, libsqa_calib.so (built beside libsqa.so; not part of
    the library's interface)."""
    import ctypes as C
    path = os.path.join(ROOT, "paper_1603_03755_amd", "libsqa_calib.so")
    if not os.path.exists(path):
        raise RuntimeError(f"{path} is missing: build it with `python -m paper_1603_03755_amd.build`")
    L = C.CDLL(path)
    L.sqa_calib_valu_issue.restype = C.c_int
    L.sqa_calib_valu_issue.argtypes = [C.c_int32, C.c_int32, C.POINTER(C.c_float), C.POINTER(C.c_double)]
    return L


def valu_issue(op: int, iters: int):
    """(kernel ms, VALU wave-instructions) of one issue-rate launch of instruction kind `op`."""
    import ctypes as C
    ms, instr = C.c_float(), C.c_double()
    rc = calib_lib().sqa_calib_valu_issue(op, iters, C.byref(ms), C.byref(instr))
    if rc != 0:
        raise RuntimeError(f"sqa_calib_valu_issue({op}, {iters}) failed with code {rc}")
    return ms.value, instr.value


def valu_calibration():
    """Issue rate of each instruction kind, in wave-instructions per SIMD per clock at
    2.4 GHz and in 32-bit lane-ops/s, against PEAK_LANE_OPS (0.25 per SIMD per clock)."""
    import torch
    torch.cuda.set_device(0)
    simds = 4 * torch.cuda.get_device_properties(0).multi_processor_count
    out = {}
    for op, name in VALU_CALIB_OPS.items():
        ms, instr = valu_issue(op, 100_000)
        rate = instr / (ms * 1e-3)
        out[name] = {"kernel_ms": ms, "wave_instructions": instr,
                     "per_simd_per_clock_at_2p4GHz": rate / (simds * 2.4e9),
                     "lane_ops_per_s": 64 * rate, "frac_of_peak": 64 * rate / PEAK_LANE_OPS}
    print(json.dumps({"valu_calibration": out, "peak_lane_ops_per_s": PEAK_LANE_OPS, "simds": simds}), flush=True)


def main():
    args = parse()
    if args.copy_calibration:
        copy_calibration()
        return
    if args.valu_calibration:
        valu_calibration()
        return
    if args.gpus != 1:
        print(f"bench.py measures one GPU only; --gpus {args.gpus} is not supported (instances and replicas are "
              f"independent: several GPUs would each take their own share of the batch).", file=sys.stderr)
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
    # one graph per step: init -> sweeps -> energies -> decoding of every replica's slice 0
    # (majority vote of the ME chains, exhaustive minimum-weight decoding of the LHZ states)
    decoders = [(sqa.SQA_DEC_ME_MAJORITY if j.kind == ME else sqa.SQA_DEC_LHZ_MWD, 0) for j in jobs]
    batch = sqa.Batch(handles, decoders=decoders)     # launch shape from the package's tuning cache
    waves, gpc = batch.config()
    setup_s = time.perf_counter() - t_setup
    attempts_per_step = sum(j.attempts for j in jobs)
    log(f"setup {setup_s:.1f} s: {len(handles)} handles, {attempts_per_step:.3e} attempts per step")

    stream = torch.cuda.Stream()

    def step():
        batch.run(stream)
        stream.synchronize()

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    log("warm-up done")
    kernel_ms, decode_ms = [], []
    t0 = time.perf_counter()
    for _ in range(args.steps):
        step()
        a_ms, d_ms = batch.timing()      # HIP events on the launch stream, around and inside the graph
        kernel_ms.append(a_ms)
        decode_ms.append(d_ms)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    value = attempts_per_step * args.steps / wall
    kernel_s = float(np.mean(kernel_ms)) / 1e3
    log(f"timed steps done: {wall / args.steps * 1e3:.1f} ms per step")

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
        "dtype": "int32",
        "dtype_note": "integer path: +-1 spins (int8 in HBM, bits in LDS), int32 fields and energies, "
                      "uint32 Philox words compared with uint32 thresholds",
        "data": "synthetic: seeded SK instances J=+-1 standing in for the paper's K8/K16 sets",
        "config": {"workload": f"batched SQA, {args.instances} instances N in {{12,16,20,24}}, half ME half LHZ, "
                               f"64 replicas, L=64, {args.sweeps} sweeps, beta=10, Gamma 3->0.01, penalty -2",
                   "attempts_per_step": attempts_per_step, "launch": {"waves_per_group": waves,
                                                                      "groups_per_cu": gpc,
                                                                      "tuning_cache": os.path.basename(
                                                                          sqa.TUNING_CACHE)},
                   "parallelism": "single GPU, one persistent launch"},
        "roofline": {"bound": "alu", "achieved": achieved / 1e12, "peak": PEAK_LANE_OPS / 1e12,
                     "unit": "TOP/s (32-bit VALU lane-op slots)", "frac": achieved / PEAK_LANE_OPS,
                     "traffic": measured_traffic(args), "kernel": "sqa_anneal_kernel",
                     "kernel_ms": kernel_s * 1e3, "decode_ms": float(np.mean(decode_ms)),
                     "ops_per_attempt": ops},
        "kernel_attempts_per_s": attempts_per_step / kernel_s,
        # the per-sweep streaming view: 1 byte read + 1 byte written per attempt at 8 TB/s
        "hbm_yardstick": {"bytes_per_attempt": 2, "attempts_per_s_at_peak": 4.0e12,
                          "frac": (attempts_per_step / kernel_s) / 4.0e12},
        "setup_s": setup_s,
    }
    legs = set() if args.no_extras else {x.strip() for x in args.legs.split(",") if x.strip()}
    if "per_instance" in legs:
        log("leg per_instance")
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
    if "single" in legs:
        log("leg single")
        out["single_instance"] = single_leg(sqa)
    if "decoders" in legs:
        log("leg decoders")
        out["decoders"] = decoders_leg(sqa)
    if "serving" in legs:
        log("leg serving")
        out["serving"] = serving_leg(sqa)
    if "pt" in legs:
        log("leg pt")
        out["parallel_tempering"] = pt_leg(sqa, O, args.pt_sweeps)
    if "wolff" in legs:
        log("leg wolff")
        out["wolff"] = wolff_leg(sqa, O, jobs, stream, kernel_s, measured_traffic(args, wolff=True))
    if "scan" in legs:
        log("leg scan")
        out["penalty_scan"] = scan_leg(sqa)
    if "ptscan" in legs:
        log("leg ptscan")
        out["pt_penalty_scan"] = pt_scan_leg(sqa, out.get("penalty_scan"))
    if "cpu" in legs:
        log("leg cpu")
        out["cpu_baseline"] = cpu_baseline(jobs)
    log("done")
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
