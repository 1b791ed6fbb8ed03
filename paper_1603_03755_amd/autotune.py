"""Tunes the launch shape of the benchmark's batches (Metropolis and Wolff moves)
with sqa_autotune and records the choices in a tuning cache file.

    python -m paper_1603_03755_amd.autotune --out <path>

sqa_autotune times every candidate (waves per workgroup in {2, 4, 8}, workgroups
per compute unit from half to full occupancy) on short runs of the real batch
and keeps the fastest; the cache maps "<arch>/<shape class>" to the choice.
Copy the written file to paper_1603_03755_amd/autotune_gfx950.json to make it
the package default.
"""
from __future__ import annotations

import argparse
import json
import os


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--out", required=True, help="cache file to write (existing entries are kept)")
    ap.add_argument("--instances", type=int, default=512)
    ap.add_argument("--sweeps", type=int, default=10_000)
    args = ap.parse_args()
    import torch
    assert torch.cuda.is_available(), "needs a GPU"
    from . import sqa
    from .workloads import batch_jobs
    jobs = batch_jobs(count=args.instances, sweeps=args.sweeps)
    out = {}
    for move, name in ((sqa.SQA_MOVE_METROPOLIS, "metropolis"), (sqa.SQA_MOVE_WOLFF, "wolff")):
        hs = [sqa.SQA(j.kind, j.J, j.penalty, j.beta, j.slices, j.sweeps, j.replicas, j.gamma0, j.gamma1, j.seed,
                      move=move) for j in jobs]
        out[name] = sqa.sqa_autotune(hs, os.path.abspath(args.out))
        print(f"{name}: waves_per_group, groups_per_cu = {out[name]}", flush=True)
        for h in hs:
            h.close()
    print(json.dumps(out))


if __name__ == "__main__":
    main()
