"""GPU parity at the measured workloads' own sizes.

* Parallel tempering at its full shape (Appendix B): all 256 ladders of the
  benchmark (128 N = 24 instances, LHZ and clique-chain ME), 32 temperatures,
  a swap phase after every sweep, 10^5 sweeps, in the one batched launch the
  benchmark times; sampled ladders equal the oracle's.
* Serving at its real job sizes: a slice of the job stream (N 8..32, ME or
  LHZ, L 32 or 64, 16 replicas, >= 10^3 sweeps) plus the largest job (ME
  N = 32, 992 sites, L = 64), through a server whose budget admits only some
  of them at once; every job equals its alone run and the oracle.
* Clique-chain ME at N = 32 (992 sites, L = 64) with both update moves.
* Minimum-weight decoding (Sec. IV A) for N = 25..32, where exhaustive
  oracle search is too slow: planted codewords.  A readout sigma_i sigma_j
  with f < (N-1)/2 pairs flipped has sigma as its unique nearest valid state,
  because two distinct logical states (up to the global flip) give parity
  states that differ in k(N-k) >= N-1 pairs.
"""
import os
from concurrent.futures import ThreadPoolExecutor

import numpy as np
import pytest

import oracle as O
from paper_1603_03755_amd.workloads import (LHZ, ME, ANNEAL_SEED_BASE, AnnealJob, pt_jobs, serving_stream,
                                            sk_instance)

pytestmark = pytest.mark.gpu
NTH = min(os.cpu_count() or 1, 16)


@pytest.fixture(scope="module")
def sqa():
    import torch
    assert torch.cuda.is_available()
    from paper_1603_03755_amd import sqa as s
    s.lib()
    return s


def _oracle_pt(j):
    emb = O.Embedding(j.kind, j.J, j.penalty)
    return O.pt_run(emb, O.pt_ladder(j.beta_min, j.beta_max, j.temps), j.sweeps, j.sweeps_per_swap, j.seed)


@pytest.mark.timeout(1200)
def test_pt_full_workload_sampled_ladders(sqa):
    """256 ladders x 32 temperatures, swap after every sweep, 10^5 sweeps, one batched
    launch; the LHZ (276 sites) and ME (552 sites) ladders of the first and the last
    instance equal the oracle's: spins and energies by slot, slot map, swap counts."""
    jobs = pt_jobs()
    assert len(jobs) == 256 and all(j.sweeps == 100_000 and j.temps == 32 for j in jobs)
    sample = [0, 1, len(jobs) - 2, len(jobs) - 1]
    print(f"PT full workload: oracle on ladders {sample} in threads, 256 ladders on the GPU", flush=True)
    with ThreadPoolExecutor(max_workers=len(sample)) as ex:
        futs = {i: ex.submit(_oracle_pt, jobs[i]) for i in sample}
        hs = [sqa.PT(j.kind, j.J, j.penalty, j.beta_min, j.beta_max, j.temps, j.sweeps, j.sweeps_per_swap, j.seed)
              for j in jobs]
        sqa.pt_run_batch(hs)
        dev = {i: hs[i].read() for i in sample}
        for h in hs:
            h.close()
        print("PT full workload: GPU done, waiting for the oracle", flush=True)
        for i in sample:
            spins, E, rep, acc = dev[i]
            ospins, oE, orep, oacc = futs[i].result()
            assert (rep == orep).all(), i
            assert (spins == ospins[orep]).all(), i
            assert (E == oE[orep]).all(), i
            assert (acc == oacc).all(), i
            assert acc.sum() > 0


def _serving_jobs():
    jobs = [j for _, j in serving_stream(count=10, rate_per_s=1.0, sweeps_range=(1000, 2000))]
    jobs.append(AnnealJob(ME, 32, sk_instance(32, 4242), -2, 10.0, 64, 1000, 16, 3.0, 0.01,
                          ANNEAL_SEED_BASE + 0x2FFFFF))
    return jobs


@pytest.mark.timeout(1200)
def test_serving_stream_real_sizes_alone_mix_oracle(sqa):
    """Jobs of the serving workload's sizes through a server that can hold only a few of
    them: each result equals the same job run alone and the oracle's."""
    jobs = _serving_jobs()
    assert max(j.n for j in jobs) == 32 and any(j.kind == ME and j.n == 32 and j.slices == 64 for j in jobs)
    assert min(j.sweeps for j in jobs) >= 1000 and all(j.replicas == 16 for j in jobs)
    print("serving at real sizes: " + ", ".join(f"{'ME' if j.kind == ME else 'LHZ'}{j.n}/L{j.slices}/{j.sweeps}"
                                              for j in jobs), flush=True)
    with ThreadPoolExecutor(max_workers=4) as ex:
        refs = [ex.submit(O.sqa_anneal, j.kind, j.J, j.penalty, j.beta, j.slices, j.sweeps, j.replicas, j.gamma0,
                          j.gamma1, j.seed, nthreads=max(1, NTH // 4)) for j in jobs]
        budget = 3 << 20
        srv = sqa.Server(hbm_budget_bytes=budget, max_slots=8, chunk_sweeps=250)
        tickets = [srv.submit(j.kind, j.J, j.penalty, j.beta, j.slices, j.sweeps, j.replicas, j.gamma0, j.gamma1,
                              j.seed) for j in jobs]
        served = []
        for t in tickets:
            srv.wait(t, 600_000)
            served.append(srv.result(t))
        completed, launches, peak = srv.stats()
        srv.close()
        assert completed == len(jobs)
        assert launches > max(j.sweeps for j in jobs) // 250       # the jobs did not all run side by side
        print(f"served {completed} jobs in {launches} launches, peak resident {peak} bytes", flush=True)
        for q, (j, (spins, E, lat), ref) in enumerate(zip(jobs, served, refs)):
            alone = sqa.SQA(j.kind, j.J, j.penalty, j.beta, j.slices, j.sweeps, j.replicas, j.gamma0, j.gamma1,
                            j.seed).anneal()
            assert (spins == alone.spins()).all() and (E == alone.energies()).all(), q
            alone.close()
            _, _, ospins, oE = ref.result()
            assert (spins == ospins).all() and (E == oE).all(), q


@pytest.mark.parametrize("move", [0, 1])
def test_me_n32_clique_chains(sqa, move):
    """Clique-chain ME at N = 32 (chains of 31, 992 sites), L = 64: alone and in a
    batch beside a small LHZ handle, identical to the oracle."""
    J = sk_instance(32, 3232)
    R, M = 4, 240
    print(f"ME N=32 move={move}", flush=True)
    h = sqa.SQA(ME, J, -2, 10.0, 64, M, R, 3.0, 0.01, 0x3232 + move, move=move).anneal()
    other = sqa.SQA(LHZ, sk_instance(9, 99), -2, 10.0, 64, M, 8, 3.0, 0.01, 0x99, move=move)
    h2 = sqa.SQA(ME, J, -2, 10.0, 64, M, R, 3.0, 0.01, 0x3232 + move, move=move)
    sqa.sqa_anneal_batch([h2, other])
    if move == 0:
        _, _, ospins, oE = O.sqa_anneal(ME, J, -2, 10.0, 64, M, R, 3.0, 0.01, 0x3232 + move, nthreads=R)
    else:
        _, _, ospins, oE = O.sqa_anneal_wolff(ME, J, -2, 10.0, 64, M, R, 3.0, 0.01, 0x3232 + move, nthreads=R)
    assert h.sites == 992
    for x in (h, h2):
        assert (x.spins() == ospins).all()
        assert (x.energies() == oE).all()
    # the decoded chains are the oracle's majority votes
    q, E = h.decode(sqa.SQA_DEC_ME_MAJORITY, 5)
    emb = O.Embedding(ME, J, -2)
    for r in range(R):
        oq = O.me_majority(emb, ospins[r, 5])
        assert (q[r] == oq).all() and E[r] == O.logical_energy(J, oq)


@pytest.mark.parametrize("N", [25, 27, 30, 32])
def test_mwd_planted_codewords_large_n(sqa, N):
    """MWD for N = 25..32 recovers a planted logical state from its parity readout with
    0, 1 and floor((N-2)/2) pairs flipped (always fewer than half the minimum distance
    N - 1 between valid states)."""
    print(f"mwd planted N={N}", flush=True)
    rng = np.random.default_rng(2500 + N)
    R, L = 6, 2
    J = sk_instance(N, 900 + N)
    h = sqa.SQA(LHZ, J, -2, 5.0, L, 4, R, 3.0, 0.05, 5)
    h.anneal()
    K = N * (N - 1) // 2
    iu = np.triu_indices(N, 1)           # row-major i < j: the LHZ site order k(i, j)
    sig = np.where(rng.random((R, N)) < 0.5, -1, 1).astype(np.int8)
    sig[:, 0] = 1
    flips = [0, 1, (N - 2) // 2, (N - 2) // 2, 1, (N - 2) // 2]
    spins = np.ones((R, L, K), dtype=np.int8)
    for r in range(R):
        s = (sig[r][iu[0]] * sig[r][iu[1]]).astype(np.int8)
        pos = rng.choice(K, size=flips[r], replace=False)
        s[pos] = -s[pos]
        spins[r, 1] = s
        spins[r, 0] = np.where(rng.random(K) < 0.5, -1, 1)
    h.write_spins(spins)
    logical, E = h.decode(sqa.SQA_DEC_LHZ_MWD, 1)
    for r in range(R):
        assert (logical[r] == sig[r]).all(), (N, r, flips[r])
        assert E[r] == O.logical_energy(J, sig[r])
