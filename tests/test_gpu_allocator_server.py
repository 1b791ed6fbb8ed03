"""Device memory through the caller's allocator, failure paths forced from the
host, and the server's memory budget, decoded results and cancellation.

Every failure here is forced on the host (an allocator that refuses, a launch
that the library is told to report as failed before queueing it), so no
kernel ever faults."""
import os

import numpy as np
import pytest

import oracle as O
from paper_1603_03755_amd.workloads import LHZ, ME, MEC, serving_stream, sk_instance

pytestmark = pytest.mark.gpu
NTH = min(os.cpu_count() or 1, 16)


@pytest.fixture(scope="module")
def sqa():
    import torch
    assert torch.cuda.is_available()
    from paper_1603_03755_amd import sqa as s
    s.lib()
    return s


def _r512(b):
    return (b + 511) // 512 * 512


def test_torch_allocator_holds_the_handle_memory(sqa):
    """A handle built on torch's caching allocator: torch's allocated bytes grow by
    the handle's device bytes (and the decoder scratch when an LHZ decoder runs), the
    results equal a hipMalloc handle's and the oracle's, and closing the handle gives
    every byte back."""
    import torch
    torch.cuda.synchronize()
    base = torch.cuda.memory_allocated()
    a = sqa.TorchAllocator()
    J = sk_instance(9, 31)
    args = (LHZ, J, -2, 6.0, 16, 60, 8, 3.0, 0.05, 0xA110C)
    h = sqa.SQA(*args, allocator=a)
    assert a.calls == 1 and len(a.live) == 1
    assert h.device_bytes() == a.live_bytes
    assert torch.cuda.memory_allocated() - base == _r512(a.live_bytes)
    h.anneal()
    ref = sqa.SQA(*args).anneal()
    assert (h.spins() == ref.spins()).all() and (h.energies() == ref.energies()).all()
    _, _, ospins, oE = O.sqa_anneal(LHZ, J, -2, 6.0, 16, 60, 8, 3.0, 0.05, 0xA110C, nthreads=NTH)
    assert (h.spins() == ospins).all() and (h.energies() == oE).all()
    q, E = h.decode(sqa.SQA_DEC_LHZ_MWD, 2)
    assert len(a.live) == 2                                   # the decoder scratch
    assert h.device_bytes() == a.live_bytes
    assert torch.cuda.memory_allocated() - base == sum(_r512(b) for b in a.live.values())
    q2, E2 = ref.decode(sqa.SQA_DEC_LHZ_MWD, 2)
    assert (q == q2).all() and (E == E2).all()
    h.close()
    ref.close()
    torch.cuda.synchronize()
    assert a.live == {} and torch.cuda.memory_allocated() == base


def test_decoder_scratch_refused_leaves_the_handle_valid(sqa):
    """The allocator refuses the decoder scratch: the decode reports SQA_ERR_OOM and
    the handle keeps its state (spins, energies, decoders that need no scratch)."""
    import torch
    budget = {"n": 1}

    def alloc(nbytes):
        if budget["n"] == 0:
            return None
        budget["n"] -= 1
        return torch.cuda.caching_allocator_alloc(nbytes, 0, torch.cuda.default_stream(0))

    a = sqa.CallbackAllocator(alloc, torch.cuda.caching_allocator_delete)
    J = sk_instance(7, 32)
    h = sqa.SQA(LHZ, J, -2, 6.0, 8, 40, 4, 3.0, 0.05, 77, allocator=a).anneal()
    with pytest.raises(sqa.SqaError) as e:
        h.decode(sqa.SQA_DEC_LHZ_MWD, 0)
    assert e.value.status == sqa.SQA_ERR_OOM
    _, _, ospins, oE = O.sqa_anneal(LHZ, J, -2, 6.0, 8, 40, 4, 3.0, 0.05, 77)
    assert (h.spins() == ospins).all() and (h.energies() == oE).all()
    budget["n"] = 1                                           # memory again: the same call now works
    q, E = h.decode(sqa.SQA_DEC_LHZ_MWD, 0)
    for r in range(4):
        assert (q[r] == O.lhz_mwd(7, ospins[r, 0])).all()
    h.close()
    assert a.live == {}
    budget["n"] = 1
    me = sqa.SQA(ME, J, -2, 6.0, 8, 40, 4, 3.0, 0.05, 78, allocator=a).anneal()
    budget["n"] = 0
    q, E = me.decode(sqa.SQA_DEC_ME_MAJORITY, 1)             # majority vote needs no scratch
    assert q.shape == (4, 7)
    me.close()


def test_injected_launch_fault_poisons_the_handle(sqa, monkeypatch):
    """A launch reported as failed (forced on the host: nothing is queued) poisons the
    handle: later calls on it report SQA_ERR_DEVICE, it can still be destroyed, and
    other handles are unaffected."""
    J = sk_instance(6, 33)
    h = sqa.SQA(ME, J, -2, 6.0, 8, 30, 4, 3.0, 0.05, 5)
    monkeypatch.setenv("SQA_FAULT_INJECT", "launch")
    with pytest.raises(sqa.SqaError) as e:
        h.anneal()
    assert e.value.status == sqa.SQA_ERR_DEVICE
    for call in (h.spins, h.energies, h.anneal, lambda: h.decode(sqa.SQA_DEC_ME_MAJORITY, 0)):
        with pytest.raises(sqa.SqaError) as e:
            call()
        assert e.value.status == sqa.SQA_ERR_DEVICE
    # batches and PT report it too
    b1 = sqa.SQA(ME, J, -2, 6.0, 8, 30, 4, 3.0, 0.05, 6)
    with pytest.raises(sqa.SqaError) as e:
        sqa.sqa_anneal_batch([b1])
    assert e.value.status == sqa.SQA_ERR_DEVICE
    pt = sqa.PT(LHZ, J, -2, 0.2, 3.0, 8, 20, 1, 9)
    with pytest.raises(sqa.SqaError) as e:
        pt.run()
    assert e.value.status == sqa.SQA_ERR_DEVICE
    with pytest.raises(sqa.SqaError):
        pt.run()
    monkeypatch.delenv("SQA_FAULT_INJECT")
    with pytest.raises(sqa.SqaError) as e:
        h.anneal()                                            # still poisoned
    assert e.value.status == sqa.SQA_ERR_DEVICE
    h.close()
    pt.close()
    ok = sqa.SQA(ME, J, -2, 6.0, 8, 30, 4, 3.0, 0.05, 5).anneal()
    _, _, ospins, _ = O.sqa_anneal(ME, J, -2, 6.0, 8, 30, 4, 3.0, 0.05, 5)
    assert (ok.spins() == ospins).all()


def _jobs(count, seed=40_000, sweeps=(300, 700), n_range=(8, 20)):
    return [j for _, j in serving_stream(count=count, rate_per_s=1.0, seed=seed, sweeps_range=sweeps,
                                         n_range=n_range)]


def test_server_budget_is_real_device_memory(sqa):
    """The server on torch's caching allocator, with a budget that admits only a few of
    the jobs at once: torch's peak allocated memory stays within the budget, every job
    equals its alone run (spins, energies and the default decoder's logical states), and
    closing the server frees everything."""
    import torch
    jobs = _jobs(12)
    torch.cuda.synchronize()
    base = torch.cuda.memory_allocated()
    a = sqa.TorchAllocator()
    probe = sqa.Server(1 << 40, 1, 100)
    sizes = []
    for j in jobs:
        t = probe.submit(j.kind, j.J, j.penalty, j.beta, j.slices, j.sweeps, j.replicas, j.gamma0, j.gamma1, j.seed)
        sizes.append(probe.job_bytes(t))
        probe.cancel(t)
    probe.close()
    budget = sum(sorted(sizes)[-3:]) + 4096
    assert budget < sum(sizes)
    torch.cuda.reset_peak_memory_stats()
    srv = sqa.Server(budget, 16, 97, allocator=a)
    tickets = [srv.submit(j.kind, j.J, j.penalty, j.beta, j.slices, j.sweeps, j.replicas, j.gamma0, j.gamma1, j.seed)
               for j in jobs]
    out = []
    for t in tickets:
        srv.wait(t, 300_000)
        out.append(srv.result(t, logical=True))
    completed, launches, peak = srv.stats()
    torch.cuda.synchronize()
    used = torch.cuda.max_memory_allocated() - base
    print(f"budget {budget} B, charged peak {peak} B, torch peak {used} B, {launches} launches", flush=True)
    assert completed == len(jobs) and peak <= budget and used <= budget
    srv.close()
    torch.cuda.synchronize()
    assert a.live == {} and torch.cuda.memory_allocated() == base
    for j, (spins, E, q, qE, lat) in zip(jobs, out):
        alone = sqa.SQA(j.kind, j.J, j.penalty, j.beta, j.slices, j.sweeps, j.replicas, j.gamma0, j.gamma1,
                        j.seed).anneal()
        assert (spins == alone.spins()).all() and (E == alone.energies()).all()
        dec = sqa.SQA_DEC_ME_MAJORITY if j.kind == ME else sqa.SQA_DEC_LHZ_MWD
        aq, aE = alone.decode(dec, 0)
        assert (q == aq).all() and (qE == aE).all()
        alone.close()


def test_server_decoders_chosen_per_job(sqa):
    """Explicit decoders per job (trees, parity-check, maximum-likelihood, majority on
    another slice, ME on Chimera) equal the same decoders on the alone run and the
    oracle's."""
    trees = sqa.sqa_random_trees(5, 9, 3)
    specs = [(LHZ, 9, dict(decoder=sqa.SQA_DEC_LHZ_TREES, readout_slice=3, trees=trees)),
             (LHZ, 9, dict(decoder=sqa.SQA_DEC_LHZ_BP, readout_slice=1, trees=trees[:1], error_rate=0.2,
                           iterations=10)),
             (LHZ, 10, dict(decoder=sqa.SQA_DEC_LHZ_MLD, readout_slice=0, error_rate=0.1)),
             (ME, 7, dict(decoder=sqa.SQA_DEC_ME_MAJORITY, readout_slice=5)),
             (MEC, 11, dict(decoder=sqa.SQA_DEC_ME_MAJORITY, readout_slice=2))]
    srv = sqa.Server(64 << 20, 2, 50)
    tk = []
    for q, (kind, N, d) in enumerate(specs):
        J = sk_instance(N, 500 + q)
        tk.append((srv.submit(kind, J, -2, 7.0, 8, 120, 6, 3.0, 0.05, 0xDEC0 + q, **d), kind, N, J, d, q))
    for t, kind, N, J, d, q in tk:
        srv.wait(t, 120_000)
        spins, E, lq, lE, _ = srv.result(t, logical=True)
        alone = sqa.SQA(kind, J, -2, 7.0, 8, 120, 6, 3.0, 0.05, 0xDEC0 + q).anneal()
        aq, aE = alone.decode(d["decoder"], d["readout_slice"], trees=d.get("trees"),
                              error_rate=d.get("error_rate", 0.2), iterations=d.get("iterations", 10))
        assert (lq == aq).all() and (lE == aE).all(), (kind, d["decoder"])
        emb = O.Embedding(kind, J, -2)
        for r in range(6):
            s = spins[r, d["readout_slice"]]
            if d["decoder"] == sqa.SQA_DEC_LHZ_TREES:
                ref = O.lhz_tree_decode(N, s, trees)
            elif d["decoder"] == sqa.SQA_DEC_LHZ_BP:
                ref = O.lhz_bp(N, s, trees[:1], 0.2, 10)[0]
            elif d["decoder"] == sqa.SQA_DEC_LHZ_MLD:
                ref = O.lhz_mld(N, s, 0.1)[0]
            else:
                ref = O.me_majority(emb, s)
            assert (lq[r] == ref).all() and lE[r] == O.logical_energy(J, ref)
    srv.close()


def test_server_rejects_bad_decoders(sqa):
    srv = sqa.Server(64 << 20, 2, 50)
    J = sk_instance(8, 3)
    for kind, d, st in ((ME, dict(decoder=sqa.SQA_DEC_LHZ_MWD), "INVALID"),
                        (LHZ, dict(decoder=sqa.SQA_DEC_ME_MAJORITY), "INVALID"),
                        (LHZ, dict(decoder=sqa.SQA_DEC_LHZ_TREES), "INVALID"),            # no trees
                        (LHZ, dict(decoder=sqa.SQA_DEC_LHZ_MWD, readout_slice=8), "INVALID"),
                        (LHZ, dict(decoder=sqa.SQA_DEC_LHZ_MLD, error_rate=0.7), "INVALID")):
        with pytest.raises(sqa.SqaError) as e:
            srv.submit(kind, J, -2, 7.0, 8, 10, 2, 3.0, 0.05, 1, **d)
        assert e.value.status == getattr(sqa, "SQA_ERR_" + st)
    with pytest.raises(sqa.SqaError) as e:
        srv.submit(LHZ, sk_instance(33, 1), -2, 7.0, 2, 10, 2, 3.0, 0.05, 1, decoder=sqa.SQA_DEC_LHZ_MWD)
    assert e.value.status == sqa.SQA_ERR_UNSUPPORTED
    srv.close()


def test_server_cancel_waiting_and_running_jobs(sqa):
    """One slot: the first job runs while the others wait.  Cancelling a waiting job
    drops it at once; cancelling the running one drops it at the next launch boundary;
    the remaining jobs still equal their alone runs; finished and unknown tickets cannot
    be cancelled."""
    jobs = _jobs(4, seed=41_000, sweeps=(3000, 3000), n_range=(16, 20))
    srv = sqa.Server(256 << 20, 1, 25)
    tk = [srv.submit(j.kind, j.J, j.penalty, j.beta, j.slices, j.sweeps, j.replicas, j.gamma0, j.gamma1, j.seed)
          for j in jobs]
    srv.cancel(tk[2])                                        # waiting
    assert srv.poll(tk[2])
    with pytest.raises(sqa.SqaError) as e:
        srv.wait(tk[2], 1000)
    assert e.value.status == sqa.SQA_ERR_CANCELLED
    srv.cancel(tk[0])                                        # running (or about to run)
    with pytest.raises(sqa.SqaError) as e:
        srv.wait(tk[0], 60_000)
    assert e.value.status == sqa.SQA_ERR_CANCELLED
    with pytest.raises(sqa.SqaError) as e:
        srv.result(tk[0])
    assert e.value.status == sqa.SQA_ERR_CANCELLED
    for i in (1, 3):
        srv.wait(tk[i], 300_000)
    with pytest.raises(sqa.SqaError) as e:
        srv.cancel(tk[1])                                    # already finished
    assert e.value.status == sqa.SQA_ERR_INVALID
    with pytest.raises(sqa.SqaError) as e:
        srv.cancel(987654)
    assert e.value.status == sqa.SQA_ERR_INVALID
    for i in (1, 3):
        j = jobs[i]
        spins, E, _ = srv.result(tk[i])
        alone = sqa.SQA(j.kind, j.J, j.penalty, j.beta, j.slices, j.sweeps, j.replicas, j.gamma0, j.gamma1,
                        j.seed).anneal()
        assert (spins == alone.spins()).all() and (E == alone.energies()).all()
    completed, _, _ = srv.stats()
    assert completed == 2
    srv.close()
