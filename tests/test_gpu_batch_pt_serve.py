"""GPU parity of the batched persistent launch, parallel tempering and the
continuous-batching server against the CPU oracle (bit-exact), plus the
full-size batched workload checked on sampled replicas."""
import os

import numpy as np
import pytest

import oracle as O
from paper_1603_03755_amd.workloads import LHZ, ME, MEC, batch_jobs, pt_jobs, sk_instance

pytestmark = pytest.mark.gpu
NTH = min(os.cpu_count() or 1, 16)


@pytest.fixture(scope="module")
def sqa():
    import torch
    assert torch.cuda.is_available()
    from paper_1603_03755_amd import sqa as s
    s.lib()
    return s


def _mixed_jobs():
    """Uneven handles: both embeddings, several N, L and replica counts."""
    spec = [(ME, 5, 32, 7), (LHZ, 8, 64, 16), (ME, 12, 16, 3), (LHZ, 6, 8, 9), (ME, 8, 64, 4),
            (LHZ, 12, 32, 5), (ME, 3, 2, 2), (LHZ, 4, 1, 6)]
    out = []
    for q, (kind, N, L, R) in enumerate(spec):
        out.append(dict(kind=kind, J=sk_instance(N, 900 + q), pen=-2, beta=8.0, L=L, M=40 + 7 * q, R=R,
                        g0=3.0, g1=0.02, seed=0xBA7C0000 + q))
    return out


@pytest.mark.parametrize("waves", [1, 2, 4, 8])
def test_batch_equals_oracle_for_every_handle(sqa, waves):
    specs = _mixed_jobs()
    print(f"batch of {len(specs)} uneven handles, waves_per_group={waves}", flush=True)
    hs = [sqa.SQA(s["kind"], s["J"], s["pen"], s["beta"], s["L"], s["M"], s["R"], s["g0"], s["g1"], s["seed"])
          for s in specs]
    b = sqa.Batch(hs, waves_per_group=waves)
    b.run()
    for s, h in zip(specs, hs):
        emb, table, ospins, oE = O.sqa_anneal(s["kind"], s["J"], s["pen"], s["beta"], s["L"], s["M"], s["R"],
                                              s["g0"], s["g1"], s["seed"], nthreads=NTH)
        assert (h.spins() == ospins).all()
        assert (h.energies() == oE).all()
    # graph replay gives the same result again (state re-initialised from the seed)
    first = [h.spins() for h in hs]
    b.run()
    for f, h in zip(first, hs):
        assert (h.spins() == f).all()
    b.close()


def test_team_and_wave_modes_agree(sqa):
    """Team mode (a workgroup's waves share one replica) and one wave per replica give
    identical lattices and energies: the same handles in an automatic batch above the
    team-mode replica limit (one wave per replica), alone (team mode), and in a small
    automatic batch (team mode), including ragged classes, L = 1, 2 and odd bytes."""
    spec = [(ME, 7, 64), (LHZ, 9, 32), (ME, 5, 2), (LHZ, 6, 1), (ME, 10, 22), (LHZ, 8, 64), (ME, 4, 10),
            (LHZ, 11, 16), (ME, 12, 64)]
    specs = []
    for q, (kind, N, L) in enumerate(spec):
        specs.append(dict(kind=kind, J=sk_instance(N, 300 + q), pen=-2, beta=8.0, L=L, M=25, R=64, g0=3.0,
                          g1=0.05, seed=0x7EA00 + q))
    # pad with extra handles so that the batch holds more than 1024 replicas
    pad = [dict(kind=LHZ, J=sk_instance(5, 400 + q), pen=-2, beta=6.0, L=16, M=10, R=64, g0=2.0, g1=0.1,
                seed=0x7EB00 + q) for q in range(9)]
    mk = lambda s: sqa.SQA(s["kind"], s["J"], s["pen"], s["beta"], s["L"], s["M"], s["R"], s["g0"], s["g1"],
                           s["seed"])
    print(f"wave-mode batch of {len(specs) + len(pad)} handles x 64 replicas", flush=True)
    big = [mk(s) for s in specs + pad]
    b = sqa.Batch(big)
    b.run()
    wave = [(h.spins(), h.energies()) for h in big[:len(specs)]]
    b.close()
    print("same handles alone and as a small batch (team mode)", flush=True)
    alone = [mk(s).anneal() for s in specs]
    small = [mk(s) for s in specs[:4]]
    b2 = sqa.Batch(small)
    b2.run()
    for (ws, we), a in zip(wave, alone):
        assert (a.spins() == ws).all() and (a.energies() == we).all()
    for (ws, we), h in zip(wave, small):
        assert (h.spins() == ws).all() and (h.energies() == we).all()
    b2.close()
    _, _, ospins, oE = O.sqa_anneal(specs[0]["kind"], specs[0]["J"], -2, 8.0, 64, 25, 64, 3.0, 0.05,
                                    specs[0]["seed"], nthreads=NTH)
    assert (wave[0][0] == ospins).all() and (wave[0][1] == oE).all()


def test_team_mode_mixed_sizes(sqa):
    """Team mode over handles of very different sizes in one launch: the workgroup's
    waves (capped at 8) are set by the largest handle (N = 32 ME, L = 64, colour classes
    of 992 items, two passes each), and the small handles' replicas run on the same
    wide workgroups, with replica counts of 3 to 16: every handle equals the oracle."""
    spec = [(ME, 32, 64, 3), (ME, 16, 64, 5), (LHZ, 12, 64, 7), (ME, 8, 32, 16), (LHZ, 6, 16, 3)]
    specs = [dict(kind=kind, J=sk_instance(N, 330 + q), pen=-2, beta=8.0, L=L, M=20, R=R, g0=3.0, g1=0.05,
                  seed=0x7EC00 + q) for q, (kind, N, L, R) in enumerate(spec)]
    print("team mode, handles of mixed sizes in one launch", flush=True)
    hs = [sqa.SQA(s["kind"], s["J"], s["pen"], s["beta"], s["L"], s["M"], s["R"], s["g0"], s["g1"], s["seed"])
          for s in specs]
    b = sqa.Batch(hs)
    b.run()
    for s, h in zip(specs, hs):
        _, _, ospins, oE = O.sqa_anneal(s["kind"], s["J"], s["pen"], s["beta"], s["L"], s["M"], s["R"], s["g0"],
                                        s["g1"], s["seed"], nthreads=NTH)
        assert (h.spins() == ospins).all() and (h.energies() == oE).all()
    b.close()


def test_team_mode_other_paths(sqa):
    """Team mode on the sweep paths the mixed-size test leaves out: ME on Chimera (six-term
    records), a runtime L (24, the last byte of each parity ragged), and field sums above 10
    (6-bit and 8-bit field modes), beside a compile-time-L handle in the same launch: every
    handle equals the oracle."""
    spec = [(MEC, 8, 32, 4, -2), (ME, 10, 24, 6, -2), (LHZ, 9, 64, 5, -6), (ME, 8, 32, 3, -40),
            (ME, 12, 64, 8, -2)]
    specs = [dict(kind=kind, J=sk_instance(N, 420 + q), pen=pen, beta=6.0, L=L, M=16, R=R, g0=3.0, g1=0.05,
                  seed=0x7ED00 + q) for q, (kind, N, L, R, pen) in enumerate(spec)]
    print("team mode, Chimera records, runtime L and larger fields", flush=True)
    hs = [sqa.SQA(s["kind"], s["J"], s["pen"], s["beta"], s["L"], s["M"], s["R"], s["g0"], s["g1"], s["seed"])
          for s in specs]
    assert max(h.fmax for h in hs) > 63          # an 8-bit field handle is in the set
    b = sqa.Batch(hs)
    b.run()
    for s, h in zip(specs, hs):
        _, _, ospins, oE = O.sqa_anneal(s["kind"], s["J"], s["pen"], s["beta"], s["L"], s["M"], s["R"], s["g0"],
                                        s["g1"], s["seed"], nthreads=NTH)
        assert (h.spins() == ospins).all() and (h.energies() == oE).all()
    b.close()


def test_batch_graph_replays_with_eager_work_between(sqa):
    specs = _mixed_jobs()[:4]
    hs = [sqa.SQA(s["kind"], s["J"], s["pen"], s["beta"], s["L"], s["M"], s["R"], s["g0"], s["g1"], s["seed"])
          for s in specs]
    ref = []
    for h in hs:
        h.anneal()
        ref.append((h.spins(), h.energies()))
    b = sqa.Batch(hs)
    for rep in range(3):
        b.run()
        for (s0, e0), h in zip(ref, hs):
            assert (h.spins() == s0).all() and (h.energies() == e0).all()
        hs[rep].anneal_range(0, 5)          # eager work on a handle between replays
    b.close()


def test_anneal_batch_one_shot(sqa):
    specs = _mixed_jobs()[2:6]
    hs = [sqa.SQA(s["kind"], s["J"], s["pen"], s["beta"], s["L"], s["M"], s["R"], s["g0"], s["g1"], s["seed"])
          for s in specs]
    sqa.sqa_anneal_batch(hs)
    for s, h in zip(specs, hs):
        _, _, ospins, _ = O.sqa_anneal(s["kind"], s["J"], s["pen"], s["beta"], s["L"], s["M"], s["R"], s["g0"],
                                       s["g1"], s["seed"], nthreads=NTH)
        assert (h.spins() == ospins).all()


def test_full_size_batched_workload_sampled(sqa):
    """The benchmark's workload at full size (512 instances, 64 replicas, L = 64,
    10^4 sweeps, one persistent launch): sampled replicas of every (embedding, N)
    stratum equal the oracle's; every replica's energies equal its spins' energies."""
    jobs = batch_jobs()
    hs = [sqa.SQA(j.kind, j.J, j.penalty, j.beta, j.slices, j.sweeps, j.replicas, j.gamma0, j.gamma1, j.seed)
          for j in jobs]
    print("full-size batch: 512 handles, running", flush=True)
    b = sqa.Batch(hs)
    b.run()
    hs[0].sync()
    print("full-size batch done, checking samples", flush=True)
    seen = {}
    rng = np.random.default_rng(0)
    for i, j in enumerate(jobs):
        if (j.kind, j.n) not in seen:
            seen[(j.kind, j.n)] = (i, int(rng.integers(0, j.replicas)))
    from concurrent.futures import ThreadPoolExecutor

    def oracle_replica(ir):
        i, r = ir
        j = jobs[i]
        return O.sqa_anneal(j.kind, j.J, j.penalty, j.beta, j.slices, j.sweeps, 1, j.gamma0, j.gamma1, j.seed,
                            nthreads=1, r0=r)

    with ThreadPoolExecutor(max_workers=8) as ex:
        refs = list(ex.map(oracle_replica, seen.values()))
    for (i, r), (emb, _, ospins, oE) in zip(seen.values(), refs):
        spins, E = hs[i].spins(), hs[i].energies()
        assert (spins[r] == ospins[0]).all(), (i, r)
        assert (E[r] == oE[0]).all(), (i, r)
        assert (O.sqa_energies(emb, spins) == E).all()
    b.close()


# ------------------------------------------------------------------ PT
PT_CASES = [(LHZ, 5, 8, 300, 1), (ME, 4, 5, 200, 2), (LHZ, 3, 1, 50, 1), (ME, 6, 64, 40, 3), (LHZ, 8, 32, 500, 1),
            (ME, 2, 3, 30, 1)]


@pytest.mark.parametrize("kind,N,R,sweeps,sps", PT_CASES)
def test_pt_bit_exact(sqa, kind, N, R, sweeps, sps):
    J = sk_instance(N, 700 + N)
    seed = 0x9700 + N
    print(f"PT kind={kind} N={N} R={R} sweeps={sweeps}", flush=True)
    dev = sqa.PT(kind, J, -2, 0.1, 5.0, R, sweeps, sps, seed).run()
    spins, E, rep, acc = dev.read()
    emb = O.Embedding(kind, J, -2)
    betas = O.pt_ladder(0.1, 5.0, R)
    ospins, oE, orep, oacc = O.pt_run(emb, betas, sweeps, sps, seed)
    assert (rep == orep).all()
    assert (spins == ospins[orep]).all()       # device returns spins by slot
    assert (E == oE[orep]).all()
    assert (acc == oacc).all()


@pytest.mark.parametrize("stage", ["1", "0"])
def test_pt_swap_table_in_lds_or_device_memory(sqa, monkeypatch, stage):
    """The swap thresholds read from the packed table staged in LDS and from device
    memory give the same ladder (and the oracle's), on swaps that happen every sweep."""
    monkeypatch.setenv("SQA_PT_STAGE_SWAPS", stage)
    print(f"PT swap table staged={stage}", flush=True)
    for kind, N, R in ((ME, 7, 32), (LHZ, 6, 13)):
        J = sk_instance(N, 750 + N)
        seed = 0x9800 + N
        dev = sqa.PT(kind, J, -2, 0.2, 4.0, R, 120, 1, seed).run()
        spins, E, rep, acc = dev.read()
        emb = O.Embedding(kind, J, -2)
        ospins, oE, orep, oacc = O.pt_run(emb, O.pt_ladder(0.2, 4.0, R), 120, 1, seed)
        assert (rep == orep).all() and (spins == ospins[orep]).all()
        assert (E == oE[orep]).all() and (acc == oacc).all()
        assert acc.sum() > 0


@pytest.mark.parametrize("mode", ["bounds", "bisect", "table"])
def test_pt_swap_decisions_by_bounds_or_thresholds(sqa, monkeypatch, mode):
    """A swap phase compares each pair's energy gap with the pair's acceptance
    bound, found from a float estimate checked against the staged table
    (default) or by bisection from 0 (bisect), or it reads the gap's threshold
    (table): each gives the oracle's ladder, with swaps every sweep over wide,
    narrow and zero temperature spans."""
    if mode == "bounds":
        monkeypatch.delenv("SQA_DEBUG_PT_SWAP", raising=False)
    else:
        monkeypatch.setenv("SQA_DEBUG_PT_SWAP", mode)
    for kind, N, R, bmin, bmax in ((ME, 8, 32, 0.1, 5.0), (LHZ, 7, 20, 0.05, 20.0), (ME, 5, 64, 1.0, 1.2),
                                   (LHZ, 4, 8, 2.0, 2.0)):
        print(f"PT swap decisions mode={mode} kind={kind} N={N} R={R} beta=[{bmin},{bmax}]", flush=True)
        J = sk_instance(N, 760 + N)
        seed = 0x9900 + N + R
        dev = sqa.PT(kind, J, -2, bmin, bmax, R, 150, 1, seed).run()
        spins, E, rep, acc = dev.read()
        emb = O.Embedding(kind, J, -2)
        ospins, oE, orep, oacc = O.pt_run(emb, O.pt_ladder(bmin, bmax, R), 150, 1, seed)
        assert (rep == orep).all() and (spins == ospins[orep]).all()
        assert (E == oE[orep]).all() and (acc == oacc).all()
        assert acc.sum() > 0


@pytest.mark.parametrize("phases", ["merged", "4"])
def test_pt_merged_colour_classes(sqa, monkeypatch, phases):
    """ME ladders sweep classes 1 and 2, which share no term, as one phase (three
    per sweep); the four classes one after the other (SQA_DEBUG_PT_PHASES=4) give
    the same ladder, and both are the oracle's, on ME, on ME on Chimera and with
    waves that take two items of the merged phase."""
    if phases == "merged":
        monkeypatch.delenv("SQA_DEBUG_PT_PHASES", raising=False)
    else:
        monkeypatch.setenv("SQA_DEBUG_PT_PHASES", phases)
    for kind, N, R, waves in ((ME, 9, 32, None), (ME, 12, 16, "3"), (MEC, 8, 24, None)):
        print(f"PT phases={phases} kind={kind} N={N} R={R} waves={waves}", flush=True)
        if waves is None:
            monkeypatch.delenv("SQA_PT_WAVES", raising=False)
        else:
            monkeypatch.setenv("SQA_PT_WAVES", waves)
        J = sk_instance(N, 780 + N)
        seed = 0x9A00 + N
        dev = sqa.PT(kind, J, -2, 0.1, 5.0, R, 120, 1, seed).run()
        spins, E, rep, acc = dev.read()
        emb = O.Embedding(kind, J, -2)
        ospins, oE, orep, oacc = O.pt_run(emb, O.pt_ladder(0.1, 5.0, R), 120, 1, seed)
        assert (rep == orep).all() and (spins == ospins[orep]).all()
        assert (E == oE[orep]).all() and (acc == oacc).all()


@pytest.mark.parametrize("waves", ["1", "3", "10"])
def test_pt_results_do_not_depend_on_wave_count(sqa, monkeypatch, waves):
    """The last wave decides the swap phases and every wave keeps its own energy
    partials: one wave (several items per thread, and the swap decisions), three,
    or the most a ladder may use give the oracle's ladder, with replica bytes from
    one to eight and swap intervals of one and three sweeps."""
    monkeypatch.setenv("SQA_PT_WAVES", waves)
    print(f"PT waves={waves}", flush=True)
    for kind, N, R, sps in ((ME, 7, 32, 1), (LHZ, 8, 64, 1), (ME, 5, 9, 3), (LHZ, 6, 5, 1)):
        J = sk_instance(N, 770 + N)
        seed = 0x9900 + 7 * N + R
        dev = sqa.PT(kind, J, -2, 0.2, 4.0, R, 90, sps, seed).run()
        spins, E, rep, acc = dev.read()
        emb = O.Embedding(kind, J, -2)
        ospins, oE, orep, oacc = O.pt_run(emb, O.pt_ladder(0.2, 4.0, R), 90, sps, seed)
        assert (rep == orep).all() and (spins == ospins[orep]).all()
        assert (E == oE[orep]).all() and (acc == oacc).all()
        assert acc.sum() > 0


@pytest.mark.parametrize("kind,N,R,sweeps,sps,waves", [(LHZ, 6, 16, 400, 150, None), (ME, 5, 32, 300, 1000, None),
                                                       (LHZ, 10, 64, 300, 120, "1"), (ME, 7, 24, 260, 97, "1")])
def test_pt_long_intervals_between_swaps(sqa, monkeypatch, kind, N, R, sweeps, sps, waves):
    """Many sweeps between swap phases (and none at all when the interval exceeds the
    run): a thread's 16-bit flip sums are emptied into 32-bit sums many times before
    an energy reduction; with one wave a thread also takes several items per class."""
    if waves is None:
        monkeypatch.delenv("SQA_PT_WAVES", raising=False)
    else:
        monkeypatch.setenv("SQA_PT_WAVES", waves)
    print(f"PT long swap interval kind={kind} N={N} R={R} sweeps={sweeps} sps={sps} waves={waves}", flush=True)
    J = sk_instance(N, 790 + N)
    seed = 0x9A00 + 3 * N + R
    dev = sqa.PT(kind, J, -2, 0.2, 4.0, R, sweeps, sps, seed).run()
    spins, E, rep, acc = dev.read()
    emb = O.Embedding(kind, J, -2)
    ospins, oE, orep, oacc = O.pt_run(emb, O.pt_ladder(0.2, 4.0, R), sweeps, sps, seed)
    assert (rep == orep).all() and (spins == ospins[orep]).all()
    assert (E == oE[orep]).all() and (acc == oacc).all()


def test_pt_workload_shape_sampled(sqa):
    """PT workload shape (N = 24, 32 temperatures, both embeddings) in one batched
    launch, at a reduced sweep count the oracle can finish: two instances exact."""
    jobs = pt_jobs(instances=2, sweeps=2000)
    hs = [sqa.PT(j.kind, j.J, j.penalty, j.beta_min, j.beta_max, j.temps, j.sweeps, j.sweeps_per_swap, j.seed)
          for j in jobs]
    sqa.pt_run_batch(hs)
    for j, h in zip(jobs, hs):
        spins, E, rep, acc = h.read()
        emb = O.Embedding(j.kind, j.J, j.penalty)
        ospins, oE, orep, oacc = O.pt_run(emb, O.pt_ladder(j.beta_min, j.beta_max, j.temps), j.sweeps,
                                          j.sweeps_per_swap, j.seed)
        assert (rep == orep).all() and (spins == ospins[orep]).all() and (E == oE[orep]).all()
        assert (acc == oacc).all()


# ------------------------------------------------------------------ serving
def test_server_results_equal_alone_runs(sqa):
    """Jobs of mixed size run together through the server equal the same jobs run
    alone (and the oracle), whatever else shares their launches."""
    specs = _mixed_jobs()
    srv = sqa.Server(hbm_budget_bytes=3 << 20, max_slots=3, chunk_sweeps=13)
    tickets = [srv.submit(s["kind"], s["J"], s["pen"], s["beta"], s["L"], s["M"], s["R"], s["g0"], s["g1"],
                          s["seed"]) for s in specs]
    for t, s in zip(tickets, specs):
        srv.wait(t, 120_000)
        spins, E, lat = srv.result(t)
        assert lat > 0
        alone = sqa.SQA(s["kind"], s["J"], s["pen"], s["beta"], s["L"], s["M"], s["R"], s["g0"], s["g1"],
                        s["seed"]).anneal()
        assert (spins == alone.spins()).all() and (E == alone.energies()).all()
        _, _, ospins, oE = O.sqa_anneal(s["kind"], s["J"], s["pen"], s["beta"], s["L"], s["M"], s["R"], s["g0"],
                                        s["g1"], s["seed"], nthreads=NTH)
        assert (spins == ospins).all() and (E == oE).all()
    completed, launches, peak = srv.stats()
    assert completed == len(specs)
    assert peak <= 3 << 20
    srv.close()


def test_server_rejects_job_over_budget(sqa):
    srv = sqa.Server(hbm_budget_bytes=1 << 16, max_slots=2, chunk_sweeps=10)
    with pytest.raises(sqa.SqaError) as e:
        srv.submit(ME, sk_instance(24, 1), -2, 10.0, 64, 100, 64, 3.0, 0.01, 1)
    assert e.value.status == sqa.SQA_ERR_BUSY
    srv.close()


def test_batch_mixed_field_ranges_and_slices(sqa):
    """One launch mixing handles on the fast path (L in {16, 32, 64}, F <= 10), the
    general small-F path (other L) and the wide-field path (F > 10)."""
    specs = [dict(kind=ME, J=sk_instance(6, 11), pen=-2, L=32, R=5),            # fast, F = 5
             dict(kind=LHZ, J=sk_instance(7, 12), pen=-2, L=16, R=3),           # fast, F = 9
             dict(kind=ME, J=sk_instance(5, 13), pen=-6, L=64, R=4),            # F = 13: wide path
             dict(kind=LHZ, J=sk_instance(6, 14), pen=-3, L=10, R=6),           # F = 13, ragged L
             dict(kind=ME, J=sk_instance(4, 15), pen=-2, L=6, R=2),             # small F, ragged L
             dict(kind=LHZ, J=sk_instance(5, 16), pen=-2, L=1, R=7)]            # classical
    hs = []
    for q, s in enumerate(specs):
        s.update(beta=7.0, M=30 + 5 * q, g0=2.0, g1=0.05, seed=0xF1E1D + q)
        hs.append(sqa.SQA(s["kind"], s["J"], s["pen"], s["beta"], s["L"], s["M"], s["R"], s["g0"], s["g1"],
                          s["seed"]))
    sqa.sqa_anneal_batch(hs)
    for s, h in zip(specs, hs):
        _, _, ospins, oE = O.sqa_anneal(s["kind"], s["J"], s["pen"], s["beta"], s["L"], s["M"], s["R"], s["g0"],
                                        s["g1"], s["seed"], nthreads=NTH)
        assert (h.spins() == ospins).all() and (h.energies() == oE).all()


def test_autotune_writes_cache_and_batch_uses_it(sqa, tmp_path, monkeypatch):
    specs = _mixed_jobs()[:4]
    hs = [sqa.SQA(s["kind"], s["J"], s["pen"], s["beta"], s["L"], s["M"], s["R"], s["g0"], s["g1"], s["seed"])
          for s in specs]
    hs[0].anneal()
    before = hs[0].spins()
    cache = tmp_path / "tune.json"
    best = sqa.sqa_autotune(hs, str(cache))
    assert best[0] in (1, 2, 4, 8) and best[1] >= 1
    assert (hs[0].spins() == before).all()          # tuning restores the device state
    text = cache.read_text()
    assert "gfx950" in text
    monkeypatch.setenv("SQA_AUTOTUNE_CACHE", str(cache))
    b = sqa.Batch(hs)
    assert b.config() == best
    b.run()
    for s, h in zip(specs, hs):
        _, _, ospins, _ = O.sqa_anneal(s["kind"], s["J"], s["pen"], s["beta"], s["L"], s["M"], s["R"], s["g0"],
                                       s["g1"], s["seed"], nthreads=NTH)
        assert (h.spins() == ospins).all()
    b.close()


def test_async_anneals_on_torch_streams(sqa):
    """sqa_anneal is asynchronous on the given stream; two handles on two streams."""
    import torch
    specs = _mixed_jobs()[:2]
    hs = [sqa.SQA(s["kind"], s["J"], s["pen"], s["beta"], s["L"], s["M"], s["R"], s["g0"], s["g1"], s["seed"])
          for s in specs]
    streams = [torch.cuda.Stream(), torch.cuda.Stream()]
    for h, st in zip(hs, streams):
        h.anneal(st)
    for s, h in zip(specs, hs):
        _, _, ospins, _ = O.sqa_anneal(s["kind"], s["J"], s["pen"], s["beta"], s["L"], s["M"], s["R"], s["g0"],
                                       s["g1"], s["seed"], nthreads=NTH)
        assert (h.spins() == ospins).all()


@pytest.mark.parametrize("kind,N,pen", [(ME, 6, -40), (LHZ, 6, -30)])
def test_pt_large_field_sums(sqa, kind, N, pen):
    """PT with couplings in {+-1..+-10} and per-site field sums above 63."""
    J = sk_instance(N, 650 + N, values=tuple(v for v in range(-10, 11) if v != 0))
    emb = O.Embedding(kind, J, pen)
    assert emb.fmax > 63
    dev = sqa.PT(kind, J, pen, 0.01, 0.5, 8, 60, 1, 99).run()
    spins, E, rep, acc = dev.read()
    ospins, oE, orep, oacc = O.pt_run(emb, O.pt_ladder(0.01, 0.5, 8), 60, 1, 99)
    assert (rep == orep).all() and (spins == ospins[orep]).all() and (E == oE[orep]).all()
    assert (acc == oacc).all()


@pytest.mark.parametrize("kind,N,pen,fmin,fmax", [(ME, 6, -8, 11, 31), (LHZ, 6, -4, 11, 31),
                                                  (ME, 6, -15, 32, 63), (LHZ, 6, -8, 32, 63)])
def test_pt_field_sum_modes(sqa, kind, N, pen, fmin, fmax):
    """PT in its byte mode (field sums up to 31, signed-weight records) and its 6-bit
    mode (32..63): couplings in {+-1..+-10}, identical to the oracle."""
    J = sk_instance(N, 660 + N, values=tuple(v for v in range(-10, 11) if v != 0))
    emb = O.Embedding(kind, J, pen)
    assert fmin <= emb.fmax <= fmax
    print(f"PT modes kind={kind} F={emb.fmax}", flush=True)
    dev = sqa.PT(kind, J, pen, 0.02, 1.0, 16, 80, 2, 77).run()
    spins, E, rep, acc = dev.read()
    ospins, oE, orep, oacc = O.pt_run(emb, O.pt_ladder(0.02, 1.0, 16), 80, 2, 77)
    assert (rep == orep).all() and (spins == ospins[orep]).all() and (E == oE[orep]).all()
    assert (acc == oacc).all()


def test_pt_many_ladder_shapes_in_one_batch(sqa):
    """Ladders of many sizes (every LDS layout size between them, swap tables staged)
    in one batched launch, each identical to the oracle."""
    cases = [(kind, N, R) for kind in (ME, LHZ) for N, R in ((3, 2), (4, 5), (5, 8), (6, 13), (7, 20), (5, 31),
                                                              (8, 32), (6, 47), (4, 64))]
    hs, refs, emb_J = [], [], []
    for i, (kind, N, R) in enumerate(cases):
        J = sk_instance(N, 900 + i)
        emb_J.append(J)
        hs.append(sqa.PT(kind, J, -2, 0.1, 5.0, R, 25, 1, 0x5A00 + i))
        refs.append((O.Embedding(kind, J, -2), O.pt_ladder(0.1, 5.0, R), 0x5A00 + i))
    print(f"PT batch of {len(hs)} ladders", flush=True)
    sqa.pt_run_batch(hs)
    for h, (emb, betas, seed) in zip(hs, refs):
        spins, E, rep, acc = h.read()
        ospins, oE, orep, oacc = O.pt_run(emb, betas, 25, 1, seed)
        assert (rep == orep).all() and (spins == ospins[orep]).all() and (E == oE[orep]).all()
        assert (acc == oacc).all()
    for h in hs:
        h.close()
    # the same ladders one launch each: every one with its own LDS size
    for i, (kind, N, R) in enumerate(cases):
        emb, betas, seed = refs[i]
        h = sqa.PT(kind, emb_J[i], -2, 0.1, 5.0, R, 25, 1, seed).run()
        spins, E, rep, acc = h.read()
        ospins, oE, orep, oacc = O.pt_run(emb, betas, 25, 1, seed)
        assert (rep == orep).all() and (spins == ospins[orep]).all() and (E == oE[orep]).all()
        h.close()


@pytest.mark.parametrize("order", ["reverse", "shuffle"])
def test_results_do_not_depend_on_work_item_order(sqa, monkeypatch, order):
    """Race check: the batch's work items handed out in another order (host-side debug
    switch) give identical spins and energies for every handle, both moves, one wave
    per replica and team mode."""
    specs = _mixed_jobs()
    mk = lambda s, move: sqa.SQA(s["kind"], s["J"], s["pen"], s["beta"], s["L"], s["M"], s["R"], s["g0"], s["g1"],
                                 s["seed"], move=move)
    for move in (sqa.SQA_MOVE_METROPOLIS, sqa.SQA_MOVE_WOLFF):
        for waves in (0, 2):
            print(f"item order {order} move={move} waves={waves}", flush=True)
            monkeypatch.delenv("SQA_DEBUG_ITEM_ORDER", raising=False)
            ref = [mk(s, move) for s in specs]
            b = sqa.Batch(ref, waves_per_group=waves)
            b.run()
            want = [(h.spins(), h.energies()) for h in ref]
            b.close()
            monkeypatch.setenv("SQA_DEBUG_ITEM_ORDER", order)
            hs = [mk(s, move) for s in specs]
            b = sqa.Batch(hs, waves_per_group=waves)
            b.run()
            for (ws, we), h in zip(want, hs):
                assert (h.spins() == ws).all() and (h.energies() == we).all()
            b.close()
