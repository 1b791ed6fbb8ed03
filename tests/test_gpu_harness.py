"""GPU tests of the exhaustive ground-state search and the penalty-scan harness:
success probabilities equal those computed from the oracle's anneals, oracle
decoders and oracle ground states."""
import numpy as np
import pytest

import oracle as O
from paper_1603_03755_amd.workloads import LHZ, ME, MEC, sk_instance

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def sqa():
    import torch
    assert torch.cuda.is_available()
    from paper_1603_03755_amd import sqa as s
    s.lib()
    return s


@pytest.mark.parametrize("N,vals,with_h", [(2, (-1, 1), False), (3, (-5, 7), True), (8, (-1, 1), False),
                                            (12, tuple(range(-10, 0)) + tuple(range(1, 11)), False),
                                            (16, (-3, -1, 2), True), (21, (-1, 1), False),
                                            (24, tuple(range(-10, 0)) + tuple(range(1, 11)), True)])
def test_ground_state_matches_oracle(sqa, N, vals, with_h):
    print(f"ground N={N}", flush=True)
    rng = np.random.default_rng(N)
    J = sk_instance(N, 70 + N, values=vals)
    h = rng.integers(-6, 7, N).astype(np.int32) if with_h else None
    E, state = sqa.sqa_ground_state(J, h)
    E0, states, count = O.ground_states(J, h)
    assert E == E0
    assert O.logical_energy(J, state, h) == E0


def test_ground_state_limits(sqa):
    with pytest.raises(sqa.SqaError) as e:
        sqa.sqa_ground_state(sk_instance(33, 1))
    assert e.value.status == sqa.SQA_ERR_UNSUPPORTED
    J = sk_instance(5, 1)
    J[0, 1] = 40000
    with pytest.raises(sqa.SqaError):
        sqa.sqa_ground_state(J)


def test_penalty_scan_equals_oracle(sqa):
    """A small scan (2 instances, 3 penalties, both schemes, Wolff moves): every p_s
    equals the one computed from the oracle's anneal, decoders and ground state."""
    from paper_1603_03755_amd import harness as H
    cfg = H.ScanConfig(sweeps=40, reads=12, slices=8, schemes=("mec", "me", "lhz"),
                       lhz_decoders=("mvd", "mwd", "bp"), trees=3)
    instances = [H.paper_instance(5, 11), H.paper_instance(6, 12)]
    penalties = [0.5, 1.5, 3.0]
    res = H.penalty_scan(instances, penalties, cfg)
    beta = cfg.beta_eff / H.SCALE
    for i, J in enumerate(instances):
        N = J.shape[0]
        E0 = O.ground_states(J)[0]
        assert res.ground_energy[i] == E0
        trees = O.random_trees(cfg.seed + i, N, cfg.trees)
        for k, lam in enumerate(penalties):
            pen = H.penalty_coefficient(lam)
            for kind in (MEC, ME, LHZ):
                seed = cfg.seed + 1000 * i + 10 * k + kind
                emb, _, spins, _ = O.sqa_anneal_wolff(kind, J, pen, beta, cfg.slices, cfg.sweeps, cfg.reads,
                                                      H.SCALE * cfg.gamma_start, H.SCALE * cfg.gamma_end, seed,
                                                      nthreads=8)
                if kind != LHZ:
                    ok = [O.logical_energy(J, O.me_majority(emb, spins[r, 0])) == E0 for r in range(cfg.reads)]
                    assert res.p_s["mec" if kind == MEC else "me"][i, k] == np.mean(ok)
                    continue
                dec = {"mvd": lambda s: O.lhz_tree_decode(N, s, trees),
                       "mwd": lambda s: O.lhz_mwd(N, s),
                       "bp": lambda s: O.lhz_bp(N, s, trees[:1], 0.2, 10)[0]}
                for d, fn in dec.items():
                    ok = [O.logical_energy(J, fn(spins[r, 0])) == E0 for r in range(cfg.reads)]
                    assert res.p_s["lhz_" + d][i, k] == np.mean(ok), (i, k, d)
    pen_me, ps_me = res.optimal("mec")
    assert len(pen_me) == 2 and all(0 <= p <= 1 for p in ps_me)


def test_valu_calibration_launch(sqa):
    """The issue-rate calibration runs on every CU (eight waves per SIMD) and counts its
    chains' instructions; the rate itself is the benchmark's business, not a test bound."""
    import torch
    import bench
    cus = torch.cuda.get_device_properties(0).multi_processor_count
    for op in (0, 1, 2):
        print(f"valu calibration op={op}", flush=True)
        ms, instr = bench.valu_issue(op, 2000)
        assert ms > 0.0
        assert instr == cus * 8 * 4 * 2000 * 8


def test_pt_penalty_scan_equals_oracle(sqa):
    """A small PT scan (2 instances, 3 penalties, ME on Chimera, clique-chain ME and LHZ,
    6 ladders of 8 temperatures each): every p_s, at every temperature, equals the one
    computed from the oracle's ladders, the oracle's decoders and the exhaustive ground
    state; the critical penalties follow from those p_s."""
    from paper_1603_03755_amd import harness as H
    cfg = H.PTScanConfig(temps=8, swaps=60, sweeps_per_swap=2, runs=6, schemes=("mec", "me", "lhz"), trees=3)
    instances = [H.paper_instance(5, 21), H.paper_instance(6, 22)]
    penalties = [0.5, 1.5, 3.0]
    res = H.pt_penalty_scan(instances, penalties, cfg)
    betas = O.pt_ladder(cfg.beta_min / H.SCALE, cfg.beta_max / H.SCALE, cfg.temps)
    assert np.allclose(res.betas / H.SCALE, betas, rtol=1e-12, atol=0)
    for i, J in enumerate(instances):
        N = J.shape[0]
        E0 = O.ground_states(J)[0]
        assert res.ground_energy[i] == E0
        trees = O.random_trees(cfg.seed + i, N, cfg.trees)
        for k, lam in enumerate(penalties):
            pen = H.penalty_coefficient(lam)
            for scheme in cfg.schemes:
                kind = H.KINDS[scheme]
                emb = O.Embedding(kind, J, pen)
                hits = np.zeros(cfg.temps)
                for run in range(cfg.runs):
                    ospins, _, orep, _ = O.pt_run(emb, betas, cfg.sweeps, cfg.sweeps_per_swap,
                                                  H.pt_seed(cfg, i, k, kind, run))
                    for slot in range(cfg.temps):
                        s = ospins[orep[slot]]
                        q = O.me_majority(emb, s) if kind != LHZ else O.lhz_tree_decode(N, s, trees)
                        hits[slot] += O.logical_energy(J, q) == E0
                assert (res.p_s[scheme][i, k] == hits / cfg.runs).all(), (scheme, i, k)
    for scheme in cfg.schemes:
        crit = res.critical(scheme)
        assert len(crit) == len(instances)
        for i, c in enumerate(crit):
            ps = res.p_s[scheme][i, :, 0]
            assert np.isnan(c) == (ps.max() < 0.5)
