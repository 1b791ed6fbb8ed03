"""GPU parity of ME on Chimera (chains of ceil(N/4)+1, up to six terms per site):
SQA with both moves, PT and majority-vote decoding against the oracle."""
import numpy as np
import pytest

import oracle as O
from paper_1603_03755_amd.workloads import MEC, batch_jobs, sk_instance

pytestmark = pytest.mark.gpu
NTH = 8


@pytest.fixture(scope="module")
def sqa():
    import torch
    assert torch.cuda.is_available()
    from paper_1603_03755_amd import sqa as s
    s.lib()
    return s


CASES = [
    # N, L, M, R, penalty, values, move
    (2, 4, 30, 3, -2, (-1, 1), 0),
    (5, 2, 40, 5, -2, (-1, 1), 1),
    (8, 32, 60, 8, -2, (-1, 1), 0),
    (8, 32, 60, 8, -2, (-1, 1), 1),
    (11, 10, 30, 6, -3, (-2, -1, 1, 3), 0),
    (16, 64, 20, 4, -2, (-1, 1), 1),
    (16, 64, 20, 4, -2, (-1, 1), 0),
    (24, 16, 10, 3, -20, tuple(v for v in range(-10, 11) if v != 0), 0),    # field sums above 63
    (24, 16, 10, 3, -20, tuple(v for v in range(-10, 11) if v != 0), 1),
    (32, 64, 5, 2, -2, (-1, 1), 0),
]


@pytest.mark.parametrize("N,L,M,R,pen,vals,move", CASES)
def test_chimera_sqa_bit_exact(sqa, N, L, M, R, pen, vals, move):
    print(f"chimera N={N} L={L} move={move}", flush=True)
    J = sk_instance(N, 800 + N, values=vals)
    h = np.random.default_rng(N).integers(-2, 3, N).astype(np.int32) if N == 11 else None
    dev = sqa.SQA(MEC, J, pen, 2.0, L, M, R, 3.0, 0.05, 555 + N, h=h, move=move)
    if move == 0:
        emb, table, ospins, oE = O.sqa_anneal(MEC, J, pen, 2.0, L, M, R, 3.0, 0.05, 555 + N, h=h, nthreads=NTH)
        assert (dev.table() == table).all()
    else:
        emb, _, ospins, oE = O.sqa_anneal_wolff(MEC, J, pen, 2.0, L, M, R, 3.0, 0.05, 555 + N, h=h, nthreads=NTH)
    assert dev.sites == emb.n_sites == N * ((N + 3) // 4 + 1)
    dev.anneal()
    assert (dev.spins() == ospins).all()
    assert (dev.energies() == oE).all()
    for sl in (0, L - 1):
        logical, E = dev.decode(sqa.SQA_DEC_ME_MAJORITY, sl)
        for r in range(R):
            q = O.me_majority(emb, ospins[r, sl])
            assert (logical[r] == q).all() and E[r] == O.logical_energy(J, q, h)


@pytest.mark.parametrize("N,R,sweeps", [(8, 16, 300), (16, 32, 100)])
def test_chimera_pt_bit_exact(sqa, N, R, sweeps):
    J = sk_instance(N, 820 + N)
    dev = sqa.PT(MEC, J, -2, 0.1, 5.0, R, sweeps, 1, 77 + N).run()
    spins, E, rep, acc = dev.read()
    emb = O.Embedding(MEC, J, -2)
    ospins, oE, orep, oacc = O.pt_run(emb, O.pt_ladder(0.1, 5.0, R), sweeps, 1, 77 + N)
    assert (rep == orep).all() and (spins == ospins[orep]).all() and (E == oE[orep]).all()
    assert (acc == oacc).all()


def test_chimera_in_a_mixed_batch(sqa):
    """Chimera, clique-chain ME and LHZ handles, both moves, in one batch."""
    jobs = batch_jobs(count=6, sweeps=30, replicas=5, slices=16, sizes=(8, 12, 16))
    hs, refs = [], []
    for i, j in enumerate(jobs):
        kind = MEC if i % 3 == 2 else j.kind
        move = i % 2
        hs.append(sqa.SQA(kind, j.J, j.penalty, j.beta, j.slices, j.sweeps, j.replicas, j.gamma0, j.gamma1,
                          j.seed, move=move))
        run = O.sqa_anneal_wolff if move else O.sqa_anneal
        refs.append(run(kind, j.J, j.penalty, j.beta, j.slices, j.sweeps, j.replicas, j.gamma0, j.gamma1, j.seed,
                        nthreads=NTH))
    b = sqa.Batch(hs)
    b.run()
    hs[0].sync()
    for h, (_, _, ospins, oE) in zip(hs, refs):
        assert (h.spins() == ospins).all() and (h.energies() == oE).all()
    b.close()
