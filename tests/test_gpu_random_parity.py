"""Seeded random SQA cases against the oracle, bit-exact: every embedding kind, both
moves, coupling scales that land in each field mode of the kernels (F up to 10, up to
63, up to 255), local fields on ME sites, odd and even slice counts, small replica
counts.  The cases are drawn once from a fixed seed, so the test is deterministic."""
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


def _cases(count=24, seed=20240601):
    rng = np.random.default_rng(seed)
    scales = [((-1, 1), -2), (tuple(v for v in range(-3, 4) if v), -4), (tuple(v for v in range(-10, 11) if v), -12),
              (tuple(v for v in range(-10, 11) if v), -60)]
    out = []
    for i in range(count):
        kind = int(rng.choice([ME, LHZ, MEC]))
        N = int(rng.integers(3, 9))
        vals, pen = scales[int(rng.integers(0, len(scales)))]
        L = int(rng.choice([1, 2, 6, 16, 24, 32, 64]))
        R = int(rng.integers(1, 7))
        M = int(rng.integers(8, 30))
        move = int(rng.integers(0, 2))
        if move == 1 and L == 1:
            L = 2                          # Wolff moves act along imaginary time
        with_h = kind != LHZ and bool(rng.integers(0, 2))
        out.append((i, kind, N, vals, pen, L, R, M, move, with_h))
    return out


@pytest.mark.parametrize("case", _cases(), ids=lambda c: f"c{c[0]}")
def test_random_case_bit_exact(sqa, case):
    i, kind, N, vals, pen, L, R, M, move, with_h = case
    rng = np.random.default_rng(1000 + i)
    J = sk_instance(N, 4000 + i, values=vals)
    h = rng.integers(-3, 4, N).astype(np.int32) if with_h else None
    emb = O.Embedding(kind, J, pen, h)
    if emb.fmax > 255:
        pytest.skip("field sum above the library's limit")
    seed = 0x7700 + i
    print(f"random case {i}: kind={kind} N={N} F={emb.fmax} L={L} R={R} M={M} move={move} h={with_h}", flush=True)
    if move == 0:
        dev = sqa.SQA(kind, J, pen, 4.0, L, M, R, 2.0, 0.05, seed, h=h).anneal()
        _, _, ospins, oE = O.sqa_anneal(kind, J, pen, 4.0, L, M, R, 2.0, 0.05, seed, h=h, nthreads=8)
    else:
        dev = sqa.SQA(kind, J, pen, 4.0, L, M, R, 2.0, 0.05, seed, h=h, move=sqa.SQA_MOVE_WOLFF).anneal()
        _, _, ospins, oE = O.sqa_anneal_wolff(kind, J, pen, 4.0, L, M, R, 2.0, 0.05, seed, h=h, nthreads=8)
    assert (dev.spins() == ospins).all()
    assert (dev.energies() == oE).all()


def _pt_cases(count=12, seed=20240602):
    rng = np.random.default_rng(seed)
    scales = [((-1, 1), -2), (tuple(v for v in range(-10, 11) if v), -8), (tuple(v for v in range(-10, 11) if v), -15),
              (tuple(v for v in range(-10, 11) if v), -40)]
    out = []
    for i in range(count):
        kind = int(rng.choice([ME, LHZ, MEC]))
        N = int(rng.integers(3, 8))
        vals, pen = scales[int(rng.integers(0, len(scales)))]
        R = int(rng.integers(1, 41))
        sweeps = int(rng.integers(10, 40))
        sps = int(rng.integers(1, 4))
        with_h = kind != LHZ and bool(rng.integers(0, 2))
        out.append((i, kind, N, vals, pen, R, sweeps, sps, with_h))
    return out


@pytest.mark.parametrize("case", _pt_cases(), ids=lambda c: f"pt{c[0]}")
def test_random_pt_case_bit_exact(sqa, case):
    i, kind, N, vals, pen, R, sweeps, sps, with_h = case
    rng = np.random.default_rng(2000 + i)
    J = sk_instance(N, 5000 + i, values=vals)
    h = rng.integers(-3, 4, N).astype(np.int32) if with_h else None
    emb = O.Embedding(kind, J, pen, h)
    seed = 0x8800 + i
    print(f"random PT case {i}: kind={kind} N={N} F={emb.fmax} R={R} sweeps={sweeps} sps={sps} h={with_h}", flush=True)
    spins, E, rep, acc = sqa.PT(kind, J, pen, 0.05, 2.0, R, sweeps, sps, seed, h=h).run().read()
    ospins, oE, orep, oacc = O.pt_run(emb, O.pt_ladder(0.05, 2.0, R), sweeps, sps, seed)
    assert (rep == orep).all() and (spins == ospins[orep]).all() and (E == oE[orep]).all()
    assert (acc == oacc).all()
