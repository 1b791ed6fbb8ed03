"""sqa_anneal_batch_noalloc (the batch whose launch scratch is the library's
static array) against sqa_anneal_batch (fresh scratch) through the C ABI: two
calls in a row, the second on a smaller batch, bit-identical spins and
energies; sizes beyond the static array are refused before any device work."""
import os

import numpy as np
import pytest

from paper_1603_03755_amd.workloads import LHZ, ME, MEC, sk_instance

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def sqa():
    import torch
    assert torch.cuda.is_available()
    from paper_1603_03755_amd import sqa as s
    s.lib()
    return s


def _specs(count, salt):
    kinds = (ME, LHZ, MEC)
    out = []
    for q in range(count):
        kind = kinds[q % 3]
        N = 5 + (q * 7 + salt) % 14
        L = (1, 2, 8, 16, 32, 64)[(q + salt) % 6]
        out.append(dict(kind=kind, J=sk_instance(N, 1000 * salt + q), L=L, M=20 + 3 * q, R=1 + (q * 5 + salt) % 70,
                        seed=0xA0A0 + 97 * salt + q, move=(q // 3) % 2))
    return out


def _handles(sqa, specs):
    return [sqa.SQA(s["kind"], s["J"], -2, 7.0, s["L"], s["M"], s["R"], 3.0, 0.05, s["seed"], move=s["move"])
            for s in specs]


@pytest.mark.parametrize("first,second", [(24, 7), (40, 1)])
def test_noalloc_batch_equals_allocating_batch_twice(sqa, first, second):
    import torch
    for call, count in enumerate((first, second)):
        specs = _specs(count, salt=first + call)
        print(f"no-alloc batch call {call}: {count} handles", flush=True)
        a, b = _handles(sqa, specs), _handles(sqa, specs)
        sqa.sqa_anneal_batch(a)
        stream = torch.cuda.Stream()
        sqa.sqa_anneal_batch_noalloc(b, stream)
        for s, x, y in zip(specs, a, b):
            assert (x.spins() == y.spins()).all(), s
            assert (x.energies() == y.energies()).all(), s
        for h in a + b:
            h.close()


def test_noalloc_batch_runs_again_on_the_same_handles(sqa):
    """Handles annealed by the no-alloc batch once, then re-annealed from their seeds by
    it again, give the same state (the static scratch keeps nothing between calls)."""
    specs = _specs(9, salt=3)
    hs = _handles(sqa, specs)
    sqa.sqa_anneal_batch_noalloc(hs)
    first = [(h.spins(), h.energies()) for h in hs]
    hs[2].anneal_range(0, 5)
    sqa.sqa_anneal_batch_noalloc(hs)
    for (s0, e0), h in zip(first, hs):
        assert (h.spins() == s0).all() and (h.energies() == e0).all()


def test_noalloc_batch_refuses_scratch_beyond_its_array(sqa):
    """32 handles of 65536 replicas need more work items (one per four replicas: over
    6 MB) than the static array holds: refused with SQA_ERR_UNSUPPORTED, nothing
    launched; a small batch right after runs."""
    J = sk_instance(3, 1)
    h = sqa.SQA(ME, J, -2, 5.0, 1, 1, 65536, 3.0, 0.1, 1)
    hs = [h] * 32
    with pytest.raises(sqa.SqaError) as e:
        sqa.sqa_anneal_batch_noalloc(hs)
    assert e.value.status == sqa.SQA_ERR_UNSUPPORTED
    assert "static scratch" in str(e.value)
    h2 = sqa.SQA(ME, J, -2, 5.0, 1, 1, 3, 3.0, 0.1, 1)
    sqa.sqa_anneal_batch_noalloc([h2])
    assert h2.spins().shape == (3, 1, 6)
