"""Failures the host can force without a GPU: an allocator that has no memory,
and arguments the library rejects before it allocates anything.  Every case
here returns before the library makes a HIP call, so it runs on the CPU."""
import ctypes as C
import os

import numpy as np
import pytest

from paper_1603_03755_amd.workloads import LHZ, ME, MEC, sk_instance

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
LIB = os.path.join(ROOT, "paper_1603_03755_amd", "libsqa.so")
pytestmark = pytest.mark.skipif(not os.path.exists(LIB), reason="library not built")


@pytest.fixture(scope="module")
def sqa():
    from paper_1603_03755_amd import sqa as s
    s.lib()
    return s


def _args(kind=ME, n=6, L=8, sweeps=10, R=4, pen=-2, J=None, h=None, beta=5.0):
    return dict(kind=kind, J=sk_instance(n, 11) if J is None else J, penalty=pen, beta=beta, slices=L, sweeps=sweeps,
                replicas=R, gamma_start=3.0, gamma_end=0.1, seed=1, h=h)


@pytest.mark.parametrize("kind,n", [(ME, 6), (LHZ, 9), (MEC, 12)])
def test_allocator_returning_null_gives_oom_and_leaves_nothing(sqa, kind, n):
    """An allocator with no memory: sqa_create reports SQA_ERR_OOM, returns no
    handle, and holds nothing of the allocator's."""
    freed = []
    a = sqa.CallbackAllocator(lambda nbytes: None, lambda p: freed.append(p))
    with pytest.raises(sqa.SqaError) as e:
        sqa.SQA(allocator=a, **_args(kind=kind, n=n))
    assert e.value.status == sqa.SQA_ERR_OOM
    assert "allocator returned NULL" in str(e.value)
    assert a.calls == 1 and a.failures == 1 and a.live == {} and freed == []
    # the library stays usable: the next failing create reports the same way
    with pytest.raises(sqa.SqaError) as e:
        sqa.SQA(allocator=a, **_args(kind=kind, n=n, R=7))
    assert e.value.status == sqa.SQA_ERR_OOM and a.calls == 2


def test_allocator_raising_counts_as_no_memory(sqa):
    def boom(nbytes):
        raise MemoryError("no device memory")

    a = sqa.CallbackAllocator(boom, lambda p: None)
    with pytest.raises(sqa.SqaError) as e:
        sqa.SQA(allocator=a, **_args())
    assert e.value.status == sqa.SQA_ERR_OOM


def test_allocator_without_both_callbacks_is_rejected(sqa):
    from paper_1603_03755_amd.sqa import ALLOC_FN, FREE_FN, sqa_allocator, sqa_embedding, sqa_schedule, make_problem
    prob, keep = make_problem(sk_instance(5, 3))
    emb = sqa_embedding(ME, -2)
    sched = sqa_schedule(5.0, 8, 10, 4, 3.0, 0.1, None, None, 1, 0)
    half = sqa_allocator(ALLOC_FN(lambda n, c: None), FREE_FN(), None)   # free is NULL
    out = C.c_void_p()
    st = sqa.lib().sqa_create(C.byref(prob), C.byref(emb), C.byref(sched), C.byref(half), C.byref(out))
    assert st == sqa.SQA_ERR_INVALID and not out.value


@pytest.mark.parametrize("case,status", [
    (dict(L=3), "INVALID"),                       # odd slice count above 1
    (dict(L=66), "UNSUPPORTED"),                  # more than 64 slices
    (dict(R=0), "INVALID"),
    (dict(sweeps=0), "INVALID"),
    (dict(beta=0.0), "INVALID"),
    (dict(kind=LHZ, n=2), "INVALID"),             # LHZ needs n >= 3
    (dict(kind=ME, n=1), "INVALID"),
    (dict(kind=LHZ, n=5, h=[1, 0, 0, 0, 0]), "UNSUPPORTED"),   # logical fields need an ancilla
    (dict(kind=LHZ, n=6, pen=-200), "UNSUPPORTED"),            # field sum above 255 at a site
    (dict(kind=7, n=5), "INVALID"),               # unknown embedding
])
def test_invalid_arguments_rejected_before_any_allocation(sqa, case, status):
    a = sqa.CallbackAllocator(lambda nbytes: None, lambda p: None)
    with pytest.raises(sqa.SqaError) as e:
        sqa.SQA(allocator=a, **_args(**case))
    assert e.value.status == getattr(sqa, "SQA_ERR_" + status)
    assert a.calls == 0


def test_negative_gamma_and_nonfinite_schedule_rejected(sqa):
    a = sqa.CallbackAllocator(lambda nbytes: None, lambda p: None)
    for g in ([3.0, -0.1, 0.0], [np.nan, 1.0, 0.5]):
        with pytest.raises(sqa.SqaError) as e:
            sqa.SQA(allocator=a, gamma=np.array(g), **_args(sweeps=3))
        assert e.value.status == sqa.SQA_ERR_INVALID
    with pytest.raises(sqa.SqaError) as e:
        sqa.SQA(allocator=a, bscale=np.array([1.0, np.inf, 1.0]), **_args(sweeps=3))
    assert e.value.status == sqa.SQA_ERR_INVALID
    assert a.calls == 0
