"""The C-ABI library loads and exports every function include/sqa.h declares
(no compute calls: this runs without a GPU)."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "sqa.h")
LIB = os.path.join(ROOT, "paper_1603_03755_amd", "libsqa.so")


def declared():
    text = open(HEADER).read()
    return sorted(set(re.findall(r"SQA_API\s+[\w\s\*]*?\b((?:sqa|pt)_\w+)\s*\(", text)))


def test_header_declares_the_boundary():
    names = declared()
    for must in ("sqa_create", "sqa_anneal", "sqa_anneal_batch", "sqa_decode", "pt_run", "sqa_server_submit",
                 "sqa_destroy", "sqa_last_error"):
        assert must in names
    assert len(names) >= 35


@pytest.mark.skipif(not os.path.exists(LIB), reason="library not built")
def test_library_exports_every_declared_symbol():
    lib = ctypes.CDLL(LIB)
    missing = [n for n in declared() if not hasattr(lib, n)]
    assert not missing, missing


@pytest.mark.skipif(not os.path.exists(LIB), reason="library not built")
def test_library_exports_nothing_else():
    out = os.popen(f"nm -D --defined-only {LIB}").read()
    exported = {ln.split()[-1] for ln in out.splitlines() if " T " in ln}
    assert exported <= set(declared()), sorted(exported - set(declared()))


@pytest.mark.skipif(not os.path.exists(LIB), reason="library not built")
def test_host_only_queries():
    from paper_1603_03755_amd import sqa
    assert sqa.sqa_physical_sites(sqa.SQA_EMB_ME, 24) == 552
    assert sqa.sqa_physical_sites(sqa.SQA_EMB_LHZ, 24) == 276
    assert sqa.sqa_physical_sites(sqa.SQA_EMB_LHZ, 2) == -1
    assert b"gfx950" in sqa.lib().sqa_version()


@pytest.mark.skipif(not os.path.exists(LIB), reason="library not built")
def test_random_trees_match_oracle_on_host():
    """Tree generation is host code: the library's Pruefer trees equal the oracle's."""
    import numpy as np
    import oracle as O
    from paper_1603_03755_amd import sqa
    for n in (2, 3, 8, 17):
        assert (sqa.sqa_random_trees(99, n, 12) == O.random_trees(99, n, 12)).all()


CALIB_LIB = os.path.join(ROOT, "paper_1603_03755_amd", "libsqa_calib.so")


@pytest.mark.skipif(not os.path.exists(CALIB_LIB), reason="calibration probe not built")
def test_valu_calibration_probe_is_separate_and_rejects_bad_arguments_on_host():
    """The benchmark's issue-rate probe lives in its own library, not in the
    library's interface; argument errors are reported before any device call."""
    import ctypes as C
    import bench
    assert "sqa_valu_calibrate" not in declared()
    out = os.popen(f"nm -D --defined-only {LIB}").read()
    assert "calib" not in out
    L = bench.calib_lib()
    ms, instr = C.c_float(), C.c_double()
    for op, iters in ((3, 10), (-1, 10), (0, 0)):
        assert L.sqa_calib_valu_issue(op, iters, C.byref(ms), C.byref(instr)) == 1
