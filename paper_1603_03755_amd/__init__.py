"""MI355X (gfx950) simulated quantum annealing and parallel tempering over
minor-embedded and LHZ-embedded all-to-all Ising problems
(arXiv:1603.03755).

The compute path is the C-ABI library libsqa.so (include/sqa.h); `sqa` is its
ctypes binding.  Import `paper_1603_03755_amd.sqa` to use it; this package
module itself loads nothing so that input generators can be used without a GPU.
"""
__all__ = ["sqa", "workloads", "build"]
