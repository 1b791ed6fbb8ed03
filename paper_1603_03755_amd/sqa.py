"""ctypes binding of libsqa.so (C ABI in include/sqa.h).

Every function here only marshals arguments: device work, tables and
decoding all happen in the library.  Import fails loudly if the library has
not been built (python -m paper_1603_03755_amd.build); there is no CPU
fallback.
"""
from __future__ import annotations

import ctypes as C
import os
from typing import Optional, Sequence

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
# SQA_LIBRARY names another build of the library (the sanitizer build of the host
# code, build.build_host_sanitized); default: libsqa.so beside this file.
LIB_PATH = os.environ.get("SQA_LIBRARY") or os.path.join(_HERE, "libsqa.so")

SQA_OK, SQA_ERR_INVALID, SQA_ERR_OOM, SQA_ERR_DEVICE, SQA_ERR_UNSUPPORTED, SQA_ERR_BUSY, SQA_ERR_NOT_READY = \
    0, -1, -2, -3, -4, -5, -6
SQA_ERR_CANCELLED = -7
SQA_EMB_ME, SQA_EMB_LHZ, SQA_EMB_ME_CHIMERA = 0, 1, 2
SQA_DEC_ME_MAJORITY, SQA_DEC_LHZ_TREES, SQA_DEC_LHZ_MWD, SQA_DEC_LHZ_MLD, SQA_DEC_LHZ_BP = 0, 1, 2, 3, 4
SQA_MOVE_METROPOLIS, SQA_MOVE_WOLFF = 0, 1


class SqaError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"sqa status {status}: {msg}")
        self.status = status


class sqa_problem(C.Structure):
    _fields_ = [("n", C.c_int32), ("J", C.POINTER(C.c_int32)), ("h", C.POINTER(C.c_int32))]


class sqa_embedding(C.Structure):
    _fields_ = [("kind", C.c_int32), ("penalty", C.c_int32)]


class sqa_schedule(C.Structure):
    _fields_ = [("beta", C.c_double), ("slices", C.c_int32), ("sweeps", C.c_int32), ("replicas", C.c_int32),
                ("gamma_start", C.c_double), ("gamma_end", C.c_double),
                ("gamma", C.POINTER(C.c_double)), ("bscale", C.POINTER(C.c_double)), ("seed", C.c_uint64),
                ("move", C.c_int32)]


class sqa_decode_params(C.Structure):
    _fields_ = [("decoder", C.c_int32), ("readout_slice", C.c_int32), ("tree_parents", C.POINTER(C.c_int32)),
                ("n_trees", C.c_int32), ("error_rate", C.c_double), ("iterations", C.c_int32)]


class sqa_launch_config(C.Structure):
    _fields_ = [("waves_per_group", C.c_int32), ("groups_per_cu", C.c_int32)]


ALLOC_FN = C.CFUNCTYPE(C.c_void_p, C.c_size_t, C.c_void_p)
FREE_FN = C.CFUNCTYPE(None, C.c_void_p, C.c_void_p)


class sqa_allocator(C.Structure):
    _fields_ = [("alloc", ALLOC_FN), ("free", FREE_FN), ("ctx", C.c_void_p)]


class pt_params(C.Structure):
    _fields_ = [("beta_min", C.c_double), ("beta_max", C.c_double), ("temps", C.c_int32), ("sweeps", C.c_int32),
                ("sweeps_per_swap", C.c_int32), ("seed", C.c_uint64)]


_lib = None
_VP = C.c_void_p
_PVP = C.POINTER(C.c_void_p)
_SIGS = {
    "sqa_create": (C.c_int, [C.POINTER(sqa_problem), C.POINTER(sqa_embedding), C.POINTER(sqa_schedule),
                             C.POINTER(sqa_allocator), _PVP]),
    "sqa_handle_device_bytes": (C.c_int, [_VP, C.POINTER(C.c_size_t)]),
    "sqa_anneal": (C.c_int, [_VP, _VP]),
    "sqa_anneal_range": (C.c_int, [_VP, C.c_int32, C.c_int32, _VP]),
    "sqa_reset": (C.c_int, [_VP, _VP]),
    "sqa_sync": (C.c_int, [_VP]),
    "sqa_read_spins": (C.c_int, [_VP, _VP, C.c_size_t]),
    "sqa_read_energies": (C.c_int, [_VP, _VP, C.c_size_t]),
    "sqa_write_spins": (C.c_int, [_VP, _VP, C.c_size_t]),
    "sqa_device_spins": (_VP, [_VP]),
    "sqa_device_energies": (_VP, [_VP]),
    "sqa_decode": (C.c_int, [_VP, C.c_int32, C.c_int32, _VP, C.c_int32, _VP, _VP]),
    "sqa_decode_ex": (C.c_int, [_VP, C.POINTER(sqa_decode_params), _VP, _VP, _VP]),
    "sqa_device_logical": (_VP, [_VP]),
    "sqa_device_logical_energies": (_VP, [_VP]),
    "sqa_read_logical": (C.c_int, [_VP, _VP, C.c_size_t, _VP, C.c_size_t]),
    "sqa_ground_state": (C.c_int, [C.POINTER(sqa_problem), C.POINTER(C.c_int32), _VP]),
    "sqa_random_trees": (C.c_int, [C.c_uint64, C.c_int32, C.c_int32, _VP]),
    "sqa_export_table": (C.c_int, [_VP, _VP, C.c_size_t, C.POINTER(C.c_int32)]),
    "sqa_export_wolff_tables": (C.c_int, [_VP, _VP, C.c_size_t, _VP, C.c_size_t, C.POINTER(C.c_int32),
                                          C.POINTER(C.c_int32)]),
    "sqa_physical_sites": (C.c_int64, [C.c_int32, C.c_int32]),
    "sqa_handle_info": (C.c_int, [_VP] + [C.POINTER(C.c_int32)] * 5),
    "sqa_destroy": (None, [_VP]),
    "sqa_batch_create": (C.c_int, [_PVP, C.c_int32, C.POINTER(sqa_launch_config), _PVP]),
    "sqa_batch_create_decoded": (C.c_int, [_PVP, C.c_int32, C.POINTER(sqa_launch_config),
                                           C.POINTER(sqa_decode_params), _PVP]),
    "sqa_batch_run": (C.c_int, [_VP, _VP]),
    "sqa_batch_timing": (C.c_int, [_VP, C.POINTER(C.c_float), C.POINTER(C.c_float)]),
    "sqa_batch_config": (C.c_int, [_VP, C.POINTER(sqa_launch_config)]),
    "sqa_batch_destroy": (None, [_VP]),
    "sqa_anneal_batch": (C.c_int, [_PVP, C.c_int32, _VP]),
    "sqa_anneal_batch_noalloc": (C.c_int, [_PVP, C.c_int32, _VP]),
    "sqa_autotune": (C.c_int, [_PVP, C.c_int32, C.c_char_p, C.POINTER(sqa_launch_config)]),
    "pt_create": (C.c_int, [C.POINTER(sqa_problem), C.POINTER(sqa_embedding), C.POINTER(pt_params), _PVP]),
    "pt_run_handle": (C.c_int, [_VP, _VP]),
    "pt_run_batch": (C.c_int, [_PVP, C.c_int32, _VP]),
    "pt_read": (C.c_int, [_VP, _VP, C.c_size_t, _VP, _VP, _VP]),
    "pt_destroy": (None, [_VP]),
    "pt_run": (C.c_int, [C.POINTER(sqa_problem), C.POINTER(sqa_embedding), C.POINTER(pt_params), _VP, _VP,
                         C.c_size_t, _VP, _VP, _VP]),
    "sqa_server_create": (C.c_int, [C.c_size_t, C.c_int32, C.c_int32, C.POINTER(sqa_allocator), _PVP]),
    "sqa_server_submit": (C.c_int, [_VP, C.POINTER(sqa_problem), C.POINTER(sqa_embedding), C.POINTER(sqa_schedule),
                                    C.POINTER(sqa_decode_params), C.POINTER(C.c_uint64)]),
    "sqa_server_job_bytes": (C.c_int, [_VP, C.c_uint64, C.POINTER(C.c_size_t)]),
    "sqa_server_cancel": (C.c_int, [_VP, C.c_uint64]),
    "sqa_server_poll": (C.c_int, [_VP, C.c_uint64, C.POINTER(C.c_int32)]),
    "sqa_server_wait": (C.c_int, [_VP, C.c_uint64, C.c_int32]),
    "sqa_server_result": (C.c_int, [_VP, C.c_uint64, _VP, C.c_size_t, _VP, C.c_size_t, _VP, C.c_size_t, _VP,
                                    C.c_size_t, C.POINTER(C.c_double)]),
    "sqa_server_stats": (C.c_int, [_VP] + [C.POINTER(C.c_uint64)] * 3),
    "sqa_server_destroy": (None, [_VP]),
    "sqa_last_error": (C.c_char_p, []),
    "sqa_version": (C.c_char_p, []),
}


# Launch shapes chosen by sqa_autotune for this package's benchmark batches on
# gfx950 (written by `python -m paper_1603_03755_amd.autotune`).  Batches created
# with an automatic shape look their shape class up here unless the environment
# names another cache file.
TUNING_CACHE = os.path.join(os.path.dirname(os.path.abspath(__file__)), "autotune_gfx950.json")


def lib():
    """The loaded library; raises if it has not been built."""
    global _lib
    if _lib is None:
        if os.path.exists(TUNING_CACHE):
            os.environ.setdefault("SQA_AUTOTUNE_CACHE", TUNING_CACHE)
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: build it with `python -m paper_1603_03755_amd.build`")
        L = C.CDLL(LIB_PATH)
        for name, (res, args) in _SIGS.items():
            f = getattr(L, name)
            f.restype = res
            f.argtypes = args
        _lib = L
    return _lib


def _check(st: int):
    if st != SQA_OK:
        msg = lib().sqa_last_error()
        raise SqaError(st, msg.decode() if msg else "")


def _ptr(a: Optional[np.ndarray]):
    return None if a is None else C.c_void_p(a.ctypes.data)


def _stream(stream) -> Optional[int]:
    """Accepts None, an int hipStream_t, or a torch.cuda.Stream."""
    if stream is None:
        return None
    if hasattr(stream, "cuda_stream"):
        return C.c_void_p(stream.cuda_stream)
    return C.c_void_p(int(stream))


def make_problem(J, h=None):
    J = np.ascontiguousarray(J, dtype=np.int32)
    hh = None if h is None else np.ascontiguousarray(h, dtype=np.int32)
    p = sqa_problem(J.shape[0], J.ctypes.data_as(C.POINTER(C.c_int32)),
                    hh.ctypes.data_as(C.POINTER(C.c_int32)) if hh is not None else None)
    return p, (J, hh)


# ---------------------------------------------------------------- allocators
class CallbackAllocator:
    """An sqa_allocator whose callbacks are Python functions: alloc(nbytes) -> device
    address (int) or None, free(address).  It counts live allocations and bytes.
    Keep the object alive while anything created with it lives."""

    def __init__(self, alloc, free):
        self._alloc_py, self._free_py = alloc, free
        self.live = {}
        self.calls = 0
        self.failures = 0

        def _a(nbytes, ctx):
            self.calls += 1
            try:
                p = self._alloc_py(int(nbytes))
            except Exception:
                p = None
            if not p:
                self.failures += 1
                return None
            self.live[int(p)] = int(nbytes)
            return int(p)

        def _f(ptr, ctx):
            if ptr:
                self.live.pop(int(ptr), None)
                self._free_py(int(ptr))

        self._afn, self._ffn = ALLOC_FN(_a), FREE_FN(_f)
        self.struct = sqa_allocator(self._afn, self._ffn, None)

    @property
    def live_bytes(self) -> int:
        return sum(self.live.values())


class TorchAllocator(CallbackAllocator):
    """Device memory from torch's caching allocator on `device` (default: the
    current one), tied to that device's default stream; the library frees a
    buffer only after its own queued work on it has finished."""

    def __init__(self, device=None):
        import torch
        dev = torch.cuda.current_device() if device is None else int(device)
        stream = torch.cuda.default_stream(dev)
        super().__init__(lambda n: torch.cuda.caching_allocator_alloc(n, dev, stream),
                         lambda p: torch.cuda.caching_allocator_delete(p))


def _alloc_ptr(allocator):
    return None if allocator is None else C.byref(allocator.struct)


# ---------------------------------------------------------------- SQA handle
class SQA:
    """One problem x embedding x schedule on the GPU (sqa_create / sqa_destroy)."""

    def __init__(self, kind: int, J, penalty: int, beta: float, slices: int, sweeps: int, replicas: int,
                 gamma_start: float, gamma_end: float, seed: int, h=None, gamma=None, bscale=None,
                 move: int = SQA_MOVE_METROPOLIS, allocator: Optional[CallbackAllocator] = None):
        prob, self._keep = make_problem(J, h)
        self.allocator = allocator
        g = None if gamma is None else np.ascontiguousarray(gamma, dtype=np.float64)
        b = None if bscale is None else np.ascontiguousarray(bscale, dtype=np.float64)
        sched = sqa_schedule(beta, slices, sweeps, replicas, gamma_start, gamma_end,
                             g.ctypes.data_as(C.POINTER(C.c_double)) if g is not None else None,
                             b.ctypes.data_as(C.POINTER(C.c_double)) if b is not None else None, seed, move)
        emb = sqa_embedding(kind, penalty)
        out = C.c_void_p()
        _check(lib().sqa_create(C.byref(prob), C.byref(emb), C.byref(sched), _alloc_ptr(allocator), C.byref(out)))
        self.h = out
        self.kind, self.N, self.move = kind, int(np.asarray(J).shape[0]), move
        vals = [C.c_int32() for _ in range(5)]
        _check(lib().sqa_handle_info(self.h, *[C.byref(v) for v in vals]))
        self.sites, self.slices, self.replicas, self.sweeps, self.fmax = [v.value for v in vals]

    def close(self):
        if getattr(self, "h", None):
            lib().sqa_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def anneal(self, stream=None):
        _check(lib().sqa_anneal(self.h, _stream(stream)))
        return self

    def anneal_range(self, m0: int, m1: int, stream=None):
        _check(lib().sqa_anneal_range(self.h, m0, m1, _stream(stream)))
        return self

    def reset(self, stream=None):
        _check(lib().sqa_reset(self.h, _stream(stream)))

    def sync(self):
        _check(lib().sqa_sync(self.h))

    def spins(self) -> np.ndarray:
        out = np.empty((self.replicas, self.slices, self.sites), dtype=np.int8)
        _check(lib().sqa_read_spins(self.h, _ptr(out), out.size))
        return out

    def energies(self) -> np.ndarray:
        out = np.empty((self.replicas, self.slices), dtype=np.int32)
        _check(lib().sqa_read_energies(self.h, _ptr(out), out.size))
        return out

    def write_spins(self, s):
        s = np.ascontiguousarray(s, dtype=np.int8)
        _check(lib().sqa_write_spins(self.h, _ptr(s), s.size))

    def table(self):
        F = C.c_int32()
        _check(lib().sqa_export_table(self.h, None, 0, C.byref(F)))
        out = np.empty((self.sweeps, 2 * F.value + 1, 3), dtype=np.uint32)
        _check(lib().sqa_export_table(self.h, _ptr(out), out.size, C.byref(F)))
        return out

    def wolff_tables(self):
        """(join thresholds [sweeps], acceptance thresholds [rows][2 L F + 1]) of a Wolff handle."""
        rows, width = C.c_int32(), C.c_int32()
        _check(lib().sqa_export_wolff_tables(self.h, None, 0, None, 0, C.byref(rows), C.byref(width)))
        padd = np.empty(self.sweeps, dtype=np.uint32)
        acc = np.empty((rows.value, width.value), dtype=np.uint32)
        _check(lib().sqa_export_wolff_tables(self.h, _ptr(padd), padd.size, _ptr(acc), acc.size, C.byref(rows),
                                             C.byref(width)))
        return padd, acc

    def decode(self, decoder: int, readout_slice: int = 0, trees=None, error_rate: float = 0.2,
               iterations: int = 10, stream=None, host: bool = True):
        """Decodes slice `readout_slice` of every replica (sqa_decode_ex).  host=False queues
        the decoder on `stream` and leaves the results in device memory."""
        t = None if trees is None else np.ascontiguousarray(trees, dtype=np.int32).reshape(-1, self.N)
        p = sqa_decode_params(decoder, readout_slice,
                              t.ctypes.data_as(C.POINTER(C.c_int32)) if t is not None else None,
                              0 if t is None else t.shape[0], error_rate, iterations)
        if not host:
            _check(lib().sqa_decode_ex(self.h, C.byref(p), None, None, _stream(stream)))
            return None
        logical = np.empty((self.replicas, self.N), dtype=np.int8)
        energy = np.empty(self.replicas, dtype=np.int32)
        _check(lib().sqa_decode_ex(self.h, C.byref(p), _ptr(logical), _ptr(energy), _stream(stream)))
        return logical, energy

    def logical(self):
        """(logical states, logical energies) of the last decode, after waiting for it."""
        q = np.empty((self.replicas, self.N), dtype=np.int8)
        E = np.empty(self.replicas, dtype=np.int32)
        _check(lib().sqa_read_logical(self.h, _ptr(q), q.size, _ptr(E), E.size))
        return q, E

    def device_spins(self) -> int:
        return lib().sqa_device_spins(self.h)

    def device_bytes(self) -> int:
        """Device bytes the handle holds through its allocator."""
        b = C.c_size_t()
        _check(lib().sqa_handle_device_bytes(self.h, C.byref(b)))
        return b.value


def sqa_random_trees(seed: int, n: int, n_trees: int) -> np.ndarray:
    out = np.empty((n_trees, n), dtype=np.int32)
    _check(lib().sqa_random_trees(seed, n, n_trees, _ptr(out)))
    return out


def sqa_ground_state(J, h=None):
    """(ground energy, one ground state) of the logical problem, exhaustive on the device."""
    prob, keep = make_problem(J, h)
    n = int(np.asarray(J).shape[0])
    E = C.c_int32()
    state = np.empty(n, dtype=np.int8)
    _check(lib().sqa_ground_state(C.byref(prob), C.byref(E), _ptr(state)))
    return int(E.value), state


def sqa_physical_sites(kind: int, n: int) -> int:
    return int(lib().sqa_physical_sites(kind, n))


def _handle_array(handles: Sequence[SQA]):
    arr = (C.c_void_p * len(handles))(*[h.h.value for h in handles])
    return arr


def decode_params(decoder: int, readout_slice: int = 0, trees=None, n: int = 0, error_rate: float = 0.2,
                  iterations: int = 10):
    """An sqa_decode_params (decoder -1 = none) and the tree array it points into."""
    t = None if trees is None else np.ascontiguousarray(trees, dtype=np.int32).reshape(-1, n)
    p = sqa_decode_params(decoder, readout_slice, t.ctypes.data_as(C.POINTER(C.c_int32)) if t is not None else None,
                          0 if t is None else t.shape[0], error_rate, iterations)
    return p, t


class Batch:
    """All handles' full anneals in one persistent launch, replayed from a HIP graph;
    with `decoders` (one (decoder, readout slice[, trees]) per handle, or None for a
    handle), each handle's decoder runs in the same graph after the anneal."""

    def __init__(self, handles: Sequence[SQA], waves_per_group: int = 0, groups_per_cu: int = 0, decoders=None):
        self.handles = list(handles)
        self._arr = _handle_array(self.handles)
        cfg = sqa_launch_config(waves_per_group, groups_per_cu)
        out = C.c_void_p()
        if decoders is None:
            _check(lib().sqa_batch_create(C.cast(self._arr, _PVP), len(self.handles), C.byref(cfg), C.byref(out)))
        else:
            arr = (sqa_decode_params * len(self.handles))()
            keep = []
            for i, (h, d) in enumerate(zip(self.handles, decoders)):
                if d is None:
                    arr[i] = sqa_decode_params(-1, 0, None, 0, 0.2, 10)
                    continue
                p, t = decode_params(d[0], d[1] if len(d) > 1 else 0, d[2] if len(d) > 2 else None, h.N)
                arr[i] = p
                keep.append(t)
            _check(lib().sqa_batch_create_decoded(C.cast(self._arr, _PVP), len(self.handles), C.byref(cfg), arr,
                                                  C.byref(out)))
        self.b = out

    def run(self, stream=None):
        _check(lib().sqa_batch_run(self.b, _stream(stream)))

    def config(self):
        c = sqa_launch_config()
        _check(lib().sqa_batch_config(self.b, C.byref(c)))
        return c.waves_per_group, c.groups_per_cu

    def timing(self):
        """(anneal ms, decode ms) of the last run, from HIP events on its stream."""
        a, d = C.c_float(), C.c_float()
        _check(lib().sqa_batch_timing(self.b, C.byref(a), C.byref(d)))
        return a.value, d.value

    def close(self):
        if getattr(self, "b", None):
            lib().sqa_batch_destroy(self.b)
            self.b = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def sqa_anneal_batch(handles: Sequence[SQA], stream=None):
    arr = _handle_array(handles)
    _check(lib().sqa_anneal_batch(C.cast(arr, _PVP), len(handles), _stream(stream)))


def sqa_anneal_batch_noalloc(handles: Sequence[SQA], stream=None):
    """sqa_anneal_batch without allocating: the launch scratch is the library's static array."""
    arr = _handle_array(handles)
    _check(lib().sqa_anneal_batch_noalloc(C.cast(arr, _PVP), len(handles), _stream(stream)))


def sqa_autotune(handles: Sequence[SQA], cache_path: Optional[str] = None):
    arr = _handle_array(handles)
    best = sqa_launch_config()
    _check(lib().sqa_autotune(C.cast(arr, _PVP), len(handles), cache_path.encode() if cache_path else None,
                              C.byref(best)))
    return best.waves_per_group, best.groups_per_cu


# ---------------------------------------------------------------- PT
class PT:
    def __init__(self, kind: int, J, penalty: int, beta_min: float, beta_max: float, temps: int, sweeps: int,
                 sweeps_per_swap: int, seed: int, h=None):
        prob, self._keep = make_problem(J, h)
        emb = sqa_embedding(kind, penalty)
        p = pt_params(beta_min, beta_max, temps, sweeps, sweeps_per_swap, seed)
        out = C.c_void_p()
        _check(lib().pt_create(C.byref(prob), C.byref(emb), C.byref(p), C.byref(out)))
        self.h = out
        self.temps = temps
        self.sites = sqa_physical_sites(kind, int(np.asarray(J).shape[0]))

    def run(self, stream=None):
        _check(lib().pt_run_handle(self.h, _stream(stream)))
        return self

    def read(self):
        spins = np.empty((self.temps, self.sites), dtype=np.int8)
        E = np.empty(self.temps, dtype=np.int32)
        rep = np.empty(self.temps, dtype=np.int32)
        acc = np.zeros(max(self.temps - 1, 1), dtype=np.uint64)
        _check(lib().pt_read(self.h, _ptr(spins), spins.size, _ptr(E), _ptr(rep), _ptr(acc)))
        return spins, E, rep, acc[:max(self.temps - 1, 0)]

    def close(self):
        if getattr(self, "h", None):
            lib().pt_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def pt_run_batch(handles: Sequence[PT], stream=None):
    arr = (C.c_void_p * len(handles))(*[h.h.value for h in handles])
    _check(lib().pt_run_batch(C.cast(arr, _PVP), len(handles), _stream(stream)))


# ---------------------------------------------------------------- server
class Server:
    """Continuous-batching server (sqa_server_*).  `allocator` supplies its device
    memory (None = hipMalloc)."""

    def __init__(self, hbm_budget_bytes: int, max_slots: int, chunk_sweeps: int,
                 allocator: Optional[CallbackAllocator] = None):
        out = C.c_void_p()
        self.allocator = allocator
        _check(lib().sqa_server_create(hbm_budget_bytes, max_slots, chunk_sweeps, _alloc_ptr(allocator),
                                       C.byref(out)))
        self.s = out
        self._keep = {}

    def submit(self, kind, J, penalty, beta, slices, sweeps, replicas, gamma_start, gamma_end, seed, h=None,
               move: int = SQA_MOVE_METROPOLIS, decoder: Optional[int] = None, readout_slice: int = 0,
               trees=None, error_rate: float = 0.2, iterations: int = 10) -> int:
        """Queues a job; `decoder` None = the default decoder for the embedding."""
        prob, keep = make_problem(J, h)
        n = int(np.asarray(J).shape[0])
        emb = sqa_embedding(kind, penalty)
        sched = sqa_schedule(beta, slices, sweeps, replicas, gamma_start, gamma_end, None, None, seed, move)
        dp = None
        if decoder is not None:
            t = None if trees is None else np.ascontiguousarray(trees, dtype=np.int32).reshape(-1, n)
            dp = sqa_decode_params(decoder, readout_slice,
                                   t.ctypes.data_as(C.POINTER(C.c_int32)) if t is not None else None,
                                   0 if t is None else t.shape[0], error_rate, iterations)
        t = C.c_uint64()
        _check(lib().sqa_server_submit(self.s, C.byref(prob), C.byref(emb), C.byref(sched),
                                       C.byref(dp) if dp is not None else None, C.byref(t)))
        self._keep[t.value] = (replicas, slices, sqa_physical_sites(kind, n), n)
        return t.value

    def job_bytes(self, ticket: int) -> int:
        b = C.c_size_t()
        _check(lib().sqa_server_job_bytes(self.s, ticket, C.byref(b)))
        return b.value

    def cancel(self, ticket: int):
        _check(lib().sqa_server_cancel(self.s, ticket))

    def poll(self, ticket: int) -> bool:
        d = C.c_int32()
        _check(lib().sqa_server_poll(self.s, ticket, C.byref(d)))
        return bool(d.value)

    def wait(self, ticket: int, timeout_ms: int = -1):
        _check(lib().sqa_server_wait(self.s, ticket, timeout_ms))

    def result(self, ticket: int, logical: bool = False):
        """(spins, energies, latency) or, with logical=True, (spins, energies, decoded
        logical states, their energies, latency)."""
        R, L, n, N = self._keep[ticket]
        spins = np.empty((R, L, n), dtype=np.int8)
        E = np.empty((R, L), dtype=np.int32)
        q = np.empty((R, N), dtype=np.int8)
        qE = np.empty(R, dtype=np.int32)
        lat = C.c_double()
        st = lib().sqa_server_result(self.s, ticket, _ptr(spins), spins.size, _ptr(E), E.size, _ptr(q), q.size,
                                     _ptr(qE), qE.size, C.byref(lat))
        if st != SQA_ERR_NOT_READY:
            self._keep.pop(ticket, None)
        _check(st)
        return (spins, E, q, qE, lat.value) if logical else (spins, E, lat.value)

    def stats(self):
        v = [C.c_uint64() for _ in range(3)]
        _check(lib().sqa_server_stats(self.s, *[C.byref(x) for x in v]))
        return tuple(x.value for x in v)

    def close(self):
        if getattr(self, "s", None):
            lib().sqa_server_destroy(self.s)
            self.s = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
