"""Python view of the CPU oracle (test infrastructure only).

The oracle is a plain C statement of the method (liboracle.so, built by
oracle/build.sh).  Only the tests, the package's smoke check and the CPU
baseline leg of the benchmark use it; the GPU library never does.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
# SQA_ORACLE_LIB names another build of the same sources (the sanitizer build of
# oracle/build_sanitized.sh); default: liboracle.so beside this file.
_LIB_PATH = os.environ.get("SQA_ORACLE_LIB") or os.path.join(_HERE, "liboracle.so")
_lib = None

ME, LHZ, MEC = 0, 1, 2
STREAM_INIT, STREAM_SQA, STREAM_PT, STREAM_SWAP, STREAM_TREE, STREAM_PT_INIT, STREAM_WOLFF = 1, 2, 3, 4, 5, 6, 7
STREAM_SQA_LO, STREAM_WOLFF_LO, STREAM_PT_LO = 8, 9, 10
ALWAYS = 0xFFFFFFFF


def build() -> None:
    subprocess.run(["sh", os.path.join(_HERE, "build.sh")], check=True)


class OEmb(C.Structure):
    _fields_ = [("kind", C.c_int32), ("N", C.c_int32), ("n_sites", C.c_int32),
                ("n_terms", C.c_int32), ("fmax", C.c_int32), ("emax", C.c_int32),
                ("h", C.POINTER(C.c_int32)), ("colour", C.POINTER(C.c_int32)),
                ("w", C.POINTER(C.c_int32)), ("arity", C.POINTER(C.c_int32)),
                ("tsite", C.POINTER(C.c_int32)), ("row", C.POINTER(C.c_int32)),
                ("inc", C.POINTER(C.c_int32))]


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB_PATH):
            build()
        _lib = C.CDLL(_LIB_PATH)
        L = _lib
        L.oracle_sqa_word.restype = C.c_uint32
        L.oracle_sqa_word.argtypes = [C.c_uint64, C.c_uint32, C.c_uint32, C.c_uint32, C.c_uint32, C.c_uint32]
        L.oracle_sqa_uniform.restype = C.c_uint32
        L.oracle_sqa_uniform.argtypes = [C.c_uint64, C.c_uint32, C.c_uint32, C.c_uint32, C.c_uint32]
        L.oracle_pt_word.restype = C.c_uint32
        L.oracle_pt_word.argtypes = [C.c_uint64, C.c_uint32, C.c_uint32, C.c_uint32, C.c_uint32]
        L.oracle_pt_uniform.restype = C.c_uint32
        L.oracle_pt_uniform.argtypes = [C.c_uint64, C.c_uint32, C.c_uint32, C.c_uint32]
        L.oracle_threshold.restype = C.c_uint32
        L.oracle_threshold.argtypes = [C.c_double]
        L.oracle_embed.restype = C.c_int
        L.oracle_local_field.restype = C.c_int32
        L.oracle_energy.restype = C.c_int32
        L.oracle_logical_energy.restype = C.c_int32
        L.oracle_sqa_sweep_order.restype = C.c_int32
        L.oracle_sqa_attempt_threshold.restype = C.c_uint32
        L.oracle_ground_states.restype = C.c_int32
        L.oracle_random_trees.restype = C.c_int
        L.oracle_me_site.restype = C.c_int32
        L.oracle_wolff_bond_uniform.restype = C.c_uint32
        L.oracle_wolff_bond_uniform.argtypes = [C.c_uint64, C.c_uint32, C.c_uint32, C.c_uint32, C.c_uint32]
        L.oracle_wolff_site_order.restype = C.c_int32
        L.oracle_lhz_site.restype = C.c_int32
    return _lib


def _p(a, ct):
    return a.ctypes.data_as(C.POINTER(ct))


def _i32(a):
    return np.ascontiguousarray(a, dtype=np.int32)


# ---------------------------------------------------------------- Philox
def philox4x32(ctr, key):
    c = np.ascontiguousarray(ctr, dtype=np.uint32)
    k = np.ascontiguousarray(key, dtype=np.uint32)
    out = np.zeros(4, dtype=np.uint32)
    lib().oracle_philox4x32(_p(c, C.c_uint32), _p(k, C.c_uint32), _p(out, C.c_uint32))
    return out


def philox4x64(ctr, key):
    c = np.ascontiguousarray(ctr, dtype=np.uint64)
    k = np.ascontiguousarray(key, dtype=np.uint64)
    out = np.zeros(4, dtype=np.uint64)
    lib().oracle_philox4x64(_p(c, C.c_uint64), _p(k, C.c_uint64), _p(out, C.c_uint64))
    return out


def sqa_word(seed, stream, replica, site, slice_, sweep) -> int:
    return int(lib().oracle_sqa_word(seed, stream, replica, site, slice_, sweep))


def sqa_uniform(seed, replica, site, slice_, sweep) -> int:
    """The 32-bit uniform of one Metropolis attempt (high half stream SQA, low half SQA_LO)."""
    return int(lib().oracle_sqa_uniform(seed, replica, site, slice_, sweep))


def pt_word(seed, stream, replica, site, sweep) -> int:
    return int(lib().oracle_pt_word(seed, stream, replica, site, sweep))


def pt_uniform(seed, replica, site, sweep) -> int:
    """The 32-bit uniform of one PT Metropolis attempt (high half stream PT, low half PT_LO)."""
    return int(lib().oracle_pt_uniform(seed, replica, site, sweep))


# ---------------------------------------------------------------- embeddings
class Embedding:
    """An embedded physical Hamiltonian built by the oracle."""

    def __init__(self, kind: int, J, penalty: int, h=None):
        J = _i32(J)
        N = J.shape[0]
        self.J = J
        self.h_logical = None if h is None else _i32(h)
        self._e = OEmb()
        hp = _p(self.h_logical, C.c_int32) if h is not None else None
        rc = lib().oracle_embed(kind, N, _p(J, C.c_int32), hp, penalty, C.byref(self._e))
        if rc != 0:
            raise ValueError("invalid embedding arguments")
        e = self._e
        n, t = e.n_sites, e.n_terms
        self.kind, self.N, self.n_sites, self.n_terms = kind, N, n, t
        self.fmax, self.emax = e.fmax, e.emax
        self.h = np.ctypeslib.as_array(e.h, (n,)).copy()
        self.colour = np.ctypeslib.as_array(e.colour, (n,)).copy()
        self.w = np.ctypeslib.as_array(e.w, (max(t, 1),))[:t].copy()
        self.arity = np.ctypeslib.as_array(e.arity, (max(t, 1),))[:t].copy()
        self.tsite = np.ctypeslib.as_array(e.tsite, (max(t, 1) * 4,))[:4 * t].reshape(t, 4).copy()
        self.row = np.ctypeslib.as_array(e.row, (n + 1,)).copy()
        self.inc = np.ctypeslib.as_array(e.inc, (max(int(self.row[-1]), 1),))[:int(self.row[-1])].copy()

    def __del__(self):
        try:
            lib().oracle_emb_free(C.byref(self._e))
        except Exception:
            pass

    @property
    def ptr(self):
        return C.byref(self._e)

    def local_field(self, s, k) -> int:
        s = np.ascontiguousarray(s, dtype=np.int8)
        return int(lib().oracle_local_field(self.ptr, _p(s, C.c_int8), k))

    def energy(self, s) -> int:
        s = np.ascontiguousarray(s, dtype=np.int8)
        return int(lib().oracle_energy(self.ptr, _p(s, C.c_int8)))


def me_site(N, i, r) -> int:
    return int(lib().oracle_me_site(N, i, r))


def chimera_m(N) -> int:
    return int(lib().oracle_chimera_m(N))


def chimera_site(N, i, t) -> int:
    """Physical site of slot t of chain i in the Chimera ME layout."""
    return int(lib().oracle_chimera_site(N, i, t))


def chimera_qubit(N, i, t):
    """(row, column, side (0 = vertical, 1 = horizontal), k) of slot t of chain i."""
    v = [C.c_int32() for _ in range(4)]
    lib().oracle_chimera_qubit(N, i, t, *[C.byref(x) for x in v])
    return tuple(int(x.value) for x in v)


def lhz_site(N, i, j) -> int:
    return int(lib().oracle_lhz_site(N, i, j))


def logical_energy(J, sigma, h=None) -> int:
    J = _i32(J)
    s = np.ascontiguousarray(sigma, dtype=np.int8)
    hp = _p(_i32(h), C.c_int32) if h is not None else None
    return int(lib().oracle_logical_energy(J.shape[0], _p(J, C.c_int32), hp, _p(s, C.c_int8)))


# ---------------------------------------------------------------- tables
def threshold(x: float) -> int:
    return int(lib().oracle_threshold(C.c_double(x)))


def gamma_schedule(g0, g1, M):
    out = np.zeros(M, dtype=np.float64)
    lib().oracle_gamma_schedule(C.c_double(g0), C.c_double(g1), M, _p(out, C.c_double))
    return out


def sqa_table(beta, L, gamma, F, bscale=None):
    gamma = np.ascontiguousarray(gamma, dtype=np.float64)
    M = gamma.shape[0]
    out = np.zeros((M, 2 * F + 1, 3), dtype=np.uint32)
    bp = None
    if bscale is not None:
        bscale = np.ascontiguousarray(bscale, dtype=np.float64)
        bp = _p(bscale, C.c_double)
    lib().oracle_sqa_table(C.c_double(beta), L, M, _p(gamma, C.c_double), bp, F, _p(out, C.c_uint32))
    return out


def pt_ladder(beta_min, beta_max, R):
    out = np.zeros(R, dtype=np.float64)
    lib().oracle_pt_ladder(C.c_double(beta_min), C.c_double(beta_max), R, _p(out, C.c_double))
    return out


def pt_table(betas, F):
    betas = np.ascontiguousarray(betas, dtype=np.float64)
    out = np.zeros((betas.shape[0], 2 * F + 1), dtype=np.uint32)
    lib().oracle_pt_table(_p(betas, C.c_double), betas.shape[0], F, _p(out, C.c_uint32))
    return out


def swap_table(betas, Dmax):
    betas = np.ascontiguousarray(betas, dtype=np.float64)
    R = betas.shape[0]
    out = np.zeros((max(R - 1, 1), Dmax + 1), dtype=np.uint32)
    lib().oracle_swap_table(_p(betas, C.c_double), R, Dmax, _p(out, C.c_uint32))
    return out[:max(R - 1, 0)]


# ---------------------------------------------------------------- SQA
def sqa_init(emb: Embedding, L, R, seed, r0=0):
    """Initial lattices of replicas r0..r0+R-1."""
    out = np.zeros((R, L, emb.n_sites), dtype=np.int8)
    lib().oracle_sqa_init_from(emb.ptr, L, r0, R, C.c_uint64(seed), _p(out, C.c_int8))
    return out


def sqa_sweep_order(emb: Embedding, L):
    n = emb.n_sites * L
    k = np.zeros(n, dtype=np.int32)
    t = np.zeros(n, dtype=np.int32)
    cnt = lib().oracle_sqa_sweep_order(emb.ptr, L, _p(k, C.c_int32), _p(t, C.c_int32))
    return k[:cnt], t[:cnt]


def sqa_attempt_threshold(emb: Embedding, L, table, lat, k, tau, m) -> int:
    table = np.ascontiguousarray(table, dtype=np.uint32)
    F = (table.shape[1] - 1) // 2
    lat = np.ascontiguousarray(lat, dtype=np.int8)
    return int(lib().oracle_sqa_attempt_threshold(emb.ptr, L, _p(table, C.c_uint32), F,
                                                  _p(lat, C.c_int8), k, tau, m))


def sqa_run(emb: Embedding, L, spins, m0, m1, table, seed, nthreads=1, r0=0):
    """Runs sweeps m0..m1-1 in place on spins[R][L][n] holding replicas r0..r0+R-1."""
    assert spins.dtype == np.int8 and spins.flags.c_contiguous
    table = np.ascontiguousarray(table, dtype=np.uint32)
    F = (table.shape[1] - 1) // 2
    lib().oracle_sqa_run_from(emb.ptr, L, r0, spins.shape[0], m0, m1, _p(table, C.c_uint32), F,
                              C.c_uint64(seed), _p(spins, C.c_int8), nthreads)
    return spins


def sqa_energies(emb: Embedding, spins):
    R, L, _ = spins.shape
    E = np.zeros((R, L), dtype=np.int32)
    s = np.ascontiguousarray(spins, dtype=np.int8)
    lib().oracle_sqa_energies(emb.ptr, L, R, _p(s, C.c_int8), _p(E, C.c_int32))
    return E


def sqa_anneal(kind, J, penalty, beta, L, sweeps, replicas, gamma0, gamma1, seed,
               h=None, gamma=None, bscale=None, nthreads=1, fmax=None, r0=0):
    """The whole single-instance SQA path: embed, tabulate, init, anneal, energies,
    for replicas r0..r0+replicas-1.  `fmax` widens the table's field range beyond the
    embedding's own (results do not depend on it)."""
    emb = Embedding(kind, J, penalty, h)
    g = gamma_schedule(gamma0, gamma1, sweeps) if gamma is None else np.asarray(gamma, dtype=np.float64)
    F = emb.fmax if fmax is None else fmax
    table = sqa_table(beta, L, g, F, bscale)
    spins = sqa_init(emb, L, replicas, seed, r0)
    sqa_run(emb, L, spins, 0, sweeps, table, seed, nthreads, r0)
    return emb, table, spins, sqa_energies(emb, spins)


# ---------------------------------------------------------------- SQA, Wolff moves
def wolff_bond_uniform(seed, replica, site, bond, sweep) -> int:
    """The 32-bit uniform of one ring bond's join decision (high half stream WOLFF, low half WOLFF_LO)."""
    return int(lib().oracle_wolff_bond_uniform(seed, replica, site, bond, sweep))


def wolff_site_words(seed, replica, site, sweep):
    """(seed-slice word, acceptance word) of one site move."""
    us, ua = C.c_uint32(), C.c_uint32()
    lib().oracle_wolff_site_words(C.c_uint64(seed), replica, site, sweep, C.byref(us), C.byref(ua))
    return int(us.value), int(ua.value)


def wolff_tables(beta, L, gamma, F, bscale=None):
    """(join thresholds padd[M], acceptance thresholds acc[rows][2 L F + 1])."""
    gamma = np.ascontiguousarray(gamma, dtype=np.float64)
    M = gamma.shape[0]
    rows = M if bscale is not None else 1
    padd = np.zeros(M, dtype=np.uint32)
    acc = np.zeros((rows, 2 * L * F + 1), dtype=np.uint32)
    bp = None
    if bscale is not None:
        bscale = np.ascontiguousarray(bscale, dtype=np.float64)
        bp = _p(bscale, C.c_double)
    lib().oracle_wolff_tables(C.c_double(beta), L, M, _p(gamma, C.c_double), bp, F, _p(padd, C.c_uint32),
                              _p(acc, C.c_uint32))
    return padd, acc


def wolff_move(emb: Embedding, L, lats, k, tau0, bond_u, u_acc, padd, acc_row):
    """Applies one cluster move of site k with the given words to every lattice of
    lats[count][L][n] in place; returns (thresholds[count], cluster bit masks[count])."""
    assert lats.dtype == np.int8 and lats.flags.c_contiguous and lats.ndim == 3
    bond_u = np.ascontiguousarray(bond_u, dtype=np.uint32)
    acc_row = np.ascontiguousarray(acc_row, dtype=np.uint32)
    F = (acc_row.shape[0] - 1) // (2 * L)
    count = lats.shape[0]
    thr = np.zeros(count, dtype=np.uint32)
    cl = np.zeros(count, dtype=np.uint64)
    lib().oracle_wolff_move(emb.ptr, L, count, _p(lats, C.c_int8), k, tau0, _p(bond_u, C.c_uint32),
                            C.c_uint32(u_acc), C.c_uint32(int(padd)), _p(acc_row, C.c_uint32), F,
                            _p(thr, C.c_uint32), _p(cl, C.c_uint64))
    return thr, cl


def wolff_site_order(emb: Embedding):
    out = np.zeros(emb.n_sites, dtype=np.int32)
    cnt = lib().oracle_wolff_site_order(emb.ptr, _p(out, C.c_int32))
    return out[:cnt]


def wolff_run(emb: Embedding, L, spins, m0, m1, padd, acc, seed, nthreads=1, r0=0):
    """Runs Wolff sweeps m0..m1-1 in place on spins[R][L][n] (replicas r0..r0+R-1)."""
    assert spins.dtype == np.int8 and spins.flags.c_contiguous
    padd = np.ascontiguousarray(padd, dtype=np.uint32)
    acc = np.ascontiguousarray(acc, dtype=np.uint32)
    F = (acc.shape[1] - 1) // (2 * L)
    lib().oracle_wolff_run(emb.ptr, L, r0, spins.shape[0], m0, m1, _p(padd, C.c_uint32), _p(acc, C.c_uint32),
                           acc.shape[0], F, C.c_uint64(seed), _p(spins, C.c_int8), nthreads)
    return spins


def sqa_anneal_wolff(kind, J, penalty, beta, L, sweeps, replicas, gamma0, gamma1, seed, h=None, gamma=None,
                     bscale=None, nthreads=1, r0=0):
    """SQA with time-like Wolff moves: embed, tabulate, init (INIT stream), anneal, energies."""
    emb = Embedding(kind, J, penalty, h)
    g = gamma_schedule(gamma0, gamma1, sweeps) if gamma is None else np.asarray(gamma, dtype=np.float64)
    padd, acc = wolff_tables(beta, L, g, emb.fmax, bscale)
    spins = sqa_init(emb, L, replicas, seed, r0)
    wolff_run(emb, L, spins, 0, sweeps, padd, acc, seed, nthreads, r0)
    return emb, (padd, acc), spins, sqa_energies(emb, spins)


# ---------------------------------------------------------------- PT
def pt_init(emb: Embedding, R, seed):
    out = np.zeros((R, emb.n_sites), dtype=np.int8)
    lib().oracle_pt_init(emb.ptr, R, C.c_uint64(seed), _p(out, C.c_int8))
    return out


def pt_run(emb: Embedding, betas, sweeps, sweeps_per_swap, seed):
    betas = np.ascontiguousarray(betas, dtype=np.float64)
    R = betas.shape[0]
    F = emb.fmax
    Dmax = 2 * emb.emax
    mt = pt_table(betas, F)
    st = swap_table(betas, Dmax)
    st_c = np.ascontiguousarray(st if st.size else np.zeros((1, Dmax + 1), np.uint32))
    spins = np.zeros((R, emb.n_sites), dtype=np.int8)
    E = np.zeros(R, dtype=np.int32)
    rep_at = np.zeros(R, dtype=np.int32)
    acc = np.zeros(max(R - 1, 1), dtype=np.uint64)
    lib().oracle_pt_run(emb.ptr, R, sweeps, sweeps_per_swap, _p(mt, C.c_uint32), F,
                        _p(st_c, C.c_uint32), Dmax, C.c_uint64(seed), _p(spins, C.c_int8),
                        _p(E, C.c_int32), _p(rep_at, C.c_int32), _p(acc, C.c_uint64))
    return spins, E, rep_at, acc[:max(R - 1, 0)]


# ---------------------------------------------------------------- decoders
def me_majority(emb: Embedding, slice_):
    s = np.ascontiguousarray(slice_, dtype=np.int8)
    out = np.zeros(emb.N, dtype=np.int8)
    lib().oracle_me_majority(emb.ptr, _p(s, C.c_int8), _p(out, C.c_int8))
    return out


def lhz_tree_decode(N, slice_, parents):
    s = np.ascontiguousarray(slice_, dtype=np.int8)
    par = _i32(parents).reshape(-1, N)
    out = np.zeros(N, dtype=np.int8)
    lib().oracle_lhz_tree_decode(N, _p(s, C.c_int8), _p(par, C.c_int32), par.shape[0], _p(out, C.c_int8))
    return out


def random_trees(seed, N, n_trees):
    out = np.zeros((n_trees, N), dtype=np.int32)
    rc = lib().oracle_random_trees(C.c_uint64(seed), N, n_trees, _p(out, C.c_int32))
    if rc != 0:
        raise ValueError("N must be >= 1")
    return out


def lhz_mwd(N, slice_):
    s = np.ascontiguousarray(slice_, dtype=np.int8)
    out = np.zeros(N, dtype=np.int8)
    lib().oracle_lhz_mwd(N, _p(s, C.c_int8), _p(out, C.c_int8))
    return out


def lhz_bp(N, slice_, parents, error_rate=0.2, iterations=10):
    """Weight-3 parity-check decoding; returns (logical[N], final pair values[K])."""
    s = np.ascontiguousarray(slice_, dtype=np.int8)
    par = _i32(parents).reshape(-1, N)
    out = np.zeros(N, dtype=np.int8)
    pairs = np.zeros(N * (N - 1) // 2, dtype=np.int8)
    lib().oracle_lhz_bp(N, _p(s, C.c_int8), C.c_double(error_rate), iterations, _p(par, C.c_int32), par.shape[0],
                        _p(out, C.c_int8), _p(pairs, C.c_int8))
    return out, pairs


def lhz_mld(N, slice_, error_rate):
    """Maximum-likelihood decoding at the Nishimori temperature; returns (logical[N],
    integer numerators of <sigma_0 sigma_i>)."""
    assert 3 <= N <= 24
    s = np.ascontiguousarray(slice_, dtype=np.int8)
    out = np.zeros(N, dtype=np.int8)
    corr = np.zeros(N, dtype=np.int64)
    lib().oracle_lhz_mld(N, _p(s, C.c_int8), C.c_double(error_rate), _p(out, C.c_int8), _p(corr, C.c_int64))
    return out, corr


def ground_states(J, h=None, max_states=64):
    J = _i32(J)
    N = J.shape[0]
    out = np.zeros((max_states, N), dtype=np.int8)
    cnt = C.c_int32(0)
    hp = _p(_i32(h), C.c_int32) if h is not None else None
    E = lib().oracle_ground_states(N, _p(J, C.c_int32), hp, _p(out, C.c_int8), max_states, C.byref(cnt))
    return int(E), out[:min(cnt.value, max_states)], cnt.value


def chain_tree(N):
    """Eq. (A1): parent(v) = v-1."""
    return np.array([-1] + list(range(N - 1)), dtype=np.int32)


def star_tree(N):
    """Eq. (A2): parent(v) = 0."""
    return np.array([-1] + [0] * (N - 1), dtype=np.int32)
