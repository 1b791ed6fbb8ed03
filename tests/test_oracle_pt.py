"""Pins of the oracle's parallel tempering (Appendix B, Eqs. (B1)-(B2)).

Exact stationarity: with R replicas of an n-site system, the joint state
(spins of every replica, slot permutation) has the stationary law
    pi ~ prod_slots exp(-beta_slot E(replica in that slot)).
One PT step (a Metropolis sweep with the oracle's PT table, then a swap phase
with the oracle's swap table) is applied exactly to pi, following the order
the oracle documents, and pi must come back unchanged.  A separate test
replays the oracle's run from its random words, tying the run to the tables.
"""
import itertools
import json
import os

import numpy as np
import pytest

import oracle as O
from paper_1603_03755_amd.workloads import sk_instance

TOL = 2e-8
GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "paper_counts.json")


def test_ladder_golden():
    g = json.load(open(GOLDEN))["pt_ladder"]
    b = O.pt_ladder(g["beta_last"], g["beta_first"], g["temps"])
    assert b[0] == g["beta_first"]
    assert abs(b[-1] - g["beta_last"]) < 1e-12
    # Eq. (B2): constant ratio (0.1/20)^(1/63)
    assert np.allclose(b[1:] / b[:-1], (0.1 / 20) ** (1 / 63), rtol=1e-12)
    assert (np.diff(b) < 0).all()


def _states(n):
    return np.array(list(itertools.product([1, -1], repeat=n)), dtype=np.int8)


@pytest.mark.parametrize("kind,N,R", [(O.LHZ, 3, 2), (O.ME, 2, 3), (O.LHZ, 3, 3)])
def test_pt_step_preserves_joint_gibbs(kind, N, R):
    J = sk_instance(N, 80 + N)
    emb = O.Embedding(kind, J, -2)
    n, F = emb.n_sites, emb.fmax
    betas = O.pt_ladder(0.4, 2.5, R)
    mt = O.pt_table(betas, F)
    Dmax = 2 * emb.emax
    st = O.swap_table(betas, Dmax)
    S = _states(n)
    E = np.array([emb.energy(s) for s in S])
    perms = list(itertools.permutations(range(R)))           # perm[slot] = replica
    pidx = {p: i for i, p in enumerate(perms)}
    ns = len(S)
    # joint index: (perm, config of replica 0, ..., replica R-1)
    shape = (len(perms),) + (ns,) * R
    pi = np.zeros(shape)
    for p in perms:
        for cfg in itertools.product(range(ns), repeat=R):
            pi[(pidx[p],) + cfg] = np.exp(-sum(betas[slot] * E[cfg[p[slot]]] for slot in range(R)))
    pi /= pi.sum()
    v = pi.copy()
    flipidx = np.array([[int(''.join('1' if x < 0 else '0' for x in (S[c] * np.where(np.arange(n) == k, -1, 1))), 2)
                         for k in range(n)] for c in range(ns)])
    # map config index -> integer code used in flipidx: configs are enumerated in product order
    code = np.array([int(''.join('1' if x < 0 else '0' for x in s), 2) for s in S])
    inv = np.empty_like(code)
    inv[code] = np.arange(ns)
    # sweep: colours 0..3, replicas, sites of that colour
    for c in range(4):
        for rho in range(R):
            for k in range(n):
                if emb.colour[k] != c:
                    continue
                p_acc = np.zeros((len(perms), ns))
                for pi_i, p in enumerate(perms):
                    slot = p.index(rho)
                    for ci in range(ns):
                        a = int(S[ci][k]) * emb.local_field(S[ci], k)
                        T = int(mt[slot, a + F])
                        p_acc[pi_i, ci] = 1.0 if T == O.ALWAYS else T / 2.0**32
                fl = inv[flipidx[:, k]]
                vm = np.moveaxis(v, rho + 1, 1)          # (perm, cfg_rho, rest...)
                pa = p_acc.reshape(p_acc.shape + (1,) * (R - 1))
                new = vm * (1 - pa) + vm[:, fl] * pa[:, fl]
                v = np.moveaxis(new, 1, rho + 1)
    assert np.abs(v - pi).max() <= TOL * pi.max()
    # swap phase: even pairs then odd pairs
    for q in (0, 1):
        for r in range(q, R - 1, 2):
            new = v.copy()
            for pi_i, p in enumerate(perms):
                p2 = list(p)
                p2[r], p2[r + 1] = p2[r + 1], p2[r]
                pj = pidx[tuple(p2)]
                for cfg in itertools.product(range(ns), repeat=R):
                    D = E[cfg[p[r + 1]]] - E[cfg[p[r]]]
                    T = O.ALWAYS if D <= 0 else int(st[r, D])
                    acc = 1.0 if T == O.ALWAYS else T / 2.0**32
                    mass = v[(pi_i,) + cfg] * acc
                    new[(pi_i,) + cfg] -= mass
                    new[(pj,) + cfg] += mass
            v = new
    assert np.abs(v - pi).max() <= TOL * pi.max()


def test_pt_swap_table_is_eq_b1():
    """Threshold of a swap with D = E_{r+1} - E_r > 0 is exp(D (beta_{r+1} - beta_r)) in 2^-32 units."""
    betas = O.pt_ladder(0.1, 5.0, 32)
    st = O.swap_table(betas, 300)
    for r in (0, 7, 30):
        for D in (1, 5, 40, 299):
            p = np.exp(D * (betas[r + 1] - betas[r]))
            assert abs(int(st[r, D]) / 2.0**32 - p) <= 2.0**-32
        assert st[r, 0] == O.ALWAYS


@pytest.mark.parametrize("kind,N,R,sweeps,sps", [(O.LHZ, 5, 4, 6, 1), (O.ME, 4, 5, 7, 2), (O.LHZ, 4, 1, 3, 1)])
def test_pt_run_replay(kind, N, R, sweeps, sps):
    seed = 0x1234
    emb = O.Embedding(kind, sk_instance(N, 90), -2)
    n, F = emb.n_sites, emb.fmax
    betas = O.pt_ladder(0.1, 5.0, R)
    mt = O.pt_table(betas, F)
    Dmax = 2 * emb.emax
    st = O.swap_table(betas, Dmax)
    spins, E, rep_at, acc = O.pt_run(emb, betas, sweeps, sps, seed)
    # replay
    s = O.pt_init(emb, R, seed)
    perm = list(range(R))
    Er = [emb.energy(s[r]) for r in range(R)]
    acc2 = np.zeros(max(R - 1, 0), dtype=np.uint64)
    phase = 0
    for m in range(sweeps):
        for c in range(4):
            for rho in range(R):
                for k in range(n):
                    if emb.colour[k] != c:
                        continue
                    a = int(s[rho, k]) * emb.local_field(s[rho], k)
                    T = int(mt[perm.index(rho), a + F])
                    u = O.pt_uniform(seed, rho, k, m)
                    if T == O.ALWAYS or u < T:
                        s[rho, k] = -s[rho, k]
                        Er[rho] -= 2 * a
        if (m + 1) % sps == 0:
            for q in (0, 1):
                for r in range(q, R - 1, 2):
                    D = Er[perm[r + 1]] - Er[perm[r]]
                    ok = D <= 0
                    if not ok:
                        u = int(O.philox4x32([r, 0, phase, O.STREAM_SWAP << 24], [seed & 0xFFFFFFFF, seed >> 32])[0])
                        T = int(st[r, D])
                        ok = T == O.ALWAYS or u < T
                    if ok:
                        perm[r], perm[r + 1] = perm[r + 1], perm[r]
                        acc2[r] += 1
            phase += 1
    assert (spins == s).all()
    assert list(E) == Er
    assert list(rep_at) == perm
    assert (acc == acc2).all()
    for r in range(R):
        assert E[r] == emb.energy(spins[r])   # incremental energy equals recomputed


def test_pt_cold_ladder_finds_ground_state():
    J = sk_instance(8, 5)
    emb = O.Embedding(O.LHZ, J, -3)
    betas = O.pt_ladder(0.2, 6.0, 8)
    spins, E, rep_at, acc = O.pt_run(emb, betas, 3000, 1, 42)
    Eg, _, _ = O.ground_states(J)
    cold = rep_at[0]
    # the coldest replica sits in a physical ground state: a logical GS with all constraints satisfied
    assert E[cold] == Eg + (-3) * 21
    assert acc.sum() > 0
