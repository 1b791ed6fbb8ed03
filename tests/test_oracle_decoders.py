"""Pins of the oracle's decoders: ME majority vote (Eq. (4)), LHZ spanning-tree
majority vote (Eq. (5), Appendix A), random spanning trees, minimum-weight
decoding (Sec. IV A) against brute force over all physical states."""
import itertools

import networkx as nx
import numpy as np
import pytest

import oracle as O
from paper_1603_03755_amd.workloads import sk_instance


def _q(sig):
    N = len(sig)
    return np.array([sig[i] * sig[j] for i in range(N) for j in range(i + 1, N)], dtype=np.int8)


@pytest.mark.parametrize("N", [3, 4, 8, 9])
def test_me_majority_recovers_aligned_and_minority_flips(N):
    rng = np.random.default_rng(N)
    emb = O.Embedding(O.ME, sk_instance(N, 1), -2)
    for _ in range(20):
        sig = rng.choice([-1, 1], N).astype(np.int8)
        phys = np.repeat(sig, N - 1).astype(np.int8)
        assert (O.me_majority(emb, phys) == sig).all()
        # flip a strict minority of every chain: the vote does not change
        for i in range(N):
            nflip = (N - 2) // 2
            for r in rng.choice(N - 1, nflip, replace=False):
                phys[O.me_site(N, i, int(r))] *= -1
        assert (O.me_majority(emb, phys) == sig).all()


def test_me_majority_tie_goes_plus():
    N = 5      # chains of 4 spins can tie
    emb = O.Embedding(O.ME, sk_instance(N, 1), -2)
    phys = np.ones(emb.n_sites, dtype=np.int8)
    for i in range(N):
        phys[O.me_site(N, i, 0)] = -1
        phys[O.me_site(N, i, 1)] = -1
    assert (O.me_majority(emb, phys) == 1).all()


@pytest.mark.parametrize("N", [3, 5, 7])
def test_trees_decode_valid_states_exactly(N):
    """On a constraint-satisfying state every spanning tree returns the logical
    state (up to the global flip fixed by qbar_0 = +1), so chain (A1) = star (A2)."""
    trees = np.vstack([O.chain_tree(N), O.star_tree(N), O.random_trees(7, N, 9)])
    for bits in itertools.product([1, -1], repeat=N - 1):
        sig = np.array((1,) + bits, dtype=np.int8)
        q = _q(sig)
        for t in trees:
            assert (O.lhz_tree_decode(N, q, t[None, :]) == sig).all()
        assert (O.lhz_tree_decode(N, q, trees) == sig).all()


def test_chain_and_star_can_differ_on_leaked_state():
    """Appendix A: on a leaked state different trees may decode differently."""
    N = 4
    sig = np.ones(N, dtype=np.int8)
    q = _q(sig)
    q[O.lhz_site(N, 1, 2)] = -1       # on the chain tree, off the star
    chain = O.lhz_tree_decode(N, q, O.chain_tree(N)[None, :])
    star = O.lhz_tree_decode(N, q, O.star_tree(N)[None, :])
    assert (star == sig).all()
    assert not (chain == sig).all()


@pytest.mark.parametrize("N", [2, 3, 6, 12, 24])
def test_random_trees_are_spanning_trees(N):
    par = O.random_trees(123, N, 20)
    for p in par:
        assert p[0] == -1
        G = nx.Graph()
        G.add_nodes_from(range(N))
        G.add_edges_from((v, int(p[v])) for v in range(1, N))
        assert nx.is_tree(G)


def test_random_trees_uniform_over_labelled_trees():
    """Cayley: 4^2 = 16 labelled trees on 4 vertices, each equally likely."""
    N, T = 4, 16000
    par = O.random_trees(2024, N, T)
    keys = {}
    for p in par:
        k = tuple(sorted(tuple(sorted((v, int(p[v])))) for v in range(1, N)))
        keys[k] = keys.get(k, 0) + 1
    assert len(keys) == 16
    cnt = np.array(list(keys.values()), dtype=float)
    chi2 = ((cnt - T / 16) ** 2 / (T / 16)).sum()
    assert chi2 < 45.0      # 15 dof


@pytest.mark.parametrize("N", [3, 4, 5])
def test_mwd_is_nearest_valid_state_bruteforce(N):
    """Sec. IV A: MWD returns a constraint-satisfying state at minimum Hamming
    distance from the read-out state; checked over every physical state."""
    K = N * (N - 1) // 2
    valid = [_q(np.array((1,) + b, dtype=np.int8)) for b in itertools.product([1, -1], repeat=N - 1)]
    valid = np.array(valid)
    for bits in itertools.product([1, -1], repeat=K):
        s = np.array(bits, dtype=np.int8)
        dmin = (valid != s).sum(axis=1).min()
        sig = O.lhz_mwd(N, s)
        assert sig[0] == 1
        assert (_q(sig) != s).sum() == dmin


def test_mwd_tie_takes_smallest_candidate():
    N = 3
    s = np.array([1, 1, -1], dtype=np.int8)   # one violated triangle: three nearest states
    sig = O.lhz_mwd(N, s)
    # candidates m = 0 (all +1) is at distance 1 and is the smallest index
    assert (sig == 1).all()


@pytest.mark.parametrize("seed", range(6))
def test_mwd_zero_penalty_recovers_logical_ground_state(seed):
    """Sec. IV E: at zero penalty the physical ground state aligns every parity
    spin against its field, s = -sign(J); MWD then solves J -> sign(J), which for
    J in {-1, +1} is the logical problem itself."""
    N = 8
    J = sk_instance(N, 500 + seed)
    emb = O.Embedding(O.LHZ, J, 0)
    s = -np.sign(emb.h).astype(np.int8)
    sig = O.lhz_mwd(N, s)
    Eg, _, _ = O.ground_states(J)
    assert O.logical_energy(J, sig) == Eg


def test_mwd_gauge_equivalence():
    """Sec. IV A: decoding s and its logical gauge transform s_ij tau_i tau_j gives
    the gauge-transformed state (the score is gauge invariant)."""
    rng = np.random.default_rng(3)
    N = 7
    for _ in range(10):
        s = rng.choice([-1, 1], N * (N - 1) // 2).astype(np.int8)
        tau = rng.choice([-1, 1], N).astype(np.int8)
        s2 = s * _q(tau)
        a, b = O.lhz_mwd(N, s), O.lhz_mwd(N, s2)
        score = lambda ss, sg: int((ss.astype(int) * _q(sg)).sum())
        assert score(s2, b) == score(s, a)
        assert score(s2, a * tau) == score(s, a)
