"""Pins of the oracle's weight-3 parity-check decoder (Sec. IV D) and
maximum-likelihood decoder (Sec. IV B, Eq. (11)) for the LHZ scheme."""
import itertools

import numpy as np
import pytest

import oracle as O


def _pairs(N, tau):
    return np.array([tau[i] * tau[j] for i in range(N) for j in range(i + 1, N)], dtype=np.int8)


def _site(N, i, j):
    i, j = min(i, j), max(i, j)
    return i * (2 * N - i - 1) // 2 + (j - i - 1)


def _random_tau(N, rng):
    tau = np.where(rng.random(N) < 0.5, -1, 1).astype(np.int8)
    tau[0] = 1
    return tau


# ------------------------------------------------------------------ BP
@pytest.mark.parametrize("N", [3, 5, 8, 13])
def test_bp_valid_readout_is_a_fixed_point(N):
    rng = np.random.default_rng(N)
    for _ in range(5):
        tau = _random_tau(N, rng)
        s = _pairs(N, tau)
        q, x = O.lhz_bp(N, s, O.random_trees(N, N, 1), 0.2, 10)
        assert (x == s).all() and (q == tau).all()


@pytest.mark.parametrize("N", [4, 6, 9])
def test_bp_corrects_one_error_in_one_iteration(N):
    """One flipped pair: its N-2 checks all disagree with it (they outvote it for
    N >= 4 at p = 0.2), every other pair sees one bad check of N-2."""
    rng = np.random.default_rng(10 + N)
    tau = _random_tau(N, rng)
    s = _pairs(N, tau)
    for k in range(len(s)):
        bad = s.copy()
        bad[k] = -bad[k]
        q, x = O.lhz_bp(N, bad, O.chain_tree(N), 0.2, 1)
        assert (x == s).all(), k
        assert (q == tau).all()


def _single_pair_decision(s01, c, p):
    """N = 5, pair (0,1) with readout s01 and its three checks q_0l q_l1 (l = 2, 3, 4)
    summing to c; all other pairs consistent with an all-up state except the (0, l)
    pairs chosen to set c.  Returns the pair's value after one iteration."""
    N = 5
    s = _pairs(N, np.ones(N, np.int8))
    s[_site(N, 0, 1)] = s01
    n_neg = (3 - c) // 2                 # checks with product -1
    for idx, l in enumerate((2, 3, 4)):
        if idx < n_neg:
            s[_site(N, 0, l)] = -1
    _, x = O.lhz_bp(N, s, O.chain_tree(N), p, 1)
    return int(x[_site(N, 0, 1)])


def test_bp_vote_weights_follow_the_error_rate():
    """At p = 0.2 the own readout weighs ln 4 = 1.39 and a two-bit check ln(0.68/0.32)
    = 0.75: one check against it is outvoted, three are not.  At p = 0.4 (own 0.41,
    check 0.080) even three checks cannot overturn the readout."""
    assert _single_pair_decision(+1, -1, 0.2) == +1
    assert _single_pair_decision(+1, -3, 0.2) == -1
    assert _single_pair_decision(-1, +1, 0.2) == -1
    assert _single_pair_decision(-1, +3, 0.2) == +1
    assert _single_pair_decision(-1, +3, 0.4) == -1
    assert _single_pair_decision(+1, -3, 0.4) == +1


@pytest.mark.parametrize("N", [4, 7, 10])
def test_bp_without_iterations_is_tree_decoding(N):
    rng = np.random.default_rng(30 + N)
    trees = O.random_trees(77, N, 3)
    for _ in range(10):
        s = np.where(rng.random(N * (N - 1) // 2) < 0.5, -1, 1).astype(np.int8)
        q, x = O.lhz_bp(N, s, trees, 0.2, 0)
        assert (x == s).all()
        assert (q == O.lhz_tree_decode(N, s, trees)).all()


def test_bp_corrects_sparse_random_errors():
    """Errors at rate 0.05 on N = 16 (about 6 of 120 pairs): ten rounds restore the
    codeword in nearly every trial, far better than a single tree."""
    rng = np.random.default_rng(4)
    N, ok_bp, ok_tree = 16, 0, 0
    for t in range(40):
        tau = _random_tau(N, rng)
        s = _pairs(N, tau)
        flips = rng.random(len(s)) < 0.05
        bad = np.where(flips, -s, s).astype(np.int8)
        tree = O.random_trees(100 + t, N, 1)
        ok_bp += int((O.lhz_bp(N, bad, tree, 0.2, 10)[0] == tau).all())
        ok_tree += int((O.lhz_tree_decode(N, bad, tree) == tau).all())
    assert ok_bp >= 38 and ok_bp > ok_tree


# ------------------------------------------------------------------ MLD
def _float_mld(N, s, p):
    """Thermal average numerators, weights relative to the best state, in float64."""
    beta = 0.5 * np.log((1 - p) / p)
    sigs, scores = [], []
    for bits in itertools.product((1, -1), repeat=N - 1):
        sig = np.array((1,) + bits, dtype=np.float64)
        sigs.append(sig)
        scores.append(sum(s[_site(N, i, j)] * sig[i] * sig[j] for i in range(N) for j in range(i + 1, N)))
    omax = max(scores)
    return sum(np.exp(-beta * (omax - o)) * sig for o, sig in zip(scores, sigs))


@pytest.mark.parametrize("N,p", [(3, 0.1), (5, 0.2), (7, 0.3), (9, 0.15), (10, 0.45)])
def test_mld_matches_float_thermal_average(N, p):
    """Against the thermal average summed in floating point by brute force: the
    integer numerators agree to the quantisation (2^-36 per state) and every
    decision away from a zero average is the same."""
    rng = np.random.default_rng(N)
    for _ in range(6):
        s = np.where(rng.random(N * (N - 1) // 2) < 0.3, -1, 1).astype(np.int8)
        q, num = O.lhz_mld(N, s, p)
        ref = _float_mld(N, s, p)
        assert np.allclose(num / 2.0**36, ref, rtol=0, atol=2.0**(N - 36) + 1e-12 * np.abs(ref).max())
        for i in range(N):
            if abs(ref[i]) > 1e-6 * ref[0]:
                assert q[i] == (1 if ref[i] > 0 else -1)
        assert q[0] == 1 and num[0] > 0


@pytest.mark.parametrize("N", [4, 8, 12])
def test_mld_decodes_codewords_and_is_gauge_covariant(N):
    rng = np.random.default_rng(50 + N)
    for p in (0.05, 0.3, 0.49):
        tau = _random_tau(N, rng)
        assert (O.lhz_mld(N, _pairs(N, tau), p)[0] == tau).all()
    s = np.where(rng.random(N * (N - 1) // 2) < 0.25, -1, 1).astype(np.int8)
    t = _random_tau(N, rng)
    gauged = np.array([t[i] * t[j] * s[_site(N, i, j)] for i in range(N) for j in range(i + 1, N)], np.int8)
    q, _ = O.lhz_mld(N, s, 0.2)
    qg, _ = O.lhz_mld(N, gauged, 0.2)
    assert (qg == t * q).all()


def test_mld_at_low_error_rate_is_mwd():
    """Footnote of Sec. IV C: as P -> 0 (beta_N -> infinity) MLD becomes MWD, checked
    where the minimum-weight state is unique."""
    rng = np.random.default_rng(8)
    N, checked = 9, 0
    for _ in range(30):
        s = np.where(rng.random(N * (N - 1) // 2) < 0.2, -1, 1).astype(np.int8)
        scores = []
        for bits in itertools.product((1, -1), repeat=N - 1):
            sig = (1,) + bits
            scores.append(sum(s[_site(N, i, j)] * sig[i] * sig[j] for i in range(N) for j in range(i + 1, N)))
        if sorted(scores)[-1] == sorted(scores)[-2]:
            continue
        checked += 1
        assert (O.lhz_mld(N, s, 1e-6)[0] == O.lhz_mwd(N, s)).all()
    assert checked >= 10
