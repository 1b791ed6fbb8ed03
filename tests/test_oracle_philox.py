"""Pins of the oracle's Philox generator and counter layout.

Philox4x32-10 and Philox4x64-10 are instantiated from one round definition in
oracle/philox.c; the 64-bit instance is checked against numpy.random.Philox
(an independent implementation of Philox4x64-10), which pins the round
structure, output order and key schedule shared by the 32-bit instance.
The published 32-bit known-answer vectors are not available here, so exact
equality of the 32-bit instance with other Philox4x32 implementations is
parity unpinned; uniformity and avalanche checks cover gross mistakes.
"""
import numpy as np
import pytest

import oracle as O


@pytest.mark.parametrize("key", [(0, 0), (5, 7), (2**64 - 1, 12345678901234567), (0xDEADBEEF, 1 << 63)])
@pytest.mark.parametrize("start", [0, 1, 41, 2**40])
def test_philox4x64_matches_numpy(key, start):
    # numpy increments its 256-bit counter before producing each block of four words.
    g = np.random.Philox(key=np.array(key, dtype=np.uint64),
                         counter=np.array([start, 0, 0, 0], dtype=np.uint64))
    raw = g.random_raw(12)
    for blk in range(3):
        ours = O.philox4x64([start + blk + 1, 0, 0, 0], key)
        assert [int(x) for x in ours] == [int(x) for x in raw[4 * blk:4 * blk + 4]]


def test_philox4x64_matches_numpy_high_counter_words():
    g = np.random.Philox(key=np.array([3, 9], dtype=np.uint64),
                         counter=np.array([2**64 - 1, 17, 5, 2], dtype=np.uint64))
    raw = g.random_raw(4)   # counter wraps word 0 and carries into word 1
    assert [int(x) for x in O.philox4x64([0, 18, 5, 2], [3, 9])] == [int(x) for x in raw]


def test_philox4x32_uniform_top_bits():
    counts = np.zeros(256, dtype=np.int64)
    for c in range(4096):
        out = O.philox4x32([c, 3, 7, 1 << 24], [11, 13])
        for w in out:
            counts[int(w) >> 24] += 1
    exp = counts.sum() / 256.0
    chi2 = float(((counts - exp) ** 2 / exp).sum())
    assert chi2 < 350.0     # 255 dof: mean 255, sd ~22.6


def test_philox4x32_avalanche():
    rng = np.random.default_rng(0)
    flips = []
    for _ in range(200):
        ctr = [int(x) for x in rng.integers(0, 2**32, 4, dtype=np.uint64)]
        key = [int(x) for x in rng.integers(0, 2**32, 2, dtype=np.uint64)]
        bit = int(rng.integers(0, 128))
        ctr2 = list(ctr)
        ctr2[bit // 32] ^= 1 << (bit % 32)
        a, b = O.philox4x32(ctr, key), O.philox4x32(ctr2, key)
        flips.append(sum(bin(int(x) ^ int(y)).count("1") for x, y in zip(a, b)))
    assert 60 < np.mean(flips) < 68


def test_init_word_counter_layout():
    seed = 0x0123456789ABCDEF
    key = [seed & 0xFFFFFFFF, seed >> 32]
    for (r, k, tau) in [(0, 0, 0), (3, 17, 13), (63, 551, 63), (5, 2, 1)]:
        g, p = tau >> 3, tau & 1
        out = O.philox4x32([k, (g << 1) | p, 0, (O.STREAM_INIT << 24) | r], key)
        # the four same-parity slices 8g+p+2w of one site share one call
        for w in range(4):
            t2 = 8 * g + p + 2 * w
            assert O.sqa_word(seed, O.STREAM_INIT, r, k, t2, 0) == int(out[w])


def test_sqa_uniform_counter_layout():
    seed = 0x0123456789ABCDEF
    key = [seed & 0xFFFFFFFF, seed >> 32]
    for (r, k, tau, m) in [(0, 0, 0, 0), (3, 17, 13, 999), (63, 551, 63, 9999), (5, 2, 1, 1), (9, 4, 0, 7)]:
        b, p = tau >> 4, tau & 1
        hi = O.philox4x32([k, (b << 1) | p, m, (O.STREAM_SQA << 24) | r], key)
        lo = O.philox4x32([k, (b << 1) | p, m, (O.STREAM_SQA_LO << 24) | r], key)
        # the eight same-parity slices 16b+p+2j of one site share one call per stream
        for j in range(8):
            t2 = 16 * b + p + 2 * j
            sh = 16 * (j >> 2)
            want = (((int(hi[j & 3]) >> sh) & 0xFFFF) << 16) | ((int(lo[j & 3]) >> sh) & 0xFFFF)
            assert O.sqa_uniform(seed, r, k, t2, m) == want


@pytest.mark.parametrize("fn", ["sqa", "wolff", "pt"])
def test_attempt_uniforms_are_uniform_with_independent_halves(fn):
    """The 32-bit attempt uniforms: both halves uniform, the low half independent of
    the high half (a low half drawn from the high half's stream would coincide with
    it), and all 2^32 values reachable in the sense that the top byte and the bottom
    byte are each uniform."""
    seed = 0x5EED
    if fn == "sqa":
        u = np.array([O.sqa_uniform(seed, r, k, t, m) for r in range(2) for k in range(6)
                      for t in range(64) for m in range(8)], dtype=np.uint64)
    elif fn == "wolff":
        u = np.array([O.wolff_bond_uniform(seed, r, k, b, m) for r in range(2) for k in range(6)
                      for b in range(64) for m in range(8)], dtype=np.uint64)
    else:
        u = np.array([O.pt_uniform(seed, rho, k, m) for rho in range(64) for k in range(12)
                      for m in range(8)], dtype=np.uint64)
    n = u.size
    hi, lo = u >> 16, u & 0xFFFF
    assert np.mean(hi == lo) < 5.0 / n + 1e-3
    assert len(np.unique(u)) > n - 3
    for part in (u >> 24, u & 0xFF, (hi & 0xFF), (lo >> 8)):
        counts = np.bincount(part.astype(np.int64), minlength=256)
        chi2 = float(((counts - n / 256.0) ** 2 / (n / 256.0)).sum())
        assert chi2 < 255 + 6 * np.sqrt(2 * 255)
    c = np.corrcoef(hi.astype(float), lo.astype(float))[0, 1]
    assert abs(c) < 5 / np.sqrt(n)


def test_pt_init_word_counter_layout():
    seed = 77
    for (rho, k) in [(0, 0), (5, 9), (31, 551)]:
        out = O.philox4x32([k, rho >> 2, 0, O.STREAM_PT_INIT << 24], [77, 0])
        assert O.pt_word(seed, O.STREAM_PT_INIT, rho, k, 0) == int(out[rho & 3])


def test_pt_uniform_counter_layout():
    seed = 77
    for (rho, k, m) in [(0, 0, 0), (5, 9, 3), (31, 551, 99999), (63, 7, 12), (12, 3, 5)]:
        hi = O.philox4x32([k, rho >> 3, m, O.STREAM_PT << 24], [77, 0])
        lo = O.philox4x32([k, rho >> 3, m, O.STREAM_PT_LO << 24], [77, 0])
        sh = 16 * ((rho >> 2) & 1)
        want = (((int(hi[rho & 3]) >> sh) & 0xFFFF) << 16) | ((int(lo[rho & 3]) >> sh) & 0xFFFF)
        assert O.pt_uniform(seed, rho, k, m) == want
