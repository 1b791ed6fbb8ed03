"""Exact pins of the oracle's SQA with time-like Wolff cluster moves (Sec. III).

The Trotter distribution of H = -Gamma sum sigma^x + B H_P (Eq. (2)) at inverse
temperature beta with L slices is built here directly from the transfer-matrix
elements <s|e^{(beta Gamma/L) sigma^x}|s'> = cosh or sinh (not from the
oracle's p_add formula).  One oracle cluster move of site k is applied to that
distribution EXACTLY: every seed slice (probability 1/L), every joined/not-joined
outcome of every ring bond (probability padd/2^32 or its complement, realised by
handing the oracle's move function the bond words 0 or 0xFFFFFFFF), and both
outcomes of the acceptance test (probability threshold/2^32, from the threshold
the move reports).  The distribution must come back unchanged after every site
of a sweep.  A wrong join probability, a cluster that crosses a misaligned bond
or stops early, a wrong sign or scale of the acceptance exponent, or a wrong
local field all break it (the planted-mistake tests show the check is sharp).
"""
import itertools

import numpy as np
import pytest

import oracle as O
from paper_1603_03755_amd.workloads import sk_instance

TOL = 2e-8
MAXW = 0xFFFFFFFF


def _lattices(n, L):
    nb = n * L
    x = np.arange(1 << nb, dtype=np.int64)
    bits = (x[:, None] >> np.arange(nb)) & 1
    return (1 - 2 * bits).astype(np.int8).reshape(-1, L, n)


def _index(lats):
    n, L = lats.shape[2], lats.shape[1]
    bits = (lats.reshape(len(lats), L * n) < 0).astype(np.int64)
    return (bits << np.arange(L * n)).sum(axis=1)


def _path_weight(emb, lats, beta, gamma, L, B=1.0):
    a = beta * gamma / L
    logw = np.zeros(len(lats))
    for tau in range(L):
        logw -= beta * B / L * np.array([emb.energy(s[tau]) for s in lats], dtype=np.float64)
    if L > 1:
        for tau in range(L):
            same = lats[:, tau, :] == lats[:, (tau + 1) % L, :]
            logw += np.where(same, np.log(np.cosh(a)), np.log(np.sinh(a))).sum(axis=1)
    w = np.exp(logw - logw.max())
    return w / w.sum()


def _prob(T):
    return 1.0 if int(T) == MAXW else int(T) / 2.0**32


def _apply_site(emb, L, lats, v, k, padd, acc_row):
    """Exact action of one oracle cluster move of site k on the distribution v."""
    out = np.zeros_like(v)
    p_join = _prob(padd)
    for tau0 in range(L):
        for z in itertools.product((0, 1), repeat=L):
            pz = 1.0
            for zb in z:
                pz *= p_join if zb else 1.0 - p_join
            if pz == 0.0:
                continue
            words = np.array([0 if zb else MAXW for zb in z], dtype=np.uint32)
            acc_l = lats.copy()
            thr, _ = O.wolff_move(emb, L, acc_l, k, tau0, words, 0, padd, acc_row)
            rej_l = lats.copy()
            thr2, _ = O.wolff_move(emb, L, rej_l, k, tau0, words, MAXW, padd, acc_row)
            assert (thr == thr2).all()
            pa = np.array([_prob(t) for t in thr])
            w = v * (pz / L)
            out += np.bincount(_index(acc_l), weights=w * pa, minlength=len(v))
            out += np.bincount(_index(rej_l), weights=w * (1.0 - pa), minlength=len(v))
    return out


def _apply_sweep(emb, L, lats, pi, padd, acc_row, check_each=False):
    v = pi.copy()
    for k in O.wolff_site_order(emb).tolist():
        v = _apply_site(emb, L, lats, v, k, padd, acc_row)
        if check_each:
            assert np.abs(v - pi).max() <= TOL * pi.max()
    return v


CASES = [
    # kind, N, penalty, logical h, L, beta, gamma, B
    (O.LHZ, 3, -2, None, 4, 1.3, 0.7, 1.0),
    (O.ME, 2, -2, (1, -2), 4, 2.0, 0.4, 1.0),
    (O.ME, 3, -2, (0, 1, 0), 2, 0.9, 1.1, 1.0),
    (O.LHZ, 4, -1, None, 2, 1.7, 0.3, 0.6),
    (O.ME, 2, -1, (1, 1), 6, 3.0, 2.5, 1.0),
    (O.LHZ, 3, -2, None, 2, 5.0, 0.01, 1.0),   # stiff time bonds: clusters span the ring
    (O.LHZ, 3, -2, None, 4, 0.5, 20.0, 1.0),   # weak time bonds: single-slice clusters
    (O.MEC, 3, -2, (1, 0, -1), 2, 1.1, 0.6, 1.0),   # Chimera chains of two
    (O.MEC, 2, -1, (2, -1), 2, 1.5, 0.9, 0.8),
]


@pytest.mark.parametrize("kind,N,pen,h,L,beta,gamma,B", CASES)
def test_sweep_preserves_trotter_distribution(kind, N, pen, h, L, beta, gamma, B):
    J = sk_instance(N, 40 + N)
    emb = O.Embedding(kind, J, pen, None if h is None else np.array(h, dtype=np.int32))
    padd, acc = O.wolff_tables(beta, L, np.array([gamma]), emb.fmax, bscale=np.array([B]))
    lats = _lattices(emb.n_sites, L)
    pi = _path_weight(emb, lats, beta, gamma, L, B)
    v = _apply_sweep(emb, L, lats, pi, padd[0], acc[0], check_each=True)
    assert np.abs(v - pi).max() <= TOL * pi.max()


@pytest.mark.parametrize("kind,N", [(O.LHZ, 4), (O.ME, 3)])
def test_single_slice_is_classical_metropolis(kind, N):
    """L = 1: no ring bonds, the cluster is the one spin and the move is the
    classical min(1, exp(-beta B dE)) rule; the Boltzmann law is stationary."""
    beta, B = 0.8, 1.5
    emb = O.Embedding(kind, sk_instance(N, 50 + N), -2)
    padd, acc = O.wolff_tables(beta, 1, np.array([0.5]), emb.fmax, bscale=np.array([B]))
    assert padd[0] == 0
    lats = _lattices(emb.n_sites, 1)
    E = np.array([emb.energy(s[0]) for s in lats], dtype=np.float64)
    pi = np.exp(-beta * B * (E - E.min()))
    pi /= pi.sum()
    v = _apply_sweep(emb, 1, lats, pi, padd[0], acc[0])
    assert np.abs(v - pi).max() <= TOL * pi.max()
    for s in lats[:64]:
        for k in range(emb.n_sites):
            s2 = s[0].copy()
            s2[k] = -s2[k]
            dE = emb.energy(s2) - emb.energy(s[0])
            thr, cl = O.wolff_move(emb, 1, s[None].copy(), k, 0, np.zeros(1, np.uint32), MAXW, padd[0], acc[0])
            assert int(cl[0]) == 1
            if dE <= 0:
                assert int(thr[0]) == MAXW
            else:
                assert abs(int(thr[0]) / 2.0**32 - np.exp(-beta * B * dE)) <= 2.0**-32


@pytest.mark.parametrize("mutation", ["padd_is_tanh", "gamma_x2", "acc_sign", "acc_beta_over_2"])
def test_stationarity_check_detects_planted_mistakes(mutation):
    kind, N, pen, L, beta, gamma = O.LHZ, 3, -2, 4, 1.3, 0.7
    emb = O.Embedding(kind, sk_instance(N, 43), pen)
    F = emb.fmax
    padd, acc = O.wolff_tables(beta, L, np.array([gamma]), F)
    if mutation == "padd_is_tanh":
        padd = np.array([O.threshold(np.log(np.tanh(beta * gamma / L)))], dtype=np.uint32)
    elif mutation == "gamma_x2":
        padd, _ = O.wolff_tables(beta, L, np.array([2 * gamma]), F)
    elif mutation == "acc_sign":
        acc = acc[:, ::-1].copy()
    else:
        _, acc = O.wolff_tables(beta, L, np.array([gamma]), F, bscale=np.array([0.5]))
    lats = _lattices(emb.n_sites, L)
    pi = _path_weight(emb, lats, beta, gamma, L)
    v = _apply_sweep(emb, L, lats, pi, padd[0], acc[0])
    assert np.abs(v - pi).max() > 1e3 * TOL * pi.max()


def test_join_probability_is_one_minus_tanh():
    """p_add = 1 - exp(-2 J_perp) with J_perp = -1/2 ln tanh(beta Gamma / L):
    the ratio of the aligned-bond weights sinh/cosh, written via the matrix elements."""
    beta, L = 2.0, 8
    g = np.array([0.0, 1e-3, 0.3, 1.0, 4.0, 1e6])
    padd, _ = O.wolff_tables(beta, L, g, 3)
    assert int(padd[0]) == MAXW                       # Gamma = 0: every aligned bond joins
    for m in range(1, len(g)):
        a = beta * g[m] / L
        want = 2.0 * np.exp(-2 * a) / (1.0 + np.exp(-2 * a))   # (cosh a - sinh a) / cosh a
        assert abs(int(padd[m]) / 2.0**32 - want) <= 2.0**-31
    assert int(padd[-1]) == 0                         # Gamma -> infinity: clusters are single slices


def test_acceptance_row_is_exp_of_twice_beta_b_over_l():
    beta, L, F = 1.5, 4, 3
    B = np.array([0.25, 1.0])
    _, acc = O.wolff_tables(beta, L, np.array([1.0, 1.0]), F, bscale=B)
    assert acc.shape == (2, 2 * L * F + 1)
    for row in range(2):
        for A in range(-L * F, L * F + 1):
            T = int(acc[row, A + L * F])
            if A >= 0:
                assert T == MAXW
            else:
                assert abs(T / 2.0**32 - np.exp(2 * beta * B[row] / L * A)) <= 2.0**-32


def _component(lat, k, tau0, joined):
    """Slices reachable from tau0 through joined ring bonds, by graph search."""
    L = lat.shape[0]
    seen, todo = {tau0}, [tau0]
    while todo:
        t = todo.pop()
        for b, (x, y) in enumerate((i, (i + 1) % L) for i in range(L)):
            if joined[b] and t in (x, y):
                o = y if t == x else x
                if o not in seen:
                    seen.add(o)
                    todo.append(o)
    return seen


@pytest.mark.parametrize("L", [2, 3, 8, 17, 64])
def test_cluster_is_component_of_seed(L):
    """The flipped set is the connected component of the seed slice in the graph of
    joined bonds; a bond joins only aligned slices; the ring closes (L = 64 too)."""
    rng = np.random.default_rng(L)
    emb = O.Embedding(O.ME, sk_instance(3, 9), -2)
    n = emb.n_sites
    _, acc = O.wolff_tables(1.0, L, np.array([1.0]), emb.fmax)
    padd = 1 << 31
    for trial in range(40):
        lat = np.where(rng.random((1, L, n)) < 0.3, -1, 1).astype(np.int8)
        if trial % 5 == 0:
            lat[0, :, 1] = 1                           # aligned ring
        k = int(rng.integers(0, n))
        tau0 = int(rng.integers(0, L))
        words = rng.integers(0, 2**32, L, dtype=np.uint64).astype(np.uint32)
        if trial % 5 == 0:
            k, words[:] = 1, 0                         # every bond joins: the whole ring
        before = lat.copy()
        thr, cl = O.wolff_move(emb, L, lat, k, tau0, words, 0, padd, acc[0])
        joined = [before[0, b, k] == before[0, (b + 1) % L, k] and int(words[b]) < padd for b in range(L)]
        comp = _component(before[0], k, tau0, joined)
        assert {t for t in range(L) if (int(cl[0]) >> t) & 1} == comp
        if trial % 5 == 0:
            assert len(comp) == L
        # A = sum over the cluster of s f, from the logical-energy change of flipping it
        flipped = before.copy()
        for t in comp:
            flipped[0, t, k] = -flipped[0, t, k]
        dE = sum(emb.energy(flipped[0, t]) - emb.energy(before[0, t]) for t in range(L))
        A = -dE // 2
        assert int(thr[0]) == int(acc[0, A + L * emb.fmax])
        if int(thr[0]) > 0:
            assert (lat == flipped).all()
        else:
            assert (lat == before).all()


def test_words_follow_counter_layout():
    seed = 0x0123456789ABCDEF
    key = [seed & 0xFFFFFFFF, seed >> 32]
    for (r, k, b, m) in [(0, 0, 0, 0), (3, 17, 63, 9999), (65535, 275, 5, 123456), (1, 2, 12, 3)]:
        # bonds 8q..8q+7 share one call per stream; bond 8q+j takes half j >> 2 of word j & 3
        hi = int(O.philox4x32([k, b >> 3, m, (O.STREAM_WOLFF << 24) | r], key)[b & 3])
        lo = int(O.philox4x32([k, b >> 3, m, (O.STREAM_WOLFF_LO << 24) | r], key)[b & 3])
        sh = 16 * ((b >> 2) & 1)
        assert O.wolff_bond_uniform(seed, r, k, b, m) == ((((hi >> sh) & 0xFFFF) << 16) | ((lo >> sh) & 0xFFFF))
        ph = O.philox4x32([k, 64, m, (O.STREAM_WOLFF << 24) | r], key)
        assert O.wolff_site_words(seed, r, k, m) == (int(ph[0]), int(ph[1]))


@pytest.mark.parametrize("kind,N,L,R", [(O.ME, 4, 4, 2), (O.LHZ, 5, 6, 3), (O.LHZ, 4, 1, 2), (O.ME, 3, 64, 1)])
def test_run_is_order_words_and_moves(kind, N, L, R):
    """The oracle's anneal equals replaying its site order with its bond uniforms and
    WOLFF-stream site words (seed slice floor(u L / 2^32)), its per-sweep join
    threshold and its acceptance row."""
    seed = 0xABCDEF12345
    emb = O.Embedding(kind, sk_instance(N, 70), -2)
    M = 4
    padd, acc = O.wolff_tables(4.0, L, O.gamma_schedule(2.0, 0.1, M), emb.fmax)
    spins = O.sqa_init(emb, L, R, seed)
    ref = spins.copy()
    O.wolff_run(emb, L, spins, 0, M, padd, acc, seed)
    order = O.wolff_site_order(emb).tolist()
    assert sorted(order) == list(range(emb.n_sites))
    assert [int(emb.colour[k]) for k in order] == sorted(int(emb.colour[k]) for k in order)
    for r in range(R):
        for m in range(M):
            for k in order:
                us, ua = O.wolff_site_words(seed, r, k, m)
                tau0 = (us * L) >> 32
                words = np.array([O.wolff_bond_uniform(seed, r, k, b, m) for b in range(L)], dtype=np.uint32)
                O.wolff_move(emb, L, ref[r:r + 1], k, tau0, words, ua, padd[m], acc[0])
    assert (spins == ref).all()


def test_resume_and_threads_are_bit_identical():
    emb = O.Embedding(O.LHZ, sk_instance(6, 3), -2)
    M, L = 30, 8
    padd, acc = O.wolff_tables(5.0, L, O.gamma_schedule(3.0, 0.01, M), emb.fmax)
    a = O.sqa_init(emb, L, 4, 17)
    b = a.copy()
    O.wolff_run(emb, L, a, 0, M, padd, acc, 17)
    O.wolff_run(emb, L, b, 0, 11, padd, acc, 17)
    O.wolff_run(emb, L, b, 11, M, padd, acc, 17, nthreads=3)
    assert (a == b).all()
    c = O.sqa_init(emb, L, 2, 17, r0=2)
    O.wolff_run(emb, L, c, 0, M, padd, acc, 17, r0=2)
    assert (c == a[2:]).all()


def test_anneal_reaches_ground_state_of_small_instance():
    """End-to-end sanity: slow annealing with Wolff moves finds the logical ground
    energy (ME, chains intact) for a small instance on most replicas."""
    J = sk_instance(4, 11)
    e0 = O.ground_states(J)[0]
    emb, _, spins, E = O.sqa_anneal_wolff(O.ME, J, -2, 8.0, 8, 400, 16, 3.0, 0.01, 5, nthreads=4)
    le = np.array([O.logical_energy(J, O.me_majority(emb, spins[r, 0])) for r in range(16)])
    assert (le == e0).mean() >= 0.6
