/*
 * Decoders and exact ground states for the oracle (test infrastructure only).
 */
#include <math.h>
#include <stdlib.h>
#include <string.h>
#include "oracle.h"

/* Eq. (4), Sec. II D: majority vote over each ME chain, qbar_i = sign sum_r q_{i,r}.
 * Tie (possible when the chain length is even) -> +1, a reading.  Chains of
 * N-1 spins (clique chains) or ceil(N/4)+1 spins (Chimera). */
void oracle_me_majority(const OEmb *e, const int8_t *slice, int8_t *logical) {
  int N = e->N;
  int len = e->kind == OR_MEC ? oracle_chimera_m(N) + 1 : N - 1;
  for (int i = 0; i < N; ++i) {
    int sum = 0;
    for (int r = 0; r < len; ++r) sum += slice[i * len + r];
    logical[i] = (sum >= 0) ? (int8_t)1 : (int8_t)-1;
  }
}

static int pair_site(int N, int a, int b) {
  return a < b ? oracle_lhz_site(N, a, b) : oracle_lhz_site(N, b, a);
}

static int8_t tree_value(int N, const int8_t *slice, const int32_t *parent, int8_t *memo, int v) {
  if (memo[v]) return memo[v];
  int8_t val;
  if (parent[v] < 0) val = 1;
  else val = (int8_t)(tree_value(N, slice, parent, memo, parent[v]) * slice[pair_site(N, v, parent[v])]);
  memo[v] = val;
  return val;
}

/* Eq. (5), Sec. II E and Appendix A: each spanning tree of K_N, rooted at
 * logical spin 0 with qbar_0 = +1, decodes qbar_child = qbar_parent * q_{child,parent};
 * the result is the majority over the trees, tie -> +1 (a reading).
 * parents[t*N + v] is the parent of v in tree t, -1 for the root 0.
 * The chain tree of Eq. (A1) is parent(v) = v-1, the star of Eq. (A2) parent(v) = 0. */
void oracle_lhz_tree_decode(int32_t N, const int8_t *slice, const int32_t *parents,
                            int32_t n_trees, int8_t *logical) {
  int *votes = (int *)calloc((size_t)N, sizeof(int));
  int8_t *memo = (int8_t *)malloc((size_t)N);
  for (int t = 0; t < n_trees; ++t) {
    memset(memo, 0, (size_t)N);
    for (int v = 0; v < N; ++v) votes[v] += tree_value(N, slice, parents + (size_t)t * N, memo, v);
  }
  for (int v = 0; v < N; ++v) logical[v] = votes[v] >= 0 ? (int8_t)1 : (int8_t)-1;
  free(votes);
  free(memo);
}

/* Random spanning trees (the paper draws "random spanning trees" without a
 * distribution; the reading is uniform labelled trees).  Tree t is decoded
 * from a Pruefer sequence whose entry i is floor(u * N / 2^32), u = word 0 of
 * the TREE-stream Philox call with counter (i, t, 0, TREE<<24); the sequence
 * is turned into edges with the smallest-leaf rule and rooted at vertex 0.
 * Returns 0, or -1 if N < 1. */
int oracle_random_trees(uint64_t seed, int32_t N, int32_t n_trees, int32_t *parents) {
  if (N < 1) return -1;
  int *seq = (int *)malloc(sizeof(int) * (size_t)(N > 2 ? N - 2 : 1));
  int *deg = (int *)malloc(sizeof(int) * (size_t)N);
  int *eu = (int *)malloc(sizeof(int) * (size_t)N);
  int *ev = (int *)malloc(sizeof(int) * (size_t)N);
  int *queue = (int *)malloc(sizeof(int) * (size_t)N);
  uint32_t key[2] = {(uint32_t)seed, (uint32_t)(seed >> 32)};
  for (int t = 0; t < n_trees; ++t) {
    int32_t *par = parents + (size_t)t * N;
    int ne = 0;
    for (int i = 0; i + 2 < N; ++i) {
      uint32_t ctr[4] = {(uint32_t)i, (uint32_t)t, 0u, (uint32_t)OR_STREAM_TREE << 24};
      uint32_t out[4];
      oracle_philox4x32(ctr, key, out);
      seq[i] = (int)(((uint64_t)out[0] * (uint64_t)N) >> 32);
    }
    for (int v = 0; v < N; ++v) deg[v] = 1;
    for (int i = 0; i + 2 < N; ++i) deg[seq[i]]++;
    for (int i = 0; i + 2 < N; ++i) {
      int leaf = 0;
      while (deg[leaf] != 1) ++leaf;
      eu[ne] = leaf; ev[ne] = seq[i]; ++ne;
      deg[leaf]--;
      deg[seq[i]]--;
    }
    if (N >= 2) {
      int a = -1, b = -1;
      for (int v = 0; v < N; ++v)
        if (deg[v] == 1) { if (a < 0) a = v; else b = v; }
      eu[ne] = a; ev[ne] = b; ++ne;
    }
    /* root at 0 by breadth-first search */
    for (int v = 0; v < N; ++v) par[v] = -2;
    par[0] = -1;
    int head = 0, tail = 0;
    queue[tail++] = 0;
    while (head < tail) {
      int x = queue[head++];
      for (int q = 0; q < ne; ++q) {
        int y = -1;
        if (eu[q] == x) y = ev[q];
        else if (ev[q] == x) y = eu[q];
        if (y >= 0 && par[y] == -2) { par[y] = x; queue[tail++] = y; }
      }
    }
  }
  free(seq); free(deg); free(eu); free(ev); free(queue);
  return 0;
}

/* Minimum-weight decoding, Sec. IV A, Eqs. (6)-(10).  The MWD state is the
 * constraint-satisfying physical state nearest to s in Hamming distance.
 * Constraint-satisfying states are exactly q_ij = sigma_i sigma_j, and
 * Hamming(s, q) = K/2 - (1/2) sum_{i<j} s_ij sigma_i sigma_j, so the decoded
 * logical state maximises sum_{i<j} s_ij sigma_i sigma_j: the ground state of
 * Eq. (9) with the gauge g = s.  (Read literally, Eq. (10) with e^g_k as
 * defined before it applies g twice; the Hamming-distance definition of MWD is
 * followed.)  Enumeration: sigma_0 = +1, candidate m = 0 .. 2^(N-1)-1 with
 * sigma_{b+1} = -1 iff bit b of m is set; ties go to the smallest m (a
 * reading). */
void oracle_lhz_mwd(int32_t N, const int8_t *slice, int8_t *logical) {
  int8_t *sig = (int8_t *)malloc((size_t)N);
  long best = -(1L << 40);
  uint64_t best_m = 0;
  uint64_t count = 1ull << (N - 1);
  for (uint64_t m = 0; m < count; ++m) {
    sig[0] = 1;
    for (int b = 0; b + 1 < N; ++b) sig[b + 1] = ((m >> b) & 1u) ? (int8_t)-1 : (int8_t)1;
    long score = 0;
    for (int i = 0; i < N; ++i)
      for (int j = i + 1; j < N; ++j) score += slice[oracle_lhz_site(N, i, j)] * sig[i] * sig[j];
    if (score > best) { best = score; best_m = m; }
  }
  logical[0] = 1;
  for (int b = 0; b + 1 < N; ++b) logical[b + 1] = ((best_m >> b) & 1u) ? (int8_t)-1 : (int8_t)1;
  free(sig);
}

/* Exact ground states of Eq. (1) by enumerating all 2^N states in Gray-code
 * order (one spin flip per step, energy updated by the flip's change).
 * Writes up to max_states ground states to states[max_states][N]; returns the
 * ground energy and stores the total number of ground states in *n_found. */
int32_t oracle_ground_states(int32_t N, const int32_t *J, const int32_t *h,
                             int8_t *states, int32_t max_states, int32_t *n_found) {
  int8_t *sig = (int8_t *)malloc((size_t)N);
  for (int i = 0; i < N; ++i) sig[i] = 1;
  int32_t E = oracle_logical_energy(N, J, h, sig);
  int32_t best = E;
  int32_t found = 0;
  uint64_t total = 1ull << N;
  for (uint64_t g = 0; g < total; ++g) {
    if (g > 0) {
      int b = __builtin_ctzll(g);   /* Gray code: step g flips bit ctz(g) */
      int32_t f = h ? h[b] : 0;
      for (int j = 0; j < N; ++j)
        if (j != b) f += (j < b ? J[j * N + b] : J[b * N + j]) * sig[j];
      E += -2 * sig[b] * f;
      sig[b] = (int8_t)-sig[b];
    }
    if (E < best) { best = E; found = 0; }
    if (E == best) {
      if (found < max_states) memcpy(states + (size_t)found * N, sig, (size_t)N);
      ++found;
    }
  }
  *n_found = found;
  free(sig);
  return best;
}

/* Weight-3 parity-check decoding (Sec. IV D; its settings in Sec. IV E and
 * Appendix C).  The paper follows an implementation it cites and describes it
 * only in words: the alignment of each pair (i, j) is updated iteratively by a
 * majority vote over the N-2 weight-3 checks q_il q_lj (l != i, j), given an
 * error rate, and one spanning tree then reads the logical state.  Reading:
 * the vote weighs the pair's own readout s_ij by its log-likelihood ratio
 * w0 = ln((1-p)/p) and each check by the ratio of a product of two bits,
 * w1 = ln((1-p2)/p2) with p2 = 2p(1-p); all pairs are updated together from
 * the previous iteration's values,
 *   x_ij <- sign(w0 s_ij + w1 sum_l x_il x_lj),  an exact tie keeps s_ij,
 * starting from x = s; after `iterations` rounds the trees decode x as in
 * Eq. (5).  0 < p < 1/2.  pairs_out (K entries, LHZ site order) may be NULL. */
void oracle_lhz_bp(int32_t N, const int8_t *slice, double error_rate, int32_t iterations,
                   const int32_t *parents, int32_t n_trees, int8_t *logical, int8_t *pairs_out) {
  int K = N * (N - 1) / 2;
  double p = error_rate, p2 = 2.0 * p * (1.0 - p);
  double w0 = log((1.0 - p) / p), w1 = log((1.0 - p2) / p2);
  int8_t *x = (int8_t *)malloc((size_t)K), *xn = (int8_t *)malloc((size_t)K);
  memcpy(x, slice, (size_t)K);
  for (int it = 0; it < iterations; ++it) {
    for (int i = 0; i < N; ++i)
      for (int j = i + 1; j < N; ++j) {
        int c = 0;
        for (int l = 0; l < N; ++l)
          if (l != i && l != j) c += x[pair_site(N, i, l)] * x[pair_site(N, l, j)];
        int k = oracle_lhz_site(N, i, j);
        double v = w0 * (double)slice[k] + w1 * (double)c;
        xn[k] = v > 0.0 ? (int8_t)1 : (v < 0.0 ? (int8_t)-1 : slice[k]);
      }
    memcpy(x, xn, (size_t)K);
  }
  oracle_lhz_tree_decode(N, x, parents, n_trees, logical);
  if (pairs_out) memcpy(pairs_out, x, (size_t)K);
  free(x);
  free(xn);
}

/* Maximum-likelihood decoding, Sec. IV B, Eq. (11): the thermal average at the
 * Nishimori inverse temperature beta_N = (1/2) ln((1-p)/p) of the decoding
 * problem of Eq. (9) in the gauge g = s, P(sigma) ~ exp(beta_N sum_{i<j}
 * s_ij sigma_i sigma_j).  That law is symmetric under sigma -> -sigma, so the
 * gauge is fixed by sigma_0 = +1 and qbar_i = sign <sigma_0 sigma_i> (tie ->
 * +1).  With O = sum s_ij sigma_i sigma_j and O_max its maximum over the states
 * (the MWD score), every state's weight exp(-beta_N (O_max - O)) is quantised
 * to round(2^36 exp(-beta_N (O_max - O))) and the averages are summed in 64-bit
 * integers (exact, independent of summation order); N <= 24 keeps the sums
 * below 2^63.  corr_out[i] (may be NULL) receives the integer numerator of
 * <sigma_0 sigma_i>. */
static int pair_score(int32_t N, const int8_t *slice, const int8_t *sig) {
  int o = 0;
  for (int i = 0; i < N; ++i)
    for (int j = i + 1; j < N; ++j) o += slice[oracle_lhz_site(N, i, j)] * sig[i] * sig[j];
  return o;
}

static void candidate(int32_t N, uint64_t m, int8_t *sig) {
  sig[0] = 1;
  for (int b = 0; b + 1 < N; ++b) sig[b + 1] = ((m >> b) & 1u) ? (int8_t)-1 : (int8_t)1;
}

void oracle_lhz_mld(int32_t N, const int8_t *slice, double error_rate, int8_t *logical, int64_t *corr_out) {
  int K = N * (N - 1) / 2;
  double beta = 0.5 * log((1.0 - error_rate) / error_rate);
  int8_t *sig = (int8_t *)malloc((size_t)N);
  uint64_t count = 1ull << (N - 1);
  int omax = -K;
  for (uint64_t m = 0; m < count; ++m) {
    candidate(N, m, sig);
    int o = pair_score(N, slice, sig);
    if (o > omax) omax = o;
  }
  uint64_t *w = (uint64_t *)malloc(sizeof(uint64_t) * (size_t)(2 * K + 1));
  for (int d = 0; d <= 2 * K; ++d) w[d] = (uint64_t)llround(ldexp(exp(-beta * (double)d), 36));
  int64_t *acc = (int64_t *)calloc((size_t)N, sizeof(int64_t));
  for (uint64_t m = 0; m < count; ++m) {
    candidate(N, m, sig);
    int64_t wt = (int64_t)w[omax - pair_score(N, slice, sig)];
    for (int i = 0; i < N; ++i) acc[i] += sig[i] > 0 ? wt : -wt;
  }
  for (int i = 0; i < N; ++i) {
    logical[i] = acc[i] >= 0 ? (int8_t)1 : (int8_t)-1;
    if (corr_out) corr_out[i] = acc[i];
  }
  free(w);
  free(acc);
  free(sig);
}
