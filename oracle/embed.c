/*
 * Embedded physical Hamiltonians for the oracle (test infrastructure only).
 *
 * Logical problem, Eq. (1) of Sec. II:
 *   H_P = sum_i h_i s_i + sum_{i<j} J_ij s_i s_j,
 * with J < 0 ferromagnetic.  Two embeddings of the complete graph K_N:
 *
 * ME (Sec. II A).  Each logical spin becomes a chain of physical spins tied by
 * ferromagnetic penalty couplings.  The paper's Chimera layout (chains of
 * ceil(N/4)+1 spins) is only drawn in a figure; the reading used here is the
 * clique-chain layout: chain i holds N-1 spins p(i,r) = i(N-1)+r, consecutive
 * chain spins are coupled with the penalty coefficient J_F, and J_ij sits on
 * the single edge between slot j-1 of chain i and slot i of chain j (i<j).
 * A logical field h_i sits on p(i,0).
 *
 * LHZ (Sec. II B, Eq. (3)).  One physical spin q_ij per logical pair, index
 * k(i,j) = i(2N-i-1)/2 + (j-i-1), carrying the field J_ij.  Constraint terms
 * C * prod(q) with the signed coefficient C (the paper's -lambda):
 *   4-body plaquettes {(i,j),(i,j+1),(i+1,j),(i+1,j+1)}, i+2 <= j <= N-2,
 *   3-body triangles  {(i,i+1),(i,i+2),(i+1,i+2)},        0 <= i <= N-3,
 * i.e. (N-3)(N-2)/2 + (N-2) = C(N-1,2) constraints, the count the paper gives.
 * The triangle row along the diagonal is the three-body edge of the LHZ graph.
 * Logical fields need an ancilla qubit (Sec. II B) and are rejected here.
 *
 * ME on Chimera (Sec. II A).  Chimera C_m is an m x m grid of K_{4,4} cells;
 * qubit (r, c, side, k) with side V (vertical) or H (horizontal), k = 0..3.
 * Couplers: inside a cell every V qubit with every H qubit; between cells
 * V(r,c,k)-V(r+1,c,k) and H(r,c,k)-H(r,c+1,k).  The paper uses Choi's clique
 * embedding with chains of ceil(N/4)+1 qubits (drawn only in a figure); the
 * reading here is the triangle construction with m = ceil(N/4): logical spin i
 * of block b = i/4, k = i%4, owns the H qubits of row b in columns 0..b and the
 * V qubits of column b in rows b..m-1, m+1 qubits joined at cell (b, b).  Its
 * chain slots t = 0..m are H(b, t, k) for t <= b and V(t-1, b, k) for t > b,
 * physical site i(m+1)+t; consecutive slots are coupled with J_F.  Chains of
 * blocks a < b meet in cell (b, a): J_ij (i in block a, j in block b) sits on
 * V(b, a, k_i)-H(b, a, k_j), i.e. slot b+1 of chain i and slot a of chain j;
 * chains of one block (k_i < k_j) meet in cell (a, a): slot a+1 of chain i
 * (V) with slot a of chain j (H).  h_i sits on slot 0.
 *
 * Colouring (a reading; the paper fixes no update order): four colours with
 * no term joining two sites of one colour,
 *   ME : colour(p(i,r)) = (r&1) | ((i&1)<<1)
 *   LHZ: colour(k(i,j)) = (i&1) | ((j&1)<<1)
 *   ME on Chimera: colour = (row + column + side) & 1, side H = 1 (Chimera is
 *   bipartite: every coupler joins qubits of different colour).
 */
#include <stdlib.h>
#include <string.h>
#include "oracle.h"

int32_t oracle_me_site(int32_t N, int32_t i, int32_t r) { return i * (N - 1) + r; }

int32_t oracle_chimera_m(int32_t N) { return (N + 3) / 4; }

int32_t oracle_chimera_site(int32_t N, int32_t i, int32_t t) { return i * (oracle_chimera_m(N) + 1) + t; }

/* Cell coordinates of slot t of chain i: row, column, side (0 = V, 1 = H), k. */
void oracle_chimera_qubit(int32_t N, int32_t i, int32_t t, int32_t *row, int32_t *col, int32_t *side,
                          int32_t *k) {
  (void)N;
  int b = i / 4;
  *k = i % 4;
  if (t <= b) { *row = b; *col = t; *side = 1; }
  else { *row = t - 1; *col = b; *side = 0; }
}

int32_t oracle_lhz_site(int32_t N, int32_t i, int32_t j) {
  return i * (2 * N - i - 1) / 2 + (j - i - 1);
}

static int iabs(int v) { return v < 0 ? -v : v; }

static void add_term(OEmb *e, int32_t w, int32_t a, int32_t b, int32_t c, int32_t d) {
  int t = e->n_terms++;
  int32_t *ts = e->tsite + 4 * t;
  e->w[t] = w;
  ts[0] = a; ts[1] = b; ts[2] = c; ts[3] = d;
  e->arity[t] = (c < 0) ? 2 : (d < 0 ? 3 : 4);
}

static void finish(OEmb *e) {
  int n = e->n_sites;
  e->row = (int32_t *)calloc((size_t)n + 1, sizeof(int32_t));
  int *cnt = (int *)calloc((size_t)n, sizeof(int));
  for (int t = 0; t < e->n_terms; ++t)
    for (int q = 0; q < e->arity[t]; ++q) cnt[e->tsite[4 * t + q]]++;
  for (int k = 0; k < n; ++k) e->row[k + 1] = e->row[k] + cnt[k];
  e->inc = (int32_t *)malloc(sizeof(int32_t) * (size_t)(e->row[n] > 0 ? e->row[n] : 1));
  memset(cnt, 0, sizeof(int) * (size_t)n);
  for (int t = 0; t < e->n_terms; ++t)
    for (int q = 0; q < e->arity[t]; ++q) {
      int k = e->tsite[4 * t + q];
      e->inc[e->row[k] + cnt[k]++] = t;
    }
  free(cnt);
  e->fmax = 0;
  e->emax = 0;
  for (int k = 0; k < n; ++k) {
    int f = iabs(e->h[k]);
    for (int q = e->row[k]; q < e->row[k + 1]; ++q) f += iabs(e->w[e->inc[q]]);
    if (f > e->fmax) e->fmax = f;
    e->emax += iabs(e->h[k]);
  }
  for (int t = 0; t < e->n_terms; ++t) e->emax += iabs(e->w[t]);
}

static void alloc_emb(OEmb *e, int n, int max_terms) {
  e->n_sites = n;
  e->n_terms = 0;
  e->h = (int32_t *)calloc((size_t)n, sizeof(int32_t));
  e->colour = (int32_t *)calloc((size_t)n, sizeof(int32_t));
  e->w = (int32_t *)calloc((size_t)(max_terms > 0 ? max_terms : 1), sizeof(int32_t));
  e->arity = (int32_t *)calloc((size_t)(max_terms > 0 ? max_terms : 1), sizeof(int32_t));
  e->tsite = (int32_t *)calloc((size_t)(max_terms > 0 ? max_terms : 1) * 4, sizeof(int32_t));
}

/* Returns 0 on success, -1 on invalid arguments. */
int oracle_embed(int32_t kind, int32_t N, const int32_t *J, const int32_t *h,
                 int32_t penalty, OEmb *e) {
  memset(e, 0, sizeof(*e));
  e->kind = kind;
  e->N = N;
  if (kind == OR_ME) {
    if (N < 2) return -1;
    int n = N * (N - 1);
    alloc_emb(e, n, N * (N - 2) + N * (N - 1) / 2);
    for (int i = 0; i < N; ++i)
      for (int r = 0; r < N - 1; ++r)
        e->colour[oracle_me_site(N, i, r)] = (r & 1) | ((i & 1) << 1);
    for (int i = 0; i < N; ++i)
      for (int r = 0; r + 1 < N - 1; ++r)
        add_term(e, penalty, oracle_me_site(N, i, r), oracle_me_site(N, i, r + 1), -1, -1);
    for (int i = 0; i < N; ++i)
      for (int j = i + 1; j < N; ++j)
        add_term(e, J[i * N + j], oracle_me_site(N, i, j - 1), oracle_me_site(N, j, i), -1, -1);
    if (h)
      for (int i = 0; i < N; ++i) e->h[oracle_me_site(N, i, 0)] = h[i];
  } else if (kind == OR_LHZ) {
    if (N < 3) return -1;
    if (h)
      for (int i = 0; i < N; ++i)
        if (h[i] != 0) return -1;
    int n = N * (N - 1) / 2;
    alloc_emb(e, n, (N - 1) * (N - 2) / 2);
    for (int i = 0; i < N; ++i)
      for (int j = i + 1; j < N; ++j) {
        int k = oracle_lhz_site(N, i, j);
        e->h[k] = J[i * N + j];
        e->colour[k] = (i & 1) | ((j & 1) << 1);
      }
    for (int i = 0; i + 2 < N; ++i)
      add_term(e, penalty, oracle_lhz_site(N, i, i + 1), oracle_lhz_site(N, i, i + 2),
               oracle_lhz_site(N, i + 1, i + 2), -1);
    for (int i = 0; i < N; ++i)
      for (int j = i + 2; j + 1 < N; ++j)
        add_term(e, penalty, oracle_lhz_site(N, i, j), oracle_lhz_site(N, i, j + 1),
                 oracle_lhz_site(N, i + 1, j), oracle_lhz_site(N, i + 1, j + 1));
  } else if (kind == OR_MEC) {
    if (N < 2) return -1;
    int m = oracle_chimera_m(N);
    int n = N * (m + 1);
    alloc_emb(e, n, N * m + N * (N - 1) / 2);
    for (int i = 0; i < N; ++i)
      for (int t = 0; t <= m; ++t) {
        int r, c, sd, k;
        oracle_chimera_qubit(N, i, t, &r, &c, &sd, &k);
        e->colour[oracle_chimera_site(N, i, t)] = (r + c + sd) & 1;
      }
    for (int i = 0; i < N; ++i)
      for (int t = 0; t < m; ++t)
        add_term(e, penalty, oracle_chimera_site(N, i, t), oracle_chimera_site(N, i, t + 1), -1, -1);
    for (int i = 0; i < N; ++i)
      for (int j = i + 1; j < N; ++j) {
        int a = i / 4, b = j / 4;
        /* V qubit of chain i in row b (slot b+1), H qubit of chain j in column a (slot a) */
        add_term(e, J[i * N + j], oracle_chimera_site(N, i, b + 1), oracle_chimera_site(N, j, a), -1, -1);
      }
    if (h)
      for (int i = 0; i < N; ++i) e->h[oracle_chimera_site(N, i, 0)] = h[i];
  } else {
    return -1;
  }
  finish(e);
  return 0;
}

void oracle_emb_free(OEmb *e) {
  free(e->h); free(e->colour); free(e->w); free(e->arity); free(e->tsite);
  free(e->row); free(e->inc);
  memset(e, 0, sizeof(*e));
}

/* f_k = h_k + sum over terms t containing k of w_t * prod_{k' in t, k' != k} s_k'. */
int32_t oracle_local_field(const OEmb *e, const int8_t *s, int32_t k) {
  int32_t f = e->h[k];
  for (int q = e->row[k]; q < e->row[k + 1]; ++q) {
    int t = e->inc[q];
    int32_t prod = 1;
    for (int a = 0; a < e->arity[t]; ++a) {
      int k2 = e->tsite[4 * t + a];
      if (k2 != k) prod *= s[k2];
    }
    f += e->w[t] * prod;
  }
  return f;
}

/* Energy of one physical configuration, Eq. (1) / Eq. (3) with the terms above. */
int32_t oracle_energy(const OEmb *e, const int8_t *s) {
  int32_t E = 0;
  for (int k = 0; k < e->n_sites; ++k) E += e->h[k] * s[k];
  for (int t = 0; t < e->n_terms; ++t) {
    int32_t prod = 1;
    for (int a = 0; a < e->arity[t]; ++a) prod *= s[e->tsite[4 * t + a]];
    E += e->w[t] * prod;
  }
  return E;
}

/* Eq. (1) on a logical state. */
int32_t oracle_logical_energy(int32_t N, const int32_t *J, const int32_t *h, const int8_t *sigma) {
  int32_t E = 0;
  for (int i = 0; i < N; ++i) {
    if (h) E += h[i] * sigma[i];
    for (int j = i + 1; j < N; ++j) E += J[i * N + j] * sigma[i] * sigma[j];
  }
  return E;
}
