/*
 * SQA with time-like Wolff cluster updates, for the oracle (test
 * infrastructure only: nothing in the library links or calls this file).
 *
 * Sec. III: in the paper's SQA one sweep applies, for every spatial site, a
 * Wolff cluster update along imaginary time (the implementation itself is
 * described in a reference the paper cites; what follows is the textbook
 * form of that move, reconstructed from the Trotter action of tables.c).
 * The L slices of site k form a ring; neighbouring slices are coupled
 * ferromagnetically with J_perp = -1/2 ln tanh(beta Gamma / L), and slice tau
 * feels the field f_k^tau of the other sites of the same slice.  The move:
 *   1. a seed slice tau0, uniform on 0..L-1;
 *   2. ring bond b joins slices b and b+1 (mod L) with probability
 *      p_add = 1 - exp(-2 J_perp) = 1 - tanh(beta Gamma / L) when their spins
 *      are equal, never otherwise (one independent decision per bond);
 *   3. the cluster C is the set of slices connected to tau0 by joined bonds
 *      (a run of the ring, or the whole ring);
 *   4. flipping C changes only the spatial part of the action, by
 *      -2 (beta B / L) A with A = sum_{tau in C} s_k^tau f_k^tau; the flip is
 *      accepted with min(1, exp(2 (beta B / L) A)).
 * Bonds inside C keep their alignment, and the join probabilities make the
 * proposal ratio of the two boundary bonds cancel their J_perp weight, so
 * the move satisfies detailed balance for the Trotter distribution.  With L = 1
 * there are no bonds (p_add = 0) and the move is single-spin Metropolis.
 *
 * Readings where the paper is silent: every sweep visits the sites by colour
 * class 0..3 and, inside a class, by increasing site index (sites of one
 * class share no term, so their moves commute); tau0 = floor(u L / 2^32).
 * Random numbers (Philox4x32-10, key = seed):
 *   bond b of site k, sweep m, replica r: the 32-bit uniform (hi << 16) | lo,
 *     hi and lo being the 16-bit half (b >> 2) & 1 (0 = low, 1 = high) of
 *     word b & 3 of counter (k, b >> 3, m, stream << 24 | r), with stream
 *     WOLFF = 7 for hi and WOLFF_LO = 9 for lo (one call serves the eight
 *     bonds 8q..8q+7; lo matters only when hi equals the threshold's top half);
 *   seed word and acceptance word: words 0 and 1 of counter (k, 64, m, 7 << 24 | r).
 * Decisions use the threshold rule of tables.c (accept iff always-code or
 * u < threshold).  Tables: padd[m] per sweep; acc[row][A + L F] with A in
 * [-L F, L F], one row per sweep when B varies (bscale given), else one row.
 */
#include <math.h>
#include <pthread.h>
#include <stdlib.h>
#include <string.h>
#include "oracle.h"

static uint32_t wolff_word(uint64_t seed, uint32_t stream, uint32_t r, uint32_t k, uint32_t c1, uint32_t m,
                           int w) {
  uint32_t ctr[4], key[2], out[4];
  ctr[0] = k;
  ctr[1] = c1;
  ctr[2] = m;
  ctr[3] = (stream << 24) | r;
  key[0] = (uint32_t)seed;
  key[1] = (uint32_t)(seed >> 32);
  oracle_philox4x32(ctr, key, out);
  return out[w];
}

uint32_t oracle_wolff_bond_uniform(uint64_t seed, uint32_t r, uint32_t k, uint32_t b, uint32_t m) {
  int half = (int)((b >> 2) & 1u);
  uint32_t whi = wolff_word(seed, OR_STREAM_WOLFF, r, k, b >> 3, m, (int)(b & 3u));
  uint32_t wlo = wolff_word(seed, OR_STREAM_WOLFF_LO, r, k, b >> 3, m, (int)(b & 3u));
  uint32_t hi = half ? (whi >> 16) : (whi & 0xFFFFu);
  uint32_t lo = half ? (wlo >> 16) : (wlo & 0xFFFFu);
  return (hi << 16) | lo;
}

void oracle_wolff_site_words(uint64_t seed, uint32_t r, uint32_t k, uint32_t m, uint32_t *u_seed,
                             uint32_t *u_acc) {
  *u_seed = wolff_word(seed, OR_STREAM_WOLFF, r, k, 64u, m, 0);
  *u_acc = wolff_word(seed, OR_STREAM_WOLFF, r, k, 64u, m, 1);
}

void oracle_wolff_tables(double beta, int32_t L, int32_t M, const double *gamma,
                         const double *bscale, int32_t F, uint32_t *padd, uint32_t *acc) {
  int rows = bscale ? M : 1;
  int width = 2 * L * F + 1;
  for (int m = 0; m < M; ++m)
    padd[m] = (L > 1) ? oracle_threshold(log(1.0 - tanh(beta * gamma[m] / (double)L))) : 0u;
  for (int row = 0; row < rows; ++row) {
    double B = bscale ? bscale[row] : 1.0;
    double bl = beta * B / (double)L;
    for (int A = -L * F; A <= L * F; ++A)
      acc[(size_t)row * width + (A + L * F)] = oracle_threshold(2.0 * (bl * (double)A));
  }
}

static int passes(uint32_t u, uint32_t T) { return T == 0xFFFFFFFFu || u < T; }

/* One cluster move of site k on each of `count` lattices [L][n], all with the
 * same random words: seed slice tau0, bond words bond_u[L], acceptance word
 * u_acc, join threshold padd and acceptance row acc_row[2 L F + 1].  The
 * acceptance threshold used for lattice i is written to thr_out[i] (if not
 * NULL) and the cluster (bit tau = slice tau in C) to cl_out[i] (if not NULL). */
void oracle_wolff_move(const OEmb *e, int32_t L, int32_t count, int8_t *lats, int32_t k, int32_t tau0,
                       const uint32_t *bond_u, uint32_t u_acc, uint32_t padd, const uint32_t *acc_row,
                       int32_t F, uint32_t *thr_out, uint64_t *cl_out) {
  int n = e->n_sites;
  int8_t joined[64], in[64];
  for (int i = 0; i < count; ++i) {
    int8_t *lat = lats + (size_t)i * L * n;
    for (int b = 0; b < L; ++b) {
      int nb = (b + 1) % L;
      int equal = lat[(size_t)b * n + k] == lat[(size_t)nb * n + k];
      joined[b] = (int8_t)(L > 1 && equal && passes(bond_u[b], padd));
    }
    /* connected component of tau0 on the ring */
    memset(in, 0, sizeof in);
    in[tau0] = 1;
    for (int t = tau0; joined[t] && !in[(t + 1) % L]; t = (t + 1) % L) in[(t + 1) % L] = 1;
    for (int t = tau0; joined[(t - 1 + L) % L] && !in[(t - 1 + L) % L]; t = (t - 1 + L) % L) in[(t - 1 + L) % L] = 1;
    int A = 0;
    uint64_t cl = 0;
    for (int t = 0; t < L; ++t) {
      if (!in[t]) continue;
      A += lat[(size_t)t * n + k] * oracle_local_field(e, lat + (size_t)t * n, k);
      cl |= 1ull << t;
    }
    uint32_t T = acc_row[A + L * F];
    if (thr_out) thr_out[i] = T;
    if (cl_out) cl_out[i] = cl;
    if (passes(u_acc, T))
      for (int t = 0; t < L; ++t)
        if (in[t]) lat[(size_t)t * n + k] = (int8_t)-lat[(size_t)t * n + k];
  }
}

/* Sites of one sweep in update order (colour class, then index). */
int32_t oracle_wolff_site_order(const OEmb *e, int32_t *site_out) {
  int cnt = 0;
  for (int c = 0; c < 4; ++c)
    for (int k = 0; k < e->n_sites; ++k)
      if (e->colour[k] == c) site_out[cnt++] = k;
  return cnt;
}

typedef struct {
  const OEmb *e;
  int32_t L, r0, R, m0, m1, rows, F, first, stride;
  const uint32_t *padd, *acc;
  uint64_t seed;
  int8_t *spins;
} WJob;

static void *wolff_worker(void *arg) {
  WJob *j = (WJob *)arg;
  const OEmb *e = j->e;
  int n = e->n_sites, L = j->L, width = 2 * L * j->F + 1;
  int32_t *order = (int32_t *)malloc(sizeof(int32_t) * (size_t)n);
  int cnt = oracle_wolff_site_order(e, order);
  uint32_t bond_u[64];
  for (int r = j->first; r < j->R; r += j->stride) {
    int8_t *lat = j->spins + (size_t)L * n * r;
    uint32_t rep = (uint32_t)(j->r0 + r);
    for (int m = j->m0; m < j->m1; ++m) {
      const uint32_t *row = j->acc + (size_t)(j->rows > 1 ? m : 0) * width;
      for (int i = 0; i < cnt; ++i) {
        int k = order[i];
        uint32_t us, ua;
        oracle_wolff_site_words(j->seed, rep, (uint32_t)k, (uint32_t)m, &us, &ua);
        int tau0 = (int)(((uint64_t)us * (uint64_t)L) >> 32);
        for (int b = 0; b < L; ++b) bond_u[b] = oracle_wolff_bond_uniform(j->seed, rep, (uint32_t)k, (uint32_t)b, (uint32_t)m);
        oracle_wolff_move(e, L, 1, lat, k, tau0, bond_u, ua, j->padd[m], row, j->F, NULL, NULL);
      }
    }
  }
  free(order);
  return NULL;
}

/* Sweeps m0..m1-1 on replicas r0..r0+R-1 held in spins[R][L][n] (L <= 64). */
void oracle_wolff_run(const OEmb *e, int32_t L, int32_t r0, int32_t R, int32_t m0, int32_t m1,
                      const uint32_t *padd, const uint32_t *acc, int32_t rows, int32_t F,
                      uint64_t seed, int8_t *spins, int32_t nthreads) {
  if (R <= 0) return;
  if (nthreads < 1) nthreads = 1;
  if (nthreads > R) nthreads = R;
  WJob *jobs = (WJob *)malloc(sizeof(WJob) * (size_t)nthreads);
  pthread_t *th = (pthread_t *)malloc(sizeof(pthread_t) * (size_t)nthreads);
  for (int t = 0; t < nthreads; ++t) {
    WJob j = {e, L, r0, R, m0, m1, rows, F, t, nthreads, padd, acc, seed, spins};
    jobs[t] = j;
  }
  for (int t = 1; t < nthreads; ++t) pthread_create(&th[t], NULL, wolff_worker, &jobs[t]);
  wolff_worker(&jobs[0]);
  for (int t = 1; t < nthreads; ++t) pthread_join(th[t], NULL);
  free(jobs);
  free(th);
}
