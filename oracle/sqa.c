/*
 * Simulated quantum annealing for the oracle (test infrastructure only).
 *
 * Discrete-time path-integral Monte Carlo (Sec. III; Appendix B): L Trotter
 * slices of the embedded physical system, periodic in imaginary time, updated
 * by single-site Metropolis moves with the acceptance tables of tables.c while
 * Gamma is annealed, one schedule step per sweep.  (The paper's own move, a
 * time-like Wolff cluster update, is in wolff.c; this file is the single-site
 * Metropolis move on the space-time lattice.)
 *
 * Sweep order, a reading (the paper only says "sweep"): for slice parity
 * p = 0, 1; for colour c = 0..3; for every slice tau with tau = p (mod 2); for
 * every site k of colour c in increasing order: one attempt on (k, tau).
 * L must be even (or 1, the classical limit) so that slices of one parity are
 * not time neighbours.  Within one (parity, colour) class no two attempts share
 * a term or a time bond, so the order inside a class does not change results.
 *
 * Initial state (paper silent): s = -1 if bit 31 of the INIT-stream word for
 * (replica, slice, site, sweep 0) is set, else +1.
 *
 * Metropolis test: flip iff the threshold is the always-code or u < threshold,
 * with u the attempt's 32-bit uniform (oracle_sqa_uniform, philox.c).
 */
#include <pthread.h>
#include <stdlib.h>
#include "oracle.h"

/* Replicas r0 .. r0+R-1 into spins[R][L][n]. */
void oracle_sqa_init_from(const OEmb *e, int32_t L, int32_t r0, int32_t R, uint64_t seed, int8_t *spins) {
  int n = e->n_sites;
  for (int r = 0; r < R; ++r)
    for (int tau = 0; tau < L; ++tau)
      for (int k = 0; k < n; ++k) {
        uint32_t u = oracle_sqa_word(seed, OR_STREAM_INIT, (uint32_t)(r0 + r), (uint32_t)k,
                                     (uint32_t)tau, 0u);
        spins[((size_t)r * L + tau) * n + k] = (u >> 31) ? (int8_t)-1 : (int8_t)1;
      }
}

void oracle_sqa_init(const OEmb *e, int32_t L, int32_t R, uint64_t seed, int8_t *spins) {
  oracle_sqa_init_from(e, L, 0, R, seed, spins);
}

/* The attempt sequence of one sweep; returns its length n*L. */
int32_t oracle_sqa_sweep_order(const OEmb *e, int32_t L, int32_t *site_out, int32_t *slice_out) {
  int cnt = 0;
  int parities = (L == 1) ? 1 : 2;
  for (int p = 0; p < parities; ++p)
    for (int c = 0; c < 4; ++c)
      for (int tau = p; tau < L; tau += 2)
        for (int k = 0; k < e->n_sites; ++k)
          if (e->colour[k] == c) {
            site_out[cnt] = k;
            slice_out[cnt] = tau;
            ++cnt;
          }
  return cnt;
}

/* Threshold for flipping s_k^tau of one replica lattice lat[L][n] at sweep m. */
uint32_t oracle_sqa_attempt_threshold(const OEmb *e, int32_t L, const uint32_t *table,
                                      int32_t F, const int8_t *lat, int32_t k,
                                      int32_t tau, int32_t m) {
  int n = e->n_sites;
  const int8_t *cur = lat + (size_t)tau * n;
  int s = cur[k];
  int f = oracle_local_field(e, cur, k);
  int nb = 0;
  if (L > 1) nb = lat[(size_t)((tau - 1 + L) % L) * n + k] + lat[(size_t)((tau + 1) % L) * n + k];
  int a = s * f;
  int b = s * nb;
  return table[((size_t)m * (2 * F + 1) + (a + F)) * 3 + (b + 2) / 2];
}

static void run_replica(const OEmb *e, int32_t L, int32_t r, int32_t m0, int32_t m1,
                        const uint32_t *table, int32_t F, uint64_t seed, int8_t *lat) {
  int n = e->n_sites;
  int parities = (L == 1) ? 1 : 2;
  for (int m = m0; m < m1; ++m)
    for (int p = 0; p < parities; ++p)
      for (int c = 0; c < 4; ++c)
        for (int tau = p; tau < L; tau += 2)
          for (int k = 0; k < n; ++k) {
            if (e->colour[k] != c) continue;
            uint32_t R = oracle_sqa_attempt_threshold(e, L, table, F, lat, k, tau, m);
            uint32_t u = oracle_sqa_uniform(seed, (uint32_t)r, (uint32_t)k, (uint32_t)tau, (uint32_t)m);
            if (R == 0xFFFFFFFFu || u < R) lat[(size_t)tau * n + k] = (int8_t)-lat[(size_t)tau * n + k];
          }
}

typedef struct {
  const OEmb *e;
  int32_t L, r0, R, m0, m1, F, first, stride;
  const uint32_t *table;
  uint64_t seed;
  int8_t *spins;
} Job;

static void *worker(void *arg) {
  Job *j = (Job *)arg;
  size_t per = (size_t)j->L * j->e->n_sites;
  for (int r = j->first; r < j->R; r += j->stride)
    run_replica(j->e, j->L, j->r0 + r, j->m0, j->m1, j->table, j->F, j->seed, j->spins + per * r);
  return NULL;
}

/* Sweeps m0 .. m1-1 on replicas r0 .. r0+R-1 held in spins[R][L][n].
 * Replicas are independent lattices; nthreads > 1 spreads them over host
 * threads. */
void oracle_sqa_run_from(const OEmb *e, int32_t L, int32_t r0, int32_t R, int32_t m0, int32_t m1,
                         const uint32_t *table, int32_t F, uint64_t seed,
                         int8_t *spins, int32_t nthreads) {
  if (nthreads < 1) nthreads = 1;
  if (nthreads > R) nthreads = R;
  Job *jobs = (Job *)malloc(sizeof(Job) * (size_t)(nthreads > 0 ? nthreads : 1));
  pthread_t *th = (pthread_t *)malloc(sizeof(pthread_t) * (size_t)(nthreads > 0 ? nthreads : 1));
  for (int t = 0; t < nthreads; ++t) {
    Job j = {e, L, r0, R, m0, m1, F, t, nthreads, table, seed, spins};
    jobs[t] = j;
  }
  for (int t = 1; t < nthreads; ++t) pthread_create(&th[t], NULL, worker, &jobs[t]);
  if (nthreads > 0) worker(&jobs[0]);
  for (int t = 1; t < nthreads; ++t) pthread_join(th[t], NULL);
  free(jobs);
  free(th);
}

void oracle_sqa_run(const OEmb *e, int32_t L, int32_t R, int32_t m0, int32_t m1,
                    const uint32_t *table, int32_t F, uint64_t seed,
                    int8_t *spins, int32_t nthreads) {
  oracle_sqa_run_from(e, L, 0, R, m0, m1, table, F, seed, spins, nthreads);
}

/* E[r][tau] = energy of slice tau of replica r. */
void oracle_sqa_energies(const OEmb *e, int32_t L, int32_t R, const int8_t *spins, int32_t *E) {
  int n = e->n_sites;
  for (int r = 0; r < R; ++r)
    for (int tau = 0; tau < L; ++tau)
      E[(size_t)r * L + tau] = oracle_energy(e, spins + ((size_t)r * L + tau) * n);
}
