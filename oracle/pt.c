/*
 * Parallel tempering for the oracle (test infrastructure only).
 *
 * Appendix B: R replicas of the classical embedded Hamiltonian at inverse
 * temperatures beta_0 > beta_1 > ... (Eq. (B2) ladder), evolved by
 * single-spin Metropolis sweeps (Sec. III restricts PT to single-spin moves),
 * followed after every sweeps_per_swap sweeps by a swap phase that exchanges
 * the temperatures of neighbouring slots with the probability of Eq. (B1).
 *
 * Readings where the paper is silent:
 *   - a sweep visits colour c = 0..3, and within a colour every replica and
 *     every site of that colour in increasing order (replicas are
 *     independent, colour classes have no internal terms);
 *   - a swap phase tries every even pair (r, r+1), r even, then every odd
 *     pair, each once, with D = E(slot r+1) - E(slot r); swapping moves
 *     temperatures, spins stay with their replica;
 *   - the swap word for pair r in swap phase q is word 0 of the SWAP-stream
 *     Philox call with counter (r, 0, q, SWAP<<24);
 *   - energies are kept incrementally: an accepted flip of a site with
 *     a = s*f changes E by -2a.
 *   - replica rho starts in slot rho; its initial spins use the PT_INIT stream;
 *   - the Metropolis test flips iff the threshold is the always-code or
 *     u < threshold, u the attempt's 32-bit uniform (oracle_pt_uniform).
 */
#include <stdlib.h>
#include "oracle.h"

void oracle_pt_init(const OEmb *e, int32_t R, uint64_t seed, int8_t *spins) {
  int n = e->n_sites;
  for (int rho = 0; rho < R; ++rho)
    for (int k = 0; k < n; ++k) {
      uint32_t u = oracle_pt_word(seed, OR_STREAM_PT_INIT, (uint32_t)rho, (uint32_t)k, 0u);
      spins[(size_t)rho * n + k] = (u >> 31) ? (int8_t)-1 : (int8_t)1;
    }
}

/* Runs `sweeps` sweeps from the PT_INIT state.  Outputs, all indexed by replica
 * id rho except rep_at (slot -> replica): spins[R][n], E[R], rep_at[R],
 * swap_acc[R-1] (accepted swaps per slot pair). */
void oracle_pt_run(const OEmb *e, int32_t R, int32_t sweeps, int32_t sweeps_per_swap,
                   const uint32_t *mtab, int32_t F, const uint32_t *stab, int32_t Dmax,
                   uint64_t seed, int8_t *spins, int32_t *E, int32_t *rep_at,
                   uint64_t *swap_acc) {
  int n = e->n_sites;
  int width = 2 * F + 1;
  int *slot_of = (int *)malloc(sizeof(int) * (size_t)R);
  oracle_pt_init(e, R, seed, spins);
  for (int rho = 0; rho < R; ++rho) {
    rep_at[rho] = rho;
    slot_of[rho] = rho;
    E[rho] = oracle_energy(e, spins + (size_t)rho * n);
  }
  for (int r = 0; r + 1 < R; ++r) swap_acc[r] = 0;
  uint32_t phase = 0;
  for (int m = 0; m < sweeps; ++m) {
    for (int c = 0; c < 4; ++c)
      for (int rho = 0; rho < R; ++rho) {
        int8_t *s = spins + (size_t)rho * n;
        for (int k = 0; k < n; ++k) {
          if (e->colour[k] != c) continue;
          int a = s[k] * oracle_local_field(e, s, k);
          uint32_t T = mtab[(size_t)slot_of[rho] * width + (a + F)];
          uint32_t u = oracle_pt_uniform(seed, (uint32_t)rho, (uint32_t)k, (uint32_t)m);
          if (T == 0xFFFFFFFFu || u < T) {
            s[k] = (int8_t)-s[k];
            E[rho] += -2 * a;
          }
        }
      }
    if ((m + 1) % sweeps_per_swap == 0) {
      for (int q = 0; q < 2; ++q)
        for (int r = q; r + 1 < R; r += 2) {
          int D = E[rep_at[r + 1]] - E[rep_at[r]];
          int accept = 0;
          if (D <= 0) {
            accept = 1;
          } else {
            uint32_t T = stab[(size_t)r * (Dmax + 1) + D];
            uint32_t ctr[4] = {(uint32_t)r, 0u, phase, (uint32_t)OR_STREAM_SWAP << 24};
            uint32_t key[2] = {(uint32_t)seed, (uint32_t)(seed >> 32)};
            uint32_t out[4];
            oracle_philox4x32(ctr, key, out);
            accept = (T == 0xFFFFFFFFu || out[0] < T);
          }
          if (accept) {
            int x = rep_at[r];
            rep_at[r] = rep_at[r + 1];
            rep_at[r + 1] = x;
            slot_of[rep_at[r]] = r;
            slot_of[rep_at[r + 1]] = r + 1;
            swap_acc[r] += 1;
          }
        }
      ++phase;
    }
  }
  free(slot_of);
}
