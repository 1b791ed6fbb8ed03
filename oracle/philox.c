/*
 * Counter-based random numbers for the oracle (test infrastructure only).
 *
 * Philox4xW-10 as defined by Salmon, Moraes, Dror and Shaw, "Parallel random
 * numbers: as easy as 1, 2, 3" (SC'11): ten rounds of two multiply-high/low
 * products mixed with the key, with a Weyl-sequence key bump between rounds.
 * The 64-bit-word variant is built from the same round definition so that the
 * round structure can be checked against numpy.random.Philox, which
 * implements Philox4x64-10.
 *
 * The paper does not say which generator it used (its SQA code is described
 * in another reference).  Counter layout, a reading taken here
 * (key = (seed low 32 bits, seed high 32 bits) throughout):
 *   Initial spin of (replica r, slice tau, site k), stream INIT:
 *     counter = (k, ((tau>>3)<<1) | (tau&1), 0, (INIT<<24) | r),
 *     word    = (tau>>1) & 3 (its top bit is used).
 *   Metropolis uniform of attempt (replica r, slice tau, site k, sweep m): a
 *     32-bit number u = (hi << 16) | lo.  hi and lo are 16-bit halves taken at
 *     the same place from two calls that differ only in the stream, SQA for
 *     hi and SQA_LO for lo:
 *       counter = (k, ((tau>>4)<<1) | (tau&1), m, (stream<<24) | r),
 *       j = (tau>>1) & 7, half j>>2 (0 = low, 1 = high) of word j & 3.
 *     One call thus serves the eight same-parity slices 16b+p+2j (j = 0..7)
 *     of one site.  u is uniform on 0 .. 2^32-1 because hi and lo are
 *     independent uniform halves; since lo matters only when hi equals the
 *     top half of the threshold, an implementation may draw it only then.
 *   PT initial spin (replica rho, site k), stream PT_INIT:
 *     counter = (k, rho>>2, 0, PT_INIT<<24), word = rho & 3 (its top bit).
 *   PT Metropolis uniform of attempt (replica rho, site k, sweep m): the
 *     32-bit u = (hi << 16) | lo with hi and lo the 16-bit half (rho>>2) & 1
 *     of word rho & 3 of the calls with counter (k, rho>>3, m, stream<<24),
 *     stream PT for hi and PT_LO for lo: one call per stream serves the eight
 *     replicas 8g..8g+7 of a site, and lo matters only on a tie of hi with the
 *     threshold's top half.
 */
#include "oracle.h"

static void mulhilo32(uint32_t a, uint32_t b, uint32_t *hi, uint32_t *lo) {
  uint64_t p = (uint64_t)a * (uint64_t)b;
  *hi = (uint32_t)(p >> 32);
  *lo = (uint32_t)p;
}

static void mulhilo64(uint64_t a, uint64_t b, uint64_t *hi, uint64_t *lo) {
  unsigned __int128 p = (unsigned __int128)a * (unsigned __int128)b;
  *hi = (uint64_t)(p >> 64);
  *lo = (uint64_t)p;
}

/* One definition of the rounds, instantiated at two word widths. */
#define DEFINE_PHILOX(NAME, T, MULHILO, M0, M1, W0, W1)                      \
  void NAME(const T ctr[4], const T key[2], T out[4]) {                      \
    T c0 = ctr[0], c1 = ctr[1], c2 = ctr[2], c3 = ctr[3];                    \
    T k0 = key[0], k1 = key[1];                                              \
    for (int round = 0; round < 10; ++round) {                               \
      T hi0, lo0, hi1, lo1;                                                  \
      MULHILO((T)(M0), c0, &hi0, &lo0);                                      \
      MULHILO((T)(M1), c2, &hi1, &lo1);                                      \
      T n0 = hi1 ^ c1 ^ k0;                                                  \
      T n1 = lo1;                                                            \
      T n2 = hi0 ^ c3 ^ k1;                                                  \
      T n3 = lo0;                                                            \
      c0 = n0; c1 = n1; c2 = n2; c3 = n3;                                    \
      k0 = (T)(k0 + (T)(W0));                                                \
      k1 = (T)(k1 + (T)(W1));                                                \
    }                                                                        \
    out[0] = c0; out[1] = c1; out[2] = c2; out[3] = c3;                      \
  }

DEFINE_PHILOX(oracle_philox4x32, uint32_t, mulhilo32,
              0xD2511F53u, 0xCD9E8D57u, 0x9E3779B9u, 0xBB67AE85u)
DEFINE_PHILOX(oracle_philox4x64, uint64_t, mulhilo64,
              0xD2E7470EE14C6C93ull, 0xCA5A826395121157ull,
              0x9E3779B97F4A7C15ull, 0xBB67AE8584CAA73Bull)

uint32_t oracle_sqa_word(uint64_t seed, uint32_t stream, uint32_t replica,
                         uint32_t site, uint32_t slice, uint32_t sweep) {
  uint32_t ctr[4], key[2], out[4];
  ctr[0] = site;
  ctr[1] = ((slice >> 3) << 1) | (slice & 1u);
  ctr[2] = sweep;
  ctr[3] = (stream << 24) | replica;
  key[0] = (uint32_t)seed;
  key[1] = (uint32_t)(seed >> 32);
  oracle_philox4x32(ctr, key, out);
  return out[(slice >> 1) & 3u];
}

static uint32_t sqa_half(uint64_t seed, uint32_t stream, uint32_t replica, uint32_t site,
                         uint32_t slice, uint32_t sweep) {
  uint32_t ctr[4], key[2], out[4];
  ctr[0] = site;
  ctr[1] = ((slice >> 4) << 1) | (slice & 1u);
  ctr[2] = sweep;
  ctr[3] = (stream << 24) | replica;
  key[0] = (uint32_t)seed;
  key[1] = (uint32_t)(seed >> 32);
  oracle_philox4x32(ctr, key, out);
  uint32_t j = (slice >> 1) & 7u;
  uint32_t w = out[j & 3u];
  return (j >> 2) ? (w >> 16) : (w & 0xFFFFu);
}

uint32_t oracle_sqa_uniform(uint64_t seed, uint32_t replica, uint32_t site, uint32_t slice, uint32_t sweep) {
  return (sqa_half(seed, OR_STREAM_SQA, replica, site, slice, sweep) << 16) |
         sqa_half(seed, OR_STREAM_SQA_LO, replica, site, slice, sweep);
}

static uint32_t pt_half(uint64_t seed, uint32_t stream, uint32_t replica, uint32_t site, uint32_t sweep) {
  uint32_t ctr[4], key[2], out[4];
  ctr[0] = site;
  ctr[1] = replica >> 3;
  ctr[2] = sweep;
  ctr[3] = stream << 24;
  key[0] = (uint32_t)seed;
  key[1] = (uint32_t)(seed >> 32);
  oracle_philox4x32(ctr, key, out);
  uint32_t w = out[replica & 3u];
  return ((replica >> 2) & 1u) ? (w >> 16) : (w & 0xFFFFu);
}

uint32_t oracle_pt_uniform(uint64_t seed, uint32_t replica, uint32_t site, uint32_t sweep) {
  return (pt_half(seed, OR_STREAM_PT, replica, site, sweep) << 16) |
         pt_half(seed, OR_STREAM_PT_LO, replica, site, sweep);
}

uint32_t oracle_pt_word(uint64_t seed, uint32_t stream, uint32_t replica,
                        uint32_t site, uint32_t sweep) {
  uint32_t ctr[4], key[2], out[4];
  ctr[0] = site;
  ctr[1] = replica >> 2;
  ctr[2] = sweep;
  ctr[3] = stream << 24;
  key[0] = (uint32_t)seed;
  key[1] = (uint32_t)(seed >> 32);
  oracle_philox4x32(ctr, key, out);
  return out[replica & 3u];
}
