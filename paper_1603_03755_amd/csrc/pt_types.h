// Layout constants and the per-ladder descriptor of the parallel-tempering
// kernel (App. B, Eqs. (B1)-(B2)), shared by the kernel and its host side.
#pragma once

#include <cstdint>

#include "device_types.h"

namespace sqa {

// Waves per PT workgroup at most (the PT kernel's launch bound is 64 x this).
constexpr int kPTMaxWaves = 10;
// Largest field sum of the PT kernel's byte mode (signed-weight records, one
// byte per replica holding 4F - 4F_site + 8S <= 8F).
constexpr int kPTByteF = 31;
// LDS words of the PT kernel's per-ladder arrays after its table: E, rep_at,
// slot_of, acc (64 each), the swap words of two phases (2 x 64), and per wave
// 64 words of energy partials.
constexpr int kPTLadderWords = 4 * 64 + 2 * 64 + kPTMaxWaves * 64;
// LDS words of the PT kernel's byte tables: kSpreadEntries uint2 spreads (bit i
// of the byte -> value 4 in byte i of a nibble's word), then kSpreadEntries
// uint4 byte-permute selectors of a flip byte f: for the words of replicas
// (0, 2), (1, 3) of the low nibble and the same of the high nibble, bytes 0
// and 2 select the replica's byte of the second source where its bit of f is
// set, of the first elsewhere, and bytes 1 and 3 give zero.
constexpr int kPTSpreadWords = 6 * kSpreadEntries;

// PT ladder state for one handle.
struct PTDev {
  const uint32_t *rec;      // same record layouts as SQA
  const int32_t *hfield;
  const int32_t *term_w;
  const uint32_t *term_s;
  const uint32_t *mtab;     // [R][2F+1]  Metropolis thresholds by slot
  const uint32_t *stab;     // [R-1][Dmax+1] swap thresholds
  const uint32_t *spack;    // the same without trailing zeros: R offsets, then the rows
  const uint16_t *dev_of;
  int8_t *spins;            // [R][n] by replica, physical order
  int32_t *energy;          // [R] by replica
  int32_t *rep_at;          // [R] slot -> replica
  uint64_t *swap_acc;       // [R-1]
  int32_t kind, n, n_terms, R, F, Dmax, sweeps, sweeps_per_swap, spack_words;
  int32_t swap_falling;     // rows non-increasing in D: 1 bounds, 2 bounds by bisection only; 0 table reads
  uint32_t seed_lo, seed_hi;
  int32_t cls[5];
  int32_t nph;              // sweep phases: 4 (the colour classes) or 3 (byte mode, two classes merged)
  int32_t ph[5];            // phase c: device sites [ph[c], ph[c + 1])
};

}  // namespace sqa
