// Structures passed from the host library to the gfx950 kernels.
//
// Device site order: sites are renumbered so that each of the four colour
// classes is contiguous (class c occupies [cls[c], cls[c+1])) and increasing
// by physical site id inside a class.  The lattice of one replica lives in
// LDS as one 64-bit word per site (a set bit = spin -1; the Metropolis kernel
// keeps even slices in the low half and odd slices in the high half, the
// Wolff kernel keeps slice tau at bit tau), followed by one all-zero word
// (index n) that unused partner slots point to.
#pragma once
#include <cstdint>

namespace sqa {

constexpr int kKindME = 0;
constexpr int kKindLHZ = 1;
constexpr int kKindMEC = 2;     // ME on Chimera

// Per-site records, kind-specific layouts (32-bit words).  Plain layout
// (Wolff and PT records, and SQA Metropolis records when F > kSmallF):
//  ME  (6 words, 24 B, 8-byte aligned): terms T=3, one partner each
//    w0 = site | base << 16
//    w1 = |w0| | |w1| << 8 | |w2| << 16 | |h| << 24
//    w2 = negmask | part0 << 16
//    w3 = part1 | part2 << 16
//    w4 = w5 = 0
//  (part = byte offset 8*d of the partner's lattice word)
//  LHZ (12 words, 48 B): terms T=4, three partners each (a 3-body term's
//  third partner is the zero word)
//    w0 = site | base << 16
//    w1 = |w0..w3| bytes
//    w2 = |h| | negmask << 8
//    w3 = 0
//    w4..w9 = part[0..11] as u16 pairs (term t partner q at index 3t+q)
//    w10, w11 = 0
//  ME on Chimera (8 words, 32 B): terms T=6, one partner each
//    w0 = site | base << 16
//    w1 = |w0..w3| bytes
//    w2 = |w4| | |w5| << 8 | |h| << 16 | negmask << 24
//    w3..w5 = part[0..5] as u16 pairs, w6 = w7 = 0
// negmask bit t (t < T): weight of term t is negative; h < 0 is bit 4 (ME,
// LHZ) or bit 6 (ME on Chimera).
// base = 3 * (F_site + F) + 2, F_site = |h| + sum |w_t|.
//
// Signed-weight layouts (SQA Metropolis records when F <= kSmallF, Wolff
// records when F <= kMidF): each term t (and h) enters its site's per-slice sum
// as W_t y_t plus a constant, y_t being the plain product bit (own spin ^
// partners; the own spin for h).  Metropolis: the sum is c + 6 A (A: weight of
// the terms whose product bit equals their sign bit, c = 3 (F - F_site)), the
// table index itself; W = -6|w| (its 6|w| in the constant c') for w >= 0 and
// +6|w| for w < 0.  Wolff: the sum is S = sum |w| X (X: the product bit
// differs from the sign bit); W = +|w| for w >= 0 and -|w| (|w| in c') for
// w < 0.  W is stored modulo 2^16; the kernels keep 4 (c' + sum W y) per byte.
//    w0 = site | (4c' | 4c' << 8) << 16
//  ME:  w1 = W0 | W1 << 16, w2 = W2 | Wh << 16, w3 = part0 | part1 << 16,
//       w4 = part2 | X << 16, w5 = 0
//  LHZ: w1 = W0 | W1 << 16, w2 = W2 | W3 << 16, w3 = Wh | X << 16, w4..w9 as
//       above
//  ME on Chimera: w1..w3 = W0..W5 as pairs, w4 = Wh | X << 16, w5..w7 =
//       part[0..5]
//  X = F_site for Wolff records, 0 for Metropolis and PT records.
// PT records (byte mode, F <= kPTByteF): W = +2|w| for w >= 0 and -2|w| (2|w|
// in c') for w < 0, c' = F - F_site + sum of those 2|w|: the kernel's byte for
// a replica, 4 (c' + sum W y) = 4F - 4F_site + 8S, addresses its threshold
// entry directly.
constexpr int kSmallF = 10;
// Largest per-site field sum of the 6-bit-field sweep path, and of the library.
constexpr int kMidF = 63;
constexpr int kLargeF = 255;
// Field modes of the sweep kernels (see sweep_class).
constexpr int kFieldSmall = 0, kFieldMid = 1, kFieldLarge = 2;
constexpr int kRecWordsME = 6;
constexpr int kRecWordsLHZ = 12;
constexpr int kRecWordsMEC = 8;
constexpr int kFieldSignMEC = 6;

constexpr int rec_words_of(int kind) {
  return kind == kKindME ? kRecWordsME : (kind == kKindMEC ? kRecWordsMEC : kRecWordsLHZ);
}

constexpr uint32_t kStreamInit = 1;
constexpr uint32_t kStreamSQA = 2;
constexpr uint32_t kStreamPT = 3;
constexpr uint32_t kStreamSwap = 4;
constexpr uint32_t kStreamTree = 5;
constexpr uint32_t kStreamPTInit = 6;
constexpr uint32_t kStreamWolff = 7;
// Low 16 bits of the 32-bit uniforms of Metropolis attempts and Wolff bonds:
// a uniform is (hi << 16) | lo with hi from the SQA (WOLFF) stream and lo from
// these, at the same counter, word and half.
// LDS table at the start of the anneal kernel's dynamic LDS, two halves of
// kSpreadEntries uint2 each: entry x maps byte x to (spread of its low nibble,
// spread of its high nibble) into 6-bit fields (bit 0 of fields at bits 0, 6,
// 12, 18); entry kSpreadEntries + x does the same into bytes at value 4 (bit 2
// of each byte), for the small-field sweep mode.
constexpr int kSpreadEntries = 256;
constexpr int kSpreadWords = 4 * kSpreadEntries;
constexpr uint32_t kStreamSQALo = 8;
constexpr uint32_t kStreamWolffLo = 9;
constexpr uint32_t kStreamPTLo = 10;

// SQA update move of a handle.
constexpr int kMoveMetropolis = 0;   // single-site Metropolis on the space-time lattice
constexpr int kMoveWolff = 1;        // time-like Wolff cluster per site (records with plain weights)
// Counter word 1 of the Philox call that draws a Wolff move's seed slice and acceptance word.
constexpr uint32_t kWolffSiteCtr = 64;
// LDS scratch of one wave for Wolff moves, per site of a chunk of a colour class (32-bit words):
// the 64-bit join mask and the 64 per-slice disagreement sums as bytes; chunks of at most
// kWolffChunk sites.
constexpr int kWolffScratchWords = 18;
constexpr int kWolffChunk = 64;

constexpr uint32_t kAlways = 0xFFFFFFFFu;

// Flags of one anneal launch for one handle.
constexpr int kFlagInit = 1;        // build the lattice from the INIT stream instead of loading it
constexpr int kFlagEnergy = 2;      // compute per-slice energies after the last sweep

struct HandleDev {
  const uint32_t *rec;      // [n][rec_words], device order
  const uint16_t *dev_of;   // [n] physical site -> device index
  const int32_t *hfield;    // [n] field of each device-order site
  const int32_t *term_w;    // [n_terms]
  const uint32_t *term_s;   // [n_terms][2]: four u16 device indices (zero word = n)
  const uint32_t *table;    // Metropolis: [M][tw]; Wolff: join thresholds [M] (tw = 1)
  const uint32_t *wacc;     // Wolff: acceptance thresholds [wrows][wwidth], index A + L F
  int8_t *spins;            // [R][L][n] physical order, +1/-1
  int32_t *energy;          // [R][L]
  int32_t kind, n, n_terms, L, M, R, F, tw;
  int32_t m0, m1, flags;
  uint32_t seed_lo, seed_hi;
  int32_t cls[5];
  int32_t move, wrows, wwidth;
};

// One unit of persistent-kernel work: handle index, first replica, count.
struct WorkItem {
  int32_t handle;
  int32_t rep0;
  int32_t nrep;
};

}  // namespace sqa
