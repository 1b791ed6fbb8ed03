// Device helpers shared by the SQA and PT kernels: Philox4x32-10, LDS
// ordering inside a wavefront, the per-kind site-record shapes and the
// carry-free bit spreading used to sum four slices side by side.
#pragma once
#include <hip/hip_runtime.h>

#include "device_types.h"

namespace sqa {

// ---------------------------------------------------------------- Philox
// Philox4x32-10 (Salmon et al., SC'11): ten rounds, each multiplying counter
// words 0 and 2 by fixed odd constants, swapping the high halves with the key
// mixed in; the key advances by a Weyl increment between rounds.
struct Words4 {
  uint32_t v[4];
};

// Philox4x32 state between rounds: counter words and the round's key.
struct PhiloxState {
  uint32_t x0, x1, x2, x3, key0, key1;
};

__device__ __forceinline__ PhiloxState philox_start(uint32_t x0, uint32_t x1, uint32_t x2, uint32_t x3,
                                                    uint32_t key0, uint32_t key1) {
  return PhiloxState{x0, x1, x2, x3, key0, key1};
}

// N rounds of Philox4x32 on st (a full draw is ten rounds).  Splitting the ten
// rounds lets a caller place independent work, such as waiting LDS reads,
// between the halves.
template <int N>
__device__ __forceinline__ void philox_rounds(PhiloxState &st) {
  constexpr uint32_t kMulA = 0xD2511F53u, kMulB = 0xCD9E8D57u;
  constexpr uint32_t kWeylA = 0x9E3779B9u, kWeylB = 0xBB67AE85u;
#pragma unroll
  for (int round = 0; round < N; ++round) {
    const uint64_t pa = static_cast<uint64_t>(kMulA) * st.x0;
    const uint64_t pb = static_cast<uint64_t>(kMulB) * st.x2;
    // three-input XORs (truth table 0x96)
    const uint32_t y0 = __builtin_amdgcn_bitop3_b32(static_cast<uint32_t>(pb >> 32), st.x1, st.key0, 0x96);
    const uint32_t y2 = __builtin_amdgcn_bitop3_b32(static_cast<uint32_t>(pa >> 32), st.x3, st.key1, 0x96);
    st.x1 = static_cast<uint32_t>(pb);
    st.x3 = static_cast<uint32_t>(pa);
    st.x0 = y0;
    st.x2 = y2;
    st.key0 += kWeylA;
    st.key1 += kWeylB;
  }
}

// Makes the state's counter words count as used at this point, so that IR
// passes cannot sink the rounds computed so far past a later scheduling
// barrier (the empty asm emits no instruction).
__device__ __forceinline__ void philox_pin(PhiloxState &st) {
  asm volatile("" : "+v"(st.x0), "+v"(st.x1), "+v"(st.x2), "+v"(st.x3));
}

__device__ __forceinline__ Words4 philox_words(const PhiloxState &st) {
  Words4 r;
  r.v[0] = st.x0; r.v[1] = st.x1; r.v[2] = st.x2; r.v[3] = st.x3;
  return r;
}

__device__ __forceinline__ Words4 philox4x32_10(uint32_t x0, uint32_t x1, uint32_t x2, uint32_t x3,
                                               uint32_t key0, uint32_t key1) {
  PhiloxState st = philox_start(x0, x1, x2, x3, key0, key1);
  philox_rounds<10>(st);
  return philox_words(st);
}

// Philox4x32 on counters (site, x1, x2, x3) whose words x1..x3 and key are
// fixed over many sites: in the first two rounds only the products with the
// site depend on it, so the rest is prepared once (philox_two_prep) and each
// site's state after two rounds costs two multiplies and three XORs
// (philox_two).
struct PhiloxTwo {
  uint32_t c1;       // x3 ^ key1: round 1's x2 = hi(A site) ^ c1
  uint32_t c2;       // lo(B x2) ^ (key0 + Weyl0): round 2's x0 = hi(B x2') ^ c2
  uint32_t d;        // hi(A x0') ^ (key1 + Weyl1), x0' = hi(B x2) ^ x1 ^ key0: round 2's x2 = d ^ lo(A site)
  uint32_t l;        // lo(A x0'): round 2's x3
  uint32_t k0, k1;   // the key after two rounds
};

__device__ __forceinline__ PhiloxTwo philox_two_prep(uint32_t x1, uint32_t x2, uint32_t x3, uint32_t key0,
                                                     uint32_t key1) {
  constexpr uint32_t kMulA = 0xD2511F53u, kMulB = 0xCD9E8D57u;
  constexpr uint32_t kWeylA = 0x9E3779B9u, kWeylB = 0xBB67AE85u;
  const uint64_t pb = static_cast<uint64_t>(kMulB) * x2;
  const uint32_t x0 = static_cast<uint32_t>(pb >> 32) ^ x1 ^ key0;
  const uint64_t pa2 = static_cast<uint64_t>(kMulA) * x0;
  PhiloxTwo w;
  w.c1 = x3 ^ key1;
  w.c2 = static_cast<uint32_t>(pb) ^ (key0 + kWeylA);
  w.d = static_cast<uint32_t>(pa2 >> 32) ^ (key1 + kWeylB);
  w.l = static_cast<uint32_t>(pa2);
  w.k0 = key0 + 2u * kWeylA;
  w.k1 = key1 + 2u * kWeylB;
  return w;
}

__device__ __forceinline__ PhiloxState philox_two(uint32_t site, const PhiloxTwo &w) {
  constexpr uint32_t kMulA = 0xD2511F53u, kMulB = 0xCD9E8D57u;
  const uint64_t pa = static_cast<uint64_t>(kMulA) * site;
  const uint32_t x2 = static_cast<uint32_t>(pa >> 32) ^ w.c1;
  const uint64_t pb = static_cast<uint64_t>(kMulB) * x2;
  return PhiloxState{static_cast<uint32_t>(pb >> 32) ^ w.c2, static_cast<uint32_t>(pb), w.d ^ static_cast<uint32_t>(pa),
                     w.l, w.k0, w.k1};
}

// Orders LDS accesses of one wavefront around a phase boundary.  A wave's LDS
// operations are executed in program order, so only the compiler needs fencing.
__device__ __forceinline__ void wave_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

__device__ __forceinline__ uint32_t bit_at(uint32_t v, int q) { return (v >> q) & 1u; }

template <int KIND>
struct Site;

// T terms per site, P partners per term, RW record words, HB negmask bit of h.
template <>
struct Site<kKindME> {
  static constexpr int T = 3, P = 1, RW = kRecWordsME, HB = 4;
};
template <>
struct Site<kKindLHZ> {
  static constexpr int T = 4, P = 3, RW = kRecWordsLHZ, HB = 4;
};
template <>
struct Site<kKindMEC> {
  static constexpr int T = 6, P = 1, RW = kRecWordsMEC, HB = kFieldSignMEC;
};

// Four record words from an 8-byte aligned address (ME records are 24 bytes
// long, so only every other one is 16-byte aligned).
__device__ __forceinline__ uint4 load_rec4(const uint32_t *r) {
  const uint2 a = *reinterpret_cast<const uint2 *>(r);
  const uint2 b = *reinterpret_cast<const uint2 *>(r + 2);
  return make_uint4(a.x, a.y, b.x, b.y);
}

// Record of an ME-on-Chimera site: site, base, term weights, |h|, signs, partners.
__device__ __forceinline__ void load_rec_mec(const uint32_t *r, uint32_t &site, uint32_t &base, uint32_t &wts,
                                             uint32_t &wts2, uint32_t &hw, uint32_t &neg, uint32_t *poff) {
  const uint4 r0 = *reinterpret_cast<const uint4 *>(r);
  const uint2 r1 = *reinterpret_cast<const uint2 *>(r + 4);
  site = r0.x & 0xFFFFu;
  base = r0.x >> 16;
  wts = r0.y;
  wts2 = r0.z & 0xFFFFu;
  hw = (r0.z >> 16) & 0xFFu;
  neg = r0.z >> 24;
  poff[0] = r0.w & 0xFFFFu; poff[1] = r0.w >> 16;
  poff[2] = r1.x & 0xFFFFu; poff[3] = r1.x >> 16;
  poff[4] = r1.y & 0xFFFFu; poff[5] = r1.y >> 16;
}

// Weight byte of term t (t < 4 from the first weight word, else the second).
__device__ __forceinline__ uint32_t term_weight(uint32_t wts, uint32_t wts2, int t) {
  return t < 4 ? ((wts >> (8 * t)) & 0xFFu) : ((wts2 >> (8 * (t - 4))) & 0xFFu);
}

// Four bits of a nibble moved to bit 0 of four 6-bit fields (bits 0, 6, 12,
// 18): every partial product of the 24-bit multiply lands on a distinct bit.
__device__ __forceinline__ uint32_t spread6(uint32_t nib) { return __umul24(nib & 0xFu, 0x8421u) & 0x41041u; }
// The same for bits 4..7 of a byte.
__device__ __forceinline__ uint32_t spread6_hi(uint32_t byte) {
  return (__umul24(byte & 0xF0u, 0x8421u) >> 4) & 0x41041u;
}

// Bits 0..2 moved to bits 0, 8, 16 (partial products at j + 7i, distinct):
// three 8-bit fields whose spread value stays below 2^24, so it can be an
// operand of a 24-bit multiply.
__device__ __forceinline__ uint32_t spread3(uint32_t bits) { return __umul24(bits & 7u, 0x4081u) & 0x10101u; }

// Four bits of a nibble moved to bit 0 of the four bytes of a word (partial
// products at bits j + 7i, all distinct: no carries).  The result has bit 24
// set for nibble bit 3, so it must not be an operand of a 24-bit multiply.
__device__ __forceinline__ uint32_t spread8(uint32_t nib) { return __umul24(nib & 0xFu, 0x204081u) & 0x01010101u; }

// Two 16-bit lanes of one register, for packed 16-bit integer arithmetic
// (v_pk_* instructions: both lanes in one operation).
typedef unsigned short u16x2 __attribute__((ext_vector_type(2)));
__device__ __forceinline__ u16x2 as_u16x2(uint32_t x) { return __builtin_bit_cast(u16x2, x); }
__device__ __forceinline__ uint32_t as_u32(u16x2 x) { return __builtin_bit_cast(uint32_t, x); }
// Entry x of the byte -> spread table; each word holds bits 0, 6, 12, 18 at
// most (the assumption lets the multiplies by it be 24-bit ones).
__device__ __forceinline__ uint2 spread_of(const uint2 *stab, uint32_t x) {
  const uint2 v = stab[x];
  __builtin_assume(v.x <= 0x41041u);
  __builtin_assume(v.y <= 0x41041u);
  return v;
}

// ------------------------------------------------- signed-weight records
// Site record in the signed-weight layout (Metropolis records with F <= 10,
// Wolff records with F <= 63): the site, record word 0 (4c' in both bytes of
// its high half), for each weight (terms, then h) the record word holding it
// and its half, the partners' byte offsets, and the high half of the word
// after the weights (F_site in Wolff records).
template <int KIND>
struct SignedRec {
  static constexpr int NW = Site<KIND>::T + 1, NP = Site<KIND>::T * Site<KIND>::P;
  uint32_t site, c4w, xtra;
  uint32_t wsg[NW];
  int wsh[NW];
  uint32_t poff[NP];
  // term t's weight (t = T: h's) in both 16-bit lanes
  __device__ __forceinline__ u16x2 weight(int t) const {
    const u16x2 w = as_u16x2(wsg[t]);
    return wsh[t] ? w.yy : w.xx;
  }
  // 4c' in all four bytes, as two 16-bit lanes
  __device__ __forceinline__ u16x2 c4() const { return as_u16x2(c4w).yy; }
};

template <int KIND>
__device__ __forceinline__ SignedRec<KIND> load_signed_rec(const uint32_t *r) {
  SignedRec<KIND> x;
  const uint4 r0 = load_rec4(r);
  x.site = r0.x & 0xFFFFu;
  x.c4w = r0.x;
  if constexpr (KIND == kKindME) {
    const uint32_t r4 = r[4];
    const uint32_t ws[4] = {r0.y, r0.y, r0.z, r0.z};
#pragma unroll
    for (int t = 0; t < 4; ++t) { x.wsg[t] = ws[t]; x.wsh[t] = t & 1; }
    x.poff[0] = r0.w & 0xFFFFu; x.poff[1] = r0.w >> 16; x.poff[2] = r4 & 0xFFFFu;
    x.xtra = r4 >> 16;
  } else if constexpr (KIND == kKindMEC) {
    const uint4 r1 = load_rec4(r + 4);
    const uint32_t ws[7] = {r0.y, r0.y, r0.z, r0.z, r0.w, r0.w, r1.x};
#pragma unroll
    for (int t = 0; t < 7; ++t) { x.wsg[t] = ws[t]; x.wsh[t] = t & 1; }
    x.xtra = r1.x >> 16;
    const uint32_t pw[3] = {r1.y, r1.z, r1.w};
#pragma unroll
    for (int q = 0; q < 3; ++q) {
      x.poff[2 * q] = pw[q] & 0xFFFFu;
      x.poff[2 * q + 1] = pw[q] >> 16;
    }
  } else {
    const uint4 r1 = load_rec4(r + 4);
    const uint2 r2 = *reinterpret_cast<const uint2 *>(r + 8);
    const uint32_t ws[5] = {r0.y, r0.y, r0.z, r0.z, r0.w};
#pragma unroll
    for (int t = 0; t < 5; ++t) { x.wsg[t] = ws[t]; x.wsh[t] = t & 1; }
    x.xtra = r0.w >> 16;
    const uint32_t pw[6] = {r1.x, r1.y, r1.z, r1.w, r2.x, r2.y};
#pragma unroll
    for (int q = 0; q < 6; ++q) {
      x.poff[2 * q] = pw[q] & 0xFFFFu;
      x.poff[2 * q + 1] = pw[q] >> 16;
    }
  }
  return x;
}

// 4 (c' + sum_t W_t y_t + W_h own) of the eight slices of one byte, slices
// 0..3 in the bytes of .x and 4..7 in .y: packed 16-bit multiply-adds of the
// spreads (bit 2 of each byte, second half of the spread table) of the plain
// product bytes.  Exact modulo 2^16 per lane; the caller's sums lie in [0, 256)
// per byte, so the lanes hold them without carries between bytes.
template <int KIND>
__device__ __forceinline__ uint2 signed_sums(const SignedRec<KIND> &x, const uint2 *st8, uint32_t own,
                                             const uint32_t *pbyte) {
  using S = Site<KIND>;
  const uint2 so = st8[own];
  u16x2 a_lo = as_u16x2(so.x) * x.weight(S::T) + x.c4();
  u16x2 a_hi = as_u16x2(so.y) * x.weight(S::T) + x.c4();
#pragma unroll
  for (int t = 0; t < S::T; ++t) {
    uint32_t prod = own;
#pragma unroll
    for (int q = 0; q < S::P; ++q) prod ^= pbyte[S::P * t + q];
    const uint2 sx = st8[prod];
    a_lo = as_u16x2(sx.x) * x.weight(t) + a_lo;
    a_hi = as_u16x2(sx.y) * x.weight(t) + a_hi;
  }
  return make_uint2(as_u32(a_lo), as_u32(a_hi));
}

}  // namespace sqa
