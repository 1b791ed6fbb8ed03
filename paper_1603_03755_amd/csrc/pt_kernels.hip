// gfx950 parallel-tempering kernel (Appendix B, Eqs. (B1)-(B2)): one
// workgroup per temperature ladder, replicas bit-packed per site word.
#include <hip/hip_runtime.h>

#include "device_common.h"
#include "pt_types.h"

namespace sqa {

// ------------------------------------------------------ parallel tempering
// Appendix B: `R` replicas of the classical embedded Hamiltonian, replica rho
// at the inverse temperature of its slot.  One workgroup owns a whole ladder.
// LDS word of site d: bit rho = 1 <=> replica rho has spin -1 there.
//
// An item is (site of colour c, replica byte a = replicas 8a..8a+7); a thread
// keeps one byte a for the whole run (a = thread index mod RG, RG = the number
// of bytes rounded up to a power of two), so the table rows of its eight
// replicas' slots stay in registers between swap phases.  Random numbers:
// replica 8a+w takes the 16-bit half w >> 2 of word w & 3 of the PT call with
// counter (site, a, sweep, PT<<24) and is accepted when that half is below the
// top half of its threshold, rejected when above; only on a tie does the item
// draw the PT_LO call and decide on the full 32 bits.  The item owns its byte,
// so flips go back with one byte store.  Energies: per-thread deltas of the
// eight replicas (a flip with a = s*f changes E by -2a), summed over each wave
// (DPP row sums, lane permutes across rows) into the wave's own LDS partials
// before the last class barrier of a sweep that ends in a swap phase.  One
// wave, the last, decides that swap phase at the start of the next sweep's
// colour class 0, while the others compute what their first item of the class
// needs before its thresholds (partner bytes, field sums, Philox words): lane s
// holds the replica at slot s and its energy, adds every wave's partial of that
// replica, and the lanes of a pair exchange both (DPP for the even pairs, a lane
// permute for the odd ones).  The new slot of every replica goes to LDS, and
// after one barrier each thread reads its replicas' table rows and finishes.
//
// Field sums: F <= 31 (byte mode): the records are in the signed-weight layout
// and packed 16-bit multiply-adds form, per replica, a byte that addresses its
// threshold directly; F <= 63: the weighted disagreement sums s_w of the eight
// replicas in two words of four 6-bit fields; otherwise per replica.
// Sum of v over the lanes l, l - g, l - 2g, ... of a 16-lane row (G = g a power
// of two below 16): DPP row shifts, so lane l with l % 16 >= 16 - G ends with
// the row's total for its residue l % G.
template <int CTRL>
__device__ __forceinline__ uint32_t dpp_row_shr(uint32_t x) {
  return static_cast<uint32_t>(__builtin_amdgcn_update_dpp(0, static_cast<int>(x), CTRL, 0xF, 0xF, true));
}

template <int G>
__device__ __forceinline__ uint32_t row_sum_stride(uint32_t v) {
  if constexpr (G < 2) v += dpp_row_shr<0x111>(v);   // row_shr:1
  if constexpr (G < 4) v += dpp_row_shr<0x112>(v);   // row_shr:2
  if constexpr (G < 8) v += dpp_row_shr<0x114>(v);   // row_shr:4
  v += dpp_row_shr<0x118>(v);                        // row_shr:8
  return v;
}

// Row folds of four values: v_permlane16_swap(A, B) yields rows (A0, B0, A2, B2)
// and (A1, B1, A3, B3), so one add merges two values' row pairs, and
// v_permlane32_swap of two such merged values yields (X0, X1, Y0, Y1) and
// (X2, X3, Y2, Y3), whose sum holds in row k the four rows' total of value k.
__device__ __forceinline__ uint32_t fold_rows4(uint32_t v0, uint32_t v1, uint32_t v2, uint32_t v3) {
  const auto p01 = __builtin_amdgcn_permlane16_swap(v0, v1, false, false);
  const auto p23 = __builtin_amdgcn_permlane16_swap(v2, v3, false, false);
  const uint32_t s01 = static_cast<uint32_t>(p01[0]) + static_cast<uint32_t>(p01[1]);
  const uint32_t s23 = static_cast<uint32_t>(p23[0]) + static_cast<uint32_t>(p23[1]);
  const auto q = __builtin_amdgcn_permlane32_swap(s01, s23, false, false);
  return static_cast<uint32_t>(q[0]) + static_cast<uint32_t>(q[1]);
}

// Sums the eight per-thread values of replica byte a over the wave (modulo
// 2^32) and stores the wave's totals in its own array: word 8a + w holds
// replica 8a + w's.  DPP row sums, then two four-value row folds.
template <int G>
__device__ __forceinline__ void flush_partials(uint32_t *dE, uint32_t *part, int a, int lane) {
#pragma unroll
  for (int w = 0; w < 8; ++w) dE[w] = row_sum_stride<G>(dE[w]);
  const uint32_t t0 = fold_rows4(dE[0], dE[1], dE[2], dE[3]), t1 = fold_rows4(dE[4], dE[5], dE[6], dE[7]);
  if ((lane & 15) >= 16 - G) {               // row k = lane / 16 holds values k and 4 + k
    const int k = lane >> 4;
    part[8 * a + k] = t0;
    part[8 * a + 4 + k] = t1;
  }
#pragma unroll
  for (int w = 0; w < 8; ++w) dE[w] = 0;
}

// Byte mode, while each 16-bit half of the packed sums vpk stays below 2^16
// over the wave: the four packed words are summed instead of eight values
// (halves of vpk[k]: replicas (k & 1) + 4 (k >> 1) and that + 2).
template <int G>
__device__ __forceinline__ void flush_packed(uint32_t *vpk, uint32_t *part, int a, int lane) {
#pragma unroll
  for (int k = 0; k < 4; ++k) vpk[k] = row_sum_stride<G>(vpk[k]);
  const uint32_t t = fold_rows4(vpk[0], vpk[1], vpk[2], vpk[3]);
  if ((lane & 15) >= 16 - G) {               // row k holds packed word k
    const int k = lane >> 4;
    const int w = (k & 1) + 4 * (k >> 1);
    part[8 * a + w] = t & 0xFFFFu;
    part[8 * a + w + 2] = t >> 16;
  }
#pragma unroll
  for (int k = 0; k < 4; ++k) vpk[k] = 0;
}

// Explicit LDS and global address spaces: pointers that are updated inside the
// sweep loop (the byte-mode threshold bases) or passed out of line would
// otherwise become generic, and their loads flat loads.
using lds_u8 = __attribute__((address_space(3))) const uint8_t;
using lds_u16 = __attribute__((address_space(3))) const uint16_t;
using lds_u32 = __attribute__((address_space(3))) uint32_t;
using lds_i32 = __attribute__((address_space(3))) int32_t;
using glb_u32 = __attribute__((address_space(1))) const uint32_t;

// Field modes of the PT kernel: byte mode (F <= kPTByteF, signed-weight
// records), four 6-bit fields per word (F <= kMidF), or per replica.
constexpr int kPTBytes = 0, kPTSwar = 1, kPTWide = 2;

// Raw record words of one site (ME: the first 4 of its 6 words, 5 in byte mode;
// LHZ: 10; ME on Chimera: 6, 8 in byte mode).
// The ladder's Philox key, held in scalar registers for the whole run (a
// scalar reload per item would make each item's LDS reads wait with it).
struct PTKey {
  uint32_t lo, hi;
};

template <int KIND> struct PTRec;
template <> struct PTRec<kKindME> { uint4 a; uint32_t b; };
template <> struct PTRec<kKindLHZ> { uint4 a, b; uint2 c; };
template <> struct PTRec<kKindMEC> { uint4 a, b; };

template <int KIND, int MODE>
__device__ __forceinline__ PTRec<KIND> load_pt_rec(const uint32_t *r) {
  PTRec<KIND> x;
  if constexpr (KIND == kKindME) {
    x.a = load_rec4(r);     // 24-byte records: 8-byte aligned
    x.b = (MODE == kPTBytes) ? r[4] : 0u;
  } else if constexpr (KIND == kKindMEC) {
    x.a = *reinterpret_cast<const uint4 *>(r);
    if constexpr (MODE == kPTBytes) {
      x.b = *reinterpret_cast<const uint4 *>(r + 4);
    } else {
      const uint2 b = *reinterpret_cast<const uint2 *>(r + 4);
      x.b = make_uint4(b.x, b.y, 0u, 0u);
    }
  } else {
    x.a = *reinterpret_cast<const uint4 *>(r);
    x.b = *reinterpret_cast<const uint4 *>(r + 4);
    x.c = *reinterpret_cast<const uint2 *>(r + 8);
  }
  return x;
}

// The signed-weight record (byte mode) held in a PTRec.
template <int KIND>
__device__ __forceinline__ SignedRec<KIND> signed_from_pt(const PTRec<KIND> &x) {
  SignedRec<KIND> s;
  s.site = x.a.x & 0xFFFFu;
  s.c4w = x.a.x;
  s.xtra = 0;
  if constexpr (KIND == kKindME) {
    const uint32_t ws[4] = {x.a.y, x.a.y, x.a.z, x.a.z};
#pragma unroll
    for (int t = 0; t < 4; ++t) { s.wsg[t] = ws[t]; s.wsh[t] = t & 1; }
    s.poff[0] = x.a.w & 0xFFFFu; s.poff[1] = x.a.w >> 16; s.poff[2] = x.b;   // the host leaves x.b's top half 0
  } else if constexpr (KIND == kKindMEC) {
    const uint32_t ws[7] = {x.a.y, x.a.y, x.a.z, x.a.z, x.a.w, x.a.w, x.b.x};
#pragma unroll
    for (int t = 0; t < 7; ++t) { s.wsg[t] = ws[t]; s.wsh[t] = t & 1; }
    const uint32_t pw[3] = {x.b.y, x.b.z, x.b.w};
#pragma unroll
    for (int q = 0; q < 3; ++q) {
      s.poff[2 * q] = pw[q] & 0xFFFFu;
      s.poff[2 * q + 1] = pw[q] >> 16;
    }
  } else {
    const uint32_t ws[5] = {x.a.y, x.a.y, x.a.z, x.a.z, x.a.w};
#pragma unroll
    for (int t = 0; t < 5; ++t) { s.wsg[t] = ws[t]; s.wsh[t] = t & 1; }
    const uint32_t pw[6] = {x.b.x, x.b.y, x.b.z, x.b.w, x.c.x, x.c.y};
#pragma unroll
    for (int q = 0; q < 6; ++q) {
      s.poff[2 * q] = pw[q] & 0xFFFFu;
      s.poff[2 * q + 1] = pw[q] >> 16;
    }
  }
  return s;
}

// Threshold top halves of the byte's eight replicas, addressed by their V bytes.
__device__ __forceinline__ void pt_thresholds(const lds_u8 *const *thb, uint2 V, uint32_t *th) {
#pragma unroll
  for (int w = 0; w < 8; ++w)
    th[w] = *reinterpret_cast<const lds_u16 *>(thb[w] - (((w < 4 ? V.x : V.y) >> (8 * (w & 3))) & 0xFFu));
}

// The decisions of a byte-mode item from its Philox words u and threshold top
// halves th: D = hi - top half is negative iff accepted on hi alone, zero on a
// tie (the sign bits are shifted into `flip` from replica 7 down); a tie decides
// all eight on 32 bits with the PT_LO call.  Then the byte store and the flip sums.
__device__ __forceinline__ void pt_item_bytes_decide(PTKey K, uint32_t site, int d, uint8_t *latb,
                                                     const uint2 *st8, int a, uint32_t vmask,
                                                     const lds_u8 *const *thb, uint32_t f4, uint32_t *vpk,
                                                     uint32_t m, uint32_t own, uint2 V,
                                                     const Words4 &u, const uint32_t *th) {
  uint32_t flip = 0, dmin = 0xFFFFFFFFu;
#pragma unroll
  for (int w = 7; w >= 0; --w) {
    const uint32_t hi = (w < 4) ? (u.v[w] & 0xFFFFu) : (u.v[w - 4] >> 16);
    const uint32_t D = hi - th[w];
    flip = __builtin_amdgcn_alignbit(flip, D, 31);
    dmin = min(dmin, D);
  }
  if (dmin == 0) {     // some half equals its threshold's top half: decide all eight on 32 bits
    const Words4 v = philox4x32_10(site, static_cast<uint32_t>(a), m, kStreamPTLo << 24, K.lo, K.hi);
    flip = 0;
#pragma unroll
    for (int w = 0; w < 8; ++w) {
      const uint32_t vb = ((w < 4 ? V.x : V.y) >> (8 * (w & 3))) & 0xFFu;
      const uint32_t R = *reinterpret_cast<const lds_u32 *>(thb[w] - 2 - vb);
      const uint32_t uu = (w < 4) ? ((u.v[w] << 16) | (v.v[w] & 0xFFFFu))
                                  : ((u.v[w - 4] & 0xFFFF0000u) | (v.v[w - 4] >> 16));
      if (min(uu, 0xFFFFFFFEu) < R) flip |= 1u << w;
    }
  }
  flip &= vmask;
  latb[8 * d + a] = static_cast<uint8_t>(own ^ flip);
  const uint4 fsel = reinterpret_cast<const uint4 *>(st8 + kSpreadEntries)[flip];
  vpk[0] += __builtin_amdgcn_perm(f4, V.x, fsel.x);
  vpk[1] += __builtin_amdgcn_perm(f4, V.x, fsel.y);
  vpk[2] += __builtin_amdgcn_perm(f4, V.y, fsel.z);
  vpk[3] += __builtin_amdgcn_perm(f4, V.y, fsel.w);
}

// One item: site d (record x), replica byte a, sweep m.
// Byte mode: the signed-weight sums give, per replica w, the byte
// V_w = 4F - 4F_site + 8 S_w in [0, 8F]; its threshold's top half is the u16 at
// thb[w] - V_w (thb[w] = the table's byte address + 4 row[w] + 8F + 2, so this is
// entry row[w] + F_site + F - 2 S_w), and a flip changes the energy by
// 4 S_w - 2 F_site = (V_w - 4F) / 2.  One byte permute per word takes V_w for
// the flipped replicas and 4F for the others (selectors from a table); the
// thread adds those bytes into 16-bit halves (vpk: replicas 0 and 2, 1 and 3,
// 4 and 6, 5 and 7).  Every site is an item of every replica byte once per
// sweep, so over k sweeps the sum for replica w less 4F n k (n sites) is the
// sum of V_w - 4F over its flips: twice its energy change.
// The item stream's counter is (site, replica byte a, sweep m, PT << 24): its
// first two rounds prepared once per thread and sweep (philox_two_prep).
using PTSweepWords = PhiloxTwo;

__device__ __forceinline__ PTSweepWords pt_sweep_words(PTKey K, int a, uint32_t m) {
  return philox_two_prep(static_cast<uint32_t>(a), m, kStreamPT << 24, K.lo, K.hi);
}

// The temperature-free front of a byte-mode item: own and partner bytes, the
// spread-table rows of the own byte and of each term's product byte, and V.
// The first six Philox rounds run in two parts while those two rounds of LDS
// reads are in flight; the last four are left to the caller.
template <int KIND>
__device__ __forceinline__ uint2 pt_item_front(const PTSweepWords &sw, const SignedRec<KIND> &sr, int d,
                                               const uint8_t *latb, const uint2 *st8, int a, uint32_t &own,
                                               PhiloxState &ps) {
  using S = Site<KIND>;
  own = latb[8 * d + a];
  uint32_t pbyte[S::T * S::P];
#pragma unroll
  for (int i = 0; i < S::T * S::P; ++i) pbyte[i] = latb[sr.poff[i] + a];
  __builtin_amdgcn_sched_barrier(0);
  ps = philox_two(sr.site, sw);
  philox_rounds<1>(ps);
  philox_pin(ps);
  asm volatile("" : "+v"(own));                   // nothing derived from own ahead of the rounds
  __builtin_amdgcn_sched_barrier(0);
  own &= 0xFFu;                                   // (a byte again for the compiler: no masks on the products)
  uint2 sx[S::T + 1];                             // spread rows: terms 0..T-1, then h's (the own byte)
#pragma unroll
  for (int t = 0; t < S::T; ++t) {
    uint32_t prod = own;
#pragma unroll
    for (int q = 0; q < S::P; ++q) prod ^= pbyte[S::P * t + q];
    sx[t] = st8[prod];
  }
  sx[S::T] = st8[own];
  __builtin_amdgcn_sched_barrier(0);
  philox_rounds<3>(ps);
  philox_pin(ps);
  __builtin_amdgcn_sched_barrier(0);
  u16x2 a_lo = as_u16x2(sx[S::T].x) * sr.weight(S::T) + sr.c4();
  u16x2 a_hi = as_u16x2(sx[S::T].y) * sr.weight(S::T) + sr.c4();
#pragma unroll
  for (int t = 0; t < S::T; ++t) {
    a_lo = as_u16x2(sx[t].x) * sr.weight(t) + a_lo;
    a_hi = as_u16x2(sx[t].y) * sr.weight(t) + a_hi;
  }
  return make_uint2(as_u32(a_lo), as_u32(a_hi));
}

template <int KIND>
__device__ __forceinline__ void pt_item_bytes(PTKey K, const PTSweepWords &sw, const PTRec<KIND> &x, int d,
                                              uint8_t *latb, const uint2 *st8, int a, uint32_t vmask,
                                              const lds_u8 *const *thb, uint32_t f4, uint32_t *vpk, uint32_t m) {
  const SignedRec<KIND> sr = signed_from_pt<KIND>(x);
  uint32_t own;
  PhiloxState ps;
  const uint2 V = pt_item_front<KIND>(sw, sr, d, latb, st8, a, own, ps);
  uint32_t th[8];
  pt_thresholds(thb, V, th);
  __builtin_amdgcn_sched_barrier(0);
  philox_rounds<4>(ps);
  __builtin_amdgcn_sched_barrier(0);
  const Words4 u = philox_words(ps);
  pt_item_bytes_decide(K, sr.site, d, latb, st8, a, vmask, thb, f4, vpk, m, own, V, u, th);
}

// The part of a byte-mode item that does not depend on the replicas'
// temperatures (own and partner bytes, the sums V, the Philox words), for the
// first item of a colour class that begins while a swap phase is decided.
struct PTItemHead {
  uint32_t own, site;
  uint2 V;
  Words4 u;
};

template <int KIND>
__device__ __forceinline__ PTItemHead pt_item_bytes_head(const PTSweepWords &sw, const PTRec<KIND> &x, int d,
                                                         const uint8_t *latb, const uint2 *st8, int a) {
  const SignedRec<KIND> sr = signed_from_pt<KIND>(x);
  PTItemHead hd;
  hd.site = sr.site;
  PhiloxState ps;
  hd.V = pt_item_front<KIND>(sw, sr, d, latb, st8, a, hd.own, ps);
  philox_rounds<4>(ps);
  hd.u = philox_words(ps);
  return hd;
}

// One item of the 6-bit-field or per-replica modes: site d (record x), replica
// byte a, sweep m; row: the table row offsets of the byte's eight replicas; dE:
// their energy deltas.
template <int KIND, bool SWAR>
__device__ __forceinline__ void pt_item(const PTDev &P, PTKey K, const PTRec<KIND> &x, int d, uint8_t *latb,
                                        const uint32_t *mtab, int a, uint32_t vmask, const int32_t *row,
                                        uint32_t *dE, uint32_t m) {
  using S = Site<KIND>;
  const int F = P.F;
  const uint16_t *mtab16 = reinterpret_cast<const uint16_t *>(mtab);
  uint32_t site, wts, wts2 = 0, ah, neg;
  uint32_t part[S::T * S::P];
  if constexpr (KIND == kKindME) {
    site = x.a.x & 0xFFFFu;
    wts = x.a.y & 0xFFFFFFu;
    ah = x.a.y >> 24;
    neg = x.a.z & 0xFFu;
    part[0] = x.a.z >> 16; part[1] = x.a.w & 0xFFFFu; part[2] = x.a.w >> 16;
  } else if constexpr (KIND == kKindMEC) {
    site = x.a.x & 0xFFFFu;
    wts = x.a.y;
    wts2 = x.a.z & 0xFFFFu;
    ah = (x.a.z >> 16) & 0xFFu;
    neg = x.a.z >> 24;
    part[0] = x.a.w & 0xFFFFu; part[1] = x.a.w >> 16;
    part[2] = x.b.x & 0xFFFFu; part[3] = x.b.x >> 16;
    part[4] = x.b.y & 0xFFFFu; part[5] = x.b.y >> 16;
  } else {
    site = x.a.x & 0xFFFFu;
    wts = x.a.y;
    ah = x.a.z & 0xFFu;
    neg = (x.a.z >> 8) & 0xFFu;
    const uint32_t pw[6] = {x.b.x, x.b.y, x.b.z, x.b.w, x.c.x, x.c.y};
#pragma unroll
    for (int q = 0; q < 6; ++q) {
      part[2 * q] = pw[q] & 0xFFFFu;
      part[2 * q + 1] = pw[q] >> 16;
    }
  }
  // own and partner bytes (LDS reads), the first Philox rounds while they are in flight
  const uint32_t own = latb[8 * d + a];
  uint32_t pbyte[S::T * S::P];
#pragma unroll
  for (int i = 0; i < S::T * S::P; ++i) pbyte[i] = latb[part[i] + a];
  PhiloxState ps = philox_start(site, static_cast<uint32_t>(a), m, kStreamPT << 24, K.lo, K.hi);
  __builtin_amdgcn_sched_barrier(0);
  philox_rounds<5>(ps);
  philox_pin(ps);
  __builtin_amdgcn_sched_barrier(0);

  // F_site = |h| + sum of the term weights
  uint32_t fs = __builtin_amdgcn_sad_u8(wts, 0u, ah);
  if constexpr (KIND == kKindMEC) fs = __builtin_amdgcn_sad_u8(wts2, 0u, fs);
  const uint32_t ox = (own ^ (0u - ((neg >> S::HB) & 1u))) & 0xFFu;
  uint32_t sw[8];                                  // weighted disagreement sum of replica 8a+w
  if constexpr (SWAR) {
    // four 6-bit fields per word; the spreads are computed (no table round trip:
    // this kernel is bound by latency, not by issue)
    uint32_t acc_lo = __umul24(spread6(ox & 0xFu), ah), acc_hi = __umul24(spread6(ox >> 4), ah);
#pragma unroll
    for (int t = 0; t < S::T; ++t) {
      uint32_t prod = own;
#pragma unroll
      for (int q = 0; q < S::P; ++q) prod ^= pbyte[S::P * t + q];
      const uint32_t xt = (prod ^ (0u - ((neg >> t) & 1u))) & 0xFFu;
      const uint32_t wt = term_weight(wts, wts2, t);
      acc_lo += __umul24(spread6(xt & 0xFu), wt);
      acc_hi += __umul24(spread6(xt >> 4), wt);
    }
#pragma unroll
    for (int w = 0; w < 4; ++w) {
      sw[w] = __builtin_amdgcn_ubfe(acc_lo, 6 * w, 6);
      sw[w + 4] = __builtin_amdgcn_ubfe(acc_hi, 6 * w, 6);
    }
  } else {
    uint32_t X[S::T];
#pragma unroll
    for (int t = 0; t < S::T; ++t) {
      uint32_t prod = own;
#pragma unroll
      for (int q = 0; q < S::P; ++q) prod ^= pbyte[S::P * t + q];
      X[t] = prod ^ (0u - ((neg >> t) & 1u));
    }
#pragma unroll
    for (int w = 0; w < 8; ++w) {
      uint32_t v = ah * bit_at(ox, w);
#pragma unroll
      for (int t = 0; t < S::T; ++t) v += term_weight(wts, wts2, t) * bit_at(X[t], w);
      sw[w] = v;
    }
  }
  // thresholds: T = mtab[slot row + (F_site - 2 s) + F]; top halves first
  int32_t ix[8];
  uint32_t th[8];
#pragma unroll
  for (int w = 0; w < 8; ++w) {
    ix[w] = row[w] + static_cast<int32_t>(fs) + F - 2 * static_cast<int32_t>(sw[w]);
    th[w] = mtab16[2 * ix[w] + 1];
  }
  __builtin_amdgcn_sched_barrier(0);
  philox_rounds<5>(ps);
  __builtin_amdgcn_sched_barrier(0);
  const Words4 u = philox_words(ps);
  uint32_t flip = 0;
  bool tie = false;
#pragma unroll
  for (int w = 0; w < 8; ++w) {
    const uint32_t hi = (w < 4) ? (u.v[w] & 0xFFFFu) : (u.v[w - 4] >> 16);
    if (hi < th[w]) flip |= 1u << w;
    tie |= (hi == th[w]);
  }
  if (tie) {     // some half equals its threshold's top half: decide all eight on 32 bits
    const Words4 v = philox4x32_10(site, static_cast<uint32_t>(a), m, kStreamPTLo << 24, K.lo, K.hi);
    flip = 0;
#pragma unroll
    for (int w = 0; w < 8; ++w) {
      const uint32_t uu = (w < 4) ? ((u.v[w] << 16) | (v.v[w] & 0xFFFFu))
                                  : ((u.v[w - 4] & 0xFFFF0000u) | (v.v[w - 4] >> 16));
      if (min(uu, 0xFFFFFFFEu) < mtab[ix[w]]) flip |= 1u << w;
    }
  }
  flip &= vmask;
  latb[8 * d + a] = static_cast<uint8_t>(own ^ flip);
#pragma unroll
  for (int w = 0; w < 8; ++w)
    if ((flip >> w) & 1u) dE[w] += static_cast<uint32_t>(4 * static_cast<int32_t>(sw[w]) - 2 * static_cast<int32_t>(fs));
}

struct SwapSlot {
  int rep;        // replica at this lane's slot
  int e;          // its energy
  uint32_t acc;   // accepted swaps of pair (lane, lane + 1)
};

// The staged row of pair r of the two swap phases of a lane (o0[q]: its first
// entry in the packed table, len[q]: its length; entries past the end are 0).
struct SwapRows {
  uint32_t o0[2], len[2];
};

__device__ __forceinline__ SwapRows swap_rows(const lds_u32 *spk, bool staged, int R) {
  const int lane = static_cast<int>(threadIdx.x & 63u);
  SwapRows sr{};
#pragma unroll
  for (int q = 0; q < 2; ++q) {
    const int r = lane - ((lane - q) & 1);
    const int rc = (r >= 0 && r + 1 < R) ? r : 0;
    if (staged) {
      sr.o0[q] = spk[rc];
      sr.len[q] = spk[rc + 1] - sr.o0[q];
    }
  }
  return sr;
}

// ln(t 2^-32) for 0 < t < 2^32, as log1p(-(2^32 - t) 2^-32): full float
// precision also where t is close to 2^32.
__device__ __forceinline__ float log1m_frac32(uint32_t t) {
  return log1pf(-static_cast<float>(0xFFFFFFFFu - t + 1u) * 0x1p-32f);
}

// Pair r's acceptance bound for its swap word u: with the staged row T of pair
// r non-increasing in D (thresholds of exp(D (beta_{r+1} - beta_r)), a gap D >
// Dmax clamping to Dmax), the test min(u, 2^32 - 2) < T(min(D, Dmax)) holds
// exactly for D <= D*, and D* = 2^32 - 1 when it holds at Dmax.  A float
// estimate from ln(u 2^-32) / ln(T(1) 2^-32) (T(1) ~ 2^32 exp(beta_{r+1} - beta_r)) is
// checked against the table at D* and D* + 1; a bisection over the table
// settles any estimate that misses.  `inv` is 1 / ln(T(1) 2^-32).
__device__ __forceinline__ uint32_t swap_bound(uint32_t u, uint32_t o0, uint32_t len, int Dmax, float inv,
                                               const lds_u32 *spk) {
  const uint32_t uq = min(u, 0xFFFFFFFEu);
  auto T = [&](int i) { return static_cast<uint32_t>(i) < len ? spk[o0 + i] : 0u; };
  const float x = log1m_frac32(uq) * inv;   // gaps below x pass
  const int d0 = static_cast<int>(fminf(fmaxf(ceilf(x) - 1.0f, 0.0f), static_cast<float>(max(Dmax - 1, 0))));
  const uint32_t t_max = T(Dmax), t0 = T(d0), t1 = T(d0 + 1);
  if (uq < t_max) return 0xFFFFFFFFu;
  if (uq < t0 && !(uq < t1)) return static_cast<uint32_t>(d0);
  int lo = 0, hi = Dmax;                          // T(0) passes, T(Dmax) does not
  while (hi - lo > 1) {
    const int mid = (lo + hi) >> 1;
    if (uq < T(mid)) lo = mid;
    else hi = mid;
  }
  return static_cast<uint32_t>(lo);
}

// The partner lane's energy and replica in swap phase q (0: even pairs, quad
// perm [1,0,3,2]; 1: odd pairs, a low lane takes lane + 1 (wave_shl:1) and a
// high lane lane - 1 (wave_shr:1), across row boundaries; lanes 0 and 63 have
// no pair).
__device__ __forceinline__ void swap_partner(int q, bool low, int e, int rep_s, int &pe, int &prep) {
  if (q == 0) {
    pe = __builtin_amdgcn_mov_dpp(e, 0xB1, 0xF, 0xF, true);
    prep = __builtin_amdgcn_mov_dpp(rep_s, 0xB1, 0xF, 0xF, true);
  } else {
    const int up_e = __builtin_amdgcn_update_dpp(0, e, 0x130, 0xF, 0xF, false);
    const int up_r = __builtin_amdgcn_update_dpp(0, rep_s, 0x130, 0xF, 0xF, false);
    const int dn_e = __builtin_amdgcn_update_dpp(0, e, 0x138, 0xF, 0xF, false);
    const int dn_r = __builtin_amdgcn_update_dpp(0, rep_s, 0x138, 0xF, 0xF, false);
    pe = low ? up_e : dn_e;
    prep = low ? up_r : dn_r;
  }
}

// One swap phase (Eq. (B1)) as one wave sees it: lane s holds the replica at
// slot s and its energy as of the last phase; it adds every wave's partial of
// that replica (their sum less `off`, shifted right by `sh`, is the energy
// change), then the even pairs (r, r + 1), then the odd ones, are decided by
// both of their lanes from the same inputs, here by comparing the gap with
// pair r's bound (lane r's `bound`, see swap_bound).  Lane r counts the
// accepted swaps of pair r in `acc`.  Kept out of line so that its registers
// do not weigh on the sweep's.
__device__ __noinline__ SwapSlot swap_phase_bounded(int rep_s, int e, uint32_t acc, uint32_t off, int sh, int R,
                                                    uint32_t bound, const lds_u32 *parts) {
  const int lane = static_cast<int>(threadIdx.x & 63u);
  uint32_t de = 0;
#pragma unroll
  for (int v = 0; v < kPTMaxWaves; ++v) de += parts[64 * v + (rep_s & 63)];
  e += static_cast<int32_t>(de - off) >> sh;
  // the bounds of this lane's pairs: (lane & ~1) in the even phase, from that
  // lane (quad_perm [0,0,2,2]); in the odd phase its own (odd lanes) or lane - 1's
  const uint32_t b_even = static_cast<uint32_t>(__builtin_amdgcn_mov_dpp(static_cast<int>(bound), 0xA0, 0xF, 0xF, true));
  const uint32_t b_dn = static_cast<uint32_t>(__builtin_amdgcn_update_dpp(0, static_cast<int>(bound), 0x138, 0xF, 0xF, false));
#pragma unroll
  for (int q = 0; q < 2; ++q) {
    const bool low = ((lane - q) & 1) == 0;       // this lane is slot r of its pair (r, r + 1)
    const int r = lane - ((lane - q) & 1);
    int pe, prep;
    swap_partner(q, low, e, rep_s, pe, prep);
    const int D = low ? pe - e : e - pe;          // E(slot r + 1) - E(slot r)
    const uint32_t b = (q == 0) ? b_even : (low ? bound : b_dn);
    if (r >= 0 && r + 1 < R && (D <= 0 || static_cast<uint32_t>(D) <= b)) {
      e = pe;
      rep_s = prep;
      if (low) ++acc;
    }
  }
  return SwapSlot{rep_s, e, acc};
}

// The same with each gap's threshold read from the swap table (staged in LDS,
// else in device memory) and compared with the pair's swap word.
__device__ __noinline__ SwapSlot swap_phase(int rep_s, int e, uint32_t acc, uint32_t off, int sh, int R, int Dmax,
                                            bool staged, SwapRows rows, const lds_u32 *spk, glb_u32 *stab,
                                            const lds_u32 *sw, const lds_u32 *parts) {
  const int lane = static_cast<int>(threadIdx.x & 63u);
  uint32_t word[2];                               // both phases' swap words, read ahead of the energies
#pragma unroll
  for (int q = 0; q < 2; ++q) {
    const int r = lane - ((lane - q) & 1);
    word[q] = sw[(r >= 0 && r + 1 < R) ? r : 0];
  }
  uint32_t de = 0;
#pragma unroll
  for (int v = 0; v < kPTMaxWaves; ++v) de += parts[64 * v + (rep_s & 63)];
  e += static_cast<int32_t>(de - off) >> sh;
#pragma unroll
  for (int q = 0; q < 2; ++q) {
    const bool low = ((lane - q) & 1) == 0;
    const int r = lane - ((lane - q) & 1);
    const bool valid = r >= 0 && r + 1 < R;
    const uint32_t o0 = rows.o0[q], len = rows.len[q];
    int pe, prep;
    swap_partner(q, low, e, rep_s, pe, prep);
    if (valid) {
      const int D = low ? pe - e : e - pe;
      bool ok = D <= 0;
      if (!ok) {
        const int Dc = min(D, Dmax);
        const uint32_t T = staged ? ((static_cast<uint32_t>(Dc) < len) ? spk[o0 + Dc] : 0u)
                               : stab[static_cast<size_t>(r) * (Dmax + 1) + Dc];
        ok = min(word[q], 0xFFFFFFFEu) < T;
      }
      if (ok) {
        e = pe;
        rep_s = prep;
        if (low) ++acc;
      }
    }
  }
  return SwapSlot{rep_s, e, acc};
}

// NPH: phases per sweep, each a run of consecutive colour classes with no term
// between them (updated together, they give what one class after the other
// gives); 4 (the classes) or 3 (one pair merged).
template <int KIND, int MODE, int NPH>
__device__ __forceinline__ void pt_ladder(const PTDev &P, const uint32_t *rec, uint64_t *lat, const uint32_t *mtab,
                                          const uint2 *st8, int32_t *E, int32_t *rep_at, int32_t *slot_of,
                                          uint32_t *acc, uint32_t *swapw, const uint32_t *spk) {
  constexpr bool SWAR = MODE == kPTSwar;
  using S = Site<KIND>;
  const int R = P.R, F = P.F;
  const int width = 2 * F + 1;
  const int tid = threadIdx.x, nth = blockDim.x;
  const int lane = tid & 63, wave = tid >> 6;
  PTKey K{P.seed_lo, P.seed_hi};
  asm volatile("" : "+s"(K.lo), "+s"(K.hi));      // not re-read from P inside the sweep loop
  int RG = 1, lgRG = 0;
  while (RG * 8 < R) {
    RG <<= 1;
    ++lgRG;
  }
  const int a = tid & (RG - 1);                    // this thread's replica byte never changes
  const bool group_live = 8 * a < R;
  const int nvalid = group_live ? min(8, R - 8 * a) : 0;
  const uint32_t vmask = (1u << nvalid) - 1u;
  uint8_t *latb = reinterpret_cast<uint8_t *>(lat);
  uint32_t dE[8];                                   // energy deltas (modulo 2^32; byte mode: see pt_item_bytes)
  uint32_t vsum[8], vpk[4];                         // byte mode: byte sums (see pt_item_bytes)
  int pend = 0;                                     // byte mode: most items per thread since vpk was emptied
  bool widened = false;                             // byte mode: vsum holds sums since the last flush
  int pmax = 0;                                     // most items of a thread in one colour class (<= 256)
  const uint32_t f4 = static_cast<uint32_t>(4 * F) * 0x01010101u;
  int32_t row[8];                                  // table row offsets of the byte's replicas
  const lds_u8 *thb[8];                            // byte mode: their threshold base addresses
  const lds_u8 *mtabb = (const lds_u8 *)(reinterpret_cast<const uint8_t *>(mtab)) + 8 * F + 2;
#pragma unroll
  for (int w = 0; w < 4; ++w) vpk[w] = 0;
#pragma unroll
  for (int w = 0; w < 8; ++w) {
    dE[w] = 0;
    vsum[w] = 0;
    row[w] = (w < nvalid) ? slot_of[8 * a + w] * width : 0;
    thb[w] = mtabb + 4 * row[w];
  }
  // The record of a thread's first item in the next phase is read into
  // registers before the current phase is processed, so its LDS latency overlaps
  // the current item and the phase barrier (records are read-only).
  int ph[NPH + 1];                                  // phase c: device sites [ph[c], ph[c + 1])
#pragma unroll
  for (int c = 0; c <= NPH; ++c) ph[c] = P.ph[c];
  bool has_first[NPH];
#pragma unroll
  for (int c = 0; c < NPH; ++c) {
    has_first[c] = group_live && tid < ((ph[c + 1] - ph[c]) << lgRG);
    pmax = max(pmax, (((ph[c + 1] - ph[c]) << lgRG) + nth - 1) / nth);
  }
  constexpr int NB = (NPH % 2 == 0) ? 2 : NPH;      // record buffers: phase c's in rb[c % NB]
  PTRec<KIND> rb[NB];
  if (has_first[0]) rb[0] = load_pt_rec<KIND, MODE>(rec + (ph[0] + (tid >> lgRG)) * S::RW);
  // energy deltas into E (RG is a power of two up to 8, so it divides the 16-lane rows)
  uint32_t *parts = swapw + 2 * 64;   // 64 words per wave
  uint32_t *part = parts + 64 * wave;
  // byte mode: the 16-bit halves into the per-replica sums (a half gains at most
  // 8F <= 248 per item, so 256 items fit)
  auto widen = [&]() {
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      const int w = (k & 1) + 4 * (k >> 1);      // halves of vpk[k]: replicas w and w + 2
      vsum[w] += vpk[k] & 0xFFFFu;
      vsum[w + 2] += vpk[k] >> 16;
      vpk[k] = 0;
    }
    pend = 0;
    widened = true;
  };
  // Every wave's sums into its partials.  Byte mode: the packed halves when a
  // half of the wave total stays below 2^16 (8F per item, 64 / RG lanes per
  // replica byte), else the widened sums; the 4F n k offset is removed where
  // the partials are gathered.
  auto flush = [&](uint32_t *d) {
    if constexpr (MODE == kPTBytes) {
      if (!widened && pend * 8 * F * (64 >> lgRG) <= 0xFFFF) {
        if (RG == 1) flush_packed<1>(vpk, part, a, lane);
        else if (RG == 2) flush_packed<2>(vpk, part, a, lane);
        else if (RG == 4) flush_packed<4>(vpk, part, a, lane);
        else flush_packed<8>(vpk, part, a, lane);
        pend = 0;
        return;
      }
      widen();
#pragma unroll
      for (int w = 0; w < 8; ++w) {
        d[w] = vsum[w];
        vsum[w] = 0;
      }
      widened = false;
    }
    if (RG == 1) flush_partials<1>(d, part, a, lane);
    else if (RG == 2) flush_partials<2>(d, part, a, lane);
    else if (RG == 4) flush_partials<4>(d, part, a, lane);
    else flush_partials<8>(d, part, a, lane);
  };
  // Gathering every wave's partials of a replica over k sweeps: the sum less
  // `off` k, shifted right by `sh` (byte mode: 4F n and 1, else 0 and 0).
  const uint32_t off = (MODE == kPTBytes) ? 4u * static_cast<uint32_t>(F) * static_cast<uint32_t>(P.n) : 0u;
  const int sh = (MODE == kPTBytes) ? 1 : 0;
  auto gathered = [&](int rho, uint32_t k) {
    uint32_t s = 0;
#pragma unroll
    for (int v = 0; v < kPTMaxWaves; ++v) s += parts[64 * v + rho];
    return static_cast<int32_t>(s - off * k) >> sh;
  };
  // Swap state.  One wave, the last (it has the fewest sweep items, none when the
  // ladder has a wave to spare), keeps the slot map in registers (lane s: the
  // replica at slot s, and its energy as of the last swap phase), draws the swap
  // words (word 0 of the SWAP call (pair r, 0, phase q), in LDS two phases apart)
  // and decides each swap phase at the start of the next sweep's colour class 0,
  // while the other waves compute the part of their first item of that class
  // that does not depend on temperatures.  It publishes every replica's new slot
  // in slot_of; after a barrier each thread takes its replicas' table rows from
  // there and finishes the item.
  const int swap_wave = nth / 64 - 1;
  const bool swapper = wave == swap_wave;
  int rep_s = lane;                                 // replica at slot `lane` (swap wave)
  int e = E[lane];                                  // and its energy as of the last swap phase
  uint32_t word0 = 0;
  if (swapper && lane + 1 < R) {
    word0 = philox4x32_10(static_cast<uint32_t>(lane), 0u, 0u, kStreamSwap << 24, K.lo, K.hi).v[0];
    swapw[lane] = word0;
  }
  uint32_t phase = 0;
  bool pending = false;                             // a swap phase is due before class 0's thresholds
  // (an LDS null pointer is not zero: the staging flag travels on its own)
  const lds_u32 *spk_lds = (const lds_u32 *)(spk ? spk : swapw);
  SwapRows srows{};
  if (swapper) srows = swap_rows(spk_lds, spk != nullptr, R);
  // With the table staged and its rows non-increasing, the swap wave turns each
  // swap word into its pair's acceptance bound (swap_bound) when it draws it,
  // two phases ahead, so that a swap phase reads no table.
  const bool bounded = spk != nullptr && P.swap_falling != 0;
  uint32_t bnd0 = 0u, bnd1 = 0u, w_next = 0u;       // bounds of the phases of parity 0 and 1
  uint32_t b_o0 = 0, b_len = 0;                     // pair `lane`'s staged row
  float b_inv = 0.0f;
  if (swapper && bounded && lane + 1 < R) {
    b_o0 = spk_lds[lane];
    b_len = spk_lds[lane + 1] - b_o0;
    const uint32_t t1 = (1u < b_len) ? spk_lds[b_o0 + 1] : 0u;
    b_inv = (t1 == 0u || P.swap_falling == 2) ? 0.0f : 1.0f / log1m_frac32(t1);
    bnd0 = swap_bound(word0, b_o0, b_len, P.Dmax, b_inv, spk_lds);
  }
  uint32_t acc_r = 0;                               // swaps accepted by pair (lane, lane + 1)
  const uint32_t off_swap = off * static_cast<uint32_t>(P.sweeps_per_swap);
  // During the sweeps slot_of[rho] holds what a thread needs of replica rho's
  // slot s: byte mode the LDS address of its threshold base (thb), else the
  // row offset s (2F + 1).  The slot map itself is written back at the end.
  const uint32_t pub0 = static_cast<uint32_t>(reinterpret_cast<uintptr_t>(mtabb));
  auto decide_swaps = [&]() {
    __builtin_amdgcn_s_setprio(3);               // ahead of the item waves on its SIMD
    const SwapSlot ns =
        bounded ? swap_phase_bounded(rep_s, e, acc_r, off_swap, sh, R, (phase & 1) ? bnd1 : bnd0,
                                     (const lds_u32 *)parts)
                : swap_phase(rep_s, e, acc_r, off_swap, sh, R, P.Dmax, spk != nullptr, srows, spk_lds,
                             (glb_u32 *)P.stab, (const lds_u32 *)(swapw + 64 * (phase & 1)), (const lds_u32 *)parts);
    rep_s = ns.rep;
    e = ns.e;
    acc_r = ns.acc;
    if (lane < R)
      slot_of[rep_s & 63] = static_cast<int32_t>(MODE == kPTBytes ? pub0 + 4u * static_cast<uint32_t>(lane * width)
                                                                  : static_cast<uint32_t>(lane * width));
    __builtin_amdgcn_s_setprio(0);
    ++phase;
  };
  // the byte's eight entries in two 16-byte reads (slot_of has 64 entries and
  // 8a + 7 < 64; entries of absent replicas are read and not used)
  auto take_rows = [&]() {
    const int4 s0 = *reinterpret_cast<const int4 *>(slot_of + 8 * a);
    const int4 s1 = *reinterpret_cast<const int4 *>(slot_of + 8 * a + 4);
    const int32_t sl[8] = {s0.x, s0.y, s0.z, s0.w, s1.x, s1.y, s1.z, s1.w};
#pragma unroll
    for (int w = 0; w < 8; ++w) {
      if constexpr (MODE == kPTBytes)
        thb[w] = (w < nvalid) ? reinterpret_cast<const lds_u8 *>(static_cast<uintptr_t>(static_cast<uint32_t>(sl[w])))
                              : mtabb;
      else
        row[w] = (w < nvalid) ? sl[w] : 0;
    }
  };
  for (int m = 0; m < P.sweeps; ++m) {
    const bool swap_now = (m + 1) % P.sweeps_per_swap == 0;
    const uint32_t mm = static_cast<uint32_t>(m);
    const PTSweepWords swd = pt_sweep_words(K, a, mm);
#pragma unroll
    for (int c = 0; c < NPH; ++c) {
      const int lo = ph[c];
      const int cnt = (ph[c + 1] - lo) << lgRG;
      const PTRec<KIND> &cur = rb[c % NB];
      const int cn = (c + 1) % NPH;
      if (has_first[cn]) rb[(c + 1) % NB] = load_pt_rec<KIND, MODE>(rec + (ph[cn] + (tid >> lgRG)) * S::RW);
      if constexpr (MODE == kPTBytes) {
        if (pend + pmax > 256) widen();
        pend += pmax;
        if (c == 0 && pending) {
          // the previous sweep's swap phase beside the first item's head
          PTItemHead hd;
          if (swapper) decide_swaps();
          if (has_first[0]) hd = pt_item_bytes_head<KIND>(swd, cur, lo + (tid >> lgRG), latb, st8, a);
          __syncthreads();
          take_rows();
          if (has_first[0]) {
            uint32_t th[8];
            pt_thresholds(thb, hd.V, th);
            pt_item_bytes_decide(K, hd.site, lo + (tid >> lgRG), latb, st8, a, vmask, thb, f4, vpk, mm, hd.own,
                                 hd.V, hd.u, th);
          }
        } else if (has_first[c]) {
          pt_item_bytes<KIND>(K, swd, cur, lo + (tid >> lgRG), latb, st8, a, vmask, thb, f4, vpk, mm);
        }
        for (int it = tid + nth; group_live && it < cnt; it += nth) {
          const int d = lo + (it >> lgRG);
          pt_item_bytes<KIND>(K, swd, load_pt_rec<KIND, MODE>(rec + d * S::RW), d, latb, st8, a, vmask, thb, f4,
                              vpk, mm);
        }
      } else {
        if (c == 0 && pending) {
          if (swapper) decide_swaps();
          __syncthreads();
          take_rows();
        }
        if (has_first[c]) pt_item<KIND, SWAR>(P, K, cur, lo + (tid >> lgRG), latb, mtab, a, vmask, row, dE, mm);
        for (int it = tid + nth; group_live && it < cnt; it += nth) {
          const int d = lo + (it >> lgRG);
          pt_item<KIND, SWAR>(P, K, load_pt_rec<KIND, MODE>(rec + d * S::RW), d, latb, mtab, a, vmask, row, dE, mm);
        }
      }
      if (c == 0) pending = false;
      // In a sweep that ends in a swap phase: the swap wave draws the next swap
      // phase's words in phase 1 (their buffer was last read by that wave in
      // phase 0) and their bounds in phase 2, and every wave stores its energy
      // deltas ahead of the last phase's barrier (their array was last read in
      // phase 0, before that phase's barrier).
      if (c == 1 && swap_now && swapper && lane + 1 < R) {
        w_next = philox4x32_10(static_cast<uint32_t>(lane), 0u, phase + 1, kStreamSwap << 24, K.lo, K.hi).v[0];
        swapw[64 * ((phase + 1) & 1) + lane] = w_next;
      }
      if (c == 2 && swap_now && swapper && bounded && lane + 1 < R) {
        const uint32_t b = swap_bound(w_next, b_o0, b_len, P.Dmax, b_inv, spk_lds);
        if ((phase + 1) & 1) bnd1 = b;
        else bnd0 = b;
      }
      if (c == NPH - 1 && swap_now) flush(dE);
      __syncthreads();
    }
    pending = swap_now;
  }
  if (pending && swapper) decide_swaps();    // the last sweep's swap phase (reads every wave's partials)
  __syncthreads();
  flush(dE);                                 // deltas of the sweeps after the last swap phase
  __syncthreads();
  if (swapper) {                             // energies, slot map and swap counts for the results
    e += gathered(rep_s & 63, static_cast<uint32_t>(P.sweeps % P.sweeps_per_swap));
    if (lane < R) E[rep_s] = e;
    rep_at[lane] = rep_s;
    slot_of[rep_s & 63] = lane;
    acc[lane] = acc_r;
  }
  __syncthreads();
}

// Dynamic LDS: [byte-spread table: kPTSpreadWords][rec_cap words][lat_cap u64][mtab_cap words]
// [E, rep_at, slot_of, acc: 64 each][swap words: 2 x 64][energy partials: 64 per wave]
// [spack_cap words: the packed swap table when it is staged].
__global__ __launch_bounds__(64 * kPTMaxWaves) void pt_kernel(const PTDev *__restrict__ pts, int rec_cap, int lat_cap,
                                                              int mtab_cap, int spack_cap) {
  extern __shared__ __align__(16) uint32_t smem[];
  const PTDev &P = pts[blockIdx.x];       // read in place: uniform fields become scalar loads
  uint2 *st8 = reinterpret_cast<uint2 *>(smem);
  uint32_t *rec = smem + kPTSpreadWords;
  uint64_t *lat = reinterpret_cast<uint64_t *>(rec + rec_cap);
  uint32_t *mtab = rec + rec_cap + 2 * lat_cap;
  int32_t *E = reinterpret_cast<int32_t *>(mtab + mtab_cap);
  int32_t *rep_at = E + 64;
  int32_t *slot_of = rep_at + 64;
  uint32_t *acc = reinterpret_cast<uint32_t *>(slot_of + 64);
  uint32_t *swapw = acc + 64;
  uint32_t *spk = reinterpret_cast<uint32_t *>(E) + kPTLadderWords;   // after the wave scratch
  static_assert(kPTLadderWords == 4 * 64 + 2 * 64 + kPTMaxWaves * 64,
                "E, rep_at, slot_of, acc, two phases of swap words and an energy partial per wave");
  const int tid = threadIdx.x, nth = blockDim.x;
  const int rw = rec_words_of(P.kind);
  for (int x = tid; x < kSpreadEntries; x += nth) {
    const uint32_t lo = static_cast<uint32_t>(x) & 0xFu, hi = static_cast<uint32_t>(x) >> 4;
    st8[x] = make_uint2(spread8(lo) << 2, spread8(hi) << 2);
    // v_perm selector of the byte pair (i, i + 2) of a word: i where flipped
    // (second source, the V byte), 4 + i elsewhere (first source, 4F); 0x0C: zero
    auto pair_sel = [](uint32_t nib, uint32_t i) {
      const uint32_t s0 = ((nib >> i) & 1u) ? i : 4u + i, s2 = ((nib >> (i + 2)) & 1u) ? i + 2 : 6u + i;
      return s0 | (0x0Cu << 8) | (s2 << 16) | (0x0Cu << 24);
    };
    reinterpret_cast<uint4 *>(st8 + kSpreadEntries)[x] =
        make_uint4(pair_sel(lo, 0), pair_sel(lo, 1), pair_sel(hi, 0), pair_sel(hi, 1));
  }
  for (int i = tid; i < P.n * rw; i += nth) rec[i] = P.rec[i];
  const int width = 2 * P.F + 1;
  for (int i = tid; i < P.R * width; i += nth) mtab[i] = P.mtab[i];
  const bool staged = spack_cap > 0 && P.spack_words <= spack_cap;
  if (staged)
    for (int i = tid; i < P.spack_words; i += nth) spk[i] = P.spack[i];
  for (int r = tid; r < kPTMaxWaves * 64; r += nth)      // the waves' energy partials
    swapw[2 * 64 + r] = 0;
  for (int r = tid; r < 64; r += nth) {
    rep_at[r] = r;
    slot_of[r] = r;
    acc[r] = 0;
    E[r] = 0;
  }
  // initial spins from the PT_INIT stream: replica rho, site k -> word rho&3 of (k, rho>>2, 0, PT_INIT<<24)
  const int RG4 = (P.R + 3) >> 2;
  for (int d = tid; d < P.n; d += nth) {
    const uint32_t site = P.rec[d * rw] & 0xFFFFu;
    uint64_t w = 0;
    for (int a = 0; a < RG4; ++a) {
      const Words4 u = philox4x32_10(site, static_cast<uint32_t>(a), 0u, kStreamPTInit << 24, P.seed_lo, P.seed_hi);
      for (int k = 0; k < 4; ++k)
        if (4 * a + k < P.R) w |= static_cast<uint64_t>(u.v[k] >> 31) << (4 * a + k);
    }
    lat[d] = w;
  }
  if (tid == 0) lat[P.n] = 0;
  __syncthreads();
  // initial energies, one thread per replica
  if (tid < P.R) {
    int32_t e = 0;
    for (int d = 0; d < P.n; ++d) e += P.hfield[d] * (1 - 2 * static_cast<int32_t>((lat[d] >> tid) & 1ull));
    for (int t = 0; t < P.n_terms; ++t) {
      const uint32_t s01 = P.term_s[2 * t], s23 = P.term_s[2 * t + 1];
      const uint64_t x = lat[s01 & 0xFFFFu] ^ lat[s01 >> 16] ^ lat[s23 & 0xFFFFu] ^ lat[s23 >> 16];
      e += P.term_w[t] * (1 - 2 * static_cast<int32_t>((x >> tid) & 1ull));
    }
    E[tid] = e;
  }
  __syncthreads();
  const int mode = (P.F <= kPTByteF) ? kPTBytes : (P.F <= kMidF ? kPTSwar : kPTWide);
  const uint32_t *sp = staged ? spk : nullptr;
  // three phases only where the host merged two classes (byte mode, ME kinds)
  if (P.kind == kKindME) {
    if (mode == kPTBytes && P.nph == 3)
      pt_ladder<kKindME, kPTBytes, 3>(P, rec, lat, mtab, st8, E, rep_at, slot_of, acc, swapw, sp);
    else if (mode == kPTBytes)
      pt_ladder<kKindME, kPTBytes, 4>(P, rec, lat, mtab, st8, E, rep_at, slot_of, acc, swapw, sp);
    else if (mode == kPTSwar)
      pt_ladder<kKindME, kPTSwar, 4>(P, rec, lat, mtab, st8, E, rep_at, slot_of, acc, swapw, sp);
    else pt_ladder<kKindME, kPTWide, 4>(P, rec, lat, mtab, st8, E, rep_at, slot_of, acc, swapw, sp);
  } else if (P.kind == kKindLHZ) {
    if (mode == kPTBytes) pt_ladder<kKindLHZ, kPTBytes, 4>(P, rec, lat, mtab, st8, E, rep_at, slot_of, acc, swapw, sp);
    else if (mode == kPTSwar)
      pt_ladder<kKindLHZ, kPTSwar, 4>(P, rec, lat, mtab, st8, E, rep_at, slot_of, acc, swapw, sp);
    else pt_ladder<kKindLHZ, kPTWide, 4>(P, rec, lat, mtab, st8, E, rep_at, slot_of, acc, swapw, sp);
  } else {
    if (mode == kPTBytes && P.nph == 3)
      pt_ladder<kKindMEC, kPTBytes, 3>(P, rec, lat, mtab, st8, E, rep_at, slot_of, acc, swapw, sp);
    else if (mode == kPTBytes)
      pt_ladder<kKindMEC, kPTBytes, 4>(P, rec, lat, mtab, st8, E, rep_at, slot_of, acc, swapw, sp);
    else if (mode == kPTSwar)
      pt_ladder<kKindMEC, kPTSwar, 4>(P, rec, lat, mtab, st8, E, rep_at, slot_of, acc, swapw, sp);
    else pt_ladder<kKindMEC, kPTWide, 4>(P, rec, lat, mtab, st8, E, rep_at, slot_of, acc, swapw, sp);
  }
  // results: spins by replica in physical order, energies by replica, slot map, swap counts
  for (size_t i = tid; i < static_cast<size_t>(P.R) * P.n; i += nth) {
    const int rho = static_cast<int>(i / P.n), k = static_cast<int>(i % P.n);
    P.spins[i] = ((lat[P.dev_of[k]] >> rho) & 1ull) ? int8_t(-1) : int8_t(1);
  }
  if (tid < P.R) {
    P.energy[tid] = E[tid];
    P.rep_at[tid] = rep_at[tid];
    if (tid + 1 < P.R) P.swap_acc[tid] = acc[tid];
  }

}

// ----------------------------------------------------------- host launchers
hipError_t launch_pt(const PTDev *pts, int count, int waves, int rec_cap, int lat_cap, int mtab_cap, int spack_cap,
                     hipStream_t stream) {
  const size_t lds =
      (static_cast<size_t>(kPTSpreadWords) + rec_cap + 2ull * lat_cap + mtab_cap + kPTLadderWords + spack_cap) * 4;
  (void)hipGetLastError();
  hipLaunchKernelGGL(pt_kernel, dim3(count), dim3(64 * waves), lds, stream, pts, rec_cap, lat_cap, mtab_cap,
                     spack_cap);
  return hipGetLastError();
}

hipError_t set_pt_lds_limit(size_t bytes) {
  return hipFuncSetAttribute(reinterpret_cast<const void *>(pt_kernel), hipFuncAttributeMaxDynamicSharedMemorySize,
                             static_cast<int>(bytes));
}

}  // namespace sqa
