// Metropolis sweep of the SQA kernels (Sec. III, Appendix B): the lattice's
// LDS I/O and the item loop of one colour class, shared by the one-wave-per-
// replica kernel and the team kernel (one replica per workgroup).  The data
// layout and the acceptance rule are those stated at the top of sqa_kernels.hip.
#pragma once

#include <hip/hip_runtime.h>

#include "device_common.h"

namespace sqa {

// Byte -> spread tables of the Metropolis and Wolff items, filled by the whole
// workgroup at kernel start (layout in device_types.h).
__device__ __forceinline__ void fill_spread_tables(uint2 *stab) {
  for (int x = threadIdx.x; x < kSpreadEntries; x += blockDim.x) {
    const uint32_t lo = static_cast<uint32_t>(x) & 0xFu, hi = static_cast<uint32_t>(x) >> 4;
    stab[x] = make_uint2(spread6(lo), spread6(hi));
    stab[kSpreadEntries + x] = make_uint2(spread8(lo) << 2, spread8(hi) << 2);
  }
}
// ------------------------------------------------------------ lattice I/O
// LDS word of a site, a set bit is spin -1.  Parity-split layout (Metropolis
// kernel): bits 0..31 hold the even slices (bit j = slice 2j), bits 32..63 the
// odd slices (bit 32+j = slice 2j+1).  Natural layout (NAT, Wolff kernel):
// bit tau = slice tau.  With L = 1 only bit 0 is used.
template <bool NAT>
__device__ __forceinline__ int slice_bit(int tau) { return NAT ? tau : (tau >> 1) + ((tau & 1) << 5); }

// Builds the initial lattice in LDS: s = -1 iff bit 31 of the INIT-stream word
// of (replica, slice, site, sweep 0).
template <bool NAT>
__device__ __forceinline__ void init_lattice(const HandleDev &H, uint64_t *lat, int rep, int lane, int nthr) {
  const int L = H.L, n = H.n;
  const int G = (L + 7) >> 3;
  const uint32_t c3 = (kStreamInit << 24) | static_cast<uint32_t>(rep);
  const int rw = rec_words_of(H.kind);
  for (int d = lane; d < n; d += nthr) {
    const uint32_t site = H.rec[d * rw] & 0xFFFFu;
    uint64_t w = 0;
    for (int g = 0; g < G; ++g) {
      for (int p = 0; p < 2; ++p) {
        const Words4 u = philox4x32_10(site, static_cast<uint32_t>((g << 1) | p), 0u, c3, H.seed_lo, H.seed_hi);
#pragma unroll
        for (int k = 0; k < 4; ++k) {
          const int tau = 8 * g + p + 2 * k;
          if (tau < L) w |= static_cast<uint64_t>(u.v[k] >> 31) << slice_bit<NAT>(tau);
        }
      }
    }
    lat[d] = w;
  }
  if (lane == 0) lat[n] = 0;
}

// Loads [L][n] int8 spins of one replica (physical order) into LDS words.
template <bool NAT>
__device__ __forceinline__ void load_lattice(const HandleDev &H, uint64_t *lat, int rep, int lane, int nthr) {
  const int L = H.L, n = H.n;
  const int8_t *src = H.spins + static_cast<size_t>(rep) * L * n;
  for (int k = lane; k < n; k += nthr) {
    uint64_t w = 0;
    for (int tau = 0; tau < L; ++tau)
      w |= static_cast<uint64_t>(src[static_cast<size_t>(tau) * n + k] < 0) << slice_bit<NAT>(tau);
    lat[H.dev_of[k]] = w;
  }
  if (lane == 0) lat[n] = 0;
}

template <bool NAT>
__device__ __forceinline__ void store_lattice(const HandleDev &H, const uint64_t *lat, int rep, int lane, int nthr) {
  const int L = H.L, n = H.n;
  int8_t *dst = H.spins + static_cast<size_t>(rep) * L * n;
  for (int k = lane; k < n; k += nthr) {
    const uint64_t w = lat[H.dev_of[k]];
    for (int tau = 0; tau < L; ++tau)
      dst[static_cast<size_t>(tau) * n + k] = ((w >> slice_bit<NAT>(tau)) & 1ull) ? int8_t(-1) : int8_t(1);
  }
}

// E^tau = sum_k h_k s_k + sum_t w_t prod s, one lane per slice.
template <bool NAT>
__device__ __forceinline__ void slice_energies(const HandleDev &H, const uint64_t *lat, int rep, int lane) {
  const int tau = lane;
  if (tau >= H.L) return;
  const int b = slice_bit<NAT>(tau);
  int32_t E = 0;
  for (int d = 0; d < H.n; ++d) E += H.hfield[d] * (1 - 2 * static_cast<int32_t>((lat[d] >> b) & 1ull));
  for (int t = 0; t < H.n_terms; ++t) {
    const uint32_t s01 = H.term_s[2 * t], s23 = H.term_s[2 * t + 1];
    const uint64_t x = lat[s01 & 0xFFFFu] ^ lat[s01 >> 16] ^ lat[s23 & 0xFFFFu] ^ lat[s23 >> 16];
    E += H.term_w[t] * (1 - 2 * static_cast<int32_t>((x >> b) & 1ull));
  }
  H.energy[static_cast<size_t>(rep) * H.L + tau] = E;
}

// ------------------------------------------------------------ SQA sweep
// Item loop over one (slice parity p, colour c) class of one replica, by the
// nthr threads of its team (one wave, or the whole workgroup).
// Item = (site of colour c, byte b of its parity-p half word): the eight slices
// tau = 16b + 2k + p (k = 0..7), whose random halves come from one Philox call
// (counter word 1 = 2b + p).  For each slice the acceptance index is
// base - (6 S + e), with
//   S = sum_t |w_t| X_t + |h| O   (X_t = 1 iff term t's product with the own
//       spin disagrees with the sign of w_t; O likewise for the field),
//   e = number of time neighbours whose spin differs from the own spin;
// S and e by field mode:
// kFieldSmall (F <= 10): signed-weight records (see device_types.h); packed
//   16-bit multiply-adds form 4 (c + 6 A) per slice in byte fields (A = F_site
//   - S, the agreeing weight; c = 3 (F - F_site)), and the spreads of the
//   agreeing time neighbours add 4 e' (e' = 2 - e).  4 (c + 6 A + e') =
//   4 (base - (6 S + e)) < 256 is the byte offset of the slice's table entry;
// kFieldMid (F <= 63): S and e in 6-bit fields, four slices per word;
// kFieldLarge (F <= 255): S in 8-bit fields, three slices per word (at bits
//   0, 8, 16, so both operands of the 24-bit multiplies stay below 2^24).
// FL: 0 for any L, or the compile-time L in {16, 32, 64} (whole bytes,
//   replicated-word rotation, L > 1); items are then taken site-major (the
//   B = L/16 bytes of one site in neighbouring lanes share their record and
//   partner words).
// P: the slice parity.
template <int KIND, int MODE, int FL, int P>
__device__ __forceinline__ void sweep_class(const HandleDev &H, const uint32_t *__restrict__ rec, uint32_t *lat32,
                                            const uint32_t *tab, const uint2 *stab, int c, uint32_t m, uint32_t c3,
                                            int tid, int nthr) {
  constexpr int p = P;
  constexpr bool FASTL = FL != 0;
  using S = Site<KIND>;
  const int L = FASTL ? FL : H.L;
  const int Hp = (L == 1) ? 1 : (L >> 1);       // slices of one parity
  const int B = (Hp + 7) >> 3;                  // bytes per parity half
  const int lo = H.cls[c];
  const int nc = H.cls[c + 1] - lo;
  if (nc <= 0) return;
  const int cnt = nc * B;
  uint8_t *latb = reinterpret_cast<uint8_t *>(lat32);
  const bool ring32 = FASTL || (Hp & (Hp - 1)) == 0;   // Hp divides 32: rotate a replicated word
  const bool ragged = !FASTL && (Hp & 7) != 0;          // last byte has fewer than eight slices
  // FASTL: item it = j * B + b (B a power of two).  Otherwise it = b * nc + j,
  // threads advancing by nthr items: (j, b) += (nthr % nc, nthr / nc).
  const int lgB = (B >= 4) ? 2 : (B - 1);
  const int dq = nthr / nc, dr = nthr - dq * nc;
  int b = FASTL ? (tid & (B - 1)) : tid / nc;
  int j = FASTL ? (tid >> lgB) : tid - b * nc;
  for (int it = tid; it < cnt; it += nthr, j += dr, b += dq) {
    if constexpr (FASTL) {
      j = it >> lgB;
      b = it & (B - 1);
    } else if (j >= nc) {
      j -= nc;
      b += 1;
    }
    const int d = lo + j;
    const uint32_t *r = rec + d * S::RW;

    uint32_t site, base = 0, wts = 0, wts2 = 0, hw = 0, neg = 0;
    uint32_t poff[S::T * S::P];
    SignedRec<KIND> sr;
    if constexpr (MODE == kFieldSmall) {
      sr = load_signed_rec<KIND>(r);
      site = sr.site;
#pragma unroll
      for (int q = 0; q < S::T * S::P; ++q) poff[q] = sr.poff[q];
    } else if constexpr (KIND == kKindME) {
      const uint4 r0 = load_rec4(r);
      site = r0.x & 0xFFFFu; base = r0.x >> 16;
      wts = r0.y & 0xFFFFFFu;
      hw = r0.y >> 24;
      neg = r0.z & 0xFFu;
      poff[0] = r0.z >> 16; poff[1] = r0.w & 0xFFFFu; poff[2] = r0.w >> 16;
    } else if constexpr (KIND == kKindMEC) {
      load_rec_mec(r, site, base, wts, wts2, hw, neg, poff);
    } else {
      const uint4 r0 = *reinterpret_cast<const uint4 *>(r);
      const uint4 r1 = *reinterpret_cast<const uint4 *>(r + 4);
      const uint2 r2 = *reinterpret_cast<const uint2 *>(r + 8);
      site = r0.x & 0xFFFFu; base = r0.x >> 16;
      wts = r0.y;
      hw = r0.z & 0xFFu;
      neg = (r0.z >> 8) & 0xFFu;
      const uint32_t pw[6] = {r1.x, r1.y, r1.z, r1.w, r2.x, r2.y};
#pragma unroll
      for (int q = 0; q < 6; ++q) {
        poff[2 * q] = pw[q] & 0xFFFFu;
        poff[2 * q + 1] = pw[q] >> 16;
      }
    }
    const uint32_t negh = 0u - ((neg >> S::HB) & 1u);   // 0 or all ones: field sign

    const uint2 word = *reinterpret_cast<const uint2 *>(lat32 + 2 * d);
    // partner bytes of the terms (LDS reads), then the first half of the Philox
    // rounds while they are in flight (the scheduling barriers keep that order)
    const uint8_t *lb = latb + (4 * p + b);        // the item's byte in any site word
    uint32_t pbyte[S::T * S::P];
#pragma unroll
    for (int i = 0; i < S::T * S::P; ++i) pbyte[i] = lb[poff[i]];
    const uint32_t ctr1 = static_cast<uint32_t>((b << 1) | p);
    PhiloxState ps = philox_start(site, ctr1, m, c3, H.seed_lo, H.seed_hi);
    __builtin_amdgcn_sched_barrier(0);
    philox_rounds<5>(ps);
    philox_pin(ps);
    __builtin_amdgcn_sched_barrier(0);

    const uint32_t own_half = p ? word.y : word.x;
    const uint32_t oth_half = p ? word.x : word.y;
    const int sh = 8 * b;
    const uint32_t own = (own_half >> sh) & 0xFFu;

    // time neighbours: other-parity bits j (n0) and j-1 (p = 0) or j+1 (p = 1), ring of Hp
    uint32_t dn, up;
    if (!FASTL && L == 1) {
      dn = own;               // no time coupling: exactly one "differing neighbour", b = 0
      up = own ^ 0xFFu;
    } else {
      const uint32_t n0 = (oth_half >> sh) & 0xFFu;
      const int s1 = p ? ((!FASTL && sh + 1 == Hp) ? 0 : sh + 1) : ((b == 0) ? Hp - 1 : sh - 1);
      uint32_t n1;
      if (ring32) {
        uint32_t y = oth_half;
        for (int k = Hp; k < 32; k <<= 1) y |= y << k;
        n1 = __builtin_amdgcn_alignbit(y, y, static_cast<uint32_t>(s1)) & 0xFFu;
      } else {
        const uint64_t yy = static_cast<uint64_t>(oth_half) | (static_cast<uint64_t>(oth_half) << Hp);
        n1 = static_cast<uint32_t>(yy >> s1) & 0xFFu;
      }
      dn = p ? n0 : n1;
      up = p ? n1 : n0;
    }
    // disagreeing (agreeing, kFieldSmall) time neighbours
    const uint32_t agree = (MODE == kFieldSmall) ? 0xFFu : 0u;
    const uint32_t e1 = own ^ dn ^ agree, e2 = own ^ up ^ agree;
    const uint32_t ox = (own ^ negh) & 0xFFu;
    uint32_t flip = 0;
    if constexpr (MODE == kFieldSmall) {
      // Byte fields, slices k = 0..3 in f_lo and 4..7 in f_hi, each holding
      // 4 (c + 6 A + e') < 256: the byte offset of the slice's table entry.
      // 4 (c + 6 A) comes from the signed-weight record; the spreads of the
      // agreeing time neighbours are added as plain 32-bit sums (no field
      // reaches 256, so nothing carries between fields).
      const uint2 *st8 = stab + kSpreadEntries;
      const uint2 a = signed_sums<KIND>(sr, st8, own, pbyte);
      const uint2 se1 = st8[e1], se2 = st8[e2];
      const uint32_t f_lo = a.x + se1.x + se2.x;
      const uint32_t f_hi = a.y + se1.y + se2.y;

      // top halves of the eight thresholds (LDS reads), the second half of the
      // Philox rounds while they are in flight, then slice k: D = hi - top half
      // (hi: half k >> 2 of word k & 3), negative iff the flip is accepted on hi
      // alone, zero on a tie; the sign bits are shifted into `flip` from slice 7
      // down, and a tie shows as a zero minimum of the D taken unsigned
      const uint8_t *tabb = reinterpret_cast<const uint8_t *>(tab);
      uint32_t th[8];
#pragma unroll
      for (int k = 0; k < 8; ++k)
        th[k] = *reinterpret_cast<const uint16_t *>(tabb + (((k < 4 ? f_lo : f_hi) >> (8 * (k & 3))) & 0xFFu) + 2);
      __builtin_amdgcn_sched_barrier(0);
      philox_rounds<5>(ps);
      __builtin_amdgcn_sched_barrier(0);
      const Words4 u = philox_words(ps);
      uint32_t dmin = 0xFFFFFFFFu;
#pragma unroll
      for (int k = 7; k >= 0; --k) {
        const uint32_t hi = (k < 4) ? (u.v[k] & 0xFFFFu) : (u.v[k - 4] >> 16);
        const uint32_t D = hi - th[k];
        flip = __builtin_amdgcn_alignbit(flip, D, 31);
        dmin = min(dmin, D);
      }
      if (dmin == 0) {     // some hi equals its threshold's top half: decide all eight on the full 32 bits
        const uint32_t c3lo = (c3 & 0xFFFFFFu) | (kStreamSQALo << 24);
        const Words4 v = philox4x32_10(site, ctr1, m, c3lo, H.seed_lo, H.seed_hi);
        flip = 0;
#pragma unroll
        for (int k = 0; k < 8; ++k) {
          const uint32_t fb = ((k < 4 ? f_lo : f_hi) >> (8 * (k & 3))) & 0xFFu;
          const uint32_t R = *reinterpret_cast<const uint32_t *>(tabb + fb);
          const uint32_t uu = (k < 4) ? ((u.v[k] << 16) | (v.v[k] & 0xFFFFu))
                                      : ((u.v[k - 4] & 0xFFFF0000u) | (v.v[k - 4] >> 16));
          if (min(uu, 0xFFFFFFFEu) < R) flip |= 1u << k;
        }
      }
    } else {
      const uint2 se1 = spread_of(stab, e1), se2 = spread_of(stab, e2);
      const uint32_t ev_lo = se1.x + se2.x;
      const uint32_t ev_hi = se1.y + se2.y;

      // weighted disagreement counts, slices k = 0..3 in acc_lo and 4..7 in acc_hi
      uint32_t acc_lo = 0, acc_hi = 0, acc_x = 0;     // kFieldLarge: slices 0-2, 3-5, 6-7
      if constexpr (MODE == kFieldLarge) {
        acc_lo = __umul24(spread3(ox), hw);
        acc_hi = __umul24(spread3(ox >> 3), hw);
        acc_x = __umul24(spread3(ox >> 6), hw);
      } else {
        const uint2 so = spread_of(stab, ox);
        acc_lo = __umul24(so.x, hw);
        acc_hi = __umul24(so.y, hw);
      }
#pragma unroll
      for (int t = 0; t < S::T; ++t) {
        uint32_t prod = own;
#pragma unroll
        for (int q = 0; q < S::P; ++q) prod ^= pbyte[S::P * t + q];
        const uint32_t x = (prod ^ (0u - ((neg >> t) & 1u))) & 0xFFu;
        const uint32_t wt = term_weight(wts, wts2, t);
        if constexpr (MODE == kFieldLarge) {
          acc_lo += __umul24(spread3(x), wt);
          acc_hi += __umul24(spread3(x >> 3), wt);
          acc_x += __umul24(spread3(x >> 6), wt);
        } else {
          const uint2 sx = spread_of(stab, x);
          acc_lo += __umul24(sx.x, wt);
          acc_hi += __umul24(sx.y, wt);
        }
      }

      // table index of each of the eight slices
      uint32_t ix[8];
      if constexpr (MODE == kFieldMid) {
#pragma unroll
        for (int w = 0; w < 4; ++w) {
          ix[w] = base - (6u * __builtin_amdgcn_ubfe(acc_lo, 6 * w, 6) + __builtin_amdgcn_ubfe(ev_lo, 6 * w, 2));
          ix[w + 4] = base - (6u * __builtin_amdgcn_ubfe(acc_hi, 6 * w, 6) + __builtin_amdgcn_ubfe(ev_hi, 6 * w, 2));
        }
      } else {
        const uint32_t sums[3] = {acc_lo, acc_hi, acc_x};
#pragma unroll
        for (int w = 0; w < 4; ++w) {
          const uint32_t s0 = __builtin_amdgcn_ubfe(sums[w / 3], 8 * (w % 3), 8);
          const uint32_t s1 = __builtin_amdgcn_ubfe(sums[(w + 4) / 3], 8 * ((w + 4) % 3), 8);
          ix[w] = base - (6u * s0 + __builtin_amdgcn_ubfe(ev_lo, 6 * w, 2));
          ix[w + 4] = base - (6u * s1 + __builtin_amdgcn_ubfe(ev_hi, 6 * w, 2));
        }
      }

      // top halves of the eight thresholds (LDS reads), the second half of the
      // Philox rounds while they are in flight, then slice k: random half k >> 2
      // of word k & 3 against the top half of its threshold
      const uint16_t *tab16 = reinterpret_cast<const uint16_t *>(tab);
      uint32_t th[8];
#pragma unroll
      for (int k = 0; k < 8; ++k) th[k] = tab16[2 * ix[k] + 1];
      __builtin_amdgcn_sched_barrier(0);
      philox_rounds<5>(ps);
      __builtin_amdgcn_sched_barrier(0);
      const Words4 u = philox_words(ps);
      bool tie = false;
#pragma unroll
      for (int k = 0; k < 8; ++k) {
        const uint32_t hi = (k < 4) ? (u.v[k] & 0xFFFFu) : (u.v[k - 4] >> 16);
        if (hi < th[k]) flip |= 1u << k;
        tie |= (hi == th[k]);
      }
      if (tie) {     // some hi equals its threshold's top half: decide all eight on the full 32 bits
        const uint32_t c3lo = (c3 & 0xFFFFFFu) | (kStreamSQALo << 24);
        const Words4 v = philox4x32_10(site, ctr1, m, c3lo, H.seed_lo, H.seed_hi);
        flip = 0;
#pragma unroll
        for (int k = 0; k < 8; ++k) {
          const uint32_t uu = (k < 4) ? ((u.v[k] << 16) | (v.v[k] & 0xFFFFu))
                                      : ((u.v[k - 4] & 0xFFFF0000u) | (v.v[k - 4] >> 16));
          if (min(uu, 0xFFFFFFFEu) < tab[ix[k]]) flip |= 1u << k;
        }
      }
    }
    if (ragged) {            // slices beyond the parity's last one stay put
      const int valid = Hp - sh;
      if (valid < 8) flip &= (1u << valid) - 1u;
    }
    latb[8 * d + 4 * p + b] = static_cast<uint8_t>(own ^ flip);
  }
}

// One replica through sweeps m0..m1-1 by a team: one wave (team = false; tid
// = lane, nthr = 64) or the whole workgroup (team = true; tid = thread index,
// nthr = block size), which then synchronises with workgroup barriers.  Each
// wave keeps its own copy of the sweep's table row in `tab`.
template <int KIND>
__device__ __forceinline__ void anneal_replica(const HandleDev &H, const uint32_t *rec, uint64_t *lat, uint32_t *tab,
                                               const uint2 *stab, int rep, int lane, int tid, int nthr, bool team) {
  auto team_sync = [&]() {
    if (team) __syncthreads();
    else wave_sync();
  };
  if (H.flags & kFlagInit) init_lattice<false>(H, lat, rep, tid, nthr);
  else load_lattice<false>(H, lat, rep, tid, nthr);
  team_sync();
  const uint32_t c3 = (kStreamSQA << 24) | static_cast<uint32_t>(rep);
  const int parities = (H.L == 1) ? 1 : 2;
  const bool smallf = H.F <= kSmallF;
  const bool midf = H.F <= kMidF;
  const int fast = (smallf && (H.L == 16 || H.L == 32 || H.L == 64)) ? H.L : 0;   // compile-time L variants
  // the next sweep's table row is fetched into a register during the current sweep
  const bool row_in_reg = H.tw <= 64;
  uint32_t next_row = 0;
  if (row_in_reg && lane < H.tw) next_row = H.table[static_cast<size_t>(H.m0) * H.tw + lane];
  for (int m = H.m0; m < H.m1; ++m) {
    if (row_in_reg) {
      if (lane < H.tw) tab[lane] = next_row;
      if (m + 1 < H.m1 && lane < H.tw) next_row = H.table[static_cast<size_t>(m + 1) * H.tw + lane];
    } else {
      const uint32_t *row = H.table + static_cast<size_t>(m) * H.tw;
      for (int i = lane; i < H.tw; i += 64) tab[i] = row[i];
    }
    team_sync();
    uint32_t *lat32 = reinterpret_cast<uint32_t *>(lat);
    const uint32_t mm = static_cast<uint32_t>(m);
    for (int c = 0; c < 4; ++c) {
      if (fast == 64) sweep_class<KIND, kFieldSmall, 64, 0>(H, rec, lat32, tab, stab, c, mm, c3, tid, nthr);
      else if (fast == 32) sweep_class<KIND, kFieldSmall, 32, 0>(H, rec, lat32, tab, stab, c, mm, c3, tid, nthr);
      else if (fast == 16) sweep_class<KIND, kFieldSmall, 16, 0>(H, rec, lat32, tab, stab, c, mm, c3, tid, nthr);
      else if (smallf) sweep_class<KIND, kFieldSmall, 0, 0>(H, rec, lat32, tab, stab, c, mm, c3, tid, nthr);
      else if (midf) sweep_class<KIND, kFieldMid, 0, 0>(H, rec, lat32, tab, stab, c, mm, c3, tid, nthr);
      else sweep_class<KIND, kFieldLarge, 0, 0>(H, rec, lat32, tab, stab, c, mm, c3, tid, nthr);
      team_sync();
    }
    if (parities > 1)
      for (int c = 0; c < 4; ++c) {
        if (fast == 64) sweep_class<KIND, kFieldSmall, 64, 1>(H, rec, lat32, tab, stab, c, mm, c3, tid, nthr);
        else if (fast == 32) sweep_class<KIND, kFieldSmall, 32, 1>(H, rec, lat32, tab, stab, c, mm, c3, tid, nthr);
        else if (fast == 16) sweep_class<KIND, kFieldSmall, 16, 1>(H, rec, lat32, tab, stab, c, mm, c3, tid, nthr);
        else if (smallf) sweep_class<KIND, kFieldSmall, 0, 1>(H, rec, lat32, tab, stab, c, mm, c3, tid, nthr);
        else if (midf) sweep_class<KIND, kFieldMid, 0, 1>(H, rec, lat32, tab, stab, c, mm, c3, tid, nthr);
        else sweep_class<KIND, kFieldLarge, 0, 1>(H, rec, lat32, tab, stab, c, mm, c3, tid, nthr);
        team_sync();
      }
  }
  store_lattice<false>(H, lat, rep, tid, nthr);
  if (H.flags & kFlagEnergy) slice_energies<false>(H, lat, rep, tid);
  team_sync();
}

// Host side of the team kernel (team_kernels.hip), called by the launchers in
// sqa_kernels.hip: the launch itself (the work counter already cleared on
// `stream`; lds = the dynamic LDS bytes), the resident workgroups per compute
// unit, and the dynamic-LDS limit.
hipError_t launch_sqa_team(const HandleDev *hds, const WorkItem *items, int n_items, int *counter, int grid, int waves,
                           int rec_cap, int lat_cap, int tab_cap, size_t lds, hipStream_t stream);
int sqa_team_occupancy(int waves, size_t lds_bytes);
hipError_t set_sqa_team_lds_limit(size_t bytes);

}  // namespace sqa
