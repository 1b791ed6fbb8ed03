// gfx950 SQA kernels: lattice initialisation, the persistent sweep kernels
// (single-site Metropolis moves, and the time-like Wolff cluster moves of
// Sec. III), per-slice energies and ME majority-vote decoding.
//
// Method (arXiv:1603.03755): discrete-time path-integral Monte Carlo on L
// Trotter slices of an embedded Ising Hamiltonian (Sec. III, Appendix B);
// majority-vote decoding of ME chains (Eq. (4)).
//
// Data layout on the device.  Each replica's space-time lattice is held in
// LDS for the whole anneal, one 64-bit word per site: even slices in the low
// half (bit j = slice 2j), odd slices in the high half, a set bit = spin -1.
// A lane processes one "item": one site, one slice parity p and one byte b of
// the parity-p half, i.e. the eight same-parity slices 16b+p+2k (k = 0..7).
// Each attempt's uniform is the 32-bit number (hi << 16) | lo; hi is half
// k >> 2 of word k & 3 of the Philox4x32-10 call with counter
// (site, 2b+p, sweep, SQA<<24 | replica), and lo the same half of the call
// with stream SQA_LO.  Acceptance compares u with a threshold R read from a
// per-sweep table indexed by (s*f, s*(time-neighbour sum)): hi < R >> 16
// accepts and hi > R >> 16 rejects whatever lo is, so the item draws the
// SQA_LO call only when some hi equals its threshold's top half (probability
// 2^-16 per attempt).  All arithmetic is integer.
#include <hip/hip_runtime.h>

#include "sqa_sweep.h"

namespace sqa {


// ------------------------------------------------------ SQA, Wolff moves
// Time-like Wolff cluster moves (Sec. III), lattice in natural layout.  For
// each colour class, two phases separated by a wave-level barrier:
//  1. item = (site of the class, byte q of its word): the eight slices
//     8q..8q+7 and the ring bonds that start at them.  Bond b = 8q+k joins
//     when its two spins are equal and its 32-bit uniform (hi << 16) | lo
//     passes the sweep's join threshold; hi is half k >> 2 of word k & 3 of
//     the WOLFF call with counter word 1 = q, lo the same from the WOLFF_LO
//     call, drawn only on a tie of hi with the threshold's top half.  The
//     item also forms, per slice, the weighted disagreement sum
//     S = sum_t |w_t| X_t + |h| O (s f = F_site - 2 S) as one byte per slice:
//     4 S from the signed-weight record when F <= 63, else S from the plain
//     record.  Join bits and S bytes go to the wave's LDS scratch.
//  2. one lane per site: the seed slice tau0 = floor(u L / 2^32) and the
//     acceptance word (counter word 1 = 64); the cluster is the run of joined
//     bonds through tau0 (ring rotation, trailing and leading ones); with
//     A = |C| F_site - 2 sum_{tau in C} S_tau the move is accepted when the
//     acceptance word passes the threshold at A + L F, and the cluster's bits
//     are flipped.
// Sites of one class share no term, so their moves commute and every read in
// phase 1 sees the state left by the previous class.  Large classes are
// processed in chunks of kWolffChunk sites.

// Cluster through slice t0 of a ring of L slices whose joined bonds are the
// bits of jn (bit b: slices b and b+1 mod L; bits L..63 are ignored).
__device__ __forceinline__ uint64_t ring_cluster(uint64_t jn, int t0, int L) {
  const uint64_t full = (L == 64) ? ~0ull : ((1ull << L) - 1ull);
  jn &= full;
  const uint64_t r = t0 ? (((jn >> t0) | (jn << (L - t0))) & full) : jn;   // bond t0 at bit 0
  if (r == full) return full;
  const int f = __builtin_ctzll(~r);                     // joined bonds forward of t0
  const int g = __builtin_clzll(~(r << (64 - L)));       // joined bonds backward of t0
  uint64_t cr = (2ull << f) - 1ull;                      // slices t0 .. t0+f
  if (g) cr |= full ^ (full >> g);                       // slices t0-g .. t0-1
  return t0 ? (((cr << t0) | (cr >> (L - t0))) & full) : cr;
}

// The same for L = 64 (rotations by t0 without masks).
__device__ __forceinline__ uint64_t ring_cluster64(uint64_t jn, int t0) {
  const uint64_t r = (jn >> t0) | (jn << ((64 - t0) & 63));   // bond t0 at bit 0
  if (r == ~0ull) return ~0ull;
  const int f = __builtin_ctzll(~r);                         // joined bonds forward of t0
  const int g = __builtin_clzll(~r);                         // joined bonds backward of t0
  uint64_t cr = (2ull << f) - 1ull;                          // slices t0 .. t0+f
  if (g) cr |= ~(~0ull >> g);                                // slices t0-g .. t0-1
  return (cr << t0) | (cr >> ((64 - t0) & 63));
}

template <int KIND, bool LARGE, bool L64>
__device__ __forceinline__ void wolff_bonds(const HandleDev &H, const uint32_t *__restrict__ rec, const uint64_t *lat,
                                            uint32_t *scr, const uint2 *stab, int lo, int nc, uint32_t m, uint32_t c3,
                                            uint32_t padd, const PhiloxTwo &pql, int lane) {
  using S = Site<KIND>;
  const int L = H.L;
  const int Q = (L + 7) >> 3;
  const int cnt = nc * Q;
  const uint8_t *latb = reinterpret_cast<const uint8_t *>(lat);
  uint8_t *jb = reinterpret_cast<uint8_t *>(scr);        // [nc] 64-bit join masks
  uint32_t *sb = scr + 2 * nc;                            // [16][nc] S bytes of slices 4i..4i+3
  // item (j, q): site lo + j, slices 8q .. 8q + 7; its S bytes go to words 2q nc + j
  // and (2q + 1) nc + j of sb
  // pq: the site-free part of the item call's first two rounds (counter (site, q, m, c3))
  // srp, wp: the site's record and lattice word when the caller has them
  auto item = [&](int j, int q, const PhiloxTwo &pq, const SignedRec<KIND> *srp, const uint64_t *wp) {
    const int d = lo + j;
    const uint32_t *r = rec + d * S::RW;
    uint32_t site, wts = 0, wts2 = 0, hw = 0, neg = 0;
    uint32_t poff[S::T * S::P];
    SignedRec<KIND> sr;
    if constexpr (!LARGE) {
      sr = srp ? *srp : load_signed_rec<KIND>(r);
      site = sr.site;
#pragma unroll
      for (int x = 0; x < S::T * S::P; ++x) poff[x] = sr.poff[x];
    } else if constexpr (KIND == kKindME) {
      const uint4 r0 = load_rec4(r);
      site = r0.x & 0xFFFFu;
      wts = r0.y & 0xFFFFFFu;
      hw = r0.y >> 24;
      neg = r0.z & 0xFFu;
      poff[0] = r0.z >> 16; poff[1] = r0.w & 0xFFFFu; poff[2] = r0.w >> 16;
    } else if constexpr (KIND == kKindMEC) {
      uint32_t base_unused;
      load_rec_mec(r, site, base_unused, wts, wts2, hw, neg, poff);
    } else {
      const uint4 r0 = *reinterpret_cast<const uint4 *>(r);
      const uint4 r1 = *reinterpret_cast<const uint4 *>(r + 4);
      const uint2 r2 = *reinterpret_cast<const uint2 *>(r + 8);
      site = r0.x & 0xFFFFu;
      wts = r0.y;
      hw = r0.z & 0xFFu;
      neg = (r0.z >> 8) & 0xFFu;
      const uint32_t pw[6] = {r1.x, r1.y, r1.z, r1.w, r2.x, r2.y};
#pragma unroll
      for (int x = 0; x < 6; ++x) {
        poff[2 * x] = pw[x] & 0xFFFFu;
        poff[2 * x + 1] = pw[x] >> 16;
      }
    }
    const uint64_t w = wp ? *wp : lat[d];
    // partner bytes of the terms (LDS reads) stay in flight during the Philox rounds
    const uint8_t *lb = latb + q;
    uint32_t pbyte[S::T * S::P];
#pragma unroll
    for (int i = 0; i < S::T * S::P; ++i) pbyte[i] = lb[poff[i]];
    __builtin_amdgcn_sched_barrier(0);
    PhiloxState ps = philox_two(site, pq);
    philox_rounds<8>(ps);
    const Words4 u = philox_words(ps);
    __builtin_amdgcn_sched_barrier(0);
    uint32_t own, eq;                               // the byte's spins; its bonds between equal spins
    if constexpr (L64) {
      // bytes q < 4 in the low word, q >= 4 in the high one; the next slices are
      // a funnel shift by one (slice 63's next is slice 0, bit 0 of the low word)
      const uint32_t lo32 = static_cast<uint32_t>(w), hi32 = static_cast<uint32_t>(w >> 32);
      const bool upper = q >= 4;
      const uint32_t wa = upper ? hi32 : lo32, wb = upper ? lo32 : hi32;
      const uint32_t s8 = static_cast<uint32_t>(8 * q) & 31u;
      own = __builtin_amdgcn_ubfe(wa, s8, 8);
      eq = ~(own ^ __builtin_amdgcn_alignbit(wb, wa, s8 + 1u)) & 0xFFu;
    } else {
      const int sh = 8 * q;
      own = static_cast<uint32_t>(w >> sh) & 0xFFu;
      // bit tau of nx: the spin of slice tau + 1 (mod L)
      const uint64_t nx = (w >> 1) | ((w & 1ull) << (L - 1));
      const uint32_t nb = static_cast<uint32_t>(nx >> sh) & 0xFFu;
      const uint32_t valid = (L - sh >= 8) ? 0xFFu : ((1u << (L - sh)) - 1u);
      eq = ~(own ^ nb) & valid;
    }

    // bond 8q+k: uniform (hi << 16) | lo, hi = half k >> 2 of word k & 3 of the
    // WOLFF call (site, q, sweep), lo the same from the WOLFF_LO call, drawn only
    // when some hi equals the top half of the join threshold.  D = hi - top
    // half is negative iff the bond joins on hi alone and zero on a tie; the
    // sign bits are shifted into `join` from bond 7 down.
    const uint32_t ph = padd >> 16;
    uint32_t join = 0, dmin = 0xFFFFFFFFu;
#pragma unroll
    for (int k = 7; k >= 0; --k) {
      const uint32_t hi = (k < 4) ? (u.v[k] & 0xFFFFu) : (u.v[k - 4] >> 16);
      const uint32_t D = hi - ph;
      join = __builtin_amdgcn_alignbit(join, D, 31);
      dmin = min(dmin, D);
    }
    if (dmin == 0) {
      const uint32_t c3lo = (c3 & 0xFFFFFFu) | (kStreamWolffLo << 24);
      const Words4 v = philox4x32_10(site, static_cast<uint32_t>(q), m, c3lo, H.seed_lo, H.seed_hi);
      join = 0;
#pragma unroll
      for (int k = 0; k < 8; ++k) {
        const uint32_t uu = (k < 4) ? ((u.v[k] << 16) | (v.v[k] & 0xFFFFu))
                                    : ((u.v[k - 4] & 0xFFFF0000u) | (v.v[k - 4] >> 16));
        if (min(uu, 0xFFFFFFFEu) < padd) join |= 1u << k;
      }
    }
    jb[8 * j + q] = static_cast<uint8_t>(join & eq);

    if constexpr (!LARGE) {
      // 4 S of the eight slices, one byte each (F <= 63), from the record's
      // signed weights: slices 8q..8q+3 in word 2q, 8q+4..8q+7 in word 2q+1
      const uint2 a = signed_sums<KIND>(sr, stab + kSpreadEntries, own, pbyte);
      sb[2 * q * nc + j] = a.x;
      sb[2 * q * nc + j + nc] = a.y;
    } else {
      // S of the eight slices in 8-bit fields, three slices per word (acc_lo
      // 0-2, acc_hi 3-5, acc_x 6-7; the operands of the 24-bit multiplies stay
      // below 2^24), repacked to one byte per slice for the store
      const uint32_t negh = 0u - ((neg >> S::HB) & 1u);
      const uint32_t ox = (own ^ negh) & 0xFFu;
      uint32_t acc_lo = __umul24(spread3(ox), hw);
      uint32_t acc_hi = __umul24(spread3(ox >> 3), hw);
      uint32_t acc_x = __umul24(spread3(ox >> 6), hw);
#pragma unroll
      for (int t = 0; t < S::T; ++t) {
        uint32_t prod = own;
#pragma unroll
        for (int x = 0; x < S::P; ++x) prod ^= pbyte[S::P * t + x];
        const uint32_t xt = (prod ^ (0u - ((neg >> t) & 1u))) & 0xFFu;
        const uint32_t wt = term_weight(wts, wts2, t);
        acc_lo += __umul24(spread3(xt), wt);
        acc_hi += __umul24(spread3(xt >> 3), wt);
        acc_x += __umul24(spread3(xt >> 6), wt);
      }
      sb[2 * q * nc + j] = (acc_lo & 0xFFFFFFu) | (acc_hi << 24);
      sb[2 * q * nc + j + nc] = ((acc_hi >> 8) & 0xFFFFu) | (acc_x << 16);
    }
  };
  if (L64 && nc == 64) {
    // a full chunk: lane j takes site j, and the byte q is the same in every lane
    // (a uniform loop counter, so its part of the counter words stays scalar)
    // (the site's record and lattice word are read once for its eight bytes)
    SignedRec<KIND> sr0{};
    if constexpr (!LARGE) sr0 = load_signed_rec<KIND>(rec + (lo + lane) * S::RW);
    const uint64_t w0 = lat[lo + lane];
    for (int q = 0; q < 8; ++q) {
      const int qs = __builtin_amdgcn_readfirstlane(q);   // uniform: its two-round part in scalar registers
      item(lane, qs, philox_two_prep(static_cast<uint32_t>(qs), m, c3, H.seed_lo, H.seed_hi),
           LARGE ? nullptr : &sr0, &w0);
    }
  } else if (L64) {
    // a partial chunk: items site-major (8 j + q), so a lane keeps the byte
    // q = lane & 7, whose two-round part the caller prepared once per sweep (pql),
    // and the eight lanes of a site read the same partner words
    for (int it = lane; it < cnt; it += 64) item(it >> 3, lane & 7, pql, nullptr, nullptr);
  } else {
    const int dq = 64 / nc, dr = 64 - dq * nc;
    int q = lane / nc;
    int j = lane - q * nc;
    for (int it = lane; it < cnt; it += 64, j += dr, q += dq) {
      if (j >= nc) { j -= nc; q += 1; }
      item(j, q, philox_two_prep(static_cast<uint32_t>(q), m, c3, H.seed_lo, H.seed_hi), nullptr, nullptr);
    }
  }
}

template <int KIND, bool LARGE, bool L64>
__device__ __forceinline__ void wolff_flips(const HandleDev &H, const uint32_t *__restrict__ rec, uint64_t *lat,
                                            const uint32_t *scr, const uint2 *stab, int lo, int nc,
                                            const PhiloxTwo &sw2, const uint32_t *arow, int lane) {
  using S = Site<KIND>;
  const int L = H.L;
  const uint64_t *jw = reinterpret_cast<const uint64_t *>(scr);
  const uint32_t *sb = scr + 2 * nc;
  for (int j = lane; j < nc; j += 64) {
    const int d = lo + j;
    const uint32_t *r = rec + d * S::RW;
    const uint32_t r0x = r[0];
    const uint32_t site = r0x & 0xFFFFu;
    // F_site = |h| + sum |w_t|: stored in the signed-weight records; in the
    // plain ones the bytes of record word 1 (and, for LHZ, |h|)
    // (ME: w0..w2, |h|; LHZ: w0..w3 then |h|; ME on Chimera: w0..w3 then w4, w5, |h|)
    uint32_t fs;
    if constexpr (!LARGE) {
      fs = r[KIND == kKindLHZ ? 3 : 4] >> 16;
    } else {
      const uint32_t r1 = r[1], r2 = r[2];
      fs = (KIND == kKindME)    ? __builtin_amdgcn_sad_u8(r1, 0u, 0u)
           : (KIND == kKindLHZ) ? __builtin_amdgcn_sad_u8(r1, 0u, r2 & 0xFFu)
                                : __builtin_amdgcn_sad_u8(r1, 0u, __builtin_amdgcn_sad_u8(r2 & 0xFFFFFFu, 0u, 0u));
    }
    PhiloxState ps = philox_two(site, sw2);
    philox_rounds<8>(ps);
    const Words4 u = philox_words(ps);
    const int t0 = static_cast<int>(__umulhi(u.v[0], static_cast<uint32_t>(L)));
    const uint64_t cl = L64 ? ring_cluster64(jw[j], t0) : ring_cluster(jw[j], t0, L);
    const uint32_t clh[2] = {static_cast<uint32_t>(cl), static_cast<uint32_t>(cl >> 32)};
    uint32_t ssum;
    if constexpr (!LARGE) {
      // bytes of 4 S, masked by the spreads (value 4 per slice) of each cluster
      // byte: the dot products sum 16 S over the cluster
      const uint2 *st8 = stab + kSpreadEntries;
      uint32_t s16 = 0;
      if constexpr (L64) {      // eight cluster bytes: every read issued before the sums
        // (a full chunk's stride is a constant: the sums' reads take immediate offsets)
        const uint32_t *sbj = sb + j;
        uint2 mk[8];
#pragma unroll
        for (int k = 0; k < 8; ++k) mk[k] = st8[(clh[k >> 2] >> (8 * (k & 3))) & 0xFFu];
        if (nc == kWolffChunk) {
#pragma unroll
          for (int k = 0; k < 8; ++k) {
            s16 = __builtin_amdgcn_udot4(sbj[(2 * k) * kWolffChunk], mk[k].x, s16, false);
            s16 = __builtin_amdgcn_udot4(sbj[(2 * k + 1) * kWolffChunk], mk[k].y, s16, false);
          }
        } else {
#pragma unroll
          for (int k = 0; k < 8; ++k) {
            s16 = __builtin_amdgcn_udot4(sbj[(2 * k) * nc], mk[k].x, s16, false);
            s16 = __builtin_amdgcn_udot4(sbj[(2 * k + 1) * nc], mk[k].y, s16, false);
          }
        }
      } else {
        const int Q = (L + 7) >> 3;
        for (int k = 0; k < Q; ++k) {
          const uint2 mk = st8[(clh[k >> 2] >> (8 * (k & 3))) & 0xFFu];
          s16 = __builtin_amdgcn_udot4(sb[(2 * k) * nc + j], mk.x, s16, false);
          s16 = __builtin_amdgcn_udot4(sb[(2 * k + 1) * nc + j], mk.y, s16, false);
        }
      }
      ssum = s16 >> 4;
    } else {
      const int words = (L + 3) >> 2;
      ssum = 0;
      for (int i = 0; i < words; ++i)
        ssum = __builtin_amdgcn_udot4(sb[i * nc + j], spread8(clh[i >> 3] >> (4 * (i & 7))), ssum, false);
    }
    const int a = __popcll(cl) * static_cast<int>(fs) - 2 * static_cast<int>(ssum);
    // (a global load: the table row is read in place)
    const uint32_t thr = ((const __attribute__((address_space(1))) uint32_t *)arow)[a];
    if (min(u.v[1], 0xFFFFFFFEu) < thr) lat[d] ^= cl;
  }
}

template <int KIND>
__device__ __forceinline__ void wolff_replica(const HandleDev &H, const uint32_t *rec, uint64_t *lat, uint32_t *scr,
                                              const uint2 *stab, int rep, int lane) {
  if (H.flags & kFlagInit) init_lattice<true>(H, lat, rep, lane, 64);
  else load_lattice<true>(H, lat, rep, lane, 64);
  wave_sync();
  const uint32_t c3 = (kStreamWolff << 24) | static_cast<uint32_t>(rep);
  for (int m = H.m0; m < H.m1; ++m) {
    const uint32_t padd = H.table[m];
    // the site call's counter (site, kWolffSiteCtr, m, c3): its first two rounds' site-free part
    const PhiloxTwo sw2 = philox_two_prep(kWolffSiteCtr, static_cast<uint32_t>(m), c3, H.seed_lo, H.seed_hi);
    // the bond calls of a lane's byte lane & 7 in partial chunks (L = 64): the same per sweep
    const PhiloxTwo pql = philox_two_prep(static_cast<uint32_t>(lane & 7), static_cast<uint32_t>(m), c3, H.seed_lo,
                                          H.seed_hi);
    const uint32_t *arow = H.wacc + static_cast<size_t>(H.wrows > 1 ? m : 0) * H.wwidth + H.L * H.F;
    // each colour class in chunks of at most 64 sites (one lane per site in
    // phase 2; sites of a class commute, so chunking does not change results)
    for (int c = 0; c < 4; ++c)
      for (int lo = H.cls[c]; lo < H.cls[c + 1]; lo += kWolffChunk) {
        const int nc = min(kWolffChunk, H.cls[c + 1] - lo);
        const uint32_t mm = static_cast<uint32_t>(m);
        if (H.F > kMidF) {
          wolff_bonds<KIND, true, false>(H, rec, lat, scr, stab, lo, nc, mm, c3, padd, pql, lane);
          wave_sync();
          wolff_flips<KIND, true, false>(H, rec, lat, scr, stab, lo, nc, sw2, arow, lane);
        } else if (H.L == 64) {
          wolff_bonds<KIND, false, true>(H, rec, lat, scr, stab, lo, nc, mm, c3, padd, pql, lane);
          wave_sync();
          wolff_flips<KIND, false, true>(H, rec, lat, scr, stab, lo, nc, sw2, arow, lane);
        } else {
          wolff_bonds<KIND, false, false>(H, rec, lat, scr, stab, lo, nc, mm, c3, padd, pql, lane);
          wave_sync();
          wolff_flips<KIND, false, false>(H, rec, lat, scr, stab, lo, nc, sw2, arow, lane);
        }
        wave_sync();
      }
  }
  store_lattice<true>(H, lat, rep, lane, 64);
  if (H.flags & kFlagEnergy) slice_energies<true>(H, lat, rep, lane);
  wave_sync();
}

// Persistent kernels, one per move type (each keeps its own register budget;
// team mode has a kernel of its own in team_kernels.hip): each workgroup
// repeatedly takes the next work item (handle, replica group) from `counter`,
// stages the handle's site records in LDS, and runs one replica per wavefront
// through sweeps m0..m1-1.
// Dynamic LDS: [kSpreadWords: byte -> spread table][rec_cap words][waves x lat_cap u64]
// [waves x tab_cap words] (tab: the Metropolis table row, or the Wolff phase scratch).
#ifndef SQA_WAVES_PER_EU
#define SQA_WAVES_PER_EU 1
#endif
template <int MOVE>
__global__ __launch_bounds__(512) __attribute__((amdgpu_waves_per_eu(SQA_WAVES_PER_EU, 8))) void sqa_anneal_kernel(const HandleDev *__restrict__ hds,
                                                         const WorkItem *__restrict__ items, int n_items,
                                                         int *__restrict__ counter, int rec_cap,
                                                         int lat_cap, int tab_cap) {
  extern __shared__ __align__(16) uint32_t smem[];
  __shared__ int s_item;
  const int waves = blockDim.x >> 6;
  const int wave = threadIdx.x >> 6;
  const int lane = threadIdx.x & 63;
  uint2 *stab = reinterpret_cast<uint2 *>(smem);
  uint32_t *rec = smem + kSpreadWords;
  uint64_t *lat = reinterpret_cast<uint64_t *>(rec + rec_cap) + static_cast<size_t>(wave) * lat_cap;
  uint32_t *tab = rec + rec_cap + 2 * waves * lat_cap + wave * tab_cap;
  fill_spread_tables(stab);
  for (;;) {
    if (threadIdx.x == 0) s_item = atomicAdd(counter, 1);
    __syncthreads();
    const int it = __builtin_amdgcn_readfirstlane(s_item);   // uniform: handle fields go to SGPRs
    if (it >= n_items) break;
    const WorkItem wi = items[it];
    const HandleDev &H = hds[wi.handle];      // read in place: uniform fields become scalar loads
    const int rw = rec_words_of(H.kind);
    const int nwords = H.n * rw;
    for (int i = threadIdx.x; i < nwords; i += blockDim.x) rec[i] = H.rec[i];
    __syncthreads();
    if (wave < wi.nrep) {
      const int rep = wi.rep0 + wave;
      if constexpr (MOVE == kMoveWolff) {
        if (H.kind == kKindME) wolff_replica<kKindME>(H, rec, lat, tab, stab, rep, lane);
        else if (H.kind == kKindLHZ) wolff_replica<kKindLHZ>(H, rec, lat, tab, stab, rep, lane);
        else wolff_replica<kKindMEC>(H, rec, lat, tab, stab, rep, lane);
      } else {
        if (H.kind == kKindME) anneal_replica<kKindME>(H, rec, lat, tab, stab, rep, lane, lane, 64, false);
        else if (H.kind == kKindLHZ) anneal_replica<kKindLHZ>(H, rec, lat, tab, stab, rep, lane, lane, 64, false);
        else anneal_replica<kKindMEC>(H, rec, lat, tab, stab, rep, lane, lane, 64, false);
      }
    }
    __syncthreads();
  }
}

__global__ void reset_counter_kernel(int *counter) {
  if (threadIdx.x == 0 && blockIdx.x == 0) *counter = 0;
}

// Standalone K1: initial lattice in device memory, one thread per (replica,
// site, slice group of 8).
__global__ void sqa_init_kernel(HandleDev H) {
  const int G = (H.L + 7) >> 3;
  const size_t total = static_cast<size_t>(H.R) * H.n * G;
  const size_t i = static_cast<size_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i >= total) return;
  const int k = static_cast<int>(i % H.n);
  const size_t rest = i / H.n;
  const int g = static_cast<int>(rest % G);
  const int rep = static_cast<int>(rest / G);
  const uint32_t c3 = (kStreamInit << 24) | static_cast<uint32_t>(rep);
  int8_t *dst = H.spins + static_cast<size_t>(rep) * H.L * H.n;
  for (int p = 0; p < 2; ++p) {
    const Words4 u = philox4x32_10(static_cast<uint32_t>(k), static_cast<uint32_t>((g << 1) | p), 0u, c3,
                                   H.seed_lo, H.seed_hi);
#pragma unroll
    for (int w = 0; w < 4; ++w) {
      const int tau = 8 * g + p + 2 * w;
      if (tau < H.L) dst[static_cast<size_t>(tau) * H.n + k] = (u.v[w] >> 31) ? int8_t(-1) : int8_t(1);
    }
  }
}

// ------------------------------------------------------ ME majority vote
// Eq. (4): qbar_i = sign(sum_r s_{i len + r}) on slice `slice`, tie -> +1, and
// the logical energy of Eq. (1); chains of len = N-1 (clique chains) or
// ceil(N/4)+1 (Chimera) consecutive sites.  One workgroup per replica, thread
// i <-> chain i.
__global__ void me_majority_kernel(const int8_t *__restrict__ spins, int N, int len, int n_sites, int L, int slice,
                                   const int32_t *__restrict__ J, const int32_t *__restrict__ h,
                                   int8_t *__restrict__ logical, int32_t *__restrict__ energy) {
  __shared__ int8_t q[256];
  __shared__ int32_t part[256];
  const int rep = blockIdx.x;
  const int8_t *s = spins + (static_cast<size_t>(rep) * L + slice) * n_sites;
  for (int i = threadIdx.x; i < N; i += blockDim.x) {
    int sum = 0;
    for (int r = 0; r < len; ++r) sum += s[i * len + r];
    q[i] = (sum >= 0) ? int8_t(1) : int8_t(-1);
    if (logical) logical[static_cast<size_t>(rep) * N + i] = q[i];
  }
  __syncthreads();
  int32_t e = 0;
  for (int i = threadIdx.x; i < N; i += blockDim.x) {
    if (h) e += h[i] * q[i];
    for (int j = i + 1; j < N; ++j) e += J[i * N + j] * q[i] * q[j];
  }
  part[threadIdx.x] = e;
  __syncthreads();
  for (int stride = blockDim.x >> 1; stride > 0; stride >>= 1) {
    if (threadIdx.x < stride) part[threadIdx.x] += part[threadIdx.x + stride];
    __syncthreads();
  }
  if (threadIdx.x == 0 && energy) energy[rep] = part[0];
}

// ----------------------------------------------------------- host launchers
hipError_t launch_sqa_anneal(int move, const HandleDev *hds, const WorkItem *items, int n_items, int *counter,
                             int grid, int waves, int rec_cap, int lat_cap, int tab_cap, bool team,
                             hipStream_t stream) {
  team = team && move == kMoveMetropolis;
  const int lattices = team ? 1 : waves;
  const size_t lds = (static_cast<size_t>(kSpreadWords) + rec_cap + 2ull * lattices * lat_cap +
                      static_cast<size_t>(waves) * tab_cap) * 4;
  (void)hipGetLastError();
  hipLaunchKernelGGL(reset_counter_kernel, dim3(1), dim3(64), 0, stream, counter);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  if (team) return launch_sqa_team(hds, items, n_items, counter, grid, waves, rec_cap, lat_cap, tab_cap, lds, stream);
  if (move == kMoveWolff)
    hipLaunchKernelGGL(sqa_anneal_kernel<kMoveWolff>, dim3(grid), dim3(64 * waves), lds, stream, hds, items, n_items,
                       counter, rec_cap, lat_cap, tab_cap);
  else
    hipLaunchKernelGGL(sqa_anneal_kernel<kMoveMetropolis>, dim3(grid), dim3(64 * waves), lds, stream, hds, items,
                       n_items, counter, rec_cap, lat_cap, tab_cap);
  return hipGetLastError();
}

// Resident workgroups of `waves` waves per compute unit for the given dynamic LDS.
int sqa_anneal_occupancy(int move, int waves, size_t lds_bytes, bool team) {
  if (team && move == kMoveMetropolis) return sqa_team_occupancy(waves, lds_bytes);
  int blocks = 0;
  hipError_t e = (move == kMoveWolff)
                     ? hipOccupancyMaxActiveBlocksPerMultiprocessor(&blocks, sqa_anneal_kernel<kMoveWolff>, 64 * waves,
                                                                    lds_bytes)
                     : hipOccupancyMaxActiveBlocksPerMultiprocessor(&blocks, sqa_anneal_kernel<kMoveMetropolis>,
                                                                    64 * waves, lds_bytes);
  if (e != hipSuccess) {
    (void)hipGetLastError();
    return 0;
  }
  return blocks;
}

hipError_t set_sqa_anneal_lds_limit(size_t bytes) {
  hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void *>(sqa_anneal_kernel<kMoveMetropolis>),
                                     hipFuncAttributeMaxDynamicSharedMemorySize, static_cast<int>(bytes));
  hipError_t e2 = hipFuncSetAttribute(reinterpret_cast<const void *>(sqa_anneal_kernel<kMoveWolff>),
                                      hipFuncAttributeMaxDynamicSharedMemorySize, static_cast<int>(bytes));
  hipError_t e3 = set_sqa_team_lds_limit(bytes);
  return e != hipSuccess ? e : (e2 != hipSuccess ? e2 : e3);
}

hipError_t launch_sqa_init(const HandleDev &H, hipStream_t stream) {
  const int G = (H.L + 7) >> 3;
  const size_t total = static_cast<size_t>(H.R) * H.n * G;
  const int block = 256;
  const size_t grid = (total + block - 1) / block;
  (void)hipGetLastError();
  hipLaunchKernelGGL(sqa_init_kernel, dim3(static_cast<unsigned>(grid)), dim3(block), 0, stream, H);
  return hipGetLastError();
}

hipError_t launch_me_majority(const int8_t *spins, int R, int N, int len, int n_sites, int L, int slice,
                              const int32_t *J, const int32_t *h, int8_t *logical, int32_t *energy,
                              hipStream_t stream) {
  (void)hipGetLastError();
  hipLaunchKernelGGL(me_majority_kernel, dim3(R), dim3(256), 0, stream, spins, N, len, n_sites, L, slice, J, h,
                     logical, energy);
  return hipGetLastError();
}

}  // namespace sqa
