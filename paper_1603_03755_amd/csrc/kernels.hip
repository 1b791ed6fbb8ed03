// gfx950 kernels: SQA init, the persistent SQA sweep kernel, per-slice
// energies, ME majority-vote decoding and parallel tempering.
//
// Method (arXiv:1603.03755): discrete-time path-integral Monte Carlo on L
// Trotter slices of an embedded Ising Hamiltonian (Sec. III, Appendix B) with
// single-site Metropolis moves; parallel tempering of the classical embedded
// Hamiltonian (Appendix B, Eqs. (B1)-(B2)); majority-vote decoding of ME
// chains (Eq. (4)).
//
// Data layout on the device.  Each replica's space-time lattice is held in
// LDS for the whole anneal, one 64-bit word per site: even slices in the low
// half (bit j = slice 2j), odd slices in the high half, a set bit = spin -1.
// A lane processes one "item": one site, one slice parity p and one byte b of
// the parity-p half, i.e. the eight same-parity slices 16b+p+2k (k = 0..7).
// Four same-parity slices 8g+p+2w (w = 0..3) share one Philox4x32-10 call
// (counter (site, 2g+p, sweep, SQA<<24 | replica), one 32-bit word per
// slice), so an item uses the calls of groups g = 2b and 2b+1.  All
// arithmetic is integer; acceptance compares the word with a threshold read
// from a per-sweep table indexed by (s*f, s*(time-neighbour sum)).
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

__device__ __forceinline__ Words4 philox4x32_10(uint32_t x0, uint32_t x1, uint32_t x2, uint32_t x3,
                                               uint32_t key0, uint32_t key1) {
  constexpr uint32_t kMulA = 0xD2511F53u, kMulB = 0xCD9E8D57u;
  constexpr uint32_t kWeylA = 0x9E3779B9u, kWeylB = 0xBB67AE85u;
#pragma unroll
  for (int round = 0; round < 10; ++round) {
    const uint64_t pa = static_cast<uint64_t>(kMulA) * x0;
    const uint64_t pb = static_cast<uint64_t>(kMulB) * x2;
    // three-input XORs (truth table 0x96)
    const uint32_t y0 = __builtin_amdgcn_bitop3_b32(static_cast<uint32_t>(pb >> 32), x1, key0, 0x96);
    const uint32_t y2 = __builtin_amdgcn_bitop3_b32(static_cast<uint32_t>(pa >> 32), x3, key1, 0x96);
    x1 = static_cast<uint32_t>(pb);
    x3 = static_cast<uint32_t>(pa);
    x0 = y0;
    x2 = y2;
    key0 += kWeylA;
    key1 += kWeylB;
  }
  Words4 r;
  r.v[0] = x0; r.v[1] = x1; r.v[2] = x2; r.v[3] = x3;
  return r;
}

// Orders LDS accesses of one wavefront around a phase boundary.  A wave's LDS
// operations are executed in program order, so only the compiler needs fencing.
__device__ __forceinline__ void wave_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

__device__ __forceinline__ uint32_t bit_at(uint32_t v, int q) { return (v >> q) & 1u; }

// ------------------------------------------------------------ lattice I/O
// LDS word of a site: bits 0..31 hold the even slices (bit j = slice 2j),
// bits 32..63 the odd slices (bit 32+j = slice 2j+1); a set bit is spin -1.
// With L = 1 only bit 0 is used.
__device__ __forceinline__ int slice_bit(int tau) { return (tau >> 1) + ((tau & 1) << 5); }

// Builds the initial lattice in LDS: s = -1 iff bit 31 of the INIT-stream word
// of (replica, slice, site, sweep 0).
__device__ __forceinline__ void init_lattice(const HandleDev &H, uint64_t *lat, int rep, int lane) {
  const int L = H.L, n = H.n;
  const int G = (L + 7) >> 3;
  const uint32_t c3 = (kStreamInit << 24) | static_cast<uint32_t>(rep);
  const int rw = (H.kind == kKindME) ? kRecWordsME : kRecWordsLHZ;
  for (int d = lane; d < n; d += 64) {
    const uint32_t site = H.rec[d * rw] & 0xFFFFu;
    uint64_t w = 0;
    for (int g = 0; g < G; ++g) {
      for (int p = 0; p < 2; ++p) {
        const Words4 u = philox4x32_10(site, static_cast<uint32_t>((g << 1) | p), 0u, c3, H.seed_lo, H.seed_hi);
#pragma unroll
        for (int k = 0; k < 4; ++k) {
          const int tau = 8 * g + p + 2 * k;
          if (tau < L) w |= static_cast<uint64_t>(u.v[k] >> 31) << slice_bit(tau);
        }
      }
    }
    lat[d] = w;
  }
  if (lane == 0) lat[n] = 0;
}

// Loads [L][n] int8 spins of one replica (physical order) into LDS words.
__device__ __forceinline__ void load_lattice(const HandleDev &H, uint64_t *lat, int rep, int lane) {
  const int L = H.L, n = H.n;
  const int8_t *src = H.spins + static_cast<size_t>(rep) * L * n;
  for (int k = lane; k < n; k += 64) {
    uint64_t w = 0;
    for (int tau = 0; tau < L; ++tau)
      w |= static_cast<uint64_t>(src[static_cast<size_t>(tau) * n + k] < 0) << slice_bit(tau);
    lat[H.dev_of[k]] = w;
  }
  if (lane == 0) lat[n] = 0;
}

__device__ __forceinline__ void store_lattice(const HandleDev &H, const uint64_t *lat, int rep, int lane) {
  const int L = H.L, n = H.n;
  int8_t *dst = H.spins + static_cast<size_t>(rep) * L * n;
  for (int k = lane; k < n; k += 64) {
    const uint64_t w = lat[H.dev_of[k]];
    for (int tau = 0; tau < L; ++tau)
      dst[static_cast<size_t>(tau) * n + k] = ((w >> slice_bit(tau)) & 1ull) ? int8_t(-1) : int8_t(1);
  }
}

// E^tau = sum_k h_k s_k + sum_t w_t prod s, one lane per slice.
__device__ __forceinline__ void slice_energies(const HandleDev &H, const uint64_t *lat, int rep, int lane) {
  const int tau = lane;
  if (tau >= H.L) return;
  const int b = slice_bit(tau);
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
template <int KIND>
struct Site;

template <>
struct Site<kKindME> {
  static constexpr int T = 3, P = 1, RW = kRecWordsME;
};
template <>
struct Site<kKindLHZ> {
  static constexpr int T = 4, P = 3, RW = kRecWordsLHZ;
};

// Four bits of a nibble moved to bit 0 of four 6-bit fields (bits 0, 6, 12,
// 18): every partial product of the 24-bit multiply lands on a distinct bit.
__device__ __forceinline__ uint32_t spread6(uint32_t nib) { return __umul24(nib & 0xFu, 0x8421u) & 0x41041u; }
// The same for bits 4..7 of a byte.
__device__ __forceinline__ uint32_t spread6_hi(uint32_t byte) {
  return (__umul24(byte & 0xF0u, 0x8421u) >> 4) & 0x41041u;
}

// 64-lane item loop over one (slice parity p, colour c) class of one replica.
// Item = (site of colour c, byte b of its parity-p half word): the eight slices
// tau = 16b + 2k + p (k = 0..7), served by the two Philox calls of slice groups
// 2b and 2b+1 (four words each).  For each slice the acceptance index is
// base - (6 S + e), with
//   S = sum_t |w_t| X_t + |h| O   (X_t = 1 iff term t's product with the own
//       spin disagrees with the sign of w_t; O likewise for the field),
//   e = number of time neighbours whose spin differs from the own spin;
// S and e are accumulated four slices at a time in 6-bit fields.
// SMALLF (F <= 10): the records carry 6|w| and 6|h|, so the fields hold 6 S
//   directly and 6 S + e < 64 stays inside a field.
// FASTL: L in {16, 32, 64} (whole bytes, replicated-word rotation, L > 1).
template <int KIND, bool SMALLF, bool FASTL>
__device__ __forceinline__ void sweep_class(const HandleDev &H, const uint32_t *__restrict__ rec, uint32_t *lat32,
                                            const uint32_t *tab, int c, int p, uint32_t m, uint32_t c3, int lane) {
  using S = Site<KIND>;
  const int L = H.L;
  const int Hp = (L == 1) ? 1 : (L >> 1);       // slices of one parity
  const int B = (Hp + 7) >> 3;                  // bytes per parity half
  const int lo = H.cls[c];
  const int nc = H.cls[c + 1] - lo;
  if (nc <= 0) return;
  const int cnt = nc * B;
  uint8_t *latb = reinterpret_cast<uint8_t *>(lat32);
  const bool ring32 = FASTL || (Hp & (Hp - 1)) == 0;   // Hp divides 32: rotate a replicated word
  const bool ragged = !FASTL && (Hp & 7) != 0;          // last byte has fewer than eight slices
  // item it = b * nc + j; lanes advance by 64 items: (j, b) += (64 % nc, 64 / nc)
  const int dq = 64 / nc, dr = 64 - dq * nc;
  int b = lane / nc;
  int j = lane - b * nc;
  for (int it = lane; it < cnt; it += 64, j += dr, b += dq) {
    if (j >= nc) { j -= nc; b += 1; }
    const int d = lo + j;
    const uint32_t *r = rec + d * S::RW;

    uint32_t site, base, wts, hw, neg;
    uint32_t poff[S::T * S::P];
    if constexpr (KIND == kKindME) {
      const uint4 r0 = *reinterpret_cast<const uint4 *>(r);
      site = r0.x & 0xFFFFu; base = r0.x >> 16;
      wts = r0.y & 0xFFFFFFu;
      hw = r0.y >> 24;
      neg = r0.z & 0xFFu;
      poff[0] = r0.z >> 16; poff[1] = r0.w & 0xFFFFu; poff[2] = r0.w >> 16;
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
    const uint32_t negh = 0u - ((neg >> 4) & 1u);   // 0 or all ones: field sign

    const uint2 word = *reinterpret_cast<const uint2 *>(lat32 + 2 * d);
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
    const uint32_t e1 = own ^ dn, e2 = own ^ up;
    const uint32_t ev_lo = spread6(__builtin_amdgcn_ubfe(e1, 0, 4)) + spread6(__builtin_amdgcn_ubfe(e2, 0, 4));
    const uint32_t ev_hi = spread6_hi(e1) + spread6_hi(e2);

    // weighted disagreement counts, slices k = 0..3 in acc_lo and 4..7 in acc_hi
    const uint8_t *lb = latb + (4 * p + b);        // the item's byte in any site word
    const uint32_t ox = (own ^ negh) & 0xFFu;
    uint32_t acc_lo = __umul24(spread6(__builtin_amdgcn_ubfe(ox, 0, 4)), hw);
    uint32_t acc_hi = __umul24(spread6(__builtin_amdgcn_ubfe(ox, 4, 4)), hw);
#pragma unroll
    for (int t = 0; t < S::T; ++t) {
      uint32_t prod = own;
#pragma unroll
      for (int q = 0; q < S::P; ++q) prod ^= lb[poff[S::P * t + q]];
      const uint32_t x = prod ^ (0u - ((neg >> t) & 1u));
      const uint32_t wt = (wts >> (8 * t)) & 0xFFu;
      acc_lo += __umul24(spread6(__builtin_amdgcn_ubfe(x, 0, 4)), wt);
      acc_hi += __umul24(spread6(__builtin_amdgcn_ubfe(x, 4, 4)), wt);
    }

    const Words4 u0 = philox4x32_10(site, static_cast<uint32_t>((b << 2) | p), m, c3, H.seed_lo, H.seed_hi);
    const Words4 u1 = philox4x32_10(site, static_cast<uint32_t>((b << 2) | 2 | p), m, c3, H.seed_lo, H.seed_hi);
    const uint32_t *tb = tab + base;                  // thresholds are read at tb[-(6 S + e)]
    uint32_t flip = 0;
    if constexpr (SMALLF) {
      const uint32_t f_lo = acc_lo + ev_lo;
      const uint32_t f_hi = acc_hi + ev_hi;
#pragma unroll
      for (int w = 0; w < 4; ++w) {
        const uint32_t R0 = *(tb - __builtin_amdgcn_ubfe(f_lo, 6 * w, 6));
        const uint32_t R1 = *(tb - __builtin_amdgcn_ubfe(f_hi, 6 * w, 6));
        if (min(u0.v[w], 0xFFFFFFFEu) < R0) flip |= 1u << w;
        if (min(u1.v[w], 0xFFFFFFFEu) < R1) flip |= 16u << w;
      }
    } else {
#pragma unroll
      for (int w = 0; w < 4; ++w) {
        const uint32_t i0 = 6u * __builtin_amdgcn_ubfe(acc_lo, 6 * w, 6) + __builtin_amdgcn_ubfe(ev_lo, 6 * w, 2);
        const uint32_t i1 = 6u * __builtin_amdgcn_ubfe(acc_hi, 6 * w, 6) + __builtin_amdgcn_ubfe(ev_hi, 6 * w, 2);
        if (min(u0.v[w], 0xFFFFFFFEu) < *(tb - i0)) flip |= 1u << w;
        if (min(u1.v[w], 0xFFFFFFFEu) < *(tb - i1)) flip |= 16u << w;
      }
    }
    if (ragged) {            // slices beyond the parity's last one stay put
      const int valid = Hp - sh;
      if (valid < 8) flip &= (1u << valid) - 1u;
    }
    latb[8 * d + 4 * p + b] = static_cast<uint8_t>(own ^ flip);
  }
}

template <int KIND>
__device__ __forceinline__ void anneal_replica(const HandleDev &H, const uint32_t *rec, uint64_t *lat, uint32_t *tab,
                               int rep, int lane) {
  if (H.flags & kFlagInit) init_lattice(H, lat, rep, lane);
  else load_lattice(H, lat, rep, lane);
  wave_sync();
  const uint32_t c3 = (kStreamSQA << 24) | static_cast<uint32_t>(rep);
  const int parities = (H.L == 1) ? 1 : 2;
  const bool smallf = H.F <= kSmallF;
  const bool fast = smallf && (H.L == 16 || H.L == 32 || H.L == 64);
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
    wave_sync();
    uint32_t *lat32 = reinterpret_cast<uint32_t *>(lat);
    for (int p = 0; p < parities; ++p)
      for (int c = 0; c < 4; ++c) {
        if (fast) sweep_class<KIND, true, true>(H, rec, lat32, tab, c, p, static_cast<uint32_t>(m), c3, lane);
        else if (smallf) sweep_class<KIND, true, false>(H, rec, lat32, tab, c, p, static_cast<uint32_t>(m), c3, lane);
        else sweep_class<KIND, false, false>(H, rec, lat32, tab, c, p, static_cast<uint32_t>(m), c3, lane);
        wave_sync();
      }
  }
  store_lattice(H, lat, rep, lane);
  if (H.flags & kFlagEnergy) slice_energies(H, lat, rep, lane);
  wave_sync();
}

// Persistent kernel: each workgroup repeatedly takes the next work item
// (handle, replica group) from `counter`, stages the handle's site records in
// LDS, and runs one replica per wavefront through sweeps m0..m1-1.
// Dynamic LDS: [rec_cap words][waves x lat_cap u64][waves x tab_cap words].
#ifndef SQA_WAVES_PER_EU
#define SQA_WAVES_PER_EU 1
#endif
__global__ __launch_bounds__(512) __attribute__((amdgpu_waves_per_eu(SQA_WAVES_PER_EU, 8))) void sqa_anneal_kernel(const HandleDev *__restrict__ hds,
                                                         const WorkItem *__restrict__ items, int n_items,
                                                         int *__restrict__ counter, int rec_cap,
                                                         int lat_cap, int tab_cap) {
  extern __shared__ __align__(16) uint32_t smem[];
  __shared__ int s_item;
  const int waves = blockDim.x >> 6;
  const int wave = threadIdx.x >> 6;
  const int lane = threadIdx.x & 63;
  uint32_t *rec = smem;
  uint64_t *lat = reinterpret_cast<uint64_t *>(smem + rec_cap) + static_cast<size_t>(wave) * lat_cap;
  uint32_t *tab = smem + rec_cap + 2 * waves * lat_cap + wave * tab_cap;
  for (;;) {
    if (threadIdx.x == 0) s_item = atomicAdd(counter, 1);
    __syncthreads();
    const int it = __builtin_amdgcn_readfirstlane(s_item);   // uniform: handle fields go to SGPRs
    if (it >= n_items) break;
    const WorkItem wi = items[it];
    const HandleDev &H = hds[wi.handle];      // read in place: uniform fields become scalar loads
    const int rw = (H.kind == kKindME) ? kRecWordsME : kRecWordsLHZ;
    const int nwords = H.n * rw;
    for (int i = threadIdx.x; i < nwords; i += blockDim.x) rec[i] = H.rec[i];
    __syncthreads();
    if (wave < wi.nrep) {
      if (H.kind == kKindME) anneal_replica<kKindME>(H, rec, lat, tab, wi.rep0 + wave, lane);
      else anneal_replica<kKindLHZ>(H, rec, lat, tab, wi.rep0 + wave, lane);
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
// Eq. (4): qbar_i = sign(sum_r s_{i(N-1)+r}) on slice `slice`, tie -> +1, and
// the logical energy of Eq. (1).  One workgroup per replica, thread i <-> chain i.
__global__ void me_majority_kernel(const int8_t *__restrict__ spins, int N, int n_sites, int L, int slice,
                                   const int32_t *__restrict__ J, const int32_t *__restrict__ h,
                                   int8_t *__restrict__ logical, int32_t *__restrict__ energy) {
  __shared__ int8_t q[256];
  __shared__ int32_t part[256];
  const int rep = blockIdx.x;
  const int8_t *s = spins + (static_cast<size_t>(rep) * L + slice) * n_sites;
  for (int i = threadIdx.x; i < N; i += blockDim.x) {
    int sum = 0;
    for (int r = 0; r < N - 1; ++r) sum += s[i * (N - 1) + r];
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

// ------------------------------------------------------ parallel tempering
// Appendix B: `R` replicas of the classical embedded Hamiltonian, replica rho
// at the inverse temperature of its slot.  One workgroup owns a whole ladder.
// LDS word of site d: bit rho = 1 <=> replica rho has spin -1 there.  An item
// is (site of colour c, replica group a = 4 replicas) and uses one Philox call
// (counter (site, a, sweep, PT<<24)).  Flips are applied with an LDS atomic
// XOR, so items of neighbouring replica groups never overwrite each other.
// Energies are kept incrementally (a flip with a = s*f changes E by -2a).
template <int KIND>
__device__ void pt_ladder(const PTDev &P, const uint32_t *rec, uint64_t *lat, const uint32_t *mtab, int32_t *E,
                          int32_t *rep_at, int32_t *slot_of, uint32_t *acc) {
  using S = Site<KIND>;
  const int R = P.R, F = P.F;
  const int width = 2 * F + 1;
  const int tid = threadIdx.x, nth = blockDim.x;
  int RG = 1;
  while (RG * 4 < R) RG <<= 1;      // replica groups, padded to a power of two (divides nth)
  const int a = tid & (RG - 1);     // this thread's replica group never changes
  const bool group_live = 4 * a < R;
  uint32_t *lat32 = reinterpret_cast<uint32_t *>(lat);
  const uint8_t *latb = reinterpret_cast<const uint8_t *>(lat);
  int32_t dE[4] = {0, 0, 0, 0};
  uint32_t phase = 0;
  for (int m = 0; m < P.sweeps; ++m) {
    for (int c = 0; c < 4; ++c) {
      const int lo = P.cls[c];
      const int nc = P.cls[c + 1] - lo;
      const int cnt = nc * RG;
      for (int it = tid; it < cnt; it += nth) {
        if (!group_live) continue;
        const int d = lo + it / RG;
        const uint32_t *r = rec + d * S::RW;
        uint32_t site, base, aw[4], ah, neg;
        uint32_t part[S::T * S::P];
        if constexpr (KIND == kKindME) {
          const uint4 r0 = *reinterpret_cast<const uint4 *>(r);
          site = r0.x & 0xFFFFu; base = r0.x >> 16;
          aw[0] = r0.y & 0xFFu; aw[1] = (r0.y >> 8) & 0xFFu; aw[2] = (r0.y >> 16) & 0xFFu; aw[3] = 0;
          ah = r0.y >> 24;
          neg = r0.z & 0xFFu;
          part[0] = r0.z >> 16; part[1] = r0.w & 0xFFFFu; part[2] = r0.w >> 16;
        } else {
          const uint4 r0 = *reinterpret_cast<const uint4 *>(r);
          const uint4 r1 = *reinterpret_cast<const uint4 *>(r + 4);
          const uint2 r2 = *reinterpret_cast<const uint2 *>(r + 8);
          site = r0.x & 0xFFFFu; base = r0.x >> 16;
          aw[0] = r0.y & 0xFFu; aw[1] = (r0.y >> 8) & 0xFFu; aw[2] = (r0.y >> 16) & 0xFFu; aw[3] = r0.y >> 24;
          ah = r0.z & 0xFFu;
          neg = (r0.z >> 8) & 0xFFu;
          const uint32_t pw[6] = {r1.x, r1.y, r1.z, r1.w, r2.x, r2.y};
#pragma unroll
          for (int q = 0; q < 6; ++q) {
            part[2 * q] = pw[q] & 0xFFFFu;
            part[2 * q + 1] = pw[q] >> 16;
          }
        }
        const int pbase = static_cast<int>((base - 2u) / 3u);   // F_site + F
        const int fsite = pbase - F;
        const int byte = a >> 1, nsh = (a & 1) * 4;
        const uint32_t own = (latb[d * 8 + byte] >> nsh) & 0xFu;
        uint32_t X[S::T];
#pragma unroll
        for (int t = 0; t < S::T; ++t) {
          uint32_t prod = 0;
#pragma unroll
          for (int q = 0; q < S::P; ++q) prod ^= latb[part[S::P * t + q] + byte];
          X[t] = own ^ (prod >> nsh) ^ (0u - ((neg >> t) & 1u));
        }
        const uint32_t O = own ^ (0u - ((neg >> 4) & 1u));
        const Words4 u = philox4x32_10(site, static_cast<uint32_t>(a), static_cast<uint32_t>(m), kStreamPT << 24,
                                       P.seed_lo, P.seed_hi);
        uint32_t flip = 0;
#pragma unroll
        for (int w = 0; w < 4; ++w) {
          const int rho = 4 * a + w;
          if (rho >= R) break;
          uint32_t s = ah * bit_at(O, w);
#pragma unroll
          for (int t = 0; t < S::T; ++t) s += aw[t] * bit_at(X[t], w);
          const int idx = slot_of[rho] * width + pbase - 2 * static_cast<int>(s);
          const uint32_t T = mtab[idx];
          if (min(u.v[w], 0xFFFFFFFEu) < T) {
            flip |= 1u << w;
            dE[w] += 4 * static_cast<int32_t>(s) - 2 * fsite;
          }
        }
        if (flip) atomicXor(&lat32[2 * d + (a >> 3)], flip << (4 * (a & 7)));
      }
      __syncthreads();
    }
    if ((m + 1) % P.sweeps_per_swap == 0) {
      if (group_live)
        for (int w = 0; w < 4; ++w)
          if (dE[w] != 0 && 4 * a + w < R) {
            atomicAdd(&E[4 * a + w], dE[w]);
            dE[w] = 0;
          }
      __syncthreads();
      for (int q = 0; q < 2; ++q) {
        const int r = 2 * tid + q;
        if (r + 1 < R) {
          const int lo_rep = rep_at[r], hi_rep = rep_at[r + 1];
          const int D = E[hi_rep] - E[lo_rep];
          bool ok = D <= 0;
          if (!ok) {
            const Words4 u = philox4x32_10(static_cast<uint32_t>(r), 0u, phase, kStreamSwap << 24, P.seed_lo,
                                           P.seed_hi);
            const uint32_t T = P.stab[static_cast<size_t>(r) * (P.Dmax + 1) + min(D, P.Dmax)];
            ok = min(u.v[0], 0xFFFFFFFEu) < T;
          }
          if (ok) {
            rep_at[r] = hi_rep;
            rep_at[r + 1] = lo_rep;
            slot_of[hi_rep] = r;
            slot_of[lo_rep] = r + 1;
            acc[r] += 1;
          }
        }
        __syncthreads();
      }
      ++phase;
    }
  }
  if (group_live)
    for (int w = 0; w < 4; ++w)
      if (dE[w] != 0 && 4 * a + w < R) atomicAdd(&E[4 * a + w], dE[w]);
  __syncthreads();
}

// Dynamic LDS: [rec_cap words][lat_cap u64][mtab_cap words][E, rep_at, slot_of, acc: 64 each].
__global__ __launch_bounds__(1024) void pt_kernel(const PTDev *__restrict__ pts, int rec_cap, int lat_cap,
                                                 int mtab_cap) {
  extern __shared__ __align__(16) uint32_t smem[];
  const PTDev P = pts[blockIdx.x];
  uint32_t *rec = smem;
  uint64_t *lat = reinterpret_cast<uint64_t *>(smem + rec_cap);
  uint32_t *mtab = smem + rec_cap + 2 * lat_cap;
  int32_t *E = reinterpret_cast<int32_t *>(mtab + mtab_cap);
  int32_t *rep_at = E + 64;
  int32_t *slot_of = rep_at + 64;
  uint32_t *acc = reinterpret_cast<uint32_t *>(slot_of + 64);
  const int tid = threadIdx.x, nth = blockDim.x;
  const int rw = (P.kind == kKindME) ? kRecWordsME : kRecWordsLHZ;
  for (int i = tid; i < P.n * rw; i += nth) rec[i] = P.rec[i];
  const int width = 2 * P.F + 1;
  for (int i = tid; i < P.R * width; i += nth) mtab[i] = P.mtab[i];
  for (int r = tid; r < 64; r += nth) {
    rep_at[r] = r;
    slot_of[r] = r;
    acc[r] = 0;
    E[r] = 0;
  }
  // initial spins from the PT_INIT stream: replica rho, site k -> word rho&3 of (k, rho>>2, 0, PT_INIT<<24)
  const int RG = (P.R + 3) >> 2;
  for (int d = tid; d < P.n; d += nth) {
    const uint32_t site = P.rec[d * rw] & 0xFFFFu;
    uint64_t w = 0;
    for (int a = 0; a < RG; ++a) {
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
  if (P.kind == kKindME) pt_ladder<kKindME>(P, rec, lat, mtab, E, rep_at, slot_of, acc);
  else pt_ladder<kKindLHZ>(P, rec, lat, mtab, E, rep_at, slot_of, acc);
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
hipError_t launch_sqa_anneal(const HandleDev *hds, const WorkItem *items, int n_items, int *counter,
                             int grid, int waves, int rec_cap, int lat_cap, int tab_cap,
                             hipStream_t stream) {
  const size_t lds = (static_cast<size_t>(rec_cap) + 2ull * waves * lat_cap + static_cast<size_t>(waves) * tab_cap) * 4;
  (void)hipGetLastError();
  hipLaunchKernelGGL(reset_counter_kernel, dim3(1), dim3(64), 0, stream, counter);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(sqa_anneal_kernel, dim3(grid), dim3(64 * waves), lds, stream, hds, items, n_items, counter,
                     rec_cap, lat_cap, tab_cap);
  return hipGetLastError();
}

// Resident workgroups of `waves` waves per compute unit for the given dynamic LDS.
int sqa_anneal_occupancy(int waves, size_t lds_bytes) {
  int blocks = 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&blocks, sqa_anneal_kernel, 64 * waves, lds_bytes) != hipSuccess) {
    (void)hipGetLastError();
    return 0;
  }
  return blocks;
}

hipError_t set_sqa_anneal_lds_limit(size_t bytes) {
  return hipFuncSetAttribute(reinterpret_cast<const void *>(sqa_anneal_kernel),
                             hipFuncAttributeMaxDynamicSharedMemorySize, static_cast<int>(bytes));
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

hipError_t launch_me_majority(const int8_t *spins, int R, int N, int n_sites, int L, int slice, const int32_t *J,
                              const int32_t *h, int8_t *logical, int32_t *energy, hipStream_t stream) {
  (void)hipGetLastError();
  hipLaunchKernelGGL(me_majority_kernel, dim3(R), dim3(256), 0, stream, spins, N, n_sites, L, slice, J, h,
                     logical, energy);
  return hipGetLastError();
}

hipError_t launch_pt(const PTDev *pts, int count, int waves, int rec_cap, int lat_cap, int mtab_cap,
                     hipStream_t stream) {
  const size_t lds = (static_cast<size_t>(rec_cap) + 2ull * lat_cap + mtab_cap + 4 * 64) * 4;
  (void)hipGetLastError();
  hipLaunchKernelGGL(pt_kernel, dim3(count), dim3(64 * waves), lds, stream, pts, rec_cap, lat_cap, mtab_cap);
  return hipGetLastError();
}

hipError_t set_pt_lds_limit(size_t bytes) {
  return hipFuncSetAttribute(reinterpret_cast<const void *>(pt_kernel), hipFuncAttributeMaxDynamicSharedMemorySize,
                             static_cast<int>(bytes));
}

}  // namespace sqa
