// gfx950 parallel-tempering kernel (Appendix B, Eqs. (B1)-(B2)): one
// workgroup per temperature ladder, replicas bit-packed per site word.
#include <hip/hip_runtime.h>

#include "device_common.h"

namespace sqa {

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
        uint32_t site, base, aw[S::T], ah, neg;
        uint32_t part[S::T * S::P];
        if constexpr (KIND == kKindMEC) {
          uint32_t w1, w2;
          load_rec_mec(r, site, base, w1, w2, ah, neg, part);
#pragma unroll
          for (int t = 0; t < S::T; ++t) aw[t] = term_weight(w1, w2, t);
        } else if constexpr (KIND == kKindME) {
          const uint4 r0 = *reinterpret_cast<const uint4 *>(r);
          site = r0.x & 0xFFFFu; base = r0.x >> 16;
          aw[0] = r0.y & 0xFFu; aw[1] = (r0.y >> 8) & 0xFFu; aw[2] = (r0.y >> 16) & 0xFFu;
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
        const uint32_t O = own ^ (0u - ((neg >> S::HB) & 1u));
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
  const int rw = rec_words_of(P.kind);
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
  else if (P.kind == kKindLHZ) pt_ladder<kKindLHZ>(P, rec, lat, mtab, E, rep_at, slot_of, acc);
  else pt_ladder<kKindMEC>(P, rec, lat, mtab, E, rep_at, slot_of, acc);
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
