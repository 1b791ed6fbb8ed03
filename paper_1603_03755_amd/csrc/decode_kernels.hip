// gfx950 decoders of the LHZ scheme (arXiv:1603.03755): spanning-tree majority
// vote (Eq. (5), Appendix A), minimum-weight decoding (Sec. IV A, Eqs. (6)-(10)),
// maximum-likelihood decoding at the Nishimori temperature (Sec. IV B, Eq. (11))
// and weight-3 parity-check decoding (Sec. IV D), plus the logical energy of
// Eq. (1) of every decoded state.
//
// The readout slice of every replica is first packed into N row masks: bit j
// of row i is set iff s_ij = -1 (i != j; bit i clear).  With the logical state
// as a bit vector z (bit i set iff sigma_i = -1, sigma_0 = +1 fixed),
// s_ij sigma_i sigma_j = -1 iff bit j of (row_i ^ z ^ (z_i ? ~0 : 0)) is set,
// so a row's disagreement count is one popcount.
//
// Exhaustive decoders enumerate the 2^(N-1) candidates m (sigma_{b+1} = -1 iff
// bit b of m) in Gray-code order: each lane walks an aligned chunk of 2^c Gray
// indices, so the bit flipped at a step is the same in every lane (the row it
// needs is a wave-uniform read) and the score changes by 4 d - 2 (N - 1), d the
// flipped row's disagreement count.
#include <hip/hip_runtime.h>

#include <cstdint>

namespace sqa {

__device__ __forceinline__ int lhz_site(int N, int i, int j) {
  if (i > j) {
    const int t = i;
    i = j;
    j = t;
  }
  return i * (2 * N - i - 1) / 2 + (j - i - 1);
}

// rows[r][i] from spins [R][L][K] at slice `slice`.  One thread per (replica, i).
__global__ void lhz_rows_kernel(const int8_t *__restrict__ spins, int R, int L, int K, int N, int slice,
                                uint32_t *__restrict__ rows) {
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= R * N) return;
  const int r = t / N, i = t - r * N;
  const int8_t *s = spins + (static_cast<size_t>(r) * L + slice) * K;
  uint32_t m = 0;
  for (int j = 0; j < N; ++j)
    if (j != i && s[lhz_site(N, i, j)] < 0) m |= 1u << j;
  rows[t] = m;
}

// Fill kernels (no memset nodes, so the decoders can sit in a captured graph).
__global__ void fill_u64_kernel(uint64_t *p, size_t n, uint64_t v) {
  const size_t i = static_cast<size_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i < n) p[i] = v;
}

__device__ __forceinline__ int row_disagreements(uint32_t row, uint32_t z, int p, uint32_t maskN) {
  const uint32_t zp = 0u - ((z >> p) & 1u);
  return __popc((row ^ z ^ zp) & maskN);
}

// Score O(z) = sum_{i<j} s_ij sigma_i sigma_j = K - 2 (number of disagreeing pairs).
__device__ __forceinline__ int full_score(const uint32_t *rows, uint32_t z, int N, int K, uint32_t maskN) {
  int bad = 0;
  for (int i = 0; i < N; ++i) {
    const uint32_t above = maskN & ~((2u << i) - 1u);     // bits j > i
    const uint32_t zi = 0u - ((z >> i) & 1u);
    bad += __popc((rows[i] ^ z ^ zi) & above);
  }
  return K - 2 * bad;
}

__device__ __forceinline__ uint64_t wave_max_u64(uint64_t v) {
  for (int off = 32; off > 0; off >>= 1) {
    const uint32_t lo = __shfl_xor(static_cast<uint32_t>(v), off);
    const uint32_t hi = __shfl_xor(static_cast<uint32_t>(v >> 32), off);
    const uint64_t o = (static_cast<uint64_t>(hi) << 32) | lo;
    v = o > v ? o : v;
  }
  return v;
}

__device__ __forceinline__ int64_t wave_sum_i64(int64_t v) {
  for (int off = 32; off > 0; off >>= 1) {
    const uint32_t lo = __shfl_xor(static_cast<uint32_t>(static_cast<uint64_t>(v)), off);
    const uint32_t hi = __shfl_xor(static_cast<uint32_t>(static_cast<uint64_t>(v) >> 32), off);
    v += static_cast<int64_t>((static_cast<uint64_t>(hi) << 32) | lo);
  }
  return v;
}

// Minimum-weight decoding: for replica blockIdx.x, lanes take Gray chunks of
// 2^c indices; best[r] receives max over candidates of the key
// (O + K) << 32 | (0xFFFFFFFF - m): the highest score, then the smallest m
// (one atomic per block after a wave and a block reduction).  best[] must
// start at 0.  Block: 256 threads.
__global__ __launch_bounds__(256) void lhz_mwd_kernel(const uint32_t *__restrict__ rows_all, int N, int c,
                                                      unsigned long long *__restrict__ best) {
  __shared__ uint32_t rows[32];
  const int r = blockIdx.x;
  if (threadIdx.x < N) rows[threadIdx.x] = rows_all[static_cast<size_t>(r) * N + threadIdx.x];
  __syncthreads();
  const int K = N * (N - 1) / 2;
  const uint32_t maskN = (N == 32) ? ~0u : ((1u << N) - 1u);
  const uint64_t total = 1ull << (N - 1);
  const uint64_t chunk = 1ull << c;
  const uint64_t g0 = (static_cast<uint64_t>(blockIdx.y) * blockDim.x + threadIdx.x) * chunk;
  uint64_t key = 0;
  if (g0 < total) {
    const uint32_t m0 = static_cast<uint32_t>(g0 ^ (g0 >> 1));
    uint32_t z = m0 << 1;
    // Within a chunk (aligned, 2^c candidates) the bits of m from c up stay those of m0, so the
    // chunk's candidates compare by the 32-bit key (bad << (c + 1)) | (z mod 2^(c+1)), smallest
    // first (z = 2 m): bad = (K - O) / 2 <= 496 disagreeing pairs, c <= 22.
    const uint32_t lowz = (2u << c) - 2u;
    const int sb = c + 1;
    int bsh = ((K - full_score(rows, z, N, K, maskN)) >> 1) << sb;     // bad << (c + 1)
    uint32_t kmin = static_cast<uint32_t>(bsh) | (z & lowz);
    const int cst = (N - 1) << sb, dsc = -(4 << c);
    // step t of the chunk flips logical bit b = ctz(t) < c (spin p = b + 1): every pair (p, j)
    // changes sign, so bad gains the N - 1 - d pairs that agreed and loses the d that did not
    auto step = [&](uint32_t row, int p) {
      const int d = row_disagreements(row, z, p, maskN);
      bsh = __mul24(d, dsc) + (bsh + cst);
      z ^= 1u << p;
      const uint32_t k = static_cast<uint32_t>(bsh) | (z & lowz);
      kmin = k < kmin ? k : kmin;
    };
    if (chunk >= 8) {
      // eight steps at a time: t = u + 1 .. u + 7 flip bits 0, 1, 0, 2, 0, 1, 0 (rows 1..3
      // in registers), t = u (u > 0) bit ctz(u) >= 3, the same in every lane (chunks are aligned)
      const uint32_t r1 = rows[1], r2 = rows[2], r3 = rows[3];
      for (uint64_t u = 0; u < chunk; u += 8) {
        if (u) {
          const int p = __builtin_ctzll(u) + 1;
          step(rows[p], p);
        }
        step(r1, 1);
        step(r2, 2);
        step(r1, 1);
        step(r3, 3);
        step(r1, 1);
        step(r2, 2);
        step(r1, 1);
      }
    } else {
      for (uint64_t t = 1; t < chunk; ++t) {
        const int p = __builtin_ctzll(t) + 1;
        step(rows[p], p);
      }
    }
    // the chunk's best as the global key (O + K) << 32 | (0xFFFFFFFF - m)
    const uint32_t mb = (m0 & ~(lowz >> 1)) | ((kmin & lowz) >> 1);
    const uint32_t okb = 2u * (static_cast<uint32_t>(K) - (kmin >> sb));  // O + K, O = K - 2 bad
    key = (static_cast<uint64_t>(okb) << 32) | (0xFFFFFFFFu - mb);
  }
  key = wave_max_u64(key);
  __shared__ uint64_t wbest[4];
  if ((threadIdx.x & 63) == 0) wbest[threadIdx.x >> 6] = key;
  __syncthreads();
  if (threadIdx.x == 0) {
    uint64_t k = wbest[0];
    for (int w = 1; w < static_cast<int>(blockDim.x >> 6); ++w) k = wbest[w] > k ? wbest[w] : k;
    atomicMax(best + r, static_cast<unsigned long long>(k));
  }
}

// Maximum-likelihood decoding: with O_max from the MWD keys, every candidate's
// weight wtab[O_max - O] (round(2^36 exp(-beta_N d)), built on the host) is
// summed into W, and the weight of the states with sigma_i = -1 into S_i by
// interval bookkeeping: when bit i turns on, S_i -= W so far; when it turns
// off, S_i += W so far; bits still on at the end add the final W.  Then
// acc[r][0] += W and acc[r][i] += W - 2 S_i (integer, order independent).
// Block: 64 threads (one wave); dynamic LDS: N x 64 int64 for S.
__global__ __launch_bounds__(64) void lhz_mld_kernel(const uint32_t *__restrict__ rows_all, int N, int c,
                                                     const unsigned long long *__restrict__ best,
                                                     const uint64_t *__restrict__ wtab_g, int wlen,
                                                     unsigned long long *__restrict__ acc) {
  extern __shared__ int64_t sacc[];              // [N][64]
  __shared__ uint32_t rows[32];
  __shared__ uint64_t wtab[1024];
  const int r = blockIdx.x;
  const int lane = threadIdx.x;
  if (lane < N) rows[lane] = rows_all[static_cast<size_t>(r) * N + lane];
  for (int i = lane; i < wlen; i += 64) wtab[i] = wtab_g[i];
  for (int i = 0; i < N; ++i) sacc[i * 64 + lane] = 0;
  __syncthreads();
  const int K = N * (N - 1) / 2;
  const int omax = static_cast<int>(best[r] >> 32) - K;
  const uint32_t maskN = (N == 32) ? ~0u : ((1u << N) - 1u);
  const uint64_t total = 1ull << (N - 1);
  const uint64_t chunk = 1ull << c;
  const uint64_t g0 = (static_cast<uint64_t>(blockIdx.y) * 64 + lane) * chunk;
  int64_t W = 0;
  uint32_t z = 0;
  if (g0 < total) {
    const uint32_t m = static_cast<uint32_t>(g0 ^ (g0 >> 1));
    z = m << 1;
    int o = full_score(rows, z, N, K, maskN);
    W = static_cast<int64_t>(wtab[omax - o]);
    // step t of the chunk flips spin p = ctz(t) + 1; its interval sum opens (bit turned on) or
    // closes (off) at the total W of the states before this one
    auto step = [&](uint32_t row, int p, int64_t &sp) {
      const int d = row_disagreements(row, z, p, maskN);
      o += 4 * d - 2 * (N - 1);
      z ^= 1u << p;
      sp += ((z >> p) & 1u) ? -W : W;
      W += static_cast<int64_t>(wtab[omax - o]);
    };
    if (chunk >= 8) {
      // eight steps at a time, as in the MWD walk: spins 1..3 (seven of every eight steps) keep
      // their rows and interval sums in registers, the eighth step's in LDS
      const uint32_t r1 = rows[1], r2 = rows[2], r3 = rows[3];
      int64_t s1 = 0, s2 = 0, s3 = 0;
      for (uint64_t u = 0; u < chunk; u += 8) {
        if (u) {
          const int p = __builtin_ctzll(u) + 1;
          step(rows[p], p, sacc[p * 64 + lane]);
        }
        step(r1, 1, s1);
        step(r2, 2, s2);
        step(r1, 1, s1);
        step(r3, 3, s3);
        step(r1, 1, s1);
        step(r2, 2, s2);
        step(r1, 1, s1);
      }
      sacc[64 + lane] += s1;
      sacc[128 + lane] += s2;
      sacc[192 + lane] += s3;
    } else {
      for (uint64_t t = 1; t < chunk; ++t) {
        const int p = __builtin_ctzll(t) + 1;
        step(rows[p], p, sacc[p * 64 + lane]);
      }
    }
  }
  // close the intervals of bits still on; S_i -> W - 2 S_i
  for (int i = 0; i < N; ++i) {
    int64_t s = sacc[i * 64 + lane];
    if ((z >> i) & 1u) s += W;
    const int64_t v = wave_sum_i64(i == 0 ? W : W - 2 * s);
    if (lane == 0) atomicAdd(acc + static_cast<size_t>(r) * N + i, static_cast<unsigned long long>(v));
  }
}

// Weight-3 parity-check decoding: one wave per replica, lane i owns row i.
// x starts at s; each round, for every pair (i, j),
//   c = sum_{l != i,j} x_il x_lj = (N - 2) - 2 popcount((X_i ^ X_j) & ~bits{i, j}),
// and the new x_ij = dec[(s_ij < 0) * (2N - 3) + c + N - 2] (host table).
// The final values go to pairs[r][K] (LHZ site order) as +1/-1.
__global__ __launch_bounds__(64) void lhz_bp_kernel(const uint32_t *__restrict__ rows_all, int N, int iterations,
                                                    const int8_t *__restrict__ dec, int8_t *__restrict__ pairs) {
  __shared__ uint32_t xa[32], xb[32];
  const int r = blockIdx.x;
  const int i = threadIdx.x;
  const uint32_t maskN = (N == 32) ? ~0u : ((1u << N) - 1u);
  const int width = 2 * N - 3;
  uint32_t srow = 0;
  if (i < N) {
    srow = rows_all[static_cast<size_t>(r) * N + i];
    xa[i] = srow;
  }
  __syncthreads();
  uint32_t *cur = xa, *nxt = xb;
  for (int it = 0; it < iterations; ++it) {
    if (i < N) {
      const uint32_t xi = cur[i];
      uint32_t row = 0;
      for (int j = 0; j < N; ++j) {
        if (j == i) continue;
        const uint32_t others = maskN & ~(1u << i) & ~(1u << j);
        const int c = (N - 2) - 2 * __popc((xi ^ cur[j]) & others);
        const int neg = (srow >> j) & 1u;
        if (dec[neg * width + c + N - 2] < 0) row |= 1u << j;
      }
      nxt[i] = row;
    }
    __syncthreads();
    uint32_t *t = cur;
    cur = nxt;
    nxt = t;
  }
  if (i < N) {
    const int K = N * (N - 1) / 2;
    for (int j = i + 1; j < N; ++j)
      pairs[static_cast<size_t>(r) * K + lhz_site(N, i, j)] = ((cur[i] >> j) & 1u) ? int8_t(-1) : int8_t(1);
  }
}

// Spanning-tree majority vote (Eq. (5)): one workgroup of 64 per replica.
// Pair values x are read from pairs + r * stride (LHZ site order).  `order`
// lists, per tree, the vertices so that every parent precedes its children
// (root 0 first); qbar_0 = +1, qbar_v = qbar_parent * x(v, parent); majority
// over the trees, tie -> +1.  N <= 256.
__global__ __launch_bounds__(64) void lhz_tree_kernel(const int8_t *__restrict__ pairs, size_t stride, int N,
                                                      const int32_t *__restrict__ parents,
                                                      const int32_t *__restrict__ order, int n_trees,
                                                      int8_t *__restrict__ logical) {
  __shared__ int8_t q[256];
  __shared__ int32_t votes[256];
  const int r = blockIdx.x;
  const int8_t *x = pairs + static_cast<size_t>(r) * stride;
  for (int v = threadIdx.x; v < N; v += 64) votes[v] = 0;
  for (int t = 0; t < n_trees; ++t) {
    if (threadIdx.x == 0) {
      const int32_t *par = parents + static_cast<size_t>(t) * N;
      const int32_t *ord = order + static_cast<size_t>(t) * N;
      q[0] = 1;
      for (int k = 1; k < N; ++k) {
        const int v = ord[k], p = par[v];
        q[v] = static_cast<int8_t>(q[p] * x[lhz_site(N, v, p)]);
      }
    }
    __syncthreads();
    for (int v = threadIdx.x; v < N; v += 64) votes[v] += q[v];
    __syncthreads();
  }
  for (int v = threadIdx.x; v < N; v += 64)
    logical[static_cast<size_t>(r) * N + v] = votes[v] >= 0 ? int8_t(1) : int8_t(-1);
}

// Logical states from MWD keys or MLD sums; one thread per (replica, i).
__global__ void mwd_logical_kernel(const unsigned long long *__restrict__ best, int R, int N,
                                   int8_t *__restrict__ logical) {
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= R * N) return;
  const int r = t / N, i = t - r * N;
  const uint32_t m = 0xFFFFFFFFu - static_cast<uint32_t>(best[r]);
  logical[t] = (i > 0 && ((m >> (i - 1)) & 1u)) ? int8_t(-1) : int8_t(1);
}

__global__ void mld_logical_kernel(const unsigned long long *__restrict__ acc, int R, int N,
                                   int8_t *__restrict__ logical) {
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= R * N) return;
  logical[t] = static_cast<int64_t>(acc[t]) >= 0 ? int8_t(1) : int8_t(-1);
}

// Eq. (1) energy of each decoded logical state; one workgroup of 64 per replica.
__global__ __launch_bounds__(64) void logical_energy_kernel(const int8_t *__restrict__ logical, int N,
                                                            const int32_t *__restrict__ J,
                                                            const int32_t *__restrict__ h,
                                                            int32_t *__restrict__ energy) {
  const int r = blockIdx.x;
  const int8_t *q = logical + static_cast<size_t>(r) * N;
  int32_t e = 0;
  for (int i = threadIdx.x; i < N; i += 64) {
    if (h) e += h[i] * q[i];
    for (int j = i + 1; j < N; ++j) e += J[i * N + j] * q[i] * q[j];
  }
  for (int off = 32; off > 0; off >>= 1) e += __shfl_xor(e, off);
  if (threadIdx.x == 0) energy[r] = e;
}


// Exact ground state of Eq. (1) for integer J, h (n <= 32, |J|, |h| < 2^15):
// exhaustive search over sigma_0 = +1 (candidate m: sigma_{b+1} = -1 iff bit b
// of m) in Gray-code chunks, each candidate also taken with all spins flipped.
// With E_J = sum_{i<j} J_ij s_i s_j and E_h = sum_i h_i s_i, the better of the
// pair has energy E_J - |E_h|.  Flipping spin p changes E_J by -2 s_p g_p,
// g_p = sum_j J_pj s_j, and E_h by -2 s_p h_p; g_p is rebuilt from bit planes
// of |J|: pos[b][p] / neg[b][p] mark the j with J_pj > 0 / < 0 and bit b of
// |J_pj| set, so g_p = c_p - 2 sum_b 2^b (popc(pos & z) - popc(neg & z)) with
// c_p = sum_j J_pj and z the bit vector of the -1 spins.
// best: min over candidates of ((E + 2^31) << 32) | (m << 1 | flipped).
__global__ __launch_bounds__(256) void ground_kernel(const uint32_t *__restrict__ planes, const int32_t *__restrict__ cj,
                                                     const int32_t *__restrict__ hv, int N, int B, int c,
                                                     unsigned long long *__restrict__ best) {
  __shared__ uint32_t pos[16][32], neg[16][32];
  __shared__ int32_t cp[32], hp[32];
  for (int i = threadIdx.x; i < B * N; i += blockDim.x) {
    const int b = i / N, p = i - b * N;
    pos[b][p] = planes[(2 * b) * N + p];
    neg[b][p] = planes[(2 * b + 1) * N + p];
  }
  if (threadIdx.x < N) {
    cp[threadIdx.x] = cj[threadIdx.x];
    hp[threadIdx.x] = hv[threadIdx.x];
  }
  __syncthreads();
  const uint64_t total = 1ull << (N - 1);
  const uint64_t chunk = 1ull << c;
  const uint64_t g0 = (static_cast<uint64_t>(blockIdx.x) * blockDim.x + threadIdx.x) * chunk;
  uint64_t key = ~0ull;
  if (g0 < total) {
    uint32_t m = static_cast<uint32_t>(g0 ^ (g0 >> 1));
    uint32_t z = m << 1;
    // energies of the chunk's first candidate, from scratch
    int ej = 0, eh = 0;
    for (int p = 0; p < N; ++p) {
      const int sp = ((z >> p) & 1u) ? -1 : 1;
      int g = cp[p];
      for (int b = 0; b < B; ++b) g -= (2 << b) * (__popc(pos[b][p] & z) - __popc(neg[b][p] & z));
      ej += sp * g;                        // counts every pair twice
      eh += sp * hp[p];
    }
    ej /= 2;
    auto make_key = [&](int e, uint32_t mm, uint32_t fl) {
      return (static_cast<uint64_t>(static_cast<uint32_t>(e) ^ 0x80000000u) << 32) | (mm << 1) | fl;
    };
    {
      const int e = ej - (eh > 0 ? eh : -eh);
      key = make_key(e, m, eh > 0 ? 1u : 0u);
    }
    for (uint64_t t = 1; t < chunk; ++t) {
      const int bflip = __builtin_ctzll(t);
      const int p = bflip + 1;
      const int sp = ((z >> p) & 1u) ? -1 : 1;
      int g = cp[p];
      for (int b = 0; b < B; ++b) g -= (2 << b) * (__popc(pos[b][p] & z) - __popc(neg[b][p] & z));
      ej -= 2 * sp * g;
      eh -= 2 * sp * hp[p];
      z ^= 1u << p;
      m ^= 1u << bflip;
      const int e = ej - (eh > 0 ? eh : -eh);
      const uint64_t k = make_key(e, m, eh > 0 ? 1u : 0u);
      key = k < key ? k : key;
    }
  }
  for (int off = 32; off > 0; off >>= 1) {
    const uint32_t lo = __shfl_xor(static_cast<uint32_t>(key), off);
    const uint32_t hi = __shfl_xor(static_cast<uint32_t>(key >> 32), off);
    const uint64_t o = (static_cast<uint64_t>(hi) << 32) | lo;
    key = o < key ? o : key;
  }
  if ((threadIdx.x & 63) == 0) atomicMin(best, static_cast<unsigned long long>(key));
}

// ----------------------------------------------------------- host launchers
static unsigned blocks_for(size_t n, unsigned b) { return static_cast<unsigned>((n + b - 1) / b); }

// Gray chunk exponent: 2^c candidates per lane, c <= N - 1.
static int chunk_exponent(int N) { return (N - 1) < 12 ? (N - 1) : 12; }
// MWD walks chunks of 2^6 candidates per lane up to N = 20 (short serial walks, many lanes for
// small N) and of 2^10 from N = 21 on, so that a lane's setup (the full score of its first
// candidate) and its block's reduction amortise over its walk: N = 30 with 16 replicas took
// 3.48 ms with 2^6-chunks and 1.77 ms with 2^10.  The grid's y dimension, 2^(N-1-c) / 256
// blocks per replica, stays within its limit up to N = 32.
static int mwd_chunk_exponent(int N) {
  const int c = (N <= 20) ? 6 : ((N - 22) > 10 ? (N - 22) : 10);
  return (N - 1) < c ? (N - 1) : c;
}

hipError_t launch_lhz_rows(const int8_t *spins, int R, int L, int K, int N, int slice, uint32_t *rows,
                           hipStream_t s) {
  (void)hipGetLastError();
  hipLaunchKernelGGL(lhz_rows_kernel, dim3(blocks_for(static_cast<size_t>(R) * N, 256)), dim3(256), 0, s, spins, R, L,
                     K, N, slice, rows);
  return hipGetLastError();
}

hipError_t launch_lhz_mwd(const uint32_t *rows, int R, int N, unsigned long long *best, int8_t *logical,
                          hipStream_t s) {
  (void)hipGetLastError();
  hipLaunchKernelGGL(fill_u64_kernel, dim3(blocks_for(R, 256)), dim3(256), 0, s, reinterpret_cast<uint64_t *>(best),
                     static_cast<size_t>(R), uint64_t(0));
  const int c = mwd_chunk_exponent(N);
  const uint64_t lanes = (1ull << (N - 1)) >> c;
  hipLaunchKernelGGL(lhz_mwd_kernel, dim3(R, blocks_for(lanes, 256)), dim3(256), 0, s, rows, N, c, best);
  if (logical)
    hipLaunchKernelGGL(mwd_logical_kernel, dim3(blocks_for(static_cast<size_t>(R) * N, 256)), dim3(256), 0, s, best,
                       R, N, logical);
  return hipGetLastError();
}

hipError_t launch_lhz_mld(const uint32_t *rows, int R, int N, unsigned long long *best, const uint64_t *wtab,
                          int wlen, unsigned long long *acc, int8_t *logical, hipStream_t s) {
  hipError_t e = launch_lhz_mwd(rows, R, N, best, nullptr, s);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(fill_u64_kernel, dim3(blocks_for(static_cast<size_t>(R) * N, 256)), dim3(256), 0, s,
                     reinterpret_cast<uint64_t *>(acc), static_cast<size_t>(R) * N, uint64_t(0));
  const int c = chunk_exponent(N);
  const uint64_t lanes = (1ull << (N - 1)) >> c;
  hipLaunchKernelGGL(lhz_mld_kernel, dim3(R, blocks_for(lanes, 64)), dim3(64), sizeof(int64_t) * 64 * N, s, rows, N,
                     c, best, wtab, wlen, acc);
  hipLaunchKernelGGL(mld_logical_kernel, dim3(blocks_for(static_cast<size_t>(R) * N, 256)), dim3(256), 0, s, acc, R, N,
                     logical);
  return hipGetLastError();
}

hipError_t launch_lhz_bp(const uint32_t *rows, int R, int N, int iterations, const int8_t *dec, int8_t *pairs,
                         hipStream_t s) {
  (void)hipGetLastError();
  hipLaunchKernelGGL(lhz_bp_kernel, dim3(R), dim3(64), 0, s, rows, N, iterations, dec, pairs);
  return hipGetLastError();
}

hipError_t launch_lhz_trees(const int8_t *pairs, size_t stride, int R, int N, const int32_t *parents,
                            const int32_t *order, int n_trees, int8_t *logical, hipStream_t s) {
  (void)hipGetLastError();
  hipLaunchKernelGGL(lhz_tree_kernel, dim3(R), dim3(64), 0, s, pairs, stride, N, parents, order, n_trees, logical);
  return hipGetLastError();
}

hipError_t launch_logical_energy(const int8_t *logical, int R, int N, const int32_t *J, const int32_t *h,
                                 int32_t *energy, hipStream_t s) {
  (void)hipGetLastError();
  hipLaunchKernelGGL(logical_energy_kernel, dim3(R), dim3(64), 0, s, logical, N, J, h, energy);
  return hipGetLastError();
}

hipError_t launch_ground(const uint32_t *planes, const int32_t *cj, const int32_t *hv, int N, int B,
                         unsigned long long *best, hipStream_t s) {
  (void)hipGetLastError();
  hipLaunchKernelGGL(fill_u64_kernel, dim3(1), dim3(64), 0, s, reinterpret_cast<uint64_t *>(best), size_t(1), ~uint64_t(0));
  const int c = chunk_exponent(N);
  const uint64_t lanes = (1ull << (N - 1)) >> c;
  hipLaunchKernelGGL(ground_kernel, dim3(blocks_for(lanes, 256)), dim3(256), 0, s, planes, cj, hv, N, B, c, best);
  return hipGetLastError();
}

}  // namespace sqa
