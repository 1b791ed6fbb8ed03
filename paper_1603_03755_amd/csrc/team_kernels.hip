// gfx950 team kernel of the SQA Metropolis moves (Sec. III, Appendix B): one
// replica per workgroup, its waves (up to 8) sharing the replica's lattice in
// LDS and taking a colour class's items together, so that a launch holding few
// replicas in all still spreads each replica's sweep over many lanes.  Same
// moves, random numbers and results as the one-wave-per-replica kernel in
// sqa_kernels.hip (the sweep code is shared through sqa_sweep.h); a kernel of
// its own so that the team path's code does not enter that kernel's register
// allocation.
#include <hip/hip_runtime.h>

#include "sqa_sweep.h"

namespace sqa {

// Persistent: each workgroup repeatedly takes the next work item (handle, one
// replica) from `counter`, stages the handle's site records in LDS, and runs the
// replica through sweeps m0..m1-1 with all its waves.
// Dynamic LDS: [kSpreadWords: byte -> spread table][rec_cap words][one lattice, lat_cap u64]
// [waves x tab_cap words] (each wave's copy of the sweep's table row).
__global__ __launch_bounds__(512) void sqa_team_kernel(const HandleDev *__restrict__ hds,
                                                       const WorkItem *__restrict__ items, int n_items,
                                                       int *__restrict__ counter, int rec_cap, int lat_cap,
                                                       int tab_cap) {
  extern __shared__ __align__(16) uint32_t smem[];
  __shared__ int s_item;
  const int wave = threadIdx.x >> 6;
  const int lane = threadIdx.x & 63;
  uint2 *stab = reinterpret_cast<uint2 *>(smem);
  uint32_t *rec = smem + kSpreadWords;
  uint64_t *lat = reinterpret_cast<uint64_t *>(rec + rec_cap);
  uint32_t *tab = rec + rec_cap + 2 * lat_cap + wave * tab_cap;
  fill_spread_tables(stab);
  const int tid = threadIdx.x, nthr = blockDim.x;
  for (;;) {
    if (threadIdx.x == 0) s_item = atomicAdd(counter, 1);
    __syncthreads();
    const int it = __builtin_amdgcn_readfirstlane(s_item);   // uniform: handle fields go to SGPRs
    if (it >= n_items) break;
    const WorkItem wi = items[it];
    const HandleDev &H = hds[wi.handle];
    const int nwords = H.n * rec_words_of(H.kind);
    for (int i = threadIdx.x; i < nwords; i += blockDim.x) rec[i] = H.rec[i];
    __syncthreads();
    if (nthr == 64) {
      // a one-wave team synchronises as a wave: no workgroup barrier, whose memory fence would wait
      // for the next sweep's table-row load at the first class boundary
      if (H.kind == kKindME) anneal_replica<kKindME>(H, rec, lat, tab, stab, wi.rep0, lane, lane, 64, false);
      else if (H.kind == kKindLHZ) anneal_replica<kKindLHZ>(H, rec, lat, tab, stab, wi.rep0, lane, lane, 64, false);
      else anneal_replica<kKindMEC>(H, rec, lat, tab, stab, wi.rep0, lane, lane, 64, false);
    } else {
      if (H.kind == kKindME) anneal_replica<kKindME>(H, rec, lat, tab, stab, wi.rep0, lane, tid, nthr, true);
      else if (H.kind == kKindLHZ) anneal_replica<kKindLHZ>(H, rec, lat, tab, stab, wi.rep0, lane, tid, nthr, true);
      else anneal_replica<kKindMEC>(H, rec, lat, tab, stab, wi.rep0, lane, tid, nthr, true);
    }
    __syncthreads();
  }
}

hipError_t launch_sqa_team(const HandleDev *hds, const WorkItem *items, int n_items, int *counter, int grid, int waves,
                           int rec_cap, int lat_cap, int tab_cap, size_t lds, hipStream_t stream) {
  (void)hipGetLastError();
  hipLaunchKernelGGL(sqa_team_kernel, dim3(grid), dim3(64 * waves), lds, stream, hds, items, n_items, counter, rec_cap,
                     lat_cap, tab_cap);
  return hipGetLastError();
}

int sqa_team_occupancy(int waves, size_t lds_bytes) {
  int blocks = 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&blocks, sqa_team_kernel, 64 * waves, lds_bytes) != hipSuccess) {
    (void)hipGetLastError();
    return 0;
  }
  return blocks;
}

hipError_t set_sqa_team_lds_limit(size_t bytes) {
  return hipFuncSetAttribute(reinterpret_cast<const void *>(sqa_team_kernel),
                             hipFuncAttributeMaxDynamicSharedMemorySize, static_cast<int>(bytes));
}

}  // namespace sqa
