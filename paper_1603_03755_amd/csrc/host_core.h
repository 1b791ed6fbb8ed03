// Host-side pieces of the library shared between its translation units:
// embedding construction, device-order site records, acceptance tables,
// error reporting and the handle structures.
#pragma once
#include <hip/hip_runtime.h>

#include <cstdint>
#include <string>
#include <vector>

#include "../../include/sqa.h"
#include "device_types.h"
#include "pt_types.h"

namespace sqa {

// ------------------------------------------------------------- errors
void set_error(const std::string &msg);
sqa_status fail(sqa_status st, const std::string &msg);
sqa_status hip_fail(hipError_t e, const char *what);

// -------------------------------------------------------- embeddings
// One k-body term (k = 2..4) of the physical Hamiltonian.
struct Term {
  int32_t w;
  int32_t arity;
  int32_t s[4];
};

// Physical Hamiltonian of an embedded problem (Sec. II A / II B).
struct Embedded {
  int32_t kind = 0, N = 0, n = 0;
  std::vector<int32_t> h;        // [n] fields
  std::vector<int32_t> colour;   // [n] 0..3
  std::vector<Term> terms;
  int32_t fmax = 0;              // max_k |h_k| + sum_{t ni k} |w_t|
  int32_t emax = 0;              // sum |h| + sum |w|
};

sqa_status build_embedding(const sqa_problem &p, const sqa_embedding &e, Embedded *out);

// Device-ready form: colour-sorted order, packed records, terms in device indices.
struct DeviceLayout {
  int32_t rec_words = 0;                 // per site
  std::vector<uint32_t> rec;             // [n][rec_words]
  std::vector<uint16_t> dev_of;          // [n] physical -> device
  std::vector<int32_t> phys_of;          // [n] device -> physical
  std::vector<int32_t> hfield;           // [n] device order
  std::vector<int32_t> term_w;           // [n_terms]
  std::vector<uint32_t> term_s;          // [n_terms][2]
  int32_t cls[5] = {0, 0, 0, 0, 0};
};

// Record layouts (the word layouts are documented with the kernel structures):
// kLayoutPlain: byte weights and sign masks (PT; SQA records whose kernel path
// takes them); kLayoutMetropolis: the signed-weight small-field layout when
// F <= kSmallF, else plain; kLayoutWolff: the signed-weight layout of the
// Wolff bond phase when F <= kMidF, else plain; kLayoutPT: the signed-weight
// layout of the PT kernel's byte mode when F <= kPTByteF, else plain.
enum RecordLayout { kLayoutPlain = 0, kLayoutMetropolis = 1, kLayoutWolff = 2, kLayoutPT = 3 };
sqa_status build_layout(const Embedded &emb, int32_t F, RecordLayout layout, DeviceLayout *out);

// ---------------------------------------------------------- tables
uint32_t threshold_from_log(double x);
std::vector<double> linear_gamma(double g0, double g1, int32_t M);
// T[m][a+F][(b+2)/2]
std::vector<uint32_t> sqa_threshold_table(double beta, int32_t L, const std::vector<double> &gamma,
                                          const std::vector<double> *bscale, int32_t F);
// Wolff moves (Sec. III): join thresholds of aligned ring bonds, p = 1 - tanh(beta Gamma_m / L),
// per sweep; acceptance thresholds of a cluster with sum s f = A, exp(2 beta B / L A), indexed
// [row][A + L F] with one row per sweep when B varies, else one row.
std::vector<uint32_t> wolff_join_table(double beta, int32_t L, const std::vector<double> &gamma);
std::vector<uint32_t> wolff_accept_table(double beta, int32_t L, const std::vector<double> *bscale, int32_t F,
                                         int32_t *rows);
std::vector<double> pt_betas(double beta_min, double beta_max, int32_t R);
std::vector<uint32_t> pt_metropolis_table(const std::vector<double> &betas, int32_t F);
std::vector<uint32_t> pt_swap_table(const std::vector<double> &betas, int32_t Dmax);
// Swap table without the trailing zeros of each pair's row: words 0..R-1 hold
// the offsets (within the packed array) of rows 0..R-2 and the end, then the rows.
std::vector<uint32_t> pt_swap_pack(const std::vector<uint32_t> &stab, int32_t R, int32_t Dmax);

// ---------------------------------------------------------- host Philox
void host_philox4x32(const uint32_t ctr[4], uint32_t k0, uint32_t k1, uint32_t out[4]);

// ------------------------------------------------------ device memory
// Device memory from a caller's allocator (sqa_allocator with both callbacks
// set) or, for a null allocator, hipMalloc / hipFree.  device_alloc returns
// SQA_ERR_OOM when the allocator returns NULL or hipMalloc runs out.
sqa_status device_alloc(const sqa_allocator *a, void **p, size_t bytes, const char *what);
void device_free(const sqa_allocator *a, void *p);
// Granularity in which the server counts a job's device bytes.
constexpr size_t kServerGranule = 4096;
inline size_t round_granule(size_t b) { return (b + kServerGranule - 1) & ~(kServerGranule - 1); }

// --------------------------------------------------------- device arena
// One device allocation carved into aligned sub-buffers.
struct Arena {
  void *base = nullptr;
  size_t size = 0;
  size_t used = 0;
  size_t take(size_t bytes) {
    size_t off = (used + 255) & ~size_t(255);
    used = off + bytes;
    return off;
  }
  template <class T>
  T *at(size_t off) const { return reinterpret_cast<T *>(static_cast<char *>(base) + off); }
};

// Kernel launchers (sqa_kernels.hip, which hands team-mode launches to
// team_kernels.hip; pt_kernels.hip; decode_kernels.hip).
hipError_t launch_sqa_anneal(int move, const HandleDev *hds, const WorkItem *items, int n_items, int *counter, int grid,
                             int waves, int rec_cap, int lat_cap, int tab_cap, bool team, hipStream_t stream);
hipError_t set_sqa_anneal_lds_limit(size_t bytes);
int sqa_anneal_occupancy(int move, int waves, size_t lds_bytes, bool team);
hipError_t launch_sqa_init(const HandleDev &H, hipStream_t stream);
hipError_t launch_me_majority(const int8_t *spins, int R, int N, int len, int n_sites, int L, int slice,
                              const int32_t *J, const int32_t *h, int8_t *logical, int32_t *energy,
                              hipStream_t stream);
hipError_t launch_lhz_rows(const int8_t *spins, int R, int L, int K, int N, int slice, uint32_t *rows, hipStream_t s);
hipError_t launch_lhz_mwd(const uint32_t *rows, int R, int N, unsigned long long *best, int8_t *logical,
                          hipStream_t s);
hipError_t launch_lhz_mld(const uint32_t *rows, int R, int N, unsigned long long *best, const uint64_t *wtab,
                          int wlen, unsigned long long *acc, int8_t *logical, hipStream_t s);
hipError_t launch_lhz_bp(const uint32_t *rows, int R, int N, int iterations, const int8_t *dec, int8_t *pairs,
                         hipStream_t s);
hipError_t launch_lhz_trees(const int8_t *pairs, size_t stride, int R, int N, const int32_t *parents,
                            const int32_t *order, int n_trees, int8_t *logical, hipStream_t s);
hipError_t launch_ground(const uint32_t *planes, const int32_t *cj, const int32_t *hv, int N, int B,
                         unsigned long long *best, hipStream_t s);
hipError_t launch_logical_energy(const int8_t *logical, int R, int N, const int32_t *J, const int32_t *h,
                                 int32_t *energy, hipStream_t s);
hipError_t launch_pt(const PTDev *pts, int count, int waves, int rec_cap, int lat_cap, int mtab_cap, int spack_cap,
                     hipStream_t stream);
hipError_t set_pt_lds_limit(size_t bytes);

// Size of the file-scope launch scratch of sqa_anneal_batch_noalloc (per GPU),
// and the current device's address of it (looked up once per device).
constexpr size_t kNoAllocScratchBytes = size_t(4) << 20;
sqa_status noalloc_scratch(void **ptr_out);

// hipErrorLaunchFailure when the environment asks for injected launch faults
// (SQA_FAULT_INJECT=launch), else hipSuccess.
hipError_t injected_launch_fault();

// LDS budget of one workgroup on gfx950 (160 KiB, less room for the kernels'
// static LDS variables).
constexpr size_t kMaxLds = 160 * 1024 - 512;

// Launch geometry for a set of handles.
struct LaunchShape {
  int move = kMoveMetropolis;
  int waves = 4;
  int grid = 0;
  int rec_cap = 0, lat_cap = 0, tab_cap = 0;
  bool team = false;   // Metropolis: the workgroup's waves run one replica together
  size_t lds_bytes() const {
    const int lattices = team ? 1 : waves;
    return (static_cast<size_t>(kSpreadWords) + rec_cap + 2ull * lattices * lat_cap +
            static_cast<size_t>(waves) * tab_cap) * 4;
  }
};

// Team mode for a Metropolis launch: when the handles hold few replicas in all
// (at most kTeamMaxReplicas), one wave per replica leaves most of the GPU idle
// and a replica's anneal time is the launch's latency, so each workgroup runs a
// single replica with enough waves (up to 8) that a colour class takes about
// one pass.
constexpr int kTeamMaxReplicas = 1024;

int device_cu_count();
int occupancy_groups_per_cu(const LaunchShape &s);

}  // namespace sqa

struct sqa_handle;

namespace sqa {
// One persistent launch over several handles, each advancing sweeps
// [m0[i], m1[i]) with its own flags.  `scratch` is a device buffer owned by the
// caller, taken from `alloc` and grown on demand.  Blocks until the launch has
// finished.
sqa_status run_handles(const std::vector<sqa_handle *> &hs, const std::vector<int> &m0, const std::vector<int> &m1,
                       const std::vector<int> &flags, hipStream_t stream, const sqa_allocator *alloc, void **scratch,
                       size_t *scratch_bytes);
// Bytes of the launch scratch of run_handles for a set of handles: at most
// kLaunchScratchFixed plus launch_scratch_share() of each handle.
constexpr size_t kLaunchScratchFixed = 4096;
size_t launch_scratch_share(const sqa_handle *h);
size_t launch_scratch_bytes(const std::vector<sqa_handle *> &hs);

// A handle in two steps: prepare (host only: validation, embedding, layout,
// tables, the sizes of its device block) and upload (device block from the
// allocator, site data and tables copied in, event).  The pinned staging of
// single-handle launches is taken at the first such launch.
sqa_status handle_prepare(const sqa_problem &problem, const sqa_embedding &embedding, const sqa_schedule &schedule,
                          sqa_handle **out);
sqa_status handle_upload(sqa_handle *h, const sqa_allocator *alloc);
// Bytes of the handle's device block, and of the scratch its decoder needs
// (`tree_entries` = n_trees * n for the tree decoders).
size_t handle_block_bytes(const sqa_handle *h);
size_t decode_scratch_bytes(const sqa_handle *h, int decoder, size_t tree_entries);

// A decoder in three steps: check it against the handle (and order the trees'
// vertices), copy its host tables into a scratch laid out for it (synchronous),
// and queue its kernels (kernels only, so a graph can hold them).
sqa_status decode_check(const sqa_handle *h, const sqa_decode_params &p, std::vector<int32_t> *order);
sqa_status decode_tables(const sqa_handle *h, const sqa_decode_params &p, const std::vector<int32_t> &order, char *base);
hipError_t decode_enqueue(const sqa_handle *h, const sqa_decode_params &p, size_t tree_entries, char *base,
                          hipStream_t s);
}  // namespace sqa

// Handle: one problem x embedding x schedule, its device buffers and state.
struct sqa_handle {
  sqa::Embedded emb;
  sqa::DeviceLayout lay;
  int32_t N = 0, L = 0, M = 0, R = 0, F = 0, tw = 0;
  int32_t move = 0;                  // kMoveMetropolis or kMoveWolff
  int32_t wrows = 0, wwidth = 0;     // Wolff acceptance table shape
  std::vector<uint32_t> wacc;        // Wolff acceptance table, host copy
  double beta = 0;
  uint64_t seed = 0;
  std::vector<int32_t> J, h;         // logical problem (n*n, n)
  bool has_h = false;
  std::vector<uint32_t> table;       // per-sweep table, host copy (Metropolis T[m][a][b]; Wolff join thresholds)
  sqa::Arena arena;
  size_t off_rec = 0, off_devof = 0, off_hfield = 0, off_tw = 0, off_ts = 0, off_table = 0, off_spins = 0,
         off_energy = 0, off_wacc = 0, off_J = 0, off_h = 0, off_logical = 0, off_lenergy = 0, off_hd = 0, off_items = 0,
         off_counter = 0;
  sqa_allocator alloc{};             // device-memory provider (null callbacks: hipMalloc)
  bool initialised = false;          // device lattice holds a state
  bool poisoned = false;
  hipEvent_t done = nullptr;
  size_t device_bytes = 0;
  // pinned staging of the single-handle launch descriptor: HandleDev then R work items
  void *staging = nullptr;
  // device scratch of the LHZ decoders (grown on demand)
  void *dec_buf = nullptr;
  size_t dec_bytes = 0;
  sqa::HandleDev dev(int m0, int m1, int flags) const;
};
