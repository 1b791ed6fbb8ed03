// C ABI: SQA handles, batched persistent launches, decoders, autotuner.
#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <fstream>
#include <map>
#include <mutex>
#include <new>
#include <sstream>
#include <string>
#include <vector>

#include <sys/stat.h>

#include "host_core.h"

using namespace sqa;

namespace sqa {
const char *last_error_cstr();

static std::once_flag g_lds_once;
static hipError_t g_lds_status = hipSuccess;

// Raises the kernels' dynamic-LDS limit where the runtime supports the
// attribute; a refusal is not an error (launches above the default limit then
// fail and are reported at launch).
static hipError_t ensure_lds_limits() {
  std::call_once(g_lds_once, [] {
    (void)set_sqa_anneal_lds_limit(kMaxLds);
    (void)set_pt_lds_limit(kMaxLds);
    (void)hipGetLastError();
  });
  return g_lds_status;
}

// Work items (handle, replica group) of the handles with update move `move`,
// longest first.
static std::vector<WorkItem> plan_items(const std::vector<const sqa_handle *> &hs, const std::vector<int> &m0,
                                        const std::vector<int> &m1, int waves, int move) {
  std::vector<std::pair<double, WorkItem>> v;
  for (size_t i = 0; i < hs.size(); ++i) {
    const sqa_handle *h = hs[i];
    if (h->move != move) continue;
    const double cost = static_cast<double>(h->emb.n) * h->L * std::max(1, m1[i] - m0[i]);
    for (int r = 0; r < h->R; r += waves) {
      WorkItem w{static_cast<int32_t>(i), r, std::min(waves, h->R - r)};
      v.push_back({cost * w.nrep / waves, w});
    }
  }
  std::stable_sort(v.begin(), v.end(), [](const auto &a, const auto &b) { return a.first > b.first; });
  std::vector<WorkItem> out;
  out.reserve(v.size());
  for (auto &p : v) out.push_back(p.second);
  // Race check: results must not depend on which workgroup takes which item or
  // when; SQA_DEBUG_ITEM_ORDER=reverse or =shuffle hands the items out in
  // another order (shuffle: a fixed permutation from a 64-bit LCG).
  if (const char *o = std::getenv("SQA_DEBUG_ITEM_ORDER")) {
    if (std::strcmp(o, "reverse") == 0) {
      std::reverse(out.begin(), out.end());
    } else if (std::strcmp(o, "shuffle") == 0) {
      uint64_t x = 0x9E3779B97F4A7C15ull;
      for (size_t i = out.size(); i > 1; --i) {
        x = x * 6364136223846793005ull + 1442695040888963407ull;
        std::swap(out[i - 1], out[(x >> 33) % i]);
      }
    }
  }
  return out;
}

static LaunchShape shape_for(const std::vector<const sqa_handle *> &hs, int waves, int groups_per_cu,
                             size_t n_items, int move, bool team = false) {
  LaunchShape s;
  s.move = move;
  s.waves = waves;
  s.team = team && move == kMoveMetropolis;
  for (const sqa_handle *h : hs) {
    if (h->move != move) continue;
    s.rec_cap = std::max(s.rec_cap, h->emb.n * h->lay.rec_words);
    s.lat_cap = std::max(s.lat_cap, h->emb.n + 1);
    if (move == kMoveWolff) {
      int maxclass = 0;
      for (int c = 0; c < 4; ++c) maxclass = std::max(maxclass, h->lay.cls[c + 1] - h->lay.cls[c]);
      s.tab_cap = std::max(s.tab_cap, kWolffScratchWords * std::min(maxclass, kWolffChunk));
    } else {
      s.tab_cap = std::max(s.tab_cap, h->tw);
    }
  }
  s.rec_cap = (s.rec_cap + 3) & ~3;
  s.lat_cap = (s.lat_cap + 1) & ~1;
  s.tab_cap = (s.tab_cap + 3) & ~3;
  int gpc = groups_per_cu > 0 ? groups_per_cu : occupancy_groups_per_cu(s);
  long long grid = static_cast<long long>(device_cu_count()) * gpc;
  s.grid = static_cast<int>(std::max<long long>(1, std::min<long long>(grid, static_cast<long long>(n_items))));
  return s;
}

// Team mode (see kTeamMaxReplicas): applies to the Metropolis handles of a set
// that hold at most kTeamMaxReplicas replicas in all; *team_waves is then the
// number of waves that makes the largest colour class about one pass.
static bool use_team(const std::vector<const sqa_handle *> &hs, int move, int *team_waves) {
  if (move != kMoveMetropolis) return false;
  long long replicas = 0;
  int max_items = 1;
  for (const sqa_handle *h : hs) {
    if (h->move != move) continue;
    replicas += h->R;
    const int half = (h->L == 1) ? 1 : (h->L >> 1);
    const int bytes = (half + 7) >> 3;
    for (int c = 0; c < 4; ++c) max_items = std::max(max_items, (h->lay.cls[c + 1] - h->lay.cls[c]) * bytes);
  }
  if (replicas == 0 || replicas > kTeamMaxReplicas) return false;
  *team_waves = std::max(1, std::min(8, (max_items + 63) / 64));
  return true;
}

// One persistent launch per update move present in a handle set.  Device
// buffer of a set: [HandleDev x handles][items of each group][a counter per group].
struct MoveGroup {
  int move = kMoveMetropolis;
  std::vector<WorkItem> items;
  LaunchShape shape;
  size_t items_off = 0, counter_off = 0;
};

static sqa_status plan_groups(const std::vector<const sqa_handle *> &hs, const std::vector<int> &m0,
                              const std::vector<int> &m1, int waves, int gpc, std::vector<MoveGroup> *out,
                              size_t *bytes, bool allow_team = true) {
  out->clear();
  size_t off = (sizeof(HandleDev) * hs.size() + 255) & ~size_t(255);
  for (int move : {kMoveMetropolis, kMoveWolff}) {
    MoveGroup g;
    g.move = move;
    int tw = 0;
    const bool team = allow_team && use_team(hs, move, &tw);
    g.items = plan_items(hs, m0, m1, team ? 1 : waves, move);
    if (g.items.empty()) continue;
    g.shape = team ? shape_for(hs, tw, 0, g.items.size(), move, true) : shape_for(hs, waves, gpc, g.items.size(), move);
    if (g.shape.lds_bytes() > kMaxLds) return fail(SQA_ERR_UNSUPPORTED, "lattices do not fit in LDS");
    g.items_off = off;
    off = (off + sizeof(WorkItem) * g.items.size() + 255) & ~size_t(255);
    out->push_back(std::move(g));
  }
  for (MoveGroup &g : *out) {
    g.counter_off = off;
    off += 256;
  }
  *bytes = off;
  return SQA_OK;
}

static hipError_t upload_groups(char *base, const std::vector<HandleDev> &hds, const std::vector<MoveGroup> &gs,
                                hipStream_t stream) {
  hipError_t e = hipMemcpyAsync(base, hds.data(), sizeof(HandleDev) * hds.size(), hipMemcpyHostToDevice, stream);
  for (const MoveGroup &g : gs) {
    if (e != hipSuccess) break;
    e = hipMemcpyAsync(base + g.items_off, g.items.data(), sizeof(WorkItem) * g.items.size(), hipMemcpyHostToDevice,
                       stream);
  }
  return e;
}

// Fault injection for tests of the error paths: with SQA_FAULT_INJECT=launch in
// the environment, every sweep-kernel launch reports hipErrorLaunchFailure
// instead of being queued (nothing runs on the device).
hipError_t injected_launch_fault() {
  const char *f = std::getenv("SQA_FAULT_INJECT");
  return (f && std::strcmp(f, "launch") == 0) ? hipErrorLaunchFailure : hipSuccess;
}

static hipError_t launch_groups(char *base, const std::vector<MoveGroup> &gs, hipStream_t stream) {
  hipError_t e = injected_launch_fault();
  if (e != hipSuccess) return e;
  for (const MoveGroup &g : gs) {
    e = launch_sqa_anneal(g.move, reinterpret_cast<HandleDev *>(base), reinterpret_cast<WorkItem *>(base + g.items_off),
                          static_cast<int>(g.items.size()), reinterpret_cast<int *>(base + g.counter_off), g.shape.grid,
                          g.shape.waves, g.shape.rec_cap, g.shape.lat_cap, g.shape.tab_cap, g.shape.team, stream);
    if (e != hipSuccess) break;
  }
  return e;
}

// ---------------------------------------------------------------- autotune cache
static std::string device_arch() {
  int dev = 0;
  hipDeviceProp_t prop;
  if (hipGetDevice(&dev) != hipSuccess || hipGetDeviceProperties(&prop, dev) != hipSuccess) return "unknown";
  std::string a = prop.gcnArchName;
  size_t c = a.find(':');
  return c == std::string::npos ? a : a.substr(0, c);
}

// Shape class: largest lattice (sites x slices) rounded up to a power of two,
// replica count rounded up to a power of two, and whether both kinds are present.
static std::string shape_class(const std::vector<const sqa_handle *> &hs) {
  int maxcells = 1, maxrep = 1;
  bool me = false, lhz = false, wolff = false;
  for (const sqa_handle *h : hs) {
    maxcells = std::max(maxcells, h->emb.n * h->L);
    maxrep = std::max(maxrep, h->R);
    (h->emb.kind == SQA_EMB_LHZ ? lhz : me) = true;
    wolff = wolff || h->move == kMoveWolff;
  }
  auto p2 = [](int v) {
    int p = 1;
    while (p < v) p <<= 1;
    return p;
  };
  char buf[96];
  std::snprintf(buf, sizeof(buf), "cells%d_rep%d_%s%s", p2(maxcells), p2(maxrep), me && lhz ? "mix" : (me ? "me" : "lhz"),
                wolff ? "_wolff" : "");
  return buf;
}

static const char *cache_path_or_env(const char *p) {
  if (p && *p) return p;
  const char *e = std::getenv("SQA_AUTOTUNE_CACHE");
  return (e && *e) ? e : nullptr;
}

// The cache is a flat JSON object {"<arch>/<class>": [waves, groups_per_cu], ...}.
static std::map<std::string, std::pair<int, int>> read_cache(const char *path) {
  std::map<std::string, std::pair<int, int>> m;
  if (!path) return m;
  std::ifstream f(path);
  if (!f) return m;
  std::stringstream ss;
  ss << f.rdbuf();
  const std::string s = ss.str();
  size_t i = 0;
  while ((i = s.find('"', i)) != std::string::npos) {
    size_t j = s.find('"', i + 1);
    if (j == std::string::npos) break;
    std::string key = s.substr(i + 1, j - i - 1);
    size_t lb = s.find('[', j), rb = s.find(']', j);
    if (lb == std::string::npos || rb == std::string::npos) break;
    int a = 0, b = 0;
    if (std::sscanf(s.c_str() + lb + 1, "%d , %d", &a, &b) == 2) m[key] = {a, b};
    i = rb + 1;
  }
  return m;
}

// The parsed cache file of the last lookup, reused while the file's path, size and
// modification time are unchanged (every launch looks its shape up; the tuner's writes
// drop it).  Used under the cache mutex.
struct CacheMemo {
  std::string path;
  off_t size = -1;
  struct timespec mtime {};
  std::map<std::string, std::pair<int, int>> m;
};
static CacheMemo g_cache_memo;

static const std::map<std::string, std::pair<int, int>> &read_cache_memo(const char *path) {
  struct stat st {};
  if (stat(path, &st) != 0) {
    g_cache_memo = CacheMemo{};
    return g_cache_memo.m;
  }
  if (g_cache_memo.path != path || g_cache_memo.size != st.st_size ||
      g_cache_memo.mtime.tv_sec != st.st_mtim.tv_sec || g_cache_memo.mtime.tv_nsec != st.st_mtim.tv_nsec) {
    g_cache_memo.m = read_cache(path);
    g_cache_memo.path = path;
    g_cache_memo.size = st.st_size;
    g_cache_memo.mtime = st.st_mtim;
  }
  return g_cache_memo.m;
}

static void write_cache(const char *path, const std::map<std::string, std::pair<int, int>> &m) {
  if (!path) return;
  g_cache_memo = CacheMemo{};
  std::ofstream f(path);
  f << "{\n";
  size_t k = 0;
  for (auto &kv : m) {
    f << "  \"" << kv.first << "\": [" << kv.second.first << ", " << kv.second.second << "]"
      << (++k < m.size() ? ",\n" : "\n");
  }
  f << "}\n";
}

static std::mutex g_cache_mu;


static bool cached_config(const std::vector<const sqa_handle *> &hs, sqa_launch_config *out) {
  const char *path = cache_path_or_env(nullptr);
  if (!path) return false;
  std::lock_guard<std::mutex> lk(g_cache_mu);
  const auto &m = read_cache_memo(path);
  auto it = m.find(device_arch() + "/" + shape_class(hs));
  if (it == m.end()) return false;
  out->waves_per_group = it->second.first;
  out->groups_per_cu = it->second.second;
  return true;
}

static void resolve_config(const std::vector<const sqa_handle *> &hs, const sqa_launch_config *cfg, int *waves,
                           int *gpc) {
  sqa_launch_config c{0, 0};
  if (cfg) c = *cfg;
  if (c.waves_per_group == 0 || c.groups_per_cu == 0) {
    sqa_launch_config cached{0, 0};
    if (cached_config(hs, &cached)) {
      if (c.waves_per_group == 0) c.waves_per_group = cached.waves_per_group;
      if (c.groups_per_cu == 0) c.groups_per_cu = cached.groups_per_cu;
    }
  }
  *waves = c.waves_per_group > 0 ? c.waves_per_group : 4;
  *gpc = c.groups_per_cu;   // 0 = from occupancy
}

static bool valid_waves(int w) { return w >= 1 && w <= 8; }

sqa_status handle_prepare(const sqa_problem &problem, const sqa_embedding &embedding, const sqa_schedule &s,
                          sqa_handle **out) {
  *out = nullptr;
  if (!problem.J) return fail(SQA_ERR_INVALID, "J is null");
  if (!(s.beta > 0.0) || !std::isfinite(s.beta)) return fail(SQA_ERR_INVALID, "beta must be positive and finite");
  if (s.slices < 1 || (s.slices > 1 && (s.slices & 1))) return fail(SQA_ERR_INVALID, "slices must be 1 or even");
  if (s.slices > 64) return fail(SQA_ERR_UNSUPPORTED, "at most 64 Trotter slices");
  if (s.sweeps < 1) return fail(SQA_ERR_INVALID, "sweeps must be >= 1");
  if (s.replicas < 1 || s.replicas > 65536) return fail(SQA_ERR_INVALID, "replicas must be in 1..65536");
  if (s.move != SQA_MOVE_METROPOLIS && s.move != SQA_MOVE_WOLFF) return fail(SQA_ERR_INVALID, "unknown update move");
  std::vector<double> gamma;
  if (s.gamma) gamma.assign(s.gamma, s.gamma + s.sweeps);
  else gamma = linear_gamma(s.gamma_start, s.gamma_end, s.sweeps);
  for (double g : gamma)
    if (!(g >= 0.0) || !std::isfinite(g)) return fail(SQA_ERR_INVALID, "Gamma must be finite and >= 0");
  std::vector<double> bscale;
  if (s.bscale) {
    bscale.assign(s.bscale, s.bscale + s.sweeps);
    for (double b : bscale)
      if (!std::isfinite(b)) return fail(SQA_ERR_INVALID, "B must be finite");
  }

  sqa_handle *h = new (std::nothrow) sqa_handle();
  if (!h) return fail(SQA_ERR_OOM, "host allocation");
  sqa_status st = build_embedding(problem, embedding, &h->emb);
  if (st != SQA_OK) {
    delete h;
    return st;
  }
  h->N = problem.n;
  h->L = s.slices;
  h->M = s.sweeps;
  h->R = s.replicas;
  h->beta = s.beta;
  h->seed = s.seed;
  h->F = h->emb.fmax;
  h->move = s.move;
  h->tw = (h->move == kMoveWolff) ? 1 : 3 * (2 * h->F + 1);
  h->J.assign(problem.J, problem.J + static_cast<size_t>(h->N) * h->N);
  h->h.assign(h->N, 0);
  if (problem.h) {
    h->has_h = true;
    std::copy(problem.h, problem.h + h->N, h->h.begin());
  }
  // Wolff moves sum plain weights per slice; Metropolis records carry 6|w| when F is small
  st = build_layout(h->emb, h->F, h->move == kMoveWolff ? kLayoutWolff : kLayoutMetropolis, &h->lay);
  if (st != SQA_OK) {
    delete h;
    return st;
  }
  if (h->move == kMoveWolff) {
    h->table = wolff_join_table(s.beta, s.slices, gamma);
    h->wacc = wolff_accept_table(s.beta, s.slices, s.bscale ? &bscale : nullptr, h->F, &h->wrows);
    h->wwidth = 2 * s.slices * h->F + 1;
  } else {
    h->table = sqa_threshold_table(s.beta, s.slices, gamma, s.bscale ? &bscale : nullptr, h->F);
  }

  const int n = h->emb.n, R = h->R, L = h->L, N = h->N;
  const size_t nt = h->emb.terms.size();
  Arena &A = h->arena;
  // the uploaded regions first: the small ones (one copy from a host image), then the table
  h->off_rec = A.take(h->lay.rec.size() * 4);
  h->off_devof = A.take(static_cast<size_t>(n) * 2);
  h->off_hfield = A.take(static_cast<size_t>(n) * 4);
  h->off_tw = A.take(std::max<size_t>(nt, 1) * 4);
  h->off_ts = A.take(std::max<size_t>(nt, 1) * 8);
  h->off_wacc = A.take(std::max<size_t>(h->wacc.size(), 1) * 4);
  h->off_J = A.take(static_cast<size_t>(N) * N * 4);
  h->off_h = A.take(static_cast<size_t>(N) * 4);
  h->off_table = A.take(h->table.size() * 4);
  h->off_spins = A.take(static_cast<size_t>(R) * L * n);
  h->off_energy = A.take(static_cast<size_t>(R) * L * 4);
  h->off_logical = A.take(static_cast<size_t>(R) * N);
  h->off_lenergy = A.take(static_cast<size_t>(R) * 4);
  h->off_hd = A.take(sizeof(HandleDev));
  h->off_items = A.take(sizeof(WorkItem) * static_cast<size_t>(R));
  h->off_counter = A.take(256);
  A.size = A.used;
  *out = h;
  return SQA_OK;
}

size_t handle_block_bytes(const sqa_handle *h) { return h->arena.size; }

sqa_status handle_upload(sqa_handle *h, const sqa_allocator *alloc) {
  if (alloc) h->alloc = *alloc;
  Arena &A = h->arena;
  sqa_status st = device_alloc(&h->alloc, &A.base, A.size, "device block of the handle");
  if (st != SQA_OK) return st;
  h->device_bytes = A.size;
  const int n = h->emb.n, N = h->N;
  const size_t nt = h->emb.terms.size();
  struct Up {
    size_t off;
    const void *p;
    size_t bytes;
  } ups[] = {
      {h->off_rec, h->lay.rec.data(), h->lay.rec.size() * 4},
      {h->off_devof, h->lay.dev_of.data(), static_cast<size_t>(n) * 2},
      {h->off_hfield, h->lay.hfield.data(), static_cast<size_t>(n) * 4},
      {h->off_tw, h->lay.term_w.data(), nt * 4},
      {h->off_ts, h->lay.term_s.data(), nt * 8},
      {h->off_wacc, h->wacc.data(), h->wacc.size() * 4},
      {h->off_J, h->J.data(), static_cast<size_t>(N) * N * 4},
      {h->off_h, h->h.data(), static_cast<size_t>(N) * 4},
  };
  // the small regions (they precede the table in the block) in one copy from a host
  // image, the table in a second
  std::vector<char> img;
  try {
    img.assign(h->off_table, 0);
  } catch (const std::bad_alloc &) {
    return fail(SQA_ERR_OOM, "host allocation (handle upload)");
  }
  for (const Up &u : ups)
    if (u.bytes) std::memcpy(img.data() + u.off, u.p, u.bytes);
  hipError_t e = hipMemcpy(A.base, img.data(), img.size(), hipMemcpyHostToDevice);
  if (e == hipSuccess && !h->table.empty())
    e = hipMemcpy(A.at<char>(h->off_table), h->table.data(), h->table.size() * 4, hipMemcpyHostToDevice);
  if (e != hipSuccess) return hip_fail(e, "hipMemcpy (handle setup)");
  e = hipEventCreateWithFlags(&h->done, hipEventDisableTiming);
  if (e != hipSuccess) {
    h->done = nullptr;
    return hip_fail(e, "hipEventCreate (handle setup)");
  }
  return SQA_OK;
}

}  // namespace sqa

// =================================================================== C ABI
extern "C" {

const char *sqa_last_error(void) { return sqa::last_error_cstr(); }
const char *sqa_version(void) { return "sqa-mi355x 0.1 (gfx950)"; }

int64_t sqa_physical_sites(int32_t kind, int32_t n) {
  if (kind == SQA_EMB_ME) return n >= 2 ? static_cast<int64_t>(n) * (n - 1) : -1;
  if (kind == SQA_EMB_LHZ) return n >= 3 ? static_cast<int64_t>(n) * (n - 1) / 2 : -1;
  if (kind == SQA_EMB_ME_CHIMERA) return n >= 2 ? static_cast<int64_t>(n) * ((n + 3) / 4 + 1) : -1;
  return -1;
}

sqa_status sqa_create(const sqa_problem *problem, const sqa_embedding *embedding, const sqa_schedule *schedule,
                      const sqa_allocator *allocator, sqa_handle **out) {
  if (!problem || !embedding || !schedule || !out) return fail(SQA_ERR_INVALID, "null argument");
  *out = nullptr;
  if (allocator && (!allocator->alloc || !allocator->free))
    return fail(SQA_ERR_INVALID, "an allocator needs both callbacks");
  sqa_handle *h = nullptr;
  sqa_status st;
  try {
    st = handle_prepare(*problem, *embedding, *schedule, &h);
  } catch (const std::bad_alloc &) {
    return fail(SQA_ERR_OOM, "host allocation (tables)");
  }
  if (st != SQA_OK) return st;
  st = handle_upload(h, allocator);
  if (st != SQA_OK) {
    sqa_destroy(h);
    return st;
  }
  *out = h;
  return SQA_OK;
}

void sqa_destroy(sqa_handle *h) {
  if (!h) return;
  if (h->done) {
    (void)hipEventSynchronize(h->done);
    (void)hipEventDestroy(h->done);
  }
  device_free(&h->alloc, h->arena.base);
  device_free(&h->alloc, h->dec_buf);
  if (h->staging) (void)hipHostFree(h->staging);
  delete h;
}

sqa_status sqa_handle_device_bytes(sqa_handle *h, size_t *bytes_out) {
  if (!h || !bytes_out) return fail(SQA_ERR_INVALID, "null argument");
  *bytes_out = (h->arena.base ? h->arena.size : 0) + h->dec_bytes;
  return SQA_OK;
}

static sqa_status check_handle(sqa_handle *h) {
  if (!h) return fail(SQA_ERR_INVALID, "null handle");
  if (h->poisoned) return fail(SQA_ERR_DEVICE, "handle is poisoned by an earlier device error");
  return SQA_OK;
}

static sqa_status run_single(sqa_handle *h, int m0, int m1, int flags, hipStream_t stream) {
  hipError_t e = ensure_lds_limits();
  if (e != hipSuccess) return hip_fail(e, "hipFuncSetAttribute");
  std::vector<const sqa_handle *> hs{h};
  int waves = 4, gpc = 0;
  resolve_config(hs, nullptr, &waves, &gpc);
  int tw = 0;
  const bool team = use_team(hs, h->move, &tw);
  std::vector<WorkItem> items = plan_items(hs, {m0}, {m1}, team ? 1 : waves, h->move);
  LaunchShape shape = team ? shape_for(hs, tw, 0, items.size(), h->move, true)
                           : shape_for(hs, waves, gpc, items.size(), h->move);
  if (shape.lds_bytes() > kMaxLds) return fail(SQA_ERR_UNSUPPORTED, "lattice does not fit in LDS");
  // previous work on this handle must have consumed the pinned staging copy
  e = hipEventSynchronize(h->done);
  if (e != hipSuccess) {
    h->poisoned = true;
    return hip_fail(e, "hipEventSynchronize");
  }
  if (!h->staging) {     // taken at the first single-handle launch (batches and the server do not use it)
    e = hipHostMalloc(&h->staging, sizeof(HandleDev) + sizeof(WorkItem) * static_cast<size_t>(h->R), 0);
    if (e != hipSuccess) {
      h->staging = nullptr;
      return hip_fail(e, "hipHostMalloc (handle staging)");
    }
  }
  HandleDev *hd = static_cast<HandleDev *>(h->staging);
  WorkItem *st_items = reinterpret_cast<WorkItem *>(hd + 1);
  *hd = h->dev(m0, m1, flags);
  std::copy(items.begin(), items.end(), st_items);
  e = hipMemcpyAsync(h->arena.at<void>(h->off_hd), hd, sizeof(HandleDev), hipMemcpyHostToDevice, stream);
  if (e == hipSuccess)
    e = hipMemcpyAsync(h->arena.at<void>(h->off_items), st_items, items.size() * sizeof(WorkItem),
                       hipMemcpyHostToDevice, stream);
  if (e == hipSuccess) e = injected_launch_fault();
  if (e == hipSuccess)
    e = launch_sqa_anneal(h->move, h->arena.at<HandleDev>(h->off_hd), h->arena.at<WorkItem>(h->off_items),
                          static_cast<int>(items.size()), h->arena.at<int>(h->off_counter), shape.grid, shape.waves,
                          shape.rec_cap, shape.lat_cap, shape.tab_cap, shape.team, stream);
  if (e == hipSuccess) e = hipEventRecord(h->done, stream);
  if (e != hipSuccess) {
    h->poisoned = true;
    return hip_fail(e, "anneal launch");
  }
  h->initialised = true;
  return SQA_OK;
}

sqa_status sqa_anneal(sqa_handle *h, void *stream) {
  sqa_status st = check_handle(h);
  if (st != SQA_OK) return st;
  return run_single(h, 0, h->M, kFlagInit | kFlagEnergy, static_cast<hipStream_t>(stream));
}

sqa_status sqa_anneal_range(sqa_handle *h, int32_t m0, int32_t m1, void *stream) {
  sqa_status st = check_handle(h);
  if (st != SQA_OK) return st;
  if (m0 < 0 || m1 > h->M || m0 >= m1) return fail(SQA_ERR_INVALID, "need 0 <= m0 < m1 <= sweeps");
  return run_single(h, m0, m1, (h->initialised ? 0 : kFlagInit) | kFlagEnergy, static_cast<hipStream_t>(stream));
}

sqa_status sqa_reset(sqa_handle *h, void *stream) {
  sqa_status st = check_handle(h);
  if (st != SQA_OK) return st;
  hipStream_t s = static_cast<hipStream_t>(stream);
  hipError_t e = launch_sqa_init(h->dev(0, 0, 0), s);
  if (e == hipSuccess) e = hipEventRecord(h->done, s);
  if (e != hipSuccess) {
    h->poisoned = true;
    return hip_fail(e, "init launch");
  }
  h->initialised = true;
  return SQA_OK;
}

sqa_status sqa_sync(sqa_handle *h) {
  if (!h) return fail(SQA_ERR_INVALID, "null handle");
  hipError_t e = hipEventSynchronize(h->done);
  if (e != hipSuccess) {
    h->poisoned = true;
    return hip_fail(e, "hipEventSynchronize");
  }
  return h->poisoned ? fail(SQA_ERR_DEVICE, "handle is poisoned") : SQA_OK;
}

sqa_status sqa_read_spins(sqa_handle *h, int8_t *out, size_t len) {
  sqa_status st = check_handle(h);
  if (st != SQA_OK) return st;
  const size_t need = static_cast<size_t>(h->R) * h->L * h->emb.n;
  if (!out || len < need) return fail(SQA_ERR_INVALID, "spin buffer too short");
  if (!h->initialised) return fail(SQA_ERR_INVALID, "no state yet: anneal or reset first");
  if ((st = sqa_sync(h)) != SQA_OK) return st;
  hipError_t e = hipMemcpy(out, h->arena.at<void>(h->off_spins), need, hipMemcpyDeviceToHost);
  return e == hipSuccess ? SQA_OK : hip_fail(e, "hipMemcpy spins");
}

sqa_status sqa_read_energies(sqa_handle *h, int32_t *out, size_t len) {
  sqa_status st = check_handle(h);
  if (st != SQA_OK) return st;
  const size_t need = static_cast<size_t>(h->R) * h->L;
  if (!out || len < need) return fail(SQA_ERR_INVALID, "energy buffer too short");
  if (!h->initialised) return fail(SQA_ERR_INVALID, "no state yet: anneal first");
  if ((st = sqa_sync(h)) != SQA_OK) return st;
  hipError_t e = hipMemcpy(out, h->arena.at<void>(h->off_energy), need * 4, hipMemcpyDeviceToHost);
  return e == hipSuccess ? SQA_OK : hip_fail(e, "hipMemcpy energies");
}

sqa_status sqa_write_spins(sqa_handle *h, const int8_t *in, size_t len) {
  sqa_status st = check_handle(h);
  if (st != SQA_OK) return st;
  const size_t need = static_cast<size_t>(h->R) * h->L * h->emb.n;
  if (!in || len < need) return fail(SQA_ERR_INVALID, "spin buffer too short");
  for (size_t i = 0; i < need; ++i)
    if (in[i] != 1 && in[i] != -1) return fail(SQA_ERR_INVALID, "spins must be +1 or -1");
  if ((st = sqa_sync(h)) != SQA_OK) return st;
  hipError_t e = hipMemcpy(h->arena.at<void>(h->off_spins), in, need, hipMemcpyHostToDevice);
  if (e != hipSuccess) return hip_fail(e, "hipMemcpy spins");
  h->initialised = true;
  return SQA_OK;
}

void *sqa_device_spins(sqa_handle *h) { return h ? h->arena.at<void>(h->off_spins) : nullptr; }
void *sqa_device_energies(sqa_handle *h) { return h ? h->arena.at<void>(h->off_energy) : nullptr; }

sqa_status sqa_handle_info(sqa_handle *h, int32_t *sites, int32_t *slices, int32_t *replicas, int32_t *sweeps,
                           int32_t *fmax) {
  if (!h) return fail(SQA_ERR_INVALID, "null handle");
  if (sites) *sites = h->emb.n;
  if (slices) *slices = h->L;
  if (replicas) *replicas = h->R;
  if (sweeps) *sweeps = h->M;
  if (fmax) *fmax = h->F;
  return SQA_OK;
}

sqa_status sqa_export_table(sqa_handle *h, uint32_t *out, size_t len, int32_t *F_out) {
  if (!h) return fail(SQA_ERR_INVALID, "null handle");
  if (h->move != kMoveMetropolis) return fail(SQA_ERR_INVALID, "Wolff handle: use sqa_export_wolff_tables");
  if (F_out) *F_out = h->F;
  if (!out) return SQA_OK;
  if (len < h->table.size()) return fail(SQA_ERR_INVALID, "table buffer too short");
  std::memcpy(out, h->table.data(), h->table.size() * 4);
  return SQA_OK;
}

sqa_status sqa_export_wolff_tables(sqa_handle *h, uint32_t *padd_out, size_t padd_len, uint32_t *acc_out,
                                   size_t acc_len, int32_t *rows_out, int32_t *width_out) {
  if (!h) return fail(SQA_ERR_INVALID, "null handle");
  if (h->move != kMoveWolff) return fail(SQA_ERR_INVALID, "not a Wolff handle");
  if (rows_out) *rows_out = h->wrows;
  if (width_out) *width_out = h->wwidth;
  if (padd_out) {
    if (padd_len < h->table.size()) return fail(SQA_ERR_INVALID, "join-threshold buffer too short");
    std::memcpy(padd_out, h->table.data(), h->table.size() * 4);
  }
  if (acc_out) {
    if (acc_len < h->wacc.size()) return fail(SQA_ERR_INVALID, "acceptance buffer too short");
    std::memcpy(acc_out, h->wacc.data(), h->wacc.size() * 4);
  }
  return SQA_OK;
}

// ------------------------------------------------------------------ decoders
void *sqa_device_logical(sqa_handle *h) { return h ? h->arena.at<void>(h->off_logical) : nullptr; }
void *sqa_device_logical_energies(sqa_handle *h) { return h ? h->arena.at<void>(h->off_lenergy) : nullptr; }

}  // extern "C"

namespace {

// Device scratch of the LHZ decoders, grown on demand (after the handle's queued
// work, which may still read the old buffer, has finished).
sqa_status decode_scratch(sqa_handle *h, size_t bytes) {
  if (h->dec_bytes >= bytes) return SQA_OK;
  hipError_t e = hipEventSynchronize(h->done);
  if (e != hipSuccess) {
    h->poisoned = true;
    return hip_fail(e, "hipEventSynchronize");
  }
  device_free(&h->alloc, h->dec_buf);
  h->dec_buf = nullptr;
  h->dec_bytes = 0;
  sqa_status st = device_alloc(&h->alloc, &h->dec_buf, bytes, "decoder scratch");
  if (st != SQA_OK) return st;
  h->dec_bytes = bytes;
  return SQA_OK;
}

// Checks parent arrays (trees of K_N rooted at 0) and lists each tree's
// vertices parents-first (breadth-first from 0).
sqa_status tree_orders(int N, const int32_t *tree_parents, int n_trees, std::vector<int32_t> *order) {
  if (!tree_parents || n_trees < 1) return fail(SQA_ERR_INVALID, "tree decoding needs at least one tree");
  order->assign(static_cast<size_t>(n_trees) * N, 0);
  std::vector<std::vector<int>> kids(N);
  for (int t = 0; t < n_trees; ++t) {
    const int32_t *par = tree_parents + static_cast<size_t>(t) * N;
    if (par[0] != -1) return fail(SQA_ERR_INVALID, "tree must be rooted at logical spin 0");
    for (auto &k : kids) k.clear();
    for (int v = 1; v < N; ++v) {
      if (par[v] < 0 || par[v] >= N || par[v] == v) return fail(SQA_ERR_INVALID, "bad parent array");
      kids[par[v]].push_back(v);
    }
    int32_t *ord = order->data() + static_cast<size_t>(t) * N;
    int head = 0, tail = 0;
    ord[tail++] = 0;
    while (head < tail) {
      const int x = ord[head++];
      for (int y : kids[x])
        if (tail < N) ord[tail++] = y;
    }
    if (tail != N) return fail(SQA_ERR_INVALID, "parent array is not a tree rooted at 0");
  }
  return SQA_OK;
}

size_t align256(size_t x) { return (x + 255) & ~size_t(255); }

// Decoder scratch of the LHZ decoders: packed rows, best keys, MLD sums, BP pair
// values, MLD weight table, BP vote table, tree parents and orders.
struct DecodeLayout {
  size_t rows = 0, best = 0, acc = 0, pairs = 0, wtab = 0, dec = 0, par = 0, ord = 0, bytes = 0;
};

DecodeLayout decode_layout(int R, int N, int K, size_t tree_entries) {
  DecodeLayout d;
  d.rows = 0;
  d.best = align256(d.rows + static_cast<size_t>(R) * N * 4);
  d.acc = align256(d.best + static_cast<size_t>(R) * 8);
  d.pairs = align256(d.acc + static_cast<size_t>(R) * N * 8);
  d.wtab = align256(d.pairs + static_cast<size_t>(R) * K);
  d.dec = align256(d.wtab + static_cast<size_t>(2 * K + 1) * 8);
  d.par = align256(d.dec + static_cast<size_t>(2 * (2 * N - 3) + 1));
  d.ord = align256(d.par + tree_entries * 4);
  d.bytes = align256(d.ord + tree_entries * 4);
  return d;
}

}  // namespace

namespace sqa {
size_t decode_scratch_bytes(const sqa_handle *h, int decoder, size_t tree_entries) {
  if (decoder == SQA_DEC_ME_MAJORITY) return 0;
  return decode_layout(h->R, h->N, h->emb.n, tree_entries).bytes;
}

// Checks a decoder against the handle and, for the tree decoders, lists each
// tree's vertices parents-first.  No device work.
sqa_status decode_check(const sqa_handle *h, const sqa_decode_params &p, std::vector<int32_t> *order) {
  const int N = h->N;
  if (p.readout_slice < 0 || p.readout_slice >= h->L) return fail(SQA_ERR_INVALID, "readout slice out of range");
  if (p.decoder == SQA_DEC_ME_MAJORITY) {
    if (h->emb.kind != SQA_EMB_ME && h->emb.kind != SQA_EMB_ME_CHIMERA)
      return fail(SQA_ERR_INVALID, "majority decoding of chains needs an ME handle");
    return SQA_OK;
  }
  if (p.decoder != SQA_DEC_LHZ_TREES && p.decoder != SQA_DEC_LHZ_MWD && p.decoder != SQA_DEC_LHZ_MLD &&
      p.decoder != SQA_DEC_LHZ_BP)
    return fail(SQA_ERR_INVALID, "unknown decoder");
  if (h->emb.kind != SQA_EMB_LHZ) return fail(SQA_ERR_INVALID, "LHZ decoders need an LHZ handle");
  if (p.decoder == SQA_DEC_LHZ_MWD && N > 32)
    return fail(SQA_ERR_UNSUPPORTED, "exhaustive minimum-weight decoding limited to n <= 32");
  if (p.decoder == SQA_DEC_LHZ_MLD && N > 24)
    return fail(SQA_ERR_UNSUPPORTED, "exhaustive maximum-likelihood decoding limited to n <= 24");
  if (p.decoder == SQA_DEC_LHZ_BP && N > 32) return fail(SQA_ERR_UNSUPPORTED, "parity-check decoding limited to n <= 32");
  if ((p.decoder == SQA_DEC_LHZ_MLD || p.decoder == SQA_DEC_LHZ_BP) && !(p.error_rate > 0.0 && p.error_rate < 0.5))
    return fail(SQA_ERR_INVALID, "error rate must be in (0, 1/2)");
  if (p.decoder == SQA_DEC_LHZ_BP && p.iterations < 0) return fail(SQA_ERR_INVALID, "negative iteration count");
  if (p.decoder == SQA_DEC_LHZ_TREES || p.decoder == SQA_DEC_LHZ_BP) return tree_orders(N, p.tree_parents, p.n_trees, order);
  order->clear();
  return SQA_OK;
}

// Copies the decoder's host tables into its scratch `base` (laid out by
// decode_layout): tree parents and orders, MLD weights, BP votes.  Synchronous;
// the scratch must not be in use by queued work.
sqa_status decode_tables(const sqa_handle *h, const sqa_decode_params &p, const std::vector<int32_t> &order, char *base) {
  const int N = h->N, K = h->emb.n;
  const DecodeLayout dl = decode_layout(h->R, N, K, order.size());
  hipError_t e = hipSuccess;
  if (p.decoder == SQA_DEC_LHZ_TREES || p.decoder == SQA_DEC_LHZ_BP) {
    e = hipMemcpy(base + dl.par, p.tree_parents, order.size() * 4, hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipMemcpy(base + dl.ord, order.data(), order.size() * 4, hipMemcpyHostToDevice);
  }
  if (e == hipSuccess && p.decoder == SQA_DEC_LHZ_MLD) {
    // Sec. IV B: weights round(2^36 exp(-beta_N d)), d = O_max - O, beta_N = ln((1-p)/p) / 2
    const double beta = 0.5 * std::log((1.0 - p.error_rate) / p.error_rate);
    std::vector<uint64_t> w(2 * K + 1);
    for (int d = 0; d <= 2 * K; ++d)
      w[d] = static_cast<uint64_t>(std::llround(std::ldexp(std::exp(-beta * static_cast<double>(d)), 36)));
    e = hipMemcpy(base + dl.wtab, w.data(), w.size() * 8, hipMemcpyHostToDevice);
  }
  if (e == hipSuccess && p.decoder == SQA_DEC_LHZ_BP) {
    // Sec. IV D: x_ij <- sign(w0 s_ij + w1 c), tie keeps s_ij; w0 = ln((1-p)/p), w1 = ln((1-p2)/p2), p2 = 2p(1-p)
    const double q = p.error_rate, q2 = 2.0 * q * (1.0 - q);
    const double w0 = std::log((1.0 - q) / q), w1 = std::log((1.0 - q2) / q2);
    std::vector<int8_t> d(2 * (2 * N - 3) + 1, 1);
    for (int neg = 0; neg < 2; ++neg)
      for (int c = -(N - 2); c <= N - 2; ++c) {
        const int sv = neg ? -1 : 1;
        const double v = w0 * static_cast<double>(sv) + w1 * static_cast<double>(c);
        d[neg * (2 * N - 3) + c + N - 2] = static_cast<int8_t>(v > 0.0 ? 1 : (v < 0.0 ? -1 : sv));
      }
    e = hipMemcpy(base + dl.dec, d.data(), d.size(), hipMemcpyHostToDevice);
  }
  return e == hipSuccess ? SQA_OK : hip_fail(e, "hipMemcpy (decoder tables)");
}

// Queues the decoder's kernels on `s` (readout slice, decoder, logical
// energies), reading the scratch `base` (LHZ decoders) that decode_tables
// filled.  Kernels only: no host work and no copies, so a graph can hold it.
hipError_t decode_enqueue(const sqa_handle *h, const sqa_decode_params &p, size_t tree_entries, char *base,
                          hipStream_t s) {
  const int N = h->N, R = h->R, n = h->emb.n, L = h->L, K = n;
  const int8_t *spins = h->arena.at<int8_t>(h->off_spins);
  int8_t *logical = h->arena.at<int8_t>(h->off_logical);
  int32_t *lenergy = h->arena.at<int32_t>(h->off_lenergy);
  const int32_t *dJ = h->arena.at<int32_t>(h->off_J);
  const int32_t *dh = h->has_h ? h->arena.at<int32_t>(h->off_h) : nullptr;
  if (p.decoder == SQA_DEC_ME_MAJORITY) {
    const int len = h->emb.kind == SQA_EMB_ME ? N - 1 : (N + 3) / 4 + 1;
    return launch_me_majority(spins, R, N, len, n, L, p.readout_slice, dJ, dh, logical, lenergy, s);
  }
  const DecodeLayout dl = decode_layout(R, N, K, tree_entries);
  auto *rows = reinterpret_cast<uint32_t *>(base + dl.rows);
  auto *best = reinterpret_cast<unsigned long long *>(base + dl.best);
  auto *acc = reinterpret_cast<unsigned long long *>(base + dl.acc);
  auto *pairs = reinterpret_cast<int8_t *>(base + dl.pairs);
  auto *wtab = reinterpret_cast<uint64_t *>(base + dl.wtab);
  auto *dec = reinterpret_cast<int8_t *>(base + dl.dec);
  auto *par = reinterpret_cast<int32_t *>(base + dl.par);
  auto *ord = reinterpret_cast<int32_t *>(base + dl.ord);
  hipError_t e = hipSuccess;
  if (p.decoder != SQA_DEC_LHZ_TREES) e = launch_lhz_rows(spins, R, L, K, N, p.readout_slice, rows, s);
  if (e == hipSuccess) {
    switch (p.decoder) {
      case SQA_DEC_LHZ_TREES:
        e = launch_lhz_trees(spins + static_cast<size_t>(p.readout_slice) * K, static_cast<size_t>(L) * K, R, N, par,
                             ord, p.n_trees, logical, s);
        break;
      case SQA_DEC_LHZ_MWD:
        e = launch_lhz_mwd(rows, R, N, best, logical, s);
        break;
      case SQA_DEC_LHZ_MLD:
        e = launch_lhz_mld(rows, R, N, best, wtab, 2 * K + 1, acc, logical, s);
        break;
      default:
        e = launch_lhz_bp(rows, R, N, p.iterations, dec, pairs, s);
        if (e == hipSuccess) e = launch_lhz_trees(pairs, static_cast<size_t>(K), R, N, par, ord, p.n_trees, logical, s);
        break;
    }
  }
  if (e == hipSuccess) e = launch_logical_energy(logical, R, N, dJ, dh, lenergy, s);
  return e;
}

}  // namespace sqa

extern "C" {

sqa_status sqa_decode_ex(sqa_handle *h, const sqa_decode_params *prm, int8_t *logical_out,
                         int32_t *logical_energy_out, void *stream) {
  sqa_status st = check_handle(h);
  if (st != SQA_OK) return st;
  if (!prm) return fail(SQA_ERR_INVALID, "null decode parameters");
  const sqa_decode_params p = *prm;
  if (!h->initialised) return fail(SQA_ERR_INVALID, "no state yet: anneal first");
  std::vector<int32_t> order;
  st = decode_check(h, p, &order);
  if (st != SQA_OK) return st;
  const int N = h->N, R = h->R;
  hipStream_t s = static_cast<hipStream_t>(stream);
  char *base = nullptr;
  if (p.decoder != SQA_DEC_ME_MAJORITY) {
    st = decode_scratch(h, decode_layout(R, N, h->emb.n, order.size()).bytes);
    if (st != SQA_OK) return st;
    base = static_cast<char *>(h->dec_buf);
    // host tables (the earlier decodes that read this scratch have finished first)
    if (p.decoder != SQA_DEC_LHZ_MWD) {
      hipError_t e = hipEventSynchronize(h->done);
      if (e != hipSuccess) {
        h->poisoned = true;
        return hip_fail(e, "hipEventSynchronize");
      }
      st = decode_tables(h, p, order, base);
      if (st != SQA_OK) return st;
    }
  }
  hipError_t e = hipStreamWaitEvent(s, h->done, 0);
  if (e == hipSuccess) e = decode_enqueue(h, p, order.size(), base, s);
  if (e == hipSuccess) e = hipEventRecord(h->done, s);
  if (e != hipSuccess) {
    h->poisoned = true;
    return hip_fail(e, "decode launch");
  }
  if (!logical_out && !logical_energy_out) return SQA_OK;    // results stay on the device
  int8_t *logical = h->arena.at<int8_t>(h->off_logical);
  int32_t *lenergy = h->arena.at<int32_t>(h->off_lenergy);
  e = hipEventSynchronize(h->done);
  if (e == hipSuccess && logical_out) e = hipMemcpy(logical_out, logical, static_cast<size_t>(R) * N, hipMemcpyDeviceToHost);
  if (e == hipSuccess && logical_energy_out)
    e = hipMemcpy(logical_energy_out, lenergy, static_cast<size_t>(R) * 4, hipMemcpyDeviceToHost);
  if (e != hipSuccess) {
    h->poisoned = true;
    return hip_fail(e, "decode read-back");
  }
  return SQA_OK;
}

sqa_status sqa_ground_state(const sqa_problem *problem, int32_t *energy_out, int8_t *state_out) {
  if (!problem || !problem->J) return fail(SQA_ERR_INVALID, "null problem");
  const int N = problem->n;
  if (N < 2) return fail(SQA_ERR_INVALID, "n must be >= 2");
  if (N > 32) return fail(SQA_ERR_UNSUPPORTED, "exhaustive ground-state search limited to n <= 32");
  int maxabs = 1;
  for (int i = 0; i < N; ++i) {
    if (problem->h) maxabs = std::max(maxabs, std::abs(problem->h[i]));
    for (int j = i + 1; j < N; ++j) maxabs = std::max(maxabs, std::abs(problem->J[i * N + j]));
  }
  if (maxabs > 32767) return fail(SQA_ERR_UNSUPPORTED, "couplings and fields limited to |x| < 2^15");
  int B = 0;
  while ((1 << B) <= maxabs) ++B;
  // bit planes of |J| split by sign, c_p = sum_j J_pj, fields
  std::vector<uint32_t> planes(static_cast<size_t>(2 * B) * N, 0u);
  std::vector<int32_t> cj(N, 0), hv(N, 0);
  for (int p = 0; p < N; ++p) {
    if (problem->h) hv[p] = problem->h[p];
    for (int j = 0; j < N; ++j) {
      if (j == p) continue;
      const int32_t v = p < j ? problem->J[p * N + j] : problem->J[j * N + p];
      cj[p] += v;
      const uint32_t a = static_cast<uint32_t>(std::abs(v));
      for (int b = 0; b < B; ++b)
        if ((a >> b) & 1u) planes[static_cast<size_t>(2 * b + (v < 0 ? 1 : 0)) * N + p] |= 1u << j;
    }
  }
  const size_t o_c = align256(planes.size() * 4), o_h = align256(o_c + N * 4), o_k = align256(o_h + N * 4);
  void *dev = nullptr;
  hipError_t e = hipMalloc(&dev, o_k + 256);
  if (e != hipSuccess) return hip_fail(e, "hipMalloc (ground state)");
  char *base = static_cast<char *>(dev);
  unsigned long long key = 0;
  e = hipMemcpy(base, planes.data(), planes.size() * 4, hipMemcpyHostToDevice);
  if (e == hipSuccess) e = hipMemcpy(base + o_c, cj.data(), N * 4, hipMemcpyHostToDevice);
  if (e == hipSuccess) e = hipMemcpy(base + o_h, hv.data(), N * 4, hipMemcpyHostToDevice);
  if (e == hipSuccess)
    e = launch_ground(reinterpret_cast<uint32_t *>(base), reinterpret_cast<int32_t *>(base + o_c),
                      reinterpret_cast<int32_t *>(base + o_h), N, B, reinterpret_cast<unsigned long long *>(base + o_k),
                      nullptr);
  if (e == hipSuccess) e = hipMemcpy(&key, base + o_k, 8, hipMemcpyDeviceToHost);
  (void)hipFree(dev);
  if (e != hipSuccess) return hip_fail(e, "ground-state search");
  if (energy_out) *energy_out = static_cast<int32_t>(static_cast<uint32_t>(key >> 32) ^ 0x80000000u);
  if (state_out) {
    const uint32_t low = static_cast<uint32_t>(key);
    const uint32_t m = low >> 1;
    const int8_t sgn = (low & 1u) ? int8_t(-1) : int8_t(1);
    state_out[0] = sgn;
    for (int b = 0; b + 1 < N; ++b) state_out[b + 1] = static_cast<int8_t>(((m >> b) & 1u) ? -sgn : sgn);
  }
  return SQA_OK;
}

sqa_status sqa_read_logical(sqa_handle *h, int8_t *logical_out, size_t len, int32_t *energy_out, size_t elen) {
  sqa_status st = check_handle(h);
  if (st != SQA_OK) return st;
  const size_t nq = static_cast<size_t>(h->R) * h->N, ne = static_cast<size_t>(h->R);
  if ((logical_out && len < nq) || (energy_out && elen < ne)) return fail(SQA_ERR_INVALID, "buffer too short");
  if ((st = sqa_sync(h)) != SQA_OK) return st;
  hipError_t e = hipSuccess;
  if (logical_out) e = hipMemcpy(logical_out, h->arena.at<void>(h->off_logical), nq, hipMemcpyDeviceToHost);
  if (e == hipSuccess && energy_out) e = hipMemcpy(energy_out, h->arena.at<void>(h->off_lenergy), ne * 4, hipMemcpyDeviceToHost);
  return e == hipSuccess ? SQA_OK : hip_fail(e, "hipMemcpy logical");
}

sqa_status sqa_decode(sqa_handle *h, int32_t decoder, int32_t readout_slice, const int32_t *tree_parents,
                      int32_t n_trees, int8_t *logical_out, int32_t *logical_energy_out) {
  sqa_decode_params p{};
  p.decoder = decoder;
  p.readout_slice = readout_slice;
  p.tree_parents = tree_parents;
  p.n_trees = n_trees;
  p.error_rate = 0.2;
  p.iterations = 10;
  sqa_status st = sqa_decode_ex(h, &p, logical_out, logical_energy_out, nullptr);
  if (st != SQA_OK || logical_out || logical_energy_out) return st;
  return sqa_sync(h);
}

// Uniform labelled spanning trees from Pruefer sequences, entry i of tree t =
// floor(u N / 2^32) with u = word 0 of Philox(i, t, 0, TREE<<24); the
// smallest-leaf rule turns the sequence into edges, rooted at 0 by BFS.
sqa_status sqa_random_trees(uint64_t seed, int32_t n, int32_t n_trees, int32_t *parents_out) {
  if (n < 1 || n_trees < 0 || (!parents_out && n_trees > 0)) return fail(SQA_ERR_INVALID, "bad tree arguments");
  std::vector<int> seq(n > 2 ? n - 2 : 0), deg(n);
  std::vector<std::vector<int>> adj(n);
  for (int t = 0; t < n_trees; ++t) {
    for (int i = 0; i + 2 < n; ++i) {
      const uint32_t ctr[4] = {static_cast<uint32_t>(i), static_cast<uint32_t>(t), 0u, kStreamTree << 24};
      uint32_t o[4];
      host_philox4x32(ctr, static_cast<uint32_t>(seed), static_cast<uint32_t>(seed >> 32), o);
      seq[i] = static_cast<int>((static_cast<uint64_t>(o[0]) * static_cast<uint64_t>(n)) >> 32);
    }
    for (auto &a : adj) a.clear();
    std::fill(deg.begin(), deg.end(), 1);
    for (int x : seq) deg[x]++;
    for (int x : seq) {
      int leaf = 0;
      while (deg[leaf] != 1) ++leaf;
      adj[leaf].push_back(x);
      adj[x].push_back(leaf);
      deg[leaf]--;
      deg[x]--;
    }
    if (n >= 2) {
      int a = -1, b = -1;
      for (int v = 0; v < n; ++v)
        if (deg[v] == 1) (a < 0 ? a : b) = v;
      adj[a].push_back(b);
      adj[b].push_back(a);
    }
    int32_t *par = parents_out + static_cast<size_t>(t) * n;
    for (int v = 0; v < n; ++v) par[v] = -2;
    par[0] = -1;
    std::vector<int> queue{0};
    for (size_t qi = 0; qi < queue.size(); ++qi) {
      const int x = queue[qi];
      std::vector<int> nb = adj[x];
      std::sort(nb.begin(), nb.end());
      for (int y : nb)
        if (par[y] == -2) {
          par[y] = x;
          queue.push_back(y);
        }
    }
  }
  return SQA_OK;
}

// -------------------------------------------------------------- batches
}  // extern "C"

namespace sqa {

// The launch scratch of a set (plan_groups): the HandleDev array and at most one
// work item per replica, each part 256-aligned, and a 256-byte counter per move.
size_t launch_scratch_share(const sqa_handle *h) {
  return sizeof(HandleDev) + sizeof(WorkItem) * static_cast<size_t>(h->R);
}

size_t launch_scratch_bytes(const std::vector<sqa_handle *> &hs) {
  size_t b = kLaunchScratchFixed;
  for (const sqa_handle *h : hs) b += launch_scratch_share(h);
  return b;
}

sqa_status run_handles(const std::vector<sqa_handle *> &hs, const std::vector<int> &m0, const std::vector<int> &m1,
                       const std::vector<int> &flags, hipStream_t stream, const sqa_allocator *alloc, void **scratch,
                       size_t *scratch_bytes) {
  hipError_t e = ensure_lds_limits();
  if (e != hipSuccess) return hip_fail(e, "hipFuncSetAttribute");
  std::vector<const sqa_handle *> ch(hs.begin(), hs.end());
  int waves = 4, gpc = 0;
  resolve_config(ch, nullptr, &waves, &gpc);
  std::vector<MoveGroup> groups;
  size_t need = 0;
  sqa_status st = plan_groups(ch, m0, m1, waves, gpc, &groups, &need);
  if (st != SQA_OK) return st;
  std::vector<HandleDev> hds(hs.size());
  for (size_t i = 0; i < hs.size(); ++i) hds[i] = hs[i]->dev(m0[i], m1[i], flags[i]);
  if (need > launch_scratch_bytes(hs)) return fail(SQA_ERR_DEVICE, "launch scratch above its bound");
  if (*scratch_bytes < need) {
    device_free(alloc, *scratch);
    *scratch = nullptr;
    *scratch_bytes = 0;
    st = device_alloc(alloc, scratch, need, "launch scratch");
    if (st != SQA_OK) return st;
    *scratch_bytes = need;
  }
  char *base = static_cast<char *>(*scratch);
  e = upload_groups(base, hds, groups, stream);
  if (e == hipSuccess) e = launch_groups(base, groups, stream);
  if (e == hipSuccess)
    for (sqa_handle *h : hs) {
      e = hipEventRecord(h->done, stream);
      if (e != hipSuccess) break;
    }
  if (e == hipSuccess) e = hipStreamSynchronize(stream);
  if (e != hipSuccess) {
    for (sqa_handle *h : hs) h->poisoned = true;
    return hip_fail(e, "multi-handle launch");
  }
  for (sqa_handle *h : hs) h->initialised = true;
  return SQA_OK;
}

}  // namespace sqa

struct sqa_batch {
  std::vector<sqa_handle *> handles;
  sqa_launch_config config{0, 0};
  std::vector<sqa::MoveGroup> groups;
  void *dev = nullptr;
  hipStream_t capture_stream = nullptr;
  hipGraph_t graph = nullptr, graph_dec = nullptr;
  hipGraphExec_t exec = nullptr, exec_dec = nullptr;
  // decoders captured after the anneal: per handle its parameters (decoder -1:
  // none), tree copies and orders, and a scratch the batch owns
  std::vector<sqa_decode_params> dec;
  std::vector<std::vector<int32_t>> trees, orders;
  std::vector<void *> dec_buf;
  bool decodes = false;
  // timing of the last run: before the anneal graph, between it and the decoder
  // graph, after both
  hipEvent_t ev0 = nullptr, ev_mid = nullptr, ev1 = nullptr;
  bool ran = false;
};

static sqa_status batch_build(sqa_handle *const *handles, int32_t count, int waves, int gpc, bool allow_team,
                              sqa_batch **out) {
  std::vector<const sqa_handle *> hs(handles, handles + count);
  std::vector<int> m0(count, 0), m1(count);
  for (int i = 0; i < count; ++i) m1[i] = handles[i]->M;
  std::vector<MoveGroup> groups;
  size_t bytes = 0;
  sqa_status st = plan_groups(hs, m0, m1, waves, gpc, &groups, &bytes, allow_team);
  if (st != SQA_OK) return st;
  std::vector<HandleDev> hds(count);
  for (int i = 0; i < count; ++i) hds[i] = handles[i]->dev(0, handles[i]->M, kFlagInit | kFlagEnergy);
  sqa_batch *b = new (std::nothrow) sqa_batch();
  if (!b) return fail(SQA_ERR_OOM, "host allocation");
  b->handles.assign(handles, handles + count);
  b->config.waves_per_group = waves;
  b->config.groups_per_cu = gpc > 0 ? gpc : occupancy_groups_per_cu(groups.front().shape);
  b->groups = std::move(groups);
  hipError_t e = hipMalloc(&b->dev, bytes);
  if (e != hipSuccess) {
    delete b;
    return hip_fail(e, "hipMalloc (batch)");
  }
  e = upload_groups(static_cast<char *>(b->dev), hds, b->groups, nullptr);
  if (e == hipSuccess) e = hipStreamSynchronize(nullptr);
  if (e != hipSuccess) {
    (void)hipFree(b->dev);
    delete b;
    return hip_fail(e, "hipMemcpy (batch)");
  }
  *out = b;
  return SQA_OK;
}

// Checks each handle's decoder, copies its trees, gives it a scratch of its own
// and fills the scratch's host tables, all before capture.
static sqa_status batch_decoders(sqa_batch *b, const sqa_decode_params *decoders) {
  const size_t n = b->handles.size();
  b->dec.assign(n, sqa_decode_params{});
  b->trees.assign(n, {});
  b->orders.assign(n, {});
  b->dec_buf.assign(n, nullptr);
  for (size_t i = 0; i < n; ++i) {
    sqa_decode_params p = decoders[i];
    b->dec[i] = p;
    if (p.decoder == -1) continue;
    const sqa_handle *h = b->handles[i];
    sqa_status st = decode_check(h, p, &b->orders[i]);
    if (st != SQA_OK) return st;
    if (p.decoder == SQA_DEC_LHZ_TREES || p.decoder == SQA_DEC_LHZ_BP) {
      b->trees[i].assign(p.tree_parents, p.tree_parents + static_cast<size_t>(p.n_trees) * h->N);
      b->dec[i].tree_parents = b->trees[i].data();
    } else {
      b->dec[i].tree_parents = nullptr;
    }
    b->decodes = true;
    if (p.decoder == SQA_DEC_ME_MAJORITY) continue;
    hipError_t e = hipMalloc(&b->dec_buf[i], decode_layout(h->R, h->N, h->emb.n, b->orders[i].size()).bytes);
    if (e != hipSuccess) {
      b->dec_buf[i] = nullptr;
      return hip_fail(e, "hipMalloc (batch decoder scratch)");
    }
    st = decode_tables(h, b->dec[i], b->orders[i], static_cast<char *>(b->dec_buf[i]));
    if (st != SQA_OK) return st;
  }
  return SQA_OK;
}

static sqa_status batch_capture(sqa_batch *b) {
  hipError_t e = hipEventCreate(&b->ev0);
  if (e == hipSuccess) e = hipEventCreate(&b->ev_mid);
  if (e == hipSuccess) e = hipEventCreate(&b->ev1);
  if (e != hipSuccess) return hip_fail(e, "hipEventCreate (batch timing)");
  e = hipStreamCreateWithFlags(&b->capture_stream, hipStreamNonBlocking);
  if (e != hipSuccess) return hip_fail(e, "hipStreamCreate");
  e = hipStreamBeginCapture(b->capture_stream, hipStreamCaptureModeThreadLocal);
  if (e != hipSuccess) return hip_fail(e, "hipStreamBeginCapture");
  hipError_t le = launch_groups(static_cast<char *>(b->dev), b->groups, b->capture_stream);
  e = hipStreamEndCapture(b->capture_stream, &b->graph);
  if (le != hipSuccess) return hip_fail(le, "capture anneal launch");
  if (e != hipSuccess) return hip_fail(e, "hipStreamEndCapture");
  e = hipGraphInstantiate(&b->exec, b->graph, nullptr, nullptr, 0);
  if (e != hipSuccess) return hip_fail(e, "hipGraphInstantiate");
  if (!b->decodes) return SQA_OK;
  // the decoders in a second graph, replayed right after the first on the same stream
  e = hipStreamBeginCapture(b->capture_stream, hipStreamCaptureModeThreadLocal);
  if (e != hipSuccess) return hip_fail(e, "hipStreamBeginCapture");
  le = hipSuccess;
  for (size_t i = 0; i < b->handles.size() && le == hipSuccess; ++i)
    if (b->dec[i].decoder != -1)
      le = decode_enqueue(b->handles[i], b->dec[i], b->orders[i].size(), static_cast<char *>(b->dec_buf[i]),
                          b->capture_stream);
  e = hipStreamEndCapture(b->capture_stream, &b->graph_dec);
  if (le != hipSuccess) return hip_fail(le, "capture decoder launch");
  if (e != hipSuccess) return hip_fail(e, "hipStreamEndCapture");
  e = hipGraphInstantiate(&b->exec_dec, b->graph_dec, nullptr, nullptr, 0);
  if (e != hipSuccess) return hip_fail(e, "hipGraphInstantiate");
  return SQA_OK;
}

static void batch_free(sqa_batch *b) {
  if (!b) return;
  if (b->exec) (void)hipGraphExecDestroy(b->exec);
  if (b->graph) (void)hipGraphDestroy(b->graph);
  if (b->exec_dec) (void)hipGraphExecDestroy(b->exec_dec);
  if (b->graph_dec) (void)hipGraphDestroy(b->graph_dec);
  if (b->capture_stream) (void)hipStreamDestroy(b->capture_stream);
  if (b->dev) (void)hipFree(b->dev);
  for (void *p : b->dec_buf)
    if (p) (void)hipFree(p);
  for (hipEvent_t ev : {b->ev0, b->ev_mid, b->ev1})
    if (ev) (void)hipEventDestroy(ev);
  delete b;
}

extern "C" {

sqa_status sqa_batch_create(sqa_handle *const *handles, int32_t count, const sqa_launch_config *config,
                            sqa_batch **out) {
  return sqa_batch_create_decoded(handles, count, config, nullptr, out);
}

sqa_status sqa_batch_create_decoded(sqa_handle *const *handles, int32_t count, const sqa_launch_config *config,
                                    const sqa_decode_params *decoders, sqa_batch **out) {
  if (!handles || count < 1 || !out) return fail(SQA_ERR_INVALID, "bad batch arguments");
  *out = nullptr;
  for (int i = 0; i < count; ++i) {
    sqa_status st = check_handle(handles[i]);
    if (st != SQA_OK) return st;
  }
  if (config && ((config->waves_per_group != 0 && !valid_waves(config->waves_per_group)) || config->groups_per_cu < 0))
    return fail(SQA_ERR_INVALID, "waves_per_group must be in 1..8");
  hipError_t e = ensure_lds_limits();
  if (e != hipSuccess) return hip_fail(e, "hipFuncSetAttribute");
  std::vector<const sqa_handle *> hs(handles, handles + count);
  int waves = 4, gpc = 0;
  resolve_config(hs, config, &waves, &gpc);
  sqa_batch *b = nullptr;
  // an explicit waves_per_group keeps one wave per replica; otherwise team mode may apply
  const bool allow_team = !(config && config->waves_per_group > 0);
  sqa_status st = batch_build(handles, count, waves, gpc, allow_team, &b);
  if (st != SQA_OK) return st;
  if (decoders) st = batch_decoders(b, decoders);
  if (st == SQA_OK) st = batch_capture(b);
  if (st != SQA_OK) {
    batch_free(b);
    return st;
  }
  *out = b;
  return SQA_OK;
}

sqa_status sqa_batch_run(sqa_batch *b, void *stream) {
  if (!b) return fail(SQA_ERR_INVALID, "null batch");
  hipStream_t s = static_cast<hipStream_t>(stream);
  for (sqa_handle *h : b->handles) {
    if (h->poisoned) return fail(SQA_ERR_DEVICE, "a handle of the batch is poisoned");
    hipError_t e = hipStreamWaitEvent(s, h->done, 0);
    if (e != hipSuccess) return hip_fail(e, "hipStreamWaitEvent");
  }
  hipError_t e = hipEventRecord(b->ev0, s);
  if (e == hipSuccess) e = hipGraphLaunch(b->exec, s);
  if (e == hipSuccess && b->decodes) {
    e = hipEventRecord(b->ev_mid, s);
    if (e == hipSuccess) e = hipGraphLaunch(b->exec_dec, s);
  }
  if (e == hipSuccess) e = hipEventRecord(b->ev1, s);
  if (e != hipSuccess) {
    for (sqa_handle *h : b->handles) h->poisoned = true;
    return hip_fail(e, "hipGraphLaunch");
  }
  for (sqa_handle *h : b->handles) {
    e = hipEventRecord(h->done, s);
    if (e != hipSuccess) return hip_fail(e, "hipEventRecord");
    h->initialised = true;
  }
  b->ran = true;
  return SQA_OK;
}

sqa_status sqa_batch_timing(sqa_batch *b, float *anneal_ms, float *decode_ms) {
  if (!b) return fail(SQA_ERR_INVALID, "null batch");
  if (!b->ran) return fail(SQA_ERR_INVALID, "the batch has not run yet");
  hipError_t e = hipEventSynchronize(b->ev1);
  float a = 0.0f, d = 0.0f;
  if (e == hipSuccess) e = hipEventElapsedTime(&a, b->ev0, b->decodes ? b->ev_mid : b->ev1);
  if (e == hipSuccess && b->decodes) e = hipEventElapsedTime(&d, b->ev_mid, b->ev1);
  if (e != hipSuccess) return hip_fail(e, "batch timing");
  if (anneal_ms) *anneal_ms = a;
  if (decode_ms) *decode_ms = d;
  return SQA_OK;
}

sqa_status sqa_batch_config(sqa_batch *b, sqa_launch_config *out) {
  if (!b || !out) return fail(SQA_ERR_INVALID, "null argument");
  *out = b->config;
  return SQA_OK;
}

void sqa_batch_destroy(sqa_batch *b) {
  if (!b) return;
  (void)hipDeviceSynchronize();
  batch_free(b);
}

sqa_status sqa_anneal_batch(sqa_handle *const *handles, int32_t count, void *stream) {
  sqa_batch *b = nullptr;
  sqa_status st = sqa_batch_create(handles, count, nullptr, &b);
  if (st != SQA_OK) return st;
  st = sqa_batch_run(b, stream);
  (void)hipStreamSynchronize(static_cast<hipStream_t>(stream));
  sqa_batch_destroy(b);
  return st;
}

// The one-shot batch without allocations: the same plan and kernels, with the
// descriptors, work items and counters in the library's file-scope launch
// scratch (this device's copy) instead of a fresh device buffer, and no graph.
sqa_status sqa_anneal_batch_noalloc(sqa_handle *const *handles, int32_t count, void *stream) {
  if (!handles || count < 1) return fail(SQA_ERR_INVALID, "bad batch arguments");
  for (int i = 0; i < count; ++i) {
    sqa_status st = check_handle(handles[i]);
    if (st != SQA_OK) return st;
  }
  hipError_t e = ensure_lds_limits();
  if (e != hipSuccess) return hip_fail(e, "hipFuncSetAttribute");
  std::vector<const sqa_handle *> hs(handles, handles + count);
  int waves = 4, gpc = 0;
  resolve_config(hs, nullptr, &waves, &gpc);
  std::vector<int> m0(count, 0), m1(count);
  for (int i = 0; i < count; ++i) m1[i] = handles[i]->M;
  std::vector<MoveGroup> groups;
  size_t bytes = 0;
  sqa_status st = plan_groups(hs, m0, m1, waves, gpc, &groups, &bytes, true);
  if (st != SQA_OK) return st;
  if (bytes > kNoAllocScratchBytes)
    return fail(SQA_ERR_UNSUPPORTED, "launch scratch of " + std::to_string(bytes) + " bytes exceeds the " +
                                         std::to_string(kNoAllocScratchBytes) +
                                         "-byte static scratch: use sqa_anneal_batch");
  void *base = nullptr;
  st = noalloc_scratch(&base);
  if (st != SQA_OK) return st;
  std::vector<HandleDev> hds(count);
  for (int i = 0; i < count; ++i) hds[i] = handles[i]->dev(0, handles[i]->M, kFlagInit | kFlagEnergy);
  hipStream_t s = static_cast<hipStream_t>(stream);
  for (sqa_handle *h : std::vector<sqa_handle *>(handles, handles + count)) {
    e = hipStreamWaitEvent(s, h->done, 0);
    if (e != hipSuccess) return hip_fail(e, "hipStreamWaitEvent");
  }
  e = upload_groups(static_cast<char *>(base), hds, groups, s);
  if (e == hipSuccess) e = launch_groups(static_cast<char *>(base), groups, s);
  if (e == hipSuccess)
    for (int i = 0; i < count && e == hipSuccess; ++i) e = hipEventRecord(handles[i]->done, s);
  if (e == hipSuccess) e = hipStreamSynchronize(s);
  if (e != hipSuccess) {
    for (int i = 0; i < count; ++i) handles[i]->poisoned = true;
    return hip_fail(e, "batch launch (static scratch)");
  }
  for (int i = 0; i < count; ++i) handles[i]->initialised = true;
  return SQA_OK;
}

// Times each candidate shape on a short sweep range of the handles' full
// batch (state saved and restored), keeps the fastest.
sqa_status sqa_autotune(sqa_handle *const *handles, int32_t count, const char *cache_path, sqa_launch_config *best) {
  if (!handles || count < 1) return fail(SQA_ERR_INVALID, "bad autotune arguments");
  for (int i = 0; i < count; ++i) {
    sqa_status st = check_handle(handles[i]);
    if (st != SQA_OK) return st;
  }
  hipError_t e = ensure_lds_limits();
  if (e != hipSuccess) return hip_fail(e, "hipFuncSetAttribute");
  std::vector<const sqa_handle *> hs(handles, handles + count);
  // save device state
  std::vector<void *> saved(count, nullptr);
  for (int i = 0; i < count; ++i) {
    sqa_handle *h = handles[i];
    const size_t bytes = static_cast<size_t>(h->R) * h->L * h->emb.n + static_cast<size_t>(h->R) * h->L * 4;
    e = hipMalloc(&saved[i], bytes);
    if (e != hipSuccess) break;
    e = hipMemcpy(saved[i], h->arena.at<void>(h->off_spins), static_cast<size_t>(h->R) * h->L * h->emb.n,
                  hipMemcpyDeviceToDevice);
    if (e == hipSuccess)
      e = hipMemcpy(static_cast<char *>(saved[i]) + static_cast<size_t>(h->R) * h->L * h->emb.n,
                    h->arena.at<void>(h->off_energy), static_cast<size_t>(h->R) * h->L * 4, hipMemcpyDeviceToDevice);
    if (e != hipSuccess) break;
  }
  double best_t = 1e300;
  int best_w = 4, best_g = 0;
  if (e == hipSuccess) {
    hipEvent_t a, z;
    (void)hipEventCreate(&a);
    (void)hipEventCreate(&z);
    const int trial_sweeps = 100;
    for (int w : {2, 4, 8}) {   // multiples of the 4 SIMDs of a CU keep waves balanced
      std::vector<int> m0(count, 0), m1(count);
      for (int i = 0; i < count; ++i) m1[i] = std::min(handles[i]->M, trial_sweeps);
      std::vector<MoveGroup> base;
      size_t bytes = 0;
      if (plan_groups(hs, m0, m1, w, 0, &base, &bytes, false) != SQA_OK) continue;
      // groups-per-CU candidates: every count from half the occupancy of the first
      // group's kernel up to all of it (the count sets how evenly the work items
      // divide into rounds of resident workgroups)
      const int occ = occupancy_groups_per_cu(base.front().shape);
      std::vector<int> gpcs;
      for (int g = occ; g >= std::max(1, occ / 2); --g) gpcs.push_back(g);
      for (int g : gpcs) {
        std::vector<MoveGroup> groups;
        if (plan_groups(hs, m0, m1, w, g, &groups, &bytes, false) != SQA_OK) continue;
        std::vector<HandleDev> hds(count);
        for (int i = 0; i < count; ++i) hds[i] = handles[i]->dev(0, m1[i], kFlagInit);
        void *dev = nullptr;
        if (hipMalloc(&dev, bytes) != hipSuccess) continue;
        hipError_t le = upload_groups(static_cast<char *>(dev), hds, groups, nullptr);
        // the second of two identical launches is timed (the first warms caches and code)
        float ms = 0;
        for (int rep = 0; rep < 2 && le == hipSuccess; ++rep) {
          (void)hipEventRecord(a, nullptr);
          le = launch_groups(static_cast<char *>(dev), groups, nullptr);
          (void)hipEventRecord(z, nullptr);
          (void)hipEventSynchronize(z);
          (void)hipEventElapsedTime(&ms, a, z);
        }
        (void)hipFree(dev);
        if (le == hipSuccess && ms < best_t) {
          best_t = ms;
          best_w = w;
          best_g = g;
        }
      }
    }
    (void)hipEventDestroy(a);
    (void)hipEventDestroy(z);
  }
  // restore device state
  for (int i = 0; i < count; ++i) {
    sqa_handle *h = handles[i];
    if (!saved[i]) continue;
    (void)hipMemcpy(h->arena.at<void>(h->off_spins), saved[i], static_cast<size_t>(h->R) * h->L * h->emb.n,
              hipMemcpyDeviceToDevice);
    (void)hipMemcpy(h->arena.at<void>(h->off_energy), static_cast<char *>(saved[i]) + static_cast<size_t>(h->R) * h->L * h->emb.n,
              static_cast<size_t>(h->R) * h->L * 4, hipMemcpyDeviceToDevice);
    (void)hipFree(saved[i]);
  }
  if (e != hipSuccess) return hip_fail(e, "autotune state save");
  if (best_t >= 1e300) return fail(SQA_ERR_UNSUPPORTED, "no launch shape fits");
  if (best) {
    best->waves_per_group = best_w;
    best->groups_per_cu = best_g;
  }
  const char *path = cache_path_or_env(cache_path);
  if (path) {
    std::lock_guard<std::mutex> lk(g_cache_mu);
    auto m = read_cache(path);
    m[device_arch() + "/" + shape_class(hs)] = {best_w, best_g};
    write_cache(path, m);
  }
  return SQA_OK;
}

}  // extern "C"
