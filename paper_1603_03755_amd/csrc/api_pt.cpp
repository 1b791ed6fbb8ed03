// C ABI: parallel tempering handles (Appendix B, Eqs. (B1)-(B2)).
#include <algorithm>
#include <cmath>
#include <cstdlib>
#include <cstring>
#include <new>
#include <vector>

#include "host_core.h"

using namespace sqa;

struct pt_handle {
  Embedded emb;
  DeviceLayout lay;
  int32_t R = 0, F = 0, Dmax = 0, sweeps = 0, sps = 1;
  bool swap_falling = false;   // every row of stab is non-increasing in D
  int32_t nph = 4, ph[5] = {0, 0, 0, 0, 0};   // sweep phases (see pt_phases)
  uint64_t seed = 0;
  std::vector<double> betas;
  std::vector<uint32_t> mtab, stab, spack;
  Arena arena;
  size_t off_rec = 0, off_devof = 0, off_hfield = 0, off_tw = 0, off_ts = 0, off_mtab = 0, off_stab = 0, off_spack = 0,
         off_spins = 0, off_energy = 0, off_repat = 0, off_acc = 0, off_pd = 0;
  bool ran = false;
  bool poisoned = false;
  hipEvent_t done = nullptr;

  PTDev dev() const {
    PTDev P{};
    P.rec = arena.at<uint32_t>(off_rec);
    P.hfield = arena.at<int32_t>(off_hfield);
    P.term_w = arena.at<int32_t>(off_tw);
    P.term_s = arena.at<uint32_t>(off_ts);
    P.mtab = arena.at<uint32_t>(off_mtab);
    P.stab = arena.at<uint32_t>(off_stab);
    P.spack = arena.at<uint32_t>(off_spack);
    P.spack_words = static_cast<int32_t>(spack.size());
    P.dev_of = arena.at<uint16_t>(off_devof);
    P.spins = arena.at<int8_t>(off_spins);
    P.energy = arena.at<int32_t>(off_energy);
    P.rep_at = arena.at<int32_t>(off_repat);
    P.swap_acc = arena.at<uint64_t>(off_acc);
    P.kind = emb.kind;
    P.n = emb.n;
    P.n_terms = static_cast<int32_t>(emb.terms.size());
    P.R = R;
    P.F = F;
    P.Dmax = Dmax;
    // 1: swap phases compare gaps with precomputed acceptance bounds; 0: they
    // read the threshold of each gap.  For the tests, SQA_DEBUG_PT_SWAP=table
    // forces 0 and =bisect (2) starts every bound's search from 0 instead of
    // the estimate, so that most bounds are found by bisection.
    const char *dbg = std::getenv("SQA_DEBUG_PT_SWAP");
    P.swap_falling = !swap_falling ? 0 : (dbg && std::strcmp(dbg, "table") == 0) ? 0
                                         : (dbg && std::strcmp(dbg, "bisect") == 0) ? 2 : 1;
    P.sweeps = sweeps;
    P.sweeps_per_swap = sps;
    P.seed_lo = static_cast<uint32_t>(seed);
    P.seed_hi = static_cast<uint32_t>(seed >> 32);
    for (int c = 0; c < 5; ++c) P.cls[c] = lay.cls[c];
    // SQA_DEBUG_PT_PHASES=4 keeps the four classes (for the tests)
    const char *phs = std::getenv("SQA_DEBUG_PT_PHASES");
    const bool classes = phs && std::strcmp(phs, "4") == 0;
    P.nph = classes ? 4 : nph;
    for (int c = 0; c < 5; ++c) P.ph[c] = classes ? lay.cls[c] : ph[c];
    return P;
  }
};

namespace {

struct PTShape {
  int waves = 4;
  int rec_cap = 0, lat_cap = 0, mtab_cap = 0;
  int spack_cap = 0;   // packed swap table staged in LDS (0: read from device memory)
  size_t lds() const {
    return (static_cast<size_t>(kPTSpreadWords) + rec_cap + 2ull * lat_cap + mtab_cap + kPTLadderWords + spack_cap) * 4;
  }
};

PTShape pt_shape(const std::vector<const pt_handle *> &hs) {
  PTShape s;
  int max_items = 0;
  for (const pt_handle *h : hs) {
    s.rec_cap = std::max(s.rec_cap, h->emb.n * h->lay.rec_words);
    s.lat_cap = std::max(s.lat_cap, h->emb.n + 1);
    s.mtab_cap = std::max(s.mtab_cap, h->R * (2 * h->F + 1));
    // items of a colour class: its sites x the replica bytes (rounded up to a power of two)
    int rg = 1;
    while (rg * 8 < h->R) rg <<= 1;
    for (int c = 0; c < 4; ++c) max_items = std::max(max_items, (h->lay.cls[c + 1] - h->lay.cls[c]) * rg);
  }
  s.rec_cap = (s.rec_cap + 3) & ~3;
  s.lat_cap = (s.lat_cap + 1) & ~1;
  s.mtab_cap = (s.mtab_cap + 3) & ~3;
  // the packed swap tables go to LDS when the largest one fits beside the rest
  // (SQA_PT_STAGE_SWAPS=0 keeps them in device memory)
  int spack = 0;
  for (const pt_handle *h : hs) spack = std::max(spack, static_cast<int>(h->spack.size()));
  s.spack_cap = (spack + 3) & ~3;
  const char *stage = std::getenv("SQA_PT_STAGE_SWAPS");
  if (s.lds() > kMaxLds || (stage && std::atoi(stage) == 0)) s.spack_cap = 0;
  // one workgroup owns a ladder: enough waves that the largest colour class is one
  // pass, and one more without items (the last wave draws the swap words, off the
  // sweep's path), at most kPTMaxWaves (the kernel's launch bound; larger classes loop)
  const char *env = std::getenv("SQA_PT_WAVES");
  s.waves = env ? std::max(1, std::min(kPTMaxWaves, std::atoi(env)))
                : std::max(2, std::min(kPTMaxWaves, (max_items + 63) / 64 + 1));
  // the byte mode sums a thread's items in 16-bit halves, emptied before any
  // colour class that could take them past 256 items: a class gives a thread at
  // most 256 of them
  s.waves = std::max(s.waves, std::min(kPTMaxWaves, (max_items + 256 * 64 - 1) / (256 * 64)));
  return s;
}

sqa_status pt_launch(const std::vector<pt_handle *> &hs, hipStream_t stream) {
  std::vector<const pt_handle *> ch(hs.begin(), hs.end());
  PTShape s = pt_shape(ch);
  if (s.lds() > kMaxLds) return fail(SQA_ERR_UNSUPPORTED, "PT ladder does not fit in LDS");
  (void)set_pt_lds_limit(kMaxLds);
  (void)hipGetLastError();
  hipError_t e = hipSuccess;
  std::vector<PTDev> pds;
  for (pt_handle *h : hs) {
    e = hipEventSynchronize(h->done);
    if (e != hipSuccess) return hip_fail(e, "hipEventSynchronize");
    pds.push_back(h->dev());
  }
  void *dev = nullptr;
  e = hipMalloc(&dev, sizeof(PTDev) * pds.size());
  if (e != hipSuccess) return hip_fail(e, "hipMalloc (PT descriptors)");
  e = hipMemcpy(dev, pds.data(), sizeof(PTDev) * pds.size(), hipMemcpyHostToDevice);
  if (e == hipSuccess) e = injected_launch_fault();
  if (e == hipSuccess)
    e = launch_pt(static_cast<const PTDev *>(dev), static_cast<int>(pds.size()), s.waves, s.rec_cap, s.lat_cap,
                  s.mtab_cap, s.spack_cap, stream);
  if (e == hipSuccess)
    for (pt_handle *h : hs) {
      e = hipEventRecord(h->done, stream);
      if (e != hipSuccess) break;
    }
  hipError_t e2 = hipStreamSynchronize(stream);
  (void)hipFree(dev);
  if (e == hipSuccess) e = e2;
  if (e != hipSuccess) {
    for (pt_handle *h : hs) h->poisoned = true;
    return hip_fail(e, "PT launch");
  }
  for (pt_handle *h : hs) h->ran = true;
  return SQA_OK;
}

}  // namespace

extern "C" {

// Eq. (B1) for a pair with beta_{r+1} < beta_r: the threshold of the energy
// gap D falls with D and is 0 once exp(D (beta_{r+1} - beta_r)) < 2^-32.  The
// swap table needs its columns only up to the first D at which every pair's
// threshold is 0; larger gaps clamp to that column.  Pairs of equal
// temperatures always swap, so their rows never reach 0 and the table keeps
// the whole range 0..2 E_max.
static int64_t swap_table_width(const std::vector<double> &betas, int64_t dfull) {
  int64_t cut = 0;
  for (size_t r = 0; r + 1 < betas.size(); ++r) {
    const double db = betas[r + 1] - betas[r];
    if (!(db < 0.0)) return dfull;
    // first D in [0, dfull] whose threshold is 0 (the thresholds do not rise with D)
    if (threshold_from_log(static_cast<double>(dfull) * db) != 0u) return dfull;
    int64_t lo = 0, hi = dfull;
    while (lo < hi) {
      const int64_t mid = lo + (hi - lo) / 2;
      if (threshold_from_log(static_cast<double>(mid) * db) == 0u) hi = mid;
      else lo = mid + 1;
    }
    cut = std::max(cut, lo);
  }
  return std::min(cut, dfull);
}

// A sweep updates the colour classes in order (sites of one class share no
// term).  Two consecutive classes that share no term either update together in
// one phase: each site's field reads only sites of the other classes, so the
// spins, energies and random words are those of the class-by-class sweep.  The
// byte-mode kernel of the ME kinds merges the first such pair (clique-chain ME:
// classes 1 and 2); every other ladder sweeps the four classes.
static void pt_phases(const Embedded &emb, const DeviceLayout &lay, int32_t F, int32_t *nph, int32_t ph[5]) {
  for (int c = 0; c < 5; ++c) ph[c] = lay.cls[c];
  *nph = 4;
  if (F > kPTByteF || (emb.kind != kKindME && emb.kind != kKindMEC)) return;
  auto cls_of = [&](int s) {
    const int d = lay.dev_of[s];
    int c = 0;
    while (c < 3 && d >= lay.cls[c + 1]) ++c;
    return c;
  };
  bool joined[4][4] = {};
  for (const Term &t : emb.terms)
    for (int i = 0; i < t.arity; ++i)
      for (int j = 0; j < t.arity; ++j)
        if (i != j) joined[cls_of(t.s[i])][cls_of(t.s[j])] = true;
  for (int c = 0; c < 3; ++c)
    if (!joined[c][c + 1]) {
      for (int k = c + 1; k < 4; ++k) ph[k] = lay.cls[k + 1];
      ph[4] = lay.cls[4];
      *nph = 3;
      return;
    }
}

// Widest swap-table row accepted (entries).
constexpr int64_t kMaxSwapRow = int64_t(1) << 22;

static sqa_status pt_create_impl(const sqa_problem *problem, const sqa_embedding *embedding, const pt_params *params,
                                 pt_handle **out);

sqa_status pt_create(const sqa_problem *problem, const sqa_embedding *embedding, const pt_params *params,
                     pt_handle **out) {
  try {
    return pt_create_impl(problem, embedding, params, out);
  } catch (const std::bad_alloc &) {
    if (out) *out = nullptr;
    return fail(SQA_ERR_OOM, "host allocation (PT tables)");
  }
}

static sqa_status pt_create_impl(const sqa_problem *problem, const sqa_embedding *embedding, const pt_params *params,
                                 pt_handle **out) {
  if (!problem || !embedding || !params || !out || !problem->J) return fail(SQA_ERR_INVALID, "null argument");
  *out = nullptr;
  const pt_params &p = *params;
  if (p.temps < 1 || p.temps > 64) return fail(SQA_ERR_INVALID, "temps must be in 1..64");
  if (p.sweeps < 1 || p.sweeps_per_swap < 1) return fail(SQA_ERR_INVALID, "sweeps and sweeps_per_swap must be >= 1");
  if (!(p.beta_min > 0) || !(p.beta_max >= p.beta_min) || !std::isfinite(p.beta_max))
    return fail(SQA_ERR_INVALID, "need 0 < beta_min <= beta_max");
  pt_handle *h = new (std::nothrow) pt_handle();
  if (!h) return fail(SQA_ERR_OOM, "host allocation");
  sqa_status st = build_embedding(*problem, *embedding, &h->emb);
  if (st == SQA_OK) st = build_layout(h->emb, h->emb.fmax, kLayoutPT, &h->lay);
  if (st != SQA_OK) {
    delete h;
    return st;
  }
  h->R = p.temps;
  h->F = h->emb.fmax;
  h->sweeps = p.sweeps;
  h->sps = p.sweeps_per_swap;
  h->seed = p.seed;
  h->betas = pt_betas(p.beta_min, p.beta_max, p.temps);
  const int64_t dmax = swap_table_width(h->betas, 2 * static_cast<int64_t>(h->emb.emax));
  if (dmax + 1 > kMaxSwapRow) {
    delete h;
    return fail(SQA_ERR_UNSUPPORTED, "swap table too wide (energy range too large for equal temperatures)");
  }
  h->Dmax = static_cast<int32_t>(dmax);
  h->mtab = pt_metropolis_table(h->betas, h->F);
  pt_phases(h->emb, h->lay, h->F, &h->nph, h->ph);
  h->stab = pt_swap_table(h->betas, h->Dmax);
  h->swap_falling = true;
  for (int32_t r = 0; r + 1 < h->R; ++r)
    for (int32_t D = 1; D <= h->Dmax; ++D)
      if (h->stab[static_cast<size_t>(r) * (h->Dmax + 1) + D] > h->stab[static_cast<size_t>(r) * (h->Dmax + 1) + D - 1])
        h->swap_falling = false;
  h->spack = pt_swap_pack(h->stab, h->R, h->Dmax);
  const int n = h->emb.n;
  const size_t nt = h->emb.terms.size();
  Arena &A = h->arena;
  h->off_rec = A.take(h->lay.rec.size() * 4);
  h->off_devof = A.take(static_cast<size_t>(n) * 2);
  h->off_hfield = A.take(static_cast<size_t>(n) * 4);
  h->off_tw = A.take(std::max<size_t>(nt, 1) * 4);
  h->off_ts = A.take(std::max<size_t>(nt, 1) * 8);
  h->off_mtab = A.take(h->mtab.size() * 4);
  h->off_stab = A.take(h->stab.size() * 4);
  h->off_spack = A.take(h->spack.size() * 4);
  h->off_spins = A.take(static_cast<size_t>(h->R) * n);
  h->off_energy = A.take(static_cast<size_t>(h->R) * 4);
  h->off_repat = A.take(static_cast<size_t>(h->R) * 4);
  h->off_acc = A.take(64 * 8);
  A.size = A.used;
  hipError_t e = hipMalloc(&A.base, A.size);
  if (e != hipSuccess) {
    delete h;
    return hip_fail(e, "hipMalloc (PT handle)");
  }
  struct Up {
    size_t off;
    const void *ptr;
    size_t bytes;
  } ups[] = {{h->off_rec, h->lay.rec.data(), h->lay.rec.size() * 4},
             {h->off_devof, h->lay.dev_of.data(), static_cast<size_t>(n) * 2},
             {h->off_hfield, h->lay.hfield.data(), static_cast<size_t>(n) * 4},
             {h->off_tw, h->lay.term_w.data(), nt * 4},
             {h->off_ts, h->lay.term_s.data(), nt * 8},
             {h->off_mtab, h->mtab.data(), h->mtab.size() * 4},
             {h->off_stab, h->stab.data(), h->stab.size() * 4},
             {h->off_spack, h->spack.data(), h->spack.size() * 4}};
  for (const Up &u : ups) {
    if (!u.bytes) continue;
    e = hipMemcpy(A.at<char>(u.off), u.ptr, u.bytes, hipMemcpyHostToDevice);
    if (e != hipSuccess) break;
  }
  if (e == hipSuccess) e = hipMemset(A.at<char>(h->off_acc), 0, 64 * 8);
  if (e == hipSuccess) e = hipEventCreateWithFlags(&h->done, hipEventDisableTiming);
  if (e != hipSuccess) {
    (void)hipFree(A.base);
    delete h;
    return hip_fail(e, "PT handle setup");
  }
  *out = h;
  return SQA_OK;
}

sqa_status pt_run_handle(pt_handle *h, void *stream) {
  if (!h) return fail(SQA_ERR_INVALID, "null handle");
  if (h->poisoned) return fail(SQA_ERR_DEVICE, "handle is poisoned");
  return pt_launch({h}, static_cast<hipStream_t>(stream));
}

sqa_status pt_run_batch(pt_handle *const *handles, int32_t count, void *stream) {
  if (!handles || count < 1) return fail(SQA_ERR_INVALID, "bad batch arguments");
  std::vector<pt_handle *> hs(handles, handles + count);
  for (pt_handle *h : hs) {
    if (!h) return fail(SQA_ERR_INVALID, "null handle");
    if (h->poisoned) return fail(SQA_ERR_DEVICE, "handle is poisoned");
  }
  return pt_launch(hs, static_cast<hipStream_t>(stream));
}

sqa_status pt_read(pt_handle *h, int8_t *spins_out, size_t spins_len, int32_t *energies_out,
                   int32_t *slot_to_replica_out, uint64_t *swap_accepts_out) {
  if (!h) return fail(SQA_ERR_INVALID, "null handle");
  if (!h->ran) return fail(SQA_ERR_INVALID, "run the handle first");
  hipError_t e = hipEventSynchronize(h->done);
  if (e != hipSuccess) return hip_fail(e, "hipEventSynchronize");
  const int R = h->R, n = h->emb.n;
  std::vector<int8_t> sp(static_cast<size_t>(R) * n);
  std::vector<int32_t> E(R), rep(R);
  std::vector<uint64_t> acc(64);
  e = hipMemcpy(sp.data(), h->arena.at<void>(h->off_spins), sp.size(), hipMemcpyDeviceToHost);
  if (e == hipSuccess) e = hipMemcpy(E.data(), h->arena.at<void>(h->off_energy), R * 4, hipMemcpyDeviceToHost);
  if (e == hipSuccess) e = hipMemcpy(rep.data(), h->arena.at<void>(h->off_repat), R * 4, hipMemcpyDeviceToHost);
  if (e == hipSuccess) e = hipMemcpy(acc.data(), h->arena.at<void>(h->off_acc), 64 * 8, hipMemcpyDeviceToHost);
  if (e != hipSuccess) return hip_fail(e, "hipMemcpy (PT results)");
  if (spins_out) {
    if (spins_len < sp.size()) return fail(SQA_ERR_INVALID, "spin buffer too short");
    for (int slot = 0; slot < R; ++slot)
      std::memcpy(spins_out + static_cast<size_t>(slot) * n, sp.data() + static_cast<size_t>(rep[slot]) * n, n);
  }
  if (energies_out)
    for (int slot = 0; slot < R; ++slot) energies_out[slot] = E[rep[slot]];
  if (slot_to_replica_out) std::memcpy(slot_to_replica_out, rep.data(), R * 4);
  if (swap_accepts_out)
    for (int r = 0; r + 1 < R; ++r) swap_accepts_out[r] = acc[r];
  return SQA_OK;
}

void pt_destroy(pt_handle *h) {
  if (!h) return;
  if (h->done) {
    (void)hipEventSynchronize(h->done);
    (void)hipEventDestroy(h->done);
  }
  if (h->arena.base) (void)hipFree(h->arena.base);
  delete h;
}

sqa_status pt_run(const sqa_problem *problem, const sqa_embedding *embedding, const pt_params *params, void *stream,
                  int8_t *spins_out, size_t spins_len, int32_t *energies_out, int32_t *slot_to_replica_out,
                  uint64_t *swap_accepts_out) {
  pt_handle *h = nullptr;
  sqa_status st = pt_create(problem, embedding, params, &h);
  if (st != SQA_OK) return st;
  st = pt_run_handle(h, stream);
  if (st == SQA_OK) st = pt_read(h, spins_out, spins_len, energies_out, slot_to_replica_out, swap_accepts_out);
  pt_destroy(h);
  return st;
}

}  // extern "C"
