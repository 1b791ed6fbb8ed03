// C ABI: continuous-batching anneal server.
//
// Jobs wait in FIFO order and are admitted while the sum of their device
// bytes stays within the budget and a slot is free.  A job's handle is
// prepared on the submitting thread (embedding, layout, tables: host only),
// so its device bytes are known exactly before admission; its device block is
// allocated when it is admitted.  All admitted jobs advance together: each
// device launch runs the next `chunk` sweeps of every resident job in one
// persistent kernel (counter-based random numbers make a split anneal
// bit-identical to an uninterrupted one).  A job that reaches its last sweep
// gets its energies, is decoded on the device, is copied to the host, and
// releases its slot and memory before the next launch, where waiting jobs
// join.
#include <algorithm>
#include <chrono>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <map>
#include <mutex>
#include <new>
#include <thread>
#include <vector>

#include "host_core.h"

using namespace sqa;
using Clock = std::chrono::steady_clock;

namespace {

struct Job {
  uint64_t ticket = 0;
  sqa_handle *handle = nullptr;     // prepared at submit, uploaded at admission
  bool uploaded = false;
  sqa_decode_params dec{};
  std::vector<int32_t> trees;       // copy of dec.tree_parents
  size_t bytes = 0;                 // device bytes charged while resident
  int next = 0;                     // first sweep of the next chunk
  bool running = false;
  bool cancel = false;              // cancel at the next launch boundary
  bool done = false;
  sqa_status status = SQA_OK;
  std::vector<int8_t> spins, logical;
  std::vector<int32_t> energies, lenergy;
  Clock::time_point t_submit, t_done;
};

// The decoder a job runs when it finishes: the caller's, or majority vote of
// the chains (ME kinds) / minimum-weight decoding (LHZ, n <= 32) / chain-tree
// decoding (LHZ above), on slice 0.
sqa_status job_decoder(Job *j, const sqa_decode_params *p, int kind, int n, int L) {
  sqa_decode_params d{};
  d.error_rate = 0.2;
  d.iterations = 10;
  if (p) {
    d = *p;
    d.tree_parents = nullptr;
    if (p->tree_parents && p->n_trees > 0) j->trees.assign(p->tree_parents, p->tree_parents + static_cast<size_t>(p->n_trees) * n);
  } else if (kind == SQA_EMB_LHZ) {
    d.decoder = n <= 32 ? SQA_DEC_LHZ_MWD : SQA_DEC_LHZ_TREES;
    if (d.decoder == SQA_DEC_LHZ_TREES) {      // Eq. (A1): parent(v) = v - 1
      d.n_trees = 1;
      j->trees.resize(n);
      for (int v = 0; v < n; ++v) j->trees[v] = v - 1;
    }
  } else {
    d.decoder = SQA_DEC_ME_MAJORITY;
  }
  if (d.readout_slice < 0 || d.readout_slice >= L) return fail(SQA_ERR_INVALID, "readout slice out of range");
  const bool me = kind == SQA_EMB_ME || kind == SQA_EMB_ME_CHIMERA;
  if (d.decoder == SQA_DEC_ME_MAJORITY ? !me : (kind != SQA_EMB_LHZ || d.decoder < SQA_DEC_LHZ_TREES ||
                                                d.decoder > SQA_DEC_LHZ_BP))
    return fail(SQA_ERR_INVALID, "decoder does not fit the embedding");
  if ((d.decoder == SQA_DEC_LHZ_MWD && n > 32) || (d.decoder == SQA_DEC_LHZ_MLD && n > 24) ||
      (d.decoder == SQA_DEC_LHZ_BP && n > 32))
    return fail(SQA_ERR_UNSUPPORTED, "decoder above its size limit");
  if ((d.decoder == SQA_DEC_LHZ_MLD || d.decoder == SQA_DEC_LHZ_BP) && !(d.error_rate > 0.0 && d.error_rate < 0.5))
    return fail(SQA_ERR_INVALID, "error rate must be in (0, 1/2)");
  const bool trees = d.decoder == SQA_DEC_LHZ_TREES || d.decoder == SQA_DEC_LHZ_BP;
  if (trees && j->trees.empty()) return fail(SQA_ERR_INVALID, "tree decoding needs tree parents");
  if (trees && !p) d.n_trees = 1;
  d.tree_parents = j->trees.empty() ? nullptr : j->trees.data();
  j->dec = d;
  return SQA_OK;
}

}  // namespace

struct sqa_server {
  size_t budget = 0;
  int max_slots = 0;
  int chunk = 0;
  sqa_allocator alloc{};
  std::mutex mu;
  std::condition_variable cv_work, cv_done;
  std::deque<Job *> waiting;
  std::vector<Job *> active;
  std::map<uint64_t, Job *> jobs;
  uint64_t next_ticket = 1;
  size_t resident = 0, peak = 0;     // charged bytes of the resident jobs (launch scratch's fixed part included)
  uint64_t completed = 0, launches = 0;
  bool stop = false;
  hipStream_t stream = nullptr;
  void *scratch = nullptr;
  size_t scratch_bytes = 0;
  int device = 0;
  std::thread worker;

  void loop();
  void finish(Job *j, sqa_status st);   // under mu
};

void sqa_server::finish(Job *j, sqa_status st) {
  if (j->handle) {
    sqa_destroy(j->handle);
    j->handle = nullptr;
  }
  if (j->running) {
    resident -= j->bytes;
    active.erase(std::find(active.begin(), active.end(), j));
    j->running = false;
  }
  j->status = st;
  j->done = true;
  j->t_done = Clock::now();
  if (st == SQA_OK) ++completed;
}

void sqa_server::loop() {
  (void)hipSetDevice(device);
  for (;;) {
    std::vector<Job *> admit;
    {
      std::unique_lock<std::mutex> lk(mu);
      cv_work.wait(lk, [&] { return stop || !waiting.empty() || !active.empty(); });
      if (stop) return;
      // cancellations of running jobs take effect at this launch boundary
      bool any = false;
      for (Job *j : std::vector<Job *>(active))
        if (j->cancel) {
          finish(j, SQA_ERR_CANCELLED);
          any = true;
        }
      if (any) cv_done.notify_all();
      while (!waiting.empty() && static_cast<int>(active.size() + admit.size()) < max_slots &&
             resident + waiting.front()->bytes <= budget) {
        Job *j = waiting.front();
        waiting.pop_front();
        resident += j->bytes;
        j->running = true;
        admit.push_back(j);
      }
      peak = std::max(peak, resident);
    }
    for (Job *j : admit) {
      sqa_status st = handle_upload(j->handle, &alloc);
      std::lock_guard<std::mutex> lk(mu);
      if (st != SQA_OK) {
        resident -= j->bytes;
        j->running = false;
        finish(j, st);
        cv_done.notify_all();
      } else {
        j->uploaded = true;
        active.push_back(j);
      }
    }
    std::vector<sqa_handle *> hs;
    std::vector<int> m0, m1, fl;
    std::vector<Job *> act;
    {
      std::lock_guard<std::mutex> lk(mu);
      act = active;
    }
    if (act.empty()) continue;
    for (Job *j : act) {
      const int M = j->handle->M;
      const int a = j->next, b = std::min(M, j->next + chunk);
      hs.push_back(j->handle);
      m0.push_back(a);
      m1.push_back(b);
      fl.push_back((a == 0 ? kFlagInit : 0) | (b == M ? kFlagEnergy : 0));
    }
    // the scratch holds no more than the resident set's bound (admission charged that)
    if (scratch_bytes > launch_scratch_bytes(hs)) {
      device_free(&alloc, scratch);
      scratch = nullptr;
      scratch_bytes = 0;
    }
    sqa_status st = run_handles(hs, m0, m1, fl, stream, &alloc, &scratch, &scratch_bytes);
    std::vector<std::pair<Job *, sqa_status>> finished;
    for (size_t i = 0; i < act.size(); ++i) {
      Job *j = act[i];
      if (st != SQA_OK) {
        finished.push_back({j, st});
        continue;
      }
      j->next = m1[i];
      if (j->next == j->handle->M) {
        sqa_handle *h = j->handle;
        const size_t ns = static_cast<size_t>(h->R) * h->L * h->emb.n;
        j->spins.resize(ns);
        j->energies.resize(static_cast<size_t>(h->R) * h->L);
        j->logical.resize(static_cast<size_t>(h->R) * h->N);
        j->lenergy.resize(h->R);
        sqa_status s1 = sqa_read_spins(h, j->spins.data(), j->spins.size());
        if (s1 == SQA_OK) s1 = sqa_read_energies(h, j->energies.data(), j->energies.size());
        if (s1 == SQA_OK) s1 = sqa_decode_ex(h, &j->dec, j->logical.data(), j->lenergy.data(), stream);
        finished.push_back({j, s1});
      }
    }
    std::lock_guard<std::mutex> lk(mu);
    ++launches;
    for (auto &f : finished) finish(f.first, f.second);
    if (!finished.empty()) cv_done.notify_all();
  }
}

extern "C" {

sqa_status sqa_server_create(size_t hbm_budget_bytes, int32_t max_slots, int32_t chunk_sweeps,
                             const sqa_allocator *allocator, sqa_server **out) {
  if (!out || hbm_budget_bytes == 0 || max_slots < 1 || chunk_sweeps < 1) return fail(SQA_ERR_INVALID, "bad server arguments");
  *out = nullptr;
  if (allocator && (!allocator->alloc || !allocator->free))
    return fail(SQA_ERR_INVALID, "an allocator needs both callbacks");
  sqa_server *s = new (std::nothrow) sqa_server();
  if (!s) return fail(SQA_ERR_OOM, "host allocation");
  s->budget = hbm_budget_bytes;
  s->max_slots = max_slots;
  s->chunk = chunk_sweeps;
  if (allocator) s->alloc = *allocator;
  s->resident = kLaunchScratchFixed;
  (void)hipGetDevice(&s->device);
  hipError_t e = hipStreamCreateWithFlags(&s->stream, hipStreamNonBlocking);
  if (e != hipSuccess) {
    delete s;
    return hip_fail(e, "hipStreamCreate");
  }
  s->worker = std::thread([s] { s->loop(); });
  *out = s;
  return SQA_OK;
}

sqa_status sqa_server_submit(sqa_server *s, const sqa_problem *problem, const sqa_embedding *embedding,
                             const sqa_schedule *schedule, const sqa_decode_params *decode, uint64_t *ticket) {
  if (!s || !problem || !embedding || !schedule || !ticket) return fail(SQA_ERR_INVALID, "null argument");
  Job *j = new (std::nothrow) Job();
  if (!j) return fail(SQA_ERR_OOM, "host allocation");
  sqa_status st;
  try {
    st = handle_prepare(*problem, *embedding, *schedule, &j->handle);
    if (st == SQA_OK) st = job_decoder(j, decode, embedding->kind, problem->n, schedule->slices);
  } catch (const std::bad_alloc &) {
    st = fail(SQA_ERR_OOM, "host allocation (job)");
  }
  if (st != SQA_OK) {
    sqa_destroy(j->handle);
    delete j;
    return st;
  }
  const sqa_handle *h = j->handle;
  j->bytes = round_granule(handle_block_bytes(h)) + round_granule(decode_scratch_bytes(h, j->dec.decoder, j->trees.size())) +
             launch_scratch_share(h);
  if (j->bytes + kLaunchScratchFixed > s->budget) {
    sqa_destroy(j->handle);
    delete j;
    return fail(SQA_ERR_BUSY, "job alone exceeds the device-memory budget");
  }
  j->t_submit = Clock::now();
  {
    std::lock_guard<std::mutex> lk(s->mu);
    j->ticket = s->next_ticket++;
    s->jobs[j->ticket] = j;
    s->waiting.push_back(j);
  }
  s->cv_work.notify_one();
  *ticket = j->ticket;
  return SQA_OK;
}

sqa_status sqa_server_job_bytes(sqa_server *s, uint64_t ticket, size_t *bytes_out) {
  if (!s || !bytes_out) return fail(SQA_ERR_INVALID, "null argument");
  std::lock_guard<std::mutex> lk(s->mu);
  auto it = s->jobs.find(ticket);
  if (it == s->jobs.end()) return fail(SQA_ERR_INVALID, "unknown ticket");
  *bytes_out = it->second->bytes;
  return SQA_OK;
}

sqa_status sqa_server_cancel(sqa_server *s, uint64_t ticket) {
  if (!s) return fail(SQA_ERR_INVALID, "null server");
  std::lock_guard<std::mutex> lk(s->mu);
  auto it = s->jobs.find(ticket);
  if (it == s->jobs.end()) return fail(SQA_ERR_INVALID, "unknown ticket");
  Job *j = it->second;
  if (j->done) return fail(SQA_ERR_INVALID, "job already finished");
  auto w = std::find(s->waiting.begin(), s->waiting.end(), j);
  if (w != s->waiting.end()) {
    s->waiting.erase(w);
    s->finish(j, SQA_ERR_CANCELLED);      // a waiting job holds no device memory
    s->cv_done.notify_all();
  } else {
    j->cancel = true;                     // running: dropped at the next launch boundary
    s->cv_work.notify_one();
  }
  return SQA_OK;
}

sqa_status sqa_server_poll(sqa_server *s, uint64_t ticket, int32_t *done) {
  if (!s || !done) return fail(SQA_ERR_INVALID, "null argument");
  std::lock_guard<std::mutex> lk(s->mu);
  auto it = s->jobs.find(ticket);
  if (it == s->jobs.end()) return fail(SQA_ERR_INVALID, "unknown ticket");
  *done = it->second->done ? 1 : 0;
  return SQA_OK;
}

sqa_status sqa_server_wait(sqa_server *s, uint64_t ticket, int32_t timeout_ms) {
  if (!s) return fail(SQA_ERR_INVALID, "null server");
  std::unique_lock<std::mutex> lk(s->mu);
  auto it = s->jobs.find(ticket);
  if (it == s->jobs.end()) return fail(SQA_ERR_INVALID, "unknown ticket");
  Job *j = it->second;
  if (timeout_ms < 0) {
    s->cv_done.wait(lk, [&] { return j->done; });
  } else if (!s->cv_done.wait_for(lk, std::chrono::milliseconds(timeout_ms), [&] { return j->done; })) {
    return fail(SQA_ERR_NOT_READY, "job not finished");
  }
  if (j->status == SQA_ERR_CANCELLED) return fail(SQA_ERR_CANCELLED, "job was cancelled");
  if (j->status != SQA_OK) return fail(j->status, "job failed");
  return SQA_OK;
}

sqa_status sqa_server_result(sqa_server *s, uint64_t ticket, int8_t *spins, size_t spins_len, int32_t *energies,
                             size_t energies_len, int8_t *logical, size_t logical_len, int32_t *logical_energies,
                             size_t logical_energies_len, double *latency_s) {
  if (!s) return fail(SQA_ERR_INVALID, "null server");
  std::lock_guard<std::mutex> lk(s->mu);
  auto it = s->jobs.find(ticket);
  if (it == s->jobs.end()) return fail(SQA_ERR_INVALID, "unknown ticket");
  Job *j = it->second;
  if (!j->done) return fail(SQA_ERR_NOT_READY, "job not finished");
  if (j->status != SQA_OK) {
    sqa_status st = j->status;
    s->jobs.erase(it);
    delete j;
    return fail(st, st == SQA_ERR_CANCELLED ? "job was cancelled" : "job failed on the device");
  }
  if ((spins && spins_len < j->spins.size()) || (energies && energies_len < j->energies.size()) ||
      (logical && logical_len < j->logical.size()) || (logical_energies && logical_energies_len < j->lenergy.size()))
    return fail(SQA_ERR_INVALID, "result buffer too short");
  if (spins) std::memcpy(spins, j->spins.data(), j->spins.size());
  if (energies) std::memcpy(energies, j->energies.data(), j->energies.size() * 4);
  if (logical) std::memcpy(logical, j->logical.data(), j->logical.size());
  if (logical_energies) std::memcpy(logical_energies, j->lenergy.data(), j->lenergy.size() * 4);
  if (latency_s) *latency_s = std::chrono::duration<double>(j->t_done - j->t_submit).count();
  s->jobs.erase(it);
  delete j;
  return SQA_OK;
}

sqa_status sqa_server_stats(sqa_server *s, uint64_t *completed, uint64_t *launches, uint64_t *peak_bytes) {
  if (!s) return fail(SQA_ERR_INVALID, "null server");
  std::lock_guard<std::mutex> lk(s->mu);
  if (completed) *completed = s->completed;
  if (launches) *launches = s->launches;
  if (peak_bytes) *peak_bytes = s->peak;
  return SQA_OK;
}

void sqa_server_destroy(sqa_server *s) {
  if (!s) return;
  {
    std::lock_guard<std::mutex> lk(s->mu);
    s->stop = true;
  }
  s->cv_work.notify_all();
  if (s->worker.joinable()) s->worker.join();
  for (auto &kv : s->jobs) {
    if (kv.second->handle) sqa_destroy(kv.second->handle);
    delete kv.second;
  }
  device_free(&s->alloc, s->scratch);
  if (s->stream) (void)hipStreamDestroy(s->stream);
  delete s;
}

}  // extern "C"
