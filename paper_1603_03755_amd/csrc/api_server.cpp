// C ABI: continuous-batching anneal server.
//
// Jobs wait in FIFO order and are admitted while the sum of their device
// bytes stays within the budget and a slot is free.  All admitted jobs
// advance together: each device launch runs the next `chunk` sweeps of every
// resident job in one persistent kernel (counter-based random numbers make a
// split anneal bit-identical to an uninterrupted one).  A job that reaches its
// last sweep gets its energies, is copied to the host, and releases its slot
// and memory before the next launch, where waiting jobs join.
#include <chrono>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <map>
#include <mutex>
#include <thread>
#include <vector>

#include "host_core.h"

using namespace sqa;
using Clock = std::chrono::steady_clock;

namespace {

struct Job {
  uint64_t ticket = 0;
  std::vector<int32_t> J, h;
  bool has_h = false;
  sqa_problem prob{};
  sqa_embedding emb{};
  sqa_schedule sched{};
  std::vector<double> gamma, bscale;
  size_t bytes = 0;
  sqa_handle *handle = nullptr;
  int next = 0;
  bool done = false;
  sqa_status status = SQA_OK;
  std::vector<int8_t> spins;
  std::vector<int32_t> energies;
  Clock::time_point t_submit, t_done;
};

// Device bytes of a job: spins, energies, table, records and terms.
size_t estimate_bytes(const Embedded &e, const sqa_schedule &s) {
  const size_t n = e.n, R = s.replicas, L = s.slices, M = s.sweeps;
  const size_t F = e.fmax;
  const size_t rw = rec_words_of(e.kind);
  size_t b = R * L * n + R * L * 4 + n * (rw * 4 + 6) + e.terms.size() * 12;
  if (s.move == SQA_MOVE_WOLFF)
    b += M * 4 + (s.bscale ? M : 1) * (2 * L * F + 1) * 4;   // join thresholds, acceptance rows
  else
    b += M * 3 * (2 * F + 1) * 4;
  b += static_cast<size_t>(e.N) * e.N * 4 + R * (e.N + 4) + 4096;
  return b;
}

}  // namespace

struct sqa_server {
  size_t budget = 0;
  int max_slots = 0;
  int chunk = 0;
  std::mutex mu;
  std::condition_variable cv_work, cv_done;
  std::deque<Job *> waiting;
  std::vector<Job *> active;
  std::map<uint64_t, Job *> jobs;
  uint64_t next_ticket = 1;
  size_t resident = 0, peak = 0;
  uint64_t completed = 0, launches = 0;
  bool stop = false;
  hipStream_t stream = nullptr;
  void *scratch = nullptr;
  size_t scratch_bytes = 0;
  int device = 0;
  std::thread worker;

  void loop();
};

void sqa_server::loop() {
  (void)hipSetDevice(device);
  for (;;) {
    std::vector<Job *> admit;
    {
      std::unique_lock<std::mutex> lk(mu);
      cv_work.wait(lk, [&] { return stop || !waiting.empty() || !active.empty(); });
      if (stop) return;
      while (!waiting.empty() && static_cast<int>(active.size() + admit.size()) < max_slots &&
             resident + waiting.front()->bytes <= budget) {
        Job *j = waiting.front();
        waiting.pop_front();
        resident += j->bytes;
        admit.push_back(j);
      }
      peak = std::max(peak, resident);
    }
    for (Job *j : admit) {
      sqa_status st = sqa_create(&j->prob, &j->emb, &j->sched, &j->handle);
      std::lock_guard<std::mutex> lk(mu);
      if (st != SQA_OK) {
        j->status = st;
        j->done = true;
        j->t_done = Clock::now();
        resident -= j->bytes;
        cv_done.notify_all();
      } else {
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
      const int M = j->sched.sweeps;
      const int a = j->next, b = std::min(M, j->next + chunk);
      hs.push_back(j->handle);
      m0.push_back(a);
      m1.push_back(b);
      fl.push_back((a == 0 ? kFlagInit : 0) | (b == M ? kFlagEnergy : 0));
    }
    sqa_status st = run_handles(hs, m0, m1, fl, stream, &scratch, &scratch_bytes);
    std::vector<Job *> finished;
    for (size_t i = 0; i < act.size(); ++i) {
      Job *j = act[i];
      if (st != SQA_OK) {
        j->status = st;
        finished.push_back(j);
        continue;
      }
      j->next = m1[i];
      if (j->next == j->sched.sweeps) {
        const size_t ns = static_cast<size_t>(j->sched.replicas) * j->sched.slices * sqa_physical_sites(j->emb.kind, j->prob.n);
        j->spins.resize(ns);
        j->energies.resize(static_cast<size_t>(j->sched.replicas) * j->sched.slices);
        sqa_status s1 = sqa_read_spins(j->handle, j->spins.data(), j->spins.size());
        sqa_status s2 = sqa_read_energies(j->handle, j->energies.data(), j->energies.size());
        j->status = s1 != SQA_OK ? s1 : s2;
        finished.push_back(j);
      }
    }
    std::lock_guard<std::mutex> lk(mu);
    ++launches;
    for (Job *j : finished) {
      sqa_destroy(j->handle);
      j->handle = nullptr;
      resident -= j->bytes;
      j->done = true;
      j->t_done = Clock::now();
      ++completed;
      active.erase(std::find(active.begin(), active.end(), j));
    }
    if (!finished.empty()) cv_done.notify_all();
  }
}

extern "C" {

sqa_status sqa_server_create(size_t hbm_budget_bytes, int32_t max_slots, int32_t chunk_sweeps, sqa_server **out) {
  if (!out || hbm_budget_bytes == 0 || max_slots < 1 || chunk_sweeps < 1) return fail(SQA_ERR_INVALID, "bad server arguments");
  sqa_server *s = new (std::nothrow) sqa_server();
  if (!s) return fail(SQA_ERR_OOM, "host allocation");
  s->budget = hbm_budget_bytes;
  s->max_slots = max_slots;
  s->chunk = chunk_sweeps;
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
                             const sqa_schedule *schedule, uint64_t *ticket) {
  if (!s || !problem || !embedding || !schedule || !ticket || !problem->J) return fail(SQA_ERR_INVALID, "null argument");
  const sqa_schedule &sc = *schedule;
  if (sc.slices < 1 || (sc.slices > 1 && (sc.slices & 1)) || sc.slices > 64 || sc.sweeps < 1 || sc.replicas < 1 ||
      sc.replicas > 65536 || !(sc.beta > 0) || (sc.move != SQA_MOVE_METROPOLIS && sc.move != SQA_MOVE_WOLFF))
    return fail(SQA_ERR_INVALID, "bad schedule");
  Embedded e;
  sqa_status st = build_embedding(*problem, *embedding, &e);
  if (st != SQA_OK) return st;
  Job *j = new (std::nothrow) Job();
  if (!j) return fail(SQA_ERR_OOM, "host allocation");
  const int N = problem->n;
  j->J.assign(problem->J, problem->J + static_cast<size_t>(N) * N);
  j->has_h = problem->h != nullptr;
  if (j->has_h) j->h.assign(problem->h, problem->h + N);
  j->prob.n = N;
  j->prob.J = j->J.data();
  j->prob.h = j->has_h ? j->h.data() : nullptr;
  j->emb = *embedding;
  j->sched = sc;
  if (sc.gamma) {
    j->gamma.assign(sc.gamma, sc.gamma + sc.sweeps);
    j->sched.gamma = j->gamma.data();
  }
  if (sc.bscale) {
    j->bscale.assign(sc.bscale, sc.bscale + sc.sweeps);
    j->sched.bscale = j->bscale.data();
  }
  j->bytes = estimate_bytes(e, sc);
  if (j->bytes > s->budget) {
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
  return j->status;
}

sqa_status sqa_server_result(sqa_server *s, uint64_t ticket, int8_t *spins, size_t spins_len, int32_t *energies,
                             size_t energies_len, double *latency_s) {
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
    return fail(st, "job failed on the device");
  }
  if ((spins && spins_len < j->spins.size()) || (energies && energies_len < j->energies.size()))
    return fail(SQA_ERR_INVALID, "result buffer too short");
  if (spins) std::memcpy(spins, j->spins.data(), j->spins.size());
  if (energies) std::memcpy(energies, j->energies.data(), j->energies.size() * 4);
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
  for (Job *j : s->active)
    if (j->handle) sqa_destroy(j->handle);
  for (auto &kv : s->jobs) delete kv.second;
  if (s->scratch) (void)hipFree(s->scratch);
  if (s->stream) (void)hipStreamDestroy(s->stream);
  delete s;
}

}  // extern "C"
