// kk_serve.cpp -- a job server over the batch engine: simulation jobs arrive
// at any time, wait in a FIFO queue until their device memory fits an HBM
// budget, and are advanced together in steps of at most chunk_sweeps sweeps
// (continuous batching: jobs join and leave between steps, never inside one).
// A finished job's N_AB, energy and cluster histogram of species 1 are taken
// on the device and kept on the host until released.  Because no slot or
// replica index enters any random counter, each job's result equals what
// kk_create_ex + kk_sweep(job.sweeps) gives alone.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <deque>
#include <map>
#include <new>
#include <vector>

#include "../../include/kk.h"
#include "kk_host.hpp"

using namespace kk;

namespace {

struct Job {
  uint64_t id = 0;
  kk_replica spec{};
  kk_sim* sim = nullptr;
  uint64_t done_sweeps = 0;
  size_t footprint = 0;
  double t_arrival = 0, t_admit = 0, t_done = 0;
  kk_status status = KK_OK;
  uint64_t accepted = 0, n_unlike = 0;
  double energy = 0;
  std::vector<kk_hist_entry> hist;
  std::vector<uint8_t> lattice;
};

using Clock = std::chrono::steady_clock;

}  // namespace

struct kk_server {
  kk_server_config cfg{};
  Clock::time_point t0;
  hipStream_t stream = nullptr;
  bool own_stream = false;
  kk_batch* batch = nullptr;
  std::deque<Job*> queue;
  std::vector<Job*> active;
  std::deque<Job*> unpolled;          // finished, not yet returned by kk_server_poll
  std::map<uint64_t, Job*> finished;  // finished, not yet released
  bool dirty = true;                  // active set changed since the batch was planned
  uint64_t next_id = 1;
  kk_server_stats stats{};
  bool poisoned = false;
};

namespace {

double now_s(const kk_server* s) { return std::chrono::duration<double>(Clock::now() - s->t0).count(); }

int resolve_layout(const kk_replica& r) {
  if (r.layout == KK_LAYOUT_AUTO) return r.L % 32 == 0 ? KK_LAYOUT_BITPACKED : KK_LAYOUT_INT8;
  return (int)r.layout;
}

// Upper bound of the device bytes a job's handle holds at any time.  Always:
// two lattice buffers, the energy counters and one accepted-move sum per
// sweep tile.  On top, the larger of the two phases that need scratch:
// placement (8-byte keys per site and the radix tables, freed after it) and
// retirement (the cluster-labelling arrays, 8 bytes per site plus the size
// tables, and for a bit-packed lattice kept on the host the N-byte unpack
// buffer of kk_get_lattice, taken while the labelling arrays are still held).
// 64 KiB of slack covers the job's share of the batch tables.
size_t job_footprint(const kk_replica& r, bool keep_lattice) {
  const int layout = resolve_layout(r);
  const size_t N = (size_t)r.L * r.L;
  const size_t lat = layout == KK_LAYOUT_BITPACKED ? N / 8 : N;
  TileConfig tc;
  kk::default_tile((int)r.L, layout == KK_LAYOUT_BITPACKED ? kk::kLayoutBits : kk::kLayoutInt8, &tc);
  SweepParams p{};
  kk::tile_geometry((int)r.L, tc, &p);
  const size_t tiles = (size_t)p.tiles_x * (size_t)(((int)r.L + p.th - 1) / p.th);
  const size_t base = 2 * lat + 2 * sizeof(unsigned long long) + tiles * sizeof(unsigned long long);
  const size_t placement = 8 * N + (256 + 1 + 4096) * sizeof(unsigned);
  const size_t labelling = 8 * N + kk::kSmallSizes * sizeof(unsigned) + 4 * (N / 4096 + 1) + sizeof(unsigned) +
                           ((keep_lattice && layout == KK_LAYOUT_BITPACKED) ? N : 0);
  return base + std::max(placement, labelling) + (64u << 10);
}

void destroy_job(Job* j) {
  if (j->sim) kk_destroy(j->sim);
  delete j;
}

// Finish a job: observables, optional lattice copy, device memory released.
void retire(kk_server* s, Job* j) {
  kk_status st = j->status;
  if (st == KK_OK) {
    uint64_t sw = 0, att = 0;
    st = kk_stats(j->sim, &sw, &att, &j->accepted);
  }
  if (st == KK_OK) st = kk_energy(j->sim, &j->n_unlike, &j->energy);
  if (st == KK_OK) {
    size_t n = 0;
    st = kk_cluster_hist(j->sim, 1, nullptr, 0, &n);
    if (st == KK_OK || st == KK_ETRUNC) {
      j->hist.resize(n);
      st = kk_cluster_hist(j->sim, 1, j->hist.data(), n, &n);
    }
  }
  if (st == KK_OK && s->cfg.keep_lattice) {
    j->lattice.resize((size_t)j->spec.L * j->spec.L);
    st = kk_get_lattice(j->sim, j->lattice.data(), j->lattice.size());
  }
  j->status = st;
  if (j->sim) {
    kk_destroy(j->sim);
    j->sim = nullptr;
  }
  s->stats.bytes_in_use -= j->footprint;
  j->t_done = now_s(s);
  s->stats.completed += 1;
  s->unpolled.push_back(j);
  s->finished[j->id] = j;
}

// Admit queued jobs in arrival order while they fit the budget and the slots.
void admit(kk_server* s) {
  while (!s->queue.empty() && s->active.size() < s->cfg.max_active) {
    Job* j = s->queue.front();
    if (s->stats.bytes_in_use + j->footprint > s->cfg.hbm_budget_bytes) break;
    s->queue.pop_front();
    s->stats.bytes_in_use += j->footprint;
    s->stats.peak_bytes = std::max(s->stats.peak_bytes, s->stats.bytes_in_use);
    s->stats.admitted += 1;
    j->t_admit = now_s(s);
    j->status = kk_create_ex(&j->sim, j->spec.L, j->spec.composition, j->spec.omega_kT, j->spec.seed,
                             j->spec.layout, s->stream);
    if (j->status == KK_OK && j->spec.start != KK_START_RANDOM) j->status = kk_restart(j->sim, j->spec.start);
    if (j->status != KK_OK || j->spec.sweeps == 0) {
      retire(s, j);  // a job that cannot be placed (or has nothing to run) finishes at once
      continue;
    }
    s->active.push_back(j);
    s->dirty = true;
  }
}

}  // namespace

extern "C" {

kk_status kk_server_create(kk_server** out, const kk_server_config* cfg) {
  if (!out) return set_error(KK_EINVAL, "out is NULL");
  *out = nullptr;
  kk_server* s = new (std::nothrow) kk_server();
  if (!s) return set_error(KK_ENOMEM, "host allocation failed");
  if (cfg) s->cfg = *cfg;
  if (s->cfg.max_active == 0) s->cfg.max_active = 256;
  if (s->cfg.chunk_sweeps == 0) s->cfg.chunk_sweeps = 1000;
  if (s->cfg.chunk_sweeps > 0x7FFFFFFFull) {
    delete s;
    return set_error(KK_EINVAL, "chunk_sweeps must be below 2^31");
  }
  hipError_t e;
  if (s->cfg.hbm_budget_bytes == 0) {
    size_t fr = 0, tot = 0;
    if ((e = hipMemGetInfo(&fr, &tot)) != hipSuccess) {
      delete s;
      return set_error(KK_EDEVICE, "hipMemGetInfo: %s", hipGetErrorString(e));
    }
    s->cfg.hbm_budget_bytes = fr / 4 * 3;
  }
  s->stats.budget = s->cfg.hbm_budget_bytes;
  if (s->cfg.hip_stream) s->stream = static_cast<hipStream_t>(s->cfg.hip_stream);
  else {
    if ((e = hipStreamCreateWithFlags(&s->stream, hipStreamNonBlocking)) != hipSuccess) {
      delete s;
      return set_error(KK_EDEVICE, "stream: %s", hipGetErrorString(e));
    }
    s->own_stream = true;
  }
  kk_status st = batch_over({}, {}, s->stream, &s->batch);
  if (st != KK_OK) {
    if (s->own_stream) (void)hipStreamDestroy(s->stream);
    delete s;
    return st;
  }
  s->t0 = Clock::now();
  *out = s;
  return KK_OK;
}

kk_status kk_server_job_bytes(const kk_replica* job, uint32_t keep_lattice, uint64_t* bytes) {
  if (!job || !bytes) return set_error(KK_EINVAL, "NULL argument");
  if (job->L < 4 || job->L % 4 != 0 || job->L > 32768)
    return set_error(KK_EINVAL, "L must be a multiple of 4 in [4, 32768] (got %u)", job->L);
  if (job->layout > KK_LAYOUT_BITPACKED) return set_error(KK_EINVAL, "unknown layout %u", job->layout);
  if (job->layout == KK_LAYOUT_BITPACKED && job->L % 32 != 0)
    return set_error(KK_EINVAL, "bit-packed layout needs L %% 32 == 0 (got %u)", job->L);
  *bytes = job_footprint(*job, keep_lattice != 0);
  return KK_OK;
}

kk_status kk_server_now(kk_server* s, double* t) {
  if (!s || !t) return set_error(KK_EINVAL, "NULL argument");
  *t = now_s(s);
  return KK_OK;
}

kk_status kk_server_submit(kk_server* s, const kk_replica* job, double arrival_s, uint64_t* job_id) {
  if (!s || !job) return set_error(KK_EINVAL, "NULL argument");
  if (s->poisoned) return set_error(KK_ESTATE, "server poisoned by an earlier error");
  if (job->L < 4 || job->L % 4 != 0 || job->L > 32768)
    return set_error(KK_EINVAL, "L must be a multiple of 4 in [4, 32768] (got %u)", job->L);
  if (!(job->composition >= 0.0 && job->composition <= 1.0))
    return set_error(KK_EINVAL, "composition must lie in [0, 1]");
  if (!std::isfinite(job->omega_kT)) return set_error(KK_EINVAL, "omega must be finite");
  if (job->layout > KK_LAYOUT_BITPACKED) return set_error(KK_EINVAL, "unknown layout %u", job->layout);
  if (job->layout == KK_LAYOUT_BITPACKED && job->L % 32 != 0)
    return set_error(KK_EINVAL, "bit-packed layout needs L %% 32 == 0 (got %u)", job->L);
  if (job->sweeps >= ((uint64_t)1 << 60)) return set_error(KK_EINVAL, "too many sweeps");
  if (job->start != KK_START_RANDOM && job->start != KK_START_SEGREGATED)
    return set_error(KK_EINVAL, "unknown start %u", job->start);
  const size_t fp = job_footprint(*job, s->cfg.keep_lattice != 0);
  if (fp > s->cfg.hbm_budget_bytes)
    return set_error(KK_ENOMEM, "job needs %zu device bytes, budget is %llu", fp,
                     (unsigned long long)s->cfg.hbm_budget_bytes);
  Job* j = new (std::nothrow) Job();
  if (!j) return set_error(KK_ENOMEM, "host allocation failed");
  j->id = s->next_id++;
  j->spec = *job;
  j->footprint = fp;
  j->t_arrival = arrival_s >= 0.0 ? arrival_s : now_s(s);
  s->queue.push_back(j);
  s->stats.submitted += 1;
  if (job_id) *job_id = j->id;
  return KK_OK;
}

kk_status kk_server_step(kk_server* s, size_t* n_active, size_t* n_queued) {
  if (!s) return set_error(KK_EINVAL, "NULL server");
  if (s->poisoned) return set_error(KK_ESTATE, "server poisoned by an earlier error");
  admit(s);
  if (!s->active.empty()) {
    std::vector<kk_sim*> sims;
    std::vector<uint64_t> sweeps;
    for (Job* j : s->active) {
      sims.push_back(j->sim);
      sweeps.push_back(std::min<uint64_t>(s->cfg.chunk_sweeps, j->spec.sweeps - j->done_sweeps));
    }
    kk_status st = s->dirty ? batch_replan(s->batch, sims, sweeps) : batch_set_sweeps(s->batch, sweeps);
    if (st == KK_OK) {
      s->dirty = false;
      const auto t0 = Clock::now();
      st = kk_batch_run(s->batch);
      s->stats.gpu_busy_s += std::chrono::duration<double>(Clock::now() - t0).count();
    }
    if (st != KK_OK) {
      s->poisoned = true;
      return st;
    }
    s->stats.steps += 1;
    std::vector<Job*> still;
    for (size_t i = 0; i < s->active.size(); ++i) {
      Job* j = s->active[i];
      j->done_sweeps += sweeps[i];
      s->stats.attempts += sweeps[i] * (uint64_t)j->spec.L * j->spec.L;
      if (j->done_sweeps >= j->spec.sweeps) {
        retire(s, j);
        s->dirty = true;
      } else {
        still.push_back(j);
      }
    }
    s->active.swap(still);
    admit(s);  // freed memory goes to waiting jobs before the caller returns
  }
  if (n_active) *n_active = s->active.size();
  if (n_queued) *n_queued = s->queue.size();
  return KK_OK;
}

kk_status kk_server_poll(kk_server* s, kk_job_result* out, size_t cap, size_t* n_out) {
  if (!s || !n_out) return set_error(KK_EINVAL, "NULL argument");
  if (cap > 0 && !out) return set_error(KK_EINVAL, "out is NULL with cap > 0");
  size_t n = 0;
  while (n < cap && !s->unpolled.empty()) {
    const Job* j = s->unpolled.front();
    s->unpolled.pop_front();
    kk_job_result& r = out[n++];
    r.id = j->id;
    r.status = (int32_t)j->status;
    r.L = j->spec.L;
    r.sweeps = j->done_sweeps;
    r.attempts = j->done_sweeps * (uint64_t)j->spec.L * j->spec.L;
    r.accepted = j->accepted;
    r.n_unlike = j->n_unlike;
    r.energy_kT = j->energy;
    r.t_arrival = j->t_arrival;
    r.t_admit = j->t_admit;
    r.t_done = j->t_done;
    r.hist_entries = j->hist.size();
  }
  *n_out = n;
  return KK_OK;
}

kk_status kk_server_job_hist(kk_server* s, uint64_t job_id, kk_hist_entry* out, size_t cap, size_t* n_out) {
  if (!s || !n_out) return set_error(KK_EINVAL, "NULL argument");
  auto it = s->finished.find(job_id);
  if (it == s->finished.end()) return set_error(KK_EINVAL, "job %llu is not finished or was released",
                                                (unsigned long long)job_id);
  const std::vector<kk_hist_entry>& h = it->second->hist;
  *n_out = h.size();
  if (cap < h.size()) return set_error(KK_ETRUNC, "histogram has %zu entries, cap %zu", h.size(), cap);
  if (!h.empty() && !out) return set_error(KK_EINVAL, "out is NULL");
  std::copy(h.begin(), h.end(), out);
  return KK_OK;
}

kk_status kk_server_job_lattice(kk_server* s, uint64_t job_id, uint8_t* out, size_t n) {
  if (!s || !out) return set_error(KK_EINVAL, "NULL argument");
  auto it = s->finished.find(job_id);
  if (it == s->finished.end()) return set_error(KK_EINVAL, "job %llu is not finished or was released",
                                                (unsigned long long)job_id);
  const std::vector<uint8_t>& lat = it->second->lattice;
  if (lat.empty()) return set_error(KK_ESTATE, "lattice not kept (keep_lattice = 0 or the job failed)");
  if (n != lat.size()) return set_error(KK_EINVAL, "buffer holds %zu sites, lattice has %zu", n, lat.size());
  std::copy(lat.begin(), lat.end(), out);
  return KK_OK;
}

kk_status kk_server_release(kk_server* s, uint64_t job_id) {
  if (!s) return set_error(KK_EINVAL, "NULL server");
  auto it = s->finished.find(job_id);
  if (it == s->finished.end()) return set_error(KK_EINVAL, "job %llu is not finished or was released",
                                                (unsigned long long)job_id);
  Job* j = it->second;
  if (std::find(s->unpolled.begin(), s->unpolled.end(), j) != s->unpolled.end())
    return set_error(KK_ESTATE, "job %llu has not been polled yet", (unsigned long long)job_id);
  s->finished.erase(it);
  destroy_job(j);
  return KK_OK;
}

kk_status kk_server_get_stats(kk_server* s, kk_server_stats* out) {
  if (!s || !out) return set_error(KK_EINVAL, "NULL argument");
  *out = s->stats;
  out->queued = s->queue.size();
  out->active = s->active.size();
  return KK_OK;
}

void kk_server_destroy(kk_server* s) {
  if (!s) return;
  if (s->batch) kk_batch_destroy(s->batch);  // borrowed sims stay alive here
  for (Job* j : s->queue) destroy_job(j);
  for (Job* j : s->active) destroy_job(j);
  for (auto& kv : s->finished) destroy_job(kv.second);
  if (s->own_stream && s->stream) {
    (void)hipStreamSynchronize(s->stream);
    (void)hipStreamDestroy(s->stream);
  }
  delete s;
}

}  // extern "C"
