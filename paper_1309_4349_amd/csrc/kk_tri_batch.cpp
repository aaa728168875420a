// kk_tri_batch.cpp -- many triangular lattices (replicas) advanced together.
//
// Replicas on the conflict-free class schedule whose whole ring fits one
// workgroup's LDS are "resident" when the batch holds at least
// kMinResident of them: one launch per run gives each its own workgroup,
// which runs all of the replica's sweeps with no halo.  Other class-schedule
// replicas whose lattice takes a whole-sweep tile are "tiled": every sweep of
// a run is one launch whose workgroups are the (replica, tile) jobs of all
// tiled replicas that still have sweeps to make.  Tiled replicas are ordered
// by their sweep count, longest first, so the jobs of sweep k are a prefix of
// one job table.  The rest (literal MPKK, lattices too small for a tile) run
// through their own launches on the same stream.  No replica index enters a
// random counter, so every replica ends exactly where kk_sweep would have
// left it.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <new>
#include <numeric>
#include <vector>

#include "../../include/kk.h"
#include "kk_host.hpp"
#include "kk_kernels.hpp"
#include "kk_tri.hpp"

using namespace kk;

namespace {
constexpr size_t kMinResident = 64;  // resident replicas fill a quarter of the CUs at least
}

struct kk_tri_batch {
  std::vector<kk_sim*> sims;
  std::vector<uint64_t> sweeps;
  hipStream_t stream = nullptr;
  bool own_stream = false;
  bool poisoned = false;
  std::vector<size_t> res;       // resident replicas
  size_t res_lds = 0;            // largest resident ring
  TriResidentRep* d_res = nullptr;
  std::vector<size_t> order;     // tiled replicas, sweeps descending
  std::vector<uint32_t> tw, tr;  // their tiles, fixed at creation (the job table depends on them)
  std::vector<size_t> plain;     // the others
  std::vector<size_t> job_end;   // jobs of order[0..i] = [0, job_end[i])
  size_t lds_bytes = 0;          // largest window of the batched replicas
  TriBatchRep* d_reps = nullptr;
  uint2* d_jobs = nullptr;
};

namespace {

#define TB_HIP(expr)                                                                              \
  do {                                                                                            \
    hipError_t e_ = (expr);                                                                       \
    if (e_ != hipSuccess) {                                                                       \
      b->poisoned = true;                                                                         \
      return set_error(KK_EDEVICE, "%s failed: %s (%s:%d)", #expr, hipGetErrorString(e_), __FILE__, \
                       __LINE__);                                                                 \
    }                                                                                             \
  } while (0)

void free_tri_batch(kk_tri_batch* b) {
  for (kk_sim* h : b->sims) kk_destroy(h);
  b->sims.clear();
  if (b->d_reps) (void)hipFree(b->d_reps);
  if (b->d_res) (void)hipFree(b->d_res);
  if (b->d_jobs) (void)hipFree(b->d_jobs);
  if (b->own_stream && b->stream) (void)hipStreamDestroy(b->stream);
}

}  // namespace

extern "C" {

kk_status kk_tri_batch_create(kk_tri_batch** out, const kk_tri_replica* reps, size_t n, void* hip_stream) {
  if (!out) return set_error(KK_EINVAL, "out is NULL");
  *out = nullptr;
  if (!reps || n == 0) return set_error(KK_EINVAL, "need at least one replica");
  for (size_t i = 0; i < n; ++i) {
    if (reps[i].start != KK_START_RANDOM && reps[i].start != KK_START_SEGREGATED)
      return set_error(KK_EINVAL, "replica %zu: unknown start %u", i, reps[i].start);
    if (reps[i].sweeps > 0x7FFFFFFFull) return set_error(KK_EINVAL, "replica %zu: at most 2^31-1 sweeps", i);
  }
  kk_tri_batch* b = new (std::nothrow) kk_tri_batch();
  if (!b) return set_error(KK_ENOMEM, "host allocation failed");
  auto fail = [&](kk_status st) {
    free_tri_batch(b);
    delete b;
    return st;
  };
  if (hip_stream) {
    b->stream = static_cast<hipStream_t>(hip_stream);
  } else {
    hipError_t e = hipStreamCreateWithFlags(&b->stream, hipStreamNonBlocking);
    if (e != hipSuccess) return fail(set_error(KK_EDEVICE, "hipStreamCreate failed: %s", hipGetErrorString(e)));
    b->own_stream = true;
  }
  for (size_t i = 0; i < n; ++i) {
    const kk_tri_replica& r = reps[i];
    kk_sim* h = nullptr;
    kk_status st = kk_create_triangular_ex(&h, r.L, r.H, r.scheme, r.composition, r.omega_kT, r.seed, b->stream);
    if (st != KK_OK) return fail(set_error(st, "replica %zu: %s", i, kk_last_error()));  // formats before storing
    b->sims.push_back(h);
    b->sweeps.push_back(r.sweeps);
    if (r.start != KK_START_RANDOM) {
      st = kk_restart(h, r.start);
      if (st != KK_OK) return fail(st);
    }
  }
  size_t fits = 0;
  for (const kk_sim* h : b->sims) fits += h->geom == 1 && tri_resident_fits(h->L, h->H);
  for (size_t i = 0; i < n; ++i) {
    const kk_sim* h = b->sims[i];
    const bool whole = h->tri_tw == h->L && h->tri_tr == h->H;
    if (h->geom == 1 && fits >= kMinResident && tri_resident_fits(h->L, h->H)) {
      b->res.push_back(i);
      b->res_lds = std::max(b->res_lds, (size_t)h->L * (size_t)h->H);
    } else if (h->geom == 1 && h->tri_tw > 0 && !whole) {
      b->order.push_back(i);
    } else {
      b->plain.push_back(i);
    }
  }
  if (!b->res.empty()) {
    const kk_status st = device_alloc((void**)&b->d_res, b->res.size() * sizeof(TriResidentRep));
    if (st != KK_OK) return fail(st);
  }
  std::stable_sort(b->order.begin(), b->order.end(),
                   [&](size_t a, size_t c) { return b->sweeps[a] > b->sweeps[c]; });
  // the job table: replica order, tiles in order
  std::vector<uint2> jobs;
  for (size_t k = 0; k < b->order.size(); ++k) {
    const kk_sim* h = b->sims[b->order[k]];
    b->tw.push_back((uint32_t)h->tri_tw);
    b->tr.push_back((uint32_t)h->tri_tr);
    const uint32_t ntx = (uint32_t)((h->L + h->tri_tw - 1) / h->tri_tw);
    const uint32_t nty = (uint32_t)((h->H + h->tri_tr - 1) / h->tri_tr);
    for (uint32_t t = 0; t < ntx * nty; ++t) jobs.push_back(make_uint2((uint32_t)k, t));
    b->job_end.push_back(jobs.size());
    b->lds_bytes = std::max(b->lds_bytes, tri_window_bytes((uint32_t)h->tri_tw, (uint32_t)h->tri_tr));
  }
  if (!b->order.empty()) {
    kk_status st = device_alloc((void**)&b->d_reps, b->order.size() * sizeof(TriBatchRep));
    if (st == KK_OK) st = device_alloc((void**)&b->d_jobs, jobs.size() * sizeof(uint2));
    if (st != KK_OK) return fail(st);
    hipError_t e = hipMemcpyAsync(b->d_jobs, jobs.data(), jobs.size() * sizeof(uint2), hipMemcpyHostToDevice,
                                  b->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(b->stream);
    if (e != hipSuccess) return fail(set_error(KK_EDEVICE, "job table upload: %s", hipGetErrorString(e)));
  }
  *out = b;
  return KK_OK;
}

namespace {
kk_status tri_batch_run(kk_tri_batch* b);
}

kk_status kk_tri_batch_run(kk_tri_batch* b) {
  if (!b) return set_error(KK_EINVAL, "NULL batch");
  if (b->poisoned) return set_error(KK_ESTATE, "batch poisoned by an earlier error");
  const kk_status st = tri_batch_run(b);
  // a run that fails part way leaves the replicas' device and host state apart
  if (st != KK_OK && b->poisoned)
    for (kk_sim* h : b->sims) h->poisoned = true;
  return st;
}

}  // extern "C"

namespace {
kk_status tri_batch_run(kk_tri_batch* b) {
  for (size_t i = 0; i < b->sims.size(); ++i) {
    const kk_sim* h = b->sims[i];
    if (h->poisoned) return set_error(KK_ESTATE, "replica %zu poisoned", i);
    if (h->t + b->sweeps[i] >= ((uint64_t)1 << 60)) return set_error(KK_EINVAL, "sweep counter overflow");
  }
  // every replica's stream is the batch stream, so the order below is the order on the device
  std::vector<TriResidentRep> res_reps(b->res.size());  // alive until the final synchronisation
  if (!b->res.empty()) {
    std::vector<TriResidentRep>& reps = res_reps;
    for (size_t k = 0; k < b->res.size(); ++k) {
      kk_sim* h = b->sims[b->res[k]];
      TriResidentRep& R = reps[k];
      R.lat = static_cast<uint8_t*>(h->lat[h->cur]);
      R.L = (uint32_t)h->L;
      R.H = (uint32_t)h->H;
      R.sweeps = (uint32_t)b->sweeps[b->res[k]];
      R.k0 = h->k0;
      R.k1 = h->k1;
      R.t0 = h->t;
      R.acc = h->tacc;
      R.partials = h->partials;
    }
    TB_HIP(hipMemcpyAsync(b->d_res, reps.data(), reps.size() * sizeof(TriResidentRep), hipMemcpyHostToDevice,
                          b->stream));
    TB_HIP(launch_tri_resident(b->d_res, (uint32_t)b->res.size(), b->res_lds, b->stream));
    for (size_t i : b->res) {
      kk_sim* h = b->sims[i];
      h->t += b->sweeps[i];
      h->attempts += b->sweeps[i] * (uint64_t)h->L * (uint64_t)h->H;
      if (b->sweeps[i]) h->epoch += 1;
    }
  }
  std::vector<TriBatchRep> tile_reps(b->order.size());  // alive until the final synchronisation
  if (!b->order.empty()) {
    std::vector<TriBatchRep>& reps = tile_reps;
    uint64_t mx = 0;
    for (size_t k = 0; k < b->order.size(); ++k) {
      kk_sim* h = b->sims[b->order[k]];
      TriBatchRep& R = reps[k];
      R.lat[0] = static_cast<uint8_t*>(h->lat[0]);
      R.lat[1] = static_cast<uint8_t*>(h->lat[1]);
      R.L = (uint32_t)h->L;
      R.H = (uint32_t)h->H;
      // the tile of the job table, whatever the handle's own setting is now (results do not depend on it)
      R.TW = b->tw[k];
      R.TR = b->tr[k];
      R.ntx = (R.L + R.TW - 1) / R.TW;
      R.cur = (uint32_t)h->cur;
      R.k0 = h->k0;
      R.k1 = h->k1;
      R.t0 = h->t;
      R.acc = h->tacc;
      R.partials = h->partials;
      mx = std::max(mx, b->sweeps[b->order[k]]);
    }
    TB_HIP(hipMemcpyAsync(b->d_reps, reps.data(), reps.size() * sizeof(TriBatchRep), hipMemcpyHostToDevice,
                          b->stream));
    // sweep k: the replicas with more than k sweeps, a prefix of `order`
    size_t active = b->order.size();
    for (uint64_t k = 0; k < mx; ++k) {
      while (active > 0 && b->sweeps[b->order[active - 1]] <= k) --active;
      TB_HIP(launch_tri_tile_sweep_batch(b->d_reps, b->d_jobs, (uint32_t)b->job_end[active - 1], (uint32_t)k,
                                         b->lds_bytes, b->stream));
    }
    for (size_t k = 0; k < b->order.size(); ++k) {
      kk_sim* h = b->sims[b->order[k]];
      const uint64_t s = b->sweeps[b->order[k]];
      h->t += s;
      h->attempts += s * (uint64_t)h->L * (uint64_t)h->H;
      h->cur ^= (int)(s & 1u);
      if (s) h->epoch += 1;
    }
  }
  for (size_t i : b->plain) {
    const kk_status st = kk_sweep_async(b->sims[i], b->sweeps[i]);
    if (st != KK_OK) {
      b->poisoned = true;
      return st;
    }
  }
  TB_HIP(hipStreamSynchronize(b->stream));
  return KK_OK;
}
}  // namespace

extern "C" {

kk_status kk_tri_batch_sim(kk_tri_batch* b, size_t i, kk_sim** sim_out) {
  if (!b || !sim_out) return set_error(KK_EINVAL, "NULL argument");
  if (i >= b->sims.size()) return set_error(KK_EINVAL, "replica %zu out of range (%zu)", i, b->sims.size());
  *sim_out = b->sims[i];
  return KK_OK;
}

kk_status kk_tri_batch_info(kk_tri_batch* b, size_t* n_resident, size_t* n_batched, size_t* n_plain,
                            size_t* n_jobs) {
  if (!b) return set_error(KK_EINVAL, "NULL batch");
  if (n_resident) *n_resident = b->res.size();
  if (n_batched) *n_batched = b->order.size();
  if (n_plain) *n_plain = b->plain.size();
  if (n_jobs) *n_jobs = b->job_end.empty() ? 0 : b->job_end.back();
  return KK_OK;
}

void kk_tri_batch_destroy(kk_tri_batch* b) {
  if (!b) return;
  free_tri_batch(b);
  delete b;
}

}  // extern "C"
