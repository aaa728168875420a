// kk_batch.cpp -- many independent lattices (replicas) of uneven size,
// composition and omega advanced together on one GPU.
//
// Replicas whose whole lattice fits one workgroup (L % 32 == 0, 64 <= L <=
// 32 * kResidentMaxC) are "resident": one persistent launch gives each its own
// workgroup, which keeps the lattice in LDS for all of its sweeps.  The others
// are "tiled": they are split into a few groups of equal work, and for each
// group every sweep is one launch over all of the group's halo tiles.
// Resident replicas of at most kResidentSmallMaxC words per row run in
// 256-thread workgroups (three per CU), larger ones in 768-thread workgroups.
// One HIP graph holds a chunk of kBatchChunk sweeps of everything: a branch
// per tile group (kBatchChunk chained launches) and a branch per resident
// kernel (one launch of kBatchChunk sweeps), forked from and joined to one
// stream; the graph is replayed once per chunk.  Branches of one graph run
// concurrently, which separate streams replaying their own graphs did not
// do here (measured).  No slot or replica index
// enters any random counter, so every replica ends exactly where kk_sweep
// would have left it.
//
// The streams live as long as the batch; the plan (tables, graphs) is rebuilt
// whenever the replica set changes, which the job server does between steps.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cstring>
#include <new>
#include <vector>

#include "../../include/kk.h"
#include "kk_host.hpp"
#include "kk_kernels.hpp"
#include "kk_ccl.hpp"

using namespace kk;

namespace {
constexpr int kMaxTileGroups = 4;
// sweep hand-off words (two each): one per tile group, then the small and the
// large resident launch
constexpr int kCtlSlots = kMaxTileGroups + 2, kCtlSmall = kMaxTileGroups, kCtlLarge = kMaxTileGroups + 1;
// tile workgroups that fill the device once (256 CUs, two per CU)
constexpr size_t kFillWorkgroups = 512;
}

struct kk_batch {
  std::vector<kk_sim*> sims;
  std::vector<uint64_t> sweeps;
  bool own_sims = true;
  int tile_th = kBatchTh;        // largest tile height of tiled replicas (rows, even)
  int tile_tww = kBatchMaxTww / 2;  // largest tile width of tiled replicas (words)
  int tile_ku = 2;                  // units per thread of the tile kernel (1 or 2)
  // streams and events, created once
  hipStream_t sA = nullptr, sB = nullptr;  // large resident launch; uploads and joins
  hipStream_t sC = nullptr;                 // small resident launch
  bool own_sB = false;
  hipEvent_t ev_upload = nullptr, ev_res = nullptr;
  hipStream_t tg_stream[kMaxTileGroups] = {};
  // batched labelling (kk_batch_cluster_hists), made on first use: the table
  // of lattices, the staging rows of the result blocks and their pinned image
  CclRep* d_ccl = nullptr;
  uint32_t* d_hist_stage = nullptr;
  uint32_t* h_hist_stage = nullptr;
  hipEvent_t tg_done[kMaxTileGroups] = {};
  // plan, rebuilt by batch_plan
  std::vector<int> resident, tiled;
  size_t n_small = 0;  // resident[0, n_small) run in the small kernel, the rest in the large one
  std::vector<size_t> count_off, count_n;
  size_t ncounts = 0;
  std::vector<int> tg_off, tg_n;  // tiled groups: slices of the tile-job table
  std::vector<int> job_rep;       // host copy: replica of every tile job
  hipGraph_t graph = nullptr;     // one chunk of kBatchChunk sweeps of every branch
  hipGraphExec_t gexec = nullptr;
  hipEvent_t ev_fork = nullptr;
  SweepParams* d_params = nullptr;
  BatchTileJob* d_jobs = nullptr;
  int njobs = 0;
  int* d_res = nullptr;
  size_t res_lds = 0, small_lds = 0;
  unsigned* d_ctl = nullptr;
  unsigned long long* d_counts = nullptr;
  bool poisoned = false;
};

namespace {

#define KB_HIP(expr)                                                                              \
  do {                                                                                            \
    hipError_t e_ = (expr);                                                                       \
    if (e_ != hipSuccess) {                                                                       \
      b->poisoned = true;                                                                         \
      return set_error(KK_EDEVICE, "%s failed: %s (%s:%d)", #expr, hipGetErrorString(e_), __FILE__, \
                       __LINE__);                                                                 \
    }                                                                                             \
  } while (0)

bool is_resident(const kk_sim* h) { return h->L % 32 == 0 && h->L >= 64 && h->L / 32 <= kResidentMaxC; }

void clear_plan(kk_batch* b) {
  if (b->gexec) (void)hipGraphExecDestroy(b->gexec);
  if (b->graph) (void)hipGraphDestroy(b->graph);
  b->gexec = nullptr;
  b->graph = nullptr;
  for (void* p : {(void*)b->d_params, (void*)b->d_jobs, (void*)b->d_res, (void*)b->d_ctl, (void*)b->d_counts})
    if (p) (void)hipFree(p);
  b->d_params = nullptr;
  b->d_jobs = nullptr;
  b->d_res = nullptr;
  b->d_ctl = nullptr;
  b->d_counts = nullptr;
  b->resident.clear();
  b->tiled.clear();
  b->count_off.clear();
  b->count_n.clear();
  b->ncounts = 0;
  b->tg_off.clear();
  b->tg_n.clear();
  b->job_rep.clear();
  b->njobs = 0;
  b->res_lds = 0;
  b->small_lds = 0;
  b->n_small = 0;
}

void free_batch(kk_batch* b) {
  clear_plan(b);
  if (b->own_sims)
    for (kk_sim* h : b->sims) kk_destroy(h);
  b->sims.clear();
  for (int g = 0; g < kMaxTileGroups; ++g) {
    if (b->tg_stream[g]) (void)hipStreamDestroy(b->tg_stream[g]);
    if (b->tg_done[g]) (void)hipEventDestroy(b->tg_done[g]);
  }
  if (b->ev_upload) (void)hipEventDestroy(b->ev_upload);
  if (b->ev_res) (void)hipEventDestroy(b->ev_res);
  if (b->ev_fork) (void)hipEventDestroy(b->ev_fork);
  if (b->sA) (void)hipStreamDestroy(b->sA);
  if (b->sC) (void)hipStreamDestroy(b->sC);
  if (b->d_ccl) (void)hipFree(b->d_ccl);
  if (b->d_hist_stage) (void)hipFree(b->d_hist_stage);
  if (b->h_hist_stage) (void)hipHostFree(b->h_hist_stage);
  if (b->own_sB && b->sB) (void)hipStreamDestroy(b->sB);
}

kk_status make_streams(kk_batch* b, void* hip_stream) {
  hipError_t e;
  if (hip_stream) b->sB = static_cast<hipStream_t>(hip_stream);
  else {
    if ((e = hipStreamCreateWithFlags(&b->sB, hipStreamNonBlocking)) != hipSuccess)
      return set_error(KK_EDEVICE, "stream: %s", hipGetErrorString(e));
    b->own_sB = true;
  }
  if ((e = hipStreamCreateWithFlags(&b->sA, hipStreamNonBlocking)) != hipSuccess ||
      (e = hipStreamCreateWithFlags(&b->sC, hipStreamNonBlocking)) != hipSuccess ||
      (e = hipEventCreateWithFlags(&b->ev_upload, hipEventDisableTiming)) != hipSuccess ||
      (e = hipEventCreateWithFlags(&b->ev_res, hipEventDisableTiming)) != hipSuccess ||
      (e = hipEventCreateWithFlags(&b->ev_fork, hipEventDisableTiming)) != hipSuccess)
    return set_error(KK_EDEVICE, "stream/event: %s", hipGetErrorString(e));
  for (int g = 0; g < kMaxTileGroups; ++g)
    if ((e = hipStreamCreateWithFlags(&b->tg_stream[g], hipStreamNonBlocking)) != hipSuccess ||
        (e = hipEventCreateWithFlags(&b->tg_done[g], hipEventDisableTiming)) != hipSuccess)
      return set_error(KK_EDEVICE, "stream/event: %s", hipGetErrorString(e));
  return KK_OK;
}

// Geometry of a replica's batch launch (resident: whole lattice; tiled: tiles
// of max_tww (8 or 16) words by at most max_th rows).
void batch_geometry(const kk_sim* h, bool resident, int max_tww, int max_th, int ku, SweepParams* p) {
  TileConfig tc;
  if (resident) {
    tc.cyclic = true;
    tc.tww = h->L / 32;
    tc.th = h->L;
  } else {
    // tiles max_tww (8 or 16) words wide, the last column possibly ragged, and
    // balanced heights of at most max_th rows that fit one workgroup
    int ty = (h->L + max_th - 1) / max_th;
    tc.cyclic = false;
    tc.tww = max_tww;
    tc.th = std::min(h->L, (((h->L + ty - 1) / ty) + 1) & ~1);
    while (!batch_tile_fits(tc.tww, tc.th, ku)) {  // more rows of tiles until one fits a workgroup
      ++ty;
      tc.th = std::min(h->L, (((h->L + ty - 1) / ty) + 1) & ~1);
    }
  }
  tc.ku = resident ? 2 : ku;
  tile_geometry(h->L, tc, p);
  p->k0 = h->k0;
  p->k1 = h->k1;
  p->acc = h->acc;
  p->layout = h->layout;
}


// Plan the current replica set: resident list, tile jobs split into groups of
// equal work, device tables and one captured graph per group.
kk_status batch_plan(kk_batch* b) {
  clear_plan(b);
  const size_t n = b->sims.size();
  if (n == 0) return KK_OK;
  std::vector<BatchTileJob> jobs;
  for (size_t i = 0; i < n; ++i) {
    kk_sim* h = b->sims[i];
    const bool res = is_resident(h);
    SweepParams p{};
    batch_geometry(h, res, b->tile_tww, b->tile_th, b->tile_ku, &p);
    const size_t tiles = res ? 1 : (size_t)p.tiles_x * (size_t)((h->L + p.th - 1) / p.th);
    b->count_off.push_back(b->ncounts);
    b->count_n.push_back(tiles);
    b->ncounts += tiles;
    if (res) {
      b->resident.push_back((int)i);
      if (h->L / 32 <= kResidentSmallMaxC) b->small_lds = std::max(b->small_lds, batch_resident_lds_bytes(h->L));
      else b->res_lds = std::max(b->res_lds, batch_resident_lds_bytes(h->L));
    } else {
      b->tiled.push_back((int)i);
    }
  }
  // small resident replicas first (their own launch), then the large ones,
  // each part widest first (the widest run longest)
  std::stable_sort(b->resident.begin(), b->resident.end(), [&](int a, int c) {
    const bool sa = b->sims[a]->L / 32 <= kResidentSmallMaxC, sc = b->sims[c]->L / 32 <= kResidentSmallMaxC;
    if (sa != sc) return sa;
    return b->sims[a]->L > b->sims[c]->L;
  });
  for (int i : b->resident) b->n_small += b->sims[i]->L / 32 <= kResidentSmallMaxC;
  // longest-processing-time split of the tiled replicas by work per run.  Two
  // tile chains fill each other's launch tails when the tiles can fill the
  // device; fewer tiles run best as one chain.  Graph branches run
  // concurrently only up to the device's hardware queues (four): the two tile
  // chains plus at most two resident launches stay within that (measured: a
  // fifth branch serialises behind another).
  size_t tile_jobs = 0;
  for (int i : b->tiled) tile_jobs += b->count_n[i];
  const int ngroups = (int)std::min<size_t>(tile_jobs >= kFillWorkgroups ? 2 : 1, b->tiled.size());
  std::vector<std::vector<int>> groups(ngroups);
  {
    std::vector<int> order = b->tiled;
    auto work = [&](int i) { return (double)b->sims[i]->L * b->sims[i]->L * (double)b->sweeps[i]; };
    std::stable_sort(order.begin(), order.end(), [&](int a, int c) { return work(a) > work(c); });
    std::vector<double> load(ngroups, 0.0);
    for (int i : order) {
      const int g = (int)(std::min_element(load.begin(), load.end()) - load.begin());
      groups[g].push_back(i);
      load[g] += work(i);
    }
  }
  std::vector<uint64_t> maxsw(ngroups, 0);
  for (int g = 0; g < ngroups; ++g) {
    b->tg_off.push_back((int)jobs.size());
    for (int i : groups[g]) {
      for (size_t t = 0; t < b->count_n[i]; ++t) jobs.push_back(BatchTileJob{i, (int)t});
      maxsw[g] = std::max(maxsw[g], b->sweeps[i]);
    }
    b->tg_n.push_back((int)jobs.size() - b->tg_off.back());
  }
  b->njobs = (int)jobs.size();
  for (const BatchTileJob& j : jobs) b->job_rep.push_back(j.rep);
  kk_status st = KK_OK;
  if (st == KK_OK) st = device_alloc((void**)&b->d_params, n * sizeof(SweepParams));
  if (st == KK_OK) st = device_alloc((void**)&b->d_ctl, 2 * sizeof(unsigned) * kCtlSlots);
  if (st == KK_OK) st = device_alloc((void**)&b->d_counts, b->ncounts * sizeof(unsigned long long));
  if (st == KK_OK && b->njobs) st = device_alloc((void**)&b->d_jobs, jobs.size() * sizeof(BatchTileJob));
  if (st == KK_OK && !b->resident.empty()) st = device_alloc((void**)&b->d_res, b->resident.size() * sizeof(int));
  if (st != KK_OK) return st;
  hipError_t e;
  if (b->njobs && (e = hipMemcpy(b->d_jobs, jobs.data(), jobs.size() * sizeof(BatchTileJob),
                                 hipMemcpyHostToDevice)) != hipSuccess)
    return set_error(KK_EDEVICE, "upload jobs: %s", hipGetErrorString(e));
  if (!b->resident.empty() && (e = hipMemcpy(b->d_res, b->resident.data(), b->resident.size() * sizeof(int),
                                             hipMemcpyHostToDevice)) != hipSuccess)
    return set_error(KK_EDEVICE, "upload ids: %s", hipGetErrorString(e));
  // one graph: fork from tile group 0's stream, a branch per tile group and
  // per resident launch, join back
  const size_t n_small = b->n_small, n_large = b->resident.size() - b->n_small;
  hipStream_t origin = b->tg_stream[0];
  if ((e = hipStreamBeginCapture(origin, hipStreamCaptureModeThreadLocal)) != hipSuccess)
    return set_error(KK_EDEVICE, "capture: %s", hipGetErrorString(e));
  std::vector<hipStream_t> branches;
  for (int g = 1; g < ngroups; ++g) branches.push_back(b->tg_stream[g]);
  if (n_small) branches.push_back(b->sC);
  if (n_large) branches.push_back(b->sA);
  e = hipEventRecord(b->ev_fork, origin);
  for (hipStream_t bs : branches)
    if (e == hipSuccess) e = hipStreamWaitEvent(bs, b->ev_fork, 0);
  for (int g = 0; g < ngroups && e == hipSuccess; ++g) {
    for (int r = 0; r < kBatchChunk && e == hipSuccess; ++r)
      e = launch_batch_tiles(b->d_params, b->d_jobs + b->tg_off[g], b->tg_n[g], b->d_ctl + 2 * g, (unsigned)r,
                             b->tile_ku, b->tg_stream[g]);
    if (e == hipSuccess) e = launch_batch_advance(b->d_ctl + 2 * g, (unsigned)kBatchChunk, b->tg_stream[g]);
  }
  if (e == hipSuccess && n_small) {
    e = launch_batch_resident(b->d_params, b->d_res, (int)n_small, b->small_lds, true, b->d_ctl + 2 * kCtlSmall, b->sC);
    if (e == hipSuccess) e = launch_batch_advance(b->d_ctl + 2 * kCtlSmall, (unsigned)kBatchChunk, b->sC);
  }
  if (e == hipSuccess && n_large) {
    e = launch_batch_resident(b->d_params, b->d_res + n_small, (int)n_large, b->res_lds, false,
                              b->d_ctl + 2 * kCtlLarge, b->sA);
    if (e == hipSuccess) e = launch_batch_advance(b->d_ctl + 2 * kCtlLarge, (unsigned)kBatchChunk, b->sA);
  }
  for (size_t i = 0; i < branches.size() && e == hipSuccess; ++i) {
    e = hipEventRecord(b->tg_done[i % kMaxTileGroups], branches[i]);
    if (e == hipSuccess) e = hipStreamWaitEvent(origin, b->tg_done[i % kMaxTileGroups], 0);
  }
  hipGraph_t graph = nullptr;
  const hipError_t ee = hipStreamEndCapture(origin, &graph);  // always end the capture
  if (e == hipSuccess) e = ee;
  b->graph = graph;
  if (e == hipSuccess) e = hipGraphInstantiate(&b->gexec, graph, nullptr, nullptr, 0);
  if (e != hipSuccess) return set_error(KK_EDEVICE, "batch graph: %s", hipGetErrorString(e));
  return KK_OK;
}

}  // namespace

namespace kk {

kk_status batch_replan(kk_batch* b, const std::vector<kk_sim*>& sims, const std::vector<uint64_t>& sweeps) {
  if (b->poisoned) return set_error(KK_ESTATE, "batch poisoned by an earlier error");
  if (sims.size() != sweeps.size()) return set_error(KK_EINVAL, "sims and sweeps differ in length");
  b->sims = sims;
  b->sweeps = sweeps;
  const kk_status st = batch_plan(b);
  if (st != KK_OK) b->poisoned = true;
  return st;
}

kk_status batch_over(const std::vector<kk_sim*>& sims, const std::vector<uint64_t>& sweeps, void* hip_stream,
                     kk_batch** out) {
  *out = nullptr;
  kk_batch* b = new (std::nothrow) kk_batch();
  if (!b) return set_error(KK_ENOMEM, "host allocation failed");
  b->own_sims = false;
  kk_status st = make_streams(b, hip_stream);
  if (st == KK_OK) st = batch_replan(b, sims, sweeps);
  if (st != KK_OK) {
    free_batch(b);
    delete b;
    return st;
  }
  *out = b;
  return KK_OK;
}

kk_status batch_set_sweeps(kk_batch* b, const std::vector<uint64_t>& sweeps) {
  if (sweeps.size() != b->sims.size()) return set_error(KK_EINVAL, "sweeps differ in length");
  b->sweeps = sweeps;
  return KK_OK;
}

}  // namespace kk

extern "C" {

kk_status kk_batch_create(kk_batch** out, const kk_replica* reps, size_t n, void* hip_stream) {
  if (!out) return set_error(KK_EINVAL, "out is NULL");
  *out = nullptr;
  if (!reps || n == 0) return set_error(KK_EINVAL, "need at least one replica");
  kk_batch* b = new (std::nothrow) kk_batch();
  if (!b) return set_error(KK_ENOMEM, "host allocation failed");
  auto fail = [&](kk_status st) {
    free_batch(b);
    delete b;
    return st;
  };
  kk_status st = make_streams(b, hip_stream);
  if (st != KK_OK) return fail(st);
  std::vector<kk_sim*> sims;
  std::vector<uint64_t> sweeps;
  for (size_t i = 0; i < n; ++i) {
    kk_sim* h = nullptr;
    if (reps[i].start != KK_START_RANDOM && reps[i].start != KK_START_SEGREGATED)
      return fail(set_error(KK_EINVAL, "replica %zu: unknown start %u", i, reps[i].start));
    st = kk_create_ex(&h, reps[i].L, reps[i].composition, reps[i].omega_kT, reps[i].seed, reps[i].layout, b->sB);
    if (st != KK_OK) return fail(st);
    b->sims.push_back(h);  // owned from here on, also if planning fails
    if (reps[i].start != KK_START_RANDOM) {
      st = kk_restart(h, reps[i].start);
      if (st != KK_OK) return fail(st);
    }
    sims.push_back(h);
    sweeps.push_back(reps[i].sweeps);
  }
  st = batch_replan(b, sims, sweeps);
  if (st != KK_OK) return fail(st);
  *out = b;
  return KK_OK;
}

kk_status kk_batch_run(kk_batch* b) {
  if (!b) return set_error(KK_EINVAL, "NULL batch");
  if (b->poisoned) return set_error(KK_ESTATE, "batch poisoned by an earlier error");
  const size_t n = b->sims.size();
  if (n == 0) return KK_OK;
  std::vector<SweepParams> params(n);
  std::vector<uint64_t> nsw(n);
  for (size_t i = 0; i < n; ++i) {
    kk_sim* h = b->sims[i];
    if (h->poisoned) return set_error(KK_ESTATE, "replica %zu poisoned", i);
    if (h->t + b->sweeps[i] >= ((uint64_t)1 << 60)) return set_error(KK_EINVAL, "sweep counter overflow");
    if (b->sweeps[i] > 0x7FFFFFFFull) return set_error(KK_EINVAL, "at most 2^31-1 sweeps per replica per run");
    const bool res = is_resident(h);
    SweepParams& p = params[i];
    batch_geometry(h, res, b->tile_tww, b->tile_th, b->tile_ku, &p);
    p.t0 = h->t;
    p.accepted = b->d_counts + b->count_off[i];
    // resident replicas sweep in place; tiled ones ping-pong src -> dst -> src ...
    p.src = h->lat[h->cur];
    p.dst = res ? h->lat[h->cur] : h->lat[h->cur ^ 1];
    p.nsweeps = (int)b->sweeps[i];
    nsw[i] = b->sweeps[i];
  }
  // every replica's own stream has finished its earlier work (placement, queries)
  for (kk_sim* h : b->sims)
    if (h->stream != b->sB) KB_HIP(hipStreamSynchronize(h->stream));
  KB_HIP(hipMemcpyAsync(b->d_params, params.data(), n * sizeof(SweepParams), hipMemcpyHostToDevice, b->sB));
  KB_HIP(hipMemsetAsync(b->d_counts, 0, b->ncounts * sizeof(unsigned long long), b->sB));
  KB_HIP(hipMemsetAsync(b->d_ctl, 0, 2 * sizeof(unsigned) * kCtlSlots, b->sB));
  KB_HIP(hipEventRecord(b->ev_upload, b->sB));
  // replay the chunk graph until the longest replica is done
  uint64_t mx = 0;
  for (size_t i = 0; i < n; ++i) mx = std::max<uint64_t>(mx, nsw[i]);
  hipStream_t origin = b->tg_stream[0];
  KB_HIP(hipStreamWaitEvent(origin, b->ev_upload, 0));
  for (uint64_t r = 0; r < (mx + kBatchChunk - 1) / kBatchChunk; ++r) KB_HIP(hipGraphLaunch(b->gexec, origin));
  KB_HIP(hipEventRecord(b->ev_res, origin));
  KB_HIP(hipStreamWaitEvent(b->sB, b->ev_res, 0));
  KB_HIP(hipStreamSynchronize(b->sB));
  std::vector<unsigned long long> counts(b->ncounts);
  KB_HIP(hipMemcpy(counts.data(), b->d_counts, b->ncounts * sizeof(unsigned long long), hipMemcpyDeviceToHost));
  for (size_t i = 0; i < n; ++i) {
    kk_sim* h = b->sims[i];
    for (size_t k = 0; k < b->count_n[i]; ++k) h->accepted_base += counts[b->count_off[i] + k];
    h->t += b->sweeps[i];
    if (b->sweeps[i]) h->epoch += 1;
    h->attempts += b->sweeps[i] * (uint64_t)h->L * (uint64_t)h->L;
    if (!is_resident(h)) h->cur ^= (int)(b->sweeps[i] & 1u);
  }
  return KK_OK;
}

kk_status kk_batch_autotune(kk_batch* b, uint32_t trial_sweeps, uint32_t* tile_words, uint32_t* tile_rows,
                            double* ms_per_sweep) {
  if (!b) return set_error(KK_EINVAL, "NULL batch");
  if (b->poisoned) return set_error(KK_ESTATE, "batch poisoned by an earlier error");
  if (trial_sweeps == 0) trial_sweeps = 10;
  if (trial_sweeps > 100000) return set_error(KK_EINVAL, "trial_sweeps must be at most 100000");
  const size_t n = b->sims.size();
  // save every replica: lattice, counters, buffer parity
  struct Saved {
    void* lat;
    size_t bytes;
    uint64_t t, attempts, accepted;
    int cur;
  };
  std::vector<Saved> saved(n);
  auto free_saved = [&]() {
    for (Saved& sv : saved)
      if (sv.lat) (void)hipFree(sv.lat);
  };
  for (size_t i = 0; i < n; ++i) {
    kk_sim* h = b->sims[i];
    Saved& sv = saved[i];
    sv.lat = nullptr;
    sv.bytes = h->layout == kLayoutBits ? (size_t)h->L * (size_t)(h->L / 32) * 4 : (size_t)h->L * h->L;
    uint64_t sw = 0;
    kk_status st = kk_stats(h, &sw, &sv.attempts, &sv.accepted);
    if (st == KK_OK) st = device_alloc(&sv.lat, sv.bytes);
    if (st != KK_OK) {
      free_saved();
      return st;
    }
    sv.t = h->t;
    sv.cur = h->cur;
    KB_HIP(hipMemcpyAsync(sv.lat, h->lat[h->cur], sv.bytes, hipMemcpyDeviceToDevice, h->stream));
    KB_HIP(hipStreamSynchronize(h->stream));
  }
  auto restore_all = [&]() -> kk_status {
    for (size_t i = 0; i < n; ++i) {
      kk_sim* h = b->sims[i];
      const Saved& sv = saved[i];
      h->cur = sv.cur;
      KB_HIP(hipMemcpyAsync(h->lat[h->cur], sv.lat, sv.bytes, hipMemcpyDeviceToDevice, h->stream));
      KB_HIP(hipStreamSynchronize(h->stream));
      h->t = sv.t;
      h->attempts = sv.attempts;
      // the handle's own tile partials are untouched by batch runs: the total
      // is accepted_base + partials, so put back the saved difference
      uint64_t sw = 0, att = 0, acc = 0;
      kk_status st = kk_stats(h, &sw, &att, &acc);
      if (st != KK_OK) return st;
      h->accepted_base -= acc - sv.accepted;
      h->epoch += 1;
    }
    return KK_OK;
  };
  const std::vector<uint64_t> sweeps0 = b->sweeps;
  const int th0 = b->tile_th, tw0 = b->tile_tww, ku0 = b->tile_ku;
  int best_th = th0, best_tw = tw0, best_ku = ku0;
  double best_ms = 1e300;
  kk_status st = KK_OK;
  // (words, rows, units per thread): large tiles for batches that fill the
  // device, small one-unit-per-thread tiles that spread a few mid-sized
  // replicas over many workgroups
  static const int cand[][3] = {{8, 128, 2}, {16, 84, 2}, {8, 64, 2}, {16, 42, 2}, {8, 32, 2}, {8, 16, 2},
                                {16, 28, 1}, {16, 20, 1}, {8, 72, 1}, {8, 50, 1}, {8, 32, 1}};
  for (const auto& c : cand) {
    const int tw = c[0], th = c[1];
    b->tile_th = th;
    b->tile_tww = tw;
    b->tile_ku = c[2];
    st = batch_replan(b, b->sims, std::vector<uint64_t>(n, trial_sweeps));
    if (st == KK_OK) st = kk_batch_run(b);  // warm-up (also checks the plan)
    double ms = 0.0;
    if (st == KK_OK) {
      const auto t0 = std::chrono::steady_clock::now();
      st = kk_batch_run(b);
      ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
    }
    const kk_status rs = restore_all();
    if (st == KK_OK) st = rs;
    if (st != KK_OK) break;
    if (ms < best_ms) {
      best_ms = ms;
      best_th = th;
      best_tw = tw;
      best_ku = c[2];
    }
  }
  free_saved();
  b->tile_th = st == KK_OK ? best_th : th0;
  b->tile_tww = st == KK_OK ? best_tw : tw0;
  b->tile_ku = st == KK_OK ? best_ku : ku0;
  const kk_status ps = batch_replan(b, b->sims, sweeps0);
  if (st == KK_OK) st = ps;
  if (st != KK_OK) return st;
  if (tile_words) *tile_words = (uint32_t)best_tw;
  if (tile_rows) *tile_rows = (uint32_t)best_th;
  if (ms_per_sweep) *ms_per_sweep = best_ms / trial_sweeps;
  return KK_OK;
}

kk_status kk_batch_sim(kk_batch* b, size_t i, kk_sim** sim_out) {
  if (!b || !sim_out) return set_error(KK_EINVAL, "NULL argument");
  if (i >= b->sims.size()) return set_error(KK_EINVAL, "replica %zu out of range (%zu)", i, b->sims.size());
  *sim_out = b->sims[i];
  return KK_OK;
}

kk_status kk_batch_set_tile(kk_batch* b, uint32_t tile_words, uint32_t tile_rows, uint32_t units_per_thread) {
  if (!b) return set_error(KK_EINVAL, "NULL batch");
  if (b->poisoned) return set_error(KK_ESTATE, "batch poisoned by an earlier error");
  if (tile_rows % 2 != 0 || tile_words > 16 || tile_rows > (uint32_t)kBatchTh || units_per_thread > 2 ||
      !batch_tile_fits((int)tile_words, (int)tile_rows, (int)units_per_thread))
    return set_error(KK_EINVAL, "tile %u x %u at %u units per thread: words 8 or 16, rows even and at most %d, "
                     "and (rows + 28) / 2 * (words + 2) at most %d * units per thread",
                     tile_words, tile_rows, units_per_thread, kBatchTh, kBatchTileThreads);
  b->tile_tww = (int)tile_words;
  b->tile_th = (int)tile_rows;
  b->tile_ku = (int)units_per_thread;
  return batch_replan(b, b->sims, b->sweeps);
}

kk_status kk_batch_cluster_hists(kk_batch* b, int species) {
  if (!b) return set_error(KK_EINVAL, "NULL batch");
  if (b->poisoned) return set_error(KK_ESTATE, "batch poisoned by an earlier error");
  if (species != 0 && species != 1) return set_error(KK_EINVAL, "species must be 0 or 1");
  // every replica's own stream has finished its earlier work
  for (kk_sim* h : b->sims) {
    if (h->poisoned) return set_error(KK_ESTATE, "a replica is poisoned");
    if (h->stream != b->sB) KB_HIP(hipStreamSynchronize(h->stream));
  }
  // every lattice that needs it labelled in one set of launches (replica =
  // blockIdx.y), the result blocks gathered into one staging array, one copy
  // and one wait
  std::vector<kk_sim*> todo;
  std::vector<CclRep> reps;
  size_t max_sites = 0;
  for (kk_sim* h : b->sims) {
    if (hist_cached(h, species)) continue;
    const kk_status st = hist_buffers(h);
    if (st != KK_OK) return st;
    todo.push_back(h);
    reps.push_back(CclRep{h->lat[h->cur], h->layout, h->L, h->ccl});
    max_sites = std::max(max_sites, (size_t)h->L * (size_t)h->L);
  }
  if (todo.empty()) return KK_OK;
  const uint32_t words = (uint32_t)kSmallSizes + 1u + kHistBigPrefix;
  const size_t n = b->sims.size();
  if (!b->d_ccl) {
    kk_status st = device_alloc((void**)&b->d_ccl, n * sizeof(CclRep));
    if (st == KK_OK) st = device_alloc((void**)&b->d_hist_stage, n * words * sizeof(uint32_t));
    if (st != KK_OK) return st;
    KB_HIP(hipHostMalloc((void**)&b->h_hist_stage, n * words * sizeof(uint32_t), hipHostMallocDefault));
  }
  KB_HIP(hipMemcpyAsync(b->d_ccl, reps.data(), reps.size() * sizeof(CclRep), hipMemcpyHostToDevice, b->sB));
  KB_HIP(launch_ccl_many(b->d_ccl, (int)reps.size(), max_sites, species, b->d_hist_stage, words, b->sB));
  KB_HIP(hipMemcpyAsync(b->h_hist_stage, b->d_hist_stage, todo.size() * words * sizeof(uint32_t),
                        hipMemcpyDeviceToHost, b->sB));
  KB_HIP(hipStreamSynchronize(b->sB));
  for (size_t i = 0; i < todo.size(); ++i)
    std::memcpy(todo[i]->hist_host, b->h_hist_stage + i * words, words * sizeof(uint32_t));
  for (kk_sim* h : todo) {
    const kk_status st = hist_finish(h, species);
    if (st != KK_OK) return st;
  }
  return KK_OK;
}

kk_status kk_batch_info(kk_batch* b, size_t* n_resident, size_t* n_tiled, size_t* n_tile_jobs) {
  if (!b) return set_error(KK_EINVAL, "NULL batch");
  if (n_resident) *n_resident = b->resident.size();
  if (n_tiled) *n_tiled = b->tiled.size();
  if (n_tile_jobs) *n_tile_jobs = (size_t)b->njobs;
  return KK_OK;
}

void kk_batch_destroy(kk_batch* b) {
  if (!b) return;
  if (b->sB) (void)hipStreamSynchronize(b->sB);
  if (b->sA) (void)hipStreamSynchronize(b->sA);
  if (b->sC) (void)hipStreamSynchronize(b->sC);
  for (int g = 0; g < kMaxTileGroups; ++g)
    if (b->tg_stream[g]) (void)hipStreamSynchronize(b->tg_stream[g]);
  free_batch(b);
  delete b;
}

}  // extern "C"
