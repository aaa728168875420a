// kk_api.cpp -- host side of libkk: the C ABI declared in include/kk.h.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <map>
#include <mutex>
#include <string>
#include <vector>

#include "../../include/kk.h"
#include "kk_host.hpp"
#include "kk_kernels.hpp"

namespace kk {

thread_local std::string g_last_error;

kk_status set_error(kk_status st, const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof buf, fmt, ap);
  va_end(ap);
  g_last_error = buf;
  return st;
}

void acceptance_table(double omega, uint64_t T[7], Accept* acc) {
  const double two42 = 4398046511104.0;
  for (int n = 0; n <= 6; ++n) {
    const double p = std::exp(-omega * (6.0 - 2.0 * n));
    const double v = std::ceil(p * two42);
    T[n] = (v < two42) ? (uint64_t)v : (uint64_t)1 << 42;
  }
  std::memset(acc, 0, sizeof *acc);
  // omega == 0: every unlike exchange is accepted, and every slot below holds
  // 2^42 (prefix 1024), which accepts every site without a branch
  acc->restricted = omega == 0.0 ? 0u : 0xFFFFFFFFu;
  acc->negmask = omega < 0.0 ? 0xFFFFFFFFu : 0u;
  // slot j covers m & 3 == j + 1 with m = n + 1: n = j (omega > 0) or n = 4 + j (omega < 0)
  for (int j = 0; j < 3; ++j) {
    const uint64_t v = T[omega > 0.0 ? j : 4 + j];
    acc->hi[j] = (uint32_t)(v >> 32);  // 1024 when the move is always accepted
    acc->lo[j] = (uint32_t)(v & 0xFFFFFFFFu);
  }
}

int max_threads(int ku) { return ku == 1 ? 1024 : 768; }

bool cyclic_fits(int L) {
  return (L % 32) == 0 && (size_t)(L / 2) * (size_t)(L / 32) <= (size_t)2 * max_threads(2);
}

// Tiles chosen by kk_autotune, per (L, layout), for the rest of the process.
std::mutex g_tuned_mu;
std::map<std::pair<int, int>, TileConfig> g_tuned;

void default_tile(int L, int layout, TileConfig* tc) {
  {
    std::lock_guard<std::mutex> lk(g_tuned_mu);
    auto it = g_tuned.find({L, layout});
    if (it != g_tuned.end()) {
      *tc = it->second;
      return;
    }
  }
  if (cyclic_fits(L)) {
    tc->cyclic = true;
    tc->tww = L / 32;
    tc->th = L;
    const int units = (L / 2) * (L / 32);
    tc->ku = units > max_threads(1) ? 2 : 1;
    return;
  }
  // Largest tile (least halo work) that still gives the GPU enough workgroups;
  // two units per thread only when the tiles saturate the device.
  static const int cand[][2] = {{16, 128}, {8, 128}, {8, 64}, {4, 64}, {2, 64}, {2, 32}, {2, 16}, {1, 16}};
  const int ncand = (int)(sizeof cand / sizeof cand[0]);
  int pick = ncand - 1;
  long tiles = 0;
  for (int i = 0; i < ncand; ++i) {
    const int tww = std::min(cand[i][0], (L + 31) / 32);
    const int th = std::min(cand[i][1], L);
    tiles = (long)((L + 32 * tww - 1) / (32 * tww)) * ((L + th - 1) / th);
    if (tiles >= 128) {
      pick = i;
      break;
    }
  }
  tc->cyclic = false;
  tc->tww = std::min(cand[pick][0], (L + 31) / 32);
  tc->th = std::min(cand[pick][1], L);
  // Two units per thread pay off only when the tiles oversubscribe the device;
  // small lattices are latency-bound and run faster with one.
  tc->ku = (tiles >= 256 && L >= 2048) ? 2 : 1;
}

// Fill the geometry fields of p for lattice side L and tile config tc.
// Returns the workgroup size.
int tile_geometry(int L, const TileConfig& tc, SweepParams* p) {
  p->L = L;
  p->wpr = L / 32;
  p->tww = tc.tww;
  p->th = tc.th;
  if (tc.cyclic) {
    p->hx = 0;
    p->hy = 0;
    p->tiles_x = 1;
    p->C = L / 32;
    p->R = L;
    p->row0 = 0;
    p->npairs = L / 2;
  } else {
    p->hx = 1;
    p->hy = 16;
    p->tiles_x = (L + 32 * tc.tww - 1) / (32 * tc.tww);
    p->C = tc.tww + 2;
    p->R = tc.th + 32;
    p->row0 = 2;
    p->npairs = (p->R - 4) / 2;
  }
  p->nunits = p->npairs * p->C;
  const int per = (p->nunits + tc.ku - 1) / tc.ku;
  return ((per + 63) / 64) * 64;
}

bool tile_valid(int L, const TileConfig& tc, std::string* why) {
  if (tc.ku != 1 && tc.ku != 2) { *why = "units_per_thread must be 1 or 2"; return false; }
  if (tc.cyclic) {
    if (!cyclic_fits(L)) { *why = "cyclic tile needs L % 32 == 0 and (L/2)*(L/32) <= 1536"; return false; }
  } else {
    if (tc.tww < 1 || tc.th < 2 || (tc.th & 1)) {
      *why = "tile_words >= 1 and an even tile_rows >= 2 needed";
      return false;
    }
  }
  SweepParams p{};
  const int threads = tile_geometry(L, tc, &p);
  if (threads > max_threads(tc.ku)) { *why = "tile needs more threads than a workgroup allows"; return false; }
  const size_t lds = (size_t)p.R * (p.C + 2) * 4;
  if (lds > 160 * 1024) { *why = "tile does not fit in 160 KiB of LDS"; return false; }
  return true;
}

}  // namespace kk

using namespace kk;


namespace {

#define KK_HIP(expr)                                                                                     \
  do {                                                                                                   \
    hipError_t e_ = (expr);                                                                              \
    if (e_ != hipSuccess) {                                                                              \
      if (h) h->poisoned = true;                                                                         \
      return set_error(KK_EDEVICE, "%s failed: %s (%s:%d)", #expr, hipGetErrorString(e_), __FILE__,     \
                       __LINE__);                                                                        \
    }                                                                                                    \
  } while (0)

#define KK_GUARD(hh)                                                                       \
  do {                                                                                     \
    if (!(hh)) return set_error(KK_EINVAL, "NULL handle");                                 \
    if ((hh)->poisoned) return set_error(KK_ESTATE, "handle poisoned by an earlier error"); \
  } while (0)

size_t lattice_bytes(const kk_sim* h) {
  return h->layout == kLayoutBits ? (size_t)h->H * (size_t)(h->L / 32) * 4 : (size_t)h->L * (size_t)h->H;
}

void free_all(kk_sim* h) {
  for (int i = 0; i < 2; ++i)
    if (h->lat[i]) (void)hipFree(h->lat[i]);
  if (h->counters) (void)hipFree(h->counters);
  if (h->partials) (void)hipFree(h->partials);
  if (h->ccl.parent) (void)hipFree(h->ccl.parent);
  if (h->ccl.size) (void)hipFree(h->ccl.size);
  if (h->ccl.hist) (void)hipFree(h->ccl.hist);  // also holds big_count and big
  if (h->hist_host) (void)hipHostFree(h->hist_host);
  if (h->own_stream && h->stream) (void)hipStreamDestroy(h->stream);
}

kk_status dmalloc(kk_sim* h, void** p, size_t bytes) {
  hipError_t e = hipMalloc(p, bytes);
  if (e != hipSuccess) {
    (void)hipGetLastError();
    *p = nullptr;
    (void)h;
    return set_error(KK_ENOMEM, "hipMalloc(%zu) failed: %s", bytes, hipGetErrorString(e));
  }
  return KK_OK;
}

// Uniform random subset of exactly n1 sites: radix select of the n1-th
// smallest Philox key, then ties (equal 64-bit keys) broken by site index.
kk_status place_initial(kk_sim* h) {
  const int L = h->L, H = h->H;
  const size_t N = (size_t)L * H;
  const uint64_t n1 = place_count(L, H, h->composition);
  void* dst = h->lat[h->cur];
  const size_t bytes = lattice_bytes(h);
  if (n1 == 0) {
    KK_HIP(hipMemsetAsync(dst, 0, bytes, h->stream));
    KK_HIP(hipStreamSynchronize(h->stream));
    return KK_OK;
  }
  if (n1 == N) {
    KK_HIP(hipMemsetAsync(dst, h->layout == kLayoutBits ? 0xFF : 0x01, bytes, h->stream));
    KK_HIP(hipStreamSynchronize(h->stream));
    return KK_OK;
  }
  uint64_t* keys = nullptr;
  unsigned* hist = nullptr;
  kk_status st = dmalloc(h, (void**)&keys, N * sizeof(uint64_t));
  if (st != KK_OK) return st;
  const unsigned eq_cap = 4096;
  st = dmalloc(h, (void**)&hist, (256 + 1 + eq_cap) * sizeof(unsigned));
  if (st != KK_OK) {
    (void)hipFree(keys);
    return st;
  }
  unsigned* eq_count = hist + 256;
  uint32_t* eq_list = reinterpret_cast<uint32_t*>(hist + 257);
  auto fail = [&](const char* what, hipError_t e) {
    (void)hipFree(keys);
    (void)hipFree(hist);
    h->poisoned = true;
    return set_error(KK_EDEVICE, "%s failed: %s", what, hipGetErrorString(e));
  };
  hipError_t e = launch_init_keys(keys, L, H, h->k0, h->k1, h->stream);
  if (e != hipSuccess) return fail("init_keys", e);
  uint64_t prefix = 0, need = n1;
  for (int shift = 56; shift >= 0; shift -= 8) {
    unsigned hh[256];
    if ((e = hipMemsetAsync(hist, 0, 256 * sizeof(unsigned), h->stream)) != hipSuccess) return fail("memset", e);
    if ((e = launch_radix_hist(keys, N, prefix, shift, hist, h->stream)) != hipSuccess) return fail("radix_hist", e);
    if ((e = hipMemcpyAsync(hh, hist, sizeof hh, hipMemcpyDeviceToHost, h->stream)) != hipSuccess)
      return fail("copy hist", e);
    if ((e = hipStreamSynchronize(h->stream)) != hipSuccess) return fail("sync", e);
    uint64_t cum = 0;
    int d = 0;
    for (; d < 256; ++d) {
      if (cum + hh[d] >= need) break;
      cum += hh[d];
    }
    prefix |= (uint64_t)d << shift;
    need -= cum;
  }
  // sites with key < prefix are ones; `need` of the sites with key == prefix too
  if ((e = hipMemsetAsync(eq_count, 0, sizeof(unsigned), h->stream)) != hipSuccess) return fail("memset", e);
  if ((e = launch_init_mark(keys, L, H, h->layout, prefix, dst, eq_count, eq_list, eq_cap, h->stream)) != hipSuccess)
    return fail("init_mark", e);
  unsigned neq = 0;
  if ((e = hipMemcpyAsync(&neq, eq_count, sizeof neq, hipMemcpyDeviceToHost, h->stream)) != hipSuccess)
    return fail("copy eq", e);
  if ((e = hipStreamSynchronize(h->stream)) != hipSuccess) return fail("sync", e);
  if (neq > eq_cap || need > neq) {
    (void)hipFree(keys);
    (void)hipFree(hist);
    return set_error(KK_EDEVICE, "initial placement: %u equal keys (cap %u), need %llu", neq, eq_cap,
                     (unsigned long long)need);
  }
  std::vector<uint32_t> idx(neq);
  if (neq) {
    if ((e = hipMemcpyAsync(idx.data(), eq_list, neq * sizeof(uint32_t), hipMemcpyDeviceToHost, h->stream)) !=
        hipSuccess)
      return fail("copy eq list", e);
    if ((e = hipStreamSynchronize(h->stream)) != hipSuccess) return fail("sync", e);
    std::sort(idx.begin(), idx.end());
    idx.resize((size_t)need);
    if ((e = hipMemcpyAsync(eq_list, idx.data(), idx.size() * sizeof(uint32_t), hipMemcpyHostToDevice,
                            h->stream)) != hipSuccess)
      return fail("upload ties", e);
    if ((e = launch_set_sites(eq_list, (unsigned)idx.size(), L, h->layout, dst, h->stream)) != hipSuccess)
      return fail("set_sites", e);
  }
  if ((e = hipStreamSynchronize(h->stream)) != hipSuccess) return fail("sync", e);
  (void)hipFree(keys);
  (void)hipFree(hist);
  return KK_OK;
}

size_t tile_count(int L, const TileConfig& tc) {
  SweepParams p{};
  tile_geometry(L, tc, &p);
  return (size_t)p.tiles_x * (size_t)((L + p.th - 1) / p.th);
}

uint64_t sum_partials(kk_sim* h, kk_status* st) {
  std::vector<unsigned long long> v(h->npartials);
  *st = KK_OK;
  hipError_t e = hipMemcpyAsync(v.data(), h->partials, h->npartials * sizeof(unsigned long long),
                                hipMemcpyDeviceToHost, h->stream);
  if (e == hipSuccess) e = hipStreamSynchronize(h->stream);
  if (e != hipSuccess) {
    h->poisoned = true;
    *st = set_error(KK_EDEVICE, "reading accepted counts: %s", hipGetErrorString(e));
    return 0;
  }
  uint64_t s = 0;
  for (auto x : v) s += x;
  return s;
}

// Size the per-tile accepted-move sums for the current tile shape, folding
// the counts gathered under the previous shape into accepted_base.
kk_status reset_partials(kk_sim* h) {
  if (h->partials) {
    kk_status st;
    const uint64_t s = sum_partials(h, &st);
    if (st != KK_OK) return st;
    h->accepted_base += s;
    (void)hipFree(h->partials);
    h->partials = nullptr;
  }
  h->npartials = h->geom != 0 ? (size_t)kTriPartials : tile_count(h->L, h->tile);
  kk_status st = dmalloc(h, (void**)&h->partials, h->npartials * sizeof(unsigned long long));
  if (st != KK_OK) return st;
  KK_HIP(hipMemsetAsync(h->partials, 0, h->npartials * sizeof(unsigned long long), h->stream));
  KK_HIP(hipStreamSynchronize(h->stream));
  return KK_OK;
}

// Launch sweeps [h->t, h->t + n) on the handle's stream.  With `timing`, an
// event pair brackets every launch and the kernel time is accumulated.
// A pair of HIP events, destroyed on every way out.
struct EventPair {
  hipEvent_t ev[2] = {nullptr, nullptr};
  ~EventPair() {
    for (hipEvent_t e : ev)
      if (e) (void)hipEventDestroy(e);
  }
};

kk_status enqueue_sweeps(kk_sim* h, uint64_t n, double* kernel_ms, uint64_t* launches) {
  // the counter carries 60 bits (28 of them in the fourth Philox word); after
  // the run it must still be a valid resume point, as kk_set_lattice requires
  if (n >= ((uint64_t)1 << 60) || h->t + n >= ((uint64_t)1 << 60))
    return set_error(KK_EINVAL, "sweep counter would reach 2^60");
  EventPair tm;
  if (kernel_ms) {
    *kernel_ms = 0.0;
    KK_HIP(hipEventCreate(&tm.ev[0]));
    KK_HIP(hipEventCreate(&tm.ev[1]));
    KK_HIP(hipEventRecord(tm.ev[0], h->stream));
  }
  if (n > 0) h->epoch += 1;
  uint64_t nl = 0;
  const uint64_t sites = (uint64_t)h->L * (uint64_t)h->H;
  if (h->geom != 0) {
    // triangular: the whole ring in one workgroup (many sweeps per launch, in
    // place), one whole-sweep tile launch per sweep, or 16 launches (one per
    // class) in place per sweep; literal MPKK: one whole-step tile launch or 7
    // synchronous iterations per step between the two buffers
    const bool whole = h->geom == 1 && h->tri_tw == h->L && h->tri_tr == h->H;
    for (uint64_t left = whole ? n : 0; left > 0;) {
      const uint64_t m = std::min<uint64_t>(left, kTriResidentChunk);
      TriResidentRep R{};
      R.lat = static_cast<uint8_t*>(h->lat[h->cur]);
      R.L = (uint32_t)h->L;
      R.H = (uint32_t)h->H;
      R.sweeps = (uint32_t)m;
      R.k0 = h->k0;
      R.k1 = h->k1;
      R.t0 = h->t;
      R.acc = h->tacc;
      R.partials = h->partials;
      KK_HIP(launch_tri_resident_one(R, sites, h->stream));
      nl += 1;
      h->t += m;
      h->attempts += m * sites;
      left -= m;
    }
    for (uint64_t k = 0; k < (whole ? 0 : n); ++k) {
      if (h->geom == 1 && h->tri_tw > 0) {
        KK_HIP(launch_tri_tile_sweep(static_cast<const uint8_t*>(h->lat[h->cur]),
                                     static_cast<uint8_t*>(h->lat[h->cur ^ 1]), h->L, h->H, h->tri_tw, h->tri_tr,
                                     h->k0, h->k1, h->t, h->tacc, h->partials, h->stream));
        h->cur ^= 1;
        nl += 1;
      } else if (h->geom == 1) {
        for (int ph = 0; ph < 16; ++ph)
          KK_HIP(launch_tri_phase(static_cast<uint8_t*>(h->lat[h->cur]), h->L, h->H, h->k0, h->k1, h->t, ph,
                                  h->tacc, h->partials, h->stream));
        nl += 16;
      } else if (h->tri_tw > 0) {
        KK_HIP(launch_mpkk_tile_step(static_cast<const uint8_t*>(h->lat[h->cur]),
                                     static_cast<uint8_t*>(h->lat[h->cur ^ 1]), h->L, h->H, h->tri_tw, h->tri_tr,
                                     h->k0, h->k1, h->t, h->tacc, h->partials, h->stream));
        h->cur ^= 1;
        nl += 1;
      } else {
        for (int j = 0; j < 7; ++j) {
          KK_HIP(launch_mpkk_iteration(static_cast<const uint8_t*>(h->lat[h->cur]),
                                       static_cast<uint8_t*>(h->lat[h->cur ^ 1]), h->L, h->H, h->k0, h->k1, h->t, j,
                                       h->tacc, h->partials, h->stream));
          h->cur ^= 1;
        }
        nl += 7;
      }
      h->t += 1;
      h->attempts += sites;
    }
  } else {
    SweepParams p{};
    const int threads = tile_geometry(h->L, h->tile, &p);
    p.accepted = h->partials;
    p.k0 = h->k0;
    p.k1 = h->k1;
    p.acc = h->acc;
    const uint64_t per_launch = h->tile.cyclic ? 256 : 1;
    while (n > 0) {
      const uint64_t k = n < per_launch ? n : per_launch;
      p.src = h->lat[h->cur];
      p.dst = h->lat[h->cur ^ 1];
      p.t0 = h->t;
      p.nsweeps = (int)k;
      KK_HIP(launch_sweep(p, h->layout, h->tile.cyclic, h->tile.ku, threads, h->stream));
      h->cur ^= 1;
      h->t += k;
      h->attempts += k * sites;
      n -= k;
      ++nl;
    }
  }
  if (kernel_ms) {
    // one event pair around the back-to-back launches: the elapsed time is
    // their summed duration plus whatever gaps the device leaves between them
    KK_HIP(hipEventRecord(tm.ev[1], h->stream));
    KK_HIP(hipEventSynchronize(tm.ev[1]));
    float ms = 0.f;
    KK_HIP(hipEventElapsedTime(&ms, tm.ev[0], tm.ev[1]));
    *kernel_ms = ms;
  }
  if (launches) *launches = nl;
  return KK_OK;
}

}  // namespace

namespace kk {
kk_status device_alloc(void** p, size_t bytes) { return dmalloc(nullptr, p, bytes); }

kk_status fold_accepted(kk_sim* h, const unsigned long long* dev_counts, size_t n) {
  if (n == 0) return KK_OK;
  std::vector<unsigned long long> v(n);
  KK_HIP(hipMemcpyAsync(v.data(), dev_counts, n * sizeof(unsigned long long), hipMemcpyDeviceToHost, h->stream));
  KK_HIP(hipStreamSynchronize(h->stream));
  for (auto x : v) h->accepted_base += x;
  return KK_OK;
}

// Whole-sweep (or whole-step) tile of a triangular lattice.  Small rings of
// the class schedule take the whole ring in one workgroup.  Otherwise a workgroup
// works on (T + h)^2 cells per phase on average -- its window shrinks from
// T + 2 halo to about T across the phases, h = 32 for the 16 classes and 21
// for the 7 MPKK iterations -- plus a fixed cost per phase; a CU runs about
// one workgroup's worth of cells at a time, so a launch takes about
// ceil(tiles / 256) of those.  Pick the square tile of least modelled cost
// (ties: the larger), or 0 -- one launch per class or iteration -- when no
// tile fits.
// Modelled time of a triangular / MPKK tile: rounds of 256 workgroups times the
// mean window area a workgroup works per phase, plus a fixed cost per round.
double tri_tile_cost(int L, int H, bool mpkk, int cw, int cr) {
  const int h = mpkk ? 21 : 32;
  const double tiles = (double)((L + cw - 1) / cw) * (double)((H + cr - 1) / cr);
  return std::ceil(tiles / 256.0) * ((double)(cw + h) * (cr + h) + 4096.0);
}

// The tiles that cut the ring into an nx x ny grid (nx, ny <= 64), so that the
// workgroups fill whole rounds of the 256 CUs, in ascending modelled time
// (measured for MPKK at 4098 x 4095: 16 x 16 tiles of 257 x 256 take 123 us
// per step, 22 x 22 tiles of 192 take 157).
std::vector<std::pair<int, int>> tri_grid_tiles(int L, int H, bool mpkk) {
  std::vector<std::pair<double, std::pair<int, int>>> v;
  for (int ny = 1; ny <= 64; ++ny)
    for (int nx = 1; nx <= 64; ++nx) {
      const int cw = (L + nx - 1) / nx, cr = (H + ny - 1) / ny;
      if (!(mpkk ? mpkk_tile_fits(L, H, cw, cr) : tri_tile_fits(L, H, cw, cr))) continue;
      v.push_back({tri_tile_cost(L, H, mpkk, cw, cr), {cw, cr}});
    }
  std::stable_sort(v.begin(), v.end(), [](const auto& a, const auto& b) { return a.first < b.first; });
  std::vector<std::pair<int, int>> out;
  for (const auto& e : v)
    if (std::find(out.begin(), out.end(), e.second) == out.end()) out.push_back(e.second);
  return out;
}

const int kTriSquareTiles[] = {320, 256, 192, 160, 128, 96, 64, 48, 32, 16};

void tri_default_tile(int L, int H, bool mpkk, int* tw, int* tr) {
  double best = 0.0;
  *tw = *tr = 0;
  // rings of up to 12288 sites: the whole ring in one workgroup (measured: 10 us
  // per sweep at 20^2, 16.7 at 100^2 against 19.9 with tiles; tiles win from
  // about 13000 sites on)
  if (!mpkk && (long)L * H <= 12288 && tri_resident_fits(L, H)) {
    *tw = L;
    *tr = H;
    return;
  }
  for (int c : kTriSquareTiles) {
    if (!(mpkk ? mpkk_tile_fits(L, H, c, c) : tri_tile_fits(L, H, c, c))) continue;
    const double cost = tri_tile_cost(L, H, mpkk, c, c);
    if (*tw == 0 || cost < best) {
      best = cost;
      *tw = *tr = c;
    }
  }
  const auto grid = tri_grid_tiles(L, H, mpkk);
  if (!grid.empty()) {
    const double cost = tri_tile_cost(L, H, mpkk, grid[0].first, grid[0].second);
    if (*tw == 0 || cost < best) {
      *tw = grid[0].first;
      *tr = grid[0].second;
    }
  }
}

uint64_t place_count(int L, int H, double composition) {
  const double N = (double)L * (double)H;
  double v = std::floor(composition * N + 0.5);
  if (v < 0.0) v = 0.0;
  if (v > N) v = N;
  return (uint64_t)v;
}
}  // namespace kk

extern "C" {

const char* kk_last_error(void) { return g_last_error.c_str(); }

kk_status kk_create(kk_sim** out, uint32_t L, double composition, double omega_kT, uint64_t seed) {
  return kk_create_ex(out, L, composition, omega_kT, seed, KK_LAYOUT_AUTO, nullptr);
}

kk_status kk_create_ex(kk_sim** out, uint32_t L, double composition, double omega_kT, uint64_t seed,
                       uint32_t layout, void* hip_stream) {
  if (!out) return set_error(KK_EINVAL, "out is NULL");
  *out = nullptr;
  if (L < 4 || (L % 4) != 0 || L > 32768)
    return set_error(KK_EINVAL, "L must be a multiple of 4 in [4, 32768] (got %u)", L);
  if (!(composition >= 0.0 && composition <= 1.0))
    return set_error(KK_EINVAL, "composition must lie in [0, 1]");
  if (!std::isfinite(omega_kT)) return set_error(KK_EINVAL, "omega must be finite");
  int lay;
  if (layout == KK_LAYOUT_AUTO) lay = (L % 32 == 0) ? kLayoutBits : kLayoutInt8;
  else if (layout == KK_LAYOUT_INT8) lay = kLayoutInt8;
  else if (layout == KK_LAYOUT_BITPACKED) {
    if (L % 32 != 0) return set_error(KK_EINVAL, "bit-packed layout needs L %% 32 == 0 (got %u)", L);
    lay = kLayoutBits;
  } else return set_error(KK_EINVAL, "unknown layout %u", layout);
  return create_handle(out, L, L, 0, composition, omega_kT, seed, lay, hip_stream);
}

}  // extern "C"

namespace kk {
// A handle of H rows of L sites on geometry `geom` (0 square torus; 1 triangular,
// conflict-free classes; 2 triangular, literal MPKK), arguments already validated.
kk_status create_handle(kk_sim** out, uint32_t L, uint32_t H, int geom, double composition, double omega_kT,
                        uint64_t seed, int lay, void* hip_stream) {
  kk_sim* h = new (std::nothrow) kk_sim();
  if (!h) return set_error(KK_ENOMEM, "host allocation failed");
  h->L = (int)L;
  h->H = (int)H;
  h->geom = geom;
  for (int n = 0; n <= 10; ++n) {
    const double p = std::exp(-omega_kT * (double)(10 - 2 * n));
    const double v = std::ceil(p * 4294967296.0);
    h->tacc.T[n] = (v >= 4294967296.0) ? 4294967296ull : (uint64_t)v;
  }
  h->layout = lay;
  h->composition = composition;
  h->omega = omega_kT;
  h->seed = seed;
  h->k0 = (uint32_t)(seed & 0xFFFFFFFFu);
  h->k1 = (uint32_t)(seed >> 32);
  acceptance_table(omega_kT, h->T, &h->acc);
  if (geom == 0) default_tile(h->L, lay, &h->tile);
  kk_status st = KK_OK;
  hipError_t e = hipGetDevice(&h->device);
  if (e != hipSuccess) {
    delete h;
    return set_error(KK_EDEVICE, "hipGetDevice failed: %s", hipGetErrorString(e));
  }
  if (hip_stream) h->stream = static_cast<hipStream_t>(hip_stream);
  else {
    e = hipStreamCreateWithFlags(&h->stream, hipStreamNonBlocking);
    if (e != hipSuccess) {
      delete h;
      return set_error(KK_EDEVICE, "hipStreamCreate failed: %s", hipGetErrorString(e));
    }
    h->own_stream = true;
  }
  const size_t bytes = lattice_bytes(h);
  for (int i = 0; i < 2 && st == KK_OK; ++i) st = dmalloc(h, &h->lat[i], bytes);
  if (st == KK_OK) st = dmalloc(h, (void**)&h->counters, 2 * sizeof(unsigned long long));
  if (st == KK_OK) {
    e = hipMemsetAsync(h->counters, 0, 2 * sizeof(unsigned long long), h->stream);
    if (e != hipSuccess) st = set_error(KK_EDEVICE, "memset failed: %s", hipGetErrorString(e));
  }
  if (st == KK_OK) st = reset_partials(h);
  if (st == KK_OK) st = place_initial(h);
  if (st != KK_OK) {
    free_all(h);
    delete h;
    return st;
  }
  *out = h;
  return KK_OK;
}

}  // namespace kk

extern "C" {

kk_status kk_create_triangular_ex(kk_sim** out, uint32_t L, uint32_t H, uint32_t scheme, double composition,
                                  double omega_kT, uint64_t seed, void* hip_stream) {
  if (!out) return set_error(KK_EINVAL, "out is NULL");
  *out = nullptr;
  if (!(composition >= 0.0 && composition <= 1.0))
    return set_error(KK_EINVAL, "composition must lie in [0, 1]");
  if (!std::isfinite(omega_kT)) return set_error(KK_EINVAL, "omega must be finite");
  if ((uint64_t)L * H > 0x7FFFFFFFull || L > 65535 || H > 65535)
    return set_error(KK_EINVAL, "lattice too large (%u x %u)", L, H);
  if (scheme == KK_TRI_CLASSES) {
    if (L < 4 || L % 8 != 4 || H < 4 || H % 4 != 0)
      return set_error(KK_EINVAL, "the 16-class schedule needs L %% 8 == 4 and H %% 4 == 0 (got %u x %u)", L, H);
  } else if (scheme == KK_TRI_MPKK) {
    if (L < 3 || (L % 7 != 3 && L % 7 != 5) || H < 7 || H % 7 != 0)
      return set_error(KK_EINVAL, "the 7-site domain cover needs L %% 7 in {3, 5} and H %% 7 == 0 (got %u x %u)", L,
                       H);
  } else {
    return set_error(KK_EINVAL, "unknown scheme %u", scheme);
  }
  const kk_status st = create_handle(out, L, H, scheme == KK_TRI_CLASSES ? 1 : 2, composition, omega_kT, seed,
                                     kLayoutInt8, hip_stream);
  if (st == KK_OK) tri_default_tile((int)L, (int)H, scheme == KK_TRI_MPKK, &(*out)->tri_tw, &(*out)->tri_tr);
  return st;
}

kk_status kk_tri_set_tile(kk_sim* h, uint32_t cols, uint32_t rows) {
  KK_GUARD(h);
  if (h->geom == 0) return set_error(KK_EINVAL, "tiles apply to triangular lattices only");
  if (cols == 0) {
    h->tri_tw = h->tri_tr = 0;
    return KK_OK;
  }
  const bool mp = h->geom == 2;
  if (!mp && cols == (uint32_t)h->L && rows == (uint32_t)h->H) {
    // the whole ring in one workgroup
    if (!tri_resident_fits(h->L, h->H))
      return set_error(KK_EINVAL, "the whole ring (%d bytes) does not fit one workgroup's LDS (%zu)", h->L * h->H,
                       kTriResidentMaxBytes);
    h->tri_tw = h->L;
    h->tri_tr = h->H;
    return KK_OK;
  }
  const uint32_t halo = mp ? kMpkkHalo : kTriHalo;
  const bool fits = mp ? mpkk_tile_fits(h->L, h->H, (int)cols, (int)rows)
                        : tri_tile_fits(h->L, h->H, (int)cols, (int)rows);
  if (!fits)
    return set_error(KK_EINVAL, "tile %u x %u does not fit: needs >= 16 each, cols + %u <= L, rows + %u <= H and %zu "
                     "window bytes <= 159 KiB", cols, rows, 2 * halo, 2 * halo,
                     mp ? mpkk_window_bytes(cols, rows) : tri_window_bytes(cols, rows));
  h->tri_tw = (int)cols;
  h->tri_tr = (int)rows;
  return KK_OK;
}

kk_status kk_tri_autotune(kk_sim* h, uint32_t trial_sweeps, uint32_t* cols, uint32_t* rows, double* us_per_sweep) {
  KK_GUARD(h);
  if (h->geom == 0) return set_error(KK_EINVAL, "square lattice: use kk_autotune");
  if (trial_sweeps == 0) trial_sweeps = 20;
  if (trial_sweeps > 100000) return set_error(KK_EINVAL, "trial_sweeps must be at most 100000");
  const bool mp = h->geom == 2;
  // candidates: one launch per class / iteration, the whole ring in one
  // workgroup, the handle's current tile, the default pick, every square tile
  // that fits and the four grid-cut tiles of least modelled time
  std::vector<std::pair<int, int>> cands = {{0, 0}};
  auto add = [&](int cw, int cr) {
    if (std::find(cands.begin(), cands.end(), std::make_pair(cw, cr)) == cands.end()) cands.push_back({cw, cr});
  };
  if (!mp && tri_resident_fits(h->L, h->H)) add(h->L, h->H);
  add(h->tri_tw, h->tri_tr);
  int dw = 0, dr = 0;
  tri_default_tile(h->L, h->H, mp, &dw, &dr);
  add(dw, dr);
  for (int c : kTriSquareTiles)
    if (mp ? mpkk_tile_fits(h->L, h->H, c, c) : tri_tile_fits(h->L, h->H, c, c)) add(c, c);
  const auto grid = tri_grid_tiles(h->L, h->H, mp);
  for (size_t i = 0; i < grid.size() && i < 4; ++i) add(grid[i].first, grid[i].second);
  // save the state; the trials run on the live buffers and everything is restored
  uint64_t sw0 = 0, att0 = 0, acc0 = 0;
  kk_status st = kk_stats(h, &sw0, &att0, &acc0);
  if (st != KK_OK) return st;
  const int cur0 = h->cur, tw0 = h->tri_tw, tr0 = h->tri_tr;
  const size_t bytes = lattice_bytes(h);
  void* save = nullptr;
  st = dmalloc(h, &save, bytes);
  if (st != KK_OK) return st;
  auto restore = [&](int tw, int tr) -> kk_status {
    h->tri_tw = tw;
    h->tri_tr = tr;
    hipError_t e = hipMemcpyAsync(h->lat[cur0], save, bytes, hipMemcpyDeviceToDevice, h->stream);
    if (e == hipSuccess) e = hipMemsetAsync(h->partials, 0, h->npartials * sizeof(unsigned long long), h->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(h->stream);
    (void)hipFree(save);
    if (e != hipSuccess) {
      h->poisoned = true;
      return set_error(KK_EDEVICE, "autotune restore: %s", hipGetErrorString(e));
    }
    h->cur = cur0;
    h->t = sw0;
    h->attempts = att0;
    h->accepted_base = acc0;  // the partials were just zeroed
    h->epoch += 1;
    return KK_OK;
  };
  hipError_t e = hipMemcpyAsync(save, h->lat[cur0], bytes, hipMemcpyDeviceToDevice, h->stream);
  if (e != hipSuccess) {
    (void)hipFree(save);
    h->poisoned = true;
    return set_error(KK_EDEVICE, "autotune save: %s", hipGetErrorString(e));
  }
  std::pair<int, int> best = {tw0, tr0};
  double best_us = 1e300;
  for (const auto& c : cands) {
    h->tri_tw = c.first;
    h->tri_tr = c.second;
    st = enqueue_sweeps(h, 2, nullptr, nullptr);  // warm-up
    double ms = 0.0;
    uint64_t nl = 0;
    if (st == KK_OK) st = enqueue_sweeps(h, trial_sweeps, &ms, &nl);
    if (st != KK_OK) {
      (void)restore(tw0, tr0);
      return st;
    }
    const double us = ms * 1e3 / trial_sweeps;
    if (us < best_us) {
      best_us = us;
      best = c;
    }
  }
  st = restore(best.first, best.second);
  if (st != KK_OK) return st;
  if (cols) *cols = (uint32_t)h->tri_tw;
  if (rows) *rows = (uint32_t)h->tri_tr;
  if (us_per_sweep) *us_per_sweep = best_us;
  return KK_OK;
}

kk_status kk_tri_get_tile(kk_sim* h, uint32_t* cols, uint32_t* rows) {
  KK_GUARD(h);
  if (h->geom == 0) return set_error(KK_EINVAL, "tiles apply to triangular lattices only");
  if (cols) *cols = (uint32_t)h->tri_tw;
  if (rows) *rows = (uint32_t)h->tri_tr;
  return KK_OK;
}

kk_status kk_create_triangular(kk_sim** out, uint32_t L, double composition, double omega_kT, uint64_t seed,
                               void* hip_stream) {
  return kk_create_triangular_ex(out, L, L, KK_TRI_CLASSES, composition, omega_kT, seed, hip_stream);
}

kk_status kk_shape(kk_sim* h, uint32_t* L, uint32_t* H) {
  KK_GUARD(h);
  if (L) *L = (uint32_t)h->L;
  if (H) *H = (uint32_t)h->H;
  return KK_OK;
}

kk_status kk_restart(kk_sim* h, uint32_t start) {
  KK_GUARD(h);
  if (start != KK_START_RANDOM && start != KK_START_SEGREGATED)
    return set_error(KK_EINVAL, "unknown start %u", start);
  if (start == KK_START_RANDOM) {
    const kk_status st = place_initial(h);
    if (st != KK_OK) return st;
  } else {
    KK_HIP(launch_fill_segregated(h->lat[h->cur], h->layout, h->L, h->H, place_count(h->L, h->H, h->composition),
                                  h->stream));
  }
  KK_HIP(hipMemsetAsync(h->partials, 0, h->npartials * sizeof(unsigned long long), h->stream));
  KK_HIP(hipStreamSynchronize(h->stream));
  h->t = 0;
  h->attempts = 0;
  h->accepted_base = 0;
  h->epoch += 1;
  return KK_OK;
}

kk_status kk_tri_thresholds(kk_sim* h, uint64_t out[11]) {
  KK_GUARD(h);
  if (!out) return set_error(KK_EINVAL, "out is NULL");
  if (h->geom == 0) return set_error(KK_EINVAL, "square lattice: use kk_thresholds");
  for (int i = 0; i < 11; ++i) out[i] = h->tacc.T[i];
  return KK_OK;
}

kk_status kk_geometry(kk_sim* h, uint32_t* geometry) {
  KK_GUARD(h);
  if (!geometry) return set_error(KK_EINVAL, "geometry is NULL");
  *geometry = (uint32_t)h->geom;
  return KK_OK;
}

kk_status kk_sweep_async(kk_sim* h, uint64_t n) {
  KK_GUARD(h);
  return enqueue_sweeps(h, n, nullptr, nullptr);
}

kk_status kk_sync(kk_sim* h) {
  KK_GUARD(h);
  KK_HIP(hipStreamSynchronize(h->stream));
  return KK_OK;
}

kk_status kk_sweep(kk_sim* h, uint64_t n) {
  KK_GUARD(h);
  kk_status st = enqueue_sweeps(h, n, nullptr, nullptr);
  if (st != KK_OK) return st;
  KK_HIP(hipStreamSynchronize(h->stream));
  return KK_OK;
}

kk_status kk_sweep_timed(kk_sim* h, uint64_t n, double* kernel_ms, uint64_t* launches) {
  KK_GUARD(h);
  double ms = 0.0;
  uint64_t nl = 0;
  kk_status st = enqueue_sweeps(h, n, &ms, &nl);
  if (st != KK_OK) return st;
  KK_HIP(hipStreamSynchronize(h->stream));
  if (kernel_ms) *kernel_ms = ms;
  if (launches) *launches = nl;
  return KK_OK;
}

kk_status kk_energy(kk_sim* h, uint64_t* n_unlike, double* energy_kT) {
  KK_GUARD(h);
  KK_HIP(hipMemsetAsync(h->counters + 1, 0, sizeof(unsigned long long), h->stream));
  if (h->geom != 0)
    KK_HIP(launch_tri_energy(static_cast<const uint8_t*>(h->lat[h->cur]), h->L, h->H, h->counters + 1, h->stream));
  else
    KK_HIP(launch_energy(h->lat[h->cur], h->layout, h->L, h->counters + 1, h->stream));
  unsigned long long v = 0;
  KK_HIP(hipMemcpyAsync(&v, h->counters + 1, sizeof v, hipMemcpyDeviceToHost, h->stream));
  KK_HIP(hipStreamSynchronize(h->stream));
  if (n_unlike) *n_unlike = v;
  if (energy_kT) *energy_kT = h->omega * (double)v;
  return KK_OK;
}

}  // extern "C"

namespace kk {

// Labelling buffers of a handle, made on its first histogram: parent and size
// (N words each), then one block holding the small-size histogram, the count
// of large sizes and their list, so that one copy brings back the histogram,
// the count and the first kHistBigPrefix large sizes; its pinned host image.
kk_status hist_buffers(kk_sim* h) {
  if (h->ccl_ready) return KK_OK;
  const size_t N = (size_t)h->L * h->H;
  const unsigned big_cap = (unsigned)(N / kSmallSizes + 1);
  kk_status st = dmalloc(h, (void**)&h->ccl.parent, N * 4);
  if (st == KK_OK) st = dmalloc(h, (void**)&h->ccl.size, N * 4);
  if (st == KK_OK) st = dmalloc(h, (void**)&h->ccl.hist, ((size_t)kSmallSizes + 1 + big_cap) * 4);
  if (st == KK_OK && !h->hist_host) {
    const hipError_t e = hipHostMalloc((void**)&h->hist_host, ((size_t)kSmallSizes + 1 + kHistBigPrefix) * 4,
                                       hipHostMallocDefault);
    if (e != hipSuccess) {
      (void)hipGetLastError();
      h->hist_host = nullptr;
      st = set_error(KK_ENOMEM, "hipHostMalloc: %s", hipGetErrorString(e));
    }
  }
  if (st != KK_OK) return st;
  h->ccl.big_count = h->ccl.hist + kSmallSizes;
  h->ccl.big = h->ccl.hist + kSmallSizes + 1;
  h->ccl.big_cap = big_cap;
  h->ccl_ready = true;
  return KK_OK;
}

bool hist_cached(const kk_sim* h, int species) { return h->hist_epoch == h->epoch && h->hist_species == species; }

// Label species, count and histogram on `stream`, and copy the result block
// to the pinned image.  The result is read by hist_finish once the stream has
// drained.
kk_status hist_enqueue(kk_sim* h, int species, hipStream_t stream) {
  kk_status st = hist_buffers(h);
  if (st != KK_OK) return st;
  KK_HIP(launch_ccl(h->lat[h->cur], h->layout, h->L, h->H, species, h->ccl, h->geom != 0, stream));
  const size_t words = (size_t)kSmallSizes + 1 + std::min<size_t>(h->ccl.big_cap, kHistBigPrefix);
  KK_HIP(hipMemcpyAsync(h->hist_host, h->ccl.hist, words * 4, hipMemcpyDeviceToHost, stream));
  return KK_OK;
}

// Turn the pinned image into the handle's cached histogram (sizes ascending).
kk_status hist_finish(kk_sim* h, int species) {
  const uint32_t* hs = h->hist_host;
  const unsigned nbig = hs[kSmallSizes];
  if (nbig > h->ccl.big_cap) return set_error(KK_EDEVICE, "cluster list overflow (%u > %u)", nbig, h->ccl.big_cap);
  std::vector<uint32_t> big(hs + kSmallSizes + 1, hs + kSmallSizes + 1 + std::min<unsigned>(nbig, kHistBigPrefix));
  if (nbig > kHistBigPrefix) {  // more large clusters than the copied prefix
    big.resize(nbig);
    KK_HIP(hipMemcpyAsync(big.data() + kHistBigPrefix, h->ccl.big + kHistBigPrefix, (nbig - kHistBigPrefix) * 4,
                          hipMemcpyDeviceToHost, h->stream));
    KK_HIP(hipStreamSynchronize(h->stream));
  }
  std::map<uint64_t, uint64_t> bigh;
  for (uint32_t s : big) bigh[s] += 1;
  h->hist_cache.clear();
  for (int s = 1; s < kSmallSizes; ++s)
    if (hs[s]) h->hist_cache.push_back(kk_hist_entry{(uint64_t)s, (uint64_t)hs[s]});
  for (auto& kv : bigh) h->hist_cache.push_back(kk_hist_entry{kv.first, kv.second});
  h->hist_epoch = h->epoch;
  h->hist_species = species;
  return KK_OK;
}

}  // namespace kk

extern "C" {

kk_status kk_cluster_hist(kk_sim* h, int species, kk_hist_entry* out, size_t cap, size_t* n_out) {
  KK_GUARD(h);
  if (species != 0 && species != 1) return set_error(KK_EINVAL, "species must be 0 or 1");
  if (!n_out) return set_error(KK_EINVAL, "n_out is NULL");
  if (cap > 0 && !out) return set_error(KK_EINVAL, "out is NULL with cap > 0");
  if (!hist_cached(h, species)) {
    // the result is cached until the lattice changes, so a size query
    // followed by the fill labels only once
    kk_status st = hist_enqueue(h, species, h->stream);
    if (st != KK_OK) return st;
    KK_HIP(hipStreamSynchronize(h->stream));
    st = hist_finish(h, species);
    if (st != KK_OK) return st;
  }
  const size_t n = h->hist_cache.size();
  *n_out = n;
  if (cap < n) return set_error(KK_ETRUNC, "histogram has %zu entries, cap %zu", n, cap);
  std::copy(h->hist_cache.begin(), h->hist_cache.end(), out);
  return KK_OK;
}

kk_status kk_observe(kk_sim* h, int species, kk_observables* out) {
  KK_GUARD(h);
  if (!out) return set_error(KK_EINVAL, "out is NULL");
  if (species != 0 && species != 1) return set_error(KK_EINVAL, "species must be 0 or 1");
  kk_observables o{};
  o.sweep = h->t;
  kk_status st = kk_energy(h, &o.n_unlike, &o.energy_kT);
  if (st != KK_OK) return st;
  const uint64_t N = (uint64_t)h->L * (uint64_t)h->H;
  // the lattice has 2N bonds (square) or 3N (triangular)
  o.similar_exact = 1.0 - (double)o.n_unlike / (double)((h->geom != 0 ? 3 : 2) * N);
  KK_HIP(hipMemsetAsync(h->counters, 0, sizeof(unsigned long long), h->stream));
  if (h->geom != 0)
    KK_HIP(launch_tri_similar(static_cast<const uint8_t*>(h->lat[h->cur]), h->L, h->H, h->k0, h->k1, h->t,
                              h->counters, h->stream));
  else
    KK_HIP(launch_similar_sampled(h->lat[h->cur], h->layout, h->L, h->k0, h->k1, h->t, h->counters, h->stream));
  unsigned long long same = 0;
  KK_HIP(hipMemcpyAsync(&same, h->counters, sizeof same, hipMemcpyDeviceToHost, h->stream));
  KK_HIP(hipStreamSynchronize(h->stream));
  o.similar_sampled = (double)same / (double)N;
  size_t n = 0;
  st = kk_cluster_hist(h, species, nullptr, 0, &n);
  if (st != KK_OK && st != KK_ETRUNC) return st;
  uint64_t nc = 0, s1 = 0, s2 = 0, smax = 0;
  for (const kk_hist_entry& e : h->hist_cache) {  // filled by the call above
    nc += e.count;
    s1 += e.size * e.count;
    s2 += e.size * e.size * e.count;
    smax = std::max(smax, e.size);
  }
  o.n_clusters = nc;
  o.size_number_avg = nc ? (double)s1 / (double)nc : 0.0;
  o.size_weight_avg = s1 ? (double)s2 / (double)s1 : 0.0;
  o.size_max = smax;
  *out = o;
  return KK_OK;
}

kk_status kk_sweep_series(kk_sim* h, uint64_t every, uint64_t count, int species, kk_observables* out) {
  KK_GUARD(h);
  if (every == 0) return set_error(KK_EINVAL, "every must be at least 1");
  if (count > 0 && !out) return set_error(KK_EINVAL, "out is NULL");
  const uint64_t lim = (uint64_t)1 << 60;
  if (count > 0 && (every >= lim || count >= lim / every || h->t + every * count >= lim))
    return set_error(KK_EINVAL, "sweep counter would reach 2^60");
  for (uint64_t i = 0; i < count; ++i) {
    kk_status st = kk_sweep(h, every);
    if (st == KK_OK) st = kk_observe(h, species, &out[i]);
    if (st != KK_OK) return st;
  }
  return KK_OK;
}

kk_status kk_get_lattice(kk_sim* h, uint8_t* host_out, size_t n) {
  KK_GUARD(h);
  const size_t N = (size_t)h->L * h->H;
  if (!host_out || n != N) return set_error(KK_EINVAL, "need a buffer of exactly L*H = %zu bytes", N);
  if (h->layout == kLayoutInt8) {
    KK_HIP(hipMemcpyAsync(host_out, h->lat[h->cur], N, hipMemcpyDeviceToHost, h->stream));
    KK_HIP(hipStreamSynchronize(h->stream));
    return KK_OK;
  }
  uint8_t* tmp = nullptr;
  kk_status st = dmalloc(h, (void**)&tmp, N);
  if (st != KK_OK) return st;
  hipError_t e = launch_unpack(static_cast<const uint32_t*>(h->lat[h->cur]), tmp, h->L, h->stream);
  if (e == hipSuccess) e = hipMemcpyAsync(host_out, tmp, N, hipMemcpyDeviceToHost, h->stream);
  if (e == hipSuccess) e = hipStreamSynchronize(h->stream);
  (void)hipFree(tmp);
  if (e != hipSuccess) {
    h->poisoned = true;
    return set_error(KK_EDEVICE, "get_lattice: %s", hipGetErrorString(e));
  }
  return KK_OK;
}

kk_status kk_set_lattice(kk_sim* h, const uint8_t* host_in, size_t n, uint64_t sweep_t) {
  KK_GUARD(h);
  const size_t N = (size_t)h->L * h->H;
  if (!host_in || n != N) return set_error(KK_EINVAL, "need a buffer of exactly L*H = %zu bytes", N);
  for (size_t i = 0; i < N; ++i)
    if (host_in[i] > 1) return set_error(KK_EINVAL, "site %zu holds %u; sites must be 0 or 1", i, host_in[i]);
  if (sweep_t >= ((uint64_t)1 << 60)) return set_error(KK_EINVAL, "sweep counter must be < 2^60");
  if (h->layout == kLayoutInt8) {
    KK_HIP(hipMemcpyAsync(h->lat[h->cur], host_in, N, hipMemcpyHostToDevice, h->stream));
  } else {
    uint8_t* tmp = nullptr;
    kk_status st = dmalloc(h, (void**)&tmp, N);
    if (st != KK_OK) return st;
    hipError_t e = hipMemcpyAsync(tmp, host_in, N, hipMemcpyHostToDevice, h->stream);
    if (e == hipSuccess) e = launch_pack(tmp, static_cast<uint32_t*>(h->lat[h->cur]), h->L, h->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(h->stream);
    (void)hipFree(tmp);
    if (e != hipSuccess) {
      h->poisoned = true;
      return set_error(KK_EDEVICE, "set_lattice: %s", hipGetErrorString(e));
    }
  }
  KK_HIP(hipStreamSynchronize(h->stream));
  h->t = sweep_t;
  h->epoch += 1;
  return KK_OK;
}

kk_status kk_stats(kk_sim* h, uint64_t* sweeps, uint64_t* attempts, uint64_t* accepted) {
  KK_GUARD(h);
  kk_status st;
  const uint64_t acc = h->accepted_base + sum_partials(h, &st);
  if (st != KK_OK) return st;
  if (sweeps) *sweeps = h->t;
  if (attempts) *attempts = h->attempts;
  if (accepted) *accepted = acc;
  return KK_OK;
}

kk_status kk_thresholds(kk_sim* h, uint64_t out[7]) {
  KK_GUARD(h);
  if (!out) return set_error(KK_EINVAL, "out is NULL");
  if (h->geom != 0) return set_error(KK_EINVAL, "triangular lattice: use kk_tri_thresholds (11 entries)");
  for (int i = 0; i < 7; ++i) out[i] = h->T[i];
  return KK_OK;
}

kk_status kk_info(kk_sim* h, uint32_t* L, uint32_t* layout) {
  KK_GUARD(h);
  if (L) *L = (uint32_t)h->L;
  if (layout) *layout = h->layout == kLayoutBits ? KK_LAYOUT_BITPACKED : KK_LAYOUT_INT8;
  return KK_OK;
}

kk_status kk_set_tile(kk_sim* h, uint32_t tile_words, uint32_t tile_rows, uint32_t units_per_thread) {
  KK_GUARD(h);
  if (h->geom != 0) return set_error(KK_EINVAL, "the triangular lattice has no sweep tiles");
  TileConfig tc{};
  tc.ku = (int)units_per_thread;
  if (tile_words == 0) {
    tc.cyclic = true;
    tc.tww = h->L / 32;
    tc.th = h->L;
  } else {
    tc.cyclic = false;
    tc.tww = (int)tile_words;
    tc.th = (int)tile_rows;
  }
  std::string why;
  if (!tile_valid(h->L, tc, &why)) return set_error(KK_EINVAL, "invalid tile: %s", why.c_str());
  h->tile = tc;
  return reset_partials(h);
}

kk_status kk_autotune(kk_sim* h, uint32_t trial_sweeps, uint32_t* tile_words, uint32_t* tile_rows,
                      uint32_t* units_per_thread, double* us_per_sweep) {
  KK_GUARD(h);
  if (h->geom != 0) return set_error(KK_EINVAL, "the triangular lattice has no sweep tiles");
  if (trial_sweeps == 0) trial_sweeps = 20;
  if (trial_sweeps > 100000) return set_error(KK_EINVAL, "trial_sweeps must be at most 100000");
  const int L = h->L;
  // candidates: the cyclic tile when it fits, and halo tiles of the compiled widths
  std::vector<TileConfig> cands;
  for (int ku = 1; ku <= 2; ++ku) {
    TileConfig tc;
    tc.ku = ku;
    std::string why;
    if (cyclic_fits(L)) {
      tc.cyclic = true;
      tc.tww = L / 32;
      tc.th = L;
      if (tile_valid(L, tc, &why)) cands.push_back(tc);
    }
    for (int tww : {16, 8, 4, 2, 1}) {
      if (tww > (L + 31) / 32) continue;
      for (int th : {32, 48, 64, 96, 128, 192, 256}) {
        tc.cyclic = false;
        tc.tww = tww;
        tc.th = std::min(th, L);
        bool dup = false;
        for (const TileConfig& c : cands)
          dup |= !c.cyclic && c.tww == tc.tww && c.th == tc.th && c.ku == tc.ku;
        if (!dup && tile_valid(L, tc, &why)) cands.push_back(tc);
      }
    }
  }
  // save the state; trials run on the live buffers and everything is restored
  uint64_t sw0 = 0, att0 = 0, acc0 = 0;
  kk_status st = kk_stats(h, &sw0, &att0, &acc0);
  if (st != KK_OK) return st;
  const int cur0 = h->cur;
  const TileConfig orig = h->tile;
  const size_t bytes = lattice_bytes(h);
  void* save = nullptr;
  st = dmalloc(h, &save, bytes);
  if (st != KK_OK) return st;
  auto restore = [&](const TileConfig& keep) -> kk_status {
    h->tile = keep;
    kk_status s2 = reset_partials(h);
    hipError_t e = hipMemcpyAsync(h->lat[cur0], save, bytes, hipMemcpyDeviceToDevice, h->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(h->stream);
    (void)hipFree(save);
    if (e != hipSuccess) {
      h->poisoned = true;
      return set_error(KK_EDEVICE, "autotune restore: %s", hipGetErrorString(e));
    }
    h->cur = cur0;
    h->t = sw0;
    h->attempts = att0;
    h->accepted_base = acc0;  // the partials were just zeroed
    h->epoch += 1;
    return s2;
  };
  hipError_t e = hipMemcpyAsync(save, h->lat[cur0], bytes, hipMemcpyDeviceToDevice, h->stream);
  if (e != hipSuccess) {
    (void)hipFree(save);
    h->poisoned = true;
    return set_error(KK_EDEVICE, "autotune save: %s", hipGetErrorString(e));
  }
  TileConfig best = orig;
  double best_us = 1e300;
  for (const TileConfig& tc : cands) {
    h->tile = tc;
    st = reset_partials(h);
    if (st == KK_OK) st = enqueue_sweeps(h, 2, nullptr, nullptr);  // warm-up
    double ms = 0.0;
    uint64_t nl = 0;
    if (st == KK_OK) st = enqueue_sweeps(h, trial_sweeps, &ms, &nl);
    if (st != KK_OK) {
      (void)restore(orig);
      return st;
    }
    const double us = ms * 1e3 / trial_sweeps;
    if (us < best_us) {
      best_us = us;
      best = tc;
    }
  }
  st = restore(best);
  if (st != KK_OK) return st;
  {
    std::lock_guard<std::mutex> lk(g_tuned_mu);
    g_tuned[{L, h->layout}] = best;
  }
  if (tile_words) *tile_words = best.cyclic ? 0u : (uint32_t)best.tww;
  if (tile_rows) *tile_rows = (uint32_t)best.th;
  if (units_per_thread) *units_per_thread = (uint32_t)best.ku;
  if (us_per_sweep) *us_per_sweep = best_us;
  return KK_OK;
}

kk_status kk_get_tile(kk_sim* h, uint32_t* tile_words, uint32_t* tile_rows, uint32_t* units_per_thread) {
  KK_GUARD(h);
  if (h->geom != 0) return set_error(KK_EINVAL, "the triangular lattice has no sweep tiles");
  if (tile_words) *tile_words = h->tile.cyclic ? 0u : (uint32_t)h->tile.tww;
  if (tile_rows) *tile_rows = (uint32_t)h->tile.th;
  if (units_per_thread) *units_per_thread = (uint32_t)h->tile.ku;
  return KK_OK;
}

kk_status kk_stream(kk_sim* h, void** stream_out) {
  KK_GUARD(h);
  if (!stream_out) return set_error(KK_EINVAL, "stream_out is NULL");
  *stream_out = h->stream;
  return KK_OK;
}

void kk_destroy(kk_sim* h) {
  if (!h) return;
  if (h->stream) (void)hipStreamSynchronize(h->stream);
  free_all(h);
  delete h;
}

}  // extern "C"
