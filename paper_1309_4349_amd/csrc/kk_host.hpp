// kk_host.hpp -- host helpers shared by the libkk C-ABI translation units.
#pragma once
#include <stdarg.h>
#include <stdint.h>

#include <string>
#include <vector>

#include "../../include/kk.h"
#include "kk_kernels.hpp"
#include "kk_tri.hpp"

namespace kk {

struct TileConfig {
  bool cyclic = false;  // one tile = whole lattice, wrapping inside LDS
  int tww = 8;          // interior words per tile row
  int th = 256;         // interior rows per tile
  int ku = 2;           // (row pair, word) units per thread
};

kk_status set_error(kk_status st, const char* fmt, ...);
void acceptance_table(double omega, uint64_t T[7], Accept* acc);
uint64_t place_count(int L, int H, double composition);
void tri_default_tile(int L, int H, bool mpkk, int* tw, int* tr);
int max_threads(int ku);
bool cyclic_fits(int L);
void default_tile(int L, int layout, TileConfig* tc);
int tile_geometry(int L, const TileConfig& tc, SweepParams* p);
bool tile_valid(int L, const TileConfig& tc, std::string* why);

}  // namespace kk

// A simulation handle (the opaque kk_sim of kk.h).
struct kk_sim {
  int L = 0;                             // sites per row
  int H = 0;                             // rows (H == L on the square torus)
  int layout = 0;
  double composition = 0, omega = 0;
  uint64_t seed = 0;
  uint32_t k0 = 0, k1 = 0;
  uint64_t t = 0;
  uint64_t attempts = 0;
  void* lat[2] = {nullptr, nullptr};
  int cur = 0;
  unsigned long long* counters = nullptr;  // [0] unused, [1] energy scratch
  unsigned long long* partials = nullptr;  // accepted moves, one running sum per sweep tile
  size_t npartials = 0;
  uint64_t accepted_base = 0;              // accepted moves folded in from earlier tile shapes
  hipStream_t stream = nullptr;
  bool own_stream = false;
  int device = 0;
  uint64_t T[7] = {};
  kk::Accept acc{};
  kk::TileConfig tile{};
  kk::CclBuffers ccl{};
  bool ccl_ready = false;
  uint32_t* hist_host = nullptr;  // pinned image of the histogram block (hist_enqueue)
  int geom = 0;                          // 0 square torus; triangular helical int8 ring: 1 with the
                                         // conflict-free 16 classes, 2 with the literal MPKK cover
  kk::TriAccept tacc{};                  // triangular thresholds
  int tri_tw = 0, tri_tr = 0;            // whole-sweep tile of the class schedule (0: one launch per class;
                                         // L x H: the whole ring in one workgroup)
  uint64_t epoch = 0;                    // bumped whenever the lattice may change
  uint64_t hist_epoch = ~(uint64_t)0;    // epoch and species of the cached histogram
  int hist_species = -1;
  std::vector<kk_hist_entry> hist_cache;
  bool poisoned = false;
};

namespace kk {
// helpers shared with the batch engine (kk_api.cpp)
kk_status device_alloc(void** p, size_t bytes);
// cluster histograms: a handle's labelling is enqueued on a stream and read
// back after that stream drains, so that many handles share one wait
constexpr unsigned kHistBigPrefix = 1024;  // large sizes copied back with the histogram
bool hist_cached(const kk_sim* h, int species);
kk_status hist_buffers(kk_sim* h);  // the labelling buffers and the pinned image, made once
kk_status hist_enqueue(kk_sim* h, int species, hipStream_t stream);
kk_status hist_finish(kk_sim* h, int species);
kk_status fold_accepted(kk_sim* h, const unsigned long long* dev_counts, size_t n);

// batch engine over borrowed handles (kk_batch.cpp), used by the job server:
// the batch never destroys these sims; replan after the set changes.
kk_status create_handle(kk_sim** out, uint32_t L, uint32_t H, int geom, double composition, double omega_kT,
                        uint64_t seed, int lay, void* hip_stream);
kk_status batch_over(const std::vector<kk_sim*>& sims, const std::vector<uint64_t>& sweeps, void* hip_stream,
                     kk_batch** out);
kk_status batch_replan(kk_batch* b, const std::vector<kk_sim*>& sims, const std::vector<uint64_t>& sweeps);
kk_status batch_set_sweeps(kk_batch* b, const std::vector<uint64_t>& sweeps);
}  // namespace kk
