// kk_kernels.hpp -- launch parameter blocks and host-side launchers of the
// libkk HIP kernels (internal to the library; the public API is kk.h).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "kk_common.hpp"

namespace kk {

constexpr int kLayoutInt8 = 1;  // one byte (0/1) per site, row-major
constexpr int kLayoutBits = 2;  // one bit per site, L/32 words per row, bit b of word g = site 32g + b

struct SweepParams {
  const void* src;
  void* dst;
  unsigned long long* accepted;  // one running sum per tile (grid index)
  int L, wpr;                // side; words per row of the bit-packed layout
  int tww, th;               // interior words / rows per tile
  int hx, hy;                // halo words / rows on each side (1/16, or 0/0 for the cyclic tile)
  int tiles_x;
  int C, R;                  // LDS words per row, rows (tile + halo)
  int row0, npairs, nunits;  // first computed LDS row, computed row pairs, units = pairs * C
  int nsweeps;               // sweeps in this launch
  int layout;                // kLayoutInt8 or kLayoutBits (read by the batch kernels)
  uint32_t k0, k1;           // Philox key (seed)
  uint64_t t0;               // first sweep index
  Accept acc;
};

hipError_t launch_sweep(const SweepParams& p, int layout, bool cyclic, int ku, int threads, hipStream_t stream);

// Batch kernels.  Tiled replicas: one workgroup per (replica, tile) job and one
// launch per sweep; ctl[0] holds the run sweep at which the current chunk of a
// captured graph starts, each tile launch adds its position `rel` in the chunk,
// and launch_batch_advance (one thread, the last node of a branch) moves ctl[0]
// on by the chunk, so the graph replays unchanged.  A replica runs p.nsweeps sweeps from
// p.t0, ping-ponging between p.src (its lattice at the start) and p.dst.  Resident replicas (L % 32 == 0,
// 2 <= L/32 <= kResidentMaxC): one launch, one workgroup per replica running
// all of its sweeps with the whole lattice in LDS.
constexpr int kBatchMaxTww = 16, kBatchTh = 128, kBatchThreads = 768;
// Tiled replicas run in 512-thread workgroups, ku (1 or 2) units per thread,
// in tiles 8 or 16 words wide: a tile of tww words by th rows fits when its
// (th + 28) / 2 computed row pairs times tww + 2 words stay within ku * 512
// units.
constexpr int kBatchTileThreads = 512;
constexpr bool batch_tile_fits(int tww, int th, int ku = 2) {
  return (tww == 8 || tww == 16) && (ku == 1 || ku == 2) && th >= 2 && th <= kBatchTh &&
         ((th + 28) / 2) * (tww + 2) <= ku * kBatchTileThreads;
}
struct BatchTileJob {
  int rep, tile;
};
hipError_t launch_batch_tiles(const SweepParams* reps, const BatchTileJob* jobs, int njobs, const unsigned* ctl,
                              unsigned rel, int ku, hipStream_t stream);
hipError_t launch_batch_advance(unsigned* ctl, unsigned step, hipStream_t stream);
// small: the 256-thread kernel for replicas of at most kResidentSmallMaxC words
// per row.  A launch runs up to kBatchChunk sweeps from sweep ctl[0] of the run
// (launch_batch_advance then moves ctl[0] on by kBatchChunk).
hipError_t launch_batch_resident(const SweepParams* reps, const int* ids, int n, size_t lds_bytes, bool small,
                                 const unsigned* ctl, hipStream_t stream);
// Sweeps per replay of a batch graph: kBatchChunk tile launches per tile group
// and one resident launch of kBatchChunk sweeps.
constexpr int kBatchChunk = 64;
constexpr int kResidentMaxC = 9;
constexpr int kResidentSmallMaxC = 5, kResidentSmallThreads = 256;
size_t batch_tile_lds_bytes();
size_t batch_resident_lds_bytes(int L);

// N_AB (unlike nearest-neighbour bonds) added into *out.
hipError_t launch_energy(const void* lat, int layout, int L, unsigned long long* out, hipStream_t stream);

// Count of sites whose randomly drawn neighbour has the same type, added into *out.
hipError_t launch_similar_sampled(const void* lat, int layout, int L, uint32_t k0, uint32_t k1, uint64_t t,
                                 unsigned long long* out, hipStream_t stream);

// Initial placement.
hipError_t launch_init_keys(uint64_t* keys, int L, int H, uint32_t k0, uint32_t k1, hipStream_t stream);
hipError_t launch_radix_hist(const uint64_t* keys, size_t n, uint64_t prefix, int shift, unsigned* hist256,
                             hipStream_t stream);
hipError_t launch_init_mark(const uint64_t* keys, int L, int H, int layout, uint64_t kth, void* lat, unsigned* eq_count,
                            uint32_t* eq_list, unsigned eq_cap, hipStream_t stream);
hipError_t launch_set_sites(const uint32_t* idx, unsigned n, int L, int layout, void* lat, hipStream_t stream);

// Connected components of one species (4-neighbour, periodic) and their size histogram.
struct CclBuffers {
  uint32_t* parent;     // N
  uint32_t* size;       // N
  unsigned* hist;       // small-size histogram, kSmallSizes entries
  uint32_t* big;        // sizes >= kSmallSizes, appended
  unsigned* big_count;  // number of appended sizes
  unsigned big_cap;
};
constexpr int kSmallSizes = 4096;
// triangular: six neighbours under helical boundaries (the int8 ring of kk_tri.hip).
hipError_t launch_ccl(const void* lat, int layout, int L, int H, int species, const CclBuffers& b, bool triangular,
                      hipStream_t stream);

// Segregated start: sites 0 .. n1-1 (index y*L + x) set to 1, the rest 0.
hipError_t launch_fill_segregated(void* lat, int layout, int L, int H, uint64_t n1, hipStream_t stream);

// int8 <-> bit-packed conversion on the device (bit-packed needs L % 32 == 0).
hipError_t launch_pack(const uint8_t* in, uint32_t* out, int L, hipStream_t stream);
hipError_t launch_unpack(const uint32_t* in, uint8_t* out, int L, hipStream_t stream);

}  // namespace kk
