// kk_tri.hpp -- launchers of the triangular-lattice kernels (kk_tri.hip).
#pragma once

#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

namespace kk {

// Triangular lattice, helical boundaries (kk_tri.hip): H rows of L sites on
// one ring of N = L*H.  Conflict-free classes: one launch per phase.  The
// literal MPKK variant: one launch per iteration, ping-pong buffers.
constexpr int kTriPartials = 64;  // accepted-move sums, indexed by workgroup % kTriPartials
struct TriAccept {
  uint64_t T[11];  // U < T[n] accepts, n = unlike neighbours of the pair (each excluding the other)
};
hipError_t launch_tri_phase(uint8_t* lat, int L, int H, uint32_t k0, uint32_t k1, uint64_t t, int p,
                            const TriAccept& acc, unsigned long long* partials, hipStream_t stream);
// Whole-sweep tiles (16 phases per launch on an LDS window, `in` -> `out`).
constexpr uint32_t kTriHalo = 33;  // 2 cells per phase, plus 1 for the first phase's reads
__host__ __device__ inline uint32_t tri_window_stride(uint32_t TW) {
  const uint32_t s = (TW + 2 * kTriHalo + 3u) & ~3u;  // whole words, an odd number of them
  return ((s >> 2) & 1u) ? s : s + 4u;
}
// Per workgroup, after the window: each of the 16 waves keeps a ring of 128
// pending centres (8 bytes each) whose pair is unlike, so that the decisions
// run on full waves (tri_tile_sweep).
constexpr uint32_t kTriQueue = 128, kTriQueueBytes = 16u * kTriQueue * 8u;
__host__ __device__ inline size_t tri_window_area(uint32_t TW, uint32_t TR) {
  return ((size_t)tri_window_stride(TW) * (TR + 2 * kTriHalo) + 7u) & ~(size_t)7u;
}
__host__ __device__ inline size_t tri_window_bytes(uint32_t TW, uint32_t TR) {
  return tri_window_area(TW, TR) + kTriQueueBytes;
}
inline bool tri_tile_fits(int L, int H, int TW, int TR) {
  return TW >= 16 && TR >= 16 && TW + 2 * (int)kTriHalo <= L && TR + 2 * (int)kTriHalo <= H &&
         tri_window_bytes((uint32_t)TW, (uint32_t)TR) <= 160u * 1024u - 1024u;
}
// The whole ring in one workgroup's LDS (small lattices): N = L * H bytes.
constexpr size_t kTriResidentMaxBytes = 160u * 1024u - 1024u;
inline bool tri_resident_fits(int L, int H) {
  return (size_t)L * (size_t)H <= kTriResidentMaxBytes;
}
struct TriResidentRep {
  uint8_t* lat;  // the current buffer, updated in place
  uint32_t L, H, sweeps;
  uint32_t k0, k1;
  uint64_t t0;
  TriAccept acc;
  unsigned long long* partials;
};
// Workgroup b runs replica b (reps[b].sweeps sweeps); lds_bytes = the largest N.
hipError_t launch_tri_resident(const TriResidentRep* reps, uint32_t nreps, size_t lds_bytes, hipStream_t stream);
// One replica, its descriptor passed by value.
hipError_t launch_tri_resident_one(const TriResidentRep& rep, size_t lds_bytes, hipStream_t stream);
constexpr uint64_t kTriResidentChunk = 1024;  // sweeps per launch of a single handle

// One replica of a batched launch of whole-sweep tiles.  Sweep k of a run reads
// lat[cur ^ (k & 1)] and writes the other buffer with sweep counter t0 + k.
struct TriBatchRep {
  uint8_t* lat[2];
  uint32_t L, H, TW, TR, ntx, cur;
  uint32_t k0, k1;
  uint64_t t0;
  TriAccept acc;
  unsigned long long* partials;  // kTriPartials sums of the replica
};
// jobs[b] = (replica, tile) for workgroup b; lds_bytes = the largest window.
hipError_t launch_tri_tile_sweep_batch(const TriBatchRep* reps, const uint2* jobs, uint32_t njobs, uint32_t k,
                                       size_t lds_bytes, hipStream_t stream);
hipError_t launch_tri_tile_sweep(const uint8_t* in, uint8_t* out, int L, int H, int TW, int TR, uint32_t k0,
                                uint32_t k1, uint64_t t, const TriAccept& acc, unsigned long long* partials,
                                hipStream_t stream);
// Whole-step MPKK tiles (7 iterations per launch on an LDS window, `in` -> `out`).
constexpr uint32_t kMpkkHalo = 21;  // 3 cells per iteration
__host__ __device__ inline uint32_t mpkk_window_stride(uint32_t TW) {
  const uint32_t s = (TW + 2 * kMpkkHalo + 3u) & ~3u;  // whole words, an odd number of them
  return ((s >> 2) & 1u) ? s : s + 4u;
}
// The window, then the per-wave rings of pending attempts (as for the class
// schedule's tile kernel).
__host__ __device__ inline size_t mpkk_window_area(uint32_t TW, uint32_t TR) {
  return ((size_t)mpkk_window_stride(TW) * (TR + 2 * kMpkkHalo) + 15u) & ~(size_t)15u;
}
__host__ __device__ inline size_t mpkk_window_bytes(uint32_t TW, uint32_t TR) {
  return mpkk_window_area(TW, TR) + kTriQueueBytes;
}
inline bool mpkk_tile_fits(int L, int H, int TW, int TR) {
  return TW >= 16 && TR >= 16 && TW + 2 * (int)kMpkkHalo <= L && TR + 2 * (int)kMpkkHalo <= H &&
         mpkk_window_bytes((uint32_t)TW, (uint32_t)TR) <= 160u * 1024u - 1024u;
}
hipError_t launch_mpkk_tile_step(const uint8_t* in, uint8_t* out, int L, int H, int TW, int TR, uint32_t k0,
                                 uint32_t k1, uint64_t t, const TriAccept& acc, unsigned long long* partials,
                                 hipStream_t stream);
hipError_t launch_mpkk_iteration(const uint8_t* in, uint8_t* out, int L, int H, uint32_t k0, uint32_t k1, uint64_t t,
                                 int j, const TriAccept& acc, unsigned long long* partials, hipStream_t stream);
hipError_t launch_tri_energy(const uint8_t* lat, int L, int H, unsigned long long* out, hipStream_t stream);
hipError_t launch_tri_similar(const uint8_t* lat, int L, int H, uint32_t k0, uint32_t k1, uint64_t t,
                              unsigned long long* out, hipStream_t stream);

}  // namespace kk
