// kk_common.hpp -- device helpers and launch parameter blocks shared by the
// HIP kernels of libkk.  Written for gfx950 (CDNA4, wave64).
//
// The random-number layout, class schedule and acceptance rule implemented
// here are the ones fixed for the square-lattice version of the paper's
// Massive Parallel Kawasaki Kinetics (section "Massive Parallel Kawasaki
// Kinetics"): a 4-neighbour torus, 8 conflict-free centre classes visited in
// a per-sweep random order, Philox4x32-10 counters keyed by the seed, and a
// 42-bit Metropolis threshold (section "Monte Carlo model with Kawasaki based
// kinetics", the Metropolis criterion and the omega_AB interaction).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace kk {

// Stream tags (top 4 bits of the fourth Philox counter word).
constexpr uint32_t kTagSweep = 1u;  // per-sweep bit-sliced random planes
constexpr uint32_t kTagExt = 2u;    // low 32 bits of a 42-bit uniform (ties only)
constexpr uint32_t kTagOrder = 3u;  // per-sweep class order
constexpr uint32_t kTagInit = 4u;   // initial-placement sort keys
constexpr uint32_t kTagObserve = 5u;  // random-neighbour draws of the observables

constexpr int kPlanes = 12;  // 2 direction planes + 10 uniform-prefix planes

struct Philox4 {
  uint32_t x, y, z, w;
};

// Philox4x32-10 (Salmon et al., SC'11).  The key schedule is uniform across a
// wavefront, so the compiler keeps it in SGPRs; each round is two
// v_mad_u64_u32 and two three-input xors per lane.
__device__ __forceinline__ Philox4 philox10(uint32_t c0, uint32_t c1, uint32_t c2, uint32_t c3,
                                            uint32_t k0, uint32_t k1) {
#pragma unroll
  for (int i = 0; i < 10; ++i) {
    const uint64_t p0 = (uint64_t)c0 * 0xD2511F53u;
    const uint64_t p1 = (uint64_t)c2 * 0xCD9E8D57u;
    // three-input xors as one v_bitop3_b32 each (truth table 0x96 = a ^ b ^ c)
    const uint32_t n0 = __builtin_amdgcn_bitop3_b32((uint32_t)(p1 >> 32), c1, k0, 0x96);
    const uint32_t n2 = __builtin_amdgcn_bitop3_b32((uint32_t)(p0 >> 32), c3, k1, 0x96);
    c1 = (uint32_t)p1;
    c3 = (uint32_t)p0;
    c0 = n0;
    c2 = n2;
    k0 += 0x9E3779B9u;
    k1 += 0xBB67AE85u;
  }
  return Philox4{c0, c1, c2, c3};
}

__host__ __device__ __forceinline__ uint32_t ctr_hi(uint64_t t, uint32_t tag) {
  return (uint32_t)((t >> 32) & 0x0FFFFFFFu) | (tag << 28);
}

__device__ __forceinline__ int imod(int v, int m) {
  int r = v % m;
  return r < 0 ? r + m : r;
}

// Fisher-Yates order of the 8 classes for sweep t.
__device__ __forceinline__ uint32_t class_order(uint32_t k0, uint32_t k1, uint64_t t) {
  const uint32_t tl = (uint32_t)t, th = ctr_hi(t, kTagOrder);
  const Philox4 a = philox10(0u, 0u, tl, th, k0, k1);
  const Philox4 b = philox10(0u, 1u, tl, th, k0, k1);
  const uint32_t w[8] = {a.x, a.y, a.z, a.w, b.x, b.y, b.z, b.w};
  // perm packed as 8 nibbles: nibble p = class of phase p
  uint32_t perm = 0x76543210u;
#pragma unroll
  for (int i = 7; i >= 1; --i) {
    const uint32_t j = (uint32_t)(((uint64_t)w[7 - i] * (uint64_t)(i + 1)) >> 32);
    const uint32_t vi = (perm >> (4 * i)) & 0xFu, vj = (perm >> (4 * j)) & 0xFu;
    perm &= ~((0xFu << (4 * i)) | (0xFu << (4 * j)));
    perm |= (vj << (4 * i)) | (vi << (4 * j));
  }
  return perm;
}

// Acceptance parameters for one lattice.  For an unlike pair with n unlike
// neighbours (excluding each other) the bit-sliced counter yields m = n + 1.
// For omega > 0 only m in {1,2,3} (dU = 6,4,2) can be rejected; for
// omega < 0 only m in {5,6,7}.  Slot j (0..2) holds the threshold for
// m & 3 == j + 1: its top 10 bits (compared with the uniform prefix) and low
// 32 bits (compared with the extension word on a tie).
struct Accept {
  uint32_t hi[3];
  uint32_t lo[3];
  uint32_t restricted;  // 0xFFFFFFFF when some move can be rejected (omega != 0)
  uint32_t negmask;     // 0xFFFFFFFF when omega < 0
};

// Tile of workgroup b in a grid of n tiles numbered row by row.  Workgroups
// are dispatched to the 8 XCDs in turn (workgroup b to XCD b mod 8), and each
// XCD has its own L2: this gives every XCD a contiguous run of tile numbers,
// i.e. a band of tile rows, so that most of the rows a tile stages were written
// through the same L2 by the previous launch.  A bijection on [0, n) for any
// n; which workgroup sweeps a tile does not affect the result.
__host__ __device__ __forceinline__ int xcd_tile(int b, int n) {
  constexpr int kXcds = 8;
  const int per = (n + kXcds - 1) / kXcds;  // tiles of each of the first `tall` XCDs
  const int tall = n - (per - 1) * kXcds;   // 1..8 XCDs take `per` tiles, the rest per - 1
  const int x = b % kXcds, l = b / kXcds;
  return x < tall ? x * per + l : tall * per + (x - tall) * (per - 1) + l;
}

}  // namespace kk
