// kk_tri.hip -- the triangular lattice with helical boundary conditions, the
// paper's own model (Materials and Methods, "Monte Carlo model with Kawasaki
// based kinetics", Fig. 2; six neighbours under helical boundaries, "Cluster
// Analysis methods"), and the paper's literal MPKK on it ("Massive Parallel
// Kawasaki Kinetics", Fig. 4).  Gfx950 (CDNA4, wave64).
//
// H rows of L sites, i = y*L + x, 0 <= i < N = L*H, form one ring; the
// neighbours of i are i +- 1, i +- L and i +- (L - 1) modulo N.  The lattice is
// stored one byte per site.
//
// Conflict-free schedule: class(i) = i mod 16, which for L % 8 == 4 and
// H % 4 == 0 puts two sites of a class at least 4 steps apart, so the
// exchanges of one class never read a site another writes; a sweep runs the 16
// classes in a random order, one launch per class, in place.  Random numbers:
//   site i at sweep t: Philox block (i/2, 0, t_lo, t_hi28 | 6<<28), words
//   2(i%2) (direction, d = (w * 6) >> 32 picks +1, -1, +L, -L, +(L-1),
//   -(L-1)) and 2(i%2)+1 (the 32-bit uniform U);
//   class order: blocks (j, 0, t_lo, t_hi28 | 7<<28), j = 0..3, Fisher-Yates
//   over 16 (step i swaps entries i and (w[15-i] * (i+1)) >> 32).
// An attempt with n unlike neighbours of the centre and the partner (each
// other excluded, n in 0..10) changes N_AB by 10 - 2n and is accepted iff
// U < T[n] = min(2^32, ceil(exp(-omega (10 - 2n)) 2^32)).
//
// Literal MPKK: for L % 7 in {3, 5} and H % 7 == 0 the 7-site domains (a
// centre and its six neighbours) centred on c = k (mod 7) partition the ring.
// A step is 7 iterations j; iteration j draws k_j = (w * 7) >> 32 from word
// j%4 of block (j/4, 2, t_lo, t_hi28 | 8<<28) and makes one attempt in every
// domain m (centre k_j + 7m) with the direction and U of block (m/2, j, t_lo,
// t_hi28 | 9<<28), words 2(m%2) and 2(m%2)+1.  Every domain decides from the
// lattice as it stood at the start of the iteration (read from one buffer,
// written whole to the other), which is how simultaneous exchanges are read.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "kk_common.hpp"
#include "kk_kernels.hpp"

namespace kk {
namespace {

constexpr uint32_t kTagTri = 6u, kTagTriOrder = 7u, kTagMpkkK = 8u, kTagMpkk = 9u;

__device__ __forceinline__ uint32_t tri_nb(uint32_t i, uint32_t d, uint32_t L, uint32_t N) {
  // +1, -1, +L, -L, +(L-1), -(L-1) on the ring of N sites
  const uint32_t mag = d < 2 ? 1u : (d < 4 ? L : L - 1u);
  if ((d & 1u) == 0u) {
    const uint32_t j = i + mag;
    return j >= N ? j - N : j;
  }
  return i >= mag ? i - mag : i + N - mag;
}

__device__ __forceinline__ uint32_t tri_order(uint32_t k0, uint32_t k1, uint64_t t, int p) {
  const uint32_t tl = (uint32_t)t, th = ctr_hi(t, kTagTriOrder);
  uint32_t w[16];
#pragma unroll
  for (int j = 0; j < 4; ++j) {
    const Philox4 b = philox10((uint32_t)j, 0u, tl, th, k0, k1);
    w[4 * j] = b.x;
    w[4 * j + 1] = b.y;
    w[4 * j + 2] = b.z;
    w[4 * j + 3] = b.w;
  }
  // the permutation as 16 nibbles of one 64-bit word (nibble e = entry e)
  uint64_t perm = 0xFEDCBA9876543210ull;
#pragma unroll
  for (int i = 15; i >= 1; --i) {
    const int k = (int)(((uint64_t)w[15 - i] * (uint64_t)(i + 1)) >> 32);
    const uint64_t vi = (perm >> (4 * i)) & 0xFull, vk = (perm >> (4 * k)) & 0xFull;
    perm &= ~((0xFull << (4 * i)) | (0xFull << (4 * k)));
    perm |= (vk << (4 * i)) | (vi << (4 * k));
  }
  return (uint32_t)((perm >> (4 * p)) & 0xFull);
}

__device__ __forceinline__ int tri_unlike_except(const uint8_t* s, uint32_t i, uint32_t other, uint32_t L,
                                                 uint32_t N) {
  const uint8_t v = s[i];
  int n = 0;
#pragma unroll
  for (uint32_t d = 0; d < 6; ++d) {
    const uint32_t j = tri_nb(i, d, L, N);
    n += (j != other) & (s[j] != v);
  }
  return n;
}

__device__ __forceinline__ void block_count(unsigned long long cnt, unsigned long long* red,
                                            unsigned long long* partials) {
  for (int off = 32; off > 0; off >>= 1) cnt += __shfl_down(cnt, off, 64);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = cnt;
  __syncthreads();
  if (threadIdx.x == 0) {
    const unsigned long long tot = red[0] + red[1] + red[2] + red[3];
    if (tot) atomicAdd(&partials[blockIdx.x % kTriPartials], tot);
  }
}

// One phase (class perm[p] of sweep t): one thread per centre.
__global__ __launch_bounds__(256) void tri_phase(uint8_t* s, uint32_t L, uint32_t N, uint32_t k0, uint32_t k1,
                                                 uint64_t t, int p, TriAccept acc, unsigned long long* partials) {
  __shared__ uint32_t cls_s;
  __shared__ unsigned long long red[4];
  if (threadIdx.x < 64) {
    const uint32_t c = tri_order(k0, k1, t, p);
    if (threadIdx.x == 0) cls_s = c;
  }
  __syncthreads();
  const uint32_t cls = cls_s;
  const uint32_t M = N >> 4;
  const uint32_t tl = (uint32_t)t, th = ctr_hi(t, kTagTri);
  unsigned long long cnt = 0;
  for (uint32_t j = blockIdx.x * blockDim.x + threadIdx.x; j < M; j += gridDim.x * blockDim.x) {
    const uint32_t i = cls + 16u * j;
    const Philox4 r = philox10(i >> 1, 0u, tl, th, k0, k1);
    const uint32_t wd = (i & 1u) ? r.z : r.x, u = (i & 1u) ? r.w : r.y;
    const uint32_t d = (uint32_t)(((uint64_t)wd * 6u) >> 32);
    const uint32_t b = tri_nb(i, d, L, N);
    const uint8_t si = s[i], sb = s[b];
    if (si == sb) continue;
    const int n = tri_unlike_except(s, i, b, L, N) + tri_unlike_except(s, b, i, L, N);
    if ((uint64_t)u < acc.T[n]) {
      s[i] = sb;
      s[b] = si;
      ++cnt;
    }
  }
  block_count(cnt, red, partials);
}

// One literal-MPKK iteration: one thread per domain, decisions from `in`, the
// whole domain written to `out` (the domains partition the ring, so every
// site of `out` is written exactly once).
__global__ __launch_bounds__(256) void mpkk_iter(const uint8_t* __restrict__ in, uint8_t* __restrict__ out,
                                                 uint32_t L, uint32_t N, uint32_t k0, uint32_t k1, uint64_t t, int j,
                                                 TriAccept acc, unsigned long long* partials) {
  __shared__ uint32_t k_s;
  __shared__ unsigned long long red[4];
  const uint32_t tl = (uint32_t)t;
  if (threadIdx.x == 0) {
    const Philox4 b = philox10((uint32_t)(j >> 2), 2u, tl, ctr_hi(t, kTagMpkkK), k0, k1);
    const uint32_t w = (j & 3) == 0 ? b.x : (j & 3) == 1 ? b.y : (j & 3) == 2 ? b.z : b.w;
    k_s = (uint32_t)(((uint64_t)w * 7u) >> 32);
  }
  __syncthreads();
  const uint32_t k = k_s, M = N / 7u, th = ctr_hi(t, kTagMpkk);
  unsigned long long cnt = 0;
  for (uint32_t m = blockIdx.x * blockDim.x + threadIdx.x; m < M; m += gridDim.x * blockDim.x) {
    const uint32_t c = k + 7u * m;
    const Philox4 r = philox10(m >> 1, (uint32_t)j, tl, th, k0, k1);
    const uint32_t wd = (m & 1u) ? r.z : r.x, u = (m & 1u) ? r.w : r.y;
    const uint32_t d = (uint32_t)(((uint64_t)wd * 6u) >> 32);
    const uint32_t b = tri_nb(c, d, L, N);
    uint8_t vc = in[c], vb = in[b];
    if (vc != vb) {
      const int n = tri_unlike_except(in, c, b, L, N) + tri_unlike_except(in, b, c, L, N);
      if ((uint64_t)u < acc.T[n]) {
        const uint8_t x = vc;
        vc = vb;
        vb = x;
        ++cnt;
      }
    }
    out[c] = vc;
#pragma unroll
    for (uint32_t e = 0; e < 6; ++e) {
      const uint32_t q = tri_nb(c, e, L, N);
      out[q] = (q == b) ? vb : in[q];
    }
  }
  block_count(cnt, red, partials);
}

// N_AB over the 3N bonds (i, i+1), (i, i+L), (i, i+L-1).
__global__ __launch_bounds__(256) void tri_energy(const uint8_t* s, uint32_t L, uint32_t N, unsigned long long* out) {
  unsigned long long a = 0;
  for (uint32_t i = blockIdx.x * blockDim.x + threadIdx.x; i < N; i += gridDim.x * blockDim.x) {
    const uint8_t v = s[i];
    a += (v != s[tri_nb(i, 0, L, N)]) + (v != s[tri_nb(i, 2, L, N)]) + (v != s[tri_nb(i, 4, L, N)]);
  }
  for (int off = 32; off > 0; off >>= 1) a += __shfl_down(a, off, 64);
  if ((threadIdx.x & 63) == 0 && a) atomicAdd(out, a);
}

// Random-neighbour draw: site i uses word i%4 of block (i/4, 1, t_lo, t_hi28 | 5<<28).
__global__ __launch_bounds__(256) void tri_similar(const uint8_t* s, uint32_t L, uint32_t N, uint32_t k0, uint32_t k1,
                                                   uint64_t t, unsigned long long* out) {
  const uint32_t Q = (N + 3u) >> 2;
  const uint32_t tl = (uint32_t)t, th = ctr_hi(t, kTagObserve);
  unsigned long long a = 0;
  for (uint32_t q = blockIdx.x * blockDim.x + threadIdx.x; q < Q; q += gridDim.x * blockDim.x) {
    const Philox4 r = philox10(q, 1u, tl, th, k0, k1);
    const uint32_t w[4] = {r.x, r.y, r.z, r.w};
#pragma unroll
    for (uint32_t m = 0; m < 4; ++m) {
      const uint32_t i = 4u * q + m;
      if (i >= N) break;
      const uint32_t d = (uint32_t)(((uint64_t)w[m] * 6u) >> 32);
      a += (s[i] == s[tri_nb(i, d, L, N)]);
    }
  }
  for (int off = 32; off > 0; off >>= 1) a += __shfl_down(a, off, 64);
  if ((threadIdx.x & 63) == 0 && a) atomicAdd(out, a);
}

int tri_grid(size_t n) {
  const size_t g = (n + 255) / 256;
  return (int)(g < 8192 ? (g < 1 ? 1 : g) : 8192);
}

}  // namespace

hipError_t launch_tri_phase(uint8_t* lat, int L, int H, uint32_t k0, uint32_t k1, uint64_t t, int p,
                            const TriAccept& acc, unsigned long long* partials, hipStream_t stream) {
  const uint32_t N = (uint32_t)L * (uint32_t)H;
  hipLaunchKernelGGL(tri_phase, dim3(tri_grid(N / 16)), dim3(256), 0, stream, lat, (uint32_t)L, N, k0, k1, t, p, acc,
                     partials);
  return hipGetLastError();
}

hipError_t launch_mpkk_iteration(const uint8_t* in, uint8_t* out, int L, int H, uint32_t k0, uint32_t k1, uint64_t t,
                                 int j, const TriAccept& acc, unsigned long long* partials, hipStream_t stream) {
  const uint32_t N = (uint32_t)L * (uint32_t)H;
  hipLaunchKernelGGL(mpkk_iter, dim3(tri_grid(N / 7)), dim3(256), 0, stream, in, out, (uint32_t)L, N, k0, k1, t, j,
                     acc, partials);
  return hipGetLastError();
}

hipError_t launch_tri_energy(const uint8_t* lat, int L, int H, unsigned long long* out, hipStream_t stream) {
  const uint32_t N = (uint32_t)L * (uint32_t)H;
  hipLaunchKernelGGL(tri_energy, dim3(tri_grid(N)), dim3(256), 0, stream, lat, (uint32_t)L, N, out);
  return hipGetLastError();
}

hipError_t launch_tri_similar(const uint8_t* lat, int L, int H, uint32_t k0, uint32_t k1, uint64_t t,
                              unsigned long long* out, hipStream_t stream) {
  const uint32_t N = (uint32_t)L * (uint32_t)H;
  hipLaunchKernelGGL(tri_similar, dim3(tri_grid((N + 3) / 4)), dim3(256), 0, stream, lat, (uint32_t)L, N, k0, k1, t,
                     out);
  return hipGetLastError();
}

}  // namespace kk
