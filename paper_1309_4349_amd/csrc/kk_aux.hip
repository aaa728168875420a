// kk_aux.hip -- initial placement, energy, cluster labelling and layout
// conversion kernels of libkk.
#include "kk_common.hpp"
#include "kk_kernels.hpp"
#include "kk_ccl.hpp"

namespace kk {

namespace {

constexpr uint32_t kNone = 0xFFFFFFFFu;
// workgroups per replica in a many-lattice labelling pass (grid-stride beyond)
constexpr int kCclManyBlocks = 512;

__device__ __forceinline__ int site_bit(const void* lat, int layout, int L, int x, int y) {
  if (layout == kLayoutBits)
    return (int)((static_cast<const uint32_t*>(lat)[(size_t)y * (L >> 5) + (x >> 5)] >> (x & 31)) & 1u);
  return (int)(static_cast<const uint8_t*>(lat)[(size_t)y * L + x] & 1u);
}

// ---------------------------------------------------------------------------
// Energy: N_AB = sum over sites of [s(x,y) != s(x+1,y)] + [s(x,y) != s(x,y+1)]
// (the Almeida one-parameter model, E/kT = omega * N_AB + const).
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void energy_bits(const uint32_t* lat, int L, unsigned long long* out) {
  const int wpr = L >> 5;
  const size_t nw = (size_t)L * wpr;
  unsigned long long acc = 0;
  for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < nw; i += (size_t)gridDim.x * blockDim.x) {
    const int y = (int)(i / wpr), g = (int)(i - (size_t)y * wpr);
    const uint32_t v = lat[i];
    const uint32_t nxt = lat[(size_t)y * wpr + (g + 1 == wpr ? 0 : g + 1)];
    const uint32_t east = __builtin_amdgcn_alignbit(nxt, v, 1);
    const uint32_t below = lat[(size_t)(y + 1 == L ? 0 : y + 1) * wpr + g];
    acc += (unsigned)__builtin_popcount(v ^ east) + (unsigned)__builtin_popcount(v ^ below);
  }
  for (int off = 32; off > 0; off >>= 1) acc += __shfl_down(acc, off, 64);
  if ((threadIdx.x & 63) == 0 && acc) atomicAdd(out, acc);
}

__global__ __launch_bounds__(256) void energy_int8(const uint8_t* lat, int L, unsigned long long* out) {
  const size_t n = (size_t)L * L;
  unsigned long long acc = 0;
  for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x) {
    const int y = (int)(i / L), x = (int)(i - (size_t)y * L);
    const uint8_t v = lat[i];
    acc += (v != lat[(size_t)y * L + (x + 1 == L ? 0 : x + 1)]);
    acc += (v != lat[(size_t)(y + 1 == L ? 0 : y + 1) * L + x]);
  }
  for (int off = 32; off > 0; off >>= 1) acc += __shfl_down(acc, off, 64);
  if ((threadIdx.x & 63) == 0 && acc) atomicAdd(out, acc);
}

// Random-neighbour estimate of the similar first-neighbour fraction: every
// site draws one of its 4 neighbours (top two bits of its word of Philox block
// (y, x / 4, t, tag 5): +x, -x, +y, -y) and counts when both are of the same
// type.  One thread per 4-site group (one Philox block); L % 4 == 0.
__global__ __launch_bounds__(256) void similar_sampled(const void* lat, int layout, int L, uint32_t k0, uint32_t k1,
                                                       uint64_t t, unsigned long long* out) {
  const int g4 = L >> 2;
  const size_t n = (size_t)L * g4;
  const uint32_t tl = (uint32_t)t, th = ctr_hi(t, kTagObserve);
  unsigned long long acc = 0;
  for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x) {
    const int y = (int)(i / g4), q = (int)(i - (size_t)y * g4);
    const Philox4 r = philox10((uint32_t)y, (uint32_t)q, tl, th, k0, k1);
    const uint32_t w[4] = {r.x, r.y, r.z, r.w};
#pragma unroll
    for (int m = 0; m < 4; ++m) {
      const int x = 4 * q + m;
      const uint32_t dir = w[m] >> 30;
      int nx = x, ny = y;
      if (dir == 0u) nx = (x + 1 == L) ? 0 : x + 1;
      else if (dir == 1u) nx = (x == 0) ? L - 1 : x - 1;
      else if (dir == 2u) ny = (y + 1 == L) ? 0 : y + 1;
      else ny = (y == 0) ? L - 1 : y - 1;
      acc += (site_bit(lat, layout, L, x, y) == site_bit(lat, layout, L, nx, ny));
    }
  }
  for (int off = 32; off > 0; off >>= 1) acc += __shfl_down(acc, off, 64);
  if ((threadIdx.x & 63) == 0 && acc) atomicAdd(out, acc);
}

// ---------------------------------------------------------------------------
// Initial placement: each site's 64-bit key is Philox block (y, x, 0, tag 4)
// words 0 and 1; the n1 sites with the smallest (key, index) get type 1.
// The n1-th smallest key is found by an 8-pass MSB-first radix select.
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void init_keys(uint64_t* keys, int L, int H, uint32_t k0, uint32_t k1) {
  const size_t n = (size_t)L * H;
  for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x) {
    const uint32_t y = (uint32_t)(i / L), x = (uint32_t)(i - (size_t)y * L);
    const Philox4 r = philox10(y, x, 0u, kTagInit << 28, k0, k1);
    keys[i] = ((uint64_t)r.x << 32) | (uint64_t)r.y;
  }
}

__global__ __launch_bounds__(256) void radix_hist(const uint64_t* keys, size_t n, uint64_t prefix, int shift,
                                                  unsigned* hist) {
  __shared__ unsigned h[256];
  h[threadIdx.x] = 0;
  __syncthreads();
  const int hs = shift + 8;
  for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x) {
    const uint64_t k = keys[i];
    if (hs >= 64 || (k >> hs) == (prefix >> hs)) atomicAdd(&h[(k >> shift) & 0xFFu], 1u);
  }
  __syncthreads();
  if (h[threadIdx.x]) atomicAdd(&hist[threadIdx.x], h[threadIdx.x]);
}

__global__ __launch_bounds__(256) void init_mark(const uint64_t* keys, int L, int H, int layout, uint64_t kth,
                                                 void* lat, unsigned* eq_count, uint32_t* eq_list,
                                                 unsigned eq_cap) {
  if (layout == kLayoutBits) {
    const int wpr = L >> 5;
    const size_t nw = (size_t)H * wpr;
    for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < nw; i += (size_t)gridDim.x * blockDim.x) {
      uint32_t v = 0;
      const size_t base = i * 32;  // words tile rows exactly, so site index = 32 * word + bit
      for (int b = 0; b < 32; ++b) {
        const uint64_t k = keys[base + b];
        if (k < kth) v |= 1u << b;
        else if (k == kth) {
          const unsigned slot = atomicAdd(eq_count, 1u);
          if (slot < eq_cap) eq_list[slot] = (uint32_t)(base + b);
        }
      }
      static_cast<uint32_t*>(lat)[i] = v;
    }
  } else {
    const size_t n = (size_t)L * H;
    for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x) {
      const uint64_t k = keys[i];
      uint8_t v = 0;
      if (k < kth) v = 1;
      else if (k == kth) {
        const unsigned slot = atomicAdd(eq_count, 1u);
        if (slot < eq_cap) eq_list[slot] = (uint32_t)i;
      }
      static_cast<uint8_t*>(lat)[i] = v;
    }
  }
}

__global__ void set_sites(const uint32_t* idx, unsigned n, int L, int layout, void* lat) {
  const unsigned i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const uint32_t s = idx[i];
  if (layout == kLayoutBits) atomicOr(&static_cast<uint32_t*>(lat)[s >> 5], 1u << (s & 31u));
  else static_cast<uint8_t*>(lat)[s] = 1;
  (void)L;
}

// ---------------------------------------------------------------------------
// Cluster labelling: lock-free union-find with atomicMin on parent links
// (parents always point to smaller indices, so no cycle can form), then
// path flattening, per-root site counts and a size histogram.  Small sizes
// go to a dense histogram through a per-block LDS copy; the few sizes of
// kSmallSizes or more are appended to a list.
// ---------------------------------------------------------------------------
__device__ __forceinline__ uint32_t ld_parent(const uint32_t* parent, uint32_t x) {
  return __hip_atomic_load(&parent[x], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Root of x with path halving: every visited node is re-linked to its
// grandparent.  Links only ever decrease (atomicMin) and always point to an
// ancestor in the same tree, so concurrent finds and unions stay consistent.
__device__ __forceinline__ uint32_t find_root_halving(uint32_t* parent, uint32_t x) {
  uint32_t p = ld_parent(parent, x);
  while (p != x) {
    const uint32_t g = ld_parent(parent, p);
    if (g != p) atomicMin(&parent[x], g);
    x = p;
    p = g;
  }
  return x;
}

__device__ void unite(uint32_t* parent, uint32_t a, uint32_t b) {
  for (;;) {
    a = find_root_halving(parent, a);
    b = find_root_halving(parent, b);
    if (a == b) return;
    if (a > b) {
      const uint32_t t = a;
      a = b;
      b = t;
    }
    const uint32_t old = atomicMin(&parent[b], a);
    if (old == b) return;
    b = old;
  }
}

// With `runs` (the square torus), a site of the species starts linked
// straight to the first site of its run: the longest stretch of sites of the
// species that ends at it, lies in one row and in its 64-site segment (sites
// 64k .. 64k + 63, one wavefront of the pass: two ballots find it).  The
// merge pass then needs a horizontal union only at segment ends and across
// the row's wrap, and the trees it starts from are one level deep.  Without
// it every site of the species starts as its own root.  Also clears what the
// later passes accumulate into: the cluster sizes, the small-size histogram
// and the count of large sizes.
__device__ __forceinline__ void ccl_init_body(const void* lat, int layout, int L, int H, int species, bool runs,
                                              uint32_t* parent, uint32_t* size, unsigned* hist, unsigned* big_count) {
  const size_t n = (size_t)L * H;
  const size_t tid = blockIdx.x * (size_t)blockDim.x + threadIdx.x, nth = (size_t)gridDim.x * blockDim.x;
  // the stride is a whole number of wavefronts, so lane l of a wavefront
  // always holds a site i with i % 64 == l, and the lanes past n are the top ones
  for (size_t i = tid; i < n; i += nth) {
    const int y = (int)(i / L), x = (int)(i - (size_t)y * L);
    const bool me = site_bit(lat, layout, L, x, y) == species;
    uint32_t pi = me ? (uint32_t)i : kNone;
    if (runs) {
      const uint64_t other = __ballot(!me), row0 = __ballot(me && x == 0);
      const uint32_t lane = (uint32_t)(i & 63u);
      const uint64_t upto = (2ull << lane) - 1ull;  // lanes 0 .. lane
      const uint64_t bo = other & upto, bz = row0 & upto;
      // one past the last lane of another species, and the last row start
      const uint32_t so = bo ? 64u - (uint32_t)__clzll((long long)bo) : 0u;
      const uint32_t sz = bz ? 63u - (uint32_t)__clzll((long long)bz) : 0u;
      if (me) pi = (uint32_t)i - (lane - max(so, sz));
    }
    parent[i] = pi;
    size[i] = 0u;
  }
  for (size_t i = tid; i < (size_t)kSmallSizes; i += nth) hist[i] = 0u;
  if (tid == 0) *big_count = 0u;
}

__device__ __forceinline__ void ccl_merge_body(const void* lat, int layout, int L, int species, uint32_t* parent) {
  const size_t n = (size_t)L * L;
  for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x) {
    const int y = (int)(i / L), x = (int)(i - (size_t)y * L);
    if (site_bit(lat, layout, L, x, y) != species) continue;
    const int xr = (x + 1 == L) ? 0 : x + 1, yd = (y + 1 == L) ? 0 : y + 1;
    // within a row and a 64-site segment the bond to the right is already a
    // link of the initial runs
    if ((xr == 0 || (i & 63u) == 63u) && site_bit(lat, layout, L, xr, y) == species)
      unite(parent, (uint32_t)i, (uint32_t)((size_t)y * L + xr));
    if (site_bit(lat, layout, L, x, yd) == species) unite(parent, (uint32_t)i, (uint32_t)((size_t)yd * L + x));
  }
}

// Segregated start: the first n1 sites in index order i = y*L + x hold type 1
// (full rows 0 .. n1/L - 1 and the start of the next one).  Bit-packed words
// tile rows exactly, so word w holds sites 32w .. 32w + 31.
__global__ __launch_bounds__(256) void fill_segregated(void* lat, int layout, int L, int H, uint64_t n1) {
  const size_t n = (size_t)L * H;
  if (layout == kLayoutBits) {
    uint32_t* w = static_cast<uint32_t*>(lat);
    for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < n / 32; i += (size_t)gridDim.x * blockDim.x) {
      const uint64_t lo = 32 * (uint64_t)i;
      w[i] = n1 >= lo + 32 ? 0xFFFFFFFFu : (n1 <= lo ? 0u : ((1u << (uint32_t)(n1 - lo)) - 1u));
    }
  } else {
    uint8_t* b = static_cast<uint8_t*>(lat);
    for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x)
      b[i] = (uint64_t)i < n1 ? 1 : 0;
  }
}

// Triangular lattice, helical boundaries (H rows of L sites, i = y*L + x on one ring of N = L*H):
// unite i with i+1, i+L and i+L-1 (mod N) when both are of the species; the
// other three of the six bonds are forward bonds of the neighbours.
__global__ __launch_bounds__(256) void ccl_merge_tri(const uint8_t* lat, int L, int H, int species, uint32_t* parent) {
  const uint32_t N = (uint32_t)L * (uint32_t)H;
  const uint32_t off[3] = {1u, (uint32_t)L, (uint32_t)L - 1u};
  for (uint32_t i = blockIdx.x * blockDim.x + threadIdx.x; i < N; i += gridDim.x * blockDim.x) {
    if (lat[i] != species) continue;
#pragma unroll
    for (int k = 0; k < 3; ++k) {
      uint32_t j = i + off[k];
      if (j >= N) j -= N;
      if (lat[j] == species) unite(parent, i, j);
    }
  }
}

// After all unions: point every site straight at its root.
__device__ __forceinline__ void ccl_flatten_body(uint32_t* parent, int L, int H) {
  const size_t n = (size_t)L * H;
  for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x) {
    if (ld_parent(parent, (uint32_t)i) == kNone) continue;
    const uint32_t r = find_root_halving(parent, (uint32_t)i);
    atomicMin(&parent[i], r);
  }
}

// Cluster sizes (parents flattened): one add per site onto its root, aggregated over the
// wavefront first (lanes with the same root add once, by their lowest lane),
// so a spanning cluster costs one atomic per wave instead of one per site.
__device__ __forceinline__ void ccl_count_body(uint32_t* parent, int L, int H, uint32_t* size) {
  const size_t n = (size_t)L * H;
  const size_t stride = (size_t)gridDim.x * blockDim.x;
  const int lane = (int)__lane_id();
  // the loop bound is uniform over the block, so every lane joins every ballot
  for (size_t base = (size_t)blockIdx.x * blockDim.x; base < n; base += stride) {
    const size_t i = base + threadIdx.x;
    bool todo = i < n && parent[i] != kNone;
    const uint32_t r = todo ? parent[i] : 0u;
    uint64_t left = __ballot(todo);
    while (left) {
      const int leader = __builtin_ctzll(left);
      const uint32_t rl = __shfl(r, leader);
      const uint64_t same = __ballot(todo && r == rl);
      if (lane == leader) atomicAdd(&size[rl], (unsigned)__popcll(same));
      if (todo && r == rl) todo = false;
      left &= ~same;
    }
  }
}

__device__ __forceinline__ void ccl_hist_body(const uint32_t* size, int L, int H, unsigned* hist, uint32_t* big,
                                              unsigned* big_count, unsigned big_cap, unsigned* h) {
  for (int k = threadIdx.x; k < kSmallSizes; k += blockDim.x) h[k] = 0;
  __syncthreads();
  const size_t n = (size_t)L * H;
  for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x) {
    const uint32_t s = size[i];
    if (s == 0) continue;
    if (s < (uint32_t)kSmallSizes) atomicAdd(&h[s], 1u);
    else {
      const unsigned slot = atomicAdd(big_count, 1u);
      if (slot < big_cap) big[slot] = s;
    }
  }
  __syncthreads();
  for (int k = threadIdx.x; k < kSmallSizes; k += blockDim.x)
    if (h[k]) atomicAdd(&hist[k], h[k]);
}

// The passes as kernels for one lattice (grid-stride over blockIdx.x), and
// for many square lattices at once: replica blockIdx.y of a table, each with
// its own buffers, the same grid-stride over blockIdx.x.
__global__ __launch_bounds__(256) void ccl_init(const void* lat, int layout, int L, int H, int species, int runs,
                                                uint32_t* parent, uint32_t* size, unsigned* hist,
                                                unsigned* big_count) {
  ccl_init_body(lat, layout, L, H, species, runs != 0, parent, size, hist, big_count);
}
__global__ __launch_bounds__(256) void ccl_merge(const void* lat, int layout, int L, int species, uint32_t* parent) {
  ccl_merge_body(lat, layout, L, species, parent);
}
__global__ __launch_bounds__(256) void ccl_flatten(uint32_t* parent, int L, int H) { ccl_flatten_body(parent, L, H); }
__global__ __launch_bounds__(256) void ccl_count(uint32_t* parent, int L, int H, uint32_t* size) {
  ccl_count_body(parent, L, H, size);
}
__global__ __launch_bounds__(256) void ccl_hist(const uint32_t* size, int L, int H, unsigned* hist, uint32_t* big,
                                                unsigned* big_count, unsigned big_cap) {
  __shared__ unsigned h[kSmallSizes];
  ccl_hist_body(size, L, H, hist, big, big_count, big_cap, h);
}
__global__ __launch_bounds__(256) void ccl_init_many(const CclRep* reps, int species) {
  const CclRep& r = reps[blockIdx.y];
  ccl_init_body(r.lat, r.layout, r.L, r.L, species, true, r.b.parent, r.b.size, r.b.hist, r.b.big_count);
}
__global__ __launch_bounds__(256) void ccl_merge_many(const CclRep* reps, int species) {
  const CclRep& r = reps[blockIdx.y];
  ccl_merge_body(r.lat, r.layout, r.L, species, r.b.parent);
}
__global__ __launch_bounds__(256) void ccl_flatten_many(const CclRep* reps) {
  const CclRep& r = reps[blockIdx.y];
  ccl_flatten_body(r.b.parent, r.L, r.L);
}
__global__ __launch_bounds__(256) void ccl_count_many(const CclRep* reps) {
  const CclRep& r = reps[blockIdx.y];
  ccl_count_body(r.b.parent, r.L, r.L, r.b.size);
}
__global__ __launch_bounds__(256) void ccl_hist_many(const CclRep* reps) {
  __shared__ unsigned h[kSmallSizes];
  const CclRep& r = reps[blockIdx.y];
  ccl_hist_body(r.b.size, r.L, r.L, r.b.hist, r.b.big, r.b.big_count, r.b.big_cap, h);
}
// Every replica's result block (histogram, large-size count, first large
// sizes) into row blockIdx.y of one staging array of `words` per replica.
__global__ __launch_bounds__(256) void ccl_gather_many(const CclRep* reps, uint32_t* stage, uint32_t words) {
  const CclRep& r = reps[blockIdx.y];
  const uint32_t n = min(words, (uint32_t)kSmallSizes + 1u + r.b.big_cap);
  uint32_t* dst = stage + (size_t)blockIdx.y * words;
  for (uint32_t i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) dst[i] = r.b.hist[i];
}

// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void pack_bits(const uint8_t* in, uint32_t* out, int L) {
  const size_t nw = (size_t)L * (L >> 5);
  for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < nw; i += (size_t)gridDim.x * blockDim.x) {
    uint32_t v = 0;
    for (int b = 0; b < 32; ++b) v |= (uint32_t)(in[i * 32 + b] & 1u) << b;
    out[i] = v;
  }
}

__global__ __launch_bounds__(256) void unpack_bits(const uint32_t* in, uint8_t* out, int L) {
  const size_t nw = (size_t)L * (L >> 5);
  for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < nw; i += (size_t)gridDim.x * blockDim.x) {
    const uint32_t v = in[i];
    for (int b = 0; b < 32; ++b) out[i * 32 + b] = (uint8_t)((v >> b) & 1u);
  }
}

int grid_for(size_t n, int block) {
  size_t g = (n + block - 1) / block;
  if (g > 4096) g = 4096;
  if (g < 1) g = 1;
  return (int)g;
}

}  // namespace

hipError_t launch_energy(const void* lat, int layout, int L, unsigned long long* out, hipStream_t stream) {
  if (layout == kLayoutBits)
    hipLaunchKernelGGL(energy_bits, dim3(grid_for((size_t)L * (L >> 5), 256)), dim3(256), 0, stream,
                       static_cast<const uint32_t*>(lat), L, out);
  else
    hipLaunchKernelGGL(energy_int8, dim3(grid_for((size_t)L * L, 256)), dim3(256), 0, stream,
                       static_cast<const uint8_t*>(lat), L, out);
  return hipGetLastError();
}

hipError_t launch_similar_sampled(const void* lat, int layout, int L, uint32_t k0, uint32_t k1, uint64_t t,
                                 unsigned long long* out, hipStream_t stream) {
  hipLaunchKernelGGL(similar_sampled, dim3(grid_for((size_t)L * (L >> 2), 256)), dim3(256), 0, stream, lat, layout, L,
                     k0, k1, t, out);
  return hipGetLastError();
}

hipError_t launch_init_keys(uint64_t* keys, int L, int H, uint32_t k0, uint32_t k1, hipStream_t stream) {
  hipLaunchKernelGGL(init_keys, dim3(grid_for((size_t)L * H, 256)), dim3(256), 0, stream, keys, L, H, k0, k1);
  return hipGetLastError();
}

hipError_t launch_radix_hist(const uint64_t* keys, size_t n, uint64_t prefix, int shift, unsigned* hist256,
                             hipStream_t stream) {
  hipLaunchKernelGGL(radix_hist, dim3(grid_for(n, 256)), dim3(256), 0, stream, keys, n, prefix, shift, hist256);
  return hipGetLastError();
}

hipError_t launch_init_mark(const uint64_t* keys, int L, int H, int layout, uint64_t kth, void* lat, unsigned* eq_count,
                            uint32_t* eq_list, unsigned eq_cap, hipStream_t stream) {
  const size_t n = layout == kLayoutBits ? (size_t)H * (L >> 5) : (size_t)L * H;
  hipLaunchKernelGGL(init_mark, dim3(grid_for(n, 256)), dim3(256), 0, stream, keys, L, H, layout, kth, lat, eq_count,
                     eq_list, eq_cap);
  return hipGetLastError();
}

hipError_t launch_set_sites(const uint32_t* idx, unsigned n, int L, int layout, void* lat, hipStream_t stream) {
  if (n == 0) return hipSuccess;
  hipLaunchKernelGGL(set_sites, dim3((n + 255) / 256), dim3(256), 0, stream, idx, n, L, layout, lat);
  return hipGetLastError();
}

hipError_t launch_ccl(const void* lat, int layout, int L, int H, int species, const CclBuffers& b, bool triangular,
                      hipStream_t stream) {
  const size_t n = (size_t)L * H;
  const int g = grid_for(n, 256);
  hipLaunchKernelGGL(ccl_init, dim3(g), dim3(256), 0, stream, lat, layout, L, H, species, triangular ? 0 : 1,
                     b.parent, b.size, b.hist, b.big_count);
  if (triangular) {
    hipLaunchKernelGGL(ccl_merge_tri, dim3(g), dim3(256), 0, stream, static_cast<const uint8_t*>(lat), L, H, species,
                       b.parent);
  } else {
    // the square torus: H == L
    hipLaunchKernelGGL(ccl_merge, dim3(g), dim3(256), 0, stream, lat, layout, L, species, b.parent);
  }
  hipLaunchKernelGGL(ccl_flatten, dim3(g), dim3(256), 0, stream, b.parent, L, H);
  hipLaunchKernelGGL(ccl_count, dim3(g), dim3(256), 0, stream, b.parent, L, H, b.size);
  // each workgroup clears and flushes a whole LDS histogram, and every one of
  // them adds into the hot small sizes: few workgroups, each streaming many sites
  hipLaunchKernelGGL(ccl_hist, dim3(g < 128 ? g : 128), dim3(256), 0, stream, b.size, L, H, b.hist, b.big,
                     b.big_count, b.big_cap);
  return hipGetLastError();
}

hipError_t launch_ccl_many(const CclRep* d_reps, int nreps, size_t max_sites, int species, uint32_t* stage,
                           uint32_t words, hipStream_t stream) {
  if (nreps <= 0) return hipSuccess;
  // every pass strides over its lattice, so a replica needs no more
  // workgroups than fill the device with the others; workgroups past a
  // smaller replica's sites exit at once
  const int g = std::min(grid_for(max_sites, 256), kCclManyBlocks);
  const dim3 grid((unsigned)g, (unsigned)nreps), hgrid((unsigned)(g < 128 ? g : 128), (unsigned)nreps);
  hipLaunchKernelGGL(ccl_init_many, grid, dim3(256), 0, stream, d_reps, species);
  hipLaunchKernelGGL(ccl_merge_many, grid, dim3(256), 0, stream, d_reps, species);
  hipLaunchKernelGGL(ccl_flatten_many, grid, dim3(256), 0, stream, d_reps);
  hipLaunchKernelGGL(ccl_count_many, grid, dim3(256), 0, stream, d_reps);
  hipLaunchKernelGGL(ccl_hist_many, hgrid, dim3(256), 0, stream, d_reps);
  hipLaunchKernelGGL(ccl_gather_many, dim3(8, (unsigned)nreps), dim3(256), 0, stream, d_reps, stage, words);
  return hipGetLastError();
}

hipError_t launch_pack(const uint8_t* in, uint32_t* out, int L, hipStream_t stream) {
  hipLaunchKernelGGL(pack_bits, dim3(grid_for((size_t)L * (L >> 5), 256)), dim3(256), 0, stream, in, out, L);
  return hipGetLastError();
}

hipError_t launch_unpack(const uint32_t* in, uint8_t* out, int L, hipStream_t stream) {
  hipLaunchKernelGGL(unpack_bits, dim3(grid_for((size_t)L * (L >> 5), 256)), dim3(256), 0, stream, in, out, L);
  return hipGetLastError();
}

hipError_t launch_fill_segregated(void* lat, int layout, int L, int H, uint64_t n1, hipStream_t stream) {
  hipLaunchKernelGGL(fill_segregated, dim3(grid_for((size_t)L * H, 256)), dim3(256), 0, stream, lat, layout, L, H,
                     n1);
  return hipGetLastError();
}

}  // namespace kk
