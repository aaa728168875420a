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
#include "kk_tri.hpp"

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

// ---------------------------------------------------------------------------
// One whole sweep of the 16 classes in one launch.  Each workgroup owns a tile
// of TW x TR sites (columns x0 .. x0+TW-1 of rows y0 .. y0+TR-1; the last tile
// of a row or column may be narrower) and holds in LDS the window of the ring
// around it: kTriHalo more rows and columns on every side, read from `in`.
// Window cell (r, c) is ring site (y0 - kTriHalo + r) * L + x0 - kTriHalo + c
// mod N, so the six neighbours are (r, c +- 1), (r +- 1, c), (r +- 1, c -+ 1)
// everywhere in the window, across row ends included.  The workgroup runs the
// 16 phases on its window; a phase only needs centres within one step of the
// cells that must stay exact, whose reads lie within two steps, so the exact
// region shrinks by two cells per phase: phase p works on the cells at least
// 2p + 2 from the window edge, and after 16 phases the cells at least 33 from
// the edge -- the tile -- hold exactly what the in-place class sweep gives.
// The tile is then written to `out`.  Centres are counted as accepted only in
// the tile, so every attempt of the sweep is counted once.  Needs the window
// to fit the ring: TW + 2 kTriHalo <= L and TR + 2 kTriHalo <= H.
// The work of one workgroup: tile (tx, ty) of TW x TR on the ring of H rows of
// L sites, one sweep t from `in` to `out`; `win` is the dynamic LDS window.
__device__ __forceinline__ void tri_tile_body(const uint8_t* __restrict__ in, uint8_t* __restrict__ out, uint32_t L,
                                              uint32_t H, uint32_t TW, uint32_t TR, uint32_t tx, uint32_t ty,
                                              uint32_t k0, uint32_t k1, uint64_t t, const TriAccept& acc,
                                              unsigned long long* partials, uint8_t* win) {
  __shared__ uint32_t perm_s[16], thr_s[11];
  __shared__ uint32_t all_s;
  __shared__ unsigned long long red[16];
  const uint32_t N = L * H;
  const uint32_t WC = TW + 2 * kTriHalo, WR = TR + 2 * kTriHalo, S = tri_window_stride(TW);
  const uint32_t x0 = tx * TW, y0 = ty * TR;
  const uint32_t TWe = min(TW, L - x0), TRe = min(TR, H - y0);
  // ring index of window cell (0, 0)
  const uint32_t base =
      (uint32_t)(((uint64_t)y0 * L + x0 + 2ull * N - (uint64_t)kTriHalo * L - kTriHalo) % (uint64_t)N);
  const uint32_t lane = threadIdx.x & 63u, wave = threadIdx.x >> 6, nwaves = blockDim.x >> 6;
  if (threadIdx.x < 64) {
    const uint32_t c = tri_order(k0, k1, t, (int)(threadIdx.x & 15u));
    if (threadIdx.x < 16) perm_s[threadIdx.x] = c;
  } else if (threadIdx.x < 64 + 11) {
    const uint32_t n = threadIdx.x - 64;
    const uint64_t T = acc.T[n];
    thr_s[n] = T >= 0xFFFFFFFFull ? 0xFFFFFFFFu : (uint32_t)T;
    const uint32_t always = (uint32_t)__ballot(T >= 0x100000000ull);  // lanes 0..10 of wave 1
    if (n == 0) all_s = always;
  }
  // the window: each wave takes two rows at a time and issues all of their
  // byte loads (up to 16 per lane) before storing any, so the loads overlap
  for (uint32_t r0 = 2 * wave; r0 < WR; r0 += 2 * nwaves) {
    for (uint32_t c0 = 0; c0 < WC; c0 += 512) {
      uint8_t v[16];
#pragma unroll
      for (uint32_t k = 0; k < 16; ++k) {
        // out-of-window lanes read the window's first site and drop it: no branch
        // around the load
        const uint32_t r = r0 + (k >> 3), c = c0 + lane + 64u * (k & 7u);
        const bool ok = r < WR && c < WC;
        uint32_t rb = base + (ok ? r : 0u) * L;
        rb = rb >= N ? rb - N : rb;
        uint32_t i = rb + (ok ? c : 0u);
        i = i >= N ? i - N : i;
        v[k] = in[i];
      }
#pragma unroll
      for (uint32_t k = 0; k < 16; ++k) {
        const uint32_t r = r0 + (k >> 3), c = c0 + lane + 64u * (k & 7u);
        if (r < WR && c < WC) win[r * S + c] = v[k];
      }
    }
  }
  __syncthreads();
  const uint32_t always = all_s;
  const uint32_t tl = (uint32_t)t, th = ctr_hi(t, kTagTri);
  // per-lane parts of the row addresses; the wave index is uniform, so the
  // work-item arithmetic below stays in scalar registers
  const uint32_t lane_ring = lane * L, lane_win = lane * S;
  const uint32_t wave_u = __builtin_amdgcn_readfirstlane(wave);
  unsigned long long cnt = 0;
  // this wave's ring of pending centres: the pair's window cell a, direction,
  // a's species and whether the centre lies in the tile, then the uniform u
  uint2* ring = reinterpret_cast<uint2*>(win + tri_window_area(TW, TR)) + wave * kTriQueue;
  auto site = [&](uint32_t k) {  // sites hold 0 or 1, so x ^ v counts an unlike neighbour
    const uint32_t x = win[k];
    __builtin_assume(x <= 1u);
    return x;
  };
  // decide the first k pending centres of the ring (lanes below k)
  auto decide = [&](uint32_t head, uint32_t k) {
    if (lane < k) {
      const uint2 e = ring[(head + lane) & (kTriQueue - 1u)];
      const uint32_t a = e.x & 0xFFFFFu, d = (e.x >> 20) & 7u, va = (e.x >> 23) & 1u, vb = va ^ 1u;
      const uint32_t mag = d < 2 ? 1u : (d < 4 ? S : S - 1u);
      const uint32_t b = (d & 1u) ? a - mag : a + mag;
      // the a-b bond is unlike and appears once in each neighbourhood
      const uint32_t n = (site(a + 1) ^ va) + (site(a - 1) ^ va) + (site(a + S) ^ va) + (site(a - S) ^ va) +
                         (site(a + S - 1) ^ va) + (site(a - S + 1) ^ va) + (site(b + 1) ^ vb) + (site(b - 1) ^ vb) +
                         (site(b + S) ^ vb) + (site(b - S) ^ vb) + (site(b + S - 1) ^ vb) + (site(b - S + 1) ^ vb) -
                         2u;
      if (e.y < thr_s[n] || ((always >> n) & 1u)) {
        win[a] = (uint8_t)vb;
        win[b] = (uint8_t)va;
        cnt += (e.x >> 24) & 1u;
      }
    }
  };
  for (int p = 0; p < 16; ++p) {
    const uint32_t cls = perm_s[p];
    const uint32_t lo = 2u * (uint32_t)p + 2u;
    const uint32_t rhi = WR - lo, chi = WC - lo;
    const uint32_t nrg = (rhi - lo + 63u) >> 6, Q = (chi - lo + 15u) >> 4;
    // Centres of one class never share a site or a neighbourhood, so their
    // decisions may run in any order: a wave draws the random numbers of 64
    // centres, queues those whose pair is unlike (a fraction of them once the
    // lattice has ordered) and decides 64 queued centres at a time.
    uint32_t qhead = 0, qtail = 0;  // uniform
    for (uint32_t it = wave_u; it < nrg * Q; it += nwaves) {
      const uint32_t rg = it / Q, q = it - rg * Q;
      const uint32_t r0 = lo + rg * 64u;  // uniform first row of the item
      const uint32_t r = r0 + lane;
      uint32_t rb0 = base + r0 * L;
      rb0 = rb0 >= N ? rb0 - N : rb0;
      uint32_t rb = rb0 + lane_ring;
      rb = rb >= N ? rb - N : rb;
      const uint32_t c = lo + ((cls - rb - lo) & 15u) + 16u * q;
      const bool ok = r < rhi && c < chi;
      uint32_t i = rb + c;
      i = i >= N ? i - N : i;
      const Philox4 rr = philox10(i >> 1, 0u, tl, th, k0, k1);
      const uint32_t wd = (i & 1u) ? rr.z : rr.x, u = (i & 1u) ? rr.w : rr.y;
      const uint32_t d = (uint32_t)(((uint64_t)wd * 6u) >> 32);
      // a lane past the phase's region looks at window cell (1, 1) and its
      // neighbour, inside the window, and queues nothing
      const uint32_t a = ok ? r0 * S + lane_win + c : S + 1u;
      const uint32_t mag = d < 2 ? 1u : (d < 4 ? S : S - 1u);
      const uint32_t b = (d & 1u) ? a - mag : a + mag;
      const uint32_t va = site(a), vb = site(b);
      const bool live = ok && va != vb;
      const uint64_t m = __ballot(live);
      if (m == 0) continue;
      if (live) {
        const uint32_t pos = __builtin_amdgcn_mbcnt_hi((uint32_t)(m >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)m, 0u));
        const uint32_t counted = (r - kTriHalo < TRe) & (c - kTriHalo < TWe);
        ring[(qtail + pos) & (kTriQueue - 1u)] = make_uint2(a | (d << 20) | (va << 23) | (counted << 24), u);
      }
      qtail += (uint32_t)__popcll(m);
      if (qtail - qhead >= 64u) {  // at most 127 pending: the ring never overflows
        decide(qhead, 64u);
        qhead += 64u;
      }
    }
    while (qtail != qhead) {
      const uint32_t k = min(qtail - qhead, 64u);
      decide(qhead, k);
      qhead += k;
    }
    __syncthreads();
  }
  // the tile
  for (uint32_t r = kTriHalo + wave; r < kTriHalo + TRe; r += nwaves) {
    uint32_t rb = base + r * L;
    if (rb >= N) rb -= N;
    for (uint32_t c = kTriHalo + lane; c < kTriHalo + TWe; c += 64) {
      uint32_t i = rb + c;
      if (i >= N) i -= N;
      out[i] = win[r * S + c];
    }
  }
  for (int off = 32; off > 0; off >>= 1) cnt += __shfl_down(cnt, off, 64);
  if (lane == 0) red[wave] = cnt;
  __syncthreads();
  if (threadIdx.x == 0) {
    unsigned long long tot = 0;
    for (uint32_t w = 0; w < nwaves; ++w) tot += red[w];
    if (tot) atomicAdd(&partials[blockIdx.x % kTriPartials], tot);
  }
}

__global__ __launch_bounds__(1024) void tri_tile_sweep(const uint8_t* __restrict__ in, uint8_t* __restrict__ out,
                                                       uint32_t L, uint32_t H, uint32_t TW, uint32_t TR, uint32_t ntx,
                                                       uint32_t k0, uint32_t k1, uint64_t t, TriAccept acc,
                                                       unsigned long long* partials) {
  extern __shared__ uint8_t win[];
  const uint32_t tile = (uint32_t)xcd_tile((int)blockIdx.x, (int)gridDim.x);
  tri_tile_body(in, out, L, H, TW, TR, tile % ntx, tile / ntx, k0, k1, t, acc, partials, win);
}

// Many lattices in one launch: workgroup b does tile jobs[b].y of replica
// jobs[b].x, sweep k of the run (buffers and sweep counter from the table).
__global__ __launch_bounds__(1024) void tri_tile_sweep_batch(const TriBatchRep* reps, const uint2* jobs,
                                                             uint32_t k) {
  extern __shared__ uint8_t win[];
  const uint2 jb = jobs[blockIdx.x];
  const TriBatchRep& R = reps[jb.x];
  const uint32_t par = R.cur ^ (k & 1u);
  tri_tile_body(R.lat[par], R.lat[par ^ 1u], R.L, R.H, R.TW, R.TR, jb.y % R.ntx, jb.y / R.ntx, R.k0, R.k1,
                R.t0 + k, R.acc, R.partials, win);
}

// ---------------------------------------------------------------------------
// Small lattices: the whole ring of one replica in one workgroup's LDS (no
// halo), all of its sweeps in one launch, written back in place.  The 16
// classes of a sweep run in the sweep's order with a barrier between them;
// neighbours wrap modulo N inside LDS.  Workgroup b runs replica b of the
// table.
__device__ __forceinline__ void tri_resident_body(const TriResidentRep& R, uint8_t* ring) {
  __shared__ uint32_t perm_s[16], thr_s[11];
  __shared__ uint32_t all_s;
  __shared__ unsigned long long red[16];
  const uint32_t L = R.L, N = R.L * R.H;
  uint8_t* lat = R.lat;
  const uint32_t lane = threadIdx.x & 63u, wave = threadIdx.x >> 6, nwaves = blockDim.x >> 6;
  if (threadIdx.x >= 64 && threadIdx.x < 64 + 11) {
    const uint32_t n = threadIdx.x - 64;
    const uint64_t T = R.acc.T[n];
    thr_s[n] = T >= 0xFFFFFFFFull ? 0xFFFFFFFFu : (uint32_t)T;
    const uint32_t always = (uint32_t)__ballot(T >= 0x100000000ull);  // lanes 0..10 of wave 1
    if (n == 0) all_s = always;
  }
  for (uint32_t i = threadIdx.x; i < N; i += blockDim.x) ring[i] = lat[i];
  unsigned long long cnt = 0;
  const uint32_t M = N >> 4;
  for (uint32_t s = 0; s < R.sweeps; ++s) {
    const uint64_t t = R.t0 + s;
    __syncthreads();  // the previous sweep's last phase (and the load) are complete
    if (threadIdx.x < 64) {
      const uint32_t c = tri_order(R.k0, R.k1, t, (int)(threadIdx.x & 15u));
      if (threadIdx.x < 16) perm_s[threadIdx.x] = c;
    }
    __syncthreads();
    const uint32_t always = all_s;
    const uint32_t tl = (uint32_t)t, th = ctr_hi(t, kTagTri);
    for (int p = 0; p < 16; ++p) {
      const uint32_t cls = perm_s[p];
      for (uint32_t j = threadIdx.x; j < M; j += blockDim.x) {
        const uint32_t i = cls + 16u * j;
        const Philox4 r = philox10(i >> 1, 0u, tl, th, R.k0, R.k1);
        const uint32_t wd = (i & 1u) ? r.z : r.x, u = (i & 1u) ? r.w : r.y;
        const uint32_t d = (uint32_t)(((uint64_t)wd * 6u) >> 32);
        const uint32_t b = tri_nb(i, d, L, N);
        const uint32_t vi = ring[i], vb = ring[b];
        if (vi == vb) continue;
        // the i-b bond is unlike and appears once in each neighbourhood
        uint32_t n = 0;
#pragma unroll
        for (uint32_t e = 0; e < 6; ++e) n += ring[tri_nb(i, e, L, N)] != vi;
#pragma unroll
        for (uint32_t e = 0; e < 6; ++e) n += ring[tri_nb(b, e, L, N)] != vb;
        n -= 2u;
        if (u < thr_s[n] || ((always >> n) & 1u)) {
          ring[i] = (uint8_t)vb;
          ring[b] = (uint8_t)vi;
          ++cnt;
        }
      }
      __syncthreads();
    }
  }
  __syncthreads();
  for (uint32_t i = threadIdx.x; i < N; i += blockDim.x) lat[i] = ring[i];
  for (int off = 32; off > 0; off >>= 1) cnt += __shfl_down(cnt, off, 64);
  if (lane == 0) red[wave] = cnt;
  __syncthreads();
  if (threadIdx.x == 0) {
    unsigned long long tot = 0;
    for (uint32_t w = 0; w < nwaves; ++w) tot += red[w];
    if (tot) atomicAdd(&R.partials[0], tot);
  }
}

__global__ __launch_bounds__(1024) void tri_resident(const TriResidentRep* reps) {
  extern __shared__ uint8_t ring[];
  tri_resident_body(reps[blockIdx.x], ring);
}

__global__ __launch_bounds__(1024) void tri_resident_one(TriResidentRep R) {
  extern __shared__ uint8_t ring[];
  tri_resident_body(R, ring);
}

// ---------------------------------------------------------------------------
// One whole literal-MPKK step (7 iterations) in one launch.  As in
// tri_tile_sweep, each workgroup owns a TW x TR tile and holds the window of
// the ring around it, kMpkkHalo more rows and columns on every side.  A cell's
// value after an iteration depends only on cells within three steps (its
// domain's centre is one step away and that centre's decision reads two
// further), so iteration j works on the centres at least 3j + 2 from the
// window edge and the tile is exact after 7.  The iteration stays synchronous
// inside one buffer: an accepted exchange of two unlike sites flips both, so
// a deciding domain only sets bit 1 (flip) of its two bytes and every reader
// looks at bit 0 (the value at the start of the iteration); after a barrier
// one pass folds the flips into the values.  Domains are disjoint, so no byte
// is marked twice.  Needs TW + 2 kMpkkHalo <= L and TR + 2 kMpkkHalo <= H.
__global__ __launch_bounds__(1024) void mpkk_tile_step(const uint8_t* __restrict__ in, uint8_t* __restrict__ out,
                                                       uint32_t L, uint32_t H, uint32_t TW, uint32_t TR, uint32_t ntx,
                                                       uint32_t k0, uint32_t k1, uint64_t t, TriAccept acc,
                                                       unsigned long long* partials) {
  extern __shared__ __attribute__((aligned(16))) uint8_t win[];  // read as words by the flip pass
  __shared__ uint32_t k_s[7], thr_s[11];
  __shared__ uint32_t all_s;
  __shared__ unsigned long long red[16];
  const uint32_t N = L * H;
  const uint32_t WC = TW + 2 * kMpkkHalo, WR = TR + 2 * kMpkkHalo, S = mpkk_window_stride(TW);
  const uint32_t tile = (uint32_t)xcd_tile((int)blockIdx.x, (int)gridDim.x);
  const uint32_t tx = tile % ntx, ty = tile / ntx;
  const uint32_t x0 = tx * TW, y0 = ty * TR;
  const uint32_t TWe = min(TW, L - x0), TRe = min(TR, H - y0);
  const uint32_t base =
      (uint32_t)(((uint64_t)y0 * L + x0 + 2ull * N - (uint64_t)kMpkkHalo * L - kMpkkHalo) % (uint64_t)N);
  const uint32_t lane = threadIdx.x & 63u, wave = threadIdx.x >> 6, nwaves = blockDim.x >> 6;
  const uint32_t tl = (uint32_t)t;
  if (threadIdx.x < 7) {
    const uint32_t j = threadIdx.x;
    const Philox4 b = philox10(j >> 2, 2u, tl, ctr_hi(t, kTagMpkkK), k0, k1);
    const uint32_t w = (j & 3) == 0 ? b.x : (j & 3) == 1 ? b.y : (j & 3) == 2 ? b.z : b.w;
    k_s[j] = (uint32_t)(((uint64_t)w * 7u) >> 32);
  } else if (threadIdx.x >= 64 && threadIdx.x < 64 + 11) {
    const uint32_t n = threadIdx.x - 64;
    const uint64_t T = acc.T[n];
    thr_s[n] = T >= 0xFFFFFFFFull ? 0xFFFFFFFFu : (uint32_t)T;
    const uint32_t always = (uint32_t)__ballot(T >= 0x100000000ull);  // lanes 0..10 of wave 1
    if (n == 0) all_s = always;
  }
  // the window, two rows per wave at a time, all loads of a batch issued first
  for (uint32_t r0 = 2 * wave; r0 < WR; r0 += 2 * nwaves) {
    for (uint32_t c0 = 0; c0 < WC; c0 += 512) {
      uint8_t v[16];
#pragma unroll
      for (uint32_t k = 0; k < 16; ++k) {
        // out-of-window lanes read the window's first site and drop it
        const uint32_t r = r0 + (k >> 3), c = c0 + lane + 64u * (k & 7u);
        const bool ok = r < WR && c < WC;
        uint32_t rb = base + (ok ? r : 0u) * L;
        rb = rb >= N ? rb - N : rb;
        uint32_t i = rb + (ok ? c : 0u);
        i = i >= N ? i - N : i;
        v[k] = in[i];
      }
#pragma unroll
      for (uint32_t k = 0; k < 16; ++k) {
        const uint32_t r = r0 + (k >> 3), c = c0 + lane + 64u * (k & 7u);
        if (r < WR && c < WC) win[r * S + c] = v[k];
      }
    }
  }
  __syncthreads();
  const uint32_t always = all_s;
  const uint32_t th = ctr_hi(t, kTagMpkk);
  const uint32_t lane_ring = lane * L, lane_win = lane * S;
  const uint32_t wave_u = __builtin_amdgcn_readfirstlane(wave);
  uint32_t* win32 = reinterpret_cast<uint32_t*>(win);
  const uint32_t nwords = (S >> 2) * WR;
  unsigned long long cnt = 0;
  // this wave's ring of pending attempts whose pair is unlike (domains are
  // disjoint and every read uses the start-of-iteration bit, so the order of
  // the decisions does not matter): cell a, direction, a's species and whether
  // the centre lies in the tile, then the uniform u
  uint2* ring = reinterpret_cast<uint2*>(win + mpkk_window_area(TW, TR)) + wave * kTriQueue;
  auto decide = [&](uint32_t head, uint32_t kq) {
    if (lane < kq) {
      const uint2 e = ring[(head + lane) & (kTriQueue - 1u)];
      const uint32_t a = e.x & 0xFFFFFu, d = (e.x >> 20) & 7u, va = (e.x >> 23) & 1u, vb = va ^ 1u;
      const uint32_t mag = d < 2 ? 1u : (d < 4 ? S : S - 1u);
      const uint32_t b = (d & 1u) ? a - mag : a + mag;
      const uint32_t n = ((win[a + 1] ^ va) & 1u) + ((win[a - 1] ^ va) & 1u) + ((win[a + S] ^ va) & 1u) +
                         ((win[a - S] ^ va) & 1u) + ((win[a + S - 1] ^ va) & 1u) + ((win[a - S + 1] ^ va) & 1u) +
                         ((win[b + 1] ^ vb) & 1u) + ((win[b - 1] ^ vb) & 1u) + ((win[b + S] ^ vb) & 1u) +
                         ((win[b - S] ^ vb) & 1u) + ((win[b + S - 1] ^ vb) & 1u) + ((win[b - S + 1] ^ vb) & 1u) - 2u;
      if (e.y < thr_s[n] || ((always >> n) & 1u)) {
        win[a] = (uint8_t)(va | 2u);
        win[b] = (uint8_t)(vb | 2u);
        cnt += (e.x >> 24) & 1u;
      }
    }
  };
  for (int j = 0; j < 7; ++j) {
    const uint32_t k = k_s[j];
    const uint32_t lo = 3u * (uint32_t)j + 2u;
    uint32_t qhead = 0, qtail = 0;  // uniform
    const uint32_t rhi = WR - lo, chi = WC - lo;
    // A work item is a lane's pair of consecutive domains m, m + 1 along its
    // row (7 sites apart) with m even: both take their numbers from Philox
    // block m/2, computed once.  The row's first pair may start one centre
    // before the region; the ring end can break the pairing in one row of the
    // window, where the second domain computes its own block.
    const uint32_t nrg = (rhi - lo + 63u) >> 6, Q = (chi - lo + 26u) / 14u;
    for (uint32_t it = wave_u; it < nrg * Q; it += nwaves) {
      const uint32_t rg = it / Q, q = it - rg * Q;
      const uint32_t r0 = lo + rg * 64u;
      const uint32_t r = r0 + lane;
      const bool rok = r < rhi;
      uint32_t rb0 = base + r0 * L;
      rb0 = rb0 >= N ? rb0 - N : rb0;
      uint32_t rb = rb0 + lane_ring;
      rb = rb >= N ? rb - N : rb;
      // the row's first centre in the region and its domain's index
      const uint32_t cf = lo + (k + 7u - (rb + lo) % 7u) % 7u;
      uint32_t i_f = rb + cf;
      i_f = i_f >= N ? i_f - N : i_f;
      const uint32_t mf = (i_f - k) / 7u;
      // the item's second centre (never before cf) and first centre
      const uint32_t c2 = cf + 7u * (1u - (mf & 1u)) + 14u * q;
      const bool ok1 = rok && c2 >= lo + 7u && c2 - 7u < chi, ok2 = rok && c2 < chi;
      uint32_t i2 = rb + c2;
      i2 = i2 >= N ? i2 - N : i2;
      const uint32_t i1 = i2 >= 7u ? i2 - 7u : i2 + N - 7u;
      const uint32_t m1 = (i1 - k) / 7u, m2 = (i2 - k) / 7u;
      const Philox4 r1 = philox10(m1 >> 1, (uint32_t)j, tl, th, k0, k1);
      Philox4 r2 = r1;
      if ((m2 >> 1) != (m1 >> 1)) r2 = philox10(m2 >> 1, (uint32_t)j, tl, th, k0, k1);
      const uint32_t rowa = r0 * S + lane_win;
      // one domain: centre at column c, direction word wd, uniform u; queued
      // when its pair is unlike (every lane takes part in the ballot)
      auto attempt = [&](bool ok, uint32_t c, uint32_t wd, uint32_t u) {
        const uint32_t d = (uint32_t)(((uint64_t)wd * 6u) >> 32);
        // a lane without this domain looks at window cell (1, 1) and its neighbour
        const uint32_t a = ok ? rowa + c : S + 1u;
        const uint32_t mag = d < 2 ? 1u : (d < 4 ? S : S - 1u);
        const uint32_t b = (d & 1u) ? a - mag : a + mag;
        // bit 0 of a byte is the value at the start of the iteration
        const uint32_t va = win[a] & 1u, vb = win[b] & 1u;
        const bool live = ok && va != vb;
        const uint64_t mk = __ballot(live);
        if (mk == 0) return;
        if (live) {
          const uint32_t pos =
              __builtin_amdgcn_mbcnt_hi((uint32_t)(mk >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)mk, 0u));
          const uint32_t counted = (r - kMpkkHalo < TRe) & (c - kMpkkHalo < TWe);
          ring[(qtail + pos) & (kTriQueue - 1u)] = make_uint2(a | (d << 20) | (va << 23) | (counted << 24), u);
        }
        qtail += (uint32_t)__popcll(mk);
        if (qtail - qhead >= 64u) {  // at most 127 pending: the ring never overflows
          decide(qhead, 64u);
          qhead += 64u;
        }
      };
      attempt(ok1, c2 - 7u, (m1 & 1u) ? r1.z : r1.x, (m1 & 1u) ? r1.w : r1.y);
      attempt(ok2, c2, (m2 & 1u) ? r2.z : r2.x, (m2 & 1u) ? r2.w : r2.y);
    }
    while (qtail != qhead) {
      const uint32_t kk = min(qtail - qhead, 64u);
      decide(qhead, kk);
      qhead += kk;
    }
    __syncthreads();
    // fold the flips: value ^= flip, four bytes at a time
    for (uint32_t w = threadIdx.x; w < nwords; w += blockDim.x) {
      const uint32_t x = win32[w];
      win32[w] = (x & 0x01010101u) ^ ((x >> 1) & 0x01010101u);
    }
    __syncthreads();
  }
  // the tile
  for (uint32_t r = kMpkkHalo + wave; r < kMpkkHalo + TRe; r += nwaves) {
    uint32_t rb = base + r * L;
    if (rb >= N) rb -= N;
    for (uint32_t c = kMpkkHalo + lane; c < kMpkkHalo + TWe; c += 64) {
      uint32_t i = rb + c;
      if (i >= N) i -= N;
      out[i] = win[r * S + c];
    }
  }
  for (int off = 32; off > 0; off >>= 1) cnt += __shfl_down(cnt, off, 64);
  if (lane == 0) red[wave] = cnt;
  __syncthreads();
  if (threadIdx.x == 0) {
    unsigned long long tot = 0;
    for (uint32_t w = 0; w < nwaves; ++w) tot += red[w];
    if (tot) atomicAdd(&partials[blockIdx.x % kTriPartials], tot);
  }
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

hipError_t launch_tri_tile_sweep(const uint8_t* in, uint8_t* out, int L, int H, int TW, int TR, uint32_t k0,
                                uint32_t k1, uint64_t t, const TriAccept& acc, unsigned long long* partials,
                                hipStream_t stream) {
  if (!tri_tile_fits(L, H, TW, TR)) return hipErrorInvalidValue;
  const uint32_t ntx = ((uint32_t)L + TW - 1) / TW, nty = ((uint32_t)H + TR - 1) / TR;
  hipLaunchKernelGGL(tri_tile_sweep, dim3(ntx * nty), dim3(1024), tri_window_bytes(TW, TR), stream, in, out,
                     (uint32_t)L, (uint32_t)H, (uint32_t)TW, (uint32_t)TR, ntx, k0, k1, t, acc, partials);
  return hipGetLastError();
}

hipError_t launch_mpkk_iteration(const uint8_t* in, uint8_t* out, int L, int H, uint32_t k0, uint32_t k1, uint64_t t,
                                 int j, const TriAccept& acc, unsigned long long* partials, hipStream_t stream) {
  const uint32_t N = (uint32_t)L * (uint32_t)H;
  hipLaunchKernelGGL(mpkk_iter, dim3(tri_grid(N / 7)), dim3(256), 0, stream, in, out, (uint32_t)L, N, k0, k1, t, j,
                     acc, partials);
  return hipGetLastError();
}

hipError_t launch_tri_tile_sweep_batch(const TriBatchRep* reps, const uint2* jobs, uint32_t njobs, uint32_t k,
                                       size_t lds_bytes, hipStream_t stream) {
  if (njobs == 0) return hipSuccess;
  hipLaunchKernelGGL(tri_tile_sweep_batch, dim3(njobs), dim3(1024), lds_bytes, stream, reps, jobs, k);
  return hipGetLastError();
}

hipError_t launch_tri_resident(const TriResidentRep* reps, uint32_t nreps, size_t lds_bytes, hipStream_t stream) {
  if (nreps == 0) return hipSuccess;
  hipLaunchKernelGGL(tri_resident, dim3(nreps), dim3(1024), lds_bytes, stream, reps);
  return hipGetLastError();
}

hipError_t launch_tri_resident_one(const TriResidentRep& rep, size_t lds_bytes, hipStream_t stream) {
  hipLaunchKernelGGL(tri_resident_one, dim3(1), dim3(1024), lds_bytes, stream, rep);
  return hipGetLastError();
}

hipError_t launch_mpkk_tile_step(const uint8_t* in, uint8_t* out, int L, int H, int TW, int TR, uint32_t k0,
                                 uint32_t k1, uint64_t t, const TriAccept& acc, unsigned long long* partials,
                                 hipStream_t stream) {
  if (!mpkk_tile_fits(L, H, TW, TR)) return hipErrorInvalidValue;
  const uint32_t ntx = ((uint32_t)L + TW - 1) / TW, nty = ((uint32_t)H + TR - 1) / TR;
  hipLaunchKernelGGL(mpkk_tile_step, dim3(ntx * nty), dim3(1024), mpkk_window_bytes(TW, TR), stream, in, out,
                     (uint32_t)L, (uint32_t)H, (uint32_t)TW, (uint32_t)TR, ntx, k0, k1, t, acc, partials);
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
