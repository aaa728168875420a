// kk_noalloc.hip -- kk_sweep_noalloc: square-torus sweeps of a caller-held
// device lattice with no allocation of any kind, for callers that cannot
// allocate (code under HIP graph capture, tight serving loops).
//
// The sweep kernels read one lattice buffer and write the other, and add
// each tile's accepted exchanges into a per-tile running sum.  Here the
// caller's lattice is one buffer; the other buffer and the per-tile sums live
// in `scratch`, a file-scope device array of fixed size that every GPU the
// library runs on holds until the process ends.
#include <hip/hip_runtime.h>

#include <cmath>
#include <mutex>

#include "../../include/kk.h"
#include "kk_host.hpp"
#include "kk_kernels.hpp"

namespace {

// The second lattice buffer (up to 8 MiB: bit-packed L <= 8192, int8 L <= 2896)
// followed by one running sum per sweep tile.
constexpr size_t kLatticeMax = (size_t)8 << 20;
constexpr size_t kPartialsMax = 4096;
constexpr size_t kScratchBytes = kLatticeMax + kPartialsMax * sizeof(unsigned long long);
static_assert(kScratchBytes == KK_NOALLOC_SCRATCH_BYTES, "kk.h states the scratch size");

static __device__ __align__(256) unsigned char scratch[kScratchBytes];

// Device address of `scratch` on each device, looked up once per device
// (the array's name on the host is only a stand-in for the symbol).
constexpr int kMaxDevices = 64;
std::mutex g_mu;
unsigned char* g_scratch[kMaxDevices] = {};

kk_status scratch_on_current_device(unsigned char** out) {
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return kk::set_error(KK_EDEVICE, "hipGetDevice failed: %s", hipGetErrorString(e));
  if (dev < 0 || dev >= kMaxDevices) return kk::set_error(KK_EDEVICE, "device %d beyond %d", dev, kMaxDevices);
  std::lock_guard<std::mutex> lk(g_mu);
  if (!g_scratch[dev]) {
    void* ptr = nullptr;
    e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !ptr)
      return kk::set_error(KK_EDEVICE, "hipGetSymbolAddress(scratch) failed: %s", hipGetErrorString(e));
    g_scratch[dev] = static_cast<unsigned char*>(ptr);
  }
  *out = g_scratch[dev];
  return KK_OK;
}

__global__ void zero_u64(unsigned long long* p, int n) {
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) p[i] = 0ull;
}

// One workgroup: sum the n per-tile counts and add the total into *out.
__global__ __launch_bounds__(256) void add_partials(const unsigned long long* p, int n, unsigned long long* out) {
  __shared__ unsigned long long red[4];
  unsigned long long s = 0;
  for (int i = threadIdx.x; i < n; i += blockDim.x) s += p[i];
  for (int off = 32; off > 0; off >>= 1) s += __shfl_down(s, off, 64);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = s;
  __syncthreads();
  if (threadIdx.x == 0) *out += red[0] + red[1] + red[2] + red[3];
}

}  // namespace

using namespace kk;

extern "C" kk_status kk_sweep_noalloc(void* lattice, uint32_t L, uint32_t layout, double omega_kT, uint64_t seed,
                                      uint64_t t0, uint64_t n_sweeps, unsigned long long* accepted,
                                      void* hip_stream) {
  if (!lattice) return set_error(KK_EINVAL, "lattice is NULL");
  if (L < 4 || (L % 4) != 0) return set_error(KK_EINVAL, "L must be a multiple of 4, at least 4 (got %u)", L);
  if (!std::isfinite(omega_kT)) return set_error(KK_EINVAL, "omega must be finite");
  int lay;
  if (layout == KK_LAYOUT_INT8) lay = kLayoutInt8;
  else if (layout == KK_LAYOUT_BITPACKED) {
    if (L % 32 != 0) return set_error(KK_EINVAL, "bit-packed layout needs L %% 32 == 0 (got %u)", L);
    lay = kLayoutBits;
  } else return set_error(KK_EINVAL, "layout must be KK_LAYOUT_INT8 or KK_LAYOUT_BITPACKED (got %u)", layout);
  const uint64_t lim = (uint64_t)1 << 60;
  if (t0 >= lim || n_sweeps >= lim || t0 + n_sweeps >= lim)
    return set_error(KK_EINVAL, "sweep counter would reach 2^60");
  const size_t bytes = lay == kLayoutBits ? (size_t)L * (L / 32) * 4 : (size_t)L * L;
  if (bytes > kLatticeMax)
    return set_error(KK_EINVAL, "lattice of %zu bytes exceeds the %zu-byte scratch lattice", bytes, kLatticeMax);
  TileConfig tc;
  default_tile((int)L, lay, &tc);
  SweepParams p{};
  const int threads = tile_geometry((int)L, tc, &p);
  const size_t tiles = (size_t)p.tiles_x * (size_t)(((int)L + p.th - 1) / p.th);
  if (tiles > kPartialsMax)
    return set_error(KK_EINVAL, "%zu sweep tiles exceed the %zu scratch counts", tiles, kPartialsMax);
  if (n_sweeps == 0) return KK_OK;

  unsigned char* base = nullptr;
  kk_status st = scratch_on_current_device(&base);
  if (st != KK_OK) return st;
  void* other = base;
  unsigned long long* partials = reinterpret_cast<unsigned long long*>(base + kLatticeMax);
  hipStream_t stream = static_cast<hipStream_t>(hip_stream);

#define KK_NA_HIP(expr)                                                                                  \
  do {                                                                                                   \
    hipError_t e_ = (expr);                                                                              \
    if (e_ != hipSuccess)                                                                                \
      return set_error(KK_EDEVICE, "%s failed: %s", #expr, hipGetErrorString(e_));                      \
  } while (0)

  // the counts of the previous call on this device are still there
  hipLaunchKernelGGL(zero_u64, dim3(((unsigned)tiles + 255) / 256), dim3(256), 0, stream, partials, (int)tiles);
  KK_NA_HIP(hipGetLastError());
  uint64_t T[7];
  acceptance_table(omega_kT, T, &p.acc);
  p.accepted = partials;
  p.k0 = (uint32_t)(seed & 0xFFFFFFFFu);
  p.k1 = (uint32_t)(seed >> 32);
  void* buf[2] = {lattice, other};
  int cur = 0;
  uint64_t t = t0, n = n_sweeps;
  const uint64_t per_launch = tc.cyclic ? 256 : 1;
  while (n > 0) {
    const uint64_t k = n < per_launch ? n : per_launch;
    p.src = buf[cur];
    p.dst = buf[cur ^ 1];
    p.t0 = t;
    p.nsweeps = (int)k;
    KK_NA_HIP(launch_sweep(p, lay, tc.cyclic, tc.ku, threads, stream));
    cur ^= 1;
    t += k;
    n -= k;
  }
  if (cur != 0) KK_NA_HIP(hipMemcpyAsync(lattice, other, bytes, hipMemcpyDeviceToDevice, stream));
  if (accepted) {
    hipLaunchKernelGGL(add_partials, dim3(1), dim3(256), 0, stream, partials, (int)tiles, accepted);
    KK_NA_HIP(hipGetLastError());
  }
#undef KK_NA_HIP
  return KK_OK;
}
