// kk_probe.hip -- VALU issue cost of the instruction kinds the sweep kernels
// are built from, measured on the device.  Used to price the sweep kernels'
// roofline: on gfx950 the plain 32-bit bitwise and add instructions issue a
// wave64 in about half the SIMD cycles that a 32-bit multiply, a
// 32 x 32 -> 64 multiply-add or an fp32 FMA takes, so the VALU peak of a
// kernel depends on its instruction mix.
//
// Each probe kernel runs eight independent chains of one instruction kind
// (written in inline asm so that the compiler neither merges nor removes
// them) over enough waves to fill every SIMD; the time per instruction
// follows from the launch time, the wave count and the device's CU count
// and clock.
#include <hip/hip_runtime.h>

#include "../../include/kk.h"
#include "kk_host.hpp"

namespace {

constexpr int kIters = 1024;

#define KK_X8(S) S S S S S S S S
#define KK_CHAIN8(OP)                                                                                        \
  KK_X8(asm volatile(OP " %0, %0, %8\n" OP " %1, %1, %8\n" OP " %2, %2, %8\n" OP " %3, %3, %8\n" OP       \
                     " %4, %4, %8\n" OP " %5, %5, %8\n" OP " %6, %6, %8\n" OP " %7, %7, %8"                   \
                     : "+v"(a0), "+v"(a1), "+v"(a2), "+v"(a3), "+v"(a4), "+v"(a5), "+v"(a6), "+v"(a7)       \
                     : "v"(b));)

#define KK_PROBE2(NAME, OP)                                                                        \
  __global__ __launch_bounds__(512) void NAME(uint32_t* out, uint32_t seed) {                      \
    uint32_t a0 = threadIdx.x, a1 = a0 + 1, a2 = a0 + 2, a3 = a0 + 3, a4 = a0 + 4, a5 = a0 + 5,     \
             a6 = a0 + 6, a7 = a0 + 7;                                                             \
    const uint32_t b = seed | 1u;                                                                  \
    for (int it = 0; it < kIters; ++it) { KK_CHAIN8(OP) }                                          \
    out[blockIdx.x * blockDim.x + threadIdx.x] = a0 ^ a1 ^ a2 ^ a3 ^ a4 ^ a5 ^ a6 ^ a7;            \
  }

KK_PROBE2(probe_xor, "v_xor_b32")
KK_PROBE2(probe_add, "v_add_u32")
KK_PROBE2(probe_mul_lo, "v_mul_lo_u32")
KK_PROBE2(probe_lshl, "v_lshlrev_b32")
KK_PROBE2(probe_bcnt, "v_bcnt_u32_b32")

__global__ __launch_bounds__(512) void probe_fma(uint32_t* out, uint32_t seed) {
  float a0 = 1.0f + threadIdx.x * 1e-6f, a1 = a0 + 1e-3f, a2 = a0 + 2e-3f, a3 = a0 + 3e-3f, a4 = a0 + 4e-3f,
        a5 = a0 + 5e-3f, a6 = a0 + 6e-3f, a7 = a0 + 7e-3f;
  const float b = 0.5f + (float)(seed & 7u) * 1e-3f;
  for (int it = 0; it < kIters; ++it) {
    KK_X8(asm volatile("v_fma_f32 %0, %0, %8, %8\n v_fma_f32 %1, %1, %8, %8\n v_fma_f32 %2, %2, %8, %8\n"
                       "v_fma_f32 %3, %3, %8, %8\n v_fma_f32 %4, %4, %8, %8\n v_fma_f32 %5, %5, %8, %8\n"
                       "v_fma_f32 %6, %6, %8, %8\n v_fma_f32 %7, %7, %8, %8"
                       : "+v"(a0), "+v"(a1), "+v"(a2), "+v"(a3), "+v"(a4), "+v"(a5), "+v"(a6), "+v"(a7)
                       : "v"(b));)
  }
  out[blockIdx.x * blockDim.x + threadIdx.x] = __float_as_uint(a0 + a1 + a2 + a3 + a4 + a5 + a6 + a7);
}

__global__ __launch_bounds__(512) void probe_bitop3(uint32_t* out, uint32_t seed) {
  uint32_t a0 = threadIdx.x, a1 = a0 + 1, a2 = a0 + 2, a3 = a0 + 3, a4 = a0 + 4, a5 = a0 + 5, a6 = a0 + 6, a7 = a0 + 7;
  const uint32_t b = seed | 1u, c = seed * 3u;
  for (int it = 0; it < kIters; ++it) {
    KK_X8(asm volatile("v_bitop3_b32 %0, %0, %8, %9 bitop3:0x96\n v_bitop3_b32 %1, %1, %8, %9 bitop3:0x96\n"
                       "v_bitop3_b32 %2, %2, %8, %9 bitop3:0x96\n v_bitop3_b32 %3, %3, %8, %9 bitop3:0x96\n"
                       "v_bitop3_b32 %4, %4, %8, %9 bitop3:0x96\n v_bitop3_b32 %5, %5, %8, %9 bitop3:0x96\n"
                       "v_bitop3_b32 %6, %6, %8, %9 bitop3:0x96\n v_bitop3_b32 %7, %7, %8, %9 bitop3:0x96"
                       : "+v"(a0), "+v"(a1), "+v"(a2), "+v"(a3), "+v"(a4), "+v"(a5), "+v"(a6), "+v"(a7)
                       : "v"(b), "v"(c));)
  }
  out[blockIdx.x * blockDim.x + threadIdx.x] = a0 ^ a1 ^ a2 ^ a3 ^ a4 ^ a5 ^ a6 ^ a7;
}

__global__ __launch_bounds__(512) void probe_alignbit(uint32_t* out, uint32_t seed) {
  uint32_t a0 = threadIdx.x, a1 = a0 + 1, a2 = a0 + 2, a3 = a0 + 3, a4 = a0 + 4, a5 = a0 + 5, a6 = a0 + 6, a7 = a0 + 7;
  const uint32_t b = seed | 1u, c = 7u;
  for (int it = 0; it < kIters; ++it) {
    KK_X8(asm volatile("v_alignbit_b32 %0, %0, %8, %9\n v_alignbit_b32 %1, %1, %8, %9\n"
                       "v_alignbit_b32 %2, %2, %8, %9\n v_alignbit_b32 %3, %3, %8, %9\n"
                       "v_alignbit_b32 %4, %4, %8, %9\n v_alignbit_b32 %5, %5, %8, %9\n"
                       "v_alignbit_b32 %6, %6, %8, %9\n v_alignbit_b32 %7, %7, %8, %9"
                       : "+v"(a0), "+v"(a1), "+v"(a2), "+v"(a3), "+v"(a4), "+v"(a5), "+v"(a6), "+v"(a7)
                       : "v"(b), "v"(c));)
  }
  out[blockIdx.x * blockDim.x + threadIdx.x] = a0 ^ a1 ^ a2 ^ a3 ^ a4 ^ a5 ^ a6 ^ a7;
}

__global__ __launch_bounds__(512) void probe_mad64(uint32_t* out, uint32_t seed) {
  uint64_t a0 = threadIdx.x, a1 = a0 + 1, a2 = a0 + 2, a3 = a0 + 3, a4 = a0 + 4, a5 = a0 + 5, a6 = a0 + 6, a7 = a0 + 7;
  const uint32_t b = seed | 1u;
  uint64_t s0, s1, s2, s3, s4, s5, s6, s7;
  for (int it = 0; it < kIters; ++it) {
    KK_X8(asm volatile("v_mad_u64_u32 %0, %8, %16, %16, %0\n v_mad_u64_u32 %1, %9, %16, %16, %1\n"
                       "v_mad_u64_u32 %2, %10, %16, %16, %2\n v_mad_u64_u32 %3, %11, %16, %16, %3\n"
                       "v_mad_u64_u32 %4, %12, %16, %16, %4\n v_mad_u64_u32 %5, %13, %16, %16, %5\n"
                       "v_mad_u64_u32 %6, %14, %16, %16, %6\n v_mad_u64_u32 %7, %15, %16, %16, %7"
                       : "+v"(a0), "+v"(a1), "+v"(a2), "+v"(a3), "+v"(a4), "+v"(a5), "+v"(a6), "+v"(a7),
                         "=s"(s0), "=s"(s1), "=s"(s2), "=s"(s3), "=s"(s4), "=s"(s5), "=s"(s6), "=s"(s7)
                       : "v"(b));)
  }
  out[blockIdx.x * blockDim.x + threadIdx.x] = (uint32_t)(a0 ^ a1 ^ a2 ^ a3 ^ a4 ^ a5 ^ a6 ^ (a7 >> 32));
}

}  // namespace

using namespace kk;

extern "C" kk_status kk_valu_issue_cycles(double out[KK_VALU_PROBES]) {
  if (!out) return set_error(KK_EINVAL, "out is NULL");
  int dev = 0, cus = 0, khz = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e == hipSuccess) e = hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
  if (e == hipSuccess) e = hipDeviceGetAttribute(&khz, hipDeviceAttributeClockRate, dev);
  if (e != hipSuccess || cus <= 0 || khz <= 0)
    return set_error(KK_EDEVICE, "device attributes: %s", hipGetErrorString(e));
  // 32 waves per CU: 4 workgroups of 512 threads per CU
  const int threads = 512, blocks = cus * 4;
  uint32_t* buf = nullptr;
  e = hipMalloc(&buf, (size_t)blocks * threads * sizeof(uint32_t));
  if (e != hipSuccess) return set_error(KK_ENOMEM, "hipMalloc: %s", hipGetErrorString(e));
  hipEvent_t ev[2] = {nullptr, nullptr};
  typedef void (*Probe)(uint32_t*, uint32_t);
  const Probe probes[KK_VALU_PROBES] = {probe_xor, probe_bitop3, probe_alignbit, probe_add, probe_mad64,
                                        probe_mul_lo, probe_fma, probe_lshl, probe_bcnt};
  kk_status st = KK_OK;
  if ((e = hipEventCreate(&ev[0])) != hipSuccess || (e = hipEventCreate(&ev[1])) != hipSuccess)
    st = set_error(KK_EDEVICE, "hipEventCreate: %s", hipGetErrorString(e));
  for (int i = 0; i < KK_VALU_PROBES && st == KK_OK; ++i) {
    hipLaunchKernelGGL(probes[i], dim3(blocks), dim3(threads), 0, 0, buf, 1u);  // warm-up
    e = hipEventRecord(ev[0], 0);
    for (int r = 0; r < 3 && e == hipSuccess; ++r) {
      hipLaunchKernelGGL(probes[i], dim3(blocks), dim3(threads), 0, 0, buf, (uint32_t)r + 2u);
      e = hipGetLastError();
    }
    if (e == hipSuccess) e = hipEventRecord(ev[1], 0);
    if (e == hipSuccess) e = hipEventSynchronize(ev[1]);
    float ms = 0.f;
    if (e == hipSuccess) e = hipEventElapsedTime(&ms, ev[0], ev[1]);
    if (e != hipSuccess) {
      st = set_error(KK_EDEVICE, "probe %d: %s", i, hipGetErrorString(e));
      break;
    }
    // SIMD cycles per wave64 instruction: time x clock x SIMDs / (waves x instructions per wave)
    const double waves = (double)blocks * threads / 64.0, instr = 64.0 * kIters;
    out[i] = (ms / 3.0) * 1e-3 * (khz * 1e3) * (4.0 * cus) / (waves * instr);
  }
  for (hipEvent_t x : ev)
    if (x) (void)hipEventDestroy(x);
  (void)hipFree(buf);
  return st;
}
