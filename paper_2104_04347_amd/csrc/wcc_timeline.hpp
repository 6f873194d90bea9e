// wcc_timeline.hpp -- per-wave timestamps for the diagnostic build of the
// half-step kernels (libwcc_timeline.so; the product library never includes
// this file).
//
// A diagnostic translation unit includes this header, then the kernel source
// with `step_time` and `publish` redirected to the wrappers below: every
// half-step kernel calls step_time first and publish last, so the wrappers
// bracket each wave's life without any change to the kernel source.  Lane 0
// of each wave writes one record: the 100 MHz constant clock and the shader
// clock counter at both ends, and the hardware placement (HW_ID, XCC_ID).
// The ratio of the two clocks over a wave's life is the shader clock the wave
// ran at.  Records are indexed by the global wave index; each launch
// overwrites the records of its waves, so after a run of half-steps they hold
// the last launch.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "wcc_tile.hpp"

namespace wcc {

struct TimelineRec {
  unsigned long long t0, t1;   // s_memrealtime (100 MHz) at entry and exit
  unsigned long long c0, c1;   // s_memtime (shader clock) at entry and exit
  unsigned int hw_id;          // hardware register HW_ID: wave, SIMD, CU, SH, SE fields
  unsigned int xcc_id;         // hardware register XCC_ID
  unsigned int pad[2];
};
static_assert(sizeof(TimelineRec) == 48, "timeline record layout");
constexpr int kTimelineWaves = 16384;

// one array per diagnostic translation unit
static __device__ TimelineRec g_timeline[kTimelineWaves];

__device__ __forceinline__ int timeline_wave() {
  return (int)blockIdx.x * (int)(blockDim.x >> 6) + (int)(threadIdx.x >> 6);
}

// s_getreg operand: size - 1 in bits 15:11, offset in bits 10:6, register id
// in bits 5:0 (HW_ID = 4, XCC_ID = 20), the whole 32-bit register
constexpr int kGetregHwId = (31 << 11) | 4;
constexpr int kGetregXccId = (31 << 11) | 20;

__device__ __forceinline__ bool step_time_tl(Ctrl* ctrl, unsigned long long* parts, int slot, double dx,
                                             double dt_fixed, bool leader_wave, double& dt) {
  const unsigned long long t0 = __builtin_amdgcn_s_memrealtime();
  const unsigned long long c0 = __builtin_amdgcn_s_memtime();
  const int w = timeline_wave();
  if ((threadIdx.x & 63) == 0 && w < kTimelineWaves) {
    g_timeline[w].t0 = t0;
    g_timeline[w].c0 = c0;
  }
  return step_time(ctrl, parts, slot, dx, dt_fixed, leader_wave, dt);
}

__device__ __forceinline__ void publish_tl(Ctrl* ctrl, unsigned long long* parts, int slot, double smax,
                                           unsigned flags) {
  const unsigned long long t1 = __builtin_amdgcn_s_memrealtime();
  const unsigned long long c1 = __builtin_amdgcn_s_memtime();
  const int w = timeline_wave();
  if ((threadIdx.x & 63) == 0 && w < kTimelineWaves) {
    g_timeline[w].t1 = t1;
    g_timeline[w].c1 = c1;
    g_timeline[w].hw_id = __builtin_amdgcn_s_getreg(kGetregHwId);
    g_timeline[w].xcc_id = __builtin_amdgcn_s_getreg(kGetregXccId);
  }
  publish(ctrl, parts, slot, smax, flags);
}

}  // namespace wcc

// Host side of one diagnostic translation unit: clear the records (before a
// run), copy them out (after it).  Synchronous copies on the null stream.
#define WCC_TIMELINE_ENTRY_POINTS(suffix)                                                                      \
  extern "C" int wcc_timeline_clear_##suffix(void) {                                                           \
    static const wcc::TimelineRec zero[wcc::kTimelineWaves] = {};                                              \
    return (int)hipMemcpyToSymbol(HIP_SYMBOL(wcc::g_timeline), zero, sizeof zero, 0, hipMemcpyHostToDevice);   \
  }                                                                                                            \
  extern "C" int wcc_timeline_read_##suffix(void* dst, size_t bytes) {                                         \
    if (!dst || bytes < sizeof(wcc::g_timeline)) return 1;                                                     \
    return (int)hipMemcpyFromSymbol(dst, HIP_SYMBOL(wcc::g_timeline), sizeof(wcc::g_timeline), 0,              \
                                    hipMemcpyDeviceToHost);                                                    \
  }
