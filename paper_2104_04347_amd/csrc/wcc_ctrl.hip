// wcc_ctrl.hip -- small stream-ordered kernels that set fields of the
// time-control blocks from values passed as kernel arguments (the host side
// then owns no buffer that an enqueued copy would still read).
#include <hip/hip_runtime.h>

#include "wcc_internal.hpp"
#include "wcc_ctrl.hpp"

namespace wcc {

__global__ void k_set_fields(Ctrl* ctrl, double t_end, double cfl) {
  if (threadIdx.x == 0) {
    ctrl->t_end = t_end;
    ctrl->cfl = cfl;
  }
}

hipError_t launch_set_fields(Ctrl* ctrl, double t_end, double cfl, hipStream_t s) {
  hipLaunchKernelGGL(k_set_fields, dim3(1), dim3(64), 0, s, ctrl, t_end, cfl);
  return hipGetLastError();
}

__global__ void k_batch_set_cfl(Ctrl* ctrl, const BatchInst* inst, int B, CflByDegree cfl) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < B) ctrl[i].cfl = cfl.v[inst[i].P];
}

hipError_t launch_batch_set_cfl(Ctrl* ctrl, const BatchInst* inst, int B, CflByDegree cfl, hipStream_t s) {
  if (B <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_batch_set_cfl, dim3((B + 255) / 256), dim3(256), 0, s, ctrl, inst, B, cfl);
  return hipGetLastError();
}

__global__ void k_init_ring(Ctrl* ctrl, unsigned long long* parts, RingInit init) {
  constexpr int n = (int)(kSmaxPartsBytes / sizeof(unsigned long long));
  for (int i = threadIdx.x; i < n; i += blockDim.x) parts[i] = 0ull;
  if (threadIdx.x == 0) {
    for (int k = 0; k < 3; ++k) {
      ctrl->t[k] = init.t;
      ctrl->smax[k] = 0ull;
      ctrl->flags[k] = 0u;
    }
    ctrl->pad0 = 0u;
    ctrl->t_end = __builtin_inf();
    ctrl->cfl = init.cfl;
    ctrl->steps_done = 0;
    for (int k = 0; k < 5; ++k) ctrl->pad1[k] = 0;
    for (int side = 0; side < 2; ++side)
      for (int k = 0; k < 3; ++k) ctrl->ghost[side][k] = init.ghost[side][k];
    ctrl->pad2[0] = ctrl->pad2[1] = 0.0;
  }
}

hipError_t launch_init_ring(Ctrl* ctrl, unsigned long long* parts, RingInit init, hipStream_t s) {
  hipLaunchKernelGGL(k_init_ring, dim3(1), dim3(256), 0, s, ctrl, parts, init);
  return hipGetLastError();
}

}  // namespace wcc
