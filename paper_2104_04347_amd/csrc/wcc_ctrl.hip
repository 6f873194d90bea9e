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

}  // namespace wcc
