// wcc2d_internal.hpp -- kernel argument block of the 2D half-step and the
// launchers (host library <-> kernels; not part of the public ABI).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "wcc2d_cell.hpp"
#include "wcc_internal.hpp"

namespace wcc2d {

struct Step2Args {
  const double* q_old;    // state of the old mesh: planes [c][dof], index j*Nx + i
  double* q_new;
  int64_t plane;          // doubles per plane (cells of the larger mesh rounded up to 64)
  int32_t Nx, Ny;         // mesh intervals (dx = domain width / Nx)
  int32_t nxo, nyo;       // cells of the old mesh (row width nxo)
  int32_t nxn, nyn;       // cells of the new mesh
  int32_t periodic_x;     // 1: indices wrap; 0: transmissive, indices clamp to the edge cell
  int32_t periodic_y;
  int32_t parity_old;     // 0: original -> staggered mesh, 1: back
  int32_t slot;           // ring slot of this launch
  double dx, dy;
  double idx, idy;        // 1/dx, 1/dy
  double dt_fixed;        // > 0: fixed dt instead of the CFL step
  Phys2 ph;
  wcc::Ctrl* ctrl;
  unsigned long long* parts;
};

// variant 0: 8 x 8 wave tiles; 1: row marching over 64-column strips; 2: the
// same with the next row prefetched; 3: the same with band-major work items
// (identical results)
hipError_t launch_half_step2(const Step2Args& a, int eq, int P, bool lim, int variant, int blocks, int threads,
                             hipStream_t s);
hipError_t launch_state_speed2(const Step2Args& a, int eq, int P, int blocks, hipStream_t s);
// plane: doubles per plane of the state (selects the kernel form launched for it)
hipError_t occupancy_half_step2(int eq, int P, bool lim, int variant, int threads, int64_t plane,
                                int* blocks_per_cu);

}  // namespace wcc2d
