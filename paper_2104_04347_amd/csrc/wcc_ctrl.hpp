// wcc_ctrl.hpp -- stream-ordered updates of the time-control blocks from
// values passed as kernel arguments (host side of the library only).
#pragma once

#include <hip/hip_runtime.h>

#include "wcc_internal.hpp"

namespace wcc {

// Ctrl::t_end and Ctrl::cfl of one control block.  The values travel as
// kernel arguments, so no host buffer has to outlive the call.
hipError_t launch_set_fields(Ctrl* ctrl, double t_end, double cfl, hipStream_t s);

// Per-degree CFL numbers of the batched form, passed by value.
struct CflByDegree {
  double v[5];
};
// ctrl[i].cfl = cfl.v[inst[i].P] for the B instances.
hipError_t launch_batch_set_cfl(Ctrl* ctrl, const BatchInst* inst, int B, CflByDegree cfl, hipStream_t s);

// Initial contents of a time-control block: time t in every slot, no wave
// speed, no flags, no end time, the CFL number and the Dirichlet ghost states.
struct RingInit {
  double t;
  double cfl;
  double ghost[2][3];
};
// Resets the control block and clears the partial wave-speed maxima
// (kSmaxPartsBytes at parts); a fill by kernel, no memset node.
hipError_t launch_init_ring(Ctrl* ctrl, unsigned long long* parts, RingInit init, hipStream_t s);

}  // namespace wcc
