// wcc_internal.hpp -- device-side control block and kernel argument blocks
// shared by the kernels and the host library (not part of the public ABI).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "wcc_cell.hpp"

namespace wcc {

// Time-control ring in device memory.  Launch n uses slot n % 3: it reads
// t[slot], smax[slot] and flags[slot], writes t[slot+1], max-reduces the new
// wave speeds into smax[slot+1], ORs new status bits into flags[slot+1] and
// clears slot+2 for the launch after.  smax holds the bit pattern of a
// non-negative double, so an unsigned integer max is the floating-point max.
struct Ctrl {
  double t[3];
  unsigned long long smax[3];
  unsigned int flags[3];
  unsigned int pad0;
  double t_end;
  double cfl;
  long long steps_done;   // half-steps actually taken since the last write
  long long pad1[5];
  double ghost[2][3];     // Dirichlet ghost states (left, right), conserved variables
  double pad2[2];
};
static_assert(sizeof(Ctrl) == 192, "control block layout");

// Partial wave-speed maxima of the single-instance kernels: 64 entries per
// ring slot, one 64-byte line each, so the blocks of a launch spread their
// atomics over 64 addresses instead of queueing on one; the next launch
// reduces the 64 entries with one wave-wide max.
constexpr int kSmaxParts = 64;
constexpr int kSmaxStride = 8;  // unsigned long long per entry (64 bytes)
constexpr size_t kSmaxPartsBytes = 3 * kSmaxParts * kSmaxStride * sizeof(unsigned long long);

template <class R>
struct StepArgs {
  const double* p_old;    // point values of the old mesh, [c][j]
  const R* d_old;         // derivatives of the old mesh, [c][k-1][j]
  double* p_new;
  R* d_new;
  int64_t ld;             // row length (cells) of every [c] / [c][k-1] row
  int64_t n_old, n_new, N;
  int32_t parity_old;     // 0: original -> staggered, 1: staggered -> original
  int32_t bc;
  double dx;
  double dt_fixed;        // > 0: fixed dt instead of the CFL step
  Phys<R> ph;
  Ctrl* ctrl;
  unsigned long long* parts;  // partial maxima (single instance), or null: Ctrl::smax (batched)
  int32_t slot;
  int32_t pad;
};

// Batched instances: one table row per instance and one per tile.
struct BatchInst {
  int64_t p_off;          // offset of the instance's point-value block (doubles)
  int64_t d_off;          // offset of its derivative block (bulk elements)
  int64_t ld;             // row length
  int64_t N;              // mesh intervals
  double dx;
  double cfl;
  int32_t P;
  int32_t pad;
};

struct BatchTile {
  int32_t inst;           // instance
  int32_t first;          // first new cell / 63 (wave tile index inside the instance)
};

template <class R>
struct BatchArgs {
  const double* p_in;     // point values of all instances, buffer of this step's input
  const R* d_in;
  double* p_out;
  R* d_out;
  const BatchInst* inst;
  const BatchTile* tiles; // sorted by instance, tiles of one instance contiguous
  int64_t n_tiles;
  Ctrl* ctrl;             // one control block per instance
  Phys<R> ph;
  int32_t parity_old;     // same for every instance (all start on the original mesh)
  int32_t slot;
};

template <class R>
hipError_t launch_half_step(const StepArgs<R>& a, int eq, int P, bool lim, int prefetch, int blocks, int threads,
                            hipStream_t s);
template <class R>
hipError_t launch_state_speed(const StepArgs<R>& a, int eq, int P, int blocks, hipStream_t s);
template <class R>
hipError_t occupancy_half_step(int eq, int P, bool lim, int prefetch, int threads, int* blocks_per_cu);

}  // namespace wcc
