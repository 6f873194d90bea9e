// wcc_kernels_wide.hip -- the fused WCC half-step with a second tile shape:
// two old cells per lane (the same per-cell arithmetic as wcc_kernels.hip,
// so the results are identical bit for bit).
//
// A wavefront owns a tile of 128 consecutive OLD cells and produces the 127
// NEW cells whose two parents both lie in it.  Lane l holds old cells l (the
// tile's first half, "A") and l + 64 (the second half, "B"); both are loaded
// as whole 64-cell row segments.  Every lane expands its two cells (two
// independent Cauchy-Kovalewski chains the compiler interleaves), then:
//   * new cell l of the first half has parents A_l and A_{l+1}: the right
//     parent's interface data come from lane l+1 by DPP wave_shl:1, except for
//     lane 63, whose right parent is B_0 -- its data are broadcast from lane 0
//     and enter as the DPP "old" value of the one lane without a source;
//   * new cell 64 + l (l < 63) has parents B_l and B_{l+1}, again by DPP.
// Compared with the 64-cell tile (63 new cells per 64 expansions) a tile
// repeats one expansion per 128 instead of one per 64, and each lane carries
// two cells' registers (fewer waves per SIMD, two chains per wave).
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "wcc_cell.hpp"
#include "wcc_internal.hpp"
#include "wcc_tile.hpp"
#include "wcc_wide.hpp"

namespace wcc {

namespace {

// DPP wave_shl:1 with a given value for lane 63 (the lane without a source).
__device__ __forceinline__ int dpp_next_or(int x, int last) {
  return __builtin_amdgcn_update_dpp(last, x, 0x130, 0xF, 0xF, false);
}
__device__ __forceinline__ float dpp_next_or(float x, float last) {
  return __int_as_float(dpp_next_or(__float_as_int(x), __float_as_int(last)));
}
__device__ __forceinline__ double dpp_next_or(double x, double last) {
  const long long v = __double_as_longlong(x), w = __double_as_longlong(last);
  const int lo = dpp_next_or((int)(v & 0xffffffffll), (int)(w & 0xffffffffll));
  const int hi = dpp_next_or((int)(v >> 32), (int)(w >> 32));
  return __longlong_as_double(((long long)hi << 32) | (long long)(unsigned)lo);
}

// Lane 0's value, the same in every lane.
__device__ __forceinline__ float lane0(float x) {
  return __int_as_float(__builtin_amdgcn_readfirstlane(__float_as_int(x)));
}
__device__ __forceinline__ double lane0(double x) {
  const long long v = __double_as_longlong(x);
  const unsigned lo = (unsigned)__builtin_amdgcn_readfirstlane((int)(v & 0xffffffffll));
  const unsigned hi = (unsigned)__builtin_amdgcn_readfirstlane((int)(v >> 32));
  return __longlong_as_double((long long)(((unsigned long long)hi << 32) | lo));
}

// The inputs of the old cell with index o (before the boundary mapping).
template <int EQ, int P, class R>
__device__ __forceinline__ void fetch_old(const StepArgs<R>& a, int o_raw, TileIn<EQ, P, R>& in) {
  constexpr int NC = ncomp<EQ>();
  int ghost;
  const int o = map_old(o_raw, (int)a.n_old, (int)a.N, a.bc, a.parity_old, ghost);
#pragma unroll
  for (int c = 0; c < NC; ++c) {
    in.p[c] = row_at(row_base(a.p_old + c * a.ld), (uint32_t)o);
    in.d[c][0] = (R)0;
#pragma unroll
    for (int k = 1; k <= P; ++k) in.d[c][k] = row_at(row_base(a.d_old + (c * P + (k - 1)) * a.ld), (uint32_t)o);
  }
  if (ghost) {
    const double* g = a.ctrl->ghost[ghost - 1];
#pragma unroll
    for (int c = 0; c < NC; ++c) {
      in.p[c] = g[c];
#pragma unroll
      for (int k = 1; k <= P; ++k) in.d[c][k] = (R)0;
    }
  }
}

template <int EQ, int P, class R>
__device__ __forceinline__ void store_new(const StepArgs<R>& a, int j, const double (&pn)[ncomp<EQ>()],
                                          const R (&dn)[ncomp<EQ>()][P + 1]) {
  constexpr int NC = ncomp<EQ>();
#pragma unroll
  for (int c = 0; c < NC; ++c) {
    row_store(row_base(a.p_new + c * a.ld), (uint32_t)j, pn[c]);
#pragma unroll
    for (int k = 1; k <= P; ++k) row_store(row_base(a.d_new + (c * P + (k - 1)) * a.ld), (uint32_t)j, dn[c][k]);
  }
}

template <int EQ, int P, bool LIM, class R>
__device__ __forceinline__ void wide_tile(const StepArgs<R>& a, int64_t tile, double lam, R nlam, int lane,
                                          double& smax, unsigned& flags) {
  constexpr int NC = ncomp<EQ>();
  constexpr int PV = P > 0 ? P : 1;
  // cell indices fit 32 bits (N <= 2^28, checked at creation)
  const int j0 = (int)tile * 127;
  const int shift = a.parity_old == 1 ? 1 : 0;   // odd->even: the left parent of new cell j is old cell j-1
  TileIn<EQ, P, R> inA, inB;
  fetch_old<EQ, P, R>(a, j0 + lane - shift, inA);
  fetch_old<EQ, P, R>(a, j0 + 64 + lane - shift, inB);
  OldOut<EQ, P, R> XA, XB;
  old_cell<EQ, P, R>(inA.p, inA.d, nlam, a.ph, XA);
  old_cell<EQ, P, R>(inB.p, inB.d, nlam, a.ph, XB);
  __builtin_amdgcn_sched_barrier(0);

  // first half: right parents A_{l+1}, and B_0 for lane 63
  {
    double uL_R[NC];
    R fbar_R[NC];
    R V_R[NC][PV];
#pragma unroll
    for (int c = 0; c < NC; ++c) {
      uL_R[c] = dpp_next_or(XA.uL[c], lane0(XB.uL[c]));
      fbar_R[c] = dpp_next_or(XA.fbar[c], lane0(XB.fbar[c]));
#pragma unroll
      for (int k = 0; k < P; ++k) V_R[c][k] = dpp_next_or(XA.V[c][k], lane0(XB.V[c][k]));
      if (P == 0) V_R[c][0] = (R)0;
    }
    const int j = j0 + lane;
    if (j < (int)a.n_new) {
      double pn[NC], sp;
      R dn[NC][P + 1];
      flags |= (unsigned)new_cell<EQ, P, LIM, R>(XA, uL_R, fbar_R, V_R, lam, a.ph, pn, dn, sp);
      smax = __builtin_fmax(smax, sp);
      if (!(sp == sp)) smax = sp;
      store_new<EQ, P, R>(a, j, pn, dn);
    }
  }
  // second half: right parents B_{l+1}
  {
    double uL_R[NC];
    R fbar_R[NC];
    R V_R[NC][PV];
#pragma unroll
    for (int c = 0; c < NC; ++c) {
      uL_R[c] = dpp_from_next(XB.uL[c]);
      fbar_R[c] = dpp_from_next(XB.fbar[c]);
#pragma unroll
      for (int k = 0; k < P; ++k) V_R[c][k] = dpp_from_next(XB.V[c][k]);
      if (P == 0) V_R[c][0] = (R)0;
    }
    const int j = j0 + 64 + lane;
    if (lane < 63 && j < (int)a.n_new) {
      double pn[NC], sp;
      R dn[NC][P + 1];
      flags |= (unsigned)new_cell<EQ, P, LIM, R>(XB, uL_R, fbar_R, V_R, lam, a.ph, pn, dn, sp);
      smax = __builtin_fmax(smax, sp);
      if (!(sp == sp)) smax = sp;
      store_new<EQ, P, R>(a, j, pn, dn);
    }
  }
}

}  // namespace

// Blocks own contiguous ranges of 128-cell tiles, their waves walk them
// blockDim/64 apart; time control and the wave-speed reduction as in
// k_half_step.
template <int EQ, int P, bool LIM, class R>
__global__ __launch_bounds__(256) void k_half_step_wide(const StepArgs<R> a) {
  double dt;
  if (!step_time(a.ctrl, a.parts, a.slot, a.dx, a.dt_fixed, blockIdx.x == 0 && threadIdx.x < 64, dt)) return;
  const double lam = div_rn(dt, a.dx);
  const R nlam = (R)(-lam);
  const int lane = threadIdx.x & 63, wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6),
            nw = blockDim.x >> 6;
  const int64_t tiles = (a.n_new + 126) / 127;
  const int64_t per_block = (tiles + gridDim.x - 1) / gridDim.x;
  const int64_t t_begin = (int64_t)blockIdx.x * per_block;
  const int64_t t_stop = t_begin + per_block < tiles ? t_begin + per_block : tiles;
  double smax = 0.0;
  unsigned flags = 0u;
  for (int64_t tile = t_begin + wave; tile < t_stop; tile += nw)
    wide_tile<EQ, P, LIM, R>(a, tile, lam, nlam, lane, smax, flags);
  publish(a.ctrl, a.parts, a.slot, smax, flags);
}

namespace {

template <int EQ, int P, class R>
hipError_t launch_wide_lim(const StepArgs<R>& a, bool lim, int blocks, int threads, hipStream_t s) {
  if (lim && P >= 1)
    hipLaunchKernelGGL((k_half_step_wide<EQ, P, (P >= 1), R>), dim3(blocks), dim3(threads), 0, s, a);
  else
    hipLaunchKernelGGL((k_half_step_wide<EQ, P, false, R>), dim3(blocks), dim3(threads), 0, s, a);
  return hipGetLastError();
}

template <int EQ, class R>
hipError_t launch_wide_p(const StepArgs<R>& a, int P, bool lim, int blocks, int threads, hipStream_t s) {
  switch (P) {
    case 0: return launch_wide_lim<EQ, 0, R>(a, false, blocks, threads, s);
    case 1: return launch_wide_lim<EQ, 1, R>(a, lim, blocks, threads, s);
    case 2: return launch_wide_lim<EQ, 2, R>(a, lim, blocks, threads, s);
    case 3: return launch_wide_lim<EQ, 3, R>(a, lim, blocks, threads, s);
    case 4: return launch_wide_lim<EQ, 4, R>(a, lim, blocks, threads, s);
  }
  return hipErrorInvalidValue;
}

template <int EQ, int P, bool LIM, class R>
const void* wide_fn() {
  return reinterpret_cast<const void*>(&k_half_step_wide<EQ, P, LIM, R>);
}

template <int EQ, class R>
const void* wide_fn_p(int P, bool lim) {
  switch (P) {
    case 0: return wide_fn<EQ, 0, false, R>();
    case 1: return lim ? wide_fn<EQ, 1, true, R>() : wide_fn<EQ, 1, false, R>();
    case 2: return lim ? wide_fn<EQ, 2, true, R>() : wide_fn<EQ, 2, false, R>();
    case 3: return lim ? wide_fn<EQ, 3, true, R>() : wide_fn<EQ, 3, false, R>();
    case 4: return lim ? wide_fn<EQ, 4, true, R>() : wide_fn<EQ, 4, false, R>();
  }
  return nullptr;
}

}  // namespace

template <class R>
hipError_t launch_half_step_wide(const StepArgs<R>& a, int eq, int P, bool lim, int blocks, int threads,
                                 hipStream_t s) {
  switch (eq) {
    case kAdvection: return launch_wide_p<kAdvection, R>(a, P, lim, blocks, threads, s);
    case kBurgers: return launch_wide_p<kBurgers, R>(a, P, lim, blocks, threads, s);
    case kEuler: return launch_wide_p<kEuler, R>(a, P, lim, blocks, threads, s);
  }
  return hipErrorInvalidValue;
}

template <class R>
hipError_t occupancy_half_step_wide(int eq, int P, bool lim, int threads, int* blocks_per_cu) {
  const void* f = eq == kAdvection ? wide_fn_p<kAdvection, R>(P, lim)
                  : eq == kBurgers ? wide_fn_p<kBurgers, R>(P, lim)
                                   : wide_fn_p<kEuler, R>(P, lim);
  if (!f) return hipErrorInvalidValue;
  return hipOccupancyMaxActiveBlocksPerMultiprocessor(blocks_per_cu, f, threads, 0);
}

template hipError_t launch_half_step_wide<double>(const StepArgs<double>&, int, int, bool, int, int, hipStream_t);
template hipError_t launch_half_step_wide<float>(const StepArgs<float>&, int, int, bool, int, int, hipStream_t);
template hipError_t occupancy_half_step_wide<double>(int, int, bool, int, int*);
template hipError_t occupancy_half_step_wide<float>(int, int, bool, int, int*);

}  // namespace wcc
