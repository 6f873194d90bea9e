// wcc_kernels.hip -- the fused WCC half-step kernels for gfx950 (MI355X).
//
// One launch = one half-step of one instance (Section 2.1 of Shen & Parsani,
// arXiv:2104.04347).  Work decomposition:
//   * a wavefront owns a tile of 64 consecutive OLD cells and produces the 63
//     NEW cells whose two parents both lie in the tile (one old cell of
//     overlap between neighbouring tiles: 1/64 redundant expansion work);
//   * every lane expands its own old cell (Cauchy-Kovalewski in registers),
//     then takes the right parent's half of the interface data from lane+1
//     with DPP wave_shl:1 row moves -- no LDS, no barrier (the staged
//     variants add LDS and two block barriers per iteration for the stores);
//   * a block owns a contiguous run of tiles (its waves walk it four apart),
//     so neighbouring tiles share cache lines inside one CU / XCD;
//   * the state is structure of arrays: point values [c][j] in binary64 and
//     derivatives [c][k-1][j] in the bulk type, rows padded to 64 cells, so
//     every load and store of a wave is a contiguous 256/512-byte segment
//     (64-aligned in the staged variants).
// Time control is on the device: the kernel reads t and s_max from a ring of
// three slots, writes the next time to the next slot, max-reduces its wave
// speeds into the next slot and clears the slot after that, so consecutive
// launches (and captured graphs of them) need no host round trip.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "wcc_cell.hpp"
#include "wcc_internal.hpp"
#include "wcc_tile.hpp"

namespace wcc {

// Register budget: the least number of waves per SIMD a kernel is compiled
// for (1: no bound, the compiler's own allocation).  The binary64 Euler
// kernels of degree 3 with direct stores allocate 130 VGPRs when left free,
// two over the 128 that four waves per SIMD allow; held to four waves they fit
// without spilling and ran ~2.5% faster on the N = 2^20 workload.  Held to four
// waves, the prefetching variants of the same kernel spill and run 30-40%
// slower, the binary32 kernels already run at four to six, and the other
// binary64 kernels sit well below or well above a step of the register file.
template <int EQ, int P, class R, int PF>
constexpr int min_waves_per_simd() {
  return (EQ == kEuler && P == 3 && sizeof(R) == 8 && PF == 0) ? 4 : 1;
}

// Variant bits.  PF & 1: each wave loads the inputs of its next tile before
// expanding the current one, so every wave keeps one tile of loads in flight
// while it computes (costs the registers of one tile's inputs).  PF & 2: the
// new cells go through LDS and are stored in whole 64-cell groups (two block
// barriers per iteration of the block's waves; pays where the state does not
// fit the caches).
template <int EQ, int P, bool LIM, class R, int PF>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(min_waves_per_simd<EQ, P, R, PF>())))
void k_half_step(const StepArgs<R> a) {
  double dt;
  if (!step_time(a.ctrl, a.parts, a.slot, a.dx, a.dt_fixed, blockIdx.x == 0 && threadIdx.x < 64, dt)) return;
  const double lam = div_rn(dt, a.dx);
  const R nlam = (R)(-lam);
  // the wave index is the same in every lane: say so, so that tile and
  // instance indices live in scalar registers
  const int lane = threadIdx.x & 63, wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6),
            nw = blockDim.x >> 6;
  const int64_t tiles = (a.n_new + 62) / 63;
  const int64_t per_block = (tiles + gridDim.x - 1) / gridDim.x;
  const int64_t t_begin = (int64_t)blockIdx.x * per_block;
  const int64_t t_stop = t_begin + per_block < tiles ? t_begin + per_block : tiles;
  double smax = 0.0;
  unsigned flags = 0u;
  if constexpr ((PF & 2) != 0) {
    constexpr int NC = ncomp<EQ>();
    __shared__ Stage<EQ, P, R> st;
    int cur = 0;
    TileIn<EQ, P, R> in;
    if ((PF & 1) && t_begin + wave < t_stop) fetch_tile<EQ, P, R>(a, t_begin + wave, lane, in);
    // every wave runs every iteration (the barriers are block-wide)
    for (int64_t tb = t_begin; tb < t_stop; tb += nw) {
      const int64_t tile = tb + wave;
      int lo = 0, hi = 0;
      if (tile < t_stop) {
        TileIn<EQ, P, R> nxt;
        if constexpr ((PF & 1) != 0) {
          const int64_t t2 = tile + nw < t_stop ? tile + nw : tile;   // in bounds; unused at the end
          fetch_tile<EQ, P, R>(a, t2, lane, nxt);
          __builtin_amdgcn_sched_barrier(0);
        } else {
          fetch_tile<EQ, P, R>(a, tile, lane, in);
        }
        double pn[NC];
        R dn[NC][P + 1];
        if (tile_cells<EQ, P, LIM, R>(a, tile, in, lam, nlam, lane, smax, flags, pn, dn))
          stage_put<EQ, P, R>(st, wave * 64 + lane, pn, dn);
        if constexpr ((PF & 1) != 0) in = nxt;
        lo = (int)tile * 63;
        hi = lo + 63 < (int)a.n_new ? lo + 63 : (int)a.n_new;
      }
      __syncthreads();
      stage_flush<EQ, P, R>(st, cur, wave, nw, lane, lo, hi, tile > t_begin, tile + 1 < t_stop, a.p_new, a.d_new,
                            a.ld);
      __syncthreads();
      cur ^= 1;
    }
  } else if constexpr (PF == 0) {
    for (int64_t tile = t_begin + wave; tile < t_stop; tile += nw)
      run_tile<EQ, P, LIM, R>(a, tile, lam, nlam, lane, smax, flags);
  } else {
    int64_t tile = t_begin + wave;
    if (tile < t_stop) {
      TileIn<EQ, P, R> cur;
      fetch_tile<EQ, P, R>(a, tile, lane, cur);
      for (; tile < t_stop; tile += nw) {
        TileIn<EQ, P, R> nxt;
        const int64_t t2 = tile + nw < t_stop ? tile + nw : tile;   // in bounds; unused at the end
        fetch_tile<EQ, P, R>(a, t2, lane, nxt);
        __builtin_amdgcn_sched_barrier(0);
        compute_tile<EQ, P, LIM, R>(a, tile, cur, lam, nlam, lane, smax, flags);
        cur = nxt;
      }
    }
  }
  publish(a.ctrl, a.parts, a.slot, smax, flags);
}

// Largest wave speed of the stored state (first time step after a write).
template <int EQ, int P, class R>
__global__ __launch_bounds__(256) void k_state_speed(const StepArgs<R> a) {
  constexpr int NC = ncomp<EQ>();
  double smax = 0.0;
  unsigned flags = 0u;
  const int64_t n = a.n_old;
  for (int64_t o = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; o < n; o += (int64_t)gridDim.x * blockDim.x) {
    double p[NC];
    R d[NC][P + 1];
    load_cell<EQ, P, R>(a.p_old, a.d_old, a.ld, o, 0, a, p, d);
    const double sp = stored_speed<EQ, P, R>(p, d, a.ph);
    smax = __builtin_fmax(smax, sp);
    if (!(sp == sp)) flags |= 1u;
#pragma unroll
    for (int c = 0; c < NC; ++c) {
      bool ok = __builtin_isfinite(p[c]);
#pragma unroll
      for (int k = 1; k <= P; ++k) ok = ok && finiteT(d[c][k]);
      if (!ok) flags |= 1u;
    }
  }
  // publish into the CURRENT slot: pass slot-1 so that publish's "next" is slot
  publish(a.ctrl, a.parts, a.slot == 0 ? 2 : a.slot - 1, smax, flags);
}

// ---------------------------------------------------------------------------
// Host-side dispatch over the compile-time variants.
// ---------------------------------------------------------------------------
template <int EQ, int P, bool LIM, class R>
static hipError_t launch_one(const StepArgs<R>& a, int pf, int blocks, int threads, hipStream_t s) {
  switch (pf) {
    case 0: hipLaunchKernelGGL((k_half_step<EQ, P, LIM, R, 0>), dim3(blocks), dim3(threads), 0, s, a); break;
    case 1: hipLaunchKernelGGL((k_half_step<EQ, P, LIM, R, 1>), dim3(blocks), dim3(threads), 0, s, a); break;
    case 2: hipLaunchKernelGGL((k_half_step<EQ, P, LIM, R, 2>), dim3(blocks), dim3(threads), 0, s, a); break;
    case 3: hipLaunchKernelGGL((k_half_step<EQ, P, LIM, R, 3>), dim3(blocks), dim3(threads), 0, s, a); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

template <int EQ, int P, class R>
static hipError_t launch_lim(const StepArgs<R>& a, bool lim, int pf, int blocks, int threads, hipStream_t s) {
  if (lim && P >= 1) return launch_one<EQ, P, true, R>(a, pf, blocks, threads, s);
  return launch_one<EQ, P, false, R>(a, pf, blocks, threads, s);
}

template <int EQ, class R>
static hipError_t launch_p(const StepArgs<R>& a, int P, bool lim, int pf, int blocks, int threads, hipStream_t s) {
  switch (P) {
    case 0: return launch_lim<EQ, 0, R>(a, false, pf, blocks, threads, s);
    case 1: return launch_lim<EQ, 1, R>(a, lim, pf, blocks, threads, s);
    case 2: return launch_lim<EQ, 2, R>(a, lim, pf, blocks, threads, s);
    case 3: return launch_lim<EQ, 3, R>(a, lim, pf, blocks, threads, s);
    case 4: return launch_lim<EQ, 4, R>(a, lim, pf, blocks, threads, s);
  }
  return hipErrorInvalidValue;
}

template <class R>
hipError_t launch_half_step(const StepArgs<R>& a, int eq, int P, bool lim, int pf, int blocks, int threads,
                            hipStream_t s) {
  switch (eq) {
    case kAdvection: return launch_p<kAdvection, R>(a, P, lim, pf, blocks, threads, s);
    case kBurgers: return launch_p<kBurgers, R>(a, P, lim, pf, blocks, threads, s);
    case kEuler: return launch_p<kEuler, R>(a, P, lim, pf, blocks, threads, s);
  }
  return hipErrorInvalidValue;
}

template <int EQ, class R>
static hipError_t launch_speed_p(const StepArgs<R>& a, int P, int blocks, hipStream_t s) {
  switch (P) {
    case 0: hipLaunchKernelGGL((k_state_speed<EQ, 0, R>), dim3(blocks), dim3(256), 0, s, a); break;
    case 1: hipLaunchKernelGGL((k_state_speed<EQ, 1, R>), dim3(blocks), dim3(256), 0, s, a); break;
    case 2: hipLaunchKernelGGL((k_state_speed<EQ, 2, R>), dim3(blocks), dim3(256), 0, s, a); break;
    case 3: hipLaunchKernelGGL((k_state_speed<EQ, 3, R>), dim3(blocks), dim3(256), 0, s, a); break;
    case 4: hipLaunchKernelGGL((k_state_speed<EQ, 4, R>), dim3(blocks), dim3(256), 0, s, a); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

template <class R>
hipError_t launch_state_speed(const StepArgs<R>& a, int eq, int P, int blocks, hipStream_t s) {
  switch (eq) {
    case kAdvection: return launch_speed_p<kAdvection, R>(a, P, blocks, s);
    case kBurgers: return launch_speed_p<kBurgers, R>(a, P, blocks, s);
    case kEuler: return launch_speed_p<kEuler, R>(a, P, blocks, s);
  }
  return hipErrorInvalidValue;
}

template <class R>
hipError_t occupancy_half_step(int eq, int P, bool lim, int pf, int threads, int* blocks_per_cu) {
  // Queried for the heaviest variant that can run; the kernel is the same for
  // every equation except in register use, so ask for the exact one.
  const void* f = nullptr;
#define WCC_K(E, PP, L)                                                            \
  (pf == 3   ? reinterpret_cast<const void*>(&k_half_step<E, PP, L, R, 3>)             \
   : pf == 2 ? reinterpret_cast<const void*>(&k_half_step<E, PP, L, R, 2>)             \
   : pf == 1 ? reinterpret_cast<const void*>(&k_half_step<E, PP, L, R, 1>)             \
             : reinterpret_cast<const void*>(&k_half_step<E, PP, L, R, 0>))
#define WCC_PSWITCH(E)                                                            \
  switch (P) {                                                                    \
    case 0: f = WCC_K(E, 0, false); break;                                        \
    case 1: f = lim ? WCC_K(E, 1, true) : WCC_K(E, 1, false); break;              \
    case 2: f = lim ? WCC_K(E, 2, true) : WCC_K(E, 2, false); break;              \
    case 3: f = lim ? WCC_K(E, 3, true) : WCC_K(E, 3, false); break;              \
    case 4: f = lim ? WCC_K(E, 4, true) : WCC_K(E, 4, false); break;              \
  }
  if (eq == kAdvection) { WCC_PSWITCH(kAdvection) }
  else if (eq == kBurgers) { WCC_PSWITCH(kBurgers) }
  else { WCC_PSWITCH(kEuler) }
#undef WCC_PSWITCH
#undef WCC_K
  if (!f) return hipErrorInvalidValue;
  return hipOccupancyMaxActiveBlocksPerMultiprocessor(blocks_per_cu, f, threads, 0);
}

template hipError_t launch_half_step<double>(const StepArgs<double>&, int, int, bool, int, int, int, hipStream_t);
template hipError_t launch_half_step<float>(const StepArgs<float>&, int, int, bool, int, int, int, hipStream_t);
template hipError_t launch_state_speed<double>(const StepArgs<double>&, int, int, int, hipStream_t);
template hipError_t launch_state_speed<float>(const StepArgs<float>&, int, int, int, hipStream_t);
template hipError_t occupancy_half_step<double>(int, int, bool, int, int, int*);
template hipError_t occupancy_half_step<float>(int, int, bool, int, int, int*);

}  // namespace wcc
