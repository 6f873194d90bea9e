// wcc2d_kernels.hip -- the fused 2D half-step kernel for gfx950 (Section 3,
// Appendix B; the 2D Euler step of Section 4).
//
// Work decomposition:
//   * a wavefront owns an 8 x 8 tile of OLD cells (lane = 8*ly + lx) and
//     produces the 7 x 7 NEW cells whose four parents all lie in the tile;
//     every lane expands its own old cell in registers;
//   * the parents of the new cell at (lx, ly) are the old cells at lanes
//     l (lower-left), l+8 (upper-left), l+1 (lower-right), l+9 (upper-right):
//     their interface quantities arrive by wave shuffles, one component at a
//     time;
//   * blocks own contiguous ranges of tiles (row-major over the tile grid);
//   * the time step comes from the same device-side ring as the 1D kernels
//     (dt = cfl / smax with smax the largest s_x/dx + s_y/dy of the previous
//     step's new averages), reduced through 64 partial slots.
#include <hip/hip_runtime.h>

#include "wcc2d_cell.hpp"
#include "wcc2d_internal.hpp"
#include "wcc_tile.hpp"

namespace wcc2d {

// periodic index of an old cell; a tile reaches one cell before 0 and seven
// past its first cell, so one wrap suffices unless the mesh is narrower than 8
__device__ __forceinline__ int wrap(int i, int n) {
  if (n >= 8) {
    if (i < 0) return i + n;
    if (i >= n) return i - n;
    return i;
  }
  int r = i % n;
  return r < 0 ? r + n : r;
}

template <int EQ, int P, bool LIM>
__device__ __forceinline__ void run_tile2(const Step2Args& a, int tile, int tiles_x, double nlx, double nly,
                                          double hx, double hy, int lane, double& smax, unsigned& flags) {
  constexpr int NC = ncomp<EQ>(), ND = ndof(P), NV = nvert(P) > 0 ? nvert(P) : 1;
  const int tx = tile % tiles_x, ty = tile / tiles_x;
  const int lx = lane & 7, ly = lane >> 3;
  const int off = a.parity_old == 0 ? 0 : -1;
  const int i = wrap(7 * tx + lx + off, a.Nx), j = wrap(7 * ty + ly + off, a.Ny);
  const uint32_t cell = (uint32_t)(j * a.Nx + i);
  double q[NC][ND];
#pragma unroll
  for (int c = 0; c < NC; ++c)
#pragma unroll
    for (int d = 0; d < ND; ++d) q[c][d] = wcc::row_at(wcc::row_base(a.q_old + (int64_t)(c * ND + d) * a.plane), cell);
  Old2<EQ, P> o;
  old_cell2<EQ, P>(q, nlx, nly, a.ph, o);

  const int ni = 7 * tx + lx, nj = 7 * ty + ly;
  const bool mine = lx < 7 && ly < 7 && ni < a.Nx && nj < a.Ny;
  const uint32_t ncell = (uint32_t)(nj * a.Nx + ni);
  double ab[NC];
  if constexpr (EQ == kEuler && LIM && P >= 1) {
    // the characteristic limiter couples the components: form all four new
    // averages and derivatives first
    double D[4][P + 1][P + 1], vx[4][4];
#pragma unroll
    for (int c = 0; c < 4; ++c) {
      const double B_RD = __shfl(o.RD[c], lane + 8, 64), B_fD = __shfl(o.fD[c], lane + 8, 64),
                   B_gR = __shfl(o.gR[c], lane + 8, 64);
      const double C_LU = __shfl(o.LU[c], lane + 1, 64), C_fU = __shfl(o.fU[c], lane + 1, 64),
                   C_gL = __shfl(o.gL[c], lane + 1, 64);
      const double E_LD = __shfl(o.LD[c], lane + 9, 64), E_fD = __shfl(o.fD[c], lane + 9, 64),
                   E_gL = __shfl(o.gL[c], lane + 9, 64);
      double VB[NV], VC[NV], VE[NV];
#pragma unroll
      for (int d = 0; d < NV; ++d) {
        VB[d] = __shfl(o.V[c][d], lane + 8, 64);
        VC[d] = __shfl(o.V[c][d], lane + 1, 64);
        VE[d] = __shfl(o.V[c][d], lane + 9, 64);
      }
      const double h = 0.25 * (((o.RU[c] + B_RD) + C_LU) + E_LD);
      const double fx = (o.fU[c] - C_fU) + (B_fD - E_fD);
      const double gy = (o.gR[c] - B_gR) + (C_gL - E_gL);
      ab[c] = __builtin_fma(hy, gy, __builtin_fma(hx, fx, h));
      new_derivatives<P>(o.V[c], VB, VC, VE, D[c]);
      vx[c][0] = o.V[c][0];
      vx[c][1] = VC[0];
      vx[c][2] = VE[0];
      vx[c][3] = VB[0];
    }
    char_limit2d<P>(a.ph, a.dx, a.dy, ab, D, vx);
    if (mine) {
#pragma unroll
      for (int c = 0; c < 4; ++c) {
        const double pv = point_value<P>(ab[c], D[c]);
        bool ok = __builtin_isfinite(pv);
        wcc::row_store(wcc::row_base(a.q_new + (int64_t)(c * ND) * a.plane), ncell, pv);
#pragma unroll
        for (int n = 1; n <= P; ++n)
#pragma unroll
          for (int l = 0; l <= n; ++l) {
            const double x = D[c][n - l][l];
            ok = ok && __builtin_isfinite(x);
            wcc::row_store(wcc::row_base(a.q_new + (int64_t)(c * ND + dof(n - l, l)) * a.plane), ncell, x);
          }
        if (!ok) flags |= 1u;
      }
    }
  } else {
#pragma unroll
  for (int c = 0; c < NC; ++c) {
    // right / upper parents' halves of this component
    const double B_RD = __shfl(o.RD[c], lane + 8, 64), B_fD = __shfl(o.fD[c], lane + 8, 64),
                 B_gR = __shfl(o.gR[c], lane + 8, 64);
    const double C_LU = __shfl(o.LU[c], lane + 1, 64), C_fU = __shfl(o.fU[c], lane + 1, 64),
                 C_gL = __shfl(o.gL[c], lane + 1, 64);
    const double E_LD = __shfl(o.LD[c], lane + 9, 64), E_fD = __shfl(o.fD[c], lane + 9, 64),
                 E_gL = __shfl(o.gL[c], lane + 9, 64);
    double VB[NV], VC[NV], VE[NV];
#pragma unroll
    for (int d = 0; d < NV; ++d) {
      VB[d] = __shfl(o.V[c][d], lane + 8, 64);
      VC[d] = __shfl(o.V[c][d], lane + 1, 64);
      VE[d] = __shfl(o.V[c][d], lane + 9, 64);
    }
    // Eq. 2DIntegral
    const double h = 0.25 * (((o.RU[c] + B_RD) + C_LU) + E_LD);
    const double fx = (o.fU[c] - C_fU) + (B_fD - E_fD);
    const double gy = (o.gR[c] - B_gR) + (C_gL - E_gL);
    const double abar = __builtin_fma(hy, gy, __builtin_fma(hx, fx, h));
    ab[c] = abar;
    double D[P + 1][P + 1];
    if constexpr (P >= 1) new_derivatives<P>(o.V[c], VB, VC, VE, D);
    if constexpr (LIM && P >= 1) limit2d<P>(a.ph.eps, abar, D, o.V[c][0], VC[0], VE[0], VB[0]);
    const double pv = point_value<P>(abar, D);
    if (mine) {
      bool ok = __builtin_isfinite(pv);
      wcc::row_store(wcc::row_base(a.q_new + (int64_t)(c * ND) * a.plane), ncell, pv);
#pragma unroll
      for (int n = 1; n <= P; ++n)
#pragma unroll
        for (int l = 0; l <= n; ++l) {
          const double x = D[n - l][l];
          ok = ok && __builtin_isfinite(x);
          wcc::row_store(wcc::row_base(a.q_new + (int64_t)(c * ND + dof(n - l, l)) * a.plane), ncell, x);
        }
      if (!ok) flags |= 1u;
    }
  }
  }
  if (mine) {
    const double sr = speed_rate<EQ>(ab, a.ph, a.idx, a.idy, flags);
    if (!__builtin_isfinite(sr)) flags |= 1u;
    smax = __builtin_fmax(smax, sr);
  }
}

template <int EQ, int P, bool LIM>
__global__ __launch_bounds__(256) void k2d_half_step(const Step2Args a) {
  const int lane = threadIdx.x & 63, wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6),
            nw = blockDim.x >> 6;
  const int tiles_x = (a.Nx + 6) / 7, tiles_y = (a.Ny + 6) / 7;
  const int tiles = tiles_x * tiles_y;
  const int per_block = (tiles + (int)gridDim.x - 1) / (int)gridDim.x;
  const int t_begin = (int)blockIdx.x * per_block;
  const int t_stop = t_begin + per_block < tiles ? t_begin + per_block : tiles;
  double dt;
  // dx = 1: the ring forms dt = (cfl * 1) / smax, smax being a rate (1/time)
  if (!wcc::step_time(a.ctrl, a.parts, a.slot, 1.0, a.dt_fixed, blockIdx.x == 0 && threadIdx.x < 64, dt)) return;
  const double lamx = dt / a.dx, lamy = dt / a.dy;
  const double nlx = -lamx, nly = -lamy, hx = 0.5 * lamx, hy = 0.5 * lamy;
  double smax = 0.0;
  unsigned flags = 0u;
  for (int tile = t_begin + wave; tile < t_stop; tile += nw)
    run_tile2<EQ, P, LIM>(a, tile, tiles_x, nlx, nly, hx, hy, lane, smax, flags);
  wcc::publish(a.ctrl, a.parts, a.slot, smax, flags);
}

// Largest wave-speed rate of the stored state (first time step after a write).
template <int EQ, int P>
__global__ __launch_bounds__(256) void k2d_state_speed(const Step2Args a) {
  constexpr int NC = ncomp<EQ>(), ND = ndof(P);
  double smax = 0.0;
  unsigned flags = 0u;
  const int64_t n = (int64_t)a.Nx * a.Ny;
  for (int64_t o = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; o < n; o += (int64_t)gridDim.x * blockDim.x) {
    double ab[NC];
    bool ok = true;
#pragma unroll
    for (int c = 0; c < NC; ++c) {
      double s = a.q_old[(int64_t)(c * ND) * a.plane + o];
      ok = ok && __builtin_isfinite(s);
#pragma unroll
      for (int nn = 1; nn <= P; ++nn)
#pragma unroll
        for (int l = 0; l <= nn; ++l) {
          const int k = nn - l;
          const double x = a.q_old[(int64_t)(c * ND + dof(k, l)) * a.plane + o];
          ok = ok && __builtin_isfinite(x);
          if (nn >= 2 && k % 2 == 0 && l % 2 == 0) s = __builtin_fma(-nqa(k, l), x, s);
        }
      ab[c] = s;
    }
    if (!ok) flags |= 1u;
    const double sr = speed_rate<EQ>(ab, a.ph, a.idx, a.idy, flags);
    smax = __builtin_fmax(smax, sr);
  }
  wcc::publish(a.ctrl, a.parts, a.slot == 0 ? 2 : a.slot - 1, smax, flags);
}

template <int EQ, int P>
static hipError_t launch_ep(const Step2Args& a, bool lim, int blocks, int threads, hipStream_t s) {
  if (lim)
    hipLaunchKernelGGL((k2d_half_step<EQ, P, true>), dim3(blocks), dim3(threads), 0, s, a);
  else
    hipLaunchKernelGGL((k2d_half_step<EQ, P, false>), dim3(blocks), dim3(threads), 0, s, a);
  return hipGetLastError();
}

template <int EQ>
static hipError_t launch_e(const Step2Args& a, int P, bool lim, int blocks, int threads, hipStream_t s) {
  switch (P) {
    case 0: return launch_ep<EQ, 0>(a, lim, blocks, threads, s);
    case 1: return launch_ep<EQ, 1>(a, lim, blocks, threads, s);
    case 2: return launch_ep<EQ, 2>(a, lim, blocks, threads, s);
    case 3: return launch_ep<EQ, 3>(a, lim, blocks, threads, s);
  }
  return hipErrorInvalidValue;
}

hipError_t launch_half_step2(const Step2Args& a, int eq, int P, bool lim, int blocks, int threads, hipStream_t s) {
  switch (eq) {
    case kAdvection: return launch_e<kAdvection>(a, P, lim, blocks, threads, s);
    case kBurgers: return launch_e<kBurgers>(a, P, lim, blocks, threads, s);
    case kEuler: return launch_e<kEuler>(a, P, lim, blocks, threads, s);
  }
  return hipErrorInvalidValue;
}

template <int EQ>
static hipError_t speed_e(const Step2Args& a, int P, int blocks, hipStream_t s) {
  switch (P) {
    case 0: hipLaunchKernelGGL((k2d_state_speed<EQ, 0>), dim3(blocks), dim3(256), 0, s, a); break;
    case 1: hipLaunchKernelGGL((k2d_state_speed<EQ, 1>), dim3(blocks), dim3(256), 0, s, a); break;
    case 2: hipLaunchKernelGGL((k2d_state_speed<EQ, 2>), dim3(blocks), dim3(256), 0, s, a); break;
    case 3: hipLaunchKernelGGL((k2d_state_speed<EQ, 3>), dim3(blocks), dim3(256), 0, s, a); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

hipError_t launch_state_speed2(const Step2Args& a, int eq, int P, int blocks, hipStream_t s) {
  switch (eq) {
    case kAdvection: return speed_e<kAdvection>(a, P, blocks, s);
    case kBurgers: return speed_e<kBurgers>(a, P, blocks, s);
    case kEuler: return speed_e<kEuler>(a, P, blocks, s);
  }
  return hipErrorInvalidValue;
}

template <int EQ, int P>
static hipError_t occ_ep(bool lim, int threads, int* per_cu) {
  if (lim)
    return hipOccupancyMaxActiveBlocksPerMultiprocessor(per_cu, k2d_half_step<EQ, P, true>, threads, 0);
  return hipOccupancyMaxActiveBlocksPerMultiprocessor(per_cu, k2d_half_step<EQ, P, false>, threads, 0);
}

template <int EQ>
static hipError_t occ_e(int P, bool lim, int threads, int* per_cu) {
  switch (P) {
    case 0: return occ_ep<EQ, 0>(lim, threads, per_cu);
    case 1: return occ_ep<EQ, 1>(lim, threads, per_cu);
    case 2: return occ_ep<EQ, 2>(lim, threads, per_cu);
    case 3: return occ_ep<EQ, 3>(lim, threads, per_cu);
  }
  return hipErrorInvalidValue;
}

hipError_t occupancy_half_step2(int eq, int P, bool lim, int threads, int* per_cu) {
  switch (eq) {
    case kAdvection: return occ_e<kAdvection>(P, lim, threads, per_cu);
    case kBurgers: return occ_e<kBurgers>(P, lim, threads, per_cu);
    case kEuler: return occ_e<kEuler>(P, lim, threads, per_cu);
  }
  return hipErrorInvalidValue;
}

}  // namespace wcc2d
