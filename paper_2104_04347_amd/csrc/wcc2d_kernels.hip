// wcc2d_kernels.hip -- the fused 2D half-step kernel for gfx950 (Section 3,
// Appendix B; the 2D Euler step of Section 4).
//
// Two work decompositions with identical results (the launch variant):
// 8 x 8 wave tiles exchanged by shuffles, and 64-column strips walked row by
// row with a one-row carry in LDS, with or without prefetch of the next row
// (described at each kernel).  The time step comes from the same device-side
// ring as the 1D kernels (dt = cfl / smax with smax the largest
// s_x/dx + s_y/dy of the previous step's new averages), reduced through 64
// partial slots.
#include <hip/hip_runtime.h>

#include "wcc2d_cell.hpp"
#include "wcc2d_internal.hpp"
#include "wcc_tile.hpp"

namespace wcc2d {

// periodic index of an old cell; a tile or strip reaches one cell before 0
// and at most 63 past its first cell, so one wrap suffices unless the mesh is
// narrower than 64
__device__ __forceinline__ int wrap(int i, int n) {
  if (n >= 64) {
    if (i < 0) return i + n;
    if (i >= n) return i - n;
    return i;
  }
  int r = i % n;
  return r < 0 ? r + n : r;
}

// Old-mesh index of a parent: wrapped (periodic) or clamped to the edge cell
// (transmissive ghosts are copies of the adjacent cell, Section 3.1 meshes).
__device__ __forceinline__ int map_idx(int i, int n, int periodic) {
  if (periodic) return wrap(i, n);
  return i < 0 ? 0 : (i >= n ? n - 1 : i);
}

// One component's parent data at a lane, as the new cell uses it: the
// quarter-average sum h and the flux differences fx, gy of Eq. 2DIntegral
// (grouped per pair of opposite half-edges, so that data uniform in the
// transverse direction cancel exactly) and the vertex values of the four
// parents, A lower-left, B upper-left, C lower-right, E upper-right.
template <int P>
struct Par2 {
  static constexpr int NV = nvert(P) > 0 ? nvert(P) : 1;
  double h, fx, gy;
  double VA[NV], VB[NV], VC[NV], VE[NV];
};

template <int P>
__device__ __forceinline__ void combine(Par2<P>& g, double A_RU, double B_RD, double C_LU, double E_LD, double A_fU,
                                        double C_fU, double B_fD, double E_fD, double A_gR, double B_gR,
                                        double C_gL, double E_gL) {
  g.h = 0.25 * (((A_RU + B_RD) + C_LU) + E_LD);
  g.fx = (A_fU - C_fU) + (B_fD - E_fD);
  g.gy = (A_gR - B_gR) + (C_gL - E_gL);
}

// ---- buffer addressing of the state (row-marching kernels) -----------------
// A row kernel loads and stores nc * ndof planes per mesh row (40 for Euler at
// P = 3).  With a 64-bit base pointer per plane the row loop needs a scalar
// register pair per plane for the loads and another for the stores -- more
// than the scalar register file holds, so the spilled pointers are reloaded
// from vector lanes on every row.  Buffer instructions take one resource per
// state buffer, a per-lane 32-bit offset (the cell and the component's group
// of planes) and a scalar 32-bit offset (the plane of the degree of freedom
// within the group): ndof - 1 scalar offsets, shared by loads and stores.
// Every offset is 32-bit, so this form serves state buffers below 2 GiB
// (`buffer_form`); larger states take the pointer form.
typedef unsigned int u32x2 __attribute__((__vector_size__(2 * sizeof(unsigned int))));

__host__ __device__ constexpr bool buffer_form(int64_t doubles_per_buffer) {
  return doubles_per_buffer * 8 < ((int64_t)1 << 31);
}

__device__ __forceinline__ __amdgpu_buffer_rsrc_t state_rsrc(const double* p) {
  // raw buffer (stride 0) with 2^31 - 1 bytes of range; word 3 as for
  // untyped dword accesses on gfx9-family parts
  return __builtin_amdgcn_make_buffer_rsrc(const_cast<double*>(p), (short)0, 0x7fffffff, 0x00020000);
}

// Per-lane byte offset of the first plane of a group at `cell`, kept opaque so
// that the compiler does not fold the uniform part into one scalar offset per
// plane again.
__device__ __forceinline__ uint32_t group_offset(uint32_t cell, int group, uint32_t plane_bytes) {
  uint32_t v = cell * 8u + (uint32_t)group * plane_bytes;
  asm("" : "+v"(v));
  return v;
}

__device__ __forceinline__ double buf_load(__amdgpu_buffer_rsrc_t r, uint32_t voff, uint32_t soff) {
  return __builtin_bit_cast(double, __builtin_amdgcn_raw_buffer_load_b64(r, (int)voff, (int)soff, 0));
}

__device__ __forceinline__ void buf_store(__amdgpu_buffer_rsrc_t r, uint32_t voff, uint32_t soff, double x) {
  __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(u32x2, x), r, (int)voff, (int)soff, 0);
}

// Store the new cell's DOFs of component c (point value, then u_{kx,ly} in
// DOF order) and flag non-finite values.
template <int EQ, int P, bool BUF>
__device__ __forceinline__ void store_cell(const Step2Args& a, int c, uint32_t ncell, double pv,
                                           const double (&D)[P + 1][P + 1], unsigned& flags) {
  constexpr int ND = ndof(P);
  bool ok = __builtin_isfinite(pv);
  if constexpr (BUF) {
    const __amdgpu_buffer_rsrc_t r = state_rsrc(a.q_new);
    const uint32_t pb = (uint32_t)a.plane * 8u, vo = group_offset(ncell, c * ND, pb);
    buf_store(r, vo, 0u, pv);
#pragma unroll
    for (int n = 1; n <= P; ++n)
#pragma unroll
      for (int l = 0; l <= n; ++l) {
        const double x = D[n - l][l];
        ok = ok && __builtin_isfinite(x);
        buf_store(r, vo, (uint32_t)dof(n - l, l) * pb, x);
      }
  } else {
    wcc::row_store(wcc::row_base(a.q_new + (int64_t)(c * ND) * a.plane), ncell, pv);
#pragma unroll
    for (int n = 1; n <= P; ++n)
#pragma unroll
      for (int l = 0; l <= n; ++l) {
        const double x = D[n - l][l];
        ok = ok && __builtin_isfinite(x);
        wcc::row_store(wcc::row_base(a.q_new + (int64_t)(c * ND + dof(n - l, l)) * a.plane), ncell, x);
      }
  }
  if (!ok) flags |= 1u;
}

// New cell of this lane from its parents' data (gather(c, g) fills Par2 for
// component c): average (Eq. 2DIntegral), derivatives (Eq. 2DDerivatives),
// limiter (Section 3.2; characteristic fields for Euler, Section 4), point
// value, store (store(c, point value, D, flags)), wave-speed rate.
template <int EQ, int P, bool LIM, class Gather, class Store>
__device__ __forceinline__ void new_cell2(const Step2Args& a, Gather&& gather, Store&& store, bool mine, double hx,
                                          double hy, double& smax, unsigned& flags) {
  constexpr int NC = ncomp<EQ>();
  double ab[NC];
  if constexpr (EQ == kEuler && LIM && P >= 1) {
    // the characteristic limiter couples the components: form all four new
    // averages and derivatives first
    double D[4][P + 1][P + 1], vx[4][4];
#pragma unroll
    for (int c = 0; c < 4; ++c) {
      Par2<P> g;
      gather(c, g);
      ab[c] = __builtin_fma(hy, g.gy, __builtin_fma(hx, g.fx, g.h));
      new_derivatives<P>(g.VA, g.VB, g.VC, g.VE, D[c]);
      vx[c][0] = g.VA[0];
      vx[c][1] = g.VC[0];
      vx[c][2] = g.VE[0];
      vx[c][3] = g.VB[0];
    }
    char_limit2d<P>(a.ph, a.dx, a.dy, ab, D, vx);
    if (mine) {
#pragma unroll
      for (int c = 0; c < 4; ++c) store(c, point_value<P>(ab[c], D[c]), D[c], flags);
    }
  } else {
#pragma unroll
    for (int c = 0; c < NC; ++c) {
      Par2<P> g;
      gather(c, g);
      const double abar = __builtin_fma(hy, g.gy, __builtin_fma(hx, g.fx, g.h));
      ab[c] = abar;
      double D[P + 1][P + 1];
      if constexpr (P >= 1) new_derivatives<P>(g.VA, g.VB, g.VC, g.VE, D);
      if constexpr (LIM && P >= 1) limit2d<P>(a.ph.eps, abar, D, g.VA[0], g.VC[0], g.VE[0], g.VB[0]);
      const double pv = point_value<P>(abar, D);
      if (mine) store(c, pv, D, flags);
    }
  }
  if (mine) {
    const double sr = speed_rate<EQ>(ab, a.ph, a.idx, a.idy, flags);
    if (!__builtin_isfinite(sr)) flags |= 1u;
    smax = __builtin_fmax(smax, sr);
  }
}

// Load the state of the old cell (i, j) of this lane.
template <int EQ, int P, bool BUF = false>
__device__ __forceinline__ void load_old(const Step2Args& a, int i, int j, double (&q)[ncomp<EQ>()][ndof(P)]) {
  constexpr int NC = ncomp<EQ>(), ND = ndof(P);
  const uint32_t cell = (uint32_t)(j * a.nxo + i);
  if constexpr (BUF) {
    const __amdgpu_buffer_rsrc_t r = state_rsrc(a.q_old);
    const uint32_t pb = (uint32_t)a.plane * 8u;
#pragma unroll
    for (int c = 0; c < NC; ++c) {
      const uint32_t vo = group_offset(cell, c * ND, pb);
#pragma unroll
      for (int d = 0; d < ND; ++d) q[c][d] = buf_load(r, vo, (uint32_t)d * pb);
    }
  } else {
#pragma unroll
    for (int c = 0; c < NC; ++c)
#pragma unroll
      for (int d = 0; d < ND; ++d)
        q[c][d] = wcc::row_at(wcc::row_base(a.q_old + (int64_t)(c * ND + d) * a.plane), cell);
  }
}

// Load and expand the old cell (i, j) of this lane.
template <int EQ, int P, bool BUF = false>
__device__ __forceinline__ void old_of(const Step2Args& a, int i, int j, double nlx, double nly, Old2<EQ, P>& o) {
  double q[ncomp<EQ>()][ndof(P)];
  load_old<EQ, P, BUF>(a, i, j, q);
  old_cell2<EQ, P>(q, nlx, nly, a.ph, o);
}

// ---- variant 0: 8 x 8 wave tiles ------------------------------------------
// A wavefront owns an 8 x 8 tile of old cells (lane = 8*ly + lx) and
// produces the 7 x 7 new cells whose four parents lie in the tile; the
// parents of the new cell at (lx, ly) are the old cells at lanes l (A),
// l+8 (B), l+1 (C), l+9 (E), exchanged by wave shuffles.  Blocks own
// contiguous ranges of tiles (row-major over the tile grid).
template <int EQ, int P, bool LIM>
__device__ __forceinline__ void run_tile2(const Step2Args& a, int tile, int tiles_x, double nlx, double nly,
                                          double hx, double hy, int lane, double& smax, unsigned& flags) {
  constexpr int NV = Par2<P>::NV;
  const int tx = tile % tiles_x, ty = tile / tiles_x;
  const int lx = lane & 7, ly = lane >> 3;
  const int off = a.parity_old == 0 ? 0 : -1;
  Old2<EQ, P> o;
  old_of<EQ, P>(a, map_idx(7 * tx + lx + off, a.nxo, a.periodic_x), map_idx(7 * ty + ly + off, a.nyo, a.periodic_y), nlx,
                nly, o);
  const int ni = 7 * tx + lx, nj = 7 * ty + ly;
  const bool mine = lx < 7 && ly < 7 && ni < a.nxn && nj < a.nyn;
  auto gather = [&](int c, Par2<P>& g) {
    const double B_RD = __shfl(o.RD[c], lane + 8, 64), B_fD = __shfl(o.fD[c], lane + 8, 64),
                 B_gR = __shfl(o.gR[c], lane + 8, 64);
    const double C_LU = __shfl(o.LU[c], lane + 1, 64), C_fU = __shfl(o.fU[c], lane + 1, 64),
                 C_gL = __shfl(o.gL[c], lane + 1, 64);
    const double E_LD = __shfl(o.LD[c], lane + 9, 64), E_fD = __shfl(o.fD[c], lane + 9, 64),
                 E_gL = __shfl(o.gL[c], lane + 9, 64);
#pragma unroll
    for (int d = 0; d < NV; ++d) {
      g.VA[d] = o.V[c][d];
      g.VB[d] = __shfl(o.V[c][d], lane + 8, 64);
      g.VC[d] = __shfl(o.V[c][d], lane + 1, 64);
      g.VE[d] = __shfl(o.V[c][d], lane + 9, 64);
    }
    combine<P>(g, o.RU[c], B_RD, C_LU, E_LD, o.fU[c], C_fU, B_fD, E_fD, o.gR[c], B_gR, C_gL, E_gL);
  };
  const uint32_t ncell = (uint32_t)(nj * a.nxn + ni);
  auto store = [&](int c, double pv, const double (&D)[P + 1][P + 1], unsigned& fl) {
    store_cell<EQ, P, false>(a, c, ncell, pv, D, fl);
  };
  new_cell2<EQ, P, LIM>(a, gather, store, mine, hx, hy, smax, flags);
}

template <int EQ, int P, bool LIM>
__global__ __launch_bounds__(256) void k2d_half_step(const Step2Args a) {
  const int lane = threadIdx.x & 63, wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6),
            nw = blockDim.x >> 6;
  const int tiles_x = (a.nxn + 6) / 7, tiles_y = (a.nyn + 6) / 7;
  const int tiles = tiles_x * tiles_y;
  const int per_block = (tiles + (int)gridDim.x - 1) / (int)gridDim.x;
  const int t_begin = (int)blockIdx.x * per_block;
  const int t_stop = t_begin + per_block < tiles ? t_begin + per_block : tiles;
  double dt;
  // dx = 1: the ring forms dt = (cfl * 1) / smax, smax being a rate (1/time)
  if (!wcc::step_time(a.ctrl, a.parts, a.slot, 1.0, a.dt_fixed, blockIdx.x == 0 && threadIdx.x < 64, dt)) return;
  const double lamx = wcc::div_rn(dt, a.dx), lamy = wcc::div_rn(dt, a.dy);
  const double nlx = -lamx, nly = -lamy, hx = 0.5 * lamx, hy = 0.5 * lamy;
  double smax = 0.0;
  unsigned flags = 0u;
  for (int tile = t_begin + wave; tile < t_stop; tile += nw)
    run_tile2<EQ, P, LIM>(a, tile, tiles_x, nlx, nly, hx, hy, lane, smax, flags);
  wcc::publish(a.ctrl, a.parts, a.slot, smax, flags);
}

// ---- variant 1: row marching -----------------------------------------------
// The mesh is cut into strips of 64 old columns (63 new columns each; the
// 64th old column holds the right parents of the 63rd new one).  A wavefront
// walks a contiguous run of (strip, row) units, strip-major, one mesh row at
// a time, lane = column in the strip.  At unit (strip, r) it expands the old
// row above new row r: the lane's old cell is the upper-left parent B of its
// new cell and the next lane's the upper-right parent E (DPP shift by one
// lane); the lower parents A and C are the previous row's expansion, kept by
// each lane in its own LDS slot (C again from the next lane).  Every old cell
// is expanded once per strip -- plus one extra row where a run starts or
// enters a new strip -- and every row is loaded and stored 64 cells wide.
template <int EQ, int P>
struct RowCarry {
  static constexpr int NQ = 5 + nvert(P);   // RU, LU, fU, gR, gL, V[0..nvert)
  double v[ncomp<EQ>()][NQ][64];
};

template <int EQ, int P>
__device__ __forceinline__ void put_carry(RowCarry<EQ, P>& carry, int c, int lane, const Old2<EQ, P>& o) {
  carry.v[c][0][lane] = o.RU[c];
  carry.v[c][1][lane] = o.LU[c];
  carry.v[c][2][lane] = o.fU[c];
  carry.v[c][3][lane] = o.gR[c];
  carry.v[c][4][lane] = o.gL[c];
#pragma unroll
  for (int d = 0; d < nvert(P); ++d) carry.v[c][5 + d][lane] = o.V[c][d];
}

// PF: load the next unit's upper row before expanding the current one (one
// row of state in flight per wave, at the cost of its registers).
// BANDS: band-major work items.  A strip's 64-cell row pieces start every 63
// cells, so each piece shares its edge cache lines with the neighbouring
// strips' pieces; with BANDS the waves of a block take neighbouring strips
// over the same band of rows (they load the shared lines at about the same
// time, through the same L2), and the blocks of one XCD (the hardware places
// block b on XCD b mod 8) take consecutive items.  Each wave owns one strip
// over one band of rows: no run crosses a strip.  Without BANDS (or with
// fewer waves than strips) the waves split the strip-major (strip, row)
// units evenly.  The arithmetic of every unit is the same either way.
// BUF: buffer addressing of the state (see buffer_form).
template <int EQ, int P, bool LIM, bool PF, bool BANDS, bool BUF>
__global__ __launch_bounds__(256) void k2d_half_step_rows(const Step2Args a) {
  constexpr int NC = ncomp<EQ>(), NV = nvert(P), ND = ndof(P);
  __shared__ RowCarry<EQ, P> carry_all[4];
  const int lane = threadIdx.x & 63, wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6),
            nw = blockDim.x >> 6;
  RowCarry<EQ, P>& carry = carry_all[wave];
  const int strips = (a.nxn + 62) / 63, rows = a.nyn;
  const int64_t units = (int64_t)strips * rows, waves = (int64_t)gridDim.x * nw;
  const int64_t gw = (int64_t)blockIdx.x * nw + wave;
  int u_begin = (int)(gw * units / waves), u_end = (int)((gw + 1) * units / waves);
  if (BANDS && waves >= strips) {
    const int G = (int)gridDim.x;
    const int lb = (G & 7) == 0 ? (int)(blockIdx.x & 7) * (G >> 3) + (int)(blockIdx.x >> 3) : (int)blockIdx.x;
    const int64_t item = (int64_t)lb * nw + wave;
    const int bands = (int)(waves / strips);
    u_begin = u_end = 0;
    if (item < (int64_t)bands * strips) {
      const int band = (int)(item / strips), sx = (int)(item - (int64_t)band * strips);
      u_begin = sx * rows + (int)((int64_t)band * rows / bands);
      u_end = sx * rows + (int)((int64_t)(band + 1) * rows / bands);
    }
  }
  double dt;
  if (!wcc::step_time(a.ctrl, a.parts, a.slot, 1.0, a.dt_fixed, blockIdx.x == 0 && threadIdx.x < 64, dt)) return;
  const double lamx = wcc::div_rn(dt, a.dx), lamy = wcc::div_rn(dt, a.dy);
  const double nlx = -lamx, nly = -lamy, hx = 0.5 * lamx, hy = 0.5 * lamy;
  const int off = a.parity_old == 0 ? 0 : -1;
  double smax = 0.0;
  unsigned flags = 0u;
  double qn[NC][ND];
  if (PF && u_begin < u_end) {
    const int sx = u_begin / rows, r = u_begin - sx * rows;
    load_old<EQ, P, BUF>(a, map_idx(63 * sx + lane + off, a.nxo, a.periodic_x), map_idx(r + 1 + off, a.nyo, a.periodic_y),
                         qn);
  }
  for (int u = u_begin; u < u_end; ++u) {
    const int sx = u / rows, r = u - sx * rows;
    const int i = map_idx(63 * sx + lane + off, a.nxo, a.periodic_x);
    if (u == u_begin || r == 0) {
      // lower parents of new row r: the old row below, expanded afresh
      Old2<EQ, P> o;
      old_of<EQ, P, BUF>(a, i, map_idx(r + off, a.nyo, a.periodic_y), nlx, nly, o);
#pragma unroll
      for (int c = 0; c < NC; ++c) put_carry<EQ, P>(carry, c, lane, o);
    }
    double q[NC][ND];
    if constexpr (PF) {
#pragma unroll
      for (int c = 0; c < NC; ++c)
#pragma unroll
        for (int d = 0; d < ND; ++d) q[c][d] = qn[c][d];
      if (u + 1 < u_end) {
        const int sx2 = (u + 1) / rows, r2 = u + 1 - sx2 * rows;
        load_old<EQ, P, BUF>(a, map_idx(63 * sx2 + lane + off, a.nxo, a.periodic_x),
                             map_idx(r2 + 1 + off, a.nyo, a.periodic_y), qn);
      }
      __builtin_amdgcn_sched_barrier(0);
    } else {
      load_old<EQ, P, BUF>(a, i, map_idx(r + 1 + off, a.nyo, a.periodic_y), q);
    }
    Old2<EQ, P> o;
    old_cell2<EQ, P>(q, nlx, nly, a.ph, o);
    const int ni = 63 * sx + lane;
    const bool mine = lane < 63 && ni < a.nxn;
    auto gather = [&](int c, Par2<P>& g) {
      // the lane's own slot: read the row below, then leave this row for the
      // next unit
      const double A_RU = carry.v[c][0][lane], A_LU = carry.v[c][1][lane], A_fU = carry.v[c][2][lane],
                   A_gR = carry.v[c][3][lane], A_gL = carry.v[c][4][lane];
#pragma unroll
      for (int d = 0; d < NV; ++d) g.VA[d] = carry.v[c][5 + d][lane];
      put_carry<EQ, P>(carry, c, lane, o);
      const double C_LU = wcc::dpp_from_next(A_LU), C_fU = wcc::dpp_from_next(A_fU),
                   C_gL = wcc::dpp_from_next(A_gL);
      const double E_LD = wcc::dpp_from_next(o.LD[c]), E_fD = wcc::dpp_from_next(o.fD[c]),
                   E_gL = wcc::dpp_from_next(o.gL[c]);
#pragma unroll
      for (int d = 0; d < NV; ++d) {
        g.VB[d] = o.V[c][d];
        g.VC[d] = wcc::dpp_from_next(g.VA[d]);
        g.VE[d] = wcc::dpp_from_next(o.V[c][d]);
      }
      combine<P>(g, A_RU, o.RD[c], C_LU, E_LD, A_fU, C_fU, o.fD[c], E_fD, A_gR, o.gR[c], C_gL, E_gL);
    };
    const uint32_t ncell = (uint32_t)(r * a.nxn + ni);
    auto store = [&](int c, double pv, const double (&D)[P + 1][P + 1], unsigned& fl) {
      store_cell<EQ, P, BUF>(a, c, ncell, pv, D, fl);
    };
    new_cell2<EQ, P, LIM>(a, gather, store, mine, hx, hy, smax, flags);
  }
  wcc::publish(a.ctrl, a.parts, a.slot, smax, flags);
}

// Largest wave-speed rate of the stored state (first time step after a write).
template <int EQ, int P>
__global__ __launch_bounds__(256) void k2d_state_speed(const Step2Args a) {
  constexpr int NC = ncomp<EQ>(), ND = ndof(P);
  double smax = 0.0;
  unsigned flags = 0u;
  const int64_t n = (int64_t)a.nxo * a.nyo;
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

// Variants 2 and 3 take the buffer-addressed kernel when a state buffer is
// below 2 GiB; variant 1 and larger states the pointer form.
template <int EQ, int P, bool LIM>
static hipError_t launch_epl(const Step2Args& a, int variant, int blocks, int threads, hipStream_t s) {
  const bool buf = buffer_form((int64_t)ncomp<EQ>() * ndof(P) * a.plane);
  if (variant == 3 && buf)
    hipLaunchKernelGGL((k2d_half_step_rows<EQ, P, LIM, true, true, true>), dim3(blocks), dim3(threads), 0, s, a);
  else if (variant == 3)
    hipLaunchKernelGGL((k2d_half_step_rows<EQ, P, LIM, true, true, false>), dim3(blocks), dim3(threads), 0, s, a);
  else if (variant == 2 && buf)
    hipLaunchKernelGGL((k2d_half_step_rows<EQ, P, LIM, true, false, true>), dim3(blocks), dim3(threads), 0, s, a);
  else if (variant == 2)
    hipLaunchKernelGGL((k2d_half_step_rows<EQ, P, LIM, true, false, false>), dim3(blocks), dim3(threads), 0, s, a);
  else if (variant == 1)
    hipLaunchKernelGGL((k2d_half_step_rows<EQ, P, LIM, false, false, false>), dim3(blocks), dim3(threads), 0, s, a);
  else
    hipLaunchKernelGGL((k2d_half_step<EQ, P, LIM>), dim3(blocks), dim3(threads), 0, s, a);
  return hipGetLastError();
}

template <int EQ, int P>
static hipError_t launch_ep(const Step2Args& a, bool lim, int variant, int blocks, int threads, hipStream_t s) {
  if (lim) return launch_epl<EQ, P, true>(a, variant, blocks, threads, s);
  return launch_epl<EQ, P, false>(a, variant, blocks, threads, s);
}

template <int EQ>
static hipError_t launch_e(const Step2Args& a, int P, bool lim, int variant, int blocks, int threads,
                           hipStream_t s) {
  switch (P) {
    case 0: return launch_ep<EQ, 0>(a, lim, variant, blocks, threads, s);
    case 1: return launch_ep<EQ, 1>(a, lim, variant, blocks, threads, s);
    case 2: return launch_ep<EQ, 2>(a, lim, variant, blocks, threads, s);
    case 3: return launch_ep<EQ, 3>(a, lim, variant, blocks, threads, s);
  }
  return hipErrorInvalidValue;
}

hipError_t launch_half_step2(const Step2Args& a, int eq, int P, bool lim, int variant, int blocks, int threads,
                             hipStream_t s) {
  switch (eq) {
    case kAdvection: return launch_e<kAdvection>(a, P, lim, variant, blocks, threads, s);
    case kBurgers: return launch_e<kBurgers>(a, P, lim, variant, blocks, threads, s);
    case kEuler: return launch_e<kEuler>(a, P, lim, variant, blocks, threads, s);
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

template <int EQ, int P, bool LIM>
static hipError_t occ_epl(int variant, int threads, int64_t plane, int* per_cu) {
  const bool buf = buffer_form((int64_t)ncomp<EQ>() * ndof(P) * plane);
  if (variant == 3 && buf)
    return hipOccupancyMaxActiveBlocksPerMultiprocessor(per_cu, k2d_half_step_rows<EQ, P, LIM, true, true, true>,
                                                        threads, 0);
  if (variant == 3)
    return hipOccupancyMaxActiveBlocksPerMultiprocessor(per_cu, k2d_half_step_rows<EQ, P, LIM, true, true, false>,
                                                        threads, 0);
  if (variant == 2 && buf)
    return hipOccupancyMaxActiveBlocksPerMultiprocessor(per_cu, k2d_half_step_rows<EQ, P, LIM, true, false, true>,
                                                        threads, 0);
  if (variant == 2)
    return hipOccupancyMaxActiveBlocksPerMultiprocessor(per_cu, k2d_half_step_rows<EQ, P, LIM, true, false, false>,
                                                        threads, 0);
  if (variant == 1)
    return hipOccupancyMaxActiveBlocksPerMultiprocessor(per_cu, k2d_half_step_rows<EQ, P, LIM, false, false, false>,
                                                        threads, 0);
  return hipOccupancyMaxActiveBlocksPerMultiprocessor(per_cu, k2d_half_step<EQ, P, LIM>, threads, 0);
}

template <int EQ, int P>
static hipError_t occ_ep(bool lim, int variant, int threads, int64_t plane, int* per_cu) {
  if (lim) return occ_epl<EQ, P, true>(variant, threads, plane, per_cu);
  return occ_epl<EQ, P, false>(variant, threads, plane, per_cu);
}

template <int EQ>
static hipError_t occ_e(int P, bool lim, int variant, int threads, int64_t plane, int* per_cu) {
  switch (P) {
    case 0: return occ_ep<EQ, 0>(lim, variant, threads, plane, per_cu);
    case 1: return occ_ep<EQ, 1>(lim, variant, threads, plane, per_cu);
    case 2: return occ_ep<EQ, 2>(lim, variant, threads, plane, per_cu);
    case 3: return occ_ep<EQ, 3>(lim, variant, threads, plane, per_cu);
  }
  return hipErrorInvalidValue;
}

hipError_t occupancy_half_step2(int eq, int P, bool lim, int variant, int threads, int64_t plane, int* per_cu) {
  switch (eq) {
    case kAdvection: return occ_e<kAdvection>(P, lim, variant, threads, plane, per_cu);
    case kBurgers: return occ_e<kBurgers>(P, lim, variant, threads, plane, per_cu);
    case kEuler: return occ_e<kEuler>(P, lim, variant, threads, plane, per_cu);
  }
  return hipErrorInvalidValue;
}

}  // namespace wcc2d
