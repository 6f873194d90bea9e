// wcc_tile.hpp -- wave-level building blocks shared by the single-instance and
// batched half-step kernels: lane exchange by DPP, wave/block reductions, the
// device-side time step, the body that turns one tile of 64 old cells into
// 63 new cells, and the LDS staging that stores new cells in whole 64-cell
// groups.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "wcc_cell.hpp"
#include "wcc_internal.hpp"

namespace wcc {

// wave_shl:1 -- lane i receives lane i+1; lane 63, which has no source lane,
// receives 0 (bound_ctrl), so the destination needs no initialising move.
__device__ __forceinline__ int dpp_from_next(int x) { return __builtin_amdgcn_update_dpp(0, x, 0x130, 0xF, 0xF, true); }
__device__ __forceinline__ float dpp_from_next(float x) {
  return __int_as_float(dpp_from_next(__float_as_int(x)));
}
__device__ __forceinline__ double dpp_from_next(double x) {
  const long long v = __double_as_longlong(x);
  const int lo = dpp_from_next((int)(v & 0xffffffffll));
  const int hi = dpp_from_next((int)(v >> 32));
  return __longlong_as_double(((long long)hi << 32) | (long long)(unsigned)lo);
}

__device__ __forceinline__ double wave_max(double v) {
#pragma unroll
  for (int o = 32; o >= 1; o >>= 1) v = __builtin_fmax(v, __shfl_xor(v, o));
  return v;
}
__device__ __forceinline__ unsigned wave_or(unsigned v) {
#pragma unroll
  for (int o = 32; o >= 1; o >>= 1) v |= (unsigned)__shfl_xor((int)v, o);
  return v;
}

// Time-step bookkeeping shared by the single and batched kernels.  Returns
// false when this launch must do nothing (end time reached or a flag raised
// by an earlier step); in that case the slot is propagated unchanged.  With
// `parts` (single-instance kernels) the wave speed of the previous step is
// the max of the 64 partial entries of the slot; the first wave of block 0
// (`leader_wave`) maintains the ring.  Called by every lane of every wave.
__device__ __forceinline__ bool step_time(Ctrl* ctrl, unsigned long long* parts, int slot, double dx,
                                          double dt_fixed, bool leader_wave, double& dt) {
  const int s1 = slot == 2 ? 0 : slot + 1;
  const int s2 = s1 == 2 ? 0 : s1 + 1;
  const int lane = threadIdx.x & 63;
  const double t = ctrl->t[slot];
  const unsigned flags_in = ctrl->flags[slot];
  bool done = flags_in != 0u;
  double tn;
  unsigned long long mine = 0ull;  // this lane's partial entry of the slot (parts mode)
  if (parts) mine = parts[(slot * kSmaxParts + lane) * kSmaxStride];
  if (dt_fixed > 0.0) {
    dt = dt_fixed;
    tn = t + dt;
  } else {
    const double smax = parts ? wave_max(__longlong_as_double((long long)mine))
                              : __longlong_as_double((long long)ctrl->smax[slot]);
    const double tend = ctrl->t_end;
    done = done || !(t < tend);
    dt = div_rn(ctrl->cfl * dx, smax);
    const double rem = tend - t;
    if (dt >= rem) {
      dt = rem;
      tn = tend;
    } else {
      tn = t + dt;
    }
  }
  if (leader_wave) {
    if (parts) {
      // Slot s1 was cleared by the previous launch (as its s2) and is being
      // raised by the other blocks' atomics now; only a finished run, where
      // no block publishes, carries the maximum forward.
      if (done) parts[(s1 * kSmaxParts + lane) * kSmaxStride] = mine;
      parts[(s2 * kSmaxParts + lane) * kSmaxStride] = 0ull;
    }
    if (lane == 0) {
      if (done) {
        ctrl->t[s1] = t;
        ctrl->smax[s1] = ctrl->smax[slot];
        ctrl->flags[s1] = flags_in;
      } else {
        ctrl->t[s1] = tn;
        ctrl->steps_done += 1;
      }
      ctrl->smax[s2] = 0ull;
      ctrl->flags[s2] = 0u;
    }
  }
  return !done;
}

// Per-block reduction of the wave speeds and flags, then one atomic each into
// the next slot, skipped when it cannot raise the stored maximum.  With
// `parts` the block's atomic goes to entry (block index mod 64).
__device__ __forceinline__ void publish(Ctrl* ctrl, unsigned long long* parts, int slot, double smax,
                                        unsigned flags) {
  __shared__ double red_s[16];
  __shared__ unsigned red_f[16];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6, nw = blockDim.x >> 6;
  smax = wave_max(smax);
  flags = wave_or(flags);
  if (lane == 0) {
    red_s[wave] = smax;
    red_f[wave] = flags;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    for (int w = 1; w < nw; ++w) {
      smax = __builtin_fmax(smax, red_s[w]);
      flags |= red_f[w];
    }
    const int s1 = slot == 2 ? 0 : slot + 1;
    const unsigned long long bits = (unsigned long long)__double_as_longlong(smax);
    unsigned long long* dst =
        parts ? &parts[(s1 * kSmaxParts + (int)(blockIdx.x % kSmaxParts)) * kSmaxStride] : &ctrl->smax[s1];
    if (bits > __hip_atomic_load(dst, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)) atomicMax(dst, bits);
    if (flags) atomicOr(&ctrl->flags[s1], flags);
  }
}

// Element i of a row: uniform base pointer plus a 32-bit byte offset, the
// form the global load/store instructions take with an SGPR base.
template <class T>
__device__ __forceinline__ T row_at(const T* base, uint32_t i) {
  return *reinterpret_cast<const T*>(reinterpret_cast<const char*>(base) + (uint32_t)(i * (uint32_t)sizeof(T)));
}
template <class T>
__device__ __forceinline__ void row_store(T* base, uint32_t i, T v) {
  *reinterpret_cast<T*>(reinterpret_cast<char*>(base) + (uint32_t)(i * (uint32_t)sizeof(T))) = v;
}

// Base pointer of one row, made opaque in a scalar register pair.  Without
// this the compiler folds the row offset (row x ld) into a 64-bit per-lane
// address, two vector instructions per load or store; with it every access
// is one instruction with an SGPR base and the lane's 32-bit offset.  The
// pointer must be uniform across the wavefront (it is: one wave handles one
// tile of one instance).
template <class T>
using global_ptr = __attribute__((address_space(1))) T*;

template <class T>
__device__ __forceinline__ global_ptr<T> row_base(T* p) {
  const uint64_t v = reinterpret_cast<uint64_t>(p);
  const uint32_t lo = __builtin_amdgcn_readfirstlane((uint32_t)v), hi = __builtin_amdgcn_readfirstlane((uint32_t)(v >> 32));
  global_ptr<T> g = (global_ptr<T>)reinterpret_cast<T*>(((uint64_t)hi << 32) | lo);
  asm("" : "+s"(g));
  return g;
}
template <class T>
__device__ __forceinline__ T row_at(global_ptr<const T> base, uint32_t i) {
  return *(global_ptr<const T>)((global_ptr<const char>)base + (uint32_t)(i * (uint32_t)sizeof(T)));
}
template <class T>
__device__ __forceinline__ void row_store(global_ptr<T> base, uint32_t i, T v) {
  *(global_ptr<T>)((global_ptr<char>)base + (uint32_t)(i * (uint32_t)sizeof(T))) = v;
}

// Load the old cell `o` (already mapped into [0, n_old)), or a Dirichlet ghost.
template <int EQ, int P, class R>
__device__ __forceinline__ void load_cell(const double* __restrict__ pv, const R* __restrict__ dv, int64_t ld,
                                          int64_t o, int ghost, const StepArgs<R>& a,
                                          double (&p)[ncomp<EQ>()], R (&d)[ncomp<EQ>()][P + 1]) {
  constexpr int NC = ncomp<EQ>();
#pragma unroll
  for (int c = 0; c < NC; ++c) {
    p[c] = pv[c * ld + o];
    d[c][0] = (R)0;
#pragma unroll
    for (int k = 1; k <= P; ++k) d[c][k] = dv[(c * P + (k - 1)) * ld + o];
  }
  if (ghost) {
    const double* g = a.ctrl->ghost[ghost - 1];
#pragma unroll
    for (int c = 0; c < NC; ++c) {
      p[c] = g[c];
#pragma unroll
      for (int k = 1; k <= P; ++k) d[c][k] = (R)0;
    }
  }
}

// Map the lane's old-cell index onto storage: periodic wrap, transmissive
// copies of the end cells for the ghosts of the odd->even step, Dirichlet
// ghost states, clamping for lanes past the end (their results are unused).
__device__ __forceinline__ int map_old(int o, int n_old, int N, int bc, int parity_old, int& ghost) {
  ghost = 0;
  if (bc == kPeriodic) {
    // a tile reaches at most one cell before 0 and 63 past the end, so one
    // wrap suffices unless N < 64 (then fall back to the remainder)
    if (o < 0) o += N;
    else if (o >= N) o -= N;
    if (o >= N) o %= N;
    return o;
  }
  if (o < 0) {
    if (bc == kDirichlet && parity_old == 1) ghost = 1;
    return 0;
  }
  if (o >= n_old) {
    if (bc == kDirichlet && parity_old == 1 && o == n_old) ghost = 2;
    return n_old - 1;
  }
  return o;
}

// The old-cell inputs of one lane for one tile (loaded ahead of use when the
// kernel prefetches the next tile while computing the current one).
template <int EQ, int P, class R>
struct TileIn {
  double p[ncomp<EQ>()];
  R d[ncomp<EQ>()][P + 1];
};

template <int EQ, int P, class R>
__device__ __forceinline__ void fetch_tile(const StepArgs<R>& a, int64_t tile, int lane, TileIn<EQ, P, R>& in) {
  constexpr int NC = ncomp<EQ>();
  // cell indices fit 32 bits (N <= 2^28, checked at creation)
  const int j0 = (int)tile * 63;
  int ghost;
  const int o = map_old(j0 + lane - (a.parity_old == 1 ? 1 : 0), (int)a.n_old, (int)a.N, a.bc, a.parity_old, ghost);
  // rows addressed by a uniform 64-bit base and a 32-bit byte offset (rows
  // are shorter than 4 GiB, checked at creation)
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

// The new cell of this lane (lanes 0..62, cell 63 tile + lane, if it exists):
// returns whether there is one and leaves it in pn / dn.
template <int EQ, int P, bool LIM, class R>
__device__ __forceinline__ bool tile_cells(const StepArgs<R>& a, int64_t tile, const TileIn<EQ, P, R>& in,
                                          double lam, R nlam, int lane, double& smax, unsigned& flags,
                                          double (&pn)[ncomp<EQ>()], R (&dn)[ncomp<EQ>()][P + 1]) {
  constexpr int NC = ncomp<EQ>();
  constexpr int PV = P > 0 ? P : 1;
  OldOut<EQ, P, R> X;
  old_cell<EQ, P, R>(in.p, in.d, nlam, a.ph, X);
  __builtin_amdgcn_sched_barrier(0);

  // Right parent's half of the interface data from lane + 1.
  double uL_R[NC];
  R fbar_R[NC];
  R V_R[NC][PV];
#pragma unroll
  for (int c = 0; c < NC; ++c) {
    uL_R[c] = dpp_from_next(X.uL[c]);
    fbar_R[c] = dpp_from_next(X.fbar[c]);
#pragma unroll
    for (int k = 0; k < P; ++k) V_R[c][k] = dpp_from_next(X.V[c][k]);
    if (P == 0) V_R[c][0] = (R)0;
  }

  const int j = (int)tile * 63 + lane;
  if (lane < 63 && j < (int)a.n_new) {
    double sp;
    flags |= (unsigned)new_cell<EQ, P, LIM, R>(X, uL_R, fbar_R, V_R, lam, a.ph, pn, dn, sp);
    smax = __builtin_fmax(smax, sp);
    if (!(sp == sp)) smax = sp;
    return true;
  }
  return false;
}

template <int EQ, int P, bool LIM, class R>
__device__ __forceinline__ void compute_tile(const StepArgs<R>& a, int64_t tile, const TileIn<EQ, P, R>& in,
                                             double lam, R nlam, int lane, double& smax, unsigned& flags) {
  constexpr int NC = ncomp<EQ>();
  double pn[NC];
  R dn[NC][P + 1];
  if (tile_cells<EQ, P, LIM, R>(a, tile, in, lam, nlam, lane, smax, flags, pn, dn)) {
    const int j = (int)tile * 63 + lane;
#pragma unroll
    for (int c = 0; c < NC; ++c) {
      row_store(row_base(a.p_new + c * a.ld), (uint32_t)j, pn[c]);
#pragma unroll
      for (int k = 1; k <= P; ++k) row_store(row_base(a.d_new + (c * P + (k - 1)) * a.ld), (uint32_t)j, dn[c][k]);
    }
  }
}

// ---------------------------------------------------------------------------
// Line-aligned stores.  A tile writes 63 new cells, so every tile edge falls
// inside a cache line that two waves write in parts; once the state no longer
// fits the caches such partial-line stores cost a quarter of the HBM
// bandwidth.  In the staged variants the waves of a block put their new cells
// into LDS; after a barrier each 64-cell group of new cells (64-aligned, cut
// to the contiguous run of tiles it lies in) is written whole, by the wave
// whose tile holds the group's last cell, or by the run's last wave for the
// run's final group.  A group that the block's next iteration completes is
// kept in a carry region until then.  The values written are the same.
// ---------------------------------------------------------------------------
template <int EQ, int PMAX, class R>
struct Stage {
  static constexpr int NC = ncomp<EQ>();
  static constexpr int ND = NC * (PMAX > 0 ? PMAX : 1);
  static constexpr int kSlots = 6 * 64;   // wave regions 0..3 (64 slots each), carry regions 4 and 5
  double p[NC][kSlots];
  R d[ND][kSlots];
  int32_t carry_lo[2];                     // first cell held in carry region 4 + i
};

template <int EQ, int P, class R, class S>
__device__ __forceinline__ void stage_put(S& s, int slot, const double (&pn)[ncomp<EQ>()],
                                          const R (&dn)[ncomp<EQ>()][P + 1]) {
  constexpr int NC = ncomp<EQ>();
#pragma unroll
  for (int c = 0; c < NC; ++c) {
    s.p[c][slot] = pn[c];
#pragma unroll
    for (int k = 1; k <= P; ++k) s.d[c * P + (k - 1)][slot] = dn[c][k];
  }
}

template <int EQ, int P, class R, class S>
__device__ __forceinline__ void stage_store(const S& s, int slot, double* p_new, R* d_new, int64_t ld, uint32_t j) {
  constexpr int NC = ncomp<EQ>();
#pragma unroll
  for (int c = 0; c < NC; ++c) {
    row_store(row_base(p_new + c * ld), j, s.p[c][slot]);
#pragma unroll
    for (int k = 1; k <= P; ++k) row_store(row_base(d_new + (c * P + (k - 1)) * ld), j, s.d[c * P + (k - 1)][slot]);
  }
}

template <int EQ, int P, class S>
__device__ __forceinline__ void stage_copy(S& s, int from, int to) {
  constexpr int NC = ncomp<EQ>();
#pragma unroll
  for (int c = 0; c < NC; ++c) {
    s.p[c][to] = s.p[c][from];
#pragma unroll
    for (int k = 1; k <= P; ++k) s.d[c * P + (k - 1)][to] = s.d[c * P + (k - 1)][from];
  }
}

// One wave's share of a block iteration's write-out (between the barrier that
// follows staging and the one before the next staging).
//   [lo, hi) : the wave's staged cells (region `wave`); lo == hi: none
//   prev     : the 63 cells below lo are staged by the previous wave, or for
//              wave 0 the cells from carry_lo[cur] up to lo are in carry
//              region 4 + cur
//   next     : the next wave (or, for the last wave, the first wave of the
//              next iteration) continues the run at hi
// Every argument is uniform across the wave.
template <int EQ, int P, class R, class S>
__device__ __forceinline__ void stage_flush(S& s, int cur, int wave, int nw, int lane, int lo, int hi, bool prev,
                                            bool next, double* p_new, R* d_new, int64_t ld) {
  if (lo >= hi) return;
  int avail = lo;
  if (prev) {
    // the carried cells start at most 63 below lo (clamped: every write stays
    // within the 63 cells below this tile)
    const int cl = wave > 0 ? lo - 63 : s.carry_lo[cur];
    avail = cl < lo - 63 ? lo - 63 : (cl > lo ? lo : cl);
  }
  auto slot_of = [&](int c) {
    if (c >= lo) return wave * 64 + (c - lo);
    return wave > 0 ? (wave - 1) * 64 + (c - (lo - 63)) : (4 + cur) * 64 + (c - avail);
  };
  const int e = (hi & ~63) - 1;            // end of the last whole group inside [.., hi)
  if (e >= lo) {                           // the group ending in this tile
    const int c = e - 63 + lane;
    if (c >= avail) stage_store<EQ, P, R>(s, slot_of(c), p_new, d_new, ld, (uint32_t)c);
  }
  const int t0 = avail > e + 1 ? avail : e + 1;   // cells after it
  if (!next) {
    const int c = t0 + lane;
    if (c < hi) stage_store<EQ, P, R>(s, slot_of(c), p_new, d_new, ld, (uint32_t)c);
  } else if (wave == nw - 1) {
    const int c = t0 + lane;
    if (c < hi) stage_copy<EQ, P>(s, slot_of(c), (5 - cur) * 64 + lane);
    if (lane == 0) s.carry_lo[1 - cur] = t0;
  }
}

template <int EQ, int P, bool LIM, class R>
__device__ __forceinline__ void run_tile(const StepArgs<R>& a, int64_t tile, double lam, R nlam, int lane,
                                         double& smax, unsigned& flags) {
  TileIn<EQ, P, R> in;
  fetch_tile<EQ, P, R>(a, tile, lane, in);
  compute_tile<EQ, P, LIM, R>(a, tile, in, lam, nlam, lane, smax, flags);
}

}  // namespace wcc
