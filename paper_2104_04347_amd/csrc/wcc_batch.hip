// wcc_batch.hip -- batched half-steps: many independent 1D instances of uneven
// size N_b and degree P_b advanced by persistent kernels over a tile table.
//
// Each tile is one wave's worth of work inside ONE instance (64 old cells ->
// 63 new cells, exactly the single-instance tile body), so batched results are
// bit-identical to single-instance runs.  Every instance keeps its own
// time-control ring (its own t, s_max and CFL step).  Two schedules:
//   fused   : one launch per half-step over all tiles; the degree is a switch
//             per tile (all degrees compiled into one kernel, so the register
//             budget is that of the largest degree);
//   grouped : one launch per degree per half-step over that degree's tiles
//             (each launch runs at its own occupancy).
// Blocks own contiguous, cost-balanced ranges of the tile table; a wave walks
// its block's range with stride = waves per block, merging consecutive tiles
// of one instance into one wave-level speed reduction and one atomic.  Either
// schedule can stage the new cells in LDS and store them in whole 64-cell
// groups (runs of consecutive tiles of one instance), which keeps partial
// cache-line stores off HBM when the batch does not fit the caches.  The
// grouped schedule can also capture each degree's launches as a branch of
// its own in the run's graphs: instances of different degrees never depend
// on each other, so their launches may overlap and fill each other's tails.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <limits>
#include <string>
#include <vector>

#include "wcc.h"
#include "wcc_cell.hpp"
#include "wcc_internal.hpp"
#include "wcc_ctrl.hpp"
#include "wcc_tile.hpp"

namespace wcc {

constexpr int kBatchPMax = 3;

__device__ __forceinline__ void publish_wave(Ctrl* ctrl, int slot, double smax, unsigned flags) {
  smax = wave_max(smax);
  flags = wave_or(flags);
  if ((threadIdx.x & 63) == 0) {
    const int s1 = slot == 2 ? 0 : slot + 1;
    const unsigned long long bits = (unsigned long long)__double_as_longlong(smax);
    if (bits > __hip_atomic_load(&ctrl->smax[s1], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT))
      atomicMax(&ctrl->smax[s1], bits);
    if (flags) atomicOr(&ctrl->flags[s1], flags);
  }
}

// The single-instance view of instance `in` for this launch.
template <class R>
__device__ __forceinline__ StepArgs<R> instance_args(const BatchArgs<R>& a, const BatchInst& in, int bc, Ctrl* ctrl) {
  StepArgs<R> s;
  s.p_old = a.p_in + in.p_off;
  s.d_old = a.d_in + in.d_off;
  s.p_new = a.p_out + in.p_off;
  s.d_new = a.d_out + in.d_off;
  s.ld = in.ld;
  const int64_t n0 = bc == kPeriodic ? in.N : in.N + 1, n1 = in.N;
  s.n_old = a.parity_old == 0 ? n0 : n1;
  s.n_new = a.parity_old == 0 ? n1 : n0;
  s.N = in.N;
  s.parity_old = a.parity_old;
  s.bc = bc;
  s.dx = in.dx;
  s.dt_fixed = 0.0;
  s.ph = a.ph;
  s.ctrl = ctrl;
  s.parts = nullptr;
  s.slot = a.slot;
  return s;
}

template <int EQ, int P, bool LIM, class R>
__device__ __forceinline__ void batch_tile(const BatchArgs<R>& a, const BatchInst& in, int first, int bc,
                                           Ctrl* ctrl, int lane, double& smax, unsigned& flags) {
  double dt;
  const bool go = step_time(ctrl, nullptr, a.slot, in.dx, 0.0, first == 0, dt);
  if (!go) return;
  const StepArgs<R> s = instance_args(a, in, bc, ctrl);
  const double lam = div_rn(dt, in.dx);
  if ((int64_t)first * 63 < s.n_new) run_tile<EQ, P, LIM, R>(s, first, lam, (R)(-lam), lane, smax, flags);
}

// Staged form: the tile's new cells go to the wave's LDS region; [lo, hi)
// returns the cells staged (empty when the instance is finished or the tile
// lies beyond this mesh's last cell).
template <int EQ, int P, bool LIM, class R, class S>
__device__ __forceinline__ void batch_tile_staged(const BatchArgs<R>& a, const BatchInst& in, int first, int bc,
                                                  Ctrl* ctrl, int lane, int wave, S& st, double& smax,
                                                  unsigned& flags, int& lo, int& hi) {
  constexpr int NC = ncomp<EQ>();
  double dt;
  const bool go = step_time(ctrl, nullptr, a.slot, in.dx, 0.0, first == 0, dt);
  if (!go) return;
  const StepArgs<R> s = instance_args(a, in, bc, ctrl);
  const double lam = div_rn(dt, in.dx);
  if ((int64_t)first * 63 >= s.n_new) return;
  TileIn<EQ, P, R> ti;
  fetch_tile<EQ, P, R>(s, first, lane, ti);
  double pn[NC];
  R dn[NC][P + 1];
  if (tile_cells<EQ, P, LIM, R>(s, first, ti, lam, (R)(-lam), lane, smax, flags, pn, dn))
    stage_put<EQ, P, R>(st, wave * 64 + lane, pn, dn);
  lo = first * 63;
  hi = lo + 63 < (int)s.n_new ? lo + 63 : (int)s.n_new;
}

// P < 0: fused schedule (switch on the instance's degree); P >= 0: the
// grouped schedule's launch for that degree.  STG: staged, line-aligned
// stores (the block's waves advance in lockstep, two barriers per iteration).
// Waves per SIMD the compiler must leave room for: the staged degree-1
// kernel, whose light tiles depend on many waves hiding load latency, is held
// to 80 registers (6 waves; it needs 83 otherwise); the others are free.
constexpr int batch_min_waves(int psel, bool stg) { return psel == 1 && stg ? 6 : 1; }

template <int EQ, int PSEL, bool LIM, class R, bool STG>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(batch_min_waves(PSEL, STG))))
void k_batch_step(const BatchArgs<R> a, const int64_t* __restrict__ block_start, int bc) {
  // the wave index is the same in every lane: say so, so that tile and
  // instance indices live in scalar registers
  const int lane = threadIdx.x & 63, wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6),
            nw = blockDim.x >> 6;
  const int64_t t0 = block_start[blockIdx.x], t1 = block_start[blockIdx.x + 1];
  int cur = -1;
  double smax = 0.0;
  unsigned flags = 0u;
  if constexpr (!STG) {
    for (int64_t w = t0 + wave; w < t1; w += nw) {
      const BatchTile tl = a.tiles[w];
      if (tl.inst != cur) {
        if (cur >= 0) publish_wave(a.ctrl + cur, a.slot, smax, flags);
        cur = tl.inst;
        smax = 0.0;
        flags = 0u;
      }
      const BatchInst in = a.inst[tl.inst];
      Ctrl* ctrl = a.ctrl + tl.inst;
      if constexpr (PSEL >= 0) {
        batch_tile<EQ, PSEL, LIM, R>(a, in, tl.first, bc, ctrl, lane, smax, flags);
      } else {
        switch (in.P) {
          case 0: batch_tile<EQ, 0, false, R>(a, in, tl.first, bc, ctrl, lane, smax, flags); break;
          case 1: batch_tile<EQ, 1, LIM, R>(a, in, tl.first, bc, ctrl, lane, smax, flags); break;
          case 2: batch_tile<EQ, 2, LIM, R>(a, in, tl.first, bc, ctrl, lane, smax, flags); break;
          default: batch_tile<EQ, 3, LIM, R>(a, in, tl.first, bc, ctrl, lane, smax, flags); break;
        }
      }
    }
  } else {
    using S = Stage<EQ, (PSEL >= 0 ? PSEL : kBatchPMax), R>;
    __shared__ S st;
    int side = 0;                                   // carry region of this iteration
    // every wave runs every iteration (the barriers are block-wide)
    for (int64_t wb = t0; wb < t1; wb += nw) {
      const int64_t w = wb + wave;
      int lo = 0, hi = 0, P = 0;
      BatchTile tl{0, 0};
      BatchInst in{};
      if (w < t1) {
        tl = a.tiles[w];
        if (tl.inst != cur) {
          if (cur >= 0) publish_wave(a.ctrl + cur, a.slot, smax, flags);
          cur = tl.inst;
          smax = 0.0;
          flags = 0u;
        }
        in = a.inst[tl.inst];
        Ctrl* ctrl = a.ctrl + tl.inst;
        P = PSEL >= 0 ? PSEL : in.P;
        if constexpr (PSEL >= 0) {
          batch_tile_staged<EQ, PSEL, LIM, R>(a, in, tl.first, bc, ctrl, lane, wave, st, smax, flags, lo, hi);
        } else {
          switch (in.P) {
            case 0:
              batch_tile_staged<EQ, 0, false, R>(a, in, tl.first, bc, ctrl, lane, wave, st, smax, flags, lo, hi);
              break;
            case 1:
              batch_tile_staged<EQ, 1, LIM, R>(a, in, tl.first, bc, ctrl, lane, wave, st, smax, flags, lo, hi);
              break;
            case 2:
              batch_tile_staged<EQ, 2, LIM, R>(a, in, tl.first, bc, ctrl, lane, wave, st, smax, flags, lo, hi);
              break;
            default:
              batch_tile_staged<EQ, 3, LIM, R>(a, in, tl.first, bc, ctrl, lane, wave, st, smax, flags, lo, hi);
              break;
          }
        }
      }
      __syncthreads();
      if (lo < hi) {
        // runs: consecutive table entries of one instance with consecutive tiles
        bool prev = false, next = false;
        if (w > t0) {
          const BatchTile tp = a.tiles[w - 1];
          prev = tp.inst == tl.inst && tp.first == tl.first - 1;
        }
        if (w + 1 < t1) {
          // the next tile continues the run only if it has cells on this mesh
          const BatchTile tn = a.tiles[w + 1];
          const int64_t n_new = a.parity_old == 0 ? in.N : (bc == kPeriodic ? in.N : in.N + 1);
          next = tn.inst == tl.inst && tn.first == tl.first + 1 && (int64_t)tn.first * 63 < n_new;
        }
        double* p_new = a.p_out + in.p_off;
        R* d_new = a.d_out + in.d_off;
        if constexpr (PSEL >= 0) {
          stage_flush<EQ, PSEL, R>(st, side, wave, nw, lane, lo, hi, prev, next, p_new, d_new, in.ld);
        } else {
          switch (P) {
            case 0: stage_flush<EQ, 0, R>(st, side, wave, nw, lane, lo, hi, prev, next, p_new, d_new, in.ld); break;
            case 1: stage_flush<EQ, 1, R>(st, side, wave, nw, lane, lo, hi, prev, next, p_new, d_new, in.ld); break;
            case 2: stage_flush<EQ, 2, R>(st, side, wave, nw, lane, lo, hi, prev, next, p_new, d_new, in.ld); break;
            default: stage_flush<EQ, 3, R>(st, side, wave, nw, lane, lo, hi, prev, next, p_new, d_new, in.ld); break;
          }
        }
      }
      __syncthreads();
      side ^= 1;
    }
  }
  if (cur >= 0) publish_wave(a.ctrl + cur, a.slot, smax, flags);
}

template <int EQ, int PSEL, class R>
static hipError_t launch_b(const BatchArgs<R>& a, const int64_t* bs, int bc, bool lim, bool stg, int blocks,
                           int threads, hipStream_t s) {
  const bool l = lim && PSEL != 0;
  if (l && stg)
    hipLaunchKernelGGL((k_batch_step<EQ, PSEL, true, R, true>), dim3(blocks), dim3(threads), 0, s, a, bs, bc);
  else if (l)
    hipLaunchKernelGGL((k_batch_step<EQ, PSEL, true, R, false>), dim3(blocks), dim3(threads), 0, s, a, bs, bc);
  else if (stg)
    hipLaunchKernelGGL((k_batch_step<EQ, PSEL, false, R, true>), dim3(blocks), dim3(threads), 0, s, a, bs, bc);
  else
    hipLaunchKernelGGL((k_batch_step<EQ, PSEL, false, R, false>), dim3(blocks), dim3(threads), 0, s, a, bs, bc);
  return hipGetLastError();
}

template <int EQ, class R>
static hipError_t launch_bp(const BatchArgs<R>& a, const int64_t* bs, int bc, int psel, bool lim, bool stg,
                            int blocks, int threads, hipStream_t s) {
  switch (psel) {
    case -1: return launch_b<EQ, -1, R>(a, bs, bc, lim, stg, blocks, threads, s);
    case 0: return launch_b<EQ, 0, R>(a, bs, bc, lim, stg, blocks, threads, s);
    case 1: return launch_b<EQ, 1, R>(a, bs, bc, lim, stg, blocks, threads, s);
    case 2: return launch_b<EQ, 2, R>(a, bs, bc, lim, stg, blocks, threads, s);
    case 3: return launch_b<EQ, 3, R>(a, bs, bc, lim, stg, blocks, threads, s);
  }
  return hipErrorInvalidValue;
}

template <class R>
static hipError_t launch_batch(const BatchArgs<R>& a, const int64_t* bs, int eq, int bc, int psel, bool lim,
                               bool stg, int blocks, int threads, hipStream_t s) {
  switch (eq) {
    case kAdvection: return launch_bp<kAdvection, R>(a, bs, bc, psel, lim, stg, blocks, threads, s);
    case kBurgers: return launch_bp<kBurgers, R>(a, bs, bc, psel, lim, stg, blocks, threads, s);
    case kEuler: return launch_bp<kEuler, R>(a, bs, bc, psel, lim, stg, blocks, threads, s);
  }
  return hipErrorInvalidValue;
}

template <class R>
static hipError_t occupancy_batch(int eq, int psel, bool lim, bool stg, int threads, int* per_cu) {
  const void* f = nullptr;
#define WCC_BK(E, PS, L)                                                             \
  (stg ? reinterpret_cast<const void*>(&k_batch_step<E, PS, L, R, true>)             \
       : reinterpret_cast<const void*>(&k_batch_step<E, PS, L, R, false>))
#define WCC_BSEL(E)                                                                  \
  switch (psel) {                                                                    \
    case -1: f = lim ? WCC_BK(E, -1, true) : WCC_BK(E, -1, false); break;            \
    case 0: f = WCC_BK(E, 0, false); break;                                          \
    case 1: f = lim ? WCC_BK(E, 1, true) : WCC_BK(E, 1, false); break;               \
    case 2: f = lim ? WCC_BK(E, 2, true) : WCC_BK(E, 2, false); break;               \
    case 3: f = lim ? WCC_BK(E, 3, true) : WCC_BK(E, 3, false); break;               \
  }
  if (eq == kAdvection) { WCC_BSEL(kAdvection) }
  else if (eq == kBurgers) { WCC_BSEL(kBurgers) }
  else { WCC_BSEL(kEuler) }
#undef WCC_BSEL
#undef WCC_BK
  if (!f) return hipErrorInvalidValue;
  return hipOccupancyMaxActiveBlocksPerMultiprocessor(per_cu, f, threads, 0);
}

}  // namespace wcc

using wcc::BatchArgs;
using wcc::BatchInst;
using wcc::BatchTile;
using wcc::Ctrl;

namespace {
inline size_t al256(size_t x) { return (x + 255) & ~size_t(255); }
constexpr int kBatchChunk = 24;  // half-steps per captured graph (multiple of 6)
}  // namespace

struct wcc_batch {
  int eq = 0, bc = 0, nc = 1, B = 0;
  wcc_params prm{};
  size_t elem = 8;
  std::vector<BatchInst> inst;
  std::vector<BatchTile> tiles;          // all tiles, grouped by degree, instances contiguous
  int64_t group_begin[wcc::kBatchPMax + 2] = {};  // tile range of degree p: [group_begin[p], group_begin[p+1])
  int64_t p_total = 0, d_total = 0;      // elements per buffer
  // schedule
  bool grouped = true;
  bool staged = false;                   // line-aligned stores through LDS
  bool branches = true;                  // grouped: the degrees' launches as parallel graph branches
  int threads = 256, blocks = 0, cu = 256;
  std::vector<int64_t> block_start;      // fused: blocks+1 entries; grouped: per group blocks+1 entries, concatenated
  std::vector<int> group_blocks;         // grouped: blocks per degree
  // binding
  char* ws = nullptr;
  size_t ws_bytes = 0;
  hipStream_t stream = nullptr;
  Ctrl* ctrl = nullptr;
  BatchInst* d_inst = nullptr;
  BatchTile* d_tiles = nullptr;
  int64_t* d_bs = nullptr;
  size_t bs_cap = 0;
  double* p[2] = {};
  void* d[2] = {};
  bool bound = false, tables_dirty = true;
  int64_t launched = 0;
  hipStream_t capture = nullptr;
  hipStream_t branch[wcc::kBatchPMax + 1] = {};   // capture-time streams of the degree branches
  hipEvent_t fork = nullptr, join[wcc::kBatchPMax + 1] = {};
  hipGraphExec_t graphs[6] = {};
  hipEvent_t ev0 = nullptr, ev1 = nullptr;
  std::string err;
  std::vector<float> stage;
  double cfl_set[WCC_PMAX + 1] = {-1, -1, -1, -1, -1};
};

namespace {

int bfail(wcc_batch* b, int code, const char* fmt, ...) {
  if (b) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    b->err = buf;
  }
  return code;
}

#define BHIP(bt, call)                                                                              \
  do {                                                                                              \
    hipError_t e_ = (call);                                                                         \
    if (e_ != hipSuccess) return bfail((bt), WCC_EDEVICE, "%s: %s", #call, hipGetErrorString(e_));  \
  } while (0)

int64_t b_ncells(const wcc_batch* b, int i, int parity) {
  const int64_t N = b->inst[i].N;
  if (b->bc == WCC_BC_PERIODIC) return N;
  return parity == 0 ? N + 1 : N;
}

template <class R>
wcc::Phys<R> b_phys(const wcc_batch* b) {
  wcc::Phys<R> ph;
  ph.a = (R)b->prm.a;
  ph.gamma = (R)b->prm.gamma;
  ph.gm1 = (R)(b->prm.gamma - 1.0);
  ph.eps = (R)b->prm.eps;
  return ph;
}

// Relative cost of one tile of degree p (CK work grows roughly with the
// number of Taylor-product terms; measured ratios refine it).
double tile_cost(int p) {
  static const double c[4] = {1.0, 2.0, 3.2, 5.5};
  return c[p < 0 ? 0 : (p > 3 ? 3 : p)];
}

// Split [lo, hi) of the tile table into `nb` contiguous ranges of equal cost.
void split_range(const wcc_batch* b, int64_t lo, int64_t hi, int nb, std::vector<int64_t>& out) {
  double total = 0.0;
  for (int64_t t = lo; t < hi; ++t) total += tile_cost(b->inst[b->tiles[t].inst].P);
  out.push_back(lo);
  double acc = 0.0;
  int k = 1;
  for (int64_t t = lo; t < hi && k < nb; ++t) {
    acc += tile_cost(b->inst[b->tiles[t].inst].P);
    if (acc >= total * (double)k / nb) {
      out.push_back(t + 1);
      ++k;
    }
  }
  while ((int)out.size() < nb) out.push_back(hi);
  out.push_back(hi);
}

int occupancy_for(wcc_batch* b, int psel) {
  int per_cu = 0;
  hipError_t e = b->prm.precision == WCC_FP64
                     ? wcc::occupancy_batch<double>(b->eq, psel, b->prm.limiter != 0, b->staged, b->threads, &per_cu)
                     : wcc::occupancy_batch<float>(b->eq, psel, b->prm.limiter != 0, b->staged, b->threads, &per_cu);
  if (e != hipSuccess || per_cu < 1) per_cu = 1;
  return per_cu;
}

int build_schedule(wcc_batch* b) {
  b->block_start.clear();
  b->group_blocks.clear();
  const int waves = b->threads / 64;
  if (!b->grouped) {
    const int64_t n = (int64_t)b->tiles.size();
    int nb = b->blocks > 0 ? b->blocks : occupancy_for(b, -1) * b->cu;
    nb = (int)std::max<int64_t>(1, std::min<int64_t>(nb, (n + waves - 1) / waves));
    split_range(b, 0, n, nb, b->block_start);
    b->group_blocks.push_back(nb);
  } else {
    for (int p = 0; p <= wcc::kBatchPMax; ++p) {
      const int64_t lo = b->group_begin[p], hi = b->group_begin[p + 1];
      if (hi <= lo) {
        b->group_blocks.push_back(0);
        continue;
      }
      int nb = b->blocks > 0 ? b->blocks : occupancy_for(b, p) * b->cu;
      nb = (int)std::max<int64_t>(1, std::min<int64_t>(nb, (hi - lo + waves - 1) / waves));
      split_range(b, lo, hi, nb, b->block_start);
      b->group_blocks.push_back(nb);
    }
  }
  b->tables_dirty = true;
  for (auto& g : b->graphs)
    if (g) { (void)hipGraphExecDestroy(g); g = nullptr; }
  return WCC_OK;
}

size_t tables_bytes(const wcc_batch* b, size_t bs_entries) {
  return al256(sizeof(Ctrl) * (size_t)b->B) + al256(sizeof(BatchInst) * (size_t)b->B) +
         al256(sizeof(BatchTile) * b->tiles.size()) + al256(sizeof(int64_t) * bs_entries);
}

// Upper bound of the block-start table: grouped schedules need blocks+1
// entries per degree; the bound covers any schedule up to 64k blocks each.
size_t bs_capacity(const wcc_batch* b) { return (size_t)(wcc::kBatchPMax + 1) * (65536 + 1) + (size_t)b->B * 0; }

int upload_tables(wcc_batch* b) {
  if (!b->tables_dirty) return WCC_OK;
  if (b->block_start.size() > b->bs_cap) return bfail(b, WCC_ESIZE, "schedule table too large");
  BHIP(b, hipMemcpyAsync(b->d_inst, b->inst.data(), sizeof(BatchInst) * b->inst.size(), hipMemcpyHostToDevice,
                         b->stream));
  BHIP(b, hipMemcpyAsync(b->d_tiles, b->tiles.data(), sizeof(BatchTile) * b->tiles.size(), hipMemcpyHostToDevice,
                         b->stream));
  BHIP(b, hipMemcpyAsync(b->d_bs, b->block_start.data(), sizeof(int64_t) * b->block_start.size(),
                         hipMemcpyHostToDevice, b->stream));
  BHIP(b, hipStreamSynchronize(b->stream));
  b->tables_dirty = false;
  return WCC_OK;
}

// One half-step of every instance on stream s; with only_p >= 0 (grouped
// schedule) just the launch of that degree.
template <class R>
int enqueue_batch_step(wcc_batch* b, int parity, int slot, hipStream_t s, int only_p = -1) {
  BatchArgs<R> a{};
  a.p_in = b->p[parity];
  a.d_in = static_cast<const R*>(b->d[parity]);
  a.p_out = b->p[1 - parity];
  a.d_out = static_cast<R*>(b->d[1 - parity]);
  a.inst = b->d_inst;
  a.tiles = b->d_tiles;
  a.n_tiles = (int64_t)b->tiles.size();
  a.ctrl = b->ctrl;
  a.ph = b_phys<R>(b);
  a.parity_old = parity;
  a.slot = slot;
  const bool lim = b->prm.limiter != 0;
  size_t off = 0;
  if (!b->grouped) {
    hipError_t e = wcc::launch_batch<R>(a, b->d_bs, b->eq, b->bc, -1, lim, b->staged, b->group_blocks[0], b->threads, s);
    if (e != hipSuccess) return bfail(b, WCC_EDEVICE, "batch launch: %s", hipGetErrorString(e));
    return WCC_OK;
  }
  for (int p = 0; p <= wcc::kBatchPMax; ++p) {
    const int nb = b->group_blocks[p];
    if (nb == 0) continue;
    if (only_p >= 0 && p != only_p) {
      off += (size_t)nb + 1;
      continue;
    }
    hipError_t e = wcc::launch_batch<R>(a, b->d_bs + off, b->eq, b->bc, p, lim, b->staged, nb, b->threads, s);
    if (e != hipSuccess) return bfail(b, WCC_EDEVICE, "batch launch (P=%d): %s", p, hipGetErrorString(e));
    off += (size_t)nb + 1;
  }
  return WCC_OK;
}

int enqueue_b(wcc_batch* b, int parity, int slot, hipStream_t s, int only_p = -1) {
  return b->prm.precision == WCC_FP64 ? enqueue_batch_step<double>(b, parity, slot, s, only_p)
                                      : enqueue_batch_step<float>(b, parity, slot, s, only_p);
}

// Capture a chunk with one graph branch per degree: the instances of one
// degree depend only on their own previous half-steps, so the launches of
// different degrees may run side by side (filling each other's tails).
int capture_branches(wcc_batch* b, int slot0, int parity0) {
  if (!b->fork) BHIP(b, hipEventCreateWithFlags(&b->fork, hipEventDisableTiming));
  BHIP(b, hipEventRecord(b->fork, b->capture));
  for (int p = 0; p <= wcc::kBatchPMax; ++p) {
    if (b->group_blocks[p] == 0) continue;
    if (!b->branch[p]) BHIP(b, hipStreamCreateWithFlags(&b->branch[p], hipStreamNonBlocking));
    if (!b->join[p]) BHIP(b, hipEventCreateWithFlags(&b->join[p], hipEventDisableTiming));
    BHIP(b, hipStreamWaitEvent(b->branch[p], b->fork, 0));
  }
  int rc = WCC_OK;
  for (int p = 0; p <= wcc::kBatchPMax && rc == WCC_OK; ++p) {
    if (b->group_blocks[p] == 0) continue;
    for (int i = 0; i < kBatchChunk && rc == WCC_OK; ++i)
      rc = enqueue_b(b, (parity0 + i) & 1, (slot0 + i) % 3, b->branch[p], p);
  }
  // join every branch back into the capturing stream (also after an error,
  // so that the capture can end)
  for (int p = 0; p <= wcc::kBatchPMax; ++p) {
    if (b->group_blocks[p] == 0) continue;
    BHIP(b, hipEventRecord(b->join[p], b->branch[p]));
    BHIP(b, hipStreamWaitEvent(b->capture, b->join[p], 0));
  }
  return rc;
}

int batch_graph(wcc_batch* b, int slot0, int parity0, hipGraphExec_t* out) {
  const int key = slot0 * 2 + parity0;
  if (b->graphs[key]) {
    *out = b->graphs[key];
    return WCC_OK;
  }
  if (!b->capture) BHIP(b, hipStreamCreateWithFlags(&b->capture, hipStreamNonBlocking));
  BHIP(b, hipStreamBeginCapture(b->capture, hipStreamCaptureModeThreadLocal));
  int rc = WCC_OK;
  if (b->grouped && b->branches)
    rc = capture_branches(b, slot0, parity0);
  else
    for (int i = 0; i < kBatchChunk && rc == WCC_OK; ++i)
      rc = enqueue_b(b, (parity0 + i) & 1, (slot0 + i) % 3, b->capture);
  hipGraph_t g = nullptr;
  hipError_t e = hipStreamEndCapture(b->capture, &g);
  if (rc != WCC_OK) {
    if (g) (void)hipGraphDestroy(g);
    return rc;
  }
  if (e != hipSuccess) return bfail(b, WCC_EDEVICE, "graph capture: %s", hipGetErrorString(e));
  hipGraphExec_t ex = nullptr;
  e = hipGraphInstantiate(&ex, g, nullptr, nullptr, 0);
  (void)hipGraphDestroy(g);
  if (e != hipSuccess) return bfail(b, WCC_EDEVICE, "graph instantiate: %s", hipGetErrorString(e));
  b->graphs[key] = ex;
  *out = ex;
  return WCC_OK;
}

}  // namespace

extern "C" {

int wcc_batch_create(int equation, int B, const int32_t* P, const int64_t* N, int bc, const wcc_params* params,
                     wcc_batch** out) {
  if (!out) return WCC_EINVAL;
  *out = nullptr;
  if (equation < WCC_ADVECTION || equation > WCC_EULER || B < 1 || !P || !N) return WCC_EINVAL;
  if (bc < WCC_BC_PERIODIC || bc > WCC_BC_DIRICHLET) return WCC_EINVAL;
  wcc_params prm;
  if (params) prm = *params; else wcc_params_default(&prm);
  if (!(prm.x_right > prm.x_left) || (prm.precision != WCC_FP64 && prm.precision != WCC_FP32_MIXED))
    return WCC_EINVAL;
  if (equation == WCC_EULER && !(prm.gamma > 1.0)) return WCC_EINVAL;
  for (int i = 0; i < B; ++i)
    if (P[i] < 0 || P[i] > wcc::kBatchPMax || N[i] < 2 || N[i] > (1LL << 28)) return WCC_EINVAL;
  wcc_batch* b = new wcc_batch();
  b->eq = equation;
  b->bc = bc;
  b->nc = equation == WCC_EULER ? 3 : 1;
  b->B = B;
  b->prm = prm;
  b->elem = prm.precision == WCC_FP64 ? 8 : 4;
  b->inst.resize(B);
  for (int i = 0; i < B; ++i) {
    BatchInst& in = b->inst[i];
    in.N = N[i];
    in.P = P[i];
    const int64_t nmax = bc == WCC_BC_PERIODIC ? N[i] : N[i] + 1;
    in.ld = (nmax + 63) / 64 * 64;
    in.dx = (prm.x_right - prm.x_left) / (double)N[i];
    in.cfl = 0.0;
    in.p_off = b->p_total;
    in.d_off = b->d_total;
    b->p_total += (int64_t)b->nc * in.ld;
    b->d_total += (int64_t)b->nc * P[i] * in.ld;
  }
  // tiles grouped by degree, instances in input order inside a group
  for (int p = 0; p <= wcc::kBatchPMax; ++p) {
    b->group_begin[p] = (int64_t)b->tiles.size();
    for (int i = 0; i < B; ++i) {
      if (b->inst[i].P != p) continue;
      const int64_t nmax = bc == WCC_BC_PERIODIC ? N[i] : N[i] + 1;
      const int64_t nt = (nmax + 62) / 63;
      for (int64_t t = 0; t < nt; ++t) b->tiles.push_back(BatchTile{i, (int32_t)t});
    }
  }
  b->group_begin[wcc::kBatchPMax + 1] = (int64_t)b->tiles.size();
  int dev = 0;
  hipDeviceProp_t prop;
  if (hipGetDevice(&dev) == hipSuccess && hipGetDeviceProperties(&prop, dev) == hipSuccess)
    b->cu = prop.multiProcessorCount;
  b->bs_cap = bs_capacity(b);
  build_schedule(b);
  *out = b;
  return WCC_OK;
}

int wcc_batch_workspace_bytes(const wcc_batch* b, size_t* bytes) {
  if (!b || !bytes) return WCC_EINVAL;
  *bytes = tables_bytes(b, b->bs_cap) + 2 * al256((size_t)b->p_total * 8) + 2 * al256((size_t)b->d_total * b->elem);
  return WCC_OK;
}

int wcc_batch_bind(wcc_batch* b, void* dev_ptr, size_t bytes, void* hip_stream) {
  if (!b || !dev_ptr) return WCC_EINVAL;
  if (((uintptr_t)dev_ptr & 255u) != 0) return bfail(b, WCC_EINVAL, "workspace must be 256-byte aligned");
  size_t need = 0;
  wcc_batch_workspace_bytes(b, &need);
  if (bytes < need) return bfail(b, WCC_ESIZE, "workspace of %zu bytes, need %zu", bytes, need);
  for (auto& g : b->graphs)
    if (g) { (void)hipGraphExecDestroy(g); g = nullptr; }
  b->ws = static_cast<char*>(dev_ptr);
  b->ws_bytes = bytes;
  b->stream = static_cast<hipStream_t>(hip_stream);
  char* q = b->ws;
  b->ctrl = reinterpret_cast<Ctrl*>(q);
  q += al256(sizeof(Ctrl) * (size_t)b->B);
  b->d_inst = reinterpret_cast<BatchInst*>(q);
  q += al256(sizeof(BatchInst) * (size_t)b->B);
  b->d_tiles = reinterpret_cast<BatchTile*>(q);
  q += al256(sizeof(BatchTile) * b->tiles.size());
  b->d_bs = reinterpret_cast<int64_t*>(q);
  q += al256(sizeof(int64_t) * b->bs_cap);
  b->p[0] = reinterpret_cast<double*>(q);
  q += al256((size_t)b->p_total * 8);
  b->p[1] = reinterpret_cast<double*>(q);
  q += al256((size_t)b->p_total * 8);
  b->d[0] = q;
  q += al256((size_t)b->d_total * b->elem);
  b->d[1] = q;
  b->bound = true;
  b->tables_dirty = true;
  b->launched = 0;
  // every instance starts at t = 0 with an empty ring
  std::vector<Ctrl> h((size_t)b->B);
  std::memset(h.data(), 0, sizeof(Ctrl) * h.size());
  for (auto& c : h) {
    c.t_end = std::numeric_limits<double>::infinity();
    for (int i = 0; i < 3; ++i) {
      c.ghost[0][i] = b->prm.left_state[i];
      c.ghost[1][i] = b->prm.right_state[i];
    }
  }
  BHIP(b, hipMemcpyAsync(b->ctrl, h.data(), sizeof(Ctrl) * h.size(), hipMemcpyHostToDevice, b->stream));
  BHIP(b, hipStreamSynchronize(b->stream));
  return upload_tables(b);
}

int wcc_batch_write_dofs(wcc_batch* b, int i, const double* host, int64_t n_cells, double t) {
  if (!b) return WCC_EINVAL;
  if (!b->bound) return bfail(b, WCC_ESTATE, "write before bind");
  if (i < 0 || i >= b->B || !host || !std::isfinite(t)) return bfail(b, WCC_EINVAL, "bad arguments");
  if (b->launched != 0) return bfail(b, WCC_ESTATE, "instances are written before the first run (rebind to restart)");
  const int64_t n = b_ncells(b, i, 0);
  if (n_cells != n) return bfail(b, WCC_ESIZE, "instance %d has %lld cells", i, (long long)n);
  const BatchInst& in = b->inst[i];
  const int P = in.P, nc = b->nc;
  for (int c = 0; c < nc; ++c)
    BHIP(b, hipMemcpyAsync(b->p[0] + in.p_off + (size_t)c * in.ld, host + (size_t)(c * (P + 1)) * n, n * 8,
                           hipMemcpyHostToDevice, b->stream));
  if (P > 0) {
    if (b->prm.precision == WCC_FP64) {
      double* db = static_cast<double*>(b->d[0]) + in.d_off;
      for (int c = 0; c < nc; ++c)
        for (int k = 1; k <= P; ++k)
          BHIP(b, hipMemcpyAsync(db + (size_t)(c * P + k - 1) * in.ld, host + (size_t)(c * (P + 1) + k) * n, n * 8,
                                 hipMemcpyHostToDevice, b->stream));
    } else {
      float* db = static_cast<float*>(b->d[0]) + in.d_off;
      b->stage.resize((size_t)nc * P * n);
      for (int c = 0; c < nc; ++c)
        for (int k = 1; k <= P; ++k) {
          const double* src = host + (size_t)(c * (P + 1) + k) * n;
          float* dst = b->stage.data() + (size_t)(c * P + k - 1) * n;
          for (int64_t j = 0; j < n; ++j) dst[j] = (float)src[j];
        }
      for (int r = 0; r < nc * P; ++r)
        BHIP(b, hipMemcpyAsync(db + (size_t)r * in.ld, b->stage.data() + (size_t)r * n, n * 4,
                               hipMemcpyHostToDevice, b->stream));
    }
  }
  double tt[3] = {t, t, t};
  BHIP(b, hipMemcpyAsync(&b->ctrl[i].t[0], tt, sizeof tt, hipMemcpyHostToDevice, b->stream));
  BHIP(b, hipStreamSynchronize(b->stream));
  return WCC_OK;
}

int wcc_batch_prepare(wcc_batch* b) {
  if (!b) return WCC_EINVAL;
  if (!b->bound) return bfail(b, WCC_ESTATE, "prepare before bind");
  // wave speed of every written instance into its slot 0
  for (int i = 0; i < b->B; ++i) {
    const BatchInst& in = b->inst[i];
    hipError_t e;
    const int64_t n = b_ncells(b, i, 0);
    const int blocks = (int)std::min<int64_t>((n + 255) / 256, 1024);
    if (b->prm.precision == WCC_FP64) {
      wcc::StepArgs<double> a{};
      a.p_old = b->p[0] + in.p_off;
      a.d_old = static_cast<const double*>(b->d[0]) + in.d_off;
      a.ld = in.ld;
      a.n_old = n;
      a.N = in.N;
      a.bc = b->bc;
      a.dx = in.dx;
      a.ph = b_phys<double>(b);
      a.ctrl = b->ctrl + i;
      a.parts = nullptr;
      a.slot = 0;
      e = wcc::launch_state_speed<double>(a, b->eq, in.P, blocks, b->stream);
    } else {
      wcc::StepArgs<float> a{};
      a.p_old = b->p[0] + in.p_off;
      a.d_old = static_cast<const float*>(b->d[0]) + in.d_off;
      a.ld = in.ld;
      a.n_old = n;
      a.N = in.N;
      a.bc = b->bc;
      a.dx = in.dx;
      a.ph = b_phys<float>(b);
      a.ctrl = b->ctrl + i;
      a.parts = nullptr;
      a.slot = 0;
      e = wcc::launch_state_speed<float>(a, b->eq, in.P, blocks, b->stream);
    }
    if (e != hipSuccess) return bfail(b, WCC_EDEVICE, "speed kernel: %s", hipGetErrorString(e));
  }
  BHIP(b, hipStreamSynchronize(b->stream));
  return WCC_OK;
}

int wcc_batch_advance(wcc_batch* b, int64_t half_steps, const double cfl_by_P[WCC_PMAX + 1]) {
  if (!b || !cfl_by_P || half_steps < 0) return WCC_EINVAL;
  if (!b->bound) return bfail(b, WCC_ESTATE, "run before bind");
  // per-instance CFL numbers live in each control block
  bool changed = false;
  for (int p = 0; p <= WCC_PMAX; ++p)
    if (cfl_by_P[p] != b->cfl_set[p]) changed = true;
  if (changed) {
    for (int p = 0; p <= wcc::kBatchPMax; ++p)
      if (!(cfl_by_P[p] > 0.0 && cfl_by_P[p] <= 1.0)) {
        bool used = false;
        for (const auto& in : b->inst) used = used || in.P == p;
        if (used) return bfail(b, WCC_EINVAL, "cfl for P=%d outside (0, 1]", p);
      }
  }
  int rc = upload_tables(b);
  if (rc) return rc;
  if (changed) {
    // the per-instance CFL numbers go to the control blocks by a kernel whose
    // arguments carry the values (after the instance table is on the device)
    wcc::CflByDegree v;
    for (int p = 0; p <= WCC_PMAX; ++p) v.v[p] = cfl_by_P[p];
    BHIP(b, wcc::launch_batch_set_cfl(b->ctrl, b->d_inst, b->B, v, b->stream));
    for (int p = 0; p <= WCC_PMAX; ++p) b->cfl_set[p] = cfl_by_P[p];
  }
  // every chunk graph a run can start on, built before the timed events
  if (half_steps >= kBatchChunk) {
    for (int key = 0; key < 6; ++key) {
      hipGraphExec_t g;
      rc = batch_graph(b, key / 2, key % 2, &g);
      if (rc) return rc;
    }
  }
  if (!b->ev0) BHIP(b, hipEventCreate(&b->ev0));
  if (!b->ev1) BHIP(b, hipEventCreate(&b->ev1));
  BHIP(b, hipEventRecord(b->ev0, b->stream));
  int64_t left = half_steps;
  while (left > 0) {
    const int slot = (int)(b->launched % 3), par = (int)(b->launched & 1);
    if (left >= kBatchChunk) {
      hipGraphExec_t g;
      rc = batch_graph(b, slot, par, &g);
      if (rc) return rc;
      BHIP(b, hipGraphLaunch(g, b->stream));
      b->launched += kBatchChunk;
      left -= kBatchChunk;
    } else {
      rc = enqueue_b(b, par, slot, b->stream);
      if (rc) return rc;
      b->launched += 1;
      left -= 1;
    }
  }
  BHIP(b, hipEventRecord(b->ev1, b->stream));
  return WCC_OK;
}

int wcc_batch_read_dofs(wcc_batch* b, int i, double* host, int64_t cap, wcc_state_info* info) {
  if (!b) return WCC_EINVAL;
  if (!b->bound) return bfail(b, WCC_ESTATE, "read before bind");
  if (i < 0 || i >= b->B) return bfail(b, WCC_EINVAL, "bad instance");
  Ctrl h;
  BHIP(b, hipMemcpyAsync(&h, &b->ctrl[i], sizeof h, hipMemcpyDeviceToHost, b->stream));
  BHIP(b, hipStreamSynchronize(b->stream));
  const int parity = (int)(h.steps_done & 1);
  const int64_t n = b_ncells(b, i, parity);
  const BatchInst& in = b->inst[i];
  const int P = in.P, nc = b->nc;
  if (host) {
    if (cap < (int64_t)nc * (P + 1) * n) return bfail(b, WCC_ESIZE, "host buffer too small");
    for (int c = 0; c < nc; ++c)
      BHIP(b, hipMemcpyAsync(host + (size_t)(c * (P + 1)) * n, b->p[parity] + in.p_off + (size_t)c * in.ld, n * 8,
                             hipMemcpyDeviceToHost, b->stream));
    if (P > 0) {
      if (b->prm.precision == WCC_FP64) {
        const double* db = static_cast<const double*>(b->d[parity]) + in.d_off;
        for (int c = 0; c < nc; ++c)
          for (int k = 1; k <= P; ++k)
            BHIP(b, hipMemcpyAsync(host + (size_t)(c * (P + 1) + k) * n, db + (size_t)(c * P + k - 1) * in.ld, n * 8,
                                   hipMemcpyDeviceToHost, b->stream));
      } else {
        const float* db = static_cast<const float*>(b->d[parity]) + in.d_off;
        b->stage.resize((size_t)nc * P * n);
        for (int r = 0; r < nc * P; ++r)
          BHIP(b, hipMemcpyAsync(b->stage.data() + (size_t)r * n, db + (size_t)r * in.ld, n * 4,
                                 hipMemcpyDeviceToHost, b->stream));
      }
    }
    BHIP(b, hipStreamSynchronize(b->stream));
    if (P > 0 && b->prm.precision != WCC_FP64)
      for (int c = 0; c < nc; ++c)
        for (int k = 1; k <= P; ++k) {
          const float* src = b->stage.data() + (size_t)(c * P + k - 1) * n;
          double* dst = host + (size_t)(c * (P + 1) + k) * n;
          for (int64_t j = 0; j < n; ++j) dst[j] = (double)src[j];
        }
  }
  if (info) {
    const int s = (int)(b->launched % 3);
    info->t = h.t[s];
    info->parity = parity;
    info->flags = (int32_t)h.flags[s];
    info->n_cells = n;
    info->dx = in.dx;
    info->x_first_center = b->prm.x_left + 0.5 * (double)parity * in.dx;
    info->half_steps = h.steps_done;
    unsigned long long bits = h.smax[s];
    std::memcpy(&info->s_max, &bits, 8);
  }
  return WCC_OK;
}

int wcc_batch_set_schedule(wcc_batch* b, int threads_per_block, int blocks, int mode) {
  if (!b) return WCC_EINVAL;
  if (threads_per_block != 0 && (threads_per_block % 64 != 0 || threads_per_block < 64 || threads_per_block > 256))
    return bfail(b, WCC_EINVAL, "threads per block must be 64..256 in steps of 64");
  if (blocks < 0 || blocks > 65536) return bfail(b, WCC_EINVAL, "blocks outside [0, 65536]");
  if (threads_per_block) b->threads = threads_per_block;
  b->blocks = blocks;
  if (mode < 0 || mode > 6) return bfail(b, WCC_EINVAL, "schedule mode must be 0..6");
  if (mode != 0) {
    b->grouped = mode == 2 || mode == 4 || mode >= 5;
    b->staged = mode == 3 || mode == 4 || mode == 6;
    b->branches = mode >= 5;
  }
  return build_schedule(b);
}

int wcc_batch_last_run_ms(wcc_batch* b, double* ms) {
  if (!b || !ms) return WCC_EINVAL;
  if (!b->ev0 || !b->ev1) return bfail(b, WCC_ESTATE, "no timed run");
  BHIP(b, hipEventSynchronize(b->ev1));
  float f = 0.f;
  BHIP(b, hipEventElapsedTime(&f, b->ev0, b->ev1));
  *ms = f;
  return WCC_OK;
}

const char* wcc_batch_last_error(const wcc_batch* b) { return b ? b->err.c_str() : "null batch"; }

void wcc_batch_destroy(wcc_batch* b) {
  if (!b) return;
  for (auto& g : b->graphs)
    if (g) (void)hipGraphExecDestroy(g);
  if (b->capture) (void)hipStreamDestroy(b->capture);
  for (int p = 0; p <= wcc::kBatchPMax; ++p) {
    if (b->branch[p]) (void)hipStreamDestroy(b->branch[p]);
    if (b->join[p]) (void)hipEventDestroy(b->join[p]);
  }
  if (b->fork) (void)hipEventDestroy(b->fork);
  if (b->ev0) (void)hipEventDestroy(b->ev0);
  if (b->ev1) (void)hipEventDestroy(b->ev1);
  delete b;
}

}  // extern "C"
