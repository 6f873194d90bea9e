// wcc2d_api.hip -- host side of the C ABI declared in include/wcc2d.h.
//
// Same structure as the 1D context: host-side sizes and layout, a half-step
// counter, a cache of instantiated graphs; device memory and the stream come
// from the caller.
//
// Workspace layout (256-byte aligned pieces):
//   [ctrl: Ctrl] [parts: 3 x 64 partial wave-speed maxima] [q0] [q1]
// with q_b = nc*ndof planes of `plane` doubles (Nx*Ny rounded up to 64);
// buffer b holds the state of mesh parity b.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <limits>
#include <string>
#include <vector>

#include "wcc2d.h"
#include "wcc2d_internal.hpp"
#include "wcc_ctrl.hpp"

using wcc::Ctrl;
using wcc2d::Step2Args;

namespace {

constexpr int kChunk2 = 48;  // half-steps per captured graph (multiple of 6)

inline size_t al256(size_t x) { return (x + 255) & ~size_t(255); }

}  // namespace

struct wcc2d_ctx {
  int eq = 0, P = 0, nc = 1, nd = 1;
  int64_t Nx = 0, Ny = 0, plane = 0;
  int bc = WCC_BC_PERIODIC, bc_y = WCC_BC_PERIODIC;   // x and y edges
  wcc2d_params prm{};
  char* ws = nullptr;
  size_t ws_bytes = 0;
  hipStream_t stream = nullptr;
  Ctrl* ctrl = nullptr;
  unsigned long long* parts = nullptr;
  double* q[2] = {nullptr, nullptr};
  bool bound = false, written = false;
  int parity_w = 0;
  int64_t launched = 0, steps = 0;
  int threads = 256, blocks = 0, cu = 0;
  int variant = 3;   // 0: 8 x 8 wave tiles, 1: row marching over 64-column strips, 2: the same with prefetch,
                     // 3 (default): as 2 with band-major work items (neighbouring strips on one CU / XCD)
  hipStream_t capture = nullptr;
  hipGraphExec_t graphs[6] = {};
  hipEvent_t ev0 = nullptr, ev1 = nullptr;
  std::string err;
  std::vector<unsigned long long> stage_zero;
};

namespace {

int fail2(wcc2d_ctx* c, int code, const char* fmt, ...) {
  if (c) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    c->err = buf;
  }
  return code;
}

#define HIPCHK2(ctx, call)                                                                          \
  do {                                                                                              \
    hipError_t e_ = (call);                                                                         \
    if (e_ != hipSuccess) return fail2((ctx), WCC_EDEVICE, "%s: %s", #call, hipGetErrorString(e_)); \
  } while (0)

double dx_of(const wcc2d_ctx* c) { return (c->prm.x_right - c->prm.x_left) / (double)c->Nx; }
double dy_of(const wcc2d_ctx* c) { return (c->prm.y_right - c->prm.y_left) / (double)c->Ny; }

// Cells of the mesh of this parity: Nx x Ny (periodic, and the staggered
// transmissive mesh) or (Nx+1) x (Ny+1) (the transmissive mesh of the mesh
// points).
int64_t mesh_nx(const wcc2d_ctx* c, int parity) { return c->Nx + (c->bc == WCC_BC_PERIODIC || parity ? 0 : 1); }
int64_t mesh_ny(const wcc2d_ctx* c, int parity) { return c->Ny + (c->bc_y == WCC_BC_PERIODIC || parity ? 0 : 1); }

Step2Args args_for(const wcc2d_ctx* c, int parity, int slot, double dt_fixed) {
  Step2Args a{};
  a.q_old = c->q[parity];
  a.q_new = c->q[1 - parity];
  a.plane = c->plane;
  a.Nx = (int32_t)c->Nx;
  a.Ny = (int32_t)c->Ny;
  a.nxo = (int32_t)mesh_nx(c, parity);
  a.nyo = (int32_t)mesh_ny(c, parity);
  a.nxn = (int32_t)mesh_nx(c, 1 - parity);
  a.nyn = (int32_t)mesh_ny(c, 1 - parity);
  a.periodic_x = c->bc == WCC_BC_PERIODIC ? 1 : 0;
  a.periodic_y = c->bc_y == WCC_BC_PERIODIC ? 1 : 0;
  a.parity_old = parity;
  a.slot = slot;
  a.dx = dx_of(c);
  a.dy = dy_of(c);
  a.idx = 1.0 / a.dx;
  a.idy = 1.0 / a.dy;
  a.dt_fixed = dt_fixed;
  a.ph.a = c->prm.a;
  a.ph.b = c->prm.b;
  a.ph.gamma = c->prm.gamma;
  a.ph.gm1 = c->prm.gamma - 1.0;
  a.ph.eps = c->prm.eps;
  a.ctrl = c->ctrl;
  a.parts = c->parts;
  return a;
}

int blocks_for(wcc2d_ctx* c, int parity) {
  if (c->blocks > 0) return c->blocks;
  // work units over the new mesh: 8 x 8 tiles (variant 0) or rows of
  // 64-column strips
  const int64_t nx = mesh_nx(c, 1 - parity), ny = mesh_ny(c, 1 - parity);
  const int64_t units = c->variant >= 1 ? ((nx + 62) / 63) * ny : ((nx + 6) / 7) * ((ny + 6) / 7);
  const int waves = c->threads / 64;
  int per_cu = 0;
  if (wcc2d::occupancy_half_step2(c->eq, c->P, c->prm.limiter != 0, c->variant, c->threads, c->plane, &per_cu) !=
          hipSuccess ||
      per_cu < 1)
    per_cu = 1;
  const int64_t full = (int64_t)per_cu * c->cu, need = (units + waves - 1) / waves;
  return (int)std::max<int64_t>(1, std::min(full, need));
}

int enqueue2(wcc2d_ctx* c, int parity, int slot, double dt_fixed, hipStream_t s) {
  hipError_t e = wcc2d::launch_half_step2(args_for(c, parity, slot, dt_fixed), c->eq, c->P, c->prm.limiter != 0,
                                          c->variant, blocks_for(c, parity), c->threads, s);
  if (e != hipSuccess) return fail2(c, WCC_EDEVICE, "2D half-step launch: %s", hipGetErrorString(e));
  return WCC_OK;
}

int parity_now(const wcc2d_ctx* c) { return (int)((c->parity_w + c->steps) & 1); }

int graph2(wcc2d_ctx* c, int slot0, int parity0, hipGraphExec_t* out) {
  const int key = slot0 * 2 + parity0;
  if (c->graphs[key]) {
    *out = c->graphs[key];
    return WCC_OK;
  }
  if (!c->capture) HIPCHK2(c, hipStreamCreateWithFlags(&c->capture, hipStreamNonBlocking));
  HIPCHK2(c, hipStreamBeginCapture(c->capture, hipStreamCaptureModeThreadLocal));
  int rc = WCC_OK;
  for (int i = 0; i < kChunk2 && rc == WCC_OK; ++i) rc = enqueue2(c, (parity0 + i) & 1, (slot0 + i) % 3, 0.0, c->capture);
  hipGraph_t g = nullptr;
  hipError_t e = hipStreamEndCapture(c->capture, &g);
  if (rc != WCC_OK) {
    if (g) (void)hipGraphDestroy(g);
    return rc;
  }
  if (e != hipSuccess) return fail2(c, WCC_EDEVICE, "graph capture: %s", hipGetErrorString(e));
  hipGraphExec_t ex = nullptr;
  e = hipGraphInstantiate(&ex, g, nullptr, nullptr, 0);
  (void)hipGraphDestroy(g);
  if (e != hipSuccess) return fail2(c, WCC_EDEVICE, "graph instantiate: %s", hipGetErrorString(e));
  c->graphs[key] = ex;
  *out = ex;
  return WCC_OK;
}

void drop_graphs(wcc2d_ctx* c) {
  for (auto& g : c->graphs)
    if (g) { (void)hipGraphExecDestroy(g); g = nullptr; }
}

int set_fields(wcc2d_ctx* c, double t_end, double cfl) {
  HIPCHK2(c, wcc::launch_set_fields(c->ctrl, t_end, cfl, c->stream));
  return WCC_OK;
}

int read_ctrl2(wcc2d_ctx* c, Ctrl* h) {
  std::vector<unsigned long long> parts(wcc::kSmaxPartsBytes / sizeof(unsigned long long));
  HIPCHK2(c, hipMemcpyAsync(h, c->ctrl, sizeof(Ctrl), hipMemcpyDeviceToHost, c->stream));
  HIPCHK2(c, hipMemcpyAsync(parts.data(), c->parts, wcc::kSmaxPartsBytes, hipMemcpyDeviceToHost, c->stream));
  HIPCHK2(c, hipStreamSynchronize(c->stream));
  for (int s = 0; s < 3; ++s) {
    unsigned long long m = 0;
    for (int i = 0; i < wcc::kSmaxParts; ++i) m = std::max(m, parts[(size_t)(s * wcc::kSmaxParts + i) * wcc::kSmaxStride]);
    h->smax[s] = m;
  }
  c->steps = h->steps_done;
  return WCC_OK;
}

bool cfl_ok(double cfl) { return cfl > 0.0 && cfl <= 1.0 && std::isfinite(cfl); }

int run2(wcc2d_ctx* c, int64_t n, bool timed) {
  if (n >= kChunk2)
    for (int key = 0; key < 6; ++key) {
      hipGraphExec_t g;
      const int rc = graph2(c, key / 2, key % 2, &g);
      if (rc) return rc;
    }
  if (timed) {
    if (!c->ev0) HIPCHK2(c, hipEventCreate(&c->ev0));
    if (!c->ev1) HIPCHK2(c, hipEventCreate(&c->ev1));
    HIPCHK2(c, hipEventRecord(c->ev0, c->stream));
  }
  int64_t left = n;
  while (left > 0) {
    const int slot = (int)(c->launched % 3), par = parity_now(c);
    if (left >= kChunk2) {
      hipGraphExec_t g;
      const int rc = graph2(c, slot, par, &g);
      if (rc) return rc;
      HIPCHK2(c, hipGraphLaunch(g, c->stream));
      c->launched += kChunk2;
      c->steps += kChunk2;
      left -= kChunk2;
    } else {
      const int rc = enqueue2(c, par, slot, 0.0, c->stream);
      if (rc) return rc;
      c->launched += 1;
      c->steps += 1;
      left -= 1;
    }
  }
  if (timed) HIPCHK2(c, hipEventRecord(c->ev1, c->stream));
  return WCC_OK;
}

}  // namespace

extern "C" {

int wcc2d_params_default(wcc2d_params* p) {
  if (!p) return WCC_EINVAL;
  std::memset(p, 0, sizeof *p);
  p->x_right = 1.0;
  p->y_right = 1.0;
  p->a = 1.0;
  p->b = 1.0;
  p->gamma = 1.4;
  p->eps = 1e-40;
  p->limiter = 1;
  p->bc_y = -1;
  return WCC_OK;
}

int wcc2d_create(int equation, int P, int64_t Nx, int64_t Ny, const wcc2d_params* params, wcc2d_ctx** out) {
  if (!out) return WCC_EINVAL;
  *out = nullptr;
  if (equation < WCC_ADVECTION || equation > WCC_EULER || P < 0 || P > WCC2D_PMAX) return WCC_EINVAL;
  if (Nx < 2 || Ny < 2 || (Nx + 1) * (Ny + 1) > ((int64_t)1 << 28)) return WCC_EINVAL;   // 32-bit byte offsets
  wcc2d_params prm;
  if (params) prm = *params; else wcc2d_params_default(&prm);
  if (prm.bc != WCC_BC_PERIODIC && prm.bc != WCC_BC_TRANSMISSIVE) return WCC_EINVAL;
  if (prm.bc_y != -1 && prm.bc_y != WCC_BC_PERIODIC && prm.bc_y != WCC_BC_TRANSMISSIVE) return WCC_EINVAL;
  if (!(prm.x_right > prm.x_left) || !(prm.y_right > prm.y_left) || !(prm.eps >= 0.0)) return WCC_EINVAL;
  if (equation == WCC_EULER && !(prm.gamma > 1.0)) return WCC_EINVAL;
  wcc2d_ctx* c = new wcc2d_ctx();
  c->eq = equation;
  c->P = P;
  c->nc = equation == WCC_EULER ? 4 : 1;
  c->nd = (P + 1) * (P + 2) / 2;
  c->Nx = Nx;
  c->Ny = Ny;
  c->bc = prm.bc;
  c->bc_y = prm.bc_y < 0 ? prm.bc : prm.bc_y;
  c->plane = (mesh_nx(c, 0) * mesh_ny(c, 0) + 63) / 64 * 64;
  c->prm = prm;
  int dev = 0;
  if (hipGetDevice(&dev) == hipSuccess) {
    hipDeviceProp_t prop;
    if (hipGetDeviceProperties(&prop, dev) == hipSuccess) c->cu = prop.multiProcessorCount;
  }
  if (c->cu <= 0) c->cu = 256;
  *out = c;
  return WCC_OK;
}

int wcc2d_workspace_bytes(const wcc2d_ctx* c, size_t* bytes) {
  if (!c || !bytes) return WCC_EINVAL;
  const size_t qb = al256((size_t)c->nc * c->nd * (size_t)c->plane * 8);
  *bytes = al256(sizeof(Ctrl)) + wcc::kSmaxPartsBytes + 2 * qb;
  return WCC_OK;
}

int wcc2d_bind(wcc2d_ctx* c, void* dev_ptr, size_t bytes, void* hip_stream) {
  if (!c || !dev_ptr) return WCC_EINVAL;
  if (((uintptr_t)dev_ptr & 255u) != 0) return fail2(c, WCC_EINVAL, "workspace must be 256-byte aligned");
  size_t need = 0;
  wcc2d_workspace_bytes(c, &need);
  if (bytes < need) return fail2(c, WCC_ESIZE, "workspace of %zu bytes, need %zu", bytes, need);
  drop_graphs(c);
  c->ws = static_cast<char*>(dev_ptr);
  c->ws_bytes = bytes;
  c->stream = static_cast<hipStream_t>(hip_stream);
  const size_t qb = al256((size_t)c->nc * c->nd * (size_t)c->plane * 8);
  char* p = c->ws;
  c->ctrl = reinterpret_cast<Ctrl*>(p);
  p += al256(sizeof(Ctrl));
  c->parts = reinterpret_cast<unsigned long long*>(p);
  p += wcc::kSmaxPartsBytes;
  c->q[0] = reinterpret_cast<double*>(p);
  p += qb;
  c->q[1] = reinterpret_cast<double*>(p);
  c->bound = true;
  c->written = false;
  return WCC_OK;
}

int wcc2d_write_dofs(wcc2d_ctx* c, const double* host, int parity, double t) {
  if (!c) return WCC_EINVAL;
  if (!c->bound) return fail2(c, WCC_ESTATE, "wcc2d_write_dofs before wcc2d_bind");
  if (!host || (parity != 0 && parity != 1) || !std::isfinite(t)) return fail2(c, WCC_EINVAL, "bad arguments");
  const size_t cells = (size_t)(mesh_nx(c, parity) * mesh_ny(c, parity));
  for (int r = 0; r < c->nc * c->nd; ++r)
    HIPCHK2(c, hipMemcpyAsync(c->q[parity] + (size_t)r * c->plane, host + (size_t)r * cells, cells * 8,
                              hipMemcpyHostToDevice, c->stream));
  Ctrl h;
  std::memset(&h, 0, sizeof h);
  h.t[0] = h.t[1] = h.t[2] = t;
  h.t_end = std::numeric_limits<double>::infinity();
  HIPCHK2(c, hipMemcpyAsync(c->ctrl, &h, sizeof h, hipMemcpyHostToDevice, c->stream));
  c->stage_zero.assign(wcc::kSmaxPartsBytes / sizeof(unsigned long long), 0ull);
  HIPCHK2(c, hipMemcpyAsync(c->parts, c->stage_zero.data(), wcc::kSmaxPartsBytes, hipMemcpyHostToDevice, c->stream));
  const int blocks = (int)std::min<int64_t>((int64_t)(cells + 255) / 256, 4LL * c->cu);
  hipError_t e = wcc2d::launch_state_speed2(args_for(c, parity, 0, 0.0), c->eq, c->P, blocks, c->stream);
  if (e != hipSuccess) return fail2(c, WCC_EDEVICE, "speed kernel: %s", hipGetErrorString(e));
  Ctrl back;
  const int rc = read_ctrl2(c, &back);
  if (rc) return rc;
  c->written = true;
  c->parity_w = parity;
  c->launched = 0;
  c->steps = 0;
  if (back.flags[0]) return fail2(c, WCC_ENONFINITE, "written state holds a non-finite value or a non-positive "
                                                     "density/pressure");
  return WCC_OK;
}

int wcc2d_step(wcc2d_ctx* c, double cfl, double dt_fixed) {
  if (!c) return WCC_EINVAL;
  if (!c->bound || !c->written) return fail2(c, WCC_ESTATE, "no state written");
  if (dt_fixed > 0.0) {
    if (!std::isfinite(dt_fixed)) return fail2(c, WCC_EINVAL, "bad dt");
  } else if (!cfl_ok(cfl)) {
    return fail2(c, WCC_EINVAL, "cfl %g outside (0, 1]", cfl);
  }
  int rc = set_fields(c, std::numeric_limits<double>::infinity(), cfl);
  if (rc) return rc;
  rc = enqueue2(c, parity_now(c), (int)(c->launched % 3), dt_fixed, c->stream);
  if (rc) return rc;
  c->launched += 1;
  c->steps += 1;
  return WCC_OK;
}

int wcc2d_run(wcc2d_ctx* c, int64_t half_steps, double cfl) {
  if (!c) return WCC_EINVAL;
  if (!c->bound || !c->written) return fail2(c, WCC_ESTATE, "no state written");
  if (!cfl_ok(cfl) || half_steps < 0) return fail2(c, WCC_EINVAL, "bad cfl or step count");
  const int rc = set_fields(c, std::numeric_limits<double>::infinity(), cfl);
  if (rc) return rc;
  return run2(c, half_steps, true);
}

int wcc2d_advance(wcc2d_ctx* c, double t_end, double cfl, int64_t max_half_steps, int64_t* taken) {
  if (taken) *taken = 0;
  if (!c) return WCC_EINVAL;
  if (!c->bound || !c->written) return fail2(c, WCC_ESTATE, "no state written");
  if (!cfl_ok(cfl) || !std::isfinite(t_end)) return fail2(c, WCC_EINVAL, "bad cfl or t_end");
  Ctrl h;
  int rc = read_ctrl2(c, &h);
  if (rc) return rc;
  const int s0 = (int)(c->launched % 3);
  if (t_end < h.t[s0]) return fail2(c, WCC_EINVAL, "t_end %g before the current time %g", t_end, h.t[s0]);
  if (h.flags[s0]) return fail2(c, WCC_ENONFINITE, "state holds a flagged value; write a new state");
  rc = set_fields(c, t_end, cfl);
  if (rc) return rc;
  const int64_t start = c->steps;
  const int64_t cap = max_half_steps > 0 ? max_half_steps : std::numeric_limits<int64_t>::max();
  while (true) {
    const int64_t done = c->steps - start;
    if (done >= cap) break;
    const int64_t want = std::min<int64_t>(cap - done, kChunk2);
    rc = run2(c, want, false);
    if (rc) return rc;
    rc = read_ctrl2(c, &h);
    if (rc) return rc;
    const int s = (int)(c->launched % 3);
    if (h.flags[s]) {
      if (taken) *taken = c->steps - start;
      return fail2(c, WCC_ENONFINITE, "a half-step produced a non-finite value or a non-positive density/pressure");
    }
    if (!(h.t[s] < t_end)) break;
  }
  if (taken) *taken = c->steps - start;
  return WCC_OK;
}

int wcc2d_read_dofs(wcc2d_ctx* c, double* host, int64_t cap, wcc2d_state_info* info) {
  if (!c) return WCC_EINVAL;
  if (!c->bound || !c->written) return fail2(c, WCC_ESTATE, "no state written");
  Ctrl h;
  int rc = read_ctrl2(c, &h);
  if (rc) return rc;
  const int parity = parity_now(c);
  const size_t cells = (size_t)(mesh_nx(c, parity) * mesh_ny(c, parity));
  if (host) {
    if (cap < (int64_t)(c->nc * c->nd * cells)) return fail2(c, WCC_ESIZE, "host buffer too small");
    for (int r = 0; r < c->nc * c->nd; ++r)
      HIPCHK2(c, hipMemcpyAsync(host + (size_t)r * cells, c->q[parity] + (size_t)r * c->plane, cells * 8,
                                hipMemcpyDeviceToHost, c->stream));
    HIPCHK2(c, hipStreamSynchronize(c->stream));
  }
  if (info) {
    const int s = (int)(c->launched % 3);
    info->t = h.t[s];
    info->parity = parity;
    info->flags = (int32_t)h.flags[s];
    info->Nx = mesh_nx(c, parity);
    info->Ny = mesh_ny(c, parity);
    info->dx = dx_of(c);
    info->dy = dy_of(c);
    info->half_steps = c->steps;
    double sm;
    std::memcpy(&sm, &h.smax[s], 8);
    info->s_max = sm;
  }
  return WCC_OK;
}

int wcc2d_totals(wcc2d_ctx* c, double* per_component) {
  if (!c || !per_component) return WCC_EINVAL;
  wcc2d_state_info info;
  const size_t cap = (size_t)c->nc * c->nd * (size_t)(mesh_nx(c, 0) * mesh_ny(c, 0));
  std::vector<double> buf(cap);
  const int rc = wcc2d_read_dofs(c, buf.data(), (int64_t)cap, &info);
  if (rc) return rc;
  const int64_t cells = info.Nx * info.Ny;
  const int P = c->P, nd = c->nd;
  // cell average of the cell polynomial: the point value plus the even-even
  // moments, 1/((k+1)! 2^k (l+1)! 2^l) u_{kx,ly} (the quarter averages summed)
  std::vector<double> w(nd, 0.0);
  for (int n = 2; n <= P; ++n)
    for (int l = 0; l <= n; ++l) {
      const int k = n - l;
      if (k % 2 || l % 2) continue;
      double f = 1.0;
      for (int i = 2; i <= k + 1; ++i) f *= i;
      for (int i = 2; i <= l + 1; ++i) f *= i;
      w[(n * (n + 1)) / 2 + l] = 1.0 / (f * std::ldexp(1.0, k + l));
    }
  for (int cc = 0; cc < c->nc; ++cc) {
    double tot = 0.0;
    for (int64_t j = 0; j < cells; ++j) {
      double a = buf[(size_t)(cc * nd) * cells + j];
      for (int d = 1; d < nd; ++d)
        if (w[d] != 0.0) a += w[d] * buf[(size_t)(cc * nd + d) * cells + j];
      tot += a;
    }
    per_component[cc] = tot * info.dx * info.dy;
  }
  return WCC_OK;
}

int wcc2d_get_launch(wcc2d_ctx* c, int* threads_per_block, int* blocks, int* variant) {
  if (!c || !threads_per_block || !blocks || !variant) return WCC_EINVAL;
  *threads_per_block = c->threads;
  *blocks = blocks_for(c, parity_now(c));
  *variant = c->variant;
  return WCC_OK;
}

int wcc2d_set_launch(wcc2d_ctx* c, int threads_per_block, int blocks, int variant) {
  if (!c) return WCC_EINVAL;
  if (variant < -1 || variant > 3) return fail2(c, WCC_EINVAL, "variant must be -1 (keep), 0, 1, 2 or 3");
  if (threads_per_block != 0 && (threads_per_block % 64 != 0 || threads_per_block < 64 || threads_per_block > 256))
    return fail2(c, WCC_EINVAL, "threads per block must be 64, 128, 192 or 256");
  if (blocks < 0) return fail2(c, WCC_EINVAL, "negative block count");
  c->threads = threads_per_block ? threads_per_block : 256;
  c->blocks = blocks;
  if (variant >= 0) c->variant = variant;
  drop_graphs(c);
  return WCC_OK;
}

int wcc2d_last_run_ms(wcc2d_ctx* c, double* ms) {
  if (!c || !ms) return WCC_EINVAL;
  if (!c->ev0 || !c->ev1) return fail2(c, WCC_ESTATE, "no timed run");
  HIPCHK2(c, hipEventSynchronize(c->ev1));
  float f = 0.f;
  HIPCHK2(c, hipEventElapsedTime(&f, c->ev0, c->ev1));
  *ms = f;
  return WCC_OK;
}

const char* wcc2d_last_error(const wcc2d_ctx* c) { return c ? c->err.c_str() : "null context"; }

void wcc2d_destroy(wcc2d_ctx* c) {
  if (!c) return;
  drop_graphs(c);
  if (c->capture) (void)hipStreamDestroy(c->capture);
  if (c->ev0) (void)hipEventDestroy(c->ev0);
  if (c->ev1) (void)hipEventDestroy(c->ev1);
  delete c;
}

}  // extern "C"
