// wcc_api.hip -- host side of the C ABI declared in include/wcc.h.
//
// The context owns only host state: sizes, the layout of the caller's device
// workspace, the half-step counter and a small cache of instantiated HIP
// graphs.  Device memory and the stream come from the caller (wcc_bind).
//
// Workspace layout (all offsets 256-byte aligned):
//   [ctrl: Ctrl] [parts: 3 x 64 partial wave-speed maxima, 64 B apart]
//   [p0: nc*ld doubles]  [p1]  [d0: nc*P*ld R]  [d1]
// with ld = max cells per mesh rounded up to 64.  Buffer b holds the state
// of mesh parity b; a half-step reads buffer `parity` and writes the other.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <limits>
#include <map>
#include <mutex>
#include <string>
#include <vector>

#include "wcc.h"
#include "wcc_internal.hpp"
#include "wcc_ctrl.hpp"
#include "wcc_wide.hpp"

using wcc::Ctrl;
using wcc::StepArgs;

namespace {

constexpr int kChunk = 48;  // half-steps per captured graph (multiple of 6)
constexpr int kWideVariant = 4;  // launch variant: 128-cell wave tiles, two old cells per lane

inline size_t align256(size_t x) { return (x + 255) & ~size_t(255); }

// Linear stability limits of the unlimited scheme per degree (von Neumann
// analysis of the linear scheme, Table 2 / Appendix A).
constexpr double kLinearLimit[5] = {0.5, 0.5, 0.384, 0.2887, 0.2820};

}  // namespace

struct wcc_ctx {
  int eq = 0, P = 0, bc = 0, nc = 1;
  int64_t N = 0;
  wcc_params prm{};
  int64_t ld = 0;
  size_t elem = 8;  // bytes per derivative element
  // binding
  char* ws = nullptr;
  size_t ws_bytes = 0;
  hipStream_t stream = nullptr;
  Ctrl* ctrl = nullptr;
  unsigned long long* parts = nullptr;
  double* p[2] = {nullptr, nullptr};
  void* d[2] = {nullptr, nullptr};
  // host-side view of the march
  bool bound = false, written = false;
  int parity_w = 0;         // parity at the last write
  int64_t launched = 0;     // kernels enqueued since the write (slot = launched % 3)
  int64_t steps = 0;        // half-steps known to be done (exact after a sync)
  int threads = 256, blocks = 0;
  int default_blocks = 0;    // device-filling grid of the current shape (0: not computed yet)
  int prefetch = 1;          // kernel variant bits: 1 = prefetch the next tile's inputs, 2 = aligned stores
  int cu = 0;
  hipStream_t capture = nullptr;
  // captured chunks of kChunk half-steps from (slot, parity), key slot*2 + parity
  std::map<int, hipGraphExec_t> graphs;
  hipEvent_t ev0 = nullptr, ev1 = nullptr;
  double last_run_ms = 0.0;
  // t_end and cfl the device control block holds (valid while fields_known)
  bool fields_known = false;
  double known_t_end = 0.0, known_cfl = 0.0;
  std::string err;
  std::vector<float> stage;
  std::vector<unsigned long long> stage_zero;
};

namespace {

int fail(wcc_ctx* c, int code, const char* fmt, ...) {
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

#define HIPCHK(ctx, call)                                                                          \
  do {                                                                                             \
    hipError_t e_ = (call);                                                                        \
    if (e_ != hipSuccess) return fail((ctx), WCC_EDEVICE, "%s: %s", #call, hipGetErrorString(e_)); \
  } while (0)

int64_t ncells_of(const wcc_ctx* c, int parity) {
  if (c->bc == WCC_BC_PERIODIC) return c->N;
  return parity == 0 ? c->N + 1 : c->N;
}

double dx_of(const wcc_ctx* c) { return (c->prm.x_right - c->prm.x_left) / (double)c->N; }

template <class R>
wcc::Phys<R> phys_of(const wcc_ctx* c) {
  wcc::Phys<R> ph;
  ph.a = (R)c->prm.a;
  ph.gamma = (R)c->prm.gamma;
  ph.gm1 = (R)(c->prm.gamma - 1.0);
  ph.eps = (R)c->prm.eps;
  return ph;
}

// Device addresses a half-step works on: the time-control block, the
// partial wave-speed maxima and the two state buffers.
struct Lay {
  Ctrl* ctrl;
  unsigned long long* parts;
  double* p[2];
  void* d[2];
};

Lay bound_lay(const wcc_ctx* c) { return Lay{c->ctrl, c->parts, {c->p[0], c->p[1]}, {c->d[0], c->d[1]}}; }

// The state buffers inside a state region laid out as the workspace after its
// control block: [p0][p1][d0][d1].
void state_lay(const wcc_ctx* c, char* q, Lay& L) {
  const size_t pb = align256((size_t)c->nc * (size_t)c->ld * 8);
  const size_t db = align256((size_t)c->nc * (size_t)c->P * (size_t)c->ld * c->elem);
  L.p[0] = reinterpret_cast<double*>(q);
  q += pb;
  L.p[1] = reinterpret_cast<double*>(q);
  q += pb;
  L.d[0] = q;
  q += db;
  L.d[1] = q;
}

template <class R>
StepArgs<R> args_at(const wcc_ctx* c, const Lay& L, int parity, int slot, double dt_fixed) {
  StepArgs<R> a{};
  a.p_old = L.p[parity];
  a.d_old = static_cast<const R*>(L.d[parity]);
  a.p_new = L.p[1 - parity];
  a.d_new = static_cast<R*>(L.d[1 - parity]);
  a.ld = c->ld;
  a.n_old = ncells_of(c, parity);
  a.n_new = ncells_of(c, 1 - parity);
  a.N = c->N;
  a.parity_old = parity;
  a.bc = c->bc;
  a.dx = dx_of(c);
  a.dt_fixed = dt_fixed;
  a.ph = phys_of<R>(c);
  a.ctrl = L.ctrl;
  a.parts = L.parts;
  a.slot = slot;
  return a;
}

template <class R>
StepArgs<R> args_for(const wcc_ctx* c, int parity, int slot, double dt_fixed) {
  return args_at<R>(c, bound_lay(c), parity, slot, dt_fixed);
}

int blocks_for(wcc_ctx* c) {
  if (c->blocks > 0) return c->blocks;
  // the device-filling grid of the current shape, computed once (the
  // occupancy query costs host time on every launch otherwise)
  if (c->default_blocks > 0) return c->default_blocks;
  const bool wide = c->prefetch == kWideVariant;
  const int64_t span = wide ? 127 : 63;   // new cells per wave tile
  const int64_t tiles = (std::max(ncells_of(c, 0), ncells_of(c, 1)) + span - 1) / span;
  const int waves = c->threads / 64;
  int per_cu = 0;
  const bool lim = c->prm.limiter != 0;
  hipError_t e;
  if (wide)
    e = c->prm.precision == WCC_FP64 ? wcc::occupancy_half_step_wide<double>(c->eq, c->P, lim, c->threads, &per_cu)
                                     : wcc::occupancy_half_step_wide<float>(c->eq, c->P, lim, c->threads, &per_cu);
  else
    e = c->prm.precision == WCC_FP64
            ? wcc::occupancy_half_step<double>(c->eq, c->P, lim, c->prefetch, c->threads, &per_cu)
            : wcc::occupancy_half_step<float>(c->eq, c->P, lim, c->prefetch, c->threads, &per_cu);
  if (e != hipSuccess || per_cu < 1) per_cu = 1;
  int64_t full = (int64_t)per_cu * c->cu;
  int64_t need = (tiles + waves - 1) / waves;
  c->default_blocks = (int)std::max<int64_t>(1, std::min(full, need));
  return c->default_blocks;
}

// Enqueue one half-step kernel on the buffers of L: launch number `launched`
// -> slot and buffers.
int enqueue_step_at(wcc_ctx* c, const Lay& L, int parity, int slot, double dt_fixed, hipStream_t s) {
  const int blocks = blocks_for(c);
  hipError_t e;
  if (c->prefetch == kWideVariant) {
    if (c->prm.precision == WCC_FP64)
      e = wcc::launch_half_step_wide<double>(args_at<double>(c, L, parity, slot, dt_fixed), c->eq, c->P,
                                             c->prm.limiter != 0, blocks, c->threads, s);
    else
      e = wcc::launch_half_step_wide<float>(args_at<float>(c, L, parity, slot, dt_fixed), c->eq, c->P,
                                            c->prm.limiter != 0, blocks, c->threads, s);
  } else if (c->prm.precision == WCC_FP64)
    e = wcc::launch_half_step<double>(args_at<double>(c, L, parity, slot, dt_fixed), c->eq, c->P,
                                      c->prm.limiter != 0, c->prefetch, blocks, c->threads, s);
  else
    e = wcc::launch_half_step<float>(args_at<float>(c, L, parity, slot, dt_fixed), c->eq, c->P,
                                     c->prm.limiter != 0, c->prefetch, blocks, c->threads, s);
  if (e != hipSuccess) return fail(c, WCC_EDEVICE, "half-step launch: %s", hipGetErrorString(e));
  return WCC_OK;
}

int enqueue_step(wcc_ctx* c, int parity, int slot, double dt_fixed, hipStream_t s) {
  return enqueue_step_at(c, bound_lay(c), parity, slot, dt_fixed, s);
}

int current_parity(const wcc_ctx* c) { return (int)((c->parity_w + c->steps) & 1); }

void drop_graphs(wcc_ctx* c) {
  for (auto& kv : c->graphs) (void)hipGraphExecDestroy(kv.second);
  c->graphs.clear();
}

// Graph of kChunk consecutive half-steps starting at (slot0, parity0).
int chunk_graph(wcc_ctx* c, int slot0, int parity0, hipGraphExec_t* out) {
  const int len = kChunk;
  const int key = slot0 * 2 + parity0;
  auto it = c->graphs.find(key);
  if (it != c->graphs.end()) {
    *out = it->second;
    return WCC_OK;
  }
  if (!c->capture) HIPCHK(c, hipStreamCreateWithFlags(&c->capture, hipStreamNonBlocking));
  HIPCHK(c, hipStreamBeginCapture(c->capture, hipStreamCaptureModeThreadLocal));
  int rc = WCC_OK;
  for (int i = 0; i < len && rc == WCC_OK; ++i)
    rc = enqueue_step(c, (parity0 + i) & 1, (slot0 + i) % 3, 0.0, c->capture);
  hipGraph_t g = nullptr;
  hipError_t e = hipStreamEndCapture(c->capture, &g);
  if (rc != WCC_OK) {
    if (g) (void)hipGraphDestroy(g);
    return rc;
  }
  if (e != hipSuccess) return fail(c, WCC_EDEVICE, "graph capture: %s", hipGetErrorString(e));
  hipGraphExec_t ex = nullptr;
  e = hipGraphInstantiate(&ex, g, nullptr, nullptr, 0);
  (void)hipGraphDestroy(g);
  if (e != hipSuccess) return fail(c, WCC_EDEVICE, "graph instantiate: %s", hipGetErrorString(e));
  c->graphs[key] = ex;
  *out = ex;
  return WCC_OK;
}

int set_ctrl_fields(wcc_ctx* c, double t_end, double cfl) {
  // the device block already holds these values (set by this context since
  // the last write): no kernel needed
  if (c->fields_known && c->known_t_end == t_end && c->known_cfl == cfl) return WCC_OK;
  HIPCHK(c, wcc::launch_set_fields(c->ctrl, t_end, cfl, c->stream));
  c->fields_known = true;
  c->known_t_end = t_end;
  c->known_cfl = cfl;
  return WCC_OK;
}

// Read the control block (synchronising the stream); smax[slot] of the copy
// is replaced by the max of the slot's partial entries.
int read_ctrl(wcc_ctx* c, Ctrl* h) {
  static_assert(wcc::kSmaxPartsBytes % 256 == 0, "parts region size");
  std::vector<unsigned long long> parts(wcc::kSmaxPartsBytes / sizeof(unsigned long long));
  HIPCHK(c, hipMemcpyAsync(h, c->ctrl, sizeof(Ctrl), hipMemcpyDeviceToHost, c->stream));
  HIPCHK(c, hipMemcpyAsync(parts.data(), c->parts, wcc::kSmaxPartsBytes, hipMemcpyDeviceToHost, c->stream));
  HIPCHK(c, hipStreamSynchronize(c->stream));
  for (int s = 0; s < 3; ++s) {
    unsigned long long m = 0;
    for (int i = 0; i < wcc::kSmaxParts; ++i) m = std::max(m, parts[(size_t)(s * wcc::kSmaxParts + i) * wcc::kSmaxStride]);
    h->smax[s] = m;
  }
  c->steps = h->steps_done;
  return WCC_OK;
}

bool check_cfl(double cfl) { return cfl > 0.0 && cfl <= 1.0 && std::isfinite(cfl); }

// ---------------------------------------------------------------------------
// Static device scratch of wcc_run_noalloc: the time-control block and the
// partial wave-speed maxima of one run, in a file-scope device array instead
// of the caller's workspace.  Every GPU the library runs on holds its own copy
// until the process ends.  Host code never uses the array's name as an
// address: the device address is looked up once per device with
// hipGetSymbolAddress (with that device current) and kept per device.
// ---------------------------------------------------------------------------
static_assert(256 + wcc::kSmaxPartsBytes == WCC_WORKSPACE_STATE_OFFSET, "state offset of the workspace");
static_assert(sizeof(Ctrl) <= 256, "control block fits its 256-byte slot");
static_assert(WCC_WORKSPACE_STATE_OFFSET <= WCC_NOALLOC_SCRATCH_BYTES, "scratch holds control block and parts");

static __device__ __align__(256) unsigned char scratch[WCC_NOALLOC_SCRATCH_BYTES];

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
char* g_scratch_ptr[kMaxDevices] = {};

// Device address of this device's scratch array (device `dev` current).
int scratch_of(wcc_ctx* c, int dev, char** out) {
  if (dev < 0 || dev >= kMaxDevices) return fail(c, WCC_EDEVICE, "device %d outside the scratch table", dev);
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void* ptr = nullptr;
    const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !ptr)
      return fail(c, WCC_EDEVICE, "hipGetSymbolAddress(scratch): %s", hipGetErrorString(e));
    g_scratch_ptr[dev] = static_cast<char*>(ptr);
  }
  *out = g_scratch_ptr[dev];
  return WCC_OK;
}

}  // namespace

extern "C" {

int wcc_run_noalloc(wcc_ctx* c, void* state, size_t bytes, int parity, double t, int64_t half_steps, double cfl,
                    void* hip_stream, double* t_out) {
  if (!c) return WCC_EINVAL;
  if (!state || ((uintptr_t)state & 255u) != 0) return fail(c, WCC_EINVAL, "state must be a 256-byte aligned device pointer");
  if ((parity != 0 && parity != 1) || !std::isfinite(t) || half_steps < 0 || !check_cfl(cfl))
    return fail(c, WCC_EINVAL, "bad parity, time, step count or cfl");
  size_t ws = 0;
  wcc_workspace_bytes(c, &ws);
  const size_t need = ws - WCC_WORKSPACE_STATE_OFFSET;
  if (bytes < need) return fail(c, WCC_ESIZE, "state region of %zu bytes, need %zu", bytes, need);
  // the scratch a run needs (control block + partial maxima) does not depend
  // on the problem size; refuse anything that would not fit the array
  const size_t scratch_need = WCC_WORKSPACE_STATE_OFFSET;
  if (scratch_need > WCC_NOALLOC_SCRATCH_BYTES)
    return fail(c, WCC_ESIZE, "run needs %zu scratch bytes, the static array holds %d", scratch_need,
                WCC_NOALLOC_SCRATCH_BYTES);
  int dev = 0;
  HIPCHK(c, hipGetDevice(&dev));
  char* sp = nullptr;
  int rc = scratch_of(c, dev, &sp);
  if (rc) return rc;
  hipStream_t s = static_cast<hipStream_t>(hip_stream);
  Lay L;
  L.ctrl = reinterpret_cast<Ctrl*>(sp);
  L.parts = reinterpret_cast<unsigned long long*>(sp + 256);
  state_lay(c, static_cast<char*>(state), L);
  // time ring and partial maxima from scratch (they keep the last call's contents)
  wcc::RingInit init{};
  init.t = t;
  init.cfl = cfl;
  for (int i = 0; i < 3; ++i) {
    init.ghost[0][i] = c->prm.left_state[i];
    init.ghost[1][i] = c->prm.right_state[i];
  }
  HIPCHK(c, wcc::launch_init_ring(L.ctrl, L.parts, init, s));
  // wave speed of the input state into slot 0, as wcc_write_dofs does
  const int64_t n = ncells_of(c, parity);
  const int blocks = (int)std::min<int64_t>((n + 255) / 256, 4LL * c->cu);
  hipError_t e;
  if (c->prm.precision == WCC_FP64) {
    StepArgs<double> a = args_at<double>(c, L, parity, 0, 0.0);
    a.n_old = n;
    e = wcc::launch_state_speed<double>(a, c->eq, c->P, blocks, s);
  } else {
    StepArgs<float> a = args_at<float>(c, L, parity, 0, 0.0);
    a.n_old = n;
    e = wcc::launch_state_speed<float>(a, c->eq, c->P, blocks, s);
  }
  if (e != hipSuccess) return fail(c, WCC_EDEVICE, "speed kernel: %s", hipGetErrorString(e));
  for (int64_t i = 0; i < half_steps; ++i) {
    rc = enqueue_step_at(c, L, (int)((parity + i) & 1), (int)(i % 3), 0.0, s);
    if (rc) return rc;
  }
  if (t_out) {
    Ctrl h;
    HIPCHK(c, hipMemcpyAsync(&h, L.ctrl, sizeof h, hipMemcpyDeviceToHost, s));
    HIPCHK(c, hipStreamSynchronize(s));
    const int slot = (int)(half_steps % 3);
    *t_out = h.t[slot];
    if (h.flags[slot] & 3u) return fail(c, WCC_ENONFINITE, "a half-step produced a non-finite value or a "
                                                          "non-positive density/pressure");
  }
  return WCC_OK;
}

int wcc_params_default(wcc_params* p) {
  if (!p) return WCC_EINVAL;
  std::memset(p, 0, sizeof *p);
  p->x_left = 0.0;
  p->x_right = 1.0;
  p->a = 1.0;
  p->gamma = 1.4;
  p->eps = 1e-40;
  p->limiter = 1;
  p->precision = WCC_FP64;
  return WCC_OK;
}

int wcc_create(int equation, int P, int64_t N, int bc, const wcc_params* params, wcc_ctx** out) {
  if (!out) return WCC_EINVAL;
  *out = nullptr;
  if (equation < WCC_ADVECTION || equation > WCC_EULER) return WCC_EINVAL;
  if (P < 0 || P > WCC_PMAX || N < 2 || bc < WCC_BC_PERIODIC || bc > WCC_BC_DIRICHLET) return WCC_EINVAL;
  wcc_params prm;
  if (params) prm = *params; else wcc_params_default(&prm);
  if (!(prm.x_right > prm.x_left) || !(prm.eps >= 0.0)) return WCC_EINVAL;
  if (prm.precision != WCC_FP64 && prm.precision != WCC_FP32_MIXED) return WCC_EINVAL;
  if (equation == WCC_EULER && !(prm.gamma > 1.0)) return WCC_EINVAL;
  // rows are addressed with 32-bit byte offsets: ld * 8 bytes < 4 GiB
  if (N > ((int64_t)1 << 28)) return WCC_EINVAL;
  wcc_ctx* c = new wcc_ctx();
  c->eq = equation;
  c->P = P;
  c->N = N;
  c->bc = bc;
  c->nc = equation == WCC_EULER ? 3 : 1;
  c->prm = prm;
  c->elem = prm.precision == WCC_FP64 ? 8 : 4;
  const int64_t nmax = std::max(ncells_of(c, 0), ncells_of(c, 1));
  c->ld = (nmax + 63) / 64 * 64;
  // Default kernel variant by state size (measured on MI355X, P = 3 and 4,
  // both precisions): once the two state buffers outgrow the 256 MB Infinity
  // Cache by about a factor two, the staged stores with prefetch are fastest
  // (the crossover lies between 0.50 and 0.60 GB); below, prefetch alone.
  const double state_bytes = 2.0 * (double)c->nc * (double)c->ld * (8.0 + (double)(c->P * c->elem));
  c->prefetch = state_bytes > 512.0 * 1048576.0 ? 3 : 1;
  int dev = 0;
  if (hipGetDevice(&dev) == hipSuccess) {
    hipDeviceProp_t prop;
    if (hipGetDeviceProperties(&prop, dev) == hipSuccess) c->cu = prop.multiProcessorCount;
  }
  if (c->cu <= 0) c->cu = 256;
  *out = c;
  return WCC_OK;
}

int wcc_workspace_bytes(const wcc_ctx* c, size_t* bytes) {
  if (!c || !bytes) return WCC_EINVAL;
  const size_t pb = align256((size_t)c->nc * (size_t)c->ld * 8);
  const size_t db = align256((size_t)c->nc * (size_t)c->P * (size_t)c->ld * c->elem);
  *bytes = align256(sizeof(Ctrl)) + wcc::kSmaxPartsBytes + 2 * pb + 2 * db;
  return WCC_OK;
}

int wcc_bind(wcc_ctx* c, void* dev_ptr, size_t bytes, void* hip_stream) {
  if (!c || !dev_ptr) return WCC_EINVAL;
  if (((uintptr_t)dev_ptr & 255u) != 0) return fail(c, WCC_EINVAL, "workspace must be 256-byte aligned");
  size_t need = 0;
  wcc_workspace_bytes(c, &need);
  if (bytes < need) return fail(c, WCC_ESIZE, "workspace of %zu bytes, need %zu", bytes, need);
  drop_graphs(c);
  c->ws = static_cast<char*>(dev_ptr);
  c->ws_bytes = bytes;
  c->stream = static_cast<hipStream_t>(hip_stream);
  const size_t pb = align256((size_t)c->nc * (size_t)c->ld * 8);
  const size_t db = align256((size_t)c->nc * (size_t)c->P * (size_t)c->ld * c->elem);
  char* q = c->ws;
  c->ctrl = reinterpret_cast<Ctrl*>(q);
  q += align256(sizeof(Ctrl));
  c->parts = reinterpret_cast<unsigned long long*>(q);
  q += wcc::kSmaxPartsBytes;
  c->p[0] = reinterpret_cast<double*>(q);
  q += pb;
  c->p[1] = reinterpret_cast<double*>(q);
  q += pb;
  c->d[0] = q;
  q += db;
  c->d[1] = q;
  c->bound = true;
  c->written = false;
  c->fields_known = false;
  return WCC_OK;
}

int wcc_write_dofs(wcc_ctx* c, const double* host, int64_t n_cells, int parity, double t) {
  if (!c) return WCC_EINVAL;
  if (!c->bound) return fail(c, WCC_ESTATE, "wcc_write_dofs before wcc_bind");
  if (!host || (parity != 0 && parity != 1) || !std::isfinite(t)) return fail(c, WCC_EINVAL, "bad arguments");
  const int64_t n = ncells_of(c, parity);
  if (n_cells != n) return fail(c, WCC_ESIZE, "n_cells %lld, mesh of parity %d has %lld", (long long)n_cells, parity,
                                (long long)n);
  const int P = c->P, nc = c->nc;
  // point values
  for (int cc = 0; cc < nc; ++cc)
    HIPCHK(c, hipMemcpyAsync(c->p[parity] + (size_t)cc * c->ld, host + (size_t)(cc * (P + 1)) * n, n * 8,
                             hipMemcpyHostToDevice, c->stream));
  // derivatives
  if (P > 0) {
    char* dbase = static_cast<char*>(c->d[parity]);
    if (c->prm.precision == WCC_FP64) {
      for (int cc = 0; cc < nc; ++cc)
        for (int k = 1; k <= P; ++k)
          HIPCHK(c, hipMemcpyAsync(dbase + ((size_t)(cc * P + k - 1) * c->ld) * 8,
                                   host + (size_t)(cc * (P + 1) + k) * n, n * 8, hipMemcpyHostToDevice, c->stream));
    } else {
      c->stage.resize((size_t)nc * P * n);
      for (int cc = 0; cc < nc; ++cc)
        for (int k = 1; k <= P; ++k) {
          const double* src = host + (size_t)(cc * (P + 1) + k) * n;
          float* dst = c->stage.data() + (size_t)(cc * P + k - 1) * n;
          for (int64_t j = 0; j < n; ++j) dst[j] = (float)src[j];
        }
      for (int r = 0; r < nc * P; ++r)
        HIPCHK(c, hipMemcpyAsync(dbase + ((size_t)r * c->ld) * 4, c->stage.data() + (size_t)r * n, n * 4,
                                 hipMemcpyHostToDevice, c->stream));
    }
  }
  // control block: time in slot 0, everything else cleared
  Ctrl h;
  std::memset(&h, 0, sizeof h);
  h.t[0] = h.t[1] = h.t[2] = t;
  h.t_end = std::numeric_limits<double>::infinity();
  h.cfl = 0.0;
  for (int i = 0; i < 3; ++i) {
    h.ghost[0][i] = c->prm.left_state[i];
    h.ghost[1][i] = c->prm.right_state[i];
  }
  HIPCHK(c, hipMemcpyAsync(c->ctrl, &h, sizeof h, hipMemcpyHostToDevice, c->stream));
  c->fields_known = false;
  c->stage_zero.assign(wcc::kSmaxPartsBytes / sizeof(unsigned long long), 0ull);
  HIPCHK(c, hipMemcpyAsync(c->parts, c->stage_zero.data(), wcc::kSmaxPartsBytes, hipMemcpyHostToDevice, c->stream));
  // wave speed of the written state into slot 0
  hipError_t e;
  const int blocks = (int)std::min<int64_t>((n + 255) / 256, 4LL * c->cu);
  if (c->prm.precision == WCC_FP64) {
    StepArgs<double> a = args_for<double>(c, parity, 0, 0.0);
    a.n_old = n;
    e = wcc::launch_state_speed<double>(a, c->eq, P, blocks, c->stream);
  } else {
    StepArgs<float> a = args_for<float>(c, parity, 0, 0.0);
    a.n_old = n;
    e = wcc::launch_state_speed<float>(a, c->eq, P, blocks, c->stream);
  }
  if (e != hipSuccess) return fail(c, WCC_EDEVICE, "speed kernel: %s", hipGetErrorString(e));
  Ctrl back;
  int rc0 = read_ctrl(c, &back);
  if (rc0) return rc0;
  c->written = true;
  c->parity_w = parity;
  c->launched = 0;
  c->steps = 0;
  if (back.flags[0]) return fail(c, WCC_ENONFINITE, "written state holds a non-finite value");
  return WCC_OK;
}

int wcc_step(wcc_ctx* c, double cfl, double dt_fixed) {
  if (!c) return WCC_EINVAL;
  if (!c->bound || !c->written) return fail(c, WCC_ESTATE, "no state written");
  if (dt_fixed > 0.0) {
    if (!std::isfinite(dt_fixed)) return fail(c, WCC_EINVAL, "bad dt");
  } else if (!check_cfl(cfl)) {
    return fail(c, WCC_EINVAL, "cfl %g outside (0, 1]", cfl);
  }
  int rc = set_ctrl_fields(c, std::numeric_limits<double>::infinity(), cfl);
  if (rc) return rc;
  rc = enqueue_step(c, current_parity(c), (int)(c->launched % 3), dt_fixed, c->stream);
  if (rc) return rc;
  c->launched += 1;
  c->steps += 1;
  return WCC_OK;
}

static int run_chunks(wcc_ctx* c, int64_t n, bool timed) {
  // Build every chunk graph a run can start on before the first one is
  // needed, so that no capture or instantiation falls between the events.
  // The remainder of a run (fewer than kChunk half-steps) is launched kernel
  // by kernel: submitting a graph costs host time before its first kernel
  // starts, which a short run cannot hide behind earlier work (measured:
  // a 20-half-step run took ~5 us per half-step more as one graph than as 20
  // launches).
  if (n >= kChunk) {
    for (int key = 0; key < 6; ++key) {
      hipGraphExec_t g;
      const int rc = chunk_graph(c, key / 2, key % 2, &g);
      if (rc) return rc;
    }
  }
  if (timed) {
    if (!c->ev0) HIPCHK(c, hipEventCreate(&c->ev0));
    if (!c->ev1) HIPCHK(c, hipEventCreate(&c->ev1));
    HIPCHK(c, hipEventRecord(c->ev0, c->stream));
  }
  int64_t left = n;
  while (left > 0) {
    const int slot = (int)(c->launched % 3), par = current_parity(c);
    if (left >= kChunk) {
      hipGraphExec_t g;
      int rc = chunk_graph(c, slot, par, &g);
      if (rc) return rc;
      HIPCHK(c, hipGraphLaunch(g, c->stream));
      c->launched += kChunk;
      c->steps += kChunk;
      left -= kChunk;
    } else {
      int rc = enqueue_step(c, par, slot, 0.0, c->stream);
      if (rc) return rc;
      c->launched += 1;
      c->steps += 1;
      left -= 1;
    }
  }
  if (timed) HIPCHK(c, hipEventRecord(c->ev1, c->stream));
  return WCC_OK;
}

int wcc_run(wcc_ctx* c, int64_t half_steps, double cfl) {
  if (!c) return WCC_EINVAL;
  if (!c->bound || !c->written) return fail(c, WCC_ESTATE, "no state written");
  if (!check_cfl(cfl) || half_steps < 0) return fail(c, WCC_EINVAL, "bad cfl or step count");
  int rc = set_ctrl_fields(c, std::numeric_limits<double>::infinity(), cfl);
  if (rc) return rc;
  rc = run_chunks(c, half_steps, true);
  if (rc) return rc;
  c->last_run_ms = -1.0;
  return WCC_OK;
}

int wcc_last_run_ms(wcc_ctx* c, double* ms) {
  if (!c || !ms) return WCC_EINVAL;
  if (!c->ev0 || !c->ev1) return fail(c, WCC_ESTATE, "no timed run");
  HIPCHK(c, hipEventSynchronize(c->ev1));
  float f = 0.f;
  HIPCHK(c, hipEventElapsedTime(&f, c->ev0, c->ev1));
  *ms = f;
  return WCC_OK;
}

int wcc_advance(wcc_ctx* c, double t_end, double cfl, int64_t max_half_steps, int64_t* taken) {
  if (taken) *taken = 0;
  if (!c) return WCC_EINVAL;
  if (!c->bound || !c->written) return fail(c, WCC_ESTATE, "no state written");
  if (!check_cfl(cfl) || !std::isfinite(t_end)) return fail(c, WCC_EINVAL, "bad cfl or t_end");
  Ctrl h;
  int rc = read_ctrl(c, &h);
  if (rc) return rc;
  const int s0 = (int)(c->launched % 3);
  if (t_end < h.t[s0]) return fail(c, WCC_EINVAL, "t_end %g before the current time %g", t_end, h.t[s0]);
  if (h.flags[s0]) return fail(c, WCC_ENONFINITE, "state holds a flagged value; write a new state");
  rc = set_ctrl_fields(c, t_end, cfl);
  if (rc) return rc;
  const int64_t start = c->steps;
  const int64_t cap = max_half_steps > 0 ? max_half_steps : std::numeric_limits<int64_t>::max();
  while (true) {
    const int64_t done = c->steps - start;
    if (done >= cap) break;
    const int64_t want = std::min<int64_t>(cap - done, kChunk);
    rc = run_chunks(c, want >= kChunk ? kChunk : want, false);
    if (rc) return rc;
    rc = read_ctrl(c, &h);  // sets c->steps from the device
    if (rc) return rc;
    const int s = (int)(c->launched % 3);
    if (h.flags[s]) {
      if (taken) *taken = c->steps - start;
      return fail(c, WCC_ENONFINITE, "a half-step produced a non-finite value or a non-positive density/pressure");
    }
    if (!(h.t[s] < t_end)) break;
  }
  if (taken) *taken = c->steps - start;
  return WCC_OK;
}

int wcc_read_dofs(wcc_ctx* c, double* host, int64_t cap, wcc_state_info* info) {
  if (!c) return WCC_EINVAL;
  if (!c->bound || !c->written) return fail(c, WCC_ESTATE, "no state written");
  Ctrl h;
  int rc = read_ctrl(c, &h);
  if (rc) return rc;
  const int parity = current_parity(c);
  const int64_t n = ncells_of(c, parity);
  const int P = c->P, nc = c->nc;
  if (host) {
    if (cap < (int64_t)nc * (P + 1) * n) return fail(c, WCC_ESIZE, "host buffer too small");
    for (int cc = 0; cc < nc; ++cc)
      HIPCHK(c, hipMemcpyAsync(host + (size_t)(cc * (P + 1)) * n, c->p[parity] + (size_t)cc * c->ld, n * 8,
                               hipMemcpyDeviceToHost, c->stream));
    if (P > 0) {
      const char* dbase = static_cast<const char*>(c->d[parity]);
      if (c->prm.precision == WCC_FP64) {
        for (int cc = 0; cc < nc; ++cc)
          for (int k = 1; k <= P; ++k)
            HIPCHK(c, hipMemcpyAsync(host + (size_t)(cc * (P + 1) + k) * n,
                                     dbase + ((size_t)(cc * P + k - 1) * c->ld) * 8, n * 8, hipMemcpyDeviceToHost,
                                     c->stream));
      } else {
        c->stage.resize((size_t)nc * P * n);
        for (int r = 0; r < nc * P; ++r)
          HIPCHK(c, hipMemcpyAsync(c->stage.data() + (size_t)r * n, dbase + ((size_t)r * c->ld) * 4, n * 4,
                                   hipMemcpyDeviceToHost, c->stream));
      }
    }
    HIPCHK(c, hipStreamSynchronize(c->stream));
    if (P > 0 && c->prm.precision != WCC_FP64)
      for (int cc = 0; cc < nc; ++cc)
        for (int k = 1; k <= P; ++k) {
          const float* src = c->stage.data() + (size_t)(cc * P + k - 1) * n;
          double* dst = host + (size_t)(cc * (P + 1) + k) * n;
          for (int64_t j = 0; j < n; ++j) dst[j] = (double)src[j];
        }
  }
  if (info) {
    const int s = (int)(c->launched % 3);
    info->t = h.t[s];
    info->parity = parity;
    info->flags = (int32_t)h.flags[s];
    info->n_cells = n;
    info->dx = dx_of(c);
    info->x_first_center = c->prm.x_left + 0.5 * (double)parity * info->dx;
    info->half_steps = c->steps;
    unsigned long long bits = h.smax[s];
    double sm;
    std::memcpy(&sm, &bits, 8);
    info->s_max = sm;
    if (h.cfl > kLinearLimit[c->P] * (1.0 + 1e-12)) info->flags |= 4;
  }
  return WCC_OK;
}

int wcc_totals(wcc_ctx* c, double* per_component) {
  if (!c || !per_component) return WCC_EINVAL;
  wcc_state_info info;
  const int64_t n = std::max(ncells_of(c, 0), ncells_of(c, 1));
  std::vector<double> buf((size_t)c->nc * (c->P + 1) * n);
  int rc = wcc_read_dofs(c, buf.data(), (int64_t)buf.size(), &info);
  if (rc) return rc;
  const int64_t m = info.n_cells;
  const int P = c->P;
  for (int cc = 0; cc < c->nc; ++cc) {
    double tot = 0.0;
    for (int64_t j = 0; j < m; ++j) {
      // cell average of the cell polynomial (Eq. SubEq:1DCellAVG)
      double s = buf[(size_t)(cc * (P + 1)) * m + j];
      double fk = 1.0;
      for (int k = 1; k <= P; ++k) {
        fk *= (double)(k + 1);
        if (k % 2 == 0) s += buf[(size_t)(cc * (P + 1) + k) * m + j] / (fk * std::ldexp(1.0, k));
      }
      tot += s;
    }
    per_component[cc] = tot * info.dx;
  }
  return WCC_OK;
}

int wcc_get_launch(const wcc_ctx* c, int* threads_per_block, int* blocks, int* variant) {
  if (!c || !threads_per_block || !blocks || !variant) return WCC_EINVAL;
  *threads_per_block = c->threads;
  *blocks = c->blocks;
  *variant = c->prefetch;
  return WCC_OK;
}

int wcc_set_launch(wcc_ctx* c, int threads_per_block, int blocks, int variant) {
  if (!c) return WCC_EINVAL;
  if (variant < -1 || variant > kWideVariant) return fail(c, WCC_EINVAL, "variant must be -1 (keep) or 0..4");
  if (variant >= 0) {
    c->prefetch = variant;
    c->default_blocks = 0;
  }
  if (threads_per_block != 0 && (threads_per_block % 64 != 0 || threads_per_block < 64 || threads_per_block > 256))
    return fail(c, WCC_EINVAL, "threads per block must be 64, 128, 192 or 256");
  if (blocks < 0) return fail(c, WCC_EINVAL, "negative block count");
  c->threads = threads_per_block ? threads_per_block : 256;
  c->blocks = blocks;
  c->default_blocks = 0;
  drop_graphs(c);
  return WCC_OK;
}

const char* wcc_strerror(int code) {
  switch (code) {
    case WCC_OK: return "ok";
    case WCC_EINVAL: return "invalid argument";
    case WCC_ESTATE: return "call out of order (not bound or no state written)";
    case WCC_ESIZE: return "buffer too small or size mismatch";
    case WCC_EDEVICE: return "HIP runtime error";
    case WCC_ENONFINITE: return "non-finite value or non-positive density/pressure";
  }
  return "unknown error code";
}

const char* wcc_last_error(const wcc_ctx* c) { return c ? c->err.c_str() : "null context"; }

void wcc_destroy(wcc_ctx* c) {
  if (!c) return;
  drop_graphs(c);
  if (c->capture) (void)hipStreamDestroy(c->capture);
  if (c->ev0) (void)hipEventDestroy(c->ev0);
  if (c->ev1) (void)hipEventDestroy(c->ev1);
  delete c;
}

}  // extern "C"
