/* wcc.h -- C ABI of the MI355X (gfx950) library for the explicit half-step of
 * the 1D weighted compact central (WCC) schemes of Shen & Parsani,
 * "A class of high-order weighted compact central schemes for solving
 * hyperbolic conservation laws" (arXiv:2104.04347).
 *
 * The library advances u_t + f(u)_x = 0 on [x_left, x_right] with initial
 * data u0 and boundary values (problem statement, Eq. 1DHCL; for systems
 * Eq. 1DHCLSystem) on the two space-time staggered meshes of Section 2.1.
 * One half-step (t^n -> t^{n+1/2}) is one fused GPU kernel that runs the
 * Cauchy-Kovalewski expansion (Eq. 1DCauchy_Kovalewski), the Riemann-solver
 * free finite-volume update of the cell average (Eq. SubEq:1DIntegral with
 * Eq. Cal1DFlux, SubEq:1DCellAVGR, SubEq:1DCellAVGL), the central-difference
 * update of the derivatives (Eq. SubEq:Cal_1D_Derivatives_3 with
 * SubEq:Cal_1D_Derivatives_4) and the WENO-type limiter (Section 2.2; for
 * the Euler equations in characteristic variables, Section 4).
 *
 * Conventions shared by every call
 * --------------------------------
 * - Every call returns int: WCC_OK (0) or a negative WCC_E* code.  Nothing
 *   throws across the ABI.  wcc_strerror names a code; wcc_last_error gives
 *   the last detailed message of a context.
 * - State layout at the boundary: a host array of doubles indexed
 *   [c][k][j] = host[(c*(P+1) + k)*n_cells + j] with c the component
 *   (1 for scalars; rho, rho*u, rho*e for Euler), k = 0 the point value u at
 *   the cell centre and k >= 1 the scaled derivative
 *   u_kx = dx^k d^k u/dx^k at the centre (Eq. 1D_Derivative_DEF,
 *   Eq. 1DPolynomial_Space; the vector q of Eq. 1DSchemeMatrixForm).
 *   k = 0 is the POINT VALUE, not the cell average: the scheme's own state
 *   vector q (Eq. 1DSchemeMatrixForm, the matrices of Appendix A act on it)
 *   is what the library stores and exchanges, so that a written state is
 *   advanced without a conversion that would round it.  The cell average is
 *   ubar = u + sum_{k even >= 2} u_kx / ((k+1)! 2^k) (Eq. SubEq:1DCellAVG);
 *   wcc_totals returns its sums.
 * - Meshes (Section 2.1): dx = (x_right-x_left)/N.  Parity 0 is the original
 *   mesh, parity 1 the staggered one.  Periodic: N cells on both, centres
 *   x_left + (j + parity/2) dx.  Otherwise the original mesh has the N+1
 *   cells centred at x_left + j dx (j = 0..N) and the staggered mesh the N
 *   cells centred at x_left + (j+1/2) dx.
 * - Time step: the CFL number cfl is nu = max wave speed * dt / dx with dt the
 *   HALF-step (t^{n+1/2} - t^n).  dt = (cfl*dx)/s_max with s_max the largest
 *   wave speed (|a|, |u| or |u|+c) over the cell averages of the current state,
 *   computed on the device; the step that would pass t_end is clipped to it.
 * - Precision: WCC_FP64 computes everything in binary64 with a fixed,
 *   documented operation order (no contraction); WCC_FP32_MIXED keeps the
 *   point value / cell-average arithmetic in binary64 and runs the expansion,
 *   the derivatives and the limiter in binary32 (derivatives stored as
 *   float; the boundary still speaks doubles and rounds on write).
 * - Ownership: device memory and the HIP stream belong to the caller and are
 *   handed over with wcc_bind / wcc_batch_bind; the library never frees them.
 *   Host buffers stay the caller's; reads and writes copy synchronously on
 *   the bound stream.  wcc_destroy frees host-side state, graphs and the
 *   library's own capture stream.  A context is not thread-safe; separate
 *   contexts are independent.
 * - Stream order: wcc_step and wcc_run only enqueue work; wcc_advance,
 *   wcc_read_dofs, wcc_write_dofs and wcc_totals synchronise the bound
 *   stream.
 */
#ifndef WCC_H
#define WCC_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define WCC_OK 0
#define WCC_EINVAL (-1)      /* bad argument: P outside [0, WCC_PMAX], N < 2, bad enum, cfl outside (0, 1], t_end < t, ... */
#define WCC_ESTATE (-2)      /* call out of order: not bound, or no state written yet */
#define WCC_ESIZE (-3)       /* a buffer is smaller than required */
#define WCC_EDEVICE (-4)     /* a HIP runtime call failed; wcc_last_error has its message */
#define WCC_ENONFINITE (-5)  /* a non-finite value or rho <= 0 / p <= 0 appeared; the state is kept for
                                inspection and further steps do nothing until the next write */

#define WCC_PMAX 4

enum { WCC_ADVECTION = 0, WCC_BURGERS = 1, WCC_EULER = 2 };        /* f = a u ; u^2/2 ; 1D Euler (Section 5.2) */
enum { WCC_BC_PERIODIC = 0, WCC_BC_TRANSMISSIVE = 1, WCC_BC_DIRICHLET = 2 };
enum { WCC_FP64 = 0, WCC_FP32_MIXED = 1 };

typedef struct wcc_ctx wcc_ctx;       /* opaque, host side */
typedef struct wcc_batch wcc_batch;   /* opaque, host side */

typedef struct {
  double x_left, x_right;        /* domain; default [0, 1] */
  double a;                      /* advection speed (default 1) */
  double gamma;                  /* ratio of specific heats (default 1.4, Section 5.2) */
  double eps;                    /* limiter epsilon (default 1e-40, Eq. 1D2ndOrderWeights) */
  int32_t limiter;               /* 1: apply the limiter (P >= 1), 0: linear scheme */
  int32_t precision;             /* WCC_FP64 or WCC_FP32_MIXED */
  double left_state[3];          /* Dirichlet ghost states, conserved variables */
  double right_state[3];
} wcc_params;

typedef struct {
  double t;                      /* current time */
  int32_t parity;                /* mesh of the current state (0 original, 1 staggered) */
  int32_t flags;                 /* bit 0: non-finite value, bit 1: rho <= 0 or p <= 0, bit 2: cfl above the linear limit */
  int64_t n_cells;               /* cells on the current mesh */
  double x_first_center;         /* centre of cell 0 */
  double dx;
  int64_t half_steps;            /* half-steps taken since the last wcc_write_dofs */
  double s_max;                  /* largest wave speed of the current state */
} wcc_state_info;

/* Fill *p with the defaults listed above: the unit interval, a = 1, the
 * gamma = 1.4 of the paper's Euler experiments (Section 5.2) and the limiter
 * epsilon 1e-40 that follows Eq. 1D2ndOrderWeights.  Returns WCC_EINVAL for
 * p == NULL. */
int wcc_params_default(wcc_params* p);

/* Create a context for the problem of Eq. 1DHCL (scalar) or Eq. 1DHCLSystem
 * (Euler): `equation` (WCC_ADVECTION/BURGERS/EULER), degree P in
 * [0, WCC_PMAX] of the cell polynomial of Eq. 1DPolynomial_Space (scheme
 * order P+1), N >= 2 mesh intervals of the mesh of Section 2.1 and boundary
 * condition bc.  params may be NULL (defaults).  On success *out owns a new
 * host-side context (free with wcc_destroy); nothing is allocated on the
 * device.  Errors: WCC_EINVAL (bad enum, P, N, domain, gamma <= 1 for Euler,
 * N > 2^28). */
int wcc_create(int equation, int P, int64_t N, int bc, const wcc_params* params, wcc_ctx** out);

/* Device bytes the caller must provide to wcc_bind: the two ping-pong state
 * buffers of the staggered meshes of Section 2.1 (structure of arrays, rows
 * padded to 64 cells) and the control block of the CFL time step (Section 5
 * preamble).  Errors: WCC_EINVAL for NULL arguments. */
int wcc_workspace_bytes(const wcc_ctx* ctx, size_t* bytes);

/* Hand over device memory (dev_ptr, at least wcc_workspace_bytes bytes,
 * 256-byte aligned; owned by the caller, never freed by the library) and the
 * HIP stream (hipStream_t as void*, NULL = the default stream) on which all
 * work of this context is enqueued.  A new bind forgets the written state.
 * Errors: WCC_EINVAL (NULL pointer, misaligned), WCC_ESIZE. */
int wcc_bind(wcc_ctx* ctx, void* dev_ptr, size_t bytes, void* hip_stream);

/* Copy the initial data (Eq. 1DHCL, u(x, 0) = u0(x)) in: the state q of every
 * cell of mesh `parity` (layout above: q of Eq. 1DSchemeMatrixForm, k = 0 the
 * point value) at time t.  host holds nc*(P+1)*n_cells doubles and stays the
 * caller's; n_cells must equal the cell count of that mesh.  Resets the
 * half-step counter and the status flags and computes s_max of the written
 * averages (Eq. SubEq:1DCellAVG) on the device.  Synchronous.
 * Errors: WCC_ESTATE (not bound), WCC_EINVAL, WCC_ESIZE, WCC_EDEVICE,
 * WCC_ENONFINITE (a non-finite value was written). */
int wcc_write_dofs(wcc_ctx* ctx, const double* host, int64_t n_cells, int parity, double t);

/* Enqueue one half-step t^n -> t^{n+1/2} of Section 2.1 (the whole path:
 * Eq. 1DCauchy_Kovalewski, Eq. SubEq:1DIntegral with Eq. Cal1DFlux,
 * Eq. SubEq:Cal_1D_Derivatives_3/4, the limiter of Section 2.2 / Section 4,
 * Eq. 1DCalU) from the current mesh to the other one.  dt_fixed > 0 uses
 * that time step; otherwise dt = (cfl*dx)/s_max, the CFL condition of the
 * Section 5 preamble with cfl per half-step.  Stream-ordered: returns once
 * enqueued.  Errors: WCC_ESTATE, WCC_EINVAL (cfl outside (0, 1], non-finite
 * dt_fixed), WCC_EDEVICE. */
int wcc_step(wcc_ctx* ctx, double cfl, double dt_fixed);

/* Enqueue `half_steps` CFL half-steps as wcc_step (no end time), replayed
 * from captured HIP graphs of a fixed number of kernels.  Stream-ordered;
 * the device time of the enqueued work is read with wcc_last_run_ms.
 * Errors as wcc_step. */
int wcc_run(wcc_ctx* ctx, int64_t half_steps, double cfl);

/* Advance to t_end with CFL time steps (Section 5 preamble; the step that
 * would pass t_end is clipped to it), at most max_half_steps (<= 0:
 * unlimited).  Synchronises at the end of every graph chunk to read the
 * 16-byte status.  *taken (may be NULL) receives the half-steps done by this
 * call.  Errors: WCC_ESTATE, WCC_EINVAL (t_end before the current time),
 * WCC_EDEVICE, WCC_ENONFINITE if a step raised a flag (the state after that
 * step is kept for inspection). */
int wcc_advance(wcc_ctx* ctx, double t_end, double cfl, int64_t max_half_steps, int64_t* taken);

/* Copy the current state out (layout above) into host[cap]; cap must hold
 * nc*(P+1)*n_cells doubles of the current mesh (host may be NULL to read only
 * info).  info (may be NULL) receives time, parity, flags, sizes and s_max.
 * Synchronous.  Errors: WCC_ESTATE, WCC_ESIZE, WCC_EDEVICE. */
int wcc_read_dofs(wcc_ctx* ctx, double* host, int64_t cap, wcc_state_info* info);

/* Conserved totals sum_j ubar_j dx per component, with ubar the cell
 * average of the cell polynomial (Eq. SubEq:1DCellAVG), summed in cell order
 * on the host; under periodic boundaries they are invariants of the finite
 * volume update Eq. SubEq:1DIntegral up to round-off.  per_component holds
 * nc doubles.  Synchronous.  Errors: WCC_EINVAL, WCC_ESTATE, WCC_EDEVICE. */
int wcc_totals(wcc_ctx* ctx, double* per_component);

/* Launch shape of the half-step kernel (not a paper quantity: the work
 * decomposition only; results do not depend on it): threads per block (64,
 * 128, 192 or 256; 0 = 256), blocks (0 = enough to fill the device at the
 * kernel's occupancy) and kernel variant.  Variants 0..3 use wave tiles of
 * 64 old cells (one per lane, 63 new cells) and are a sum of bits: 1 = load
 * the next tile's inputs while computing the current one; 2 = store the new
 * cells in whole 64-cell groups staged through LDS instead of one 63-cell
 * tile per wave (pays when the state does not fit the caches).  Variant 4
 * is the second tile shape: wave tiles of 128 old cells, two per lane (127
 * new cells), direct stores.  -1 keeps the current variant.  At creation the
 * variant is 3 when the two state buffers exceed 512 MiB, else 1.  Used by
 * the autotuner.  Errors: WCC_EINVAL (variant outside -1..4, threads not
 * 64..256 in steps of 64, negative blocks). */
int wcc_set_launch(wcc_ctx* ctx, int threads_per_block, int blocks, int variant);

/* The current launch shape: threads per block, blocks (0 = device-filling
 * default) and kernel variant, as wcc_set_launch describes them.  Returns
 * WCC_EINVAL for a NULL argument. */
int wcc_get_launch(const wcc_ctx* ctx, int* threads_per_block, int* blocks, int* variant);

/* Device time of the last wcc_run call (HIP events around the enqueued work
 * on the bound stream), in ms; waits for that work.  Errors: WCC_EINVAL,
 * WCC_ESTATE (no timed run yet), WCC_EDEVICE. */
int wcc_last_run_ms(wcc_ctx* ctx, double* ms);

/* ------------------------------------------------------------------------
 * For callers that cannot allocate device memory or hand over a workspace
 * (code under HIP graph capture, serving loops that forbid hipMalloc): the
 * half-steps of wcc_run on a state the caller holds, with the run's scratch
 * (time-control block and partial wave-speed maxima) in a static device
 * array of the library instead of the workspace.  The call allocates nothing.
 *
 * - state: caller-owned device buffer (256-byte aligned) of at least
 *   wcc_workspace_bytes - WCC_WORKSPACE_STATE_OFFSET bytes, laid out as the
 *   part of wcc_bind's workspace that follows its first
 *   WCC_WORKSPACE_STATE_OFFSET bytes (so a bound workspace + that offset
 *   works): point-value buffers of parity 0 and 1, then the derivative
 *   buffers of parity 0 and 1, each nc (and nc*P) rows of ld cells, ld = the
 *   larger mesh's cell count rounded up to 64, each buffer rounded up to 256
 *   bytes.  It holds the state of mesh `parity` at time t on entry; after
 *   half_steps CFL half-steps (as wcc_run: dt = (cfl*dx)/s_max, no end time)
 *   the state of mesh parity ^ (half_steps & 1) is in that parity's buffers.
 * - ctx: a created context; only its sizes, parameters and launch shape are
 *   used (it need not be bound; its own time and state are not touched).
 * - t_out: NULL, or a host double that receives the time after the steps; a
 *   non-NULL t_out makes the call synchronise the stream and report
 *   WCC_ENONFINITE if a step raised a status flag.
 * - Scratch: WCC_NOALLOC_SCRATCH_BYTES per GPU, held until the process ends;
 *   a run needs the same amount at any size.  Every call on a GPU shares
 *   that GPU's array and keeps the last call's contents (each call
 *   re-initialises what it uses); calls that overlap on one GPU (other
 *   streams, other threads) race and must be serialised by the caller.
 * Errors: WCC_EINVAL (NULL or misaligned state, parity, t, cfl, negative
 * half_steps), WCC_ESIZE (state too small), WCC_EDEVICE, WCC_ENONFINITE. */
#define WCC_WORKSPACE_STATE_OFFSET 12544
#define WCC_NOALLOC_SCRATCH_BYTES 16384
int wcc_run_noalloc(wcc_ctx* ctx, void* state, size_t bytes, int parity, double t, int64_t half_steps, double cfl,
                    void* hip_stream, double* t_out);

/* Name of a WCC_* code (static string; "unknown error code" otherwise). */
const char* wcc_strerror(int code);
/* The last detailed message of a context (owned by the context). */
const char* wcc_last_error(const wcc_ctx* ctx);
/* Free the context's host state, graphs, events and capture stream; the
 * caller's device memory and stream are left alone.  NULL is ignored. */
void wcc_destroy(wcc_ctx* ctx);

/* ------------------------------------------------------------------------
 * Batched form: B independent instances of Eq. 1DHCLSystem (or the scalar
 * Eq. 1DHCL) of one equation, each with its own degree P[b] (0..3) and mesh
 * size N[b], same bc and params, advanced together.  Each instance runs the
 * same half-step of Section 2.1 with its own time, s_max and CFL time step
 * (Section 5 preamble); the tiles of all instances form one table and never
 * straddle instances, so instance b's results equal those of a
 * single-instance context bit for bit.  State layout per instance as above
 * (instances start on mesh parity 0).
 * ---------------------------------------------------------------------- */
/* New batch of B >= 1 instances with degrees P[0..B-1] in 0..3 and sizes
 * N[0..B-1] >= 2 (arrays read during the call only).  Errors: WCC_EINVAL. */
int wcc_batch_create(int equation, int B, const int32_t* P, const int64_t* N, int bc,
                     const wcc_params* params, wcc_batch** out);
/* Device bytes wcc_batch_bind needs: per-instance control blocks, the tile
 * and instance tables, and two ping-pong state buffers of all instances. */
int wcc_batch_workspace_bytes(const wcc_batch* bt, size_t* bytes);
/* Hand over caller-owned device memory and the HIP stream, as wcc_bind; every
 * instance restarts at t = 0 with an empty time-control ring.  Errors:
 * WCC_EINVAL, WCC_ESIZE, WCC_EDEVICE. */
int wcc_batch_bind(wcc_batch* bt, void* dev_ptr, size_t bytes, void* hip_stream);
/* Write the initial data (Eq. 1DHCL) of instance b on parity 0 at time t,
 * layout as wcc_write_dofs.  Allowed before the first advance only.
 * Synchronous.  Errors: WCC_EINVAL, WCC_ESTATE, WCC_ESIZE, WCC_EDEVICE. */
int wcc_batch_write_dofs(wcc_batch* bt, int b, const double* host, int64_t n_cells, double t);
/* Compute every instance's s_max of the written averages (Eq.
 * SubEq:1DCellAVG), the start of its CFL time control.  Synchronous. */
int wcc_batch_prepare(wcc_batch* bt);
/* Enqueue `half_steps` half-steps (Section 2.1) of every instance; instance
 * b uses the CFL number cfl_by_P[P[b]] per half-step (Section 5 preamble;
 * cfl_by_P is read during the call only).  Steps are replayed from captured
 * graphs; stream-ordered.  Errors: WCC_EINVAL (a used cfl outside (0, 1]),
 * WCC_ESTATE (not bound), WCC_EDEVICE. */
int wcc_batch_advance(wcc_batch* bt, int64_t half_steps, const double cfl_by_P[WCC_PMAX + 1]);
/* Copy instance b out (host may be NULL to read only info), as
 * wcc_read_dofs.  Synchronous. */
int wcc_batch_read_dofs(wcc_batch* bt, int b, double* host, int64_t cap, wcc_state_info* info);
/* Schedule of the persistent kernels (work decomposition only; results do not
 * depend on it): threads per block (64..256, 0 keeps the current value),
 * blocks per launch (0 = fill the device at the kernel's occupancy) and mode
 * (0 keeps the current one; 1 = fused: one launch per half-step over all
 * tiles, degree switched per tile; 2 = grouped: one launch per degree per
 * half-step; 3 and 4 = fused and grouped with the new cells staged in LDS and
 * stored in whole 64-cell groups; 5 (the default) and 6 = grouped with direct
 * / staged stores, the degrees' launches captured as parallel branches of the
 * run's graphs so that they may overlap on the device; other values return
 * WCC_EINVAL). */
int wcc_batch_set_schedule(wcc_batch* bt, int threads_per_block, int blocks, int mode);
/* Device time of the last wcc_batch_advance call, in ms (waits for it). */
int wcc_batch_last_run_ms(wcc_batch* bt, double* ms);
/* The last detailed message of a batch (owned by the batch). */
const char* wcc_batch_last_error(const wcc_batch* bt);
/* Free the batch's host state and graphs.  NULL is ignored. */
void wcc_batch_destroy(wcc_batch* bt);

#ifdef __cplusplus
}
#endif

#endif /* WCC_H */
