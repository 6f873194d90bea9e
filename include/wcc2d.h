/* wcc2d.h -- C ABI of the 2D half-step of the weighted compact central (WCC)
 * schemes (Shen & Parsani, arXiv:2104.04347, Section 3 and Appendix B; the
 * 2D Euler step of Section 4) on gfx950.
 *
 * The library advances u_t + f(u)_x + g(u)_y = 0 (Eq. 2DHCL) on a rectangle
 * [x_left, x_right] x [y_left, y_right] cut into Nx x Ny intervals, periodic
 * or with transmissive edges in each direction, on the two space-time
 * staggered Cartesian meshes of Section 3.1.  One half-step is
 * one fused GPU kernel: trivariate Cauchy-Kovalewski expansion of every old
 * cell, quarter-cell averages (Eq. SubEq:2DCellAVGRU/RD/LU/LD) and half-edge
 * space-time flux averages (Eq. SubEq:2DFluxFU/FD/GR/GL) combined into the new
 * cell average (Eq. 2DIntegral), the new derivatives from the vertex values at
 * the half time level (Eq. 2DDerivatives with Eq. SubEq:2DUij; cross
 * derivatives averaged) and the 2D limiter of Section 3.2 -- for the Euler
 * equations applied to characteristic fields in the rotated direction of
 * the gradient of rho e (Section 4, Eq. RotatedNormal).
 *
 * Conventions
 * -----------
 * - Return codes, ownership and stream order are those of wcc.h (same
 *   WCC_* codes; wcc_strerror names them).
 * - Equations: WCC_ADVECTION (f = a u, g = b u), WCC_BURGERS
 *   (f = g = u^2/2), WCC_EULER (rho, rho u, rho v, rho e; gamma-law gas);
 *   limiter 0 gives the unlimited LCCS form, 1 the WCCS form.
 * - State layout at the boundary: host doubles indexed
 *   [c][d][j][i] = host[((c*ndof + d)*ny + j)*nx + i] with nx x ny the cells
 *   of the state's mesh (below), ndof = (P+1)(P+2)/2,
 *   with the DOFs u_{kx,ly} = dx^k dy^l d^{k+l}u/dx^k dy^l at the cell
 *   centre in "DOF order": total degree k+l ascending, then l ascending
 *   (d = (k+l)(k+l+1)/2 + l); d = 0 is the point value (Eq.
 *   2DPolynomial_Space).
 * - Meshes: dx = (x_right-x_left)/Nx, dy = (y_right-y_left)/Ny; parity 0
 *   centres (x_left + i dx, y_left + j dy), parity 1 shifted by (dx/2, dy/2).
 *   Per direction (bc for x, bc_y for y): WCC_BC_PERIODIC, N cells on both
 *   meshes, indices wrap; WCC_BC_TRANSMISSIVE, parity 0 has the N+1 cells
 *   centred at the mesh points (the domain's edges included), parity 1 the N
 *   cells between them, and the parents an edge cell of parity 0 lacks are
 *   copies (all DOFs) of the adjacent parity-1 cell (corners likewise).
 *   nx = Nx or Nx+1 and ny = Ny or Ny+1 accordingly.
 * - Time step: dt = cfl / s_max with s_max the largest s_x/dx + s_y/dy over
 *   the current cell averages (s_x = |a|, |u| or |u|+c; s_y likewise), i.e.
 *   cfl is the CFL number of the half-step; clipped to t_end by wcc2d_advance.
 * - Arithmetic: binary64 with a fixed, documented operation order.
 */
#ifndef WCC2D_H
#define WCC2D_H

#include <stddef.h>
#include <stdint.h>

#include "wcc.h"

#ifdef __cplusplus
extern "C" {
#endif

#define WCC2D_PMAX 3

typedef struct wcc2d_ctx wcc2d_ctx;   /* opaque, host side */

typedef struct {
  double x_left, x_right, y_left, y_right;   /* domain, default [0,1] x [0,1] */
  double a, b;                                /* advection velocity, default (1, 1) */
  double gamma;                               /* Euler, default 1.4 */
  double eps;                                 /* limiter epsilon, default 1e-40 (Section 3.2) */
  int32_t limiter;                            /* 0/1, default 1 */
  int32_t bc;                                 /* x edges: WCC_BC_PERIODIC (default) or WCC_BC_TRANSMISSIVE */
  int32_t bc_y;                               /* y edges: likewise; -1 (default): as bc */
  int32_t reserved;
} wcc2d_params;

typedef struct {
  double t;             /* time of the current state */
  int32_t parity;       /* mesh of the current state */
  int32_t flags;        /* bit0 non-finite value, bit1 rho <= 0 or p <= 0 */
  int64_t Nx, Ny;       /* cells of the current mesh (see Meshes) */
  double dx, dy;
  int64_t half_steps;   /* half-steps taken since the last write */
  double s_max;         /* s_x/dx + s_y/dy of the current state */
} wcc2d_state_info;

/* Defaults listed in wcc2d_params.  Error: WCC_EINVAL for a null pointer. */
int wcc2d_params_default(wcc2d_params* p);

/* New context for the problem of Eq. 2DHCL: equation (WCC_ADVECTION,
 * WCC_BURGERS, WCC_EULER), degree P in [0, WCC2D_PMAX] of the cell
 * polynomial of Eq. 2DPolynomial_Space, Nx, Ny >= 2 intervals of the meshes of
 * Section 3.1 with (Nx+1)*(Ny+1) <= 2^28.
 * params may be null (defaults).  Errors: WCC_EINVAL for bad sizes, enums
 * (equation, boundary) or domain, gamma <= 1 for Euler. */
int wcc2d_create(int equation, int P, int64_t Nx, int64_t Ny, const wcc2d_params* params, wcc2d_ctx** out);

/* Device bytes the caller must provide to wcc2d_bind: a control block of the
 * CFL time step, the partial wave-speed slots and two state buffers of
 * nc*ndof planes (the two staggered meshes of Section 3.1).  Errors:
 * WCC_EINVAL for NULL arguments. */
int wcc2d_workspace_bytes(const wcc2d_ctx* c, size_t* bytes);

/* Hand over caller-owned device memory (256-byte aligned, at least
 * wcc2d_workspace_bytes) and the HIP stream every later call enqueues on.
 * Errors: WCC_EINVAL (null or misaligned), WCC_ESIZE (too small). */
int wcc2d_bind(wcc2d_ctx* c, void* dev_ptr, size_t bytes, void* hip_stream);

/* Copy the initial data of Eq. 2DHCL (layout above, the cells of mesh
 * `parity`; host stays the caller's) onto that mesh at time t and compute its
 * wave-speed rate from the cell averages; synchronises the stream.  Errors:
 * WCC_ESTATE before bind, WCC_EINVAL, WCC_ENONFINITE (state kept). */
int wcc2d_write_dofs(wcc2d_ctx* c, const double* host, int parity, double t);

/* Enqueue one half-step of Section 3 (Cauchy-Kovalewski expansion of
 * Eq. 2DTaylorSeries, the quarter-cell and half-edge averages of Appendix B,
 * Eq. 2DIntegral, Eq. 2DDerivatives, the limiter of Section 3.2 and
 * Section 4): dt = cfl/s_max, or dt_fixed when > 0.  Stream-ordered.
 * Errors: WCC_ESTATE, WCC_EINVAL, WCC_EDEVICE. */
int wcc2d_step(wcc2d_ctx* c, double cfl, double dt_fixed);

/* Enqueue half_steps half-steps as wcc2d_step at CFL number cfl
 * (graph-replayed chunks), timed by HIP events on the bound stream
 * (wcc2d_last_run_ms).  Errors as wcc2d_step. */
int wcc2d_run(wcc2d_ctx* c, int64_t half_steps, double cfl);

/* Advance to t_end with CFL time steps (the step that would pass t_end is
 * clipped to it), at most max_half_steps if > 0;
 * *taken = half-steps done.  Errors: WCC_ENONFINITE when a step raised a
 * status bit (the state is kept for inspection). */
int wcc2d_advance(wcc2d_ctx* c, double t_end, double cfl, int64_t max_half_steps, int64_t* taken);

/* Copy the current state to host (if host != null; cap = doubles available,
 * layout above) and fill info (if non-null); synchronises the stream.
 * Errors: WCC_ESTATE, WCC_ESIZE, WCC_EDEVICE. */
int wcc2d_read_dofs(wcc2d_ctx* c, double* host, int64_t cap, wcc2d_state_info* info);

/* Conserved totals sum over the current mesh of ubar dx dy per component
 * (cell averages of the cell polynomials of Eq. 2DPolynomial_Space), summed
 * in cell order on the host.
 * Synchronous.  With periodic edges they are invariants of the scheme up to
 * round-off.  Errors: WCC_EINVAL, WCC_ESTATE (no state). */
int wcc2d_totals(wcc2d_ctx* c, double* per_component);

/* Launch shape (the work decomposition, not a paper quantity): threads per
 * block (64..256, multiple of 64; 0 = 256),
 * blocks per launch (0 = resident capacity) and the work decomposition
 * (variant 0: every wavefront expands 8 x 8 old-cell tiles and produces their
 * 7 x 7 new cells; 1: wavefronts walk 64-column strips upward one row at a
 * time, expanding every old cell once per strip; 2: as 1, with the next
 * row's loads issued before the current row is expanded; 3, the default: as
 * 2, with each wave owning one strip over one band of rows and the waves of
 * a block (and the blocks of one XCD) taking neighbouring strips, so that
 * the cache lines neighbouring strips share are fetched once; -1 keeps the
 * current one).  Results do not depend on it.  Errors: WCC_EINVAL. */
int wcc2d_set_launch(wcc2d_ctx* c, int threads_per_block, int blocks, int variant);

/* The launch shape the next half-step uses: threads per block, the
 * effective number of blocks (the resident capacity resolved for the
 * current mesh when wcc2d_set_launch was given 0) and the variant.
 * Errors: WCC_EINVAL for a NULL argument. */
int wcc2d_get_launch(wcc2d_ctx* c, int* threads_per_block, int* blocks, int* variant);

/* Milliseconds between the HIP events around the last wcc2d_run (waits for
 * it).  Errors: WCC_EINVAL, WCC_ESTATE (no timed run), WCC_EDEVICE. */
int wcc2d_last_run_ms(wcc2d_ctx* c, double* ms);

/* The last detailed message of a context (owned by the context). */
const char* wcc2d_last_error(const wcc2d_ctx* c);
/* Free the context's host state, graphs and events; NULL is ignored. */
void wcc2d_destroy(wcc2d_ctx* c);

#ifdef __cplusplus
}
#endif
#endif /* WCC2D_H */
