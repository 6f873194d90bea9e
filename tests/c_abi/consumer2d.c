/* A C program that uses the 2D library through include/wcc2d.h alone: it
 * allocates the workspace with hipMalloc, creates its own HIP stream, and
 * advances a 2D Euler state on the square [x_left, x_right]^2 (transmissive
 * edges, rotated characteristic limiter, binary64) to an end time with CFL
 * steps.  Test infrastructure: tests/test_c_abi_consumer.py runs it and
 * compares the result with the oracle's.
 *
 *   consumer2d <in.bin> <out.bin> <P> <N> <x_left> <x_right> <t_end> <cfl>
 *
 * in.bin: the state of the parity-0 mesh ((N+1) x (N+1) cells) in the layout
 * of wcc2d_write_dofs.  out.bin: the final state (4 x (P+1)(P+2)/2 x Ny x Nx
 * values of the final mesh), then the final time, the mesh parity (as a
 * binary64) and the number of half-steps taken.  Exit status 0 on success;
 * otherwise the failing call's error is printed to stderr. */
#include <hip/hip_runtime_api.h>
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>

#include "wcc.h"
#include "wcc2d.h"

#define CHECK(call)                                                                     \
  do {                                                                                  \
    int rc_ = (call);                                                                   \
    if (rc_ != WCC_OK) {                                                                \
      fprintf(stderr, "%s: %s (%s)\n", #call, wcc_strerror(rc_), ctx ? wcc2d_last_error(ctx) : ""); \
      return 1;                                                                         \
    }                                                                                   \
  } while (0)

int main(int argc, char** argv) {
  wcc2d_ctx* ctx = NULL;
  if (argc != 9) {
    fprintf(stderr, "usage: %s in.bin out.bin P N x_left x_right t_end cfl\n", argv[0]);
    return 2;
  }
  const int P = atoi(argv[3]);
  const int64_t N = atoll(argv[4]);
  const double t_end = atof(argv[7]), cfl = atof(argv[8]);
  if (P < 0 || P > WCC2D_PMAX || N < 2 || N > 4096) {
    fprintf(stderr, "bad P or N\n");
    return 2;
  }
  const int64_t nd = (int64_t)(P + 1) * (P + 2) / 2;
  const int64_t cap = 4 * nd * (N + 1) * (N + 1);
  double* q = (double*)malloc((size_t)cap * sizeof(double));
  FILE* f = fopen(argv[1], "rb");
  if (!q || !f || fread(q, sizeof(double), (size_t)cap, f) != (size_t)cap) {
    fprintf(stderr, "cannot read %s\n", argv[1]);
    return 2;
  }
  fclose(f);

  wcc2d_params p;
  CHECK(wcc2d_params_default(&p));
  p.x_left = p.y_left = atof(argv[5]);
  p.x_right = p.y_right = atof(argv[6]);
  p.limiter = 1;
  p.bc = WCC_BC_TRANSMISSIVE;
  CHECK(wcc2d_create(WCC_EULER, P, N, N, &p, &ctx));
  size_t bytes = 0;
  CHECK(wcc2d_workspace_bytes(ctx, &bytes));
  void* dev = NULL;
  hipStream_t stream = NULL;
  if (hipMalloc(&dev, bytes) != hipSuccess || hipStreamCreate(&stream) != hipSuccess) {
    fprintf(stderr, "hipMalloc / hipStreamCreate failed\n");
    return 1;
  }
  CHECK(wcc2d_bind(ctx, dev, bytes, (void*)stream));
  CHECK(wcc2d_write_dofs(ctx, q, 0, 0.0));
  int64_t taken = 0;
  CHECK(wcc2d_advance(ctx, t_end, cfl, 0, &taken));
  wcc2d_state_info info;
  CHECK(wcc2d_read_dofs(ctx, q, cap, &info));

  const size_t n = (size_t)(4 * nd * info.Nx * info.Ny);
  f = fopen(argv[2], "wb");
  const double tail[3] = {info.t, (double)info.parity, (double)taken};
  if (!f || fwrite(q, sizeof(double), n, f) != n || fwrite(tail, sizeof(double), 3, f) != 3) {
    fprintf(stderr, "cannot write %s\n", argv[2]);
    return 2;
  }
  fclose(f);
  wcc2d_destroy(ctx);
  hipStreamDestroy(stream);
  hipFree(dev);
  free(q);
  printf("consumer2d: %lld half-steps to t = %.17g on mesh parity %d, %lld x %lld cells\n", (long long)taken, info.t,
         info.parity, (long long)info.Nx, (long long)info.Ny);
  return 0;
}
