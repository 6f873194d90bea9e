/* A C program that uses the library through include/wcc.h alone: it allocates
 * the workspace with hipMalloc, creates its own HIP stream, and advances a 1D
 * Euler state (transmissive boundaries, limiter on, binary64) to an end time
 * with CFL steps.  Test infrastructure: tests/test_c_abi_consumer.py runs it
 * and compares the result with the oracle's.
 *
 *   consumer <in.bin> <out.bin> <P> <N> <x_left> <x_right> <t_end> <cfl>
 *
 * in.bin: the state of the parity-0 mesh, 3 x (P+1) x (N+1) binary64 values in
 * the layout of wcc_write_dofs.  out.bin: the final state, 3 x (P+1) x n
 * values (n = the cells of the final mesh), then the final time, the mesh
 * parity (as a binary64) and the number of half-steps taken.  Exit status 0
 * on success; otherwise the failing call's error is printed to stderr. */
#include <hip/hip_runtime_api.h>
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>

#include "wcc.h"

#define CHECK(call)                                                                   \
  do {                                                                                \
    int rc_ = (call);                                                                 \
    if (rc_ != WCC_OK) {                                                              \
      fprintf(stderr, "%s: %s (%s)\n", #call, wcc_strerror(rc_), ctx ? wcc_last_error(ctx) : ""); \
      return 1;                                                                       \
    }                                                                                 \
  } while (0)

int main(int argc, char** argv) {
  wcc_ctx* ctx = NULL;
  if (argc != 9) {
    fprintf(stderr, "usage: %s in.bin out.bin P N x_left x_right t_end cfl\n", argv[0]);
    return 2;
  }
  const int P = atoi(argv[3]);
  const int64_t N = atoll(argv[4]);
  const double t_end = atof(argv[7]), cfl = atof(argv[8]);
  if (P < 0 || P > WCC_PMAX || N < 2) {
    fprintf(stderr, "bad P or N\n");
    return 2;
  }
  const int64_t n0 = N + 1, cap = 3 * (int64_t)(P + 1) * (N + 1);
  double* q = (double*)malloc((size_t)cap * sizeof(double));
  FILE* f = fopen(argv[1], "rb");
  if (!q || !f || fread(q, sizeof(double), (size_t)(3 * (P + 1) * n0), f) != (size_t)(3 * (P + 1) * n0)) {
    fprintf(stderr, "cannot read %s\n", argv[1]);
    return 2;
  }
  fclose(f);

  wcc_params p;
  CHECK(wcc_params_default(&p));
  p.x_left = atof(argv[5]);
  p.x_right = atof(argv[6]);
  p.limiter = 1;
  p.precision = WCC_FP64;
  CHECK(wcc_create(WCC_EULER, P, N, WCC_BC_TRANSMISSIVE, &p, &ctx));
  size_t bytes = 0;
  CHECK(wcc_workspace_bytes(ctx, &bytes));
  void* dev = NULL;
  hipStream_t stream = NULL;
  if (hipMalloc(&dev, bytes) != hipSuccess || hipStreamCreate(&stream) != hipSuccess) {
    fprintf(stderr, "hipMalloc / hipStreamCreate failed\n");
    return 1;
  }
  CHECK(wcc_bind(ctx, dev, bytes, (void*)stream));
  CHECK(wcc_write_dofs(ctx, q, n0, 0, 0.0));
  int64_t taken = 0;
  CHECK(wcc_advance(ctx, t_end, cfl, 0, &taken));
  wcc_state_info info;
  CHECK(wcc_read_dofs(ctx, q, cap, &info));

  f = fopen(argv[2], "wb");
  const double tail[3] = {info.t, (double)info.parity, (double)taken};
  if (!f || fwrite(q, sizeof(double), (size_t)(3 * (P + 1) * info.n_cells), f) != (size_t)(3 * (P + 1) * info.n_cells) ||
      fwrite(tail, sizeof(double), 3, f) != 3) {
    fprintf(stderr, "cannot write %s\n", argv[2]);
    return 2;
  }
  fclose(f);
  wcc_destroy(ctx);
  hipStreamDestroy(stream);
  hipFree(dev);
  free(q);
  printf("consumer: %lld half-steps to t = %.17g on mesh parity %d, %lld cells\n", (long long)taken, info.t,
         info.parity, (long long)info.n_cells);
  return 0;
}
