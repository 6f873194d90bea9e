// Runs the device rounding helpers of csrc/wcc_rn.hpp (div_rn, sqrt_rn) and
// the compiler's own binary64 `/` and sqrt on operands read from files, and
// writes the four results.  Test infrastructure: tests/test_gpu_rounding.py
// generates the operands and compares the results with the CPU's IEEE
// operations.
//
//   rn_check <div.bin> <sqrt.bin> <out.bin>
//
// div.bin: n numerators then n denominators (binary64); sqrt.bin: m operands.
// out.bin: div_rn (n), `/` (n), sqrt_rn (m), sqrt (m).  Exit status 0 on
// success, 1 on a HIP error, 2 on unreadable input.
#include <hip/hip_runtime.h>

#include <cstdio>
#include <vector>

#include "wcc_rn.hpp"

__global__ void k_div(const double* a, const double* b, double* rn, double* hw, long n) {
  for (long i = blockIdx.x * (long)blockDim.x + threadIdx.x; i < n; i += (long)gridDim.x * blockDim.x) {
    rn[i] = wcc::div_rn(a[i], b[i]);
    hw[i] = a[i] / b[i];
  }
}

__global__ void k_sqrt(const double* x, double* rn, double* hw, long m) {
  for (long i = blockIdx.x * (long)blockDim.x + threadIdx.x; i < m; i += (long)gridDim.x * blockDim.x) {
    rn[i] = wcc::sqrt_rn(x[i]);
    hw[i] = __builtin_sqrt(x[i]);
  }
}

static bool read_all(const char* path, std::vector<double>& v) {
  FILE* f = fopen(path, "rb");
  if (!f) return false;
  fseek(f, 0, SEEK_END);
  const long bytes = ftell(f);
  fseek(f, 0, SEEK_SET);
  if (bytes < 0 || bytes % 8) {
    fclose(f);
    return false;
  }
  v.resize(bytes / 8);
  const bool ok = fread(v.data(), 8, v.size(), f) == v.size();
  fclose(f);
  return ok;
}

#define HIP_OK(call)                                                       \
  do {                                                                     \
    hipError_t e_ = (call);                                                \
    if (e_ != hipSuccess) {                                                \
      fprintf(stderr, "%s: %s\n", #call, hipGetErrorString(e_));          \
      return 1;                                                            \
    }                                                                      \
  } while (0)

int main(int argc, char** argv) {
  if (argc != 4) {
    fprintf(stderr, "usage: %s div.bin sqrt.bin out.bin\n", argv[0]);
    return 2;
  }
  std::vector<double> ab, x;
  if (!read_all(argv[1], ab) || !read_all(argv[2], x) || ab.size() % 2 || ab.empty() || x.empty()) {
    fprintf(stderr, "cannot read the operands\n");
    return 2;
  }
  const long n = (long)ab.size() / 2, m = (long)x.size();
  double *d_ab = nullptr, *d_x = nullptr, *d_out = nullptr;
  HIP_OK(hipMalloc(&d_ab, 2 * n * sizeof(double)));
  HIP_OK(hipMalloc(&d_x, m * sizeof(double)));
  HIP_OK(hipMalloc(&d_out, (2 * n + 2 * m) * sizeof(double)));
  HIP_OK(hipMemcpy(d_ab, ab.data(), 2 * n * sizeof(double), hipMemcpyHostToDevice));
  HIP_OK(hipMemcpy(d_x, x.data(), m * sizeof(double), hipMemcpyHostToDevice));
  // grid-stride loops: any grid covers every element
  k_div<<<1024, 256>>>(d_ab, d_ab + n, d_out, d_out + n, n);
  HIP_OK(hipGetLastError());
  k_sqrt<<<1024, 256>>>(d_x, d_out + 2 * n, d_out + 2 * n + m, m);
  HIP_OK(hipGetLastError());
  std::vector<double> out(2 * n + 2 * m);
  HIP_OK(hipMemcpy(out.data(), d_out, out.size() * sizeof(double), hipMemcpyDeviceToHost));
  HIP_OK(hipFree(d_ab));
  HIP_OK(hipFree(d_x));
  HIP_OK(hipFree(d_out));
  FILE* f = fopen(argv[3], "wb");
  if (!f || fwrite(out.data(), sizeof(double), out.size(), f) != out.size()) {
    fprintf(stderr, "cannot write %s\n", argv[3]);
    return 2;
  }
  fclose(f);
  printf("rn_check: %ld quotients, %ld square roots\n", n, m);
  return 0;
}
