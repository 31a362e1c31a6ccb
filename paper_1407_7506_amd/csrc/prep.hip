// Set-up kernels: Jacobi preconditioner T = diag(H)^{-1} (the paper only
// requires T Hermitian positive definite, Theorem 2), float copy of V, and
// the scan for NaN / non-positive diagonal.
#include "common.hpp"
#include "kernels.hpp"
#include "prep.hpp"

namespace ppcg {

__global__ __launch_bounds__(256) void prep_diag_kernel(const double* V, long n, double c0, double* td, float* V32,
                                                        double* dmin_part, int* nan_flag) {
  double mn = 1e308;
  int bad = 0;
  for (long r = blockIdx.x * 256L + threadIdx.x; r < n; r += (long)gridDim.x * 256) {
    double v = V[r];
    double d = c0 + v;
    if (v != v) bad = 1;
    mn = fmin(mn, d);
    td[r] = 1.0 / d;
    if (V32) V32[r] = (float)v;
  }
  for (int o = 32; o > 0; o >>= 1) mn = fmin(mn, __shfl_xor(mn, o, 64));
  __shared__ double red[4];
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = mn;
  if (bad) atomicOr(nan_flag, 1);
  __syncthreads();
  if (threadIdx.x == 0) dmin_part[blockIdx.x] = fmin(fmin(red[0], red[1]), fmin(red[2], red[3]));
}

void launch_prep_diag(const double* V, long n, double c0, double* td, float* V32, double* dmin_part, int nparts,
                      int* nan_flag, hipStream_t st) {
  hipLaunchKernelGGL(prep_diag_kernel, dim3(nparts), dim3(256), 0, st, V, n, c0, td, V32, dmin_part, nan_flag);
}

__global__ void zero_int_kernel(int* p, int n) {
  int e = blockIdx.x * 256 + threadIdx.x;
  if (e < n) p[e] = 0;
}
void launch_zero_int(int* p, int n, hipStream_t st) {
  if (n > 0) hipLaunchKernelGGL(zero_int_kernel, dim3((n + 255) / 256), dim3(256), 0, st, p, n);
}

}  // namespace ppcg
