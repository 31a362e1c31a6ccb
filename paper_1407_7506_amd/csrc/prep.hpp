#pragma once
#include <hip/hip_runtime.h>
namespace ppcg {
void launch_prep_diag(const double* V, long n, double c0, double* td, float* V32, double* dmin_part, int nparts,
                      int* nan_flag, hipStream_t st);
void launch_zero_int(int* p, int n, hipStream_t st);
}  // namespace ppcg
