// Backward pass of the eigen-decomposition: dL/dV for
//   L = sum_i g_i lambda_i + sum_r w_r rho_r,  rho = sum_{i<=k} |x_i|^2.
// Eigenvalue part (Hellmann-Feynman): d lambda_i / d V = |x_i|^2.  Density
// part (first-order perturbation of the occupied subspace):
//   dL/dV -= 2 Re sum_i conj(z_i) x_i,  Q (H - lambda_i) Q z_i = Q (w x_i),
// Q = I - X X^H, solved by block preconditioned CG (per-column scalars,
// Jacobi preconditioner 1/(diag(H) - lambda_i)) with the stencil and the
// projection kernels of the solver.  These kernels are the element-wise and
// per-column pieces of that CG.
#include "common.hpp"
#include "kernels.hpp"

namespace ppcg {

// out[j] = sum_r A[r, j] B[r, j]  (one workgroup per column, fixed order)
__global__ __launch_bounds__(256) void coldot_kernel(const double* A, const double* B, long ld, long rows,
                                                     double* out) {
  const double* a = A + (long)blockIdx.x * ld;
  const double* b = B + (long)blockIdx.x * ld;
  double s = 0;
  for (long r = threadIdx.x; r < rows; r += 256) s += a[r] * b[r];
  __shared__ double red[4];
  s = wave_sum(s);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = s;
  __syncthreads();
  if (threadIdx.x == 0) out[blockIdx.x] = (red[0] + red[1]) + (red[2] + red[3]);
}
void launch_coldot(const double* A, const double* B, long ld, long rows, int ncols, double* out, hipStream_t st) {
  if (ncols > 0) hipLaunchKernelGGL(coldot_kernel, dim3(ncols), dim3(256), 0, st, A, B, ld, rows, out);
}

// Y[r, j] = R[r, j] / (c0 + V[r] - lam[j])  (or R when unprec); zero on padding rows.
// nc = 2: complex columns (interleaved), both parts divided by the real diagonal.
__global__ __launch_bounds__(256) void cg_precond_kernel(const double* R, double* Y, const double* V, double c0,
                                                         const double* lam, long ld, long n, long rows, int unprec,
                                                         int nc) {
  long e = blockIdx.x * 256L + threadIdx.x;  // element of the (interleaved) column
  int j = blockIdx.y;
  if (e >= rows * nc) return;
  const long r = nc == 2 ? e >> 1 : e;
  const long o = e + j * ld * nc;
  double v = R[o];
  if (r >= n) v = 0.0;
  else if (!unprec) v /= (c0 + V[r] - lam[j]);
  Y[o] = v;
}
void launch_cg_precond(const double* R, double* Y, const double* V, double c0, const double* lam, long ld, long n,
                       long rows, int ncols, int unprec, hipStream_t st, int cplx) {
  const int nc = cplx ? 2 : 1;
  if (ncols > 0)
    hipLaunchKernelGGL(cg_precond_kernel, dim3((rows * nc + 255) / 256, ncols), dim3(256), 0, st, R, Y, V, c0, lam,
                       ld, n, rows, unprec, nc);
}

// alpha_j = rz_j / pAp_j (0 when pAp_j <= 0 or the column has converged)
__global__ void cg_alpha_kernel(const double* rz, const double* pAp, const int* done, double* alpha, int k) {
  int j = blockIdx.x * 256 + threadIdx.x;
  if (j >= k) return;
  alpha[j] = (!done[j] && pAp[j] > 0) ? rz[j] / pAp[j] : 0.0;
}
// beta_j = rz_new_j / rz_j; rz <- rz_new
__global__ void cg_beta_kernel(double* rz, const double* rznew, const int* done, double* beta, int k) {
  int j = blockIdx.x * 256 + threadIdx.x;
  if (j >= k) return;
  beta[j] = (!done[j] && rz[j] > 0) ? rznew[j] / rz[j] : 0.0;
  rz[j] = rznew[j];
}
void launch_cg_alpha(const double* rz, const double* pAp, const int* done, double* alpha, int k, hipStream_t st) {
  hipLaunchKernelGGL(cg_alpha_kernel, dim3((k + 255) / 256), dim3(256), 0, st, rz, pAp, done, alpha, k);
}
void launch_cg_beta(double* rz, const double* rznew, const int* done, double* beta, int k, hipStream_t st) {
  hipLaunchKernelGGL(cg_beta_kernel, dim3((k + 255) / 256), dim3(256), 0, st, rz, rznew, done, beta, k);
}

// Z += alpha P ; R -= alpha AP
__global__ __launch_bounds__(256) void cg_xr_kernel(double* Z, double* R, const double* P, const double* AP,
                                                    const double* alpha, long ld, long rows) {
  long r = blockIdx.x * 256L + threadIdx.x;
  int j = blockIdx.y;
  if (r >= rows) return;
  double a = alpha[j];
  long o = r + j * ld;
  Z[o] += a * P[o];
  R[o] -= a * AP[o];
}
// P = Y + beta P
__global__ __launch_bounds__(256) void cg_p_kernel(double* P, const double* Y, const double* beta, long ld,
                                                   long rows) {
  long r = blockIdx.x * 256L + threadIdx.x;
  int j = blockIdx.y;
  if (r >= rows) return;
  long o = r + j * ld;
  P[o] = Y[o] + beta[j] * P[o];
}
void launch_cg_xr(double* Z, double* R, const double* P, const double* AP, const double* alpha, long ld, long rows,
                  int k, hipStream_t st) {
  hipLaunchKernelGGL(cg_xr_kernel, dim3((rows + 255) / 256, k), dim3(256), 0, st, Z, R, P, AP, alpha, ld, rows);
}
void launch_cg_p(double* P, const double* Y, const double* beta, long ld, long rows, int k, hipStream_t st) {
  hipLaunchKernelGGL(cg_p_kernel, dim3((rows + 255) / 256, k), dim3(256), 0, st, P, Y, beta, ld, rows);
}

// done_j = (|r_j|^2 <= tol^2 |b_j|^2); counts unfinished columns into *left
__global__ void cg_check_kernel(const double* rr, const double* bb, double tol, int* done, int* left, int k) {
  int j = blockIdx.x * 256 + threadIdx.x;
  if (j >= k) return;
  int d = done[j] || rr[j] <= tol * tol * bb[j];
  done[j] = d;
  if (!d) atomicAdd(left, 1);
}
void launch_cg_check(const double* rr, const double* bb, double tol, int* done, int* left, int k, hipStream_t st) {
  hipLaunchKernelGGL(cg_check_kernel, dim3((k + 255) / 256), dim3(256), 0, st, rr, bb, tol, done, left, k);
}

// out[r] = sum_j (g_j |X[r,j]|^2 - 2 Re(conj(Z[r,j]) X[r,j])) for r < n  (Z may be null; g null = all
// ones); nc = 2: complex columns (interleaved, leading dimension ld complex elements)
__global__ __launch_bounds__(256) void grad_rows_kernel(const double* X, const double* Z, const double* g, long ld,
                                                        long n, int k, double* out, int nc) {
  long r = blockIdx.x * 256L + threadIdx.x;
  if (r >= n) return;
  double s = 0;
  for (int j = 0; j < k; ++j) {
    for (int c = 0; c < nc; ++c) {
      const long o = (r + j * ld) * nc + c;
      double x = X[o];
      double t = (g ? g[j] : 1.0) * x;
      if (Z) t -= 2.0 * Z[o];
      s += t * x;
    }
  }
  out[r] = s;
}
void launch_grad_rows(const double* X, const double* Z, const double* g, long ld, long n, int k, double* out,
                      hipStream_t st, int cplx) {
  hipLaunchKernelGGL(grad_rows_kernel, dim3((n + 255) / 256), dim3(256), 0, st, X, Z, g, ld, n, k, out,
                     cplx ? 2 : 1);
}

// Y[r, j] = w[r] X[r, j] over rows (complex columns: both parts), the right-hand sides w x_i
__global__ __launch_bounds__(256) void scale_rows_c_kernel(const double* w, const double* X, double* Y, long ld,
                                                           long rows, int nc) {
  long e = blockIdx.x * 256L + threadIdx.x;
  int j = blockIdx.y;
  if (e >= rows * nc) return;
  const long o = e + j * ld * nc;
  Y[o] = w[nc == 2 ? e >> 1 : e] * X[o];
}
void launch_scale_rows_c(const double* w, const double* X, double* Y, long ld, long rows, int ncols, int cplx,
                         hipStream_t st) {
  const int nc = cplx ? 2 : 1;
  if (ncols > 0)
    hipLaunchKernelGGL(scale_rows_c_kernel, dim3((rows * nc + 255) / 256, ncols), dim3(256), 0, st, w, X, Y, ld,
                       rows, nc);
}

}  // namespace ppcg
