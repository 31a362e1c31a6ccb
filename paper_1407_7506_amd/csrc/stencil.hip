// Matrix-free Kohn-Sham operator H = -1/2 Lap_h + diag(V) on a periodic N^3
// grid (7-point or 13-point Laplacian), applied to a block of columns.  This
// is the product A X of the paper's problem statement (section 1); the
// paper's own operator is a planewave Hamiltonian, here it is a
// finite-difference one.  Streams each column once from HBM: a thread owns
// one grid point; x-neighbours share cache lines and the y/z planes are
// served from L2 because the workgroups of one column run on one XCD.
#include "common.hpp"
#include "kernels.hpp"

namespace ppcg {

template <class T, int ORDER>
__global__ __launch_bounds__(256) void stencil_kernel(StencilArgs a) {
  const long n = (long)a.N * a.N * a.N;
  const unsigned bpc = (unsigned)((n + 255) / 256);
  unsigned L = xcd_remap(blockIdx.x, gridDim.x);
  int col = L / bpc;
  long p = (long)(L % bpc) * 256 + threadIdx.x;
  if (col >= a.ncols || p >= n) return;
  const T* x = (const T*)a.X + (long)col * a.ldx;
  T* y = (T*)a.Y + (long)col * a.ldy;
  const T* V = (const T*)a.V;
  const int N = a.N;
  const int NN = N * N;
  int i = (int)(p % N);
  int t = (int)(p / N);
  int j = t % N;
  int k = t / N;
  const long b = p - i;                 // start of the x line
  const long pl = p - (long)j * N;      // (i, 0, k)
  const long pz = p - (long)k * NN;     // (i, j, 0)
  auto wr = [N](int c, int d) { int r = c + d; return r >= N ? r - N : (r < 0 ? r + N : r); };
  T xc = x[p];
  T s1 = x[b + wr(i, 1)] + x[b + wr(i, -1)] + x[pl + (long)wr(j, 1) * N] + x[pl + (long)wr(j, -1) * N] +
         x[pz + (long)wr(k, 1) * NN] + x[pz + (long)wr(k, -1) * NN];
  T out = ((T)a.c0 + V[p]) * xc + (T)a.w1 * s1;
  if (ORDER == 4) {
    T s2 = x[b + wr(i, 2)] + x[b + wr(i, -2)] + x[pl + (long)wr(j, 2) * N] + x[pl + (long)wr(j, -2) * N] +
           x[pz + (long)wr(k, 2) * NN] + x[pz + (long)wr(k, -2) * NN];
    out += (T)a.w2 * s2;
  }
  if (a.shift) out -= (T)a.shift[col] * xc;
  y[p] = out;
}

void launch_stencil(const StencilArgs& a, hipStream_t st) {
  long n = (long)a.N * a.N * a.N;
  long blocks = ((n + 255) / 256) * a.ncols;
  if (blocks == 0) return;
  if (a.f32) {
    if (a.order == 4) hipLaunchKernelGGL((stencil_kernel<float, 4>), dim3(blocks), dim3(256), 0, st, a);
    else hipLaunchKernelGGL((stencil_kernel<float, 2>), dim3(blocks), dim3(256), 0, st, a);
  } else {
    if (a.order == 4) hipLaunchKernelGGL((stencil_kernel<double, 4>), dim3(blocks), dim3(256), 0, st, a);
    else hipLaunchKernelGGL((stencil_kernel<double, 2>), dim3(blocks), dim3(256), 0, st, a);
  }
}

// ---------------------------------------------------------------------------
// small elementwise helpers
// ---------------------------------------------------------------------------
template <class T>
__global__ __launch_bounds__(256) void scale_rows_kernel(const double* d, const T* X, T* Y, long ld, long rows,
                                                         int ncols) {
  long e = blockIdx.x * 256L + threadIdx.x;
  if (e >= rows * ncols) return;
  long c = e / rows, r = e % rows;
  T v = X[r + c * ld];
  Y[r + c * ld] = d ? (T)(v * (T)d[r]) : v;
}
void launch_scale_rows(const double* d, const void* X, void* Y, long ld, long rows, int ncols, int f32,
                       hipStream_t st) {
  long tot = rows * ncols;
  if (tot == 0) return;
  long blocks = (tot + 255) / 256;
  if (f32) hipLaunchKernelGGL(scale_rows_kernel<float>, dim3(blocks), dim3(256), 0, st, d, (const float*)X,
                              (float*)Y, ld, rows, ncols);
  else hipLaunchKernelGGL(scale_rows_kernel<double>, dim3(blocks), dim3(256), 0, st, d, (const double*)X,
                          (double*)Y, ld, rows, ncols);
}

__global__ __launch_bounds__(256) void to_f32_kernel(const double* X, float* Y, long ld, long rows, int ncols) {
  long e = blockIdx.x * 256L + threadIdx.x;
  if (e >= rows * ncols) return;
  long c = e / rows, r = e % rows;
  Y[r + c * ld] = (float)X[r + c * ld];
}
void launch_to_f32(const double* X, float* Y, long ld, long rows, int ncols, hipStream_t st) {
  long tot = rows * ncols;
  if (tot == 0) return;
  hipLaunchKernelGGL(to_f32_kernel, dim3((tot + 255) / 256), dim3(256), 0, st, X, Y, ld, rows, ncols);
}

// one workgroup per column, fixed-order tree reduction
template <class T>
__global__ __launch_bounds__(256) void colnorm2_kernel(const T* X, long ld, long rows, double* out) {
  const T* x = X + (long)blockIdx.x * ld;
  double s = 0;
  for (long r = threadIdx.x; r < rows; r += 256) {
    double v = (double)x[r];
    s += v * v;
  }
  __shared__ double red[4];
  s = wave_sum(s);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = s;
  __syncthreads();
  if (threadIdx.x == 0) out[blockIdx.x] = (red[0] + red[1]) + (red[2] + red[3]);
}
void launch_colnorm2(const void* X, int f32, long ld, long rows, int ncols, double* out, hipStream_t st) {
  if (ncols <= 0) return;
  if (f32) hipLaunchKernelGGL(colnorm2_kernel<float>, dim3(ncols), dim3(256), 0, st, (const float*)X, ld, rows, out);
  else hipLaunchKernelGGL(colnorm2_kernel<double>, dim3(ncols), dim3(256), 0, st, (const double*)X, ld, rows, out);
}

__global__ __launch_bounds__(256) void ritz_resid_kernel(const double* AX, const double* X, const double* lam,
                                                         double* W, float* W32, long ld, long rows) {
  long c = blockIdx.y;
  long r = blockIdx.x * 256L + threadIdx.x;
  if (r >= rows) return;
  double v = AX[r + c * ld] - X[r + c * ld] * lam[c];
  if (W) W[r + c * ld] = v;
  if (W32) W32[r + c * ld] = (float)v;
}
void launch_ritz_resid(const double* AX, const double* X, const double* lam, double* W, float* W32, long ld,
                       long rows, int ncols, hipStream_t st) {
  if (ncols <= 0) return;
  hipLaunchKernelGGL(ritz_resid_kernel, dim3((rows + 255) / 256, ncols), dim3(256), 0, st, AX, X, lam, W, W32, ld,
                     rows);
}

}  // namespace ppcg
