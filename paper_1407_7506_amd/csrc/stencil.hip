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
PPCG_DEV void stencil_body(const StencilArgs& a, unsigned wg, unsigned nwg) {
  const long n = (long)a.N * a.N * a.N;
  const unsigned bpc = (unsigned)((n + 255) / 256);
  unsigned L = xcd_remap(wg, nwg);
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
template <class T, int ORDER>
__global__ __launch_bounds__(256) void stencil_kernel(StencilArgs a) {
  stencil_body<T, ORDER>(a, blockIdx.x, gridDim.x);
}
template <class T, int ORDER>
__global__ __launch_bounds__(256) void stencil_grouped(const StencilArgs* jobs, const unsigned* start, int nj) {
  int j = find_job(start, nj, blockIdx.x);
  stencil_body<T, ORDER>(jobs[j], blockIdx.x - start[j], start[j + 1] - start[j]);
}

void launch_stencil(const StencilArgs& a, hipStream_t st) {
  long n = (long)a.N * a.N * a.N;
  unsigned blocks = (unsigned)(((n + 255) / 256) * a.ncols);
  int kind = a.f32 ? (a.order == 4 ? OP_STENCIL_F4 : OP_STENCIL_F2) : (a.order == 4 ? OP_STENCIL_D4 : OP_STENCIL_D2);
  if (g_rec) {
    g_rec->add(kind, &a, sizeof(a), blocks);
    return;
  }
  if (blocks == 0) return;
  switch (kind) {
    case OP_STENCIL_F4: hipLaunchKernelGGL((stencil_kernel<float, 4>), dim3(blocks), dim3(256), 0, st, a); break;
    case OP_STENCIL_F2: hipLaunchKernelGGL((stencil_kernel<float, 2>), dim3(blocks), dim3(256), 0, st, a); break;
    case OP_STENCIL_D4: hipLaunchKernelGGL((stencil_kernel<double, 4>), dim3(blocks), dim3(256), 0, st, a); break;
    case OP_STENCIL_D2: hipLaunchKernelGGL((stencil_kernel<double, 2>), dim3(blocks), dim3(256), 0, st, a); break;
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

// one workgroup per column, fixed-order tree reduction
template <class T>
PPCG_DEV void colnorm2_body(const ColnormArgs& a, unsigned wg, unsigned) {
  const T* x = (const T*)a.X + (long)wg * a.ld;
  double s = 0;
  for (long r = threadIdx.x; r < a.rows; r += 256) {
    double v = (double)x[r];
    s += v * v;
  }
  __shared__ double red[4];
  s = wave_sum(s);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = s;
  __syncthreads();
  if (threadIdx.x == 0) a.out[wg] = (red[0] + red[1]) + (red[2] + red[3]);
}
template <class T>
__global__ __launch_bounds__(256) void colnorm2_kernel(ColnormArgs a) {
  colnorm2_body<T>(a, blockIdx.x, gridDim.x);
}
template <class T>
__global__ __launch_bounds__(256) void colnorm2_grouped(const ColnormArgs* jobs, const unsigned* start, int nj) {
  int j = find_job(start, nj, blockIdx.x);
  colnorm2_body<T>(jobs[j], blockIdx.x - start[j], start[j + 1] - start[j]);
}
void launch_colnorm2(const void* X, int f32, long ld, long rows, int ncols, double* out, hipStream_t st) {
  ColnormArgs a{X, f32, ld, rows, ncols, out};
  unsigned blocks = ncols > 0 ? (unsigned)ncols : 0;
  if (g_rec) {
    g_rec->add(f32 ? OP_COLNORM_F : OP_COLNORM_D, &a, sizeof(a), blocks);
    return;
  }
  if (blocks == 0) return;
  if (f32) hipLaunchKernelGGL(colnorm2_kernel<float>, dim3(blocks), dim3(256), 0, st, a);
  else hipLaunchKernelGGL(colnorm2_kernel<double>, dim3(blocks), dim3(256), 0, st, a);
}

PPCG_DEV void ritz_body(const RitzArgs& a, unsigned wg, unsigned) {
  const unsigned bpc = (unsigned)((a.rows + 255) / 256);
  long c = wg / bpc;
  long r = (long)(wg % bpc) * 256 + threadIdx.x;
  if (r >= a.rows) return;
  double v = a.AX[r + c * a.ld] - a.X[r + c * a.ld] * a.lam[c];
  if (a.W) a.W[r + c * a.ld] = v;
  if (a.W32) a.W32[r + c * a.ld] = (float)v;
}
__global__ __launch_bounds__(256) void ritz_kernel(RitzArgs a) { ritz_body(a, blockIdx.x, gridDim.x); }
__global__ __launch_bounds__(256) void ritz_grouped(const RitzArgs* jobs, const unsigned* start, int nj) {
  int j = find_job(start, nj, blockIdx.x);
  ritz_body(jobs[j], blockIdx.x - start[j], start[j + 1] - start[j]);
}
void launch_ritz_resid(const double* AX, const double* X, const double* lam, double* W, float* W32, long ld,
                       long rows, int ncols, hipStream_t st) {
  RitzArgs a{AX, X, lam, W, W32, ld, rows, ncols};
  unsigned blocks = ncols > 0 ? (unsigned)(((rows + 255) / 256) * ncols) : 0;
  if (g_rec) {
    g_rec->add(OP_RITZ, &a, sizeof(a), blocks);
    return;
  }
  if (blocks == 0) return;
  hipLaunchKernelGGL(ritz_kernel, dim3(blocks), dim3(256), 0, st, a);
}

bool launch_grouped_stencil(int kind, const void* jobs, const unsigned* start, int nj, unsigned total,
                            hipStream_t st) {
  const StencilArgs* sj = (const StencilArgs*)jobs;
  switch (kind) {
    case OP_STENCIL_F4: hipLaunchKernelGGL((stencil_grouped<float, 4>), dim3(total), dim3(256), 0, st, sj, start, nj); return true;
    case OP_STENCIL_F2: hipLaunchKernelGGL((stencil_grouped<float, 2>), dim3(total), dim3(256), 0, st, sj, start, nj); return true;
    case OP_STENCIL_D4: hipLaunchKernelGGL((stencil_grouped<double, 4>), dim3(total), dim3(256), 0, st, sj, start, nj); return true;
    case OP_STENCIL_D2: hipLaunchKernelGGL((stencil_grouped<double, 2>), dim3(total), dim3(256), 0, st, sj, start, nj); return true;
    case OP_COLNORM_D:
      hipLaunchKernelGGL(colnorm2_grouped<double>, dim3(total), dim3(256), 0, st, (const ColnormArgs*)jobs, start, nj);
      return true;
    case OP_COLNORM_F:
      hipLaunchKernelGGL(colnorm2_grouped<float>, dim3(total), dim3(256), 0, st, (const ColnormArgs*)jobs, start, nj);
      return true;
    case OP_RITZ:
      hipLaunchKernelGGL(ritz_grouped, dim3(total), dim3(256), 0, st, (const RitzArgs*)jobs, start, nj);
      return true;
  }
  return false;
}

}  // namespace ppcg
