// Set-up kernel: Jacobi preconditioner T = diag(H)^{-1} (the paper only
// requires T Hermitian positive definite, Theorem 2), float copy of V, and
// the scan for NaN / non-positive diagonal.
#include "common.hpp"
#include "kernels.hpp"

namespace ppcg {

PPCG_DEV void prep_body(const PrepArgs& a, unsigned wg, unsigned nwg) {
  double mn = 1e308;
  int bad = 0;
  for (long r = wg * 256L + threadIdx.x; r < a.n; r += (long)nwg * 256) {
    double v = a.V[r];
    double d = a.c0 + v;
    if (v != v) bad = 1;
    mn = fmin(mn, d);
    a.td[r] = 1.0 / d;
    if (a.V32) a.V32[r] = (float)v;
  }
  for (int o = 32; o > 0; o >>= 1) mn = fmin(mn, __shfl_xor(mn, o, 64));
  __shared__ double red[4];
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = mn;
  if (bad) atomicOr(a.nan_flag, 1);
  __syncthreads();
  if (threadIdx.x == 0) a.dmin_part[wg] = fmin(fmin(red[0], red[1]), fmin(red[2], red[3]));
}
__global__ __launch_bounds__(256) void prep_kernel(PrepArgs a) { prep_body(a, blockIdx.x, gridDim.x); }
__global__ __launch_bounds__(256) void prep_grouped(const PrepArgs* jobs, const unsigned* start, int nj) {
  int j = find_job(start, nj, blockIdx.x);
  prep_body(jobs[j], blockIdx.x - start[j], start[j + 1] - start[j]);
}

void launch_prep_diag(const double* V, long n, double c0, double* td, float* V32, double* dmin_part, int nparts,
                      int* nan_flag, hipStream_t st) {
  PrepArgs a{V, n, c0, td, V32, dmin_part, nparts, nan_flag};
  if (g_rec) {
    g_rec->add(OP_PREP, &a, sizeof(a), (unsigned)nparts);
    return;
  }
  hipLaunchKernelGGL(prep_kernel, dim3(nparts), dim3(256), 0, st, a);
}

// Start block X0 ~ N(0,1) drawn on the device (ppcg_solve with X0 = NULL).
// Philox-4x32-10 (Salmon, Moraes, Dror, Shaw, "Parallel random numbers: as
// easy as 1, 2, 3", SC 2011): counter (row, column, 0, 0), key (seed low,
// seed high) -> four 32-bit words -> two 53-bit uniforms in (0, 1) -> two
// normals by the Box-Muller transform.  Real blocks take the first normal;
// complex blocks take both, scaled by sqrt(1/2) (real and imaginary parts
// N(0, 1/2)).
PPCG_DEV void philox4x32_10(uint32_t c[4], uint32_t k0, uint32_t k1) {
  for (int r = 0; r < 10; ++r) {
    const uint64_t p0 = (uint64_t)0xD2511F53u * c[0], p1 = (uint64_t)0xCD9E8D57u * c[2];
    const uint32_t hi0 = (uint32_t)(p0 >> 32), lo0 = (uint32_t)p0;
    const uint32_t hi1 = (uint32_t)(p1 >> 32), lo1 = (uint32_t)p1;
    const uint32_t n0 = hi1 ^ c[1] ^ k0, n2 = hi0 ^ c[3] ^ k1;
    c[0] = n0;
    c[1] = lo1;
    c[2] = n2;
    c[3] = lo0;
    k0 += 0x9E3779B9u;
    k1 += 0xBB67AE85u;
  }
}
__global__ __launch_bounds__(256) void randn_kernel(double* X, long ld, long n, int ncols, uint64_t seed, int cplx) {
  const long r = blockIdx.x * 256L + threadIdx.x;
  const int col = blockIdx.y;
  if (r >= n || col >= ncols) return;
  uint32_t c[4] = {(uint32_t)r, (uint32_t)col, (uint32_t)(r >> 32), 0u};
  philox4x32_10(c, (uint32_t)seed, (uint32_t)(seed >> 32));
  const double two53 = 1.0 / 9007199254740992.0;
  const double u1 = ((double)(c[0] >> 5) * 67108864.0 + (double)(c[1] >> 6) + 0.5) * two53;
  const double u2 = ((double)(c[2] >> 5) * 67108864.0 + (double)(c[3] >> 6) + 0.5) * two53;
  const double rad = sqrt(-2.0 * log(u1));
  double sn, cs;
  sincospi(2.0 * u2, &sn, &cs);
  if (cplx) {
    const double s = 0.70710678118654752440;
    X[2 * (r + col * ld)] = s * rad * cs;
    X[2 * (r + col * ld) + 1] = s * rad * sn;
  } else {
    X[r + col * ld] = rad * cs;
  }
}

void launch_randn(double* X, long ld, long n, int ncols, uint64_t seed, bool cplx, hipStream_t st) {
  if (n <= 0 || ncols <= 0) return;
  hipLaunchKernelGGL(randn_kernel, dim3((unsigned)((n + 255) / 256), (unsigned)ncols), dim3(256), 0, st, X, ld, n,
                     ncols, seed, cplx ? 1 : 0);
}

bool launch_grouped_prep(int kind, const void* jobs, const unsigned* start, int nj, unsigned total, hipStream_t st) {
  if (kind != OP_PREP) return false;
  hipLaunchKernelGGL(prep_grouped, dim3(total), dim3(256), 0, st, (const PrepArgs*)jobs, start, nj);
  return true;
}

size_t op_args_size(int kind) {
  if (kind >= OP_GRAM_D0 && kind <= OP_GRAMB_2) return sizeof(GramArgs);
  if (kind >= OP_REDUCE_D && kind <= OP_REDUCE_C) return sizeof(ReduceArgs);
  if (kind >= OP_UPDATE_D0 && kind <= OP_UPDATEL_F1) return sizeof(UpdateArgs);
  if (kind >= OP_STENCIL_D2 && kind <= OP_STENCIL_C4) return sizeof(StencilArgs);
  if (kind >= OP_PENCIL24 && kind <= OP_PENCILZ96) return sizeof(PencilArgs);
  if (kind >= OP_BUPD_D4 && kind <= OP_BUPD_C32) return sizeof(BlockUpdArgs);
  switch (kind) {
    case OP_COLNORM_D: case OP_COLNORM_F: return sizeof(ColnormArgs);
    case OP_RITZ: return sizeof(RitzArgs);
    case OP_TRANSPOSE: return sizeof(TransposeArgs);
    case OP_FILL: return sizeof(FillArgs);
    case OP_SETDIAG: return sizeof(SetDiagArgs);
    case OP_SYMM: return sizeof(SymmArgs);
    case OP_OFFDIAG: return sizeof(OffdiagArgs);
    case OP_FROB2: return sizeof(Frob2Args);
    case OP_ORTH: return sizeof(OrthArgs);
    case OP_POLAR: return sizeof(PolarArgs);
    case OP_ADDDIAG: return sizeof(AddDiagArgs);
    case OP_TRACE: return sizeof(TraceArgs);
    case OP_TOF32: return sizeof(ToF32Args);
    case OP_ZEROINT: return sizeof(ZeroIntArgs);
    case OP_COPY: return sizeof(CopyArgs);
    case OP_PREP: return sizeof(PrepArgs);
    case OP_CHOL: return sizeof(CholArgs);
    case OP_D2H: return sizeof(D2HArgs);
  }
  return 0;
}

}  // namespace ppcg
