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
    case OP_ZEROINT: return sizeof(ZeroIntArgs);
    case OP_COPY: return sizeof(CopyArgs);
    case OP_PREP: return sizeof(PrepArgs);
    case OP_CHOL: return sizeof(CholArgs);
    case OP_D2H: return sizeof(D2HArgs);
  }
  return 0;
}

}  // namespace ppcg
