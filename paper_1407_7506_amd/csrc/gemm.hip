// Tall-skinny contractions on MFMA (gfx950):
//   gram    C = A^H (D B) summed over the rows of tall blocks (split-n partials)
//   reduce  deterministic fixed-order sum of the split partials
//   update  C <- beta * (D C) + alpha * A B with A tall, B small
// Used for the projections of W and P (Algorithm 3, steps 9-10), the
// Cholesky-QR Gram and X R^{-1} (section 5.5), the residual
// W = AX - X (X^H A X) (section 2) and the Rayleigh-Ritz Grams and rotation
// (section 5.6).
#include "common.hpp"
#include "kernels.hpp"

namespace ppcg {

// Column c of a segmented column set -> (pointer, is_f32).
template <class S>
PPCG_DEV const void* seg_col(const S& cs, int c, long ld, long joff, bool& f32) {
  const char* p = (const char*)cs.p[0];
  int base = 0;
  f32 = cs.f32[0];
#pragma unroll
  for (int s = 1; s < kMaxSeg; ++s) {
    if (s < cs.nseg && c >= cs.end[s - 1]) {
      p = (const char*)cs.p[s];
      base = cs.end[s - 1];
      f32 = cs.f32[s];
    }
  }
  long off = (long)(c - base) * ld + joff;
  return p + off * (f32 ? 4 : 8);
}

template <class T, int Q> struct VecLoad;
template <> struct VecLoad<double, 4> {
  static PPCG_DEV void load(const void* p, bool f32, double* o) {
    if (f32) {
      float4 v = *(const float4*)p;
      o[0] = v.x; o[1] = v.y; o[2] = v.z; o[3] = v.w;
    } else {
      const double2* q = (const double2*)p;
      double2 a = q[0], b = q[1];
      o[0] = a.x; o[1] = a.y; o[2] = b.x; o[3] = b.y;
    }
  }
};
template <> struct VecLoad<float, 4> {
  static PPCG_DEV void load(const void* p, bool, float* o) {
    float4 v = *(const float4*)p;
    o[0] = v.x; o[1] = v.y; o[2] = v.z; o[3] = v.w;
  }
};

// ---------------------------------------------------------------------------
// gram: one wave per (job, tile_i, tile_j, split); tile = (16 TM) x (16 TN).
// Lane group g = l/16 reads Q consecutive rows of its column, so the MFMA
// reduction index k = g maps to physical row r0 + g*Q + e in step e: every
// lane issues one contiguous vector load per column and step.
// ---------------------------------------------------------------------------
template <class T, int TM, int TN>
PPCG_DEV void gram_body(const GramArgs& a, unsigned wg, unsigned nwg) {
  constexpr int Q = 4;
  typedef typename AccT<T>::type acc_t;
  const int l = threadIdx.x;
  unsigned L = xcd_remap(wg, nwg);
  // logical index: tiles fastest, then split, then job
  const int ntile = a.tiles_i * a.tiles_j;
  int tile = L % ntile;
  int rest = L / ntile;
  int split = rest % a.splits;
  int job = rest / a.splits;
  int ti = tile % a.tiles_i, tj = tile / a.tiles_i;
  if (a.upper_only && ti * TM > tj * TN + TN - 1) return;  // tile wholly below diagonal
  const int i0 = ti * 16 * TM, j0 = tj * 16 * TN;
  const long joff = (long)job * a.job_col_off;
  const long rbeg = (long)split * a.chunk;
  long rend = rbeg + a.chunk;
  if (rend > a.rows) rend = a.rows;

  const int lc = l & 15, g = l >> 4;
  const void* pa[TM];
  bool fa[TM], va[TM];
  const void* pb[TN];
  bool fb[TN], vb[TN], sb[TN];
#pragma unroll
  for (int t = 0; t < TM; ++t) {
    int c = i0 + 16 * t + lc;
    va[t] = c < a.M;
    pa[t] = seg_col(a.A, va[t] ? c : 0, a.ld, joff, fa[t]);
  }
#pragma unroll
  for (int t = 0; t < TN; ++t) {
    int c = j0 + 16 * t + lc;
    vb[t] = c < a.N;
    pb[t] = seg_col(a.B, vb[t] ? c : 0, a.ld, joff, fb[t]);
    sb[t] = a.dsc != nullptr && c < a.nsc;
  }
  acc_t acc[TM][TN];
#pragma unroll
  for (int x = 0; x < TM; ++x)
#pragma unroll
    for (int y = 0; y < TN; ++y) acc[x][y] = acc_t{0, 0, 0, 0};

  for (long r = rbeg; r < rend; r += 4 * Q) {
    const long rr = r + g * Q;
    T av[TM][Q], bv[TN][Q];
#pragma unroll
    for (int t = 0; t < TM; ++t) {
      if (va[t]) {
        const char* p = (const char*)pa[t] + rr * (fa[t] ? 4 : 8);
        VecLoad<T, Q>::load(p, fa[t], av[t]);
      } else {
#pragma unroll
        for (int e = 0; e < Q; ++e) av[t][e] = 0;
      }
    }
    T dv[Q];
    if (a.dsc) {
      const double* dp = a.dsc + rr;
#pragma unroll
      for (int e = 0; e < Q; ++e) dv[e] = (T)dp[e];
    }
#pragma unroll
    for (int t = 0; t < TN; ++t) {
      if (vb[t]) {
        const char* p = (const char*)pb[t] + rr * (fb[t] ? 4 : 8);
        VecLoad<T, Q>::load(p, fb[t], bv[t]);
        if (sb[t]) {
#pragma unroll
          for (int e = 0; e < Q; ++e) bv[t][e] *= dv[e];
        }
      } else {
#pragma unroll
        for (int e = 0; e < Q; ++e) bv[t][e] = 0;
      }
    }
#pragma unroll
    for (int e = 0; e < Q; ++e)
#pragma unroll
      for (int x = 0; x < TM; ++x)
#pragma unroll
        for (int y = 0; y < TN; ++y) acc[x][y] = mfma(av[x][e], bv[y][e], acc[x][y]);
  }
  // store partial: out + (job*splits + split)*split_stride + i + j*ldo
  T* out = (T*)a.out + ((long)job * a.splits + split) * a.split_stride;
#pragma unroll
  for (int x = 0; x < TM; ++x)
#pragma unroll
    for (int y = 0; y < TN; ++y)
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        int i = i0 + 16 * x + acc_row<T>(l, v);
        int j = j0 + 16 * y + lc;
        if (i < a.M && j < a.N) out[i + (long)j * a.ldo] = acc[x][y][v];
      }
}

// SITE only distinguishes call sites in profiles (projection Grams = 1,
// per-block Grams = 2, others = 0); the code is identical.
template <class T, int TM, int TN, int SITE>
__global__ __launch_bounds__(64) void gram_kernel(GramArgs a) {
  gram_body<T, TM, TN>(a, blockIdx.x, gridDim.x);
}
template <class T, int TM, int TN, int SITE>
__global__ __launch_bounds__(64) void gram_grouped(const GramArgs* jobs, const unsigned* start, int nj) {
  int j = find_job(start, nj, blockIdx.x);
  gram_body<T, TM, TN>(jobs[j], blockIdx.x - start[j], start[j + 1] - start[j]);
}

// Sum of split partials in a fixed order.  dst[i + j*ldd] (+)= sum_s part[s].
template <class T>
PPCG_DEV void reduce_body(const ReduceArgs& r, unsigned wg, unsigned) {
  long e = wg * 256L + threadIdx.x;
  long per = (long)r.M * r.N;
  if (e >= per * r.njobs) return;
  int job = e / per;
  long ij = e % per;
  int i = ij % r.M, j = ij / r.M;
  if (r.upper_only && i > j) return;
  const T* p = (const T*)r.part + (long)job * r.splits * r.split_stride + i + (long)j * r.ldp;
  double s = 0;
  for (int t = 0; t < r.splits; ++t) s += (double)p[t * r.split_stride];
  T* dbase = (T*)r.dst + (long)job * r.dst_job_stride;
  T* d = dbase + i + (long)j * r.ldd;
  T v = (T)(r.alpha * s + (r.beta != 0 ? r.beta * (double)*d : 0.0));
  *d = v;
  // upper_only: the result is Hermitian by construction; mirror it
  if (r.upper_only && i < j) dbase[j + (long)i * r.ldd] = v;
}
template <class T>
__global__ __launch_bounds__(256) void reduce_kernel(ReduceArgs r) {
  reduce_body<T>(r, blockIdx.x, gridDim.x);
}
template <class T>
__global__ __launch_bounds__(256) void reduce_grouped(const ReduceArgs* jobs, const unsigned* start, int nj) {
  int j = find_job(start, nj, blockIdx.x);
  reduce_body<T>(jobs[j], blockIdx.x - start[j], start[j + 1] - start[j]);
}

// ---------------------------------------------------------------------------
// update: C[r, j] = beta * (D C)[r, j] + alpha * sum_k A[r, k] B[k, j]
// The MFMA computes the transposed tile (j, r) so that the epilogue writes
// 16 consecutive rows of a column per lane group.  Lane group g reads
// Q consecutive k of the small matrix B in one vector load.
// ---------------------------------------------------------------------------
template <class T, int TJ, int TR>
PPCG_DEV void update_body(const UpdateArgs& a, unsigned wg, unsigned nwg) {
  constexpr int Q = 4;
  typedef typename AccT<T>::type acc_t;
  const int l = threadIdx.x, lc = l & 15, g = l >> 4;
  unsigned L = xcd_remap(wg, nwg);
  // column tiles fastest so the row tile of A is shared inside one XCD
  int tj = L % a.tiles_j;
  int rest = L / a.tiles_j;
  int tr = rest % a.tiles_r;
  int job = rest / a.tiles_r;
  const int j0 = tj * 16 * TJ;
  const long r0 = (long)tr * 16 * TR;
  const T* A = (const T*)a.A + (long)job * a.job_a_off;
  const T* B = (const T*)a.B + (long)job * a.job_b_off;
  int kend = a.K;
  if (a.b_upper) {
    int lim = j0 + 16 * TJ;
    if (lim < kend) kend = lim;
  }
  acc_t acc[TJ][TR];
#pragma unroll
  for (int x = 0; x < TJ; ++x)
#pragma unroll
    for (int y = 0; y < TR; ++y) acc[x][y] = acc_t{0, 0, 0, 0};
  bool vj[TJ];
  const T* bcol[TJ];
#pragma unroll
  for (int x = 0; x < TJ; ++x) {
    int j = j0 + 16 * x + lc;
    vj[x] = j < a.N;
    bcol[x] = B + (long)(vj[x] ? j : 0) * a.ldb;
  }
  for (int k0 = 0; k0 < kend; k0 += 4 * Q) {
    const int kb = k0 + g * Q;
    T bv[TJ][Q], av[TR][Q];
#pragma unroll
    for (int x = 0; x < TJ; ++x)
#pragma unroll
      for (int e = 0; e < Q; ++e) bv[x][e] = (vj[x] && kb + e < kend) ? bcol[x][kb + e] : (T)0;
#pragma unroll
    for (int y = 0; y < TR; ++y) {
      const T* ap = A + r0 + 16 * y + lc;
#pragma unroll
      for (int e = 0; e < Q; ++e) av[y][e] = (kb + e < kend) ? ap[(long)(kb + e) * a.lda] : (T)0;
    }
#pragma unroll
    for (int e = 0; e < Q; ++e)
#pragma unroll
      for (int x = 0; x < TJ; ++x)
#pragma unroll
        for (int y = 0; y < TR; ++y) acc[x][y] = mfma(bv[x][e], av[y][e], acc[x][y]);
  }
  const T alpha = (T)a.alpha, beta = (T)a.beta;
#pragma unroll
  for (int x = 0; x < TJ; ++x)
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      int j = j0 + 16 * x + acc_row<T>(l, v);
      if (j >= a.N) continue;
      T* cp;
      bool scaled;
      if (j < a.N0) {
        cp = (T*)a.C0 + (long)job * a.job_c_off + (long)j * a.ldc;
        scaled = a.dsc != nullptr;
      } else {
        cp = (T*)a.C1 + (long)job * a.job_c_off + (long)(j - a.N0) * a.ldc;
        scaled = false;
      }
      float* c32 = a.C32 ? (float*)a.C32 + (long)job * a.job_c_off + (long)j * a.ldc : nullptr;
#pragma unroll
      for (int y = 0; y < TR; ++y) {
        long r = r0 + 16 * y + lc;
        T val = alpha * acc[x][y][v];
        if (a.beta != 0) {
          T c = cp[r];
          if (scaled) c *= (T)a.dsc[r];
          val += beta * c;
        }
        if (!a.c0_keep) cp[r] = val;
        if (c32) c32[r] = (float)val;
      }
    }
}

template <class T, int TJ, int TR, int SITE>
__global__ __launch_bounds__(64) void update_kernel(UpdateArgs a) {
  update_body<T, TJ, TR>(a, blockIdx.x, gridDim.x);
}
template <class T, int TJ, int TR, int SITE>
__global__ __launch_bounds__(64) void update_grouped(const UpdateArgs* jobs, const unsigned* start, int nj) {
  int j = find_job(start, nj, blockIdx.x);
  update_body<T, TJ, TR>(jobs[j], blockIdx.x - start[j], start[j + 1] - start[j]);
}

// ---------------------------------------------------------------------------
// host launchers
// ---------------------------------------------------------------------------
constexpr int GTM = 4, GTN = 4, UTJ = 4, UTR = 4;

void gram_tiles(GramArgs& a) {
  a.tiles_i = (a.M + 16 * GTM - 1) / (16 * GTM);
  a.tiles_j = (a.N + 16 * GTN - 1) / (16 * GTN);
}
void update_tiles(UpdateArgs& a) {
  a.tiles_j = (a.N + 16 * UTJ - 1) / (16 * UTJ);
  a.tiles_r = (int)(a.rows / (16 * UTR));
}

void launch_gram(const GramArgs& a0, bool f32acc, hipStream_t st) {
  GramArgs a = a0;
  gram_tiles(a);
  unsigned blocks = (unsigned)((long)a.tiles_i * a.tiles_j * a.splits * a.njobs);
  if (blocks == 0) return;
  int kind = (f32acc ? OP_GRAM_F0 : OP_GRAM_D0) + (a.site == 1 ? 1 : a.site == 2 ? 2 : 0);
  if (g_rec) {
    g_rec->add(kind, &a, sizeof(a), blocks);
    return;
  }
#define PPCG_GRAM(T, S) hipLaunchKernelGGL((gram_kernel<T, GTM, GTN, S>), dim3(blocks), dim3(64), 0, st, a)
  switch (kind) {
    case OP_GRAM_D0: PPCG_GRAM(double, 0); break;
    case OP_GRAM_D1: PPCG_GRAM(double, 1); break;
    case OP_GRAM_D2: PPCG_GRAM(double, 2); break;
    case OP_GRAM_F0: PPCG_GRAM(float, 0); break;
    case OP_GRAM_F1: PPCG_GRAM(float, 1); break;
    case OP_GRAM_F2: PPCG_GRAM(float, 2); break;
  }
#undef PPCG_GRAM
}

void launch_reduce(const ReduceArgs& r, bool f32, hipStream_t st) {
  long tot = (long)r.M * r.N * r.njobs;
  unsigned blocks = (unsigned)((tot + 255) / 256);
  if (blocks == 0) return;
  if (g_rec) {
    g_rec->add(f32 ? OP_REDUCE_F : OP_REDUCE_D, &r, sizeof(r), blocks);
    return;
  }
  if (f32) hipLaunchKernelGGL(reduce_kernel<float>, dim3(blocks), dim3(256), 0, st, r);
  else hipLaunchKernelGGL(reduce_kernel<double>, dim3(blocks), dim3(256), 0, st, r);
}

void launch_update(const UpdateArgs& a0, bool f32, hipStream_t st) {
  UpdateArgs a = a0;
  update_tiles(a);
  unsigned blocks = (unsigned)((long)a.tiles_j * a.tiles_r);
  if (blocks == 0) return;
  int kind = (f32 ? OP_UPDATE_F0 : OP_UPDATE_D0) + (a.site == 1 ? 1 : 0);
  if (g_rec) {
    g_rec->add(kind, &a, sizeof(a), blocks);
    return;
  }
#define PPCG_UPD(T, S) hipLaunchKernelGGL((update_kernel<T, UTJ, UTR, S>), dim3(blocks), dim3(64), 0, st, a)
  switch (kind) {
    case OP_UPDATE_D0: PPCG_UPD(double, 0); break;
    case OP_UPDATE_D1: PPCG_UPD(double, 1); break;
    case OP_UPDATE_F0: PPCG_UPD(float, 0); break;
    case OP_UPDATE_F1: PPCG_UPD(float, 1); break;
  }
#undef PPCG_UPD
}

bool launch_grouped_gemm(int kind, const void* jobs, const unsigned* start, int nj, unsigned total, hipStream_t st) {
#define PPCG_GG(T, S) \
  hipLaunchKernelGGL((gram_grouped<T, GTM, GTN, S>), dim3(total), dim3(64), 0, st, (const GramArgs*)jobs, start, nj)
#define PPCG_GU(T, S)                                                                                   \
  hipLaunchKernelGGL((update_grouped<T, UTJ, UTR, S>), dim3(total), dim3(64), 0, st, (const UpdateArgs*)jobs, \
                     start, nj)
  switch (kind) {
    case OP_GRAM_D0: PPCG_GG(double, 0); return true;
    case OP_GRAM_D1: PPCG_GG(double, 1); return true;
    case OP_GRAM_D2: PPCG_GG(double, 2); return true;
    case OP_GRAM_F0: PPCG_GG(float, 0); return true;
    case OP_GRAM_F1: PPCG_GG(float, 1); return true;
    case OP_GRAM_F2: PPCG_GG(float, 2); return true;
    case OP_UPDATE_D0: PPCG_GU(double, 0); return true;
    case OP_UPDATE_D1: PPCG_GU(double, 1); return true;
    case OP_UPDATE_F0: PPCG_GU(float, 0); return true;
    case OP_UPDATE_F1: PPCG_GU(float, 1); return true;
    case OP_REDUCE_D:
      hipLaunchKernelGGL(reduce_grouped<double>, dim3(total), dim3(256), 0, st, (const ReduceArgs*)jobs, start, nj);
      return true;
    case OP_REDUCE_F:
      hipLaunchKernelGGL(reduce_grouped<float>, dim3(total), dim3(256), 0, st, (const ReduceArgs*)jobs, start, nj);
      return true;
  }
#undef PPCG_GG
#undef PPCG_GU
  return false;
}

}  // namespace ppcg
