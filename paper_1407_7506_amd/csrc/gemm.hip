// Tall-skinny contractions on MFMA (gfx950):
//   gram    C = A^H (D B) summed over the rows of tall blocks (split-n partials)
//   reduce  deterministic fixed-order sum of the split partials
//   update  C <- beta * (D C) + alpha * A B with A tall, B small
// Used for the projections of W and P (Algorithm 3, steps 9-10), the
// Cholesky-QR Gram and X R^{-1} (section 5.5), the residual
// W = AX - X (X^H A X) (section 2) and the Rayleigh-Ritz Grams and rotation
// (section 5.6).  Real operands use one MFMA per 16x16x4 tile; complex
// operands four (real and imaginary parts in separate accumulators).
#include "common.hpp"
#include "kernels.hpp"

namespace ppcg {

// Column c of a segmented column set -> (pointer, single precision flag).
template <class S>
PPCG_DEV const void* seg_col(const S& cs, int c, long ld, long joff, bool& f32, int esz64) {
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
  return p + off * (f32 ? esz64 / 2 : esz64);
}

// Q = 4 consecutive rows of one column into re[] (and im[] when complex)
template <class T, bool CPLX> struct Load4;
template <> struct Load4<double, false> {
  static PPCG_DEV void go(const char* p, bool f32, double* re, double*) {
    if (f32) {
      float4 v = *(const float4*)p;
      re[0] = v.x; re[1] = v.y; re[2] = v.z; re[3] = v.w;
    } else {
      const double2* q = (const double2*)p;
      double2 a = q[0], b = q[1];
      re[0] = a.x; re[1] = a.y; re[2] = b.x; re[3] = b.y;
    }
  }
};
template <> struct Load4<float, false> {
  static PPCG_DEV void go(const char* p, bool, float* re, float*) {
    float4 v = *(const float4*)p;
    re[0] = v.x; re[1] = v.y; re[2] = v.z; re[3] = v.w;
  }
};
template <> struct Load4<double, true> {
  static PPCG_DEV void go(const char* p, bool f32, double* re, double* im) {
    if (f32) {
      const float4* q = (const float4*)p;
      float4 a = q[0], b = q[1];
      re[0] = a.x; im[0] = a.y; re[1] = a.z; im[1] = a.w;
      re[2] = b.x; im[2] = b.y; re[3] = b.z; im[3] = b.w;
    } else {
      const double2* q = (const double2*)p;
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        double2 v = q[e];
        re[e] = v.x;
        im[e] = v.y;
      }
    }
  }
};
template <> struct Load4<float, true> {
  static PPCG_DEV void go(const char* p, bool, float* re, float* im) {
    const float4* q = (const float4*)p;
    float4 a = q[0], b = q[1];
    re[0] = a.x; im[0] = a.y; re[1] = a.z; im[1] = a.w;
    re[2] = b.x; im[2] = b.y; re[3] = b.z; im[3] = b.w;
  }
};

// ---------------------------------------------------------------------------
// gram: one wave per (job, tile_i, tile_j, split); tile = (16 TM) x (16 TN).
// Lane group g = l/16 reads Q consecutive rows of its column, so the MFMA
// reduction index k = g maps to physical row r0 + g*Q + e in step e: every
// lane issues one contiguous vector load per column and step.
// ---------------------------------------------------------------------------
template <class T, int TM, int TN, bool CPLX>
PPCG_DEV void gram_body(const GramArgs& a, unsigned wg, unsigned nwg) {
  constexpr int Q = 4;
  constexpr int NC = CPLX ? 2 : 1;
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
  const int esz64 = CPLX ? 16 : 8;

  const int lc = l & 15, g = l >> 4;
  const void* pa[TM];
  bool fa[TM], va[TM];
  const void* pb[TN];
  bool fb[TN], vb[TN], sb[TN];
#pragma unroll
  for (int t = 0; t < TM; ++t) {
    int c = i0 + 16 * t + lc;
    va[t] = c < a.M;
    pa[t] = seg_col(a.A, va[t] ? c : 0, a.ld, joff, fa[t], esz64);
  }
#pragma unroll
  for (int t = 0; t < TN; ++t) {
    int c = j0 + 16 * t + lc;
    vb[t] = c < a.N;
    pb[t] = seg_col(a.B, vb[t] ? c : 0, a.ld, joff, fb[t], esz64);
    sb[t] = a.dsc != nullptr && c < a.nsc;
  }
  acc_t acc[NC][TM][TN];
#pragma unroll
  for (int z = 0; z < NC; ++z)
#pragma unroll
    for (int x = 0; x < TM; ++x)
#pragma unroll
      for (int y = 0; y < TN; ++y) acc[z][x][y] = acc_t{0, 0, 0, 0};

  for (long r = rbeg; r < rend; r += 4 * Q) {
    const long rr = r + g * Q;
    T ar[TM][Q], ai[TM][Q], br[TN][Q], bi[TN][Q];
#pragma unroll
    for (int t = 0; t < TM; ++t) {
      if (va[t]) {
        const char* p = (const char*)pa[t] + rr * (fa[t] ? esz64 / 2 : esz64);
        Load4<T, CPLX>::go(p, fa[t], ar[t], ai[t]);
      } else {
#pragma unroll
        for (int e = 0; e < Q; ++e) ar[t][e] = ai[t][e] = 0;
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
        const char* p = (const char*)pb[t] + rr * (fb[t] ? esz64 / 2 : esz64);
        Load4<T, CPLX>::go(p, fb[t], br[t], bi[t]);
        if (sb[t]) {
#pragma unroll
          for (int e = 0; e < Q; ++e) {
            br[t][e] *= dv[e];
            if (CPLX) bi[t][e] *= dv[e];
          }
        }
      } else {
#pragma unroll
        for (int e = 0; e < Q; ++e) br[t][e] = bi[t][e] = 0;
      }
    }
#pragma unroll
    for (int e = 0; e < Q; ++e)
#pragma unroll
      for (int x = 0; x < TM; ++x)
#pragma unroll
        for (int y = 0; y < TN; ++y) {
          acc[0][x][y] = mfma(ar[x][e], br[y][e], acc[0][x][y]);
          if (CPLX) {  // conj(a) b = (ar br + ai bi) + i (ar bi - ai br)
            acc[0][x][y] = mfma(ai[x][e], bi[y][e], acc[0][x][y]);
            acc[NC - 1][x][y] = mfma(ar[x][e], bi[y][e], acc[NC - 1][x][y]);
            acc[NC - 1][x][y] = mfma(-ai[x][e], br[y][e], acc[NC - 1][x][y]);
          }
        }
  }
  // store partial: out + (job*splits + split)*split_stride + i + j*ldo
  T* out = (T*)a.out + (((long)job * a.splits + split) * a.split_stride) * NC;
#pragma unroll
  for (int x = 0; x < TM; ++x)
#pragma unroll
    for (int y = 0; y < TN; ++y)
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        int i = i0 + 16 * x + acc_row<T>(l, v);
        int j = j0 + 16 * y + lc;
        if (i < a.M && j < a.N) {
          long o = (i + (long)j * a.ldo) * NC;
          out[o] = acc[0][x][y][v];
          if (CPLX) out[o + 1] = acc[NC - 1][x][y][v];
        }
      }
}

// SITE only distinguishes call sites in profiles (projection Grams = 1,
// per-block Grams = 2, others = 0); the code is identical.
template <class T, int TM, int TN, bool CPLX, int SITE>
__global__ __launch_bounds__(64) void gram_kernel(GramArgs a) {
  gram_body<T, TM, TN, CPLX>(a, blockIdx.x, gridDim.x);
}
template <class T, int TM, int TN, bool CPLX, int SITE>
__global__ __launch_bounds__(64) void gram_grouped(const GramArgs* jobs, const unsigned* start, int nj) {
  int j = find_job(start, nj, blockIdx.x);
  gram_body<T, TM, TN, CPLX>(jobs[j], blockIdx.x - start[j], start[j + 1] - start[j]);
}

// Sum of split partials in a fixed order.  dst[i + j*ldd] = alpha * sum_s part[s]
// (+ beta dst); with upper_only the result is Hermitian and is mirrored.
template <class T, bool CPLX>
PPCG_DEV void reduce_body(const ReduceArgs& r, unsigned wg, unsigned) {
  constexpr int NC = CPLX ? 2 : 1;
  long e = wg * 256L + threadIdx.x;
  long per = (long)r.M * r.N;
  if (e >= per * r.njobs) return;
  int job = e / per;
  long ij = e % per;
  int i = ij % r.M, j = ij / r.M;
  if (r.upper_only && i > j) return;
  const T* p = (const T*)r.part + ((long)job * r.splits * r.split_stride + i + (long)j * r.ldp) * NC;
  double s0 = 0, s1 = 0;
  for (int t = 0; t < r.splits; ++t) {
    s0 += (double)p[(long)t * r.split_stride * NC];
    if (CPLX) s1 += (double)p[(long)t * r.split_stride * NC + 1];
  }
  T* dbase = (T*)r.dst + (long)job * r.dst_job_stride * NC;
  T* d = dbase + (i + (long)j * r.ldd) * NC;
  T v0 = (T)(r.alpha * s0 + (r.beta != 0 ? r.beta * (double)d[0] : 0.0));
  T v1 = CPLX ? (T)(r.alpha * s1 + (r.beta != 0 ? r.beta * (double)d[1] : 0.0)) : (T)0;
  if (r.upper_only && i == j) v1 = 0;  // Hermitian diagonal is real
  d[0] = v0;
  if (CPLX) d[1] = v1;
  if (r.upper_only && i < j) {
    T* m = dbase + (j + (long)i * r.ldd) * NC;
    m[0] = v0;
    if (CPLX) m[1] = -v1;
  }
}
template <class T, bool CPLX>
__global__ __launch_bounds__(256) void reduce_kernel(ReduceArgs r) {
  reduce_body<T, CPLX>(r, blockIdx.x, gridDim.x);
}
template <class T, bool CPLX>
__global__ __launch_bounds__(256) void reduce_grouped(const ReduceArgs* jobs, const unsigned* start, int nj) {
  int j = find_job(start, nj, blockIdx.x);
  reduce_body<T, CPLX>(jobs[j], blockIdx.x - start[j], start[j + 1] - start[j]);
}

// ---------------------------------------------------------------------------
// update: C[r, j] = beta * (D C)[r, j] + alpha * sum_k A[r, k] B[k, j]
// The MFMA computes the transposed tile (j, r) so that the epilogue writes
// 16 consecutive rows of a column per lane group.  Lane group g reads
// Q consecutive k of the small matrix B in one vector load.
// ---------------------------------------------------------------------------
template <class T, int TJ, int TR, bool CPLX>
PPCG_DEV void update_body(const UpdateArgs& a, unsigned wg, unsigned nwg) {
  constexpr int Q = 4;
  constexpr int NC = CPLX ? 2 : 1;
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
  const T* A = (const T*)a.A + (long)job * a.job_a_off * NC;
  const T* B = (const T*)a.B + (long)job * a.job_b_off * NC;
  int kend = a.K;
  if (a.b_upper) {
    int lim = j0 + 16 * TJ;
    if (lim < kend) kend = lim;
  }
  acc_t acc[NC][TJ][TR];
#pragma unroll
  for (int z = 0; z < NC; ++z)
#pragma unroll
    for (int x = 0; x < TJ; ++x)
#pragma unroll
      for (int y = 0; y < TR; ++y) acc[z][x][y] = acc_t{0, 0, 0, 0};
  bool vj[TJ];
  const T* bcol[TJ];
#pragma unroll
  for (int x = 0; x < TJ; ++x) {
    int j = j0 + 16 * x + lc;
    vj[x] = j < a.N;
    bcol[x] = B + (long)(vj[x] ? j : 0) * a.ldb * NC;
  }
  for (int k0 = 0; k0 < kend; k0 += 4 * Q) {
    const int kb = k0 + g * Q;
    T br[TJ][Q], bi[TJ][Q], ar[TR][Q], ai[TR][Q];
#pragma unroll
    for (int x = 0; x < TJ; ++x)
#pragma unroll
      for (int e = 0; e < Q; ++e) {
        bool ok = vj[x] && kb + e < kend;
        br[x][e] = ok ? bcol[x][(kb + e) * NC] : (T)0;
        bi[x][e] = (CPLX && ok) ? bcol[x][(kb + e) * NC + NC - 1] : (T)0;
      }
#pragma unroll
    for (int y = 0; y < TR; ++y) {
      const T* ap = A + (r0 + 16 * y + lc) * NC;
#pragma unroll
      for (int e = 0; e < Q; ++e) {
        bool ok = kb + e < kend;
        ar[y][e] = ok ? ap[(long)(kb + e) * a.lda * NC] : (T)0;
        ai[y][e] = (CPLX && ok) ? ap[(long)(kb + e) * a.lda * NC + NC - 1] : (T)0;
      }
    }
#pragma unroll
    for (int e = 0; e < Q; ++e)
#pragma unroll
      for (int x = 0; x < TJ; ++x)
#pragma unroll
        for (int y = 0; y < TR; ++y) {
          acc[0][x][y] = mfma(br[x][e], ar[y][e], acc[0][x][y]);
          if (CPLX) {  // b a = (br ar - bi ai) + i (br ai + bi ar)
            acc[0][x][y] = mfma(-bi[x][e], ai[y][e], acc[0][x][y]);
            acc[NC - 1][x][y] = mfma(br[x][e], ai[y][e], acc[NC - 1][x][y]);
            acc[NC - 1][x][y] = mfma(bi[x][e], ar[y][e], acc[NC - 1][x][y]);
          }
        }
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
        cp = (T*)a.C0 + ((long)job * a.job_c_off + (long)j * a.ldc) * NC;
        scaled = a.dsc != nullptr;
      } else {
        cp = (T*)a.C1 + ((long)job * a.job_c_off + (long)(j - a.N0) * a.ldc) * NC;
        scaled = false;
      }
      float* c32 = a.C32 ? (float*)a.C32 + ((long)job * a.job_c_off + (long)j * a.ldc) * NC : nullptr;
#pragma unroll
      for (int y = 0; y < TR; ++y) {
        long r = (r0 + 16 * y + lc) * NC;
        T v0 = alpha * acc[0][x][y][v];
        T v1 = CPLX ? alpha * acc[NC - 1][x][y][v] : (T)0;
        if (a.beta != 0) {
          T c0 = cp[r], c1 = CPLX ? cp[r + 1] : (T)0;
          if (scaled) {
            T d = (T)a.dsc[r / NC];
            c0 *= d;
            c1 *= d;
          }
          v0 += beta * c0;
          v1 += beta * c1;
        }
        if (!a.c0_keep) {
          cp[r] = v0;
          if (CPLX) cp[r + 1] = v1;
        }
        if (c32) {
          c32[r] = (float)v0;
          if (CPLX) c32[r + 1] = (float)v1;
        }
      }
    }
}

template <class T, int TJ, int TR, bool CPLX, int SITE>
__global__ __launch_bounds__(64) void update_kernel(UpdateArgs a) {
  update_body<T, TJ, TR, CPLX>(a, blockIdx.x, gridDim.x);
}
template <class T, int TJ, int TR, bool CPLX, int SITE>
__global__ __launch_bounds__(64) void update_grouped(const UpdateArgs* jobs, const unsigned* start, int nj) {
  int j = find_job(start, nj, blockIdx.x);
  update_body<T, TJ, TR, CPLX>(jobs[j], blockIdx.x - start[j], start[j + 1] - start[j]);
}

// ---------------------------------------------------------------------------
// host launchers
// ---------------------------------------------------------------------------
constexpr int GTM = 4, GTN = 4, UTJ = 4, UTR = 4;   // real tiles
constexpr int ZTM = 2, ZTN = 2, ZTJ = 2, ZTR = 2;   // complex tiles

void gram_tiles(GramArgs& a) {
  int tm = a.cplx ? ZTM : GTM, tn = a.cplx ? ZTN : GTN;
  a.tiles_i = (a.M + 16 * tm - 1) / (16 * tm);
  a.tiles_j = (a.N + 16 * tn - 1) / (16 * tn);
}
void update_tiles(UpdateArgs& a) {
  int tj = a.cplx ? ZTJ : UTJ, tr = a.cplx ? ZTR : UTR;
  a.tiles_j = (a.N + 16 * tj - 1) / (16 * tj);
  a.tiles_r = (int)(a.rows / (16 * tr));
}

static int gram_kind(const GramArgs& a, bool f32acc) {
  int base = a.cplx ? (f32acc ? OP_GRAM_C0 : OP_GRAM_Z0) : (f32acc ? OP_GRAM_F0 : OP_GRAM_D0);
  return base + (a.site == 1 ? 1 : a.site == 2 ? 2 : 0);
}
static int update_kind(const UpdateArgs& a, bool f32) {
  int base = a.cplx ? (f32 ? OP_UPDATE_C0 : OP_UPDATE_Z0) : (f32 ? OP_UPDATE_F0 : OP_UPDATE_D0);
  return base + (a.site == 1 ? 1 : 0);
}

#define PPCG_GRAM_CASES(KERNEL, GRID, ...)                                                                       \
  case OP_GRAM_D0: hipLaunchKernelGGL((KERNEL<double, GTM, GTN, false, 0>), dim3(GRID), dim3(64), 0, st, __VA_ARGS__); break; \
  case OP_GRAM_D1: hipLaunchKernelGGL((KERNEL<double, GTM, GTN, false, 1>), dim3(GRID), dim3(64), 0, st, __VA_ARGS__); break; \
  case OP_GRAM_D2: hipLaunchKernelGGL((KERNEL<double, GTM, GTN, false, 2>), dim3(GRID), dim3(64), 0, st, __VA_ARGS__); break; \
  case OP_GRAM_F0: hipLaunchKernelGGL((KERNEL<float, GTM, GTN, false, 0>), dim3(GRID), dim3(64), 0, st, __VA_ARGS__); break;  \
  case OP_GRAM_F1: hipLaunchKernelGGL((KERNEL<float, GTM, GTN, false, 1>), dim3(GRID), dim3(64), 0, st, __VA_ARGS__); break;  \
  case OP_GRAM_F2: hipLaunchKernelGGL((KERNEL<float, GTM, GTN, false, 2>), dim3(GRID), dim3(64), 0, st, __VA_ARGS__); break;  \
  case OP_GRAM_Z0: hipLaunchKernelGGL((KERNEL<double, ZTM, ZTN, true, 0>), dim3(GRID), dim3(64), 0, st, __VA_ARGS__); break;  \
  case OP_GRAM_Z1: hipLaunchKernelGGL((KERNEL<double, ZTM, ZTN, true, 1>), dim3(GRID), dim3(64), 0, st, __VA_ARGS__); break;  \
  case OP_GRAM_Z2: hipLaunchKernelGGL((KERNEL<double, ZTM, ZTN, true, 2>), dim3(GRID), dim3(64), 0, st, __VA_ARGS__); break;  \
  case OP_GRAM_C0: hipLaunchKernelGGL((KERNEL<float, ZTM, ZTN, true, 0>), dim3(GRID), dim3(64), 0, st, __VA_ARGS__); break;   \
  case OP_GRAM_C1: hipLaunchKernelGGL((KERNEL<float, ZTM, ZTN, true, 1>), dim3(GRID), dim3(64), 0, st, __VA_ARGS__); break;   \
  case OP_GRAM_C2: hipLaunchKernelGGL((KERNEL<float, ZTM, ZTN, true, 2>), dim3(GRID), dim3(64), 0, st, __VA_ARGS__); break;

#define PPCG_UPDATE_CASES(KERNEL, GRID, ...)                                                                     \
  case OP_UPDATE_D0: hipLaunchKernelGGL((KERNEL<double, UTJ, UTR, false, 0>), dim3(GRID), dim3(64), 0, st, __VA_ARGS__); break; \
  case OP_UPDATE_D1: hipLaunchKernelGGL((KERNEL<double, UTJ, UTR, false, 1>), dim3(GRID), dim3(64), 0, st, __VA_ARGS__); break; \
  case OP_UPDATE_F0: hipLaunchKernelGGL((KERNEL<float, UTJ, UTR, false, 0>), dim3(GRID), dim3(64), 0, st, __VA_ARGS__); break;  \
  case OP_UPDATE_F1: hipLaunchKernelGGL((KERNEL<float, UTJ, UTR, false, 1>), dim3(GRID), dim3(64), 0, st, __VA_ARGS__); break;  \
  case OP_UPDATE_Z0: hipLaunchKernelGGL((KERNEL<double, ZTJ, ZTR, true, 0>), dim3(GRID), dim3(64), 0, st, __VA_ARGS__); break;  \
  case OP_UPDATE_Z1: hipLaunchKernelGGL((KERNEL<double, ZTJ, ZTR, true, 1>), dim3(GRID), dim3(64), 0, st, __VA_ARGS__); break;  \
  case OP_UPDATE_C0: hipLaunchKernelGGL((KERNEL<float, ZTJ, ZTR, true, 0>), dim3(GRID), dim3(64), 0, st, __VA_ARGS__); break;   \
  case OP_UPDATE_C1: hipLaunchKernelGGL((KERNEL<float, ZTJ, ZTR, true, 1>), dim3(GRID), dim3(64), 0, st, __VA_ARGS__); break;

void launch_gram(const GramArgs& a0, bool f32acc, hipStream_t st) {
  GramArgs a = a0;
  gram_tiles(a);
  unsigned blocks = (unsigned)((long)a.tiles_i * a.tiles_j * a.splits * a.njobs);
  if (blocks == 0) return;
  int kind = gram_kind(a, f32acc);
  if (g_rec) {
    g_rec->add(kind, &a, sizeof(a), blocks);
    return;
  }
  switch (kind) { PPCG_GRAM_CASES(gram_kernel, blocks, a) default: break; }
}

static int reduce_kind(const ReduceArgs& r, bool f32) {
  return r.cplx ? (f32 ? OP_REDUCE_C : OP_REDUCE_Z) : (f32 ? OP_REDUCE_F : OP_REDUCE_D);
}

void launch_reduce(const ReduceArgs& r, bool f32, hipStream_t st) {
  long tot = (long)r.M * r.N * r.njobs;
  unsigned blocks = (unsigned)((tot + 255) / 256);
  if (blocks == 0) return;
  int kind = reduce_kind(r, f32);
  if (g_rec) {
    g_rec->add(kind, &r, sizeof(r), blocks);
    return;
  }
  switch (kind) {
    case OP_REDUCE_D: hipLaunchKernelGGL((reduce_kernel<double, false>), dim3(blocks), dim3(256), 0, st, r); break;
    case OP_REDUCE_F: hipLaunchKernelGGL((reduce_kernel<float, false>), dim3(blocks), dim3(256), 0, st, r); break;
    case OP_REDUCE_Z: hipLaunchKernelGGL((reduce_kernel<double, true>), dim3(blocks), dim3(256), 0, st, r); break;
    case OP_REDUCE_C: hipLaunchKernelGGL((reduce_kernel<float, true>), dim3(blocks), dim3(256), 0, st, r); break;
  }
}

void launch_update(const UpdateArgs& a0, bool f32, hipStream_t st) {
  UpdateArgs a = a0;
  update_tiles(a);
  unsigned blocks = (unsigned)((long)a.tiles_j * a.tiles_r);
  if (blocks == 0) return;
  int kind = update_kind(a, f32);
  if (g_rec) {
    g_rec->add(kind, &a, sizeof(a), blocks);
    return;
  }
  switch (kind) { PPCG_UPDATE_CASES(update_kernel, blocks, a) default: break; }
}

bool launch_grouped_gemm(int kind, const void* jobs, const unsigned* start, int nj, unsigned total, hipStream_t st) {
  const GramArgs* gj = (const GramArgs*)jobs;
  const UpdateArgs* uj = (const UpdateArgs*)jobs;
  const ReduceArgs* rj = (const ReduceArgs*)jobs;
  switch (kind) {
    PPCG_GRAM_CASES(gram_grouped, total, gj, start, nj)
    PPCG_UPDATE_CASES(update_grouped, total, uj, start, nj)
    case OP_REDUCE_D: hipLaunchKernelGGL((reduce_grouped<double, false>), dim3(total), dim3(256), 0, st, rj, start, nj); break;
    case OP_REDUCE_F: hipLaunchKernelGGL((reduce_grouped<float, false>), dim3(total), dim3(256), 0, st, rj, start, nj); break;
    case OP_REDUCE_Z: hipLaunchKernelGGL((reduce_grouped<double, true>), dim3(total), dim3(256), 0, st, rj, start, nj); break;
    case OP_REDUCE_C: hipLaunchKernelGGL((reduce_grouped<float, true>), dim3(total), dim3(256), 0, st, rj, start, nj); break;
    default: return false;
  }
  return true;
}

}  // namespace ppcg
