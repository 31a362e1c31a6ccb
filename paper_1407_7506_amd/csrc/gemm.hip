// Tall-skinny contractions on MFMA (gfx950):
//   gram    C = A^H (D B) summed over the rows of tall blocks (split-n partials)
//   reduce  deterministic fixed-order sum of the split partials
//   update  C <- beta * (D C) + alpha * A B with A tall, B small
// Used for the projections of W and P (Algorithm 3, steps 9-10), the
// Cholesky-QR Gram and X R^{-1} (section 5.5), the residual
// W = AX - X (X^H A X) (section 2) and the Rayleigh-Ritz Grams and rotation
// (section 5.6).  Real operands use one MFMA per 16x16x4 tile; complex
// operands four (real and imaginary parts in separate accumulators).
#include <stdexcept>
#include <type_traits>

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
  bool fb[TN], vb[TN], sb[TN], sb2[TN];
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
    sb2[t] = a.dsc2 != nullptr && c >= a.nsc;
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
    T dv[Q], dv2[Q];
    if (a.dsc) {
      const double* dp = a.dsc + rr;
#pragma unroll
      for (int e = 0; e < Q; ++e) dv[e] = (T)dp[e];
    }
    if (a.dsc2) {
      const double* dp = a.dsc2 + rr;
#pragma unroll
      for (int e = 0; e < Q; ++e) dv2[e] = (T)dp[e];
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
        if (sb2[t]) {
#pragma unroll
          for (int e = 0; e < Q; ++e) {
            br[t][e] *= dv2[e];
            if (CPLX) bi[t][e] *= dv2[e];
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
  double s0 = 0, s1 = 0;
  if (CPLX && r.im_off > 0) {  // real partials: real parts, imaginary parts im_off further
    const T* p = (const T*)r.part + ((long)job * r.splits * r.split_stride + i + (long)j * r.ldp);
#pragma unroll 8
    for (int t = 0; t < r.splits; ++t) {
      s0 += (double)p[(long)t * r.split_stride];
      s1 += (double)p[(long)t * r.split_stride + r.im_off];
    }
  } else {
    const T* p = (const T*)r.part + ((long)job * r.splits * r.split_stride + i + (long)j * r.ldp) * NC;
#pragma unroll 8
    for (int t = 0; t < r.splits; ++t) {
      s0 += (double)p[(long)t * r.split_stride * NC];
      if (CPLX) s1 += (double)p[(long)t * r.split_stride * NC + 1];
    }
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
// epilogue of the update kernels: the wave's (16 TJ) x (16 TR) tile of the
// transposed product, at output column j0 and row r0
template <class T, int TJ, int TR, bool CPLX>
PPCG_DEV void update_epilogue(const UpdateArgs& a, int job, int j0, long r0,
                              const typename AccT<T>::type (&acc)[CPLX ? 2 : 1][TJ][TR]) {
  constexpr int NC = CPLX ? 2 : 1;
  const int l = threadIdx.x & 63, lc = l & 15;
  const T alpha = (T)a.alpha, beta = (T)a.beta;
  const bool norms = !CPLX && a.cpart != nullptr;
#pragma unroll
  for (int x = 0; x < TJ; ++x)
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const int j = j0 + 16 * x + acc_row<T>(l, v);
      const bool jv = j < a.N;
      double sq = 0;  // sum of squares of the values this lane stores in column j
      if (jv) {
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
          if (a.c64) {  // float64 input and diagonal term, combined in float64
            const long o = ((long)job * a.job_c_off + (long)j * a.ldc) * NC + r;
            const double g = a.xd ? a.gd[(long)j * a.gds * NC] : 0.0;  // real diagonal of a Hermitian G
            double w0 = a.beta * a.c64[o] + (double)v0;
            if (a.xd) w0 -= a.xd[o] * g;
            v0 = (T)w0;
            if (CPLX) {
              double w1 = a.beta * a.c64[o + 1] + (double)v1;
              if (a.xd) w1 -= a.xd[o + 1] * g;
              v1 = (T)w1;
            }
          } else if (a.beta != 0) {
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
          if (norms) {
            const double w = c32 ? (double)(float)v0 : (double)v0;
            sq += w * w;
          }
        }
      }
      if (norms) {  // the 16 lanes of a lane group hold the same column: reduce over them
#pragma unroll
        for (int o = 1; o < 16; o <<= 1) sq += __shfl_xor(sq, o, 64);
        if (jv && lc == 0 && j < a.ncn) a.cpart[r0 / (16 * TR) + (long)j * a.ldp] = sq;
      }
    }
}

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
  update_epilogue<T, TJ, TR, CPLX>(a, job, j0, r0, acc);
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
// Per-block pencil Grams for 16-column blocks (one wave per block and split):
// every slab of the block is read once per row (lane group g reads 4
// consecutive rows of column lc, as in gram_body) and only the 11 tiles of
// the overlap and H matrices that the pencil uses are accumulated, in
// float64.
// ---------------------------------------------------------------------------
template <bool F32, bool HASP, bool AXR>
PPCG_DEV void block_gram_body(const BlockGramArgs& a, unsigned wg, unsigned nwg) {
  typedef typename AccT<double>::type acc_t;
  const int l = threadIdx.x, lc = l & 15, g = l >> 4;
  const unsigned L = xcd_remap(wg, nwg);
  const int blk = (int)(L % (unsigned)a.nblocks);
  const int split = (int)(L / (unsigned)a.nblocks);
  const long rbeg = (long)split * a.chunk;
  const long rend = rbeg + a.chunk < a.rows ? rbeg + a.chunk : a.rows;
  const long col = ((long)blk * 16 + lc) * a.ld;
  const int es = F32 ? 4 : 8;
  const char* px = (const char*)(a.X + col);
  const char* pw = (const char*)a.W + col * es;
  const char* pp = HASP ? (const char*)a.P + col * es : nullptr;
  const char* paw = (const char*)a.AW + col * es;
  const char* pap = HASP ? (const char*)a.AP + col * es : nullptr;
  const char* pax = AXR ? (const char*)(a.AX + col) : nullptr;
  acc_t acc[BG_TILES];
#pragma unroll
  for (int t = 0; t < BG_TILES; ++t) acc[t] = acc_t{0, 0, 0, 0};
  // software pipeline: the raw 16-byte pieces of the next 16 rows are loaded
  // while the MFMAs of the current rows run, and decoded (float32 widened)
  // only after them; element accesses go through scalars before
  // reinterpretation
  typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));
  constexpr int NW = F32 ? 1 : 2;  // pieces per quad of W, P, AW, AP
  u32x4 rx[2], rw[NW], rp[NW], raw_[NW], rap[NW], rax[2];
  auto fetch = [&](long r) {
    const long rr = r + 4 * g;
    const char* q;
    q = px + rr * 8; rx[0] = *(const u32x4*)q; rx[1] = *(const u32x4*)(q + 16);
    q = pw + rr * es; rw[0] = *(const u32x4*)q; if constexpr (NW == 2) rw[1] = *(const u32x4*)(q + 16);
    q = paw + rr * es; raw_[0] = *(const u32x4*)q; if constexpr (NW == 2) raw_[1] = *(const u32x4*)(q + 16);
    if (HASP) {
      q = pp + rr * es; rp[0] = *(const u32x4*)q; if constexpr (NW == 2) rp[1] = *(const u32x4*)(q + 16);
      q = pap + rr * es; rap[0] = *(const u32x4*)q; if constexpr (NW == 2) rap[1] = *(const u32x4*)(q + 16);
    }
    if (AXR) { q = pax + rr * 8; rax[0] = *(const u32x4*)q; rax[1] = *(const u32x4*)(q + 16); }
  };
  auto dec64 = [](const u32x4* x, double* v) {
    const unsigned w0 = x[0].x, w1 = x[0].y, w2 = x[0].z, w3 = x[0].w;
    const unsigned w4 = x[1].x, w5 = x[1].y, w6 = x[1].z, w7 = x[1].w;
    v[0] = __hiloint2double((int)w1, (int)w0);
    v[1] = __hiloint2double((int)w3, (int)w2);
    v[2] = __hiloint2double((int)w5, (int)w4);
    v[3] = __hiloint2double((int)w7, (int)w6);
  };
  auto decw = [&](const u32x4* x, double* v) {
    if constexpr (F32) {
      const unsigned w0 = x[0].x, w1 = x[0].y, w2 = x[0].z, w3 = x[0].w;
      v[0] = (double)__uint_as_float(w0);
      v[1] = (double)__uint_as_float(w1);
      v[2] = (double)__uint_as_float(w2);
      v[3] = (double)__uint_as_float(w3);
    } else {
      dec64(x, v);
    }
  };
  if (rbeg < rend) fetch(rbeg);
  for (long r = rbeg; r < rend; r += 16) {
    double x[4], w[4], p[4], aw[4], ap[4], ax[4];
    dec64(rx, x);
    decw(rw, w);
    decw(raw_, aw);
    if (HASP) {
      decw(rp, p);
      decw(rap, ap);
    }
    if (AXR) dec64(rax, ax);
    if (r + 16 < rend) fetch(r + 16);
#pragma unroll
    for (int e = 0; e < 4; ++e) {
      acc[0] = mfma(x[e], x[e], acc[0]);
      acc[1] = mfma(x[e], w[e], acc[1]);
      acc[3] = mfma(w[e], w[e], acc[3]);
      acc[6] = mfma(w[e], aw[e], acc[6]);
      acc[9] = AXR ? mfma(ax[e], w[e], acc[9]) : mfma(x[e], aw[e], acc[9]);
      if (HASP) {
        acc[2] = mfma(x[e], p[e], acc[2]);
        acc[4] = mfma(w[e], p[e], acc[4]);
        acc[5] = mfma(p[e], p[e], acc[5]);
        acc[7] = mfma(w[e], ap[e], acc[7]);
        acc[8] = mfma(p[e], ap[e], acc[8]);
        acc[10] = AXR ? mfma(ax[e], p[e], acc[10]) : mfma(x[e], ap[e], acc[10]);
      }
    }
    // the next rows are decoded only after every MFMA of these rows (the
    // loads issued above stay in flight meanwhile)
    __builtin_amdgcn_sched_barrier(0);
  }
  double* out = a.out + ((long)blk * a.splits + split) * (BG_TILES * 256);
#pragma unroll
  for (int t = 0; t < BG_TILES; ++t) {
    if (!HASP && (t == 2 || t == 4 || t == 5 || t == 7 || t == 8 || t == 10)) continue;
#pragma unroll
    for (int v = 0; v < 4; ++v) out[t * 256 + acc_row<double>(l, v) + 16 * lc] = acc[t][v];
  }
}
template <bool F32, bool HASP, bool AXR>
__global__ __launch_bounds__(64) void block_gram_kernel(BlockGramArgs a) {
  block_gram_body<F32, HASP, AXR>(a, blockIdx.x, gridDim.x);
}

void launch_block_gram(const BlockGramArgs& a, hipStream_t st) {
  if (g_rec) throw std::invalid_argument("block gram: not available in grouped launches");
  if (a.rows % 16 || a.chunk % 16 || a.nblocks <= 0 || a.splits <= 0 || !a.X || !a.W || !a.AW || !a.out ||
      (a.hasP && (!a.P || !a.AP)))
    throw std::invalid_argument("block gram: bad arguments");
  const unsigned grid = (unsigned)a.nblocks * (unsigned)a.splits;
  const bool axr = a.AX != nullptr;
#define PPCG_BG(F, H, X) hipLaunchKernelGGL((block_gram_kernel<F, H, X>), dim3(grid), dim3(64), 0, st, a)
  if (a.f32) {
    if (a.hasP) { if (axr) PPCG_BG(true, true, true); else PPCG_BG(true, true, false); }
    else { if (axr) PPCG_BG(true, false, true); else PPCG_BG(true, false, false); }
  } else {
    if (a.hasP) { if (axr) PPCG_BG(false, true, true); else PPCG_BG(false, true, false); }
    else { if (axr) PPCG_BG(false, false, true); else PPCG_BG(false, false, false); }
  }
#undef PPCG_BG
}

// ---------------------------------------------------------------------------
// LDS-staged variants for large real shapes.  A workgroup of four waves
// (2 x 2) owns a 128 x 128 output tile.  Each chunk of KC reduction indices
// (rows of the tall operands for gram, columns of A for update) of both
// operands is loaded once per workgroup into LDS (double buffered, one
// barrier per chunk, the next chunk's global loads in flight during the
// MFMAs of the current one) and every wave computes its 64 x 64 quadrant
// from it: half the L2-to-CU traffic per flop of the one-wave kernels.
// Panels whose reads are 4 consecutive reduction indices per lane use the
// column stride KC + 2 (float64) or KC + 4 (float32) elements, so that the
// 16-byte reads of 8 consecutive lanes fall into distinct bank groups.
// ---------------------------------------------------------------------------
constexpr int LB = 128;  // workgroup tile edge of the LDS-staged kernels
template <class T, int KC> struct LdsPad { static constexpr int S = KC + (sizeof(T) == 8 ? 2 : 4); };

PPCG_DEV void put4(double* d, const double* v) {
  ((double2*)d)[0] = make_double2(v[0], v[1]);
  ((double2*)d)[1] = make_double2(v[2], v[3]);
}
PPCG_DEV void put4(float* d, const float* v) { *(float4*)d = make_float4(v[0], v[1], v[2], v[3]); }
PPCG_DEV void get4(const double* d, double* v) {
  double2 x = ((const double2*)d)[0], y = ((const double2*)d)[1];
  v[0] = x.x; v[1] = x.y; v[2] = y.x; v[3] = y.y;
}
PPCG_DEV void get4(const float* d, float* v) {
  float4 x = *(const float4*)d;
  v[0] = x.x; v[1] = x.y; v[2] = x.z; v[3] = x.w;
}

// gram, C (M x N) partial over rows [rbeg, rend) of split s; real operands
// (NBUF as for the update below)
template <class T, int KC, int NBUF = 2>
PPCG_DEV void gram_lds_body(const GramArgs& a, unsigned wg, unsigned nwg) {
  constexpr int S = LdsPad<T, KC>::S;
  constexpr int PQ = KC / 4;             // quads (4 consecutive rows) per column and chunk
  constexpr int NQ = LB * PQ / 256;      // quads per thread and panel
  constexpr int CS = 256 / PQ;           // column step between a thread's quads
  __shared__ __align__(16) T As[NBUF][LB * S];
  __shared__ __align__(16) T Bs[NBUF][LB * S];
  typedef typename AccT<T>::type acc_t;
  const int tid = threadIdx.x, l = tid & 63, lc = l & 15, g = l >> 4;
  const int wi = (tid >> 6) & 1, wj = tid >> 7;
  unsigned L = xcd_remap(wg, nwg);
  const int ntile = a.tiles_i * a.tiles_j;
  const int tile = L % ntile;
  const int rest = L / ntile;
  const int split = rest % a.splits;
  const int job = rest / a.splits;
  const int ti = tile % a.tiles_i, tj = tile / a.tiles_i;
  if (a.upper_only && ti > tj) return;  // tile wholly below the diagonal (uniform per workgroup)
  const int i0 = ti * LB, j0 = tj * LB;
  const long joff = (long)job * a.job_col_off;
  const long rbeg = (long)split * a.chunk;
  const long rend = rbeg + a.chunk < a.rows ? rbeg + a.chunk : a.rows;
  const int nch = rend > rbeg ? (int)((rend - rbeg) / KC) : 0;

  const int part = tid % PQ;
  const char* pa[NQ];
  const char* pb[NQ];
  bool fa[NQ], fb[NQ], va[NQ], vb[NQ], sb[NQ], sb2[NQ];
#pragma unroll
  for (int q = 0; q < NQ; ++q) {
    const int col = tid / PQ + q * CS;
    const int ca = i0 + col, cb = j0 + col;
    va[q] = ca < a.M;
    vb[q] = cb < a.N;
    pa[q] = (const char*)seg_col(a.A, va[q] ? ca : 0, a.ld, joff, fa[q], 8);
    pb[q] = (const char*)seg_col(a.B, vb[q] ? cb : 0, a.ld, joff, fb[q], 8);
    sb[q] = a.dsc != nullptr && cb < a.nsc;
    sb2[q] = a.dsc2 != nullptr && cb >= a.nsc;
  }
  const int dsh = a.il ? 1 : 0;  // interleaved complex rows: two real rows per grid point
  // 16 x 16 sub-tiles of this wave's quadrant that carry results: inside
  // M x N and, for a diagonal tile of an upper-only Gram, on or above the
  // diagonal (the rest is never read; skipping it leaves every used entry
  // bitwise the same)
  const int nxv = max(0, min(4, (a.M - (i0 + wi * 64) + 15) / 16));
  const int nyv = max(0, min(4, (a.N - (j0 + wj * 64) + 15) / 16));
  const bool dg = a.upper_only && ti == tj;
  const bool full = nxv == 4 && nyv == 4 && !dg;
  // Row scales and the complex rotation of the B operand: applied as the
  // chunk is loaded for float64 (measured faster there), and for float32
  // after the current chunk's MFMAs, as the chunk is stored to LDS, so that
  // its loads stay in flight meanwhile (the scales of this thread's four rows
  // are loaded once per chunk, not once per quad).
  constexpr bool DEFER = sizeof(T) == 4;
  T ra[NQ][4], rb[NQ][4];
  double dv[4], dv2[4];
  auto gload = [&](long r) {
    const long rr = r + 4 * part;
#pragma unroll
    for (int q = 0; q < NQ; ++q) {
      if (va[q]) {
        Load4<T, false>::go(pa[q] + rr * (fa[q] ? 4 : 8), fa[q], ra[q], nullptr);
      } else {
#pragma unroll
        for (int e = 0; e < 4; ++e) ra[q][e] = 0;
      }
      if (vb[q]) {
        Load4<T, false>::go(pb[q] + rr * (fb[q] ? 4 : 8), fb[q], rb[q], nullptr);
        if constexpr (!DEFER) {
          if (sb[q]) {
#pragma unroll
            for (int e = 0; e < 4; ++e) rb[q][e] *= (T)a.dsc[(rr + e) >> dsh];
          }
          if (sb2[q]) {
#pragma unroll
            for (int e = 0; e < 4; ++e) rb[q][e] *= (T)a.dsc2[(rr + e) >> dsh];
          }
          if (a.rotB) {  // (re, im) -> (im, -re): rows come in quads, so pairs do not straddle them
            const T r0 = rb[q][0], r2 = rb[q][2];
            rb[q][0] = rb[q][1];
            rb[q][1] = -r0;
            rb[q][2] = rb[q][3];
            rb[q][3] = -r2;
          }
        }
      } else {
#pragma unroll
        for (int e = 0; e < 4; ++e) rb[q][e] = 0;
      }
    }
    if constexpr (DEFER) {
      if (a.dsc) {
#pragma unroll
        for (int e = 0; e < 4; ++e) dv[e] = a.dsc[(rr + e) >> dsh];
      }
      if (a.dsc2) {
#pragma unroll
        for (int e = 0; e < 4; ++e) dv2[e] = a.dsc2[(rr + e) >> dsh];
      }
    }
  };
  auto sput = [&](int buf) {
#pragma unroll
    for (int q = 0; q < NQ; ++q) {
      const int col = tid / PQ + q * CS;
      if constexpr (DEFER) {
        if (vb[q]) {
          if (sb[q]) {
#pragma unroll
            for (int e = 0; e < 4; ++e) rb[q][e] *= (T)dv[e];
          }
          if (sb2[q]) {
#pragma unroll
            for (int e = 0; e < 4; ++e) rb[q][e] *= (T)dv2[e];
          }
          if (a.rotB) {
            const T r0 = rb[q][0], r2 = rb[q][2];
            rb[q][0] = rb[q][1];
            rb[q][1] = -r0;
            rb[q][2] = rb[q][3];
            rb[q][3] = -r2;
          }
        }
      }
      put4(&As[buf][col * S + 4 * part], ra[q]);
      put4(&Bs[buf][col * S + 4 * part], rb[q]);
    }
  };

  acc_t acc[4][4];
#pragma unroll
  for (int x = 0; x < 4; ++x)
#pragma unroll
    for (int y = 0; y < 4; ++y) acc[x][y] = acc_t{0, 0, 0, 0};
  if (nch > 0) {
    gload(rbeg);
    sput(0);
  }
  __syncthreads();
  for (int c = 0; c < nch; ++c) {
    const int buf = NBUF == 2 ? (c & 1) : 0;
    if (c + 1 < nch) gload(rbeg + (long)(c + 1) * KC);
#pragma unroll
    for (int kk = 0; kk < KC; kk += 16) {
      T av[4][4], bv[4][4];
#pragma unroll
      for (int t = 0; t < 4; ++t) {
        get4(&As[buf][(wi * 64 + 16 * t + lc) * S + kk + 4 * g], av[t]);
        get4(&Bs[buf][(wj * 64 + 16 * t + lc) * S + kk + 4 * g], bv[t]);
      }
      if (full) {
#pragma unroll
        for (int e = 0; e < 4; ++e)
#pragma unroll
          for (int x = 0; x < 4; ++x)
#pragma unroll
            for (int y = 0; y < 4; ++y) acc[x][y] = mfma(av[x][e], bv[y][e], acc[x][y]);
      } else {
#pragma unroll
        for (int e = 0; e < 4; ++e)
#pragma unroll
          for (int x = 0; x < 4; ++x)
#pragma unroll
            for (int y = 0; y < 4; ++y)
              if (x < nxv && y < nyv && !(dg && (wi > wj || (wi == wj && x > y))))
                acc[x][y] = mfma(av[x][e], bv[y][e], acc[x][y]);
      }
    }
    if (NBUF == 1) __syncthreads();
    if (c + 1 < nch) sput(NBUF == 2 ? buf ^ 1 : 0);
    __syncthreads();
  }
  T* out = (T*)a.out + ((long)job * a.splits + split) * a.split_stride;
#pragma unroll
  for (int x = 0; x < 4; ++x)
#pragma unroll
    for (int y = 0; y < 4; ++y)
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int i = i0 + wi * 64 + 16 * x + acc_row<T>(l, v);
        const int j = j0 + wj * 64 + 16 * y + lc;
        if (i < a.M && j < a.N) out[i + (long)j * a.ldo] = acc[x][y][v];
      }
}

template <class T, int KC, int SITE>
__global__ __launch_bounds__(256) void gram_lds_kernel(GramArgs a) {
  gram_lds_body<T, KC>(a, blockIdx.x, gridDim.x);
}
template <class T, int KC, int SITE>
__global__ __launch_bounds__(256) void gram_lds_grouped(const GramArgs* jobs, const unsigned* start, int nj) {
  int j = find_job(start, nj, blockIdx.x);
  gram_lds_body<T, KC>(jobs[j], blockIdx.x - start[j], start[j + 1] - start[j]);
}

// update, C (rows x N) = beta (D C) + alpha A B for one 128 x 128 tile; real.
// NBUF = 2: double-buffered LDS panels (one barrier per chunk); NBUF = 1: one
// LDS buffer refilled between two barriers (half the LDS, deeper chunks).
template <class T, int KC, int NBUF = 2, bool LEAN = false>
PPCG_DEV void update_lds_body(const UpdateArgs& a, unsigned wg, unsigned nwg) {
  constexpr int SB = LdsPad<T, KC>::S;                 // B panel [col][k]
  constexpr int SA = LB + (sizeof(T) == 8 ? 2 : 4);    // A panel [k][row]
  constexpr int PE = 16 / (int)sizeof(T);              // rows per 16-byte piece of A
  constexpr int PA = LB / PE;                          // pieces per column of the A panel
  constexpr int NA = KC * PA / 256;                    // A pieces per thread
  constexpr int PQ = KC / 4, NB = LB * PQ / 256;       // B quads per column / per thread
  typedef typename AccT<T>::type acc_t;
  typedef typename std::conditional<sizeof(T) == 8, double2, float4>::type v16;
  __shared__ __align__(16) T As[NBUF][KC * SA];
  __shared__ __align__(16) T Bs[NBUF][LB * SB];
  const int tid = threadIdx.x, l = tid & 63, lc = l & 15, g = l >> 4;
  const int wr = (tid >> 6) & 1, wj = tid >> 7;
  unsigned L = xcd_remap(wg, nwg);
  // column tiles fastest so the row panel of A is shared inside one XCD
  const int tj = L % a.tiles_j;
  const int rest = L / a.tiles_j;
  const int tr = rest % a.tiles_r;
  const int job = rest / a.tiles_r;
  const int j0 = tj * LB;
  const long r0 = (long)tr * LB;
  const T* A = (const T*)a.A + (long)job * a.job_a_off;
  const T* Bm = (const T*)a.B + (long)job * a.job_b_off;
  int kend = a.K;
  if (a.b_upper && j0 + LB < kend) kend = j0 + LB;
  const int nch = (kend + KC - 1) / KC;
  v16 ra[NA];
  T rb[NB][4];
  auto gload = [&](int k0) {
#pragma unroll
    for (int q = 0; q < NA; ++q) {
      const int pc = tid + 256 * q;
      const int k = k0 + pc / PA, rp = pc % PA;
      if (k < kend) ra[q] = *(const v16*)(A + r0 + rp * PE + (long)k * a.lda);
      else ra[q] = v16{};
    }
#pragma unroll
    for (int q = 0; q < NB; ++q) {
      const int pc = tid + 256 * q;
      const int j = j0 + pc / PQ, k = k0 + 4 * (pc % PQ);
      const T* bp = Bm + (long)(j < a.N ? j : 0) * a.ldb;
#pragma unroll
      for (int e = 0; e < 4; ++e) rb[q][e] = (j < a.N && k + e < kend) ? bp[k + e] : (T)0;
    }
  };
  auto sput = [&](int buf) {
#pragma unroll
    for (int q = 0; q < NA; ++q) {
      const int pc = tid + 256 * q;
      *(v16*)&As[buf][(pc / PA) * SA + (pc % PA) * PE] = ra[q];
    }
#pragma unroll
    for (int q = 0; q < NB; ++q) {
      const int pc = tid + 256 * q;
      put4(&Bs[buf][(pc / PQ) * SB + 4 * (pc % PQ)], rb[q]);
    }
  };
  acc_t acc[1][4][4];
#pragma unroll
  for (int x = 0; x < 4; ++x)
#pragma unroll
    for (int y = 0; y < 4; ++y) acc[0][x][y] = acc_t{0, 0, 0, 0};
  // output columns of this wave's quadrant inside N, in 16-column sub-tiles
  const int nxv = max(0, min(4, (a.N - (j0 + wj * 64) + 15) / 16));
  if (nch > 0) {
    gload(0);
    sput(0);
  }
  __syncthreads();
  // the chunk loop; MODE 0 tests for a whole quadrant inside the loop, MODE 1
  // (whole) and 2 (partial) take that choice once per wave, outside it (both
  // run the same barriers).  Measured: float64 is faster with the test inside,
  // float32 with it outside.
  auto chunks = [&](auto mode) {
    constexpr int MODE = decltype(mode)::value;
    for (int c = 0; c < nch; ++c) {
      const int buf = NBUF == 2 ? (c & 1) : 0;
      if (c + 1 < nch) gload((c + 1) * KC);
#pragma unroll
      for (int kk = 0; kk < KC; kk += 16) {
        if constexpr (LEAN) {
          // operands read one reduction step at a time (same MFMA order as
          // below): fewer live registers, so two workgroups share a CU
#pragma unroll
          for (int e = 0; e < 4; ++e) {
            T bx[4], ay[4];
#pragma unroll
            for (int x = 0; x < 4; ++x) bx[x] = Bs[buf][(wj * 64 + 16 * x + lc) * SB + kk + 4 * g + e];
#pragma unroll
            for (int y = 0; y < 4; ++y) ay[y] = As[buf][(kk + 4 * g + e) * SA + wr * 64 + 16 * y + lc];
#pragma unroll
            for (int x = 0; x < 4; ++x)
              if (MODE == 1 || (MODE == 0 && nxv == 4) || x < nxv) {
#pragma unroll
                for (int y = 0; y < 4; ++y) acc[0][x][y] = mfma(bx[x], ay[y], acc[0][x][y]);
              }
          }
          continue;
        }
        T bv[4][4], av[4][4];
#pragma unroll
        for (int x = 0; x < 4; ++x) get4(&Bs[buf][(wj * 64 + 16 * x + lc) * SB + kk + 4 * g], bv[x]);
#pragma unroll
        for (int y = 0; y < 4; ++y)
#pragma unroll
          for (int e = 0; e < 4; ++e) av[y][e] = As[buf][(kk + 4 * g + e) * SA + wr * 64 + 16 * y + lc];
        if (MODE == 1 || (MODE == 0 && nxv == 4)) {
#pragma unroll
          for (int e = 0; e < 4; ++e)
#pragma unroll
            for (int x = 0; x < 4; ++x)
#pragma unroll
              for (int y = 0; y < 4; ++y) acc[0][x][y] = mfma(bv[x][e], av[y][e], acc[0][x][y]);
        } else {
#pragma unroll
          for (int e = 0; e < 4; ++e)
#pragma unroll
            for (int x = 0; x < 4; ++x)
              if (x < nxv) {
#pragma unroll
                for (int y = 0; y < 4; ++y) acc[0][x][y] = mfma(bv[x][e], av[y][e], acc[0][x][y]);
              }
        }
      }
      if (NBUF == 1) __syncthreads();
      if (c + 1 < nch) sput(NBUF == 2 ? buf ^ 1 : 0);
      __syncthreads();
    }
  };
  if constexpr (sizeof(T) == 8) {
    chunks(std::integral_constant<int, 0>{});
  } else {
    if (nxv == 4) chunks(std::integral_constant<int, 1>{});
    else chunks(std::integral_constant<int, 2>{});
  }
  update_epilogue<T, 4, 4, false>(a, job, j0 + wj * 64, r0 + wr * 64, acc);
}

template <class T, int KC, int SITE>
__global__ __launch_bounds__(256) void update_lds_kernel(UpdateArgs a) {
  update_lds_body<T, KC>(a, blockIdx.x, gridDim.x);
}
// float64 update with 16-deep chunks (70 KB of LDS) and operands read per
// reduction step, held to 256 registers: two workgroups per CU, so one
// workgroup's barrier and load waits are covered by the other's MFMAs
template <class T, int KC, int SITE>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(2))) void update_lds_kernel_lean(UpdateArgs a) {
  update_lds_body<T, KC, 2, true>(a, blockIdx.x, gridDim.x);
}
template <class T, int KC, int SITE>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(2))) void update_lds_grouped_lean(
    const UpdateArgs* jobs, const unsigned* start, int nj) {
  int j = find_job(start, nj, blockIdx.x);
  update_lds_body<T, KC, 2, true>(jobs[j], blockIdx.x - start[j], start[j + 1] - start[j]);
}
template <class T, int KC, int SITE>
__global__ __launch_bounds__(256) void update_lds_grouped(const UpdateArgs* jobs, const unsigned* start, int nj) {
  int j = find_job(start, nj, blockIdx.x);
  update_lds_body<T, KC>(jobs[j], blockIdx.x - start[j], start[j + 1] - start[j]);
}

// ---------------------------------------------------------------------------
// Per-block Grams in one pass over the block's columns (real, float64
// accumulation).  The A and B column sets of a block share segments (X_j,
// W_j, P_j appear in both); a workgroup of four waves owns one (block, row
// split), stages each chunk of 16 rows of the union of the two sets once in
// LDS (converted to float64, double buffered) and computes the whole
// (M x N) partial Gram from it: each column is read from HBM once instead of
// once per operand and output tile.  Wave w owns output tile rows w, w+4, ...
// TR: output tile rows per wave, TC: output tile columns.
// ---------------------------------------------------------------------------
constexpr int BG_MAXU = 6 * 32;  // union columns: up to 6 segments of q <= 32
template <int TR, int TC>
PPCG_DEV void gram_block_body(const GramArgs& a, unsigned wg, unsigned nwg) {
  constexpr int KC = 16, S = KC + 2;
  typedef AccT<double>::type acc_t;
  __shared__ __align__(16) double U[2][BG_MAXU * S];
  __shared__ const char* uptr[BG_MAXU];
  __shared__ unsigned char uf32[BG_MAXU];
  __shared__ short amap[TR * 64];
  __shared__ int nU;
  const int tid = threadIdx.x, l = tid & 63, lc = l & 15, g = l >> 4, w = tid >> 6;
  unsigned L = xcd_remap(wg, nwg);
  const int split = (int)(L % a.splits), job = (int)(L / a.splits);
  const long joff = (long)job * a.job_col_off;
  const long rbeg = (long)split * a.chunk;
  const long rend = rbeg + a.chunk < a.rows ? rbeg + a.chunk : a.rows;
  const int nch = rend > rbeg ? (int)((rend - rbeg) / KC) : 0;
  // union of the column sets: every B column, then the A segments found in no B segment
  if (tid == 0) {
    int n = 0;
    for (int c = 0; c < a.N; ++c) {
      bool f;
      uptr[n] = (const char*)seg_col(a.B, c, a.ld, joff, f, 8);
      uf32[n] = f;
      ++n;
    }
    int a0 = 0;
    for (int sA = 0; sA < a.A.nseg; ++sA) {
      const int len = a.A.end[sA] - a0;
      int map0 = -1, b0 = 0;
      for (int sB = 0; sB < a.B.nseg; ++sB) {
        const int blen = a.B.end[sB] - b0;
        if (a.B.p[sB] == a.A.p[sA] && a.B.f32[sB] == a.A.f32[sA] && blen >= len) {
          map0 = b0;
          break;
        }
        b0 = a.B.end[sB];
      }
      for (int c = 0; c < len; ++c) {
        if (map0 >= 0) {
          amap[a0 + c] = (short)(map0 + c);
        } else {
          bool f;
          uptr[n] = (const char*)seg_col(a.A, a0 + c, a.ld, joff, f, 8);
          uf32[n] = f;
          amap[a0 + c] = (short)n;
          ++n;
        }
      }
      a0 = a.A.end[sA];
    }
    nU = n;
  }
  __syncthreads();
  const int nu = nU;
  const int nq = nu * (KC / 4);   // 4-row quads per chunk, at most 3 per thread
  double rq[3][4];
  auto gload = [&](long r) {  // next chunk into registers
#pragma unroll
    for (int t = 0; t < 3; ++t) {
      const int q = tid + 256 * t;
      if (q < nq) {
        const int col = q >> 2;
        const bool f = uf32[col] != 0;
        Load4<double, false>::go(uptr[col] + (r + 4 * (q & 3)) * (f ? 4 : 8), f, rq[t], nullptr);
      }
    }
  };
  auto sput = [&](int buf) {
#pragma unroll
    for (int t = 0; t < 3; ++t) {
      const int q = tid + 256 * t;
      if (q < nq) put4(&U[buf][(q >> 2) * S + 4 * (q & 3)], rq[t]);
    }
  };
  acc_t acc[TR][TC];
#pragma unroll
  for (int x = 0; x < TR; ++x)
#pragma unroll
    for (int y = 0; y < TC; ++y) acc[x][y] = acc_t{0, 0, 0, 0};
  if (nch > 0) {
    gload(rbeg);
    sput(0);
  }
  __syncthreads();
  for (int c = 0; c < nch; ++c) {
    const int buf = c & 1;
    if (c + 1 < nch) gload(rbeg + (long)(c + 1) * KC);
    double av[TR][4], bv[TC][4];
#pragma unroll
    for (int x = 0; x < TR; ++x) {
      const int i = (w + 4 * x) * 16 + lc;
      if (i < a.M) get4(&U[buf][amap[i] * S + 4 * g], av[x]);
      else av[x][0] = av[x][1] = av[x][2] = av[x][3] = 0.0;
    }
#pragma unroll
    for (int y = 0; y < TC; ++y) {
      const int j = 16 * y + lc;
      if (j < a.N) get4(&U[buf][j * S + 4 * g], bv[y]);
      else bv[y][0] = bv[y][1] = bv[y][2] = bv[y][3] = 0.0;
    }
#pragma unroll
    for (int e = 0; e < 4; ++e)
#pragma unroll
      for (int x = 0; x < TR; ++x)
#pragma unroll
        for (int y = 0; y < TC; ++y) acc[x][y] = mfma(av[x][e], bv[y][e], acc[x][y]);
    if (c + 1 < nch) sput(buf ^ 1);
    __syncthreads();
  }
  double* out = (double*)a.out + ((long)job * a.splits + split) * a.split_stride;
#pragma unroll
  for (int x = 0; x < TR; ++x)
#pragma unroll
    for (int y = 0; y < TC; ++y)
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int i = (w + 4 * x) * 16 + acc_row<double>(l, v);
        const int j = 16 * y + lc;
        if (i < a.M && j < a.N) out[i + (long)j * a.ldo] = acc[x][y][v];
      }
}

template <int TR, int TC>
__global__ __launch_bounds__(256) void gram_block_kernel(GramArgs a) {
  gram_block_body<TR, TC>(a, blockIdx.x, gridDim.x);
}
template <int TR, int TC>
__global__ __launch_bounds__(256) void gram_block_grouped(const GramArgs* jobs, const unsigned* start, int nj) {
  int j = find_job(start, nj, blockIdx.x);
  gram_block_body<TR, TC>(jobs[j], blockIdx.x - start[j], start[j + 1] - start[j]);
}

// ---------------------------------------------------------------------------
// host launchers
// ---------------------------------------------------------------------------
constexpr int GTM = 4, GTN = 4, UTJ = 4, UTR = 4;   // real tiles
constexpr int BTN = 5;  // real per-block Grams: 64 x 80 tiles, i.e. one tile per block for q <= 16
constexpr int ZTM = 2, ZTN = 2, ZTJ = 2, ZTR = 2;   // complex tiles

constexpr int GKC_D = 16, GKC_F = 32, UKC_D = 32, UKC_F = 16;  // LDS chunk depths (measured best)

void gram_tiles(GramArgs& a) {
  if (a.lds == 2) {
    a.tiles_i = a.tiles_j = 1;
    return;
  }
  if (a.lds) {
    a.tiles_i = (a.M + LB - 1) / LB;
    a.tiles_j = (a.N + LB - 1) / LB;
    return;
  }
  int tm = a.cplx ? ZTM : GTM, tn = a.cplx ? ZTN : (a.site == 2 ? BTN : GTN);
  a.tiles_i = (a.M + 16 * tm - 1) / (16 * tm);
  a.tiles_j = (a.N + 16 * tn - 1) / (16 * tn);
}
void update_tiles(UpdateArgs& a) {
  if (a.lds) {
    a.tiles_j = (a.N + LB - 1) / LB;
    a.tiles_r = (int)(a.rows / LB);
    return;
  }
  int tj = a.cplx ? ZTJ : UTJ, tr = a.cplx ? ZTR : UTR;
  a.tiles_j = (a.N + 16 * tj - 1) / (16 * tj);
  a.tiles_r = (int)(a.rows / (16 * tr));
}

static int gram_kind(const GramArgs& a, bool f32acc) {
  if (a.lds == 2) return (a.M <= 64 && a.N <= 80) ? OP_GRAMB_1 : OP_GRAMB_2;
  if (a.lds) return (f32acc ? OP_GRAML_F0 : OP_GRAML_D0) + (a.site == 1 ? 1 : 0);
  int base = a.cplx ? (f32acc ? OP_GRAM_C0 : OP_GRAM_Z0) : (f32acc ? OP_GRAM_F0 : OP_GRAM_D0);
  return base + (a.site == 1 ? 1 : a.site == 2 ? 2 : 0);
}
static int update_kind(const UpdateArgs& a, bool f32) {
  if (a.lds) return (f32 ? OP_UPDATEL_F0 : OP_UPDATEL_D0) + (a.site == 1 ? 1 : 0);
  int base = a.cplx ? (f32 ? OP_UPDATE_C0 : OP_UPDATE_Z0) : (f32 ? OP_UPDATE_F0 : OP_UPDATE_D0);
  return base + (a.site == 1 ? 1 : 0);
}

#define PPCG_GRAM_CASES(KERNEL, GRID, ...)                                                                       \
  case OP_GRAM_D0: hipLaunchKernelGGL((KERNEL<double, GTM, GTN, false, 0>), dim3(GRID), dim3(64), 0, st, __VA_ARGS__); break; \
  case OP_GRAM_D1: hipLaunchKernelGGL((KERNEL<double, GTM, GTN, false, 1>), dim3(GRID), dim3(64), 0, st, __VA_ARGS__); break; \
  case OP_GRAM_D2: hipLaunchKernelGGL((KERNEL<double, GTM, BTN, false, 2>), dim3(GRID), dim3(64), 0, st, __VA_ARGS__); break; \
  case OP_GRAM_F0: hipLaunchKernelGGL((KERNEL<float, GTM, GTN, false, 0>), dim3(GRID), dim3(64), 0, st, __VA_ARGS__); break;  \
  case OP_GRAM_F1: hipLaunchKernelGGL((KERNEL<float, GTM, GTN, false, 1>), dim3(GRID), dim3(64), 0, st, __VA_ARGS__); break;  \
  case OP_GRAM_F2: hipLaunchKernelGGL((KERNEL<float, GTM, BTN, false, 2>), dim3(GRID), dim3(64), 0, st, __VA_ARGS__); break;  \
  case OP_GRAM_Z0: hipLaunchKernelGGL((KERNEL<double, ZTM, ZTN, true, 0>), dim3(GRID), dim3(64), 0, st, __VA_ARGS__); break;  \
  case OP_GRAM_Z1: hipLaunchKernelGGL((KERNEL<double, ZTM, ZTN, true, 1>), dim3(GRID), dim3(64), 0, st, __VA_ARGS__); break;  \
  case OP_GRAM_Z2: hipLaunchKernelGGL((KERNEL<double, ZTM, ZTN, true, 2>), dim3(GRID), dim3(64), 0, st, __VA_ARGS__); break;  \
  case OP_GRAM_C0: hipLaunchKernelGGL((KERNEL<float, ZTM, ZTN, true, 0>), dim3(GRID), dim3(64), 0, st, __VA_ARGS__); break;   \
  case OP_GRAM_C1: hipLaunchKernelGGL((KERNEL<float, ZTM, ZTN, true, 1>), dim3(GRID), dim3(64), 0, st, __VA_ARGS__); break;   \
  case OP_GRAM_C2: hipLaunchKernelGGL((KERNEL<float, ZTM, ZTN, true, 2>), dim3(GRID), dim3(64), 0, st, __VA_ARGS__); break;

#define PPCG_GRAML_CASES(KERNEL, GRID, ...)                                                                      \
  case OP_GRAML_D0: hipLaunchKernelGGL((KERNEL<double, GKC_D, 0>), dim3(GRID), dim3(256), 0, st, __VA_ARGS__); break; \
  case OP_GRAML_D1: hipLaunchKernelGGL((KERNEL<double, GKC_D, 1>), dim3(GRID), dim3(256), 0, st, __VA_ARGS__); break; \
  case OP_GRAML_F0: hipLaunchKernelGGL((KERNEL<float, GKC_F, 0>), dim3(GRID), dim3(256), 0, st, __VA_ARGS__); break;  \
  case OP_GRAML_F1: hipLaunchKernelGGL((KERNEL<float, GKC_F, 1>), dim3(GRID), dim3(256), 0, st, __VA_ARGS__); break;

#define PPCG_GRAMB_CASES(KERNEL, GRID, ...)                                                                      \
  case OP_GRAMB_1: hipLaunchKernelGGL((KERNEL<1, 5>), dim3(GRID), dim3(256), 0, st, __VA_ARGS__); break;          \
  case OP_GRAMB_2: hipLaunchKernelGGL((KERNEL<2, 10>), dim3(GRID), dim3(256), 0, st, __VA_ARGS__); break;

#ifndef PPCG_UPD64_LEAN
#define PPCG_UPD64_LEAN 1
#endif
#if PPCG_UPD64_LEAN
#define PPCG_UPDATEL_D(KERNEL, SITE, GRID, ...) \
  hipLaunchKernelGGL((KERNEL##_lean<double, 16, SITE>), dim3(GRID), dim3(256), 0, st, __VA_ARGS__)
#else
#define PPCG_UPDATEL_D(KERNEL, SITE, GRID, ...) \
  hipLaunchKernelGGL((KERNEL<double, UKC_D, SITE>), dim3(GRID), dim3(256), 0, st, __VA_ARGS__)
#endif
#define PPCG_UPDATEL_CASES(KERNEL, GRID, ...)                                                                    \
  case OP_UPDATEL_D0: PPCG_UPDATEL_D(KERNEL, 0, GRID, __VA_ARGS__); break;                                         \
  case OP_UPDATEL_D1: PPCG_UPDATEL_D(KERNEL, 1, GRID, __VA_ARGS__); break;                                         \
  case OP_UPDATEL_F0: hipLaunchKernelGGL((KERNEL<float, UKC_F, 0>), dim3(GRID), dim3(256), 0, st, __VA_ARGS__); break;  \
  case OP_UPDATEL_F1: hipLaunchKernelGGL((KERNEL<float, UKC_F, 1>), dim3(GRID), dim3(256), 0, st, __VA_ARGS__); break;

#define PPCG_UPDATE_CASES(KERNEL, GRID, ...)                                                                     \
  case OP_UPDATE_D0: hipLaunchKernelGGL((KERNEL<double, UTJ, UTR, false, 0>), dim3(GRID), dim3(64), 0, st, __VA_ARGS__); break; \
  case OP_UPDATE_D1: hipLaunchKernelGGL((KERNEL<double, UTJ, UTR, false, 1>), dim3(GRID), dim3(64), 0, st, __VA_ARGS__); break; \
  case OP_UPDATE_F0: hipLaunchKernelGGL((KERNEL<float, UTJ, UTR, false, 0>), dim3(GRID), dim3(64), 0, st, __VA_ARGS__); break;  \
  case OP_UPDATE_F1: hipLaunchKernelGGL((KERNEL<float, UTJ, UTR, false, 1>), dim3(GRID), dim3(64), 0, st, __VA_ARGS__); break;  \
  case OP_UPDATE_Z0: hipLaunchKernelGGL((KERNEL<double, ZTJ, ZTR, true, 0>), dim3(GRID), dim3(64), 0, st, __VA_ARGS__); break;  \
  case OP_UPDATE_Z1: hipLaunchKernelGGL((KERNEL<double, ZTJ, ZTR, true, 1>), dim3(GRID), dim3(64), 0, st, __VA_ARGS__); break;  \
  case OP_UPDATE_C0: hipLaunchKernelGGL((KERNEL<float, ZTJ, ZTR, true, 0>), dim3(GRID), dim3(64), 0, st, __VA_ARGS__); break;   \
  case OP_UPDATE_C1: hipLaunchKernelGGL((KERNEL<float, ZTJ, ZTR, true, 1>), dim3(GRID), dim3(64), 0, st, __VA_ARGS__); break;

static bool aligned16(const void* p) { return ((uintptr_t)p & 15) == 0; }

void launch_gram(const GramArgs& a0, bool f32acc, hipStream_t st) {
  GramArgs a = a0;
  if (a.lds == 2) {  // the single-pass per-block kernel's preconditions
    int extra = 0, a0 = 0;  // A segments that are not also B segments
    for (int sA = 0; sA < a.A.nseg; ++sA) {
      const int len = a.A.end[sA] - a0;
      bool found = false;
      int b0 = 0;
      for (int sB = 0; sB < a.B.nseg && !found; ++sB) {
        found = a.B.p[sB] == a.A.p[sA] && a.B.f32[sB] == a.A.f32[sA] && a.B.end[sB] - b0 >= len;
        b0 = a.B.end[sB];
      }
      if (!found) extra += len;
      a0 = a.A.end[sA];
    }
    bool ok = !a.cplx && !f32acc && a.M <= 128 && a.N <= 160 && a.N + extra <= BG_MAXU && a.chunk % 16 == 0 &&
              a.ld % 4 == 0 && !a.dsc && !a.dsc2;  // this kernel applies no row scales
    for (int s = 0; s < a.A.nseg; ++s) ok = ok && aligned16(a.A.p[s]);
    for (int s = 0; s < a.B.nseg; ++s) ok = ok && aligned16(a.B.p[s]);
    a.lds = ok ? 2 : 0;
  } else if (a.lds) {  // the LDS-staged kernel's preconditions; otherwise the one-wave kernel
    bool ok = !a.cplx && a.njobs == 1 && a.chunk % 32 == 0 && a.ld % 4 == 0;
    if (a.il && !ok) throw std::invalid_argument("interleaved complex Gram: LDS kernel preconditions not met");
    for (int s = 0; s < a.A.nseg; ++s) ok = ok && aligned16(a.A.p[s]);
    for (int s = 0; s < a.B.nseg; ++s) ok = ok && aligned16(a.B.p[s]);
    a.lds = ok;
  }
  gram_tiles(a);
  unsigned blocks = (unsigned)((long)a.tiles_i * a.tiles_j * a.splits * a.njobs);
  if (blocks == 0) return;
  int kind = gram_kind(a, f32acc);
  if (g_rec) {
    g_rec->add(kind, &a, sizeof(a), blocks);
    return;
  }
  switch (kind) {
    PPCG_GRAM_CASES(gram_kernel, blocks, a)
    PPCG_GRAML_CASES(gram_lds_kernel, blocks, a)
    PPCG_GRAMB_CASES(gram_block_kernel, blocks, a)
    default: break;
  }
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
  if (a.c64 && (!a.c0_keep || !f32 || (a.xd && !a.gd)))
    throw std::invalid_argument("update: float64 input needs a float32 update that keeps C0");
  if (a.lds)  // the LDS-staged kernel's preconditions; otherwise the one-wave kernel
    a.lds = !a.cplx && a.rows % LB == 0 && a.lda % 4 == 0 && aligned16(a.A) && a.job_a_off == 0 &&
            a.job_b_off == 0 && a.job_c_off == 0;
  update_tiles(a);
  unsigned blocks = (unsigned)((long)a.tiles_j * a.tiles_r);
  if (blocks == 0) return;
  int kind = update_kind(a, f32);
  if (g_rec) {
    g_rec->add(kind, &a, sizeof(a), blocks);
    return;
  }
  switch (kind) {
    PPCG_UPDATE_CASES(update_kernel, blocks, a)
    PPCG_UPDATEL_CASES(update_lds_kernel, blocks, a)
    default: break;
  }
}

bool launch_grouped_gemm(int kind, const void* jobs, const unsigned* start, int nj, unsigned total, hipStream_t st) {
  const GramArgs* gj = (const GramArgs*)jobs;
  const UpdateArgs* uj = (const UpdateArgs*)jobs;
  const ReduceArgs* rj = (const ReduceArgs*)jobs;
  switch (kind) {
    PPCG_GRAM_CASES(gram_grouped, total, gj, start, nj)
    PPCG_UPDATE_CASES(update_grouped, total, uj, start, nj)
    PPCG_GRAML_CASES(gram_lds_grouped, total, gj, start, nj)
    PPCG_GRAMB_CASES(gram_block_grouped, total, gj, start, nj)
    PPCG_UPDATEL_CASES(update_lds_grouped, total, uj, start, nj)
    case OP_REDUCE_D: hipLaunchKernelGGL((reduce_grouped<double, false>), dim3(total), dim3(256), 0, st, rj, start, nj); break;
    case OP_REDUCE_F: hipLaunchKernelGGL((reduce_grouped<float, false>), dim3(total), dim3(256), 0, st, rj, start, nj); break;
    case OP_REDUCE_Z: hipLaunchKernelGGL((reduce_grouped<double, true>), dim3(total), dim3(256), 0, st, rj, start, nj); break;
    case OP_REDUCE_C: hipLaunchKernelGGL((reduce_grouped<float, true>), dim3(total), dim3(256), 0, st, rj, start, nj); break;
    default: return false;
  }
  return true;
}

}  // namespace ppcg
