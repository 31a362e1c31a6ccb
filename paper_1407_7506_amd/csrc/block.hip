// Per-sub-block work of PPCG (Algorithm 3, steps 11-16; section 5.1):
//   block_pencil  the 3q x 3q (2q x 2q while P is empty) projected problem
//                 herm(S^H A S) c = theta herm(S^H S) c, S = [X_j W_j P_j],
//                 keeping the q lowest pairs with C^H (S^H S) C = I
//                 (projected problem of section 2); one workgroup per
//                 block, everything in LDS up to nS = 48; for nS up to 96
//                 (sub-blocks of width up to 32) the four nS x nS work
//                 matrices live in a per-block device scratch area (L2
//                 resident) and only the vectors stay in LDS
//   block_update  P_j <- W_j C_W + P_j C_P ;  X_j <- X_j C_X + P_j
// In the mixed-precision path H W and H P are float32 products, whose
// rounding error (~1e-7 |H| |w|) would swamp the X-W coupling x^H H w =
// r^H T r (Theorem 2), which is second order in the residual; those entries
// are therefore taken from the float64 H X as (H X_j)^H W_j.
// Safeguards where the paper is silent: diagonal scaling of the pencil, zero
// W/P columns dropped, a Cholesky of the scaled Gram that drops columns
// whose pivot falls below pivot_tol (taken in the order X, W, P), and the
// rank indicator of Theorem 1 (C_X singular) answered by re-solving the
// block without P (Theorem 2).  S is double or zdouble (Hermitian).
#include <stdexcept>
#include <type_traits>

#include "common.hpp"
#include "jacobi.hpp"
#include "kernels.hpp"

namespace ppcg {

#ifndef PPCG_PENCIL_NT
#define PPCG_PENCIL_NT 1024
#endif
// threads of a pencil workgroup (the Jacobi rounds of the larger pencils
// spread their 2x2 updates over more waves)
template <int NB> constexpr int pencil_nt() { return NB <= 24 ? 256 : PPCG_PENCIL_NT; }

template <int NB, class S>
PPCG_DEV void block_pencil_body(const PencilArgs& a, unsigned wg, unsigned) {
  constexpr int LD = NB + 1;
  constexpr int NT = pencil_nt<NB>();
  constexpr bool IN_LDS = NB <= 48;
  static_assert(IN_LDS || 4L * NB * LD <= pencil_work_elems(), "pencil scratch too small");
  __shared__ S shm[IN_LDS ? 4 * NB * LD : 1];
  __shared__ double Dv[NB], cs[NB + 2];
  __shared__ JRot<S> jr[NB / 2 + 1];
  __shared__ int keep[NB], acc[NB], pq[NB + 2], nacc, sing;
  const int tid = threadIdx.x;
  const int blk = (int)wg;
  S* b0 = IN_LDS ? shm : (S*)a.work + (long)blk * pencil_work_elems();
  S* b1 = b0 + NB * LD;
  S* b2 = b1 + NB * LD;
  S* b3 = b2 + NB * LD;
  const int q = a.q, nS = a.nS;
  const S* gram = (const S*)a.gram + (long)blk * a.gstride;
  const S* Gm = (const S*)a.G;
  const int ldgr = nS + (a.ax_rows ? q : 0);
  const int c0 = blk * q;
  const S zero = from_real<S>(0.0);
  int flag = 0;
  for (int pass = 0; pass < 2; ++pass) {
    const bool allowP = (nS == 3 * q) && pass == 0;
    // 1. load A (b0) and B (b1)
    if (a.tiles16) {
      // 16 x 16 tiles of the upper block triangle; the lower blocks mirror them
      for (int e = tid; e < nS * nS; e += NT) {
        const int i = e % nS, j = e / nS;
        const int I = i >> 4, J = j >> 4;
        const bool up = I <= J;
        const int lo = up ? I : J, hi = up ? J : I;
        const int o = up ? (i & 15) + 16 * (j & 15) : (j & 15) + 16 * (i & 15);
        const int ts = lo == 0 ? hi : (lo == 1 ? 2 + hi : 5);
        const int th = lo == 0 ? 8 + hi : (lo == 1 ? 5 + hi : 8);
        const S vs = gram[ts * 256 + o];
        b1[i + j * LD] = up ? vs : conj_(vs);
        if (hi == 0) {
          b0[i + j * LD] = Gm[(c0 + i) + (long)(c0 + j) * a.ldg];
        } else {
          const S vh = gram[th * 256 + o];
          b0[i + j * LD] = up ? vh : conj_(vh);
        }
      }
    } else {
      for (int e = tid; e < nS * nS; e += NT) {
        int i = e % nS, j = e / nS;
        b1[i + j * LD] = gram[i + j * ldgr];
        if (j >= q) {
          // X rows of the W / P columns: (H X_j)^H W_j and (H X_j)^H P_j when available
          b0[i + j * LD] = (a.ax_rows && i < q) ? gram[(nS + i) + j * ldgr] : gram[i + (nS + j - q) * ldgr];
        } else if (i < q) {
          b0[i + j * LD] = Gm[(c0 + i) + (long)(c0 + j) * a.ldg];
        }
      }
      __syncthreads();
      for (int e = tid; e < nS * q; e += NT) {
        int j = e % q, i = q + e / q;  // fill the X columns below the X block
        if (i < nS) b0[i + j * LD] = conj_(b0[j + i * LD]);
      }
    }
    __syncthreads();
    // Hermitian parts
    for (int e = tid; e < nS * nS; e += NT) {
      int i = e % nS, j = e / nS;
      if (i < j) {
        S va = 0.5 * (b0[i + j * LD] + conj_(b0[j + i * LD]));
        S vb = 0.5 * (b1[i + j * LD] + conj_(b1[j + i * LD]));
        b0[i + j * LD] = va; b0[j + i * LD] = conj_(va);
        b1[i + j * LD] = vb; b1[j + i * LD] = conj_(vb);
      } else if (i == j) {
        b0[i + i * LD] = from_real<S>(real_(b0[i + i * LD]));
        b1[i + i * LD] = from_real<S>(real_(b1[i + i * LD]));
      }
    }
    __syncthreads();
    // 2. keep mask and scaling
    if (tid == 0) {
      double xmax = 0;
      for (int i = 0; i < q; ++i) xmax = fmax(xmax, real_(b1[i + i * LD]));
      for (int i = 0; i < nS; ++i) {
        double d = real_(b1[i + i * LD]);
        int kp = (i < q) || (d > a.drop_tol * a.drop_tol * xmax);
        if (i >= 2 * q && !allowP) kp = 0;
        if (!(d > 0)) kp = 0;
        keep[i] = kp;
        Dv[i] = kp ? 1.0 / sqrt(d) : 0.0;
      }
    }
    __syncthreads();
    for (int e = tid; e < nS * nS; e += NT) {
      int i = e % nS, j = e / nS;
      double sc = Dv[i] * Dv[j];
      b0[i + j * LD] = sc * b0[i + j * LD];
      b1[i + j * LD] = sc * b1[i + j * LD];
    }
    __syncthreads();
    // 3. greedy right-looking Cholesky of the scaled Gram (b1, in place)
    for (int c = 0; c < nS; ++c) {
      if (!keep[c]) continue;  // uniform
      double piv = real_(b1[c + c * LD]);
      if (!(piv >= a.pivot_tol)) {
        __syncthreads();
        if (tid == 0) keep[c] = 0;
        __syncthreads();
        continue;
      }
      double lcc = sqrt(piv);
      for (int i = c + 1 + tid; i < nS; i += NT)
        if (keep[i]) b1[i + c * LD] = (1.0 / lcc) * b1[i + c * LD];
      __syncthreads();
      if (tid == 0) b1[c + c * LD] = from_real<S>(lcc);
      int nr = nS - c - 1;
      for (int e = tid; e < nr * nr; e += NT) {
        int i = c + 1 + e % nr, j = c + 1 + e / nr;
        if (i >= j && keep[i] && keep[j]) b1[i + j * LD] -= b1[i + c * LD] * conj_(b1[j + c * LD]);
      }
      __syncthreads();
    }
    if (tid == 0) {
      int r = 0;
      for (int i = 0; i < nS; ++i)
        if (keep[i]) acc[r++] = i;
      nacc = r;
    }
    __syncthreads();
    const int r = nacc;
    if (r < q) {
      // rank failure: leave the block unchanged (C = [I; 0; 0]) and report
      flag |= 4;
      S* C = (S*)a.C + (long)blk * a.cstride;
      for (int e = tid; e < 3 * q * q; e += NT) {
        int i = e % (3 * q), t = e / (3 * q);
        C[i + t * 3 * q] = from_real<S>(i == t ? 1.0 : 0.0);
      }
      break;
    }
    // 4. compact: L (b2, lower r x r) and A (b3)
    for (int e = tid; e < r * r; e += NT) {
      int x = e % r, y = e / r;
      b2[x + y * LD] = (x >= y) ? b1[acc[x] + acc[y] * LD] : zero;
      b3[x + y * LD] = b0[acc[x] + acc[y] * LD];
    }
    __syncthreads();
    // 5. Linv (b1) by forward substitution, one thread per column, in column
    //    order: entry x of column y receives the terms L_xt Linv_ty in
    //    increasing t, as in the dot-product form, but the updates of one
    //    step t are independent of each other
    for (int y = tid; y < r; y += NT) {
      for (int x = 0; x < r; ++x) b1[x + y * LD] = from_real<S>(x == y ? 1.0 : 0.0);
      for (int t = y; t < r; ++t) {
        const S lt = (1.0 / real_(b2[t + t * LD])) * b1[t + y * LD];
        b1[t + y * LD] = lt;
        for (int x = t + 1; x < r; ++x) b1[x + y * LD] -= b2[x + t * LD] * lt;
      }
    }
    __syncthreads();
    // 6. T = A Linv^H (b2), M = Linv T (b3)
    for (int e = tid; e < r * r; e += NT) {
      int x = e % r, y = e / r;
      S s = zero;
      for (int t = 0; t <= y; ++t) s += b3[x + t * LD] * conj_(b1[y + t * LD]);
      b2[x + y * LD] = s;
    }
    __syncthreads();
    for (int e = tid; e < r * r; e += NT) {
      int x = e % r, y = e / r;
      S s = zero;
      for (int t = 0; t <= x; ++t) s += b1[x + t * LD] * b2[t + y * LD];
      b3[x + y * LD] = s;
    }
    __syncthreads();
    for (int e = tid; e < r * r; e += NT) {
      int x = e % r, y = e / r;
      if (x < y) {
        S v = 0.5 * (b3[x + y * LD] + conj_(b3[y + x * LD]));
        b3[x + y * LD] = v;
        b3[y + x * LD] = conj_(v);
      } else if (x == y) {
        b3[x + x * LD] = from_real<S>(real_(b3[x + x * LD]));
      }
    }
    __syncthreads();
    // 7. eigen-decomposition M = Y diag Y^H (Y in b0).  Rotations below
    //    jacobi_rel |M|_F are skipped: the pencil only has to give a good
    //    step, and the caller sizes jacobi_rel well below the X-W coupling
    //    (of the order of the residual) that the step has to resolve.
    {
      double fro = 0;
      for (int e = tid; e < r * r; e += NT) fro += abs2_(b3[(e % r) + (e / r) * LD]);
      fro = wave_sum(fro);
      if ((tid & 63) == 0) cs[tid >> 6] = fro;
      __syncthreads();
      fro = 0;
#pragma unroll
      for (int w = 0; w < NT / 64; ++w) fro += cs[w];
      __syncthreads();
      lds_jacobi<NT, S>(b3, b0, r, LD, a.jacobi_rel * sqrt(fro), 40, jr, cs);
    }
    // 8. ascending order (ties by index): rank -> keep[] reused as sel
    for (int x = tid; x < r; x += NT) {
      double lx = real_(b3[x + x * LD]);
      int rk = 0;
      for (int y = 0; y < r; ++y) {
        double ly = real_(b3[y + y * LD]);
        rk += (ly < lx) || (ly == lx && y < x);
      }
      pq[x] = rk;  // temporarily the rank of x
    }
    __syncthreads();
    for (int x = tid; x < r; x += NT) keep[pq[x]] = x;
    __syncthreads();
    // 9. C_acc = Linv^H Y[:, sel[0..q)]  (b2, r x q)
    for (int e = tid; e < r * q; e += NT) {
      int x = e % r, t = e / r;
      int col = keep[t];
      S s = zero;
      for (int y = x; y < r; ++y) s += conj_(b1[y + x * LD]) * b0[y + col * LD];
      b2[x + t * LD] = s;
    }
    __syncthreads();
    // 10. Theorem 1 indicator when P columns took part
    int usedP = 0;
    for (int x = 0; x < r; ++x) usedP |= (acc[x] >= 2 * q);
    if (usedP && pass == 0) {
      // Gc = C_X^H C_X (b3, q x q) over the kept X rows
      for (int e = tid; e < q * q; e += NT) {
        int u = e % q, v = e / q;
        S s = zero;
        for (int x = 0; x < r; ++x) {
          int i = acc[x];
          if (i >= q) break;
          s += (Dv[i] * Dv[i]) * (conj_(b2[x + u * LD]) * b2[x + v * LD]);
        }
        b3[u + v * LD] = s;
      }
      __syncthreads();
      // right-looking Cholesky of the q x q Gram over the workgroup (every
      // thread reads the same pivots, so the exit is uniform).  The columns
      // of C are B-orthonormal and X is orthonormal and orthogonal to W and
      // P, so C_X^H C_X <= I: pivots are compared with 1, and a C_X that
      // vanishes to rounding counts as singular.
      int bad = 0;
      for (int c = 0; c < q; ++c) {
        const double piv = real_(b3[c + c * LD]);
        if (!(piv >= a.sing_tol)) {
          bad = 1;
          break;
        }
        const double l = sqrt(piv);
        for (int i = c + 1 + tid; i < q; i += NT) b3[i + c * LD] = (1.0 / l) * b3[i + c * LD];
        __syncthreads();
        const int nr = q - c - 1;
        for (int e = tid; e < nr * nr; e += NT) {
          const int i = c + 1 + e % nr, j = c + 1 + e / nr;
          if (i >= j) b3[i + j * LD] -= b3[i + c * LD] * conj_(b3[j + c * LD]);
        }
        __syncthreads();
      }
      if (tid == 0) sing = bad;
      __syncthreads();
      if (sing) {
        flag |= 2;
        continue;  // pass 1 without P
      }
    }
    if (usedP) flag |= 1;
    flag |= ((allowP ? 3 * q : 2 * q) - r) << 8;  // W/P columns left out
    // 11. write C (nS x q, ld 3q): zero rows for dropped columns
    S* C = (S*)a.C + (long)blk * a.cstride;
    const int ldc = 3 * q;
    for (int e = tid; e < ldc * q; e += NT) {
      int i = e % ldc, t = e / ldc;
      C[i + t * ldc] = zero;
    }
    __syncthreads();
    for (int e = tid; e < r * q; e += NT) {
      int x = e % r, t = e / r;
      int i = acc[x];
      C[i + t * ldc] = Dv[i] * b2[x + t * LD];
    }
    break;
  }
  if (tid == 0) a.flags[blk] = flag;
}

template <int NB, class S>
__global__ __launch_bounds__(pencil_nt<NB>()) void block_pencil_kernel(PencilArgs a) {
  block_pencil_body<NB, S>(a, blockIdx.x, gridDim.x);
}
template <int NB, class S>
__global__ __launch_bounds__(pencil_nt<NB>()) void block_pencil_grouped(const PencilArgs* jobs, const unsigned* start, int nj) {
  int j = find_job(start, nj, blockIdx.x);
  block_pencil_body<NB, S>(jobs[j], blockIdx.x - start[j], start[j + 1] - start[j]);
}

static int pencil_kind(const PencilArgs& a) {
  if (a.cplx) return a.nS <= 24 ? OP_PENCILZ24 : (a.nS <= 48 ? OP_PENCILZ48 : OP_PENCILZ96);
  return a.nS <= 24 ? OP_PENCIL24 : (a.nS <= 48 ? OP_PENCIL48 : OP_PENCIL96);
}

#define PPCG_PENCIL_SWITCH(KERNEL, GRID, ...)                                                                   \
  switch (kind) {                                                                                              \
    case OP_PENCIL24: hipLaunchKernelGGL((KERNEL<24, double>), dim3(GRID), dim3(pencil_nt<24>()), 0, st, __VA_ARGS__); break;  \
    case OP_PENCIL48: hipLaunchKernelGGL((KERNEL<48, double>), dim3(GRID), dim3(pencil_nt<48>()), 0, st, __VA_ARGS__); break;  \
    case OP_PENCILZ24: hipLaunchKernelGGL((KERNEL<24, zdouble>), dim3(GRID), dim3(pencil_nt<24>()), 0, st, __VA_ARGS__); break; \
    case OP_PENCILZ48: hipLaunchKernelGGL((KERNEL<48, zdouble>), dim3(GRID), dim3(pencil_nt<48>()), 0, st, __VA_ARGS__); break; \
    case OP_PENCIL96: hipLaunchKernelGGL((KERNEL<96, double>), dim3(GRID), dim3(pencil_nt<96>()), 0, st, __VA_ARGS__); break;  \
    case OP_PENCILZ96: hipLaunchKernelGGL((KERNEL<96, zdouble>), dim3(GRID), dim3(pencil_nt<96>()), 0, st, __VA_ARGS__); break; \
    default: break;                                                                                            \
  }

// Lays out given pencils (A_j, B_j), nS x nS each (ld nS, stride nS^2), in
// the pencil kernel's input form: per block an nS x (2 nS - q) Gram holding
// B_j in columns [0, nS) and the columns [q, nS) of A_j after them, and the
// q x q X block of A_j at offset j q (q + 1) with leading dimension q (the
// kernel's G[j q + i, j q + c] addressing with ldg = q).  S: double or zdouble.
template <class S>
__global__ __launch_bounds__(256) void pencil_pack_kernel(const S* A, const S* B, int nblocks, int q, int nS, S* gram,
                                                         S* G) {
  const long e = blockIdx.x * 256L + threadIdx.x;
  const long per = (long)nS * nS;
  if (e >= per * nblocks) return;
  const int j = (int)(e / per);
  const int r = (int)(e % per);
  const int i = r % nS, c = r / nS;
  const long Nb = 2L * nS - q;
  S* gj = gram + (long)j * nS * Nb;
  gj[r] = B[e];
  const S a = A[e];
  if (c >= q) gj[per + i + (long)(c - q) * nS] = a;
  if (i < q && c < q) G[(long)j * q * (q + 1) + i + (long)c * q] = a;
}

void launch_pencil_pack(const double* A, const double* B, int nblocks, int q, int nS, int cplx, double* gram,
                        double* G, hipStream_t st) {
  const long tot = (long)nS * nS * nblocks;
  if (tot <= 0) return;
  const unsigned grid = (unsigned)((tot + 255) / 256);
  if (cplx)
    hipLaunchKernelGGL(pencil_pack_kernel<zdouble>, dim3(grid), dim3(256), 0, st, (const zdouble*)A,
                       (const zdouble*)B, nblocks, q, nS, (zdouble*)gram, (zdouble*)G);
  else
    hipLaunchKernelGGL(pencil_pack_kernel<double>, dim3(grid), dim3(256), 0, st, A, B, nblocks, q, nS, gram, G);
}

void launch_block_pencil(const PencilArgs& a, hipStream_t st) {
  unsigned blocks = a.nblocks > 0 ? (unsigned)a.nblocks : 0;
  if (a.nS > 96 || (a.nS > 48 && !a.work))
    throw std::invalid_argument("block pencil: nS > 96, or nS > 48 without device scratch");
  int kind = pencil_kind(a);
  if (g_rec) {
    g_rec->add(kind, &a, sizeof(a), blocks);
    return;
  }
  if (blocks == 0) return;
  PPCG_PENCIL_SWITCH(block_pencil_kernel, blocks, a)
}

// ---------------------------------------------------------------------------
// TW: storage of W/P (double, float, zdouble, zfloat); SX: X and arithmetic.
// Real blocks up to 16 columns: two consecutive rows per thread, read and
// written as 8- or 16-byte pairs (half the memory instructions of one row
// per thread, which matters most for the float32 W and P of the mixed path);
// complex or wider blocks: one row per thread.  The 3q x q coefficients are
// the same for every lane.
template <class SX, int QM> constexpr int bupd_rpt() { return (sc_traits<SX>::cplx || QM > 16) ? 1 : 2; }
#ifndef PPCG_BUPD_SCALAR_C
#define PPCG_BUPD_SCALAR_C 1
#endif
// a value at a workgroup-uniform address of memory the kernel does not write,
// read through the constant address space (a scalar load into SGPRs)
template <class S>
PPCG_DEV S uniform_load(const S* p) {
  typedef typename sc_traits<S>::real_t R;
  typedef const __attribute__((address_space(4))) R* CR;
  CR r = (CR)(const R*)p;
  if constexpr (sc_traits<S>::cplx) return S{r[0], r[1]};
  else return r[0];
}

// Complex or wide blocks: one row per lane, the q output columns split into
// groups of NO, one group per wave (or pair of waves) of the workgroup, and
// the inputs streamed one column at a time, so only the 2 NO accumulators of a
// group stay in registers.  Every group reads the whole row of X, W and P
// (from the CU's cache after the first); a barrier separates those reads from
// the in-place stores of X and P.  Each output receives the same operations
// in the same order as in the row-per-thread form.
template <class SX> constexpr int bupd_no() { return sc_traits<SX>::cplx ? 8 : 16; }
template <class TW, class SX, int QM>
PPCG_DEV void block_update_wide_body(const BlockUpdArgs& a, unsigned wg, unsigned nwg) {
  constexpr int NO = QM < bupd_no<SX>() ? QM : bupd_no<SX>();
  constexpr int G = QM / NO;    // output groups
  constexpr int RW = 256 / G;   // rows per workgroup (a multiple of 64: groups are whole waves)
  const int q = a.q;
  const unsigned rtiles = (unsigned)((a.rows + RW - 1) / RW);
  const unsigned L = xcd_remap(wg, nwg);
  const int blk = L / rtiles;
  const int grp = threadIdx.x / RW;
  const long r = (long)(L % rtiles) * RW + threadIdx.x % RW;
  const int t0 = grp * NO;
  const bool ok = r < a.rows;
  const SX* __restrict__ C = (const SX*)a.C + (long)blk * a.cstride;
  const int ldc = 3 * q;
  const long cb = (long)blk * q * a.ld;
  SX* X = (SX*)a.X + cb;
  TW* W = (TW*)a.W + cb;
  TW* P = (TW*)a.P + cb;
  const SX zero = from_real<SX>(0.0);
  // the block's coefficients in LDS, [input i][output t] for each of the
  // X, W and P parts, read as broadcasts (one address for the whole wave)
  __shared__ SX Cs[3 * QM * QM];
  for (int e = threadIdx.x; e < 3 * q * q; e += 256) {
    const int i = e % ldc, t = e / ldc;  // C is 3q x q, ld 3q
    const int part = i / q, ii = i % q;
    Cs[(part * QM + ii) * QM + t] = C[i + (long)t * ldc];
  }
  __syncthreads();
  SX xn[NO], pn[NO];
#pragma unroll
  for (int u = 0; u < NO; ++u) xn[u] = pn[u] = zero;
  if (ok && t0 < q) {
    for (int i = 0; i < q; ++i) {
      const long o = r + i * a.ld;
      const SX x = X[o];
      const SX w = cvt<SX, TW>(W[o]);
      const SX p = a.hasP ? cvt<SX, TW>(P[o]) : zero;
      const SX* cx_ = Cs + i * QM + t0;
      const SX* cw_ = Cs + (QM + i) * QM + t0;
      const SX* cp_ = Cs + (2 * QM + i) * QM + t0;
#pragma unroll
      for (int u = 0; u < NO; ++u) {
        if (t0 + u < q) {
          pn[u] += w * cw_[u];
          if (a.hasP) pn[u] += p * cp_[u];
          xn[u] += x * cx_[u];
        }
      }
    }
  }
  __syncthreads();  // every group has read the row before any group overwrites it
  if (ok && t0 < q) {
#pragma unroll
    for (int u = 0; u < NO; ++u) {
      const int t = t0 + u;
      if (t < q) {
        const long o = r + t * a.ld;
        xn[u] += pn[u];
        P[o] = cvt<TW, SX>(pn[u]);
        X[o] = xn[u];
      }
    }
  }
}

template <class TW, class SX, int QM>
PPCG_DEV void block_update_body(const BlockUpdArgs& a, unsigned wg, unsigned nwg) {
  if constexpr (sc_traits<SX>::cplx || QM > 16) {
    block_update_wide_body<TW, SX, QM>(a, wg, nwg);
    return;
  }
  constexpr int RPT = bupd_rpt<SX, QM>();
  const int q = a.q;
  const unsigned rtiles = (unsigned)((a.rows + 256 * RPT - 1) / (256 * RPT));
  unsigned L = xcd_remap(wg, nwg);
  int blk = L / rtiles;
  const long r0 = (long)(L % rtiles) * 256 * RPT + (long)threadIdx.x * RPT;  // rows r0 .. r0 + RPT - 1
  const SX* __restrict__ C = (const SX*)a.C + (long)blk * a.cstride;
  const int ldc = 3 * q;
#if PPCG_BUPD_SCALAR_C
  // the coefficients are the same for every lane: read through the constant
  // address space at workgroup-uniform addresses, i.e. by scalar loads into
  // SGPRs that the FMAs take as operands (C is not written by this kernel)
  const SX* Cs = C;
  constexpr int CLD = 0;  // column t of C at Cs + t * ldc
#else
  __shared__ SX Cs[3 * QM * QM];
  constexpr int CLD = 3 * QM;
  for (int e = threadIdx.x; e < 3 * q * q; e += 256) {
    int i = e % ldc, t = e / ldc;
    Cs[i + t * 3 * QM] = C[i + t * ldc];
  }
  __syncthreads();
#endif
  const long cb = (long)blk * q * a.ld;
  SX* X = (SX*)a.X + cb;
  TW* W = (TW*)a.W + cb;
  TW* P = (TW*)a.P + cb;
  const SX zero = from_real<SX>(0.0);
  SX x[RPT][QM], w[RPT][QM], p[RPT][QM];
  // rows is a multiple of 256 and r0 a multiple of RPT: a thread's rows are all in range or all out
  const bool ok = r0 < a.rows;
#pragma unroll
  for (int i = 0; i < QM; ++i) {
    if (i < q && ok) {
      const long o = r0 + i * a.ld;
      if constexpr (RPT == 2) {  // real: pairs of consecutive rows (ld and r0 even: aligned)
        typedef typename std::conditional<sizeof(TW) == 8, double2, float2>::type tw2;
        const double2 xv = *(const double2*)(X + o);
        const tw2 wv = *(const tw2*)(W + o);
        x[0][i] = xv.x;
        x[1][i] = xv.y;
        w[0][i] = (SX)wv.x;
        w[1][i] = (SX)wv.y;
        if (a.hasP) {
          const tw2 pv = *(const tw2*)(P + o);
          p[0][i] = (SX)pv.x;
          p[1][i] = (SX)pv.y;
        } else {
          p[0][i] = p[1][i] = zero;
        }
      } else {
        x[0][i] = X[o];
        w[0][i] = cvt<SX, TW>(W[o]);
        p[0][i] = a.hasP ? cvt<SX, TW>(P[o]) : zero;
      }
    } else {
#pragma unroll
      for (int u = 0; u < RPT; ++u) x[u][i] = w[u][i] = p[u][i] = zero;
    }
  }
  for (int t = 0; t < q; ++t) {
    const SX* ct = Cs + t * (CLD ? CLD : ldc);
    SX pn[RPT], xn[RPT];
#pragma unroll
    for (int u = 0; u < RPT; ++u) pn[u] = xn[u] = zero;
#pragma unroll
    for (int i = 0; i < QM; ++i) {
      if (i < q) {
#if PPCG_BUPD_SCALAR_C
        const SX cw = uniform_load(ct + q + i), cp = uniform_load(ct + 2 * q + i), cx = uniform_load(ct + i);
#else
        const SX cw = ct[q + i], cp = ct[2 * q + i], cx = ct[i];
#endif
#pragma unroll
        for (int u = 0; u < RPT; ++u) {
          pn[u] += w[u][i] * cw;
          if (a.hasP) pn[u] += p[u][i] * cp;
          xn[u] += x[u][i] * cx;
        }
      }
    }
    if (ok) {
      const long o = r0 + t * a.ld;
#pragma unroll
      for (int u = 0; u < RPT; ++u) xn[u] += pn[u];
      if constexpr (RPT == 2) {
        typedef typename std::conditional<sizeof(TW) == 8, double2, float2>::type tw2;
        tw2 pv;
        pv.x = (decltype(pv.x))pn[0];
        pv.y = (decltype(pv.y))pn[1];
        *(tw2*)(P + o) = pv;
        *(double2*)(X + o) = make_double2(xn[0], xn[1]);
      } else {
        P[o] = cvt<TW, SX>(pn[0]);
        X[o] = xn[0];
      }
    }
  }
}

template <class TW, class SX, int QM>
__global__ __launch_bounds__(256) void block_update_kernel(BlockUpdArgs a) {
  block_update_body<TW, SX, QM>(a, blockIdx.x, gridDim.x);
}
template <class TW, class SX, int QM>
__global__ __launch_bounds__(256) void block_update_grouped(const BlockUpdArgs* jobs, const unsigned* start, int nj) {
  int j = find_job(start, nj, blockIdx.x);
  block_update_body<TW, SX, QM>(jobs[j], blockIdx.x - start[j], start[j + 1] - start[j]);
}

static int bupd_kind(const BlockUpdArgs& a) {
  int base = a.cplx ? (a.f32 ? OP_BUPD_C4 : OP_BUPD_Z4) : (a.f32 ? OP_BUPD_F4 : OP_BUPD_D4);
  return base + (a.q <= 4 ? 0 : a.q <= 8 ? 1 : a.q <= 16 ? 2 : 3);
}

#define PPCG_BUPD_SWITCH(KERNEL, GRID, ...)                                                                      \
  switch (kind) {                                                                                               \
    case OP_BUPD_D4: hipLaunchKernelGGL((KERNEL<double, double, 4>), dim3(GRID), dim3(256), 0, st, __VA_ARGS__); break;    \
    case OP_BUPD_D8: hipLaunchKernelGGL((KERNEL<double, double, 8>), dim3(GRID), dim3(256), 0, st, __VA_ARGS__); break;    \
    case OP_BUPD_D16: hipLaunchKernelGGL((KERNEL<double, double, 16>), dim3(GRID), dim3(256), 0, st, __VA_ARGS__); break;  \
    case OP_BUPD_D32: hipLaunchKernelGGL((KERNEL<double, double, 32>), dim3(GRID), dim3(256), 0, st, __VA_ARGS__); break;  \
    case OP_BUPD_F4: hipLaunchKernelGGL((KERNEL<float, double, 4>), dim3(GRID), dim3(256), 0, st, __VA_ARGS__); break;     \
    case OP_BUPD_F8: hipLaunchKernelGGL((KERNEL<float, double, 8>), dim3(GRID), dim3(256), 0, st, __VA_ARGS__); break;     \
    case OP_BUPD_F16: hipLaunchKernelGGL((KERNEL<float, double, 16>), dim3(GRID), dim3(256), 0, st, __VA_ARGS__); break;   \
    case OP_BUPD_F32: hipLaunchKernelGGL((KERNEL<float, double, 32>), dim3(GRID), dim3(256), 0, st, __VA_ARGS__); break;   \
    case OP_BUPD_Z4: hipLaunchKernelGGL((KERNEL<zdouble, zdouble, 4>), dim3(GRID), dim3(256), 0, st, __VA_ARGS__); break;  \
    case OP_BUPD_Z8: hipLaunchKernelGGL((KERNEL<zdouble, zdouble, 8>), dim3(GRID), dim3(256), 0, st, __VA_ARGS__); break;  \
    case OP_BUPD_Z16: hipLaunchKernelGGL((KERNEL<zdouble, zdouble, 16>), dim3(GRID), dim3(256), 0, st, __VA_ARGS__); break; \
    case OP_BUPD_Z32: hipLaunchKernelGGL((KERNEL<zdouble, zdouble, 32>), dim3(GRID), dim3(256), 0, st, __VA_ARGS__); break; \
    case OP_BUPD_C4: hipLaunchKernelGGL((KERNEL<zfloat, zdouble, 4>), dim3(GRID), dim3(256), 0, st, __VA_ARGS__); break;   \
    case OP_BUPD_C8: hipLaunchKernelGGL((KERNEL<zfloat, zdouble, 8>), dim3(GRID), dim3(256), 0, st, __VA_ARGS__); break;   \
    case OP_BUPD_C16: hipLaunchKernelGGL((KERNEL<zfloat, zdouble, 16>), dim3(GRID), dim3(256), 0, st, __VA_ARGS__); break; \
    case OP_BUPD_C32: hipLaunchKernelGGL((KERNEL<zfloat, zdouble, 32>), dim3(GRID), dim3(256), 0, st, __VA_ARGS__); break; \
    default: break;                                                                                             \
  }

void launch_block_update(const BlockUpdArgs& a, hipStream_t st) {
  // rows per workgroup of the selected kernel: the wide form's 256 / groups,
  // else 256 times the rows per thread
  const int qm = a.q <= 4 ? 4 : a.q <= 8 ? 8 : a.q <= 16 ? 16 : 32;
  const int no = a.cplx ? 8 : 16;
  const long rpw = (a.cplx || a.q > 16) ? 256 / (qm < no ? 1 : qm / no) : 512;
  unsigned blocks = (unsigned)(((a.rows + rpw - 1) / rpw) * (a.nblocks > 0 ? a.nblocks : 0));
  int kind = bupd_kind(a);
  if (g_rec) {
    g_rec->add(kind, &a, sizeof(a), blocks);
    return;
  }
  if (blocks == 0) return;
  PPCG_BUPD_SWITCH(block_update_kernel, blocks, a)
}

bool launch_grouped_block(int kind, const void* jobs, const unsigned* start, int nj, unsigned total, hipStream_t st) {
  if (kind >= OP_PENCIL24 && kind <= OP_PENCILZ96) {
    const PencilArgs* pj = (const PencilArgs*)jobs;
    PPCG_PENCIL_SWITCH(block_pencil_grouped, total, pj, start, nj)
    return true;
  }
  if (kind >= OP_BUPD_D4 && kind <= OP_BUPD_C32) {
    const BlockUpdArgs* bj = (const BlockUpdArgs*)jobs;
    PPCG_BUPD_SWITCH(block_update_grouped, total, bj, start, nj)
    return true;
  }
  return false;
}

}  // namespace ppcg
