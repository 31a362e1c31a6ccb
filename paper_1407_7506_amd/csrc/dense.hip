// Dense m x m kernels (column-major, ld >= m):
//   chol_inverse      G = L L^H and L^{-1}, blocked (32 x 32 tiles), for
//                     Cholesky-QR (section 5.5) and the Rayleigh-Ritz
//                     reduction to a standard problem (section 5.6)
//   block_jacobi_eig  Hermitian eigen-decomposition of the reduced
//                     Rayleigh-Ritz matrix by block Jacobi: pairs of 16-wide
//                     diagonal blocks are diagonalised in LDS and their
//                     rotations applied to the block rows, then columns
//   misc              fills, transposes, diagonal set, Frobenius norms
#include "common.hpp"
#include "jacobi.hpp"
#include "kernels.hpp"

namespace ppcg {

constexpr int CB = 32;       // Cholesky tile
constexpr int CLD = CB + 1;

// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void chol_diag_kernel(double* G, int ld, int m, int p, double* L, double* Li,
                                                        int* flag) {
  __shared__ double S[CB * CLD], I[CB * CLD];
  __shared__ int bad;
  const int tid = threadIdx.x;
  const int n0 = p * CB;
  const int nb = min(CB, m - n0);
  for (int e = tid; e < CB * CB; e += 256) {
    int i = e % CB, j = e / CB;
    double v = 0.0;
    if (i < nb && j < nb) v = (i >= j) ? G[(n0 + i) + (long)(n0 + j) * ld] : G[(n0 + j) + (long)(n0 + i) * ld];
    S[i + j * CLD] = v;
  }
  if (tid == 0) bad = 0;
  __syncthreads();
  for (int c = 0; c < nb; ++c) {
    double piv = S[c + c * CLD];
    double lcc = (piv > 0) ? sqrt(piv) : 1.0;
    if (!(piv > 0) && tid == 0) bad = 1;
    __syncthreads();
    for (int i = c + 1 + tid; i < nb; i += 256) S[i + c * CLD] /= lcc;
    if (tid == 0) S[c + c * CLD] = lcc;
    __syncthreads();
    int nr = nb - c - 1;
    for (int e = tid; e < nr * nr; e += 256) {
      int i = c + 1 + e % nr, j = c + 1 + e / nr;
      if (i >= j) S[i + j * CLD] -= S[i + c * CLD] * S[j + c * CLD];
    }
    __syncthreads();
  }
  // inverse of the lower-triangular tile, one thread per column
  if (tid < nb) {
    int y = tid;
    for (int x = 0; x < nb; ++x) I[x + y * CLD] = 0.0;
    for (int x = y; x < nb; ++x) {
      double s = (x == y) ? 1.0 : 0.0;
      for (int t = y; t < x; ++t) s -= S[x + t * CLD] * I[t + y * CLD];
      I[x + y * CLD] = s / S[x + x * CLD];
    }
  }
  __syncthreads();
  for (int e = tid; e < nb * nb; e += 256) {
    int i = e % nb, j = e / nb;
    long o = (n0 + i) + (long)(n0 + j) * ld;
    L[o] = (i >= j) ? S[i + j * CLD] : 0.0;
    Li[o] = (i >= j) ? I[i + j * CLD] : 0.0;
  }
  if (tid == 0 && bad && *flag == 0) *flag = p + 1;
}

// Tiles (i, j), p < j <= i: L_ip = G_ip Li_pp^T, G_ij -= L_ip L_jp^T.
// The diagonal tile (i, i) stores L_ip and zeroes the upper tile (p, i).
__global__ __launch_bounds__(256) void chol_trail_kernel(double* G, int ld, int m, int p, double* L,
                                                         const double* Li) {
  __shared__ double Lp[CB * CLD], Ai[CB * CLD], Aj[CB * CLD];
  const int nbk = (m + CB - 1) / CB;
  const int span = nbk - p - 1;
  const int i = p + 1 + blockIdx.x % span, j = p + 1 + blockIdx.x / span;
  if (j > i) return;
  const int tid = threadIdx.x;
  const int n0 = p * CB, ni0 = i * CB, nj0 = j * CB;
  const int nbp = min(CB, m - n0), nbi = min(CB, m - ni0), nbj = min(CB, m - nj0);
  for (int e = tid; e < CB * CB; e += 256) {
    int x = e % CB, y = e / CB;
    Lp[x + y * CLD] = (x < nbp && y < nbp) ? Li[(n0 + x) + (long)(n0 + y) * ld] : 0.0;
    Ai[x + y * CLD] = (x < nbi && y < nbp) ? G[(ni0 + x) + (long)(n0 + y) * ld] : 0.0;
    Aj[x + y * CLD] = (x < nbj && y < nbp) ? G[(nj0 + x) + (long)(n0 + y) * ld] : 0.0;
  }
  __syncthreads();
  // L_ip[x][y] = sum_t A_ip[x][t] Li_pp[y][t]   (register results, 4 per thread)
  double li[4], lj[4];
  for (int s = 0; s < 4; ++s) {
    int e = tid + 256 * s, x = e % CB, y = e / CB;
    double a1 = 0, a2 = 0;
    for (int t = 0; t <= y; ++t) {
      double lv = Lp[y + t * CLD];
      a1 += Ai[x + t * CLD] * lv;
      a2 += Aj[x + t * CLD] * lv;
    }
    li[s] = a1;
    lj[s] = a2;
  }
  __syncthreads();
  for (int s = 0; s < 4; ++s) {
    int e = tid + 256 * s, x = e % CB, y = e / CB;
    Ai[x + y * CLD] = li[s];
    Aj[x + y * CLD] = lj[s];
  }
  __syncthreads();
  for (int s = 0; s < 4; ++s) {
    int e = tid + 256 * s, x = e % CB, y = e / CB;
    if (x < nbi && y < nbj && (i != j || x >= y)) {
      double acc = 0;
      for (int t = 0; t < CB; ++t) acc += Ai[x + t * CLD] * Aj[y + t * CLD];
      G[(ni0 + x) + (long)(nj0 + y) * ld] -= acc;
    }
    if (i == j && x < nbi && y < nbp) {
      L[(ni0 + x) + (long)(n0 + y) * ld] = Ai[x + y * CLD];
      L[(n0 + y) + (long)(ni0 + x) * ld] = 0.0;
    }
  }
}

// Off-diagonal tiles of L^{-1} along block diagonal d:
// Li_ij = -Li_ii sum_{t=j}^{i-1} L_it Li_tj, with i = j + d; zeroes tile (j, i).
__global__ __launch_bounds__(256) void trinv_kernel(const double* L, double* Li, int ld, int m, int d) {
  __shared__ double A[CB * CLD], B[CB * CLD], S[CB * CLD];
  const int j = blockIdx.x, i = j + d;
  const int tid = threadIdx.x;
  const int ni0 = i * CB, nj0 = j * CB;
  const int nbi = min(CB, m - ni0), nbj = min(CB, m - nj0);
  double acc[4] = {0, 0, 0, 0};
  for (int t = j; t < i; ++t) {
    const int nt0 = t * CB, nbt = min(CB, m - nt0);
    __syncthreads();
    for (int e = tid; e < CB * CB; e += 256) {
      int x = e % CB, y = e / CB;
      A[x + y * CLD] = (x < nbi && y < nbt) ? L[(ni0 + x) + (long)(nt0 + y) * ld] : 0.0;
      B[x + y * CLD] = (x < nbt && y < nbj) ? Li[(nt0 + x) + (long)(nj0 + y) * ld] : 0.0;
    }
    __syncthreads();
    for (int s = 0; s < 4; ++s) {
      int e = tid + 256 * s, x = e % CB, y = e / CB;
      double a = 0;
      for (int u = 0; u < CB; ++u) a += A[x + u * CLD] * B[u + y * CLD];
      acc[s] += a;
    }
  }
  __syncthreads();
  for (int s = 0; s < 4; ++s) {
    int e = tid + 256 * s, x = e % CB, y = e / CB;
    S[x + y * CLD] = acc[s];
  }
  for (int e = tid; e < CB * CB; e += 256) {
    int x = e % CB, y = e / CB;
    A[x + y * CLD] = (x < nbi && y < nbi) ? Li[(ni0 + x) + (long)(ni0 + y) * ld] : 0.0;
  }
  __syncthreads();
  for (int s = 0; s < 4; ++s) {
    int e = tid + 256 * s, x = e % CB, y = e / CB;
    if (x < nbi && y < nbj) {
      double a = 0;
      for (int u = 0; u <= x; ++u) a += A[x + u * CLD] * S[u + y * CLD];
      Li[(ni0 + x) + (long)(nj0 + y) * ld] = -a;
      Li[(nj0 + y) + (long)(ni0 + x) * ld] = 0.0;
    }
  }
}

void chol_inverse(double* G, double* L, double* Linv, int m, int ld, int* flag, hipStream_t st) {
  const int nbk = (m + CB - 1) / CB;
  for (int p = 0; p < nbk; ++p) {
    hipLaunchKernelGGL(chol_diag_kernel, dim3(1), dim3(256), 0, st, G, ld, m, p, L, Linv, flag);
    int span = nbk - p - 1;
    if (span > 0) hipLaunchKernelGGL(chol_trail_kernel, dim3(span * span), dim3(256), 0, st, G, ld, m, p, L, Linv);
  }
  for (int d = 1; d < nbk; ++d)
    hipLaunchKernelGGL(trinv_kernel, dim3(nbk - d), dim3(256), 0, st, L, Linv, ld, m, d);
}

// ---------------------------------------------------------------------------
__global__ void transpose_kernel(const double* src, int lds, double* dst, int ldd, int m, int n) {
  __shared__ double t[32][33];
  int bx = blockIdx.x * 32, by = blockIdx.y * 32;
  int tx = threadIdx.x, ty = threadIdx.y;
  for (int k = ty; k < 32; k += 8) {
    int r = bx + tx, c = by + k;
    if (r < m && c < n) t[k][tx] = src[r + (long)c * lds];
  }
  __syncthreads();
  for (int k = ty; k < 32; k += 8) {
    int r = by + tx, c = bx + k;  // dst is n x m
    if (r < n && c < m) dst[r + (long)c * ldd] = t[tx][k];
  }
}
void launch_transpose(const double* src, int lds, double* dst, int ldd, int m, int n, hipStream_t st) {
  dim3 g((m + 31) / 32, (n + 31) / 32);
  hipLaunchKernelGGL(transpose_kernel, g, dim3(32, 8), 0, st, src, lds, dst, ldd, m, n);
}

__global__ void fill_kernel(double* p, long count, double v) {
  long e = blockIdx.x * 256L + threadIdx.x;
  if (e < count) p[e] = v;
}
void launch_fill(double* p, long count, double v, hipStream_t st) {
  if (count <= 0) return;
  hipLaunchKernelGGL(fill_kernel, dim3((count + 255) / 256), dim3(256), 0, st, p, count, v);
}

__global__ void set_diag_kernel(double* G, int ld, int m, const double* lam) {
  long e = blockIdx.x * 256L + threadIdx.x;
  if (e >= (long)m * m) return;
  int i = e % m, j = e / m;
  G[i + (long)j * ld] = (i == j) ? lam[i] : 0.0;
}
void launch_set_diag(double* G, int ld, int m, const double* lam, hipStream_t st) {
  long t = (long)m * m;
  if (t == 0) return;
  hipLaunchKernelGGL(set_diag_kernel, dim3((t + 255) / 256), dim3(256), 0, st, G, ld, m, lam);
}

__global__ void symmetrize_kernel(double* G, int ld, int m) {
  long e = blockIdx.x * 256L + threadIdx.x;
  if (e >= (long)m * m) return;
  int i = e % m, j = e / m;
  if (i < j) {
    double v = 0.5 * (G[i + (long)j * ld] + G[j + (long)i * ld]);
    G[i + (long)j * ld] = v;
    G[j + (long)i * ld] = v;
  }
}
void launch_symmetrize(double* G, int ld, int m, hipStream_t st) {
  long t = (long)m * m;
  if (t == 0) return;
  hipLaunchKernelGGL(symmetrize_kernel, dim3((t + 255) / 256), dim3(256), 0, st, G, ld, m);
}

// out[j] = sum_{i < nw} G[i, j]^2 for j < nw (one workgroup per column)
__global__ __launch_bounds__(256) void frob2_sub_kernel(const double* G, int ld, int nw, double* out) {
  const double* g = G + (long)blockIdx.x * ld;
  double s = 0;
  for (int i = threadIdx.x; i < nw; i += 256) s += g[i] * g[i];
  __shared__ double red[4];
  s = wave_sum(s);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = s;
  __syncthreads();
  if (threadIdx.x == 0) out[blockIdx.x] = (red[0] + red[1]) + (red[2] + red[3]);
}
void launch_frob2_sub(const double* G, int ld, int nw, double* out, hipStream_t st) {
  if (nw > 0) hipLaunchKernelGGL(frob2_sub_kernel, dim3(nw), dim3(256), 0, st, G, ld, nw, out);
}

__global__ __launch_bounds__(256) void orth_err2_kernel(const double* G, int ld, int k, double* out) {
  double s = 0;
  for (long e = threadIdx.x; e < (long)k * k; e += 256) {
    long i = e % k, j = e / k;
    double v = G[i + j * ld] - (i == j ? 1.0 : 0.0);
    s += v * v;
  }
  __shared__ double red[4];
  s = wave_sum(s);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = s;
  __syncthreads();
  if (threadIdx.x == 0) *out = (red[0] + red[1]) + (red[2] + red[3]);
}
void launch_orth_err2(const double* G, int ld, int k, double* out, hipStream_t st) {
  hipLaunchKernelGGL(orth_err2_kernel, dim3(1), dim3(256), 0, st, G, ld, k, out);
}

// ---------------------------------------------------------------------------
// block Jacobi
// ---------------------------------------------------------------------------
constexpr int JB = 16;           // block width
// Rotations are skipped once |M_pq| <= rel_tol |M|_F.  Off-diagonal entries
// of that size change the Ritz residual of a column by at most
// rel_tol |M|_F sqrt(K) (the caller keeps this far below its locking
// threshold) and the eigenvalues (Rayleigh quotients of the rotated
// columns) by O(off^2 / gap).
constexpr int J2 = 2 * JB;       // pair size
constexpr int JLD = J2 + 1;

struct JacobiWork {
  double* Q;       // npairs x J2 x J2
  int* flags;      // npairs
  int* counter;    // 1
  double* tiny;    // 1
  double* Vt;      // m x m (ld m) accumulated rotations
  int* rank;       // m
};

static JacobiWork carve(void* work, int m) {
  int nblk = (m + JB - 1) / JB;
  int np = (nblk + 1) / 2;
  char* p = (char*)work;
  JacobiWork w;
  w.Q = (double*)p; p += sizeof(double) * np * J2 * J2;
  w.Vt = (double*)p; p += sizeof(double) * (size_t)m * m;
  w.tiny = (double*)p; p += 256;
  w.flags = (int*)p; p += sizeof(int) * ((np + 63) / 64 * 64);
  w.counter = (int*)p; p += 256;
  w.rank = (int*)p;
  return w;
}
size_t eig_workspace_bytes(int m) {
  int nblk = (m + JB - 1) / JB;
  int np = (nblk + 1) / 2;
  return sizeof(double) * (size_t)np * J2 * J2 + sizeof(double) * (size_t)m * m + 256 +
         sizeof(int) * ((np + 63) / 64 * 64) + 256 + sizeof(int) * (size_t)m + 256;
}

PPCG_DEV int pair_block(int t, int round, int nbe) { return rr_player(t, round, nbe); }

__global__ __launch_bounds__(256) void bj_norm_kernel(const double* M, int ld, int m, double* tiny, int* counter,
                                                      double rel_tol) {
  double s = 0;
  for (long e = threadIdx.x; e < (long)m * m; e += 256) {
    double v = M[(e % m) + (e / m) * ld];
    s += v * v;
  }
  __shared__ double red[4];
  s = wave_sum(s);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = s;
  __syncthreads();
  if (threadIdx.x == 0) {
    *tiny = rel_tol * sqrt((red[0] + red[1]) + (red[2] + red[3]));
    *counter = 0;
  }
}

__global__ void bj_zero_kernel(int* counter) { *counter = 0; }

__global__ __launch_bounds__(256) void bj_pair_kernel(double* M, int ld, int m, int nbe, int round, double* Qbuf,
                                                      int* flags, int* counter, const double* tinyp) {
  __shared__ double S[J2 * JLD], Q[J2 * JLD];
  __shared__ double cs[J2 + 2];
  __shared__ int pq[J2 + 2], cnt, any;
  const int tid = threadIdx.x, t = blockIdx.x;
  const int nblk = (m + JB - 1) / JB;
  int I = pair_block(t, round, nbe), J = pair_block(nbe - 1 - t, round, nbe);
  if (I > J) { int x = I; I = J; J = x; }
  const int i0 = I * JB, j0 = J * JB;
  const int nI = I < nblk ? min(JB, m - i0) : 0;
  const int nJ = J < nblk ? min(JB, m - j0) : 0;
  const int n2 = nI + nJ;
  auto gidx = [&](int a) { return a < nI ? i0 + a : j0 + (a - nI); };
  const double tiny = *tinyp;
  if (tid == 0) any = 0;
  __syncthreads();
  for (int e = tid; e < n2 * n2; e += 256) {
    int x = e % n2, y = e / n2;
    double v = M[gidx(x) + (long)gidx(y) * ld];
    S[x + y * JLD] = v;
    if (x != y && fabs(v) > tiny) any = 1;
  }
  __syncthreads();
  if (!any) {
    if (tid == 0) flags[t] = 0;
    return;
  }
  lds_jacobi<256>(S, Q, n2, JLD, tiny, 40, cs, pq, &cnt);
  double* Qg = Qbuf + (long)t * J2 * J2;
  for (int e = tid; e < n2 * n2; e += 256) Qg[(e % n2) + (e / n2) * J2] = Q[(e % n2) + (e / n2) * JLD];
  if (tid == 0) {
    flags[t] = 1;
    atomicAdd(counter, 1);
  }
}

// rows of each rotated pair: M[rows, chunk] <- Q^T M[rows, chunk], 64 columns per workgroup
__global__ __launch_bounds__(256) void bj_row_kernel(double* M, int ld, int m, int nbe, int round, const double* Qbuf,
                                                     const int* flags) {
  __shared__ double Q[J2 * JLD], R[J2 * 65];
  const int t = blockIdx.x;
  if (!flags[t]) return;
  const int tid = threadIdx.x;
  const int nblk = (m + JB - 1) / JB;
  int I = pair_block(t, round, nbe), J = pair_block(nbe - 1 - t, round, nbe);
  if (I > J) { int x = I; I = J; J = x; }
  const int i0 = I * JB, j0 = J * JB;
  const int nI = I < nblk ? min(JB, m - i0) : 0;
  const int nJ = J < nblk ? min(JB, m - j0) : 0;
  const int n2 = nI + nJ;
  auto gidx = [&](int a) { return a < nI ? i0 + a : j0 + (a - nI); };
  const double* Qg = Qbuf + (long)t * J2 * J2;
  for (int e = tid; e < n2 * n2; e += 256) Q[(e % n2) + (e / n2) * JLD] = Qg[(e % n2) + (e / n2) * J2];
  const int c0 = blockIdx.y * 64;
  const int nc = min(64, m - c0);
  for (int e = tid; e < n2 * nc; e += 256) {
    int x = e % n2, c = e / n2;
    R[x + c * J2] = M[gidx(x) + (long)(c0 + c) * ld];
  }
  __syncthreads();
  for (int e = tid; e < n2 * nc; e += 256) {
    int x = e % n2, c = e / n2;
    double s = 0;
    for (int u = 0; u < n2; ++u) s += Q[u + x * JLD] * R[u + c * J2];
    M[gidx(x) + (long)(c0 + c) * ld] = s;
  }
}

__global__ __launch_bounds__(256) void bj_col_kernel(double* M, int ld, double* V, int ldv, int m, int nbe,
                                                     int round, const double* Qbuf, const int* flags) {
  __shared__ double Q[J2 * JLD], R[64 * (J2 + 1)];
  const int t = blockIdx.x;
  if (!flags[t]) return;
  const int tid = threadIdx.x;
  const int nblk = (m + JB - 1) / JB;
  int I = pair_block(t, round, nbe), J = pair_block(nbe - 1 - t, round, nbe);
  if (I > J) { int x = I; I = J; J = x; }
  const int i0 = I * JB, j0 = J * JB;
  const int nI = I < nblk ? min(JB, m - i0) : 0;
  const int nJ = J < nblk ? min(JB, m - j0) : 0;
  const int n2 = nI + nJ;
  auto gidx = [&](int a) { return a < nI ? i0 + a : j0 + (a - nI); };
  const double* Qg = Qbuf + (long)t * J2 * J2;
  for (int e = tid; e < n2 * n2; e += 256) Q[(e % n2) + (e / n2) * JLD] = Qg[(e % n2) + (e / n2) * J2];
  const int r0 = blockIdx.y * 64;
  const int nr = min(64, m - r0);
  constexpr int RLD = J2 + 1;
  for (int which = 0; which < 2; ++which) {
    double* A = which ? V : M;
    const int lda = which ? ldv : ld;
    __syncthreads();
    for (int e = tid; e < nr * n2; e += 256) {
      int r = e % nr, x = e / nr;
      R[x + r * RLD] = A[(r0 + r) + (long)gidx(x) * lda];
    }
    __syncthreads();
    for (int e = tid; e < nr * n2; e += 256) {
      int r = e % nr, x = e / nr;
      double s = 0;
      for (int u = 0; u < n2; ++u) s += R[u + r * RLD] * Q[u + x * JLD];
      A[(r0 + r) + (long)gidx(x) * lda] = s;
    }
  }
}

__global__ __launch_bounds__(1024) void bj_rank_kernel(const double* M, int ld, int m, double* lam, int* rank) {
  for (int x = threadIdx.x; x < m; x += 1024) {
    double lx = M[x + (long)x * ld];
    int rk = 0;
    for (int y = 0; y < m; ++y) {
      double ly = M[y + (long)y * ld];
      rk += (ly < lx) || (ly == lx && y < x);
    }
    rank[x] = rk;
    lam[rk] = lx;
  }
}

__global__ void bj_gather_kernel(const double* Vt, int m, const int* rank, double* V, int ldv) {
  long e = blockIdx.x * 256L + threadIdx.x;
  if (e >= (long)m * m) return;
  int i = e % m, j = e / m;
  V[i + (long)rank[j] * ldv] = Vt[i + (long)j * m];
}

__global__ void identity_kernel(double* V, int m) {
  long e = blockIdx.x * 256L + threadIdx.x;
  if (e >= (long)m * m) return;
  V[e] = ((e % m) == (e / m)) ? 1.0 : 0.0;
}

int block_jacobi_eig(double* M, int ld, int m, double* V, int ldv, double* lam, void* work, int* hostbuf,
                     double rel_tol, hipStream_t st) {
  JacobiWork w = carve(work, m);
  const int nblk = (m + JB - 1) / JB;
  const int nbe = nblk + (nblk & 1);
  const int np = nbe / 2;
  long mm = (long)m * m;
  hipLaunchKernelGGL(identity_kernel, dim3((mm + 255) / 256), dim3(256), 0, st, w.Vt, m);
  hipLaunchKernelGGL(bj_norm_kernel, dim3(1), dim3(256), 0, st, M, ld, m, w.tiny, w.counter, rel_tol);
  int sweeps = 0;
  const int rounds = nbe > 1 ? nbe - 1 : 1;
  for (int sweep = 0; sweep < 40; ++sweep) {
    hipLaunchKernelGGL(bj_zero_kernel, dim3(1), dim3(1), 0, st, w.counter);
    for (int round = 0; round < rounds; ++round) {
      hipLaunchKernelGGL(bj_pair_kernel, dim3(np), dim3(256), 0, st, M, ld, m, nbe, round, w.Q, w.flags, w.counter,
                         w.tiny);
      hipLaunchKernelGGL(bj_row_kernel, dim3(np, (m + 63) / 64), dim3(256), 0, st, M, ld, m, nbe, round, w.Q,
                         w.flags);
      hipLaunchKernelGGL(bj_col_kernel, dim3(np, (m + 63) / 64), dim3(256), 0, st, M, ld, w.Vt, m, m, nbe, round,
                         w.Q, w.flags);
    }
    ++sweeps;
    hipMemcpyAsync(hostbuf, w.counter, sizeof(int), hipMemcpyDeviceToHost, st);
    hipStreamSynchronize(st);
    if (*hostbuf == 0) break;
  }
  hipLaunchKernelGGL(bj_rank_kernel, dim3(1), dim3(1024), 0, st, M, ld, m, lam, w.rank);
  hipLaunchKernelGGL(bj_gather_kernel, dim3((mm + 255) / 256), dim3(256), 0, st, w.Vt, m, w.rank, V, ldv);
  return sweeps;
}

}  // namespace ppcg
