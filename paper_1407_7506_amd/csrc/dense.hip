// Dense m x m kernels (column-major, ld >= m):
//   chol_inverse      G = L L^H and L^{-1}, blocked (32 x 32 tiles), for
//                     Cholesky-QR (section 5.5) and the Rayleigh-Ritz
//                     reduction to a standard problem (section 5.6)
//   block_jacobi_eig  Hermitian eigen-decomposition of the reduced
//                     Rayleigh-Ritz matrix by block Jacobi: pairs of 16-wide
//                     diagonal blocks are diagonalised in LDS, their
//                     rotations applied to the block rows, then to the block
//                     columns and the eigenvector accumulator
//   misc              fills, transposes, diagonal set, Frobenius norms, copies
// Both composite routines take a list of independent problems and advance
// them in lockstep, one grouped launch per step.
#include <algorithm>

#include <stdexcept>
#include <type_traits>

#include "common.hpp"
#include "jacobi.hpp"
#include "kernels.hpp"

namespace ppcg {

thread_local Recorder* g_rec = nullptr;

// ---------------------------------------------------------------------------
// staging of job arrays
// ---------------------------------------------------------------------------
Stage::~Stage() {
  for (auto* v : {&chunks, &retired})
    for (auto& c : *v) {
      hipHostFree(c.h);
      hipFree(c.d);
    }
}
void* Stage::upload(const void* src, size_t bytes, hipStream_t st) {
  size_t need = (bytes + 255) / 256 * 256;
  if (chunks.empty() || chunks.back().used + need > chunks.back().cap) {
    size_t cap = std::max<size_t>(need, 1 << 20);
    Chunk c{nullptr, nullptr, cap, 0};
    if (hipHostMalloc((void**)&c.h, cap, hipHostMallocDefault) != hipSuccess) throw std::bad_alloc();
    if (hipMalloc((void**)&c.d, cap) != hipSuccess) {
      hipHostFree(c.h);
      throw std::bad_alloc();
    }
    if (!chunks.empty()) {  // keep the full chunk alive until reset
      retired.push_back(chunks.back());
      chunks.pop_back();
    }
    chunks.push_back(c);
  }
  Chunk& c = chunks.back();
  std::memcpy(c.h + c.used, src, bytes);
  void* d = c.d + c.used;
  hipMemcpyAsync(d, c.h + c.used, bytes, hipMemcpyHostToDevice, st);
  c.used += need;
  return d;
}
void Stage::reset() {
  for (auto& c : retired) {
    hipHostFree(c.h);
    hipFree(c.d);
  }
  retired.clear();
  for (auto& c : chunks) c.used = 0;
}

// ---------------------------------------------------------------------------
// blocked Cholesky and inverse
//
// G = L L^H (lower, 32 x 32 tiles) and L^{-1}, in P + 1 launches for P tile
// columns.  Launch 0 factors the first diagonal tile.  Launch p + 1 (p =
// 0..P-1) runs, side by side:
//   trailing tiles (i, j), p < j <= i:  G_ij -= L_ip L_jp^H with
//       L_ip = G_ip Li_pp^H recomputed by the workgroup; the workgroup of
//       tile (p+1, p+1) then factors it (the next diagonal step);
//   inverse rows: with W_ic = delta_ic I - sum_{k<p} L_ik Li_kc (kept in the
//       L buffer for i > c), block row p of the inverse is final,
//       Li_pc = Li_pp W_pc (c < p), and every row below takes the step's
//       term, W_ic -= L_ip (Li_pp W_pc) (c <= p; W_pp = I).
// Block forward substitution of L Li = I in right-looking order: every
// launch is one layer of independent 32 x 32 tile products, so the inverse
// costs no launches of its own.
// ---------------------------------------------------------------------------
constexpr int CB = 32;       // Cholesky tile
constexpr int CLD = CB + 1;

struct DenseStep { double* G; double* W; double* Li; int ld, m; int* flag; };

// LDS tile <- 32 x 32 block of M at (r0, c0), zero outside nr x nc
template <class S>
PPCG_DEV void tile_get(S* T, const S* M, long ld, int r0, int c0, int nr, int nc) {
  const S zero = from_real<S>(0.0);
  for (int e = threadIdx.x; e < CB * CB; e += 256) {
    int x = e % CB, y = e / CB;
    T[x + y * CLD] = (x < nr && y < nc) ? M[(r0 + x) + (long)(c0 + y) * ld] : zero;
  }
}
// C = A op(B) for the 4 entries of this thread (op = identity or ^H)
template <class S, bool BH>
PPCG_DEV void tile_mul4(S (&c)[4], const S* A, const S* B) {
  const S zero = from_real<S>(0.0);
#pragma unroll
  for (int s = 0; s < 4; ++s) {
    int e = threadIdx.x + 256 * s, x = e % CB, y = e / CB;
    S v = zero;
    for (int t = 0; t < CB; ++t) v += A[x + t * CLD] * (BH ? conj_(B[y + t * CLD]) : B[t + y * CLD]);
    c[s] = v;
  }
}
template <class S>
PPCG_DEV void tile_put4(S* T, const S (&c)[4]) {
#pragma unroll
  for (int s = 0; s < 4; ++s) {
    int e = threadIdx.x + 256 * s;
    T[(e % CB) + (e / CB) * CLD] = c[s];
  }
}

// Float64 32 x 32 tile product on the matrix cores: each of the four waves
// forms one 16 x 16 quadrant of A op(B) (op = identity, or transpose when BH)
// from LDS tiles (ld CLD) in 8 MFMA steps; acc value v of lane l is entry
// (16 qx + 4 v + l/16, 16 qy + l%16).
template <bool BH>
PPCG_DEV d4v tile_mfma(const double* A, const double* B) {
  const int l = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int qx = w & 1, qy = w >> 1, lc = l & 15, g = l >> 4;
  d4v acc = {0, 0, 0, 0};
#pragma unroll
  for (int t0 = 0; t0 < CB; t0 += 4) {
    const double av = A[(16 * qx + lc) + (t0 + g) * CLD];
    const double bv = BH ? B[(16 * qy + lc) + (t0 + g) * CLD] : B[(t0 + g) + (16 * qy + lc) * CLD];
    acc = mfma(av, bv, acc);
  }
  return acc;
}
template <class S>
PPCG_DEV void acc_put(S* T, const d4v& acc) {
  const int l = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int qx = w & 1, qy = w >> 1;
#pragma unroll
  for (int v = 0; v < 4; ++v) T[(16 * qx + 4 * v + (l >> 4)) + (16 * qy + (l & 15)) * CLD] = acc[v];
}

// factor the diagonal tile p of G (already updated by every earlier step):
// Li_pp = L_pp^{-1}; a non-positive pivot sets *flag = p + 1.  The inverse is
// formed inside the factorization loop by forward substitution in column
// (axpy) order: once column c of L is scaled, row c of the inverse takes its
// 1 / L_cc and every row below subtracts L_xc times it.  Each entry of the
// inverse receives the same operations in the same order as row-by-row
// substitution, with no barriers beyond the factorization's own.
template <class S>
PPCG_DEV void chol_diag_body(const DenseStep& a, int p) {
  __shared__ S Sm[CB * CLD], I[CB * CLD];
  __shared__ int bad;
  const S* G = (const S*)a.G;
  S* Li = (S*)a.Li;
  const S zero = from_real<S>(0.0);
  const int tid = threadIdx.x;
  const int n0 = p * CB;
  const int nb = min(CB, a.m - n0);
  for (int e = tid; e < CB * CB; e += 256) {
    int i = e % CB, j = e / CB;
    S v = zero;
    if (i < nb && j < nb) v = (i >= j) ? G[(n0 + i) + (long)(n0 + j) * a.ld] : conj_(G[(n0 + j) + (long)(n0 + i) * a.ld]);
    Sm[i + j * CLD] = v;
    I[i + j * CLD] = from_real<S>(i == j && i < nb ? 1.0 : 0.0);
  }
  if (tid == 0) bad = 0;
  __syncthreads();
  for (int c = 0; c < nb; ++c) {
    double piv = real_(Sm[c + c * CLD]);
    double lcc = (piv > 0) ? sqrt(piv) : 1.0;
    if (!(piv > 0) && tid == 0) bad = 1;
    __syncthreads();
    const double rl = 1.0 / lcc;
    for (int i = c + 1 + tid; i < nb; i += 256) Sm[i + c * CLD] = rl * Sm[i + c * CLD];
    if (tid == 0) Sm[c + c * CLD] = from_real<S>(lcc);
    if (tid <= c) I[c + tid * CLD] = rl * I[c + tid * CLD];  // row c of the inverse is final
    __syncthreads();
    int nr = nb - c - 1;
    for (int e = tid; e < nr * nr; e += 256) {
      int i = c + 1 + e % nr, j = c + 1 + e / nr;
      if (i >= j) Sm[i + j * CLD] -= Sm[i + c * CLD] * conj_(Sm[j + c * CLD]);
    }
    for (int e = tid; e < nr * (c + 1); e += 256) {  // rows x > c, columns y <= c
      int x = c + 1 + e % nr, y = e / nr;
      I[x + y * CLD] -= Sm[x + c * CLD] * I[c + y * CLD];
    }
    __syncthreads();
  }
  for (int e = tid; e < nb * nb; e += 256) {
    int i = e % nb, j = e / nb;
    Li[(n0 + i) + (long)(n0 + j) * a.ld] = (i >= j) ? I[i + j * CLD] : zero;
  }
  if (tid == 0 && bad && *a.flag == 0) *a.flag = p + 1;
}

// one workgroup item of launch p + 1 (see above)
template <class S>
PPCG_DEV void chol_step_body(const DenseStep& a, int p, unsigned wg) {
  __shared__ S T0[CB * CLD], T1[CB * CLD], T2[CB * CLD];
  constexpr bool MF = std::is_same<S, double>::value;  // float64: tile products on the matrix cores
  __shared__ S T3[MF ? CB * CLD : 1], T4[MF ? CB * CLD : 1];
  const int ml = threadIdx.x & 63, mw = threadIdx.x >> 6;
  const int mx0 = 16 * (mw & 1) + 4 * 0 + (ml >> 4), my = 16 * (mw >> 1) + (ml & 15);  // acc value v: row mx0 + 4 v
  S* G = (S*)a.G;
  S* W = (S*)a.W;
  S* Li = (S*)a.Li;
  const int m = a.m, ld = a.ld;
  const int nbk = (m + CB - 1) / CB;
  if (p >= nbk) return;
  const int span = nbk - p - 1;
  const int n0 = p * CB, nbp = min(CB, m - n0);
  auto nb_of = [&](int t) { return min(CB, m - t * CB); };
  S c[4];
  unsigned it = wg;
  if (it < (unsigned)(span * span)) {  // trailing tile (i, j)
    const int i = p + 1 + (int)(it % span), j = p + 1 + (int)(it / span);
    if (j > i) return;
    const int nbi = nb_of(i), nbj = nb_of(j);
    tile_get(T0, Li, ld, n0, n0, nbp, nbp);          // Li_pp
    tile_get(T1, G, ld, i * CB, n0, nbi, nbp);       // G_ip
    tile_get(T2, G, ld, j * CB, n0, nbj, nbp);       // G_jp
    __syncthreads();
    if constexpr (MF) {
      acc_put(T3, tile_mfma<true>(T1, T0));          // L_ip = G_ip Li_pp^T
      acc_put(T4, tile_mfma<true>(T2, T0));          // L_jp
      __syncthreads();
      const d4v r = tile_mfma<true>(T3, T4);         // L_ip L_jp^T
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int x = mx0 + 4 * v, y = my;
        if (x < nbi && y < nbj && (i != j || x >= y)) G[(i * CB + x) + (long)(j * CB + y) * ld] -= r[v];
      }
    } else {
      S d[4];
      tile_mul4<S, true>(c, T1, T0);                 // L_ip = G_ip Li_pp^H
      tile_mul4<S, true>(d, T2, T0);                 // L_jp
      __syncthreads();
      tile_put4(T1, c);
      tile_put4(T2, d);
      __syncthreads();
      tile_mul4<S, true>(c, T1, T2);                 // L_ip L_jp^H
#pragma unroll
      for (int s = 0; s < 4; ++s) {
        int e = threadIdx.x + 256 * s, x = e % CB, y = e / CB;
        if (x < nbi && y < nbj && (i != j || x >= y)) G[(i * CB + x) + (long)(j * CB + y) * ld] -= c[s];
      }
    }
    if (i == j && i == p + 1) {  // the next diagonal step, on the tile just updated
      __syncthreads();
      chol_diag_body<S>(a, p + 1);
    }
    return;
  }
  it -= span * span;
  if (it < (unsigned)p) {  // row p of the inverse: Li_pc = Li_pp W_pc, c < p
    const int cc = (int)it, nbc = nb_of(cc);
    tile_get(T0, Li, ld, n0, n0, nbp, nbp);
    tile_get(T1, W, ld, n0, cc * CB, nbp, nbc);
    __syncthreads();
    if constexpr (MF) {
      const d4v r = tile_mfma<false>(T0, T1);
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int x = mx0 + 4 * v, y = my;
        if (x < nbp && y < nbc) Li[(n0 + x) + (long)(cc * CB + y) * ld] = r[v];
      }
    } else {
      tile_mul4<S, false>(c, T0, T1);
#pragma unroll
      for (int s = 0; s < 4; ++s) {
        int e = threadIdx.x + 256 * s, x = e % CB, y = e / CB;
        if (x < nbp && y < nbc) Li[(n0 + x) + (long)(cc * CB + y) * ld] = c[s];
      }
    }
    return;
  }
  it -= p;
  if (it < (unsigned)(span * (p + 1))) {  // W_ic -= L_ip (Li_pp W_pc), i > p, c <= p
    const int i = p + 1 + (int)(it / (p + 1)), cc = (int)(it % (p + 1));
    const int nbi = nb_of(i), nbc = nb_of(cc);
    tile_get(T0, Li, ld, n0, n0, nbp, nbp);          // Li_pp
    tile_get(T1, G, ld, i * CB, n0, nbi, nbp);       // G_ip
    if (cc < p) tile_get(T2, W, ld, n0, cc * CB, nbp, nbc);
    __syncthreads();
    if constexpr (MF) {
      acc_put(T3, tile_mfma<true>(T1, T0));          // L_ip
      if (cc < p) acc_put(T4, tile_mfma<false>(T0, T2));  // Li_pp W_pc
      __syncthreads();
      const d4v r = tile_mfma<false>(T3, cc < p ? T4 : T0);  // L_ip (Li_pp W_pc); W_pp = I
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int x = mx0 + 4 * v, y = my;
        if (x < nbi && y < nbc) {
          S* w = W + (i * CB + x) + (long)(cc * CB + y) * ld;
          *w = (cc < p) ? *w - r[v] : -r[v];
        }
      }
    } else {
      S d[4];
      tile_mul4<S, true>(c, T1, T0);                 // L_ip
      if (cc < p) tile_mul4<S, false>(d, T0, T2);    // Li_pp W_pc
      __syncthreads();
      tile_put4(T1, c);
      if (cc < p) tile_put4(T2, d);
      __syncthreads();
      tile_mul4<S, false>(c, T1, cc < p ? T2 : T0);  // L_ip (Li_pp W_pc); W_pp = I
#pragma unroll
      for (int s = 0; s < 4; ++s) {
        int e = threadIdx.x + 256 * s, x = e % CB, y = e / CB;
        if (x < nbi && y < nbc) {
          S* w = W + (i * CB + x) + (long)(cc * CB + y) * ld;
          *w = (cc < p) ? *w - c[s] : -c[s];
        }
      }
    }
  }
}

// launch 0: the first diagonal tile; launch p + 1: chol_step_body(p)
template <class S>
__global__ __launch_bounds__(256) void chol_step_grouped(const DenseStep* jobs, const unsigned* start, int nj,
                                                         int launch) {
  int j = find_job(start, nj, blockIdx.x);
  unsigned wg = blockIdx.x - start[j];
  if (launch == 0) chol_diag_body<S>(jobs[j], 0);
  else chol_step_body<S>(jobs[j], launch - 1, wg);
}

void chol_inverse_grouped(const std::vector<CholArgs>& jobs, Stage& stage, hipStream_t st) {
  const int nj = (int)jobs.size();
  if (nj == 0) return;
  const bool cplx = jobs[0].cplx;
  std::vector<DenseStep> ds(nj);
  int P = 0;
  for (int j = 0; j < nj; ++j) {
    ds[j] = DenseStep{jobs[j].G, jobs[j].L, jobs[j].Li, jobs[j].ld, jobs[j].m, jobs[j].flag};
    P = std::max(P, (jobs[j].m + CB - 1) / CB);
  }
  // workgroups of every launch and job, packed with the job array into one upload
  std::vector<unsigned> tots;
  std::vector<size_t> offs;
  std::vector<unsigned> starts;
  for (int l = 0; l <= P; ++l) {
    offs.push_back(starts.size());
    unsigned t = 0;
    for (int j = 0; j < nj; ++j) {
      starts.push_back(t);
      const int nbk = (jobs[j].m + CB - 1) / CB;
      if (l == 0) {
        t += nbk > 0 ? 1 : 0;
      } else {
        const int p = l - 1;
        if (p < nbk) {
          const int span = nbk - p - 1;
          t += (unsigned)(span * span + p + span * (p + 1));
        }
      }
    }
    starts.push_back(t);
    tots.push_back(t);
  }
  size_t jb = sizeof(DenseStep) * nj;
  std::vector<uint8_t> buf(jb + sizeof(unsigned) * starts.size());
  std::memcpy(buf.data(), ds.data(), jb);
  std::memcpy(buf.data() + jb, starts.data(), sizeof(unsigned) * starts.size());
  uint8_t* dev = (uint8_t*)stage.upload(buf.data(), buf.size(), st);
  const DenseStep* dj = (const DenseStep*)dev;
  const unsigned* sd = (const unsigned*)(dev + jb);
  for (int l = 0; l <= P; ++l) {
    if (!tots[l]) continue;
    if (cplx) hipLaunchKernelGGL(chol_step_grouped<zdouble>, dim3(tots[l]), dim3(256), 0, st, dj, sd + offs[l], nj, l);
    else hipLaunchKernelGGL(chol_step_grouped<double>, dim3(tots[l]), dim3(256), 0, st, dj, sd + offs[l], nj, l);
  }
}

// ---------------------------------------------------------------------------
// small element-wise kernels (direct and grouped)
// ---------------------------------------------------------------------------
PPCG_DEV void transpose_body(const TransposeArgs& a, unsigned wg, unsigned) {
  __shared__ double t[32][33], ti[32][33];
  const unsigned gx = (a.m + 31) / 32;
  const int nc = a.cplx ? 2 : 1;
  int bx = (wg % gx) * 32, by = (wg / gx) * 32;
  int tx = threadIdx.x % 32, ty = threadIdx.x / 32;
  for (int k = ty; k < 32; k += 8) {
    int r = bx + tx, c = by + k;
    if (r < a.m && c < a.n) {
      long o = (r + (long)c * a.lds) * nc;
      t[k][tx] = a.src[o];
      if (a.cplx) ti[k][tx] = -a.src[o + 1];
    }
  }
  __syncthreads();
  for (int k = ty; k < 32; k += 8) {
    int r = by + tx, c = bx + k;  // dst is n x m
    if (r < a.n && c < a.m) {
      long o = (r + (long)c * a.ldd) * nc;
      a.dst[o] = t[tx][k];
      if (a.cplx) a.dst[o + 1] = ti[tx][k];
    }
  }
}
PPCG_DEV void fill_body(const FillArgs& a, unsigned wg, unsigned) {
  long e = wg * 256L + threadIdx.x;
  if (e < a.count) a.p[e] = a.v;
}
PPCG_DEV void set_diag_body(const SetDiagArgs& a, unsigned wg, unsigned) {
  long e = wg * 256L + threadIdx.x;
  if (e >= (long)a.m * a.m) return;
  int i = e % a.m, j = e / a.m;
  const int nc = a.cplx ? 2 : 1;
  long o = (i + (long)j * a.ld) * nc;
  a.G[o] = (i == j) ? a.lam[i] : 0.0;
  if (a.cplx) a.G[o + 1] = 0.0;
}
PPCG_DEV void offdiag_body(const OffdiagArgs& a, unsigned wg, unsigned) {
  long e = wg * 256L + threadIdx.x;
  if (e >= (long)a.m * a.m) return;
  int i = e % a.m, j = e / a.m;
  const int nc = a.cplx ? 2 : 1;
  const long f = (i + (long)j * a.ldf) * nc, g = (i + (long)j * a.ldg) * nc;
  for (int c = 0; c < nc; ++c) a.F[f + c] = i == j ? 0.0f : (float)a.G[g + c];
}
PPCG_DEV void symm_body(const SymmArgs& a, unsigned wg, unsigned) {
  long e = wg * 256L + threadIdx.x;
  if (e >= (long)a.m * a.m) return;
  int i = e % a.m, j = e / a.m;
  const int nc = a.cplx ? 2 : 1;
  long u = (i + (long)j * a.ld) * nc, l = (j + (long)i * a.ld) * nc;
  if (i < j) {
    double v = 0.5 * (a.G[u] + a.G[l]);
    a.G[u] = v;
    a.G[l] = v;
    if (a.cplx) {
      double w = 0.5 * (a.G[u + 1] - a.G[l + 1]);
      a.G[u + 1] = w;
      a.G[l + 1] = -w;
    }
  } else if (i == j && a.cplx) {
    a.G[u + 1] = 0.0;
  }
}
// out[j] = sum_{i < nw} G[i, j]^2 for j < nw (one workgroup per column)
PPCG_DEV void frob2_body(const Frob2Args& a, unsigned wg, unsigned) {
  const int nc = a.cplx ? 2 : 1;
  const double* g = a.G + (long)wg * a.ld * nc;
  double s = 0;
  for (int i = threadIdx.x; i < a.nw * nc; i += 256) s += g[i] * g[i];
  __shared__ double red[4];
  s = wave_sum(s);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = s;
  __syncthreads();
  if (threadIdx.x == 0) a.out[wg] = (red[0] + red[1]) + (red[2] + red[3]);
}
PPCG_DEV void orth_body(const OrthArgs& a, unsigned, unsigned) {
  double s = 0;
  const int nc = a.cplx ? 2 : 1;
  for (long e = threadIdx.x; e < (long)a.k * a.k; e += 256) {
    long i = e % a.k, j = e / a.k;
    if (a.upper && i > j) continue;
    long o = (i + j * a.ld) * nc;
    double v = a.G[o] - (i == j ? 1.0 : 0.0);
    double t = v * v;
    if (a.cplx) t += a.G[o + 1] * a.G[o + 1];
    s += (a.upper && i < j) ? 2.0 * t : t;  // a Hermitian G: the lower triangle mirrors the upper
  }
  __shared__ double red[4];
  s = wave_sum(s);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = s;
  __syncthreads();
  if (threadIdx.x == 0) *a.out = (red[0] + red[1]) + (red[2] + red[3]);
}
PPCG_DEV void polar_body(const PolarArgs& a, unsigned wg, unsigned) {
  long e = wg * 256L + threadIdx.x;
  if (e >= (long)a.m * a.m) return;
  const int i = e % a.m, j = e / a.m;
  const int nc = a.cplx ? 2 : 1;
  const bool up = i <= j;
  const long src = (up ? i + (long)j * a.ld : j + (long)i * a.ld) * nc;  // Hermitian: lower = conj(upper)
  const long o = (i + (long)j * a.ld) * nc;
  const double yr = a.G[src] - (i == j ? 1.0 : 0.0);
  a.Y[o] = yr;
  a.M[o] = (i == j ? 0.375 : 0.0) - 0.3125 * yr;
  if (a.cplx) {
    const double yi = i == j ? 0.0 : (up ? a.G[src + 1] : -a.G[src + 1]);
    a.Y[o + 1] = yi;
    a.M[o + 1] = -0.3125 * yi;
  }
}
PPCG_DEV void add_diag_body(const AddDiagArgs& a, unsigned wg, unsigned) {
  int i = wg * 256 + threadIdx.x;
  if (i < a.m) a.G[(i + (long)i * a.ld) * (a.cplx ? 2 : 1)] += a.v;
}
PPCG_DEV void trace_body(const TraceArgs& a, unsigned, unsigned) {
  double s = 0;
  for (int i = threadIdx.x; i < a.m; i += 256) s += a.G[(i + (long)i * a.ld) * (a.cplx ? 2 : 1)];
  __shared__ double red[4];
  s = wave_sum(s);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = s;
  __syncthreads();
  if (threadIdx.x == 0) *a.out = (red[0] + red[1]) + (red[2] + red[3]);
}
PPCG_DEV void to_f32_body(const ToF32Args& a, unsigned wg, unsigned) {
  const int nc = a.cplx ? 2 : 1;
  const long per = a.rows * nc;
  const long e = wg * 256L + threadIdx.x;
  if (e >= per * a.ncols) return;
  const long c = e / per, r = e % per;
  a.Y[r + c * a.ld * nc] = (float)a.X[r + c * a.ld * nc];
}
PPCG_DEV void zero_int_body(const ZeroIntArgs& a, unsigned wg, unsigned) {
  int e = wg * 256 + threadIdx.x;
  if (e < a.n) a.p[e] = 0;
}
PPCG_DEV void copy_body(const CopyArgs& a, unsigned wg, unsigned) {
  long e = wg * 256L + threadIdx.x;
  if (e < a.count) a.dst[e] = a.src[e];
}

#define PPCG_SIMPLE(NAME, ARGS)                                                                          \
  __global__ __launch_bounds__(256) void NAME##_kernel(ARGS a) { NAME##_body(a, blockIdx.x, gridDim.x); } \
  __global__ __launch_bounds__(256) void NAME##_grouped(const ARGS* jobs, const unsigned* start, int nj) { \
    int j = find_job(start, nj, blockIdx.x);                                                              \
    NAME##_body(jobs[j], blockIdx.x - start[j], start[j + 1] - start[j]);                                 \
  }
PPCG_SIMPLE(transpose, TransposeArgs)
PPCG_SIMPLE(fill, FillArgs)
PPCG_SIMPLE(set_diag, SetDiagArgs)
PPCG_SIMPLE(symm, SymmArgs)
PPCG_SIMPLE(offdiag, OffdiagArgs)
PPCG_SIMPLE(frob2, Frob2Args)
PPCG_SIMPLE(orth, OrthArgs)
PPCG_SIMPLE(zero_int, ZeroIntArgs)
PPCG_SIMPLE(copy, CopyArgs)
PPCG_SIMPLE(polar, PolarArgs)
PPCG_SIMPLE(add_diag, AddDiagArgs)
PPCG_SIMPLE(trace, TraceArgs)
PPCG_SIMPLE(to_f32, ToF32Args)
#undef PPCG_SIMPLE

template <class A>
static void simple_launch(int kind, void (*k)(A), const A& a, unsigned blocks, hipStream_t st) {
  if (g_rec) {
    g_rec->add(kind, &a, sizeof(a), blocks);
    return;
  }
  if (blocks == 0) return;
  hipLaunchKernelGGL(k, dim3(blocks), dim3(256), 0, st, a);
}

void launch_transpose(const double* src, int lds, double* dst, int ldd, int m, int n, int cplx, hipStream_t st) {
  TransposeArgs a{src, lds, dst, ldd, m, n, cplx};
  simple_launch(OP_TRANSPOSE, transpose_kernel, a, (unsigned)(((m + 31) / 32) * ((n + 31) / 32)), st);
}
void launch_offdiag32(const double* G, int ldg, int m, float* F, int ldf, int cplx, hipStream_t st) {
  OffdiagArgs a{G, ldg, m, F, ldf, cplx};
  long t = (long)m * m;
  simple_launch(OP_OFFDIAG, offdiag_kernel, a, (unsigned)((t + 255) / 256), st);
}
void launch_fill(double* p, long count, double v, hipStream_t st) {
  FillArgs a{p, count, v};
  simple_launch(OP_FILL, fill_kernel, a, (unsigned)(count > 0 ? (count + 255) / 256 : 0), st);
}
void launch_set_diag(double* G, int ld, int m, const double* lam, int cplx, hipStream_t st) {
  SetDiagArgs a{G, ld, m, lam, cplx};
  long t = (long)m * m;
  simple_launch(OP_SETDIAG, set_diag_kernel, a, (unsigned)((t + 255) / 256), st);
}
void launch_symmetrize(double* G, int ld, int m, int cplx, hipStream_t st) {
  SymmArgs a{G, ld, m, cplx};
  long t = (long)m * m;
  simple_launch(OP_SYMM, symm_kernel, a, (unsigned)((t + 255) / 256), st);
}
void launch_frob2_sub(const double* G, int ld, int nw, double* out, int cplx, hipStream_t st) {
  Frob2Args a{G, ld, nw, out, cplx};
  simple_launch(OP_FROB2, frob2_kernel, a, (unsigned)(nw > 0 ? nw : 0), st);
}
void launch_orth_err2(const double* G, int ld, int k, double* out, int cplx, hipStream_t st, bool upper) {
  OrthArgs a{G, ld, k, out, cplx, upper ? 1 : 0};
  simple_launch(OP_ORTH, orth_kernel, a, 1u, st);
}
void launch_polar_prep(const double* G, int ld, int m, double* Y, double* M, int cplx, hipStream_t st) {
  PolarArgs a{G, ld, m, Y, M, cplx};
  long t = (long)m * m;
  simple_launch(OP_POLAR, polar_kernel, a, (unsigned)((t + 255) / 256), st);
}
void launch_add_diag(double* G, int ld, int m, double v, int cplx, hipStream_t st) {
  AddDiagArgs a{G, ld, m, v, cplx};
  simple_launch(OP_ADDDIAG, add_diag_kernel, a, (unsigned)((m + 255) / 256), st);
}
void launch_trace(const double* G, int ld, int m, double* out, int cplx, hipStream_t st) {
  TraceArgs a{G, ld, m, out, cplx};
  simple_launch(OP_TRACE, trace_kernel, a, 1u, st);
}
void launch_to_f32(const double* X, float* Y, long ld, long rows, int ncols, int cplx, hipStream_t st) {
  ToF32Args a{X, Y, ld, rows, ncols, cplx};
  long t = rows * (cplx ? 2 : 1) * ncols;
  simple_launch(OP_TOF32, to_f32_kernel, a, (unsigned)(t > 0 ? (t + 255) / 256 : 0), st);
}
void launch_zero_int(int* p, int n, hipStream_t st) {
  ZeroIntArgs a{p, n};
  simple_launch(OP_ZEROINT, zero_int_kernel, a, (unsigned)(n > 0 ? (n + 255) / 256 : 0), st);
}
void launch_copy(const double* src, double* dst, long count, hipStream_t st) {
  CopyArgs a{src, dst, count};
  simple_launch(OP_COPY, copy_kernel, a, (unsigned)(count > 0 ? (count + 255) / 256 : 0), st);
}
void launch_d2h(void* dst, const void* src, size_t bytes, hipStream_t st) {
  if (g_rec) {
    D2HArgs a{dst, src, bytes};
    g_rec->add(OP_D2H, &a, sizeof(a), 0);
    return;
  }
  if (bytes) hipMemcpyAsync(dst, src, bytes, hipMemcpyDeviceToHost, st);
}

bool launch_grouped_dense(int kind, const void* jobs, const unsigned* start, int nj, unsigned total, hipStream_t st) {
#define PPCG_G(NAME, ARGS) \
  hipLaunchKernelGGL(NAME##_grouped, dim3(total), dim3(256), 0, st, (const ARGS*)jobs, start, nj)
  switch (kind) {
    case OP_TRANSPOSE: PPCG_G(transpose, TransposeArgs); return true;
    case OP_FILL: PPCG_G(fill, FillArgs); return true;
    case OP_SETDIAG: PPCG_G(set_diag, SetDiagArgs); return true;
    case OP_SYMM: PPCG_G(symm, SymmArgs); return true;
    case OP_OFFDIAG: PPCG_G(offdiag, OffdiagArgs); return true;
    case OP_FROB2: PPCG_G(frob2, Frob2Args); return true;
    case OP_ORTH: PPCG_G(orth, OrthArgs); return true;
    case OP_ZEROINT: PPCG_G(zero_int, ZeroIntArgs); return true;
    case OP_COPY: PPCG_G(copy, CopyArgs); return true;
    case OP_POLAR: PPCG_G(polar, PolarArgs); return true;
    case OP_ADDDIAG: PPCG_G(add_diag, AddDiagArgs); return true;
    case OP_TRACE: PPCG_G(trace, TraceArgs); return true;
    case OP_TOF32: PPCG_G(to_f32, ToF32Args); return true;
  }
#undef PPCG_G
  return false;
}

// ---------------------------------------------------------------------------
// block Jacobi
// ---------------------------------------------------------------------------
constexpr int JB = 16;           // block width
constexpr int BJ_INIT_WG = 64;   // workgroups of the init step
constexpr int J2 = 2 * JB;       // pair size
constexpr int JLD = J2 + 1;
#ifndef PPCG_BJ_INNER
#define PPCG_BJ_INNER 1
#endif
// Inner Jacobi sweeps per pair eigensolve.  The pair problem need not be
// diagonalised exactly: the outer loop ends only after a sweep in which no
// off-diagonal entry anywhere exceeds the threshold, whatever the inner count.
constexpr int BJ_INNER = PPCG_BJ_INNER;
// Rotations are skipped once |M_pq| <= rel_tol |M|_F.  Off-diagonal entries
// of that size change the Ritz residual of a column by at most
// rel_tol |M|_F sqrt(K) (the caller keeps this far below its locking
// threshold) and the eigenvalues (Rayleigh quotients of the rotated
// columns) by O(off^2 / gap).

struct EigDev {
  double* M;
  int ld, m;
  double* V;
  int ldv;
  double* lam;
  double* Q;       // 2 x np x J2 x J2 scalars: the rotations of rounds of even / odd parity
  double* M2;      // m x m (ld m): the second buffer of M for fused rounds
  double* Vt;      // m x m accumulated rotations
  double* tiny;    // BJ_INIT_WG partial sums of |M|^2
  int* flags;      // 2 x fst: which pairs rotated, per parity
  int* rank;       // m
  int* counter;    // shared by all problems of a call
  double rel_tol;
  int nbe, np, fst;
};

static EigDev carve(const EigJob& j, int* counter) {
  int nblk = (j.m + JB - 1) / JB;
  int nbe = nblk + (nblk & 1);
  int np = nbe / 2;
  const size_t es = j.cplx ? 16 : 8;
  char* p = (char*)j.work;
  EigDev w{};
  w.M = j.M;
  w.ld = j.ld;
  w.m = j.m;
  w.V = j.V;
  w.ldv = j.ldv;
  w.lam = j.lam;
  w.fst = (np + 63) / 64 * 64;
  w.Q = (double*)p; p += es * 2 * np * J2 * J2;
  w.M2 = (double*)p; p += es * (size_t)j.m * j.m;
  w.Vt = (double*)p; p += es * (size_t)j.m * j.m;
  w.tiny = (double*)p; p += sizeof(double) * BJ_INIT_WG;
  w.flags = (int*)p; p += sizeof(int) * 2 * w.fst;
  w.rank = (int*)p;
  w.counter = counter;
  w.rel_tol = j.rel_tol;
  w.nbe = nbe;
  w.np = np;
  return w;
}
size_t eig_workspace_bytes(int m, int cplx) {
  int nblk = (m + JB - 1) / JB;
  int np = (nblk + 1) / 2;
  const size_t es = cplx ? 16 : 8;
  return es * 2 * (size_t)np * J2 * J2 + 2 * es * (size_t)m * m + sizeof(double) * BJ_INIT_WG +
         sizeof(int) * 2 * ((np + 63) / 64 * 64) + sizeof(int) * (size_t)m + 256;
}

PPCG_DEV void pair_of(const EigDev& a, int t, int round, int& nI, int& nJ, int& i0, int& j0) {
  const int nblk = (a.m + JB - 1) / JB;
  int I = rr_player(t, round, a.nbe), J = rr_player(a.nbe - 1 - t, round, a.nbe);
  if (I > J) { int x = I; I = J; J = x; }
  i0 = I * JB;
  j0 = J * JB;
  nI = I < nblk ? min(JB, a.m - i0) : 0;
  nJ = J < nblk ? min(JB, a.m - j0) : 0;
}

// step kernels; `round` is shared by all jobs of a launch
// BJ_INIT_WG workgroups: Vt = I, and partial sums of |M|^2 (one per workgroup)
// from which every pair step forms the skip threshold rel_tol |M|_F
template <class S>
PPCG_DEV void bj_init_body(const EigDev& a, unsigned wg) {
  long mm = (long)a.m * a.m;
  S* Vt = (S*)a.Vt;
  const S* M = (const S*)a.M;
  double s = 0;
  for (long e = wg * 256L + threadIdx.x; e < mm; e += 256L * BJ_INIT_WG) {
    const int i = (int)(e % a.m), j = (int)(e / a.m);
    Vt[e] = from_real<S>(i == j ? 1.0 : 0.0);
    s += abs2_(M[i + (long)j * a.ld]);
  }
  __shared__ double red[4];
  s = wave_sum(s);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = s;
  __syncthreads();
  if (threadIdx.x == 0) a.tiny[wg] = (red[0] + red[1]) + (red[2] + red[3]);
}
PPCG_DEV double bj_tiny(const EigDev& a) {
  double s = 0;
  for (int w = 0; w < BJ_INIT_WG; ++w) s += a.tiny[w];
  return a.rel_tol * sqrt(s);
}

// the pair of `round` that holds block B, and B's offset inside that pair
PPCG_DEV void locate(const EigDev& a, int B, int round, int& t, int& off) {
  const int n1 = a.nbe - 1;
  int pos = 0;
  if (B != 0) pos = ((B - 1 - round) % n1 + n1) % n1 + 1;
  t = pos < a.np ? pos : a.nbe - 1 - pos;
  int nI, nJ, i0, j0;
  pair_of(a, t, round, nI, nJ, i0, j0);
  off = (B * JB == i0) ? 0 : nI;
}

// M of the rounds: M_0 is the caller's matrix; with fused rounds, M_r (r >= 1)
// alternates between the second buffer (r odd) and the caller's matrix (r
// even), and the last round of a sweep writes the caller's matrix
template <class S>
PPCG_DEV S* bj_buf(const EigDev& a, int r, int& ld) {
  const bool second = r > 0 && (r & 1);
  ld = second ? a.m : a.ld;
  return (S*)(second ? a.M2 : a.M);
}

// Q_a^H M_ab Q_b for pairs ta (rows) and tb (columns) of `round`, read from
// src (ld lds), Q and the flags of parity par; Q = I for a pair that did not
// rotate.  Leaves the na x nb result in sh (ld JLD) and returns true, or
// returns false when neither pair rotated (the tile is src unchanged).  The
// same arithmetic serves the stored update and the fused pair step, so both
// see identical values.
template <class S>
PPCG_DEV bool bj_tile(const EigDev& a, int round, const S* src, long lds, int par, int ta, int tb, S* sh, int& na,
                      int& nb) {
  const int tid = threadIdx.x, nt = blockDim.x;
  const int* fl = a.flags + par * a.fst;
  const bool ra = fl[ta] != 0, rb = fl[tb] != 0;
  int nIa, nJa, i0a, j0a, nIb, nJb, i0b, j0b;
  pair_of(a, ta, round, nIa, nJa, i0a, j0a);
  pair_of(a, tb, round, nIb, nJb, i0b, j0b);
  na = nIa + nJa;
  nb = nIb + nJb;
  if (!ra && !rb) return false;
  auto ga = [&](int x) { return x < nIa ? i0a + x : j0a + (x - nIa); };
  auto gb = [&](int y) { return y < nIb ? i0b + y : j0b + (y - nIb); };
  const S zero = from_real<S>(0.0);
  S* Ms = sh;
  S* Ts = sh + J2 * JLD;
  S* QA = sh + 2 * J2 * JLD;
  S* QB = sh + 3 * J2 * JLD;
  const S* Qp = (const S*)a.Q + (long)par * a.np * J2 * J2;
  const S* qa = Qp + (long)ta * J2 * J2;
  const S* qb = Qp + (long)tb * J2 * J2;
  for (int e = tid; e < na * nb; e += nt) {
    int x = e % na, y = e / na;
    Ms[x + y * JLD] = src[ga(x) + (long)gb(y) * lds];
  }
  if (ra)
    for (int e = tid; e < na * na; e += nt) QA[(e % na) + (e / na) * JLD] = qa[(e % na) + (e / na) * J2];
  if (rb)
    for (int e = tid; e < nb * nb; e += nt) QB[(e % nb) + (e / nb) * JLD] = qb[(e % nb) + (e / nb) * J2];
  __syncthreads();
  for (int e = tid; e < na * nb; e += nt) {  // T = M_ab Q_b
    int x = e % na, y = e / na;
    S t = zero;
    if (rb) {
      for (int u = 0; u < nb; ++u) t += Ms[x + u * JLD] * QB[u + y * JLD];
    } else {
      t = Ms[x + y * JLD];
    }
    Ts[x + y * JLD] = t;
  }
  __syncthreads();
  for (int e = tid; e < na * nb; e += nt) {  // Q_a^H T
    int x = e % na, y = e / na;
    S t = zero;
    if (ra) {
      for (int u = 0; u < na; ++u) t += conj_(QA[u + x * JLD]) * Ts[u + y * JLD];
    } else {
      t = Ts[x + y * JLD];
    }
    Ms[x + y * JLD] = t;
  }
  __syncthreads();
  return true;
}

// Pair eigensolve t of `round` (NT threads; more waves hide the LDS latency of
// the Jacobi rounds).  The pair problem is read from M_round; with fused
// rounds and round >= 1 it is formed here from M_{round-1} and the previous
// round's rotations, tile by tile (sh: scratch for bj_tile).  Writes Q and the
// flag of parity `par`.
template <class S, int NT>
PPCG_DEV void bj_pair_body(const EigDev& a, int round, unsigned t, bool fused, int par, S* sh) {
  __shared__ S Sm[J2 * JLD], Qs[J2 * JLD];
  __shared__ double red[NT / 64];
  __shared__ JRot<S> jr[J2 / 2 + 1];
  __shared__ int any;
  const int tid = threadIdx.x;
  if (round >= a.nbe - 1) return;
  int nI, nJ, i0, j0;
  pair_of(a, t, round, nI, nJ, i0, j0);
  const int n2 = nI + nJ;
  const double tiny = bj_tiny(a);
  if (tid == 0) any = 0;
  if (fused && round > 0) {
    int lds;
    const S* src = bj_buf<S>(a, round - 1, lds);
    // blocks of this pair: (global block, size, offset in this pair)
    const int nbk = nJ > 0 ? 2 : 1;
    const int bk[2] = {i0 / JB, j0 / JB}, bs[2] = {nI, nJ}, bo[2] = {0, nI};
    int pt[2], po[2];
    for (int u = 0; u < nbk; ++u) locate(a, bk[u], round - 1, pt[u], po[u]);
    for (int u = 0; u < nbk; ++u)
      for (int v = 0; v < nbk; ++v) {
        int na, nb;
        __syncthreads();
        const bool rot = bj_tile<S>(a, round - 1, src, lds, par ^ 1, pt[u], pt[v], sh, na, nb);
        int nIu, nJu, i0u, j0u, nIv, nJv, i0v, j0v;
        pair_of(a, pt[u], round - 1, nIu, nJu, i0u, j0u);
        pair_of(a, pt[v], round - 1, nIv, nJv, i0v, j0v);
        for (int e = tid; e < bs[u] * bs[v]; e += NT) {
          const int x = e % bs[u], y = e / bs[u];
          S val;
          if (rot) {
            val = sh[(po[u] + x) + (po[v] + y) * JLD];
          } else {
            const int xx = po[u] + x, yy = po[v] + y;
            const int gx = xx < nIu ? i0u + xx : j0u + (xx - nIu);
            const int gy = yy < nIv ? i0v + yy : j0v + (yy - nIv);
            val = src[gx + (long)gy * lds];
          }
          const int xs = bo[u] + x, ys = bo[v] + y;
          Sm[xs + ys * JLD] = val;
          if (xs != ys && sqrt(abs2_(val)) > tiny) any = 1;
        }
      }
    __syncthreads();
  } else {
    int lds;
    const S* M = bj_buf<S>(a, fused ? round : 0, lds);
    auto gidx = [&](int x) { return x < nI ? i0 + x : j0 + (x - nI); };
    __syncthreads();
    for (int e = tid; e < n2 * n2; e += NT) {
      int x = e % n2, y = e / n2;
      S v = M[gidx(x) + (long)gidx(y) * lds];
      Sm[x + y * JLD] = v;
      if (x != y && sqrt(abs2_(v)) > tiny) any = 1;
    }
    __syncthreads();
  }
  int* fl = a.flags + par * a.fst;
  if (!any) {
    if (tid == 0) fl[t] = 0;
    return;
  }
  lds_jacobi<NT, S>(Sm, Qs, n2, JLD, tiny, BJ_INNER, jr, red);
  S* Qg = (S*)a.Q + ((long)par * a.np + t) * J2 * J2;
  for (int e = tid; e < n2 * n2; e += NT) Qg[(e % n2) + (e / n2) * J2] = Qs[(e % n2) + (e / n2) * JLD];
  if (tid == 0) fl[t] = 1;
}

// Stop test after a sweep: counts the workgroups that see an off-diagonal
// entry of M above the skip threshold.  Every off-diagonal entry of M lies in
// the pair problem of some round, and while nothing rotates M stays as it is,
// so the next sweep would rotate anything exactly when this count is nonzero:
// the loop ends without running a last sweep that only confirms convergence.
constexpr int BJ_CHECK_PER_WG = 256 * 16;
template <class S>
PPCG_DEV void bj_check_body(const EigDev& a, unsigned wg) {
  __shared__ int any;
  const S* M = (const S*)a.M;
  const double tiny = bj_tiny(a);
  if (threadIdx.x == 0) any = 0;
  __syncthreads();
  const long mm = (long)a.m * a.m;
  const long e1 = min(mm, (long)(wg + 1) * BJ_CHECK_PER_WG);
  bool hit = false;
  for (long e = (long)wg * BJ_CHECK_PER_WG + threadIdx.x; e < e1; e += 256) {
    const int i = (int)(e % a.m), j = (int)(e / a.m);
    if (i != j && sqrt(abs2_(M[i + (long)j * a.ld])) > tiny) hit = true;
  }
  if (hit) any = 1;
  __syncthreads();
  if (threadIdx.x == 0 && any) atomicAdd(a.counter, 1);
}

// One round's two-sided update.  Items [0, np^2): the tile (rows of pair a) x
// (columns of pair b) of M_round becomes Q_a^H M_ab Q_b in M_{round+1} (Q = I
// for a pair that did not rotate; a tile neither pair rotated is copied when
// the two buffers differ); tiles are disjoint, so no item depends on another.
// Items [np^2, np^2 + np * ceil(m/64)): 64 rows of the accumulated rotations,
// Vt[rows, cols of pair b] <- Vt[rows, cols] Q_b, in place.  Unfused rounds
// update the caller's matrix in place (src = dst, parity 0).
template <class S>
PPCG_DEV void bj_update_body(const EigDev& a, int round, unsigned wg, bool fused, int par, S* sh) {
  if (round >= a.nbe - 1) return;
  const int tid = threadIdx.x, nt = blockDim.x;
  const int np = a.np;
  const unsigned nmt = (unsigned)np * np;
  const S zero = from_real<S>(0.0);
  int lds = a.ld, ldd = a.ld;
  const S* src = (const S*)a.M;
  S* dst = (S*)a.M;
  if (fused) {
    src = bj_buf<S>(a, round, lds);
    dst = round + 1 == a.nbe - 1 ? (S*)a.M : bj_buf<S>(a, round + 1, ldd);
    if (round + 1 == a.nbe - 1) ldd = a.ld;
  }
  if (wg < nmt) {
    const int ta = (int)(wg % np), tb = (int)(wg / np);
    int na, nb;
    const bool rot = bj_tile<S>(a, round, src, lds, par, ta, tb, sh, na, nb);
    if (!rot && src == dst) return;
    int nIa, nJa, i0a, j0a, nIb, nJb, i0b, j0b;
    pair_of(a, ta, round, nIa, nJa, i0a, j0a);
    pair_of(a, tb, round, nIb, nJb, i0b, j0b);
    auto ga = [&](int x) { return x < nIa ? i0a + x : j0a + (x - nIa); };
    auto gb = [&](int y) { return y < nIb ? i0b + y : j0b + (y - nIb); };
    for (int e = tid; e < na * nb; e += nt) {
      int x = e % na, y = e / na;
      dst[ga(x) + (long)gb(y) * ldd] = rot ? sh[x + y * JLD] : src[ga(x) + (long)gb(y) * lds];
    }
    return;
  }
  const int* fl = a.flags + par * a.fst;
  const unsigned it = wg - nmt;
  const int tb = (int)(it % np), chunk = (int)(it / np);
  if (!fl[tb]) return;
  int nI, nJ, i0, j0;
  pair_of(a, tb, round, nI, nJ, i0, j0);
  const int n2 = nI + nJ;
  auto gidx = [&](int x) { return x < nI ? i0 + x : j0 + (x - nI); };
  S* Qs = sh;
  S* R = sh + J2 * JLD;  // 64 rows x n2, ld JLD
  const S* Qg = (const S*)a.Q + ((long)par * np + tb) * J2 * J2;
  for (int e = tid; e < n2 * n2; e += nt) Qs[(e % n2) + (e / n2) * JLD] = Qg[(e % n2) + (e / n2) * J2];
  const int c0 = chunk * 64;
  const int nc = min(64, a.m - c0);
  S* Vt = (S*)a.Vt;
  for (int e = tid; e < nc * n2; e += nt) {
    int r = e % nc, x = e / nc;
    R[x + r * JLD] = Vt[(c0 + r) + (long)gidx(x) * a.m];
  }
  __syncthreads();
  for (int e = tid; e < nc * n2; e += nt) {
    int r = e % nc, x = e / nc;
    S t = zero;
    for (int u = 0; u < n2; ++u) t += R[u + r * JLD] * Qs[u + x * JLD];
    Vt[(c0 + r) + (long)gidx(x) * a.m] = t;
  }
}

// ranks of the (real) diagonal (ascending, ties by index) -> lam; then Vt
// columns gathered into V.  One thread per diagonal entry, ceil(m / 256)
// workgroups; the diagonal is read through LDS in chunks of 1024.
template <class S>
PPCG_DEV void bj_rank_body(const EigDev& a, unsigned wg) {
  __shared__ double dg[1024];
  const S* M = (const S*)a.M;
  const int x = (int)wg * 256 + (int)threadIdx.x;
  const double lx = x < a.m ? real_(M[x + (long)x * a.ld]) : 0.0;
  int rk = 0;
  for (int y0 = 0; y0 < a.m; y0 += 1024) {
    const int ny = min(1024, a.m - y0);
    __syncthreads();
    for (int e = threadIdx.x; e < ny; e += 256) dg[e] = real_(M[(y0 + e) + (long)(y0 + e) * a.ld]);
    __syncthreads();
    if (x < a.m)
      for (int e = 0; e < ny; ++e) {
        const double ly = dg[e];
        rk += (ly < lx) || (ly == lx && y0 + e < x);
      }
  }
  if (x < a.m) {
    a.rank[x] = rk;
    a.lam[rk] = lx;
  }
}
template <class S>
PPCG_DEV void bj_gather_body(const EigDev& a, unsigned wg) {
  long e = wg * 256L + threadIdx.x;
  if (e >= (long)a.m * a.m) return;
  int i = e % a.m, j = e / a.m;
  ((S*)a.V)[i + (long)a.rank[j] * a.ldv] = ((const S*)a.Vt)[i + (long)j * a.m];
}

// STEP: 0 init, 1 pair eigensolves, 2 two-sided update of M and Vt, 3 rank,
// 4 gather, 5 stop test; fused rounds: 6 pair eigensolves of round 0, 7 pair
// eigensolves of `round` beside the update of round - 1, 8 the update of the
// last round
#ifndef PPCG_BJ_PAIR_NT
#define PPCG_BJ_PAIR_NT 1024
#endif
#ifndef PPCG_BJ_FUSED
#define PPCG_BJ_FUSED 0
#endif
constexpr int BJ_PAIR_NT = PPCG_BJ_PAIR_NT;
template <int STEP> constexpr int bj_threads() { return (STEP == 1 || STEP >= 6) ? BJ_PAIR_NT : 256; }
template <class S>
PPCG_DEV S* bj_scratch() {
  __shared__ S sh[4 * J2 * JLD];
  return sh;
}
template <class S, int STEP>
__global__ __launch_bounds__(bj_threads<STEP>()) void bj_grouped(const EigDev* jobs, const unsigned* start, int nj, int round) {
  int j = find_job(start, nj, blockIdx.x);
  unsigned wg = blockIdx.x - start[j];
  const EigDev& a = jobs[j];
  if constexpr (STEP == 0) bj_init_body<S>(a, wg);
  if constexpr (STEP == 1) bj_pair_body<S, BJ_PAIR_NT>(a, round, wg, false, 0, nullptr);
  if constexpr (STEP == 2) bj_update_body<S>(a, round, wg, false, 0, bj_scratch<S>());
  if constexpr (STEP == 3) bj_rank_body<S>(a, wg);
  if constexpr (STEP == 4) bj_gather_body<S>(a, wg);
  if constexpr (STEP == 5) bj_check_body<S>(a, wg);
  if constexpr (STEP == 6) bj_pair_body<S, BJ_PAIR_NT>(a, 0, wg, true, 0, bj_scratch<S>());
  if constexpr (STEP == 7) {
    if (wg < (unsigned)a.np) bj_pair_body<S, BJ_PAIR_NT>(a, round, wg, true, round & 1, bj_scratch<S>());
    else bj_update_body<S>(a, round - 1, wg - a.np, true, (round - 1) & 1, bj_scratch<S>());
  }
  if constexpr (STEP == 8) bj_update_body<S>(a, round, wg, true, round & 1, bj_scratch<S>());
}

void EigGraphCache::clear() {
  if (exec) hipGraphExecDestroy(exec);
  if (graph) hipGraphDestroy(graph);
  exec = nullptr;
  graph = nullptr;
  key.clear();
}
EigGraphCache::~EigGraphCache() {
  clear();
  if (dev) hipFree(dev);
  if (stream) hipStreamDestroy(stream);
}

int block_jacobi_eig_grouped(const std::vector<EigJob>& jobs, Stage& stage, EigGraphCache* graphs, int* dev_counter,
                             int* host_counter, hipStream_t st) {
  const int nj = (int)jobs.size();
  if (nj == 0) return 0;
  const bool cplx = jobs[0].cplx;
  bool own_stream = false;
  if (graphs) {
    if (!graphs->stream && hipStreamCreateWithFlags(&graphs->stream, hipStreamNonBlocking) != hipSuccess) {
      graphs->stream = nullptr;
      graphs = nullptr;
    } else {
      st = graphs->stream;
      own_stream = true;
    }
  }
  std::vector<EigDev> ed(nj);
  int maxr = 1;
  for (int j = 0; j < nj; ++j) {
    ed[j] = carve(jobs[j], dev_counter);
    maxr = std::max(maxr, ed[j].nbe - 1);
  }
  // start arrays for the five step shapes
  auto wgs = [&](int step, const EigDev& a) -> unsigned {
    long mm = (long)a.m * a.m;
    switch (step) {
      case 0: return (unsigned)BJ_INIT_WG;
      case 1: return (unsigned)a.np;
      case 2: return (unsigned)(a.np * a.np + a.np * ((a.m + 63) / 64));
      case 3: return (unsigned)((a.m + 255) / 256);
      case 4: return (unsigned)((mm + 255) / 256);
      case 5: return (unsigned)((mm + BJ_CHECK_PER_WG - 1) / BJ_CHECK_PER_WG);
      case 6: return (unsigned)a.np;
      case 7: return (unsigned)(a.np + a.np * a.np + a.np * ((a.m + 63) / 64));
      default: return (unsigned)(a.np * a.np + a.np * ((a.m + 63) / 64));
    }
  };
  constexpr int NSTEP = 9;
  const unsigned* sd[NSTEP];
  unsigned tot[NSTEP];
  std::vector<unsigned> starts;
  for (int step = 0; step < NSTEP; ++step) {
    unsigned t = 0;
    for (int j = 0; j < nj; ++j) {
      starts.push_back(t);
      t += wgs(step, ed[j]);
    }
    starts.push_back(t);
    tot[step] = t;
  }
  size_t jb = sizeof(EigDev) * nj;
  std::vector<uint8_t> buf(jb + sizeof(unsigned) * starts.size());
  std::memcpy(buf.data(), ed.data(), jb);
  std::memcpy(buf.data() + jb, starts.data(), sizeof(unsigned) * starts.size());
  // with a graph cache the array lives at the cache's fixed address (the
  // captured sweep reads it there); else in the per-call staging area
  bool reuse = false;
  uint8_t* dev;
  if (graphs) {
    reuse = graphs->exec && graphs->key == buf;
    if (!reuse) {
      graphs->clear();
      if (graphs->cap < buf.size()) {
        if (graphs->dev) hipFree(graphs->dev);
        graphs->dev = nullptr;
        graphs->cap = 0;
        if (hipMalloc(&graphs->dev, buf.size()) != hipSuccess) throw std::runtime_error("hipMalloc failed");
        graphs->cap = buf.size();
      }
      if (hipMemcpyAsync(graphs->dev, buf.data(), buf.size(), hipMemcpyHostToDevice, st) != hipSuccess ||
          hipStreamSynchronize(st) != hipSuccess)
        throw std::runtime_error("eigensolver job upload failed");
    }
    dev = (uint8_t*)graphs->dev;
  } else {
    dev = (uint8_t*)stage.upload(buf.data(), buf.size(), st);
  }
  const EigDev* dj = (const EigDev*)dev;
  for (int step = 0; step < NSTEP; ++step) sd[step] = (const unsigned*)(dev + jb) + step * (nj + 1);
  auto launch = [&](auto kernel, int step, int round) {
    const int nt = (step == 1 || step >= 6) ? BJ_PAIR_NT : 256;
    hipLaunchKernelGGL(kernel, dim3(tot[step]), dim3(nt), 0, st, dj, sd[step], nj, round);
  };
  auto run = [&](int step, int round) {
    if (!tot[step]) return;
    if (cplx) {
      switch (step) {
        case 0: launch(bj_grouped<zdouble, 0>, step, round); break;
        case 1: launch(bj_grouped<zdouble, 1>, step, round); break;
        case 2: launch(bj_grouped<zdouble, 2>, step, round); break;
        case 3: launch(bj_grouped<zdouble, 3>, step, round); break;
        case 4: launch(bj_grouped<zdouble, 4>, step, round); break;
        case 5: launch(bj_grouped<zdouble, 5>, step, round); break;
        case 6: launch(bj_grouped<zdouble, 6>, step, round); break;
        case 7: launch(bj_grouped<zdouble, 7>, step, round); break;
        default: launch(bj_grouped<zdouble, 8>, step, round); break;
      }
    } else {
      switch (step) {
        case 0: launch(bj_grouped<double, 0>, step, round); break;
        case 1: launch(bj_grouped<double, 1>, step, round); break;
        case 2: launch(bj_grouped<double, 2>, step, round); break;
        case 3: launch(bj_grouped<double, 3>, step, round); break;
        case 4: launch(bj_grouped<double, 4>, step, round); break;
        case 5: launch(bj_grouped<double, 5>, step, round); break;
        case 6: launch(bj_grouped<double, 6>, step, round); break;
        case 7: launch(bj_grouped<double, 7>, step, round); break;
        default: launch(bj_grouped<double, 8>, step, round); break;
      }
    }
  };
  // one sweep: every round's two launches, then the stop test into the zeroed
  // counter, read back
  auto sweep_ops = [&]() {
    if (PPCG_BJ_FUSED) {  // one launch per round: its pair eigensolves beside the previous round's update
      run(6, 0);
      for (int round = 1; round < maxr; ++round) run(7, round);
      run(8, maxr - 1);
    } else {
      for (int round = 0; round < maxr; ++round) {
        run(1, round);
        run(2, round);
      }
    }
    ZeroIntArgs z{dev_counter, 1};
    hipLaunchKernelGGL(zero_int_kernel, dim3(1), dim3(256), 0, st, z);
    run(5, 0);
    hipMemcpyAsync(host_counter, dev_counter, sizeof(int), hipMemcpyDeviceToHost, st);
  };
  if (graphs && !reuse) {
    hipGraph_t g = nullptr;
    hipGraphExec_t ge = nullptr;
    bool ok = hipStreamBeginCapture(st, hipStreamCaptureModeThreadLocal) == hipSuccess;
    if (ok) {
      sweep_ops();
      ok = hipStreamEndCapture(st, &g) == hipSuccess && g != nullptr;
    }
    if (ok) ok = hipGraphInstantiate(&ge, g, nullptr, nullptr, 0) == hipSuccess;
    if (ok) {
      graphs->graph = g;
      graphs->exec = ge;
      graphs->key = buf;
    } else {
      if (g) hipGraphDestroy(g);
      (void)hipGetLastError();
      graphs->clear();
      graphs = nullptr;  // this call runs without the graph
    }
  }
  run(0, 0);
  int sweeps = 0;
  for (int sweep = 0; sweep < 80; ++sweep) {
    if (graphs) {
      if (hipGraphLaunch(graphs->exec, st) != hipSuccess) throw std::runtime_error("hipGraphLaunch failed");
    } else {
      sweep_ops();
    }
    ++sweeps;
    if (hipStreamSynchronize(st) != hipSuccess) throw std::runtime_error("block Jacobi sweep failed");
    if (*host_counter == 0) break;
  }
  run(3, 0);
  run(4, 0);
  if (own_stream && hipStreamSynchronize(st) != hipSuccess) throw std::runtime_error("block Jacobi failed");
  return sweeps;
}

bool launch_grouped_gemm(int, const void*, const unsigned*, int, unsigned, hipStream_t);
bool launch_grouped_stencil(int, const void*, const unsigned*, int, unsigned, hipStream_t);
bool launch_grouped_block(int, const void*, const unsigned*, int, unsigned, hipStream_t);
bool launch_grouped_prep(int, const void*, const unsigned*, int, unsigned, hipStream_t);

bool launch_grouped(int kind, const void* jobs, const unsigned* start, int nj, unsigned total, hipStream_t st) {
  if (total == 0) return true;
  return launch_grouped_gemm(kind, jobs, start, nj, total, st) ||
         launch_grouped_stencil(kind, jobs, start, nj, total, st) ||
         launch_grouped_block(kind, jobs, start, nj, total, st) ||
         launch_grouped_dense(kind, jobs, start, nj, total, st) || launch_grouped_prep(kind, jobs, start, nj, total, st);
}

}  // namespace ppcg
