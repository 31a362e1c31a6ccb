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

template <class S>
PPCG_DEV S phased(S xp, S xm, const double* ph) {
  if constexpr (sc_traits<S>::cplx) {
    typedef typename sc_traits<S>::real_t R;
    cpx<R> f{(R)ph[0], (R)ph[1]};
    return f * xp + conj_(f) * xm;
  } else {
    return xp + xm;
  }
}

// S: double, float, zdouble, zfloat.  The coupling from point r to
// r + a h e_d carries exp(i kappa_d a h) (gauge form of the Bloch phase).
// A workgroup owns 256 consecutive points of an (x, y) plane and marches
// through SZ consecutive z planes: the z neighbours of a point are the
// centres of the planes before and after it, kept in registers, so each
// point issues one load for z and the x, y neighbours come from the plane
// the workgroup (or its neighbour) is loading anyway.
constexpr int SZ = 16;  // z planes per workgroup

PPCG_DEV int wrap_idx(int c, int d, int N) {
  int r = c + d;
  return r >= N ? r - N : (r < 0 ? r + N : r);
}

template <class S, int ORDER>
PPCG_DEV void stencil_body(const StencilArgs& a, unsigned wg, unsigned nwg) {
  typedef typename sc_traits<S>::real_t R;
  const int N = a.N;
  const long NN = (long)N * N;
  const unsigned tpp = (unsigned)((NN + 255) / 256);       // tiles per plane
  const unsigned kch = (unsigned)((N + SZ - 1) / SZ);      // z chunks
  unsigned L = xcd_remap(wg, nwg);
  const int col = (int)(L / (tpp * kch));
  const unsigned rest = L % (tpp * kch);
  const int kc = (int)(rest / tpp);
  const long q = (long)(rest % tpp) * 256 + threadIdx.x;  // point inside the plane
  if (col >= a.ncols || q >= NN) return;
  const S* x = (const S*)a.X + (long)col * a.ldx;
  S* y = (S*)a.Y + (long)col * a.ldy;
  const R* V = (const R*)a.V;
  const int i = (int)(q % N), j = (int)(q / N);
  const long b = q - i;            // start of the x line in the plane
  const long pl = q - (long)j * N;  // (i, 0) in the plane
  const int k0 = kc * SZ;
  const int k1 = k0 + SZ < N ? k0 + SZ : N;
  auto at = [&](int k) { return x[q + (long)k * NN]; };
  // z window: zm2 = k-2, zm1 = k-1, zc = k, zp1 = k+1, zp2 = k+2
  S zm2 = ORDER == 4 ? at(wrap_idx(k0, -2, N)) : S{};
  S zm1 = at(wrap_idx(k0, -1, N));
  S zc = at(k0);
  S zp1 = at(wrap_idx(k0, 1, N));
  for (int k = k0; k < k1; ++k) {
    S zp2 = ORDER == 4 ? at(wrap_idx(k, 2, N)) : S{};
    const long pk = (long)k * NN;
    const S* xp = x + pk;
    const long p = q + pk;
    S s1 = phased<S>(xp[b + wrap_idx(i, 1, N)], xp[b + wrap_idx(i, -1, N)], a.ph[0][0]) +
           phased<S>(xp[pl + (long)wrap_idx(j, 1, N) * N], xp[pl + (long)wrap_idx(j, -1, N) * N], a.ph[1][0]) +
           phased<S>(zp1, zm1, a.ph[2][0]);
    S out = ((R)a.c0 + V[p]) * zc + (R)a.w1 * s1;
    if (ORDER == 4) {
      S s2 = phased<S>(xp[b + wrap_idx(i, 2, N)], xp[b + wrap_idx(i, -2, N)], a.ph[0][1]) +
             phased<S>(xp[pl + (long)wrap_idx(j, 2, N) * N], xp[pl + (long)wrap_idx(j, -2, N) * N], a.ph[1][1]) +
             phased<S>(zp2, zm2, a.ph[2][1]);
      out += (R)a.w2 * s2;
    }
    if (a.shift) out -= (R)a.shift[col] * zc;
    y[p] = out;
    zm2 = zm1;
    zm1 = zc;
    zc = zp1;
    zp1 = ORDER == 4 ? zp2 : at(wrap_idx(k, 2, N));
  }
}
template <class S, int ORDER>
__global__ __launch_bounds__(256) void stencil_kernel(StencilArgs a) {
  stencil_body<S, ORDER>(a, blockIdx.x, gridDim.x);
}

// LDS-staged, software-pipelined variant (single launches).  For each z
// plane the workgroup stages a window of the flattened (x, y) plane -- its
// 256 points and R N points on either side (R = ORDER / 2, plane-periodic) --
// in LDS; the x and y neighbours of a point are then LDS reads and the z
// neighbours stay in registers.  The loads for plane k + 1 (its window, V and
// the z value entering the register window) are issued before plane k is
// computed and written to the second LDS buffer after it, so every wave keeps
// a plane's worth of loads in flight while it computes: one barrier per
// plane.  The window offsets (wrapped in the plane) are computed once.  A
// point costs (256 + 2 R N) / 256 coalesced loads for the window plus one for
// its z neighbour and one for V, instead of one load per neighbour.
template <int ORDER>
constexpr int stencil_rad() { return ORDER / 2; }
inline int stencil_window(int N, int order) { return 256 + 2 * (order / 2) * N; }

template <class S, int ORDER, int WPT>
__global__ __launch_bounds__(256) void stencil_lds_kernel(StencilArgs a) {
  typedef typename sc_traits<S>::real_t R;
  extern __shared__ __align__(16) char smem[];
  constexpr int RAD = stencil_rad<ORDER>();
  const int N = a.N;
  const int NN = N * N;
  const int W = 256 + 2 * RAD * N;  // WPT * 256 >= W (checked by the launcher)
  S* const win0 = (S*)smem;
  S* const win1 = win0 + W;
  const unsigned tpp = (unsigned)((NN + 255) / 256);
  const unsigned kch = (unsigned)((N + SZ - 1) / SZ);
  const unsigned L = xcd_remap(blockIdx.x, gridDim.x);
  const int col = (int)(L / (tpp * kch));
  const unsigned rest = L % (tpp * kch);
  const int kc = (int)(rest / tpp);
  const int q0 = (int)(rest % tpp) * 256;
  if (col >= a.ncols) return;  // uniform over the workgroup
  const int tid = threadIdx.x;
  const int q = q0 + tid;
  const bool act = q < NN;
  const S* x = (const S*)a.X + (long)col * a.ldx;
  S* y = (S*)a.Y + (long)col * a.ldy;
  const R* V = (const R*)a.V;
  const int i = act ? q % N : 0;
  const int c = tid + RAD * N;  // this point in the window
  // window offsets of the x neighbours (wrapped inside the point's x line)
  const int xp1 = c + wrap_idx(i, 1, N) - i, xm1 = c + wrap_idx(i, -1, N) - i;
  const int xp2 = c + wrap_idx(i, 2, N) - i, xm2 = c + wrap_idx(i, -2, N) - i;
  // plane offsets of this thread's window elements tid + 256 u
  int woff[WPT];
  bool wv[WPT];
#pragma unroll
  for (int u = 0; u < WPT; ++u) {
    const int e = tid + 256 * u;
    wv[u] = e < W;
    int s2 = (q0 - RAD * N + e) % NN;
    woff[u] = s2 < 0 ? s2 + NN : s2;
  }
  const int k0 = kc * SZ;
  const int k1 = k0 + SZ < N ? k0 + SZ : N;
  S wr[WPT];
  auto wload = [&](int k) {
    const S* xp = x + (long)k * NN;
#pragma unroll
    for (int u = 0; u < WPT; ++u) wr[u] = wv[u] ? xp[woff[u]] : S{};
  };
  auto wstore = [&](S* buf) {
#pragma unroll
    for (int u = 0; u < WPT; ++u)
      if (wv[u]) buf[tid + 256 * u] = wr[u];
  };
  auto at = [&](int k) { return act ? x[q + (long)k * NN] : S{}; };
  auto vat = [&](int k) { return act ? V[q + (long)k * NN] : R{}; };
  // z register window: planes k - RAD .. k + RAD
  S zm2 = ORDER == 4 ? at(wrap_idx(k0, -2, N)) : S{};
  S zm1 = at(wrap_idx(k0, -1, N));
  S zc = at(k0);
  S zp1 = at(wrap_idx(k0, 1, N));
  S zp2 = ORDER == 4 ? at(wrap_idx(k0, 2, N)) : S{};
  R vc = vat(k0);
  wload(k0);
  wstore(win0);
  __syncthreads();
  for (int k = k0; k < k1; ++k) {
    const bool odd = ((k - k0) & 1) != 0;
    const S* cur = odd ? win1 : win0;
    const bool more = k + 1 < k1;
    S znew = S{};
    R vn = R{};
    if (more) {
      wload(k + 1);
      vn = vat(k + 1);
      znew = at(wrap_idx(k + 1, RAD, N));
    }
    if (act) {
      S s1 = phased<S>(cur[xp1], cur[xm1], a.ph[0][0]) + phased<S>(cur[c + N], cur[c - N], a.ph[1][0]) +
             phased<S>(zp1, zm1, a.ph[2][0]);
      S out = ((R)a.c0 + vc) * zc + (R)a.w1 * s1;
      if (ORDER == 4) {
        S s2 = phased<S>(cur[xp2], cur[xm2], a.ph[0][1]) + phased<S>(cur[c + 2 * N], cur[c - 2 * N], a.ph[1][1]) +
               phased<S>(zp2, zm2, a.ph[2][1]);
        out += (R)a.w2 * s2;
      }
      if (a.shift) out -= (R)a.shift[col] * zc;
      y[q + (long)k * NN] = out;
    }
    if (more) wstore(odd ? win0 : win1);
    __syncthreads();
    if (ORDER == 4) {
      zm2 = zm1;
      zm1 = zc;
      zc = zp1;
      zp1 = zp2;
      zp2 = znew;
    } else {
      zm1 = zc;
      zc = zp1;
      zp1 = znew;
    }
    vc = vn;
  }
}
// Vector variant for real columns (float or double) when N, the column
// strides and the pointers allow 16-byte access: a lane owns VEC = 16 /
// sizeof(S) consecutive points of one x line (N is a multiple of VEC), so the
// plane window, the z values entering the register window, V and the output
// move as 16-byte loads and stores, and a workgroup covers 256 VEC points of
// the plane.  The y neighbours are 16-byte LDS reads at +-N, +-2N; the x
// neighbours are the lane's own centre values plus one (13-point: two) LDS
// values at each end of its run, wrapped inside the x line.  Same pipeline as
// above: the loads of plane k + 1 are issued before plane k is computed, one
// barrier per plane; the last plane of a chunk is peeled so that the loop body
// has no conditional load.  Every global load is in bounds: window offsets are
// taken modulo the plane and idle lanes read their column's first run.
template <class S, int ORDER, int WPT>
__global__ __launch_bounds__(256) void stencil_vec_kernel(StencilArgs a) {
  constexpr int VEC = 16 / (int)sizeof(S);
  typedef S VT __attribute__((ext_vector_type(VEC)));
  extern __shared__ __align__(16) char smem[];
  constexpr int RAD = stencil_rad<ORDER>();
  constexpr int P = 256 * VEC;  // points of a plane per workgroup
  const int N = a.N;
  const int NN = N * N;
  const int W = P + 2 * RAD * N;  // window elements (a multiple of VEC)
  const int WV = W / VEC;         // window vectors, <= 256 WPT (checked by the launcher)
  S* const win0 = (S*)smem;
  S* const win1 = win0 + W;
  const unsigned tpp = (unsigned)((NN + P - 1) / P);
  const unsigned kch = (unsigned)((N + SZ - 1) / SZ);
  const unsigned L = xcd_remap(blockIdx.x, gridDim.x);
  const int col = (int)(L / (tpp * kch));
  const unsigned rest = L % (tpp * kch);
  const int kc = (int)(rest / tpp);
  const int q0 = (int)(rest % tpp) * P;
  if (col >= a.ncols) return;  // uniform over the workgroup
  const int tid = threadIdx.x;
  const int q = q0 + VEC * tid;  // first point of this lane's run
  const bool act = q < NN;       // NN is a multiple of VEC: a run is wholly inside or outside
  const int qa = act ? q : 0;
  const S* x = (const S*)a.X + (long)col * a.ldx;
  S* y = (S*)a.Y + (long)col * a.ldy;
  const S* V = (const S*)a.V;
  const int i0 = qa % N;           // x index of the run's first point; the run ends at i0 + VEC - 1 < N
  const int c = RAD * N + VEC * tid;  // window position of the run's first point
  const int xl1 = c + wrap_idx(i0, -1, N) - i0, xl2 = c + wrap_idx(i0, -2, N) - i0;
  const int xr1 = c + wrap_idx(i0 + VEC - 1, 1, N) - i0, xr2 = c + wrap_idx(i0 + VEC - 1, 2, N) - i0;
  int woff[WPT];
  bool wv[WPT];
#pragma unroll
  for (int u = 0; u < WPT; ++u) {
    const int e = tid + 256 * u;
    wv[u] = e < WV;
    const int s2 = (q0 - RAD * N + VEC * e) % NN;
    woff[u] = s2 < 0 ? s2 + NN : s2;  // a multiple of VEC, at most NN - VEC
  }
  const int k0 = kc * SZ;
  const int k1 = k0 + SZ < N ? k0 + SZ : N;
  VT wr[WPT];
  auto wload = [&](int k) {
    const S* xp = x + (long)k * NN;
#pragma unroll
    for (int u = 0; u < WPT; ++u) wr[u] = *(const VT*)(xp + woff[u]);
  };
  auto wstore = [&](S* buf) {
#pragma unroll
    for (int u = 0; u < WPT; ++u)
      if (wv[u]) *(VT*)(buf + VEC * (tid + 256 * u)) = wr[u];
  };
  auto at = [&](int k) { return *(const VT*)(x + qa + (long)k * NN); };
  auto vat = [&](int k) { return *(const VT*)(V + qa + (long)k * NN); };
  VT zm2 = ORDER == 4 ? at(wrap_idx(k0, -2, N)) : VT{};
  VT zm1 = at(wrap_idx(k0, -1, N));
  VT zc = at(k0);
  VT zp1 = at(wrap_idx(k0, 1, N));
  VT zp2 = ORDER == 4 ? at(wrap_idx(k0, 2, N)) : VT{};
  VT vc = vat(k0);
  wload(k0);
  wstore(win0);
  __syncthreads();
  auto compute = [&](int k, const S* cur) {
    if (!act) return;
    const VT yp1 = *(const VT*)(cur + c + N), ym1 = *(const VT*)(cur + c - N);
    VT yp2 = VT{}, ym2 = VT{};
    if (ORDER == 4) {
      yp2 = *(const VT*)(cur + c + 2 * N);
      ym2 = *(const VT*)(cur + c - 2 * N);
    }
    S e[VEC + 4];  // x line values at i0 - 2 .. i0 + VEC + 1
    e[0] = ORDER == 4 ? cur[xl2] : S{};
    e[1] = cur[xl1];
#pragma unroll
    for (int v = 0; v < VEC; ++v) e[2 + v] = zc[v];
    e[VEC + 2] = cur[xr1];
    e[VEC + 3] = ORDER == 4 ? cur[xr2] : S{};
    VT out;
#pragma unroll
    for (int v = 0; v < VEC; ++v) {
      const S s1 = (e[v + 3] + e[v + 1]) + (yp1[v] + ym1[v]) + (zp1[v] + zm1[v]);
      S o = ((S)a.c0 + vc[v]) * zc[v] + (S)a.w1 * s1;
      if (ORDER == 4) {
        const S s2 = (e[v + 4] + e[v]) + (yp2[v] + ym2[v]) + (zp2[v] + zm2[v]);
        o += (S)a.w2 * s2;
      }
      if (a.shift) o -= (S)a.shift[col] * zc[v];
      out[v] = o;
    }
    *(VT*)(y + q + (long)k * NN) = out;
  };
  auto advance = [&](VT znew, VT vn) {
    if (ORDER == 4) {
      zm2 = zm1;
      zm1 = zc;
      zc = zp1;
      zp1 = zp2;
      zp2 = znew;
    } else {
      zm1 = zc;
      zc = zp1;
      zp1 = znew;
    }
    vc = vn;
  };
  int k = k0;
  for (; k + 1 < k1; ++k) {
    const bool odd = ((k - k0) & 1) != 0;
    wload(k + 1);
    const VT vn = vat(k + 1);
    const VT znew = at(wrap_idx(k + 1, RAD, N));
    compute(k, odd ? win1 : win0);
    wstore(odd ? win0 : win1);
    __syncthreads();
    advance(znew, vn);
  }
  compute(k, ((k - k0) & 1) != 0 ? win1 : win0);
}

template <class S, int ORDER>
__global__ __launch_bounds__(256) void stencil_grouped(const StencilArgs* jobs, const unsigned* start, int nj) {
  int j = find_job(start, nj, blockIdx.x);
  stencil_body<S, ORDER>(jobs[j], blockIdx.x - start[j], start[j + 1] - start[j]);
}

static int stencil_kind(const StencilArgs& a) {
  int base = a.cplx ? (a.f32 ? OP_STENCIL_C2 : OP_STENCIL_Z2) : (a.f32 ? OP_STENCIL_F2 : OP_STENCIL_D2);
  // D2, D4 / F2, F4 / Z2, Z4 / C2, C4 are adjacent except D and F
  if (!a.cplx && a.f32) return a.order == 4 ? OP_STENCIL_F4 : OP_STENCIL_F2;
  if (!a.cplx) return a.order == 4 ? OP_STENCIL_D4 : OP_STENCIL_D2;
  return a.order == 4 ? base + 1 : base;
}

#define PPCG_STENCIL_SWITCH(KERNEL, GRID, ...)                                                                        \
  switch (kind) {                                                                                                    \
    case OP_STENCIL_D2: hipLaunchKernelGGL((KERNEL<double, 2>), dim3(GRID), dim3(256), 0, st, __VA_ARGS__); break;    \
    case OP_STENCIL_D4: hipLaunchKernelGGL((KERNEL<double, 4>), dim3(GRID), dim3(256), 0, st, __VA_ARGS__); break;    \
    case OP_STENCIL_F2: hipLaunchKernelGGL((KERNEL<float, 2>), dim3(GRID), dim3(256), 0, st, __VA_ARGS__); break;     \
    case OP_STENCIL_F4: hipLaunchKernelGGL((KERNEL<float, 4>), dim3(GRID), dim3(256), 0, st, __VA_ARGS__); break;     \
    case OP_STENCIL_Z2: hipLaunchKernelGGL((KERNEL<zdouble, 2>), dim3(GRID), dim3(256), 0, st, __VA_ARGS__); break;   \
    case OP_STENCIL_Z4: hipLaunchKernelGGL((KERNEL<zdouble, 4>), dim3(GRID), dim3(256), 0, st, __VA_ARGS__); break;   \
    case OP_STENCIL_C2: hipLaunchKernelGGL((KERNEL<zfloat, 2>), dim3(GRID), dim3(256), 0, st, __VA_ARGS__); break;    \
    case OP_STENCIL_C4: hipLaunchKernelGGL((KERNEL<zfloat, 4>), dim3(GRID), dim3(256), 0, st, __VA_ARGS__); break;    \
    default: break;                                                                                                  \
  }

#ifndef PPCG_STENCIL_LDS
#define PPCG_STENCIL_LDS 1
#endif
#ifndef PPCG_STENCIL_VEC
#define PPCG_STENCIL_VEC 1
#endif
#ifndef PPCG_STENCIL_LDS_MIN_ES
#define PPCG_STENCIL_LDS_MIN_ES 4
#endif

void launch_stencil(const StencilArgs& a, hipStream_t st) {
  const long NN = (long)a.N * a.N;
  unsigned blocks = (unsigned)(((NN + 255) / 256) * ((a.N + SZ - 1) / SZ) * (long)a.ncols);
  int kind = stencil_kind(a);
  if (g_rec) {  // grouped launches keep the register kernel (one LDS size for every job)
    g_rec->add(kind, &a, sizeof(a), blocks);
    return;
  }
  if (blocks == 0) return;
  const size_t es = (a.f32 ? 4 : 8) * (a.cplx ? 2 : 1);
  if (PPCG_STENCIL_VEC && !a.cplx && NN < (1L << 30)) {
    const int vec = 16 / (int)es;
    const int rad = a.order / 2;
    const long P = 256L * vec;
    const long Wv = P + 2L * rad * a.N;
    const long wpt = (Wv / vec + 255) / 256;
    const size_t lds = 2 * (size_t)Wv * es;
    const bool al = ((uintptr_t)a.X % 16 == 0) && ((uintptr_t)a.Y % 16 == 0) && ((uintptr_t)a.V % 16 == 0);
    if (al && a.N % vec == 0 && a.ldx % vec == 0 && a.ldy % vec == 0 && wpt <= 4 && lds <= 64 * 1024) {
      const unsigned vblocks = (unsigned)(((NN + P - 1) / P) * ((a.N + SZ - 1) / SZ) * (long)a.ncols);
#define PPCG_STENCIL_VEC_CASE(S, ORDER)                                                                            \
  switch (wpt) {                                                                                                   \
    case 1: hipLaunchKernelGGL((stencil_vec_kernel<S, ORDER, 1>), dim3(vblocks), dim3(256), lds, st, a); break;    \
    case 2: hipLaunchKernelGGL((stencil_vec_kernel<S, ORDER, 2>), dim3(vblocks), dim3(256), lds, st, a); break;    \
    case 3: hipLaunchKernelGGL((stencil_vec_kernel<S, ORDER, 3>), dim3(vblocks), dim3(256), lds, st, a); break;    \
    default: hipLaunchKernelGGL((stencil_vec_kernel<S, ORDER, 4>), dim3(vblocks), dim3(256), lds, st, a); break;   \
  }
      switch (kind) {
        case OP_STENCIL_D2: PPCG_STENCIL_VEC_CASE(double, 2) break;
        case OP_STENCIL_D4: PPCG_STENCIL_VEC_CASE(double, 4) break;
        case OP_STENCIL_F2: PPCG_STENCIL_VEC_CASE(float, 2) break;
        case OP_STENCIL_F4: PPCG_STENCIL_VEC_CASE(float, 4) break;
        default: break;
      }
#undef PPCG_STENCIL_VEC_CASE
      return;
    }
  }
  const int W = stencil_window(a.N, a.order);
  const size_t lds = 2 * (size_t)W * es;
  const int wpt = (W + 255) / 256;
  if (PPCG_STENCIL_LDS && es >= PPCG_STENCIL_LDS_MIN_ES && lds <= 64 * 1024 && wpt <= 4 && NN < (1L << 30)) {
#define PPCG_STENCIL_LDS_CASE(S, ORDER)                                                                            \
  switch (wpt) {                                                                                                   \
    case 1: hipLaunchKernelGGL((stencil_lds_kernel<S, ORDER, 1>), dim3(blocks), dim3(256), lds, st, a); break;     \
    case 2: hipLaunchKernelGGL((stencil_lds_kernel<S, ORDER, 2>), dim3(blocks), dim3(256), lds, st, a); break;     \
    case 3: hipLaunchKernelGGL((stencil_lds_kernel<S, ORDER, 3>), dim3(blocks), dim3(256), lds, st, a); break;     \
    default: hipLaunchKernelGGL((stencil_lds_kernel<S, ORDER, 4>), dim3(blocks), dim3(256), lds, st, a); break;    \
  }
    switch (kind) {
      case OP_STENCIL_D2: PPCG_STENCIL_LDS_CASE(double, 2) break;
      case OP_STENCIL_D4: PPCG_STENCIL_LDS_CASE(double, 4) break;
      case OP_STENCIL_F2: PPCG_STENCIL_LDS_CASE(float, 2) break;
      case OP_STENCIL_F4: PPCG_STENCIL_LDS_CASE(float, 4) break;
      case OP_STENCIL_Z2: PPCG_STENCIL_LDS_CASE(zdouble, 2) break;
      case OP_STENCIL_Z4: PPCG_STENCIL_LDS_CASE(zdouble, 4) break;
      case OP_STENCIL_C2: PPCG_STENCIL_LDS_CASE(zfloat, 2) break;
      case OP_STENCIL_C4: PPCG_STENCIL_LDS_CASE(zfloat, 4) break;
      default: break;
    }
#undef PPCG_STENCIL_LDS_CASE
    return;
  }
  PPCG_STENCIL_SWITCH(stencil_kernel, blocks, a)
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
    s += a.sum ? v : v * v;
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
void launch_colsum(const double* P, long ld, long rows, int ncols, double* out, hipStream_t st) {
  ColnormArgs a{P, 0, ld, rows, ncols, out, 1};
  unsigned blocks = ncols > 0 ? (unsigned)ncols : 0;
  if (g_rec) {
    g_rec->add(OP_COLNORM_D, &a, sizeof(a), blocks);
    return;
  }
  if (blocks == 0) return;
  hipLaunchKernelGGL(colnorm2_kernel<double>, dim3(blocks), dim3(256), 0, st, a);
}
void launch_colnorm2(const void* X, int f32, long ld, long rows, int ncols, double* out, hipStream_t st) {
  ColnormArgs a{X, f32, ld, rows, ncols, out, 0};
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
  double xb = a.X[r + c * a.ld];
  if (a.b) xb *= a.b[r >> a.bshift];
  double v = a.AX[r + c * a.ld] - xb * a.lam[c];
  if (a.W) a.W[r + c * a.ld] = v;
  if (a.W32) a.W32[r + c * a.ld] = (float)v;
}
__global__ __launch_bounds__(256) void ritz_kernel(RitzArgs a) { ritz_body(a, blockIdx.x, gridDim.x); }
__global__ __launch_bounds__(256) void ritz_grouped(const RitzArgs* jobs, const unsigned* start, int nj) {
  int j = find_job(start, nj, blockIdx.x);
  ritz_body(jobs[j], blockIdx.x - start[j], start[j + 1] - start[j]);
}
void launch_ritz_resid(const double* AX, const double* X, const double* lam, double* W, float* W32, long ld,
                       long rows, int ncols, hipStream_t st, const double* b, int bshift) {
  RitzArgs a{AX, X, lam, W, W32, ld, rows, ncols, b, bshift};
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
  if (kind >= OP_STENCIL_D2 && kind <= OP_STENCIL_C4) {
    PPCG_STENCIL_SWITCH(stencil_grouped, total, sj, start, nj)
    return true;
  }
  switch (kind) {
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
