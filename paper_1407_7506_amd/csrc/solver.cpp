// Host driver of libppcg: iteration control of the PPCG method (Algorithm 3
// of the paper, with the practical aspects of section 5), workspace, locking
// and the C ABI.  Every arithmetic step runs in the HIP kernels of this
// library; the host only decides control flow from a few scalars copied
// back per iteration.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <functional>
#include <map>
#include <string>
#include <vector>

#include "kernels.hpp"
#include "ppcg.h"
#include "prep.hpp"

using namespace ppcg;

namespace {

struct PpcgError {
  ppcg_status code;
  std::string msg;
};

#define HIPCHECK(x)                                                                   \
  do {                                                                                \
    hipError_t e_ = (x);                                                              \
    if (e_ != hipSuccess) throw PpcgError{PPCG_EHIP, std::string(#x) + ": " + hipGetErrorString(e_)}; \
  } while (0)

long round_up(long a, long b) { return (a + b - 1) / b * b; }

// ---------------------------------------------------------------------------
// device buffer that grows on demand
struct DBuf {
  void* p = nullptr;
  size_t bytes = 0;
  void ensure(size_t b) {
    if (b <= bytes) return;
    if (p) hipFree(p);
    p = nullptr;
    bytes = 0;
    if (b == 0) return;
    hipError_t e = hipMalloc(&p, b);
    if (e != hipSuccess) {
      p = nullptr;
      throw PpcgError{PPCG_ENOMEM, "hipMalloc of " + std::to_string(b) + " bytes failed"};
    }
    bytes = b;
  }
  void release() {
    if (p) hipFree(p);
    p = nullptr;
    bytes = 0;
  }
  double* d() const { return (double*)p; }
  float* f() const { return (float*)p; }
  int* i() const { return (int*)p; }
};

// ---------------------------------------------------------------------------
// per-kernel event timing (options.profile)
struct Prof {
  bool on = false;
  hipStream_t st = nullptr;
  std::vector<hipEvent_t> pool;
  struct Rec { int kind; hipEvent_t a, b; };
  std::vector<Rec> pending;
  std::vector<std::string> names;
  std::map<std::string, int> ids;
  std::vector<double> ms;
  std::vector<long> counts;
  std::vector<double> flops, bytes;
  struct Open { int kind; hipEvent_t ev; double fl, by; };
  std::vector<Open> open;
  hipEvent_t get() {
    if (!pool.empty()) {
      hipEvent_t e = pool.back();
      pool.pop_back();
      return e;
    }
    hipEvent_t e;
    HIPCHECK(hipEventCreate(&e));
    return e;
  }
  int id(const char* n) {
    auto it = ids.find(n);
    if (it != ids.end()) return it->second;
    int k = (int)names.size();
    names.push_back(n);
    ids[n] = k;
    ms.push_back(0);
    counts.push_back(0);
    flops.push_back(0);
    bytes.push_back(0);
    return k;
  }
  // fl / by: algorithmic flops and compulsory HBM bytes of the launch
  void begin(const char* n, double fl = 0, double by = 0) {
    if (!on) return;
    hipEvent_t e = get();
    HIPCHECK(hipEventRecord(e, st));
    open.push_back({id(n), e, fl, by});
  }
  void end() {
    if (!on || open.empty()) return;
    Open o = open.back();
    open.pop_back();
    hipEvent_t b = get();
    HIPCHECK(hipEventRecord(b, st));
    pending.push_back({o.kind, o.ev, b});
    flops[o.kind] += o.fl;
    bytes[o.kind] += o.by;
    if (pending.size() > 4096) collect();
  }
  void collect() {
    if (pending.empty()) return;
    HIPCHECK(hipStreamSynchronize(st));
    for (auto& r : pending) {
      float t = 0;
      HIPCHECK(hipEventElapsedTime(&t, r.a, r.b));
      ms[r.kind] += t;
      counts[r.kind] += 1;
      pool.push_back(r.a);
      pool.push_back(r.b);
    }
    pending.clear();
  }
  void reset() {
    collect();
    std::fill(ms.begin(), ms.end(), 0.0);
    std::fill(counts.begin(), counts.end(), 0L);
    std::fill(flops.begin(), flops.end(), 0.0);
    std::fill(bytes.begin(), bytes.end(), 0.0);
  }
  ~Prof() {
    for (auto e : pool) hipEventDestroy(e);
  }
};

struct Scope {
  Prof& p;
  Scope(Prof& p_, const char* n, double fl = 0, double by = 0) : p(p_) { p.begin(n, fl, by); }
  ~Scope() { p.end(); }
};

}  // namespace

struct ppcg_handle {
  hipStream_t st = nullptr;
  int device = 0;
  ppcg_options opt{};
  std::string err;
  Prof prof;
  // workspace
  DBuf X, Xt, W, P, AW, AP;           // float64 blocks (W..AP only in FP64 mode)
  DBuf X32, W32, P32, AW32, AP32;     // float32 blocks (mixed mode)
  DBuf AXm;                           // float64 H X kept in mixed mode
  DBuf Vd, V32, td;
  DBuf G, GWP, L, Li, Rinv, SAS, SS, V1, Mr, Yv, Cc, lam;
  DBuf part, bgram, bC, bflags, cn, scal, iflag, eigw, dminp;
  DBuf gZ, gR, gP, gAP, gY, gw, gsc;  // backward-pass work
  // state of the last successful solve (for ppcg_grad / ppcg_density)
  bool has_state = false;
  int s_N = 0, s_order = 0, s_k = 0;
  long s_n = 0, s_rows = 0;
  double s_c0 = 0, s_w1 = 0, s_w2 = 0, s_dmin = 0;
  int* hpin = nullptr;                // pinned host scratch
  double* hpind = nullptr;
  size_t hpin_bytes = 0;
  ~ppcg_handle() {
    for (DBuf* b : {&X, &Xt, &W, &P, &AW, &AP, &X32, &W32, &P32, &AW32, &AP32, &AXm, &Vd, &V32, &td, &G, &GWP, &L, &Li,
                    &Rinv, &SAS, &SS, &V1, &Mr, &Yv, &Cc, &lam, &part, &bgram, &bC, &bflags, &cn, &scal, &iflag,
                    &eigw, &dminp, &gZ, &gR, &gP, &gAP, &gY, &gw, &gsc})
      b->release();
    if (hpin) hipHostFree(hpin);
  }
  void pinned(size_t b) {
    if (b <= hpin_bytes) return;
    if (hpin) hipHostFree(hpin);
    hpin = nullptr;
    HIPCHECK(hipHostMalloc((void**)&hpin, b, hipHostMallocDefault));
    hpind = (double*)hpin;
    hpin_bytes = b;
  }
};

namespace {

// ---------------------------------------------------------------------------
// one solve
// ---------------------------------------------------------------------------
struct Solve {
  ppcg_handle* H;
  hipStream_t st;
  Prof& prof;
  // problem
  int N, order;
  double hsp, c0, w1, w2;
  long n, rows, ld;
  int k, q, K, Kp;
  double tol;
  int rr_period, max_iter;
  bool mixed;
  double dmin = 0;
  // state
  int nl = 0;        // locked columns (absolute prefix)
  bool hasP = false;
  std::vector<double> lock_wn, lock_lam;
  ppcg_info info{};

  Solve(ppcg_handle* h) : H(h), st(h->st), prof(h->prof) {}

  // Jacobi skip thresholds relative to |M|_F, tied to the requested tolerance:
  // the RR rotation error then stays ~1e-5 tol below the Ritz residuals that
  // decide locking, and the pencils resolve X-W couplings down to ~1e-4 tol.
  double rr_rel_tol() const { return std::max(2.2e-16, std::min(1e-11, 1e-5 * tol)); }
  double pencil_rel_tol() const { return std::max(2.2e-16, std::min(1e-10, 1e-4 * tol)); }

  double* X() { return H->X.d(); }
  double* Xt() { return H->Xt.d(); }
  void swapX() { std::swap(H->X, H->Xt); }

  // W/P/AW/AP storage (f64 in plain mode, f32 in mixed mode)
  void* Wb() { return mixed ? (void*)H->W32.p : H->W.p; }
  void* Pb() { return mixed ? (void*)H->P32.p : H->P.p; }
  void* AWb() { return mixed ? (void*)H->AW32.p : H->AW.p; }
  void* APb() { return mixed ? (void*)H->AP32.p : H->AP.p; }
  size_t esz() const { return mixed ? 4 : 8; }
  void* col(void* base, long c, size_t es) { return (char*)base + (size_t)c * ld * es; }

  // ---- kernels --------------------------------------------------------------
  void stencil(const void* Xs, void* Ys, int ncols, bool f32) {
    if (ncols <= 0) return;
    double es = f32 ? 4 : 8;
    Scope s(prof, f32 ? "stencil_f32" : "stencil_f64", (order == 4 ? 16.0 : 10.0) * n * ncols,
            2.0 * es * n * ncols + es * n);
    StencilArgs a{};
    a.X = Xs;
    a.Y = Ys;
    a.ldx = a.ldy = ld;
    a.ncols = ncols;
    a.N = N;
    a.order = order;
    a.c0 = c0;
    a.w1 = w1;
    a.w2 = w2;
    a.V = f32 ? (const void*)H->V32.p : (const void*)H->Vd.p;
    a.f32 = f32;
    launch_stencil(a, st);
  }

  static ColSet cols1(const void* p, int ncols, bool f32) {
    ColSet c{};
    c.p[0] = p;
    c.end[0] = ncols;
    c.f32[0] = f32;
    c.nseg = 1;
    return c;
  }

  static int site_of(const char* name) {
    if (!strcmp(name, "gram_proj") || !strcmp(name, "update_proj")) return 1;
    if (!strcmp(name, "gram_block")) return 2;
    return 0;
  }

  int pick_splits(long tiles, long njobs, long rws) {
    long target = 2048;
    long s = (target + tiles * njobs - 1) / (tiles * njobs);
    long maxs = std::max(1L, rws / 256);
    return (int)std::max(1L, std::min(s, maxs));
  }

  // dst (M x N, ldd) = A^H (D B) over `rws` rows; njobs strided jobs
  void gram(const ColSet& A, const ColSet& B, int M, int Nn, long rws, long ldab, const double* dsc, int nsc,
            void* dst, int ldd, bool upper, bool f32acc, int njobs = 1, long job_col_off = 0,
            long dst_job_stride = 0, const char* name = "gram") {
    if (M <= 0 || Nn <= 0) return;
    long tiles = (long)((M + 63) / 64) * ((Nn + 63) / 64);
    int splits = pick_splits(tiles, njobs, rws);
    size_t es = f32acc ? 4 : 8;
    size_t one = (size_t)njobs * M * Nn * es;
    if (one > H->part.bytes) throw PpcgError{PPCG_EINVAL, "internal: partial buffer too small"};
    splits = (int)std::min<size_t>((size_t)splits, H->part.bytes / one);
    long chunk = round_up((rws + splits - 1) / splits, 16);
    splits = (int)((rws + chunk - 1) / chunk);
    GramArgs g{};
    g.A = A;
    g.B = B;
    g.dsc = dsc;
    g.nsc = nsc;
    g.M = M;
    g.N = Nn;
    g.ld = ldab;
    g.rows = rws;
    g.splits = splits;
    g.chunk = chunk;
    g.out = H->part.p;
    g.split_stride = (long)M * Nn;
    g.ldo = M;
    g.upper_only = upper;
    g.job_col_off = job_col_off;
    {
      double nn = (double)std::min(rws, n), es_in = f32acc ? 4.0 : 8.0;
      double fl = upper ? (double)M * (M + 1) * nn : 2.0 * M * Nn * nn;
      double by = (double)njobs * (upper ? M : (M + Nn)) * nn * es_in;
      Scope s(prof, name, fl * njobs, by);
      g.site = site_of(name);
      launch_gram(g, njobs, f32acc, st);
    }
    ReduceArgs r{};
    r.part = H->part.p;
    r.M = M;
    r.N = Nn;
    r.ldp = M;
    r.splits = splits;
    r.split_stride = (long)M * Nn;
    r.njobs = njobs;
    r.dst = dst;
    r.ldd = ldd;
    r.dst_job_stride = dst_job_stride;
    r.alpha = 1.0;
    r.beta = 0.0;
    r.upper_only = upper;
    Scope s(prof, "reduce");
    launch_reduce(r, f32acc, st);
  }

  // C = beta (D C) + alpha A B
  void update(const void* A, long lda, int Kk, const void* B, long ldb, int Nn, void* C0, void* C1, int N0, long ldc,
              float* C32, const double* dsc, long rws, double alpha, double beta, bool b_upper, bool f32,
              const char* name = "update", bool c0_keep = false) {
    if (Nn <= 0 || rws <= 0) return;
    UpdateArgs u{};
    u.A = A;
    u.lda = lda;
    u.B = B;
    u.ldb = ldb;
    u.C0 = C0;
    u.C1 = C1;
    u.N0 = N0;
    u.ldc = ldc;
    u.C32 = C32;
    u.dsc = dsc;
    u.K = Kk;
    u.N = Nn;
    u.rows = rws;
    u.alpha = alpha;
    u.beta = beta;
    u.b_upper = b_upper;
    u.c0_keep = c0_keep;
    double nn = (double)std::min(rws, n), es = f32 ? 4.0 : 8.0;
    double fl = b_upper ? (double)Nn * (Nn + 1) * nn : 2.0 * Kk * Nn * nn;
    double by = ((double)Kk + Nn * (beta != 0 ? 2.0 : 1.0)) * nn * es + (C32 ? 4.0 * Nn * nn : 0.0);
    Scope s(prof, name, fl, by);
    u.site = site_of(name);
    launch_update(u, 1, f32, st);
  }

  // ---- set-up ---------------------------------------------------------------
  void allocate() {
    size_t nk8 = (size_t)rows * K * 8, nk4 = (size_t)rows * K * 4;
    H->X.ensure(nk8);
    H->Xt.ensure(nk8);
    if (mixed) {
      H->AXm.ensure(nk8);
      H->X32.ensure(nk4);
      H->W32.ensure(nk4);
      H->P32.ensure(nk4);
      H->AW32.ensure(nk4);
      H->AP32.ensure(nk4);
      H->V32.ensure((size_t)rows * 4);
    } else {
      H->W.ensure(nk8);
      H->P.ensure(nk8);
      H->AW.ensure(nk8);
      H->AP.ensure(nk8);
    }
    H->Vd.ensure((size_t)rows * 8);
    H->td.ensure((size_t)rows * 8);
    size_t kk = (size_t)Kp * Kp * 8;
    for (DBuf* b : {&H->G, &H->L, &H->Li, &H->Rinv, &H->SAS, &H->SS, &H->V1, &H->Mr, &H->Yv, &H->Cc})
      b->ensure(kk);
    H->GWP.ensure((size_t)Kp * 2 * K * 8);
    H->lam.ensure((size_t)Kp * 8);
    H->cn.ensure((size_t)Kp * 8);
    H->scal.ensure((size_t)Kp * 8 + 256);
    H->iflag.ensure(256);
    H->dminp.ensure(1024 * 8);
    int s = K / q;
    int nS = 3 * q;
    H->bgram.ensure((size_t)s * (nS + q) * (2 * nS - q) * 8);
    H->bC.ensure((size_t)s * 3 * q * q * 8);
    H->bflags.ensure((size_t)s * 4 + 256);
    H->eigw.ensure(eig_workspace_bytes(K));
    // split partials: the largest Gram of the run
    size_t need = 0;
    auto acc = [&](long M, long Nn, long njobs, long rws, size_t es) {
      long tiles = ((M + 63) / 64) * ((Nn + 63) / 64);
      int sp = pick_splits(tiles, njobs, rws);
      long chunk = round_up((rws + sp - 1) / sp, 16);
      sp = (int)((rws + chunk - 1) / chunk);
      need = std::max(need, (size_t)njobs * sp * M * Nn * es);
    };
    acc(K, 2 * K, 1, rows, mixed ? 4 : 8);
    acc(K, K, 1, rows, 8);
    acc(nS + q, 2 * nS - q, s, rows, 8);
    acc(K, K, 1, Kp, 8);
    H->part.ensure(need);
    H->pinned((size_t)(4 * Kp + 64) * 8);  // doubles [0, 2Kp), ints from 4Kp + 8
    // zero everything that carries padding rows
    std::vector<DBuf*> blocks = {&H->X, &H->Xt};
    if (mixed) {
      for (DBuf* b : {&H->X32, &H->W32, &H->P32, &H->AW32, &H->AP32, &H->AXm}) blocks.push_back(b);
    } else {
      for (DBuf* b : {&H->W, &H->P, &H->AW, &H->AP}) blocks.push_back(b);
    }
    for (DBuf* b : blocks) HIPCHECK(hipMemsetAsync(b->p, 0, b->bytes, st));
    for (DBuf* b : {&H->Vd, &H->td, &H->G, &H->L, &H->Li, &H->Rinv, &H->SAS, &H->SS, &H->V1, &H->Mr, &H->Yv,
                    &H->Cc, &H->GWP})
      HIPCHECK(hipMemsetAsync(b->p, 0, b->bytes, st));
    if (mixed) HIPCHECK(hipMemsetAsync(H->V32.p, 0, H->V32.bytes, st));
  }

  void prep(const double* V) {
    HIPCHECK(hipMemcpyAsync(H->Vd.p, V, n * 8, hipMemcpyDeviceToDevice, st));
    int nparts = 256;
    launch_zero_int(H->iflag.i(), 4, st);
    launch_prep_diag(H->Vd.d(), n, c0, H->td.d(), mixed ? H->V32.f() : nullptr, H->dminp.d(), nparts, H->iflag.i(),
                     st);
    HIPCHECK(hipMemcpyAsync(H->hpind, H->dminp.p, nparts * 8, hipMemcpyDeviceToHost, st));
    HIPCHECK(hipMemcpyAsync(H->hpin + 2 * nparts, H->iflag.p, 4, hipMemcpyDeviceToHost, st));
    HIPCHECK(hipStreamSynchronize(st));
    double mn = 1e308;
    for (int i = 0; i < nparts; ++i) mn = std::min(mn, H->hpind[i]);
    if (H->hpin[2 * nparts]) throw PpcgError{PPCG_EINVAL, "V contains NaN"};
    if (!(mn > 0)) throw PpcgError{PPCG_ENOTHPD, "diag(H) has a non-positive entry: Jacobi preconditioner not HPD"};
    dmin = mn;
  }

  // X (active columns c0.., m of them) <- X R^{-1}; result lands in Xt then X/Xt swap
  void cholqr(int m) {
    double* Xa = X() + (long)nl * ld;
    {
      ColSet A = cols1(Xa, m, false);
      gram(A, A, m, m, rows, ld, nullptr, 0, H->G.p, Kp, true, false, 1, 0, 0, "gram_xx");
    }
    launch_zero_int(H->iflag.i(), 4, st);
    {
      Scope s(prof, "chol_inverse");
      chol_inverse(H->G.d(), H->L.d(), H->Li.d(), m, Kp, H->iflag.i(), st);
      launch_transpose(H->Li.d(), Kp, H->Rinv.d(), Kp, m, m, st);
    }
    double* Xn = Xt() + (long)nl * ld;
    update(Xa, ld, m, H->Rinv.p, Kp, m, Xn, nullptr, m, ld, mixed ? H->X32.f() + (long)nl * ld : nullptr, nullptr,
           rows, 1.0, 0.0, true, false, "update_xr");
    if (nl > 0) HIPCHECK(hipMemcpyAsync(Xt(), X(), (size_t)nl * ld * 8, hipMemcpyDeviceToDevice, st));
    swapX();
  }

  // residual of the active columns: AX = H X, G = X^H AX, W = AX - X G.
  // plain: AX and W live in W; mixed: in Xt (f64), then W32 = (float) W.
  // Column norms of the wanted active columns go to cn.
  void residual(int m) {
    double* Xa = X() + (long)nl * ld;
    // plain: H X and then W overwrite the W block; mixed: H X stays in AXm (float64)
    // and only the float copy W32 of the residual is written
    double* R = mixed ? H->AXm.d() + (long)nl * ld : H->W.d() + (long)nl * ld;
    stencil(Xa, R, m, false);
    ColSet A = cols1(Xa, m, false), B = cols1(R, m, false);
    gram(A, B, m, m, rows, ld, nullptr, 0, H->G.p, Kp, true, false, 1, 0, 0, "gram_xax");
    float* W32a = mixed ? H->W32.f() + (long)nl * ld : nullptr;
    update(Xa, ld, m, H->G.p, Kp, m, R, nullptr, m, ld, W32a, nullptr, rows, -1.0, 1.0, false, false, "update_resid",
           mixed);
    int nwa = std::max(0, k - nl);
    {
      Scope s(prof, "colnorm");
      if (mixed) launch_colnorm2(W32a, 1, ld, rows, nwa, H->cn.d(), st);
      else launch_colnorm2(R, 0, ld, rows, nwa, H->cn.d(), st);
      launch_frob2_sub(H->G.d(), Kp, nwa, H->scal.d(), st);
    }
  }

  // rho of the loop head from the last residual (cn, scal) and locked parts
  double rho() {
    int nwa = std::max(0, k - nl);
    HIPCHECK(hipMemcpyAsync(H->hpind, H->cn.p, (size_t)std::max(nwa, 1) * 8, hipMemcpyDeviceToHost, st));
    HIPCHECK(hipMemcpyAsync(H->hpind + Kp, H->scal.p, (size_t)std::max(nwa, 1) * 8, hipMemcpyDeviceToHost, st));
    HIPCHECK(hipMemcpyAsync(H->hpin + 4 * Kp + 8, H->iflag.p, 4, hipMemcpyDeviceToHost, st));
    HIPCHECK(hipStreamSynchronize(st));
    if (H->hpin[4 * Kp + 8]) throw PpcgError{PPCG_ERANK, "Cholesky-QR breakdown (X^H X not positive definite)"};
    double num = 0, den = 0;
    for (int i = 0; i < nwa; ++i) {
      num += H->hpind[i];
      den += H->hpind[Kp + i];
    }
    for (size_t i = 0; i < lock_wn.size(); ++i) {
      num += lock_wn[i] * lock_wn[i];
      den += lock_lam[i] * lock_lam[i];
    }
    return den > 0 ? std::sqrt(num / den) : INFINITY;
  }

  // Rayleigh-Ritz over all K columns (S = [X_lock, X_act]), then W = H X - X Lambda
  // for all columns, the locking decision and the new active split.  Returns the
  // fresh residual of the k lowest pairs.
  double rayleigh_ritz() {
    double* S = X();
    double* AS = mixed ? H->AXm.d() : H->AW.d();
    stencil(S, AS, K, false);
    ColSet A = cols1(S, K, false);
    gram(A, cols1(AS, K, false), K, K, rows, ld, nullptr, 0, H->SAS.p, Kp, true, false, 1, 0, 0, "gram_rr");
    gram(A, A, K, K, rows, ld, nullptr, 0, H->SS.p, Kp, true, false, 1, 0, 0, "gram_rr");
    launch_zero_int(H->iflag.i(), 4, st);
    {
      Scope s(prof, "chol_inverse");
      chol_inverse(H->SS.d(), H->L.d(), H->Li.d(), K, Kp, H->iflag.i(), st);
      launch_transpose(H->Li.d(), Kp, H->Rinv.d(), Kp, K, K, st);  // Rinv = Linv^T
    }
    // Mr = Linv SAS Linv^T
    update(H->SAS.p, Kp, K, H->Rinv.p, Kp, K, H->V1.p, nullptr, K, Kp, nullptr, nullptr, Kp, 1.0, 0.0, true, false,
           "update_small");
    gram(cols1(H->Rinv.p, K, false), cols1(H->V1.p, K, false), K, K, Kp, Kp, nullptr, 0, H->Mr.p, Kp, false, false,
         1, 0, 0, "gram_small");
    launch_symmetrize(H->Mr.d(), Kp, K, st);
    HIPCHECK(hipMemcpyAsync(H->hpin, H->iflag.p, 4, hipMemcpyDeviceToHost, st));
    HIPCHECK(hipStreamSynchronize(st));
    if (H->hpin[0]) throw PpcgError{PPCG_ERANK, "Rayleigh-Ritz Gram S^H S not positive definite"};
    {
      Scope s(prof, "eig");
      block_jacobi_eig(H->Mr.d(), Kp, K, H->Yv.d(), Kp, H->lam.d(), H->eigw.p, H->hpin, rr_rel_tol(), st);
    }
    // C = Linv^T Y, X <- S C
    update(H->Rinv.p, Kp, K, H->Yv.p, Kp, K, H->Cc.p, nullptr, K, Kp, nullptr, nullptr, Kp, 1.0, 0.0, false, false,
           "update_small");
    update(S, ld, K, H->Cc.p, Kp, K, Xt(), nullptr, K, ld, mixed ? H->X32.f() : nullptr, nullptr, rows, 1.0, 0.0,
           false, false, "update_rot");
    swapX();
    // fresh residual W = H X - X Lambda (all K columns)
    double* R = mixed ? H->AXm.d() : H->W.d();
    stencil(X(), R, K, false);
    {
      Scope s(prof, "ritz_resid");
      if (mixed) {
        launch_ritz_resid(R, X(), H->lam.d(), nullptr, H->W32.f(), ld, rows, K, st);
        launch_colnorm2(H->W32.p, 1, ld, rows, K, H->cn.d(), st);
      } else {
        launch_ritz_resid(R, X(), H->lam.d(), R, nullptr, ld, rows, K, st);
        launch_colnorm2(R, 0, ld, rows, K, H->cn.d(), st);
      }
    }
    HIPCHECK(hipMemcpyAsync(H->hpind, H->cn.p, (size_t)K * 8, hipMemcpyDeviceToHost, st));
    HIPCHECK(hipMemcpyAsync(H->hpind + Kp, H->lam.p, (size_t)K * 8, hipMemcpyDeviceToHost, st));
    HIPCHECK(hipStreamSynchronize(st));
    const double* wn2 = H->hpind;
    const double* lam = H->hpind + Kp;
    double lk = 0, rk = 0;
    for (int i = 0; i < k; ++i) {
      lk += lam[i] * lam[i];
      rk += wn2[i];
    }
    double fresh = lk > 0 ? std::sqrt(rk / lk) : INFINITY;
    // locking: leading run of wanted Ritz vectors with |w_i| <= tol |Lambda_k|_F / (2 sqrt(k)),
    // rounded down to a multiple of q
    double thr = 0.5 * tol * std::sqrt(lk) / std::sqrt((double)k);
    int nlnew = 0;
    while (nlnew < k && std::sqrt(wn2[nlnew]) <= thr) ++nlnew;
    nlnew = nlnew / q * q;
    if (hasP && nlnew < nl) hasP = false;  // P(J_act) undefined when the locked set shrinks
    nl = nlnew;
    lock_wn.assign(nl, 0.0);
    lock_lam.assign(nl, 0.0);
    for (int i = 0; i < nl; ++i) {
      lock_wn[i] = std::sqrt(wn2[i]);
      lock_lam[i] = lam[i];
    }
    int m = K - nl;
    // active G = diag(Lambda_act); residual bookkeeping for rho
    launch_set_diag(H->G.d(), Kp, m, H->lam.d() + nl, st);
    int nwa = std::max(0, k - nl);
    HIPCHECK(hipMemcpyAsync(H->cn.p, H->cn.d() + nl, (size_t)std::max(nwa, 1) * 8, hipMemcpyDeviceToDevice, st));
    launch_frob2_sub(H->G.d(), Kp, nwa, H->scal.d(), st);
    info.n_rr++;
    return fresh;
  }

  // one PPCG iteration body (steps 8-31)
  void iteration(int it) {
    const int m = K - nl;
    const int s = m / q;
    const long off = (long)nl * ld;
    const size_t es = esz();
    void* Wa = col(Wb(), nl, es);
    void* Pa = col(Pb(), nl, es);
    void* AWa = col(AWb(), nl, es);
    void* APa = col(APb(), nl, es);
    // steps 8-10: precondition and project W and P against all K columns of X
    {
      ColSet A = cols1(mixed ? (const void*)H->X32.p : (const void*)X(), K, mixed);
      ColSet B{};
      B.p[0] = Wa;
      B.end[0] = m;
      B.f32[0] = mixed;
      B.nseg = 1;
      if (hasP) {
        B.p[1] = Pa;
        B.end[1] = 2 * m;
        B.f32[1] = mixed;
        B.nseg = 2;
      }
      int ncol = hasP ? 2 * m : m;
      gram(A, B, K, ncol, rows, ld, H->td.d(), m, H->GWP.p, Kp, false, mixed, 1, 0, 0, "gram_proj");
      const void* Xs = mixed ? (const void*)H->X32.p : (const void*)X();
      update(Xs, ld, K, H->GWP.p, Kp, ncol, Wa, Pa, m, ld, nullptr, H->td.d(), rows, -1.0, 1.0, false, mixed,
             "update_proj");
    }
    // AW = H W, AP = H P
    stencil(Wa, AWa, m, mixed);
    if (hasP) stencil(Pa, APa, m, mixed);
    // steps 11-13: per-block Grams and pencils
    const int nS = hasP ? 3 * q : 2 * q;
    {
      ColSet A{}, B{};
      const void* segs[5] = {X() + off, Wa, Pa, AWa, APa};
      bool f[5] = {false, mixed, mixed, mixed, mixed};
      int na = hasP ? 3 : 2;
      for (int t = 0; t < na; ++t) {
        A.p[t] = segs[t];
        A.end[t] = (t + 1) * q;
        A.f32[t] = f[t];
      }
      if (mixed) {  // rows (H X_j)^H [...] from the float64 H X
        A.p[na] = H->AXm.d() + off;
        A.end[na] = (na + 1) * q;
        A.f32[na] = false;
        ++na;
      }
      A.nseg = na;
      const int Ma = na * q;
      int bi = 0;
      for (int t = 0; t < 5; ++t) {
        if (!hasP && (t == 2 || t == 4)) continue;
        B.p[bi] = segs[t];
        B.end[bi] = (bi + 1) * q;
        B.f32[bi] = f[t];
        ++bi;
      }
      B.nseg = bi;
      int Nb = 2 * nS - q;
      gram(A, B, Ma, Nb, rows, ld, nullptr, 0, H->bgram.p, Ma, false, false, s, (long)q * ld, (long)Ma * Nb,
           "gram_block");
      PencilArgs pa{};
      pa.gram = H->bgram.d();
      pa.gstride = (long)Ma * Nb;
      pa.ax_rows = mixed;
      pa.G = H->G.d();
      pa.ldg = Kp;
      pa.q = q;
      pa.nS = nS;
      pa.C = H->bC.d();
      pa.cstride = 3L * q * q;
      pa.flags = H->bflags.i();
      pa.drop_tol = 1e-14;
      pa.pivot_tol = 1e-12;
      pa.jacobi_rel = pencil_rel_tol();
      Scope sc(prof, "block_pencil", 0, 0);
      launch_block_pencil(pa, s, st);
    }
    // steps 14-15
    {
      BlockUpdArgs bu{};
      bu.X = X() + off;
      bu.W = Wa;
      bu.P = Pa;
      bu.f32 = mixed;
      bu.hasP = hasP;
      bu.ld = ld;
      bu.rows = rows;
      bu.q = q;
      bu.C = H->bC.d();
      bu.cstride = 3L * q * q;
      Scope sc(prof, "block_update", 6.0 * (double)n * q * q * s * (hasP ? 1.0 : 2.0 / 3.0),
               (double)n * q * s * (hasP ? 5.0 : 4.0) * (double)esz());
      launch_block_update(bu, s, st);
    }
    hasP = true;
    // pencil flags: rank failures / backtracks
    HIPCHECK(hipMemcpyAsync(H->hpin, H->bflags.p, (size_t)s * 4, hipMemcpyDeviceToHost, st));
    HIPCHECK(hipStreamSynchronize(st));
    for (int j = 0; j < s; ++j) {
      if (H->hpin[j] & 4) throw PpcgError{PPCG_ERANK, "sub-block pencil has rank below sbsize"};
      if (H->hpin[j] & 2) info.n_backtrack++;
    }
    if (it % rr_period != 0) {
      cholqr(m);
      residual(m);
    } else {
      rayleigh_ritz();
    }
  }

  void finish(double* Xout, double* lamout, double fresh) {
    HIPCHECK(hipMemcpy2DAsync(Xout, (size_t)n * 8, X(), (size_t)ld * 8, (size_t)n * 8, k, hipMemcpyDeviceToDevice,
                              st));
    HIPCHECK(hipMemcpyAsync(lamout, H->lam.p, (size_t)k * 8, hipMemcpyDeviceToDevice, st));
    // orthogonality of the returned block
    ColSet A = cols1(X(), k, false);
    gram(A, A, k, k, rows, ld, nullptr, 0, H->G.p, Kp, false, false, 1, 0, 0, "gram_check");
    launch_orth_err2(H->G.d(), Kp, k, H->scal.d(), st);
    HIPCHECK(hipMemcpyAsync(H->hpind, H->scal.p, 8, hipMemcpyDeviceToHost, st));
    HIPCHECK(hipStreamSynchronize(st));
    info.orth_err = std::sqrt(H->hpind[0]);
    info.resid_final = fresh;
    info.n_locked = nl;
  }

  ppcg_status run(const ppcg_operator* op, int k_, int q_, double tol_, int rrp, const double* X0, double* Xout,
                  double* lamout) {
    auto t0 = std::chrono::steady_clock::now();
    if (!op || !op->V || !X0 || !Xout || !lamout) throw PpcgError{PPCG_EINVAL, "null pointer argument"};
    if (op->kpt[0] != 0 || op->kpt[1] != 0 || op->kpt[2] != 0)
      throw PpcgError{PPCG_EINVAL, "complex (Bloch) operators are not available in this build"};
    if (op->order != 2 && op->order != 4) throw PpcgError{PPCG_EINVAL, "order must be 2 or 4"};
    if (op->precond != PPCG_PRECOND_JACOBI) throw PpcgError{PPCG_EINVAL, "only the Jacobi preconditioner"};
    if (op->nx < 4 || !(op->h > 0)) throw PpcgError{PPCG_EINVAL, "bad grid"};
    N = op->nx;
    order = op->order;
    hsp = op->h;
    double ih2 = 1.0 / (hsp * hsp);
    if (order == 2) {
      c0 = 3.0 * ih2;
      w1 = -0.5 * ih2;
      w2 = 0;
    } else {
      c0 = 3.0 * 1.25 * ih2;
      w1 = -2.0 / 3.0 * ih2;
      w2 = ih2 / 24.0;
    }
    n = (long)N * N * N;
    rows = round_up(n, 256);
    ld = rows;
    k = k_;
    q = q_;
    tol = tol_;
    rr_period = rrp;
    mixed = H->opt.precision == PPCG_MIXED;
    max_iter = H->opt.max_iter > 0 ? H->opt.max_iter : 20000;
    if (k <= 0 || q < 1 || q > 16 || !(tol > 0) || rr_period < 1)
      throw PpcgError{PPCG_EINVAL, "need k > 0, 1 <= sbsize <= 16, tol > 0, rr_period >= 1"};
    int nbuf = H->opt.nbuf;
    if (nbuf < 0) {
      int extra = std::max(2, (int)std::ceil(0.02 * k));
      nbuf = q * ((k + extra + q - 1) / q) - k;
    }
    K = k + nbuf;
    if (K % q != 0) throw PpcgError{PPCG_EINVAL, "k + nbuf must be a multiple of sbsize"};
    if ((long)K * 4 > n) throw PpcgError{PPCG_EINVAL, "k + nbuf must not exceed n/4"};
    Kp = (int)round_up(K, 64);
    H->has_state = false;
    allocate();
    prep(op->V);
    HIPCHECK(hipMemcpy2DAsync(X(), (size_t)ld * 8, X0, (size_t)n * 8, (size_t)n * 8, K, hipMemcpyDeviceToDevice, st));
    // steps 1-4: orthonormal start and first residual
    nl = 0;
    hasP = false;
    cholqr(K);
    if (mixed) {
      // X32 for the projections (cholqr wrote the active part, i.e. all K)
    }
    residual(K);
    int it = 1;
    double fresh = INFINITY;
    ppcg_status status = PPCG_OK;
    while (true) {
      double r = rho();
      if (r <= tol) {
        fresh = rayleigh_ritz();
        if (fresh <= tol) break;
        continue;
      }
      if (it > max_iter) {
        fresh = rayleigh_ritz();
        status = PPCG_ENOCONV;
        break;
      }
      iteration(it);
      info.iters = it;
      ++it;
    }
    finish(Xout, lamout, fresh);
    prof.collect();
    if (status == PPCG_OK) {
      H->has_state = true;
      H->s_N = N;
      H->s_order = order;
      H->s_k = k;
      H->s_n = n;
      H->s_rows = rows;
      H->s_c0 = c0;
      H->s_w1 = w1;
      H->s_w2 = w2;
      H->s_dmin = dmin;
    }
    info.time_s = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
    if (status == PPCG_ENOCONV) H->err = "max_iter reached";
    return status;
  }
};

// ---------------------------------------------------------------------------
// backward pass: projected Sternheimer systems by block PCG
// ---------------------------------------------------------------------------
struct Grad {
  ppcg_handle* H;
  hipStream_t st;
  Prof& prof;
  int k;
  long n, rows, ld;
  Grad(ppcg_handle* h) : H(h), st(h->st), prof(h->prof) {}

  // Y <- (I - X X^H) Y over the k saved eigenvectors
  void project(double* Y) {
    Solve s(H);
    s.n = n;
    s.rows = rows;
    s.ld = ld;
    ColSet A = Solve::cols1(H->X.p, k, false), B = Solve::cols1(Y, k, false);
    s.gram(A, B, k, k, rows, ld, nullptr, 0, H->gsc.p, (int)round_up(k, 64), false, false, 1, 0, 0, "gram_grad");
    s.update(H->X.p, ld, k, H->gsc.p, round_up(k, 64), k, Y, nullptr, k, ld, nullptr, nullptr, rows, -1.0, 1.0,
             false, false, "update_grad");
  }
  void stencil_shift(const double* P, double* Y) {
    StencilArgs a{};
    a.X = P;
    a.Y = Y;
    a.ldx = a.ldy = ld;
    a.ncols = k;
    a.N = H->s_N;
    a.order = H->s_order;
    a.c0 = H->s_c0;
    a.w1 = H->s_w1;
    a.w2 = H->s_w2;
    a.V = H->Vd.p;
    a.f32 = 0;
    a.shift = H->lam.d();
    Scope sc(prof, "stencil_f64", (H->s_order == 4 ? 17.0 : 11.0) * n * k, 16.0 * n * k);
    launch_stencil(a, st);
  }

  int run(const double* g, const double* w, double* out, double tol, int max_iter) {
    if (!H->has_state) throw PpcgError{PPCG_ENOSTATE, "ppcg_grad needs a successful ppcg_solve on this handle"};
    if (!g || !out || !(tol > 0)) throw PpcgError{PPCG_EINVAL, "null pointer or tol <= 0"};
    k = H->s_k;
    n = H->s_n;
    rows = H->s_rows;
    ld = rows;
    if (!w) {
      launch_grad_rows(H->X.d(), nullptr, g, ld, n, k, out, st);
      HIPCHECK(hipStreamSynchronize(st));
      return 0;
    }
    const size_t blk = (size_t)rows * k * 8;
    for (DBuf* b : {&H->gZ, &H->gR, &H->gP, &H->gAP, &H->gY}) b->ensure(blk);
    H->gw.ensure((size_t)rows * 8);
    int kp = (int)round_up(k, 64);
    H->gsc.ensure((size_t)kp * kp * 8 + (size_t)16 * kp * 8);
    double* sc = H->gsc.d() + (size_t)kp * kp;  // per-column scalars
    double *rz = sc, *rznew = sc + kp, *pAp = sc + 2 * kp, *alpha = sc + 3 * kp, *beta = sc + 4 * kp,
           *bb = sc + 5 * kp, *rr = sc + 6 * kp;
    int* done = (int*)(sc + 7 * kp);
    int* left = (int*)(sc + 8 * kp);
    // the partial buffer must hold a k x k Gram
    H->part.ensure((size_t)k * k * 8 * 4);
    HIPCHECK(hipMemsetAsync(H->gw.p, 0, H->gw.bytes, st));
    HIPCHECK(hipMemcpyAsync(H->gw.p, w, n * 8, hipMemcpyDeviceToDevice, st));
    double *Z = H->gZ.d(), *R = H->gR.d(), *P = H->gP.d(), *AP = H->gAP.d(), *Y = H->gY.d();
    // b = Q (w x_i)
    launch_scale_rows(H->gw.d(), H->X.p, R, ld, rows, k, 0, st);
    project(R);
    launch_coldot(R, R, ld, rows, k, bb, st);
    launch_fill(Z, (long)rows * k, 0.0, st);
    launch_zero_int(done, k, st);
    // Jacobi preconditioner 1/(diag(H) - lambda_i) when it is positive definite
    HIPCHECK(hipMemcpyAsync(H->hpind, H->lam.p, (size_t)k * 8, hipMemcpyDeviceToHost, st));
    HIPCHECK(hipStreamSynchronize(st));
    double lmax = -1e308;
    for (int j = 0; j < k; ++j) lmax = std::max(lmax, H->hpind[j]);
    int unprec = !(H->s_dmin - lmax > 0);
    auto precond = [&]() {
      launch_cg_precond(R, Y, H->Vd.d(), H->s_c0, H->lam.d(), ld, n, rows, k, unprec, st);
      project(Y);
    };
    precond();
    HIPCHECK(hipMemcpyAsync(P, Y, blk, hipMemcpyDeviceToDevice, st));
    launch_coldot(R, Y, ld, rows, k, rz, st);
    int it = 0;
    for (; it < max_iter; ++it) {
      stencil_shift(P, AP);
      project(AP);
      launch_coldot(P, AP, ld, rows, k, pAp, st);
      launch_cg_alpha(rz, pAp, done, alpha, k, st);
      launch_cg_xr(Z, R, P, AP, alpha, ld, rows, k, st);
      launch_coldot(R, R, ld, rows, k, rr, st);
      launch_zero_int(left, 1, st);
      launch_cg_check(rr, bb, tol, done, left, k, st);
      if (it % 4 == 3 || it == max_iter - 1) {
        HIPCHECK(hipMemcpyAsync(H->hpin, left, 4, hipMemcpyDeviceToHost, st));
        HIPCHECK(hipStreamSynchronize(st));
        if (H->hpin[0] == 0) {
          ++it;
          break;
        }
      }
      precond();
      launch_coldot(R, Y, ld, rows, k, rznew, st);
      launch_cg_beta(rz, rznew, done, beta, k, st);
      launch_cg_p(P, Y, beta, ld, rows, k, st);
    }
    launch_grad_rows(H->X.d(), Z, g, ld, n, k, out, st);
    HIPCHECK(hipStreamSynchronize(st));
    prof.collect();
    return it;
  }
};

ppcg_status guard(ppcg_handle* h, const std::function<ppcg_status()>& f) {
  try {
    if (h) HIPCHECK(hipSetDevice(h->device));
    return f();
  } catch (const PpcgError& e) {
    if (h) h->err = e.msg;
    return e.code;
  } catch (const std::exception& e) {
    if (h) h->err = e.what();
    return PPCG_EHIP;
  }
}

}  // namespace

extern "C" {

ppcg_status ppcg_create(ppcg_handle** out, const ppcg_options* opt, void* stream) {
  if (!out) return PPCG_EINVAL;
  ppcg_handle* h = new ppcg_handle();
  if (hipGetDevice(&h->device) != hipSuccess) {
    delete h;
    return PPCG_EHIP;
  }
  h->st = (hipStream_t)stream;
  if (opt) h->opt = *opt;
  else {
    h->opt.precision = PPCG_FP64;
    h->opt.nbuf = -1;
    h->opt.max_iter = 20000;
    h->opt.profile = 0;
  }
  if (h->opt.precision != PPCG_FP64 && h->opt.precision != PPCG_MIXED) {
    delete h;
    return PPCG_EINVAL;
  }
  h->prof.on = h->opt.profile != 0;
  h->prof.st = h->st;
  *out = h;
  return PPCG_OK;
}

ppcg_status ppcg_solve(ppcg_handle* h, const ppcg_operator* op, int32_t k, int32_t sbsize, double tol,
                       int32_t rr_period, const double* X0, double* X_out, double* lambda_out, ppcg_info* info) {
  if (!h) return PPCG_EINVAL;
  return guard(h, [&]() {
    Solve s(h);
    ppcg_status st = PPCG_OK;
    try {
      st = s.run(op, k, sbsize, tol, rr_period, X0, X_out, lambda_out);
    } catch (...) {
      if (info) *info = s.info;
      throw;
    }
    if (info) *info = s.info;
    return st;
  });
}

ppcg_status ppcg_grad(ppcg_handle* h, const double* g_lambda, const double* w, double* dL_dV, double tol,
                      int32_t max_iter, int32_t* iters) {
  if (!h) return PPCG_EINVAL;
  return guard(h, [&]() {
    Grad g(h);
    int it = g.run(g_lambda, w, dL_dV, tol, max_iter > 0 ? max_iter : 10000);
    if (iters) *iters = it;
    return PPCG_OK;
  });
}

ppcg_status ppcg_density(ppcg_handle* h, double* rho) {
  if (!h || !rho) return PPCG_EINVAL;
  return guard(h, [&]() {
    if (!h->has_state) throw PpcgError{PPCG_ENOSTATE, "ppcg_density needs a successful ppcg_solve on this handle"};
    launch_grad_rows(h->X.d(), nullptr, nullptr, h->s_rows, h->s_n, h->s_k, rho, h->st);
    HIPCHECK(hipGetLastError());
    HIPCHECK(hipStreamSynchronize(h->st));
    return PPCG_OK;
  });
}

int32_t ppcg_columns(const ppcg_handle* h, int32_t k, int32_t sbsize) {
  if (!h || k <= 0 || sbsize < 1) return -1;
  int nbuf = h->opt.nbuf;
  if (nbuf < 0) {
    int extra = std::max(2, (int)std::ceil(0.02 * k));
    nbuf = sbsize * ((k + extra + sbsize - 1) / sbsize) - k;
  }
  return k + nbuf;
}

ppcg_status ppcg_apply_h(ppcg_handle* h, const ppcg_operator* op, int32_t ncols, const double* X, double* Y) {
  if (!h || !op || !op->V || !X || !Y || ncols < 0) return PPCG_EINVAL;
  return guard(h, [&]() {
    if (op->order != 2 && op->order != 4) throw PpcgError{PPCG_EINVAL, "order must be 2 or 4"};
    if (op->kpt[0] != 0 || op->kpt[1] != 0 || op->kpt[2] != 0)
      throw PpcgError{PPCG_EINVAL, "complex (Bloch) operators are not available in this build"};
    Solve s(h);
    s.N = op->nx;
    s.order = op->order;
    double ih2 = 1.0 / (op->h * op->h);
    s.c0 = op->order == 2 ? 3.0 * ih2 : 3.75 * ih2;
    s.w1 = op->order == 2 ? -0.5 * ih2 : -2.0 / 3.0 * ih2;
    s.w2 = op->order == 2 ? 0.0 : ih2 / 24.0;
    s.n = (long)s.N * s.N * s.N;
    s.ld = s.n;
    StencilArgs a{};
    a.X = X;
    a.Y = Y;
    a.ldx = a.ldy = s.n;
    a.ncols = ncols;
    a.N = s.N;
    a.order = s.order;
    a.c0 = s.c0;
    a.w1 = s.w1;
    a.w2 = s.w2;
    a.V = op->V;
    a.f32 = 0;
    {
      Scope sc(h->prof, "stencil_f64");
      launch_stencil(a, h->st);
    }
    HIPCHECK(hipGetLastError());
    HIPCHECK(hipStreamSynchronize(h->st));
    return PPCG_OK;
  });
}

int32_t ppcg_kernel_stats(ppcg_handle* h, const char** names, double* ms, int64_t* counts, double* flops,
                          double* bytes, int32_t cap) {
  if (!h) return 0;
  int32_t w = ppcg_kernel_times(h, names, ms, counts, cap);
  for (int32_t i = 0; i < w; ++i) {
    if (flops) flops[i] = h->prof.flops[i];
    if (bytes) bytes[i] = h->prof.bytes[i];
  }
  return w;
}

int32_t ppcg_kernel_times(ppcg_handle* h, const char** names, double* ms, int64_t* counts, int32_t cap) {
  if (!h) return 0;
  try {
    h->prof.collect();
  } catch (...) {
    return 0;
  }
  int32_t nk = (int32_t)h->prof.names.size();
  int32_t w = std::min(nk, cap);
  for (int32_t i = 0; i < w; ++i) {
    if (names) names[i] = h->prof.names[i].c_str();
    if (ms) ms[i] = h->prof.ms[i];
    if (counts) counts[i] = h->prof.counts[i];
  }
  return w;
}

void ppcg_reset_kernel_times(ppcg_handle* h) {
  if (!h) return;
  try {
    h->prof.reset();
  } catch (...) {
  }
}

void ppcg_destroy(ppcg_handle* h) { delete h; }

const char* ppcg_last_error(const ppcg_handle* h) { return h ? h->err.c_str() : "null handle"; }

}  // extern "C"
