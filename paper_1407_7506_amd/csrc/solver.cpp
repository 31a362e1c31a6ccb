// Host driver of libppcg: iteration control of the PPCG method (Algorithm 3
// of the paper, with the practical aspects of section 5), workspace, locking
// and the C ABI.  Every arithmetic step runs in the HIP kernels of this
// library; the host only decides control flow from a few scalars copied
// back per iteration.
//
// One problem (`Prob`) is a sequence of enqueue phases (no synchronisation
// inside) and post-phase host logic.  The `Driver` advances a set of
// problems in lockstep: a single solve launches every kernel directly; a
// batched solve records each phase for all problems and replays it as one
// grouped launch per kernel and position (see kernels.hpp).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <functional>
#include <cstdio>
#include <map>
#include <tuple>
#include <memory>
#include <string>
#include <vector>

#include "kernels.hpp"
#include "ppcg.h"

#include <mutex>

using namespace ppcg;

// Scratch of ppcg_block_pencils_noalloc, for callers that cannot allocate
// device memory: a static array that every GPU the library runs on holds
// until the process ends (each GPU its own copy, at its own address).  Host
// code must use the address hipGetSymbolAddress returns for the current
// device, never the array's name (a host-side stand-in).  Calls that overlap
// on one GPU share it and race.
constexpr size_t NOALLOC_SCRATCH_BYTES = (size_t)32 << 20;
static __device__ __align__(256) char scratch[NOALLOC_SCRATCH_BYTES];

namespace {
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_ptr[kMaxDevices] = {};

// device address of `scratch` on `device` (which must be current), resolved
// once per device
hipError_t resolve_scratch(int device, void** out) {
  if (device < 0 || device >= kMaxDevices) return hipErrorInvalidDevice;
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (!g_scratch_ptr[device]) {
    void* p = nullptr;
    hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    g_scratch_ptr[device] = p;
  }
  *out = g_scratch_ptr[device];
  return hipSuccess;
}
}  // namespace

namespace {

struct PpcgError {
  ppcg_status code;
  std::string msg;
};

#define HIPCHECK(x)                                                                                      \
  do {                                                                                                   \
    hipError_t e_ = (x);                                                                                 \
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
  ~DBuf() { release(); }
  double* d() const { return (double*)p; }
  float* f() const { return (float*)p; }
  int* i() const { return (int*)p; }
};

// ---------------------------------------------------------------------------
// per-kernel event timing (options.profile)

// MI355X peaks of the per-launch roofline time: HBM and dense MFMA by dtype
constexpr double PEAK_HBM = 8.0e12, PEAK_F64 = 78.6e12, PEAK_F32 = 157.3e12;

// time categories of the paper's breakdown (section 6, Tables 4-5)
enum { CAT_GEMM = 0, CAT_AX = 1, CAT_RR = 2, CAT_CHOLQR = 3, CAT_SMALL = 4, CAT_OTHER = 5, NCAT = 6 };

struct Prof {
  bool on = false;
  hipStream_t st = nullptr;
  int ctx = -1;  // category of launches whose name does not fix one (Cholesky, reductions)
  std::vector<hipEvent_t> pool;
  struct Rec { int kind, cat; hipEvent_t a, b; };
  std::vector<Rec> pending;
  std::vector<std::string> names;
  std::map<std::string, int> ids;
  std::vector<double> ms;
  std::vector<long> counts;
  std::vector<double> flops, bytes;
  double cat_ms[NCAT] = {};
  double roof_ms = 0;  // sum over launches of max(bytes / HBM peak, flops / MFMA peak)
  struct Open { int kind, cat; hipEvent_t ev; double fl, by; };
  std::vector<Open> open;
  static int cat_of_name(const char* n) {
    static const std::map<std::string, int> m = {
        {"stencil_f64", CAT_AX},     {"stencil_f32", CAT_AX},     {"block_pencil", CAT_SMALL},
        {"gram_proj", CAT_GEMM},     {"update_proj", CAT_GEMM},   {"gram_block", CAT_GEMM},
        {"block_update", CAT_GEMM},  {"gram_xax", CAT_GEMM},      {"update_resid", CAT_GEMM},
        {"gram_rr", CAT_RR},         {"update_small", CAT_RR},    {"gram_small", CAT_RR},
        {"eig", CAT_RR},             {"update_rot", CAT_RR},      {"ritz_resid", CAT_RR},
        {"gram_xx", CAT_CHOLQR},     {"update_xr", CAT_CHOLQR}};
    auto it = m.find(n);
    return it == m.end() ? -1 : it->second;
  }
  // the category a launch named n is charged to
  int cat_of(const char* n) const {
    int c = cat_of_name(n);
    if (c >= 0) return c;
    return ctx >= 0 ? ctx : CAT_OTHER;
  }
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
  // events are only recorded around real launches (not while recording a batch)
  bool active() const { return on && g_rec == nullptr; }
  // fl / by: algorithmic flops and compulsory HBM bytes of the launch
  // recording a batch: the next recorded op carries this work model
  void note(const char* n, double fl, double by) {
    if (!on || !g_rec) return;
    g_rec->pend_name = (fl + by > 0) ? n : nullptr;
    g_rec->pend_fl = fl;
    g_rec->pend_by = by;
  }
  // peak: dense MFMA rate of the launch's dtype (flops / s)
  void begin(const char* n, double fl = 0, double by = 0, double peak = PEAK_F64, int cat = -1) {
    if (!active()) return;
    hipEvent_t e = get();
    HIPCHECK(hipEventRecord(e, st));
    open.push_back({id(n), cat >= 0 ? cat : cat_of(n), e, fl, by});
    roof_ms += 1e3 * std::max(by / PEAK_HBM, fl / peak);
  }
  void end() {
    if (!active() || open.empty()) return;
    Open o = open.back();
    open.pop_back();
    hipEvent_t b = get();
    HIPCHECK(hipEventRecord(b, st));
    pending.push_back({o.kind, o.cat, o.ev, b});
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
      cat_ms[r.cat] += t;
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
    std::fill(cat_ms, cat_ms + NCAT, 0.0);
    roof_ms = 0;
  }
  ~Prof() {
    for (auto e : pool) hipEventDestroy(e);
  }
};

struct Scope {
  Prof& p;
  bool live;
  Scope(Prof& p_, const char* n, double fl = 0, double by = 0, double peak = PEAK_F64, int cat = -1)
      : p(p_), live(p_.active()) {
    if (live) p.begin(n, fl, by, peak, cat);
    else p.note(n, fl, by);
  }
  ~Scope() {
    if (live) p.end();
    else p.note(nullptr, 0, 0);
  }
};

// charges launches without a category of their own (Cholesky, reductions) to cat
struct CatCtx {
  Prof& p;
  int old;
  CatCtx(Prof& p_, int cat) : p(p_), old(p_.ctx) { p.ctx = cat; }
  ~CatCtx() { p.ctx = old; }
};

// per-problem workspace
struct Work {
  DBuf X, Xt, W, P, AW, AP;           // float64 blocks (W..AP only in FP64 mode)
  DBuf X32, W32, P32, AW32, AP32;     // float32 blocks (mixed mode)
  DBuf AXm;                           // float64 H X kept in mixed mode
  DBuf Vd, V32, td;
  DBuf Bd, btd;                       // generalized problem: diag(B) and B T (padding rows zero)
  DBuf G, GWP, L, Li, Rinv, SAS, SS, V1, Mr, Yv, Cc, lam;
  DBuf part, bgram, bC, bflags, cn, scal, iflag, eigw, dminp, pwork, cpart, G32;
  int* hpin = nullptr;                // pinned host scratch: doubles [0, 2Kp), ints from 4Kp + 8
  double* hpind = nullptr;
  size_t hpin_bytes = 0;
  ~Work() {
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

}  // namespace

// Autotuner table: the fastest kernel variant and row-split schedule found
// for each shape class (powers-of-two buckets of the operand sizes).
struct TuneKey {
  int kind;     // 0 Gram, 1 update, 2 16-column block Grams
  int site;     // Gram call site (0 plain, 1 projection, 2 per-block); -1 for updates
  int f32, cplx, multi, upper;
  int mb, nb;   // buckets of M x N (Gram) or K x N (update)
  long rb;      // bucket of the rows
  bool operator<(const TuneKey& o) const {
    return std::tie(kind, site, f32, cplx, multi, upper, mb, nb, rb) <
           std::tie(o.kind, o.site, o.f32, o.cplx, o.multi, o.upper, o.mb, o.nb, o.rb);
  }
};
struct TuneChoice {
  int lds = 0;          // LDS-staged 128 x 128 kernel
  int target = 2048;    // workgroups aimed at (Gram row splits)
  int floor_rows = 256; // no fewer rows per split
  double ms = 0;        // time of the chosen candidate
  std::string tried;    // every candidate and its time
};

struct ppcg_handle {
  hipStream_t st = nullptr;
  int device = 0;
  ppcg_options opt{};
  std::string err;
  Prof prof;
  Stage stage;
  std::vector<std::unique_ptr<Work>> works;
  DBuf counter;                       // rotation counter of the grouped eigensolver
  int* hcounter = nullptr;
  EigGraphCache eig_graph;            // captured block-Jacobi sweep
  std::map<TuneKey, TuneChoice> tune; // autotuner decisions (PPCG_AUTOTUNE)
  std::string tune_path;              // options.tune_table (empty: none)
  size_t tune_saved = 0;              // entries the file holds
  DBuf tune_scratch;                  // output copy for timing non-idempotent updates
  hipEvent_t tev[2] = {nullptr, nullptr};
  DBuf gZ, gR, gP, gAP, gY, gw, gsc;  // backward-pass work
  DBuf pen_gram, pen_G, pen_work;     // ppcg_block_pencils inputs in the solver's pencil layout
  void* noalloc_scratch = nullptr;    // this device's copy of `scratch` (ppcg_block_pencils_noalloc)
  // state of the last successful single solve (for ppcg_grad / ppcg_density)
  bool has_state = false;
  bool s_cplx = false;
  int s_N = 0, s_order = 0, s_k = 0;
  long s_n = 0, s_rows = 0, s_ld = 0;
  double s_c0 = 0, s_w1 = 0, s_w2 = 0, s_dmin = 0;
  double s_ph[3][2][2] = {};          // Bloch phases of that solve's operator
  bool s_gen = false;                 // that solve was a generalized problem (H x = lambda B x)
  ~ppcg_handle() {
    if (hcounter) hipHostFree(hcounter);
    for (hipEvent_t e : tev)
      if (e) hipEventDestroy(e);
  }
  Work& work(int i) {
    while ((int)works.size() <= i) works.emplace_back(new Work());
    return *works[i];
  }
};

namespace {

void sync(ppcg_handle* H) {
  HIPCHECK(hipStreamSynchronize(H->st));
  H->stage.reset();
}

// ---------------------------------------------------------------------------
// one problem
// ---------------------------------------------------------------------------
// Bloch phases exp(i kappa_d a h) of the couplings at distance a = 1, 2 along
// direction d (the gauge form of the Bloch operator, section 1); true when the
// operator is complex (some kappa_d != 0).
static bool bloch_phases(const ppcg_operator* op, double ph[3][2][2]) {
  bool c = false;
  for (int d = 0; d < 3; ++d) {
    c = c || op->kpt[d] != 0;
    for (int a = 1; a <= 2; ++a) {
      ph[d][a - 1][0] = std::cos(op->kpt[d] * a * op->h);
      ph[d][a - 1][1] = std::sin(op->kpt[d] * a * op->h);
    }
  }
  return c;
}

struct Prob {
  ppcg_handle* H;
  Work& Wk;
  hipStream_t st;
  Prof& prof;
  // problem
  int N = 0, order = 2;
  double hsp = 0, c0 = 0, w1 = 0, w2 = 0;
  long n = 0, rows = 0, ld = 0;
  int k = 0, q = 0, K = 0, Kp = 0;
  double tol = 0;
  int rr_period = 1, max_iter = 0;
  bool mixed = false;
  bool cplx = false;          // complex Hermitian (Bloch phase) operator
  double ph[3][2][2] = {};    // exp(i kappa_d a h), a = 1, 2
  const double* V = nullptr;
  const double* Bsrc = nullptr;  // generalized problem: diag(B) (caller's), else NULL
  bool gen = false;
  bool jac = true;             // Jacobi preconditioner T = diag(H)^-1, else T = I
  const double* X0 = nullptr;  // NULL: seeded N(0,1) start block drawn on the device
  uint64_t seed = 0;
  double* Xout = nullptr;
  double* lamout = nullptr;
  // state
  double dmin = 0;
  int nl = 0;        // locked columns (absolute prefix)
  bool hasP = false;
  int it = 1;
  bool noconv = false;
  double fresh = INFINITY;
  int last_kind = 0;  // what the last iteration ended with (ppcg_iter_log.kind)
  int pend_flags = 0; // sub-block pencil flags of the last iteration still to be read (block count)
  // pinned slot of those flags (ints), clear of the slots the residual and Rayleigh-Ritz read-backs use
  int* flag_slot() { return Wk.hpin + 4 * Kp + 32; }
  // orthonormalisation policy (section 5.5) and stopping test (section 5.2)
  int orth = PPCG_ORTH_CHOLQR, stop = PPCG_STOP_RESIDUAL;
  double orth_skip = 0.1, orth_taylor = 0.3;
  double orth_e = -1;          // |Xbar^H Xbar - I|_F measured in the last iteration (-1: not measured)
  int orth_mode = 2;           // this iteration: 0 omit steps 18-19, 1 Taylor polar, 2 Cholesky-QR
  double trace_prev = NAN, trace_cur = NAN;
  // Rayleigh-Ritz schedule (section 5.6): next iteration with a Rayleigh-Ritz step, current interval
  int next_rr = 0, rr_gap = 0;
  std::vector<double> lock_wn, lock_lam;
  ppcg_info info{};
  ppcg_status status = PPCG_OK;
  std::string err;
  std::chrono::steady_clock::time_point t0;

  Prob(ppcg_handle* h, Work& w) : H(h), Wk(w), st(h->st), prof(h->prof) {}

  // Jacobi skip thresholds relative to |M|_F, tied to the requested tolerance:
  // the RR rotation error then stays ~1e-5 tol below the Ritz residuals that
  // decide locking, and the pencils resolve X-W couplings down to ~1e-4 tol.
  double rr_rel_tol() const { return std::max(2.2e-16, std::min(1e-11, 1e-5 * tol)); }
  double pencil_rel_tol() const { return std::max(2.2e-16, std::min(1e-10, 1e-4 * tol)); }

  double* X() { return Wk.X.d(); }
  // diag(B) of a generalized problem (row scale of every B inner product), else NULL
  const double* bdiag() const { return gen ? Wk.Bd.d() : nullptr; }
  double* Xt() { return Wk.Xt.d(); }
  void swapX() {
    std::swap(Wk.X.p, Wk.Xt.p);
    std::swap(Wk.X.bytes, Wk.Xt.bytes);
  }

  // W/P/AW/AP storage (f64 in plain mode, f32 in mixed mode)
  void* Wb() { return mixed ? (void*)Wk.W32.p : Wk.W.p; }
  void* Pb() { return mixed ? (void*)Wk.P32.p : Wk.P.p; }
  void* AWb() { return mixed ? (void*)Wk.AW32.p : Wk.AW.p; }
  void* APb() { return mixed ? (void*)Wk.AP32.p : Wk.AP.p; }
  size_t esz() const { return (mixed ? 4 : 8) * (cplx ? 2 : 1); }
  void* col(void* base, long c, size_t es) { return (char*)base + (size_t)c * ld * es; }
  // element sizes: float64 blocks (X, H X) and the float shadow of X
  size_t xs() const { return cplx ? 16 : 8; }
  size_t x32s() const { return cplx ? 8 : 4; }
  int nc() const { return cplx ? 2 : 1; }
  // column c of a float64 / float block
  double* xc(double* base, long c) { return (double*)col(base, c, xs()); }
  float* fc(float* base, long c) { return (float*)col(base, c, x32s()); }

  // ---- parameters -----------------------------------------------------------
  void setup(const ppcg_operator* op, int k_, int q_, double tol_, int rrp, const double* X0_, double* Xout_,
             double* lamout_) {
    t0 = std::chrono::steady_clock::now();
    if (!op || !op->V || !Xout_ || !lamout_) throw PpcgError{PPCG_EINVAL, "null pointer argument"};
    if (op->order != 2 && op->order != 4) throw PpcgError{PPCG_EINVAL, "order must be 2 or 4"};
    cplx = bloch_phases(op, ph);
    if (op->precond != PPCG_PRECOND_JACOBI && op->precond != PPCG_PRECOND_NONE)
      throw PpcgError{PPCG_EINVAL, "precond must be PPCG_PRECOND_NONE or PPCG_PRECOND_JACOBI"};
    jac = op->precond == PPCG_PRECOND_JACOBI;
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
    // column stride: 64 elements beyond the rows, so that equal row offsets of
    // different columns (at 48^3 a column is a multiple of 32 KiB) need not
    // fall on the same HBM channels.  On separately allocated operands this
    // was 5-10% faster for the block update and the projection Gram; inside
    // the solve the difference is within run-to-run noise.  The extra rows
    // are never read and stay zero.
    ld = rows + 64;
    k = k_;
    q = q_;
    tol = tol_;
    rr_period = rrp;
    mixed = H->opt.precision == PPCG_MIXED;
    orth = H->opt.orth;
    stop = H->opt.stop;
    if (orth < PPCG_ORTH_CHOLQR || orth > PPCG_ORTH_NONE || stop < PPCG_STOP_RESIDUAL || stop > PPCG_STOP_TRACE)
      throw PpcgError{PPCG_EINVAL, "bad options.orth or options.stop"};
    orth_skip = H->opt.orth_skip > 0 ? H->opt.orth_skip : 0.1;
    orth_taylor = H->opt.orth_taylor > 0 ? H->opt.orth_taylor : 0.3;
    rr_gap = std::max(H->opt.rr_max, rrp);
    next_rr = rr_gap;
    max_iter = H->opt.max_iter > 0 ? H->opt.max_iter : 20000;
    if (k <= 0 || q < 1 || q > 32 || !(tol > 0) || rr_period < 1)
      throw PpcgError{PPCG_EINVAL, "need k > 0, 1 <= sbsize <= 32, tol > 0, rr_period >= 1"};
    int nbuf = H->opt.nbuf;
    if (nbuf < 0) {
      int extra = std::max(2, (int)std::ceil(0.02 * k));
      nbuf = q * ((k + extra + q - 1) / q) - k;
    }
    K = k + nbuf;
    if (K % q != 0) throw PpcgError{PPCG_EINVAL, "k + nbuf must be a multiple of sbsize"};
    if ((long)K * 4 > n) throw PpcgError{PPCG_EINVAL, "k + nbuf must not exceed n/4"};
    Kp = (int)round_up(K, 64);
    V = op->V;
    Bsrc = op->B;
    gen = Bsrc != nullptr;
    if (gen && mixed) throw PpcgError{PPCG_EINVAL, "the generalized problem (operator B) runs in FP64 only"};
    X0 = X0_;
    Xout = Xout_;
    lamout = lamout_;
  }

  // ---- autotuner --------------------------------------------------------------
  bool tuning() const { return (H->opt.flags & PPCG_AUTOTUNE) && !g_rec; }
  static int bucket(long x) {
    long b = 32;
    while (b < x) b *= 2;
    return (int)std::min<long>(b, 1L << 30);
  }
  // each candidate: one untimed run, then one timed with HIP events on the
  // solver's stream; the fastest wins (ties: the earlier candidate)
  template <class F>
  TuneChoice time_candidates(std::vector<TuneChoice>& cands, F&& run) {
    for (hipEvent_t& e : H->tev)
      if (!e) HIPCHECK(hipEventCreate(&e));
    int best = 0;
    std::string tried;
    for (size_t i = 0; i < cands.size(); ++i) {
      run(cands[i]);
      HIPCHECK(hipEventRecord(H->tev[0], st));
      run(cands[i]);
      HIPCHECK(hipEventRecord(H->tev[1], st));
      HIPCHECK(hipEventSynchronize(H->tev[1]));
      float ms = 0;
      HIPCHECK(hipEventElapsedTime(&ms, H->tev[0], H->tev[1]));
      cands[i].ms = ms;
      char b[96];
      snprintf(b, sizeof b, "%s%s/%d/%d:%.3f", i ? " " : "",
               cands[i].lds == 3 ? "tiles16" : (cands[i].lds == 2 ? "block" : (cands[i].lds ? "lds" : "wave")), cands[i].target,
               cands[i].floor_rows, ms);
      tried += b;
      if (ms < cands[best].ms) best = (int)i;
    }
    TuneChoice c = cands[best];
    c.tried = tried;
    return c;
  }

  // ---- kernels --------------------------------------------------------------
  void stencil(const void* Xs, void* Ys, int ncols, bool f32) {
    double es = (f32 ? 4 : 8) * nc();
    Scope s(prof, f32 ? "stencil_f32" : "stencil_f64", (order == 4 ? 16.0 : 10.0) * (cplx ? 3 : 1) * n * ncols,
            2.0 * es * n * ncols + es / nc() * n, f32 ? PEAK_F32 : PEAK_F64);
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
    a.V = f32 ? (const void*)Wk.V32.p : (const void*)Wk.Vd.p;
    a.f32 = f32;
    a.cplx = cplx;
    std::memcpy(a.ph, ph, sizeof(ph));
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

  // Gram kernel choice and row splitting.  Large real single-job Grams use
  // the LDS-staged kernel (128 x 128 workgroup tiles, 4 waves): about 4096
  // workgroups but no fewer than ~1000 rows per split.  The one-wave kernel
  // (64 x 64 tiles) aims at 2048 workgroups.
  struct GramPlan {
    bool lds;
    int splits;
    long chunk;
  };
  // LDS-staged Grams: real ones, and complex ones as two real Grams over interleaved rows
  bool gram_lds_ok(int M, int Nn, int njobs) const { return njobs == 1 && std::min(M, Nn) >= 64 && !(cplx && g_rec); }
  // per-block Grams: the single-pass kernel (lds = 2) for real blocks
  bool gram_block_ok(int M, int Nn, int site) const { return !cplx && site == 2 && M <= 128 && Nn <= 160; }
  GramPlan gram_plan(int M, int Nn, int njobs, long rws, int site = 0, const TuneChoice* tc = nullptr) const {
    GramPlan g;
    if (gram_block_ok(M, Nn, site)) {
      g.lds = tc && tc->lds == 2 ? 2 : 0;  // measured: the one-wave kernel at ~4096 workgroups is as fast
    } else {
      g.lds = tc ? (tc->lds == 1 && gram_lds_ok(M, Nn, njobs)) : (gram_lds_ok(M, Nn, njobs) && std::min(M, Nn) >= 96);
    }
    const long target = tc ? tc->target : (g.lds ? (g.lds == 2 ? 2048 : 4096) : (site == 2 ? 4096 : 2048));
    const long floor_rows = tc ? tc->floor_rows : (g.lds ? (g.lds == 2 ? 512 : 1024) : 256);
    long tiles, s, maxs;
    if (g.lds == 2) {
      tiles = njobs;
    } else if (g.lds) {
      tiles = (long)((M + 127) / 128) * ((Nn + 127) / 128);
    } else {
      const int tn = (site == 2 && !cplx) ? 80 : 64;  // per-block Grams use 64 x 80 tiles
      tiles = (long)((M + 63) / 64) * ((Nn + tn - 1) / tn) * njobs;
    }
    s = (target + tiles - 1) / tiles;
    maxs = std::max(1L, rws / floor_rows);
    s = std::max(1L, std::min(s, maxs));
    g.chunk = round_up((rws + s - 1) / s, 32);
    g.splits = (int)((rws + g.chunk - 1) / g.chunk);
    return g;
  }

  // dst (M x N, ldd) = A^H (D B) over `rws` rows; njobs strided jobs
  void gram(const ColSet& A, const ColSet& B, int M, int Nn, long rws, long ldab, const double* dsc, int nsc,
            void* dst, int ldd, bool upper, bool f32acc, int njobs = 1, long job_col_off = 0,
            long dst_job_stride = 0, const char* name = "gram", const double* dsc2 = nullptr) {
    if (M <= 0 || Nn <= 0) return;
    const int site = site_of(name);
    size_t es = (f32acc ? 4 : 8) * nc();
    size_t one = (size_t)njobs * M * Nn * es;
    if (one > Wk.part.bytes) throw PpcgError{PPCG_EINVAL, "internal: partial buffer too small"};
    auto capped = [&](GramPlan pl) {
      if ((size_t)pl.splits * one > Wk.part.bytes) {  // fewer, longer splits
        long sp = (long)(Wk.part.bytes / one);
        pl.chunk = round_up((rws + sp - 1) / sp, 32);
        pl.splits = (int)((rws + pl.chunk - 1) / pl.chunk);
      }
      return pl;
    };
    GramArgs g{};
    g.A = A;
    g.B = B;
    g.dsc = dsc;
    g.nsc = nsc;
    g.dsc2 = dsc2;
    g.M = M;
    g.N = Nn;
    g.ld = ldab;
    g.rows = rws;
    g.out = Wk.part.p;
    g.split_stride = (long)M * Nn;
    g.ldo = M;
    g.upper_only = upper;
    g.job_col_off = job_col_off;
    g.njobs = njobs;
    g.site = site;
    g.cplx = cplx;
    ReduceArgs r{};
    r.part = Wk.part.p;
    r.M = M;
    r.N = Nn;
    r.ldp = M;
    r.split_stride = (long)M * Nn;
    r.njobs = njobs;
    r.dst = dst;
    r.ldd = ldd;
    r.dst_job_stride = dst_job_stride;
    r.alpha = 1.0;
    r.beta = 0.0;
    r.upper_only = upper;
    r.cplx = cplx;
    auto set_plan = [&](const GramPlan& pl) {
      g.splits = pl.splits;
      g.chunk = pl.chunk;
      g.lds = pl.lds;
      r.splits = pl.splits;
    };
    // A complex Gram on the LDS-staged kernel: the columns read as real
    // columns of 2 rows per grid point, Re(A^H B) from the plain real Gram
    // and Im(A^H B) = Re(A^H (-i B)) from the one with every B pair (re, im)
    // taken as (im, -re); both upper-only when the result is Hermitian (the
    // real part is symmetric, the imaginary part antisymmetric), their split
    // partials one after the other, joined by the reduction.
    auto launch_g = [&]() {
      if (!(cplx && g.lds == 1)) {
        r.im_off = 0;
        launch_gram(g, f32acc, st);
        return;
      }
      GramArgs gi = g;
      gi.cplx = 0;
      gi.il = 1;
      gi.ld = 2 * ldab;
      gi.rows = 2 * rws;
      gi.chunk = 2 * g.chunk;
      gi.rotB = 0;
      launch_gram(gi, f32acc, st);
      gi.rotB = 1;
      gi.out = (char*)Wk.part.p + (size_t)g.splits * M * Nn * (f32acc ? 4 : 8);
      launch_gram(gi, f32acc, st);
      r.im_off = (long)g.splits * M * Nn;
    };
    // the Gram and its reduction are idempotent (the reduction overwrites
    // dst), so candidates run in place
    const TuneChoice* tc = nullptr;
    if (tuning()) {
      TuneKey key{0, site, f32acc ? 1 : 0, cplx ? 1 : 0, njobs > 1 ? 1 : 0, upper ? 1 : 0, bucket(M), bucket(Nn),
                  bucket(rws)};
      auto it = H->tune.find(key);
      if (it == H->tune.end()) {
        std::vector<TuneChoice> cands;
        for (int tgt : {1024, 2048, 4096}) {
          TuneChoice c;
          c.target = tgt;
          cands.push_back(c);
        }
        if (gram_block_ok(M, Nn, site))
          for (int tgt : {1024, 2048, 4096}) {
            TuneChoice c;
            c.lds = 2;
            c.target = tgt;
            c.floor_rows = 512;
            cands.push_back(c);
          }
        if (gram_lds_ok(M, Nn, njobs))
          for (int tgt : {512, 1024, 2048, 4096, 8192})
            for (int fl : {512, 1024}) {
              TuneChoice c;
              c.lds = 1;
              c.target = tgt;
              c.floor_rows = fl;
              cands.push_back(c);
            }
        TuneChoice best = time_candidates(cands, [&](const TuneChoice& c) {
          set_plan(capped(gram_plan(M, Nn, njobs, rws, site, &c)));
          launch_g();
          launch_reduce(r, f32acc, st);
        });
        it = H->tune.emplace(key, best).first;
      }
      tc = &it->second;
    }
    set_plan(capped(gram_plan(M, Nn, njobs, rws, site, tc)));
    {
      double nn = (double)std::min(rws, n), es_in = (f32acc ? 4.0 : 8.0) * nc();
      double fl = (upper ? (double)M * (M + 1) * nn : 2.0 * M * Nn * nn) * (cplx ? 4 : 1);
      double by = (double)njobs * (upper ? M : (M + Nn)) * nn * es_in;
      Scope s(prof, name, fl * njobs, by, f32acc ? PEAK_F32 : PEAK_F64);
      launch_g();
    }
    Scope s(prof, "reduce", 0, 0, PEAK_F64, prof.cat_of(name));
    launch_reduce(r, f32acc, st);
  }

  // Per-block pencil Grams of 16-column real blocks (steps 12-13 input) with
  // the tile kernel: the slabs of each block are read once and only the
  // tiles the pencil uses are formed.  Returns false where it does not apply
  // (complex, other block widths, grouped launches).
  long bg_splits(long target, int s) const {
    long sp = std::max(1L, std::min((target + s - 1) / s, std::max(1L, rows / 256)));
    long chunk = round_up((rows + sp - 1) / sp, 16);
    return (rows + chunk - 1) / chunk;
  }
  bool block_gram(const void* Wa, const void* Pa, const void* AWa, const void* APa, bool hasP, int s) {
    if (cplx || gen || q != 16 || g_rec || rows % 16 || s <= 0) return false;
    BlockGramArgs b{};
    b.X = xc(X(), nl);
    b.W = Wa;
    b.P = hasP ? Pa : nullptr;
    b.AW = AWa;
    b.AP = hasP ? APa : nullptr;
    b.AX = mixed ? xc(Wk.AXm.d(), nl) : nullptr;
    b.ld = ld;
    b.rows = rows;
    b.nblocks = s;
    b.hasP = hasP;
    b.f32 = mixed;
    b.out = Wk.part.d();
    const long one = (long)s * BG_TILES * 256 * 8;
    ReduceArgs r{};
    r.part = Wk.part.p;
    r.M = BG_TILES * 256;
    r.N = 1;
    r.ldp = r.M;
    r.split_stride = r.M;
    r.njobs = s;
    r.dst = Wk.bgram.p;
    r.ldd = r.M;
    r.dst_job_stride = r.M;
    r.alpha = 1.0;
    r.beta = 0.0;
    auto set_plan = [&](long target) {
      long sp = std::min(bg_splits(target, s), std::max(1L, (long)(Wk.part.bytes / one)));
      b.chunk = round_up((rows + sp - 1) / sp, 16);
      b.splits = (int)((rows + b.chunk - 1) / b.chunk);
      r.splits = b.splits;
    };
    long target = 4096;
    if (tuning()) {
      TuneKey key{2, 2, mixed ? 1 : 0, 0, 0, hasP ? 1 : 0, bucket(s), 16, bucket(rows)};
      auto it = H->tune.find(key);
      if (it == H->tune.end()) {
        std::vector<TuneChoice> cands;
        for (int tgt : {1024, 2048, 4096, 8192}) {
          TuneChoice c;
          c.lds = 3;
          c.target = tgt;
          cands.push_back(c);
        }
        TuneChoice best = time_candidates(cands, [&](const TuneChoice& c) {
          set_plan(c.target);
          launch_block_gram(b, st);
          launch_reduce(r, false, st);
        });
        it = H->tune.emplace(key, best).first;
      }
      target = it->second.target;
    }
    set_plan(target);
    {
      const double es = mixed ? 4.0 : 8.0;
      const double tiles = hasP ? BG_TILES : 5;
      const double fl = tiles * 2.0 * 256.0 * (double)rows * s;
      const double by = (double)rows * 16.0 * s * (8.0 + (hasP ? 4 : 2) * es + (mixed ? 8.0 : 0.0));
      Scope sc(prof, "gram_block", fl, by);
      launch_block_gram(b, st);
    }
    Scope sr(prof, "reduce", 0, 0, PEAK_F64, CAT_GEMM);
    launch_reduce(r, false, st);
    return true;
  }

  // C = beta (D C) + alpha A B
  // cpart (real only): column sums of squares of the stored values, per 64-row tile, for columns < ncn
  void update(const void* A, long lda, int Kk, const void* B, long ldb, int Nn, void* C0, void* C1, int N0, long ldc,
              float* C32, const double* dsc, long rws, double alpha, double beta, bool b_upper, bool f32,
              const char* name = "update", bool c0_keep = false, double* cpart = nullptr, int ncn = 0,
              const double* c64 = nullptr, const double* xd = nullptr, const double* gd = nullptr, long gds = 0) {
    if (Nn <= 0 || rws <= 0) return;
    UpdateArgs u{};
    u.c64 = c64;
    u.xd = xd;
    u.gd = gd;
    u.gds = gds;
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
    u.site = site_of(name);
    u.cplx = cplx;
    if (cpart && !cplx && ncn > 0) {
      u.cpart = cpart;
      u.ncn = ncn;
      u.ldp = rws / 64;
    }
    const bool lds_ok = !cplx && rws % 128 == 0 && Nn >= 64;
    u.lds = lds_ok && Nn >= 96;
    if (tuning() && lds_ok) {
      TuneKey key{1, -1, f32 ? 1 : 0, 0, 0, b_upper ? 1 : 0, bucket(Kk), bucket(Nn), bucket(rws)};
      auto it = H->tune.find(key);
      if (it == H->tune.end()) {
        // C = beta (D C) + alpha A B is idempotent only with beta = 0 or an
        // unwritten C0; otherwise candidates write into a copy of C
        UpdateArgs t = u;
        const bool idem = beta == 0.0 || c0_keep;
        if (!idem) {
          const size_t esz = f32 ? 4 : 8;
          const size_t c0b = (size_t)ldc * N0 * esz, c1b = C1 ? (size_t)ldc * (Nn - N0) * esz : 0;
          H->tune_scratch.ensure(c0b + c1b);
          HIPCHECK(hipMemcpyAsync(H->tune_scratch.p, C0, c0b, hipMemcpyDeviceToDevice, st));
          if (C1) HIPCHECK(hipMemcpyAsync((char*)H->tune_scratch.p + c0b, C1, c1b, hipMemcpyDeviceToDevice, st));
          t.C0 = H->tune_scratch.p;
          t.C1 = C1 ? (char*)H->tune_scratch.p + c0b : nullptr;
          t.C32 = nullptr;
        }
        std::vector<TuneChoice> cands(2);
        cands[1].lds = 1;
        TuneChoice best = time_candidates(cands, [&](const TuneChoice& c) {
          t.lds = c.lds;
          launch_update(t, f32, st);
        });
        it = H->tune.emplace(key, best).first;
      }
      u.lds = it->second.lds;
    }
    double nn = (double)std::min(rws, n), es = (f32 ? 4.0 : 8.0) * nc();
    double fl = (b_upper ? (double)Nn * (Nn + 1) * nn : 2.0 * Kk * Nn * nn) * (cplx ? 4 : 1);
    double by = ((double)Kk + Nn * (beta != 0 ? 2.0 : 1.0)) * nn * es + (C32 ? 4.0 * nc() * Nn * nn : 0.0);
    if (c64) by += (8.0 - es + (xd ? 8.0 : 0.0)) * Nn * nn;  // float64 input (and X) instead of C0
    Scope s(prof, name, fl, by, f32 ? PEAK_F32 : PEAK_F64);
    launch_update(u, f32, st);
  }

  void chol(double* G, int m) {
    CholArgs c{G, Wk.L.d(), Wk.Li.d(), m, Kp, Wk.iflag.i(), cplx};
    Scope s(prof, "chol_inverse");
    if (g_rec) g_rec->add(OP_CHOL, &c, sizeof(c), 0);
    else chol_inverse_grouped({c}, H->stage, st);
  }

  // ---- set-up ---------------------------------------------------------------
  void allocate() {
    size_t nk8 = (size_t)ld * K * xs(), nk4 = (size_t)ld * K * x32s();
    Wk.X.ensure(nk8);
    Wk.Xt.ensure(nk8);
    if (mixed) {
      Wk.AXm.ensure(nk8);
      Wk.X32.ensure(nk4);
      Wk.W32.ensure(nk4);
      Wk.P32.ensure(nk4);
      Wk.AW32.ensure(nk4);
      Wk.AP32.ensure(nk4);
      Wk.V32.ensure((size_t)rows * 4);
    } else {
      Wk.W.ensure(nk8);
      Wk.P.ensure(nk8);
      Wk.AW.ensure(nk8);
      Wk.AP.ensure(nk8);
    }
    Wk.Vd.ensure((size_t)rows * 8);
    Wk.td.ensure((size_t)rows * 8);
    if (gen) {
      Wk.Bd.ensure((size_t)rows * 8);
      Wk.btd.ensure((size_t)rows * 8);
    }
    size_t kk = (size_t)Kp * Kp * xs();
    for (DBuf* b : {&Wk.G, &Wk.L, &Wk.Li, &Wk.Rinv, &Wk.SAS, &Wk.SS, &Wk.V1, &Wk.Mr, &Wk.Yv, &Wk.Cc}) b->ensure(kk);
    Wk.GWP.ensure((size_t)Kp * 2 * K * xs());
    Wk.lam.ensure((size_t)Kp * 8);
    Wk.cn.ensure((size_t)Kp * 8);
    Wk.scal.ensure((size_t)Kp * 8 + 256);
    Wk.iflag.ensure(256);
    Wk.dminp.ensure(1024 * 8);
    int s = K / q;
    int nS = 3 * q;
    Wk.bgram.ensure((size_t)s * (nS + q) * (2 * nS - q) * xs());
    Wk.bC.ensure((size_t)s * 3 * q * q * xs());
    Wk.bflags.ensure((size_t)s * 4 + 256);
    Wk.cpart.ensure((size_t)(rows / 64) * Kp * 8);
    if (mixed) Wk.G32.ensure((size_t)Kp * Kp * x32s());
    if (3 * q > 48) Wk.pwork.ensure((size_t)s * pencil_work_elems() * xs());
    Wk.eigw.ensure(eig_workspace_bytes(K, cplx));
    // split partials: the largest Gram of the run
    size_t need = 0;
    auto acc = [&](int M, int Nn, int njobs, long rws, size_t es, int site = 0) {
      // the largest partial set over every shape up to M x Nn (active widths
      // shrink with locking; every width is a multiple of q) and job count
      for (int jb = 1; jb <= njobs; ++jb)
        for (int mm = std::min(q, M); mm <= M; mm += q)
          for (int nn = std::min(q, Nn); nn <= Nn; nn += q) {
            GramPlan pl = gram_plan(mm, nn, jb, rws, site);
            need = std::max(need, (size_t)jb * pl.splits * mm * nn * es);
            if (H->opt.flags & PPCG_AUTOTUNE) {  // room for the finest candidate splits
              TuneChoice c;
              c.lds = 1;
              c.target = 8192;
              c.floor_rows = 512;
              pl = gram_plan(mm, nn, jb, rws, site, &c);
              need = std::max(need, (size_t)jb * pl.splits * mm * nn * es);
              c.lds = 0;
              c.target = 4096;
              pl = gram_plan(mm, nn, jb, rws, site, &c);
              need = std::max(need, (size_t)jb * pl.splits * mm * nn * es);
            }
          }
    };
    acc(K, 2 * K, 1, rows, esz());
    acc(K, K, 1, rows, xs());
    acc(nS + q, 2 * nS - q, s, rows, xs(), 2);
    acc(K, K, 1, Kp, xs());
    if (!cplx && q == 16)  // 16-column block Grams, finest candidate
      need = std::max(need, (size_t)bg_splits(8192, s) * s * BG_TILES * 256 * 8);
    Wk.part.ensure(need);
    Wk.pinned((size_t)std::max(4 * Kp + 64 + (K / q + 1) / 2, 1024) * 8);
    // zero everything that carries padding rows
    std::vector<DBuf*> blocks = {&Wk.X, &Wk.Xt};
    if (mixed) {
      for (DBuf* b : {&Wk.X32, &Wk.W32, &Wk.P32, &Wk.AW32, &Wk.AP32, &Wk.AXm}) blocks.push_back(b);
    } else {
      for (DBuf* b : {&Wk.W, &Wk.P, &Wk.AW, &Wk.AP}) blocks.push_back(b);
    }
    for (DBuf* b : blocks) HIPCHECK(hipMemsetAsync(b->p, 0, b->bytes, st));
    for (DBuf* b : {&Wk.Vd, &Wk.td, &Wk.G, &Wk.L, &Wk.Li, &Wk.Rinv, &Wk.SAS, &Wk.SS, &Wk.V1, &Wk.Mr, &Wk.Yv,
                    &Wk.Cc, &Wk.GWP})
      HIPCHECK(hipMemsetAsync(b->p, 0, b->bytes, st));
    if (mixed) HIPCHECK(hipMemsetAsync(Wk.V32.p, 0, Wk.V32.bytes, st));
    HIPCHECK(hipMemcpyAsync(Wk.Vd.p, V, n * 8, hipMemcpyDeviceToDevice, st));
    if (gen) {
      HIPCHECK(hipMemsetAsync(Wk.Bd.p, 0, Wk.Bd.bytes, st));
      HIPCHECK(hipMemsetAsync(Wk.btd.p, 0, Wk.btd.bytes, st));
      HIPCHECK(hipMemcpyAsync(Wk.Bd.p, Bsrc, n * 8, hipMemcpyDeviceToDevice, st));
    }
  }

  // phase: Jacobi preconditioner and checks of V
  void enq_prep() {
    const int nparts = 256;
    launch_zero_int(Wk.iflag.i(), 4, st);
    launch_prep_diag(Wk.Vd.d(), n, c0, Wk.td.d(), mixed ? Wk.V32.f() : nullptr, Wk.dminp.d(), nparts, Wk.iflag.i(),
                     st);
    if (!jac) launch_fill(Wk.td.d(), n, 1.0, st);  // T = I: the row scales of step 8 become ones
    launch_d2h(Wk.hpind, Wk.dminp.p, nparts * 8, st);
    launch_d2h(Wk.hpin + 2 * nparts, Wk.iflag.p, 4, st);
    if (gen) {  // min and NaN scan of B (its reciprocal lands in btd, overwritten below)
      launch_prep_diag(Wk.Bd.d(), n, 0.0, Wk.btd.d(), nullptr, Wk.dminp.d() + nparts, nparts, Wk.iflag.i() + 1, st);
      launch_d2h(Wk.hpind + 512, Wk.dminp.d() + nparts, nparts * 8, st);
      launch_d2h(Wk.hpin + 2 * nparts + 1, Wk.iflag.i() + 1, 4, st);
      launch_scale_rows(Wk.Bd.d(), Wk.td.d(), Wk.btd.d(), rows, rows, 1, 0, st);  // B T
    }
  }
  void post_prep() {
    const int nparts = 256;
    double mn = 1e308;
    for (int i = 0; i < nparts; ++i) mn = std::min(mn, Wk.hpind[i]);
    if (Wk.hpin[2 * nparts]) throw PpcgError{PPCG_EINVAL, "V contains NaN"};
    if (jac && !(mn > 0))
      throw PpcgError{PPCG_ENOTHPD, "diag(H) has a non-positive entry: Jacobi preconditioner not HPD"};
    dmin = mn;
    if (gen) {
      double bm = 1e308;
      for (int i = 0; i < nparts; ++i) bm = std::min(bm, Wk.hpind[512 + i]);
      if (Wk.hpin[2 * nparts + 1]) throw PpcgError{PPCG_EINVAL, "B contains NaN"};
      if (!(bm > 0)) throw PpcgError{PPCG_ENOTHPD, "B has a non-positive entry: not positive definite"};
    }
  }

  // phase: orthonormal start block and first residual (steps 1-4)
  void enq_init() {
    if (X0)
      HIPCHECK(hipMemcpy2DAsync(X(), (size_t)ld * xs(), X0, (size_t)n * xs(), (size_t)n * xs(), K,
                                hipMemcpyDeviceToDevice, st));
    else
      launch_randn(X(), ld, n, K, seed, cplx, st);
    nl = 0;
    hasP = false;
    it = 1;
    enq_cholqr(K);
    enq_residual(K);
    enq_rho_d2h();
  }

  // G = Xbar^H Xbar of the active columns (upper triangle)
  void enq_gram_xx(int m) {
    CatCtx cc(prof, CAT_CHOLQR);
    double* Xa = xc(X(), nl);
    ColSet A = cols1(Xa, m, false);
    gram(A, A, m, m, rows, ld, bdiag(), bdiag() ? m : 0, Wk.G.p, Kp, true, false, 1, 0, 0, "gram_xx");  // X^H B X
  }
  // |G - I|_F^2 of that Gram into scal[Kp + 1] and the pinned slot 2 Kp + 1
  void enq_orth_err() {
    launch_orth_err2(Wk.G.d(), Kp, K - nl, Wk.scal.d() + Kp + 1, cplx, st, true);
    launch_d2h(Wk.hpind + 2 * Kp + 1, Wk.scal.d() + Kp + 1, 8, st);
  }
  // X (active columns) <- X R^{-1} with G = R^H R; result lands in Xt then X/Xt swap
  void enq_chol_apply(int m) {
    CatCtx cc(prof, CAT_CHOLQR);
    double* Xa = xc(X(), nl);
    launch_zero_int(Wk.iflag.i(), 4, st);
    chol(Wk.G.d(), m);
    launch_transpose(Wk.Li.d(), Kp, Wk.Rinv.d(), Kp, m, m, cplx, st);  // R^{-1} = L^{-H}
    double* Xn = xc(Xt(), nl);
    update(Xa, ld, m, Wk.Rinv.p, Kp, m, Xn, nullptr, m, ld, mixed ? fc(Wk.X32.f(), nl) : nullptr, nullptr, rows, 1.0,
           0.0, true, false, "update_xr");
    swapX();  // the locked prefix is valid in both buffers (copied once per Rayleigh-Ritz)
  }
  void enq_cholqr(int m) {
    enq_gram_xx(m);
    enq_chol_apply(m);
  }
  // X (active) <- X (I - Y/2 + 3Y^2/8 - 5Y^3/16), Y = G - I: the orthonormal
  // polar factor by four Taylor terms (section 5.5), evaluated as
  // I + Y (-I/2 + Y (3I/8 - 5Y/16)) with small products on the K x K buffers
  void enq_taylor(int m) {
    CatCtx cc(prof, CAT_CHOLQR);
    double* Xa = xc(X(), nl);
    launch_polar_prep(Wk.G.d(), Kp, m, Wk.Yv.d(), Wk.Mr.d(), cplx, st);
    update(Wk.Yv.p, Kp, m, Wk.Mr.p, Kp, m, Wk.V1.p, nullptr, m, Kp, nullptr, nullptr, Kp, 1.0, 0.0, false, false,
           "update_polar");
    launch_add_diag(Wk.V1.d(), Kp, m, -0.5, cplx, st);
    update(Wk.Yv.p, Kp, m, Wk.V1.p, Kp, m, Wk.Cc.p, nullptr, m, Kp, nullptr, nullptr, Kp, 1.0, 0.0, false, false,
           "update_polar");
    launch_add_diag(Wk.Cc.d(), Kp, m, 1.0, cplx, st);
    double* Xn = xc(Xt(), nl);
    update(Xa, ld, m, Wk.Cc.p, Kp, m, Xn, nullptr, m, ld, mixed ? fc(Wk.X32.f(), nl) : nullptr, nullptr, rows, 1.0,
           0.0, false, false, "update_xr");
    swapX();
  }
  // steps 18-19 omitted: X stays Xbar; the float shadow follows it
  void enq_orth_skip(int m) {
    if (mixed) launch_to_f32(xc(X(), nl), fc(Wk.X32.f(), nl), ld, rows, m, cplx, st);
  }

  // residual of the active columns: AX = H X, G = X^H AX, W = AX - X G.
  // plain: H X and then W overwrite the W block; mixed: H X stays in AXm
  // (float64) and only the float copy W32 of the residual is written (the
  // off-diagonal part of X G on float32 MFMA).
  // Column norms of the wanted active columns go to cn, G's to scal.
  void enq_residual(int m) {
    double* Xa = xc(X(), nl);
    double* R = mixed ? xc(Wk.AXm.d(), nl) : xc(Wk.W.d(), nl);
    stencil(Xa, R, m, false);
    ColSet A = cols1(Xa, m, false), B = cols1(R, m, false);
    gram(A, B, m, m, rows, ld, nullptr, 0, Wk.G.p, Kp, true, false, 1, 0, 0, "gram_xax");
    float* W32a = mixed ? fc(Wk.W32.f(), nl) : nullptr;
    int nwa = std::max(0, k - nl);
    // real: column norms of the wanted active residual columns from the update's epilogue partials
    double* cpart = cplx ? nullptr : Wk.cpart.d();
    if (mixed) {
      // W = (AX - X diag(G)) - X (G - diag(G)): the first part per entry in
      // float64, the coupling of the columns (off-diagonal G, of the size of
      // the residual near convergence) as a float32 product of the X shadow
      launch_offdiag32(Wk.G.d(), Kp, m, Wk.G32.f(), Kp, cplx, st);
      update(fc(Wk.X32.f(), nl), ld, m, Wk.G32.p, Kp, m, R, nullptr, m, ld, W32a, nullptr, rows, -1.0, 1.0, false,
             true, "update_resid", true, cpart, nwa, R, Xa, Wk.G.d(), (long)Kp + 1);
    } else {
      // generalized problem: W = H X - (B X) G, with B X formed in the (free) H W buffer
      const double* XG = Xa;
      if (gen) {
        double* BXa = xc(Wk.AW.d(), nl);
        launch_scale_rows_c(Wk.Bd.d(), Xa, BXa, ld, rows, m, cplx, st);
        XG = BXa;
      }
      update(XG, ld, m, Wk.G.p, Kp, m, R, nullptr, m, ld, W32a, nullptr, rows, -1.0, 1.0, false, false,
             "update_resid", mixed, cpart, nwa);
    }
    Scope s(prof, "colnorm");
    if (!cplx) {
      launch_colsum(Wk.cpart.d(), rows / 64, rows / 64, nwa, Wk.cn.d(), st);
    } else {  // a complex column is read as a real column of twice the length
      if (mixed) launch_colnorm2(W32a, 1, ld * nc(), rows * nc(), nwa, Wk.cn.d(), st);
      else launch_colnorm2(R, 0, ld * nc(), rows * nc(), nwa, Wk.cn.d(), st);
    }
    launch_frob2_sub(Wk.G.d(), Kp, nwa, Wk.scal.d(), cplx, st);
  }

  void enq_rho_d2h() {
    launch_trace(Wk.G.d(), Kp, K - nl, Wk.scal.d() + Kp, cplx, st);
    launch_d2h(Wk.hpind + 2 * Kp, Wk.scal.d() + Kp, 8, st);
    int nwa = std::max(0, k - nl);
    launch_d2h(Wk.hpind, Wk.cn.p, (size_t)std::max(nwa, 1) * 8, st);
    launch_d2h(Wk.hpind + Kp, Wk.scal.p, (size_t)std::max(nwa, 1) * 8, st);
    launch_d2h(Wk.hpin + 4 * Kp + 8, Wk.iflag.p, 4, st);
  }

  // per-iteration record for options.log_cb
  void log(double rho) const {
    if (!H->opt.log_cb) return;
    ppcg_iter_log rec{};
    rec.iter = it - 1;
    rec.n_locked = nl;
    rec.n_active = K - nl;
    rec.kind = last_kind;
    rec.rho = rho;
    rec.time_s = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
    rec.orth_err = orth_e;
    rec.trace = trace_cur;
    H->opt.log_cb(&rec, H->opt.log_user);
  }

  // rho of the loop head from the last residual (cn, scal) and the locked parts
  double post_rho() {
    int nwa = std::max(0, k - nl);
    if (Wk.hpin[4 * Kp + 8]) throw PpcgError{PPCG_ERANK, "Cholesky-QR breakdown (X^H X not positive definite)"};
    double num = 0, den = 0;
    for (int i = 0; i < nwa; ++i) {
      num += Wk.hpind[i];
      den += Wk.hpind[Kp + i];
    }
    double tr = Wk.hpind[2 * Kp];  // trace of the active block of X^H H X
    for (size_t i = 0; i < lock_wn.size(); ++i) {
      num += lock_wn[i] * lock_wn[i];
      den += lock_lam[i] * lock_lam[i];
      tr += lock_lam[i];
    }
    trace_prev = trace_cur;
    trace_cur = tr;
    return den > 0 ? std::sqrt(num / den) : INFINITY;
  }
  // the loop head's stopping test (section 5.2) on this iteration's rho and trace
  bool converged(double rho) const {
    if (stop == PPCG_STOP_TRACE)
      return std::isfinite(trace_prev) && std::fabs(trace_cur - trace_prev) <= tol * std::fabs(trace_cur);
    return rho <= tol;
  }
  bool rr_iteration() const { return it == next_rr; }
  void advance_rr() {
    rr_gap = std::max(rr_period, rr_gap - 1);
    next_rr += rr_gap;
  }

  // Rayleigh-Ritz over all K columns (S = [X_lock, X_act]), part 1: the
  // reduced matrix Mr = L^{-1} S^H H S L^{-H} with S^H S = L L^H.
  void enq_rr1() {
    CatCtx cc(prof, CAT_RR);
    double* S = X();
    double* AS = mixed ? Wk.AXm.d() : Wk.AW.d();
    stencil(S, AS, K, false);
    ColSet A = cols1(S, K, false);
    gram(A, cols1(AS, K, false), K, K, rows, ld, nullptr, 0, Wk.SAS.p, Kp, true, false, 1, 0, 0, "gram_rr");
    gram(A, A, K, K, rows, ld, bdiag(), bdiag() ? K : 0, Wk.SS.p, Kp, true, false, 1, 0, 0, "gram_rr");  // S^H B S
    launch_zero_int(Wk.iflag.i(), 4, st);
    chol(Wk.SS.d(), K);
    launch_transpose(Wk.Li.d(), Kp, Wk.Rinv.d(), Kp, K, K, cplx, st);  // Rinv = Linv^H
    update(Wk.SAS.p, Kp, K, Wk.Rinv.p, Kp, K, Wk.V1.p, nullptr, K, Kp, nullptr, nullptr, Kp, 1.0, 0.0, true, false,
           "update_small");
    gram(cols1(Wk.Rinv.p, K, false), cols1(Wk.V1.p, K, false), K, K, Kp, Kp, nullptr, 0, Wk.Mr.p, Kp, false, false,
         1, 0, 0, "gram_small");
    launch_symmetrize(Wk.Mr.d(), Kp, K, cplx, st);
    launch_d2h(Wk.hpin, Wk.iflag.p, 4, st);
  }
  void post_rr1() {
    if (Wk.hpin[0]) throw PpcgError{PPCG_ERANK, "Rayleigh-Ritz Gram S^H S not positive definite"};
  }
  EigJob eig_job() { return EigJob{Wk.Mr.d(), Kp, K, Wk.Yv.d(), Kp, Wk.lam.d(), Wk.eigw.p, rr_rel_tol(), cplx}; }

  // part 2: C = L^{-H} Y, X <- S C, fresh W = H X - X Lambda (all columns)
  void enq_rr2() {
    CatCtx cc(prof, CAT_RR);
    double* S = X();
    update(Wk.Rinv.p, Kp, K, Wk.Yv.p, Kp, K, Wk.Cc.p, nullptr, K, Kp, nullptr, nullptr, Kp, 1.0, 0.0, false, false,
           "update_small");
    update(S, ld, K, Wk.Cc.p, Kp, K, Xt(), nullptr, K, ld, mixed ? Wk.X32.f() : nullptr, nullptr, rows, 1.0, 0.0,
           false, false, "update_rot");
    swapX();
    double* R = mixed ? Wk.AXm.d() : Wk.W.d();
    stencil(X(), R, K, false);
    {
      Scope s(prof, "ritz_resid");
      // a complex column is read as a real column of twice the length (lambda is real)
      const long ldr = ld * nc(), rowsr = rows * nc();
      if (mixed) {
        launch_ritz_resid(R, X(), Wk.lam.d(), nullptr, Wk.W32.f(), ldr, rowsr, K, st);
        launch_colnorm2(Wk.W32.p, 1, ldr, rowsr, K, Wk.cn.d(), st);
      } else {  // generalized problem: H X - B X Lambda
        launch_ritz_resid(R, X(), Wk.lam.d(), R, nullptr, ldr, rowsr, K, st, bdiag(), cplx ? 1 : 0);
        launch_colnorm2(R, 0, ldr, rowsr, K, Wk.cn.d(), st);
      }
    }
    launch_d2h(Wk.hpind, Wk.cn.p, (size_t)K * 8, st);
    launch_d2h(Wk.hpind + Kp, Wk.lam.p, (size_t)K * 8, st);
  }

  // locking decision from the fresh Ritz residuals; returns the fresh residual
  // of the k lowest pairs
  double post_rr() {
    const double* wn2 = Wk.hpind;
    const double* lam = Wk.hpind + Kp;
    double lk = 0, rk = 0;
    for (int i = 0; i < k; ++i) {
      lk += lam[i] * lam[i];
      rk += wn2[i];
    }
    fresh = lk > 0 ? std::sqrt(rk / lk) : INFINITY;
    // leading run of wanted Ritz vectors with |w_i| <= tol |Lambda_k|_F / (2 sqrt(k)),
    // rounded down to a multiple of q
    double thr = 0.5 * tol * std::sqrt(lk) / std::sqrt((double)k);
    int nlnew = 0;
    while (nlnew < k && std::sqrt(wn2[nlnew]) <= thr) ++nlnew;
    nlnew = nlnew / q * q;
    if (hasP && nlnew < nl) {  // P(J_act) undefined when the locked set shrinks
      hasP = false;
      info.n_unlock++;
    }
    nl = nlnew;
    lock_wn.assign(nl, 0.0);
    lock_lam.assign(nl, 0.0);
    for (int i = 0; i < nl; ++i) {
      lock_wn[i] = std::sqrt(wn2[i]);
      lock_lam[i] = lam[i];
    }
    info.n_rr++;
    return fresh;
  }

  // part 3: active G = diag(Lambda_act) and the residual bookkeeping for rho
  void enq_rr3() {
    CatCtx cc(prof, CAT_RR);
    int m = K - nl;
    // the locked prefix of X, unchanged until the next Rayleigh-Ritz, into the other buffer
    launch_copy(X(), Xt(), (long)nl * ld * nc(), st);
    launch_set_diag(Wk.G.d(), Kp, m, Wk.lam.d() + nl, cplx, st);
    int nwa = std::max(0, k - nl);
    launch_copy(Wk.cn.d() + nl, Wk.scal.d(), std::max(nwa, 1), st);  // shift cn by nl through scal
    launch_copy(Wk.scal.d(), Wk.cn.d(), std::max(nwa, 1), st);
    launch_frob2_sub(Wk.G.d(), Kp, nwa, Wk.scal.d(), cplx, st);
    enq_rho_d2h();
  }

  // phase: steps 8-15 of one iteration
  void enq_body1() {
    const int m = K - nl;
    const int s = m / q;
    const size_t es = esz();
    void* Wa = col(Wb(), nl, es);
    void* Pa = col(Pb(), nl, es);
    void* AWa = col(AWb(), nl, es);
    void* APa = col(APb(), nl, es);
    // steps 8-10: precondition and project W and P against all K columns of X
    {
      ColSet A = cols1(mixed ? (const void*)Wk.X32.p : (const void*)X(), K, mixed);
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
      // X^H (T W) and X^H P; generalized problem: X^H B (T W) and X^H B P (B-orthogonal projector)
      gram(A, B, K, ncol, rows, ld, gen ? Wk.btd.d() : Wk.td.d(), m, Wk.GWP.p, Kp, false, mixed, 1, 0, 0,
           "gram_proj", gen ? Wk.Bd.d() : nullptr);
      const void* Xs = mixed ? (const void*)Wk.X32.p : (const void*)X();
      update(Xs, ld, K, Wk.GWP.p, Kp, ncol, Wa, Pa, m, ld, nullptr, Wk.td.d(), rows, -1.0, 1.0, false, mixed,
             "update_proj");
    }
    // AW = H W, AP = H P (no columns while P is empty)
    stencil(Wa, AWa, m, mixed);
    stencil(Pa, APa, hasP ? m : 0, mixed);
    // steps 11-13: per-block Grams and pencils
    const int nS = hasP ? 3 * q : 2 * q;
    {
      ColSet A{}, B{};
      const void* segs[5] = {xc(X(), nl), Wa, Pa, AWa, APa};
      bool f[5] = {false, mixed, mixed, mixed, mixed};
      int na = hasP ? 3 : 2;
      for (int t = 0; t < na; ++t) {
        A.p[t] = segs[t];
        A.end[t] = (t + 1) * q;
        A.f32[t] = f[t];
      }
      if (mixed) {  // rows (H X_j)^H [...] from the float64 H X
        A.p[na] = xc(Wk.AXm.d(), nl);
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
      const bool tiles = block_gram(Wa, Pa, AWa, APa, hasP, s);
      if (!tiles)  // generalized problem: the overlap columns [0, nS) carry B
        gram(A, B, Ma, Nb, rows, ld, bdiag(), gen ? nS : 0, Wk.bgram.p, Ma, false, false, s, (long)q * ld,
             (long)Ma * Nb, "gram_block");
      PencilArgs pa{};
      pa.gram = Wk.bgram.d();
      pa.gstride = tiles ? (long)BG_TILES * 256 : (long)Ma * Nb;
      pa.tiles16 = tiles;
      pa.ax_rows = mixed;
      pa.G = Wk.G.d();
      pa.ldg = Kp;
      pa.q = q;
      pa.nS = nS;
      pa.C = Wk.bC.d();
      pa.cstride = 3L * q * q;
      pa.flags = Wk.bflags.i();
      pa.drop_tol = 1e-14;
      pa.pivot_tol = 1e-12;
      pa.sing_tol = H->opt.singular_tol;
      pa.jacobi_rel = pencil_rel_tol();
      pa.nblocks = s;
      pa.cplx = cplx;
      pa.work = Wk.pwork.p;
      Scope sc(prof, "block_pencil", 0, 0);
      launch_block_pencil(pa, st);
    }
    // steps 14-15
    {
      BlockUpdArgs bu{};
      bu.X = xc(X(), nl);
      bu.W = Wa;
      bu.P = Pa;
      bu.f32 = mixed;
      bu.hasP = hasP;
      bu.ld = ld;
      bu.rows = rows;
      bu.q = q;
      bu.C = Wk.bC.d();
      bu.cstride = 3L * q * q;
      bu.nblocks = s;
      bu.cplx = cplx;
      // reads X, W (and P), writes X and P: X at its float64 size in both modes
      Scope sc(prof, "block_update", 6.0 * (cplx ? 4 : 1) * (double)n * q * q * s * (hasP ? 1.0 : 2.0 / 3.0),
               (double)n * q * s * (2.0 * xs() + (hasP ? 3.0 : 2.0) * esz()), mixed ? PEAK_F32 : PEAK_F64);
      launch_block_update(bu, st);
    }
    // the flags are read at the next synchronisation (no wait here): a rank
    // failure leaves its block unchanged (C = [I; 0; 0]) and ends the solve there
    launch_d2h(flag_slot(), Wk.bflags.p, (size_t)s * 4, st);
    pend_flags = s;
    hasP = true;
  }
  void post_body_flags() {
    const int* f = flag_slot();
    const int s = pend_flags;
    pend_flags = 0;
    for (int j = 0; j < s; ++j) {
      if (f[j] & 4) throw PpcgError{PPCG_ERANK, "sub-block pencil has rank below sbsize"};
      if (f[j] & 2) info.n_backtrack++;
      info.n_dropped += f[j] >> 8;
    }
  }

  // phase: steps 17-20 when the orthonormalisation needs no host decision
  // (Cholesky-QR every iteration, or never)
  void enq_cq() {
    int m = K - nl;
    if (orth == PPCG_ORTH_NONE) {
      orth_e = -1;
      orth_mode = 0;
      info.n_orth_skip++;
      enq_orth_skip(m);
    } else {
      enq_gram_xx(m);
      enq_orth_err();
      enq_chol_apply(m);
      orth_mode = 2;
      info.n_cholqr++;
    }
    enq_residual(m);
    enq_rho_d2h();
  }
  // adaptive orthonormalisation (section 5.5), part 1: measure e = |Xbar^H Xbar - I|_F
  void enq_cq_a() {
    enq_gram_xx(K - nl);
    enq_orth_err();
  }
  void post_cq_a() {
    orth_e = std::sqrt(Wk.hpind[2 * Kp + 1]);
    if (orth_e <= orth_skip) orth_mode = 0;
    else if (orth == PPCG_ORTH_TAYLOR && orth_e <= orth_taylor) orth_mode = 1;
    else orth_mode = 2;
    (orth_mode == 0 ? info.n_orth_skip : orth_mode == 1 ? info.n_taylor : info.n_cholqr)++;
  }
  // part 2: the chosen step, then the residual (step 20)
  void enq_cq_b() {
    int m = K - nl;
    if (orth_mode == 0) enq_orth_skip(m);
    else if (orth_mode == 1) enq_taylor(m);
    else enq_chol_apply(m);
    enq_residual(m);
    enq_rho_d2h();
  }
  // the measured e of a Cholesky-QR iteration is read at the next loop head
  void post_cq() {
    if (orth != PPCG_ORTH_NONE) orth_e = std::sqrt(Wk.hpind[2 * Kp + 1]);
  }

  // phase: outputs and the orthogonality check of the returned block
  void enq_finish() {
    const int kout = (H->opt.flags & PPCG_RETURN_BUFFERS) ? K : k;
    HIPCHECK(hipMemcpy2DAsync(Xout, (size_t)n * xs(), X(), (size_t)ld * xs(), (size_t)n * xs(), kout,
                              hipMemcpyDeviceToDevice, st));
    HIPCHECK(hipMemcpyAsync(lamout, Wk.lam.p, (size_t)kout * 8, hipMemcpyDeviceToDevice, st));
    ColSet A = cols1(X(), k, false);
    gram(A, A, k, k, rows, ld, bdiag(), bdiag() ? k : 0, Wk.G.p, Kp, false, false, 1, 0, 0, "gram_check");
    launch_orth_err2(Wk.G.d(), Kp, k, Wk.scal.d(), cplx, st);
    launch_d2h(Wk.hpind, Wk.scal.p, 8, st);
  }
  void post_finish() {
    info.orth_err = std::sqrt(Wk.hpind[0]);
    info.resid_final = fresh;
    info.n_locked = nl;
    info.time_s = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
  }
};

// ---------------------------------------------------------------------------
// lockstep driver
// ---------------------------------------------------------------------------
struct Driver {
  ppcg_handle* H;
  bool batched;
  Recorder rec;

  Driver(ppcg_handle* h, bool b) : H(h), batched(b) {}

  static const char* op_name(int kind) {
    switch (kind) {
      case OP_GRAM_D0: case OP_GRAM_F0: case OP_GRAM_Z0: case OP_GRAM_C0: case OP_GRAML_D0: case OP_GRAML_F0:
        return "gram";
      case OP_GRAM_D1: case OP_GRAM_F1: case OP_GRAM_Z1: case OP_GRAM_C1: case OP_GRAML_D1: case OP_GRAML_F1:
        return "gram_proj";
      case OP_GRAM_D2: case OP_GRAM_F2: case OP_GRAM_Z2: case OP_GRAM_C2: case OP_GRAMB_1: case OP_GRAMB_2:
        return "gram_block";
      case OP_REDUCE_D: case OP_REDUCE_F: case OP_REDUCE_Z: case OP_REDUCE_C: return "reduce";
      case OP_UPDATE_D0: case OP_UPDATE_F0: case OP_UPDATE_Z0: case OP_UPDATE_C0: case OP_UPDATEL_D0:
      case OP_UPDATEL_F0:
        return "update";
      case OP_UPDATE_D1: case OP_UPDATE_F1: case OP_UPDATE_Z1: case OP_UPDATE_C1: case OP_UPDATEL_D1:
      case OP_UPDATEL_F1:
        return "update_proj";
      case OP_STENCIL_D2: case OP_STENCIL_D4: case OP_STENCIL_Z2: case OP_STENCIL_Z4: return "stencil_f64";
      case OP_STENCIL_F2: case OP_STENCIL_F4: case OP_STENCIL_C2: case OP_STENCIL_C4: return "stencil_f32";
      case OP_PENCIL24: case OP_PENCIL48: case OP_PENCIL96:
      case OP_PENCILZ24: case OP_PENCILZ48: case OP_PENCILZ96: return "block_pencil";
      case OP_CHOL: return "chol_inverse";
      default: return (kind >= OP_BUPD_D4 && kind <= OP_BUPD_C32) ? "block_update" : "misc";
    }
  }

  // replay the recorded lists: one grouped launch per position and kind.
  // Pass 1 packs every job array and prefix-sum array of the phase into one
  // host buffer (one upload); pass 2 issues the launches in recorded order.
  void flush() {
    auto& L = rec.lists;
    size_t len = L.empty() ? 0 : L[0].size();
    for (auto& l : L)
      if (l.size() != len) throw PpcgError{PPCG_EINVAL, "internal: batched phases diverged"};
    hipStream_t st = H->st;
    struct G { size_t pos; int kind; std::vector<int> idx; size_t jobs_off = 0, start_off = 0; unsigned tot = 0; };
    std::vector<G> groups;
    std::vector<uint8_t> buf;
    auto align = [&]() { buf.resize((buf.size() + 15) / 16 * 16); };
    for (size_t pos = 0; pos < len; ++pos) {
      std::map<int, std::vector<int>> by_kind;
      for (int i = 0; i < (int)L.size(); ++i) by_kind[L[i][pos].kind].push_back(i);
      for (auto& kv : by_kind) {
        G g;
        g.pos = pos;
        g.kind = kv.first;
        g.idx = kv.second;
        if (g.kind != OP_D2H && g.kind != OP_CHOL) {
          size_t asz = op_args_size(g.kind);
          align();
          g.jobs_off = buf.size();
          buf.resize(buf.size() + asz * g.idx.size());
          for (size_t j = 0; j < g.idx.size(); ++j)
            std::memcpy(buf.data() + g.jobs_off + j * asz, L[g.idx[j]][pos].args.data(), asz);
          align();
          g.start_off = buf.size();
          buf.resize(buf.size() + sizeof(unsigned) * (g.idx.size() + 1));
          unsigned* s = (unsigned*)(buf.data() + g.start_off);
          for (size_t j = 0; j < g.idx.size(); ++j) {
            s[j] = g.tot;
            g.tot += L[g.idx[j]][pos].nwg;
          }
          s[g.idx.size()] = g.tot;
        }
        groups.push_back(std::move(g));
      }
    }
    uint8_t* dev = buf.empty() ? nullptr : (uint8_t*)H->stage.upload(buf.data(), buf.size(), st);
    for (G& g : groups) {
      if (g.kind == OP_D2H) {
        for (int i : g.idx) {
          D2HArgs a;
          std::memcpy(&a, L[i][g.pos].args.data(), sizeof(a));
          if (a.bytes) HIPCHECK(hipMemcpyAsync(a.dst, a.src, a.bytes, hipMemcpyDeviceToHost, st));
        }
        continue;
      }
      double fl = 0, by = 0;
      const char* nm = nullptr;
      for (int i : g.idx) {
        const RecOp& op = L[i][g.pos];
        fl += op.fl;
        by += op.by;
        if (op.name) nm = op.name;
      }
      Scope sc(H->prof, nm ? nm : op_name(g.kind), fl, by);
      if (g.kind == OP_CHOL) {
        std::vector<CholArgs> jobs;
        for (int i : g.idx) {
          CholArgs a;
          std::memcpy(&a, L[i][g.pos].args.data(), sizeof(a));
          jobs.push_back(a);
        }
        chol_inverse_grouped(jobs, H->stage, st);
        continue;
      }
      if (g.tot == 0) continue;
      if (!launch_grouped(g.kind, dev + g.jobs_off, (const unsigned*)(dev + g.start_off), (int)g.idx.size(), g.tot,
                          st))
        throw PpcgError{PPCG_EINVAL, "internal: op cannot be grouped"};
    }
  }

  template <class F>
  void phase(const std::vector<Prob*>& ps, F fn) {
    if (ps.empty()) return;
    if (!batched) {
      for (Prob* p : ps) fn(*p);
      return;
    }
    rec.begin((int)ps.size());
    g_rec = &rec;
    try {
      for (int i = 0; i < (int)ps.size(); ++i) {
        rec.cur = i;
        fn(*ps[i]);
      }
    } catch (...) {
      g_rec = nullptr;
      throw;
    }
    g_rec = nullptr;
    flush();
  }

  // run fn on each problem; a problem that throws leaves the set
  template <class F>
  void post(std::vector<Prob*>& ps, F fn) {
    std::vector<Prob*> keep;
    for (Prob* p : ps) {
      try {
        fn(*p);
        keep.push_back(p);
      } catch (const PpcgError& e) {
        p->status = e.code;
        p->err = e.msg;
      }
    }
    ps.swap(keep);
  }

  void rayleigh_ritz(std::vector<Prob*>& ps) {
    phase(ps, [](Prob& p) { p.enq_rr1(); });
    sync(H);
    post(ps, [](Prob& p) { p.post_rr1(); });
    if (ps.empty()) return;
    std::vector<EigJob> jobs;
    for (Prob* p : ps) jobs.push_back(p->eig_job());
    {
      Scope s(H->prof, "eig");
      if (!H->hcounter) HIPCHECK(hipHostMalloc((void**)&H->hcounter, 64, hipHostMallocDefault));
      H->counter.ensure(256);
      EigGraphCache* gc = (H->opt.flags & PPCG_NO_GRAPHS) ? nullptr : &H->eig_graph;
      block_jacobi_eig_grouped(jobs, H->stage, gc, H->counter.i(), H->hcounter, H->st);
    }
    phase(ps, [](Prob& p) { p.enq_rr2(); });
    sync(H);
    post(ps, [](Prob& p) { p.post_rr(); });
  }

  // Algorithm 3 over a set of problems in lockstep.  Each problem ends with
  // status OK, ENOCONV or an error of its own.
  void run(std::vector<Prob*> act) {
    for (Prob* p : act) p->allocate();
    phase(act, [](Prob& p) { p.enq_prep(); });
    sync(H);
    post(act, [](Prob& p) { p.post_prep(); });
    phase(act, [](Prob& p) { p.enq_init(); });
    sync(H);
    while (!act.empty()) {
      std::vector<Prob*> fin, body, done, again;
      post(act, [&](Prob& p) {
        p.post_body_flags();
        double r = p.post_rho();
        if (p.last_kind == 1) p.post_cq();
        p.log(r);
        if (p.converged(r)) fin.push_back(&p);
        else if (p.it > p.max_iter) {
          p.noconv = true;
          fin.push_back(&p);
        } else body.push_back(&p);
      });
      // final Rayleigh-Ritz and the fresh residual check (loop head, rho <= tol)
      if (!fin.empty()) {
        rayleigh_ritz(fin);
        for (Prob* p : fin) {
          if (p->fresh <= p->tol || (p->stop == PPCG_STOP_TRACE && !p->noconv)) done.push_back(p);
          else if (p->noconv) {
            p->status = PPCG_ENOCONV;
            p->err = "max_iter reached";
            done.push_back(p);
          } else {
            p->last_kind = 3;
            again.push_back(p);
          }
        }
        phase(again, [](Prob& p) { p.enq_rr3(); });
      }
      if (!body.empty()) {
        phase(body, [](Prob& p) { p.enq_body1(); });
        std::vector<Prob*> cq, cqa, rr;
        for (Prob* p : body) {
          const bool r_it = p->rr_iteration();
          p->last_kind = r_it ? 2 : 1;
          if (r_it) rr.push_back(p);
          else if (p->orth == PPCG_ORTH_SKIP || p->orth == PPCG_ORTH_TAYLOR) cqa.push_back(p);
          else cq.push_back(p);
        }
        phase(cq, [](Prob& p) { p.enq_cq(); });
        if (!cqa.empty()) {  // the orthonormalisation step depends on the measured e
          phase(cqa, [](Prob& p) { p.enq_cq_a(); });
          sync(H);
          post(cqa, [](Prob& p) { p.post_cq_a(); });
          // one phase per decision: grouped launches need the same steps in every problem
          for (int mode = 0; mode < 3; ++mode) {
            std::vector<Prob*> grp;
            for (Prob* p : cqa)
              if (p->orth_mode == mode) grp.push_back(p);
            phase(grp, [](Prob& p) { p.enq_cq_b(); });
          }
        }
        if (!rr.empty()) {
          rayleigh_ritz(rr);
          phase(rr, [](Prob& p) {
            p.enq_rr3();
            p.orth_e = -1;
            p.advance_rr();
          });
        }
        for (Prob* p : body) {
          p->info.iters = p->it;
          p->it++;
        }
      }
      phase(done, [](Prob& p) { p.enq_finish(); });
      sync(H);
      for (Prob* p : done) p->post_finish();
      std::vector<Prob*> alive;
      for (Prob* p : again)
        if (p->status == PPCG_OK) alive.push_back(p);
      for (Prob* p : body)
        if (p->status == PPCG_OK) alive.push_back(p);
      act.swap(alive);
    }
    H->prof.collect();
  }
};

// ---------------------------------------------------------------------------
// backward pass: projected Sternheimer systems by block PCG
// ---------------------------------------------------------------------------
struct Grad {
  ppcg_handle* H;
  hipStream_t st;
  Prof& prof;
  int k = 0;
  long n = 0, rows = 0, ld = 0;
  bool cplx = false;  // complex Hermitian (Bloch) operator: interleaved complex columns
  int nc = 1;         // doubles per element
  double resid = 0;  // largest |r_i| / |b_i| over the columns at exit
  Grad(ppcg_handle* h) : H(h), st(h->st), prof(h->prof) {}

  // Y <- (I - X X^H) Y over the k saved eigenvectors
  void project(double* Y) {
    Prob s(H, H->work(0));
    s.n = n;
    s.rows = rows;
    s.ld = ld;
    s.cplx = cplx;
    ColSet A = Prob::cols1(H->work(0).X.p, k, false), B = Prob::cols1(Y, k, false);
    s.gram(A, B, k, k, rows, ld, nullptr, 0, H->gsc.p, (int)round_up(k, 64), false, false, 1, 0, 0, "gram_grad");
    s.update(H->work(0).X.p, ld, k, H->gsc.p, round_up(k, 64), k, Y, nullptr, k, ld, nullptr, nullptr, rows, -1.0,
             1.0, false, false, "update_grad");
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
    a.V = H->work(0).Vd.p;
    a.f32 = 0;
    a.shift = H->work(0).lam.d();
    a.cplx = cplx;
    std::memcpy(a.ph, H->s_ph, sizeof(a.ph));
    Scope sc(prof, "stencil_f64", (H->s_order == 4 ? 17.0 : 11.0) * (cplx ? 3 : 1) * n * k, 16.0 * nc * n * k);
    launch_stencil(a, st);
  }

  int run(const double* g, const double* w, double* out, double tol, int max_iter) {
    if (!H->has_state) throw PpcgError{PPCG_ENOSTATE, "ppcg_grad needs a successful ppcg_solve on this handle"};
    if (H->s_gen) throw PpcgError{PPCG_EINVAL, "ppcg_grad: not for a generalized problem (operator B)"};
    if (!g || !out || !(tol > 0)) throw PpcgError{PPCG_EINVAL, "null pointer or tol <= 0"};
    Work& Wk = H->work(0);
    k = H->s_k;
    n = H->s_n;
    rows = H->s_rows;
    ld = H->s_ld;
    cplx = H->s_cplx;
    nc = cplx ? 2 : 1;
    if (!w) {
      launch_grad_rows(Wk.X.d(), nullptr, g, ld, n, k, out, st, cplx);
      sync(H);
      return 0;
    }
    // complex columns are addressed as real columns of twice the length by
    // the element-wise CG kernels (the CG scalars Re(a^H b) are real dots)
    const long ldr = ld * nc, rowsr = rows * nc;
    const size_t blk = (size_t)ld * k * 8 * nc;
    for (DBuf* b : {&H->gZ, &H->gR, &H->gP, &H->gAP, &H->gY}) b->ensure(blk);
    H->gw.ensure((size_t)rows * 8);
    int kp = (int)round_up(k, 64);
    H->gsc.ensure((size_t)kp * kp * 8 * nc + (size_t)16 * kp * 8);
    double* sc = H->gsc.d() + (size_t)kp * kp * nc;  // per-column scalars
    double *rz = sc, *rznew = sc + kp, *pAp = sc + 2 * kp, *alpha = sc + 3 * kp, *beta = sc + 4 * kp,
           *bb = sc + 5 * kp, *rr = sc + 6 * kp;
    int* done = (int*)(sc + 7 * kp);
    int* left = (int*)(sc + 8 * kp);
    // the partial buffer holds the split partials of the k x k projection Gram
    {
      Prob tmp(H, Wk);
      tmp.cplx = cplx;
      Wk.part.ensure((size_t)tmp.gram_plan(k, k, 1, rows).splits * k * k * 8 * nc);
    }
    HIPCHECK(hipMemsetAsync(H->gw.p, 0, H->gw.bytes, st));
    HIPCHECK(hipMemcpyAsync(H->gw.p, w, n * 8, hipMemcpyDeviceToDevice, st));
    // the stencil writes only the n grid rows of A P and the projection keeps
    // the padding rows as they are: they must start (and stay) zero, or the
    // CG residual norms over the padded rows pick up stale memory
    HIPCHECK(hipMemsetAsync(H->gAP.p, 0, H->gAP.bytes, st));
    double *Z = H->gZ.d(), *R = H->gR.d(), *P = H->gP.d(), *AP = H->gAP.d(), *Y = H->gY.d();
    // b = Q (w x_i)
    launch_scale_rows_c(H->gw.d(), Wk.X.d(), R, ld, rows, k, cplx, st);
    project(R);
    launch_coldot(R, R, ldr, rowsr, k, bb, st);
    launch_fill(Z, (long)ld * k * nc, 0.0, st);
    launch_zero_int(done, k, st);
    // Jacobi preconditioner 1/(diag(H) - lambda_i) when it is positive definite
    HIPCHECK(hipMemcpyAsync(Wk.hpind, Wk.lam.p, (size_t)k * 8, hipMemcpyDeviceToHost, st));
    sync(H);
    double lmax = -1e308;
    for (int j = 0; j < k; ++j) lmax = std::max(lmax, Wk.hpind[j]);
    int unprec = !(H->s_dmin - lmax > 0);
    auto precond = [&]() {
      launch_cg_precond(R, Y, Wk.Vd.d(), H->s_c0, Wk.lam.d(), ld, n, rows, k, unprec, st, cplx);
      project(Y);
    };
    precond();
    HIPCHECK(hipMemcpyAsync(P, Y, blk, hipMemcpyDeviceToDevice, st));
    launch_coldot(R, Y, ldr, rowsr, k, rz, st);
    int it = 0;
    for (; it < max_iter; ++it) {
      stencil_shift(P, AP);
      project(AP);
      launch_coldot(P, AP, ldr, rowsr, k, pAp, st);
      launch_cg_alpha(rz, pAp, done, alpha, k, st);
      launch_cg_xr(Z, R, P, AP, alpha, ldr, rowsr, k, st);
      launch_coldot(R, R, ldr, rowsr, k, rr, st);
      launch_zero_int(left, 1, st);
      launch_cg_check(rr, bb, tol, done, left, k, st);
      if (it % 4 == 3 || it == max_iter - 1) {
        HIPCHECK(hipMemcpyAsync(Wk.hpin, left, 4, hipMemcpyDeviceToHost, st));
        sync(H);
        if (Wk.hpin[0] == 0) {
          ++it;
          break;
        }
      }
      precond();
      launch_coldot(R, Y, ldr, rowsr, k, rznew, st);
      launch_cg_beta(rz, rznew, done, beta, k, st);
      launch_cg_p(P, Y, beta, ldr, rowsr, k, st);
    }
    launch_grad_rows(Wk.X.d(), Z, g, ld, n, k, out, st, cplx);
    HIPCHECK(hipMemcpyAsync(Wk.hpind, rr, (size_t)k * 8, hipMemcpyDeviceToHost, st));
    HIPCHECK(hipMemcpyAsync(Wk.hpind + k, bb, (size_t)k * 8, hipMemcpyDeviceToHost, st));
    sync(H);
    resid = 0;
    for (int j = 0; j < k; ++j) {
      const double b2 = Wk.hpind[k + j];
      if (b2 > 0) resid = std::max(resid, std::sqrt(Wk.hpind[j] / b2));
    }
    prof.collect();
    return it;
  }
};

// Autotuner table file: one decision per line,
//   kind site f32 cplx multi upper mb nb rb lds target floor_rows ms
// ('#' starts a comment line).
void load_tune_table(ppcg_handle* H) {
  FILE* f = fopen(H->tune_path.c_str(), "r");
  if (!f) return;  // no table yet: the first tuned solve writes it
  char line[512];
  int ln = 0;
  while (fgets(line, sizeof line, f)) {
    ++ln;
    if (line[0] == '#' || line[0] == '\n') continue;
    TuneKey k{};
    TuneChoice c;
    long rb = 0;
    int n = sscanf(line, "%d %d %d %d %d %d %d %d %ld %d %d %d %lf", &k.kind, &k.site, &k.f32, &k.cplx, &k.multi,
                   &k.upper, &k.mb, &k.nb, &rb, &c.lds, &c.target, &c.floor_rows, &c.ms);
    k.rb = rb;
    if (n != 13 || k.kind < 0 || k.kind > 2 || c.lds < 0 || c.lds > 3 || c.target <= 0 || c.floor_rows <= 0) {
      fclose(f);
      throw PpcgError{PPCG_EINVAL, "tune table " + H->tune_path + ": malformed line " + std::to_string(ln)};
    }
    c.tried = "(from table)";
    H->tune[k] = c;
  }
  fclose(f);
  H->tune_saved = H->tune.size();
}

void save_tune_table(ppcg_handle* H) {
  if (H->tune_path.empty() || H->tune.size() == H->tune_saved) return;
  std::string tmp = H->tune_path + ".tmp";
  FILE* f = fopen(tmp.c_str(), "w");
  if (!f) throw PpcgError{PPCG_EINVAL, "cannot write tune table " + tmp};
  fprintf(f, "# libppcg autotuner decisions: kind site f32 cplx multi upper mb nb rb lds target floor_rows ms\n");
  for (const auto& kv : H->tune) {
    const TuneKey& k = kv.first;
    const TuneChoice& c = kv.second;
    fprintf(f, "%d %d %d %d %d %d %d %d %ld %d %d %d %.6f\n", k.kind, k.site, k.f32, k.cplx, k.multi, k.upper, k.mb,
            k.nb, k.rb, c.lds, c.target, c.floor_rows, c.ms);
  }
  bool ok = fclose(f) == 0;
  if (!ok || rename(tmp.c_str(), H->tune_path.c_str()) != 0)
    throw PpcgError{PPCG_EINVAL, "cannot write tune table " + H->tune_path};
  H->tune_saved = H->tune.size();
}

// Input of the block pencil kernel for given pencils: the Gram layout a
// solve builds (per block nS x (2 nS - q): B, then columns [q, nS) of A), the
// q x q X blocks of A, and for nS > 48 the per-block work matrices.
struct PencilLayout {
  size_t gram_bytes = 0, g_bytes = 0, work_bytes = 0;
  size_t g_off = 0, work_off = 0;  // offsets inside one scratch area (256-byte aligned)
  size_t total() const { return work_off + work_bytes; }
};
PencilLayout pencil_layout(int nblocks, int q, bool has_p, bool cplx) {
  const size_t es = cplx ? 16 : 8;
  const int nS = has_p ? 3 * q : 2 * q, Nb = 2 * nS - q;
  auto al = [](size_t b) { return (b + 255) / 256 * 256; };
  PencilLayout L;
  L.gram_bytes = (size_t)nblocks * nS * Nb * es;
  L.g_bytes = (size_t)nblocks * q * (q + 1) * es;
  L.work_bytes = nS > 48 ? (size_t)nblocks * pencil_work_elems() * es : 0;
  L.g_off = al(L.gram_bytes);
  L.work_off = L.g_off + al(L.g_bytes);
  return L;
}

// packs the pencils and launches the block pencil kernel on the handle's
// stream (no synchronisation)
void enqueue_pencils(ppcg_handle* h, int nblocks, int q, bool has_p, bool cplx, const double* A, const double* B,
                     double tol, double* C, int32_t* flags, double* gram, double* G, void* work) {
  const int nS = has_p ? 3 * q : 2 * q, Nb = 2 * nS - q;
  launch_pencil_pack(A, B, nblocks, q, nS, cplx ? 1 : 0, gram, G, h->st);
  PencilArgs pa{};
  pa.gram = gram;
  pa.gstride = (long)nS * Nb;
  pa.G = G;
  pa.ldg = q;
  pa.q = q;
  pa.nS = nS;
  pa.C = C;
  pa.cstride = 3L * q * q;
  pa.flags = flags;
  pa.drop_tol = 1e-14;
  pa.pivot_tol = 1e-12;
  pa.sing_tol = h->opt.singular_tol;
  pa.jacobi_rel = std::max(2.2e-16, std::min(1e-10, 1e-4 * tol));
  pa.nblocks = nblocks;
  pa.cplx = cplx ? 1 : 0;
  pa.work = work;
  Scope sc(h->prof, "block_pencil");
  launch_block_pencil(pa, h->st);
}

ppcg_status guard(ppcg_handle* h, const std::function<ppcg_status()>& f) {
  try {
    if (h) HIPCHECK(hipSetDevice(h->device));
    return f();
  } catch (const PpcgError& e) {
    g_rec = nullptr;
    if (h) h->err = e.msg;
    return e.code;
  } catch (const std::exception& e) {
    g_rec = nullptr;
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
  if (resolve_scratch(h->device, &h->noalloc_scratch) != hipSuccess) {
    delete h;
    return PPCG_EHIP;
  }
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
  if (!(h->opt.singular_tol > 0)) h->opt.singular_tol = 1e-12;
  if (h->opt.tune_table) h->tune_path = h->opt.tune_table;
  h->opt.tune_table = nullptr;  // the handle keeps its own copy of the path
  h->prof.on = h->opt.profile != 0;
  h->prof.st = h->st;
  if (!h->tune_path.empty()) {
    try {
      load_tune_table(h);
    } catch (const PpcgError& e) {
      delete h;
      return e.code;
    }
  }
  *out = h;
  return PPCG_OK;
}

ppcg_status ppcg_solve(ppcg_handle* h, const ppcg_operator* op, int32_t k, int32_t sbsize, double tol,
                       int32_t rr_period, const double* X0, double* X_out, double* lambda_out, ppcg_info* info) {
  if (!h) return PPCG_EINVAL;
  return guard(h, [&]() {
    h->has_state = false;
    Prob p(h, h->work(0));
    h->prof.collect();
    double cat0[NCAT], roof0 = h->prof.roof_ms;
    std::copy(h->prof.cat_ms, h->prof.cat_ms + NCAT, cat0);
    auto stages = [&]() {
      if (!h->prof.on) return;
      h->prof.collect();
      for (int c = 0; c < NCAT; ++c) p.info.stage_ms[c] = h->prof.cat_ms[c] - cat0[c];
      p.info.roofline_ms = h->prof.roof_ms - roof0;
    };
    try {
      p.setup(op, k, sbsize, tol, rr_period, X0, X_out, lambda_out);
      p.seed = h->opt.seed;
      Driver d(h, false);
      d.run({&p});
      stages();
    } catch (...) {
      if (info) *info = p.info;
      throw;
    }
    save_tune_table(h);
    if (info) *info = p.info;
    if (p.status != PPCG_OK) {
      h->err = p.err;
      return p.status;
    }
    h->has_state = true;
    h->s_cplx = p.cplx;
    h->s_N = p.N;
    h->s_order = p.order;
    h->s_k = p.k;
    h->s_n = p.n;
    h->s_rows = p.rows;
    h->s_ld = p.ld;
    h->s_c0 = p.c0;
    h->s_w1 = p.w1;
    h->s_w2 = p.w2;
    h->s_dmin = p.dmin;
    std::memcpy(h->s_ph, p.ph, sizeof(p.ph));
    h->s_gen = p.gen;
    return PPCG_OK;
  });
}

ppcg_status ppcg_solve_batched(ppcg_handle* h, int32_t nprob, const ppcg_operator* ops, const int32_t* k,
                               int32_t sbsize, double tol, int32_t rr_period, const double* const* X0,
                               double* const* X_out, double* const* lambda_out, ppcg_info* infos,
                               int32_t* statuses) {
  if (!h || nprob < 0 || (nprob > 0 && (!ops || !k || !X_out || !lambda_out))) return PPCG_EINVAL;
  return guard(h, [&]() {
    h->has_state = false;
    std::vector<std::unique_ptr<Prob>> ps;
    std::vector<Prob*> run;
    ppcg_status first = PPCG_OK;
    for (int b = 0; b < nprob; ++b) {
      ps.emplace_back(new Prob(h, h->work(b)));
      try {
        ps[b]->setup(&ops[b], k[b], sbsize, tol, rr_period, X0 ? X0[b] : nullptr, X_out[b], lambda_out[b]);
        ps[b]->seed = h->opt.seed + (uint64_t)b;
        if (!run.empty() && ps[b]->cplx != run[0]->cplx)
          throw PpcgError{PPCG_EINVAL, "a batch cannot mix real and complex (Bloch) operators"};
        if (ps[b]->gen) throw PpcgError{PPCG_EINVAL, "the generalized problem (operator B) is not batched"};
        run.push_back(ps[b].get());
      } catch (const PpcgError& e) {
        ps[b]->status = e.code;
        ps[b]->err = e.msg;
      }
    }
    Driver d(h, true);
    d.run(run);
    for (int b = 0; b < nprob; ++b) {
      if (infos) infos[b] = ps[b]->info;
      if (statuses) statuses[b] = ps[b]->status;
      if (ps[b]->status != PPCG_OK && first == PPCG_OK) {
        first = ps[b]->status;
        h->err = "problem " + std::to_string(b) + ": " + ps[b]->err;
      }
    }
    return first;
  });
}

ppcg_status ppcg_grad(ppcg_handle* h, const double* g_lambda, const double* w, double* dL_dV, double tol,
                      int32_t max_iter, int32_t* iters, double* resid) {
  if (!h) return PPCG_EINVAL;
  return guard(h, [&]() {
    Grad g(h);
    int it = g.run(g_lambda, w, dL_dV, tol, max_iter > 0 ? max_iter : 10000);
    if (iters) *iters = it;
    if (resid) *resid = g.resid;
    if (g.resid > tol) {
      h->err = "Sternheimer block CG stopped at max_iter with relative residual " + std::to_string(g.resid);
      return PPCG_ENOCONV;
    }
    return PPCG_OK;
  });
}

ppcg_status ppcg_density(ppcg_handle* h, double* rho) {
  if (!h || !rho) return PPCG_EINVAL;
  return guard(h, [&]() {
    if (!h->has_state) throw PpcgError{PPCG_ENOSTATE, "ppcg_density needs a successful ppcg_solve on this handle"};
    launch_grad_rows(h->work(0).X.d(), nullptr, nullptr, h->s_ld, h->s_n, h->s_k, rho, h->st, h->s_cplx);
    HIPCHECK(hipGetLastError());
    sync(h);
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
    if (op->nx < 4 || !(op->h > 0)) throw PpcgError{PPCG_EINVAL, "bad grid: need nx >= 4 and h > 0"};
    double ih2 = 1.0 / (op->h * op->h);
    long n = (long)op->nx * op->nx * op->nx;
    StencilArgs a{};
    a.X = X;
    a.Y = Y;
    a.ldx = a.ldy = n;
    a.ncols = ncols;
    a.N = op->nx;
    a.order = op->order;
    a.c0 = op->order == 2 ? 3.0 * ih2 : 3.75 * ih2;
    a.w1 = op->order == 2 ? -0.5 * ih2 : -2.0 / 3.0 * ih2;
    a.w2 = op->order == 2 ? 0.0 : ih2 / 24.0;
    a.V = op->V;
    a.f32 = 0;
    a.cplx = bloch_phases(op, a.ph);
    {
      Scope sc(h->prof, "stencil_f64");
      launch_stencil(a, h->st);
    }
    HIPCHECK(hipGetLastError());
    sync(h);
    return PPCG_OK;
  });
}

ppcg_status ppcg_start_block(ppcg_handle* h, int64_t n, int32_t ncols, int32_t cplx, uint64_t seed, double* X) {
  if (!h || n < 0 || n > (int64_t(1) << 31) || ncols < 0 || ncols > 65535 || (n > 0 && ncols > 0 && !X))
    return PPCG_EINVAL;
  return guard(h, [&]() {
    launch_randn(X, (long)n, (long)n, ncols, seed, cplx != 0, h->st);
    HIPCHECK(hipGetLastError());
    sync(h);
    return PPCG_OK;
  });
}

ppcg_status ppcg_block_pencils(ppcg_handle* h, int32_t nblocks, int32_t q, int32_t has_p, int32_t cplx,
                               const double* A, const double* B, double tol, double* C, int32_t* flags) {
  if (!h || nblocks < 0 || q < 1 || q > 32 || !(tol > 0) || (nblocks > 0 && (!A || !B || !C || !flags)))
    return PPCG_EINVAL;
  return guard(h, [&]() {
    if (nblocks == 0) return PPCG_OK;
    const PencilLayout L = pencil_layout(nblocks, q, has_p != 0, cplx != 0);
    h->pen_gram.ensure(L.gram_bytes);
    h->pen_G.ensure(L.g_bytes);
    if (L.work_bytes) h->pen_work.ensure(L.work_bytes);
    enqueue_pencils(h, nblocks, q, has_p != 0, cplx != 0, A, B, tol, C, flags, h->pen_gram.d(), h->pen_G.d(),
                    L.work_bytes ? h->pen_work.p : nullptr);
    sync(h);
    return PPCG_OK;
  });
}

ppcg_status ppcg_block_pencils_noalloc(ppcg_handle* h, int32_t nblocks, int32_t q, int32_t has_p, int32_t cplx,
                                       const double* A, const double* B, double tol, double* C, int32_t* flags) {
  if (!h || nblocks < 0 || q < 1 || q > 32 || !(tol > 0) || (nblocks > 0 && (!A || !B || !C || !flags)))
    return PPCG_EINVAL;
  return guard(h, [&]() {
    if (nblocks == 0) return PPCG_OK;
    const PencilLayout L = pencil_layout(nblocks, q, has_p != 0, cplx != 0);
    if (L.total() > NOALLOC_SCRATCH_BYTES)
      throw PpcgError{PPCG_EINVAL, "ppcg_block_pencils_noalloc: " + std::to_string(nblocks) +
                                       " pencils need " + std::to_string(L.total()) + " bytes of scratch, more than " +
                                       std::to_string(NOALLOC_SCRATCH_BYTES)};
    char* base = (char*)h->noalloc_scratch;  // this device's copy of the static array (set by ppcg_create)
    if (!base) throw PpcgError{PPCG_EHIP, "no-allocation scratch of this device not resolved"};
    enqueue_pencils(h, nblocks, q, has_p != 0, cplx != 0, A, B, tol, C, flags, (double*)base,
                    (double*)(base + L.g_off), L.work_bytes ? (void*)(base + L.work_off) : nullptr);
    HIPCHECK(hipGetLastError());
    return PPCG_OK;
  });
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

void ppcg_reset_kernel_times(ppcg_handle* h) {
  if (!h) return;
  try {
    h->prof.reset();
  } catch (...) {
  }
}

int32_t ppcg_tune_report(const ppcg_handle* h, char* buf, int32_t cap) {
  if (!h) return -1;
  std::string out;
  for (const auto& kv : h->tune) {
    const TuneKey& k = kv.first;
    const TuneChoice& c = kv.second;
    char line[256];
    snprintf(line, sizeof line, "%s site=%d %s%s%s%s %s<=%d N<=%d rows<=%ld -> %s target=%d floor=%d %.3f ms [", 
             k.kind == 2 ? "block-gram" : (k.kind ? "update" : "gram"), k.site, k.f32 ? "f32" : "f64", k.cplx ? " complex" : "",
             k.multi ? " batched-jobs" : "", k.upper ? (k.kind == 2 ? " with-P" : " upper") : "", k.kind ? "K" : "M", k.mb, k.nb, k.rb,
             c.lds == 3 ? "tiles16" : (c.lds == 2 ? "block" : (c.lds ? "lds" : "wave")), c.target, c.floor_rows, c.ms);
    out += line;
    out += c.tried;
    out += "]\n";
  }
  if (buf && cap > 0) {
    size_t w = std::min<size_t>(out.size(), (size_t)cap - 1);
    std::memcpy(buf, out.data(), w);
    buf[w] = 0;
  }
  return (int32_t)out.size();
}

void ppcg_destroy(ppcg_handle* h) { delete h; }

const char* ppcg_last_error(const ppcg_handle* h) { return h ? h->err.c_str() : "null handle"; }

}  // extern "C"
