// Kernel argument structs, host-side launchers and the launch recorder
// (internal to libppcg).
//
// Every launcher either launches its kernel directly (one job, arguments by
// value) or, while a Recorder is active, appends (op kind, arguments,
// workgroup count) to the recorder.  The batched driver records the same
// stage for many problems and then issues one grouped launch per
// (position, op kind): the grouped kernel finds its job from a device job
// array by workgroup prefix sums.
#pragma once
#include <hip/hip_runtime.h>

#include <cstdint>
#include <cstring>
#include <vector>

namespace ppcg {

constexpr int kMaxSeg = 5;

// Up to kMaxSeg column segments (each from its own buffer, shared leading
// dimension), addressed as one column range; f32[s] marks float storage.
struct ColSet {
  const void* p[kMaxSeg];
  int end[kMaxSeg];  // cumulative column count after segment s
  bool f32[kMaxSeg];
  int nseg;
};

struct GramArgs {
  ColSet A, B;
  const double* dsc;  // optional row scale of B columns [0, nsc)
  int nsc;
  const double* dsc2; // optional row scale of B columns [nsc, N) (generalized problem: B P next to B T W)
  int M, N;
  long ld;            // leading dimension of every segment
  long rows;          // rows summed (multiple of 16)
  int splits;
  long chunk;         // rows per split (multiple of 16)
  void* out;          // partials: out + (job*splits + s)*split_stride + i + j*ldo
  long split_stride;
  int ldo;
  int tiles_i, tiles_j;
  int upper_only;
  long job_col_off;   // per-job element offset added to all column pointers
  int njobs;          // strided jobs (blocks) inside this gram
  int site;           // call site (selects a distinct kernel symbol for profiling)
  int cplx;           // complex operands (f32 segments then mean complex float)
  int lds;            // 1: LDS-staged 128 x 128 workgroup tiles (real, one job, chunk % 32 == 0);
                      // 2: per-block single pass (real, float64 accumulation, M <= 128, N <= 160)
  int il;             // LDS kernel on complex columns read as real columns of interleaved (re, im)
                      // rows (ld, rows and chunk in real rows): the row scale dsc is indexed by
                      // row / 2, and with rotB every B pair (re, im) is taken as (im, -re), so the
                      // real Gram is Re(A^H B) without and Im(A^H B) with it
  int rotB;
};

// Per-block Grams of the 3q x 3q pencils for q = 16, real: only the tiles the
// pencil reads.  Block j owns columns [16 j, 16 j + 16) of every slab.  Per
// block and split, 11 tiles of 16 x 16 (column-major) in this order:
//   overlap  0 X^T X, 1 X^T W, 2 X^T P, 3 W^T W, 4 W^T P, 5 P^T P
//   H        6 W^T AW, 7 W^T AP, 8 P^T AP,
//            9 X^T H W and 10 X^T H P (from AX^T W and AX^T P when AX is given,
//              else from X^T AW and X^T AP)
// Without P the tiles that involve P are not formed.
constexpr int BG_TILES = 11;
struct BlockGramArgs {
  const double* X;   // float64 slabs, ld
  const void* W;     // W, P, AW, AP: float32 when f32, else float64
  const void* P;
  const void* AW;
  const void* AP;
  const double* AX;  // optional float64 H X (mixed precision)
  long ld;
  long rows;         // multiple of 16
  int nblocks, hasP, f32;
  int splits;
  long chunk;        // rows per split (multiple of 16)
  double* out;       // partials: out + (block * splits + split) * BG_TILES * 256
};
void launch_block_gram(const BlockGramArgs& a, hipStream_t st);

struct ReduceArgs {
  const void* part;
  int M, N, ldp, splits;
  long split_stride;
  int njobs;
  void* dst;
  int ldd;
  long dst_job_stride;
  double alpha, beta;
  int upper_only;
  int cplx;          // complex entries; the mirrored entry of upper_only is conjugated
  long im_off;       // > 0: complex result from real partials, the imaginary parts at part + im_off
                     // elements (the two real Grams of an interleaved complex Gram)
};

struct UpdateArgs {
  const void* A;   // tall, rows x K, lda
  long lda, job_a_off;
  const void* B;   // small K x N, ldb
  long ldb, job_b_off;
  void* C0;        // output columns [0, N0)
  void* C1;        // output columns [N0, N)
  int N0;
  long ldc, job_c_off;
  void* C32;       // optional float copy of the output (same ldc), columns of C0
  const double* dsc;  // optional row scale of the old C0 values
  int K, N;
  long rows;       // multiple of 64
  double alpha, beta;
  int b_upper;     // B upper triangular: k range limited per column tile
  int c0_keep;     // 1: do not overwrite C0 (only the float copy C32 is written)
  int tiles_j, tiles_r;
  int site;        // call site (selects a distinct kernel symbol for profiling)
  int cplx;        // complex A, B, C (C32 then complex float)
  int lds;         // 1: LDS-staged 128 x 128 workgroup tiles (real, one job, rows % 128 == 0)
  double* cpart;   // optional (real): per 64-row tile t and column j < ncn, the sum of squares of the
                   // stored values at cpart[t + j * ldp] (column norms without re-reading C)
  int ncn;
  long ldp;
  // optional (float32 kernels): float64 input c64 (ld ldc, complex interleaved
  // when cplx) read in place of C0, and the float64 term - xd[r, j] Re gd[j * gds]
  // added; the result is formed in float64 and stored through C32 (c0_keep)
  const double* c64;
  const double* xd;
  const double* gd;
  long gds;
};

// stencil: Y = H X on an N^3 periodic grid (7- or 13-point), columns [0, ncols)
struct StencilArgs {
  const void* X;
  void* Y;
  long ldx, ldy;
  int ncols;
  int N;
  int order;
  double c0;          // 3 w0 / h^2
  double w1, w2;      // off-diagonal weights / h^2
  const void* V;      // potential (real, same precision as X)
  int f32;
  const double* shift;  // optional per-column shift: Y[:, j] -= shift[j] X[:, j] (float64 only)
  int cplx;           // complex X, Y (interleaved); Bloch phases below
  double ph[3][2][2]; // ph[d][a-1] = exp(i kappa_d a h) as (re, im), a = 1, 2
};

// block pencils (steps 12-13): one workgroup per sub-block
struct PencilArgs {
  const double* gram;   // per block: Gram rows x (2 nS - q), ld = rows (or BG_TILES tiles), stride gstride
  long gstride;
  const double* G;      // X^H A X of the active columns (m x m, ldg); the X block is G[jq.., jq..]
  int ldg;
  int q, nS;            // nS = 2q (no P) or 3q
  int ax_rows;          // 1: the Gram has q extra rows (H X_j)^H [...] after the nS rows of S, and the
                        //    X-W / X-P blocks of the projected A are taken from them
  double* C;            // out: per block nS x q (ld 3q), stride cstride
  long cstride;
  int* flags;           // out: per block bit0 = P used, bit1 = backtracked, bit2 = rank failure,
                        //      bits 8.. = W/P columns of the solved pencil left out (zero or dependent)
  double drop_tol, pivot_tol;
  double sing_tol;      // Theorem 1 test: C_X singular when a Cholesky pivot of C_X^H C_X is below it
  double jacobi_rel;    // rotations below jacobi_rel |M|_F are skipped
  int nblocks;
  int cplx;             // complex Hermitian pencils (gram, G and C complex)
  int tiles16;          // 1: gram holds the BG_TILES tiles of the 16-column block Gram kernel
  void* work;           // nS > 48 only: per block 4 * 96 * 97 scalars of device scratch for the
                        // pencil matrices (too large for LDS), stride pencil_work_elems()
};
// scalars of device scratch one block pencil with nS > 48 uses
constexpr long pencil_work_elems() { return 4L * 96 * 97; }
// given pencils (A_j, B_j) -> the block pencil kernel's gram / G input layout (one launch)
void launch_pencil_pack(const double* A, const double* B, int nblocks, int q, int nS, int cplx, double* gram,
                        double* G, hipStream_t st);

// block update (steps 14-15): P_j <- W_j C_W + P_j C_P ; X_j <- X_j C_X + P_j
struct BlockUpdArgs {
  double* X;       // f64 master, columns of block j at X + j*q*ld
  void* W;         // f64 or f32
  void* P;         // f64 or f32
  int f32;         // W/P storage
  int hasP;
  long ld, rows;
  int q;
  const double* C;  // per block (3q x q, ld 3q), stride cstride
  long cstride;
  int nblocks;
  int cplx;         // complex X, W, P and C
};

// small per-problem kernels
struct ColnormArgs { const void* X; int f32; long ld, rows; int ncols; double* out; int sum; };  // sum: plain column sums
// W = AX - (B) X diag(lam); b: optional diagonal B of a generalized problem, indexed by row >> bshift
// (complex columns read as real columns of twice the length: bshift = 1)
struct RitzArgs { const double* AX; const double* X; const double* lam; double* W; float* W32; long ld, rows; int ncols;
                  const double* b; int bshift; };
struct TransposeArgs { const double* src; int lds; double* dst; int ldd; int m, n; int cplx; };  // cplx: conjugate
struct FillArgs { double* p; long count; double v; };
struct SetDiagArgs { double* G; int ld, m; const double* lam; int cplx; };
struct SymmArgs { double* G; int ld, m; int cplx; };
// F (float, ldf) <- G with a zero diagonal (m x m; complex interleaved when cplx)
struct OffdiagArgs { const double* G; int ldg, m; float* F; int ldf; int cplx; };
struct Frob2Args { const double* G; int ld, nw; double* out; int cplx; };
// |G - I|_F^2 of a k x k Gram; upper: only the upper triangle of G is valid
struct OrthArgs { const double* G; int ld, k; double* out; int cplx; int upper; };
// Taylor polar step (section 5.5): from the upper triangle of G = X^H X,
// Y = G - I (Hermitian) and M = (3/8) I - (5/16) Y, m x m at leading dimension ld
struct PolarArgs { const double* G; int ld, m; double* Y; double* M; int cplx; };
// G += v I on the m x m leading block
struct AddDiagArgs { double* G; int ld, m; double v; int cplx; };
// out[0] = sum_i Re G_ii over the m x m leading block (one workgroup)
struct TraceArgs { const double* G; int ld, m; double* out; int cplx; };
// float shadow of a float64 block: Y = (float) X over rows x ncols (ld in elements)
struct ToF32Args { const double* X; float* Y; long ld, rows; int ncols; int cplx; };
struct ZeroIntArgs { int* p; int n; };
struct CopyArgs { const double* src; double* dst; long count; };
struct PrepArgs { const double* V; long n; double c0; double* td; float* V32; double* dmin_part; int nparts; int* nan_flag; };
// Cholesky G = L L^H (lower) of an m x m block with L, L^{-1}; composite op
struct CholArgs { double* G; double* L; double* Li; int m, ld; int* flag; int cplx; };
// device-to-host copy (executed in order at its position, not grouped)
struct D2HArgs { void* dst; const void* src; size_t bytes; };

enum OpKind : int {
  OP_GRAM_D0, OP_GRAM_D1, OP_GRAM_D2, OP_GRAM_F0, OP_GRAM_F1, OP_GRAM_F2,
  OP_GRAM_Z0, OP_GRAM_Z1, OP_GRAM_Z2, OP_GRAM_C0, OP_GRAM_C1, OP_GRAM_C2,
  OP_GRAML_D0, OP_GRAML_D1, OP_GRAML_F0, OP_GRAML_F1, OP_GRAMB_1, OP_GRAMB_2,
  OP_REDUCE_D, OP_REDUCE_F, OP_REDUCE_Z, OP_REDUCE_C,
  OP_UPDATE_D0, OP_UPDATE_D1, OP_UPDATE_F0, OP_UPDATE_F1,
  OP_UPDATE_Z0, OP_UPDATE_Z1, OP_UPDATE_C0, OP_UPDATE_C1,
  OP_UPDATEL_D0, OP_UPDATEL_D1, OP_UPDATEL_F0, OP_UPDATEL_F1,
  OP_STENCIL_D2, OP_STENCIL_D4, OP_STENCIL_F2, OP_STENCIL_F4,
  OP_STENCIL_Z2, OP_STENCIL_Z4, OP_STENCIL_C2, OP_STENCIL_C4,
  OP_COLNORM_D, OP_COLNORM_F, OP_RITZ,
  OP_PENCIL24, OP_PENCIL48, OP_PENCIL96, OP_PENCILZ24, OP_PENCILZ48, OP_PENCILZ96,
  OP_BUPD_D4, OP_BUPD_D8, OP_BUPD_D16, OP_BUPD_D32, OP_BUPD_F4, OP_BUPD_F8, OP_BUPD_F16, OP_BUPD_F32,
  OP_BUPD_Z4, OP_BUPD_Z8, OP_BUPD_Z16, OP_BUPD_Z32, OP_BUPD_C4, OP_BUPD_C8, OP_BUPD_C16, OP_BUPD_C32,
  OP_TRANSPOSE, OP_FILL, OP_SETDIAG, OP_SYMM, OP_FROB2, OP_ORTH, OP_ZEROINT, OP_COPY, OP_PREP, OP_OFFDIAG,
  OP_POLAR, OP_ADDDIAG, OP_TRACE, OP_TOF32,
  OP_CHOL,   // composite: expanded by the grouped executor
  OP_D2H,    // host copy
  OP_COUNT
};

struct RecOp {
  int kind;
  unsigned nwg;
  std::vector<uint8_t> args;
  const char* name = nullptr;  // profiling name and algorithmic work of the op
  double fl = 0, by = 0;
};

struct Recorder {
  std::vector<std::vector<RecOp>> lists;  // one op list per problem
  int cur = -1;
  // work model of the op about to be recorded (set by the profiler scope)
  const char* pend_name = nullptr;
  double pend_fl = 0, pend_by = 0;
  void begin(int nprob) {
    lists.assign(nprob, {});
    cur = -1;
  }
  void add(int kind, const void* a, size_t sz, unsigned nwg) {
    RecOp op;
    op.kind = kind;
    op.nwg = nwg;
    op.args.resize(sz);
    std::memcpy(op.args.data(), a, sz);
    op.name = pend_name;
    op.fl = pend_fl;
    op.by = pend_by;
    pend_name = nullptr;
    pend_fl = pend_by = 0;
    lists[cur].push_back(std::move(op));
  }
};
extern thread_local Recorder* g_rec;  // non-null while the batched driver of this thread records

// Pinned host staging + device mirror for job arrays.  Bump allocation; the
// owner calls reset() only after synchronising the stream, so a region is
// never rewritten while its host-to-device copy may be pending.  Chunks that
// overflow are kept until reset.
struct Stage {
  struct Chunk { uint8_t* h; uint8_t* d; size_t cap, used; };
  std::vector<Chunk> chunks;
  std::vector<Chunk> retired;
  ~Stage();
  // copies `bytes` from src into the staging area and enqueues the upload;
  // returns the device address
  void* upload(const void* src, size_t bytes, hipStream_t st);
  void reset();
};

// Grouped launch of `nj` jobs of op `kind` (device job array, device start
// array of nj+1 prefix sums, `total` workgroups).  Returns false for kinds
// that cannot be grouped.
bool launch_grouped(int kind, const void* jobs, const unsigned* start, int nj, unsigned total, hipStream_t st);
size_t op_args_size(int kind);

void launch_gram(const GramArgs& a, bool f32acc, hipStream_t st);
void launch_reduce(const ReduceArgs& r, bool f32, hipStream_t st);
void launch_update(const UpdateArgs& a, bool f32, hipStream_t st);
void gram_tiles(GramArgs& a);
void update_tiles(UpdateArgs& a);
void launch_stencil(const StencilArgs& a, hipStream_t st);

// Y[r, j] = X[r, j] * d[r]  (d may be null: copy)
void launch_scale_rows(const double* d, const void* X, void* Y, long ld, long rows, int ncols, int f32, hipStream_t st);
// out[c] = sum_r |X[r, c]|^2 (X f64 or f32), deterministic
void launch_colnorm2(const void* X, int f32, long ld, long rows, int ncols, double* out, hipStream_t st);
// out[j] = sum_r P[r + j ld], r < rows (double; fixed reduction order)
void launch_colsum(const double* P, long ld, long rows, int ncols, double* out, hipStream_t st);
// W[r, j] = AX[r, j] - X[r, j] * lam[j] (W and/or its float copy W32)
void launch_ritz_resid(const double* AX, const double* X, const double* lam, double* W, float* W32, long ld,
                       long rows, int ncols, hipStream_t st, const double* b = nullptr, int bshift = 0);

void launch_block_pencil(const PencilArgs& a, hipStream_t st);
void launch_block_update(const BlockUpdArgs& a, hipStream_t st);

// dense m x m (column-major, ld) kernels
// Cholesky G = L L^H (lower), L and Linv written to separate buffers; flag
// set to 1 + (first failing diagonal block) on a non-positive pivot.
void chol_inverse_grouped(const std::vector<CholArgs>& jobs, Stage& stage, hipStream_t st);
// dst (n x m) = src^T (src^H when cplx)
void launch_transpose(const double* src, int lds, double* dst, int ldd, int m, int n, int cplx, hipStream_t st);
void launch_offdiag32(const double* G, int ldg, int m, float* F, int ldf, int cplx, hipStream_t st);
void launch_fill(double* p, long count, double v, hipStream_t st);
void launch_set_diag(double* G, int ld, int m, const double* lam, int cplx, hipStream_t st);
void launch_symmetrize(double* G, int ld, int m, int cplx, hipStream_t st);
// out[j] = sum_{i<nw} G[i, j]^2, j < nw
void launch_frob2_sub(const double* G, int ld, int nw, double* out, int cplx, hipStream_t st);
// out = |G[:k, :k] - I|_F^2
void launch_orth_err2(const double* G, int ld, int k, double* out, int cplx, hipStream_t st, bool upper = false);
void launch_polar_prep(const double* G, int ld, int m, double* Y, double* M, int cplx, hipStream_t st);
void launch_add_diag(double* G, int ld, int m, double v, int cplx, hipStream_t st);
void launch_trace(const double* G, int ld, int m, double* out, int cplx, hipStream_t st);
void launch_to_f32(const double* X, float* Y, long ld, long rows, int ncols, int cplx, hipStream_t st);
void launch_copy(const double* src, double* dst, long count, hipStream_t st);
void launch_d2h(void* dst, const void* src, size_t bytes, hipStream_t st);

// Hermitian eigensolver for m x m (ld) by block Jacobi; eigenvalues
// ascending in lam, eigenvectors in V (m x m, ldv).  Work buffers owned by
// the caller (size from eig_workspace_bytes).  Returns sweeps used.
size_t eig_workspace_bytes(int m, int cplx);
struct EigJob { double* M; int ld, m; double* V; int ldv; double* lam; void* work; double rel_tol; int cplx; };
// One sweep of the block Jacobi (every round's pair and update launches and the
// read-back of its rotation count) captured as a HIP graph, kept for as long
// as the job array (problem pointers and shapes) stays the same: successive
// Rayleigh-Ritz steps of a solve replay it instead of re-issuing the launches.
// With a cache the eigensolve runs on the cache's own stream; the caller's
// stream must have no pending work that the eigensolve depends on (the solver
// synchronizes it first), and the call returns with that stream drained.
struct EigGraphCache {
  std::vector<uint8_t> key;     // job array + workgroup prefix sums the graph was captured for
  void* dev = nullptr;          // device copy of that array (fixed address, read by the graph)
  size_t cap = 0;
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
  hipStream_t stream = nullptr;  // the library's own stream (capture is not possible on the null stream)
  void clear();
  ~EigGraphCache();
};
// All problems in lockstep (one workgroup set per problem and launch);
// dev_counter / host_counter: one int of device / pinned host memory for the
// stop test after each sweep.  Synchronises the stream once per sweep.
// Returns the sweeps used.
int block_jacobi_eig_grouped(const std::vector<EigJob>& jobs, Stage& stage, EigGraphCache* graphs, int* dev_counter,
                             int* host_counter,
                             hipStream_t st);

// backward pass (grad.hip)
void launch_coldot(const double* A, const double* B, long ld, long rows, int ncols, double* out, hipStream_t st);
void launch_cg_precond(const double* R, double* Y, const double* V, double c0, const double* lam, long ld, long n,
                       long rows, int ncols, int unprec, hipStream_t st, int cplx = 0);
void launch_cg_alpha(const double* rz, const double* pAp, const int* done, double* alpha, int k, hipStream_t st);
void launch_cg_beta(double* rz, const double* rznew, const int* done, double* beta, int k, hipStream_t st);
void launch_cg_xr(double* Z, double* R, const double* P, const double* AP, const double* alpha, long ld, long rows,
                  int k, hipStream_t st);
void launch_cg_p(double* P, const double* Y, const double* beta, long ld, long rows, int k, hipStream_t st);
void launch_cg_check(const double* rr, const double* bb, double tol, int* done, int* left, int k, hipStream_t st);
void launch_grad_rows(const double* X, const double* Z, const double* g, long ld, long n, int k, double* out,
                      hipStream_t st, int cplx = 0);
// Y = diag(w) X over rows x ncols (complex columns: both parts), leading dimension ld elements
void launch_scale_rows_c(const double* w, const double* X, double* Y, long ld, long rows, int ncols, int cplx,
                         hipStream_t st);

void launch_prep_diag(const double* V, long n, double c0, double* td, float* V32, double* dmin_part, int nparts,
                      int* nan_flag, hipStream_t st);
void launch_zero_int(int* p, int n, hipStream_t st);
// N(0,1) start block (Philox-4x32-10 counter (row, column), Box-Muller); launched directly, also
// while a batch records (it is the first step of the start-up phase)
void launch_randn(double* X, long ld, long n, int ncols, uint64_t seed, bool cplx, hipStream_t st);

}  // namespace ppcg
