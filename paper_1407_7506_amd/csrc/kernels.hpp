// Kernel argument structs and host-side launchers (internal to libppcg).
#pragma once
#include <hip/hip_runtime.h>

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
  int site;           // call site (selects a distinct kernel symbol for profiling)
};

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
};

void launch_gram(const GramArgs& a, int njobs, bool f32acc, hipStream_t st);
void launch_reduce(const ReduceArgs& r, bool f32, hipStream_t st);
void launch_update(const UpdateArgs& a, int njobs, bool f32, hipStream_t st);

// -------------------------------------------------------------------------
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
  const void* V;      // potential (same precision as X)
  int f32;
  const double* shift;  // optional per-column shift: Y[:, j] -= shift[j] X[:, j] (float64 only)
};
void launch_stencil(const StencilArgs& a, hipStream_t st);

// Y[r, j] = X[r, j] * d[r]  (d may be null: copy), optional float copy
void launch_scale_rows(const double* d, const void* X, void* Y, long ld, long rows, int ncols, int f32, hipStream_t st);
// Y32 = (float) X64, ncols columns
void launch_to_f32(const double* X, float* Y, long ld, long rows, int ncols, hipStream_t st);
// out[c] = sum_r |X[r, c]|^2 (X f64 or f32), deterministic
void launch_colnorm2(const void* X, int f32, long ld, long rows, int ncols, double* out, hipStream_t st);
// W[r, j] = AX[r, j] - X[r, j] * lam[j]; also out[j] = |W[:, j]|^2
void launch_ritz_resid(const double* AX, const double* X, const double* lam, double* W, float* W32, long ld,
                       long rows, int ncols, hipStream_t st);

// -------------------------------------------------------------------------
// block pencils (steps 12-13): one workgroup per sub-block
struct PencilArgs {
  const double* gram;   // per block: S^H [S | AW | AP], nS x (2 nS - q), ld = nS, stride gstride
  long gstride;
  const double* G;      // X^H A X of the active columns (m x m, ldg); the X block is G[jq.., jq..]
  int ldg;
  int q, nS;            // nS = 2q (no P) or 3q
  int ax_rows;          // 1: the Gram has q extra rows (H X_j)^H [...] after the nS rows of S, and the
                        //    X-W / X-P blocks of the projected A are taken from them
  double* C;            // out: per block nS x q (ld 3q), stride cstride
  long cstride;
  int* flags;           // out: per block bit0 = P used, bit1 = backtracked, bit2 = rank failure
  double drop_tol, pivot_tol;
  double jacobi_rel;    // rotations below jacobi_rel |M|_F are skipped
};
void launch_block_pencil(const PencilArgs& a, int nblocks, hipStream_t st);

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
};
void launch_block_update(const BlockUpdArgs& a, int nblocks, hipStream_t st);

// -------------------------------------------------------------------------
// dense m x m (column-major, ld) kernels
// Cholesky G = L L^H (lower), L and Linv written to separate buffers; flag
// set to 1 + (first failing diagonal block) on a non-positive pivot.
void chol_inverse(double* G, double* L, double* Linv, int m, int ld, int* flag, hipStream_t st);
// Upper triangle of dst = src^H (used to form R^{-1} = Linv^H)
void launch_transpose(const double* src, int lds, double* dst, int ldd, int m, int n, hipStream_t st);
void launch_fill(double* p, long count, double v, hipStream_t st);
void launch_set_diag(double* G, int ld, int m, const double* lam, hipStream_t st);
void launch_symmetrize(double* G, int ld, int m, hipStream_t st);

// Hermitian eigensolver for m x m (ld) by block Jacobi; eigenvalues
// ascending in lam, eigenvectors in V (m x m, ldv).  Work buffers owned by
// the caller (size from eig_workspace_bytes).  Returns sweeps used.
size_t eig_workspace_bytes(int m);
int block_jacobi_eig(double* M, int ld, int m, double* V, int ldv, double* lam, void* work, int* hostbuf,
                     double rel_tol, hipStream_t st);

// backward pass (grad.hip)
void launch_coldot(const double* A, const double* B, long ld, long rows, int ncols, double* out, hipStream_t st);
void launch_cg_precond(const double* R, double* Y, const double* V, double c0, const double* lam, long ld, long n,
                       long rows, int ncols, int unprec, hipStream_t st);
void launch_cg_alpha(const double* rz, const double* pAp, const int* done, double* alpha, int k, hipStream_t st);
void launch_cg_beta(double* rz, const double* rznew, const int* done, double* beta, int k, hipStream_t st);
void launch_cg_xr(double* Z, double* R, const double* P, const double* AP, const double* alpha, long ld, long rows,
                  int k, hipStream_t st);
void launch_cg_p(double* P, const double* Y, const double* beta, long ld, long rows, int k, hipStream_t st);
void launch_cg_check(const double* rr, const double* bb, double tol, int* done, int* left, int k, hipStream_t st);
void launch_grad_rows(const double* X, const double* Z, const double* g, long ld, long n, int k, double* out,
                      hipStream_t st);

// rho and helpers: out[j] = sum_{i<nw} G[i, j]^2, j < nw
void launch_frob2_sub(const double* G, int ld, int nw, double* out, hipStream_t st);
// out = |G[:k, :k] - I|_F^2
void launch_orth_err2(const double* G, int ld, int k, double* out, hipStream_t st);

}  // namespace ppcg
