// Device kernels of the block-sparse PINVIT path and their host launchers.
#pragma once
#include <hip/hip_runtime.h>

#include <cstdint>

namespace pv {

// One product C = alpha * op(A) op(B) + beta * C, all column-major.
// op(A) is M x K (ta = 0: A[i + k*lda], ta = 1: A[k + i*lda]); op(B) is K x N
// (tb = 0: B[k + j*ldb], tb = 1: B[j + k*ldb]).  [kbeg, kend) restricts the K range.
struct GemmDesc {
  const double* A;
  const double* B;
  double* C;
  int M, N, K, lda, ldb, ldc;
  int ta, tb;
  double alpha, beta;
  int tile0, tiles_n, kbeg, kend;
};

// Split-K reduction: C = alpha * sum_s P[s] + beta * C, P[s] is M x N with ld M.
struct ReduceDesc {
  double* C;
  const double* P;
  int M, N, ldc, S;
  double alpha, beta;
  int64_t elem0;  // prefix sum of M*N over descriptors
};

// Symmetric eigenproblem of the n x n matrix A (upper triangle read): eigenvalues w
// (descending) and orthonormal eigenvectors V (n x n, ld n, column j for w[j]).
struct EigDesc {
  const double* A;
  int lda, n;
  double* V;
  double* w;
  double* work;  // n*n + n(n+1)/2 doubles
  int* sweeps;   // optional: number of sweeps taken (diagnostics), may be null
  double abs_tol;  // rotations need |a_pq| > abs_tol * max_i |a_ii| (0: relative test only)
};

// W-step (application of one MPO site to a partially contracted tensor).
// Output block: T2[a, b', c'] (a < rows, b' < wq_out, c' < cols), column-major in
// (a, b', c').  For output state b' (global index bglob), with local operator
// entries of row (s_out, bglob) in the CSR arrays: value += val * src[s_in][q_in].
struct WBlock {
  double* out;
  int rows, cols, wq_out, qoff_out;
  int s_out;
  int src;  // index of the WSrc table row (8 entries: s_in*4... see kernels.hip)
};
struct WSrc {
  const double* base[2][5];  // [s_in][q_in + 2], null if absent
  int64_t ld[2][5];          // stride between consecutive c' (rows * w_q of the source)
  int rows_w[2][5];          // rows of the source (must equal the output rows)
  int col0[2][5];            // first column of the s_in part in the source block
};
struct WItem {
  int block;
  int bprime;  // global state index at the output cut
};

// Batched copies dst = alpha * src of r x c sub-blocks (column-major).
struct CopyDesc {
  const double* src;
  double* dst;
  int rows, cols, lds, ldd;
  double alpha;
  int64_t elem0;
};

// Column scaling dst[:, j] = src[:, j] * s[j] (r x c).
struct ScaleDesc {
  const double* src;
  double* dst;
  const double* s;
  int rows, cols, lds, ldd;
  int64_t elem0;
  int invert;  // 1: multiply by 1/s[j] (0 when s[j] == 0)
  int sqrt_s;  // 1: use sqrt(max(s[j], 0))
};

void launch_gemm(const GemmDesc* d_desc, int nprob, int total_tiles, hipStream_t s);
void launch_reduce(const ReduceDesc* d_desc, int nd, int64_t total, hipStream_t s);
// mode: 2 = matrix and vectors in LDS, 1 = matrix in LDS, 0 = global memory; all
// problems of one launch must admit the chosen mode at size nmax.
void launch_eig(const EigDesc* d_desc, int nprob, int nmax, int mode, hipStream_t s);
// Fastest mode available for an n x n problem on this device.
int eig_mode(int n);
// Tridiagonalisation, bisection + inverse iteration, back-transformation (three
// launches); work holds tri_work_doubles(n) doubles; abs_tol is the relative cut below
// which eigenvectors are returned as zero.
void launch_eig_tridiag(const EigDesc* d_desc, int nprob, int nmax, hipStream_t s);
inline size_t tri_work_doubles(int n) { return size_t(7) * n * n + size_t(3) * n + 1; }
// Blocked Cholesky factorisation W W^T ~ A of a symmetric positive semidefinite matrix, in
// place (lower triangle; the upper triangle is zeroed).  A column whose pivot (Schur
// complement diagonal) is at most kCholDrop times its original diagonal entry depends
// linearly on the earlier columns to working accuracy and is set to zero, so the residual
// A - W W^T stays at that level.  One launch per panel of kCholB columns: the panel kernel
// factors the diagonal block and solves for the rows below it; the caller applies the
// trailing update A22 -= L21 L21^T (a GEMM) before the next panel.  dg (n doubles) keeps
// the original diagonal.
struct CholDesc {
  double* A;
  double* dg;
  int n, lda;
};
constexpr int kCholB = 32;
constexpr double kCholDrop = 1e-12;
void launch_chol_panel(const CholDesc* d, int nprob, int j0, hipStream_t s);
void launch_wstep(const WItem* items, int nitems, const WBlock* blocks, const WSrc* srcs,
                  const int32_t* row_ptr, const int32_t* b_in, const uint8_t* s_in,
                  const int8_t* q_in, const int32_t* qoff_in, const double* val, int w_out,
                  hipStream_t s);
void launch_copy(const CopyDesc* d, int nd, int64_t total, hipStream_t s);
void launch_scale(const ScaleDesc* d, int nd, int64_t total, hipStream_t s);
void launch_sumsq(const double* x, int64_t n, double* out, hipStream_t s);
void launch_fill(double* x, int64_t n, double v, hipStream_t s);

constexpr int kGemmBM = 64, kGemmBN = 64, kGemmBK = 16;
constexpr int kEigMax = 1024;

}  // namespace pv
