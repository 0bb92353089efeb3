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
  // tile order: 0 = row blocks slowest (tiles sharing a row block of A are neighbours),
  // 1 = row blocks fastest (tiles sharing a column block of B are neighbours); tiles_m =
  // number of row blocks
  int tiles_m, colmajor;
  // m1 > 0: the rows of op(A) and C are pairs (r, s) with i = r + m1 s (ta = 0 only): row i
  // of A starts at A + r + s * a_outer, row i of C at C + r + s * c_outer.  A batch of
  // products that share B and differ by fixed strides in A and C runs as one product.
  int m1;
  int64_t a_outer, c_outer;
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
  // tridiagonal solver: eigenvectors for the nvec largest eigenvalues only (negative: all);
  // the other columns of V are zero.  The Jacobi solver always returns all.
  int nvec = -1;
};

// W-step (application of one MPO site to a partially contracted tensor).  Task t writes
// the elements x in [x0, min(x0 + kWTask, n)) of one output block, x = a + rows c',
// out[a + ldo c'] = sum over the task's entries e of val_e * src_e[a + ld_e c'].  The host
// resolves the MPO's sparse entries into (source pointer, stride, coefficient) triples.
struct WEntry {
  const double* src;
  int64_t ld;
  double val;
};
struct WTask {
  double* out;
  int64_t ldo;
  int rows, n, x0, e0, e1;
};
constexpr int kWElems = 8;              // output elements per thread
constexpr int kWTask = 256 * kWElems;   // output elements per task (one workgroup)

// Batched copies dst = alpha * src of r x c sub-blocks (column-major); a null src fills the
// block with alpha.
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

// prec 0: float64 MFMA; prec 1: operands rounded to float32, float32 MFMA accumulation;
// prec 2: float64 MFMA, the instance used for the trailing updates of the tridiagonal
// reduction; prec 3: operands rounded to bfloat16, float32 MFMA accumulation.
// d_tmap[t] = index of the descriptor that owns tile t (tiles numbered by tile0).
void launch_gemm(const GemmDesc* d_desc, const int* d_tmap, int total_tiles, int prec, hipStream_t s,
                 bool small = false, hipEvent_t ev_start = nullptr, hipEvent_t ev_stop = nullptr);
// Batches of at most kGemmPack problems pass their descriptors in the kernel arguments.
constexpr int kGemmPack = 16;
struct GemmPack {
  GemmDesc d[kGemmPack];
};
void launch_gemm_packed(const GemmPack& pack, int nprob, int total_tiles, int prec, hipStream_t s,
                        bool small = false, hipEvent_t ev_start = nullptr, hipEvent_t ev_stop = nullptr);
void launch_reduce(const ReduceDesc* d_desc, int nd, int64_t total, hipStream_t s);
// mode: 2 = matrix and vectors in LDS, 1 = matrix in LDS, 0 = global memory; all
// problems of one launch must admit the chosen mode at size nmax.
void launch_eig(const EigDesc* d_desc, int nprob, int nmax, int mode, hipStream_t s);
// Fastest mode available for an n x n problem on this device.
int eig_mode(int n);
// Tridiagonal eigensolver.  Reduction: launch_tri_prepare, then for k0 = 0, kTriPanel, ...
// while k0 + 2 < nmax one launch_tri_panel followed by the trailing update of every
// problem with k0 + 2 < n, A[o:, o:] -= P1[o:, :] P2[o:, :]^T with o = k0 + nbe,
// nbe = min(kTriPanel, n - 2 - k0), P1 = work + n^2, P2 = P1 + 2 nbe n (ld n, 2 nbe columns),
// then launch_tri_finish.  After it, launch_eig_tridiag runs eigenvalues by bisection
// (phase bit 2), eigenvectors by inverse iteration (bit 4) and the back-transformation
// (bit 8), one launch each, in that order (the eigenvalues are final after bit 2, so a
// caller may read them and set nvec before the vector phases).  work holds
// tri_work_doubles(n) doubles and carries the state between launches; abs_tol is the
// relative cut below which eigenvectors are returned as zero.
constexpr int kTriPanel = 32;
void launch_tri_prepare(const EigDesc* d_desc, int nprob, int nmax, hipStream_t s);
void launch_tri_panel(const EigDesc* d_desc, int nprob, int nmax, int k0, hipStream_t s);
void launch_tri_finish(const EigDesc* d_desc, int nprob, hipStream_t s);
// The reduction one step per launch instead of the panels: after launch_tri_prepare, one
// launch_tri_step for every k = 0 .. max(nmax - 2, 0), with G workgroups per problem; it
// leaves the same state as the panels and launch_tri_finish (no trailing GEMMs).
void launch_tri_step(const EigDesc* d_desc, int nprob, int nmax, int k, int G, hipStream_t s);
// The remaining steps of every problem from k0 = max(n - tri_tail_rows(), 0) on, one
// workgroup per problem with the trailing block in LDS; the step launches for a problem
// stop at k0 - 1.  Leaves d, e, beta and the reflectors as the step launches would.
void launch_tri_tail(const EigDesc* d_desc, int nprob, hipStream_t s);
int tri_tail_rows();
// Float64 MFMA rate probe: blocks workgroups of 256 threads, iters steps of four
// 16x16x4 products per wavefront (2048 flops each); out takes 256 doubles per workgroup.
void launch_mfma_rate(double* out, int blocks, int iters, hipStream_t s);
void launch_eig_tridiag(const EigDesc* d_desc, int nprob, int nmax, int phases, hipStream_t s);
inline size_t tri_work_doubles(int n) { return size_t(7) * n * n + size_t(5) * n + 2; }
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
void launch_wstep(const WTask* tasks, int ntasks, const WEntry* entries, hipStream_t s);
void launch_copy(const CopyDesc* d, int nd, int64_t total, hipStream_t s);
void launch_scale(const ScaleDesc* d, int nd, int64_t total, hipStream_t s);
void launch_sumsq(const double* x, int64_t n, double* out, hipStream_t s);
void launch_fill(double* x, int64_t n, double v, hipStream_t s);

constexpr int kGemmBM = 64, kGemmBN = 64, kGemmBK = 16;
// float64 launches of at most kGemmSmallTiles 64 x 64 tiles (fewer than one workgroup per
// compute unit) run kGemmSmall x kGemmSmall tiles instead: four times the workgroups for
// MFMA chains a quarter as long.  Each element's products are summed in the same order
// (same K-steps, same position in its 16 x 16 MFMA block), so the results are the same bits.
constexpr int kGemmSmall = 32;
constexpr int64_t kGemmSmallTiles = 256;
constexpr int kGemmGroup = 4;  // consecutive tiles kept on one XCD
constexpr int kEigMax = 1024;

}  // namespace pv
