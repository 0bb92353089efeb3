// HIP kernels for gfx950: grouped FP64 MFMA GEMM, batched Jacobi eigensolver,
// MPO W-step, block copies/scalings and a wavefront-shuffle reduction.
#include <hip/hip_runtime.h>

#include <cfloat>
#include <cmath>
#include <cstdint>
#include <stdexcept>
#include <string>

#include "kernels.hpp"

namespace pv {

typedef double d4 __attribute__((ext_vector_type(4)));

__device__ inline double wave_sum_d(double v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
  return v;
}

#define PV_LAUNCH_CHECK()                                                          \
  do {                                                                             \
    hipError_t e_ = hipGetLastError();                                             \
    if (e_ != hipSuccess) throw std::runtime_error(std::string("kernel launch: ") + \
                                                   hipGetErrorString(e_));         \
  } while (0)

// ---------------------------------------------------------------------------
// Grouped GEMM.  One workgroup (4 waves) computes a 64x64 tile of one problem;
// each wave owns a 32x32 quadrant as 2x2 tiles of v_mfma_f64_16x16x4f64.
// Operand layout of that instruction (wave64): lane l supplies A[l%16][l/16] and
// B[l/16][l%16]; the 16x16 result lives in 4 doubles per lane, element r of lane l
// being D[4*r + l/16][l%16] (measured with a single-instruction probe on gfx950).
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void gemm_f64_kernel(const GemmDesc* __restrict__ descs, int nprob) {
  constexpr int BM = kGemmBM, BN = kGemmBN, BK = kGemmBK;
  __shared__ double As[BK][BM + 1];
  __shared__ double Bs[BK][BN + 1];
  const int tile = blockIdx.x;
  int lo = 0, hi = nprob - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (descs[mid].tile0 <= tile) lo = mid; else hi = mid - 1;
  }
  const GemmDesc g = descs[lo];
  const int t = tile - g.tile0;
  const int row0 = (t / g.tiles_n) * BM, col0 = (t % g.tiles_n) * BN;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int wr = wave >> 1, wc = wave & 1;
  const int li = lane & 15, lk = lane >> 4;
  d4 acc[2][2];
  for (int a = 0; a < 2; ++a)
    for (int b = 0; b < 2; ++b) acc[a][b] = d4{0.0, 0.0, 0.0, 0.0};

  for (int k0 = g.kbeg; k0 < g.kend; k0 += BK) {
    for (int e = tid; e < BM * BK; e += 256) {
      int i, k;
      if (!g.ta) { i = e % BM; k = e / BM; } else { k = e % BK; i = e / BK; }
      const int gi = row0 + i, gk = k0 + k;
      double v = 0.0;
      if (gi < g.M && gk < g.kend)
        v = g.ta ? g.A[gk + (int64_t)gi * g.lda] : g.A[gi + (int64_t)gk * g.lda];
      As[k][i] = v;
    }
    for (int e = tid; e < BN * BK; e += 256) {
      int j, k;
      if (!g.tb) { k = e % BK; j = e / BK; } else { j = e % BN; k = e / BN; }
      const int gj = col0 + j, gk = k0 + k;
      double v = 0.0;
      if (gj < g.N && gk < g.kend)
        v = g.tb ? g.B[gj + (int64_t)gk * g.ldb] : g.B[gk + (int64_t)gj * g.ldb];
      Bs[k][j] = v;
    }
    __syncthreads();
#pragma unroll
    for (int kk = 0; kk < BK; kk += 4) {
      double a0 = As[kk + lk][wr * 32 + li];
      double a1 = As[kk + lk][wr * 32 + 16 + li];
      double b0 = Bs[kk + lk][wc * 32 + li];
      double b1 = Bs[kk + lk][wc * 32 + 16 + li];
      acc[0][0] = __builtin_amdgcn_mfma_f64_16x16x4f64(a0, b0, acc[0][0], 0, 0, 0);
      acc[0][1] = __builtin_amdgcn_mfma_f64_16x16x4f64(a0, b1, acc[0][1], 0, 0, 0);
      acc[1][0] = __builtin_amdgcn_mfma_f64_16x16x4f64(a1, b0, acc[1][0], 0, 0, 0);
      acc[1][1] = __builtin_amdgcn_mfma_f64_16x16x4f64(a1, b1, acc[1][1], 0, 0, 0);
    }
    __syncthreads();
  }
  for (int mi = 0; mi < 2; ++mi)
    for (int nj = 0; nj < 2; ++nj)
      for (int r = 0; r < 4; ++r) {
        const int i = row0 + wr * 32 + mi * 16 + 4 * r + lk;
        const int j = col0 + wc * 32 + nj * 16 + li;
        if (i < g.M && j < g.N) {
          double v = g.alpha * acc[mi][nj][r];
          double* c = g.C + i + (int64_t)j * g.ldc;
          if (g.beta != 0.0) v += g.beta * *c;
          *c = v;
        }
      }
}

void launch_gemm(const GemmDesc* d_desc, int nprob, int total_tiles, hipStream_t s) {
  if (total_tiles <= 0) return;
  hipLaunchKernelGGL(gemm_f64_kernel, dim3(total_tiles), dim3(256), 0, s, d_desc, nprob);
  PV_LAUNCH_CHECK();
}

__global__ void reduce_kernel(const ReduceDesc* __restrict__ d, int nd, int64_t total) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= total) return;
  int lo = 0, hi = nd - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (d[mid].elem0 <= e) lo = mid; else hi = mid - 1;
  }
  const ReduceDesc r = d[lo];
  const int64_t x = e - r.elem0;
  const int i = int(x % r.M), j = int(x / r.M);
  const int64_t mn = (int64_t)r.M * r.N;
  double acc = 0.0;
  for (int s = 0; s < r.S; ++s) acc += r.P[s * mn + x];
  double* c = r.C + i + (int64_t)j * r.ldc;
  double v = r.alpha * acc;
  if (r.beta != 0.0) v += r.beta * *c;
  *c = v;
}

void launch_reduce(const ReduceDesc* d, int nd, int64_t total, hipStream_t s) {
  if (total <= 0) return;
  hipLaunchKernelGGL(reduce_kernel, dim3((total + 255) / 256), dim3(256), 0, s, d, nd, total);
  PV_LAUNCH_CHECK();
}

// ---------------------------------------------------------------------------
// Cyclic two-sided Jacobi eigensolver, one workgroup per matrix.
// Parallel ordering: the circle method pairs the n2 (= n rounded up to even) indices
// into n2/2 disjoint pairs per step, n2-1 steps per sweep meeting every pair once.
// All rotations of a step are applied at once as 2x2 block updates
// B_ij <- J_i^T B_ij J_j over the block rows/columns of the pairs.  The working
// matrix is the packed upper triangle; depending on the size it lives in LDS together
// with V (MODE 2), in LDS with V in global memory (MODE 1), or both in global memory
// (MODE 0).  A rotation is applied when |a_pq| > 1e-14 sqrt(|a_pp a_qq|) and
// |a_pq| > abs_tol max_i |a_ii|.  On a general matrix the updates leave rounding noise
// of order eps max|a_ii| in the small-eigenvalue block, which the relative test alone
// keeps rotating; an absolute floor above that noise (abs_tol = 1e-15) ends the sweeps.
// On nearly diagonal input (the second pass of a two-pass factorisation) the noise is
// local and abs_tol = 0 keeps small eigenvalues relatively accurate.  Sweeps stop when a
// sweep applies no rotation.
// ---------------------------------------------------------------------------
constexpr int kEigMaxPairs = kEigMax / 2;
constexpr double kJacobiTol = 1e-14;

__device__ inline int pidx(int r, int c) {  // packed upper, r <= c (n <= 1024: fits int32)
  return (c * (c + 1) >> 1) + r;
}
__device__ inline int sidx(int r, int c) { return r <= c ? pidx(r, c) : pidx(c, r); }

// Dynamic LDS of one problem in each mode (bytes).
__host__ __device__ inline size_t eig_lds_bytes(int n, int mode) {
  const int P = (n + (n & 1)) / 2;
  size_t b = size_t(P) * (2 * sizeof(double) + 2 * sizeof(int));
  if (mode >= 1) b += size_t(n) * (n + 1) / 2 * sizeof(double);
  if (mode == 2) b += size_t(n) * n * sizeof(double);
  return b;
}

constexpr int kEigBlocksPerThread = 8;  // (P(P+1)/2) / threads <= 8 for n <= 1024 at 1024 threads
                                        // is not guaranteed; larger counts fall back to a loop

template <int MODE>
__global__ __launch_bounds__(1024) void jacobi_eig_kernel(const EigDesc* __restrict__ descs, int maxsweep) {
  extern __shared__ double smem[];
  __shared__ int rotated;
  __shared__ double dmax;
  const EigDesc d = descs[blockIdx.x];
  const int n = d.n;
  if (n <= 0) return;
  const int tid = threadIdx.x, bs = blockDim.x;
  const int n2 = n + (n & 1), P = n2 / 2;
  double* lds = smem;
  double* Ap;
  double* Vw;
  if (MODE == 0) { Vw = d.work; Ap = d.work + (int64_t)n * n; }
  else if (MODE == 1) { Vw = d.work; Ap = lds; lds += n * (n + 1) / 2; }
  else { Ap = lds; lds += n * (n + 1) / 2; Vw = lds; lds += n * n; }
  double* rc = lds;
  double* rs = rc + P;
  int* rp = reinterpret_cast<int*>(rs + P);
  int* rq = rp + P;
  for (int c = 0; c < n; ++c)
    for (int r = tid; r <= c; r += bs) Ap[pidx(r, c)] = d.A[r + (int64_t)c * d.lda];
  for (int e = tid; e < n * n; e += bs) {
    const int col = e / n;
    Vw[e] = (e - col * n == col) ? 1.0 : 0.0;
  }
  // this thread's 2x2 blocks (i <= j) of the pair-indexed matrix, decoded once
  const int nb = P * (P + 1) / 2;
  int myblk[kEigBlocksPerThread];
  int nmine = 0;
  for (int e = tid; e < nb && nmine < kEigBlocksPerThread; e += bs) {
    int j = int((sqrtf(8.0f * float(e) + 1.0f) - 1.0f) * 0.5f);
    while ((j + 1) * (j + 2) / 2 <= e) ++j;
    while (j * (j + 1) / 2 > e) --j;
    myblk[nmine++] = ((e - j * (j + 1) / 2) << 16) | j;
  }
  const int extra_start = tid + kEigBlocksPerThread * bs;  // blocks beyond the cached ones
  __syncthreads();
  int sweeps = 0;
  for (int sweep = 0; sweep < maxsweep; ++sweep) {
    if (tid == 0) {
      rotated = 0;
      double m = 0.0;
      for (int i = 0; i < n; ++i) m = fmax(m, fabs(Ap[pidx(i, i)]));
      dmax = m;
    }
    __syncthreads();
    ++sweeps;
    const double abs_floor = fmax(d.abs_tol * dmax, 1e-300);
    for (int step = 0; step < n2 - 1; ++step) {
      for (int k = tid; k < P; k += bs) {
        int a, b;
        if (k == 0) { a = n2 - 1; b = step; }
        else {
          a = step + k; if (a >= n2 - 1) a -= n2 - 1;
          b = step - k; if (b < 0) b += n2 - 1;
        }
        const int p = min(a, b), q = max(a, b);
        double c = 1.0, s = 0.0;
        if (q < n) {
          const double app = Ap[pidx(p, p)], aqq = Ap[pidx(q, q)], apq = Ap[pidx(p, q)];
          if (fabs(apq) > kJacobiTol * sqrt(fabs(app * aqq)) && fabs(apq) > abs_floor) {
            const double th = (aqq - app) / (2.0 * apq);
            const double t = (th >= 0.0 ? 1.0 : -1.0) / (fabs(th) + sqrt(1.0 + th * th));
            c = 1.0 / sqrt(1.0 + t * t);
            s = t * c;
            rotated = 1;
          }
        }
        rp[k] = p; rq[k] = q; rc[k] = c; rs[k] = s;
      }
      __syncthreads();
      auto update = [&](int i, int j) {
        const double si = rs[i], sj = rs[j];
        if (si == 0.0 && sj == 0.0) return;
        const double ci = rc[i], cj = rc[j];
        const int pi = rp[i], qi = rq[i], pj = rp[j], qj = rq[j];
        if (i == j) {
          if (qi >= n) return;
          const double app = Ap[pidx(pi, pi)], aqq = Ap[pidx(qi, qi)], apq = Ap[pidx(pi, qi)];
          Ap[pidx(pi, pi)] = ci * ci * app - 2.0 * ci * si * apq + si * si * aqq;
          Ap[pidx(qi, qi)] = si * si * app + 2.0 * ci * si * apq + ci * ci * aqq;
          Ap[pidx(pi, qi)] = 0.0;
        } else {
          const bool vqi = qi < n, vqj = qj < n;
          const double b00 = Ap[sidx(pi, pj)];
          const double b01 = vqj ? Ap[sidx(pi, qj)] : 0.0;
          const double b10 = vqi ? Ap[sidx(qi, pj)] : 0.0;
          const double b11 = (vqi && vqj) ? Ap[sidx(qi, qj)] : 0.0;
          const double t00 = ci * b00 - si * b10, t01 = ci * b01 - si * b11;
          const double t10 = si * b00 + ci * b10, t11 = si * b01 + ci * b11;
          Ap[sidx(pi, pj)] = t00 * cj - t01 * sj;
          if (vqj) Ap[sidx(pi, qj)] = t00 * sj + t01 * cj;
          if (vqi) Ap[sidx(qi, pj)] = t10 * cj - t11 * sj;
          if (vqi && vqj) Ap[sidx(qi, qj)] = t10 * sj + t11 * cj;
        }
      };
      for (int m = 0; m < nmine; ++m) update(myblk[m] >> 16, myblk[m] & 0xffff);
      for (int e = extra_start; e < nb; e += bs) {
        int j = int((sqrtf(8.0f * float(e) + 1.0f) - 1.0f) * 0.5f);
        while ((j + 1) * (j + 2) / 2 <= e) ++j;
        while (j * (j + 1) / 2 > e) --j;
        update(e - j * (j + 1) / 2, j);
      }
      for (int e = tid; e < P * n; e += bs) {
        const int k = e / n, r = e - k * n;
        const double s = rs[k];
        if (s == 0.0) continue;
        const double c = rc[k];
        double* vp = Vw + rp[k] * n + r;
        double* vq = Vw + rq[k] * n + r;
        const double x = *vp, y = *vq;
        *vp = c * x - s * y;
        *vq = s * x + c * y;
      }
      __syncthreads();
    }
    if (!rotated) break;
    __syncthreads();
  }
  // eigenvalues, sorted descending (ties: lower index first), and matching vectors
  for (int i = tid; i < n; i += bs) {
    const double wi = Ap[pidx(i, i)];
    int rank = 0;
    for (int j = 0; j < n; ++j) {
      const double wj = Ap[pidx(j, j)];
      rank += (wj > wi) || (wj == wi && j < i);
    }
    d.w[rank] = wi;
    for (int r = 0; r < n; ++r) d.V[r + (int64_t)rank * n] = Vw[r + i * n];
  }
  if (tid == 0 && d.sweeps) *d.sweeps = sweeps;
}

// ---------------------------------------------------------------------------
// Symmetric eigensolver by Householder tridiagonalisation, bisection and inverse
// iteration, one workgroup per matrix (used for the Gram eigenproblems of the scaled
// path, where Jacobi's O(n^3) traffic per sweep is too slow):
//  1. A = Q T Q^T with Householder reflectors H_k = I - beta_k v_k v_k^T acting on rows
//     and columns k+1..n-1 (the trailing block is updated by the symmetric rank-2 form
//     A <- A - v q^T - q v^T, q = p - (beta/2)(v^T p) v, p = beta A v);
//  2. every eigenvalue of T by bisection on the Sturm count (thread t finds the t-th
//     smallest);
//  3. eigenvectors of T by inverse iteration with a partially pivoted tridiagonal LU,
//     three iterations, members of a cluster (gap <= 1e-7 ||T||) orthogonalised against
//     each other by modified Gram-Schmidt; eigenvalues <= vec_cut * max |lambda| get a
//     zero vector (the callers drop them);
//  4. back-transformation V = H_0 H_1 ... H_{n-3} Z.
// Output as the Jacobi kernel: eigenvalues descending, eigenvectors in the columns of V.
// ---------------------------------------------------------------------------
constexpr int kTriThreads = 1024;

__device__ inline double block_sum(double v, double* red, int tid, int bs) {
  v = wave_sum_d(v);
  __syncthreads();
  if ((tid & 63) == 0) red[tid >> 6] = v;
  __syncthreads();
  double t = 0.0;
  for (int w = 0; w < (bs + 63) / 64; ++w) t += red[w];
  return t;
}

__device__ inline int sturm_count(const double* d, const double* e2, int n, double x, double tiny) {
  int cnt = 0;
  double q = d[0] - x;
  if (q == 0.0) q = -tiny;
  cnt += q < 0.0;
  for (int i = 1; i < n; ++i) {
    q = d[i] - x - e2[i - 1] / q;
    if (q == 0.0) q = -tiny;
    cnt += q < 0.0;
  }
  return cnt;
}

// Solve (T - sigma I) x = b in place for one thread; LU with partial pivoting stored in
// the thread's scratch (u, v, w, mult: n doubles each; piv as the sign of mult slot).
__device__ void tri_factor(const double* d, const double* e, int n, double sigma, double tiny,
                           double* u, double* v, double* w, double* mult, unsigned char* piv) {
  double cd = d[0] - sigma, cs1 = n > 1 ? e[0] : 0.0, cs2 = 0.0;
  for (int i = 0; i < n - 1; ++i) {
    const double sub = e[i];
    const double a1 = d[i + 1] - sigma;
    const double s1 = (i + 1 < n - 1) ? e[i + 1] : 0.0;
    if (fabs(cd) >= fabs(sub)) {
      piv[i] = 0;
      const double m = cd != 0.0 ? sub / cd : 0.0;
      mult[i] = m;
      u[i] = cd; v[i] = cs1; w[i] = cs2;
      cd = a1 - m * cs1;
      cs1 = s1 - m * cs2;
      cs2 = 0.0;
    } else {
      piv[i] = 1;
      const double m = cd / sub;
      mult[i] = m;
      u[i] = sub; v[i] = a1; w[i] = s1;
      cd = cs1 - m * a1;
      cs1 = cs2 - m * s1;
      cs2 = 0.0;
    }
    if (u[i] == 0.0) u[i] = tiny;
  }
  u[n - 1] = cd == 0.0 ? tiny : cd;
  v[n - 1] = 0.0;
  w[n - 1] = 0.0;
}

__device__ void tri_solve(int n, const double* u, const double* v, const double* w, const double* mult,
                          const unsigned char* piv, double* x) {
  // forward: apply the row operations to the right-hand side
  double cur = x[0];
  for (int i = 0; i < n - 1; ++i) {
    const double nxt = x[i + 1];
    if (!piv[i]) { x[i] = cur; cur = nxt - mult[i] * cur; }
    else { x[i] = nxt; cur = cur - mult[i] * nxt; }
  }
  x[n - 1] = cur;
  // back substitution
  x[n - 1] = x[n - 1] / u[n - 1];
  if (n >= 2) x[n - 2] = (x[n - 2] - v[n - 2] * x[n - 1]) / u[n - 2];
  for (int i = n - 3; i >= 0; --i) x[i] = (x[i] - v[i] * x[i + 1] - w[i] * x[i + 2]) / u[i];
}

__device__ inline double block_max(double v, double* red, int tid, int bs) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v = fmax(v, __shfl_xor(v, off, 64));
  __syncthreads();
  if ((tid & 63) == 0) red[tid >> 6] = v;
  __syncthreads();
  double t = 0.0;
  for (int w = 0; w < (bs + 63) / 64; ++w) t = fmax(t, red[w]);
  return t;
}

// Off-diagonal entries at most this fraction of the largest diagonal entry: the matrix is
// taken as diagonal (its diagonal has residual <= sqrt(n) * 1e-13 ||A||).
constexpr double kDiagTol = 1e-13;
// A spectrum inside the disc |lambda - mu| <= kShiftTol |mu| (mu the mean diagonal entry,
// radius by Gershgorin) is computed as mu + eig(A - mu I): a Gram matrix of nearly
// orthonormal vectors then becomes an ordinary problem instead of one huge cluster.
constexpr double kShiftTol = 1e-3;
// Off-diagonal entries of T at most this multiple of eps ||T|| split T into blocks.
constexpr double kSplitTol = 4.0 * 2.220446049250313e-16;
// Neighbouring eigenvalues (both above the zero cut) closer than
// min(kClusterTol ||T||, kClusterRel max|lambda|) form a cluster whose inverse-iteration
// vectors are orthogonalised against each other.  Outside clusters a vector is accurate to
// about eps ||T|| / gap: orthogonal to ~1e-9 where |lambda| >= 1e-5 ||T||, and in the graded
// tail only as far as eps ||T|| / (0.01 |lambda|), which weighted by sqrt(|lambda|) (as in
// a Gram factor V Lambda^{1/2}) stays below ~1e-9 ||T||.
constexpr double kClusterTol = 1e-7;
constexpr double kClusterRel = 1e-2;
// Clusters up to this size are handled by one thread, longer ones by the workgroup.
constexpr int kThreadCluster = 16;

__device__ inline bool linked(double a, double b, double cut, double ctol) {
  return fabs(a) > cut && fabs(b) > cut && b - a <= fmin(ctol, kClusterRel * fmax(fabs(a), fabs(b)));
}

__device__ inline void start_vector(double* z, int n, int s, int m, int j) {
  for (int i = 0; i < n; ++i)
    z[i] = (i >= s && i < s + m) ? 1.0 + 0.37 * (double)((i * 7919 + j * 104729) % 101) / 101.0 : 0.0;
}

__global__ __launch_bounds__(kTriThreads) void tridiag_eig_kernel(const EigDesc* __restrict__ descs) {
  __shared__ double red[kTriThreads / 64];
  __shared__ double sh_beta, sh_K;
  __shared__ int sh_nblk, sh_nruns;
  // d, e, e2, lam, beta, vsh, psh: n doubles each; block starts: n + 1 ints
  extern __shared__ double tsm[];
  const EigDesc D = descs[blockIdx.x];
  const int n = D.n;
  if (n <= 0) return;
  const int tid = threadIdx.x, bs = blockDim.x;
  const int lane = tid & 63, wave = tid >> 6, nw = bs >> 6;
  double* dd = tsm;
  double* ee = dd + n;
  double* e2 = ee + n;
  double* lam = e2 + n;
  double* betas = lam + n;
  double* vsh = betas + n;
  double* psh = vsh + n;
  int* bstart = reinterpret_cast<int*>(psh + n);
  const int lda = n;
  double* A = D.work;                         // n x n working copy
  double* scratch = D.work + (int64_t)n * n;  // per-thread inverse-iteration storage
  double* Z = D.V;                            // eigenvectors of T, then of A
  double od = 0.0, dg = 0.0;
  for (int e = tid; e < n * n; e += bs) {
    const int j = e / n, i = e - j * n;
    const double a = (i <= j) ? D.A[i + (int64_t)j * D.lda] : D.A[j + (int64_t)i * D.lda];
    A[e] = a;
    if (i == j) dg = fmax(dg, fabs(a)); else od = fmax(od, fabs(a));
  }
  od = block_max(od, red, tid, bs);
  dg = block_max(dg, red, tid, bs);
  const bool diagonal = od <= kDiagTol * dg;
  if (diagonal) {
    // 0. diagonal to working accuracy: eigenpairs (a_ii, e_i)
    for (int t = tid; t < n; t += bs) {
      lam[t] = A[t + (int64_t)t * lda];
      betas[t] = 0.0;
    }
    for (int e = tid; e < n * n; e += bs) {
      const int j = e / n, i = e - j * n;
      Z[e] = i == j ? 1.0 : 0.0;
    }
    __syncthreads();
  } else {
  double dsum = 0.0;
  for (int t = tid; t < n; t += bs) dsum += A[t + (int64_t)t * lda];
  const double mu = block_sum(dsum, red, tid, bs) / n;
  double rad = 0.0;
  for (int j = tid; j < n; j += bs) {
    double r = fabs(A[j + (int64_t)j * lda] - mu);
    for (int i = 0; i < n; ++i) r += i == j ? 0.0 : fabs(A[i + (int64_t)j * lda]);
    rad = fmax(rad, r);
  }
  rad = block_max(rad, red, tid, bs);
  const double shift = rad <= kShiftTol * fabs(mu) ? mu : 0.0;
  if (shift != 0.0)
    for (int t = tid; t < n; t += bs) A[t + (int64_t)t * lda] -= shift;
  __syncthreads();
  // 1. tridiagonalisation
  for (int k = 0; k + 2 < n; ++k) {
    const int m = n - k - 1;
    double* x = A + (k + 1) + (int64_t)k * lda;  // column k below the diagonal
    double part = 0.0;
    for (int i = tid + 1; i < m; i += bs) part += x[i] * x[i];
    const double sig2 = block_sum(part, red, tid, bs);
    const double x0 = x[0];
    if (tid == 0) {
      dd[k] = A[k + (int64_t)k * lda];
      if (sig2 == 0.0) {
        ee[k] = x0;
        sh_beta = 0.0;
      } else {
        const double nrm = sqrt(x0 * x0 + sig2);
        const double alpha = x0 > 0.0 ? -nrm : nrm;
        const double v0 = x0 - alpha;
        ee[k] = alpha;
        sh_beta = 2.0 / (v0 * v0 + sig2);
        x[0] = v0;  // v stored over the column
      }
      betas[k] = sh_beta;
    }
    __syncthreads();
    const double beta = sh_beta;
    if (beta == 0.0) continue;
    for (int i = tid; i < m; i += bs) vsh[i] = x[i];
    __syncthreads();
    // p = beta A22 v, A22 = A[k+1:, k+1:]; A22 is symmetric, so p_i is the dot product of
    // column i with v: one wavefront per column, lanes along the contiguous column
    const double* A22 = A + (k + 1) + (int64_t)(k + 1) * lda;
    for (int i0 = wave; i0 < m; i0 += 2 * nw) {
      const int i1 = i0 + nw;
      const double* c0 = A22 + (int64_t)i0 * lda;
      const double* c1 = A22 + (int64_t)(i1 < m ? i1 : i0) * lda;
      double a0 = 0.0, a1 = 0.0;
      for (int j = lane; j < m; j += 64) {
        const double vj = vsh[j];
        a0 += c0[j] * vj;
        a1 += c1[j] * vj;
      }
      a0 = wave_sum_d(a0);
      a1 = wave_sum_d(a1);
      if (lane == 0) {
        psh[i0] = beta * a0;
        if (i1 < m) psh[i1] = beta * a1;
      }
    }
    __syncthreads();
    double pv = 0.0;
    for (int i = tid; i < m; i += bs) pv += psh[i] * vsh[i];
    const double vtp = block_sum(pv, red, tid, bs);
    if (tid == 0) sh_K = 0.5 * beta * vtp;
    __syncthreads();
    const double K = sh_K;
    for (int i = tid; i < m; i += bs) psh[i] -= K * vsh[i];  // q
    __syncthreads();
    double* A22w = A + (k + 1) + (int64_t)(k + 1) * lda;
    for (int j = wave; j < m; j += nw) {
      const double vj = vsh[j], qj = psh[j];
      double* col = A22w + (int64_t)j * lda;
      for (int i = lane; i < m; i += 64) col[i] -= vsh[i] * qj + psh[i] * vj;
    }
    __syncthreads();
  }
  if (tid == 0) {
    if (n >= 2) {
      dd[n - 2] = A[(n - 2) + (int64_t)(n - 2) * lda];
      ee[n - 2] = A[(n - 1) + (int64_t)(n - 2) * lda];
      betas[n - 2] = 0.0;
    }
    dd[n - 1] = A[(n - 1) + (int64_t)(n - 1) * lda];
    ee[n - 1] = 0.0;
    betas[n - 1] = 0.0;
  }
  __syncthreads();
  // Gershgorin bound of ||T||; negligible off-diagonals split T into unreduced blocks
  double tn = 0.0;
  for (int i = 0; i < n; ++i)
    tn = fmax(tn, fabs(dd[i]) + (i > 0 ? fabs(ee[i - 1]) : 0.0) + (i < n - 1 ? fabs(ee[i]) : 0.0));
  __syncthreads();
  if (tid == 0) {
    int nb = 0;
    bstart[nb++] = 0;
    for (int i = 0; i + 1 < n; ++i)
      if (fabs(ee[i]) <= kSplitTol * tn) {
        ee[i] = 0.0;
        bstart[nb++] = i + 1;
      }
    bstart[nb] = n;
    sh_nblk = nb;
  }
  __syncthreads();
  const int nblk = sh_nblk;
  for (int i = tid; i < n; i += bs) e2[i] = ee[i] * ee[i];
  __syncthreads();
  const double tiny = fmax(tn * 1e-300, 1e-300) + tn * 2.2e-16 * 1e-3;
  // 2. bisection: position t of block b = [s, s+m) holds the (t-s)-th smallest eigenvalue
  //    of that block, so eigenvalues ascend within each block
  for (int t = tid; t < n; t += bs) {
    int lo_b = 0, hi_b = nblk - 1;
    while (lo_b < hi_b) {
      const int mid = (lo_b + hi_b + 1) >> 1;
      if (bstart[mid] <= t) lo_b = mid; else hi_b = mid - 1;
    }
    const int s = bstart[lo_b], m = bstart[lo_b + 1] - s;
    if (m == 1) { lam[t] = dd[s]; continue; }
    double lo = 1e300, hi = -1e300;
    for (int i = s; i < s + m; ++i) {
      const double r = (i > s ? fabs(ee[i - 1]) : 0.0) + (i < s + m - 1 ? fabs(ee[i]) : 0.0);
      lo = fmin(lo, dd[i] - r);
      hi = fmax(hi, dd[i] + r);
    }
    double a = lo - 1e-14 * tn - 1e-300, b = hi + 1e-14 * tn + 1e-300;
    for (int it = 0; it < 100; ++it) {
      const double mid = 0.5 * (a + b);
      if (mid <= a || mid >= b) break;
      if (b - a <= 2.2e-16 * fmax(fabs(a), fabs(b)) * 2.0 || b - a <= 1e-18 * tn) break;
      if (sturm_count(dd + s, e2 + s, m, mid, tiny + 1e-300) > t - s) b = mid; else a = mid;
    }
    lam[t] = 0.5 * (a + b);
  }
  __syncthreads();
  // 3. inverse iteration within each block; vectors vanish outside their block
  double lmax = 0.0;
  for (int i = 0; i < n; ++i) lmax = fmax(lmax, fabs(lam[i]));
  // with a shift every |eigenvalue| of A is at least (1 - kShiftTol) |mu|: nothing is cut
  const double cut = shift != 0.0 ? 0.0 : D.abs_tol * lmax;
  const double ctol = kClusterTol * fmax(tn, 1e-300);
  for (int t = tid; t < n; t += bs) {
    int lo_b = 0, hi_b = nblk - 1;
    while (lo_b < hi_b) {
      const int mid = (lo_b + hi_b + 1) >> 1;
      if (bstart[mid] <= t) lo_b = mid; else hi_b = mid - 1;
    }
    const int s = bstart[lo_b], m = bstart[lo_b + 1] - s;
    if (t > s && linked(lam[t - 1], lam[t], cut, ctol)) continue;  // not the first of its cluster
    int last = t;
    while (last + 1 < s + m && linked(lam[last], lam[last + 1], cut, ctol)) ++last;
    if (last + 1 - t > kThreadCluster) continue;  // long cluster: workgroup pass below
    double* u = scratch + (int64_t)t * 5 * n;
    double* v = u + n;
    double* w = v + n;
    double* mult = w + n;
    unsigned char* piv = reinterpret_cast<unsigned char*>(mult + n);
    for (int j = t; j <= last; ++j) {
      double* z = Z + (int64_t)j * n;
      if (fabs(lam[j]) <= cut) {
        for (int i = 0; i < n; ++i) z[i] = 0.0;
        continue;
      }
      if (m == 1) {
        for (int i = 0; i < n; ++i) z[i] = i == s ? 1.0 : 0.0;
        continue;
      }
      const double sigma = lam[j] + (j - t) * 10.0 * 2.2e-16 * tn;
      tri_factor(dd + s, ee + s, m, sigma, fmax(tn * 1e-15, 1e-300), u, v, w, mult, piv);
      start_vector(z, n, s, m, j);
      for (int it = 0; it < 3; ++it) {
        tri_solve(m, u, v, w, mult, piv, z + s);
        for (int jj = t; jj < j; ++jj) {
          const double* y = Z + (int64_t)jj * n;
          double dot = 0.0;
          for (int i = s; i < s + m; ++i) dot += y[i] * z[i];
          for (int i = s; i < s + m; ++i) z[i] -= dot * y[i];
        }
        double nn = 0.0;
        for (int i = s; i < s + m; ++i) nn += z[i] * z[i];
        nn = nn > 0.0 ? 1.0 / sqrt(nn) : 0.0;
        for (int i = s; i < s + m; ++i) z[i] *= nn;
      }
    }
  }
  __syncthreads();
  // long clusters: (first, last, block) listed in e2 (free after bisection), members
  // flagged in vsh (free until the back-transformation)
  for (int i = tid; i < n; i += bs) vsh[i] = 0.0;
  __syncthreads();
  if (tid == 0) {
    int nr = 0;
    for (int b = 0; b < nblk; ++b) {
      const int s = bstart[b], e = bstart[b + 1];
      int t = s;
      while (t < e) {
        int last = t;
        while (last + 1 < e && linked(lam[last], lam[last + 1], cut, ctol)) ++last;
        if (last + 1 - t > kThreadCluster) {
          e2[3 * nr] = t; e2[3 * nr + 1] = last; e2[3 * nr + 2] = b;
          for (int q = t; q <= last; ++q) vsh[q] = 1.0;
          ++nr;
        }
        t = last + 1;
      }
    }
    sh_nruns = nr;
  }
  __syncthreads();
  const int nruns = sh_nruns;
  // simultaneous inverse iteration: every member solves with its own shift in parallel,
  // then each cluster is orthonormalised by the workgroup (classical Gram-Schmidt, twice)
  for (int it = 0; it < 3 && nruns > 0; ++it) {
    for (int p = tid; p < n; p += bs) {
      if (vsh[p] == 0.0) continue;
      int lo_b = 0, hi_b = nblk - 1;
      while (lo_b < hi_b) {
        const int mid = (lo_b + hi_b + 1) >> 1;
        if (bstart[mid] <= p) lo_b = mid; else hi_b = mid - 1;
      }
      const int s = bstart[lo_b], m = bstart[lo_b + 1] - s;
      double* u = scratch + (int64_t)p * 5 * n;
      double* v = u + n;
      double* w = v + n;
      double* mult = w + n;
      unsigned char* piv = reinterpret_cast<unsigned char*>(mult + n);
      double* z = Z + (int64_t)p * n;
      if (it == 0) {
        tri_factor(dd + s, ee + s, m, lam[p] + (p - s) * 10.0 * 2.2e-16 * tn, fmax(tn * 1e-15, 1e-300), u, v, w, mult,
                   piv);
        start_vector(z, n, s, m, p);
      }
      tri_solve(m, u, v, w, mult, piv, z + s);
      double nn = 0.0;
      for (int i = s; i < s + m; ++i) nn += z[i] * z[i];
      nn = nn > 0.0 ? 1.0 / sqrt(nn) : 0.0;
      for (int i = s; i < s + m; ++i) z[i] *= nn;
    }
    __syncthreads();
    for (int q = 0; q < nruns; ++q) {
      const int r0 = int(e2[3 * q]), r1 = int(e2[3 * q + 1]), b = int(e2[3 * q + 2]);
      const int s = bstart[b], m = bstart[b + 1] - s;
      for (int j = r0; j <= r1; ++j) {
        double* z = Z + (int64_t)j * n;
        for (int pass = 0; pass < 2 && j > r0; ++pass) {
          for (int jj = r0 + wave; jj < j; jj += nw) {
            const double* y = Z + (int64_t)jj * n;
            double dot = 0.0;
            for (int i = s + lane; i < s + m; i += 64) dot += y[i] * z[i];
            dot = wave_sum_d(dot);
            if (lane == 0) psh[jj - r0] = dot;
          }
          __syncthreads();
          for (int i = s + tid; i < s + m; i += bs) {
            double acc = 0.0;
            for (int jj = r0; jj < j; ++jj) acc += psh[jj - r0] * Z[i + (int64_t)jj * n];
            z[i] -= acc;
          }
          __syncthreads();
        }
        double part = 0.0;
        for (int i = s + tid; i < s + m; i += bs) part += z[i] * z[i];
        const double nn2 = block_sum(part, red, tid, bs);
        const double sc = nn2 > 0.0 ? 1.0 / sqrt(nn2) : 0.0;
        for (int i = s + tid; i < s + m; i += bs) z[i] *= sc;
        __syncthreads();
      }
    }
  }
  __syncthreads();
  // 4. back-transformation: apply H_{n-3} ... H_0 to the columns of Z
  for (int k = n - 3; k >= 0; --k) {
    const double beta = betas[k];
    if (beta == 0.0) continue;
    const int m = n - k - 1;
    const double* vk = A + (k + 1) + (int64_t)k * lda;
    for (int i = tid; i < m; i += bs) vsh[i] = vk[i];
    __syncthreads();
    for (int c = wave; c < n; c += nw) {
      double* zc = Z + (int64_t)c * n + (k + 1);
      double dot = 0.0;
      for (int i = lane; i < m; i += 64) dot += vsh[i] * zc[i];
      dot = beta * wave_sum_d(dot);
      if (dot != 0.0)
        for (int i = lane; i < m; i += 64) zc[i] -= dot * vsh[i];
    }
    __syncthreads();
  }
  for (int t = tid; t < n; t += bs) lam[t] += shift;
  __syncthreads();
  }  // !diagonal
  // eigenvalues at or below the cut carry zero vectors
  double lmx = 0.0;
  for (int i = 0; i < n; ++i) lmx = fmax(lmx, fabs(lam[i]));
  const double vcut = D.abs_tol * lmx;
  // 5. descending order (ties: lower position first); Z goes through the working copy
  for (int e = tid; e < n * n; e += bs) {
    const int c = e / n;
    A[e] = fabs(lam[c]) <= vcut ? 0.0 : Z[e];
  }
  for (int t = tid; t < n; t += bs) {
    int rank = 0;
    const double lt = lam[t];
    for (int u = 0; u < n; ++u) rank += (lam[u] > lt) || (lam[u] == lt && u < t);
    e2[t] = rank;
  }
  __syncthreads();
  for (int t = tid; t < n; t += bs) D.w[int(e2[t])] = lam[t];
  for (int e = tid; e < n * n; e += bs) {
    const int c = e / n, i = e - c * n;
    Z[i + (int64_t)int(e2[c]) * n] = A[e];
  }
  if (tid == 0 && D.sweeps) *D.sweeps = diagonal ? 0 : -1;
}

void launch_eig_tridiag(const EigDesc* d, int nprob, int nmax, hipStream_t s) {
  if (nprob <= 0) return;
  if (nmax > kEigMax) throw std::runtime_error("eig: matrix larger than supported");
  const size_t shm = size_t(nmax) * 7 * sizeof(double) + size_t(nmax + 1) * sizeof(int);
  const int threads = nmax <= 64 ? 256 : kTriThreads;
  hipLaunchKernelGGL(tridiag_eig_kernel, dim3(nprob), dim3(threads), shm, s, d);
  PV_LAUNCH_CHECK();
}

static size_t g_lds_limit = size_t(-1);

// Largest dynamic LDS accepted for the LDS-resident variants (0 when the opt-in fails).
static size_t eig_lds_limit() {
  if (g_lds_limit == size_t(-1)) {
    int dev = 0, v = 0;
    (void)hipGetDevice(&dev);
    if (hipDeviceGetAttribute(&v, hipDeviceAttributeMaxSharedMemoryPerBlock, dev) != hipSuccess) v = 0;
    (void)hipGetLastError();
    size_t want = v > 1024 ? size_t(v) - 1024 : 0;  // room for the static flag
    const void* fns[3] = {(const void*)jacobi_eig_kernel<0>, (const void*)jacobi_eig_kernel<1>,
                          (const void*)jacobi_eig_kernel<2>};
    for (const void* f : fns)
      if (want > 0 && hipFuncSetAttribute(f, hipFuncAttributeMaxDynamicSharedMemorySize, int(want)) != hipSuccess) {
        (void)hipGetLastError();
        want = 0;
      }
    g_lds_limit = want;
  }
  return g_lds_limit;
}

int eig_mode(int n) {
  const size_t lim = eig_lds_limit();
  if (eig_lds_bytes(n, 2) <= lim) return 2;
  if (eig_lds_bytes(n, 1) <= lim) return 1;
  return 0;
}

void launch_eig(const EigDesc* d, int nprob, int nmax, int mode, hipStream_t s) {
  if (nprob <= 0) return;
  if (nmax > kEigMax) throw std::runtime_error("eig: matrix larger than supported");
  const size_t shm = eig_lds_bytes(nmax, mode);
  if (shm > eig_lds_limit()) throw std::runtime_error("eig: LDS request above the device limit");
  const int threads = nmax <= 48 ? 256 : (nmax <= 96 ? 512 : 1024);
  if (mode == 2)
    hipLaunchKernelGGL(jacobi_eig_kernel<2>, dim3(nprob), dim3(threads), shm, s, d, 60);
  else if (mode == 1)
    hipLaunchKernelGGL(jacobi_eig_kernel<1>, dim3(nprob), dim3(threads), shm, s, d, 60);
  else
    hipLaunchKernelGGL(jacobi_eig_kernel<0>, dim3(nprob), dim3(threads), shm, s, d, 60);
  PV_LAUNCH_CHECK();
}

// ---------------------------------------------------------------------------
// W-step: one workgroup per (output block, output state b').
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void wstep_kernel(const WItem* __restrict__ items,
                                                    const WBlock* __restrict__ blocks,
                                                    const WSrc* __restrict__ srcs,
                                                    const int32_t* __restrict__ row_ptr,
                                                    const int32_t* __restrict__ b_in,
                                                    const uint8_t* __restrict__ s_in,
                                                    const int8_t* __restrict__ q_in,
                                                    const int32_t* __restrict__ qoff_in,
                                                    const double* __restrict__ val, int w_out) {
  const WItem it = items[blockIdx.x];
  const WBlock B = blocks[it.block];
  const WSrc& S = srcs[B.src];
  const int row = B.s_out * w_out + it.bprime;
  const int e0 = row_ptr[row], e1 = row_ptr[row + 1];
  const int bl = it.bprime - B.qoff_out;
  const int64_t n = (int64_t)B.rows * B.cols;
  const int64_t ldo = (int64_t)B.rows * B.wq_out;
  for (int64_t x = threadIdx.x; x < n; x += blockDim.x) {
    const int a = int(x % B.rows);
    const int64_t c = x / B.rows;
    double acc = 0.0;
    for (int e = e0; e < e1; ++e) {
      const int b = b_in[e];
      const int q = q_in[b] + 2;
      const int si = s_in[e];
      const double* base = S.base[si][q];
      if (base == nullptr) continue;
      acc += val[e] * base[a + (int64_t)B.rows * (b - qoff_in[q]) + S.ld[si][q] * c];
    }
    B.out[a + (int64_t)B.rows * bl + ldo * c] = acc;
  }
}

void launch_wstep(const WItem* items, int nitems, const WBlock* blocks, const WSrc* srcs,
                  const int32_t* row_ptr, const int32_t* b_in, const uint8_t* s_in,
                  const int8_t* q_in, const int32_t* qoff_in, const double* val, int w_out,
                  hipStream_t s) {
  if (nitems <= 0) return;
  hipLaunchKernelGGL(wstep_kernel, dim3(nitems), dim3(256), 0, s, items, blocks, srcs, row_ptr,
                     b_in, s_in, q_in, qoff_in, val, w_out);
  PV_LAUNCH_CHECK();
}

// ---------------------------------------------------------------------------
// Batched block copy with scale, and column scaling.
// ---------------------------------------------------------------------------
__global__ void copy_kernel(const CopyDesc* __restrict__ d, int nd, int64_t total) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= total) return;
  int lo = 0, hi = nd - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (d[mid].elem0 <= e) lo = mid; else hi = mid - 1;
  }
  const CopyDesc c = d[lo];
  const int64_t x = e - c.elem0;
  const int i = int(x % c.rows), j = int(x / c.rows);
  c.dst[i + (int64_t)j * c.ldd] = c.alpha * c.src[i + (int64_t)j * c.lds];
}

void launch_copy(const CopyDesc* d, int nd, int64_t total, hipStream_t s) {
  if (total <= 0) return;
  hipLaunchKernelGGL(copy_kernel, dim3((total + 255) / 256), dim3(256), 0, s, d, nd, total);
  PV_LAUNCH_CHECK();
}

__global__ void scale_kernel(const ScaleDesc* __restrict__ d, int nd, int64_t total) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= total) return;
  int lo = 0, hi = nd - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (d[mid].elem0 <= e) lo = mid; else hi = mid - 1;
  }
  const ScaleDesc c = d[lo];
  const int64_t x = e - c.elem0;
  const int i = int(x % c.rows), j = int(x / c.rows);
  double f = c.s[j];
  if (c.sqrt_s) f = sqrt(fmax(f, 0.0));
  if (c.invert) f = f != 0.0 ? 1.0 / f : 0.0;
  c.dst[i + (int64_t)j * c.ldd] = f * c.src[i + (int64_t)j * c.lds];
}

void launch_scale(const ScaleDesc* d, int nd, int64_t total, hipStream_t s) {
  if (total <= 0) return;
  hipLaunchKernelGGL(scale_kernel, dim3((total + 255) / 256), dim3(256), 0, s, d, nd, total);
  PV_LAUNCH_CHECK();
}

// ---------------------------------------------------------------------------
// Sum of squares with wavefront shuffles: per-lane partial sums, a 64-lane
// butterfly (__shfl_xor), one value per wave through LDS, and a fixed-order final sum
// by a single workgroup, so the result is bitwise reproducible.
// ---------------------------------------------------------------------------
__device__ inline double wave_sum(double v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
  return v;
}

__global__ __launch_bounds__(1024) void sumsq_kernel(const double* __restrict__ x, int64_t n, double* out) {
  __shared__ double part[16];
  double acc = 0.0;
  for (int64_t i = threadIdx.x; i < n; i += blockDim.x) acc += x[i] * x[i];
  acc = wave_sum(acc);
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  if (lane == 0) part[wave] = acc;
  __syncthreads();
  if (threadIdx.x == 0) {
    double t = 0.0;
    for (int w = 0; w < int(blockDim.x >> 6); ++w) t += part[w];
    *out = t;
  }
}

void launch_sumsq(const double* x, int64_t n, double* out, hipStream_t s) {
  hipLaunchKernelGGL(sumsq_kernel, dim3(1), dim3(1024), 0, s, x, n, out);
  PV_LAUNCH_CHECK();
}

__global__ void fill_kernel(double* x, int64_t n, double v) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e < n) x[e] = v;
}

void launch_fill(double* x, int64_t n, double v, hipStream_t s) {
  if (n <= 0) return;
  hipLaunchKernelGGL(fill_kernel, dim3((n + 255) / 256), dim3(256), 0, s, x, n, v);
  PV_LAUNCH_CHECK();
}

}  // namespace pv
