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
// matrix is the packed upper triangle (in LDS when it fits); V is accumulated in
// global memory.  A rotation is skipped when |a_pq| <= eps sqrt(|a_pp a_qq|).
// ---------------------------------------------------------------------------
constexpr int kEigThreads = 512;
constexpr int kEigMaxPairs = kEigMax / 2;

__device__ inline int64_t pidx(int r, int c) {  // packed upper, r <= c
  return (int64_t)c * (c + 1) / 2 + r;
}
__device__ inline int64_t sidx(int r, int c) { return r <= c ? pidx(r, c) : pidx(c, r); }

template <bool LDS>
__global__ __launch_bounds__(kEigThreads) void jacobi_eig_kernel(const EigDesc* __restrict__ descs, int maxsweep) {
  extern __shared__ double smem[];
  __shared__ double rc[kEigMaxPairs], rs[kEigMaxPairs];
  __shared__ int rp[kEigMaxPairs], rq[kEigMaxPairs];
  __shared__ int rotated;
  const EigDesc d = descs[blockIdx.x];
  const int n = d.n;
  if (n <= 0) return;
  const int tid = threadIdx.x, bs = blockDim.x;
  const int n2 = n + (n & 1), P = n2 / 2;
  double* Ap = LDS ? smem : (d.work + (int64_t)n * n);
  double* Vw = d.work;
  for (int c = 0; c < n; ++c)
    for (int r = tid; r <= c; r += bs) Ap[pidx(r, c)] = d.A[r + (int64_t)c * d.lda];
  for (int64_t e = tid; e < (int64_t)n * n; e += bs) Vw[e] = (e % n == e / n) ? 1.0 : 0.0;
  __syncthreads();
  const double eps = 2.0 * DBL_EPSILON;
  for (int sweep = 0; sweep < maxsweep; ++sweep) {
    if (tid == 0) rotated = 0;
    __syncthreads();
    for (int step = 0; step < n2 - 1; ++step) {
      for (int k = tid; k < P; k += bs) {
        int a, b;
        if (k == 0) { a = n2 - 1; b = step; }
        else { a = (step + k) % (n2 - 1); b = (step - k + n2 - 1) % (n2 - 1); }
        const int p = min(a, b), q = max(a, b);
        double c = 1.0, s = 0.0;
        if (q < n) {
          const double app = Ap[pidx(p, p)], aqq = Ap[pidx(q, q)], apq = Ap[pidx(p, q)];
          if (fabs(apq) > eps * sqrt(fabs(app * aqq)) && fabs(apq) > 1e-300) {
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
      const int nb = P * (P + 1) / 2;
      for (int e = tid; e < nb; e += bs) {
        int j = int((sqrt(8.0 * e + 1.0) - 1.0) * 0.5);
        while ((j + 1) * (j + 2) / 2 <= e) ++j;
        while (j * (j + 1) / 2 > e) --j;
        const int i = e - j * (j + 1) / 2;
        const double si = rs[i], sj = rs[j];
        if (si == 0.0 && sj == 0.0) continue;
        const double ci = rc[i], cj = rc[j];
        const int pi = rp[i], qi = rq[i], pj = rp[j], qj = rq[j];
        if (i == j) {
          if (qi >= n) continue;
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
      }
      for (int64_t e = tid; e < (int64_t)P * n; e += bs) {
        const int k = int(e / n), r = int(e % n);
        const double s = rs[k];
        if (s == 0.0) continue;
        const double c = rc[k];
        double* vp = Vw + (int64_t)rp[k] * n + r;
        double* vq = Vw + (int64_t)rq[k] * n + r;
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
    for (int r = 0; r < n; ++r) d.V[r + (int64_t)rank * n] = Vw[r + (int64_t)i * n];
  }
}

// Largest dynamic LDS request accepted for the LDS variant (0 when the opt-in fails).
static size_t eig_lds_limit() {
  static size_t limit = size_t(-1);
  if (limit == size_t(-1)) {
    int dev = 0, v = 0;
    (void)hipGetDevice(&dev);
    if (hipDeviceGetAttribute(&v, hipDeviceAttributeMaxSharedMemoryPerBlock, dev) != hipSuccess) v = 0;
    (void)hipGetLastError();
    // static LDS of the kernel: rotation tables and the flag
    const size_t stat = kEigMaxPairs * (2 * sizeof(double) + 2 * sizeof(int)) + 64;
    size_t want = v > int(stat) ? size_t(v) - stat : 0;
    if (want > 0 && hipFuncSetAttribute((const void*)jacobi_eig_kernel<true>,
                                        hipFuncAttributeMaxDynamicSharedMemorySize, int(want)) != hipSuccess) {
      (void)hipGetLastError();
      want = 0;
    }
    limit = want;
  }
  return limit;
}

bool eig_fits_lds(int n) {
  return n <= kEigLdsMax && size_t(n) * (n + 1) / 2 * sizeof(double) <= eig_lds_limit();
}

void launch_eig(const EigDesc* d, int nprob, int nmax, bool lds, hipStream_t s) {
  if (nprob <= 0) return;
  if (nmax > kEigMax) throw std::runtime_error("eig: matrix larger than supported");
  if (lds) {
    const size_t shm = size_t(nmax) * (nmax + 1) / 2 * sizeof(double);
    if (shm > eig_lds_limit()) throw std::runtime_error("eig: LDS request above the device limit");
    hipLaunchKernelGGL(jacobi_eig_kernel<true>, dim3(nprob), dim3(kEigThreads), shm, s, d, 60);
  } else {
    hipLaunchKernelGGL(jacobi_eig_kernel<false>, dim3(nprob), dim3(kEigThreads), 0, s, d, 60);
  }
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
