// Kernels of the learned preconditioner correction; see learned.hpp.  All of them are
// elementwise or per-sample loops over small arrays (a few thousand rows): one thread per
// element, 256-thread workgroups.  The matrix products of the network run through the
// block GEMM of kernels.hip.
#include "learned.hpp"

namespace pv {

namespace {

constexpr int kThreads = 256;

inline unsigned blocks(int64_t n) { return unsigned((n + kThreads - 1) / kThreads); }

// round to the nearest bfloat16 (ties to even), returned as float
__device__ inline float bf16_round(float x) {
  unsigned u = __float_as_uint(x);
  u = (u + 0x7FFFu + ((u >> 16) & 1u)) & 0xFFFF0000u;
  return __uint_as_float(u);
}

__global__ void features_kernel(const double* th, const double* hd, const double* dens, int L, int N, double tbar,
                                double lam, double* X) {
  const int r = blockIdx.x * blockDim.x + threadIdx.x;
  if (r >= L * (N + 1)) return;
  const int i = r / (N + 1), n = r % (N + 1);
  double* x = X + (int64_t)r * kMlpFeat;
  x[0] = th[i] / tbar;
  x[1] = hd[i] / tbar;
  x[2] = double(n) / N;
  x[3] = double(i) / L;
  x[4] = dens[i];
  x[5] = lam / (N * tbar);
}

__global__ void bias_tanh_kernel(double* A, const double* b, int rows, int cols, int ld) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= (int64_t)rows * cols) return;
  const int u = int(e % rows), c = int(e / rows);
  double* a = A + u + (int64_t)c * ld;
  *a = tanh(*a + b[u]);
}

__global__ void output_kernel(const double* z, const double* b3, int R, double dmax, double* tz, double* delta) {
  const int r = blockIdx.x * blockDim.x + threadIdx.x;
  if (r >= R) return;
  const double t = tanh(z[r] + b3[0]);
  tz[r] = t;
  delta[r] = dmax * t;
}

__global__ void target_kernel(const uint64_t* masks, int B, const double* hd, const double* jk, double gamma, int L,
                              double* target) {
  const int b = blockIdx.x * blockDim.x + threadIdx.x;
  if (b >= B) return;
  const uint64_t m = masks[b];
  double e = gamma;
  for (int i = 0; i < L; ++i) {
    if (!((m >> i) & 1u)) continue;
    e += hd[i];
    for (int j = 0; j < L; ++j)
      if (j != i && ((m >> j) & 1u)) e += jk[i + (int64_t)j * L];
  }
  target[b] = e;
}

// one thread per sample; the workgroup accumulates its samples' contributions to G and
// to the loss in LDS (R + 1 doubles of dynamic shared memory), then adds them to global
// memory once per entry
__global__ void misfit_kernel(const uint64_t* masks, int B, const double* th, const double* delta,
                              const double* target, int L, int N, double scale, double lscale, double* G,
                              double* loss) {
  extern __shared__ double acc[];
  const int R = L * (N + 1);
  for (int r = threadIdx.x; r <= R; r += blockDim.x) acc[r] = 0.0;
  __syncthreads();
  const int b = blockIdx.x * blockDim.x + threadIdx.x;
  if (b < B) {
    const uint64_t m = masks[b];
    double d = 0.0;
    int n = 0;
    for (int i = 0; i < L && n <= N; ++i) {
      if (!((m >> i) & 1u)) continue;
      if (n < N) d += th[i] + delta[i * (N + 1) + n];
      ++n;
    }
    if (n == N) {  // an N-particle determinant (others do not contribute)
      const double e = d - target[b];
      n = 0;
      for (int i = 0; i < L; ++i) {
        if (!((m >> i) & 1u)) continue;
        atomicAdd(acc + i * (N + 1) + n, scale * e);
        ++n;
      }
      atomicAdd(acc + R, lscale * e * e);
    }
  }
  __syncthreads();
  for (int r = threadIdx.x; r < R; r += blockDim.x)
    if (acc[r] != 0.0) atomicAdd(G + r, acc[r]);
  if (threadIdx.x == 0) atomicAdd(loss, acc[R]);
}

// Solve form of the misfit: per sampled determinant b the corrected diagonal d_b, the
// preconditioned residual r_b / d_b against the exact solve t_b; loss += lscale e^2 with
// e = r_b/d_b - t_b, and d loss / d d_b = -gscale e r_b / d_b^2 scattered onto the
// correction entries of the occupied sites (LDS sums, one global add per entry).
__global__ void solve_misfit_kernel(const uint64_t* masks, int B, const double* th, const double* delta,
                                    const double* rv, const double* tv, int L, int N, double gscale,
                                    double lscale, double* G, double* loss) {
  extern __shared__ double acc[];
  const int R = L * (N + 1);
  for (int r = threadIdx.x; r <= R; r += blockDim.x) acc[r] = 0.0;
  __syncthreads();
  const int b = blockIdx.x * blockDim.x + threadIdx.x;
  if (b < B) {
    const uint64_t m = masks[b];
    double d = 0.0;
    int n = 0;
    for (int i = 0; i < L && n <= N; ++i) {
      if (!((m >> i) & 1u)) continue;
      if (n < N) d += th[i] + delta[i * (N + 1) + n];
      ++n;
    }
    if (n == N) {
      const double r = rv[b];
      const double e = r / d - tv[b];
      const double gd = -gscale * e * r / (d * d);
      n = 0;
      for (int i = 0; i < L; ++i) {
        if (!((m >> i) & 1u)) continue;
        atomicAdd(acc + i * (N + 1) + n, gd);
        ++n;
      }
      atomicAdd(acc + R, lscale * e * e);
    }
  }
  __syncthreads();
  for (int r = threadIdx.x; r < R; r += blockDim.x)
    if (acc[r] != 0.0) atomicAdd(G + r, acc[r]);
  if (threadIdx.x == 0) atomicAdd(loss, acc[R]);
}

__global__ void dz_kernel(const double* G, const double* tz, int R, double dmax, double* dz) {
  const int r = blockIdx.x * blockDim.x + threadIdx.x;
  if (r >= R) return;
  dz[r] = G[r] * dmax * (1.0 - tz[r] * tz[r]);
}

__global__ void tanh_grad_kernel(double* dA, const double* H, int64_t n) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= n) return;
  dA[e] *= 1.0 - H[e] * H[e];
}

// 64 rows per workgroup: lane l takes row 64 blockIdx.x + l, the four wavefronts take
// every fourth column, eight independent partial sums per thread; LDS sums the wavefronts
__global__ void rowsum_kernel(const double* A, int rows, int cols, int ld, double* out) {
  __shared__ double part[4][64];
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int u = blockIdx.x * 64 + lane;
  double s[8] = {0, 0, 0, 0, 0, 0, 0, 0};
  if (u < rows) {
    int c = w;
    for (; c + 28 < cols; c += 32) {
#pragma unroll
      for (int k = 0; k < 8; ++k) s[k] += A[u + (int64_t)(c + 4 * k) * ld];
    }
    for (; c < cols; c += 4) s[0] += A[u + (int64_t)c * ld];
  }
  part[w][lane] = ((s[0] + s[1]) + (s[2] + s[3])) + ((s[4] + s[5]) + (s[6] + s[7]));
  __syncthreads();
  if (w == 0 && u < rows) out[u] = (part[0][lane] + part[1][lane]) + (part[2][lane] + part[3][lane]);
}

__global__ void adam_kernel(float* w, float* m, float* v, const double* g, int64_t P, float lr, float b1, float b2,
                            float eps, float c1, float c2, double* wq) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= P) return;
  const float gi = float(g[e]);
  const float mi = b1 * m[e] + (1.0f - b1) * gi;
  const float vi = b2 * v[e] + (1.0f - b2) * gi * gi;
  m[e] = mi;
  v[e] = vi;
  const float wi = w[e] - lr * (mi / c1) / (sqrtf(vi / c2) + eps);
  w[e] = wi;
  wq[e] = double(bf16_round(wi));
}

__global__ void round_kernel(const float* w, int64_t P, double* wq) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= P) return;
  wq[e] = double(bf16_round(w[e]));
}

}  // namespace

void launch_mlp_features(const double* th, const double* hd, const double* dens, int L, int N, double tbar,
                         double lam, double* X, hipStream_t s) {
  const int R = L * (N + 1);
  if (R > 0) hipLaunchKernelGGL(features_kernel, dim3(blocks(R)), dim3(kThreads), 0, s, th, hd, dens, L, N, tbar, lam, X);
}

void launch_mlp_bias_tanh(double* A, const double* b, int rows, int cols, int ld, hipStream_t s) {
  const int64_t n = (int64_t)rows * cols;
  if (n > 0) hipLaunchKernelGGL(bias_tanh_kernel, dim3(blocks(n)), dim3(kThreads), 0, s, A, b, rows, cols, ld);
}

void launch_mlp_output(const double* z, const double* b3, int R, double dmax, double* tz, double* delta,
                       hipStream_t s) {
  if (R > 0) hipLaunchKernelGGL(output_kernel, dim3(blocks(R)), dim3(kThreads), 0, s, z, b3, R, dmax, tz, delta);
}

void launch_mlp_target(const uint64_t* masks, int B, const double* hd, const double* jk, double gamma, int L,
                       double* target, hipStream_t s) {
  if (B > 0) hipLaunchKernelGGL(target_kernel, dim3(blocks(B)), dim3(kThreads), 0, s, masks, B, hd, jk, gamma, L, target);
}

void launch_mlp_misfit(const uint64_t* masks, int B, const double* th, const double* delta, const double* target,
                       int L, int N, double scale, double lscale, double* G, double* loss, hipStream_t s) {
  const size_t shm = (size_t(L) * (N + 1) + 1) * sizeof(double);  // at most 64 x 65 + 1 doubles
  if (B > 0)
    hipLaunchKernelGGL(misfit_kernel, dim3(blocks(B)), dim3(kThreads), shm, s, masks, B, th, delta, target, L, N,
                       scale, lscale, G, loss);
}

void launch_mlp_solve_misfit(const uint64_t* masks, int B, const double* th, const double* delta, const double* rv,
                             const double* tv, int L, int N, double gscale, double lscale, double* G, double* loss,
                             hipStream_t s) {
  const size_t shm = (size_t(L) * (N + 1) + 1) * sizeof(double);
  if (B > 0)
    hipLaunchKernelGGL(solve_misfit_kernel, dim3(blocks(B)), dim3(kThreads), shm, s, masks, B, th, delta, rv, tv, L,
                       N, gscale, lscale, G, loss);
}

void launch_mlp_dz(const double* G, const double* tz, int R, double dmax, double* dz, hipStream_t s) {
  if (R > 0) hipLaunchKernelGGL(dz_kernel, dim3(blocks(R)), dim3(kThreads), 0, s, G, tz, R, dmax, dz);
}

void launch_mlp_tanh_grad(double* dA, const double* H, int64_t n, hipStream_t s) {
  if (n > 0) hipLaunchKernelGGL(tanh_grad_kernel, dim3(blocks(n)), dim3(kThreads), 0, s, dA, H, n);
}

void launch_mlp_rowsum(const double* A, int rows, int cols, int ld, double* out, hipStream_t s) {
  if (rows > 0) hipLaunchKernelGGL(rowsum_kernel, dim3((rows + 63) / 64), dim3(256), 0, s, A, rows, cols, ld, out);
}

void launch_mlp_adam(float* w, float* m, float* v, const double* g, int64_t P, float lr, float b1, float b2,
                     float eps, float c1, float c2, double* wq, hipStream_t s) {
  if (P > 0)
    hipLaunchKernelGGL(adam_kernel, dim3(blocks(P)), dim3(kThreads), 0, s, w, m, v, g, P, lr, b1, b2, eps, c1, c2, wq);
}

void launch_mlp_round(const float* w, int64_t P, double* wq, hipStream_t s) {
  if (P > 0) hipLaunchKernelGGL(round_kernel, dim3(blocks(P)), dim3(kThreads), 0, s, w, P, wq);
}

}  // namespace pv
