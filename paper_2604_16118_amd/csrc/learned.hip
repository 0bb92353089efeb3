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

__global__ void misfit_kernel(const uint64_t* masks, int B, const double* th, const double* delta,
                              const double* target, int L, int N, double scale, double lscale, double* G,
                              double* loss) {
  const int b = blockIdx.x * blockDim.x + threadIdx.x;
  if (b >= B) return;
  const uint64_t m = masks[b];
  double d = 0.0;
  int n = 0;
  for (int i = 0; i < L && n <= N; ++i) {
    if (!((m >> i) & 1u)) continue;
    if (n < N) d += th[i] + delta[i * (N + 1) + n];
    ++n;
  }
  if (n != N) return;  // not an N-particle determinant: no contribution
  const double e = d - target[b];
  n = 0;
  for (int i = 0; i < L; ++i) {
    if (!((m >> i) & 1u)) continue;
    atomicAdd(G + i * (N + 1) + n, scale * e);
    ++n;
  }
  atomicAdd(loss, lscale * e * e);
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

__global__ void rowsum_kernel(const double* A, int rows, int cols, int ld, double* out) {
  const int u = blockIdx.x * blockDim.x + threadIdx.x;
  if (u >= rows) return;
  double s = 0.0;
  for (int c = 0; c < cols; ++c) s += A[u + (int64_t)c * ld];
  out[u] = s;
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
  if (B > 0)
    hipLaunchKernelGGL(misfit_kernel, dim3(blocks(B)), dim3(kThreads), 0, s, masks, B, th, delta, target, L, N, scale,
                       lscale, G, loss);
}

void launch_mlp_dz(const double* G, const double* tz, int R, double dmax, double* dz, hipStream_t s) {
  if (R > 0) hipLaunchKernelGGL(dz_kernel, dim3(blocks(R)), dim3(kThreads), 0, s, G, tz, R, dmax, dz);
}

void launch_mlp_tanh_grad(double* dA, const double* H, int64_t n, hipStream_t s) {
  if (n > 0) hipLaunchKernelGGL(tanh_grad_kernel, dim3(blocks(n)), dim3(kThreads), 0, s, dA, H, n);
}

void launch_mlp_rowsum(const double* A, int rows, int cols, int ld, double* out, hipStream_t s) {
  if (rows > 0) hipLaunchKernelGGL(rowsum_kernel, dim3(blocks(rows)), dim3(kThreads), 0, s, A, rows, cols, ld, out);
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
