// Device kernels of the learned preconditioner correction (an extension, not in the
// paper): feature rows, the elementwise parts of a two-hidden-layer tanh network whose
// matrix products run through the block GEMM, the misfit of the corrected diagonal on
// sampled determinants, and Adam with bfloat16-rounded working weights.
#pragma once
#include <hip/hip_runtime.h>

#include <cstdint>

namespace pv {

constexpr int kMlpFeat = 6;
constexpr int kMlpWidth = 256;
// flat parameter vector: W1 (width x feat, row-major), b1, W2 (width x width), b2, W3, b3
constexpr int64_t kMlpParams = int64_t(kMlpWidth) * kMlpFeat + kMlpWidth + int64_t(kMlpWidth) * kMlpWidth +
                               kMlpWidth + kMlpWidth + 1;

// X (kMlpFeat x L(N+1), column r = i(N+1) + n): theta_i/tbar, h_ii/tbar, n/N, i/L,
// dens_i, lam/(N tbar)
void launch_mlp_features(const double* th, const double* hd, const double* dens, int L, int N, double tbar,
                         double lam, double* X, hipStream_t s);
// A (rows x cols, ld) <- tanh(A + b[row])
void launch_mlp_bias_tanh(double* A, const double* b, int rows, int cols, int ld, hipStream_t s);
// tz[r] = tanh(z[r] + b3[0]); delta[r] = dmax tz[r]
void launch_mlp_output(const double* z, const double* b3, int R, double dmax, double* tz, double* delta,
                       hipStream_t s);
// target[b] = gamma + sum_i h_ii n_i + sum_{i != j} jk[i + j L] n_i n_j (bit i of masks[b])
void launch_mlp_target(const uint64_t* masks, int B, const double* hd, const double* jk, double gamma, int L,
                       double* target, hipStream_t s);
// e_b = sum_{i occ} (theta_i + delta[i(N+1) + n_i]) - target[b]; G[i(N+1) + n_i] += scale e_b;
// loss[0] += lscale e_b^2 (G and loss cleared by the caller)
// Solve form: rv, tv (B each) the residual and its exact solve at the sampled determinants.
void launch_mlp_solve_misfit(const uint64_t* masks, int B, const double* th, const double* delta, const double* rv,
                             const double* tv, int L, int N, double gscale, double lscale, double* G, double* loss,
                             hipStream_t s);
void launch_mlp_misfit(const uint64_t* masks, int B, const double* th, const double* delta, const double* target,
                       int L, int N, double scale, double lscale, double* G, double* loss, hipStream_t s);
// dz[r] = G[r] dmax (1 - tz[r]^2)
void launch_mlp_dz(const double* G, const double* tz, int R, double dmax, double* dz, hipStream_t s);
// dA[e] *= 1 - H[e]^2 (both rows x cols with ld = rows)
void launch_mlp_tanh_grad(double* dA, const double* H, int64_t n, hipStream_t s);
// out[u] = sum_c A[u + c ld], u < rows
void launch_mlp_rowsum(const double* A, int rows, int cols, int ld, double* out, hipStream_t s);
// Adam step t on the float32 parameters w (moments m, v), gradient g; wq = bf16(w) as double
void launch_mlp_adam(float* w, float* m, float* v, const double* g, int64_t P, float lr, float b1, float b2,
                     float eps, float c1, float c2, double* wq, hipStream_t s);
// wq = bf16(w) as double
void launch_mlp_round(const float* w, int64_t P, double* wq, hipStream_t s);

}  // namespace pv
