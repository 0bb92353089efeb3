// C ABI (include/pinvit.h) and the driver of Algorithm 2.
#include <algorithm>
#include <atomic>
#include <chrono>
#include <cmath>
#include <cstring>
#include <limits>
#include <numeric>
#include <set>
#include <string>
#include <thread>
#include <vector>

#include "engine.hpp"

using namespace pv;

struct pv_ctx {
  Ctx c;
};

namespace {

thread_local std::string g_err;

template <class F>
pv_status guard(F&& f) {
  try {
    f();
    return PV_OK;
  } catch (const Error& e) {
    g_err = e.what();
    return e.code;
  } catch (const std::bad_alloc&) {
    g_err = "host allocation failed";
    return PV_ENOMEM;
  } catch (const std::exception& e) {
    g_err = e.what();
    const std::string w = e.what();
    if (w.rfind("kernel launch", 0) == 0) return PV_EDEVICE;
    return PV_EINVAL;
  }
}

Mps& get(Ctx& c, int h) {
  auto it = c.mps.find(h);
  if (it == c.mps.end()) fail(PV_EINVAL, "unknown MPS handle " + std::to_string(h));
  return *it->second;
}

int put(Ctx& c, std::unique_ptr<Mps> m) {
  const int h = c.next_handle++;
  c.mps[h] = std::move(m);
  return h;
}

// ---- exponential sum (Thm. expsum, eqs. expsum and expsumparams) ----
void expsum_params(double c0, double T, double* h, int* mp, int* mm) {
  *h = M_PI * M_PI / std::log(8.0 * std::sqrt(2.0) / c0 + 1.0);
  const double lg = std::fabs(std::log(std::sqrt(M_PI) * c0 / 4.0));
  *mp = int(std::ceil(std::log(lg) / *h));
  *mm = -int(std::ceil((2.0 * lg + std::log(T)) / *h));
}

double expsum(double t, double h, int mp, int mm) {
  double s = 0.0;
  for (int m = mm; m <= mp; ++m) s += std::exp(m * h / 2.0) * std::exp(-std::exp(m * h) * t);
  return h / std::sqrt(M_PI) * s;
}

// theta_i of Section 7.1.1 with one-based window j = k_i+1 .. k_i+N, k_i = max(0, i-N).
// theta_i of Section 7.1.1 into c.theta
void compute_theta(Ctx& c) {
  const int L = c.L, N = c.N;
  c.theta.assign(L, 0.0);
  for (int i1 = 1; i1 <= L; ++i1) {
    const int ki = std::max(0, i1 - N);
    double acc = c.gamma / N + c.h[size_t(i1 - 1) * L + (i1 - 1)];
    for (int j1 = ki + 1; j1 <= ki + N; ++j1) {
      const int i = i1 - 1, j = j1 - 1;
      auto V = [&](int a, int b, int cc, int d) { return c.v[((size_t(a) * L + b) * L + cc) * L + d]; };
      acc += V(i, j, j, i) - V(i, j, i, j);
    }
    c.theta[i1 - 1] = acc;
  }
}

void setup_precond(Ctx& c, double c0, double cl, double cu) {
  const int L = c.L, N = c.N;
  compute_theta(c);
  if (c.corr.empty()) {
    std::vector<double> s = c.theta;
    std::sort(s.begin(), s.end());
    c.t_min = std::accumulate(s.begin(), s.begin() + N, 0.0);
    c.t_max = std::accumulate(s.end() - N, s.end(), 0.0);
  } else {
    // extremes of sum_{i occ} (theta_i + Delta_{i, particles before i}) over the
    // N-particle determinants: shortest and longest path over (site, particles placed)
    const double inf = std::numeric_limits<double>::infinity();
    std::vector<double> lo(N + 1, inf), hi(N + 1, -inf);
    lo[0] = hi[0] = 0.0;
    for (int i = 0; i < L; ++i)
      for (int n = N; n >= 1; --n) {
        const double w = c.theta[i] + c.corr[size_t(i) * (N + 1) + n - 1];
        if (!(w > 0)) fail(PV_ENOTSPD, "corrected theta is not positive");
        lo[n] = std::min(lo[n], lo[n - 1] + w);
        hi[n] = std::max(hi[n], hi[n - 1] + w);
      }
    c.t_min = lo[N];
    c.t_max = hi[N];
  }
  if (!(c.t_min > 0.0)) fail(PV_ENOTSPD, "t_min <= 0: the shift does not make D positive");
  c.T_ratio = c.t_max / c.t_min;
  expsum_params(c0, c.T_ratio, &c.hs, &c.m_plus, &c.m_minus);
  c.a0 = std::sqrt(2.0 / (c.t_min * (cl * (1 - c0) * (1 - c0) + cu * (1 + c0) * (1 + c0))));
  c.alpha.clear();
  c.beta.clear();
  for (int m = c.m_minus; m <= c.m_plus; ++m) {
    c.alpha.push_back(c.hs * c.a0 / std::sqrt(M_PI) * std::exp(m * c.hs / 2.0));
    c.beta.push_back(std::exp(m * c.hs) / c.t_min);
  }
  c.s_max = c.a0 * expsum(1.0, c.hs, c.m_plus, c.m_minus);
  c.s_min = c.a0 * expsum(c.T_ratio, c.hs, c.m_plus, c.m_minus);
}

// b_delta of eq. bbetarho and the eigenvector bound of eq. everrbound.
double error_bound(double rho, double delta) {
  if (rho * rho > 1.0 / (4.0 * delta * (delta - 1.0))) return std::numeric_limits<double>::quiet_NaN();
  const double disc = 1.0 - 4.0 * (delta - 1.0) * delta * rho * rho;
  const double b = 2.0 * delta / (1.0 + 2.0 * delta * rho * rho + std::sqrt(std::max(disc, 0.0)));
  const double arg = std::sqrt(delta * b) * rho;
  if (arg > 1.0) return std::numeric_limits<double>::quiet_NaN();
  return 2.0 * std::sin(0.5 * std::asin(arg));
}

// Relative eigenvalue bound of eq. releigerr, b_delta(rho) rho^2 / (1 - b_delta(rho) rho^2)
// (NaN outside the domain of b_delta).
double rel_eig_bound(double rho, double delta) {
  const double disc = 1.0 - 4.0 * (delta - 1.0) * delta * rho * rho;
  if (disc < 0.0) return std::numeric_limits<double>::quiet_NaN();
  const double b = 2.0 * delta / (1.0 + 2.0 * delta * rho * rho + std::sqrt(disc));
  return b * rho * rho / (1.0 - b * rho * rho);
}

// Lower eigenpair of the 2x2 pencil (Rem. omegamin), v^T mm v = 1, v[0] > 0.
void ritz2(const double hm[3], const double mm[3], double* lam, double v[2]) {
  // hm = {h00, h01, h11}, mm = {m00, m01, m11}
  const double a = mm[0] * mm[2] - mm[1] * mm[1];
  if (!(a > 0.0)) fail(PV_ENOTSPD, "2x2 Ritz pencil is not definite (search direction parallel to iterate)");
  const double b = -(hm[0] * mm[2] + hm[2] * mm[0] - 2.0 * hm[1] * mm[1]);
  const double cc = hm[0] * hm[2] - hm[1] * hm[1];
  const double disc = std::max(b * b - 4.0 * a * cc, 0.0);
  double r1, r2;
  if (b < 0) { const double q = -0.5 * (b - std::sqrt(disc)); r1 = q / a; r2 = cc / q; }
  else { const double q = -0.5 * (b + std::sqrt(disc)); r1 = cc / q; r2 = q / a; }
  *lam = std::min(r1, r2);
  const double k00 = hm[0] - *lam * mm[0], k01 = hm[1] - *lam * mm[1], k11 = hm[2] - *lam * mm[2];
  double v0, v1;
  if (std::fabs(k00) + std::fabs(k01) >= std::fabs(k01) + std::fabs(k11)) { v0 = -k01; v1 = k00; }
  else { v0 = k11; v1 = -k01; }
  const double nn = std::sqrt(v0 * v0 * mm[0] + 2.0 * v0 * v1 * mm[1] + v1 * v1 * mm[2]);
  v0 /= nn; v1 /= nn;
  if (v0 < 0 || (v0 == 0 && v1 < 0)) { v0 = -v0; v1 = -v1; }
  v[0] = v0; v[1] = v1;
}

double delta_a(double rho, double q) {
  return (-q * rho + std::sqrt(q * q * rho * rho + (1.0 + rho * rho) * (1.0 - q * q))) / (1.0 + rho * rho);
}

// Lowest k eigenpairs of the symmetric pencil (B, M), n x n row-major, M positive definite:
// M = L L^T (Cholesky), cyclic Jacobi on L^{-1} B L^{-T}, eigenvalues ascending, vectors
// V (n x k, row-major) with V^T M V = I; the entry of largest magnitude of each vector
// (the first on ties) is made positive.  For the small Rayleigh-Ritz problems of the
// subspace iteration (n <= 2 PV_SUBSPACE_MAX_D).
void small_pencil(int n, const std::vector<double>& B, const std::vector<double>& M, int k, std::vector<double>& w,
                  std::vector<double>& V) {
  std::vector<double> L(size_t(n) * n, 0.0);
  for (int j = 0; j < n; ++j) {
    double d = M[size_t(j) * n + j];
    for (int q = 0; q < j; ++q) d -= L[size_t(j) * n + q] * L[size_t(j) * n + q];
    if (!(d > 0.0)) fail(PV_ENOTSPD, "Rayleigh-Ritz pencil: Gram matrix is not positive definite");
    L[size_t(j) * n + j] = std::sqrt(d);
    for (int i = j + 1; i < n; ++i) {
      double s = M[size_t(i) * n + j];
      for (int q = 0; q < j; ++q) s -= L[size_t(i) * n + q] * L[size_t(j) * n + q];
      L[size_t(i) * n + j] = s / L[size_t(j) * n + j];
    }
  }
  // X = L^{-1} B (forward substitution per column), A = X L^{-T} = L^{-1} X^T (B symmetric)
  auto lsolve = [&](std::vector<double>& Y) {  // Y <- L^{-1} Y, Y n x n row-major
    for (int c = 0; c < n; ++c)
      for (int i = 0; i < n; ++i) {
        double s = Y[size_t(i) * n + c];
        for (int q = 0; q < i; ++q) s -= L[size_t(i) * n + q] * Y[size_t(q) * n + c];
        Y[size_t(i) * n + c] = s / L[size_t(i) * n + i];
      }
  };
  std::vector<double> A(B);
  lsolve(A);
  std::vector<double> At(size_t(n) * n);
  for (int i = 0; i < n; ++i)
    for (int j = 0; j < n; ++j) At[size_t(i) * n + j] = A[size_t(j) * n + i];
  lsolve(At);
  for (int i = 0; i < n; ++i)
    for (int j = 0; j < i; ++j) {
      const double m = 0.5 * (At[size_t(i) * n + j] + At[size_t(j) * n + i]);
      At[size_t(i) * n + j] = At[size_t(j) * n + i] = m;
    }
  std::vector<double> U(size_t(n) * n, 0.0);
  for (int i = 0; i < n; ++i) U[size_t(i) * n + i] = 1.0;
  for (int sweep = 0; sweep < 100; ++sweep) {
    double off = 0.0, tot = 0.0;
    for (int i = 0; i < n; ++i)
      for (int j = 0; j < n; ++j) {
        const double a = At[size_t(i) * n + j] * At[size_t(i) * n + j];
        tot += a;
        if (i != j) off += a;
      }
    if (off <= 1e-32 * tot || off == 0.0) break;
    for (int p = 0; p < n; ++p)
      for (int q = p + 1; q < n; ++q) {
        const double apq = At[size_t(p) * n + q];
        if (apq == 0.0) continue;
        const double th = (At[size_t(q) * n + q] - At[size_t(p) * n + p]) / (2.0 * apq);
        const double t = (th >= 0 ? 1.0 : -1.0) / (std::fabs(th) + std::sqrt(1.0 + th * th));
        const double cs = 1.0 / std::sqrt(1.0 + t * t), sn = t * cs;
        for (int r = 0; r < n; ++r) {  // columns p, q
          const double x = At[size_t(r) * n + p], y = At[size_t(r) * n + q];
          At[size_t(r) * n + p] = cs * x - sn * y;
          At[size_t(r) * n + q] = sn * x + cs * y;
        }
        for (int r = 0; r < n; ++r) {  // rows p, q
          const double x = At[size_t(p) * n + r], y = At[size_t(q) * n + r];
          At[size_t(p) * n + r] = cs * x - sn * y;
          At[size_t(q) * n + r] = sn * x + cs * y;
        }
        for (int r = 0; r < n; ++r) {
          const double x = U[size_t(r) * n + p], y = U[size_t(r) * n + q];
          U[size_t(r) * n + p] = cs * x - sn * y;
          U[size_t(r) * n + q] = sn * x + cs * y;
        }
      }
  }
  std::vector<int> order(n);
  std::iota(order.begin(), order.end(), 0);
  std::stable_sort(order.begin(), order.end(),
                   [&](int a, int b) { return At[size_t(a) * n + a] < At[size_t(b) * n + b]; });
  w.assign(k, 0.0);
  V.assign(size_t(n) * k, 0.0);
  for (int j = 0; j < k; ++j) {
    const int e = order[j];
    w[j] = At[size_t(e) * n + e];
    // V[:, j] = L^{-T} U[:, e] (back substitution)
    for (int i = n - 1; i >= 0; --i) {
      double s = U[size_t(i) * n + e];
      for (int q = i + 1; q < n; ++q) s -= L[size_t(q) * n + i] * V[size_t(q) * k + j];
      V[size_t(i) * k + j] = s / L[size_t(i) * n + i];
    }
    int im = 0;
    for (int i = 1; i < n; ++i)
      if (std::fabs(V[size_t(i) * k + j]) > std::fabs(V[size_t(im) * k + j])) im = i;
    if (V[size_t(im) * k + j] < 0)
      for (int i = 0; i < n; ++i) V[size_t(i) * k + j] = -V[size_t(i) * k + j];
  }
}

// Starting columns of the subspace iteration: the determinant of the N smallest h_ii (ties
// to the lower index) and its single excitations i -> a in order of h_aa - h_ii (ties: lower
// i, then lower a).
std::vector<std::vector<int>> subspace_starts(const std::vector<double>& h, int L, int N, int D) {
  std::vector<int> idx(L);
  std::iota(idx.begin(), idx.end(), 0);
  std::stable_sort(idx.begin(), idx.end(), [&](int a, int b) { return h[size_t(a) * L + a] < h[size_t(b) * L + b]; });
  std::vector<int> occ(idx.begin(), idx.begin() + N);
  std::sort(occ.begin(), occ.end());
  std::vector<char> in(L, 0);
  for (int o : occ) in[o] = 1;
  struct Ex { double d; int i, a; };
  std::vector<Ex> ex;
  for (int i : occ)
    for (int a = 0; a < L; ++a)
      if (!in[a]) ex.push_back({h[size_t(a) * L + a] - h[size_t(i) * L + i], i, a});
  std::stable_sort(ex.begin(), ex.end(), [](const Ex& x, const Ex& y) {
    if (x.d != y.d) return x.d < y.d;
    if (x.i != y.i) return x.i < y.i;
    return x.a < y.a;
  });
  if (int(ex.size()) < D - 1) fail(PV_EINVAL, "not enough single excitations for D starting columns");
  std::vector<std::vector<int>> out{occ};
  for (int t = 0; t + 1 < D; ++t) {
    std::vector<int> o;
    for (int x : occ)
      if (x != ex[t].i) o.push_back(x);
    o.push_back(ex[t].a);
    std::sort(o.begin(), o.end());
    out.push_back(o);
  }
  return out;
}

}  // namespace

extern "C" {

const char* pv_last_error(void) { return g_err.c_str(); }

pv_status pv_create(pv_ctx** out, int device, void* stream) {
  if (!out) { g_err = "null output pointer"; return PV_EINVAL; }
  *out = nullptr;
  return guard([&] {
    int n = 0;
    if (hipGetDeviceCount(&n) != hipSuccess || n <= device || device < 0) {
      (void)hipGetLastError();
      fail(PV_EDEVICE, "no HIP device " + std::to_string(device));
    }
    PV_HIP(hipSetDevice(device));
    auto* ctx = new pv_ctx();
    try {
      ctx->c.device = device;
      if (stream) {
        ctx->c.stream = static_cast<hipStream_t>(stream);  // the caller's: not destroyed here
        ctx->c.own_stream = false;
      } else {
        PV_HIP(hipStreamCreate(&ctx->c.stream));
      }
      ctx->c.staging.init(size_t(64) << 20);
      (void)noalloc_scratch(device);  // the allocation-free entry point's array on this device
    } catch (...) {
      delete ctx;
      throw;
    }
    *out = ctx;
  });
}

void pv_destroy(pv_ctx* ctx) {
  if (!ctx) return;
  try {
    (void)hipSetDevice(ctx->c.device);
    (void)hipStreamSynchronize(ctx->c.stream);
    if (ctx->c.side_stream) (void)hipStreamSynchronize(ctx->c.side_stream);
    release_aux(ctx->c);
    for (auto e : ctx->c.event_pool) (void)hipEventDestroy(e);
    for (auto& p : ctx->c.tune_pending)
      if (p.owns) { (void)hipEventDestroy(p.a); (void)hipEventDestroy(p.b); }
    for (auto& p : ctx->c.pending) { (void)hipEventDestroy(p.a); (void)hipEventDestroy(p.b); }
    if (ctx->c.fork_event) (void)hipEventDestroy(ctx->c.fork_event);
    if (ctx->c.join_event) (void)hipEventDestroy(ctx->c.join_event);
    hipStream_t s = ctx->c.own_stream ? ctx->c.stream : nullptr, s2 = ctx->c.side_stream;
    delete ctx;
    if (s) (void)hipStreamDestroy(s);
    if (s2) (void)hipStreamDestroy(s2);
  } catch (...) {
  }
}

pv_status pv_set_hamiltonian(pv_ctx* ctx, int L, int N, const double* h, const double* v, double gamma) {
  return guard([&] {
    if (!ctx || !h || !v) fail(PV_EINVAL, "null argument");
    if (L < 2 || L > 127 || N < 1 || N > L - 1) fail(PV_EINVAL, "need 2 <= L <= 127 and 1 <= N <= L-1");
    if (!std::isfinite(gamma)) fail(PV_EINVAL, "gamma not finite");
    const size_t nv = size_t(L) * L * L * L;
    for (size_t i = 0; i < size_t(L) * L; ++i) if (!std::isfinite(h[i])) fail(PV_EINVAL, "h not finite");
    for (size_t i = 0; i < nv; ++i) if (!std::isfinite(v[i])) fail(PV_EINVAL, "v not finite");
    Ctx& c = ctx->c;
    PV_HIP(hipSetDevice(c.device));
    c.sync();
    c.mps.clear();
    c.L = L; c.N = N; c.gamma = gamma;
    c.corr.clear();  // a correction (and an attached network) belongs to one Hamiltonian
    c.net.clear();
    c.net_refresh = 0;
    c.h.assign(h, h + size_t(L) * L);
    c.v.assign(v, v + nv);
    Mpo m = build_mpo(L, h, v, gamma / N);
    c.mpo_w = m.w;
    c.hmpo = upload_mpo(c, m);
    c.ident.reset();
    setup_precond(c, 0.1, 1.0, 1.0);
  });
}

pv_status pv_precond_info(pv_ctx* ctx, double* out, int* m_range) {
  return guard([&] {
    if (!ctx || !out || !m_range) fail(PV_EINVAL, "null argument");
    Ctx& c = ctx->c;
    if (!c.hmpo) fail(PV_ESTATE, "no Hamiltonian set");
    double v[7] = {c.t_min, c.t_max, c.T_ratio, c.hs, c.a0, c.s_min, c.s_max};
    std::memcpy(out, v, sizeof(v));
    m_range[0] = c.m_minus;
    m_range[1] = c.m_plus;
  });
}

pv_status pv_mps_create(pv_ctx* ctx, const int32_t* rho, const double* data, size_t n, int* handle) {
  return guard([&] {
    if (!ctx || !rho || !handle) fail(PV_EINVAL, "null argument");
    Ctx& c = ctx->c;
    if (!c.hmpo) fail(PV_ESTATE, "no Hamiltonian set");
    const int L = c.L, N = c.N;
    std::vector<std::vector<int>> r(L + 1, std::vector<int>(N + 1, 0));
    Mps probe; probe.L = L; probe.N = N;
    for (int k = 0; k <= L; ++k)
      for (int nn = 0; nn <= N; ++nn) {
        const int x = rho[k * (N + 1) + nn];
        if (x < 0 || x > (1 << 20)) fail(PV_EINVAL, "block table entry out of range");
        if (!probe.valid(k, nn) && x != 0) fail(PV_EINVAL, "nonzero rank outside the sector set K_k");
        r[k][nn] = x;
      }
    if (r[0][0] != 1 || r[L][N] < 1 || r[L][N] > PV_SUBSPACE_MAX_D)
      fail(PV_EINVAL, "rho[0][0] must be 1 and rho[L][N] (the number of columns) 1..PV_SUBSPACE_MAX_D");
    auto m = mps_alloc(c, L, N, r);
    if (size_t(m->size()) != n) fail(PV_EINVAL, "data length does not match the block table");
    if (!data && n) fail(PV_EINVAL, "null data");
    for (size_t i = 0; i < n; ++i) if (!std::isfinite(data[i])) fail(PV_EINVAL, "MPS data not finite");
    size_t o = 0;
    for (int k = 1; k <= L; ++k) {
      const size_t s = size_t(m->site_size(k));
      if (s) PV_HIP(hipMemcpyAsync(m->site[k - 1].p, data + o, s * 8, hipMemcpyHostToDevice, c.stream));
      o += s;
    }
    c.sync();
    *handle = put(c, std::move(m));
  });
}

pv_status pv_mps_determinant(pv_ctx* ctx, const int32_t* occupied, int* handle) {
  return guard([&] {
    if (!ctx || !occupied || !handle) fail(PV_EINVAL, "null argument");
    Ctx& c = ctx->c;
    if (!c.hmpo) fail(PV_ESTATE, "no Hamiltonian set");
    std::vector<int> occ(occupied, occupied + c.N);
    std::vector<int> s = occ;
    std::sort(s.begin(), s.end());
    for (int i = 0; i < c.N; ++i)
      if (s[i] < 0 || s[i] >= c.L || (i && s[i] == s[i - 1])) fail(PV_EINVAL, "occupied orbitals must be N distinct indices in [0, L)");
    *handle = put(c, mps_determinant(c, occ));
    c.sync();
  });
}

pv_status pv_mps_layout(pv_ctx* ctx, int handle, int32_t* rho, size_t* n) {
  return guard([&] {
    if (!ctx) fail(PV_EINVAL, "null context");
    Mps& m = get(ctx->c, handle);
    if (rho)
      for (int k = 0; k <= m.L; ++k)
        for (int nn = 0; nn <= m.N; ++nn) rho[k * (m.N + 1) + nn] = m.valid(k, nn) ? m.rho[k][nn] : 0;
    if (n) *n = size_t(m.size());
  });
}

pv_status pv_mps_download(pv_ctx* ctx, int handle, double* data, size_t n) {
  return guard([&] {
    if (!ctx) fail(PV_EINVAL, "null context");
    Ctx& c = ctx->c;
    Mps& m = get(c, handle);
    if (size_t(m.size()) != n) fail(PV_EINVAL, "buffer length does not match the MPS size");
    size_t o = 0;
    for (int k = 1; k <= m.L; ++k) {
      const size_t s = size_t(m.site_size(k));
      if (s) PV_HIP(hipMemcpyAsync(data + o, m.site[k - 1].p, s * 8, hipMemcpyDeviceToHost, c.stream));
      o += s;
    }
    c.sync();
  });
}

pv_status pv_mps_free(pv_ctx* ctx, int handle) {
  return guard([&] {
    if (!ctx) fail(PV_EINVAL, "null context");
    Ctx& c = ctx->c;
    auto it = c.mps.find(handle);
    if (it == c.mps.end()) fail(PV_EINVAL, "unknown MPS handle");
    c.sync();
    c.mps.erase(it);
  });
}

pv_status pv_set_truncation(pv_ctx* ctx, int mode) {
  return guard([&] {
    if (!ctx) fail(PV_EINVAL, "null context");
    if (mode != 0 && mode != 1) fail(PV_EINVAL, "truncation mode must be 0 or 1");
    ctx->c.trunc_mode = mode;
  });
}

pv_status pv_set_tridiag_steps(pv_ctx* ctx, int max_problems) {
  return guard([&] {
    if (!ctx) fail(PV_EINVAL, "null context");
    if (max_problems < 0) fail(PV_EINVAL, "max_problems must be >= 0");
    ctx->c.tri_step_max = max_problems;
  });
}

pv_status pv_set_gemm_tiles(pv_ctx* ctx, int mode) {
  return guard([&] {
    if (!ctx) fail(PV_EINVAL, "null context");
    if (mode < PV_GEMM_TILES_RULE || mode > PV_GEMM_TILES_LARGE) fail(PV_EINVAL, "mode must lie in 0 .. 4");
    ctx->c.sync();  // samples in flight are filed under the mode that issued them
    ctx->c.gemm_tiles = mode;
  });
}

pv_status pv_gemm_tune_table(double* rows, int max_rows, int* n_rows) {
  return guard([&] {
    if (!n_rows || (max_rows > 0 && !rows)) fail(PV_EINVAL, "null argument");
    if (max_rows < 0) fail(PV_EINVAL, "max_rows must be >= 0");
    const std::vector<double> t = gemm_tune_rows();
    const int n = int(t.size() / 9);
    *n_rows = n;
    std::copy(t.begin(), t.begin() + 9 * std::min(n, max_rows), rows);
  });
}

pv_status pv_gemm_tune_clear(void) {
  return guard([&] { gemm_tune_clear(); });
}

pv_status pv_gemm_tune_load(const double* rows, int n_rows) {
  return guard([&] {
    if (n_rows < 0 || (n_rows > 0 && !rows)) fail(PV_EINVAL, "need n_rows >= 0 and rows for n_rows > 0");
    gemm_tune_load(rows, n_rows);
  });
}

pv_status pv_dot(pv_ctx* ctx, int a, int b, double* out) {
  return guard([&] {
    if (!ctx || !out) fail(PV_EINVAL, "null argument");
    *out = dot(ctx->c, get(ctx->c, a), get(ctx->c, b));
  });
}

pv_status pv_expect_h(pv_ctx* ctx, int bra, int ket, double* out) {
  return guard([&] {
    if (!ctx || !out) fail(PV_EINVAL, "null argument");
    *out = expect_h(ctx->c, get(ctx->c, bra), get(ctx->c, ket));
  });
}

pv_status pv_lincomb(pv_ctx* ctx, double a, int x, double b, int y, int* out) {
  return guard([&] {
    if (!ctx || !out) fail(PV_EINVAL, "null argument");
    if (!std::isfinite(a) || !std::isfinite(b)) fail(PV_EINVAL, "coefficients not finite");
    auto m = mps_lincomb(ctx->c, a, get(ctx->c, x), b, get(ctx->c, y));
    ctx->c.sync();
    *out = put(ctx->c, std::move(m));
  });
}

pv_status pv_round(pv_ctx* ctx, int x, double eps, int cap, int* out, int* cap_bound) {
  return guard([&] {
    if (!ctx || !out) fail(PV_EINVAL, "null argument");
    if (!(eps >= 0) || cap < 1) fail(PV_EINVAL, "need eps >= 0 and cap >= 1");
    bool cb = false;
    auto m = round_mps(ctx->c, get(ctx->c, x), eps, cap, &cb);
    ctx->c.sync();
    *out = put(ctx->c, std::move(m));
    if (cap_bound) *cap_bound = cb;
  });
}

pv_status pv_apply_h(pv_ctx* ctx, int x, double eps, int cap, int m_zip, int* out, int* cap_bound,
                     double* zip_discard) {
  return guard([&] {
    if (!ctx || !out) fail(PV_EINVAL, "null argument");
    if (!(eps >= 0) || cap < 1) fail(PV_EINVAL, "need eps >= 0 and cap >= 1");
    bool cb = false;
    double zd2 = 0.0;
    auto m = apply_h(ctx->c, get(ctx->c, x), eps, cap, m_zip, &cb, &zd2);
    if (zip_discard) *zip_discard = std::sqrt(zd2);
    ctx->c.sync();
    *out = put(ctx->c, std::move(m));
    if (cap_bound) *cap_bound = cb;
  });
}

pv_status pv_apply_s(pv_ctx* ctx, int x, double eta, int cap, int* out, int* cap_bound) {
  return guard([&] {
    if (!ctx || !out) fail(PV_EINVAL, "null argument");
    if (!(eta >= 0) || cap < 1) fail(PV_EINVAL, "need eta >= 0 and cap >= 1");
    if (!ctx->c.hmpo) fail(PV_ESTATE, "no Hamiltonian set");
    bool cb = false;
    auto m = apply_s(ctx->c, get(ctx->c, x), eta, cap, &cb);
    ctx->c.sync();
    *out = put(ctx->c, std::move(m));
    if (cap_bound) *cap_bound = cb;
  });
}

// Algorithm 2 on psi = S x (see the oracle's pinvit module for the step list).
// While alive, operator contractions use float32 MFMA if the run asked for it.
struct LowPrecision {
  Ctx& c;
  bool old;
  explicit LowPrecision(Ctx& cx) : c(cx), old(cx.lowp) { c.lowp = c.prec != 0; }
  ~LowPrecision() { c.lowp = old; }
};

// The plain S (no correction) for the life of the object: the correction and the set-up
// of its S are restored on every way out.
struct PlainS {
  Ctx& c;
  const pv_params& p;
  std::vector<double> keep;
  PlainS(Ctx& cx, const pv_params& pp) : c(cx), p(pp), keep(std::move(cx.corr)) {
    c.corr.clear();
    setup();
  }
  ~PlainS() {
    c.corr = std::move(keep);
    try {
      setup();
    } catch (...) {
    }
  }
  void setup() { setup_precond(c, p.c0, p.c_lower > 0 ? p.c_lower : 1.0, p.c_upper > 0 ? p.c_upper : 1.0); }
};

pv_status pv_run(pv_ctx* ctx, const pv_params* prm, int start, pv_result* res, pv_iter* hist,
                 int hist_cap, int* psi_out) {
  return guard([&] {
    if (!ctx || !prm || !res) fail(PV_EINVAL, "null argument");
    Ctx& c = ctx->c;
    if (!c.hmpo) fail(PV_ESTATE, "no Hamiltonian set");
    const pv_params p = *prm;
    if (p.rank_cap < 1 || p.max_iter < 0 || !(p.c > 0 && p.c < 1) || !(p.delta > 1) || !(p.c0 > 0 && p.c0 < 1) ||
        !(p.t_eig > 0 && p.t_eig < 1) || !(p.tau >= 0))
      fail(PV_EINVAL, "invalid parameters");
    if (p.precision < 0 || p.precision > 2)
      fail(PV_EINVAL, "precision must be 0 (float64), 1 (float32 contractions) or 2 (bfloat16 contractions)");
    c.prec = p.precision;
    if (p.truncation != 0 && p.truncation != 1) fail(PV_EINVAL, "truncation mode must be 0 or 1");
    c.trunc_mode = p.truncation;
    // outputs of the sequential truncation are left-orthogonal (norm = last core)
    auto mnorm = [&](const Mps& m) { return c.trunc_mode == 0 ? norm_canonical(c, m) : norm2(c, m); };
    setup_precond(c, p.c0, p.c_lower > 0 ? p.c_lower : 1.0, p.c_upper > 0 ? p.c_upper : 1.0);
    const int L = c.L, N = c.N, cap = p.rank_cap, mz = p.m_zip;
    const double eps_num = p.eps_num > 0 ? p.eps_num : 0.5 * (1.0 - p.c);
    const double zeta = eps_num / (1.0 + p.c);
    double eta = std::numeric_limits<double>::infinity();
    double s_prev = -1, s_prev2 = -1;
    if (p.resume_s > 0) {
      s_prev = p.resume_s;
      s_prev2 = p.resume_s2;
      if (p.resume_eta > 0) eta = p.resume_eta;
    }
    std::unique_ptr<Mps> psi;
    if (start >= 0) {
      const Mps& s0 = get(c, start);
      psi = mps_scaled_copy(c, s0, 1.0, nullptr);
    } else {
      std::vector<int> idx(L);
      std::iota(idx.begin(), idx.end(), 0);
      std::stable_sort(idx.begin(), idx.end(), [&](int a, int b) { return c.h[size_t(a) * L + a] < c.h[size_t(b) * L + b]; });
      std::vector<int> occ(idx.begin(), idx.begin() + N);
      psi = mps_determinant(c, occ);
    }
    // a sweep started on the auxiliary stream reads psi: on every way out, it ends first
    struct Drain {
      Ctx& c;
      ~Drain() { expect_h_drain(c); }
    } drain{c};
    int rows = 0;
    *res = pv_result{};
    c.judge_plain = c.judge_corr = 0;
    for (int it = 0; it < p.max_iter; ++it) {
      const auto t0 = std::chrono::steady_clock::now();
      const double nrm = std::sqrt(dot(c, *psi, *psi));
      if (!(nrm > 0)) fail(PV_ENOCONV, "iterate vanished");
      psi = mps_scaled_copy(c, *psi, 1.0 / nrm, nullptr);
      // the Rayleigh quotient's sweep reads psi only: it runs beside the intermediate-rank
      // application of H below and is collected where lambda is first used
      expect_h_begin(c, *psi, *psi);
      double lam = 0.0;
      bool have_lam = false;
      auto lam_now = [&] {
        if (!have_lam) {
          lam = expect_h_end(c);
          have_lam = true;
        }
        return lam;
      };
      if (!c.net.empty() && it % c.net_refresh == 0) {
        lam_now();
        // the attached network corrects theta from the current iterate's features
        std::vector<double> delta(size_t(L) * (N + 1));
        compute_theta(c);
        learned_correction(c, c.net.data(), *psi, lam, c.theta, delta.data());
        c.corr = std::move(delta);
        setup_precond(c, p.c0, p.c_lower > 0 ? p.c_lower : 1.0, p.c_upper > 0 ? p.c_upper : 1.0);
      }
      double est;
      if (s_prev < 0) {
        std::unique_ptr<Mps> y0;
        {
          LowPrecision lp(c);
          y0 = apply_h(c, *psi, 0.0, cap, mz, nullptr);
        }
        auto d0 = mps_lincomb(c, 1.0, *y0, -lam_now(), *psi);
        auto r0 = round_mps(c, *d0, 0.0, cap, nullptr);
        est = c.s_max * mnorm(*r0);
      } else if (s_prev2 <= 0) {
        est = s_prev;
      } else {
        est = s_prev * std::min(1.0, s_prev / s_prev2);
      }
      eta = std::min(2.0 * eta, 0.8 * zeta * est);
      int retries = 0;
      bool capb = false;
      std::unique_ptr<Mps> r, s;
      double ns = 0, zd2 = 0;
      while (true) {
        bool cb1 = false, cb2 = false, cb3 = false;
        const double e12 = eta / (3.0 * c.s_max);
        std::unique_ptr<Mps> y;
        zd2 = 0.0;
        {
          LowPrecision lp(c);
          y = apply_h(c, *psi, e12, cap, mz, &cb1, &zd2);
        }
        auto d = mps_lincomb(c, 1.0, *y, -lam_now(), *psi);
        y.reset();
        r = round_mps(c, *d, e12, cap, &cb2);
        d.reset();
        s = apply_s(c, *r, eta / 3.0, cap, &cb3);
        capb = cb1 || cb2 || cb3;
        ns = mnorm(*s);
        if (ns >= (1.0 + 1.0 / zeta) * eta || capb || retries >= p.max_retries) break;
        eta *= 0.8;
        ++retries;
      }
      lam_now();
      bool cb4 = false;
      auto pdir = apply_s(c, *s, c.s_max * eta / 3.0, cap, &cb4);
      const double nr = mnorm(*r);
      const double rho = (ns + eta) / (std::sqrt(1.0 - p.c) * std::sqrt(lam));
      const double bound = error_bound(rho, p.delta);
      pv_iter rec{};
      rec.lambda = lam;
      rec.energy = lam - c.gamma;
      rec.rho = rho;
      rec.bound = bound;
      rec.r_norm = nr;
      rec.s_norm = ns;
      rec.eta_res = eta;
      rec.retries = retries;
      rec.cap_bound = (capb || cb4) ? 1 : 0;
      rec.zip_discard = std::sqrt(zd2);
      rec.zip_bound = zd2 > 0.0 ? 1 : 0;
      res->energy = rec.energy;
      res->lambda = lam;
      res->rho = rho;
      res->bound = bound;
      // with a binding intermediate rank the residual is not within eta_res of the true
      // one, so the bound is not certified and the run does not stop on it
      if (bound <= p.tau && !rec.zip_bound) {
        rec.stopped = 1;
        rec.max_rank = psi->max_rank();
        c.sync();
        rec.seconds = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
        if (hist && rows < hist_cap) hist[rows] = rec;
        ++rows;
        res->converged = 1;
        break;
      }
      const double np = mnorm(*pdir);
      if (!(np > 0)) {
        // the direction vanished under the truncation tolerances: psi is an eigenvector to
        // those tolerances, the run stops (as on a sector of dimension 2)
        rec.stopped = 1;
        rec.max_rank = psi->max_rank();
        c.sync();
        rec.seconds = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
        if (hist && rows < hist_cap) hist[rows] = rec;
        ++rows;
        res->converged = 1;
        break;
      }
      auto z2 = mps_scaled_copy(c, *pdir, 1.0 / np, nullptr);
      pdir.reset();
      double h12, h22;
      {
        LowPrecision lp(c);  // the Ritz sandwiches may use the low-precision contractions
        // the two sandwiches run side by side, h12 on the auxiliary stream
        expect_h_begin(c, *psi, *z2);
        h22 = expect_h(c, *z2, *z2);
        h12 = expect_h_end(c);
      }
      const double o12 = dot(c, *psi, *z2);
      const double hm[3] = {lam, h12, h22}, mm[3] = {1.0, o12, 1.0};
      double lam_s, v[2];
      ritz2(hm, mm, &lam_s, v);
      double s_min_step = c.s_min;
      bool cbj = false;
      if (c.judge && !c.corr.empty()) {
        // the judge: the same residual r through the plain S (its own s_max and s_min, the
        // same eta); the direction whose Ritz value is lower makes the step (the corrected
        // one on ties), and the update's tolerance takes that S's s_min
        PlainS plain(c, p);
        bool cj1 = false, cj2 = false;
        auto sB = apply_s(c, *r, eta / 3.0, cap, &cj1);
        auto pB = apply_s(c, *sB, c.s_max * eta / 3.0, cap, &cj2);
        sB.reset();
        const double npB = mnorm(*pB);
        bool plain_wins = false;
        if (npB > 0) {
          auto zB = mps_scaled_copy(c, *pB, 1.0 / npB, nullptr);
          pB.reset();
          double h12B, h22B;
          {
            LowPrecision lp(c);
            expect_h_begin(c, *psi, *zB);
            h22B = expect_h(c, *zB, *zB);
            h12B = expect_h_end(c);
          }
          const double o12B = dot(c, *psi, *zB);
          const double hmB[3] = {lam, h12B, h22B}, mmB[3] = {1.0, o12B, 1.0};
          double lamB, vB[2];
          ritz2(hmB, mmB, &lamB, vB);
          if (lamB < lam_s) {
            plain_wins = true;
            lam_s = lamB;
            v[0] = vB[0];
            v[1] = vB[1];
            z2 = std::move(zB);
            s_min_step = c.s_min;
            cbj = cj1 || cj2;
          }
        }
        ++(plain_wins ? c.judge_plain : c.judge_corr);
      }
      const double q = std::sqrt(lam_s / (lam_s + p.t_eig * (lam - lam_s)));
      const double da = delta_a(rho, q);
      const double eta_in = da * std::sqrt(lam_s) / std::sqrt(1.0 + p.c);
      const double eta_psi = eta_in * s_min_step;
      auto comb = mps_lincomb(c, v[0], *psi, v[1], *z2);
      bool cb5 = false;
      psi = round_mps(c, *comb, eta_psi, cap, &cb5);
      c.sync();
      rec.cap_bound |= cbj ? 1 : 0;
      rec.lambda_star = lam_s;
      rec.eta_psi = eta_psi;
      rec.cap_bound |= cb5 ? 1 : 0;
      rec.max_rank = psi->max_rank();
      rec.seconds = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
      if (hist && rows < hist_cap) hist[rows] = rec;
      ++rows;
      s_prev2 = s_prev;
      s_prev = ns;
      res->eta_res = eta;
      res->s_last = s_prev;
      res->s_prev = s_prev2;
    }
    res->iterations = rows;
    if (psi_out) *psi_out = put(c, std::move(psi));
  });
}

// Algorithm 3 (outer iteration): PINVIT to the eigenvector tolerance
// tau_m = eta^m / (2 (1 + (1+alpha) kappa)), kappa of eq. kappadef, stop when the relative
// eigenvalue bound of eq. releigerr is below tol, else truncate the normalised iterate
// with theta eta^m (converted to psi = S x with s_min) and halve eta (Thm. quasioptr).
pv_status pv_run_outer(pv_ctx* ctx, const pv_params* prm, double alpha, double tol, int max_outer,
                       pv_result* res, pv_outer_iter* hist, int hist_cap, int* psi_out) {
  return guard([&] {
    if (!ctx || !prm || !res) fail(PV_EINVAL, "null argument");
    if (!(alpha > 0) || !(tol > 0) || max_outer < 1) fail(PV_EINVAL, "need alpha > 0, tol > 0, max_outer >= 1");
    if (!(prm->c > 0 && prm->c < 1)) fail(PV_EINVAL, "invalid parameters");
    Ctx& c = ctx->c;
    if (!c.hmpo) fail(PV_ESTATE, "no Hamiltonian set");
    const pv_params p = *prm;
    const double kappa = std::sqrt((1.0 + p.c) / (1.0 - p.c)) * std::sqrt(double(std::max(c.L - 1, 1)));
    const double ak = (1.0 + alpha) * kappa;
    const double theta = ak / (2.0 * (1.0 + ak));
    double eta = 1.0 / (2.0 * theta);
    *res = pv_result{};
    int start = -1, rows = 0;
    // the intermediate iterate is released if a step fails
    struct Release {
      Ctx& c;
      int* h;
      ~Release() { if (*h >= 0) c.mps.erase(*h); }
    } release{c, &start};
    std::vector<pv_iter> ih(size_t(std::max(p.max_iter, 1)));
    for (int m = 0; m < max_outer; ++m) {
      pv_params inner = p;
      inner.tau = eta / (2.0 * (1.0 + ak));
      inner.resume_eta = inner.resume_s = inner.resume_s2 = 0.0;  // every inner run starts afresh
      pv_result r{};
      int y = -1;
      const pv_status st = pv_run(ctx, &inner, start, &r, ih.data(), int(ih.size()), &y);
      if (st != PV_OK) fail(st, std::string("inner iteration of outer step ") + std::to_string(m) + ": " + pv_last_error());
      if (start >= 0) c.mps.erase(start);
      start = y;  // released by `release` should a later step fail
      if (r.iterations < 1) fail(PV_EINVAL, "inner iteration limit must be at least 1");
      const pv_iter& last = ih[size_t(std::min(r.iterations, int(ih.size())) - 1)];
      pv_outer_iter rec{};
      rec.eta = eta;
      rec.tau = inner.tau;
      rec.lambda = last.lambda;
      rec.energy = last.energy;
      rec.rho = last.rho;
      rec.rel_bound = rel_eig_bound(last.rho, p.delta);
      rec.inner_iterations = r.iterations;
      const double ny = norm2(c, get(c, start));
      if (!(ny > 0)) fail(PV_ENOCONV, "iterate vanished");
      auto yn = mps_scaled_copy(c, get(c, start), 1.0 / ny, nullptr);
      c.mps.erase(start);
      start = -1;
      res->energy = last.energy;
      res->lambda = last.lambda;
      res->rho = last.rho;
      res->bound = last.bound;
      if (rec.rel_bound < tol) {
        rec.stopped = 1;
        rec.max_rank = yn->max_rank();
        if (hist && rows < hist_cap) hist[rows] = rec;
        ++rows;
        res->converged = 1;
        start = put(c, std::move(yn));
        break;
      }
      const double eps = c.s_min * theta * eta;
      bool cb = false;
      auto t = round_mps(c, *yn, eps, p.rank_cap, &cb);
      c.sync();
      rec.trunc_eps = eps;
      rec.cap_bound = cb ? 1 : 0;
      rec.max_rank = t->max_rank();
      if (hist && rows < hist_cap) hist[rows] = rec;
      ++rows;
      start = put(c, std::move(t));
      eta *= 0.5;
    }
    res->iterations = rows;
    if (psi_out) {
      *psi_out = start;
      start = -1;  // handed to the caller
    }
  });
}

pv_status pv_run_batch(pv_ctx* const* ctxs, int count, const pv_params* prm, pv_result* res, pv_status* status) {
  return guard([&] {
    if (count < 0) fail(PV_EINVAL, "negative problem count");
    if (count == 0) return;
    if (!ctxs || !prm || !res) fail(PV_EINVAL, "null argument");
    std::set<pv_ctx*> seen;
    for (int i = 0; i < count; ++i) {
      if (!ctxs[i]) fail(PV_EINVAL, "null context in the batch");
      if (!seen.insert(ctxs[i]).second) fail(PV_EINVAL, "a context appears twice in the batch");
    }
    // problems are independent: each runs pv_run on its own context (own stream and memory
    // pool) in a worker thread, so the device interleaves the kernels of different problems
    const unsigned hw = std::max(1u, std::thread::hardware_concurrency());
    const int workers = std::min<int>(count, int(std::min(hw, 16u)));
    std::vector<pv_status> st(count, PV_OK);
    std::vector<std::string> msg(count);
    std::atomic<int> next{0};
    std::vector<std::thread> pool;
    for (int w = 0; w < workers; ++w)
      pool.emplace_back([&] {
        for (int i; (i = next.fetch_add(1)) < count;) {
          const int dev = ctxs[i]->c.device;
          // one stream per problem: with many contexts a second stream each measured slower
          ctxs[i]->c.use_side = false;
          st[i] = hipSetDevice(dev) == hipSuccess ? pv_run(ctxs[i], &prm[i], -1, &res[i], nullptr, 0, nullptr)
                                                  : PV_EDEVICE;
          ctxs[i]->c.use_side = true;
          if (st[i] != PV_OK) msg[i] = pv_last_error();
        }
      });
    for (auto& t : pool) t.join();
    if (status) std::copy(st.begin(), st.end(), status);
    for (int i = 0; i < count; ++i)
      if (st[i] != PV_OK) fail(st[i], "problem " + std::to_string(i) + ": " + msg[i]);
  });
}

pv_status pv_sym_eig(pv_ctx* ctx, int n, const double* A, double* w, double* V, int method) {
  return guard([&] {
    if (!ctx || !A || !w || !V) fail(PV_EINVAL, "null argument");
    if (n < 1 || n > kEigMax) fail(PV_EINVAL, "n out of range");
    if (method != 0 && method != 1) fail(PV_EINVAL, "method must be 0 or 1");
    for (size_t i = 0; i < size_t(n) * n; ++i) if (!std::isfinite(A[i])) fail(PV_EINVAL, "A not finite");
    sym_eig(ctx->c, n, A, w, V, method);
  });
}

pv_status pv_sym_eig_noalloc(pv_ctx* ctx, int n, const double* A, double* w, double* V) {
  return guard([&] {
    if (!ctx || !A || !w || !V) fail(PV_EINVAL, "null argument");
    sym_eig_noalloc(ctx->c, n, A, w, V);
  });
}

pv_status pv_mfma_f64_rate(pv_ctx* ctx, double* tflops) {
  return guard([&] {
    if (!ctx || !tflops) fail(PV_EINVAL, "null argument");
    Ctx& c = ctx->c;
    int ncu = 0;
    PV_HIP(hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, c.device));
    // eight workgroups of four wavefronts per compute unit: eight wavefronts per SIMD
    const int blocks = 8 * std::max(ncu, 1), iters = 20000;
    Buf out(c.pool, size_t(blocks) * 256);
    hipEvent_t e0 = nullptr, e1 = nullptr;
    PV_HIP(hipEventCreate(&e0));
    PV_HIP(hipEventCreate(&e1));
    struct Events {
      hipEvent_t a, b;
      ~Events() { (void)hipEventDestroy(a); (void)hipEventDestroy(b); }
    } ev{e0, e1};
    c.sync();
    launch_mfma_rate(out.p, blocks, iters, c.stream);  // warm-up
    PV_HIP(hipEventRecord(e0, c.stream));
    launch_mfma_rate(out.p, blocks, iters, c.stream);
    PV_HIP(hipEventRecord(e1, c.stream));
    PV_HIP(hipEventSynchronize(e1));
    float ms = 0.f;
    PV_HIP(hipEventElapsedTime(&ms, e0, e1));
    const double flops = double(blocks) * 4.0 * iters * 4.0 * 2048.0;
    *tflops = ms > 0.f ? flops / (double(ms) * 1e-3) / 1e12 : 0.0;
    c.sync();
  });
}

pv_status pv_gemm(pv_ctx* ctx, int M, int N, int K, const double* A, int lda, int ta, const double* B, int ldb,
                  int tb, double* C, int ldc, double alpha, double beta, int precision) {
  return guard([&] {
    if (!ctx || !C || (K > 0 && (!A || !B))) fail(PV_EINVAL, "null argument");
    if (M < 1 || N < 1 || K < 0) fail(PV_EINVAL, "sizes out of range");
    if ((ta != 0 && ta != 1) || (tb != 0 && tb != 1)) fail(PV_EINVAL, "ta, tb must be 0 or 1");
    if (lda < (ta ? K : M) || lda < 1 || ldb < (tb ? N : K) || ldb < 1 || ldc < M) fail(PV_EINVAL, "leading dimension too small");
    if (precision < 0 || precision > 2) fail(PV_EINVAL, "precision must be 0 (float64), 1 (float32) or 2 (bfloat16)");
    gemm_host(ctx->c, M, N, K, A, lda, ta, B, ldb, tb, C, ldc, alpha, beta, precision);
  });
}

pv_status pv_sym_eig_top(pv_ctx* ctx, int n, const double* A, double* w, double* V, int nvec) {
  return guard([&] {
    if (!ctx || !A || !w || !V) fail(PV_EINVAL, "null argument");
    if (n < 1 || n > kEigMax) fail(PV_EINVAL, "n out of range");
    if (nvec < 0 || nvec > n) fail(PV_EINVAL, "nvec must lie in [0, n]");
    for (size_t i = 0; i < size_t(n) * n; ++i) if (!std::isfinite(A[i])) fail(PV_EINVAL, "A not finite");
    sym_eig(ctx->c, n, A, w, V, 1, nvec);
  });
}

pv_status pv_cholesky(pv_ctx* ctx, int n, const double* A, double* W) {
  return guard([&] {
    if (!ctx || !A || !W) fail(PV_EINVAL, "null argument");
    if (n < 1 || n > kEigMax) fail(PV_EINVAL, "n out of range");
    for (size_t i = 0; i < size_t(n) * n; ++i) if (!std::isfinite(A[i])) fail(PV_EINVAL, "A not finite");
    cholesky(ctx->c, n, A, W);
  });
}

// Algorithm 2 on x (z-form): term-by-term products with A and E and the sorted sum of the
// M^2 residual terms; see the header.
pv_status pv_run_zform(pv_ctx* ctx, const pv_params* prm, int start, pv_result* res, pv_iter* hist,
                       int hist_cap, int* x_out) {
  return guard([&] {
    if (!ctx || !prm || !res) fail(PV_EINVAL, "null argument");
    Ctx& c = ctx->c;
    if (!c.hmpo) fail(PV_ESTATE, "no Hamiltonian set");
    if (!c.corr.empty()) fail(PV_ESTATE, "the z-form does not take a learned correction");
    const pv_params p = *prm;
    if (p.rank_cap < 1 || p.max_iter < 0 || !(p.c > 0 && p.c < 1) || !(p.delta > 1) || !(p.c0 > 0 && p.c0 < 1) ||
        !(p.t_eig > 0 && p.t_eig < 1) || !(p.tau >= 0))
      fail(PV_EINVAL, "invalid parameters");
    if (p.precision != 0) fail(PV_EINVAL, "the z-form runs in float64 only");
    if (p.truncation != 0 && p.truncation != 1) fail(PV_EINVAL, "truncation mode must be 0 or 1");
    c.prec = 0;
    c.trunc_mode = p.truncation;
    auto mnorm = [&](const Mps& m) { return c.trunc_mode == 0 ? norm_canonical(c, m) : norm2(c, m); };
    setup_precond(c, p.c0, p.c_lower > 0 ? p.c_lower : 1.0, p.c_upper > 0 ? p.c_upper : 1.0);
    const int L = c.L, N = c.N, cap = p.rank_cap, M = int(c.alpha.size());
    const int exact_cap = 1 << 30;
    std::vector<std::vector<double>> occ(M, std::vector<double>(L));
    for (int m = 0; m < M; ++m)
      for (int k = 0; k < L; ++k) occ[m][k] = std::exp(-c.beta[m] * c.theta[k]);
    auto term = [&](const Mps& x, int m) { return mps_scaled_copy(c, x, c.alpha[m], occ[m].data()); };
    // <a, A b> and <a, E b>, summed over all pairs (k, k')
    auto products = [&](const Mps& a, const Mps& b, double* ha, double* ea) {
      std::vector<std::unique_ptr<Mps>> sa(M), sb(M);
      for (int m = 0; m < M; ++m) {
        sa[m] = term(a, m);
        sb[m] = term(b, m);
      }
      double h = 0.0, e = 0.0;
      for (int k = 0; k < M; ++k)
        for (int k2 = 0; k2 < M; ++k2) {
          h += expect_h(c, *sa[k], *sb[k2]);
          e += dot(c, *sa[k], *sb[k2]);
        }
      *ha = h;
      *ea = e;
    };
    const double eps_num = p.eps_num > 0 ? p.eps_num : 0.5 * (1.0 - p.c);
    const double zeta = eps_num / (1.0 + p.c);
    double eta = std::numeric_limits<double>::infinity();
    std::unique_ptr<Mps> x;
    if (start >= 0) {
      x = mps_scaled_copy(c, get(c, start), 1.0, nullptr);
    } else {
      std::vector<int> idx(L);
      std::iota(idx.begin(), idx.end(), 0);
      std::stable_sort(idx.begin(), idx.end(), [&](int a, int b) { return c.h[size_t(a) * L + a] < c.h[size_t(b) * L + b]; });
      x = mps_determinant(c, std::vector<int>(idx.begin(), idx.begin() + N));
    }
    struct Term {
      double norm;
      int k, k2;
      std::unique_ptr<Mps> s;
    };
    int rows = 0;
    *res = pv_result{};
    for (int it = 0; it < p.max_iter; ++it) {
      const auto t0 = std::chrono::steady_clock::now();
      double num, den;
      products(*x, *x, &num, &den);
      if (!(num > 0 && den > 0)) fail(PV_ENOTSPD, "iterate has no positive A-norm");
      const double lam = num / den;
      x = mps_scaled_copy(c, *x, 1.0 / std::sqrt(num), nullptr);
      // residual terms S_k (H - lambda) S_k' x, exact
      std::vector<Term> terms;
      double est = 0.0;
      for (int k2 = 0; k2 < M; ++k2) {
        auto u = term(*x, k2);
        auto hu = apply_h(c, *u, 0.0, exact_cap, p.m_zip, nullptr);
        auto g = mps_lincomb(c, 1.0, *hu, -lam, *u);
        for (int k = 0; k < M; ++k) {
          auto s = term(*g, k);
          const double n = std::sqrt(std::max(dot(c, *s, *s), 0.0));
          est += n;
          terms.push_back(Term{n, k, k2, std::move(s)});
        }
      }
      std::sort(terms.begin(), terms.end(), [](const Term& a, const Term& b) {
        if (a.norm != b.norm) return a.norm < b.norm;
        if (a.k != b.k) return a.k < b.k;
        return a.k2 < b.k2;
      });
      eta = std::min(2.0 * eta, 0.8 * zeta * est);
      int retries = 0;
      bool capb = false;
      std::unique_ptr<Mps> r;
      double nr = 0.0;
      while (true) {
        capb = false;
        double csum = 0.0;
        size_t j0 = 0;
        for (size_t j = 0; j < terms.size(); ++j) {
          if (csum + terms[j].norm <= eta / 3.0) { csum += terms[j].norm; j0 = j + 1; }
          else break;
        }
        double total = 0.0;
        for (size_t j = j0; j < terms.size(); ++j) total += terms[j].norm;
        std::unique_ptr<Mps> y;
        for (size_t j = j0; j < terms.size(); ++j) {
          const double eps_j = total > 0 ? eta * terms[j].norm / (3.0 * total) : 0.0;
          bool cb = false;
          if (!y) y = round_mps(c, *terms[j].s, eps_j, cap, &cb);
          else {
            auto sum = mps_lincomb(c, 1.0, *y, 1.0, *terms[j].s);
            y = round_mps(c, *sum, eps_j, cap, &cb);
          }
          capb = capb || cb;
        }
        if (y) {
          bool cb = false;
          r = round_mps(c, *y, eta / 3.0, cap, &cb);
          capb = capb || cb;
          nr = mnorm(*r);
        } else {
          r = mps_zero_like(c, *x);
          nr = 0.0;
        }
        if (nr >= (1.0 + 1.0 / zeta) * eta || capb || retries >= p.max_retries) break;
        eta *= 0.8;
        ++retries;
      }
      terms.clear();
      const double rho = (nr + eta) / std::sqrt(1.0 - p.c);
      const double bound = error_bound(rho, p.delta);
      pv_iter rec{};
      rec.lambda = lam;
      rec.energy = lam - c.gamma;
      rec.rho = rho;
      rec.bound = bound;
      rec.r_norm = nr;
      rec.s_norm = nr;
      rec.eta_res = eta;
      rec.retries = retries;
      rec.cap_bound = capb ? 1 : 0;
      res->energy = rec.energy;
      res->lambda = lam;
      res->rho = rho;
      res->bound = bound;
      res->eta_res = eta;
      if (bound <= p.tau) {
        rec.stopped = 1;
        rec.max_rank = x->max_rank();
        c.sync();
        rec.seconds = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
        if (hist && rows < hist_cap) hist[rows] = rec;
        ++rows;
        res->converged = 1;
        break;
      }
      if (!(nr > 0)) fail(PV_ENOCONV, "residual vanished before the tolerance test succeeded");
      auto rh = mps_scaled_copy(c, *r, 1.0 / nr, nullptr);
      r.reset();
      double h01, e01, h11, e11;
      products(*x, *rh, &h01, &e01);
      products(*rh, *rh, &h11, &e11);
      // x has unit A-norm: <x, A x> = 1 and <x, E x> = den / num
      const double hm[3] = {1.0, h01, h11}, mm[3] = {den / num, e01, e11};
      double lam_s, z[2];
      ritz2(hm, mm, &lam_s, z);
      const double q = std::sqrt(lam_s / (lam_s + p.t_eig * (lam - lam_s)));
      const double eta_in = delta_a(rho, q) * std::sqrt(lam_s) / std::sqrt(1.0 + p.c);
      auto comb = mps_lincomb(c, z[0], *x, z[1], *rh);
      bool cb5 = false;
      x = round_mps(c, *comb, eta_in, cap, &cb5);
      c.sync();
      rec.lambda_star = lam_s;
      rec.eta_psi = eta_in;
      rec.cap_bound |= cb5 ? 1 : 0;
      rec.max_rank = x->max_rank();
      rec.seconds = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
      if (hist && rows < hist_cap) hist[rows] = rec;
      ++rows;
    }
    res->iterations = rows;
    if (x_out) *x_out = put(c, std::move(x));
  });
}

// Learned correction of theta (an extension): see the header.
pv_status pv_set_correction(pv_ctx* ctx, const double* delta) {
  return guard([&] {
    if (!ctx) fail(PV_EINVAL, "null argument");
    Ctx& c = ctx->c;
    if (!c.hmpo) fail(PV_ESTATE, "no Hamiltonian set");
    if (!delta) {
      c.corr.clear();
      setup_precond(c, 0.1, 1.0, 1.0);  // the default preconditioner, as after pv_set_hamiltonian
      return;
    }
    const size_t n = size_t(c.L) * (c.N + 1);
    for (size_t e = 0; e < n; ++e)
      if (!std::isfinite(delta[e])) fail(PV_EINVAL, "correction is not finite");
    std::vector<double> keep(delta, delta + n);
    compute_theta(c);
    for (int i = 0; i < c.L; ++i)
      for (int k = 0; k < c.N; ++k)
        if (!(c.theta[i] + keep[size_t(i) * (c.N + 1) + k] > 0))
          fail(PV_ENOTSPD, "corrected theta is not positive");
    c.corr = std::move(keep);
    setup_precond(c, 0.1, 1.0, 1.0);  // pv_apply_s and pv_precond_info see the corrected S
  });
}

// the iterate the features describe (psi, or the start determinant of pv_run) and its
// Rayleigh quotient
static std::unique_ptr<Mps> feature_state(Ctx& c, int psi, double* lam) {
  std::unique_ptr<Mps> x;
  if (psi >= 0) {
    x = mps_scaled_copy(c, get(c, psi), 1.0, nullptr);
  } else {
    std::vector<int> idx(c.L);
    std::iota(idx.begin(), idx.end(), 0);
    std::stable_sort(idx.begin(), idx.end(), [&](int a, int b) { return c.h[size_t(a) * c.L + a] < c.h[size_t(b) * c.L + b]; });
    x = mps_determinant(c, std::vector<int>(idx.begin(), idx.begin() + c.N));
  }
  const double nx = dot(c, *x, *x);
  if (!(nx > 0)) fail(PV_EINVAL, "zero state");
  *lam = expect_h(c, *x, *x) / nx;
  return x;
}

pv_status pv_learned_correction(pv_ctx* ctx, const float* params, int psi, double* delta) {
  return guard([&] {
    if (!ctx || !params || !delta) fail(PV_EINVAL, "null argument");
    Ctx& c = ctx->c;
    if (!c.hmpo) fail(PV_ESTATE, "no Hamiltonian set");
    compute_theta(c);
    double lam = 0;
    auto x = feature_state(c, psi, &lam);
    learned_correction(c, params, *x, lam, c.theta, delta);
  });
}

pv_status pv_learned_train(pv_ctx* ctx, float* params, int psi, const uint64_t* masks, int nmask, int steps,
                           float lr, double* loss, double* grad) {
  return guard([&] {
    if (!ctx || !params || (nmask > 0 && !masks)) fail(PV_EINVAL, "null argument");
    if (nmask < 1 || steps < 0 || !(lr >= 0)) fail(PV_EINVAL, "need nmask >= 1, steps >= 0, lr >= 0");
    Ctx& c = ctx->c;
    if (!c.hmpo) fail(PV_ESTATE, "no Hamiltonian set");
    if (c.L > 64) fail(PV_EINVAL, "sample masks hold at most 64 orbitals");
    compute_theta(c);
    double lam = 0;
    auto x = feature_state(c, psi, &lam);
    learned_train(c, params, *x, lam, c.theta, masks, nmask, steps, lr, loss, grad);
  });
}

pv_status pv_learned_train_solves(pv_ctx* ctx, float* params, int psi, const uint64_t* masks, int nmask,
                                  const double* rvals, const double* tvals, int steps, float lr, double* loss,
                                  double* grad) {
  return guard([&] {
    if (!ctx || !params || !masks || !rvals || !tvals) fail(PV_EINVAL, "null argument");
    if (nmask < 1 || steps < 0 || !(lr >= 0)) fail(PV_EINVAL, "need nmask >= 1, steps >= 0, lr >= 0");
    Ctx& c = ctx->c;
    if (!c.hmpo) fail(PV_ESTATE, "no Hamiltonian set");
    if (c.L > 64) fail(PV_EINVAL, "sample masks hold at most 64 orbitals");
    for (int b = 0; b < nmask; ++b)
      if (!std::isfinite(rvals[b]) || !std::isfinite(tvals[b])) fail(PV_EINVAL, "samples not finite");
    compute_theta(c);
    double lam = 0;
    auto x = feature_state(c, psi, &lam);
    learned_train(c, params, *x, lam, c.theta, masks, nmask, steps, lr, loss, grad, rvals, tvals);
  });
}

pv_status pv_set_learned_network(pv_ctx* ctx, const float* params, int refresh) {
  return guard([&] {
    if (!ctx) fail(PV_EINVAL, "null argument");
    Ctx& c = ctx->c;
    if (!c.hmpo) fail(PV_ESTATE, "no Hamiltonian set");
    if (!params) {
      c.net.clear();
      c.net_refresh = 0;
      return;
    }
    if (refresh < 1) fail(PV_EINVAL, "refresh must be at least 1");
    for (int i = 0; i < PV_MLP_PARAMS; ++i)
      if (!std::isfinite(params[i])) fail(PV_EINVAL, "network parameters not finite");
    c.net.assign(params, params + PV_MLP_PARAMS);
    c.net_refresh = refresh;
  });
}

pv_status pv_set_learned_judge(pv_ctx* ctx, int on) {
  return guard([&] {
    if (!ctx) fail(PV_EINVAL, "null argument");
    if (on != 0 && on != 1) fail(PV_EINVAL, "on must be 0 or 1");
    ctx->c.judge = on != 0;
  });
}

pv_status pv_learned_judge_counts(pv_ctx* ctx, int* plain, int* corrected) {
  return guard([&] {
    if (!ctx || !plain || !corrected) fail(PV_EINVAL, "null argument");
    *plain = ctx->c.judge_plain;
    *corrected = ctx->c.judge_corr;
  });
}

pv_status pv_solve_h(pv_ctx* ctx, int b, double rel_tol, int max_iter, int* out, int* iters, double* rel_res) {
  return guard([&] {
    if (!ctx || !out) fail(PV_EINVAL, "null argument");
    if (!(rel_tol > 0) || max_iter < 1) fail(PV_EINVAL, "need rel_tol > 0 and max_iter >= 1");
    Ctx& c = ctx->c;
    if (!c.hmpo) fail(PV_ESTATE, "no Hamiltonian set");
    if (c.alpha.empty()) setup_precond(c, 0.1, 1.0, 1.0);
    int it = 0;
    double rr = 0;
    auto x = solve_h(c, get(c, b), rel_tol, max_iter, &it, &rr);
    if (iters) *iters = it;
    if (rel_res) *rel_res = rr;
    *out = put(c, std::move(x));
  });
}

pv_status pv_mps_amplitudes(pv_ctx* ctx, int handle, const uint64_t* masks, int n, double* out) {
  return guard([&] {
    if (!ctx || (n > 0 && (!masks || !out))) fail(PV_EINVAL, "null argument");
    if (n < 0) fail(PV_EINVAL, "negative count");
    Ctx& c = ctx->c;
    const Mps& x = get(c, handle);
    if (x.L > 64) fail(PV_EINVAL, "masks hold at most 64 orbitals");
    amplitudes(c, x, masks, n, out);
  });
}

// Algorithm 4 (subspace iteration, Section 6) on D separate columns; see the header for the
// readings.  Phi holds the columns as stored; the Rayleigh-Ritz coefficients C of an
// iteration give the E-orthonormal basis psi_i = sum_j C_ji phi_j, formed exactly (MPS
// concatenation) where H, the residual or the update need it.
pv_status pv_run_subspace(pv_ctx* ctx, const pv_params* prm, int D, const int* starts, pv_result* res,
                          pv_subspace_iter* hist, int hist_cap, int* psi_out) {
  return guard([&] {
    if (!ctx || !prm || !res) fail(PV_EINVAL, "null argument");
    if (D < 1 || D > PV_SUBSPACE_MAX_D) fail(PV_EINVAL, "D out of range");
    Ctx& c = ctx->c;
    if (!c.hmpo) fail(PV_ESTATE, "no Hamiltonian set");
    {
      // the 2D Ritz vectors are dependent in a sector of dimension below 2D
      double dim = 1.0;
      for (int i = 1; i <= c.N; ++i) dim = dim * double(c.L - c.N + i) / double(i);
      if (2.0 * D > dim + 0.5) fail(PV_EINVAL, "the 2D Ritz vectors need a sector of dimension at least 2D");
    }
    const pv_params p = *prm;
    if (p.rank_cap < 1 || p.max_iter < 0 || !(p.c > 0 && p.c < 1) || !(p.delta > 1) || !(p.c0 > 0 && p.c0 < 1) ||
        !(p.t_eig > 0 && p.t_eig < 1) || !(p.tau >= 0))
      fail(PV_EINVAL, "invalid parameters");
    if (p.precision < 0 || p.precision > 2)
      fail(PV_EINVAL, "precision must be 0 (float64), 1 (float32 contractions) or 2 (bfloat16 contractions)");
    if (p.truncation != 0 && p.truncation != 1) fail(PV_EINVAL, "truncation mode must be 0 or 1");
    c.prec = p.precision;
    c.trunc_mode = p.truncation;
    auto mnorm = [&](const Mps& m) { return c.trunc_mode == 0 ? norm_canonical(c, m) : norm2(c, m); };
    setup_precond(c, p.c0, p.c_lower > 0 ? p.c_lower : 1.0, p.c_upper > 0 ? p.c_upper : 1.0);
    const int cap = p.rank_cap, mz = p.m_zip;
    const double eps_num = p.eps_num > 0 ? p.eps_num : 0.5 * (1.0 - p.c);
    const double zeta = eps_num / (1.0 + p.c);
    double eta = std::numeric_limits<double>::infinity();
    double s_prev = -1, s_prev2 = -1;
    std::vector<std::unique_ptr<Mps>> phi(D);
    if (starts) {
      for (int i = 0; i < D; ++i) phi[i] = mps_scaled_copy(c, get(c, starts[i]), 1.0, nullptr);
    } else {
      const auto dets = subspace_starts(c.h, c.L, c.N, D);
      for (int i = 0; i < D; ++i) phi[i] = mps_determinant(c, dets[i]);
    }
    // sum_j a_j x_j by concatenation (exact)
    auto combine = [&](const std::vector<const Mps*>& xs, const std::vector<double>& a) {
      std::unique_ptr<Mps> acc = mps_scaled_copy(c, *xs[0], a[0], nullptr);
      for (size_t j = 1; j < xs.size(); ++j) acc = mps_lincomb(c, 1.0, *acc, a[j], *xs[j]);
      return acc;
    };
    std::vector<const Mps*> phip(D);
    int rows = 0;
    *res = pv_result{};
    std::vector<std::unique_ptr<Mps>> psi(D);
    for (int it = 0; it < p.max_iter; ++it) {
      const auto t0 = std::chrono::steady_clock::now();
      pv_subspace_iter rec{};
      for (int i = 0; i < D; ++i) phip[i] = phi[i].get();
      // 1. Rayleigh-Ritz on span phi: Hm C = Em C Lambda, C^T Em C = I
      std::vector<double> Hm(size_t(D) * D), Em(size_t(D) * D);
      for (int i = 0; i < D; ++i)
        for (int j = i; j < D; ++j) {
          Hm[size_t(i) * D + j] = Hm[size_t(j) * D + i] = expect_h(c, *phi[i], *phi[j]);
          Em[size_t(i) * D + j] = Em[size_t(j) * D + i] = dot(c, *phi[i], *phi[j]);
        }
      std::vector<double> lam, Cm;
      small_pencil(D, Hm, Em, D, lam, Cm);
      for (int i = 0; i < D; ++i) {
        std::vector<double> a(D);
        for (int j = 0; j < D; ++j) a[j] = Cm[size_t(j) * D + i];
        psi[i] = combine(phip, a);
        if (!(lam[i] > 0)) fail(PV_ENOTSPD, "Rayleigh quotient is not positive (H_gamma not positive definite)");
      }
      // 2. start value of eta_res
      double est = 0.0;
      if (s_prev < 0) {
        for (int i = 0; i < D; ++i) {
          std::unique_ptr<Mps> y0;
          {
            LowPrecision lp(c);
            y0 = apply_h(c, *psi[i], 0.0, cap, mz, nullptr);
          }
          auto d0 = mps_lincomb(c, 1.0, *y0, -lam[i], *psi[i]);
          auto r0 = round_mps(c, *d0, 0.0, cap, nullptr);
          est = std::max(est, c.s_max * mnorm(*r0));
        }
      } else if (s_prev2 <= 0) {
        est = s_prev;
      } else {
        est = s_prev * std::min(1.0, s_prev / s_prev2);
      }
      eta = std::min(2.0 * eta, 0.8 * zeta * est);
      // 3.-4. residuals r_i, s_i = S r_i; eta reduced while the smallest ||s_i|| is too small
      int retries = 0;
      bool capb = false;
      std::vector<std::unique_ptr<Mps>> s(D);
      std::vector<double> ns(D);
      while (true) {
        capb = false;
        const double e12 = eta / (3.0 * c.s_max);
        double nmin = std::numeric_limits<double>::infinity();
        for (int i = 0; i < D; ++i) {
          bool cb1 = false, cb2 = false, cb3 = false;
          std::unique_ptr<Mps> y;
          {
            LowPrecision lp(c);
            y = apply_h(c, *psi[i], e12, cap, mz, &cb1);
          }
          auto d = mps_lincomb(c, 1.0, *y, -lam[i], *psi[i]);
          y.reset();
          auto r = round_mps(c, *d, e12, cap, &cb2);
          d.reset();
          s[i] = apply_s(c, *r, eta / 3.0, cap, &cb3);
          ns[i] = mnorm(*s[i]);
          nmin = std::min(nmin, ns[i]);
          capb = capb || cb1 || cb2 || cb3;
        }
        if (nmin >= (1.0 + 1.0 / zeta) * eta || capb || retries >= p.max_retries) break;
        eta *= 0.8;
        ++retries;
      }
      std::vector<double> rho(D);
      for (int i = 0; i < D; ++i) rho[i] = (ns[i] + eta) / (std::sqrt(1.0 - p.c) * std::sqrt(lam[i]));
      const double bound = error_bound(rho[0], p.delta);
      for (int i = 0; i < D; ++i) {
        rec.lambda[i] = lam[i];
        rec.energy[i] = lam[i] - c.gamma;
        rec.rho[i] = rho[i];
        rec.s_norm[i] = ns[i];
      }
      rec.bound = bound;
      rec.eta_res = eta;
      rec.retries = retries;
      rec.cap_bound = capb ? 1 : 0;
      res->energy = lam[0] - c.gamma;
      res->lambda = lam[0];
      res->rho = rho[0];
      res->bound = bound;
      res->eta_res = eta;
      if (bound <= p.tau) {
        rec.stopped = 1;
        int mr = 0;
        for (int i = 0; i < D; ++i) mr = std::max(mr, psi[i]->max_rank());
        rec.max_rank = mr;
        c.sync();
        rec.seconds = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
        if (hist && rows < hist_cap) hist[rows] = rec;
        ++rows;
        res->converged = 1;
        for (int i = 0; i < D; ++i) phi[i] = std::move(psi[i]);
        break;
      }
      // 6. directions p_i / ||p_i|| and the 2D x 2D Rayleigh-Ritz step on (psi, p)
      std::vector<std::unique_ptr<Mps>> pd(D);
      std::vector<double> np(D);
      bool cb4 = false;
      int vanished = 0;
      for (int i = 0; i < D; ++i) {
        bool cb = false;
        pd[i] = apply_s(c, *s[i], c.s_max * eta / 3.0, cap, &cb);
        cb4 = cb4 || cb;
        np[i] = mnorm(*pd[i]);
        vanished += !(np[i] > 0);
        s[i].reset();
      }
      if (vanished == D) {
        // every direction vanished under the truncation tolerances: the columns span an
        // invariant subspace to those tolerances and the run stops
        rec.stopped = 1;
        int mr = 0;
        for (int i = 0; i < D; ++i) mr = std::max(mr, psi[i]->max_rank());
        rec.max_rank = mr;
        c.sync();
        rec.seconds = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
        if (hist && rows < hist_cap) hist[rows] = rec;
        ++rows;
        res->converged = 1;
        for (int i = 0; i < D; ++i) phi[i] = std::move(psi[i]);
        break;
      }
      if (vanished) fail(PV_ENOCONV, "a search direction vanished while others did not");
      for (int i = 0; i < D; ++i) pd[i] = mps_scaled_copy(c, *pd[i], 1.0 / np[i], nullptr);
      const int n2 = 2 * D;
      std::vector<double> B(size_t(n2) * n2, 0.0), M(size_t(n2) * n2, 0.0);
      {
        LowPrecision lp(c);  // the Ritz sandwiches may use the low-precision contractions
        // <phi_j | H | p_k>, <p_i | H | p_k>
        std::vector<double> hp(size_t(D) * D), op(size_t(D) * D);
        for (int j = 0; j < D; ++j)
          for (int k = 0; k < D; ++k) {
            hp[size_t(j) * D + k] = expect_h(c, *phi[j], *pd[k]);
            op[size_t(j) * D + k] = dot(c, *phi[j], *pd[k]);
          }
        for (int i = 0; i < D; ++i)
          for (int k = i; k < D; ++k) {
            B[size_t(D + i) * n2 + D + k] = B[size_t(D + k) * n2 + D + i] = expect_h(c, *pd[i], *pd[k]);
            M[size_t(D + i) * n2 + D + k] = M[size_t(D + k) * n2 + D + i] = dot(c, *pd[i], *pd[k]);
          }
        for (int i = 0; i < D; ++i) {
          B[size_t(i) * n2 + i] = lam[i];
          M[size_t(i) * n2 + i] = 1.0;
          for (int k = 0; k < D; ++k) {
            double bh = 0.0, bo = 0.0;
            for (int j = 0; j < D; ++j) {
              bh += Cm[size_t(j) * D + i] * hp[size_t(j) * D + k];
              bo += Cm[size_t(j) * D + i] * op[size_t(j) * D + k];
            }
            B[size_t(i) * n2 + D + k] = B[size_t(D + k) * n2 + i] = bh;
            M[size_t(i) * n2 + D + k] = M[size_t(D + k) * n2 + i] = bo;
          }
        }
      }
      std::vector<double> lam_s, W;
      small_pencil(n2, B, M, D, lam_s, W);
      // 7. truncation tolerance: the smallest of the per-column tolerances
      double eta_in = std::numeric_limits<double>::infinity();
      for (int i = 0; i < D; ++i) {
        const double q = std::sqrt(lam_s[i] / (lam_s[i] + p.t_eig * (lam[i] - lam_s[i])));
        eta_in = std::min(eta_in, delta_a(rho[i], q) * std::sqrt(lam_s[i]) / std::sqrt(1.0 + p.c));
      }
      const double eta_psi = eta_in * c.s_min;
      // new column i = sum_j (C W1)_ji phi_j + sum_k W2_ki p_k, truncated
      std::vector<const Mps*> terms(n2);
      for (int j = 0; j < D; ++j) {
        terms[j] = phi[j].get();
        terms[D + j] = pd[j].get();
      }
      std::vector<std::unique_ptr<Mps>> next(D);
      bool cb5 = false;
      int mr = 0;
      for (int i = 0; i < D; ++i) {
        std::vector<double> a(n2, 0.0);
        for (int j = 0; j < D; ++j) {
          double v = 0.0;
          for (int l = 0; l < D; ++l) v += Cm[size_t(j) * D + l] * W[size_t(l) * D + i];
          a[j] = v;
          a[D + j] = W[size_t(D + j) * D + i];
        }
        auto comb = combine(terms, a);
        bool cb = false;
        next[i] = round_mps(c, *comb, eta_psi, cap, &cb);
        cb5 = cb5 || cb;
        mr = std::max(mr, next[i]->max_rank());
      }
      for (int i = 0; i < D; ++i) {
        phi[i] = std::move(next[i]);
        psi[i].reset();
      }
      c.sync();
      for (int i = 0; i < D; ++i) rec.lambda_star[i] = lam_s[i];
      rec.eta_psi = eta_psi;
      rec.cap_bound |= (cb4 || cb5) ? 1 : 0;
      rec.max_rank = mr;
      rec.seconds = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
      if (hist && rows < hist_cap) hist[rows] = rec;
      ++rows;
      s_prev2 = s_prev;
      s_prev = *std::max_element(ns.begin(), ns.end());
      res->s_last = s_prev;
      res->s_prev = s_prev2;
    }
    res->iterations = rows;
    if (psi_out)
      for (int i = 0; i < D; ++i) psi_out[i] = put(c, std::move(phi[i]));
  });
}

// Algorithm 4 with the D columns held jointly (Section 6.2): one MPS whose right boundary
// is the column index.  The same steps as pv_run_subspace, with every product, residual,
// S sum and truncation acting on all columns at once (one tolerance, shared ranks), the
// normalisation and the Ritz combinations applied to the column index (the last core).
pv_status pv_run_subspace_joint(pv_ctx* ctx, const pv_params* prm, int D, int start, pv_result* res,
                                pv_subspace_iter* hist, int hist_cap, int* psi_out) {
  return guard([&] {
    if (!ctx || !prm || !res) fail(PV_EINVAL, "null argument");
    if (D < 1 || D > PV_SUBSPACE_MAX_D) fail(PV_EINVAL, "D out of range");
    Ctx& c = ctx->c;
    if (!c.hmpo) fail(PV_ESTATE, "no Hamiltonian set");
    {
      double dim = 1.0;
      for (int i = 1; i <= c.N; ++i) dim = dim * double(c.L - c.N + i) / double(i);
      if (2.0 * D > dim + 0.5) fail(PV_EINVAL, "the 2D Ritz vectors need a sector of dimension at least 2D");
    }
    const pv_params p = *prm;
    if (p.rank_cap < 1 || p.max_iter < 0 || !(p.c > 0 && p.c < 1) || !(p.delta > 1) || !(p.c0 > 0 && p.c0 < 1) ||
        !(p.t_eig > 0 && p.t_eig < 1) || !(p.tau >= 0))
      fail(PV_EINVAL, "invalid parameters");
    if (p.precision < 0 || p.precision > 2)
      fail(PV_EINVAL, "precision must be 0 (float64), 1 (float32 contractions) or 2 (bfloat16 contractions)");
    if (p.truncation != 0 && p.truncation != 1) fail(PV_EINVAL, "truncation mode must be 0 or 1");
    c.prec = p.precision;
    c.trunc_mode = p.truncation;
    setup_precond(c, p.c0, p.c_lower > 0 ? p.c_lower : 1.0, p.c_upper > 0 ? p.c_upper : 1.0);
    const int L = c.L, N = c.N, cap = p.rank_cap, mz = p.m_zip;
    const double eps_num = p.eps_num > 0 ? p.eps_num : 0.5 * (1.0 - p.c);
    const double zeta = eps_num / (1.0 + p.c);
    double eta = std::numeric_limits<double>::infinity();
    double s_prev = -1, s_prev2 = -1;
    std::unique_ptr<Mps> phi;
    if (start >= 0) {
      const Mps& s0 = get(c, start);
      if (s0.rho[L][N] != D) fail(PV_EINVAL, "the start holds a different number of columns");
      phi = mps_scaled_copy(c, s0, 1.0, nullptr);
    } else {
      const auto dets = subspace_starts(c.h, L, N, D);
      phi = mps_determinant(c, dets[0]);
      for (int i = 1; i < D; ++i) {
        auto d = mps_determinant(c, dets[i]);
        phi = mps_lincomb(c, 1.0, *phi, 1.0, *d, true);
      }
    }
    // symmetric part of a column-major D x D result, row-major for small_pencil
    auto sym = [](const std::vector<double>& v, int n) {
      std::vector<double> o(size_t(n) * n);
      for (int i = 0; i < n; ++i)
        for (int j = 0; j < n; ++j) o[size_t(i) * n + j] = 0.5 * (v[size_t(i) + size_t(n) * j] + v[size_t(j) + size_t(n) * i]);
      return o;
    };
    auto col_norms = [&](const Mps& x) {
      auto g = dot_matrix(c, x, x);
      std::vector<double> nv(D);
      for (int i = 0; i < D; ++i) nv[i] = std::sqrt(std::max(g[size_t(i) + size_t(D) * i], 0.0));
      return nv;
    };
    auto diag = [&](const std::vector<double>& d) {
      std::vector<double> W(size_t(D) * D, 0.0);
      for (int i = 0; i < D; ++i) W[size_t(i) + size_t(D) * i] = d[i];
      return W;
    };
    int rows = 0;
    *res = pv_result{};
    for (int it = 0; it < p.max_iter; ++it) {
      const auto t0 = std::chrono::steady_clock::now();
      pv_subspace_iter rec{};
      // 1. Rayleigh-Ritz on span phi; psi = phi C (the index core times C)
      std::vector<double> lam, Cm;
      small_pencil(D, sym(expect_matrix(c, *phi, *phi), D), sym(dot_matrix(c, *phi, *phi), D), D, lam, Cm);
      std::vector<double> Wc(size_t(D) * D);
      for (int j = 0; j < D; ++j)
        for (int i = 0; i < D; ++i) Wc[size_t(j) + size_t(D) * i] = Cm[size_t(j) * D + i];
      for (int i = 0; i < D; ++i)
        if (!(lam[i] > 0)) fail(PV_ENOTSPD, "Rayleigh quotient is not positive (H_gamma not positive definite)");
      auto psi = mps_index_transform(c, *phi, Wc, D);
      auto psil = mps_index_transform(c, *psi, diag(lam), D);  // psi Lambda
      // 2. start value of eta_res (largest column norm)
      double est = 0.0;
      if (s_prev < 0) {
        std::unique_ptr<Mps> y0;
        {
          LowPrecision lp(c);
          y0 = apply_h(c, *psi, 0.0, cap, mz, nullptr);
        }
        auto d0 = mps_lincomb(c, 1.0, *y0, -1.0, *psil);
        auto r0 = round_mps(c, *d0, 0.0, cap, nullptr);
        for (double v : col_norms(*r0)) est = std::max(est, c.s_max * v);
      } else if (s_prev2 <= 0) {
        est = s_prev;
      } else {
        est = s_prev * std::min(1.0, s_prev / s_prev2);
      }
      eta = std::min(2.0 * eta, 0.8 * zeta * est);
      // 3.-4. joint residual R = H psi - psi Lambda and S = S(R)
      int retries = 0;
      bool capb = false;
      std::unique_ptr<Mps> S;
      std::vector<double> ns;
      while (true) {
        bool cb1 = false, cb2 = false, cb3 = false;
        const double e12 = eta / (3.0 * c.s_max);
        std::unique_ptr<Mps> y;
        {
          LowPrecision lp(c);
          y = apply_h(c, *psi, e12, cap, mz, &cb1);
        }
        auto d = mps_lincomb(c, 1.0, *y, -1.0, *psil);
        y.reset();
        auto r = round_mps(c, *d, e12, cap, &cb2);
        d.reset();
        S = apply_s(c, *r, eta / 3.0, cap, &cb3);
        ns = col_norms(*S);
        capb = cb1 || cb2 || cb3;
        if (*std::min_element(ns.begin(), ns.end()) >= (1.0 + 1.0 / zeta) * eta || capb || retries >= p.max_retries)
          break;
        eta *= 0.8;
        ++retries;
      }
      std::vector<double> rho(D);
      for (int i = 0; i < D; ++i) rho[i] = (ns[i] + eta) / (std::sqrt(1.0 - p.c) * std::sqrt(lam[i]));
      const double bound = error_bound(rho[0], p.delta);
      for (int i = 0; i < D; ++i) {
        rec.lambda[i] = lam[i];
        rec.energy[i] = lam[i] - c.gamma;
        rec.rho[i] = rho[i];
        rec.s_norm[i] = ns[i];
      }
      rec.bound = bound;
      rec.eta_res = eta;
      rec.retries = retries;
      rec.cap_bound = capb ? 1 : 0;
      res->energy = lam[0] - c.gamma;
      res->lambda = lam[0];
      res->rho = rho[0];
      res->bound = bound;
      res->eta_res = eta;
      auto finish = [&]() {
        rec.stopped = 1;
        rec.max_rank = psi->max_rank();
        c.sync();
        rec.seconds = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
        if (hist && rows < hist_cap) hist[rows] = rec;
        ++rows;
        res->converged = 1;
        phi = std::move(psi);
      };
      if (bound <= p.tau) {
        finish();
        break;
      }
      // 6. directions P = S(S R), columns normalised; Rayleigh-Ritz on [psi | P]
      bool cb4 = false;
      auto P = apply_s(c, *S, c.s_max * eta / 3.0, cap, &cb4);
      S.reset();
      const auto np = col_norms(*P);
      int vanished = 0;
      for (double v : np) vanished += !(v > 0);
      if (vanished == D) {
        finish();
        break;
      }
      if (vanished) fail(PV_ENOCONV, "a search direction vanished while others did not");
      std::vector<double> inv(D);
      for (int i = 0; i < D; ++i) inv[i] = 1.0 / np[i];
      auto pn = mps_index_transform(c, *P, diag(inv), D);
      P.reset();
      auto bas = mps_lincomb(c, 1.0, *psi, 1.0, *pn, true);  // 2D columns
      pn.reset();
      const int n2 = 2 * D;
      std::vector<double> Bm, Mm;
      {
        LowPrecision lp(c);
        Bm = sym(expect_matrix(c, *bas, *bas), n2);
      }
      Mm = sym(dot_matrix(c, *bas, *bas), n2);
      std::vector<double> lam_s, W;
      small_pencil(n2, Bm, Mm, D, lam_s, W);
      // 7. truncation tolerance and the update psi <- trunc(bas W)
      double eta_in = std::numeric_limits<double>::infinity();
      for (int i = 0; i < D; ++i) {
        const double q = std::sqrt(lam_s[i] / (lam_s[i] + p.t_eig * (lam[i] - lam_s[i])));
        eta_in = std::min(eta_in, delta_a(rho[i], q) * std::sqrt(lam_s[i]) / std::sqrt(1.0 + p.c));
      }
      const double eta_psi = eta_in * c.s_min;
      std::vector<double> Wc2(size_t(n2) * D);
      for (int l = 0; l < n2; ++l)
        for (int i = 0; i < D; ++i) Wc2[size_t(l) + size_t(n2) * i] = W[size_t(l) * D + i];
      auto comb = mps_index_transform(c, *bas, Wc2, D);
      bas.reset();
      bool cb5 = false;
      phi = round_mps(c, *comb, eta_psi, cap, &cb5);
      c.sync();
      for (int i = 0; i < D; ++i) rec.lambda_star[i] = lam_s[i];
      rec.eta_psi = eta_psi;
      rec.cap_bound |= (cb4 || cb5) ? 1 : 0;
      rec.max_rank = phi->max_rank();
      rec.seconds = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
      if (hist && rows < hist_cap) hist[rows] = rec;
      ++rows;
      s_prev2 = s_prev;
      s_prev = *std::max_element(ns.begin(), ns.end());
      res->s_last = s_prev;
      res->s_prev = s_prev2;
    }
    res->iterations = rows;
    if (psi_out) *psi_out = put(c, std::move(phi));
  });
}

static const char* kTimerNames[T_COUNT] = {"gemm_f64_mfma", "jacobi_eig_f64", "mpo_wstep", "copy_scale", "reduce",
                                            "tridiag_reduce_f64", "cholesky_f64", "gemm_f32_mfma",
                                            "tridiag_vectors_f64", "tridiag_back_f64", "tridiag_values_f64",
                                            "tridiag_update_gemm_f64", "gemm_bf16_mfma", "tridiag_tail_f64"};

pv_status pv_timers(pv_ctx* ctx, int n, double* ms, double* flops, double* bytes, int* calls) {
  return guard([&] {
    if (!ctx) fail(PV_EINVAL, "null context");
    Ctx& c = ctx->c;
    c.sync();
    for (int i = 0; i < n && i < T_COUNT; ++i) {
      if (ms) ms[i] = c.t_ms[i];
      if (flops) flops[i] = c.t_flops[i];
      if (bytes) bytes[i] = c.t_bytes[i];
      if (calls) calls[i] = c.t_calls[i];
    }
  });
}

const char* pv_timer_name(int i) { return (i >= 0 && i < T_COUNT) ? kTimerNames[i] : ""; }

pv_status pv_set_timer_mask(pv_ctx* ctx, uint32_t mask) {
  return guard([&] {
    if (!ctx) fail(PV_EINVAL, "null context");
    ctx->c.sync();
    ctx->c.timer_mask = mask;
  });
}

pv_status pv_set_timer_sampling(pv_ctx* ctx, uint32_t mask, int every) {
  return guard([&] {
    if (!ctx) fail(PV_EINVAL, "null context");
    if (every < 1) fail(PV_EINVAL, "sampling period must be >= 1");
    ctx->c.sync();
    ctx->c.sample_mask = mask;
    ctx->c.sample_every = every;
    for (auto& n : ctx->c.sample_count) n = 0;
  });
}

pv_status pv_timers_reset(pv_ctx* ctx) {
  return guard([&] {
    if (!ctx) fail(PV_EINVAL, "null context");
    Ctx& c = ctx->c;
    c.sync();
    for (int i = 0; i < T_COUNT; ++i) { c.t_ms[i] = 0; c.t_flops[i] = 0; c.t_bytes[i] = 0; c.t_calls[i] = 0; }
  });
}

pv_status pv_mpo_bond_dims(int L, const double* h, const double* v, int32_t* dims, int32_t* qdims) {
  return guard([&] {
    if (!h || !v || !dims) fail(PV_EINVAL, "null argument");
    if (L < 2 || L > 127) fail(PV_EINVAL, "L out of range");
    Mpo m = build_mpo(L, h, v, 0.0);
    for (int k = 0; k <= L; ++k) {
      dims[k] = m.w[k];
      if (qdims)
        for (int q = 0; q < 5; ++q) qdims[k * 5 + q] = m.qoff[k][q + 1] - m.qoff[k][q];
    }
  });
}

pv_status pv_mpo_dense(int L, const double* h, const double* v, double diag_shift, double* out) {
  return guard([&] {
    if (!h || !v || !out) fail(PV_EINVAL, "null argument");
    if (L < 1 || L > 8) fail(PV_EINVAL, "dense MPO contraction needs 1 <= L <= 8");
    Mpo m = build_mpo(L, h, v, diag_shift);
    mpo_to_dense(m, out);
  });
}

}  // extern "C"
