// Host-side runtime of the block-sparse PINVIT path: device memory pool, block-sparse
// MPS storage, batched launch builders and the operations of one iteration.
#pragma once
#include <hip/hip_runtime.h>

#include <array>
#include <cstdint>
#include <map>
#include <memory>
#include <stdexcept>
#include <string>
#include <vector>

#include "../../include/pinvit.h"
#include "kernels.hpp"
#include "mpo.hpp"

namespace pv {

struct Error : std::runtime_error {
  pv_status code;
  Error(pv_status c, const std::string& m) : std::runtime_error(m), code(c) {}
};
[[noreturn]] inline void fail(pv_status c, const std::string& m) { throw Error(c, m); }

#define PV_HIP(x)                                                                      \
  do {                                                                                 \
    hipError_t e_ = (x);                                                               \
    if (e_ != hipSuccess)                                                              \
      ::pv::fail(e_ == hipErrorOutOfMemory ? PV_ENOMEM : PV_EDEVICE,                    \
                 std::string(#x) + ": " + hipGetErrorString(e_));                      \
  } while (0)

// Caching device allocator.  Sizes are rounded to 1/8 of their power-of-two class so
// buffers are reused across iterations; release is stream ordered because the kernels of a
// context run on its main stream.  While a side stream runs beside it (Ctx::fork .. join)
// released blocks are held back until the join, after which every later launch is ordered
// behind the work of both streams.
class Pool {
 public:
  ~Pool();
  void* get(size_t bytes);
  void put(void* p, size_t bytes);
  void release();
  void hold(bool on);  // on: keep released blocks aside; off: make them reusable
  size_t in_use() const { return in_use_; }
  size_t cached() const { return cached_; }
 private:
  std::multimap<size_t, void*> free_;
  std::vector<std::pair<size_t, void*>> held_;
  bool holding_ = false;
  size_t in_use_ = 0, cached_ = 0;
};

struct Buf {
  Pool* pool = nullptr;
  double* p = nullptr;
  size_t n = 0;
  Buf() = default;
  Buf(Pool& pl, size_t count);
  Buf(const Buf&) = delete;
  Buf& operator=(const Buf&) = delete;
  Buf(Buf&& o) noexcept { *this = std::move(o); }
  Buf& operator=(Buf&& o) noexcept;
  ~Buf() { reset(); }
  void reset();
};

// Pinned host staging for launch descriptors; reset at every stream synchronisation.
class Staging {
 public:
  ~Staging();
  void* put(const void* src, size_t bytes);  // returns pinned copy
  void reset() { used_ = 0; }
  bool fits(size_t bytes) const { return used_ + ((bytes + 255) & ~size_t(255)) <= cap_; }
  void init(size_t cap);
 private:
  char* base_ = nullptr;
  size_t cap_ = 0, used_ = 0;
};

// Block-sparse MPS (Section 2.3).  Site k (1-based) stores, for each left sector n in
// K_{k-1} (ascending), the column-major matrix [U_{k,n} | O_{k,n}] with rho[k-1][n]
// rows.  This is also the export layout.
struct Mps {
  int L = 0, N = 0;
  std::vector<std::vector<int>> rho;          // [L+1][N+1]
  std::vector<Buf> site;                      // site[k-1]
  std::vector<std::vector<int64_t>> off;      // off[k-1][n]: start of [U|O] for sector n
  bool valid(int k, int n) const { return n >= 0 && n <= N && n >= N - L + k && n <= k; }
  int rows(int k, int n) const { return valid(k - 1, n) ? rho[k - 1][n] : 0; }
  int ucols(int k, int n) const { return valid(k - 1, n) && valid(k, n) ? rho[k][n] : 0; }
  int ocols(int k, int n) const { return valid(k - 1, n) && valid(k, n + 1) ? rho[k][n + 1] : 0; }
  double* U(int k, int n) const { return site[k - 1].p + off[k - 1][n]; }
  double* O(int k, int n) const { return U(k, n) + int64_t(rows(k, n)) * ucols(k, n); }
  int64_t site_size(int k) const;
  int64_t size() const;
  int max_rank() const;
};

// Device copy of an operator in the bond-charge blocked form of mpo.hpp.
struct DevMpo {
  int L = 0;
  std::vector<int> w;
  std::vector<std::array<int, 6>> qoff;
  // Dense charge block W^{s_out s_in}[b in q_in, b' in q_out] (w_in x w_out, column
  // major), applied by GEMM; its entries are removed from the sparse CSR.
  struct Dense {
    int q_in, q_out, s_in, s_out, w_in, w_out;
    Buf W;
  };
  // Sparse part (entries not in a dense block) as CSR over rows s_out * w_out + b_out,
  // kept on the host: the W-step resolves it into source pointers per launch.
  struct Site {
    std::vector<int32_t> row_ptr, b_in;
    std::vector<uint8_t> s_in;
    std::vector<double> val;
    int w_out = 0;
    std::vector<Dense> dense;
  };
  std::vector<Site> site;
  std::vector<std::vector<int8_t>> charge;  // charge of every state, per cut
  int64_t nnz = 0;
};

enum TimerClass { T_GEMM = 0, T_EIG, T_WSTEP, T_COPY, T_REDUCE, T_TRI, T_CHOL, T_GEMM32, T_TRIVEC, T_TRIBACK, T_TRIVAL, T_TRIGEMM, T_GEMMBF16, T_TRITAIL, T_COUNT };

struct Ctx {
  int device = 0;
  hipStream_t stream = nullptr;
  bool own_stream = true;  // false when the caller passed its stream to pv_create
  Pool pool;
  Staging staging;
  // problem
  int L = 0, N = 0;
  double gamma = 0.0;
  std::vector<double> h, v;
  std::unique_ptr<DevMpo> hmpo;
  std::unique_ptr<DevMpo> ident;  // identity operator (dot products)
  // precision of the contractions: 0 float64; 1 float32 MFMA, 2 bfloat16 operands on MFMA
  // with float32 accumulation, for the operator contractions (H psi and the Ritz
  // sandwiches) while truncations, norms and the Rayleigh quotient stay float64.  lowp is
  // set while such a contraction runs.
  int prec = 0;
  bool lowp = false;
  // GEMM kernel precision of an operator contraction (see launch_gemm)
  int contraction_kernel() const { return lowp ? (prec == 2 ? 3 : 1) : 0; }
  std::vector<int> mpo_w;
  // preconditioner (Section 4.3, Section 7.1.1)
  std::vector<double> theta;
  std::vector<double> corr;  // learned correction of theta, L x (N+1) row-major; empty: none
  // network parameters (float32) attached for the runs, and the refresh period of the
  // correction (iterations); empty: none
  std::vector<float> net;
  int net_refresh = 0;
  // per-step judge of a corrected S: each iteration of pv_run also forms the direction
  // with the plain S and takes the one with the lower Ritz value; steps won by each
  bool judge = false;
  int judge_plain = 0, judge_corr = 0;
  double t_min = 0, t_max = 0, T_ratio = 0, hs = 0, a0 = 0, s_min = 0, s_max = 0;
  int m_minus = 0, m_plus = 0;
  std::vector<double> alpha, beta;
  // MPS handles
  std::map<int, std::unique_ptr<Mps>> mps;
  int next_handle = 1;
  // timers
  // weight: launches the timed one stands for (sampled timing of short repeated launches)
  struct Pending { int cls; hipEvent_t a, b; double flops, bytes; int weight; };
  std::vector<Pending> pending;
  std::vector<hipEvent_t> event_pool;
  double t_ms[T_COUNT] = {0}, t_flops[T_COUNT] = {0}, t_bytes[T_COUNT] = {0};
  int t_calls[T_COUNT] = {0};
  // kernel classes timed with HIP events (bit c: class c); an untimed launch records no event
  uint32_t timer_mask = ~0u;
  // classes timed on a pseudo-random one-in-sample_every subset of their launches, each
  // timed launch standing for sample_every (selection by a hash of the launch's index)
  uint32_t sample_mask = 0;
  int sample_every = 1;
  uint64_t sample_count[32] = {0};
  // 0: sequential TT-SVD truncation with two-pass Gram factorisations (exact path);
  // 1: simultaneous Gram truncation of all bonds, single-pass factorisations in the
  //    intermediate-rank H application.
  int trunc_mode = 0;
  // float64 GEMM tile shape (PV_GEMM_TILES_*): the fixed rule by launch size, the online
  // autotuner, its table without exploration, or one shape forced
  int gemm_tiles = 0;
  // launches of the autotuner's exploration whose events are read at the next sync
  struct TunePending { int prec, bt, bk, cand; hipEvent_t a, b; double flops; bool owns; };
  std::vector<TunePending> tune_pending;
  // eigensolver batches of at most this many tridiagonal problems are reduced one step per
  // launch on several workgroups per problem; larger ones by one-workgroup panels
  int tri_step_max = PV_TRIDIAG_STEPS_DEFAULT;

  // side stream for an independent chain of launches: fork() orders it behind the main
  // stream's work so far and redirects `stream` to it; unfork() restores the main stream;
  // join() orders the main stream behind the side stream's work
  hipStream_t main_stream = nullptr, side_stream = nullptr;
  bool use_side = true;  // off while many contexts share the device (pv_run_batch)
  hipEvent_t fork_event = nullptr, join_event = nullptr;
  void fork();
  void unfork();
  void join();

  // auxiliary context on a stream of its own, for a sweep that runs beside the main
  // stream's work (expect_h_begin / expect_h_end); created on first use
  std::unique_ptr<Ctx> aux;
  hipEvent_t aux_ready = nullptr;
  double* aux_host = nullptr;  // pinned host copy of the overlapped sweep's result
  size_t aux_host_n = 0, aux_n = 0;
  bool aux_pending = false, aux_inline = false;
  int aux_da = 0, aux_db = 0;
  double aux_value = 0.0;
  // pinned host buffer of download()
  double* dl_host = nullptr;
  size_t dl_n = 0;

  void sync();
  hipEvent_t event();
  void begin(int cls, hipEvent_t& a);
  void end(int cls, hipEvent_t a, double flops, double bytes, int weight = 1);
  // the same for a launch that records its own start and stop times (an extended launch
  // given the two events): begin_ext hands out the events (nulls when the launch is not
  // timed), end_ext files them; no marker packet goes on the stream
  void begin_ext(int cls, hipEvent_t& a, hipEvent_t& b);
  void end_ext(int cls, hipEvent_t a, hipEvent_t b, double flops, double bytes, int weight = 1);
  template <class T>
  T* upload(const std::vector<T>& v);  // staged async copy into a pool buffer kept in `scratch`
  // two arrays in one copy (each copy costs a command and a gap on the stream)
  template <class T, class U>
  std::pair<T*, U*> upload2(const std::vector<T>& a, const std::vector<U>& b);
  std::vector<Buf> scratch;            // freed at sync
};

// ---- GEMM tile autotuner (engine.cpp): one table per process, shared by every context ----
// rows of 9 values: device, kernel precision, log2 bucket of the launch's 64 x 64 tiles,
// log2 bucket of its longest K, choice (-1 undecided, 0: 64 x 64, 1: 32 x 32), samples of
// each shape, and each shape's measured rate in TFLOP/s
std::vector<double> gemm_tune_rows();
void gemm_tune_clear();
// n rows in the layout of gemm_tune_rows, validated, replacing the entries of their keys
void gemm_tune_load(const double* rows, int n);

// ---- operations (engine.cpp) ----
std::unique_ptr<Mps> mps_alloc(Ctx& c, int L, int N, const std::vector<std::vector<int>>& rho);
std::unique_ptr<Mps> mps_determinant(Ctx& c, const std::vector<int>& occ);
std::unique_ptr<Mps> mps_lincomb(Ctx& c, double a, const Mps& x, double b, const Mps& y, bool index_concat = false);
// Joint MPS (several columns): the right boundary rho[L][N] = D is the column index
// (Section 6.2, the index core after orbital L).  dot and expect_h return the traces over
// the columns; the matrices of all column pairs (D_a x D_b, column-major):
std::vector<double> dot_matrix(Ctx& c, const Mps& a, const Mps& b);
std::vector<double> expect_matrix(Ctx& c, const Mps& bra, const Mps& ket);
// column j of the result = sum_i W[i + Din j] (column i of x)
std::unique_ptr<Mps> mps_index_transform(Ctx& c, const Mps& x, const std::vector<double>& W, int Dout);
std::unique_ptr<Mps> mps_scaled_copy(Ctx& c, const Mps& x, double a, const double* occ_scale);
std::unique_ptr<Mps> mps_zero_like(Ctx& c, const Mps& x);
std::unique_ptr<Mps> mps_sector_scaled_copy(Ctx& c, const Mps& x, double a, const double* occ);
std::vector<double> densities(Ctx& c, const Mps& x);
// learned correction of theta (th: theta_i, L values; hd: h_ii; lam: Rayleigh quotient of x)
void learned_correction(Ctx& c, const float* params, const Mps& x, double lam, const std::vector<double>& th,
                        double* delta);
// rvals/tvals (nmask each, host, may be null): train on the solve form of the misfit (the
// method's residual and its exact solve at the samples) instead of the exact diagonal.
void learned_train(Ctx& c, float* params, const Mps& x, double lam, const std::vector<double>& th,
                   const uint64_t* masks, int nmask, int steps, float lr, double* loss, double* grad,
                   const double* rvals = nullptr, const double* tvals = nullptr);
// x = H_gamma^{-1} b by preconditioned conjugate gradients in block-sparse form (exact
// products and sums up to numerical zeros).
std::unique_ptr<Mps> solve_h(Ctx& c, const Mps& b, double rel_tol, int max_iter, int* iters, double* rel_res);
// amplitudes <det_b|x> for determinants given as bit masks
void amplitudes(Ctx& c, const Mps& x, const uint64_t* masks, int n, double* out);
std::vector<double> env_sweep(Ctx& c, const Mps& bra, const Mps& ket, const DevMpo& op);
double dot(Ctx& c, const Mps& a, const Mps& b);
double expect_h(Ctx& c, const Mps& bra, const Mps& ket);
// <bra|H|ket> started on the auxiliary stream behind the main stream's work so far (in
// place when use_side is off) and collected by expect_h_end; bra and ket stay alive and
// unmodified until then.  expect_h_drain waits for and drops a started sweep;
// release_aux frees the auxiliary context and the pinned host buffers.
void expect_h_begin(Ctx& c, const Mps& bra, const Mps& ket);
double expect_h_end(Ctx& c);
void expect_h_drain(Ctx& c) noexcept;
void release_aux(Ctx& c) noexcept;
std::unique_ptr<Mps> round_mps(Ctx& c, const Mps& x, double eps, int cap, bool* cap_bound);
// trunc(H x; eps, cap) with intermediate rank m_zip; *zip_disc2 (may be null) is
// incremented by the sum of the squared singular values that m_zip dropped in the panels
// (in their own metric), and *cap_bound is set when that sum is positive.
std::unique_ptr<Mps> apply_h(Ctx& c, const Mps& x, double eps, int cap, int m_zip, bool* cap_bound,
                             double* zip_disc2 = nullptr);
std::unique_ptr<Mps> apply_s(Ctx& c, const Mps& x, double eta, int cap, bool* cap_bound);
std::unique_ptr<DevMpo> upload_mpo(Ctx& c, const Mpo& m);
double norm_canonical(Ctx& c, const Mps& x);
std::unique_ptr<Mps> round_parallel(Ctx& c, const Mps& x, double eps, int cap, bool* cap_bound);
double norm2(Ctx& c, const Mps& x);
void sym_eig(Ctx& c, int n, const double* A_host, double* w_host, double* V_host, int method, int nvec = -1);
void gemm_host(Ctx& c, int M, int N, int K, const double* A_host, int lda, int ta, const double* B_host, int ldb,
               int tb, double* C_host, int ldc, double alpha, double beta, int precision);
void cholesky(Ctx& c, int n, const double* A_host, double* W_host);
// Tridiagonal solver launches shared by the batched eigenproblems and the single-problem
// paths: reduction and eigenvalues, then the d[i].nvec leading eigenvectors.
void tri_values(Ctx& c, const std::vector<EigDesc>& tri, const EigDesc* d, int ntri, double ftri, double btri);
void tri_vectors(Ctx& c, const std::vector<EigDesc>& tri, const EigDesc* d, int ntri);
// All eigenpairs of the n x n matrix A (device, column-major, upper triangle read) by the
// tridiagonal solver into w, V (device), with the caller's work area (tri_work_doubles(n)
// doubles) and descriptor slot (device); allocates nothing; synchronous.
void sym_eig_tridiag_device(Ctx& c, int n, const double* A, double* w, double* V, double* work, EigDesc* desc);
// Device address of the file-scope work array of the allocation-free eigensolver entry
// point on `device` (looked up once per device; called by pv_create).
double* noalloc_scratch(int device);
// pv_sym_eig_noalloc: the tridiagonal solver on device buffers with its work area in that
// array (n <= PV_NOALLOC_MAX_N, PV_EINVAL beyond).
void sym_eig_noalloc(Ctx& c, int n, const double* A, double* w, double* V);

}  // namespace pv
