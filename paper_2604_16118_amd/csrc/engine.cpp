// Runtime pieces (pool, staging, timers) and the block-sparse MPS operations.
#include "engine.hpp"
#include "learned.hpp"

#include <algorithm>
#include <cmath>
#include <cstring>
#include <functional>
#include <mutex>
#include <numeric>
#include <tuple>

namespace pv {

// ---------------------------------------------------------------- pool
static size_t size_class(size_t bytes) {
  if (bytes <= 4096) return 4096;
  size_t p = 1;
  while ((p << 1) <= bytes) p <<= 1;
  const size_t step = std::max<size_t>(p / 8, 256);
  return (bytes + step - 1) / step * step;
}

Pool::~Pool() { release(); }

void* Pool::get(size_t bytes) {
  const size_t cls = size_class(bytes);
  auto it = free_.find(cls);
  if (it != free_.end()) {
    void* p = it->second;
    free_.erase(it);
    cached_ -= cls;
    in_use_ += cls;
    return p;
  }
  void* p = nullptr;
  hipError_t e = hipMalloc(&p, cls);
  if (e != hipSuccess) {
    (void)hipGetLastError();
    release();
    e = hipMalloc(&p, cls);
    if (e != hipSuccess) {
      (void)hipGetLastError();
      fail(PV_ENOMEM, "hipMalloc of " + std::to_string(cls) + " bytes failed");
    }
  }
  in_use_ += cls;
  return p;
}

void Pool::put(void* p, size_t bytes) {
  if (!p) return;
  const size_t cls = size_class(bytes);
  in_use_ -= cls;
  cached_ += cls;
  if (holding_) held_.emplace_back(cls, p);
  else free_.emplace(cls, p);
}

void Pool::hold(bool on) {
  holding_ = on;
  if (on) return;
  for (auto& kv : held_) free_.emplace(kv.first, kv.second);
  held_.clear();
}

void Pool::release() {
  for (auto& kv : free_) (void)hipFree(kv.second);
  for (auto& kv : held_) (void)hipFree(kv.second);
  free_.clear();
  held_.clear();
  cached_ = 0;
}

Buf::Buf(Pool& pl, size_t count) : pool(&pl), n(count) {
  p = count ? static_cast<double*>(pl.get(count * sizeof(double))) : nullptr;
}

Buf& Buf::operator=(Buf&& o) noexcept {
  if (this != &o) {
    reset();
    pool = o.pool; p = o.p; n = o.n;
    o.p = nullptr; o.n = 0;
  }
  return *this;
}

void Buf::reset() {
  if (p && pool) pool->put(p, n * sizeof(double));
  p = nullptr;
  n = 0;
}

// ---------------------------------------------------------------- staging
void Staging::init(size_t cap) {
  void* p = nullptr;
  PV_HIP(hipHostMalloc(&p, cap, hipHostMallocDefault));
  base_ = static_cast<char*>(p);
  cap_ = cap;
  used_ = 0;
}
Staging::~Staging() {
  if (base_) (void)hipHostFree(base_);
}
void* Staging::put(const void* src, size_t bytes) {
  const size_t need = (bytes + 255) & ~size_t(255);
  if (used_ + need > cap_) fail(PV_ENOMEM, "staging area exhausted");
  void* dst = base_ + used_;
  std::memcpy(dst, src, bytes);
  used_ += need;
  return dst;
}

// ---------------------------------------------------------------- ctx
hipEvent_t Ctx::event() {
  if (!event_pool.empty()) {
    hipEvent_t e = event_pool.back();
    event_pool.pop_back();
    return e;
  }
  hipEvent_t e;
  PV_HIP(hipEventCreate(&e));
  return e;
}

// whether this launch of class cls is timed (the class's mask bit, then the sample)
static bool timed_launch(Ctx& c, int cls) {
  if (!((c.timer_mask >> cls) & 1u)) return false;
  if ((c.sample_mask >> cls) & 1u) {
    // splitmix64 of the launch index: no period that a regular launch pattern could alias
    uint64_t x = c.sample_count[cls]++ + 0x9E3779B97F4A7C15ull;
    x = (x ^ (x >> 30)) * 0xBF58476D1CE4E5B9ull;
    x = (x ^ (x >> 27)) * 0x94D049BB133111EBull;
    x ^= x >> 31;
    if (x % uint64_t(c.sample_every) != 0) return false;
  }
  return true;
}

void Ctx::begin(int cls, hipEvent_t& a) {
  if (!timed_launch(*this, cls)) { a = nullptr; return; }
  a = event();
  PV_HIP(hipEventRecord(a, stream));
}

void Ctx::begin_ext(int cls, hipEvent_t& a, hipEvent_t& b) {
  a = b = nullptr;
  if (!timed_launch(*this, cls)) return;
  a = event();
  b = event();
}

void Ctx::end_ext(int cls, hipEvent_t a, hipEvent_t b, double flops, double bytes, int weight) {
  if (!a || !b) return;
  if ((sample_mask >> cls) & 1u) weight *= sample_every;
  pending.push_back({cls, a, b, flops, bytes, weight});
}

void Ctx::end(int cls, hipEvent_t a, double flops, double bytes, int weight) {
  if (!a) return;
  hipEvent_t b = event();
  PV_HIP(hipEventRecord(b, stream));
  if ((sample_mask >> cls) & 1u) weight *= sample_every;
  pending.push_back({cls, a, b, flops, bytes, weight});
}

void Ctx::fork() {
  if (!side_stream) {
    PV_HIP(hipStreamCreate(&side_stream));
    PV_HIP(hipEventCreateWithFlags(&fork_event, hipEventDisableTiming));
    PV_HIP(hipEventCreateWithFlags(&join_event, hipEventDisableTiming));
  }
  main_stream = stream;
  PV_HIP(hipEventRecord(fork_event, main_stream));
  PV_HIP(hipStreamWaitEvent(side_stream, fork_event, 0));
  pool.hold(true);
  stream = side_stream;
}

void Ctx::unfork() { stream = main_stream; }

void Ctx::join() {
  stream = main_stream;
  PV_HIP(hipEventRecord(join_event, side_stream));
  PV_HIP(hipStreamWaitEvent(main_stream, join_event, 0));
  pool.hold(false);
}

// ---------------------------------------------------------------- GEMM tile autotuner
// The two float64 tile shapes (64 x 64 and 32 x 32) run the same chain of MFMA products
// for every element of C (the same K-tiles and k-steps in the same order, the same split
// of K), so the shape changes a launch's time and never a bit of its result.  A launch is
// keyed by (device, kernel precision, floor(log2) of its count of 64 x 64 tiles including
// split-K parts, floor(log2) of its longest K range).  In the online mode the first
// 2 kTuneSamples launches of a key alternate the two shapes, each timed by the launch's own
// start and stop events; once both shapes have kTuneSamples samples, the key takes the
// shape with the smaller time per flop (the launches of one key differ in size).  Until
// then, and for keys never seen, the fixed rule decides.  The table lives for the process
// and is shared by every context (guarded by a mutex: batched runs tune from many host
// threads).
namespace {
struct TuneKey {
  int dev, prec, bt, bk;
  bool operator<(const TuneKey& o) const {
    return std::tie(dev, prec, bt, bk) < std::tie(o.dev, o.prec, o.bt, o.bk);
  }
};
struct TuneEntry {
  double ms[2] = {0, 0}, flops[2] = {0, 0};
  int n[2] = {0, 0};
  int issued = 0;
  int choice = -1;
};
constexpr int kTuneSamples = 4;
std::mutex g_tune_mu;
std::map<TuneKey, TuneEntry> g_tune;

int floor_log2(int64_t x) {
  int b = 0;
  while (x > 1) { x >>= 1; ++b; }
  return b;
}

// the tile shape of a float64 launch (true: 32 x 32); cand receives the shape an
// exploration launch times (-1: none)
bool gemm_tiles_choice(Ctx& c, int prec, int64_t tiles64, int kmax, int& cand, int& bt, int& bk) {
  cand = -1;
  const bool rule = tiles64 <= kGemmSmallTiles;
  switch (c.gemm_tiles) {
    case PV_GEMM_TILES_SMALL: return true;
    case PV_GEMM_TILES_LARGE: return false;
    case PV_GEMM_TILES_TUNE:
    case PV_GEMM_TILES_TABLE: break;
    default: return rule;
  }
  bt = floor_log2(std::max<int64_t>(tiles64, 1));
  bk = floor_log2(std::max(kmax, 1));
  std::lock_guard<std::mutex> lk(g_tune_mu);
  const TuneKey key{c.device, prec, bt, bk};
  if (c.gemm_tiles == PV_GEMM_TILES_TABLE) {
    auto it = g_tune.find(key);
    return it != g_tune.end() && it->second.choice >= 0 ? it->second.choice == 1 : rule;
  }
  TuneEntry& e = g_tune[key];
  if (e.choice >= 0) return e.choice == 1;
  if (e.issued >= 2 * kTuneSamples) return rule;  // samples still in flight
  cand = e.issued++ & 1;
  return cand == 1;
}

}  // namespace

std::vector<double> gemm_tune_rows() {
  std::lock_guard<std::mutex> lk(g_tune_mu);
  std::vector<double> rows;
  for (const auto& [k, e] : g_tune) {
    const double r0 = e.ms[0] > 0 ? e.flops[0] / (e.ms[0] * 1e9) : 0.0;
    const double r1 = e.ms[1] > 0 ? e.flops[1] / (e.ms[1] * 1e9) : 0.0;
    const double row[9] = {double(k.dev), double(k.prec), double(k.bt), double(k.bk), double(e.choice),
                           double(e.n[0]), double(e.n[1]), r0, r1};
    rows.insert(rows.end(), row, row + 9);
  }
  return rows;
}

void gemm_tune_clear() {
  std::lock_guard<std::mutex> lk(g_tune_mu);
  g_tune.clear();
}

void gemm_tune_load(const double* rows, int n) {
  // validate every row before changing the table
  for (int i = 0; i < n; ++i) {
    const double* r = rows + size_t(9) * i;
    for (int j = 0; j < 9; ++j)
      if (!std::isfinite(r[j])) fail(PV_EINVAL, "tuner row " + std::to_string(i) + " is not finite");
    const bool ints = r[0] == std::floor(r[0]) && r[1] == std::floor(r[1]) && r[2] == std::floor(r[2]) &&
                      r[3] == std::floor(r[3]) && r[4] == std::floor(r[4]) && r[5] == std::floor(r[5]) &&
                      r[6] == std::floor(r[6]);
    if (!ints || r[0] < 0 || r[0] > 63 || (r[1] != 0 && r[1] != 2) || r[2] < 0 || r[2] > 62 || r[3] < 0 ||
        r[3] > 30 || r[4] < -1 || r[4] > 1 || r[5] < 0 || r[6] < 0 || r[5] > 1e9 || r[6] > 1e9 || r[7] < 0 ||
        r[8] < 0)
      fail(PV_EINVAL, "tuner row " + std::to_string(i) + " out of range");
  }
  std::lock_guard<std::mutex> lk(g_tune_mu);
  for (int i = 0; i < n; ++i) {
    const double* r = rows + size_t(9) * i;
    TuneEntry e;
    e.choice = int(r[4]);
    e.n[0] = int(r[5]);
    e.n[1] = int(r[6]);
    // an undecided key explores again from the start (both shapes get their samples)
    e.issued = e.choice >= 0 ? e.n[0] + e.n[1] : 0;
    // one millisecond per shape at the stored rate (the table keeps rates, not times)
    for (int j = 0; j < 2; ++j) {
      e.ms[j] = r[7 + j] > 0 ? 1.0 : 0.0;
      e.flops[j] = r[7 + j] * 1e9;
    }
    g_tune[TuneKey{int(r[0]), int(r[1]), int(r[2]), int(r[3])}] = e;
  }
}

void Ctx::sync() {
  if (side_stream) PV_HIP(hipStreamSynchronize(side_stream));
  if (main_stream && main_stream != stream) PV_HIP(hipStreamSynchronize(main_stream));
  PV_HIP(hipStreamSynchronize(stream));
  // the autotuner's samples first: their events may also be a timer's, which the timer
  // loop below returns to the pool
  for (auto& p : tune_pending) {
    float ms = 0.f;
    PV_HIP(hipEventElapsedTime(&ms, p.a, p.b));
    {
      std::lock_guard<std::mutex> lk(g_tune_mu);
      TuneEntry& e = g_tune[TuneKey{device, p.prec, p.bt, p.bk}];
      e.ms[p.cand] += double(ms);
      e.flops[p.cand] += p.flops;
      e.n[p.cand] += 1;
      if (e.choice < 0 && e.n[0] >= kTuneSamples && e.n[1] >= kTuneSamples)
        e.choice = e.ms[1] * e.flops[0] < e.ms[0] * e.flops[1] ? 1 : 0;
    }
    if (p.owns) {
      event_pool.push_back(p.a);
      event_pool.push_back(p.b);
    }
  }
  tune_pending.clear();
  for (auto& p : pending) {
    float ms = 0.f;
    PV_HIP(hipEventElapsedTime(&ms, p.a, p.b));
    t_ms[p.cls] += double(ms) * p.weight;
    t_flops[p.cls] += p.flops * p.weight;
    t_bytes[p.cls] += p.bytes * p.weight;
    t_calls[p.cls] += p.weight;
    event_pool.push_back(p.a);
    event_pool.push_back(p.b);
  }
  pending.clear();
  scratch.clear();
  staging.reset();
}

template <class T>
T* Ctx::upload(const std::vector<T>& v) {
  if (v.empty()) return nullptr;
  const size_t bytes = v.size() * sizeof(T);
  if (!staging.fits(bytes)) sync();
  void* host = staging.put(v.data(), bytes);
  Buf b(pool, (bytes + sizeof(double) - 1) / sizeof(double));
  PV_HIP(hipMemcpyAsync(b.p, host, bytes, hipMemcpyHostToDevice, stream));
  T* out = reinterpret_cast<T*>(b.p);
  scratch.push_back(std::move(b));
  return out;
}
template GemmDesc* Ctx::upload(const std::vector<GemmDesc>&);
template int* Ctx::upload(const std::vector<int>&);

template <class T, class U>
std::pair<T*, U*> Ctx::upload2(const std::vector<T>& a, const std::vector<U>& b) {
  if (a.empty() || b.empty()) return {upload(a), upload(b)};
  const size_t ba = a.size() * sizeof(T), bb = b.size() * sizeof(U);
  // the staging area places each array at a 256-byte boundary, one after the other
  if (!staging.fits(ba + bb + 256)) sync();
  char* ha = static_cast<char*>(staging.put(a.data(), ba));
  char* hb = static_cast<char*>(staging.put(b.data(), bb));
  const size_t off = size_t(hb - ha), bytes = off + bb;
  Buf buf(pool, (bytes + sizeof(double) - 1) / sizeof(double));
  PV_HIP(hipMemcpyAsync(buf.p, ha, bytes, hipMemcpyHostToDevice, stream));
  char* d = reinterpret_cast<char*>(buf.p);
  scratch.push_back(std::move(buf));
  return {reinterpret_cast<T*>(d), reinterpret_cast<U*>(d + off)};
}

static Buf scratch_buf(Ctx& c, size_t n) {
  return Buf(c.pool, n);
}

// ---------------------------------------------------------------- MPS basics
int64_t Mps::site_size(int k) const {
  int64_t s = 0;
  for (int n = 0; n <= N; ++n)
    if (valid(k - 1, n)) s += int64_t(rows(k, n)) * (ucols(k, n) + ocols(k, n));
  return s;
}
int64_t Mps::size() const {
  int64_t s = 0;
  for (int k = 1; k <= L; ++k) s += site_size(k);
  return s;
}
int Mps::max_rank() const {
  int r = 0;
  for (int k = 0; k <= L; ++k) {
    int t = 0;
    for (int n = 0; n <= N; ++n) t += valid(k, n) ? rho[k][n] : 0;
    r = std::max(r, t);
  }
  return r;
}

static void layout_site(Mps& m, int k) {
  m.off[k - 1].assign(m.N + 1, 0);
  int64_t o = 0;
  for (int n = 0; n <= m.N; ++n) {
    m.off[k - 1][n] = o;
    if (m.valid(k - 1, n)) o += int64_t(m.rows(k, n)) * (m.ucols(k, n) + m.ocols(k, n));
  }
}

static void alloc_site(Ctx& c, Mps& m, int k) {
  layout_site(m, k);
  m.site[k - 1] = Buf(c.pool, size_t(std::max<int64_t>(m.site_size(k), 1)));
}

std::unique_ptr<Mps> mps_alloc(Ctx& c, int L, int N, const std::vector<std::vector<int>>& rho) {
  auto m = std::make_unique<Mps>();
  m->L = L;
  m->N = N;
  m->rho = rho;
  m->site.resize(L);
  m->off.resize(L);
  for (int k = 1; k <= L; ++k) alloc_site(c, *m, k);
  return m;
}

static std::vector<std::vector<int>> empty_rho(int L, int N) {
  return std::vector<std::vector<int>>(L + 1, std::vector<int>(N + 1, 0));
}

// ---------------------------------------------------------------- batched launches
namespace {

// events for an exploration launch of the tile autotuner that the timers did not time
// (true: the tuner owns them and returns them to the pool)
bool tune_events(Ctx& c, int cand, hipEvent_t& a, hipEvent_t& b) {
  if (cand < 0 || a) return false;
  a = c.event();
  b = c.event();
  return true;
}

struct GemmBatch {
  std::vector<GemmDesc> d;
  int prec = 0;  // 1: float32 MFMA (operator contractions in the mixed-precision mode)
  int cls = -1;  // timer class (default: by precision)
  void add(const double* A, int lda, int ta, const double* B, int ldb, int tb, double* C, int ldc,
           int M, int N, int K, double alpha, double beta) {
    if (M <= 0 || N <= 0) return;
    GemmDesc g{};
    g.A = A; g.B = B; g.C = C;
    g.M = M; g.N = N; g.K = K;
    g.lda = std::max(lda, 1); g.ldb = std::max(ldb, 1); g.ldc = std::max(ldc, 1);
    g.ta = ta; g.tb = tb; g.alpha = alpha; g.beta = beta;
    d.push_back(g);
  }
  // C_s = alpha A_s op(B) + beta C_s for s = 0 .. nouter - 1, A_s = A + s a_outer (m1 x K,
  // ld lda), C_s = C + s c_outer (m1 x N, ld ldc): one product whose rows are (r, s).  The
  // bfloat16 kernel has no such rows: it gets one problem per s.
  void add_rows2(const double* A, int lda, int64_t a_outer, const double* B, int ldb, int tb, double* C, int ldc,
                 int64_t c_outer, int m1, int nouter, int N, int K, double alpha, double beta) {
    if (m1 <= 0 || nouter <= 0 || N <= 0) return;
    if (prec == 3 || nouter == 1 || int64_t(m1) * nouter > INT32_MAX / 2) {
      for (int s = 0; s < nouter; ++s) add(A + s * a_outer, lda, 0, B, ldb, tb, C + s * c_outer, ldc, m1, N, K, alpha, beta);
      return;
    }
    add(A, lda, 0, B, ldb, tb, C, ldc, m1 * nouter, N, K, alpha, beta);
    GemmDesc& g = d.back();
    g.m1 = m1;
    g.a_outer = a_outer;
    g.c_outer = c_outer;
  }
  bool empty() const { return d.empty(); }
  void run(Ctx& c) {
    if (d.empty()) return;
    std::vector<GemmDesc> list;
    std::vector<ReduceDesc> red;
    std::vector<CopyDesc> zero_k;
    int64_t tiles = 0, red_elems = 0, zk_elems = 0;
    double red_bytes = 0;  // the S partials read, C read when beta != 0, C written
    double flops = 0, bytes = 0;
    // split-K choice on 64 x 64 tiles
    auto split_of = [](const GemmDesc& g0) {
      const int tm = (g0.M + kGemmBM - 1) / kGemmBM, tn = (g0.N + kGemmBN - 1) / kGemmBN;
      int S = 1;
      if (tm * tn < 128 && g0.K >= 1024 && g0.m1 == 0) {
        S = std::min((g0.K + 511) / 512, (256 + tm * tn - 1) / (tm * tn));
        S = std::max(S, 1);
      }
      return S;
    };
    // a float64 launch of few 64 x 64 tiles takes the small tiles
    int64_t tiles64 = 0;
    for (const GemmDesc& g0 : d)
      if (g0.K > 0)
        tiles64 += int64_t((g0.M + kGemmBM - 1) / kGemmBM) * ((g0.N + kGemmBN - 1) / kGemmBN) * split_of(g0);
    int kmax = 0;
    for (const GemmDesc& g0 : d) kmax = std::max(kmax, g0.K / split_of(g0));
    int cand = -1, bt = 0, bk = 0;
    // (a batch of K = 0 products only launches no GEMM and takes no tuning sample)
    const bool small = (prec == 0 || prec == 2) && tiles64 > 0 && gemm_tiles_choice(c, prec, tiles64, kmax, cand, bt, bk);
    const int TM = small ? kGemmSmall : kGemmBM, TN = small ? kGemmSmall : kGemmBN;
    for (const GemmDesc& g0 : d) {
      if (g0.K <= 0) {  // C = beta C (beta 0: C cleared without reading it)
        CopyDesc cd{g0.beta != 0.0 ? g0.C : nullptr, g0.C, g0.M, g0.N, g0.ldc, g0.ldc, g0.beta, zk_elems};
        zero_k.push_back(cd);
        zk_elems += int64_t(g0.M) * g0.N;
        continue;
      }
      flops += 2.0 * g0.M * g0.N * double(g0.K);
      bytes += 8.0 * (double(g0.M) * g0.K + double(g0.K) * g0.N + double(g0.M) * g0.N * (g0.beta != 0 ? 2 : 1));
      const int tm = (g0.M + TM - 1) / TM, tn = (g0.N + TN - 1) / TN;
      int S = split_of(g0);
      if (S == 1) {
        GemmDesc g = g0;
        g.tile0 = int(tiles); g.tiles_n = tn; g.kbeg = 0; g.kend = g.K;
        // the operand along the longer tile dimension is the big one: keep the tiles that
        // share one of its blocks next to each other
        g.tiles_m = tm; g.colmajor = tm < tn;
        list.push_back(g);
        tiles += int64_t(tm) * tn;
      } else {
        const int chunk = ((g0.K + S - 1) / S + kGemmBK - 1) / kGemmBK * kGemmBK;
        S = (g0.K + chunk - 1) / chunk;
        Buf part = scratch_buf(c, size_t(g0.M) * g0.N * S);
        for (int s = 0; s < S; ++s) {
          GemmDesc g = g0;
          g.C = part.p + size_t(s) * g0.M * g0.N;
          g.ldc = g0.M; g.alpha = 1.0; g.beta = 0.0;
          g.kbeg = s * chunk; g.kend = std::min(g0.K, (s + 1) * chunk);
          g.tile0 = int(tiles); g.tiles_n = tn; g.tiles_m = tm; g.colmajor = 0;
          list.push_back(g);
          tiles += int64_t(tm) * tn;
        }
        red.push_back(ReduceDesc{g0.C, part.p, g0.M, g0.N, g0.ldc, S, g0.alpha, g0.beta, red_elems});
        red_elems += int64_t(g0.M) * g0.N;
        red_bytes += 8.0 * double(g0.M) * g0.N * (S + 1 + (g0.beta != 0.0 ? 1 : 0));
        c.scratch.push_back(std::move(part));
      }
    }
    if (!zero_k.empty()) {
      CopyDesc* dz = c.upload(zero_k);
      hipEvent_t a; c.begin(T_COPY, a);
      launch_copy(dz, int(zero_k.size()), zk_elems, c.stream);
      c.end(T_COPY, a, 0, 16.0 * zk_elems);
    }
    if (!list.empty()) {
      if (tiles > INT32_MAX) fail(PV_EINVAL, "GEMM batch too large for one launch");
      const int tc = cls >= 0 ? cls : (prec == 3 ? T_GEMMBF16 : prec ? T_GEMM32 : T_GEMM);
      if (list.size() <= size_t(kGemmPack)) {  // descriptors in the kernel arguments
        GemmPack pack{};
        std::copy(list.begin(), list.end(), pack.d);
        hipEvent_t a, b;
        c.begin_ext(tc, a, b);
        const bool owns = tune_events(c, cand, a, b);
        launch_gemm_packed(pack, int(list.size()), int(tiles), prec, c.stream, small, a, b);
        if (cand >= 0) c.tune_pending.push_back({prec, bt, bk, cand, a, b, flops, owns});
        if (!owns) c.end_ext(tc, a, b, flops, bytes);
      } else {
        std::vector<int> tmap(static_cast<size_t>(tiles));
        for (size_t i = 0; i < list.size(); ++i) {
          const GemmDesc& g = list[i];
          const int64_t nt = int64_t((g.M + TM - 1) / TM) * ((g.N + TN - 1) / TN);
          std::fill(tmap.begin() + g.tile0, tmap.begin() + g.tile0 + nt, int(i));
        }
        auto [dd, dm] = c.upload2(list, tmap);
        hipEvent_t a, b;
        c.begin_ext(tc, a, b);
        const bool owns = tune_events(c, cand, a, b);
        launch_gemm(dd, dm, int(tiles), prec, c.stream, small, a, b);
        if (cand >= 0) c.tune_pending.push_back({prec, bt, bk, cand, a, b, flops, owns});
        if (!owns) c.end_ext(tc, a, b, flops, bytes);
      }
    }
    if (!red.empty()) {
      ReduceDesc* dr = c.upload(red);
      hipEvent_t a; c.begin(T_REDUCE, a);
      launch_reduce(dr, int(red.size()), red_elems, c.stream);
      c.end(T_REDUCE, a, 0, red_bytes);
    }
    d.clear();
  }
};

struct CopyBatch {
  std::vector<CopyDesc> d;
  int64_t total = 0;
  void add(const double* src, int lds, double* dst, int ldd, int rows, int cols, double alpha) {
    if (rows <= 0 || cols <= 0) return;
    d.push_back(CopyDesc{src, dst, rows, cols, std::max(lds, 1), std::max(ldd, 1), alpha, total});
    total += int64_t(rows) * cols;
  }
  // n elements of p at stride ld set to v
  void add_fill_strided(double* p, int ld, int n, double v) {
    if (n <= 0) return;
    d.push_back(CopyDesc{nullptr, p, 1, n, 1, std::max(ld, 1), v, total});
    total += n;
  }
  // n elements of p set to v (through the same launch as the copies)
  void add_fill(double* p, int64_t n, double v) {
    for (int64_t o = 0; o < n; o += int64_t(1) << 30) {
      const int m = int(std::min<int64_t>(n - o, int64_t(1) << 30));
      d.push_back(CopyDesc{nullptr, p + o, m, 1, m, m, v, total});
      total += m;
    }
  }
  void run(Ctx& c) {
    if (d.empty()) return;
    CopyDesc* dd = c.upload(d);
    hipEvent_t a; c.begin(T_COPY, a);
    launch_copy(dd, int(d.size()), total, c.stream);
    c.end(T_COPY, a, 0, 16.0 * total);
    d.clear();
    total = 0;
  }
};

struct ScaleBatch {
  std::vector<ScaleDesc> d;
  int64_t total = 0;
  void add(const double* src, int lds, double* dst, int ldd, int rows, int cols, const double* s,
           bool invert, bool sqrt_s) {
    if (rows <= 0 || cols <= 0) return;
    d.push_back(ScaleDesc{src, dst, s, rows, cols, std::max(lds, 1), std::max(ldd, 1), total,
                          invert ? 1 : 0, sqrt_s ? 1 : 0});
    total += int64_t(rows) * cols;
  }
  void run(Ctx& c) {
    if (d.empty()) return;
    ScaleDesc* dd = c.upload(d);
    hipEvent_t a; c.begin(T_COPY, a);
    launch_scale(dd, int(d.size()), total, c.stream);
    c.end(T_COPY, a, 0, 16.0 * total);
    d.clear();
    total = 0;
  }
};

struct EigJob {
  const double* A;
  int lda, n;
  double* V;
  double* w;
  double abs_tol = 1e-15;
  bool tridiag = false;  // Householder + bisection + inverse iteration (scaled path)
  bool force = false;    // use the tridiagonal solver at any size
};

constexpr double kAbsTolGeneral = 1e-15;  // first pass / Gram eigenproblems
constexpr double kAbsTolRefine = 0.0;     // second pass on nearly diagonal input
// numerical-zero level of single-pass Gram singular values: sigma <= 1e-6 sigma_max, i.e.
// eigenvalues below 1e-12 of the largest, above the rounding level of the Gram solvers
constexpr double kZeroTolPar = 1e-6;
constexpr double kVecCut = 1e-12;  // tridiagonal solver: no eigenvector below this


// Step-per-launch reduction: workgroups per launch aimed at (as many per compute unit as
// the instance's registers let run at once: three for n > 512, five for n <= 512) and the
// most per problem.
constexpr int kTriStepWorkgroups = 768, kTriStepWorkgroupsSmall = 1280;
constexpr int kTriStepMaxG = 128;
constexpr int kTriStepTimeEvery = 8;

// Matrices above this size go to the tridiagonal solver when the job allows it.
constexpr int kTridiagMin = 40;
// Algorithmic flops of a symmetric eigendecomposition with eigenvectors, counted as the
// standard Householder route: tridiagonal reduction 4/3 n^3 plus back-transformation 2 n^3
// (the same count is used for the Jacobi kernel, which does more work).
constexpr double kEigFlops = 10.0 / 3.0;

// Eigenproblems of one batch.  The tridiagonal ones keep their work areas here between
// the eigenvalue launches and the eigenvector launches.
struct EigPlan {
  std::vector<EigDesc> tri;
  std::vector<int> job;  // job index of each tridiagonal problem
  std::vector<Buf> work;
  int ntri = 0;
};

}  // namespace

static void tri_panels(Ctx& c, const std::vector<EigDesc>& tri, const EigDesc* d, int ntri, double ftri,
                       double btri);

// Tridiagonal solver, first half, for the problems `tri` (host copies of the descriptors)
// whose device copy is `d`: reduction (preparation, panels with trailing GEMM updates,
// finish) and the eigenvalues.  ftri/btri: algorithmic flops and bytes of the panels.
void tri_values(Ctx& c, const std::vector<EigDesc>& tri, const EigDesc* d, int ntri, double ftri, double btri) {
  const int np = int(tri.size());
  double bprep = 0;
  for (const EigDesc& e : tri) bprep += 16.0 * double(e.n) * e.n;
  hipEvent_t a;
  c.begin(T_COPY, a);
  launch_tri_prepare(d, np, ntri, c.stream);
  c.end(T_COPY, a, 0, bprep);
  if (np <= c.tri_step_max) {
    // one step per launch on several workgroups per problem.  The problems go in order of
    // decreasing size, so those still reducing at step k are a prefix of the list; each
    // launch covers only them and spreads the workgroup budget over them (the instances
    // for n <= 512 hold fewer registers: more workgroups fit).
    const int target = ntri <= 512 ? kTriStepWorkgroupsSmall : kTriStepWorkgroups;
    std::vector<EigDesc> srt(tri);
    std::stable_sort(srt.begin(), srt.end(), [](const EigDesc& x, const EigDesc& y) { return x.n > y.n; });
    // (a single problem uses the caller's descriptor: nothing is allocated then)
    const EigDesc* ds = np == 1 ? d : c.upload(srt);
    // a problem takes step launches for k < n - tri_tail_rows(); the tail kernel then
    // finishes every problem at once
    const int T = tri_tail_rows();
    const int last = std::max(ntri - T - 1, -1);
    int act = np;
    for (int k = 0; k <= last; ++k) {
      while (act > 0 && srt[act - 1].n - T <= k) --act;
      if (act == 0) break;
      const int G = std::clamp(target / act, 1, kTriStepMaxG);
      // every kTriStepTimeEvery-th launch is timed and stands for the launches up to the
      // next timed one: events around each of these short launches would lengthen the run
      if (k % kTriStepTimeEvery != 0) {
        launch_tri_step(ds, act, ntri, k, G, c.stream);
        continue;
      }
      // algorithmic work of step k: the trailing block of every problem read and written
      // once (read only at k = 0), 6 flops per element (rank-2 update and product)
      double fl = 0, by = 0;
      for (int i = 0; i < act; ++i) {
        const double m = std::max(srt[i].n - k - 1, 0);
        fl += 6.0 * m * m;
        by += (k > 0 ? 16.0 : 8.0) * m * m;
      }
      c.begin(T_TRI, a);
      launch_tri_step(ds, act, ntri, k, G, c.stream);
      c.end(T_TRI, a, fl, by, std::min(kTriStepTimeEvery, last + 1 - k));
    }
    {
      // the tail: per problem about 4/3 m^3 flops over its m = min(n, T) trailing rows,
      // the block read once and the reflectors written
      double fl = 0, by = 0;
      for (const EigDesc& e : tri) {
        const double m = std::min(e.n, T);
        fl += 4.0 / 3.0 * m * m * m;
        by += 8.0 * m * m;
      }
      c.begin(T_TRITAIL, a);
      launch_tri_tail(d, np, c.stream);
      c.end(T_TRITAIL, a, fl, by);
    }
  } else {
    tri_panels(c, tri, d, ntri, ftri, btri);
  }
  c.begin(T_TRIVAL, a);
  launch_eig_tridiag(d, np, ntri, 2, c.stream);
  c.end(T_TRIVAL, a, 0, 0);
}

// Blocked reduction: panel kernel (one workgroup per problem), then the trailing update of
// every problem as a GEMM, then the last 2 x 2 blocks.
static void tri_panels(Ctx& c, const std::vector<EigDesc>& tri, const EigDesc* d, int ntri, double ftri,
                       double btri) {
  const int np = int(tri.size());
  hipEvent_t a;
  const double nsteps = std::max(ntri - 2, 1);
  for (int k0 = 0; k0 + 2 < ntri; k0 += kTriPanel) {
    const double share = std::min<double>(kTriPanel, ntri - 2 - k0) / nsteps;
    c.begin(T_TRI, a);
    launch_tri_panel(d, np, ntri, k0, c.stream);
    c.end(T_TRI, a, ftri * share, btri * share);
    GemmBatch g;
    g.cls = T_TRIGEMM;
    g.prec = 2;
    for (const EigDesc& e : tri) {
      const int n = e.n;
      if (k0 + 2 >= n) continue;
      const int nbe = std::min(kTriPanel, n - 2 - k0);
      const int o = k0 + nbe, m2 = n - o;
      double* P1 = e.work + int64_t(n) * n;
      double* P2 = P1 + int64_t(2) * nbe * n;
      g.add(P1 + o, n, 0, P2 + o, n, 1, e.work + o + int64_t(o) * n, n, m2, m2, 2 * nbe, -1.0, 1.0);
    }
    g.run(c);
  }
  c.begin(T_COPY, a);
  launch_tri_finish(d, np, c.stream);
  c.end(T_COPY, a, 0, 0);
}

// Second half: eigenvectors by inverse iteration and the back-transformation, for the
// d[i].nvec leading eigenvalues of each problem (the device descriptors carry nvec).
void tri_vectors(Ctx& c, const std::vector<EigDesc>& tri, const EigDesc* d, int ntri) {
  double fb = 0;
  for (const EigDesc& e : tri) fb += 2.0 * double(e.n) * e.n * e.nvec;
  hipEvent_t a; c.begin(T_TRIVEC, a);
  launch_eig_tridiag(d, int(tri.size()), ntri, 4, c.stream);
  c.end(T_TRIVEC, a, 0, 0);
  c.begin(T_TRIBACK, a);
  launch_eig_tridiag(d, int(tri.size()), ntri, 8, c.stream);
  c.end(T_TRIBACK, a, fb, 0);
}

namespace {

// Eigenvalues of every job; the Jacobi problems (small, or not flagged tridiagonal) also
// get all their eigenvectors here.
EigPlan run_eig_values(Ctx& c, const std::vector<EigJob>& jobs) {
  EigPlan plan;
  std::vector<EigDesc> by_mode[3];
  int nmax[3] = {0, 0, 0};
  double flops[3] = {0, 0, 0}, ftri = 0, btri = 0;
  for (size_t ji = 0; ji < jobs.size(); ++ji) {
    const EigJob& j = jobs[ji];
    if (j.n <= 0) continue;
    if (j.n > kEigMax) fail(PV_EINVAL, "eigenproblem of size " + std::to_string(j.n) + " exceeds the supported maximum");
    if (j.tridiag && (j.n > kTridiagMin || j.force)) {
      Buf w(c.pool, tri_work_doubles(j.n));
      plan.tri.push_back(EigDesc{j.A, j.lda, j.n, j.V, j.w, w.p, nullptr, std::max(j.abs_tol, kVecCut)});
      plan.job.push_back(int(ji));
      plan.work.push_back(std::move(w));
      plan.ntri = std::max(plan.ntri, j.n);
      // panel kernels: the symmetric products over the stored trailing lower triangle,
      // 4 flops and 8 bytes per element read (the rank-2k updates are counted as GEMMs)
      ftri += 2.0 / 3.0 * double(j.n) * j.n * j.n;
      btri += 4.0 / 3.0 * double(j.n) * j.n * j.n;
      continue;
    }
    const int mode = eig_mode(j.n);
    const size_t wn = size_t(j.n) * j.n + size_t(j.n) * (j.n + 1) / 2;
    Buf w = scratch_buf(c, wn);
    by_mode[mode].push_back(EigDesc{j.A, j.lda, j.n, j.V, j.w, w.p, nullptr, j.abs_tol});
    c.scratch.push_back(std::move(w));
    nmax[mode] = std::max(nmax[mode], j.n);
    flops[mode] += kEigFlops * double(j.n) * j.n * j.n;
  }
  if (!plan.tri.empty()) {
    EigDesc* d = c.upload(plan.tri);
    tri_values(c, plan.tri, d, plan.ntri, ftri, btri);
  }
  for (int mode = 2; mode >= 0; --mode) {
    if (by_mode[mode].empty()) continue;
    EigDesc* d = c.upload(by_mode[mode]);
    hipEvent_t a; c.begin(T_EIG, a);
    launch_eig(d, int(by_mode[mode].size()), nmax[mode], mode, c.stream);
    c.end(T_EIG, a, flops[mode], 0);
  }
  return plan;
}

// Eigenvectors of the tridiagonal problems of a plan: for job j the nvec[j] leading ones
// (all when nvec is null), the other columns of V zero.
void run_eig_vectors(Ctx& c, EigPlan& plan, const std::vector<int>* nvec) {
  if (plan.tri.empty()) return;
  for (size_t i = 0; i < plan.tri.size(); ++i) {
    EigDesc& e = plan.tri[i];
    e.nvec = nvec ? std::min(std::max((*nvec)[plan.job[i]], 0), e.n) : e.n;
  }
  EigDesc* d = c.upload(plan.tri);
  tri_vectors(c, plan.tri, d, plan.ntri);
  for (Buf& w : plan.work) c.scratch.push_back(std::move(w));
  plan.work.clear();
  plan.tri.clear();
}

void run_eig(Ctx& c, const std::vector<EigJob>& jobs) {
  EigPlan plan = run_eig_values(c, jobs);
  run_eig_vectors(c, plan, nullptr);
}

// W W^T ~ G for every job (G symmetric positive semidefinite, n x n, ld n; W lower
// triangular, n x n, numerically dependent columns zero): panel kernels interleaved with
// batched trailing GEMMs.
struct CholJob {
  const double* G;
  int n;
  double* W;
};

void chol_all(Ctx& c, const std::vector<CholJob>& jobs) {
  std::vector<CholDesc> d;
  CopyBatch cp;
  int nmax = 0;
  int64_t ndg = 0;
  for (const CholJob& j : jobs) ndg += std::max(j.n, 0);
  Buf dg = scratch_buf(c, size_t(std::max<int64_t>(ndg, 1)));
  ndg = 0;
  for (const CholJob& j : jobs) {
    if (j.n <= 0) continue;
    cp.add(j.G, j.n, j.W, j.n, j.n, j.n, 1.0);
    d.push_back(CholDesc{j.W, dg.p + ndg, j.n, j.n});
    ndg += j.n;
    nmax = std::max(nmax, j.n);
  }
  c.scratch.push_back(std::move(dg));
  if (d.empty()) return;
  cp.run(c);
  CholDesc* dd = c.upload(d);
  for (int j0 = 0; j0 < nmax; j0 += kCholB) {
    double fl = 0;
    for (const CholDesc& x : d) {
      const int jb = std::min(kCholB, x.n - j0);
      if (jb > 0) fl += double(jb) * jb * jb / 3.0 + double(x.n - j0 - jb) * jb * jb;
    }
    hipEvent_t a; c.begin(T_CHOL, a);
    launch_chol_panel(dd, int(d.size()), j0, c.stream);
    c.end(T_CHOL, a, fl, 0);
    GemmBatch g;
    for (const CholDesc& x : d) {
      const int m2 = x.n - j0 - kCholB;
      if (m2 <= 0) continue;
      const int64_t o = j0 + kCholB;
      g.add(x.A + o + int64_t(j0) * x.n, x.n, 0, x.A + o + int64_t(j0) * x.n, x.n, 1, x.A + o + o * x.n, x.n, m2, m2,
            kCholB, -1.0, 1.0);
    }
    g.run(c);
  }
}

void fill(Ctx& c, double* p, int64_t n, double v) {
  if (n <= 0) return;
  hipEvent_t a; c.begin(T_COPY, a);
  launch_fill(p, n, v, c.stream);
  c.end(T_COPY, a, 0, 8.0 * n);
}

// Rank selection across the sectors of one bond (same rules as the truncation of the
// oracle): drop sigma <= zero_tol * sigma_max, order by sigma descending (ties: lower
// sector, then lower index), keep the least count whose discarded tail has
// sum sigma^2 <= delta^2, at most cap, at least one.
constexpr double kZeroTol = 1e-12;

// Two runs of values in descending order merged into out (ties: the first run's value first).
static void merge_desc(const double* a, size_t na, const double* b, size_t nb, double* out) {
  size_t i = 0, j = 0, k = 0;
  while (i < na && j < nb) {
    const double x = a[i], y = b[j];
    const bool t = y > x;
    out[k++] = t ? y : x;
    j += t;
    i += !t;
  }
  while (i < na) out[k++] = a[i++];
  while (j < nb) out[k++] = b[j++];
}

// The candidate values are put in descending order by merging the sectors' lists (each
// already descending from the eigensolver; sorted first otherwise); the sector counts of
// the leading s then follow from the s-th value, ties going to the lower sectors first,
// which is the order (value, sector, index) of the rule.
std::vector<int> select_ranks(const std::vector<std::vector<double>>& sig, double delta, int cap,
                              bool* cap_bound, double zero_tol = kZeroTol) {
  std::vector<int> kept(sig.size(), 0);
  double smax = 0.0;
  size_t tot = 0;
  for (const auto& v : sig) {
    tot += v.size();
    for (double x : v) smax = std::max(smax, x);
  }
  if (tot == 0 || !(smax > 0.0)) return kept;
  const double zl = zero_tol * smax;
  std::vector<double> cand, buf;
  cand.reserve(tot);
  std::vector<size_t> runs{0}, next;
  for (const auto& v : sig) {
    const size_t b0 = cand.size();
    for (double x : v)
      if (x > zl) cand.push_back(x);
    if (!std::is_sorted(cand.begin() + b0, cand.end(), std::greater<double>()))
      std::sort(cand.begin() + b0, cand.end(), std::greater<double>());
    if (cand.size() > b0) runs.push_back(cand.size());
  }
  buf.resize(cand.size());
  while (runs.size() > 2) {
    next.assign(1, 0);
    for (size_t r = 0; r + 1 < runs.size(); r += 2) {
      if (r + 2 < runs.size()) {
        merge_desc(cand.data() + runs[r], runs[r + 1] - runs[r], cand.data() + runs[r + 1], runs[r + 2] - runs[r + 1],
                   buf.data() + runs[r]);
        next.push_back(runs[r + 2]);
      } else {
        std::copy(cand.begin() + runs[r], cand.begin() + runs[r + 1], buf.begin() + runs[r]);
        next.push_back(runs[r + 1]);
      }
    }
    cand.swap(buf);
    runs.swap(next);
  }
  const int m = int(cand.size());
  // the least s whose discarded tail (summed from the smallest value up) is <= delta^2
  int s_tol = m;
  {
    std::vector<double> tail(size_t(m) + 1, 0.0);
    for (int i = m - 1; i >= 0; --i) tail[i] = tail[i + 1] + cand[i] * cand[i];
    for (int s = 0; s <= m; ++s)
      if (tail[s] <= delta * delta) { s_tol = s; break; }
  }
  if (s_tol > cap && cap_bound) *cap_bound = true;
  const int s = std::min(std::max(1, std::min(s_tol, cap)), m);
  if (s <= 0) return kept;
  const double th = cand[size_t(s) - 1];
  int taken = 0;
  for (size_t n = 0; n < sig.size(); ++n) {
    int c = 0;
    for (double x : sig[n]) c += (x > zl && x > th) ? 1 : 0;
    kept[n] = c;
    taken += c;
  }
  for (size_t n = 0; n < sig.size() && taken < s; ++n) {
    int c = 0;
    for (double x : sig[n]) c += (x > zl && x == th) ? 1 : 0;
    c = std::min(c, s - taken);
    kept[n] += c;
    taken += c;
  }
  return kept;
}

// Sum of the squares of the singular values above the numerical-zero level that a rank
// selection left out (sig[n] descending; keep[n] leading values of sector n kept).
double dropped_weight(const std::vector<std::vector<double>>& sig, const std::vector<int>& keep, double zero_tol) {
  double smax = 0.0;
  for (const auto& v : sig)
    for (double x : v) smax = std::max(smax, x);
  double d2 = 0.0;
  for (size_t n = 0; n < sig.size(); ++n)
    for (size_t j = size_t(std::max(keep[n], 0)); j < sig[n].size(); ++j)
      if (sig[n][j] > zero_tol * smax) d2 += sig[n][j] * sig[n][j];
  return d2;
}

// through a pinned buffer of the context: a copy into pageable memory would have the
// runtime lock the destination's pages first, which costs far more than the copy itself
std::vector<double> download(Ctx& c, const double* p, size_t n) {
  if (n > c.dl_n) {
    c.sync();
    if (c.dl_host) PV_HIP(hipHostFree(c.dl_host));
    c.dl_host = nullptr;
    c.dl_n = 0;
    const size_t cap = std::max<size_t>(n + n / 2, 4096);
    void* h = nullptr;
    PV_HIP(hipHostMalloc(&h, cap * sizeof(double), hipHostMallocDefault));
    c.dl_host = static_cast<double*>(h);
    c.dl_n = cap;
  }
  if (n) PV_HIP(hipMemcpyAsync(c.dl_host, p, n * sizeof(double), hipMemcpyDeviceToHost, c.stream));
  c.sync();
  return std::vector<double>(c.dl_host, c.dl_host + n);
}

// ---------------------------------------------------------------- environments
// Environment / carry at cut m: for each "bra" sector na a matrix with rho_bra rows and
// columns = concatenation over charges q of (w_q states x ket dimension of sector na-q),
// each q-part stored as [a, b, c] with a fastest.
struct EnvLayout {
  int m = 0;
  std::vector<int> rows;
  std::vector<std::array<int64_t, 5>> qcol;  // -1 when absent
  std::vector<std::array<int, 5>> kdim;
  std::vector<int64_t> ncols, off;
  int64_t total = 0;
};

EnvLayout env_layout(int m, int N, const std::vector<int>& bra_rho_m, const std::vector<int>& ket_rho_m,
                     const std::array<int, 6>& qoff, auto&& valid_bra, auto&& valid_ket) {
  EnvLayout e;
  e.m = m;
  e.rows.assign(N + 1, 0);
  e.qcol.assign(N + 1, {-1, -1, -1, -1, -1});
  e.kdim.assign(N + 1, {0, 0, 0, 0, 0});
  e.ncols.assign(N + 1, 0);
  e.off.assign(N + 1, 0);
  for (int na = 0; na <= N; ++na) {
    e.off[na] = e.total;
    if (!valid_bra(m, na)) continue;
    const int r = bra_rho_m[na];
    e.rows[na] = r;
    int64_t col = 0;
    for (int q = -2; q <= 2; ++q) {
      const int n = na - q;
      const int wq = qoff[q + 3] - qoff[q + 2];
      if (wq <= 0 || n < 0 || n > N || !valid_ket(m, n)) continue;
      const int kd = ket_rho_m[n];
      if (kd <= 0) continue;
      e.qcol[na][q + 2] = col;
      e.kdim[na][q + 2] = kd;
      col += int64_t(wq) * kd;
    }
    e.ncols[na] = col;
    e.total += int64_t(r) * col;
  }
  return e;
}

inline int wq_of(const std::array<int, 6>& qoff, int q) { return qoff[q + 3] - qoff[q + 2]; }

// One output block of the W-step (output sector n2 and s_out, output charge q', all its
// w_{q'} states b') and the T1 slices it reads: base[s_in][q_in + 2] points at the part of
// T1 with physical index s_in and input charge q_in (null if absent), ld is its stride
// between consecutive c'.
struct WBlock {
  double* out;
  int rows, cols, wq_out, qoff_out, s_out, src;
};
struct WSrc {
  const double* base[2][5];
  int64_t ld[2][5];
};

// One site of a sweep: T1 = E x_k (GEMM), T2 = W_k T1 (W-step).
// Output T2 grouped by (s_out, n2) with rows rho_bra[k-1][n2 - s_out] and the column
// layout of the environment at cut k (`Ln`).  Returns the T2 buffer and offsets.
struct T2Data {
  Buf buf;
  std::vector<int64_t> off[2];
  std::vector<int> rows[2];
};

T2Data site_contract(Ctx& c, int k, const Mps& ket, const std::vector<int>& bra_rows_prev,
                     const EnvLayout& Le, const Buf& E, const EnvLayout& Ln, const DevMpo& op) {
  const int N = ket.N;
  const auto& qo_in = op.qoff[k - 1];
  // (i) T1
  std::vector<int64_t> t1off((N + 1) * 5, -1);
  int64_t t1tot = 0;
  for (int na = 0; na <= N; ++na)
    for (int q = -2; q <= 2; ++q) {
      if (Le.qcol[na][q + 2] < 0 || Le.rows[na] == 0) continue;
      const int n = na - q;
      const int cols = ket.ucols(k, n) + ket.ocols(k, n);
      if (cols == 0) continue;
      t1off[na * 5 + q + 2] = t1tot;
      t1tot += int64_t(Le.rows[na]) * wq_of(qo_in, q) * cols;
    }
  Buf T1(c.pool, size_t(std::max<int64_t>(t1tot, 1)));
  GemmBatch gb;
  gb.prec = c.contraction_kernel();
  for (int na = 0; na <= N; ++na)
    for (int q = -2; q <= 2; ++q) {
      const int64_t o = t1off[na * 5 + q + 2];
      if (o < 0) continue;
      const int n = na - q;
      const int rw = Le.rows[na] * wq_of(qo_in, q);
      const int cols = ket.ucols(k, n) + ket.ocols(k, n);
      const double* A = E.p + Le.off[na] + int64_t(Le.rows[na]) * Le.qcol[na][q + 2];
      gb.add(A, rw, 0, ket.U(k, n), ket.rows(k, n), 0, T1.p + o, rw, rw, cols, Le.kdim[na][q + 2], 1.0, 0.0);
    }
  gb.run(c);
  // (ii) W-step
  T2Data t2;
  int64_t t2tot = 0;
  for (int s = 0; s < 2; ++s) {
    t2.off[s].assign(N + 1, -1);
    t2.rows[s].assign(N + 1, 0);
    for (int n2 = 0; n2 <= N; ++n2) {
      const int na = n2 - s;
      // output bra sector n2 at cut k; rows come from bra sector na at cut k-1
      if (na < 0 || na > N || Ln.ncols[n2] == 0 || Ln.rows[n2] == 0 || Le.rows[na] == 0) continue;
      t2.off[s][n2] = t2tot;
      t2.rows[s][n2] = Le.rows[na];
      t2tot += int64_t(Le.rows[na]) * Ln.ncols[n2];
    }
  }
  t2.buf = Buf(c.pool, size_t(std::max<int64_t>(t2tot, 1)));
  const auto& qo_out = op.qoff[k];
  const DevMpo::Site& st = op.site[k - 1];
  const std::vector<int8_t>& chg_in = op.charge[k - 1];
  std::vector<WSrc> srcs;
  std::vector<WBlock> blocks;
  std::vector<WTask> tasks;
  std::vector<WEntry> entries;
  double bytes = 0;
  for (int s = 0; s < 2; ++s)
    for (int n2 = 0; n2 <= N; ++n2) {
      if (t2.off[s][n2] < 0) continue;
      const int na = n2 - s;
      const int rows = t2.rows[s][n2];
      WSrc src{};
      for (int si = 0; si < 2; ++si)
        for (int q = -2; q <= 2; ++q) {
          src.base[si][q + 2] = nullptr;
          src.ld[si][q + 2] = 0;
          const int64_t o = t1off[na * 5 + q + 2];
          if (o < 0) continue;
          const int n = na - q;
          const int cu = ket.ucols(k, n), co = ket.ocols(k, n);
          if ((si == 0 && cu == 0) || (si == 1 && co == 0)) continue;
          const int64_t ld = int64_t(rows) * wq_of(qo_in, q);
          src.base[si][q + 2] = T1.p + o + (si ? int64_t(cu) * ld : 0);
          src.ld[si][q + 2] = ld;
        }
      const int sid = int(srcs.size());
      srcs.push_back(src);
      for (int q2 = -2; q2 <= 2; ++q2) {
        const int64_t qc = Ln.qcol[n2][q2 + 2];
        if (qc < 0) continue;
        WBlock B{};
        B.out = t2.buf.p + t2.off[s][n2] + int64_t(rows) * qc;
        B.rows = rows;
        B.cols = Ln.kdim[n2][q2 + 2];
        B.wq_out = wq_of(qo_out, q2);
        B.qoff_out = qo_out[q2 + 2];
        B.s_out = s;
        B.src = sid;
        blocks.push_back(B);
        const int nel = rows * B.cols;
        if (nel == 0) continue;
        for (int b = 0; b < B.wq_out; ++b) {
          // sparse entries of row (s_out, b') resolved to source slices of T1
          const int row = s * st.w_out + B.qoff_out + b;
          const int e0 = int(entries.size());
          for (int e = st.row_ptr[row]; e < st.row_ptr[row + 1]; ++e) {
            const int bi = st.b_in[e];
            const int q = chg_in[bi] + 2;
            const double* base = src.base[st.s_in[e]][q];
            if (!base) continue;
            entries.push_back(WEntry{base + int64_t(rows) * (bi - qo_in[q]), src.ld[st.s_in[e]][q], st.val[e]});
          }
          const int e1 = int(entries.size());
          bytes += 8.0 * nel * (e1 - e0 + 1);
          for (int x0 = 0; x0 < nel; x0 += kWTask)
            tasks.push_back(WTask{B.out + int64_t(rows) * b, int64_t(rows) * B.wq_out, rows, nel, x0, e0, e1});
        }
      }
    }
  if (!tasks.empty()) {
    auto [dt, de] = c.upload2(tasks, entries);
    hipEvent_t a; c.begin(T_WSTEP, a);
    launch_wstep(dt, int(tasks.size()), de, c.stream);
    c.end(T_WSTEP, a, 0, bytes);
  }
  // dense charge blocks of W_k: T2[a, b', c'] += sum_b T1[a, b, c'] W[b, b'], one product whose
  // rows run over the pairs (a, c')
  if (!st.dense.empty()) {
    // several dense blocks may accumulate into one output block: the k-th contribution to
    // each output goes to launch k, so no launch has two problems writing the same output
    std::vector<GemmBatch> gd;
    for (const WBlock& B : blocks) {
      int slot = 0;
      const WSrc& src = srcs[B.src];
      const int q_out = [&] {
        for (int q = -2; q <= 2; ++q)
          if (qo_out[q + 2] == B.qoff_out) return q;
        return 99;
      }();
      for (const DevMpo::Dense& D : st.dense) {
        if (D.s_out != B.s_out || D.q_out != q_out || D.w_out != B.wq_out) continue;
        const double* base = src.base[D.s_in][D.q_in + 2];
        if (!base) continue;
        const int64_t ld = src.ld[D.s_in][D.q_in + 2];
        if (int(gd.size()) <= slot) {
          gd.emplace_back();
          gd.back().prec = c.contraction_kernel();
        }
        // one product over all c': rows (a, c') of T1 and T2
        gd[slot].add_rows2(base, B.rows, ld, D.W.p, D.w_in, 0, B.out, B.rows, int64_t(B.rows) * B.wq_out, B.rows,
                           B.cols, B.wq_out, D.w_in, 1.0, 1.0);
        ++slot;
      }
    }
    for (auto& g : gd) g.run(c);
  }
  c.scratch.push_back(std::move(T1));
  (void)bra_rows_prev;
  return t2;
}

}  // namespace

// ---------------------------------------------------------------- MPO upload
std::unique_ptr<DevMpo> upload_mpo(Ctx& c, const Mpo& m) {
  c.sync();  // synchronous copies below must not overtake queued work
  auto d = std::make_unique<DevMpo>();
  d->L = m.L;
  d->w = m.w;
  d->qoff = m.qoff;
  d->site.resize(m.L);
  d->charge.resize(m.L + 1);
  auto put = [&](const void* src, size_t bytes) {
    Buf b(c.pool, std::max<size_t>((bytes + 7) / 8, 1));
    if (bytes) PV_HIP(hipMemcpy(b.p, src, bytes, hipMemcpyHostToDevice));
    return b;
  };
  for (int k = 0; k <= m.L; ++k) d->charge[k].assign(m.charge[k].begin(), m.charge[k].end());
  for (int k = 0; k < m.L; ++k) {
    const MpoSite& st = m.site[k];
    // charge blocks dense enough for a GEMM
    auto qof = [&](int cut, int b) { return int(m.charge[cut][b]); };
    std::map<std::array<int, 4>, int> cnt;  // (q_in, q_out, s_in, s_out) -> nnz
    for (size_t e = 0; e < st.val.size(); ++e)
      cnt[{qof(k, st.b_in[e]), qof(k + 1, st.b_out[e]), st.s_in[e], st.s_out[e]}]++;
    std::map<std::array<int, 4>, int> dense_id;
    for (auto& kv : cnt) {
      const int qi = kv.first[0], qo = kv.first[1];
      const int wi = m.qoff[k][qi + 3] - m.qoff[k][qi + 2];
      const int wo = m.qoff[k + 1][qo + 3] - m.qoff[k + 1][qo + 2];
      const double dens = double(kv.second) / (double(wi) * wo);
      if (kv.second >= 64 && dens >= 0.05) {
        dense_id[kv.first] = int(d->site[k].dense.size());
        DevMpo::Dense D{qi, qo, kv.first[2], kv.first[3], wi, wo, Buf()};
        d->site[k].dense.push_back(std::move(D));
      }
    }
    std::vector<std::vector<double>> dmat(d->site[k].dense.size());
    for (size_t i = 0; i < dmat.size(); ++i)
      dmat[i].assign(size_t(d->site[k].dense[i].w_in) * d->site[k].dense[i].w_out, 0.0);
    std::vector<size_t> sparse_idx;
    for (size_t e = 0; e < st.val.size(); ++e) {
      const int qi = qof(k, st.b_in[e]), qo = qof(k + 1, st.b_out[e]);
      auto it = dense_id.find({qi, qo, st.s_in[e], st.s_out[e]});
      if (it == dense_id.end()) { sparse_idx.push_back(e); continue; }
      const auto& D = d->site[k].dense[it->second];
      const int bi = st.b_in[e] - m.qoff[k][qi + 2], bo = st.b_out[e] - m.qoff[k + 1][qo + 2];
      dmat[it->second][bi + size_t(bo) * D.w_in] += st.val[e];
    }
    for (size_t i = 0; i < dmat.size(); ++i) d->site[k].dense[i].W = put(dmat[i].data(), dmat[i].size() * 8);
    const int rows = 2 * st.w_out;
    std::vector<int32_t> rp(rows + 1, 0);
    for (size_t e : sparse_idx) rp[st.s_out[e] * st.w_out + st.b_out[e] + 1]++;
    for (int r = 0; r < rows; ++r) rp[r + 1] += rp[r];
    std::vector<int32_t> bi(sparse_idx.size());
    std::vector<uint8_t> si(sparse_idx.size());
    std::vector<double> vv(sparse_idx.size());
    std::vector<int32_t> fillp(rp.begin(), rp.end() - 1);
    for (size_t e : sparse_idx) {
      const int r = st.s_out[e] * st.w_out + st.b_out[e];
      const int p = fillp[r]++;
      bi[p] = st.b_in[e];
      si[p] = st.s_in[e];
      vv[p] = st.val[e];
    }
    d->site[k].row_ptr = std::move(rp);
    d->site[k].b_in = std::move(bi);
    d->site[k].s_in = std::move(si);
    d->site[k].val = std::move(vv);
    d->site[k].w_out = st.w_out;
    d->nnz += int64_t(st.val.size());
  }
  return d;
}

// Diagonal operator with w states at every inner cut: state j applies
// diag(d0[j][k], d1[j][k]) on site k; the boundary cut 0 has one state feeding all j
// and cut L keeps the w states apart, so one sweep yields w expectation values.
static std::unique_ptr<DevMpo> diag_mpo(Ctx& c, int L, int w, const std::vector<std::vector<double>>& d0,
                                        const std::vector<std::vector<double>>& d1) {
  Mpo m;
  m.L = L;
  m.w.assign(L + 1, w);
  m.w[0] = 1;
  m.charge.resize(L + 1);
  m.qoff.resize(L + 1);
  for (int k = 0; k <= L; ++k) {
    m.charge[k].assign(m.w[k], 0);
    m.qoff[k] = {0, 0, 0, m.w[k], m.w[k], m.w[k]};
  }
  m.site.resize(L);
  for (int k = 0; k < L; ++k) {
    MpoSite& s = m.site[k];
    s.w_in = m.w[k];
    s.w_out = m.w[k + 1];
    for (int j = 0; j < w; ++j) {
      const int bin = k == 0 ? 0 : j;
      for (int o = 0; o < 2; ++o) {
        const double val = o == 0 ? d0[j][k] : d1[j][k];
        if (val == 0.0) continue;
        s.b_in.push_back(bin); s.b_out.push_back(j);
        s.s_in.push_back(uint8_t(o)); s.s_out.push_back(uint8_t(o));
        s.val.push_back(val);
      }
    }
  }
  return upload_mpo(c, m);
}

// ---------------------------------------------------------------- sweeps
// the sweep's launches on c.stream; the result is the block of bra sector N of the
// environment at cut L (rows x cols, column-major) inside E
struct EnvEnd {
  Buf E;
  const double* res = nullptr;
  int64_t rows = 0, cols = 0;
};

static EnvEnd env_sweep_dev(Ctx& c, const Mps& bra, const Mps& ket, const DevMpo& op) {
  const int L = ket.L, N = ket.N;
  if (bra.L != L || bra.N != N || op.L != L) fail(PV_EINVAL, "env_sweep: mismatched chains");
  auto vb = [&](int m, int n) { return bra.valid(m, n); };
  auto vk = [&](int m, int n) { return ket.valid(m, n); };
  EnvLayout Le = env_layout(0, N, bra.rho[0], ket.rho[0], op.qoff[0], vb, vk);
  Buf E(c.pool, size_t(std::max<int64_t>(Le.total, 1)));
  fill(c, E.p, Le.total, 1.0);  // 1 x 1 x 1 at cut 0
  for (int k = 1; k <= L; ++k) {
    EnvLayout Ln = env_layout(k, N, bra.rho[k], ket.rho[k], op.qoff[k], vb, vk);
    T2Data t2 = site_contract(c, k, ket, bra.rho[k - 1], Le, E, Ln, op);
    Buf En(c.pool, size_t(std::max<int64_t>(Ln.total, 1)));
    // the first product into a block overwrites it (beta 0); blocks without one are cleared
    GemmBatch g0, g1;
    CopyBatch zero;
    for (int n2 = 0; n2 <= N; ++n2) {
      if (Ln.rows[n2] == 0 || Ln.ncols[n2] == 0) continue;
      double* C = En.p + Ln.off[n2];
      const bool p0 = t2.off[0][n2] >= 0 && bra.ucols(k, n2) > 0;
      const bool p1 = t2.off[1][n2] >= 0 && n2 >= 1 && bra.ocols(k, n2 - 1) > 0;
      if (p0)
        g0.add(bra.U(k, n2), bra.rows(k, n2), 1, t2.buf.p + t2.off[0][n2], t2.rows[0][n2], 0, C,
               Ln.rows[n2], Ln.rows[n2], int(Ln.ncols[n2]), bra.rows(k, n2), 1.0, 0.0);
      if (p1)
        g1.add(bra.O(k, n2 - 1), bra.rows(k, n2 - 1), 1, t2.buf.p + t2.off[1][n2], t2.rows[1][n2], 0, C,
               Ln.rows[n2], Ln.rows[n2], int(Ln.ncols[n2]), bra.rows(k, n2 - 1), 1.0, p0 ? 1.0 : 0.0);
      if (!p0 && !p1) zero.add_fill(C, int64_t(Ln.rows[n2]) * Ln.ncols[n2], 0.0);
    }
    zero.run(c);
    g0.run(c);
    g1.run(c);
    c.scratch.push_back(std::move(t2.buf));
    c.scratch.push_back(std::move(E));
    E = std::move(En);
    Le = std::move(Ln);
  }
  // cut L: bra sector N, one row; columns = w_0 states x ket dim 1
  EnvEnd r;
  r.res = E.p + Le.off[N];
  r.rows = Le.rows[N];
  r.cols = Le.ncols[N];
  r.E = std::move(E);
  return r;
}

std::vector<double> env_sweep(Ctx& c, const Mps& bra, const Mps& ket, const DevMpo& op) {
  EnvEnd r = env_sweep_dev(c, bra, ket, op);
  std::vector<double> out = download(c, r.res, size_t(r.rows * r.cols));
  return out;
}

static const DevMpo& identity_mpo(Ctx& c, int L) {
  if (!c.ident || c.ident->L != L) {
    std::vector<std::vector<double>> one(1, std::vector<double>(L, 1.0));
    c.ident = diag_mpo(c, L, 1, one, one);
  }
  return *c.ident;
}

// sum_i v[i + D i] of a D x D result (column-major), v[0] for one column
static double trace_of(const std::vector<double>& v, int Da, int Db) {
  if (v.empty()) return 0.0;
  if (Da != Db) fail(PV_EINVAL, "inner product of MPS with different numbers of columns");
  double t = 0.0;
  for (int i = 0; i < Da; ++i) t += v[size_t(i) + size_t(Da) * i];
  return t;
}

double dot(Ctx& c, const Mps& a, const Mps& b) {
  auto v = env_sweep(c, a, b, identity_mpo(c, a.L));
  return trace_of(v, a.rho[a.L][a.N], b.rho[b.L][b.N]);
}

std::vector<double> dot_matrix(Ctx& c, const Mps& a, const Mps& b) {
  return env_sweep(c, a, b, identity_mpo(c, a.L));
}

std::vector<double> expect_matrix(Ctx& c, const Mps& bra, const Mps& ket) {
  if (!c.hmpo) fail(PV_ESTATE, "no Hamiltonian set");
  return env_sweep(c, bra, ket, *c.hmpo);
}

// x with its column index transformed: the last core's blocks times W (Din x Dout,
// column-major, host): column j of the result is sum_i W_ij (column i of x).
std::unique_ptr<Mps> mps_index_transform(Ctx& c, const Mps& x, const std::vector<double>& W, int Dout) {
  const int L = x.L, N = x.N, Din = x.rho[L][N];
  if (int64_t(W.size()) != int64_t(Din) * Dout) fail(PV_EINVAL, "index transform of the wrong size");
  auto rho = x.rho;
  rho[L][N] = Dout;
  auto y = mps_alloc(c, L, N, rho);
  CopyBatch cb;
  for (int k = 1; k < L; ++k) cb.add(x.site[k - 1].p, 1, y->site[k - 1].p, 1, int(x.site_size(k)), 1, 1.0);
  cb.run(c);
  Buf w(c.pool, W.size());
  PV_HIP(hipMemcpyAsync(w.p, W.data(), W.size() * 8, hipMemcpyHostToDevice, c.stream));
  GemmBatch g;
  CopyBatch zero;
  for (int n = 0; n <= N; ++n) {
    if (!x.valid(L - 1, n)) continue;
    const int r = x.rows(L, n);
    if (r == 0) continue;
    if (y->ucols(L, n)) g.add(x.U(L, n), r, 0, w.p, Din, 0, y->U(L, n), r, r, Dout, Din, 1.0, 0.0);
    if (y->ocols(L, n)) g.add(x.O(L, n), r, 0, w.p, Din, 0, y->O(L, n), r, r, Dout, Din, 1.0, 0.0);
  }
  g.run(c);
  c.sync();  // the host W goes out of scope with the caller
  c.scratch.push_back(std::move(w));
  return y;
}

double expect_h(Ctx& c, const Mps& bra, const Mps& ket) {
  if (!c.hmpo) fail(PV_ESTATE, "no Hamiltonian set");
  auto v = env_sweep(c, bra, ket, *c.hmpo);
  return trace_of(v, bra.rho[bra.L][bra.N], ket.rho[ket.L][ket.N]);
}

// ---- overlapped sweeps: an auxiliary context (pool, staging, timers) on a stream of its own
static Ctx& aux_ctx(Ctx& c) {
  if (!c.aux) {
    auto a = std::make_unique<Ctx>();
    a->device = c.device;
    a->use_side = false;
    PV_HIP(hipStreamCreate(&a->stream));
    c.aux = std::move(a);
    c.aux->staging.init(size_t(64) << 20);
    PV_HIP(hipEventCreateWithFlags(&c.aux_ready, hipEventDisableTiming));
  }
  return *c.aux;
}

void expect_h_drain(Ctx& c) noexcept {
  if (!c.aux_pending) return;
  c.aux_pending = false;
  if (!c.aux_inline && c.aux) {
    try {
      c.aux->sync();
    } catch (...) {
      (void)hipStreamSynchronize(c.aux->stream);
    }
  }
}

void expect_h_begin(Ctx& c, const Mps& bra, const Mps& ket) {
  if (!c.hmpo) fail(PV_ESTATE, "no Hamiltonian set");
  expect_h_drain(c);
  c.aux_da = bra.rho[bra.L][bra.N];
  c.aux_db = ket.rho[ket.L][ket.N];
  if (!c.use_side) {
    // contexts sharing the device from several host threads: the sweep runs in place
    c.aux_value = expect_h(c, bra, ket);
    c.aux_inline = true;
    c.aux_pending = true;
    return;
  }
  Ctx& a = aux_ctx(c);
  a.prec = c.prec;
  a.lowp = c.lowp;
  a.trunc_mode = c.trunc_mode;
  a.timer_mask = c.timer_mask;
  a.gemm_tiles = c.gemm_tiles;
  a.sample_mask = c.sample_mask;
  a.sample_every = c.sample_every;
  // the operands are complete once the main stream's work so far is
  PV_HIP(hipEventRecord(c.aux_ready, c.stream));
  PV_HIP(hipStreamWaitEvent(a.stream, c.aux_ready, 0));
  c.aux_inline = false;
  c.aux_pending = true;
  EnvEnd r = env_sweep_dev(a, bra, ket, *c.hmpo);
  const size_t n = size_t(r.rows * r.cols);
  if (n > c.aux_host_n) {
    a.sync();
    if (c.aux_host) PV_HIP(hipHostFree(c.aux_host));
    c.aux_host = nullptr;
    c.aux_host_n = 0;
    void* h = nullptr;
    PV_HIP(hipHostMalloc(&h, n * sizeof(double), hipHostMallocDefault));
    c.aux_host = static_cast<double*>(h);
    c.aux_host_n = n;
  }
  c.aux_n = n;
  if (n) PV_HIP(hipMemcpyAsync(c.aux_host, r.res, n * sizeof(double), hipMemcpyDeviceToHost, a.stream));
  a.scratch.push_back(std::move(r.E));
}

double expect_h_end(Ctx& c) {
  if (!c.aux_pending) fail(PV_ESTATE, "no overlapped sweep is running");
  c.aux_pending = false;
  if (c.aux_inline) return c.aux_value;
  Ctx& a = *c.aux;
  a.sync();
  for (int k = 0; k < T_COUNT; ++k) {
    c.t_ms[k] += a.t_ms[k];
    c.t_flops[k] += a.t_flops[k];
    c.t_bytes[k] += a.t_bytes[k];
    c.t_calls[k] += a.t_calls[k];
    a.t_ms[k] = a.t_flops[k] = a.t_bytes[k] = 0.0;
    a.t_calls[k] = 0;
  }
  std::vector<double> v(c.aux_host, c.aux_host + c.aux_n);
  return trace_of(v, c.aux_da, c.aux_db);
}

void release_aux(Ctx& c) noexcept {
  expect_h_drain(c);
  if (c.aux) {
    Ctx& a = *c.aux;
    (void)hipStreamSynchronize(a.stream);
    for (auto e : a.event_pool) (void)hipEventDestroy(e);
    for (auto& p : a.pending) { (void)hipEventDestroy(p.a); (void)hipEventDestroy(p.b); }
    a.event_pool.clear();
    a.pending.clear();
    a.scratch.clear();
    hipStream_t s = a.stream;
    c.aux.reset();
    if (s) (void)hipStreamDestroy(s);
  }
  if (c.aux_ready) (void)hipEventDestroy(c.aux_ready);
  c.aux_ready = nullptr;
  if (c.aux_host) (void)hipHostFree(c.aux_host);
  c.aux_host = nullptr;
  c.aux_host_n = 0;
  if (c.dl_host) (void)hipHostFree(c.dl_host);
  c.dl_host = nullptr;
  c.dl_n = 0;
}

void sym_eig_tridiag_device(Ctx& c, int n, const double* A, double* w, double* V, double* work, EigDesc* desc) {
  std::vector<EigDesc> tri{EigDesc{A, n, n, V, w, work, nullptr, kVecCut, n}};
  if (!c.staging.fits(sizeof(EigDesc))) c.sync();
  void* host = c.staging.put(tri.data(), sizeof(EigDesc));
  PV_HIP(hipMemcpyAsync(desc, host, sizeof(EigDesc), hipMemcpyHostToDevice, c.stream));
  tri_values(c, tri, desc, n, 2.0 / 3.0 * double(n) * n * n, 4.0 / 3.0 * double(n) * n * n);
  tri_vectors(c, tri, desc, n);
  c.sync();
}

void sym_eig(Ctx& c, int n, const double* A_host, double* w_host, double* V_host, int method, int nvec) {
  Buf A(c.pool, size_t(n) * n), V(c.pool, size_t(n) * n), w(c.pool, size_t(n));
  PV_HIP(hipMemcpyAsync(A.p, A_host, size_t(n) * n * 8, hipMemcpyHostToDevice, c.stream));
  std::vector<EigJob> jobs{EigJob{A.p, n, n, V.p, w.p, method == 1 ? kVecCut : kAbsTolGeneral, method == 1}};
  jobs[0].force = method == 1;
  if (method == 1 && nvec >= 0) {
    EigPlan plan = run_eig_values(c, jobs);
    std::vector<int> nv{nvec};
    run_eig_vectors(c, plan, &nv);
  } else {
    run_eig(c, jobs);
  }
  PV_HIP(hipMemcpyAsync(w_host, w.p, size_t(n) * 8, hipMemcpyDeviceToHost, c.stream));
  PV_HIP(hipMemcpyAsync(V_host, V.p, size_t(n) * n * 8, hipMemcpyDeviceToHost, c.stream));
  c.sync();
}

void gemm_host(Ctx& c, int M, int N, int K, const double* A_host, int lda, int ta, const double* B_host, int ldb,
               int tb, double* C_host, int ldc, double alpha, double beta, int precision) {
  const size_t na = size_t(lda) * (ta ? M : K), nb = size_t(ldb) * (tb ? K : N), nc = size_t(ldc) * N;
  Buf A(c.pool, std::max<size_t>(na, 1)), B(c.pool, std::max<size_t>(nb, 1)), C(c.pool, std::max<size_t>(nc, 1));
  if (na) PV_HIP(hipMemcpyAsync(A.p, A_host, na * 8, hipMemcpyHostToDevice, c.stream));
  if (nb) PV_HIP(hipMemcpyAsync(B.p, B_host, nb * 8, hipMemcpyHostToDevice, c.stream));
  PV_HIP(hipMemcpyAsync(C.p, C_host, nc * 8, hipMemcpyHostToDevice, c.stream));
  GemmBatch g;
  g.prec = precision == 2 ? 3 : precision;
  g.add(A.p, lda, ta, B.p, ldb, tb, C.p, ldc, M, N, K, alpha, beta);
  g.run(c);
  PV_HIP(hipMemcpyAsync(C_host, C.p, nc * 8, hipMemcpyDeviceToHost, c.stream));
  c.sync();
}

void cholesky(Ctx& c, int n, const double* A_host, double* W_host) {
  Buf A(c.pool, size_t(n) * n), W(c.pool, size_t(n) * n);
  PV_HIP(hipMemcpyAsync(A.p, A_host, size_t(n) * n * 8, hipMemcpyHostToDevice, c.stream));
  chol_all(c, {CholJob{A.p, n, W.p}});
  PV_HIP(hipMemcpyAsync(W_host, W.p, size_t(n) * n * 8, hipMemcpyDeviceToHost, c.stream));
  c.sync();
}

double norm2(Ctx& c, const Mps& x) { return std::sqrt(std::max(dot(c, x, x), 0.0)); }

double norm_canonical(Ctx& c, const Mps& x) {
  // left-orthogonal MPS: the norm is the Frobenius norm of the last core
  Buf out(c.pool, 1);
  hipEvent_t a; c.begin(T_REDUCE, a);
  launch_sumsq(x.site[x.L - 1].p, x.site_size(x.L), out.p, c.stream);
  c.end(T_REDUCE, a, 0, 8.0 * x.site_size(x.L));
  auto h = download(c, out.p, 1);
  return std::sqrt(h[0]);
}

// ---------------------------------------------------------------- simple constructions
std::unique_ptr<Mps> mps_determinant(Ctx& c, const std::vector<int>& occ) {
  const int L = c.L, N = c.N;
  std::vector<char> o(L, 0);
  for (int i : occ) o[i] = 1;
  auto rho = empty_rho(L, N);
  int n = 0;
  rho[0][0] = 1;
  for (int k = 1; k <= L; ++k) {
    n += o[k - 1];
    rho[k][n] = 1;
  }
  auto m = mps_alloc(c, L, N, rho);
  for (int k = 1; k <= L; ++k) fill(c, m->site[k - 1].p, m->site_size(k), 1.0);
  return m;
}

// The zero state in the layout of x: every core cleared, so that the norm read from the
// last core (the norm of a left-orthogonal chain) is zero as well.
std::unique_ptr<Mps> mps_zero_like(Ctx& c, const Mps& x) {
  auto m = mps_alloc(c, x.L, x.N, x.rho);
  CopyBatch zero;
  for (int k = 1; k <= x.L; ++k) zero.add_fill(m->site[k - 1].p, m->site_size(k), 0.0);
  zero.run(c);
  return m;
}

// a x with the occupied block of site k in left sector n scaled by occ[(k-1)(N+1) + n]
std::unique_ptr<Mps> mps_sector_scaled_copy(Ctx& c, const Mps& x, double a, const double* occ) {
  auto m = mps_alloc(c, x.L, x.N, x.rho);
  CopyBatch cb;
  for (int k = 1; k <= x.L; ++k)
    for (int n = 0; n <= x.N; ++n) {
      if (!x.valid(k - 1, n)) continue;
      const int r = x.rows(k, n);
      const double f = k == 1 ? a : 1.0;
      cb.add(x.U(k, n), r, m->U(k, n), r, r, x.ucols(k, n), f);
      cb.add(x.O(k, n), r, m->O(k, n), r, r, x.ocols(k, n), f * occ[size_t(k - 1) * (x.N + 1) + n]);
    }
  cb.run(c);
  return m;
}

std::unique_ptr<Mps> mps_scaled_copy(Ctx& c, const Mps& x, double a, const double* occ_scale) {
  auto m = mps_alloc(c, x.L, x.N, x.rho);
  CopyBatch cb;
  for (int k = 1; k <= x.L; ++k)
    for (int n = 0; n <= x.N; ++n) {
      if (!x.valid(k - 1, n)) continue;
      const int r = x.rows(k, n);
      const double f = k == 1 ? a : 1.0;
      cb.add(x.U(k, n), r, m->U(k, n), r, r, x.ucols(k, n), f);
      cb.add(x.O(k, n), r, m->O(k, n), r, r, x.ocols(k, n), f * (occ_scale ? occ_scale[k - 1] : 1.0));
    }
  cb.run(c);
  return m;
}

// a x + b y by concatenation of blocks (Section 2.3).  With index_concat the right
// boundaries (column indices of joint MPS) are concatenated too: the last cores go block
// diagonal and the result holds the columns of x followed by those of y (Section 6.2).
std::unique_ptr<Mps> mps_lincomb(Ctx& c, double a, const Mps& x, double b, const Mps& y, bool index_concat) {
  const int L = x.L, N = x.N;
  if (y.L != L || y.N != N) fail(PV_EINVAL, "lincomb: mismatched chains");
  if (!index_concat && x.rho[L][N] != y.rho[L][N]) fail(PV_EINVAL, "lincomb: different numbers of columns");
  auto rho = empty_rho(L, N);
  for (int k = 0; k <= L; ++k)
    for (int n = 0; n <= N; ++n)
      if (x.valid(k, n))
        rho[k][n] = k == 0 ? 1 : k < L ? x.rho[k][n] + y.rho[k][n] : index_concat ? x.rho[k][n] + y.rho[k][n] : x.rho[k][n];
  auto m = mps_alloc(c, L, N, rho);
  CopyBatch zero, cb;  // every site cleared in one launch, then the blocks copied in
  for (int k = 1; k <= L; ++k) zero.add_fill(m->site[k - 1].p, m->site_size(k), 0.0);
  zero.run(c);
  for (int k = 1; k <= L; ++k) {
    for (int n = 0; n <= N; ++n) {
      if (!x.valid(k - 1, n)) continue;
      const int R = m->rows(k, n);
      const int rx = x.rows(k, n), ry = y.rows(k, n);
      const int rx0 = (k == 1) ? 0 : 0, ry0 = (k == 1) ? 0 : rx;  // row offset of y part
      const double fx = k == 1 ? a : 1.0, fy = k == 1 ? b : 1.0;
      for (int kind = 0; kind < 2; ++kind) {
        const int cx = kind ? x.ocols(k, n) : x.ucols(k, n);
        const int cy = kind ? y.ocols(k, n) : y.ucols(k, n);
        if (cx + cy == 0 && (kind ? m->ocols(k, n) : m->ucols(k, n)) == 0) continue;
        double* dst = kind ? m->O(k, n) : m->U(k, n);
        const double* sx = kind ? x.O(k, n) : x.U(k, n);
        const double* sy = kind ? y.O(k, n) : y.U(k, n);
        const int cy0 = (k == L && !index_concat) ? 0 : cx;  // column offset of y part
        cb.add(sx, rx, dst + rx0, R, rx, cx, fx);
        cb.add(sy, ry, dst + ry0 + int64_t(R) * cy0, R, ry, cy, fy);
      }
    }
  }
  cb.run(c);
  return m;
}

// ---------------------------------------------------------------- factorisations
namespace {

// Two-pass Gram eigendecomposition of the Gram matrices G_s (n_s x n_s, ld n_s) of a set
// of sectors.  Pass 1: G = W1 L1 W1^T.  The caller forms Y = rotated data and its Gram
// G2, pass 2 gives W2 and the singular values as sqrt of its eigenvalues.
struct SectorEig {
  int n = 0;
  Buf G, W, w;
};

void eig_all(Ctx& c, std::vector<SectorEig>& se, double abs_tol, bool tridiag = false) {
  std::vector<EigJob> jobs;
  for (auto& s : se) {
    if (s.n <= 0) continue;
    s.W = Buf(c.pool, size_t(s.n) * s.n);
    s.w = Buf(c.pool, size_t(s.n));
    jobs.push_back(EigJob{s.G.p, s.n, s.n, s.W.p, s.w.p, abs_tol, tridiag});
  }
  run_eig(c, jobs);
}

std::vector<std::vector<double>> sigmas(Ctx& c, std::vector<SectorEig>& se) {
  int64_t tot = 0;
  for (auto& s : se) tot += s.n;
  Buf all(c.pool, size_t(std::max<int64_t>(tot, 1)));
  CopyBatch cb;
  int64_t o = 0;
  for (auto& s : se) {
    cb.add(s.w.p, s.n, all.p + o, s.n, s.n, 1, 1.0);
    o += s.n;
  }
  cb.run(c);
  auto h = download(c, all.p, size_t(tot));
  std::vector<std::vector<double>> out(se.size());
  o = 0;
  for (size_t i = 0; i < se.size(); ++i) {
    out[i].resize(se[i].n);
    for (int j = 0; j < se[i].n; ++j) out[i][j] = std::sqrt(std::max(h[o + j], 0.0));
    o += se[i].n;
  }
  return out;
}

// Single-pass factorisation: the second pass is the identity (W2 = I, same eigenvalues).
void identity_pass(Ctx& c, std::vector<SectorEig>& se, std::vector<SectorEig>& se2) {
  CopyBatch zero, cb;  // W2 = 0 in one launch, then the unit diagonals and the eigenvalues
  for (size_t i = 0; i < se.size(); ++i) {
    const int r = se[i].n;
    se2[i].n = r;
    if (r == 0) continue;
    se2[i].W = Buf(c.pool, size_t(r) * r);
    se2[i].w = Buf(c.pool, size_t(r));
    zero.add_fill(se2[i].W.p, int64_t(r) * r, 0.0);
    cb.add(se[i].w.p, r, se2[i].w.p, r, r, 1, 1.0);
    cb.add_fill_strided(se2[i].W.p, r + 1, r, 1.0);  // unit diagonal (stride r + 1)
  }
  zero.run(c);
  cb.run(c);
}


}  // namespace

// Right-orthogonalisation R->L (site k = L..2): per left sector n of site k the block
// C = [U|O] is factored as C = R Q with orthonormal rows Q through the two-pass Gram
// eigendecomposition of C C^T; R is multiplied into site k-1.  Directions with
// sigma <= kZeroTol * sigma_max are dropped.
static std::unique_ptr<Mps> orthogonalize_right(Ctx& c, const Mps& x, bool two_pass) {
  const int L = x.L, N = x.N;
  auto y = mps_alloc(c, L, N, x.rho);
  {
    CopyBatch cb;
    for (int k = 1; k <= L; ++k) cb.add(x.site[k - 1].p, 1, y->site[k - 1].p, 1, int(x.site_size(k)), 1, 1.0);
    cb.run(c);
  }
  for (int k = L; k >= 2; --k) {
    std::vector<SectorEig> se(N + 1);
    std::vector<int> cols(N + 1, 0);
    GemmBatch g;
    for (int n = 0; n <= N; ++n) {
      if (!y->valid(k - 1, n)) continue;
      const int r = y->rows(k, n);
      cols[n] = y->ucols(k, n) + y->ocols(k, n);
      if (r == 0 || cols[n] == 0) continue;
      se[n].n = r;
      se[n].G = Buf(c.pool, size_t(r) * r);
      g.add(y->U(k, n), r, 0, y->U(k, n), r, 1, se[n].G.p, r, r, r, cols[n], 1.0, 0.0);
    }
    g.run(c);
    eig_all(c, se, kAbsTolGeneral, !two_pass);
    // pass 2: Y = W1^T C, G2 = Y Y^T (single pass: W2 = I, eigenvalues of pass 1)
    std::vector<Buf> Y(N + 1);
    std::vector<SectorEig> se2(N + 1);
    for (int n = 0; n <= N; ++n) {
      if (se[n].n == 0) continue;
      const int r = se[n].n;
      Y[n] = Buf(c.pool, size_t(r) * cols[n]);
      g.add(se[n].W.p, r, 1, y->U(k, n), r, 0, Y[n].p, r, r, cols[n], r, 1.0, 0.0);
    }
    g.run(c);
    if (two_pass) {
      for (int n = 0; n <= N; ++n) {
        if (se[n].n == 0) continue;
        const int r = se[n].n;
        se2[n].n = r;
        se2[n].G = Buf(c.pool, size_t(r) * r);
        g.add(Y[n].p, r, 0, Y[n].p, r, 1, se2[n].G.p, r, r, r, cols[n], 1.0, 0.0);
      }
      g.run(c);
      eig_all(c, se2, kAbsTolRefine);
    } else {
      identity_pass(c, se, se2);
    }
    auto sig = sigmas(c, se2);
    double smax = 0;
    for (auto& v : sig) for (double s : v) smax = std::max(smax, s);
    const double ztol = two_pass ? kZeroTol : kZeroTolPar;
    std::vector<int> keep(N + 1, 0);
    for (int n = 0; n <= N; ++n)
      for (double s : sig[n]) keep[n] += s > ztol * smax;
    // new ranks on bond k-1
    auto rho = y->rho;
    for (int n = 0; n <= N; ++n)
      if (y->valid(k - 1, n)) rho[k - 1][n] = keep[n];
    // keep at least one direction on a nonzero bond
    int tot = 0;
    for (int n = 0; n <= N; ++n) tot += keep[n];
    auto z = std::make_unique<Mps>();
    z->L = L; z->N = N; z->rho = rho;
    z->site.resize(L); z->off.resize(L);
    for (int kk = 1; kk <= L; ++kk) {
      if (kk == k || kk == k - 1) { alloc_site(c, *z, kk); }
      else { layout_site(*z, kk); z->site[kk - 1] = std::move(y->site[kk - 1]); }
    }
    (void)tot;
    // W2s = W2[:, :s] / sigma  and  R = W1 W2[:, :s] sigma
    ScaleBatch sb;
    std::vector<Buf> W2inv(N + 1), W2sig(N + 1), R(N + 1);
    for (int n = 0; n <= N; ++n) {
      const int s = keep[n], r = se[n].n;
      if (s == 0) continue;
      W2inv[n] = Buf(c.pool, size_t(r) * s);
      W2sig[n] = Buf(c.pool, size_t(r) * s);
      sb.add(se2[n].W.p, r, W2inv[n].p, r, r, s, se2[n].w.p, true, true);
      sb.add(se2[n].W.p, r, W2sig[n].p, r, r, s, se2[n].w.p, false, true);
    }
    sb.run(c);
    for (int n = 0; n <= N; ++n) {
      const int s = keep[n], r = se[n].n;
      if (s == 0) continue;
      // Q = W2inv^T Y -> new site k block, rows s
      g.add(W2inv[n].p, r, 1, Y[n].p, r, 0, z->U(k, n), s, s, cols[n], r, 1.0, 0.0);
      R[n] = Buf(c.pool, size_t(r) * s);
      g.add(se[n].W.p, r, 0, W2sig[n].p, r, 0, R[n].p, r, r, s, r, 1.0, 0.0);
    }
    g.run(c);
    // site k-1: U(k-1,n) R_n and O(k-1,n) R_{n+1}
    for (int n = 0; n <= N; ++n) {
      if (!y->valid(k - 2, n)) continue;
      const int rr = y->rows(k - 1, n);
      if (rr == 0) continue;
      if (y->ucols(k - 1, n) > 0 && keep[n] > 0)
        g.add(y->U(k - 1, n), rr, 0, R[n].p, se[n].n, 0, z->U(k - 1, n), rr, rr, keep[n], se[n].n, 1.0, 0.0);
      if (y->ocols(k - 1, n) > 0 && n + 1 <= N && keep[n + 1] > 0)
        g.add(y->O(k - 1, n), rr, 0, R[n + 1].p, se[n + 1].n, 0, z->O(k - 1, n), rr, rr, keep[n + 1], se[n + 1].n, 1.0, 0.0);
    }
    g.run(c);
    for (auto& b : Y) c.scratch.push_back(std::move(b));
    for (auto& b : R) c.scratch.push_back(std::move(b));
    for (auto& b : W2inv) c.scratch.push_back(std::move(b));
    for (auto& b : W2sig) c.scratch.push_back(std::move(b));
    for (auto& s : se) { c.scratch.push_back(std::move(s.G)); c.scratch.push_back(std::move(s.W)); c.scratch.push_back(std::move(s.w)); }
    for (auto& s : se2) { c.scratch.push_back(std::move(s.G)); c.scratch.push_back(std::move(s.W)); c.scratch.push_back(std::move(s.w)); }
    c.scratch.push_back(std::move(y->site[k - 1]));
    c.scratch.push_back(std::move(y->site[k - 2]));
    y = std::move(z);
  }
  return y;
}

// Left-to-right truncation of a right-orthogonal MPS: at cut k the left-fused blocks
// M_n = [U_{k,n}; O_{k,n-1}] are factored through the two-pass Gram eigendecomposition
// of M^T M, ranks are selected across sectors, the kept left singular vectors form the
// new core and Sigma V^T is multiplied into site k+1.
static std::unique_ptr<Mps> truncate_ltr(Ctx& c, std::unique_ptr<Mps> y, double eps, int cap,
                                         bool* cap_bound) {
  const int L = y->L, N = y->N;
  const double delta = L > 1 ? eps / std::sqrt(double(L - 1)) : eps;
  for (int k = 1; k <= L - 1; ++k) {
    std::vector<SectorEig> se(N + 1), se2(N + 1);
    std::vector<int> r0(N + 1, 0), r1(N + 1, 0);
    GemmBatch g, g1;
    for (int n = 0; n <= N; ++n) {
      if (!y->valid(k, n)) continue;
      const int rk = y->rho[k][n];
      r0[n] = y->valid(k - 1, n) ? y->ucols(k, n) > 0 ? y->rows(k, n) : 0 : 0;
      r1[n] = (n >= 1 && y->valid(k - 1, n - 1) && y->ocols(k, n - 1) > 0) ? y->rows(k, n - 1) : 0;
      if (rk == 0 || r0[n] + r1[n] == 0) continue;
      se[n].n = rk;
      se[n].G = Buf(c.pool, size_t(rk) * rk);
      // the first product overwrites G (beta 0), the second accumulates
      if (r0[n]) g.add(y->U(k, n), r0[n], 1, y->U(k, n), r0[n], 0, se[n].G.p, rk, rk, rk, r0[n], 1.0, 0.0);
      if (r1[n])
        g1.add(y->O(k, n - 1), r1[n], 1, y->O(k, n - 1), r1[n], 0, se[n].G.p, rk, rk, rk, r1[n], 1.0, r0[n] ? 1.0 : 0.0);
    }
    g.run(c);
    g1.run(c);
    eig_all(c, se, kAbsTolGeneral);
    // Y = M W1 (stacked rows r0 + r1), G2 = Y^T Y
    std::vector<Buf> Y(N + 1);
    for (int n = 0; n <= N; ++n) {
      if (se[n].n == 0) continue;
      const int rk = se[n].n, R = r0[n] + r1[n];
      Y[n] = Buf(c.pool, size_t(R) * rk);
      if (r0[n]) g.add(y->U(k, n), r0[n], 0, se[n].W.p, rk, 0, Y[n].p, R, r0[n], rk, rk, 1.0, 0.0);
      if (r1[n]) g.add(y->O(k, n - 1), r1[n], 0, se[n].W.p, rk, 0, Y[n].p + r0[n], R, r1[n], rk, rk, 1.0, 0.0);
    }
    g.run(c);
    for (int n = 0; n <= N; ++n) {
      if (se[n].n == 0) continue;
      const int rk = se[n].n, R = r0[n] + r1[n];
      se2[n].n = rk;
      se2[n].G = Buf(c.pool, size_t(rk) * rk);
      g.add(Y[n].p, R, 1, Y[n].p, R, 0, se2[n].G.p, rk, rk, rk, R, 1.0, 0.0);
    }
    g.run(c);
    eig_all(c, se2, kAbsTolRefine);
    auto sig = sigmas(c, se2);
    std::vector<std::vector<double>> sig_all(N + 1);
    for (int n = 0; n <= N; ++n) sig_all[n] = sig[n];
    std::vector<int> keep = select_ranks(sig_all, delta, cap, cap_bound);
    auto rho = y->rho;
    for (int n = 0; n <= N; ++n)
      if (y->valid(k, n)) rho[k][n] = keep[n];
    auto z = std::make_unique<Mps>();
    z->L = L; z->N = N; z->rho = rho;
    z->site.resize(L); z->off.resize(L);
    for (int kk = 1; kk <= L; ++kk) {
      if (kk == k || kk == k + 1) alloc_site(c, *z, kk);
      else { layout_site(*z, kk); z->site[kk - 1] = std::move(y->site[kk - 1]); }
    }
    ScaleBatch sb;
    std::vector<Buf> W2inv(N + 1), W2sig(N + 1), V(N + 1);
    for (int n = 0; n <= N; ++n) {
      const int s = keep[n], rk = se[n].n;
      if (s == 0 || rk == 0) continue;
      W2inv[n] = Buf(c.pool, size_t(rk) * s);
      W2sig[n] = Buf(c.pool, size_t(rk) * s);
      sb.add(se2[n].W.p, rk, W2inv[n].p, rk, rk, s, se2[n].w.p, true, true);
      sb.add(se2[n].W.p, rk, W2sig[n].p, rk, rk, s, se2[n].w.p, false, true);
    }
    sb.run(c);
    for (int n = 0; n <= N; ++n) {
      const int s = keep[n], rk = se[n].n, R = r0[n] + r1[n];
      if (s == 0 || rk == 0) continue;
      if (r0[n]) g.add(Y[n].p, R, 0, W2inv[n].p, rk, 0, z->U(k, n), z->rows(k, n), r0[n], s, rk, 1.0, 0.0);
      if (r1[n]) g.add(Y[n].p + r0[n], R, 0, W2inv[n].p, rk, 0, z->O(k, n - 1), z->rows(k, n - 1), r1[n], s, rk, 1.0, 0.0);
      V[n] = Buf(c.pool, size_t(rk) * s);
      g1.add(se[n].W.p, rk, 0, W2sig[n].p, rk, 0, V[n].p, rk, rk, s, rk, 1.0, 0.0);
    }
    g.run(c);
    g1.run(c);
    // site k+1: rows of left sector n become (Sigma V^T) [U|O]
    for (int n = 0; n <= N; ++n) {
      if (!y->valid(k, n) || keep[n] == 0 || se[n].n == 0) continue;
      const int cols = y->ucols(k + 1, n) + y->ocols(k + 1, n);
      if (cols == 0) continue;
      g.add(V[n].p, se[n].n, 1, y->U(k + 1, n), y->rows(k + 1, n), 0, z->U(k + 1, n), keep[n], keep[n], cols,
            se[n].n, 1.0, 0.0);
    }
    g.run(c);
    for (auto& b : Y) c.scratch.push_back(std::move(b));
    for (auto& b : V) c.scratch.push_back(std::move(b));
    for (auto& b : W2inv) c.scratch.push_back(std::move(b));
    for (auto& b : W2sig) c.scratch.push_back(std::move(b));
    for (auto& s : se) { c.scratch.push_back(std::move(s.G)); c.scratch.push_back(std::move(s.W)); c.scratch.push_back(std::move(s.w)); }
    for (auto& s : se2) { c.scratch.push_back(std::move(s.G)); c.scratch.push_back(std::move(s.W)); c.scratch.push_back(std::move(s.w)); }
    c.scratch.push_back(std::move(y->site[k - 1]));
    c.scratch.push_back(std::move(y->site[k]));
    y = std::move(z);
  }
  return y;
}

std::unique_ptr<Mps> round_mps(Ctx& c, const Mps& x, double eps, int cap, bool* cap_bound) {
  if (c.trunc_mode == 1) return round_parallel(c, x, eps, cap, cap_bound);
  auto y = orthogonalize_right(c, x, true);
  return truncate_ltr(c, std::move(y), eps, cap, cap_bound);
}

// ---------------------------------------------------------------- simultaneous truncation
// Gram matrices of the left parts (G^L_k = A_k^T A_k, by a left-to-right GEMM sweep) and of
// the right parts (G^R_k = B_k B_k^T, right-to-left) of every bond, one entry per sector.
namespace {

struct BondGrams {
  std::vector<std::vector<int64_t>> off;  // off[k][n] into buf, -1 if empty
  Buf buf;
};

BondGrams alloc_grams(Ctx& c, const Mps& x) {
  BondGrams g;
  g.off.assign(x.L + 1, std::vector<int64_t>(x.N + 1, -1));
  int64_t tot = 0;
  for (int k = 0; k <= x.L; ++k)
    for (int n = 0; n <= x.N; ++n)
      if (x.valid(k, n) && x.rho[k][n] > 0) {
        g.off[k][n] = tot;
        tot += int64_t(x.rho[k][n]) * x.rho[k][n];
      }
  g.buf = Buf(c.pool, size_t(std::max<int64_t>(tot, 1)));
  return g;
}

BondGrams left_grams(Ctx& c, const Mps& x) {
  const int L = x.L, N = x.N;
  BondGrams g = alloc_grams(c, x);
  fill(c, g.buf.p, int64_t(g.buf.n), 0.0);
  fill(c, g.buf.p + g.off[0][0], 1, 1.0);
  for (int k = 1; k < L; ++k) {
    std::vector<Buf> T(N + 1);
    GemmBatch gb, g0, g1;
    for (int n = 0; n <= N; ++n) {
      if (!x.valid(k - 1, n) || g.off[k - 1][n] < 0) continue;
      const int r = x.rows(k, n), cols = x.ucols(k, n) + x.ocols(k, n);
      if (r == 0 || cols == 0) continue;
      T[n] = Buf(c.pool, size_t(r) * cols);
      gb.add(g.buf.p + g.off[k - 1][n], r, 0, x.U(k, n), r, 0, T[n].p, r, r, cols, r, 1.0, 0.0);
    }
    gb.run(c);
    for (int n = 0; n <= N; ++n) {
      if (g.off[k][n] < 0) continue;
      const int rk = x.rho[k][n];
      double* G = g.buf.p + g.off[k][n];
      if (T[n].p && x.ucols(k, n) > 0)
        g0.add(x.U(k, n), x.rows(k, n), 1, T[n].p, x.rows(k, n), 0, G, rk, rk, rk, x.rows(k, n), 1.0, 1.0);
      if (n >= 1 && T[n - 1].p && x.ocols(k, n - 1) > 0) {
        const int r = x.rows(k, n - 1);
        g1.add(x.O(k, n - 1), r, 1, T[n - 1].p + int64_t(r) * x.ucols(k, n - 1), r, 0, G, rk, rk, rk, r, 1.0, 1.0);
      }
    }
    g0.run(c);
    g1.run(c);
    for (auto& b : T) c.scratch.push_back(std::move(b));
  }
  return g;
}

BondGrams right_grams(Ctx& c, const Mps& x) {
  const int L = x.L, N = x.N;
  BondGrams g = alloc_grams(c, x);
  fill(c, g.buf.p, int64_t(g.buf.n), 0.0);
  {
    // identity over the right boundary (the column index of a joint MPS, else 1 x 1)
    CopyBatch one;
    one.add_fill_strided(g.buf.p + g.off[L][N], x.rho[L][N] + 1, x.rho[L][N], 1.0);
    one.run(c);
  }
  for (int k = L; k >= 2; --k) {
    std::vector<Buf> T(N + 1);
    GemmBatch gb, g2;
    for (int n = 0; n <= N; ++n) {
      if (!x.valid(k - 1, n) || g.off[k - 1][n] < 0) continue;
      const int r = x.rows(k, n), cu = x.ucols(k, n), co = x.ocols(k, n);
      if (r == 0 || cu + co == 0) continue;
      T[n] = Buf(c.pool, size_t(r) * (cu + co));
      if (cu) gb.add(x.U(k, n), r, 0, g.buf.p + g.off[k][n], cu, 0, T[n].p, r, r, cu, cu, 1.0, 0.0);
      if (co) gb.add(x.O(k, n), r, 0, g.buf.p + g.off[k][n + 1], co, 0, T[n].p + int64_t(r) * cu, r, r, co, co, 1.0, 0.0);
      g2.add(T[n].p, r, 0, x.U(k, n), r, 1, g.buf.p + g.off[k - 1][n], r, r, r, cu + co, 1.0, 0.0);
    }
    gb.run(c);
    g2.run(c);
    for (auto& b : T) c.scratch.push_back(std::move(b));
  }
  return g;
}

struct BondEig {
  std::vector<std::vector<int64_t>> voff, woff;  // per (k, n)
  Buf V, w;
};

// Eigendecompositions of the Gram matrices of bonds kmin..kmax, one batched launch.  With
// `values_only` the tridiagonal problems stop after their eigenvalues; their vectors come
// from run_eig_vectors on the returned plan (job order: bonds ascending, sectors ascending).
BondEig eig_grams(Ctx& c, const Mps& x, const BondGrams& g, int kmin, int kmax, EigPlan* values_only = nullptr) {
  BondEig e;
  e.voff.assign(x.L + 1, std::vector<int64_t>(x.N + 1, -1));
  e.woff = e.voff;
  int64_t tv = 0, tw = 0;
  for (int k = kmin; k <= kmax; ++k)
    for (int n = 0; n <= x.N; ++n)
      if (g.off[k][n] >= 0) {
        const int r = x.rho[k][n];
        e.voff[k][n] = tv; e.woff[k][n] = tw;
        tv += int64_t(r) * r; tw += r;
      }
  e.V = Buf(c.pool, size_t(std::max<int64_t>(tv, 1)));
  e.w = Buf(c.pool, size_t(std::max<int64_t>(tw, 1)));
  std::vector<EigJob> jobs;
  for (int k = kmin; k <= kmax; ++k)
    for (int n = 0; n <= x.N; ++n)
      if (g.off[k][n] >= 0) {
        const int r = x.rho[k][n];
        jobs.push_back(EigJob{g.buf.p + g.off[k][n], r, r, e.V.p + e.voff[k][n], e.w.p + e.woff[k][n], kAbsTolGeneral, true});
      }
  if (values_only) *values_only = run_eig_values(c, jobs);
  else run_eig(c, jobs);
  return e;
}

}  // namespace

// trunc_par(x; eps, cap) = P_1 P_2 ... P_{L-1} x with P_k the orthogonal projector onto the
// kept left singular vectors of the k-th matricisation of x, every bond decided
// independently with tolerance eps/(L-1).  With the left Gram G^L_k = A_k^T A_k factored
// as W W^T (any factor: here its Cholesky factor, columns whose pivot is at the level of
// rounding dropped) one has A_k = Q W^T with Q orthonormal, so
// the singular values of the matricisation A_k B_k are the square roots of the
// eigenvalues of M = W^T G^R W (G^R = B_k B_k^T).  For the leading eigenpairs
// (U_s, Sigma_s^2) of M the bond matrices Lk = G^R W U_s Sigma_s^{-2} and Rk = U_s^T W^T
// satisfy A_k Lk Rk = Q U_s U_s^T Q^T A_k = P_k A_k, so inserting Lk Rk on every bond
// applies all projectors; all bonds are processed in the same batched launches.  No
// inverse of W or of a Gram eigenvalue appears; the inverse Sigma_s^{-2} only involves
// kept singular values.
std::unique_ptr<Mps> round_parallel(Ctx& c, const Mps& x, double eps, int cap, bool* cap_bound) {
  const int L = x.L, N = x.N;
  // x - P_1 Y = (I - P_1) x + P_1 (x - Y), Y = P_2 ... P_{L-1} x, splits into parts with
  // complementary ranges, so ||x - y||^2 <= sum_k ||(I - P_k) x||^2 (the first inequality
  // of eq. ttsvdquasiopt) and eps/sqrt(L-1) per bond gives ||x - y|| <= eps
  const double delta = L > 1 ? eps / std::sqrt(double(L - 1)) : eps;
  // the right Grams (a chain over k = L..2) run on the side stream beside the left Grams
  // (k = 1..L-1) and their Cholesky factorisations
  struct SideChain {
    Ctx& c;
    bool joined;
    explicit SideChain(Ctx& cx) : c(cx), joined(!cx.use_side) {
      if (!joined) c.fork();
    }
    void unfork() {
      if (!joined) c.unfork();
    }
    void join() {
      if (!joined) c.join();
      joined = true;
    }
    ~SideChain() {
      if (!joined) try { c.join(); } catch (...) {}
    }
  } side(c);
  BondGrams GR = right_grams(c, x);
  side.unfork();
  BondGrams GL = left_grams(c, x);
  // W W^T = G^L (+ kCholShift max diag) by a blocked Cholesky factorisation; offsets of the
  // r x r blocks of every bond and sector
  BondEig EL;
  EL.voff.assign(L + 1, std::vector<int64_t>(N + 1, -1));
  int64_t tv = 0;
  for (int k = 1; k < L; ++k)
    for (int n = 0; n <= N; ++n)
      if (GL.off[k][n] >= 0) {
        EL.voff[k][n] = tv;
        tv += int64_t(x.rho[k][n]) * x.rho[k][n];
      }
  EL.V = Buf(c.pool, size_t(std::max<int64_t>(tv, 1)));
  Buf W(c.pool, EL.V.n);
  {
    std::vector<CholJob> jobs;
    for (int k = 1; k < L; ++k)
      for (int n = 0; n <= N; ++n)
        if (EL.voff[k][n] >= 0) jobs.push_back(CholJob{GL.buf.p + GL.off[k][n], x.rho[k][n], W.p + EL.voff[k][n]});
    chol_all(c, jobs);
  }
  side.join();
  // B = W^T G^R W for every bond and sector
  Buf Tm(c.pool, EL.V.n), Bm(c.pool, EL.V.n);
  {
    GemmBatch g1, g2;
    for (int k = 1; k < L; ++k)
      for (int n = 0; n <= N; ++n)
        if (EL.voff[k][n] >= 0) {
          const int r = x.rho[k][n];
          g1.add(GR.buf.p + GR.off[k][n], r, 0, W.p + EL.voff[k][n], r, 0, Tm.p + EL.voff[k][n], r, r, r, r, 1.0, 0.0);
          g2.add(W.p + EL.voff[k][n], r, 1, Tm.p + EL.voff[k][n], r, 0, Bm.p + EL.voff[k][n], r, r, r, r, 1.0, 0.0);
        }
    g1.run(c);
    g2.run(c);
  }
  BondGrams Bg;
  Bg.off.assign(L + 1, std::vector<int64_t>(N + 1, -1));
  for (int k = 1; k < L; ++k) Bg.off[k] = EL.voff[k];
  Bg.buf = std::move(Bm);
  EigPlan plan;
  BondEig EB = eig_grams(c, x, Bg, 1, L - 1, &plan);
  std::vector<double> sb2 = download(c, EB.w.p, EB.w.n);
  auto rho = x.rho;
  // the bonds are decided independently: on host threads unless several contexts share
  // the host already (batches)
  std::vector<char> bound(size_t(L), 0);
#pragma omp parallel for schedule(dynamic, 1) if (c.use_side)
  for (int k = 1; k < L; ++k) {
    std::vector<std::vector<double>> sig(N + 1);
    for (int n = 0; n <= N; ++n)
      if (EB.woff[k][n] >= 0) {
        sig[n].resize(size_t(x.rho[k][n]));
        for (int j = 0; j < x.rho[k][n]; ++j) sig[n][j] = std::sqrt(std::max(sb2[EB.woff[k][n] + j], 0.0));
      }
    // same selection rules with the Gram-level numerical-zero cut-off
    double smax = 0;
    for (int n = 0; n <= N; ++n)
      for (double v : sig[n]) smax = std::max(smax, v);
    std::vector<int> keep(N + 1, 0);
    if (smax > 0) {
      double floor2 = 0.0;  // weight of the values at the numerical-zero level
      for (int n = 0; n <= N; ++n)
        for (double v : sig[n])
          if (!(v > kZeroTolPar * smax)) floor2 += v * v;
      bool cb = false;
      keep = select_ranks(sig, delta, cap, &cb, kZeroTolPar);
      // the dropped zero-level values are only known to that level: the tolerance is
      // certified only when their weight fits in it too (exact requests, delta = 0, aside)
      if (delta > 0 && floor2 > delta * delta) cb = true;
      bound[size_t(k)] = cb ? 1 : 0;
    }
    for (int n = 0; n <= N; ++n)
      if (x.valid(k, n)) rho[k][n] = keep[n];
  }
  if (cap_bound)
    for (int k = 1; k < L; ++k)
      if (bound[size_t(k)]) *cap_bound = true;
  // eigenvectors of the kept singular values only
  {
    std::vector<int> nvec;
    for (int k = 1; k < L; ++k)
      for (int n = 0; n <= N; ++n)
        if (Bg.off[k][n] >= 0) nvec.push_back(rho[k][n]);
    run_eig_vectors(c, plan, &nvec);
  }
  // bond matrices: Lk = (G^R W) U_s Sigma_s^{-2} (r x s), Rt = W U_s (r x s)
  Buf Lb(c.pool, EL.V.n), Rb(c.pool, EL.V.n);
  {
    GemmBatch g;
    ScaleBatch sb;
    for (int k = 1; k < L; ++k)
      for (int n = 0; n <= N; ++n)
        if (EL.voff[k][n] >= 0 && rho[k][n] > 0) {
          const int r = x.rho[k][n], s = rho[k][n];
          g.add(Tm.p + EL.voff[k][n], r, 0, EB.V.p + EB.voff[k][n], r, 0, Lb.p + EL.voff[k][n], r, r, s, r, 1.0, 0.0);
          g.add(W.p + EL.voff[k][n], r, 0, EB.V.p + EB.voff[k][n], r, 0, Rb.p + EL.voff[k][n], r, r, s, r, 1.0, 0.0);
          sb.add(Lb.p + EL.voff[k][n], r, Lb.p + EL.voff[k][n], r, r, s, EB.w.p + EB.woff[k][n], true, false);
        }
    g.run(c);
    sb.run(c);
  }
  auto y = mps_alloc(c, L, N, rho);
  // Z = [U | O] diag(L_k[n], L_k[n+1]) then new block = R_{k-1}[n] Z
  std::vector<Buf> Z;
  GemmBatch gz, gr;
  CopyBatch cz;
  for (int k = 1; k <= L; ++k) {
    for (int n = 0; n <= N; ++n) {
      if (!x.valid(k - 1, n)) continue;
      const int r = x.rows(k, n);
      const int su = y->ucols(k, n), so = y->ocols(k, n);
      if (r == 0 || su + so == 0 || y->rows(k, n) == 0) continue;
      Buf z(c.pool, size_t(r) * (su + so));
      if (su) {
        if (k == L) cz.add(x.U(k, n), r, z.p, r, r, su, 1.0);
        else gz.add(x.U(k, n), r, 0, Lb.p + EL.voff[k][n], x.rho[k][n], 0, z.p, r, r, su, x.ucols(k, n), 1.0, 0.0);
      }
      if (so) {
        if (k == L) cz.add(x.O(k, n), r, z.p + int64_t(r) * su, r, r, so, 1.0);
        else gz.add(x.O(k, n), r, 0, Lb.p + EL.voff[k][n + 1], x.rho[k][n + 1], 0, z.p + int64_t(r) * su, r, r, so,
                    x.ocols(k, n), 1.0, 0.0);
      }
      const int sl = y->rows(k, n);
      if (k == 1) cz.add(z.p, r, y->U(k, n), sl, r, su + so, 1.0);
      else gr.add(Rb.p + EL.voff[k - 1][n], r, 1, z.p, r, 0, y->U(k, n), sl, sl, su + so, r, 1.0, 0.0);
      Z.push_back(std::move(z));
    }
  }
  gz.run(c);
  cz.run(c);  // k == L copies; the k == 1 copies need gz first (issued after it)
  gr.run(c);
  // k == 1 blocks are copies of Z (R_0 = 1): issue them now that Z is complete
  for (auto& b : Z) c.scratch.push_back(std::move(b));
  for (Buf* b : {&W, &Tm, &Lb, &Rb}) c.scratch.push_back(std::move(*b));
  c.scratch.push_back(std::move(GL.buf));
  c.scratch.push_back(std::move(GR.buf));
  c.scratch.push_back(std::move(EL.V)); c.scratch.push_back(std::move(EL.w));
  c.scratch.push_back(std::move(EB.V)); c.scratch.push_back(std::move(EB.w));
  c.scratch.push_back(std::move(Bg.buf));
  return y;
}

// ---------------------------------------------------------------- H application
// Site-by-site application of the MPO with an intermediate rank m_zip ("zip-up"): the
// carry C_{k-1}[a, b, c] (a: new bond, b: MPO bond, c: bond of x) is contracted with
// x_k and W_k; the stacked matrix [T2_0; T2_1] of each new sector is factored through
// the two-pass Gram eigendecomposition of T2 T2^T, its leading left singular vectors
// become the new core and the carry is their transpose times T2.  With m_zip <= 0 only
// numerical zeros are dropped, which gives H x up to rounding; then trunc(.; eps, cap).
std::unique_ptr<Mps> apply_h(Ctx& c, const Mps& xin, double eps, int cap, int m_zip, bool* cap_bound,
                             double* zip_disc2) {
  if (!c.hmpo) fail(PV_ESTATE, "no Hamiltonian set");
  const DevMpo& op = *c.hmpo;
  const int L = xin.L, N = xin.N;
  std::unique_ptr<Mps> xr;
  const bool two_pass = c.trunc_mode == 0 || m_zip <= 0;
  if (m_zip > 0) xr = orthogonalize_right(c, xin, two_pass);
  const Mps& x = m_zip > 0 ? *xr : xin;
  const int zcap = m_zip > 0 ? m_zip : (1 << 30);
  double disc2 = 0.0;  // squared singular values the intermediate rank dropped
  auto rho = empty_rho(L, N);
  rho[0][0] = 1;
  auto y = std::make_unique<Mps>();
  y->L = L; y->N = N; y->rho = rho;
  y->site.resize(L); y->off.resize(L);
  auto vy = [&](int m, int n) { return y->valid(m, n); };
  auto vx = [&](int m, int n) { return x.valid(m, n); };
  EnvLayout Le = env_layout(0, N, y->rho[0], x.rho[0], op.qoff[0], vy, vx);
  Buf C(c.pool, size_t(std::max<int64_t>(Le.total, 1)));
  fill(c, C.p, Le.total, 1.0);
  for (int k = 1; k <= L; ++k) {
    // rows of the new core per new sector n2: r0 = rho_y[k-1][n2], r1 = rho_y[k-1][n2-1]
    // provisional layout at cut k with unit rows to size T2 columns
    std::vector<int> unit(N + 1, 1);
    EnvLayout Ln = env_layout(k, N, unit, x.rho[k], op.qoff[k], vy, vx);
    T2Data t2 = site_contract(c, k, x, y->rho[k - 1], Le, C, Ln, op);
    std::vector<int> r0(N + 1, 0), r1(N + 1, 0);
    for (int n2 = 0; n2 <= N; ++n2) {
      if (!y->valid(k, n2) || Ln.ncols[n2] == 0) continue;
      r0[n2] = t2.off[0][n2] >= 0 ? t2.rows[0][n2] : 0;
      r1[n2] = t2.off[1][n2] >= 0 ? t2.rows[1][n2] : 0;
    }
    if (k == L) {
      // last core: the panel itself, one column per column of x (the right boundary: 1, or
      // the column index of a joint MPS)
      const int D = x.rho[L][N];
      y->rho[L][N] = D;
      alloc_site(c, *y, L);
      CopyBatch cb;
      fill(c, y->site[L - 1].p, y->site_size(L), 0.0);
      if (r0[N] && y->ucols(L, N)) cb.add(t2.buf.p + t2.off[0][N], r0[N], y->U(L, N), y->rows(L, N), r0[N], D, 1.0);
      if (r1[N] && N >= 1 && y->ocols(L, N - 1))
        cb.add(t2.buf.p + t2.off[1][N], r1[N], y->O(L, N - 1), y->rows(L, N - 1), r1[N], D, 1.0);
      cb.run(c);
      c.scratch.push_back(std::move(t2.buf));
      break;
    }
    std::vector<SectorEig> se(N + 1), se2(N + 1);
    std::vector<Buf> Y(N + 1);
    GemmBatch g;
    for (int n2 = 0; n2 <= N; ++n2) {
      const int R = r0[n2] + r1[n2];
      if (R == 0) continue;
      const int K = int(Ln.ncols[n2]);
      se[n2].n = R;
      se[n2].G = Buf(c.pool, size_t(R) * R);
      const double* X0 = t2.buf.p + t2.off[0][n2];
      const double* X1 = r1[n2] ? t2.buf.p + t2.off[1][n2] : nullptr;
      if (r0[n2]) g.add(X0, r0[n2], 0, X0, r0[n2], 1, se[n2].G.p, R, r0[n2], r0[n2], K, 1.0, 0.0);
      if (r0[n2] && r1[n2]) g.add(X0, r0[n2], 0, X1, r1[n2], 1, se[n2].G.p + int64_t(r0[n2]) * R, R, r0[n2], r1[n2], K, 1.0, 0.0);
      if (r1[n2]) g.add(X1, r1[n2], 0, X1, r1[n2], 1, se[n2].G.p + r0[n2] + int64_t(r0[n2]) * R, R, r1[n2], r1[n2], K, 1.0, 0.0);
    }
    g.run(c);
    if (!two_pass) {
      // single pass: eigenvalues, rank selection, then only the kept eigenvectors; the new
      // core is W[:, :s] and the new carry W[:, :s]^T T2
      std::vector<EigJob> jobs(N + 1);
      for (int n2 = 0; n2 <= N; ++n2) {
        if (se[n2].n <= 0) continue;
        se[n2].W = Buf(c.pool, size_t(se[n2].n) * se[n2].n);
        se[n2].w = Buf(c.pool, size_t(se[n2].n));
        jobs[n2] = EigJob{se[n2].G.p, se[n2].n, se[n2].n, se[n2].W.p, se[n2].w.p, kAbsTolGeneral, true};
      }
      EigPlan plan = run_eig_values(c, jobs);
      auto sig = sigmas(c, se);
      std::vector<int> keep = select_ranks(sig, 0.0, zcap, nullptr, kZeroTolPar);
      disc2 += dropped_weight(sig, keep, kZeroTolPar);
      std::vector<int> nvec(N + 1, 0);
      for (int n2 = 0; n2 <= N; ++n2) nvec[n2] = se[n2].n > 0 ? keep[n2] : 0;
      run_eig_vectors(c, plan, &nvec);
      for (int n2 = 0; n2 <= N; ++n2) y->rho[k][n2] = y->valid(k, n2) ? keep[n2] : 0;
      alloc_site(c, *y, k);
      fill(c, y->site[k - 1].p, y->site_size(k), 0.0);
      CopyBatch cb;
      for (int n2 = 0; n2 <= N; ++n2) {
        const int s = keep[n2], R = se[n2].n;
        if (s == 0 || R == 0) continue;
        if (r0[n2] && y->ucols(k, n2)) cb.add(se[n2].W.p, R, y->U(k, n2), y->rows(k, n2), r0[n2], s, 1.0);
        if (r1[n2] && n2 >= 1 && y->ocols(k, n2 - 1))
          cb.add(se[n2].W.p + r0[n2], R, y->O(k, n2 - 1), y->rows(k, n2 - 1), r1[n2], s, 1.0);
      }
      cb.run(c);
      EnvLayout Lc = env_layout(k, N, y->rho[k], x.rho[k], op.qoff[k], vy, vx);
      Buf Cn(c.pool, size_t(std::max<int64_t>(Lc.total, 1)));
      GemmBatch g1;
      for (int n2 = 0; n2 <= N; ++n2) {
        const int s = keep[n2], R = se[n2].n;
        if (s == 0 || R == 0 || Lc.ncols[n2] == 0) continue;
        const int K = int(Lc.ncols[n2]);
        double* out = Cn.p + Lc.off[n2];
        if (r0[n2]) g.add(se[n2].W.p, R, 1, t2.buf.p + t2.off[0][n2], r0[n2], 0, out, s, s, K, r0[n2], 1.0, 0.0);
        if (r1[n2]) g1.add(se[n2].W.p + r0[n2], R, 1, t2.buf.p + t2.off[1][n2], r1[n2], 0, out, s, s, K, r1[n2], 1.0,
                           r0[n2] ? 1.0 : 0.0);
      }
      g.run(c);
      g1.run(c);
      for (auto& s2 : se) { c.scratch.push_back(std::move(s2.G)); c.scratch.push_back(std::move(s2.W)); c.scratch.push_back(std::move(s2.w)); }
      c.scratch.push_back(std::move(t2.buf));
      c.scratch.push_back(std::move(C));
      C = std::move(Cn);
      Le = std::move(Lc);
      continue;
    }
    eig_all(c, se, kAbsTolGeneral);
    GemmBatch g1;
    for (int n2 = 0; n2 <= N; ++n2) {
      const int R = se[n2].n;
      if (R == 0) continue;
      const int K = int(Ln.ncols[n2]);
      Y[n2] = Buf(c.pool, size_t(R) * K);
      if (r0[n2]) g.add(se[n2].W.p, R, 1, t2.buf.p + t2.off[0][n2], r0[n2], 0, Y[n2].p, R, R, K, r0[n2], 1.0, 0.0);
      if (r1[n2]) g1.add(se[n2].W.p + r0[n2], R, 1, t2.buf.p + t2.off[1][n2], r1[n2], 0, Y[n2].p, R, R, K, r1[n2], 1.0,
                         r0[n2] ? 1.0 : 0.0);
    }
    g.run(c);
    g1.run(c);
    if (two_pass) {
      for (int n2 = 0; n2 <= N; ++n2) {
        const int R = se[n2].n;
        if (R == 0) continue;
        const int K = int(Ln.ncols[n2]);
        se2[n2].n = R;
        se2[n2].G = Buf(c.pool, size_t(R) * R);
        g.add(Y[n2].p, R, 0, Y[n2].p, R, 1, se2[n2].G.p, R, R, R, K, 1.0, 0.0);
      }
      g.run(c);
      eig_all(c, se2, kAbsTolRefine);
    } else {
      identity_pass(c, se, se2);
    }
    auto sig = sigmas(c, se2);
    std::vector<std::vector<double>> sig_all(N + 1);
    for (int n2 = 0; n2 <= N; ++n2) sig_all[n2] = sig[n2];
    std::vector<int> keep = select_ranks(sig_all, 0.0, zcap, nullptr, two_pass ? kZeroTol : kZeroTolPar);
    disc2 += dropped_weight(sig_all, keep, two_pass ? kZeroTol : kZeroTolPar);
    for (int n2 = 0; n2 <= N; ++n2) y->rho[k][n2] = y->valid(k, n2) ? keep[n2] : 0;
    alloc_site(c, *y, k);
    fill(c, y->site[k - 1].p, y->site_size(k), 0.0);
    // new core: W1 W2[:, :s] split into the U (rows r0) and O (rows r1) parts
    for (int n2 = 0; n2 <= N; ++n2) {
      const int s = keep[n2], R = se[n2].n;
      if (s == 0 || R == 0) continue;
      if (r0[n2] && y->ucols(k, n2)) g.add(se[n2].W.p, R, 0, se2[n2].W.p, R, 0, y->U(k, n2), y->rows(k, n2), r0[n2], s, R, 1.0, 0.0);
      if (r1[n2] && n2 >= 1 && y->ocols(k, n2 - 1))
        g.add(se[n2].W.p + r0[n2], R, 0, se2[n2].W.p, R, 0, y->O(k, n2 - 1), y->rows(k, n2 - 1), r1[n2], s, R, 1.0, 0.0);
    }
    g.run(c);
    // new carry: W2[:, :s]^T Y, layout of the environment at cut k with rows s
    EnvLayout Lc = env_layout(k, N, y->rho[k], x.rho[k], op.qoff[k], vy, vx);
    Buf Cn(c.pool, size_t(std::max<int64_t>(Lc.total, 1)));
    for (int n2 = 0; n2 <= N; ++n2) {
      const int s = keep[n2], R = se[n2].n;
      if (s == 0 || R == 0 || Lc.ncols[n2] == 0) continue;
      g.add(se2[n2].W.p, R, 1, Y[n2].p, R, 0, Cn.p + Lc.off[n2], s, s, int(Lc.ncols[n2]), R, 1.0, 0.0);
    }
    g.run(c);
    for (auto& b : Y) c.scratch.push_back(std::move(b));
    for (auto& s2 : se) { c.scratch.push_back(std::move(s2.G)); c.scratch.push_back(std::move(s2.W)); c.scratch.push_back(std::move(s2.w)); }
    for (auto& s2 : se2) { c.scratch.push_back(std::move(s2.G)); c.scratch.push_back(std::move(s2.W)); c.scratch.push_back(std::move(s2.w)); }
    c.scratch.push_back(std::move(t2.buf));
    c.scratch.push_back(std::move(C));
    C = std::move(Cn);
    Le = std::move(Lc);
  }
  c.scratch.push_back(std::move(C));
  // a binding intermediate rank is reported like a binding rank cap: the result is no
  // longer within eps of H x, so the tolerance of the caller is not certified
  if (disc2 > 0.0 && cap_bound) *cap_bound = true;
  if (zip_disc2) *zip_disc2 += disc2;
  return round_mps(c, *y, eps, cap, cap_bound);
}

// ---------------------------------------------------------------- preconditioner
// S x by the sorted sequential truncated sum (Lemma truncr): the terms
// s_m = alpha_m prod_i diag(1, exp(-beta_m theta_i)) x (Section 4.3) have exact norms from
// one diagonal-operator sweep; the terms whose norms sum to <= eta/3 are dropped, the
// rest added in increasing norm order with trunc_{eps_j}, eps_j = eta |s_j| / (3 sum |s|),
// and the sum is truncated once more with eta/3.
// The M terms alpha_m exp(-beta_m d) of S with the learned correction of theta per (site,
// particles before it): the occupied block of site k in left sector n is scaled by
// exp(-beta_m (theta_k + Delta_{k,n})).  The term norms come from the scaled copies.
static std::unique_ptr<Mps> apply_s_corrected(Ctx& c, const Mps& x, double eta, int cap, bool* cap_bound) {
  const int L = x.L, N = x.N, M = int(c.alpha.size());
  std::vector<std::unique_ptr<Mps>> terms(M);
  std::vector<double> nrm(M);
  std::vector<double> occ(size_t(L) * (N + 1));
  for (int m = 0; m < M; ++m) {
    for (int k = 0; k < L; ++k)
      for (int n = 0; n <= N; ++n)
        occ[size_t(k) * (N + 1) + n] = std::exp(-c.beta[m] * (c.theta[k] + c.corr[size_t(k) * (N + 1) + n]));
    terms[m] = mps_sector_scaled_copy(c, x, c.alpha[m], occ.data());
    nrm[m] = norm2(c, *terms[m]);
  }
  std::vector<int> order(M);
  std::iota(order.begin(), order.end(), 0);
  std::sort(order.begin(), order.end(), [&](int a, int b) { return nrm[a] != nrm[b] ? nrm[a] < nrm[b] : a < b; });
  double csum = 0.0;
  int j0 = 0;
  for (int j = 0; j < M; ++j) {
    if (csum + nrm[order[j]] <= eta / 3.0) { csum += nrm[order[j]]; j0 = j + 1; }
    else break;
  }
  double total = 0.0;
  for (int j = j0; j < M; ++j) total += nrm[order[j]];
  std::unique_ptr<Mps> y;
  for (int j = j0; j < M; ++j) {
    const int m = order[j];
    const double eps_j = total > 0 ? eta * nrm[m] / (3.0 * total) : 0.0;
    if (!y) y = round_mps(c, *terms[m], eps_j, cap, cap_bound);
    else {
      auto sum = mps_lincomb(c, 1.0, *y, 1.0, *terms[m]);
      y = round_mps(c, *sum, eps_j, cap, cap_bound);
    }
    terms[m].reset();
  }
  if (!y) return mps_zero_like(c, x);
  return round_mps(c, *y, eta / 3.0, cap, cap_bound);
}

std::unique_ptr<Mps> apply_s(Ctx& c, const Mps& x, double eta, int cap, bool* cap_bound) {
  if (!c.corr.empty()) return apply_s_corrected(c, x, eta, cap, cap_bound);
  const int L = x.L, M = int(c.alpha.size());
  std::vector<std::vector<double>> d0(M, std::vector<double>(L, 1.0)), d1(M, std::vector<double>(L, 1.0));
  std::vector<std::vector<double>> occ(M, std::vector<double>(L, 1.0));
  for (int m = 0; m < M; ++m)
    for (int k = 0; k < L; ++k) {
      occ[m][k] = std::exp(-c.beta[m] * c.theta[k]);
      d1[m][k] = occ[m][k] * occ[m][k];
      if (k == 0) { d0[m][k] = c.alpha[m] * c.alpha[m]; d1[m][k] *= c.alpha[m] * c.alpha[m]; }
    }
  auto op = diag_mpo(c, L, M, d0, d1);
  std::vector<double> n2 = env_sweep(c, x, x, *op);
  // final environment: bra column a, channel m, ket column b at a + D (m + M b)
  const int D = x.rho[L][x.N];
  std::vector<double> nrm(M);
  for (int m = 0; m < M; ++m) {
    double t = 0.0;
    for (int i = 0; i < D; ++i) t += n2[size_t(i) + size_t(D) * (m + size_t(M) * i)];
    nrm[m] = std::sqrt(std::max(t, 0.0));
  }
  std::vector<int> order(M);
  std::iota(order.begin(), order.end(), 0);
  std::sort(order.begin(), order.end(), [&](int a, int b) { return nrm[a] != nrm[b] ? nrm[a] < nrm[b] : a < b; });
  double csum = 0.0;
  int j0 = 0;
  for (int j = 0; j < M; ++j) {
    if (csum + nrm[order[j]] <= eta / 3.0) { csum += nrm[order[j]]; j0 = j + 1; }
    else break;
  }
  double total = 0.0;
  for (int j = j0; j < M; ++j) total += nrm[order[j]];
  std::unique_ptr<Mps> y;
  for (int j = j0; j < M; ++j) {
    const int m = order[j];
    const double eps_j = total > 0 ? eta * nrm[m] / (3.0 * total) : 0.0;
    auto s = mps_scaled_copy(c, x, c.alpha[m], occ[m].data());
    if (!y) y = round_mps(c, *s, eps_j, cap, cap_bound);
    else {
      auto sum = mps_lincomb(c, 1.0, *y, 1.0, *s);
      y = round_mps(c, *sum, eps_j, cap, cap_bound);
    }
  }
  if (!y) {
    // every term dropped: S x is below the tolerance; return the zero state
    return mps_zero_like(c, x);
  }
  return round_mps(c, *y, eta / 3.0, cap, cap_bound);
}


// ---------------------------------------------------------------- exact solves
// x = H_gamma^{-1} b on the N-particle space by preconditioned conjugate gradients in
// block-sparse form: the products with H (exact zip-up), the preconditioner S^2 (both
// S applications with every term kept) and every sum truncated only at the numerical
// zeros (eps 0, no rank cap).  Stops when ||b - H x|| <= rel_tol ||b|| (the recursive
// residual) or after max_iter steps.
std::unique_ptr<Mps> solve_h(Ctx& c, const Mps& b, double rel_tol, int max_iter, int* iters, double* rel_res) {
  const int big = 1 << 30;
  const double nb = norm2(c, b);
  auto x = mps_zero_like(c, b);
  if (!(nb > 0)) {
    if (iters) *iters = 0;
    if (rel_res) *rel_res = 0.0;
    return x;
  }
  auto r = round_mps(c, b, 0.0, big, nullptr);
  auto precondition = [&](const Mps& v) {
    auto s1 = apply_s(c, v, 0.0, big, nullptr);
    return apply_s(c, *s1, 0.0, big, nullptr);
  };
  auto z = precondition(*r);
  auto p = mps_scaled_copy(c, *z, 1.0, nullptr);
  double rz = dot(c, *r, *z);
  int it = 0;
  double rr = nb;
  for (; it < max_iter; ++it) {
    auto q = apply_h(c, *p, 0.0, big, 0, nullptr);
    const double pq = dot(c, *p, *q);
    if (!(pq > 0)) fail(PV_ENOTSPD, "H_gamma is not positive on the search direction");
    const double alpha = rz / pq;
    auto xs = mps_lincomb(c, 1.0, *x, alpha, *p);
    x = round_mps(c, *xs, 0.0, big, nullptr);
    auto rs = mps_lincomb(c, 1.0, *r, -alpha, *q);
    r = round_mps(c, *rs, 0.0, big, nullptr);
    rr = norm2(c, *r);
    if (rr <= rel_tol * nb) { ++it; break; }
    z = precondition(*r);
    const double rz2 = dot(c, *r, *z);
    const double beta = rz2 / rz;
    rz = rz2;
    auto ps = mps_lincomb(c, 1.0, *z, beta, *p);
    p = round_mps(c, *ps, 0.0, big, nullptr);
  }
  if (iters) *iters = it;
  if (rel_res) *rel_res = rr / nb;
  return x;
}

// x at determinants (bit i of a mask = orbital i occupied): <det|x> by a transfer sweep
// with the determinant's rank-one MPS.
void amplitudes(Ctx& c, const Mps& x, const uint64_t* masks, int n, double* out) {
  for (int b = 0; b < n; ++b) {
    std::vector<int> occ;
    for (int i = 0; i < x.L; ++i)
      if ((masks[b] >> i) & 1u) occ.push_back(i);
    if (int(occ.size()) != x.N) fail(PV_EINVAL, "a determinant with the wrong particle number");
    auto d = mps_determinant(c, occ);
    out[b] = dot(c, *d, x);
  }
}

// ---------------------------------------------------------------- learned correction
// <n_i> of x for every site in one diagonal-operator sweep (channel i: 0 on the empty and
// 1 on the occupied state of site i, 1 elsewhere), divided by <x|x>.
std::vector<double> densities(Ctx& c, const Mps& x) {
  const int L = x.L;
  std::vector<std::vector<double>> d0(L, std::vector<double>(L, 1.0)), d1(L, std::vector<double>(L, 1.0));
  for (int i = 0; i < L; ++i) d0[i][i] = 0.0;
  auto op = diag_mpo(c, L, L, d0, d1);
  std::vector<double> v = env_sweep(c, x, x, *op);
  const double nx = dot(c, x, x);
  if (!(nx > 0)) fail(PV_EINVAL, "densities of a zero state");
  v.resize(L);
  for (double& d : v) d /= nx;
  return v;
}

namespace {

// Device state of one network evaluation over the R = L(N+1) feature rows.
struct Mlp {
  Ctx& c;
  int L, N, R;
  double tbar, dmax;
  Buf wq, X, H1, H2, z, tz, delta, G, dz, dA2, dA1, grad, dev;
  Mlp(Ctx& cc, const Mps& x, double lam, const std::vector<double>& th) : c(cc), L(x.L), N(x.N) {
    R = L * (N + 1);
    tbar = 0.0;
    double tmin = th[0];
    for (double t : th) { tbar += std::fabs(t); tmin = std::min(tmin, t); }
    tbar /= L;
    if (!(tbar > 0)) fail(PV_EINVAL, "theta vanishes");
    dmax = tmin > 0 ? 0.5 * tmin : 0.0;
    auto dens = densities(c, x);
    std::vector<double> host(3 * size_t(L));
    for (int i = 0; i < L; ++i) {
      host[i] = th[i];
      host[L + i] = c.h[size_t(i) * L + i];
      host[2 * L + i] = dens[i];
    }
    dev = Buf(c.pool, host.size());
    PV_HIP(hipMemcpyAsync(dev.p, host.data(), host.size() * 8, hipMemcpyHostToDevice, c.stream));
    wq = Buf(c.pool, size_t(kMlpParams));
    X = Buf(c.pool, size_t(kMlpFeat) * R);
    H1 = Buf(c.pool, size_t(kMlpWidth) * R);
    H2 = Buf(c.pool, size_t(kMlpWidth) * R);
    z = Buf(c.pool, R);
    tz = Buf(c.pool, R);
    delta = Buf(c.pool, R);
    launch_mlp_features(dev.p, dev.p + L, dev.p + 2 * L, L, N, tbar, lam, X.p, c.stream);
    c.sync();  // the host staging vector goes out of scope
  }
  const double* W1() const { return wq.p; }
  const double* b1() const { return W1() + kMlpWidth * kMlpFeat; }
  const double* W2() const { return b1() + kMlpWidth; }
  const double* b2() const { return W2() + kMlpWidth * kMlpWidth; }
  const double* W3() const { return b2() + kMlpWidth; }
  const double* b3() const { return W3() + kMlpWidth; }
  // the matrix products in float32 MFMA with float32 accumulation
  void gemm(const double* A, int lda, int ta, const double* B, int ldb, int tb, double* C, int ldc, int M, int Nn,
            int K) {
    GemmBatch g;
    g.prec = 1;
    g.add(A, lda, ta, B, ldb, tb, C, ldc, M, Nn, K, 1.0, 0.0);
    g.run(c);
  }
  void forward() {
    const int W = kMlpWidth;
    gemm(W1(), kMlpFeat, 1, X.p, kMlpFeat, 0, H1.p, W, W, R, kMlpFeat);
    launch_mlp_bias_tanh(H1.p, b1(), W, R, W, c.stream);
    gemm(W2(), W, 1, H1.p, W, 0, H2.p, W, W, R, W);
    launch_mlp_bias_tanh(H2.p, b2(), W, R, W, c.stream);
    gemm(W3(), W, 1, H2.p, W, 0, z.p, 1, 1, R, W);
    launch_mlp_output(z.p, b3(), R, dmax, tz.p, delta.p, c.stream);
  }
  // gradient of the loss with respect to the parameters from G = d loss / d delta
  void backward() {
    const int W = kMlpWidth;
    if (!grad.p) {
      dz = Buf(c.pool, R);
      dA2 = Buf(c.pool, size_t(W) * R);
      dA1 = Buf(c.pool, size_t(W) * R);
      grad = Buf(c.pool, size_t(kMlpParams));
    }
    double* gW1 = grad.p;
    double* gb1 = gW1 + W * kMlpFeat;
    double* gW2 = gb1 + W;
    double* gb2 = gW2 + W * W;
    double* gW3 = gb2 + W;
    double* gb3 = gW3 + W;
    launch_mlp_dz(G.p, tz.p, R, dmax, dz.p, c.stream);
    gemm(H2.p, W, 0, dz.p, R, 0, gW3, W, W, 1, R);
    launch_mlp_rowsum(dz.p, 1, R, 1, gb3, c.stream);
    gemm(W3(), W, 0, dz.p, 1, 0, dA2.p, W, W, R, 1);
    launch_mlp_tanh_grad(dA2.p, H2.p, int64_t(W) * R, c.stream);
    gemm(H1.p, W, 0, dA2.p, W, 1, gW2, W, W, W, R);
    launch_mlp_rowsum(dA2.p, W, R, W, gb2, c.stream);
    gemm(W2(), W, 0, dA2.p, W, 0, dA1.p, W, W, R, W);
    launch_mlp_tanh_grad(dA1.p, H1.p, int64_t(W) * R, c.stream);
    gemm(X.p, kMlpFeat, 0, dA1.p, W, 1, gW1, kMlpFeat, kMlpFeat, W, R);
    launch_mlp_rowsum(dA1.p, W, R, W, gb1, c.stream);
  }
};

}  // namespace

void learned_correction(Ctx& c, const float* params, const Mps& x, double lam, const std::vector<double>& th,
                        double* delta) {
  Mlp net(c, x, lam, th);
  Buf w(c.pool, size_t((kMlpParams + 1) / 2));
  PV_HIP(hipMemcpyAsync(w.p, params, size_t(kMlpParams) * 4, hipMemcpyHostToDevice, c.stream));
  launch_mlp_round(reinterpret_cast<const float*>(w.p), kMlpParams, net.wq.p, c.stream);
  net.forward();
  PV_HIP(hipMemcpyAsync(delta, net.delta.p, size_t(net.R) * 8, hipMemcpyDeviceToHost, c.stream));
  c.sync();
}

void learned_train(Ctx& c, float* params, const Mps& x, double lam, const std::vector<double>& th,
                   const uint64_t* masks, int nmask, int steps, float lr, double* loss, double* grad,
                   const double* rvals, const double* tvals) {
  const int L = x.L, N = x.N;
  for (int b = 0; b < nmask; ++b) {
    if (L < 64 && (masks[b] >> L) != 0) fail(PV_EINVAL, "a sample occupies an orbital beyond L");
    if (__builtin_popcountll(masks[b]) != N) fail(PV_EINVAL, "a sample is not an N-particle determinant");
  }
  Mlp net(c, x, lam, th);
  const size_t pf = size_t((kMlpParams + 1) / 2);  // float32 arrays in double-sized units
  Buf w(c.pool, pf), mom(c.pool, 2 * pf), mk(c.pool, std::max(nmask, 1)), jk(c.pool, size_t(L) * L),
      target(c.pool, std::max(nmask, 1)), lossd(c.pool, size_t(steps) + 1);
  float* wf = reinterpret_cast<float*>(w.p);
  float* m1 = reinterpret_cast<float*>(mom.p);
  float* m2 = m1 + kMlpParams;
  fill(c, mom.p, int64_t(2 * pf), 0.0);
  fill(c, lossd.p, steps + 1, 0.0);
  std::vector<double> jkh(size_t(L) * L, 0.0);
  for (int i = 0; i < L; ++i)
    for (int j = 0; j < L; ++j) {
      auto V = [&](int a, int b2, int cc, int d) { return c.v[((size_t(a) * L + b2) * L + cc) * L + d]; };
      jkh[i + size_t(j) * L] = V(i, j, j, i) - V(i, j, i, j);
    }
  PV_HIP(hipMemcpyAsync(w.p, params, size_t(kMlpParams) * 4, hipMemcpyHostToDevice, c.stream));
  if (nmask) PV_HIP(hipMemcpyAsync(mk.p, masks, size_t(nmask) * 8, hipMemcpyHostToDevice, c.stream));
  PV_HIP(hipMemcpyAsync(jk.p, jkh.data(), jkh.size() * 8, hipMemcpyHostToDevice, c.stream));
  const uint64_t* md = reinterpret_cast<const uint64_t*>(mk.p);
  const bool solve_form = rvals != nullptr;
  Buf rt;
  double tt = 0.0;
  if (solve_form) {
    // the method's residual and its exact solve at the samples
    rt = Buf(c.pool, 2 * size_t(nmask));
    PV_HIP(hipMemcpyAsync(rt.p, rvals, size_t(nmask) * 8, hipMemcpyHostToDevice, c.stream));
    PV_HIP(hipMemcpyAsync(rt.p + nmask, tvals, size_t(nmask) * 8, hipMemcpyHostToDevice, c.stream));
    for (int b = 0; b < nmask; ++b) tt += tvals[b] * tvals[b];
    if (!(tt > 0)) fail(PV_EINVAL, "the exact solve vanishes at every sample");
  } else {
    launch_mlp_target(md, nmask, net.dev.p + L, jk.p, c.gamma, L, target.p, c.stream);
  }
  launch_mlp_round(wf, kMlpParams, net.wq.p, c.stream);
  net.G = Buf(c.pool, net.R);
  const double B = std::max(nmask, 1);
  const double scale = 2.0 / (B * net.tbar * net.tbar), lscale = 1.0 / (B * net.tbar * net.tbar);
  auto misfit = [&](int t) {
    net.forward();
    fill(c, net.G.p, net.R, 0.0);
    if (solve_form)
      launch_mlp_solve_misfit(md, nmask, net.dev.p, net.delta.p, rt.p, rt.p + nmask, L, N, 2.0 / tt, 1.0 / tt,
                              net.G.p, lossd.p + t, c.stream);
    else
      launch_mlp_misfit(md, nmask, net.dev.p, net.delta.p, target.p, L, N, scale, lscale, net.G.p, lossd.p + t,
                        c.stream);
  };
  const float b1 = 0.9f, b2 = 0.999f, eps = 1e-8f;
  float p1 = 1.0f, p2 = 1.0f;
  for (int t = 0; t < steps; ++t) {
    misfit(t);
    net.backward();
    p1 *= b1;
    p2 *= b2;
    launch_mlp_adam(wf, m1, m2, net.grad.p, kMlpParams, lr, b1, b2, eps, 1.0f - p1, 1.0f - p2, net.wq.p, c.stream);
  }
  misfit(steps);
  if (grad) {
    net.backward();
    PV_HIP(hipMemcpyAsync(grad, net.grad.p, size_t(kMlpParams) * 8, hipMemcpyDeviceToHost, c.stream));
  }
  if (loss) PV_HIP(hipMemcpyAsync(loss, lossd.p, (size_t(steps) + 1) * 8, hipMemcpyDeviceToHost, c.stream));
  PV_HIP(hipMemcpyAsync(params, w.p, size_t(kMlpParams) * 4, hipMemcpyDeviceToHost, c.stream));
  c.sync();
}

}  // namespace pv
