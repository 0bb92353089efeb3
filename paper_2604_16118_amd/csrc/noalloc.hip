// Allocation-free entry point: the symmetric eigensolver on caller-owned device buffers,
// with its work area in a file-scope device array instead of the context's memory pool.
#include <algorithm>
#include <mutex>

#include "engine.hpp"

using namespace pv;

namespace {

// Largest matrix order of pv_sym_eig_noalloc (PV_NOALLOC_MAX_N in the header).
constexpr int kNoAllocMaxN = PV_NOALLOC_MAX_N;
// The descriptor slot (256 bytes) followed by the tridiagonal solver's work area.
constexpr size_t kDescDoubles = 32;
constexpr size_t kScratchDoubles = kDescDoubles + size_t(7) * kNoAllocMaxN * kNoAllocMaxN + size_t(5) * kNoAllocMaxN + 2;
static_assert(sizeof(EigDesc) <= kDescDoubles * sizeof(double), "descriptor slot too small");

// One copy per device, held until the process ends.  In host code `scratch` only names
// the symbol: its device address comes from hipGetSymbolAddress.
static __device__ __align__(256) double scratch[kScratchDoubles];

std::mutex g_mu;
double* g_ptr[64] = {nullptr};

}  // namespace

namespace pv {

double* noalloc_scratch(int device) {
  if (device < 0 || device >= 64) fail(PV_EDEVICE, "device index out of range for the work array");
  std::lock_guard<std::mutex> lock(g_mu);
  if (!g_ptr[device]) {
    int cur = 0;
    PV_HIP(hipGetDevice(&cur));
    if (cur != device) PV_HIP(hipSetDevice(device));
    void* p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (cur != device) (void)hipSetDevice(cur);
    if (e != hipSuccess || !p) fail(PV_EDEVICE, std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(e));
    g_ptr[device] = static_cast<double*>(p);
  }
  return g_ptr[device];
}

// All eigenpairs of A (device) into w, V (device) with the work area and the descriptor
// slot in this device's copy of `scratch`; nothing is allocated and no HIP event is made.
void sym_eig_noalloc(Ctx& c, int n, const double* A, double* w, double* V) {
  if (n < 1 || n > kNoAllocMaxN)
    fail(PV_EINVAL, "n = " + std::to_string(n) + " outside 1.." + std::to_string(kNoAllocMaxN) +
                        ", the largest order the fixed work array of pv_sym_eig_noalloc holds");
  PV_HIP(hipSetDevice(c.device));
  double* base = noalloc_scratch(c.device);
  // no timing events, and the step reduction whatever the context's setting: the panel
  // reduction's trailing updates go through the GEMM, whose split-K partials are allocated
  const uint32_t mask = c.timer_mask;
  const int steps = c.tri_step_max;
  c.timer_mask = 0;
  c.tri_step_max = std::max(steps, 1);
  try {
    sym_eig_tridiag_device(c, n, A, w, V, base + kDescDoubles, reinterpret_cast<EigDesc*>(base));
  } catch (...) {
    c.timer_mask = mask;
    c.tri_step_max = steps;
    throw;
  }
  c.timer_mask = mask;
  c.tri_step_max = steps;
}

}  // namespace pv

