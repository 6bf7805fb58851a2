// The regularised FP64 Cholesky solve (T + lambda I) x = b without any
// device allocation: its factor, diagonal-block inverses, solver vector and
// tickets live in one file-scope device array.  The kernels are those of
// minsr_solve; only where their workspace comes from differs.
#include "model.hpp"
#include <mutex>

namespace minsr {

// largest n served, and the array that holds the workspace for it: the
// factor (n^2), the inverses of its 64 x 64 diagonal blocks, the solver
// vector with its per-tile contributions, and the sync words, each part
// starting on a 256-byte boundary
constexpr int NOALLOC_MAX_N = 1024;
constexpr size_t NOALLOC_DOUBLES = (size_t)NOALLOC_MAX_N * NOALLOC_MAX_N + (1u << 17);
static __device__ __align__(256) double scratch[NOALLOC_DOUBLES];

// device address of `scratch` on each device, resolved once per device
constexpr int NOALLOC_MAX_DEV = 64;
static void* g_scratch_ptr[NOALLOC_MAX_DEV];
static std::mutex g_scratch_mu;

static size_t up256(size_t bytes) { return (bytes + 255) / 256 * 256; }

static int scratch_for_current_device(char** out) {
  int dev = -1;
  MINSR_HIP(hipGetDevice(&dev));
  if (dev < 0 || dev >= NOALLOC_MAX_DEV) return fail(MINSR_E_DEVICE, "device index out of range");
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void* p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !p)
      return fail(MINSR_E_DEVICE, std::string("hipGetSymbolAddress(scratch): ") +
                                      hipGetErrorString(e));
    g_scratch_ptr[dev] = p;
  }
  *out = static_cast<char*>(g_scratch_ptr[dev]);
  return MINSR_OK;
}

}  // namespace minsr

using namespace minsr;

extern "C" int minsr_solve_noalloc(int n, const double* dev_T, double lambda,
                                   const double* dev_b, double* dev_x, uint32_t* dev_status,
                                   hipStream_t s) {
  if (n < 0 || n > NOALLOC_MAX_N)
    return fail(MINSR_E_SHAPE, "minsr_solve_noalloc: n = " + std::to_string(n) +
                                   " outside [0, " + std::to_string(NOALLOC_MAX_N) + "]");
  if (!(lambda > 0.0)) return fail(MINSR_E_INVALID_ARG, "minsr_solve_noalloc: lambda must be > 0");
  char* base = nullptr;
  int rc = scratch_for_current_device(&base);
  if (rc) return rc;
  if (n == 0) return MINSR_OK;   // the set-up call
  if (!dev_T || !dev_b || !dev_x || !dev_status)
    return fail(MINSR_E_INVALID_ARG, "null argument");
  // carve the workspace for this n
  const size_t lf = up256((size_t)n * n * 8);
  const size_t di = up256(chol_dinv_elems(n) * 8);
  const size_t ve = up256(chol_vec_elems(n) * 8);
  const size_t sy = up256(chol_sync_words(n) * 4);
  if (lf + di + ve + sy > sizeof(double) * NOALLOC_DOUBLES)
    return fail(MINSR_E_SHAPE, "minsr_solve_noalloc: workspace exceeds the static array");
  double* Lf = reinterpret_cast<double*>(base);
  double* Dinv = reinterpret_cast<double*>(base + lf);
  double* yv = reinterpret_cast<double*>(base + lf + di);
  uint32_t* sync = reinterpret_cast<uint32_t*>(base + lf + di + ve);
  // the solver's preparation kernel clears the sync words and the x marks
  // on every call, so nothing left by an earlier call is read
  return launch_cholesky_solve(n, dev_T, Lf, Dinv, 0, lambda, dev_b, dev_x, yv, sync, dev_status,
                               s);
}
