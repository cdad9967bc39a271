// hsrq_noalloc.hip -- the single-problem solve for callers that cannot
// allocate (code under stream capture, tight serving loops, harnesses that
// forbid allocation): the workspace of hsrq_dhsrq3 comes from a fixed device
// array instead of the caller.
//
// The array lives in the library's code object, so every device the library
// runs on holds its own copy until the process ends.  Host code never uses
// its name as an address: hsrq_create, with the device current, asks the
// runtime once per device for the address of that device's copy, and the
// solve passes that address to the kernels exactly as it passes a caller's
// workspace.
#include <hip/hip_runtime.h>

#include <mutex>

#include "hsrq.h"
#include "hsrq_plan.h"

namespace hsrq {

constexpr size_t kScratchBytes = size_t(HSRQ_NOALLOC_SCRATCH_BYTES);
static __device__ __align__(256) char scratch[kScratchBytes];

constexpr int kMaxDevices = 64;
static void* g_scratch[kMaxDevices];
static std::mutex g_scratch_mu;

// Called by hsrq_create with `device` current.
int scratch_init(int device) {
  if (device < 0 || device >= kMaxDevices) return -1;
  std::lock_guard<std::mutex> g(g_scratch_mu);
  if (g_scratch[device]) return 0;
  void* p = nullptr;
  if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) != hipSuccess || !p) return -1;
  g_scratch[device] = p;
  return 0;
}

static void* scratch_of(int device) {
  if (device < 0 || device >= kMaxDevices) return nullptr;
  std::lock_guard<std::mutex> g(g_scratch_mu);
  return g_scratch[device];
}

}  // namespace hsrq

extern "C" int hsrq_dhsrq3_noalloc(hsrq_handle_t h, int n, const double* H, int ldh, int m, const double* wr,
                                   const double* wi, double* X, int ldx, int32_t* scale_exp, double* scale_mant,
                                   int32_t* info, double* resid, const hsrq_opts_t* opts) {
  using namespace hsrq;
  if (!h) return -1;
  hsrq_problem_t p{n, H, ldh, m, wr, wi, X, ldx, scale_exp, scale_mant, info, resid};
  const int st = check_problem(p);
  if (st) return st;
  if (!opts_valid(opts) || (opts && (opts->precision != 0 || opts->graph > 0))) return -14;
  if (m == 0) return HSRQ_OK;
  void* work = scratch_of(handle_device(h));
  if (!work) return HSRQ_ERR_HIP;
  return run_noalloc(h, p, work, kScratchBytes, opts);
}
