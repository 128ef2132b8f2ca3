// hs_step_static: the exponential-midpoint Lanczos step of hs_step with its workspace taken
// from a fixed device array instead of a caller buffer, for callers that cannot allocate
// device memory (code under graph capture, serving loops, harnesses that forbid it).
//
// The array lives in the code object, one copy per GPU, for the life of the process.  Its
// device address is looked up once per device with that device current and kept; host
// code never passes the array's own name to a kernel (in host code it only names a
// host-side stand-in).  Every call on one GPU shares that GPU's copy: calls that overlap
// in time on one GPU (two streams, two threads) race on it and must be serialised by the
// caller.  The step writes every workspace word it reads before reading it, so nothing
// needs clearing between calls.
#include <cmath>
#include <mutex>
#include <string>

#include "hs_internal.h"

namespace hs {

int32_t launch_step(const hs_index_s *idx, const void *idx_dev, const hs_pot_s *p, void *pot_dev,
                    int32_t dtype, double t, double *t_dev, double h, int m, int reorth, void *c,
                    void *ws, double *diag, hipStream_t s);
int64_t step_workspace_bytes(const hs_index_s *idx, const hs_pot_s *p, int32_t dtype, int m);

static __device__ __align__(256) uint8_t scratch[HS_STEP_STATIC_MAX_BYTES];

constexpr int kMaxDevices = 64;
static void *g_scratch_ptr[kMaxDevices] = {};
static std::mutex g_scratch_mu;

// device address of this GPU's copy of the array (looked up on first use per device)
static int32_t scratch_address(void **out) {
  int dev = -1;
  HS_HIP(hipGetDevice(&dev));
  if (dev < 0 || dev >= kMaxDevices) return fail(HS_E_UNSUPPORTED, "hs_step_static: device id out of range");
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void *ptr = nullptr;
    HS_HIP(hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)));
    if (!ptr) return fail(HS_E_HIP, "hs_step_static: no device address for the scratch array");
    g_scratch_ptr[dev] = ptr;
  }
  *out = g_scratch_ptr[dev];
  return HS_OK;
}

}  // namespace hs

extern "C" int32_t hs_step_static(hs_index idx, const void *idx_dev, hs_pot pot, void *pot_dev,
                                  int32_t dtype, double t, double *t_dev, double h, int32_t m,
                                  int32_t reorth, void *c, double *diag_dev, void *stream) {
  if (!idx || !pot || !idx_dev || !pot_dev || !c)
    return hs::fail(HS_E_INVALID, "hs_step_static: NULL argument");
  if (pot->N != idx->N) return hs::fail(HS_E_INVALID, "hs_step_static: potential and index differ in N");
  if (dtype != HS_C128 && dtype != HS_C64) return hs::fail(HS_E_INVALID, "hs_step_static: bad dtype");
  if (m < 1 || m > 32) return hs::fail(HS_E_INVALID, "hs_step_static: m out of range 1..32");
  if (!std::isfinite(h) || (!t_dev && !std::isfinite(t)))
    return hs::fail(HS_E_NONFINITE, "hs_step_static: t or h not finite");
  const uintptr_t mis = reinterpret_cast<uintptr_t>(c) | reinterpret_cast<uintptr_t>(idx_dev) |
                        reinterpret_cast<uintptr_t>(pot_dev);
  if (mis & 15u) return hs::fail(HS_E_INVALID, "hs_step_static: device pointer not 16-byte aligned");
  const int64_t need = hs::step_workspace_bytes(idx, pot, dtype, m);
  if (need > (int64_t)HS_STEP_STATIC_MAX_BYTES)
    return hs::fail(HS_E_WORKSPACE, "hs_step_static: the step needs " + std::to_string(need) +
                                        " workspace bytes, above the fixed " +
                                        std::to_string((int64_t)HS_STEP_STATIC_MAX_BYTES));
  void *ws = nullptr;
  const int32_t st = hs::scratch_address(&ws);
  if (st != HS_OK) return st;
  return hs::launch_step(idx, idx_dev, pot, pot_dev, dtype, t, t_dev, h, m, reorth, c, ws, diag_dev,
                         static_cast<hipStream_t>(stream));
}
