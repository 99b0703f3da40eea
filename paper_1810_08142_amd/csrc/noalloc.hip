// Allocation-free ladder entry point, ri_ppl_noalloc: for callers that cannot
// allocate device memory (code under HIP graph capture, tight serving loops,
// harnesses that forbid hipMalloc).  It runs the ladder of ri_ppl_ex on a workspace
// taken from a fixed device array of this file instead of allocating one.
//
// The array `scratch` exists once per device that loads the library and lives until
// the process ends.  Its host-side name is only a handle: the device address of each
// device's copy is looked up once per device (hipGetSymbolAddress, with that device
// current) and only that address is ever handed to kernels.  Every call on a device
// uses the same memory, so calls that overlap on one device (two streams, two host
// threads) race; the caller serialises them.
#include <mutex>

#include "ppl_shared.h"

namespace ri {
namespace {

constexpr size_t SCRATCH_BYTES = RI_PPL_NOALLOC_MAX_BYTES;
static_assert(SCRATCH_BYTES % 256 == 0, "whole 256-byte units");
static_assert(SCRATCH_BYTES >= ppl::ASYM_SCRATCH_BYTES, "room for the tau check");

static __device__ __align__(256) unsigned char scratch[SCRATCH_BYTES];

constexpr int MAX_DEVICES = 64;
std::mutex g_mu;
void* g_scratch[MAX_DEVICES] = {};

// Device address of the current device's copy of `scratch` (looked up on first use).
int scratch_address(int dev, void** out) {
  if (dev < 0 || dev >= MAX_DEVICES) {
    set_error("ri_ppl_noalloc: device %d is beyond the %d devices the library tracks", dev, MAX_DEVICES);
    return RI_E_UNSUPPORTED;
  }
  std::lock_guard<std::mutex> lk(g_mu);
  if (!g_scratch[dev]) {
    void* p = nullptr;
    RI_HIP(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
    if (!p || (reinterpret_cast<uintptr_t>(p) & 255)) {
      set_error("ri_ppl_noalloc: the scratch array has no usable device address on device %d", dev);
      return RI_E_HIP;
    }
    g_scratch[dev] = p;
  }
  *out = g_scratch[dev];
  return RI_OK;
}

}  // namespace
}  // namespace ri

using namespace ri;

extern "C" int ri_ppl_noalloc(const double* B_vv, const double* tau, int o, int v, int naux, double* R,
                              int precision, void* stream) {
  clear_error();
  RI_TRY(ppl::check_ladder_args(B_vv, tau, o, v, naux, R, precision, "ri_ppl_noalloc"));
  const size_t need = ppl::min_workspace_bytes(o, v, naux, precision);
  if (need == 0 || need > SCRATCH_BYTES) {
    set_error("ri_ppl_noalloc: o=%d v=%d naux=%d needs at least %zu bytes of workspace; the fixed scratch "
              "array holds %zu (use ri_ppl_ex)", o, v, naux, need, SCRATCH_BYTES);
    return RI_E_NOMEM;
  }
  hipStream_t s = static_cast<hipStream_t>(stream);
  int dev = 0;
  RI_HIP(hipGetDevice(&dev));
  if (s) {  // the scratch address is the current device's: the stream must be on it
    int sdev = 0;
    RI_HIP(hipStreamGetDevice(s, &sdev));
    if (sdev != dev) {
      set_error("ri_ppl_noalloc: the stream belongs to device %d, the current device is %d", sdev, dev);
      return RI_E_ARG;
    }
  }
  void* ws = nullptr;
  RI_TRY(scratch_address(dev, &ws));
  ProfSuppress quiet;  // the event profiler would create HIP events
  // the optional pair-symmetry check synchronises the stream before the ladder reuses
  // the same bytes
  RI_TRY(ppl::check_tau_if_asked(tau, o, v, s, ws));
  // every workspace element the ladder reads is written by it earlier in the call,
  // so nothing is cleared
  return ppl::run_fit(B_vv, tau, o, v, naux, R, precision, ws, SCRATCH_BYTES, s);
}
