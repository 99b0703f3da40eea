// Status strings, per-thread error state and stream-ordered workspace helpers.
#include <cstdarg>
#include <mutex>
#include <vector>

#include "ri_common.h"

namespace ri {

namespace {
thread_local std::string g_msg;
thread_local int g_hip_err = 0;
std::mutex g_pool_mu;
std::vector<int> g_pool_ready;
}  // namespace

void set_error(const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof(buf), fmt, ap);
  va_end(ap);
  g_msg = buf;
}

void clear_error() {
  g_msg.clear();
  g_hip_err = 0;
}

void set_hip_error(hipError_t e, const char* where) {
  g_hip_err = static_cast<int>(e);
  set_error("%s: %s", where, hipGetErrorString(e));
}

// Keep freed stream-ordered memory in the device's default pool so repeated
// calls do not pay for mapping fresh pages every time.
static int warm_pool() {
  int dev = 0;
  RI_HIP(hipGetDevice(&dev));
  std::lock_guard<std::mutex> lk(g_pool_mu);
  if (static_cast<int>(g_pool_ready.size()) <= dev) g_pool_ready.resize(dev + 1, 0);
  if (g_pool_ready[dev]) return RI_OK;
  hipMemPool_t pool;
  RI_HIP(hipDeviceGetDefaultMemPool(&pool, dev));
  uint64_t thr = UINT64_MAX;
  RI_HIP(hipMemPoolSetAttribute(pool, hipMemPoolAttrReleaseThreshold, &thr));
  g_pool_ready[dev] = 1;
  return RI_OK;
}

int dev_alloc(void** p, size_t bytes, hipStream_t s) {
  *p = nullptr;
  if (bytes == 0) return RI_OK;
  RI_TRY(warm_pool());
  hipError_t e = hipMallocAsync(p, bytes, s);
  if (e != hipSuccess) {
    (void)hipGetLastError();
    *p = nullptr;
    set_error("device workspace of %zu bytes could not be allocated (%s)", bytes, hipGetErrorString(e));
    return RI_E_NOMEM;
  }
  return RI_OK;
}

void dev_free(void* p, hipStream_t s) {
  if (p) (void)hipFreeAsync(p, s);
}

}  // namespace ri

extern "C" {

const char* ri_status_str(int status) {
  switch (status) {
    case RI_OK: return "ok";
    case RI_E_ARG: return "invalid argument";
    case RI_E_ALIAS: return "output overlaps an input";
    case RI_E_NOMEM: return "out of device memory or workspace too small";
    case RI_E_HIP: return "HIP runtime error";
    case RI_E_NOCONV: return "not converged within the iteration limit";
    case RI_E_NUMERIC: return "non-finite values or divergence";
    case RI_E_UNSUPPORTED: return "unsupported precision or device";
    default: return "unknown status";
  }
}

const char* ri_last_error_msg(void) { return ri::g_msg.c_str(); }

int ri_last_hip_error(void) { return ri::g_hip_err; }

}  // extern "C"
