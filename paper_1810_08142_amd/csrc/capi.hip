// Status strings, per-thread error state and stream-ordered workspace helpers.
#include <cstdarg>
#include <cstring>
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

// ------------------------------------------------------------------ profiling
namespace {
struct ProfRec {
  std::string name;
  hipEvent_t start, stop;
  double flops, bytes;
};
std::mutex g_prof_mu;
bool g_prof_on = false;
std::vector<ProfRec> g_prof;
thread_local bool g_prof_suppressed = false;
}  // namespace

ProfSuppress::ProfSuppress() : prev_(g_prof_suppressed) { g_prof_suppressed = true; }
ProfSuppress::~ProfSuppress() { g_prof_suppressed = prev_; }

ProfScope::ProfScope(hipStream_t s, const char* name, double flops, double bytes) : s_(s) {
  if (g_prof_suppressed) return;
  std::lock_guard<std::mutex> lk(g_prof_mu);
  if (!g_prof_on) return;
  ProfRec r{name, nullptr, nullptr, flops, bytes};
  if (hipEventCreate(&r.start) != hipSuccess || hipEventCreate(&r.stop) != hipSuccess) {
    (void)hipGetLastError();
    return;
  }
  if (hipEventRecord(r.start, s) != hipSuccess) {
    (void)hipGetLastError();
    return;
  }
  idx_ = static_cast<int>(g_prof.size());
  g_prof.push_back(r);
}

ProfScope::~ProfScope() {
  if (idx_ < 0) return;
  std::lock_guard<std::mutex> lk(g_prof_mu);
  if (idx_ < static_cast<int>(g_prof.size())) (void)hipEventRecord(g_prof[idx_].stop, s_);
}

}  // namespace ri

extern "C" {

int ri_prof_enable(int on) {
  std::lock_guard<std::mutex> lk(ri::g_prof_mu);
  ri::g_prof_on = on != 0;
  return RI_OK;
}

int ri_prof_report(char* buf, size_t len) {
  ri::clear_error();
  if (!buf || len == 0) {
    ri::set_error("ri_prof_report: null buffer");
    return RI_E_ARG;
  }
  std::vector<ri::ProfRec> recs;
  {
    std::lock_guard<std::mutex> lk(ri::g_prof_mu);
    recs.swap(ri::g_prof);
  }
  struct Agg {
    std::string name;
    int count = 0;
    double ms = 0, flops = 0, bytes = 0;
  };
  std::vector<Agg> agg;
  int rc = RI_OK;
  for (auto& r : recs) {
    float ms = 0.f;
    hipError_t e = hipEventSynchronize(r.stop);
    if (e == hipSuccess) e = hipEventElapsedTime(&ms, r.start, r.stop);
    if (e != hipSuccess) rc = ri::check_hip(e, "ri_prof_report");
    (void)hipEventDestroy(r.start);
    (void)hipEventDestroy(r.stop);
    Agg* a = nullptr;
    for (auto& x : agg)
      if (x.name == r.name) a = &x;
    if (!a) {
      agg.push_back(Agg{r.name});
      a = &agg.back();
    }
    a->count += 1;
    a->ms += ms;
    a->flops += r.flops;
    a->bytes += r.bytes;
  }
  std::string out = "[";
  for (size_t k = 0; k < agg.size(); ++k) {
    char line[256];
    snprintf(line, sizeof(line), "%s{\"name\": \"%s\", \"count\": %d, \"ms\": %.6f, \"flops\": %.6e, \"bytes\": %.6e}",
             k ? ", " : "", agg[k].name.c_str(), agg[k].count, agg[k].ms, agg[k].flops, agg[k].bytes);
    out += line;
  }
  out += "]";
  if (out.size() + 1 > len) {
    ri::set_error("ri_prof_report: buffer of %zu bytes too small (%zu needed)", len, out.size() + 1);
    return RI_E_ARG;
  }
  memcpy(buf, out.c_str(), out.size() + 1);
  return rc;
}

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
