// Internal helpers shared by the library's translation units (not installed).
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>
#include <cstdio>
#include <string>

#include "../../include/riccsd.h"

namespace ri {

// Thread-local error state behind ri_last_error_msg / ri_last_hip_error.
void set_error(const char* fmt, ...) __attribute__((format(printf, 1, 2)));
void clear_error();
void set_hip_error(hipError_t e, const char* where);

// Returns RI_E_HIP (and records the error) when `e` is not hipSuccess.
inline int check_hip(hipError_t e, const char* where) {
  if (e == hipSuccess) return RI_OK;
  set_hip_error(e, where);
  return RI_E_HIP;
}

#define RI_TRY(expr)                 \
  do {                               \
    int _rc = (expr);                \
    if (_rc != RI_OK) return _rc;    \
  } while (0)

#define RI_HIP(expr) RI_TRY(::ri::check_hip((expr), #expr))

// Stream-ordered device allocation (pool kept warm for repeated calls).
int dev_alloc(void** p, size_t bytes, hipStream_t s);
void dev_free(void* p, hipStream_t s);

// Per-kernel timing: when enabled (ri_prof_enable), a ProfScope records HIP events
// around the launches it encloses on stream `s`; ri_prof_report sums them by name.
class ProfScope {
 public:
  ProfScope(hipStream_t s, const char* name, double flops, double bytes = 0.0);
  ~ProfScope();
  ProfScope(const ProfScope&) = delete;
  ProfScope& operator=(const ProfScope&) = delete;

 private:
  hipStream_t s_;
  int idx_ = -1;
};

// While a ProfSuppress lives, ProfScope records nothing on its thread (no HIP events
// are created), whatever ri_prof_enable says.
class ProfSuppress {
 public:
  ProfSuppress();
  ~ProfSuppress();
  ProfSuppress(const ProfSuppress&) = delete;
  ProfSuppress& operator=(const ProfSuppress&) = delete;

 private:
  bool prev_;
};

// Ladder on factors stored with strides: B[q][a][c] at B + q*qs + a*rs + c
// (R += sum_cd (ac|bd) tau^{cd}_{ij}; workspace allocated on stream s).
int ppl_strided(const double* B, long qs, long rs, const double* tau, int o, int v, int naux, double* R,
                int precision, hipStream_t s);

namespace cc {
int check_system(const ri_system* sys, const char* where);
// (ia|jb) as gov [o][v][o][v] (caller buffer).
int ovov_integrals(const ri_system* sys, double* gov, hipStream_t s);
// MP2 amplitudes with the (ia|jb) integrals kept in gov [o][v][o][v] (caller buffer).
int mp2_with_integrals(const ri_system* sys, double* gov, double* t1, double* t2, hipStream_t s);
// t2 <- (t2 + t2^T) / 2 with t2^T[i][j][a][b] = t2[j][i][b][a]
int symmetrize_pairs(double* t2, int o, int v, hipStream_t s);
}  // namespace cc

// Byte ranges [a, a+na) and [b, b+nb) overlap?
inline bool overlaps(const void* a, size_t na, const void* b, size_t nb) {
  auto pa = reinterpret_cast<uintptr_t>(a), pb = reinterpret_cast<uintptr_t>(b);
  return pa < pb + nb && pb < pa + na;
}

inline size_t round_up(size_t x, size_t m) { return (x + m - 1) / m * m; }

// Last launch error as a status.
inline int check_launch(const char* what) { return check_hip(hipGetLastError(), what); }

// Bump allocator over one workspace block.
struct Carve {
  char* base;
  size_t used = 0;
  size_t cap;
  Carve(void* b, size_t c) : base(static_cast<char*>(b)), cap(c) {}
  template <class T>
  T* take(size_t count) {
    size_t off = round_up(used, 256);
    used = off + count * sizeof(T);
    return reinterpret_cast<T*>(base + off);
  }
};

}  // namespace ri
