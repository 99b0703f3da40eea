// Helpers shared by the ladder paths (internal).
#pragma once

#include <algorithm>
#include <cmath>
#include <cstdlib>

#include "ri_common.h"

namespace ri {
namespace ppl {

constexpr int TB = 16;  // virtual block size: a block pair (X <= Y) has 256 slots
constexpr int NG = 16;  // column granule of the packed amplitudes
// Largest slice of the packed amplitudes one contraction split reads (MB); see the
// contraction splits of the ladder paths.  Measured at o=48 v=768 naux=2304: 48-96 MB
// take the FP64 contraction from 8.0 to 6.5 s; more splits cost unpack time.
constexpr long TAU_CHUNK_MB = 80;

__host__ __device__ inline void tri_decode(long p, int& x, int& y) {
  // p = y(y+1)/2 + x with 0 <= x <= y
  long yy = static_cast<long>((sqrt(8.0 * static_cast<double>(p) + 1.0) - 1.0) * 0.5);
  while ((yy + 1) * (yy + 2) / 2 <= p) ++yy;
  while (yy * (yy + 1) / 2 > p) --yy;
  y = static_cast<int>(yy);
  x = static_cast<int>(p - yy * (yy + 1) / 2);
}

// The split-bf16 path stores the 256 slots of a cd block pair in the build's wave
// order: the pair (x_in, y_in) (x_in the first index of the pair, 0..15) sits in slot
// 128h + 16w + 4i + j with h = x_in >> 3, w = 4 ((x_in >> 2) & 1) + (y_in >> 2),
// i = x_in & 3, j = y_in & 3 (the natural order is 16 x_in + y_in).
__host__ __device__ inline int split_slot(int x_in, int y_in) {
  return 128 * (x_in >> 3) + 16 * (4 * ((x_in >> 2) & 1) + (y_in >> 2)) + 4 * (x_in & 3) + (y_in & 3);
}

// Contraction column tiling: ntw 16-wide column tiles per workgroup tile (1..maxw),
// chosen to minimise the padded column count (ties: wider tiles).
// Columns per contraction tile (ntw tiles of 16) for ncols output columns.  A tile
// of `rows` rows and 16*ntw columns loads rows + 16*ntw operand rows per k step, so
// the traffic of the whole contraction goes as padded * (rows/16 + ntw) / ntw: wide
// tiles pay for some zero padding.
inline void pick_ntw(int ncols, int maxw, int rows, int& ntw, int& padded) {
  const int n16 = std::max(1, (ncols + NG - 1) / NG);
  const double r = rows / 16.0;
  ntw = 1;
  double best = 1e300;
  int best_pad = n16;
  for (int c = 1; c <= maxw; ++c) {
    const int p = (n16 + c - 1) / c * c;
    const double cost = p * (r + c) / c;
    if (cost < best * (1.0 - 1e-12)) {
      best = cost;
      ntw = c;
      best_pad = p;
    }
  }
  padded = best_pad * NG;
}

// Workgroups are dispatched to the eight XCDs round-robin by linear id; this maps
// the linear id so that each XCD works through a contiguous run of tiles (x
// fastest), so tiles that share operand rows share one L2.
__device__ inline void xcd_tile(unsigned& tx, unsigned& ty) {
  const unsigned gx = gridDim.x, nwg = gridDim.x * gridDim.y;
  const unsigned id = blockIdx.x + gx * blockIdx.y;
  const unsigned per = nwg / 8, rem = nwg % 8, x = id % 8, j = id / 8;
  const unsigned tile = (x < rem ? x * (per + 1) : rem * (per + 1) + (x - rem) * per) + j;
  tx = tile % gx;
  ty = tile / gx;
}

// Workgroups of kernel f (block threads each) resident on the current device at once:
// blocks per CU by the runtime's occupancy rule (registers, LDS, waves) times the CU
// count, or 256 * dflt_per_cu where the runtime gives no answer (no device).
inline long resident_wgs(const void* f, int block, int dflt_per_cu) {
  int dev = 0, cus = 0, per = 0;
  if (hipGetDevice(&dev) == hipSuccess &&
      hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) == hipSuccess &&
      hipOccupancyMaxActiveBlocksPerMultiprocessor(&per, f, block, 0) == hipSuccess && cus > 0 && per > 0)
    return static_cast<long>(per) * cus;
  (void)hipGetLastError();  // leave no error behind for the next launch check
  return 256L * dflt_per_cu;
}

// Split count for a launch of nwg workgroups per split, `slots` of which run at once,
// over K summed indices taken `step` at a time.  The launch lasts about
// ceil(nwg z / slots) rounds of one split's ceil(K / z) indices (rounded up to `step`):
// a last round of a few workgroups costs as much as a full one.  Among z in
// [z0, min(zmax, max(2 z0, z0 + 8))] the smallest whose modelled duration is within 3%
// of the least is taken, since every split adds a partial output to write and reduce.
inline long balance_splits(long nwg, long slots, long K, long step, long z0, long zmax) {
  auto cost = [&](long z) {
    long kz = (K + z - 1) / z;
    kz = (kz + step - 1) / step * step;
    const long zz = (K + kz - 1) / kz;  // splits launched
    return static_cast<double>((nwg * zz + slots - 1) / slots) * static_cast<double>(kz);
  };
  const long hi = std::min(zmax, std::max(2 * z0, z0 + 8));
  double best = cost(z0);
  for (long z = z0 + 1; z <= hi; ++z) best = std::min(best, cost(z));
  for (long z = z0; z <= hi; ++z)
    if (cost(z) <= best * 1.03) return z;
  return z0;
}

inline long env_long(const char* name, long dflt) {
  const char* s = getenv(name);
  if (!s || !*s) return dflt;
  char* end = nullptr;
  long x = strtol(s, &end, 10);
  return (end && *end == 0 && x > 0) ? x : dflt;
}

// Valid (a <= b) and (a < b) virtual pairs inside block pairs [p0, p0 + n), and the
// (a <= b) pairs among them that lie in diagonal block pairs (X == Y).
inline void count_pairs(int v, long p0, long n, double& le, double& lt, double& ld) {
  le = lt = ld = 0;
  for (long q = p0; q < p0 + n; ++q) {
    int X, Y;
    tri_decode(q, X, Y);
    const double nx = std::min(TB, v - X * TB), ny = std::min(TB, v - Y * TB);
    if (X < Y) {
      le += nx * ny;
      lt += nx * ny;
    } else {
      le += nx * (nx + 1) / 2;
      lt += nx * (nx - 1) / 2;
      ld += nx * (nx + 1) / 2;
    }
  }
}

// The diagonal block pairs (Y, Y), at index Y (Y + 3) / 2, inside [p0, p0 + n): Y runs
// over y0 .. y0 + count - 1.
inline void diag_pairs(long p0, long n, int& y0, int& count) {
  long y = 0;
  while (y * (y + 3) / 2 < p0) ++y;
  y0 = static_cast<int>(y);
  count = 0;
  while (y * (y + 3) / 2 < p0 + n) {
    ++count;
    ++y;
  }
}

// R += mirrored S +- A from FP32 slab results (shared unpack kernel).
// S, A: zp (zm) partial sums over k, zsp (zsm) elements apart, added in order.
// perm: S and A rows are in the split path's slot order (split_slot) instead of the
// natural one.
void launch_unpack_f32(const float* S, const float* A, int NP, int NM, int o, int v, long slab0, long npairs,
                       double* R, int zp, long zsp, int zm, long zsm, hipStream_t s, int perm = 0);

// Mixed-precision ladder (split-bf16, three products, FP32 accumulation).
// fit: choose the widest slab whose workspace fits ws_bytes (ws must be given);
// otherwise the default slab plan, which ws_bytes must hold.
size_t bf16x3_workspace_bytes(int o, int v, int naux);
size_t bf16x3_workspace_bytes_min(int o, int v, int naux);  // one-block-pair slabs
int bf16x3_run(const double* B, long qs, long rs, const double* tau, int o, int v, int naux, double* R,
               void* ws, size_t ws_bytes, int shard, int nshards, hipStream_t s, bool fit = false);

// The exchange-symmetric ladder (symmetric factors) in split bf16 with slabs of slab_bp
// block pairs; B_vv [naux][v][v] contiguous.  Workspace allocated for the call.
int bf16x3_run_sym(const double* B, const double* tau, int o, int v, int naux, double* R, long slab_bp,
                   hipStream_t s);

// Ladder argument checks shared by the entry points (status, error text set).
int check_ladder_args(const double* B_vv, const double* tau, int o, int v, int naux, const double* R,
                      int precision, const char* who);
// With RI_PPL_CHECK_TAU set: reject tau that is not pair-symmetric (synchronises s).
// scratch: a device buffer of at least ASYM_SCRATCH_BYTES, or NULL to allocate one.
constexpr size_t ASYM_SCRATCH_BYTES = (2 * 1024 + 2) * sizeof(double);
int check_tau_if_asked(const double* tau, int o, int v, hipStream_t s, void* scratch = nullptr);
// Smallest workspace any slab plan needs (one block pair per slab); 0 on invalid sizes.
size_t min_workspace_bytes(int o, int v, int naux, int precision);
// The ladder on the caller's workspace ws of ws_bytes, with the widest slab plan that
// fits in it (RI_E_NOMEM if none does); allocates nothing.
int run_fit(const double* B_vv, const double* tau, int o, int v, int naux, double* R, int precision, void* ws,
            size_t ws_bytes, hipStream_t s);

}  // namespace ppl
}  // namespace ri
