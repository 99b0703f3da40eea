// Generic strided FP64 tensor contraction on MFMA (gfx950):
//
//   C(m, n) = alpha * sum_k A(m, k) B(k, n) + beta * C(m, n)
//
// where m, n and k are compound indices: m = (m1, m2), n = (n1, n2),
// k = (k1, k2, k3), each level with its own stride, so a contraction over a
// permuted index pair of a 4-index tensor needs no transposed copy.  Each thread
// walks its k indices with incremental counters (no tables, no divisions in the
// loop).  Contractions with few output tiles and a long k range are split over k
// into partial products that a second kernel sums in a fixed order, so the result
// does not depend on scheduling.
#include <cstdlib>

#include "gemm.h"

namespace ri {
namespace gemm {

typedef double double4_t __attribute__((ext_vector_type(4)));
typedef float f32x4_t __attribute__((ext_vector_type(4)));

// Arithmetic of the large-tile kernel: FP64 operands on the FP64 MFMA, or operands
// rounded to FP32 on the FP32 MFMA (FP32 accumulation).  Both are 16x16x4 tiles with
// the same operand layout; element r of lane l holds D[drow(r, l)][l % 16].
template <class T>
struct GMma;
template <>
struct GMma<double> {
  typedef double4_t acc_t;
  __device__ static acc_t mma(double a, double b, acc_t c) {
    return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
  }
  __device__ static int drow(int r, int lane) { return 4 * r + (lane >> 4); }
  __device__ static acc_t zero() { return acc_t{0.0, 0.0, 0.0, 0.0}; }
};
template <>
struct GMma<float> {
  typedef f32x4_t acc_t;
  __device__ static acc_t mma(float a, float b, acc_t c) { return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0); }
  __device__ static int drow(int r, int lane) { return 4 * (lane >> 4) + r; }
  __device__ static acc_t zero() { return acc_t{0.f, 0.f, 0.f, 0.f}; }
};

constexpr int BM = 64, BN = 64, KC = 16;

// One operand element stream: position k (decomposed as (k1, k2, k3)) and its
// offset, advanced by KC per chunk.
struct KWalk {
  long k, k2, k3, off;
};

__device__ inline KWalk kwalk_init(long k, long K2, long K3, long s1, long s2, long s3) {
  KWalk w;
  w.k = k;
  w.k3 = k % K3;
  const long r = k / K3;
  w.k2 = r % K2;
  w.off = (r / K2) * s1 + w.k2 * s2 + w.k3 * s3;
  return w;
}

__device__ inline void kwalk_step(KWalk& w, long K2, long K3, long s1, long s2, long s3) {
  w.k += KC;
  w.k3 += KC;
  w.off += KC * s3;
  while (w.k3 >= K3) {
    w.k3 -= K3;
    w.off += s2 - K3 * s3;
    if (++w.k2 >= K2) {
      w.k2 = 0;
      w.off += s1 - K2 * s2;
    }
  }
}

// tile 64 x 64, 4 waves in a 2 x 2 arrangement, each wave 32 x 32 (2 x 2 MFMA tiles).
// a_kfast / b_kfast choose which index consecutive threads walk when loading.
// grid (ceil(N/64), ceil(M/64), batch * splits); with splits > 1 the raw products of
// k range z go to part + z * M * N (row-major [M][N]).
__global__ __launch_bounds__(256) void gemm_f64_kernel(GemmDesc g, int a_kfast, int b_kfast, int splits, long kper,
                                                       double* __restrict__ part) {
  __shared__ double sA[2][KC][BM + 1];
  __shared__ double sB[2][KC][BN + 1];
  const int t = threadIdx.x, w = t >> 6, lane = t & 63;
  const long bm = static_cast<long>(blockIdx.y) * BM, bn = static_cast<long>(blockIdx.x) * BN;
  const int zb = blockIdx.z / splits, zs = blockIdx.z % splits;
  const double* A = g.a + zb * g.a_batch;
  const double* B = g.b + zb * g.b_batch;
  const long k_lo = zs * kper, k_hi = std::min(g.K, k_lo + kper);

  // each thread loads one row (m or n) and four k of each operand per chunk
  const int am = a_kfast ? (t >> 2) : (t & 63);
  const int ak = a_kfast ? ((t & 3) << 2) : (t >> 6);
  const int akstep = a_kfast ? 1 : 4;
  const int bnn = b_kfast ? (t >> 2) : (t & 63);
  const int bk = b_kfast ? ((t & 3) << 2) : (t >> 6);
  const int bkstep = b_kfast ? 1 : 4;
  const long mrow = bm + am, ncol = bn + bnn;
  const bool arow = mrow < g.M, brow = ncol < g.N;
  const long aoff = arow ? (mrow / g.M2) * g.am1 + (mrow % g.M2) * g.am2 : 0;
  const long boff = brow ? (ncol / g.N2) * g.bn1 + (ncol % g.N2) * g.bn2 : 0;
  KWalk wa[4], wb[4];
#pragma unroll
  for (int r = 0; r < 4; ++r) {
    wa[r] = kwalk_init(k_lo + ak + r * akstep, g.K2, g.K3, g.ak1, g.ak2, g.ak3);
    wb[r] = kwalk_init(k_lo + bk + r * bkstep, g.K2, g.K3, g.bk1, g.bk2, g.bk3);
  }

  double ra[4], rb[4];
  double4_t acc[2][2];
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j) acc[i][j] = double4_t{0.0, 0.0, 0.0, 0.0};
  const int wm = (w >> 1) * 32, wn = (w & 1) * 32;
  const int l16 = lane & 15, kq = lane >> 4;
  const long nchunks = k_hi > k_lo ? (k_hi - k_lo + KC - 1) / KC : 0;
#pragma unroll
  for (int r = 0; r < 4; ++r) {
    ra[r] = (arow && wa[r].k < k_hi) ? A[aoff + wa[r].off] : 0.0;
    rb[r] = (brow && wb[r].k < k_hi) ? B[boff + wb[r].off] : 0.0;
  }
#pragma unroll
  for (int r = 0; r < 4; ++r) {
    sA[0][ak + r * akstep][am] = ra[r];
    sB[0][bk + r * bkstep][bnn] = rb[r];
  }
  __syncthreads();
  for (long ch = 0; ch < nchunks; ++ch) {
    const int buf = ch & 1;
    const bool more = ch + 1 < nchunks;
    if (more) {
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        kwalk_step(wa[r], g.K2, g.K3, g.ak1, g.ak2, g.ak3);
        kwalk_step(wb[r], g.K2, g.K3, g.bk1, g.bk2, g.bk3);
        ra[r] = (arow && wa[r].k < k_hi) ? A[aoff + wa[r].off] : 0.0;
        rb[r] = (brow && wb[r].k < k_hi) ? B[boff + wb[r].off] : 0.0;
      }
    }
#pragma unroll
    for (int s = 0; s < KC / 4; ++s) {
      const int kk = 4 * s + kq;
      double a[2], b[2];
#pragma unroll
      for (int i = 0; i < 2; ++i) a[i] = sA[buf][kk][wm + 16 * i + l16];
#pragma unroll
      for (int j = 0; j < 2; ++j) b[j] = sB[buf][kk][wn + 16 * j + l16];
#pragma unroll
      for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j) acc[i][j] = __builtin_amdgcn_mfma_f64_16x16x4f64(a[i], b[j], acc[i][j], 0, 0, 0);
    }
    if (more) {
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        sA[buf ^ 1][ak + r * akstep][am] = ra[r];
        sB[buf ^ 1][bk + r * bkstep][bnn] = rb[r];
      }
    }
    __syncthreads();
  }
  // D[4r + lane/16][lane%16] in element r
  double* C = g.c + zb * g.c_batch;
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j) {
      const long n = bn + wn + 16 * j + l16;
      if (n >= g.N) continue;
      const long cn = (n / g.N2) * g.cn1 + (n % g.N2) * g.cn2;
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const long m = bm + wm + 16 * i + 4 * r + kq;
        if (m >= g.M) continue;
        if (splits > 1) {
          part[(zs * g.M + m) * g.N + n] = acc[i][j][r];
        } else {
          double* p = C + (m / g.M2) * g.cm1 + (m % g.M2) * g.cm2 + cn;
          const double val = g.alpha * acc[i][j][r];
          *p = g.beta == 0.0 ? val : val + g.beta * *p;
        }
      }
    }
}

// Large tiles for large contractions whose innermost summed extent K3 is a multiple
// of KC: a chunk of KC summed indices then never crosses a level boundary, so its
// offset is one wave-uniform base plus dk * stride.  Tile 128 x 128, four waves in
// a 2 x 2 arrangement, each wave 64 x 64 (4 x 4 MFMA tiles).  grid (ceil(N/128),
// ceil(M/128), batch), no split.
constexpr int BL = 128;
template <class T, int a_kfast, int b_kfast>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(2, 2))) void gemm_large(GemmDesc g) {
  typedef GMma<T> MF;
  __shared__ T sA[2][KC][BL + 2];
  __shared__ T sB[2][KC][BL + 2];
  const int t = threadIdx.x, w = t >> 6, lane = t & 63;
  const long bm = static_cast<long>(blockIdx.y) * BL, bn = static_cast<long>(blockIdx.x) * BL;
  const long zb = blockIdx.z;
  const double* A = g.a + zb * g.a_batch;
  const double* B = g.b + zb * g.b_batch;

  // element r of this thread: (row, dk) of the 128 x 16 tile; k-fast operands put
  // 16 consecutive lanes on consecutive k, the others 64 lanes on consecutive rows
  // (row, dk) of element r; recomputed where used rather than kept in registers
#define A_ROW(r) (a_kfast ? (t >> 4) + 16 * (r) : (t & 127))
#define A_K(r) (a_kfast ? (t & 15) : (t >> 7) + 2 * (r))
#define B_ROW(r) (b_kfast ? (t >> 4) + 16 * (r) : (t & 127))
#define B_K(r) (b_kfast ? (t & 15) : (t >> 7) + 2 * (r))
  long aoff[8], boff[8];
#pragma unroll
  for (int r = 0; r < 8; ++r) {
    const long m = bm + A_ROW(r), n = bn + B_ROW(r);
    aoff[r] = m < g.M ? (m / g.M2) * g.am1 + (m % g.M2) * g.am2 + A_K(r) * g.ak3 : -1;
    boff[r] = n < g.N ? (n / g.N2) * g.bn1 + (n % g.N2) * g.bn2 + B_K(r) * g.bk3 : -1;
  }
  // wave-uniform position of the chunk base in (k1, k2, k3) and its offsets
  long k2 = 0, k3 = 0, ka = 0, kb = 0;
  const long nchunks = g.K / KC;

  typename MF::acc_t acc[4][4];
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int j = 0; j < 4; ++j) acc[i][j] = MF::zero();
  const int wm = (w >> 1) * 64, wn = (w & 1) * 64;
  const int l16 = lane & 15, kq = lane >> 4;
  double ra[8], rb[8];
#pragma unroll
  for (int r = 0; r < 8; ++r) {
    ra[r] = aoff[r] >= 0 ? A[aoff[r]] : 0.0;
    rb[r] = boff[r] >= 0 ? B[boff[r]] : 0.0;
  }
#pragma unroll
  for (int r = 0; r < 8; ++r) {
    sA[0][A_K(r)][A_ROW(r)] = static_cast<T>(ra[r]);
    sB[0][B_K(r)][B_ROW(r)] = static_cast<T>(rb[r]);
  }
  __syncthreads();
  for (long ch = 0; ch < nchunks; ++ch) {
    const int buf = ch & 1;
    const bool more = ch + 1 < nchunks;
    if (more) {
      // advance the base by KC (never past a K3 boundary inside the chunk)
      k3 += KC;
      ka += KC * g.ak3;
      kb += KC * g.bk3;
      if (k3 == g.K3) {
        k3 = 0;
        ka += g.ak2 - g.K3 * g.ak3;
        kb += g.bk2 - g.K3 * g.bk3;
        if (++k2 == g.K2) {
          k2 = 0;
          ka += g.ak1 - g.K2 * g.ak2;
          kb += g.bk1 - g.K2 * g.bk2;
        }
      }
#pragma unroll
      for (int r = 0; r < 8; ++r) {
        ra[r] = aoff[r] >= 0 ? A[aoff[r] + ka] : 0.0;
        rb[r] = boff[r] >= 0 ? B[boff[r] + kb] : 0.0;
      }
    }
#pragma unroll
    for (int s4 = 0; s4 < KC / 4; ++s4) {
      const int kk = 4 * s4 + kq;
      T a[4], b[4];
#pragma unroll
      for (int i = 0; i < 4; ++i) a[i] = sA[buf][kk][wm + 16 * i + l16];
#pragma unroll
      for (int j = 0; j < 4; ++j) b[j] = sB[buf][kk][wn + 16 * j + l16];
#pragma unroll
      for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int j = 0; j < 4; ++j) acc[i][j] = MF::mma(a[i], b[j], acc[i][j]);
    }
    if (more) {
#pragma unroll
      for (int r = 0; r < 8; ++r) {
        sA[buf ^ 1][A_K(r)][A_ROW(r)] = static_cast<T>(ra[r]);
        sB[buf ^ 1][B_K(r)][B_ROW(r)] = static_cast<T>(rb[r]);
      }
    }
    __syncthreads();
  }
  // element r of a lane: D[drow(r, lane)][lane % 16]
  double* C = g.c + zb * g.c_batch;
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const long n = bn + wn + 16 * j + l16;
      if (n >= g.N) continue;
      const long cn = (n / g.N2) * g.cn1 + (n % g.N2) * g.cn2;
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const long m = bm + wm + 16 * i + MF::drow(r, lane);
        if (m >= g.M) continue;
        double* p = C + (m / g.M2) * g.cm1 + (m % g.M2) * g.cm2 + cn;
        const double val = g.alpha * static_cast<double>(acc[i][j][r]);
        *p = g.beta == 0.0 ? val : val + g.beta * *p;
      }
    }
}

#undef A_ROW
#undef A_K
#undef B_ROW
#undef B_K

// C(m, n) = alpha * sum_z part[z][m][n] + beta * C(m, n), z in order
__global__ void split_reduce(GemmDesc g, int splits, const double* __restrict__ part) {
  const long idx = static_cast<long>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (idx >= g.M * g.N) return;
  const long m = idx / g.N, n = idx % g.N;
  double acc = 0.0;
  for (int z = 0; z < splits; ++z) acc += part[z * g.M * g.N + idx];
  double* p = g.c + (m / g.M2) * g.cm1 + (m % g.M2) * g.cm2 + (n / g.N2) * g.cn1 + (n % g.N2) * g.cn2;
  const double val = g.alpha * acc;
  *p = g.beta == 0.0 ? val : val + g.beta * *p;
}

// Split over k when the output has too few tiles to fill the chip: aim at about
// 2048 workgroups, each split at least 32 chunks of k, partials at most 2^26 doubles.
size_t scratch_doubles(const GemmDesc& g, int batch) {
  const long tiles = ((g.M + BM - 1) / BM) * ((g.N + BN - 1) / BN);
  if (batch > 1 || tiles >= 1024) return 0;
  long splits = std::min<long>(1024, 2048 / tiles);
  splits = std::min(splits, g.K / (32 * KC));
  splits = std::min(splits, (1L << 26) / (g.M * g.N));
  if (splits < 2) return 0;
  return static_cast<size_t>(splits) * g.M * g.N;
}

int run(const GemmDesc& g, int batch, double* scratch, size_t scratch_len, hipStream_t s, int prec) {
  if (g.M <= 0 || g.N <= 0 || batch <= 0) return RI_OK;
  if (g.K <= 0) {
    set_error("gemm: K must be positive");
    return RI_E_ARG;
  }
  // consecutive threads walk k when the innermost k stride is 1 and the m/n stride is not
  const int a_kfast = (g.ak3 == 1 && g.K3 >= 4 && g.am2 != 1) ? 1 : 0;
  const int b_kfast = (g.bk3 == 1 && g.K3 >= 4 && g.bn2 != 1) ? 1 : 0;
  // large tiles when they still give the chip a few workgroups per CU
  // (RI_GEMM_LARGE_MIN_TILES overrides the threshold, e.g. to test the path at small sizes)
  const char* env = getenv("RI_GEMM_LARGE_MIN_TILES");
  const long env_tiles = env ? strtol(env, nullptr, 10) : 0;
  const long min_tiles = env_tiles > 0 ? env_tiles : 256;
  const long tiles_l = ((g.M + BL - 1) / BL) * ((g.N + BL - 1) / BL) * batch;
  if (g.K3 % KC == 0 && tiles_l >= min_tiles) {
    dim3 grid(static_cast<unsigned>((g.N + BL - 1) / BL), static_cast<unsigned>((g.M + BL - 1) / BL),
              static_cast<unsigned>(batch));
    if (prec == RI_PREC_FP32) {
      if (a_kfast && b_kfast) gemm_large<float, 1, 1><<<grid, 256, 0, s>>>(g);
      else if (a_kfast) gemm_large<float, 1, 0><<<grid, 256, 0, s>>>(g);
      else if (b_kfast) gemm_large<float, 0, 1><<<grid, 256, 0, s>>>(g);
      else gemm_large<float, 0, 0><<<grid, 256, 0, s>>>(g);
    } else {
      if (a_kfast && b_kfast) gemm_large<double, 1, 1><<<grid, 256, 0, s>>>(g);
      else if (a_kfast) gemm_large<double, 1, 0><<<grid, 256, 0, s>>>(g);
      else if (b_kfast) gemm_large<double, 0, 1><<<grid, 256, 0, s>>>(g);
      else gemm_large<double, 0, 0><<<grid, 256, 0, s>>>(g);
    }
    return check_launch("gemm_large");
  }
  const size_t want = scratch_doubles(g, batch);
  int splits = 1;
  if (want > 0 && scratch && scratch_len >= want) splits = static_cast<int>(want / (static_cast<size_t>(g.M) * g.N));
  // k range of each split, a whole number of chunks; trailing splits may be empty
  // (they write zero partials)
  const long kper = splits > 1 ? ((g.K + splits - 1) / splits + KC - 1) / KC * KC : g.K;
  dim3 grid(static_cast<unsigned>((g.N + BN - 1) / BN), static_cast<unsigned>((g.M + BM - 1) / BM),
            static_cast<unsigned>(batch * splits));
  gemm_f64_kernel<<<grid, 256, 0, s>>>(g, a_kfast, b_kfast, splits, kper, scratch);
  RI_TRY(check_launch("gemm_f64_kernel"));
  if (splits > 1) {
    const long n = g.M * g.N;
    split_reduce<<<static_cast<unsigned>((n + 255) / 256), 256, 0, s>>>(g, splits, scratch);
    RI_TRY(check_launch("split_reduce"));
  }
  return RI_OK;
}

}  // namespace gemm
}  // namespace ri
