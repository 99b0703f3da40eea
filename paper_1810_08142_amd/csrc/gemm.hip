// Generic strided FP64 tensor contraction on MFMA (gfx950):
//
//   C(m, n) = alpha * sum_k A(m, k) B(k, n) + beta * C(m, n)
//
// where m, n and k are compound indices: m = (m1, m2), n = (n1, n2),
// k = (k1, k2, k3), each level with its own stride, so a contraction over a
// permuted index pair of a 4-index tensor needs no transposed copy.  The index
// decomposition is turned into offset tables once per call (gemm_tables), and
// the MFMA kernel gathers operand tiles through them into LDS.
#include "gemm.h"

namespace ri {
namespace gemm {

typedef double double4_t __attribute__((ext_vector_type(4)));

constexpr int BM = 64, BN = 64, KC = 16;

__global__ void gemm_tables(GemmDesc g, long* tab) {
  long* amoff = tab;
  long* cmoff = amoff + g.M;
  long* bnoff = cmoff + g.M;
  long* cnoff = bnoff + g.N;
  long* akoff = cnoff + g.N;
  long* bkoff = akoff + g.K;
  const long idx = static_cast<long>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (idx < g.M) {
    const long m1 = idx / g.M2, m2 = idx % g.M2;
    amoff[idx] = m1 * g.am1 + m2 * g.am2;
    cmoff[idx] = m1 * g.cm1 + m2 * g.cm2;
  }
  if (idx < g.N) {
    const long n1 = idx / g.N2, n2 = idx % g.N2;
    bnoff[idx] = n1 * g.bn1 + n2 * g.bn2;
    cnoff[idx] = n1 * g.cn1 + n2 * g.cn2;
  }
  if (idx < g.K) {
    const long k3 = idx % g.K3, r = idx / g.K3;
    const long k2 = r % g.K2, k1 = r / g.K2;
    akoff[idx] = k1 * g.ak1 + k2 * g.ak2 + k3 * g.ak3;
    bkoff[idx] = k1 * g.bk1 + k2 * g.bk2 + k3 * g.bk3;
  }
}

// tile 64 x 64, 4 waves in a 2 x 2 arrangement, each wave 32 x 32 (2 x 2 MFMA tiles).
// a_kfast / b_kfast choose which index consecutive threads walk when loading.
// grid (ceil(N/64), ceil(M/64), batch), block 256
__global__ __launch_bounds__(256) void gemm_f64_kernel(GemmDesc g, const long* __restrict__ tab,
                                                       int a_kfast, int b_kfast) {
  __shared__ double sA[2][KC][BM + 1];
  __shared__ double sB[2][KC][BN + 1];
  const long* amoff = tab;
  const long* cmoff = amoff + g.M;
  const long* bnoff = cmoff + g.M;
  const long* cnoff = bnoff + g.N;
  const long* akoff = cnoff + g.N;
  const long* bkoff = akoff + g.K;

  const int t = threadIdx.x, w = t >> 6, lane = t & 63;
  const long bm = static_cast<long>(blockIdx.y) * BM, bn = static_cast<long>(blockIdx.x) * BN;
  const double* A = g.a + blockIdx.z * g.a_batch;
  const double* B = g.b + blockIdx.z * g.b_batch;
  double* C = g.c + blockIdx.z * g.c_batch;

  // each thread loads one row (m or n) and four k of each operand per chunk
  const int am = a_kfast ? (t >> 2) : (t & 63);
  const int ak = a_kfast ? ((t & 3) << 2) : (t >> 6);
  const int akstep = a_kfast ? 1 : 4;
  const int bnn = b_kfast ? (t >> 2) : (t & 63);
  const int bk = b_kfast ? ((t & 3) << 2) : (t >> 6);
  const int bkstep = b_kfast ? 1 : 4;
  const bool arow = bm + am < g.M, brow = bn + bnn < g.N;
  const long aoff = arow ? amoff[bm + am] : 0;
  const long boff = brow ? bnoff[bn + bnn] : 0;

  double ra[4], rb[4];
  double4_t acc[2][2];
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j) acc[i][j] = double4_t{0.0, 0.0, 0.0, 0.0};
  const int wm = (w >> 1) * 32, wn = (w & 1) * 32;
  const int l16 = lane & 15, kq = lane >> 4;
  const long nchunks = (g.K + KC - 1) / KC;
#pragma unroll
  for (int r = 0; r < 4; ++r) {
    const long ka = ak + r * akstep, kb = bk + r * bkstep;
    ra[r] = (arow && ka < g.K) ? A[aoff + akoff[ka]] : 0.0;
    rb[r] = (brow && kb < g.K) ? B[boff + bkoff[kb]] : 0.0;
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
      const long k0 = (ch + 1) * KC;
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const long ka = k0 + ak + r * akstep, kb = k0 + bk + r * bkstep;
        ra[r] = (arow && ka < g.K) ? A[aoff + akoff[ka]] : 0.0;
        rb[r] = (brow && kb < g.K) ? B[boff + bkoff[kb]] : 0.0;
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
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j) {
      const long n = bn + wn + 16 * j + l16;
      if (n >= g.N) continue;
      const long cn = cnoff[n];
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const long m = bm + wm + 16 * i + 4 * r + kq;
        if (m >= g.M) continue;
        double* p = C + cmoff[m] + cn;
        const double val = g.alpha * acc[i][j][r];
        *p = g.beta == 0.0 ? val : val + g.beta * *p;
      }
    }
}

size_t table_longs(const GemmDesc& g) { return 2 * static_cast<size_t>(g.M) + 2 * g.N + 2 * g.K; }

int run(const GemmDesc& g, int batch, long* tab, hipStream_t s) {
  if (g.M <= 0 || g.N <= 0 || batch <= 0) return RI_OK;
  if (g.K <= 0) {
    set_error("gemm: K must be positive");
    return RI_E_ARG;
  }
  const long mx = std::max(std::max(g.M, g.N), g.K);
  gemm_tables<<<static_cast<unsigned>((mx + 255) / 256), 256, 0, s>>>(g, tab);
  RI_TRY(check_launch("gemm_tables"));
  // consecutive threads walk k when the innermost k stride is 1 and the m/n stride is not
  const int a_kfast = (g.ak3 == 1 && g.K3 >= 4 && g.am2 != 1) ? 1 : 0;
  const int b_kfast = (g.bk3 == 1 && g.K3 >= 4 && g.bn2 != 1) ? 1 : 0;
  dim3 grid(static_cast<unsigned>((g.N + BN - 1) / BN), static_cast<unsigned>((g.M + BM - 1) / BM), batch);
  gemm_f64_kernel<<<grid, 256, 0, s>>>(g, tab, a_kfast, b_kfast);
  return check_launch("gemm_f64_kernel");
}

}  // namespace gemm
}  // namespace ri
