// Learned starting guess for the doubles amplitudes: a fully connected network
// with tanh hidden layers maps per-amplitude MP2 features to a correction of the
// MP2 amplitudes.  Training (forward, backward, Adam) and inference run in these
// FP32 kernels on f32 MFMA; the result is added to the FP64 MP2 amplitudes.
//
// Parameters are one flat FP32 vector: W1 [d_in][h], b1 [h], ..., W_out [h][1], b_out [1].
// Loss: mean over the batch of (y - Y)^2.
//
// MFMA v_mfma_f32_16x16x4f32 lane layout (measured): A[m][k] at lane m + 16k,
// B[k][n] at lane n + 16k, D[m][n] at lane n + 16*(m/4), element m%4.
#include <cmath>
#include <cstdio>
#include <cstring>
#include <vector>

#include "ri_common.h"

struct ri_mlp {
  int d_in, hidden, layers;
  size_t nparams;
  float* params = nullptr;  // device
  float* grad = nullptr;
  float* m = nullptr;
  float* v = nullptr;
  long step = 0;
  std::vector<float> mean, stdv;
  float y_scale = 1.f;
  float* scratch = nullptr;  // activations and deltas for up to `rows` rows
  long rows = 0;
  size_t scratch_bytes = 0;
};

namespace ri {
namespace mlp {

typedef float f32x4_t __attribute__((ext_vector_type(4)));
constexpr int BM = 64, BN = 64, KC = 16;
constexpr int NF = 8;  // features per amplitude

// C(m, n) = epilogue(alpha * sum_k A(m, k) B(k, n)); A(m, k) = A[m*sam + k*sak],
// B(k, n) = B[k*sbk + n*sbn]; C[m*ldc + n].  epilogue: + bias[n] (if bias), tanh (if act).
// grid.z splits K into `splits` ranges whose partial results go to C + z*split_stride.
struct GemmF32 {
  long M, N, K;
  const float* A;
  long sam, sak;
  const float* B;
  long sbk, sbn;
  float* C;
  long ldc;
  const float* bias;
  int act;
  float alpha;
  long kper;          // K range per split
  long split_stride;  // elements between split outputs
};

__global__ __launch_bounds__(256) void gemm_f32_kernel(GemmF32 g, int a_kfast, int b_kfast) {
  __shared__ float sA[2][KC][BM + 1];
  __shared__ float sB[2][KC][BN + 1];
  const int t = threadIdx.x, w = t >> 6, lane = t & 63;
  const long bm = static_cast<long>(blockIdx.y) * BM, bn = static_cast<long>(blockIdx.x) * BN;
  const long k_lo = blockIdx.z * g.kper, k_hi = std::min(g.K, k_lo + g.kper);
  float* C = g.C + blockIdx.z * g.split_stride;

  const int am = a_kfast ? (t >> 2) : (t & 63);
  const int ak = a_kfast ? ((t & 3) << 2) : (t >> 6);
  const int akstep = a_kfast ? 1 : 4;
  const int bnn = b_kfast ? (t >> 2) : (t & 63);
  const int bk = b_kfast ? ((t & 3) << 2) : (t >> 6);
  const int bkstep = b_kfast ? 1 : 4;
  const bool arow = bm + am < g.M, brow = bn + bnn < g.N;
  const float* Ap = g.A + (arow ? (bm + am) * g.sam : 0);
  const float* Bp = g.B + (brow ? (bn + bnn) * g.sbn : 0);

  float ra[4], rb[4];
  f32x4_t acc[2][2];
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j) acc[i][j] = f32x4_t{0.f, 0.f, 0.f, 0.f};
  const int wm = (w >> 1) * 32, wn = (w & 1) * 32;
  const int l16 = lane & 15, kq = lane >> 4;
  const long nchunks = k_hi > k_lo ? (k_hi - k_lo + KC - 1) / KC : 0;
#pragma unroll
  for (int r = 0; r < 4; ++r) {
    const long ka = k_lo + ak + r * akstep, kb = k_lo + bk + r * bkstep;
    ra[r] = (arow && ka < k_hi) ? Ap[ka * g.sak] : 0.f;
    rb[r] = (brow && kb < k_hi) ? Bp[kb * g.sbk] : 0.f;
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
      const long k0 = k_lo + (ch + 1) * KC;
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const long ka = k0 + ak + r * akstep, kb = k0 + bk + r * bkstep;
        ra[r] = (arow && ka < k_hi) ? Ap[ka * g.sak] : 0.f;
        rb[r] = (brow && kb < k_hi) ? Bp[kb * g.sbk] : 0.f;
      }
    }
#pragma unroll
    for (int s = 0; s < KC / 4; ++s) {
      const int kk = 4 * s + kq;
      float a[2], b[2];
#pragma unroll
      for (int i = 0; i < 2; ++i) a[i] = sA[buf][kk][wm + 16 * i + l16];
#pragma unroll
      for (int j = 0; j < 2; ++j) b[j] = sB[buf][kk][wn + 16 * j + l16];
#pragma unroll
      for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j) acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x4f32(a[i], b[j], acc[i][j], 0, 0, 0);
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
  // D[m][n] at lane n + 16*(m/4), element m%4
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j) {
      const long n = bn + wn + 16 * j + l16;
      if (n >= g.N) continue;
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const long m = bm + wm + 16 * i + 4 * kq + r;
        if (m >= g.M) continue;
        float val = g.alpha * acc[i][j][r];
        if (g.bias) val += g.bias[n];
        if (g.act) val = tanhf(val);
        C[m * g.ldc + n] = val;
      }
    }
}

// out[i] = sum_z part[z * stride + i], fixed order
__global__ void sum_splits(const float* __restrict__ part, int splits, long stride, long n, float* out) {
  const long i = static_cast<long>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i >= n) return;
  float acc = 0.f;
  for (int z = 0; z < splits; ++z) acc += part[z * stride + i];
  out[i] = acc;
}

// part[z][c] = sum over rows r in chunk z of D[r][c]  (grid (ceil(cols/256), splits))
__global__ void colsum_partial(const float* __restrict__ D, long rows, int cols, long rper, float* part) {
  const int c = blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= cols) return;
  const long lo = blockIdx.y * rper, hi = std::min(rows, lo + rper);
  float acc = 0.f;
  for (long r = lo; r < hi; ++r) acc += D[r * cols + c];
  part[static_cast<long>(blockIdx.y) * cols + c] = acc;
}

// delta = dH * (1 - H^2)   (tanh')
__global__ void tanh_back(const float* __restrict__ H, float* dH, long n) {
  const long i = static_cast<long>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i < n) dH[i] *= 1.f - H[i] * H[i];
}

constexpr int LB = 1024;
// delta_out[r] = 2 (y - Y) / n and partials of sum (y - Y)^2
// (delta may be NULL: loss only)
__global__ __launch_bounds__(256) void mse_stage1(const float* __restrict__ y, const float* __restrict__ Y, long n,
                                                  float* delta, float* part) {
  __shared__ float sh[256];
  const long chunk = (n + LB - 1) / LB;
  const long lo = static_cast<long>(blockIdx.x) * chunk, hi = std::min(n, lo + chunk);
  float acc = 0.f;
  for (long i = lo + threadIdx.x; i < hi; i += 256) {
    const float r = y[i] - Y[i];
    if (delta) delta[i] = 2.f * r / static_cast<float>(n);
    acc += r * r;
  }
  sh[threadIdx.x] = acc;
  __syncthreads();
  for (int s = 128; s > 0; s >>= 1) {
    if (threadIdx.x < s) sh[threadIdx.x] += sh[threadIdx.x + s];
    __syncthreads();
  }
  if (threadIdx.x == 0) part[blockIdx.x] = sh[0];
}

__global__ __launch_bounds__(256) void mse_stage2(const float* __restrict__ part, long n, float* loss) {
  __shared__ float sh[256];
  float acc = 0.f;
  for (int i = threadIdx.x; i < LB; i += 256) acc += part[i];
  sh[threadIdx.x] = acc;
  __syncthreads();
  for (int s = 128; s > 0; s >>= 1) {
    if (threadIdx.x < s) sh[threadIdx.x] += sh[threadIdx.x + s];
    __syncthreads();
  }
  if (threadIdx.x == 0) *loss = sh[0] / static_cast<float>(n);
}

__global__ void adam_kernel(float* p, const float* __restrict__ g, float* m, float* v, long n, float lr, float b1,
                            float b2, float eps, float c1, float c2) {
  const long i = static_cast<long>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const float gi = g[i];
  const float mi = b1 * m[i] + (1.f - b1) * gi;
  const float vi = b2 * v[i] + (1.f - b2) * gi * gi;
  m[i] = mi;
  v[i] = vi;
  p[i] -= lr * (mi / c1) / (sqrtf(vi / c2) + eps);
}

// SplitMix64 (Steele, Lea and Flood, OOPSLA 2014): output number c (c = 0, 1, ...)
// of the stream seeded with `seed`.
__host__ __device__ inline unsigned long long splitmix64(unsigned long long seed, unsigned long long c) {
  unsigned long long z = seed + (c + 1) * 0x9E3779B97F4A7C15ull;
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}

// Starting parameters of one layer (parameters [off, off + fin*fout + fout) of the
// flat vector): weight number i gets N(0, 1)/sqrt(fin) by the Box-Muller transform of
// the uniforms u1 = (x_{2i} >> 11 + 1) 2^-53 in (0, 1] and u2 = (x_{2i+1} >> 11) 2^-53,
// x_c the SplitMix64 outputs of `seed` and i the flat parameter index; biases are zero.
__global__ void init_layer(float* p, long off, int fin, int fout, unsigned long long seed) {
  const long k = static_cast<long>(blockIdx.x) * blockDim.x + threadIdx.x;
  const long nw = static_cast<long>(fin) * fout;
  if (k >= nw + fout) return;
  const long i = off + k;
  if (k >= nw) {
    p[i] = 0.f;
    return;
  }
  const double two53 = 1.0 / 9007199254740992.0;
  const double u1 = static_cast<double>((splitmix64(seed, 2 * i) >> 11) + 1) * two53;
  const double u2 = static_cast<double>(splitmix64(seed, 2 * i + 1) >> 11) * two53;
  const double z = sqrt(-2.0 * log(u1)) * cos(6.283185307179586 * u2);
  p[i] = static_cast<float>(z / sqrt(static_cast<double>(fin)));
}

// rows r of (X, Y) in the order perm: Xs[r][:] = X[perm[r]][:], Ys[r] = Y[perm[r]]
__global__ void gather_rows(const float* __restrict__ X, const float* __restrict__ Y, const int* __restrict__ perm,
                            long n, int d, float* Xs, float* Ys) {
  const long t = static_cast<long>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (t >= n * (d + 1)) return;
  const long r = t / (d + 1);
  const int c = static_cast<int>(t - r * (d + 1));
  const long src = perm[r];
  if (c < d)
    Xs[r * d + c] = X[src * d + c];
  else
    Ys[r] = Y[src];
}

// acc[0] += w * x[0]  (one thread; the epoch's mean batch loss, summed in step order)
__global__ void add_scaled(float* acc, const float* __restrict__ x, float w) {
  if (threadIdx.x == 0 && blockIdx.x == 0) acc[0] += w * x[0];
}

// Features of amplitudes [row0, row0 + n) of the o*o*v*v flattened (i, j, a, b) set:
// t2_ijab, t2_ijba, (ia|jb), (ib|ja), e_i + e_j - e_a - e_b, (e_a - e_b)^2, (e_i - e_j)^2,
// sqrt((ia|ia)(jb|jb)); standardised with (x - mean) / std when mean != NULL.
struct Norm {
  float mean[NF], inv_std[NF];
  int on;
};
__global__ void features_kernel(const double* __restrict__ gov, const double* __restrict__ eps,
                                const double* __restrict__ t2, int o, int v, long row0, long n, Norm nm, float* X) {
  const long r = static_cast<long>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (r >= n) return;
  const long idx = row0 + r;
  const long vv = static_cast<long>(v) * v;
  const int b = idx % v, a = (idx / v) % v;
  const long ij = idx / vv;
  const int j = ij % o, i = ij / o;
  auto G = [&](int p, int x, int q, int y) { return gov[((static_cast<long>(p) * v + x) * o + q) * v + y]; };
  const double ea = eps[o + a], eb = eps[o + b], ei = eps[i], ej = eps[j];
  double f[NF];
  f[0] = t2[idx];
  f[1] = t2[ij * vv + static_cast<long>(b) * v + a];
  f[2] = G(i, a, j, b);
  f[3] = G(i, b, j, a);
  f[4] = ei + ej - ea - eb;
  f[5] = (ea - eb) * (ea - eb);
  f[6] = (ei - ej) * (ei - ej);
  f[7] = sqrt(G(i, a, i, a) * G(j, b, j, b));
#pragma unroll
  for (int k = 0; k < NF; ++k) {
    float x = static_cast<float>(f[k]);
    if (nm.on) x = (x - nm.mean[k]) * nm.inv_std[k];
    X[r * NF + k] = x;
  }
}

// The pair-symmetric half of the (i, j, a, b) set: rows [row0, row0 + n) of the
// amplitudes with i <= j, pair p = j (j + 1) / 2 + i, row p v^2 + a v + b.
__device__ inline long half_index(long r, int o, int v) {
  const long vv = static_cast<long>(v) * v;
  const long p = r / vv, ab = r - p * vv;
  long j = static_cast<long>((sqrt(8.0 * static_cast<double>(p) + 1.0) - 1.0) * 0.5);
  while ((j + 1) * (j + 2) / 2 <= p) ++j;
  while (j * (j + 1) / 2 > p) --j;
  const long i = p - j * (j + 1) / 2;
  return (i * o + j) * vv + ab;
}

// Features of the half-set rows [row0, row0 + n) (see features_kernel).
__global__ void features_half_kernel(const double* __restrict__ gov, const double* __restrict__ eps,
                                     const double* __restrict__ t2, int o, int v, long row0, long n, Norm nm,
                                     float* X) {
  const long r = static_cast<long>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (r >= n) return;
  const long idx = half_index(row0 + r, o, v);
  const long vv = static_cast<long>(v) * v;
  const int b = idx % v, a = (idx / v) % v;
  const long ij = idx / vv;
  const int j = ij % o, i = ij / o;
  auto G = [&](int p, int x, int q, int y) { return gov[((static_cast<long>(p) * v + x) * o + q) * v + y]; };
  const double ea = eps[o + a], eb = eps[o + b], ei = eps[i], ej = eps[j];
  double f[NF];
  f[0] = t2[idx];
  f[1] = t2[ij * vv + static_cast<long>(b) * v + a];
  f[2] = G(i, a, j, b);
  f[3] = G(i, b, j, a);
  f[4] = ei + ej - ea - eb;
  f[5] = (ea - eb) * (ea - eb);
  f[6] = (ei - ej) * (ei - ej);
  f[7] = sqrt(G(i, a, i, a) * G(j, b, j, b));
#pragma unroll
  for (int k = 0; k < NF; ++k) {
    float x = static_cast<float>(f[k]);
    if (nm.on) x = (x - nm.mean[k]) * nm.inv_std[k];
    X[r * NF + k] = x;
  }
}

// t2[ijab] = t2[jiba] = t2_MP2[ijab] * (1 + scale * y) for the half-set rows
__global__ void add_correction_half(double* t2, const double* __restrict__ t2m, int o, int v, long row0, long n,
                                    const float* __restrict__ y, float scale) {
  const long r = static_cast<long>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (r >= n) return;
  const long idx = half_index(row0 + r, o, v);
  const long vv = static_cast<long>(v) * v;
  const long b = idx % v, a = (idx / v) % v, ij = idx / vv;
  const long j = ij % o, i = ij / o;
  const double val = t2m[idx] * (1.0 + static_cast<double>(scale) * static_cast<double>(y[r]));
  t2[idx] = val;
  if (i != j) t2[(j * o + i) * vv + b * v + a] = val;  // i == j: the row (b, a) writes that one
}

// y[r] = net(X[r]), r < n, without keeping activations: each workgroup takes IR = 64
// rows through every layer.  The layer input sits in LDS, element (m, k) at
// m * HMAX + (k ^ 4 (m & 15)).  A hidden layer's W arrives in chunks of WK rows, each
// loaded into registers while the previous one is in use; in LDS element (k, c) with
// c = 16 u + l sits at k * HMAX + 16 l + 4 (u4 ^ ((l >> 2) & 3)) + (u & 3), u4 = u >> 2,
// so the sixteen B operands of a lane (one per output tile) are four 16-byte reads and
// the reads of sixteen lanes hit distinct banks.  Wave w owns rows 16w .. 16w + 15 and
// all outputs (NT = hidden / 16 tiles of the 16x16x4 FP32 MFMA; the output layer one
// tile, its weight column read directly), summing k in steps of four from zero and
// adding the bias, then tanh for the hidden layers: the operation order of forward()'s
// GEMMs, so both give the same y bit for bit.  d_in a multiple of 4, at most HMAX.
// grid ceil(n / IR), block 256.
constexpr int IR = 64, HMAX = 256, WK = 8;
template <int NT>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(2))) void infer_kernel(const float* __restrict__ X, long n, int d_in, int layers,
                                                    const float* __restrict__ params, float* __restrict__ y) {
  constexpr int HID = 16 * NT, NQ = (NT + 3) / 4;  // 16-byte groups of a lane's B operands
  constexpr int RUNS = WK * 16 * NQ, PER = (RUNS + 255) / 256;
  __shared__ float sH[IR * HMAX];
  __shared__ float sW[WK * HMAX];
  const int t = threadIdx.x, w = t >> 6, lane = t & 63;
  const int l16 = lane & 15, kq = lane >> 4, mrow = 16 * w + l16;
  const long r0 = static_cast<long>(blockIdx.x) * IR;
  auto hidx = [](int m, int k) { return m * HMAX + (k ^ (4 * (m & 15))); };
  auto wrun = [](int k, int l, int u4) { return k * HMAX + 16 * l + 4 * (u4 ^ ((l >> 2) & 3)); };
  for (int e = t; e < IR * d_in; e += 256) {
    const int m = e / d_in, k = e - m * d_in;
    sH[hidx(m, k)] = r0 + m < n ? X[(r0 + m) * d_in + k] : 0.f;
  }
  const float* Wl = params;
  int fin = d_in;
  for (int l = 0; l < layers; ++l) {
    const float* bl = Wl + static_cast<size_t>(fin) * HID;
    f32x4_t acc[NT];
#pragma unroll
    for (int u = 0; u < NT; ++u) acc[u] = f32x4_t{0.f, 0.f, 0.f, 0.f};
    // run q of a chunk: row k = q / (16 NQ), column l = (q / NQ) % 16, group u4 = q % NQ,
    // i.e. W[k][16 (4 u4 + e) + l], e = 0..3 (zero beyond the layer)
    f32x4_t pre[PER];
    auto gload = [&](int k0) {
#pragma unroll
      for (int p = 0; p < PER; ++p) {
        const int q = t + 256 * p, k = q / (16 * NQ), lc = (q / NQ) % 16, u4 = q % NQ;
#pragma unroll
        for (int e = 0; e < 4; ++e) {
          const int u = 4 * u4 + e;
          pre[p][e] = (q < RUNS && k0 + k < fin && u < NT) ? Wl[static_cast<size_t>(k0 + k) * HID + 16 * u + lc] : 0.f;
        }
      }
    };
    auto step = [&](int k0, int s4) {
      const float a = sH[hidx(mrow, k0 + s4 + kq)];
      f32x4_t bq[NQ];
#pragma unroll
      for (int g = 0; g < NQ; ++g) bq[g] = *reinterpret_cast<const f32x4_t*>(&sW[wrun(s4 + kq, l16, g)]);
#pragma unroll
      for (int u = 0; u < NT; ++u) acc[u] = __builtin_amdgcn_mfma_f32_16x16x4f32(a, bq[u >> 2][u & 3], acc[u], 0, 0, 0);
    };
    const int nch = (fin + WK - 1) / WK;
    gload(0);
    for (int ch = 0; ch < nch; ++ch) {
      const int k0 = ch * WK;
      __syncthreads();  // the layer input is complete; the previous chunk is consumed
#pragma unroll
      for (int p = 0; p < PER; ++p) {
        const int q = t + 256 * p, k = q / (16 * NQ), lc = (q / NQ) % 16, u4 = q % NQ;
        if (q < RUNS) *reinterpret_cast<f32x4_t*>(&sW[wrun(k, lc, u4)]) = pre[p];
      }
      __syncthreads();
      if (ch + 1 < nch) gload(k0 + WK);
      if (fin - k0 >= WK) {
#pragma unroll
        for (int s4 = 0; s4 < WK; s4 += 4) step(k0, s4);
      } else {
        for (int s4 = 0; s4 < fin - k0; s4 += 4) step(k0, s4);
      }
    }
    __syncthreads();  // every wave has read the layer input
    // D[m][c] at lane c + 16 (m / 4), element m % 4
#pragma unroll
    for (int u = 0; u < NT; ++u) {
      const int c = 16 * u + l16;
      const float bc = bl[c];
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        float val = 1.f * acc[u][r];
        val += bc;
        sH[hidx(16 * w + 4 * kq + r, c)] = tanhf(val);
      }
    }
    Wl = bl + HID;
    fin = HID;
  }
  // output layer: one column of weights, read directly
  __syncthreads();
  const float* bl = Wl + fin;
  f32x4_t acc = f32x4_t{0.f, 0.f, 0.f, 0.f};
  for (int k = 0; k < fin; k += 4) {
    const float a = sH[hidx(mrow, k + kq)];
    const float b = l16 == 0 ? Wl[k + kq] : 0.f;
    acc = __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, acc, 0, 0, 0);
  }
  if (l16 == 0) {
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const long m = r0 + 16 * w + 4 * kq + r;
      float val = 1.f * acc[r];
      val += bl[0];
      if (m < n) y[m] = val;
    }
  }
}

inline unsigned nblk(long n) { return static_cast<unsigned>((n + 255) / 256); }

inline bool infer_ok(const ri_mlp* net) {
  return net->d_in % 4 == 0 && net->d_in <= HMAX && net->hidden % 16 == 0 && net->hidden <= HMAX;
}

template <int NT>
static void launch_infer(const ri_mlp* net, const float* X, long n, float* y, hipStream_t s) {
  infer_kernel<NT><<<static_cast<unsigned>((n + IR - 1) / IR), 256, 0, s>>>(X, n, net->d_in, net->layers,
                                                                           net->params, y);
}
// y = net(X), n rows, by infer_kernel (chunks of 2^24 workgroups at most)
int infer(const ri_mlp* net, const float* X, long n, float* y, hipStream_t s) {
  const long step = static_cast<long>(IR) << 24;
  for (long r0 = 0; r0 < n; r0 += step) {
    const long nn = std::min(step, n - r0);
    const float* Xc = X + r0 * net->d_in;
    float* yc = y + r0;
    switch (net->hidden / 16) {
      case 1: launch_infer<1>(net, Xc, nn, yc, s); break;
      case 2: launch_infer<2>(net, Xc, nn, yc, s); break;
      case 3: launch_infer<3>(net, Xc, nn, yc, s); break;
      case 4: launch_infer<4>(net, Xc, nn, yc, s); break;
      case 5: launch_infer<5>(net, Xc, nn, yc, s); break;
      case 6: launch_infer<6>(net, Xc, nn, yc, s); break;
      case 7: launch_infer<7>(net, Xc, nn, yc, s); break;
      case 8: launch_infer<8>(net, Xc, nn, yc, s); break;
      case 9: launch_infer<9>(net, Xc, nn, yc, s); break;
      case 10: launch_infer<10>(net, Xc, nn, yc, s); break;
      case 11: launch_infer<11>(net, Xc, nn, yc, s); break;
      case 12: launch_infer<12>(net, Xc, nn, yc, s); break;
      case 13: launch_infer<13>(net, Xc, nn, yc, s); break;
      case 14: launch_infer<14>(net, Xc, nn, yc, s); break;
      case 15: launch_infer<15>(net, Xc, nn, yc, s); break;
      default: launch_infer<16>(net, Xc, nn, yc, s); break;
    }
    RI_TRY(check_launch("infer_kernel"));
  }
  return RI_OK;
}

int gemm(GemmF32 g, int splits, hipStream_t s) {
  g.kper = (g.K + splits - 1) / splits;
  const int a_kfast = (g.sak == 1 && g.sam != 1) ? 1 : 0;
  const int b_kfast = (g.sbk == 1 && g.sbn != 1) ? 1 : 0;
  dim3 grid(static_cast<unsigned>((g.N + BN - 1) / BN), static_cast<unsigned>((g.M + BM - 1) / BM), splits);
  gemm_f32_kernel<<<grid, 256, 0, s>>>(g, a_kfast, b_kfast);
  return check_launch("gemm_f32_kernel");
}

// layer k (0-based) parameter pointers
inline void layer_ptrs(const ri_mlp* net, float* base, int k, float*& W, float*& b, int& fin, int& fout) {
  size_t off = 0;
  int in = net->d_in;
  for (int l = 0; l <= net->layers; ++l) {
    const int out = l < net->layers ? net->hidden : 1;
    if (l == k) {
      W = base + off;
      b = base + off + static_cast<size_t>(in) * out;
      fin = in;
      fout = out;
      return;
    }
    off += static_cast<size_t>(in) * out + out;
    in = out;
  }
}

// scratch layout for `rows` rows: H[1..layers] [rows][h], D (delta) [rows][h] x 2, y [rows],
// dy [rows], split partials [SPLITS][h*h], loss partials [LB] + 1
constexpr int SPLITS = 32;
int reserve(ri_mlp* net, long rows, hipStream_t s) {
  if (rows <= net->rows) return RI_OK;
  const size_t h = net->hidden;
  const size_t n = static_cast<size_t>(rows);
  const size_t floats = net->layers * n * h + 2 * n * h + 2 * n + SPLITS * std::max(h * h, h * 64) + LB + 16;
  if (net->scratch) dev_free(net->scratch, s);
  net->scratch = nullptr;
  net->rows = 0;
  void* p = nullptr;
  RI_TRY(dev_alloc(&p, floats * sizeof(float), s));
  net->scratch = static_cast<float*>(p);
  net->rows = rows;
  net->scratch_bytes = floats * sizeof(float);
  return RI_OK;
}

struct Scr {
  std::vector<float*> H;  // H[1..layers]
  float *D0, *D1, *y, *dy, *part, *lpart, *loss;
};
Scr carve(const ri_mlp* net) {
  Scr c;
  const size_t h = net->hidden, n = static_cast<size_t>(net->rows);
  float* p = net->scratch;
  c.H.push_back(nullptr);
  for (int l = 0; l < net->layers; ++l) {
    c.H.push_back(p);
    p += n * h;
  }
  c.D0 = p;
  p += n * h;
  c.D1 = p;
  p += n * h;
  c.y = p;
  p += n;
  c.dy = p;
  p += n;
  c.part = p;
  p += SPLITS * std::max(h * h, h * 64);
  c.lpart = p;
  p += LB;
  c.loss = p;
  return c;
}

// y = net(X) for n <= net->rows rows; hidden activations kept in scratch
int forward(ri_mlp* net, const float* X, long n, float* y, hipStream_t s) {
  Scr c = carve(net);
  const float* in = X;
  int fin = net->d_in;
  for (int l = 0; l <= net->layers; ++l) {
    float *W, *b;
    int fi, fo;
    layer_ptrs(net, net->params, l, W, b, fi, fo);
    GemmF32 g{};
    g.M = n;
    g.N = fo;
    g.K = fi;
    g.A = in;
    g.sam = fin;
    g.sak = 1;
    g.B = W;
    g.sbk = fo;
    g.sbn = 1;
    g.bias = b;
    g.alpha = 1.f;
    g.split_stride = 0;
    if (l < net->layers) {
      g.C = c.H[l + 1];
      g.ldc = fo;
      g.act = 1;
    } else {
      g.C = y;
      g.ldc = 1;
      g.act = 0;
    }
    RI_TRY(gemm(g, 1, s));
    in = c.H[l + 1];
    fin = fo;
  }
  return RI_OK;
}

// grad (device) and loss (device scalar in scratch) for the batch
int gradient(ri_mlp* net, const float* X, const float* Y, long n, float* grad, hipStream_t s) {
  RI_TRY(forward(net, X, n, carve(net).y, s));
  Scr c = carve(net);
  mse_stage1<<<LB, 256, 0, s>>>(c.y, Y, n, c.dy, c.lpart);
  mse_stage2<<<1, 256, 0, s>>>(c.lpart, n, c.loss);
  RI_TRY(check_launch("mse"));
  // delta of the output layer: c.dy [n][1]
  const float* delta = c.dy;
  int dcols = 1;
  float* dbuf[2] = {c.D0, c.D1};
  int flip = 0;
  const long splits = std::max(1L, std::min(static_cast<long>(SPLITS), n / 256));
  for (int l = net->layers; l >= 0; --l) {
    float *W, *b, *gW, *gb;
    int fi, fo;
    layer_ptrs(net, net->params, l, W, b, fi, fo);
    layer_ptrs(net, grad, l, gW, gb, fi, fo);
    const float* Hin = l > 0 ? c.H[l] : X;
    // gW = Hin^T delta  (K = batch, deterministic split-K)
    GemmF32 g{};
    g.M = fi;
    g.N = fo;
    g.K = n;
    g.A = Hin;
    g.sam = 1;
    g.sak = fi;
    g.B = delta;
    g.sbk = dcols;
    g.sbn = 1;
    g.C = c.part;
    g.ldc = fo;
    g.bias = nullptr;
    g.act = 0;
    g.alpha = 1.f;
    g.split_stride = static_cast<long>(fi) * fo;
    RI_TRY(gemm(g, static_cast<int>(splits), s));
    sum_splits<<<nblk(static_cast<long>(fi) * fo), 256, 0, s>>>(c.part, static_cast<int>(splits),
                                                                 static_cast<long>(fi) * fo, static_cast<long>(fi) * fo, gW);
    RI_TRY(check_launch("sum_splits"));
    // gb = column sums of delta
    const long rper = (n + splits - 1) / splits;
    colsum_partial<<<dim3((fo + 255) / 256, splits), 256, 0, s>>>(delta, n, fo, rper, c.part);
    sum_splits<<<nblk(fo), 256, 0, s>>>(c.part, static_cast<int>(splits), fo, fo, gb);
    RI_TRY(check_launch("bias grad"));
    if (l == 0) break;
    // dH = delta W^T ; delta_prev = dH * (1 - H^2)
    float* dH = dbuf[flip];
    flip ^= 1;
    GemmF32 d{};
    d.M = n;
    d.N = fi;
    d.K = fo;
    d.A = delta;
    d.sam = dcols;
    d.sak = 1;
    d.B = W;
    d.sbk = 1;
    d.sbn = fo;
    d.C = dH;
    d.ldc = fi;
    d.bias = nullptr;
    d.act = 0;
    d.alpha = 1.f;
    d.split_stride = 0;
    RI_TRY(gemm(d, 1, s));
    tanh_back<<<nblk(n * fi), 256, 0, s>>>(c.H[l], dH, n * fi);
    RI_TRY(check_launch("tanh_back"));
    delta = dH;
    dcols = fi;
  }
  return RI_OK;
}

// One Adam step on net->grad with learning rate lr (beta1 0.9, beta2 0.999, eps 1e-8).
int adam_step(ri_mlp* net, float lr, hipStream_t s) {
  net->step += 1;
  const float b1 = 0.9f, b2 = 0.999f;
  const float c1 = 1.f - powf(b1, static_cast<float>(net->step)), c2 = 1.f - powf(b2, static_cast<float>(net->step));
  adam_kernel<<<nblk(net->nparams), 256, 0, s>>>(net->params, net->grad, net->m, net->v, net->nparams, lr, b1, b2,
                                                 1e-8f, c1, c2);
  return check_launch("adam_kernel");
}

// Learning rate of step `it` of `total`: linear warm-up over `warm` steps, then
// cosine decay to zero (evaluated in double, rounded once to float).
inline float schedule(float lr, long it, long warm, long total) {
  const double ramp = std::min(1.0, static_cast<double>(it + 1) / static_cast<double>(warm));
  const double cosine = 1.0 + cos(3.141592653589793 * static_cast<double>(it) / static_cast<double>(total));
  return static_cast<float>(static_cast<double>(lr) * ramp * 0.5 * cosine);
}

// Fisher-Yates shuffle of the identity permutation of n rows: for i = n-1 down to 1,
// swap entries i and j = floor(x (i+1) / 2^64), x the next output of the SplitMix64
// stream (counter *ctr, advanced by n-1).
void shuffle(std::vector<int>& perm, long n, unsigned long long seed, unsigned long long* ctr) {
  for (long r = 0; r < n; ++r) perm[r] = static_cast<int>(r);
  for (long i = n - 1; i >= 1; --i) {
    const unsigned long long x = splitmix64(seed, (*ctr)++);
    const long j = static_cast<long>((static_cast<unsigned __int128>(x) * static_cast<unsigned long long>(i + 1)) >> 64);
    std::swap(perm[i], perm[j]);
  }
}

int check_net(const ri_mlp* net, const char* where) {
  if (!net || !net->params) {
    set_error("%s: null network", where);
    return RI_E_ARG;
  }
  return RI_OK;
}

// ---------------------------------------------------------------- training data
// Importance sampling of amplitudes with probability proportional to t2_MP2^2, by the
// inverse of the cumulative weight: sample s takes u_s = ((x_s >> 11) + 1/2) 2^-53 of
// the total weight, x_s the SplitMix64 output s of `seed`, and picks the first index k
// whose running sum of weights exceeds it.  The running sums are formed per chunk of
// SCH elements (in index order) and over the chunks, in FP64.
constexpr long SCH = 4096;
__global__ __launch_bounds__(256) void weight_chunks(const double* __restrict__ t, long n, double* csum) {
  __shared__ double sh[256];
  const long lo = static_cast<long>(blockIdx.x) * SCH, hi = std::min(n, lo + SCH);
  double acc = 0.0;
  for (long k = lo + threadIdx.x; k < hi; k += 256) acc += t[k] * t[k];
  sh[threadIdx.x] = acc;
  __syncthreads();
  for (int st = 128; st > 0; st >>= 1) {
    if (threadIdx.x < st) sh[threadIdx.x] += sh[threadIdx.x + st];
    __syncthreads();
  }
  if (threadIdx.x == 0) csum[blockIdx.x] = sh[0];
}
// cum[c] = sum of the weights of chunks 0 .. c (one thread, chunk order)
__global__ void chunk_prefix(double* csum, long nch) {
  if (threadIdx.x || blockIdx.x) return;
  double acc = 0.0;
  for (long c = 0; c < nch; ++c) {
    acc += csum[c];
    csum[c] = acc;
  }
}
__global__ void sample_kernel(const double* __restrict__ t, long n, const double* __restrict__ cum, long nch,
                              unsigned long long seed, long ns, long* idx) {
  const long sidx = static_cast<long>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (sidx >= ns) return;
  const double total = cum[nch - 1];
  const double u = (static_cast<double>(splitmix64(seed, sidx) >> 11) + 0.5) * (1.0 / 9007199254740992.0) * total;
  long lo = 0, hi = nch - 1;  // first chunk whose cumulative weight exceeds u
  while (lo < hi) {
    const long mid = (lo + hi) / 2;
    if (cum[mid] > u) hi = mid; else lo = mid + 1;
  }
  double acc = lo > 0 ? cum[lo - 1] : 0.0;
  const long k0 = lo * SCH, k1 = std::min(n, k0 + SCH);
  long pick = k1 - 1;
  for (long k = k0; k < k1; ++k) {
    acc += t[k] * t[k];
    if (acc > u) {
      pick = k;
      break;
    }
  }
  idx[sidx] = pick;
}

// Y[s] = clamp(t2c[idx[s]] / t2m[idx[s]] - 1, -clip, clip)
__global__ void targets_kernel(const double* __restrict__ t2c, const double* __restrict__ t2m,
                               const long* __restrict__ idx, long n, float clip, float* Y) {
  const long sidx = static_cast<long>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (sidx >= n) return;
  const long k = idx[sidx];
  const double r = t2c[k] / t2m[k] - 1.0;
  Y[sidx] = static_cast<float>(fmin(fmax(r, -static_cast<double>(clip)), static_cast<double>(clip)));
}

// Column sums (FP64) of the d columns of X [n][d] and of Y [n], optionally about given
// means (squares of the deviations): part[b][c] for row chunk b, c < d + 1 (column d is Y).
// grid (nb), block 256: thread c < d + 1 of chunk b sums its column over the chunk.
constexpr int SROWS = 8192;
__global__ __launch_bounds__(256) void colstats_partial(const float* __restrict__ X, const float* __restrict__ Y,
                                                        long n, int d, const double* __restrict__ mean,
                                                        double* part) {
  const int c = threadIdx.x;
  if (c > d) return;
  const long lo = static_cast<long>(blockIdx.x) * SROWS, hi = std::min(n, lo + SROWS);
  const double m = mean ? mean[c] : 0.0;
  double acc = 0.0;
  for (long r = lo; r < hi; ++r) {
    const double x = (c < d ? static_cast<double>(X[r * d + c]) : static_cast<double>(Y[r])) - m;
    acc += mean ? x * x : x;
  }
  part[static_cast<long>(blockIdx.x) * (d + 1) + c] = acc;
}
// out[c] = sum over chunks of part[b][c] / n, chunk order
__global__ void colstats_final(const double* __restrict__ part, long nb, int d, long n, double* out) {
  const int c = threadIdx.x;
  if (c > d) return;
  double acc = 0.0;
  for (long b = 0; b < nb; ++b) acc += part[b * (d + 1) + c];
  out[c] = acc / static_cast<double>(n);
}

// Xn = (X - mean) * inv_std, Yn = Y * inv_y (in place allowed)
__global__ void standardize_kernel(const float* X, const float* Y, long n, int d, Norm nm, float inv_y, float* Xn,
                                   float* Yn) {
  const long t = static_cast<long>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (t >= n * (d + 1)) return;
  const long r = t / (d + 1);
  const int c = static_cast<int>(t - r * (d + 1));
  if (c < d)
    Xn[r * d + c] = (X[r * d + c] - nm.mean[c]) * nm.inv_std[c];
  else if (Y && Yn)
    Yn[r] = Y[r] * inv_y;
}

}  // namespace mlp
}  // namespace ri

using namespace ri;

extern "C" {

ri_mlp* ri_mlp_create(int d_in, int hidden, int layers) {
  clear_error();
  if (d_in <= 0 || hidden <= 0 || layers <= 0 || d_in > 4096 || hidden > 4096 || layers > 16) {
    set_error("ri_mlp_create: invalid sizes");
    return nullptr;
  }
  ri_mlp* net = new (std::nothrow) ri_mlp();
  if (!net) return nullptr;
  net->d_in = d_in;
  net->hidden = hidden;
  net->layers = layers;
  size_t n = 0;
  int in = d_in;
  for (int l = 0; l <= layers; ++l) {
    const int out = l < layers ? hidden : 1;
    n += static_cast<size_t>(in) * out + out;
    in = out;
  }
  net->nparams = n;
  net->mean.assign(d_in, 0.f);
  net->stdv.assign(d_in, 1.f);
  float* p = nullptr;
  if (hipMalloc(&p, 4 * n * sizeof(float)) != hipSuccess) {
    (void)hipGetLastError();
    set_error("ri_mlp_create: out of device memory");
    delete net;
    return nullptr;
  }
  if (hipMemset(p, 0, 4 * n * sizeof(float)) != hipSuccess) {
    (void)hipGetLastError();
    (void)hipFree(p);
    delete net;
    return nullptr;
  }
  net->params = p;
  net->grad = p + n;
  net->m = p + 2 * n;
  net->v = p + 3 * n;
  return net;
}

void ri_mlp_destroy(ri_mlp* net) {
  if (!net) return;
  if (net->scratch) (void)hipFree(net->scratch);
  if (net->params) (void)hipFree(net->params);
  delete net;
}

size_t ri_mlp_num_params(const ri_mlp* net) { return net ? net->nparams : 0; }

int ri_mlp_set_params(ri_mlp* net, const float* params_host) {
  clear_error();
  RI_TRY(mlp::check_net(net, "ri_mlp_set_params"));
  if (!params_host) {
    set_error("ri_mlp_set_params: null pointer");
    return RI_E_ARG;
  }
  RI_HIP(hipMemcpy(net->params, params_host, net->nparams * sizeof(float), hipMemcpyHostToDevice));
  RI_HIP(hipMemset(net->m, 0, 2 * net->nparams * sizeof(float)));
  net->step = 0;
  return RI_OK;
}

int ri_mlp_get_params(const ri_mlp* net, float* params_host) {
  clear_error();
  RI_TRY(mlp::check_net(net, "ri_mlp_get_params"));
  if (!params_host) {
    set_error("ri_mlp_get_params: null pointer");
    return RI_E_ARG;
  }
  RI_HIP(hipMemcpy(params_host, net->params, net->nparams * sizeof(float), hipMemcpyDeviceToHost));
  return RI_OK;
}

int ri_mlp_set_scaling(ri_mlp* net, const float* mean, const float* std, float y_scale) {
  clear_error();
  RI_TRY(mlp::check_net(net, "ri_mlp_set_scaling"));
  if (!mean || !std || !(y_scale > 0.f)) {
    set_error("ri_mlp_set_scaling: invalid argument");
    return RI_E_ARG;
  }
  for (int k = 0; k < net->d_in; ++k)
    if (!(std[k] > 0.f)) {
      set_error("ri_mlp_set_scaling: std must be positive");
      return RI_E_ARG;
    }
  net->mean.assign(mean, mean + net->d_in);
  net->stdv.assign(std, std + net->d_in);
  net->y_scale = y_scale;
  return RI_OK;
}

int ri_mlp_get_scaling(const ri_mlp* net, float* mean, float* std, float* y_scale) {
  clear_error();
  RI_TRY(mlp::check_net(net, "ri_mlp_get_scaling"));
  if (mean) memcpy(mean, net->mean.data(), net->d_in * sizeof(float));
  if (std) memcpy(std, net->stdv.data(), net->d_in * sizeof(float));
  if (y_scale) *y_scale = net->y_scale;
  return RI_OK;
}

int ri_mlp_forward(ri_mlp* net, const float* X, long n, float* y, void* stream) {
  clear_error();
  RI_TRY(mlp::check_net(net, "ri_mlp_forward"));
  if (!X || !y || n <= 0) {
    set_error("ri_mlp_forward: invalid argument");
    return RI_E_ARG;
  }
  hipStream_t s = static_cast<hipStream_t>(stream);
  const long chunk = 1L << 20;
  RI_TRY(mlp::reserve(net, std::min(n, chunk), s));
  for (long r0 = 0; r0 < n; r0 += chunk) {
    const long nn = std::min(chunk, n - r0);
    RI_TRY(mlp::forward(net, X + r0 * net->d_in, nn, y + r0, s));
  }
  return RI_OK;
}

int ri_mlp_gradient(ri_mlp* net, const float* X, const float* Y, long n, float* grad, float* loss_host, void* stream) {
  clear_error();
  RI_TRY(mlp::check_net(net, "ri_mlp_gradient"));
  if (!X || !Y || n <= 0 || n > (1L << 24)) {
    set_error("ri_mlp_gradient: invalid argument");
    return RI_E_ARG;
  }
  hipStream_t s = static_cast<hipStream_t>(stream);
  RI_TRY(mlp::reserve(net, n, s));
  float* g = grad ? grad : net->grad;
  RI_TRY(mlp::gradient(net, X, Y, n, g, s));
  if (loss_host) {
    RI_HIP(hipMemcpyAsync(loss_host, mlp::carve(net).loss, sizeof(float), hipMemcpyDeviceToHost, s));
    RI_HIP(hipStreamSynchronize(s));
  }
  return RI_OK;
}

int ri_mlp_train_step(ri_mlp* net, const float* X, const float* Y, long n, float lr, float* loss_host, void* stream) {
  clear_error();
  RI_TRY(mlp::check_net(net, "ri_mlp_train_step"));
  if (!X || !Y || n <= 0 || n > (1L << 24) || !(lr > 0.f)) {
    set_error("ri_mlp_train_step: invalid argument");
    return RI_E_ARG;
  }
  hipStream_t s = static_cast<hipStream_t>(stream);
  RI_TRY(mlp::reserve(net, n, s));
  RI_TRY(mlp::gradient(net, X, Y, n, net->grad, s));
  RI_TRY(mlp::adam_step(net, lr, s));
  if (loss_host) {
    RI_HIP(hipMemcpyAsync(loss_host, mlp::carve(net).loss, sizeof(float), hipMemcpyDeviceToHost, s));
    RI_HIP(hipStreamSynchronize(s));
  }
  return RI_OK;
}

int ri_mlp_init(ri_mlp* net, unsigned long long seed, void* stream) {
  clear_error();
  RI_TRY(mlp::check_net(net, "ri_mlp_init"));
  hipStream_t s = static_cast<hipStream_t>(stream);
  long off = 0;
  for (int l = 0; l <= net->layers; ++l) {
    float *W, *b;
    int fi, fo;
    mlp::layer_ptrs(net, net->params, l, W, b, fi, fo);
    const long cnt = static_cast<long>(fi) * fo + fo;
    mlp::init_layer<<<mlp::nblk(cnt), 256, 0, s>>>(net->params, off, fi, fo, seed);
    RI_TRY(check_launch("init_layer"));
    off += cnt;
  }
  RI_HIP(hipMemsetAsync(net->m, 0, 2 * net->nparams * sizeof(float), s));
  net->step = 0;
  return RI_OK;
}

void ri_mlp_default_train_opts(ri_mlp_train_opts* opts) {
  if (!opts) return;
  opts->epochs = 30;
  opts->batch = 4096;
  opts->lr = 5e-4f;
  opts->warmup = 0.05f;
  opts->seed = 1;
  opts->shuffle = 1;
}

int ri_mlp_train(ri_mlp* net, const float* X, const float* Y, long n, const float* X_val, const float* Y_val,
                 long n_val, const ri_mlp_train_opts* opts, float* train_loss, float* val_loss, void* stream) {
  clear_error();
  RI_TRY(mlp::check_net(net, "ri_mlp_train"));
  ri_mlp_train_opts o;
  ri_mlp_default_train_opts(&o);
  if (opts) o = *opts;
  if (!X || !Y || n <= 0 || n > (1L << 28)) {
    set_error("ri_mlp_train: need X and Y with 1 <= n <= 2^28 rows");
    return RI_E_ARG;
  }
  if (o.epochs <= 0 || o.epochs > 1000000 || o.batch <= 0 || o.batch > (1L << 24) || !(o.lr > 0.f) ||
      !std::isfinite(o.lr) || !(o.warmup >= 0.f && o.warmup <= 1.f)) {
    set_error("ri_mlp_train: invalid options (epochs %d, batch %ld, lr %g, warmup %g)", o.epochs, o.batch,
              static_cast<double>(o.lr), static_cast<double>(o.warmup));
    return RI_E_ARG;
  }
  if (n_val < 0 || n_val > (1L << 28) || (n_val > 0 && (!X_val || !Y_val)) || (val_loss && n_val == 0)) {
    set_error("ri_mlp_train: invalid validation set (n_val %ld)", n_val);
    return RI_E_ARG;
  }
  hipStream_t s = static_cast<hipStream_t>(stream);
  const int d = net->d_in;
  const long bs = std::min(o.batch, n);
  const long steps = std::max(1L, n / o.batch);
  const long total = static_cast<long>(o.epochs) * steps;
  const long warm = std::max(1L, static_cast<long>(static_cast<double>(total) * static_cast<double>(o.warmup)));
  RI_TRY(mlp::reserve(net, bs, s));

  // workspace: shuffled X [n][d] and Y [n], validation outputs [n_val], loss
  // histories [2][epochs], permutation [n]
  const size_t nf = (o.shuffle ? static_cast<size_t>(n) * (d + 1) : 0) + static_cast<size_t>(n_val) +
                    2 * static_cast<size_t>(o.epochs);
  const size_t bytes = round_up(nf * sizeof(float), 256) + (o.shuffle ? static_cast<size_t>(n) * sizeof(int) : 0);
  std::vector<int> hperm[2];
  std::vector<float> hist(2 * static_cast<size_t>(o.epochs));
  struct Guard {
    void* ws = nullptr;
    hipEvent_t ev[2] = {nullptr, nullptr};
    hipStream_t s;
    ~Guard() {
      for (hipEvent_t e : ev)
        if (e) {
          (void)hipEventSynchronize(e);  // the copy that reads a host permutation has finished
          (void)hipEventDestroy(e);
        }
      if (ws) dev_free(ws, s);
    }
  } g;
  g.s = s;
  RI_TRY(dev_alloc(&g.ws, bytes, s));
  float* fp = static_cast<float*>(g.ws);
  float* Xs = fp;
  float* Ys = Xs + (o.shuffle ? static_cast<size_t>(n) * d : 0);
  float* yv = Ys + (o.shuffle ? n : 0);
  float* tl = yv + n_val;
  float* vl = tl + o.epochs;
  int* dperm = reinterpret_cast<int*>(reinterpret_cast<char*>(g.ws) + round_up(nf * sizeof(float), 256));
  RI_HIP(hipMemsetAsync(tl, 0, 2 * static_cast<size_t>(o.epochs) * sizeof(float), s));
  if (o.shuffle) {
    for (int k = 0; k < 2; ++k) {
      hperm[k].resize(n);
      RI_HIP(hipEventCreateWithFlags(&g.ev[k], hipEventDisableTiming));
    }
  }
  unsigned long long ctr = 0;
  long it = 0;
  for (int ep = 0; ep < o.epochs; ++ep) {
    const float* Xe = X;
    const float* Ye = Y;
    if (o.shuffle) {
      const int k = ep & 1;
      RI_HIP(hipEventSynchronize(g.ev[k]));  // the copy from this host buffer two epochs ago is done
      mlp::shuffle(hperm[k], n, o.seed, &ctr);
      RI_HIP(hipMemcpyAsync(dperm, hperm[k].data(), static_cast<size_t>(n) * sizeof(int), hipMemcpyHostToDevice, s));
      RI_HIP(hipEventRecord(g.ev[k], s));
      mlp::gather_rows<<<mlp::nblk(n * (d + 1)), 256, 0, s>>>(X, Y, dperm, n, d, Xs, Ys);
      RI_TRY(check_launch("gather_rows"));
      Xe = Xs;
      Ye = Ys;
    }
    for (long st = 0; st < steps; ++st, ++it) {
      const long r0 = st * bs;
      RI_TRY(mlp::gradient(net, Xe + r0 * d, Ye + r0, bs, net->grad, s));
      mlp::add_scaled<<<1, 64, 0, s>>>(tl + ep, mlp::carve(net).loss, 1.f / static_cast<float>(steps));
      RI_TRY(check_launch("add_scaled"));
      RI_TRY(mlp::adam_step(net, mlp::schedule(o.lr, it, warm, total), s));
    }
    if (n_val > 0) {
      for (long r0 = 0; r0 < n_val; r0 += bs) {
        const long nn = std::min(bs, n_val - r0);
        RI_TRY(mlp::forward(net, X_val + r0 * d, nn, yv + r0, s));
      }
      mlp::Scr c = mlp::carve(net);
      mlp::mse_stage1<<<mlp::LB, 256, 0, s>>>(yv, Y_val, n_val, nullptr, c.lpart);
      mlp::mse_stage2<<<1, 256, 0, s>>>(c.lpart, n_val, vl + ep);
      RI_TRY(check_launch("validation loss"));
    }
  }
  if (train_loss || val_loss) {
    RI_HIP(hipMemcpyAsync(hist.data(), tl, hist.size() * sizeof(float), hipMemcpyDeviceToHost, s));
    RI_HIP(hipStreamSynchronize(s));
    if (train_loss) memcpy(train_loss, hist.data(), o.epochs * sizeof(float));
    if (val_loss) memcpy(val_loss, hist.data() + o.epochs, o.epochs * sizeof(float));
    for (int ep = 0; ep < o.epochs; ++ep)
      if (!std::isfinite(hist[ep]) || (val_loss && !std::isfinite(hist[o.epochs + ep]))) {
        set_error("ri_mlp_train: loss is not finite after epoch %d", ep + 1);
        return RI_E_NUMERIC;
      }
  }
  return RI_OK;
}

int ri_mlp_features(const ri_system* sys, const double* t2_mp2, float* X, void* stream) {
  clear_error();
  RI_TRY(cc::check_system(sys, "ri_mlp_features"));
  if (!t2_mp2 || !X) {
    set_error("ri_mlp_features: null pointer");
    return RI_E_ARG;
  }
  hipStream_t s = static_cast<hipStream_t>(stream);
  const long n = static_cast<long>(sys->o) * sys->o * sys->v * sys->v;
  void* buf = nullptr;
  RI_TRY(dev_alloc(&buf, static_cast<size_t>(n) * sizeof(double), s));
  double* gov = static_cast<double*>(buf);
  int rc = cc::ovov_integrals(sys, gov, s);
  if (rc == RI_OK) {
    mlp::Norm nm{};
    nm.on = 0;
    mlp::features_kernel<<<mlp::nblk(n), 256, 0, s>>>(gov, sys->eps, t2_mp2, sys->o, sys->v, 0, n, nm, X);
    rc = check_launch("features_kernel");
  }
  dev_free(buf, s);
  return rc;
}

int ri_mlp_sample(const double* t2_mp2, long total, long n, unsigned long long seed, long* idx, void* stream) {
  clear_error();
  if (!t2_mp2 || !idx || total <= 0 || n <= 0 || n > (1L << 30)) {
    set_error("ri_mlp_sample: invalid argument");
    return RI_E_ARG;
  }
  hipStream_t s = static_cast<hipStream_t>(stream);
  const long nch = (total + mlp::SCH - 1) / mlp::SCH;
  void* buf = nullptr;
  RI_TRY(dev_alloc(&buf, static_cast<size_t>(nch) * sizeof(double), s));
  double* cum = static_cast<double*>(buf);
  double total_w = 0.0;
  int rc = RI_OK;
  do {
    mlp::weight_chunks<<<static_cast<unsigned>(nch), 256, 0, s>>>(t2_mp2, total, cum);
    if ((rc = check_launch("weight_chunks"))) break;
    mlp::chunk_prefix<<<1, 64, 0, s>>>(cum, nch);
    if ((rc = check_launch("chunk_prefix"))) break;
    if ((rc = check_hip(hipMemcpyAsync(&total_w, cum + nch - 1, sizeof(double), hipMemcpyDeviceToHost, s),
                        "ri_mlp_sample copy")))
      break;
    if ((rc = check_hip(hipStreamSynchronize(s), "ri_mlp_sample sync"))) break;
    if (!(total_w > 0.0) || !std::isfinite(total_w)) {
      set_error("ri_mlp_sample: the weights sum to %g", total_w);
      rc = RI_E_NUMERIC;
      break;
    }
    mlp::sample_kernel<<<mlp::nblk(n), 256, 0, s>>>(t2_mp2, total, cum, nch, seed, n, idx);
    rc = check_launch("sample_kernel");
  } while (false);
  dev_free(buf, s);
  return rc;
}

int ri_mlp_targets(const double* t2_ccsd, const double* t2_mp2, const long* idx, long n, float clip, float* Y,
                   void* stream) {
  clear_error();
  if (!t2_ccsd || !t2_mp2 || !idx || !Y || n <= 0 || !(clip > 0.f)) {
    set_error("ri_mlp_targets: invalid argument");
    return RI_E_ARG;
  }
  mlp::targets_kernel<<<mlp::nblk(n), 256, 0, static_cast<hipStream_t>(stream)>>>(t2_ccsd, t2_mp2, idx, n, clip,
                                                                                 Y);
  return check_launch("targets_kernel");
}

int ri_mlp_fit_scaling(ri_mlp* net, const float* X, const float* Y, long n, void* stream) {
  clear_error();
  RI_TRY(mlp::check_net(net, "ri_mlp_fit_scaling"));
  if (!X || !Y || n <= 0 || net->d_in + 1 > 256) {
    set_error("ri_mlp_fit_scaling: invalid argument");
    return RI_E_ARG;
  }
  hipStream_t s = static_cast<hipStream_t>(stream);
  const int d = net->d_in;
  const long nb = (n + mlp::SROWS - 1) / mlp::SROWS;
  void* buf = nullptr;
  RI_TRY(dev_alloc(&buf, (static_cast<size_t>(nb) * (d + 1) + 2 * (d + 1)) * sizeof(double), s));
  double* part = static_cast<double*>(buf);
  double* mean = part + nb * (d + 1);
  double* var = mean + (d + 1);
  std::vector<double> hm(d + 1), hv(d + 1);
  int rc = RI_OK;
  do {
    mlp::colstats_partial<<<static_cast<unsigned>(nb), 256, 0, s>>>(X, Y, n, d, nullptr, part);
    mlp::colstats_final<<<1, 256, 0, s>>>(part, nb, d, n, mean);
    mlp::colstats_partial<<<static_cast<unsigned>(nb), 256, 0, s>>>(X, Y, n, d, mean, part);
    mlp::colstats_final<<<1, 256, 0, s>>>(part, nb, d, n, var);
    if ((rc = check_launch("colstats"))) break;
    if ((rc = check_hip(hipMemcpyAsync(hm.data(), mean, (d + 1) * sizeof(double), hipMemcpyDeviceToHost, s),
                        "ri_mlp_fit_scaling copy")))
      break;
    if ((rc = check_hip(hipMemcpyAsync(hv.data(), var, (d + 1) * sizeof(double), hipMemcpyDeviceToHost, s),
                        "ri_mlp_fit_scaling copy")))
      break;
    rc = check_hip(hipStreamSynchronize(s), "ri_mlp_fit_scaling sync");
  } while (false);
  dev_free(buf, s);
  RI_TRY(rc);
  for (int c = 0; c <= d; ++c)
    if (!std::isfinite(hm[c]) || !std::isfinite(hv[c])) {
      set_error("ri_mlp_fit_scaling: non-finite statistics in column %d", c);
      return RI_E_NUMERIC;
    }
  for (int c = 0; c < d; ++c) {
    const float sd = static_cast<float>(std::sqrt(hv[c]));
    net->mean[c] = static_cast<float>(hm[c]);
    net->stdv[c] = sd > 0.f ? sd : 1.f;
  }
  const float ys = static_cast<float>(std::sqrt(hv[d]));
  net->y_scale = ys > 0.f ? ys : 1.f;
  return RI_OK;
}

int ri_mlp_standardize(const ri_mlp* net, const float* X, const float* Y, long n, float* Xn, float* Yn,
                       void* stream) {
  clear_error();
  RI_TRY(mlp::check_net(net, "ri_mlp_standardize"));
  if (!X || !Xn || n <= 0 || (Y == nullptr) != (Yn == nullptr) || net->d_in > mlp::NF) {
    set_error("ri_mlp_standardize: invalid argument");
    return RI_E_ARG;
  }
  mlp::Norm nm{};
  for (int c = 0; c < net->d_in; ++c) {
    nm.mean[c] = net->mean[c];
    nm.inv_std[c] = 1.f / net->stdv[c];
  }
  nm.on = 1;
  const long total = n * (net->d_in + 1);
  mlp::standardize_kernel<<<mlp::nblk(total), 256, 0, static_cast<hipStream_t>(stream)>>>(
      X, Y, n, net->d_in, nm, 1.f / net->y_scale, Xn, Yn);
  return check_launch("standardize_kernel");
}

int ri_mlp_guess(ri_mlp* net, const ri_system* sys, double* t1, double* t2, void* stream) {
  clear_error();
  RI_TRY(mlp::check_net(net, "ri_mlp_guess"));
  RI_TRY(cc::check_system(sys, "ri_mlp_guess"));
  if (!t1 || !t2 || net->d_in != mlp::NF) {
    set_error("ri_mlp_guess: null amplitudes or a network without %d inputs", mlp::NF);
    return RI_E_ARG;
  }
  hipStream_t s = static_cast<hipStream_t>(stream);
  const int o = sys->o, v = sys->v;
  const long n = static_cast<long>(o) * o * v * v;
  // the network sees the i <= j half of the amplitudes; t2 is pair-symmetric
  const long nh = static_cast<long>(o) * (o + 1) / 2 * v * v;
  const bool fused = mlp::infer_ok(net);
  const long chunk = std::min(nh, fused ? (1L << 22) : (1L << 20));
  // gov [o][v][o][v], an unmodified copy of the MP2 t2 (features read it), X and y of a chunk
  const size_t gbytes = round_up(static_cast<size_t>(n) * sizeof(double), 256);
  void* buf = nullptr;
  RI_TRY(dev_alloc(&buf, 2 * gbytes + static_cast<size_t>(chunk) * (mlp::NF + 1) * sizeof(float), s));
  double* gov = static_cast<double*>(buf);
  double* t2m = reinterpret_cast<double*>(static_cast<char*>(buf) + gbytes);
  float* X = reinterpret_cast<float*>(static_cast<char*>(buf) + 2 * gbytes);
  float* y = X + chunk * mlp::NF;
  mlp::Norm nm{};
  nm.on = 1;
  for (int k = 0; k < mlp::NF; ++k) {
    nm.mean[k] = net->mean[k];
    nm.inv_std[k] = 1.f / net->stdv[k];
  }
  int rc = cc::mp2_with_integrals(sys, gov, t1, t2m, s);
  if (rc == RI_OK && !fused) rc = mlp::reserve(net, chunk, s);
  for (long r0 = 0; r0 < nh && rc == RI_OK; r0 += chunk) {
    const long nn = std::min(chunk, nh - r0);
    mlp::features_half_kernel<<<mlp::nblk(nn), 256, 0, s>>>(gov, sys->eps, t2m, o, v, r0, nn, nm, X);
    if ((rc = check_launch("features_half_kernel"))) break;
    if (fused) {
      rc = mlp::infer(net, X, nn, y, s);
    } else {
      rc = mlp::forward(net, X, nn, y, s);
    }
    if (rc) break;
    mlp::add_correction_half<<<mlp::nblk(nn), 256, 0, s>>>(t2, t2m, o, v, r0, nn, y, net->y_scale);
    rc = check_launch("add_correction_half");
  }
  // averages the i == j entries over (a, b) <-> (b, a); the other pairs are equal already
  if (rc == RI_OK) rc = cc::symmetrize_pairs(t2, o, v, s);
  dev_free(buf, s);
  return rc;
}

int ri_mlp_infer(const ri_mlp* net, const float* X, long n, float* y, void* stream) {
  clear_error();
  RI_TRY(mlp::check_net(net, "ri_mlp_infer"));
  if (!X || !y || n <= 0) {
    set_error("ri_mlp_infer: invalid argument");
    return RI_E_ARG;
  }
  if (!mlp::infer_ok(net)) {
    set_error("ri_mlp_infer: needs d_in a multiple of 4 and hidden a multiple of 16, both at most %d (d_in %d, "
              "hidden %d)", mlp::HMAX, net->d_in, net->hidden);
    return RI_E_ARG;
  }
  return mlp::infer(net, X, n, y, static_cast<hipStream_t>(stream));
}

int ri_mlp_save(const ri_mlp* net, const char* path) {
  clear_error();
  RI_TRY(mlp::check_net(net, "ri_mlp_save"));
  if (!path) {
    set_error("ri_mlp_save: null path");
    return RI_E_ARG;
  }
  std::vector<float> p(net->nparams);
  RI_HIP(hipMemcpy(p.data(), net->params, p.size() * sizeof(float), hipMemcpyDeviceToHost));
  FILE* f = fopen(path, "wb");
  if (!f) {
    set_error("ri_mlp_save: cannot open %s", path);
    return RI_E_ARG;
  }
  const int hdr[4] = {0x504c4d52, net->d_in, net->hidden, net->layers};  // "RMLP"
  bool ok = fwrite(hdr, sizeof(hdr), 1, f) == 1 && fwrite(net->mean.data(), sizeof(float), net->d_in, f) == (size_t)net->d_in &&
            fwrite(net->stdv.data(), sizeof(float), net->d_in, f) == (size_t)net->d_in &&
            fwrite(&net->y_scale, sizeof(float), 1, f) == 1 && fwrite(p.data(), sizeof(float), p.size(), f) == p.size();
  ok = (fclose(f) == 0) && ok;
  if (!ok) {
    set_error("ri_mlp_save: write to %s failed", path);
    return RI_E_ARG;
  }
  return RI_OK;
}

ri_mlp* ri_mlp_load(const char* path) {
  clear_error();
  if (!path) {
    set_error("ri_mlp_load: null path");
    return nullptr;
  }
  FILE* f = fopen(path, "rb");
  if (!f) {
    set_error("ri_mlp_load: cannot open %s", path);
    return nullptr;
  }
  int hdr[4];
  ri_mlp* net = nullptr;
  if (fread(hdr, sizeof(hdr), 1, f) == 1 && hdr[0] == 0x504c4d52) net = ri_mlp_create(hdr[1], hdr[2], hdr[3]);
  bool ok = net != nullptr;
  if (ok) {
    std::vector<float> mean(net->d_in), stdv(net->d_in), p(net->nparams);
    float ys = 0.f;
    ok = fread(mean.data(), sizeof(float), net->d_in, f) == (size_t)net->d_in &&
         fread(stdv.data(), sizeof(float), net->d_in, f) == (size_t)net->d_in && fread(&ys, sizeof(float), 1, f) == 1 &&
         fread(p.data(), sizeof(float), p.size(), f) == p.size();
    ok = ok && ri_mlp_set_scaling(net, mean.data(), stdv.data(), ys) == RI_OK && ri_mlp_set_params(net, p.data()) == RI_OK;
  }
  fclose(f);
  if (!ok) {
    ri_mlp_destroy(net);
    set_error("ri_mlp_load: %s is not a valid network file", path);
    return nullptr;
  }
  return net;
}

}  // extern "C"
