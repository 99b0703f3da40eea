// Particle-particle ladder on MI355X (gfx950), FP64 MFMA path.
//
//   R[i][j][a][b] += sum_cd (ac|bd) tau[i][j][c][d],  (ac|bd) = sum_Q B[Q][a][c] B[Q][b][d]
//
// (Sec. II.C, eq. pp-Ladder-0 with eq. RIM.)  The integrals are never stored at v^4
// size.  The contraction uses Scuseria's symmetric/antisymmetric split of the
// amplitudes (the 1/4-cost form mentioned in Sec. II.C):
//
//   tau(+-)^{cd}_{ij} = (tau^{cd}_{ij} +- tau^{dc}_{ij}) / 2           (pair-symmetric tau)
//   V(+-)^{ab}_{cd}   = (ac|bd) +- (ad|bc)
//   S^{ab}_{ij} = sum_{c<=d} s_cd V+ tau+,   s_cd = 1/2 if c == d else 1    (a<=b, i<=j)
//   A^{ab}_{ij} = sum_{c<d} V- tau-                                        (a<b,  i<j)
//   L^{ab}_{ij} = S + A,  L^{ba}_{ij} = L^{ab}_{ji} = S - A,  L^{ba}_{ji} = S + A
//
// so only the a<=b half of the integrals is built and the contraction runs over
// packed c<=d / i<=j pairs.  The paper itself keeps only the i<=j symmetry and
// evaluates b^{ab}_{cd} per a with three dgemm calls (Fig. 2); here the work is
// tiled for MFMA instead.
//
// Virtual indices are grouped in blocks of 16.  A "block pair" (X <= Y) has 256
// slots x_in*16 + y_in; pairs are numbered p = Y(Y+1)/2 + X.  Slots of a
// diagonal block pair with x_in > y_in, and slots touching padding, carry zero
// amplitudes (cd side) or are skipped when unpacking (ab side).
//
// Pipeline per call (all on the caller's stream):
//   1. relayout   Bc[c][Q][a] = B_vv[Q][a][c]           (MFMA-operand layout, zero padded)
//   2. pack       T+[cd slot][i<=j], T-[cd slot][i<j]     (sigma and the 1/2 folded in)
//   3. per slab of ab block pairs:
//      build      W+-[cd slot][ab slot] = (ac|bd) +- (ad|bc)  (MFMA over Q, B staged in LDS)
//      contract   S = W+^T T+, A = W-^T T-                    (MFMA over cd slots)
//      unpack     R += mirrored S +- A                         (LDS transposes, coalesced)
#include <algorithm>
#include <cmath>
#include <cstdlib>

#include "ppl_shared.h"

namespace ri {
namespace ppl {

constexpr int KC = 16;  // auxiliary functions staged per LDS step (FP64 path)

typedef double double4_t __attribute__((ext_vector_type(4)));
typedef double double2_t __attribute__((ext_vector_type(2)));  // register-promotable (unlike double2)

// D += A B on a 16x16x4 FP64 tile: lane l supplies A[l%16][l/16] and B[l/16][l%16]
// and holds D[4r + l/16][l%16] in element r.
__device__ inline double4_t mfma_f64(double a, double b, double4_t c) {
  return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
}

// ---------------------------------------------------------------- 1. relayout
// B[q][a][c] lives at B + q*qs + a*rs + c.  grid (naux_p, vp/16, vp/16), block 256
__global__ __launch_bounds__(256) void relayout_b_f64(const double* __restrict__ B, long qs, long rs, int v,
                                                      int naux, int vp, int naux_p, double* __restrict__ Bc) {
  __shared__ double tile[TB][TB + 1];
  const int q = blockIdx.x, a0 = blockIdx.y * TB, c0 = blockIdx.z * TB;
  const int tx = threadIdx.x & 15, ty = threadIdx.x >> 4;
  const int a = a0 + ty, c = c0 + tx;
  tile[ty][tx] = (a < v && c < v && q < naux) ? B[q * qs + a * rs + c] : 0.0;
  __syncthreads();
  Bc[(static_cast<size_t>(c0 + ty) * naux_p + q) * vp + a0 + tx] = tile[tx][ty];
}

// ---------------------------------------------------------------- 2. pack
// out[slot][col], slot = pcd*256 + c_in*16 + d_in, col = packed (i,j).
// sign > 0: i<=j columns, value of tau+ (with the 1/2 on c == d);
// sign < 0: i<j columns, value of tau-.  Both taken from the pair-symmetric part
// of tau.  grid (nbp, ncol/16), block 256
__global__ __launch_bounds__(256) void pack_tau_f64(const double* __restrict__ tau, int o, int v,
                                                    int ncol, int sign, double* __restrict__ out) {
  __shared__ double sv[256][NG + 1];
  int Cb, Db;
  tri_decode(blockIdx.x, Cb, Db);
  const int t = threadIdx.x, c_in = t >> 4, d_in = t & 15;
  const int c = Cb * TB + c_in, d = Db * TB + d_in;
  const bool valid = d < v && (Cb < Db || c_in <= d_in) && (sign > 0 || c != d);
  const int nreal = sign > 0 ? o * (o + 1) / 2 : o * (o - 1) / 2;
  const size_t vv = static_cast<size_t>(v) * v;
  for (int cc = 0; cc < NG; ++cc) {
    const int col = blockIdx.y * NG + cc;
    double val = 0.0;
    if (valid && col < nreal) {
      int i, j;
      tri_decode(col, i, j);
      if (sign < 0) j += 1;
      const double* tij = tau + (static_cast<size_t>(i) * o + j) * vv;
      const double* tji = tau + (static_cast<size_t>(j) * o + i) * vv;
      const size_t cd = static_cast<size_t>(c) * v + d, dc = static_cast<size_t>(d) * v + c;
      const double x1 = tij[cd], x2 = tij[dc], x3 = tji[cd], x4 = tji[dc];
      if (sign > 0) {
        val = 0.25 * ((x1 + x4) + (x2 + x3));
        if (c == d) val *= 0.5;
      } else {
        val = 0.25 * ((x1 + x4) - (x2 + x3));
      }
    }
    sv[t][cc] = val;
  }
  __syncthreads();
  for (int r = 0; r < 16; ++r) {
    const int slot = r * 16 + (t >> 4), cc = t & 15;
    out[(static_cast<size_t>(blockIdx.x) * 256 + slot) * ncol + blockIdx.y * NG + cc] = sv[slot][cc];
  }
}

// ---------------------------------------------------------------- 3a. build
// One workgroup: ab block pair (Ab, Bb) x one quarter (8 c by 8 d) of cd block pair
// (Cb, Db).  Eight waves; wave w owns c in {2*(w>>1), +1} and d in {4*(w&1) .. +3}
// of the quarter and accumulates (ac|bd) and (ad|bc) as 16x16 (a, b) MFMA tiles.
// LDS holds, per 16-wide Q chunk, Bc for the 16 c/d rows x (16 a + 16 b) columns.
// grid (nbp*4, slab_pairs), block 512
__global__ __launch_bounds__(512) void build_w_f64(const double* __restrict__ Bc, int naux_p, int vp,
                                                   long slab0, long slab_M, int want_minus,
                                                   double* __restrict__ Wp, double* __restrict__ Wm) {
  __shared__ double lds[2][16][KC][32];  // [buf][x: 8 c then 8 d][k][e: 16 a then 16 b]
  const int quarter = blockIdx.x & 3;
  const long pcd = blockIdx.x >> 2;
  const long pab_loc = blockIdx.y;
  int Cb, Db, Ab, Bb;
  tri_decode(pcd, Cb, Db);
  tri_decode(slab0 + pab_loc, Ab, Bb);
  const int c_base = Cb * TB + (quarter >> 1) * 8;
  const int d_base = Db * TB + (quarter & 1) * 8;
  const int t = threadIdx.x, w = t >> 6, lane = t & 63;

  // global -> register -> LDS staging: 8 double2 per thread per chunk.  Offsets are
  // computed once; the chunk loop only adds the Q stride.
  size_t goff[8];
  int loff[8];
#pragma unroll
  for (int r = 0; r < 8; ++r) {
    const int p2 = t + 512 * r;  // [0, 4096)
    const int x = p2 >> 8, k = (p2 >> 4) & 15, e = (p2 & 15) * 2;
    const int cg = x < 8 ? c_base + x : d_base + (x - 8);
    const int ag = e < 16 ? Ab * TB + e : Bb * TB + (e - 16);
    goff[r] = (static_cast<size_t>(cg) * naux_p + k) * vp + ag;
    loff[r] = (x * KC + k) * 32 + e;
  }
  const size_t qstride = static_cast<size_t>(vp) * KC;  // advance one chunk of Q
  double* lds0 = &lds[0][0][0][0];
  constexpr int LBUF = 16 * KC * 32;

  double4_t acc1[2][4], acc2[2][4];
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      acc1[i][j] = double4_t{0.0, 0.0, 0.0, 0.0};
      acc2[i][j] = double4_t{0.0, 0.0, 0.0, 0.0};
    }

  const int xc0 = (w >> 1) * 2, xd0 = 8 + (w & 1) * 4;
  const int m = lane & 15, kq = lane >> 4;
  const int nchunks = naux_p / KC;
  double2_t stage[8];
#pragma unroll
  for (int r = 0; r < 8; ++r) stage[r] = *reinterpret_cast<const double2_t*>(Bc + goff[r]);
#pragma unroll
  for (int r = 0; r < 8; ++r) *reinterpret_cast<double2_t*>(lds0 + loff[r]) = stage[r];
  __syncthreads();
  for (int ch = 0; ch < nchunks; ++ch) {
    const int buf = ch & 1;
    const bool more = ch + 1 < nchunks;
    if (more) {
      const size_t qo = static_cast<size_t>(ch + 1) * qstride;
#pragma unroll
      for (int r = 0; r < 8; ++r) stage[r] = *reinterpret_cast<const double2_t*>(Bc + goff[r] + qo);
    }
#pragma unroll
    for (int s = 0; s < KC / 4; ++s) {
      const int kk = 4 * s + kq;
      double a_c[2], b_c[2], a_d[4], b_d[4];
#pragma unroll
      for (int i = 0; i < 2; ++i) {
        a_c[i] = lds[buf][xc0 + i][kk][m];
        b_c[i] = lds[buf][xc0 + i][kk][16 + m];
      }
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        a_d[j] = lds[buf][xd0 + j][kk][m];
        b_d[j] = lds[buf][xd0 + j][kk][16 + m];
      }
#pragma unroll
      for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 4; ++j) {
          acc1[i][j] = mfma_f64(a_c[i], b_d[j], acc1[i][j]);  // (ac|bd)
          acc2[i][j] = mfma_f64(a_d[j], b_c[i], acc2[i][j]);  // (ad|bc)
        }
    }
    if (more) {
      double* dst = lds0 + (buf ^ 1) * LBUF;
#pragma unroll
      for (int r = 0; r < 8; ++r) *reinterpret_cast<double2_t*>(dst + loff[r]) = stage[r];
    }
    __syncthreads();
  }

  // epilogue: W+-[slot][ab slot].  The f64 16x16x4 MFMA leaves D[4r + lane/16][lane%16]
  // in register r of each lane: row a_in = 4r + (lane>>4), column b_in = lane&15.
  const size_t col0 = static_cast<size_t>(pab_loc) * 256;
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const int c_in = (quarter >> 1) * 8 + xc0 + i;
      const int d_in = (quarter & 1) * 8 + (xd0 - 8) + j;
      const size_t row = (static_cast<size_t>(pcd) * 256 + c_in * 16 + d_in) * slab_M + col0;
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int a_in = 4 * r + (lane >> 4), b_in = lane & 15;
        const double v1 = acc1[i][j][r], v2 = acc2[i][j][r];
        Wp[row + a_in * 16 + b_in] = v1 + v2;
        if (want_minus) Wm[row + a_in * 16 + b_in] = v1 - v2;
      }
    }
}

// ---------------------------------------------------------------- 3b. contract
// C[m][n] = sum_k W[k][m] T[k][n];  tile 64 (m) x 16*NTW (n); 4 waves, wave w owns
// rows 16w..16w+15 and all columns.  grid (ncol/(16*NTW), M/64), block 256
template <int NTW>
__global__ __launch_bounds__(256) void contract_f64(const double* __restrict__ W, const double* __restrict__ T,
                                                    long K, long M, int ncol, double* __restrict__ C) {
  // W rows have stride M (the slab width); C has NTW*16*gridDim.x columns
  constexpr int BN = 16 * NTW;
  __shared__ double sA[2][KC][64];
  __shared__ double sB[2][KC][BN];
  unsigned tx, ty;
  xcd_tile(tx, ty);
  const long n0 = static_cast<long>(tx) * BN, m0 = static_cast<long>(ty) * 64;
  const int t = threadIdx.x, w = t >> 6, lane = t & 63;

  // staging offsets (computed once; the chunk loop adds k0 * row stride)
  long aoff[2], boff[NTW];
  int alo[2], blo[NTW];
#pragma unroll
  for (int r = 0; r < 2; ++r) {
    const int p2 = t + 256 * r;
    const int k = p2 >> 5, mm = (p2 & 31) * 2;
    aoff[r] = k * M + m0 + mm;
    alo[r] = k * 64 + mm;
  }
#pragma unroll
  for (int r = 0; r < NTW; ++r) {
    const int e = t + 256 * r;
    const int k = e / BN, nn = e % BN;
    boff[r] = static_cast<long>(k) * ncol + n0 + nn;
    blo[r] = k * BN + nn;
  }
  double2_t ra[2];
  double rb[NTW];
  double* sA0 = &sA[0][0][0];
  double* sB0 = &sB[0][0][0];

  double4_t acc[NTW];
#pragma unroll
  for (int u = 0; u < NTW; ++u) acc[u] = double4_t{0.0, 0.0, 0.0, 0.0};
  const int m = lane & 15, kq = lane >> 4;
  const long nchunks = K / KC;
#pragma unroll
  for (int r = 0; r < 2; ++r) ra[r] = *reinterpret_cast<const double2_t*>(W + aoff[r]);
#pragma unroll
  for (int r = 0; r < NTW; ++r) rb[r] = T[boff[r]];
#pragma unroll
  for (int r = 0; r < 2; ++r) *reinterpret_cast<double2_t*>(sA0 + alo[r]) = ra[r];
#pragma unroll
  for (int r = 0; r < NTW; ++r) sB0[blo[r]] = rb[r];
  __syncthreads();
  for (long ch = 0; ch < nchunks; ++ch) {
    const int buf = ch & 1;
    const bool more = ch + 1 < nchunks;
    if (more) {
      const long k0 = (ch + 1) * KC;
#pragma unroll
      for (int r = 0; r < 2; ++r) ra[r] = *reinterpret_cast<const double2_t*>(W + aoff[r] + k0 * M);
#pragma unroll
      for (int r = 0; r < NTW; ++r) rb[r] = T[boff[r] + k0 * ncol];
    }
#pragma unroll
    for (int s = 0; s < KC / 4; ++s) {
      const int kk = 4 * s + kq;
      const double a = sA[buf][kk][w * 16 + m];
#pragma unroll
      for (int u = 0; u < NTW; ++u) acc[u] = mfma_f64(a, sB[buf][kk][u * 16 + m], acc[u]);
    }
    if (more) {
#pragma unroll
      for (int r = 0; r < 2; ++r) *reinterpret_cast<double2_t*>(sA0 + (buf ^ 1) * KC * 64 + alo[r]) = ra[r];
#pragma unroll
      for (int r = 0; r < NTW; ++r) sB0[(buf ^ 1) * KC * BN + blo[r]] = rb[r];
    }
    __syncthreads();
  }
#pragma unroll
  for (int u = 0; u < NTW; ++u)
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const long row = m0 + w * 16 + 4 * r + kq;  // D[4r + lane/16][lane%16]
      C[row * ncol + n0 + u * 16 + m] = acc[u][r];
    }
}

// ---------------------------------------------------------------- 3c. unpack
// S and A are FP64 (FP64 path) or FP32 (mixed paths); R accumulates in FP64.
// grid (slab_pairs, ceil(po/16)), block 256
template <class T>
__global__ __launch_bounds__(256) void unpack_kernel(const T* __restrict__ S, const T* __restrict__ A,
                                                     int NP, int NM, int o, int v, long slab0,
                                                     double* __restrict__ R) {
  __shared__ double sS[256][NG + 1];
  __shared__ double sA[256][NG + 1];
  int Ab, Bb;
  tri_decode(slab0 + blockIdx.x, Ab, Bb);
  const int t = threadIdx.x;
  const int po = o * (o + 1) / 2;
  const int lam0 = blockIdx.y * NG;
  const size_t row0 = static_cast<size_t>(blockIdx.x) * 256;
  for (int r = 0; r < 16; ++r) {
    const int slot = r * 16 + (t >> 4), cc = t & 15, lam = lam0 + cc;
    double s = 0.0, x = 0.0;
    if (lam < po) {
      int i, j;
      tri_decode(lam, i, j);
      s = static_cast<double>(S[(row0 + slot) * NP + lam]);
      if (i < j) x = static_cast<double>(A[(row0 + slot) * NM + j * (j - 1) / 2 + i]);
    }
    sS[slot][cc] = s;
    sA[slot][cc] = x;
  }
  __syncthreads();
  const size_t vv = static_cast<size_t>(v) * v;
  for (int cc = 0; cc < NG; ++cc) {
    const int lam = lam0 + cc;
    if (lam >= po) break;
    int i, j;
    tri_decode(lam, i, j);
    double* Rij = R + (static_cast<size_t>(i) * o + j) * vv;
    double* Rji = R + (static_cast<size_t>(j) * o + i) * vv;
    {  // a <= b: rows contiguous in b
      const int a_in = t >> 4, b_in = t & 15;
      const int a = Ab * TB + a_in, b = Bb * TB + b_in;
      if (a < v && b < v && (Ab < Bb || a_in <= b_in)) {
        const double s = sS[a_in * 16 + b_in][cc], x = sA[a_in * 16 + b_in][cc];
        Rij[static_cast<size_t>(a) * v + b] += s + x;
        if (i != j) Rji[static_cast<size_t>(a) * v + b] += s - x;
      }
    }
    {  // mirrors with a < b: rows contiguous in a
      const int b_in = t >> 4, a_in = t & 15;
      const int a = Ab * TB + a_in, b = Bb * TB + b_in;
      if (a < v && b < v && (Ab < Bb || a_in < b_in)) {
        const double s = sS[a_in * 16 + b_in][cc], x = sA[a_in * 16 + b_in][cc];
        Rij[static_cast<size_t>(b) * v + a] += s - x;
        if (i != j) Rji[static_cast<size_t>(b) * v + a] += s + x;
      }
    }
  }
}

void launch_unpack_f32(const float* S, const float* A, int NP, int NM, int o, int v, long slab0, long npairs,
                       double* R, hipStream_t s) {
  unpack_kernel<float><<<dim3(npairs, (o * (o + 1) / 2 + NG - 1) / NG), 256, 0, s>>>(S, A, NP, NM, o, v, slab0, R);
}

// ---------------------------------------------------------------- tau
__global__ void build_tau_kernel(const double* __restrict__ t1, const double* t2, int o, int v,
                                 double* tau, size_t total) {
  const size_t idx = static_cast<size_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (idx >= total) return;
  const size_t vv = static_cast<size_t>(v) * v;
  const int b = idx % v, a = (idx / v) % v;
  const size_t ij = idx / vv;
  const int j = ij % o, i = ij / o;
  tau[idx] = t2[idx] + t1[static_cast<size_t>(i) * v + a] * t1[static_cast<size_t>(j) * v + b];
}

// ---------------------------------------------------------------- host plan
struct Plan {
  int o, v, naux;
  int nb, vp, naux_p;
  long nbp, K;
  int po, pm, NP, NM, ntw_p, ntw_m;
  long slab_bp, slab_M;
  size_t n_Bc, n_Tp, n_Tm, n_W, n_S, n_A;
  size_t bytes;
};

static bool make_plan(int o, int v, int naux, Plan& p) {
  if (o <= 0 || v <= 0 || naux <= 0) return false;
  if (o > 4096 || v > 65536 || naux > (1 << 24)) return false;
  p.o = o;
  p.v = v;
  p.naux = naux;
  p.nb = (v + TB - 1) / TB;
  p.vp = p.nb * TB;
  p.naux_p = static_cast<int>(round_up(naux, KC));
  p.nbp = static_cast<long>(p.nb) * (p.nb + 1) / 2;
  p.K = p.nbp * 256;
  p.po = o * (o + 1) / 2;
  p.pm = o * (o - 1) / 2;
  pick_ntw(p.po, 10, 64, p.ntw_p, p.NP);
  pick_ntw(p.pm, 10, 64, p.ntw_m, p.NM);
  if (p.pm == 0) p.NM = 0;
  const int nw = p.pm > 0 ? 2 : 1;
  const long budget = env_long("RI_PPL_W_BYTES", 16L << 30);
  long bp = budget / (static_cast<long>(nw) * p.K * 256 * 8);
  bp = bp < 1 ? 1 : bp;
  bp = bp > p.nbp ? p.nbp : bp;
  bp = bp > 65535 ? 65535 : bp;
  const long cap = env_long("RI_PPL_SLAB_PAIRS", bp);
  p.slab_bp = cap < bp ? cap : bp;
  p.slab_M = p.slab_bp * 256;
  p.n_Bc = static_cast<size_t>(p.vp) * p.naux_p * p.vp;
  p.n_Tp = static_cast<size_t>(p.K) * p.NP;
  p.n_Tm = static_cast<size_t>(p.K) * p.NM;
  p.n_W = static_cast<size_t>(p.K) * p.slab_M;
  p.n_S = static_cast<size_t>(p.slab_M) * p.NP;
  p.n_A = static_cast<size_t>(p.slab_M) * p.NM;
  size_t b = 0;
  for (size_t n : {p.n_Bc, p.n_Tp, p.n_Tm, p.n_W, p.pm > 0 ? p.n_W : 0, p.n_S, p.n_A})
    b = round_up(b, 256) + n * sizeof(double);
  p.bytes = round_up(b, 256);
  return true;
}

// rows: number of C rows (multiple of 64) computed; ldw: row stride of W
template <int NTW>
static void launch_contract_t(const double* W, const double* T, long K, long ldw, long rows, int ncol,
                              double* C, hipStream_t s) {
  dim3 grid(ncol / (16 * NTW), rows / 64);
  contract_f64<NTW><<<grid, 256, 0, s>>>(W, T, K, ldw, ncol, C);
}

static void launch_contract(int ntw, const double* W, const double* T, long K, long ldw, long rows,
                            int ncol, double* C, hipStream_t s) {
  switch (ntw) {
    case 1: launch_contract_t<1>(W, T, K, ldw, rows, ncol, C, s); break;
    case 2: launch_contract_t<2>(W, T, K, ldw, rows, ncol, C, s); break;
    case 3: launch_contract_t<3>(W, T, K, ldw, rows, ncol, C, s); break;
    case 4: launch_contract_t<4>(W, T, K, ldw, rows, ncol, C, s); break;
    case 5: launch_contract_t<5>(W, T, K, ldw, rows, ncol, C, s); break;
    case 6: launch_contract_t<6>(W, T, K, ldw, rows, ncol, C, s); break;
    case 7: launch_contract_t<7>(W, T, K, ldw, rows, ncol, C, s); break;
    case 8: launch_contract_t<8>(W, T, K, ldw, rows, ncol, C, s); break;
    case 9: launch_contract_t<9>(W, T, K, ldw, rows, ncol, C, s); break;
    default: launch_contract_t<10>(W, T, K, ldw, rows, ncol, C, s); break;
  }
}

static int run_f64(const Plan& p, const double* B_vv, long qs, long rs, const double* tau, double* R,
                   void* ws, hipStream_t s) {
  Carve cv(ws, p.bytes);
  double* Bc = cv.take<double>(p.n_Bc);
  double* Tp = cv.take<double>(p.n_Tp);
  double* Tm = cv.take<double>(p.n_Tm);
  double* Wp = cv.take<double>(p.n_W);
  double* Wm = cv.take<double>(p.pm > 0 ? p.n_W : 0);
  double* S = cv.take<double>(p.n_S);
  double* A = cv.take<double>(p.n_A);

  const double vv = static_cast<double>(p.v) * p.v, oo = static_cast<double>(p.o) * p.o;
  const double pv = p.v * (p.v + 1.0) / 2, pvm = p.v * (p.v - 1.0) / 2;
  {
    ProfScope ps(s, "relayout_b_f64", 0.0, 8.0 * vv * p.naux * 2);
    relayout_b_f64<<<dim3(p.naux_p, p.nb, p.nb), 256, 0, s>>>(B_vv, qs, rs, p.v, p.naux, p.vp, p.naux_p, Bc);
    RI_TRY(check_launch("relayout_b_f64"));
  }
  {
    ProfScope ps(s, "pack_tau_f64", 0.0, 8.0 * (oo * vv + pv * p.po + pvm * p.pm));
    pack_tau_f64<<<dim3(p.nbp, p.NP / NG), 256, 0, s>>>(tau, p.o, p.v, p.NP, +1, Tp);
    RI_TRY(check_launch("pack_tau_f64(+)"));
    if (p.pm > 0) {
      pack_tau_f64<<<dim3(p.nbp, p.NM / NG), 256, 0, s>>>(tau, p.o, p.v, p.NM, -1, Tm);
      RI_TRY(check_launch("pack_tau_f64(-)"));
    }
  }
  for (long slab0 = 0; slab0 < p.nbp; slab0 += p.slab_bp) {
    const long npairs = (p.nbp - slab0) < p.slab_bp ? (p.nbp - slab0) : p.slab_bp;
    const long M = npairs * 256;
    double le, lt;
    count_pairs(p.v, slab0, npairs, le, lt);
    {
      // per valid (a <= b): the v x v matrix (ac|bd) over all c, d, naux products each
      ProfScope ps(s, "build_w_f64", 2.0 * p.naux * vv * le);
      build_w_f64<<<dim3(p.nbp * 4, npairs), 512, 0, s>>>(Bc, p.naux_p, p.vp, slab0, p.slab_M,
                                                          p.pm > 0 ? 1 : 0, Wp, Wm);
      RI_TRY(check_launch("build_w_f64"));
    }
    {
      ProfScope ps(s, "contract_f64", 2.0 * (le * pv * p.po + lt * pvm * p.pm));
      launch_contract(p.ntw_p, Wp, Tp, p.K, p.slab_M, M, p.NP, S, s);
      RI_TRY(check_launch("contract_f64(+)"));
      if (p.pm > 0) {
        launch_contract(p.ntw_m, Wm, Tm, p.K, p.slab_M, M, p.NM, A, s);
        RI_TRY(check_launch("contract_f64(-)"));
      }
    }
    {
      ProfScope ps(s, "unpack_f64", 0.0, 16.0 * oo * (le + lt));
      unpack_kernel<double><<<dim3(npairs, (p.po + NG - 1) / NG), 256, 0, s>>>(S, A, p.NP, p.NM, p.o, p.v, slab0, R);
      RI_TRY(check_launch("unpack_f64"));
    }
  }
  return RI_OK;
}

}  // namespace ppl

int ppl_strided(const double* B, long qs, long rs, const double* tau, int o, int v, int naux, double* R,
                int precision, hipStream_t s) {
  ppl::Plan p;
  if (!ppl::make_plan(o, v, naux, p)) {
    set_error("ladder: invalid sizes o=%d v=%d naux=%d", o, v, naux);
    return RI_E_ARG;
  }
  if (precision == RI_PREC_BF16X3) return ppl::bf16x3_run(B, qs, rs, tau, o, v, naux, R, nullptr, 0, s);
  if (precision != RI_PREC_FP64) {
    set_error("ladder: precision %d not available in this build", precision);
    return RI_E_UNSUPPORTED;
  }
  void* buf = nullptr;
  RI_TRY(dev_alloc(&buf, p.bytes, s));
  const int rc = ppl::run_f64(p, B, qs, rs, tau, R, buf, s);
  dev_free(buf, s);
  return rc;
}

}  // namespace ri

using namespace ri;

extern "C" {

size_t ri_ppl_workspace_bytes(int o, int v, int naux, int precision) {
  ppl::Plan p;
  if (precision == RI_PREC_BF16X3) return ppl::bf16x3_workspace_bytes(o, v, naux);
  if (precision != RI_PREC_FP64) return 0;
  if (!ppl::make_plan(o, v, naux, p)) return 0;
  return p.bytes;
}

double ri_ppl_flops(int o, int v, int naux) {
  if (o <= 0 || v <= 0 || naux <= 0) return 0.0;
  const double dv = v, pv = dv * (dv + 1) / 2, pvm = dv * (dv - 1) / 2;
  const double po = o * (o + 1.0) / 2, pom = o * (o - 1.0) / 2;
  return static_cast<double>(naux) * dv * dv * dv * (dv + 1) + 2.0 * (pv * pv * po + pvm * pvm * pom);
}

int ri_ppl_ex(const double* B_vv, const double* tau, int o, int v, int naux, double* R, int precision,
              void* ws, size_t ws_bytes, void* stream) {
  clear_error();
  if (!B_vv || !tau || !R) {
    set_error("ri_ppl: null pointer argument");
    return RI_E_ARG;
  }
  if (precision != RI_PREC_FP64 && precision != RI_PREC_FP32 && precision != RI_PREC_BF16X3) {
    set_error("ri_ppl: unknown precision %d", precision);
    return RI_E_ARG;
  }
  ppl::Plan p;
  if (!ppl::make_plan(o, v, naux, p)) {
    set_error("ri_ppl: invalid sizes o=%d v=%d naux=%d", o, v, naux);
    return RI_E_ARG;
  }
  if (precision == RI_PREC_FP32) {
    set_error("ri_ppl: precision %d not available in this build", precision);
    return RI_E_UNSUPPORTED;
  }
  const size_t nB = static_cast<size_t>(naux) * v * v * sizeof(double);
  const size_t nT = static_cast<size_t>(o) * o * v * v * sizeof(double);
  if (overlaps(R, nT, B_vv, nB) || overlaps(R, nT, tau, nT)) {
    set_error("ri_ppl: R overlaps an input");
    return RI_E_ALIAS;
  }
  if ((reinterpret_cast<uintptr_t>(B_vv) | reinterpret_cast<uintptr_t>(tau) |
       reinterpret_cast<uintptr_t>(R)) & 7) {
    set_error("ri_ppl: arrays must be 8-byte aligned");
    return RI_E_ARG;
  }
  hipStream_t s = static_cast<hipStream_t>(stream);
  if (ws && (reinterpret_cast<uintptr_t>(ws) & 255)) {
    set_error("ri_ppl: workspace must be 256-byte aligned");
    return RI_E_ARG;
  }
  if (precision == RI_PREC_BF16X3)
    return ppl::bf16x3_run(B_vv, static_cast<long>(v) * v, v, tau, o, v, naux, R, ws, ws_bytes, s);
  void* buf = ws;
  bool own = false;
  if (ws) {
    if (ws_bytes < p.bytes) {
      set_error("ri_ppl: workspace of %zu bytes is smaller than the %zu required", ws_bytes, p.bytes);
      return RI_E_NOMEM;
    }
    if (reinterpret_cast<uintptr_t>(ws) & 255) {
      set_error("ri_ppl: workspace must be 256-byte aligned");
      return RI_E_ARG;
    }
  } else {
    RI_TRY(dev_alloc(&buf, p.bytes, s));
    own = true;
  }
  int rc = ppl::run_f64(p, B_vv, static_cast<long>(v) * v, v, tau, R, buf, s);
  if (own) dev_free(buf, s);
  return rc;
}

int ri_ppl(const double* B_vv, const double* tau, int o, int v, int naux, double* R, void* stream) {
  return ri_ppl_ex(B_vv, tau, o, v, naux, R, RI_PREC_FP64, nullptr, 0, stream);
}

int ri_build_tau(const double* t1, const double* t2, int o, int v, double* tau, void* stream) {
  clear_error();
  if (!t1 || !t2 || !tau || o <= 0 || v <= 0) {
    set_error("ri_build_tau: invalid argument");
    return RI_E_ARG;
  }
  const size_t total = static_cast<size_t>(o) * o * v * v;
  if (tau != t2 && overlaps(tau, total * 8, t2, total * 8)) {
    set_error("ri_build_tau: tau partially overlaps t2");
    return RI_E_ALIAS;
  }
  if (overlaps(tau, total * 8, t1, static_cast<size_t>(o) * v * 8)) {
    set_error("ri_build_tau: tau overlaps t1");
    return RI_E_ALIAS;
  }
  hipStream_t s = static_cast<hipStream_t>(stream);
  const unsigned blocks = static_cast<unsigned>((total + 255) / 256);
  ppl::build_tau_kernel<<<blocks, 256, 0, s>>>(t1, t2, o, v, tau, total);
  return check_launch("build_tau_kernel");
}

}  // extern "C"
