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

constexpr int KC = 16;  // auxiliary functions (build) or cd slots (contraction) per LDS step
constexpr int CRM = 128;  // contraction tile rows (four waves of CRM / 4)

typedef double double4_t __attribute__((ext_vector_type(4)));
typedef double double2_t __attribute__((ext_vector_type(2)));  // register-promotable (unlike double2)
typedef float f32x4_t __attribute__((ext_vector_type(4)));

// The FP64 and FP32 paths share their kernels; the element type picks the MFMA.
// Both are 16x16x4 tiles with the same operand layout (lane l supplies A[l%16][l/16]
// and B[l/16][l%16]) but different result layouts: element r of lane l holds
// D[drow(r, l)][l%16].
template <class T>
struct Mfma;
template <>
struct Mfma<double> {
  typedef double4_t acc_t;
  typedef double2_t vec_t;  // one 16-byte load
  __device__ static acc_t mma(double a, double b, acc_t c) {
    return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
  }
  __device__ static int drow(int r, int lane) { return 4 * r + (lane >> 4); }
  __device__ static acc_t zero() { return acc_t{0.0, 0.0, 0.0, 0.0}; }
};
template <>
struct Mfma<float> {
  typedef f32x4_t acc_t;
  typedef f32x4_t vec_t;
  __device__ static acc_t mma(float a, float b, acc_t c) { return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0); }
  __device__ static int drow(int r, int lane) { return 4 * (lane >> 4) + r; }
  __device__ static acc_t zero() { return acc_t{0.f, 0.f, 0.f, 0.f}; }
};

// ---------------------------------------------------------------- 1. relayout
// B[q][a][c] lives at B + q*qs + a*rs + c.  grid (naux_p, vp/16, vp/16), block 256
template <class T>
__device__ __forceinline__ void relayout_body(const double* __restrict__ B, long qs, long rs, int v, int naux, int vp,
                                              int naux_p, T* __restrict__ Bc) {
  __shared__ double tile[TB][TB + 1];
  const int q = blockIdx.x, a0 = blockIdx.y * TB, c0 = blockIdx.z * TB;
  const int tx = threadIdx.x & 15, ty = threadIdx.x >> 4;
  const int a = a0 + ty, c = c0 + tx;
  tile[ty][tx] = (a < v && c < v && q < naux) ? B[q * qs + a * rs + c] : 0.0;
  __syncthreads();
  Bc[(static_cast<size_t>(c0 + ty) * naux_p + q) * vp + a0 + tx] = static_cast<T>(tile[tx][ty]);
}
__global__ __launch_bounds__(256) void relayout_b_f64(const double* __restrict__ B, long qs, long rs, int v,
                                                      int naux, int vp, int naux_p, double* __restrict__ Bc) {
  relayout_body<double>(B, qs, rs, v, naux, vp, naux_p, Bc);
}
__global__ __launch_bounds__(256) void relayout_b_f32(const double* __restrict__ B, long qs, long rs, int v,
                                                      int naux, int vp, int naux_p, float* __restrict__ Bc) {
  relayout_body<float>(B, qs, rs, v, naux, vp, naux_p, Bc);
}

// ---------------------------------------------------------------- 2. pack
// out[slot][col], slot = pcd*256 + c_in*16 + d_in, col = packed (i,j).
// sign > 0: i<=j columns, value of tau+ (with the 1/2 on c == d);
// sign < 0: i<j columns, value of tau-.  Both taken from the pair-symmetric part
// of tau, formed in FP64 and rounded once to T.  grid (nbp, ncol/16), block 256
template <class T>
__device__ __forceinline__ void pack_body(const double* __restrict__ tau, int o, int v, int ncol, int sign,
                                          T* __restrict__ out) {
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
    out[(static_cast<size_t>(blockIdx.x) * 256 + slot) * ncol + blockIdx.y * NG + cc] = static_cast<T>(sv[slot][cc]);
  }
}
__global__ __launch_bounds__(256) void pack_tau_f64(const double* __restrict__ tau, int o, int v, int ncol, int sign,
                                                    double* __restrict__ out) {
  pack_body<double>(tau, o, v, ncol, sign, out);
}
__global__ __launch_bounds__(256) void pack_tau_f32(const double* __restrict__ tau, int o, int v, int ncol, int sign,
                                                    float* __restrict__ out) {
  pack_body<float>(tau, o, v, ncol, sign, out);
}

// ---------------------------------------------------------------- 3a. build
// One workgroup: ab block pair (Ab, Bb) x one quarter (8 c by 8 d) of cd block pair
// (Cb, Db).  Eight waves; wave w owns c in {2*(w>>1), +1} and d in {4*(w&1) .. +3}
// of the quarter and accumulates (ac|bd) and (ad|bc) as 16x16 (a, b) MFMA tiles.
// LDS holds, per KC-wide Q chunk, Bc for the 16 c/d rows x (16 a + 16 b) columns.
// The launch covers cd block pairs pcd0 .. nbp-1 (rows of the others are not written).
// grid ((nbp - pcd0)*4, slab_pairs), block 512
// D: the workgroups of diagonal ab block pairs (Ab == Bb), blockIdx.y counting them
// from block Ab = diag_y0; otherwise blockIdx.y is the slab's pair and diagonal pairs
// exit at once.  In a diagonal pair a and b run over the same block, so the (ad|bc)
// tile is the transpose of the (ac|bd) tile: only the latter is built, and the
// epilogue reads it back transposed through LDS.
template <class T, bool D>
__device__ __forceinline__ void build_body(const T* __restrict__ Bc, int naux_p, int vp, long slab0, long slab_M,
                                           int want_minus, int diag_y0, long pcd0, T* __restrict__ Wp,
                                           T* __restrict__ Wm) {
  typedef Mfma<T> MF;
  typedef typename MF::vec_t vec_t;
  constexpr int VEC = 16 / sizeof(T);          // elements per 16-byte load
  constexpr int EV = 32 / VEC;                 // loads per (x, k) row of 32 e
  constexpr int NV = 16 * KC * 32 / (512 * VEC);  // loads per thread per chunk
  __shared__ T lds[2][16][KC][32];  // [buf][x: 8 c then 8 d][k][e: 16 a then 16 b]
  static_assert(2 * 16 * KC * 32 >= 8 * 8 * 256, "the staging buffer holds the transposed tiles");
  const int quarter = blockIdx.x & 3;
  const long pcd = pcd0 + (blockIdx.x >> 2);
  int Cb, Db, Ab, Bb;
  tri_decode(pcd, Cb, Db);
  long pab_loc;
  if constexpr (D) {
    Ab = Bb = diag_y0 + static_cast<int>(blockIdx.y);
    pab_loc = static_cast<long>(Ab) * (Ab + 3) / 2 - slab0;
  } else {
    pab_loc = blockIdx.y;
    tri_decode(slab0 + pab_loc, Ab, Bb);
    if (Ab == Bb) return;  // built by the diagonal launch (uniform over the workgroup)
  }
  const int c_base = Cb * TB + (quarter >> 1) * 8;
  const int d_base = Db * TB + (quarter & 1) * 8;
  const int t = threadIdx.x, w = t >> 6, lane = t & 63;

  // global -> register -> LDS staging: NV 16-byte loads per thread per chunk.
  // Offsets are computed once; the chunk loop only adds the Q stride.
  size_t goff[NV];
  int loff[NV];
#pragma unroll
  for (int r = 0; r < NV; ++r) {
    const int p2 = t + 512 * r;
    const int x = p2 / (KC * EV), k = (p2 / EV) % KC, e = (p2 % EV) * VEC;
    const int cg = x < 8 ? c_base + x : d_base + (x - 8);
    const int ag = e < 16 ? Ab * TB + e : Bb * TB + (e - 16);
    goff[r] = (static_cast<size_t>(cg) * naux_p + k) * vp + ag;
    loff[r] = (x * KC + k) * 32 + e;
  }
  const size_t qstride = static_cast<size_t>(vp) * KC;  // advance one chunk of Q
  T* lds0 = &lds[0][0][0][0];
  constexpr int LBUF = 16 * KC * 32;

  const int xc0 = (w >> 1) * 2, xd0 = 8 + (w & 1) * 4;
  const int m = lane & 15, kq = lane >> 4;
  const int nchunks = naux_p / KC;
  // In a diagonal cd block pair the quarter with c in the upper and d in the lower
  // half holds only c > d slots, whose packed amplitudes are zero: its W entries are
  // written as zeros without the build (uniform over the workgroup).
  const bool skip = Cb == Db && quarter == 2;
  const size_t col0 = static_cast<size_t>(pab_loc) * 256;

  {
    constexpr int NA2 = D ? 1 : 2;  // (ad|bc) accumulators are not needed when D
    typename MF::acc_t acc1[2][4], acc2[NA2][4];
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
      for (int j = 0; j < 4; ++j) acc1[i][j] = MF::zero();
#pragma unroll
    for (int i = 0; i < NA2; ++i)
#pragma unroll
      for (int j = 0; j < 4; ++j) acc2[i][j] = MF::zero();
    if (!skip) {
      vec_t stage[NV];
#pragma unroll
      for (int r = 0; r < NV; ++r) stage[r] = *reinterpret_cast<const vec_t*>(Bc + goff[r]);
#pragma unroll
      for (int r = 0; r < NV; ++r) *reinterpret_cast<vec_t*>(lds0 + loff[r]) = stage[r];
      __syncthreads();
      for (int ch = 0; ch < nchunks; ++ch) {
        const int buf = ch & 1;
        const bool more = ch + 1 < nchunks;
        if (more) {
          const size_t qo = static_cast<size_t>(ch + 1) * qstride;
#pragma unroll
          for (int r = 0; r < NV; ++r) stage[r] = *reinterpret_cast<const vec_t*>(Bc + goff[r] + qo);
        }
#pragma unroll
        for (int s = 0; s < KC / 4; ++s) {
          const int kk = 4 * s + kq;
          if constexpr (D) {
            T a_c[2], b_d[4];
#pragma unroll
            for (int i = 0; i < 2; ++i) a_c[i] = lds[buf][xc0 + i][kk][m];
#pragma unroll
            for (int j = 0; j < 4; ++j) b_d[j] = lds[buf][xd0 + j][kk][16 + m];
#pragma unroll
            for (int i = 0; i < 2; ++i)
#pragma unroll
              for (int j = 0; j < 4; ++j) acc1[i][j] = MF::mma(a_c[i], b_d[j], acc1[i][j]);  // (ac|bd)
          } else {
            T a_c[2], b_c[2], a_d[4], b_d[4];
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
                acc1[i][j] = MF::mma(a_c[i], b_d[j], acc1[i][j]);      // (ac|bd)
                acc2[i % NA2][j] = MF::mma(a_d[j], b_c[i], acc2[i % NA2][j]);  // (ad|bc)
              }
          }
        }
        if (more) {
          T* dst = lds0 + (buf ^ 1) * LBUF;
#pragma unroll
          for (int r = 0; r < NV; ++r) *reinterpret_cast<vec_t*>(dst + loff[r]) = stage[r];
        }
        __syncthreads();
      }
    }  // !skip

    // each wave's own 8 x 256 elements of the (now idle) staging buffer hold its
    // (ac|bd) tiles, element (a, b) of a tile at a*16 + (b ^ a)
    T* tw = lds0 + w * (8 * 256);
    if constexpr (D) {
#pragma unroll
      for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 4; ++j)
#pragma unroll
          for (int r = 0; r < 4; ++r) {
            const int a_in = MF::drow(r, lane), b_in = lane & 15;
            tw[(i * 4 + j) * 256 + a_in * 16 + (b_in ^ a_in)] = acc1[i][j][r];
          }
      __syncthreads();
    }

    // epilogue: W+-[slot][ab slot]; element r of a lane is row a_in = drow(r, lane),
    // column b_in = lane & 15 of the (a, b) tile.
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        const int c_in = (quarter >> 1) * 8 + xc0 + i;
        const int d_in = (quarter & 1) * 8 + (xd0 - 8) + j;
        const size_t row = (static_cast<size_t>(pcd) * 256 + c_in * 16 + d_in) * slab_M + col0;
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const int a_in = MF::drow(r, lane), b_in = lane & 15;
          const T v1 = acc1[i][j][r];
          T v2;
          if constexpr (D)
            v2 = tw[(i * 4 + j) * 256 + b_in * 16 + (a_in ^ b_in)];  // (ac|bd)[b][a]
          else
            v2 = acc2[i][j][r];
          Wp[row + a_in * 16 + b_in] = v1 + v2;
          if (want_minus) Wm[row + a_in * 16 + b_in] = v1 - v2;
        }
      }
  }
}
__global__ __launch_bounds__(512) void build_w_f64(const double* __restrict__ Bc, int naux_p, int vp, long slab0,
    long slab_M, int want_minus, int diag_y0, long pcd0, double* __restrict__ Wp, double* __restrict__ Wm) {
  build_body<double, false>(Bc, naux_p, vp, slab0, slab_M, want_minus, diag_y0, pcd0, Wp, Wm);
}
__global__ __launch_bounds__(512) void build_w_f64_diag(const double* __restrict__ Bc, int naux_p, int vp, long slab0,
    long slab_M, int want_minus, int diag_y0, long pcd0, double* __restrict__ Wp, double* __restrict__ Wm) {
  build_body<double, true>(Bc, naux_p, vp, slab0, slab_M, want_minus, diag_y0, pcd0, Wp, Wm);
}
__global__ __launch_bounds__(512) void build_w_f32(const float* __restrict__ Bc, int naux_p, int vp, long slab0,
    long slab_M, int want_minus, int diag_y0, long pcd0, float* __restrict__ Wp, float* __restrict__ Wm) {
  build_body<float, false>(Bc, naux_p, vp, slab0, slab_M, want_minus, diag_y0, pcd0, Wp, Wm);
}
__global__ __launch_bounds__(512) void build_w_f32_diag(const float* __restrict__ Bc, int naux_p, int vp, long slab0,
    long slab_M, int want_minus, int diag_y0, long pcd0, float* __restrict__ Wp, float* __restrict__ Wm) {
  build_body<float, true>(Bc, naux_p, vp, slab0, slab_M, want_minus, diag_y0, pcd0, Wp, Wm);
}

// ---------------------------------------------------------------- 3b. contract
// C[m][n] = sum_k W[k][m] T[k][n];  tile CRM (m) x 16*NTW (n); 4 waves, wave w owns
// rows w*CRM/4 .. (w+1)*CRM/4 - 1 (CRM/64 MFMA row tiles, each B fragment feeds all of
// them) and all columns.  Every row tile streams the whole packed tau, so taller tiles
// read it fewer times.  The k range may be split over grid.z: split z sums k in
// [z*kz, min(K, (z+1)*kz)) into C + z*zs, and the unpack adds the splits in order.
// grid (ncol/(16*NTW), M/CRM, splits), block 256
template <class T, int NTW>
__device__ __forceinline__ void contract_body(const T* __restrict__ W, const T* __restrict__ Tt, long K, long M,
                                              int ncol, T* __restrict__ C, long kz, long zs) {
  // W rows have stride M (the slab width); C has NTW*16*gridDim.x columns
  typedef Mfma<T> MF;
  typedef typename MF::vec_t vec_t;
  constexpr int BN = 16 * NTW;
  constexpr int RW = CRM / 64;                  // 16-row MFMA tiles per wave
  constexpr int VEC = 16 / sizeof(T);
  constexpr int AV = CRM / VEC;                 // loads per k row of the A tile
  constexpr int NA = KC * CRM / (256 * VEC);    // A loads per thread per chunk
  __shared__ T sA[2][KC][CRM];
  __shared__ T sB[2][KC][BN];
  unsigned tx, ty;
  xcd_tile(tx, ty);
  const long n0 = static_cast<long>(tx) * BN, m0 = static_cast<long>(ty) * CRM;
  const int t = threadIdx.x, w = t >> 6, lane = t & 63;
  {  // this split's k range (every split holds at least one chunk)
    const long k_lo = blockIdx.z * kz;
    K = (K < k_lo + kz ? K : k_lo + kz) - k_lo;
    W += k_lo * M + m0;
    Tt += k_lo * ncol + n0;
    C += blockIdx.z * zs;
  }

  // staging offsets within a chunk (the chunk loop advances the base pointers)
  int aoff[NA], boff[NTW];
  int alo[NA], blo[NTW];
#pragma unroll
  for (int r = 0; r < NA; ++r) {
    const int p2 = t + 256 * r;
    const int k = p2 / AV, mm = (p2 % AV) * VEC;
    aoff[r] = k * static_cast<int>(M) + mm;
    alo[r] = k * CRM + mm;
  }
#pragma unroll
  for (int r = 0; r < NTW; ++r) {
    const int e = t + 256 * r;
    const int k = e / BN, nn = e % BN;
    boff[r] = k * ncol + nn;
    blo[r] = k * BN + nn;
  }
  vec_t ra[NA];
  T rb[NTW];
  T* sA0 = &sA[0][0][0];
  T* sB0 = &sB[0][0][0];

  typename MF::acc_t acc[RW][NTW];
#pragma unroll
  for (int q = 0; q < RW; ++q)
#pragma unroll
    for (int u = 0; u < NTW; ++u) acc[q][u] = MF::zero();
  const int m = lane & 15, kq = lane >> 4;
  const long nchunks = K / KC;
#pragma unroll
  for (int r = 0; r < NA; ++r) ra[r] = *reinterpret_cast<const vec_t*>(W + aoff[r]);
#pragma unroll
  for (int r = 0; r < NTW; ++r) rb[r] = Tt[boff[r]];
#pragma unroll
  for (int r = 0; r < NA; ++r) *reinterpret_cast<vec_t*>(sA0 + alo[r]) = ra[r];
#pragma unroll
  for (int r = 0; r < NTW; ++r) sB0[blo[r]] = rb[r];
  __syncthreads();
  for (long ch = 0; ch < nchunks; ++ch) {
    const int buf = ch & 1;
    const bool more = ch + 1 < nchunks;
    if (more) {
      const T* Wc = W + (ch + 1) * KC * M;
      const T* Tc = Tt + (ch + 1) * KC * ncol;
#pragma unroll
      for (int r = 0; r < NA; ++r) ra[r] = *reinterpret_cast<const vec_t*>(Wc + aoff[r]);
#pragma unroll
      for (int r = 0; r < NTW; ++r) rb[r] = Tc[boff[r]];
    }
#pragma unroll
    for (int s = 0; s < KC / 4; ++s) {
      const int kk = 4 * s + kq;
      T a[RW];
#pragma unroll
      for (int q = 0; q < RW; ++q) a[q] = sA[buf][kk][(w * RW + q) * 16 + m];
#pragma unroll
      for (int u = 0; u < NTW; ++u) {
        const T b = sB[buf][kk][u * 16 + m];
#pragma unroll
        for (int q = 0; q < RW; ++q) acc[q][u] = MF::mma(a[q], b, acc[q][u]);
      }
    }
    if (more) {
#pragma unroll
      for (int r = 0; r < NA; ++r) *reinterpret_cast<vec_t*>(sA0 + (buf ^ 1) * KC * CRM + alo[r]) = ra[r];
#pragma unroll
      for (int r = 0; r < NTW; ++r) sB0[(buf ^ 1) * KC * BN + blo[r]] = rb[r];
    }
    __syncthreads();
  }
#pragma unroll
  for (int q = 0; q < RW; ++q)
#pragma unroll
    for (int u = 0; u < NTW; ++u)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const long row = m0 + (w * RW + q) * 16 + MF::drow(r, lane);
        C[row * ncol + n0 + u * 16 + m] = acc[q][u][r];
      }
}
template <int NTW>
__global__ __launch_bounds__(256) void contract_f64(const double* __restrict__ W, const double* __restrict__ Tt,
                                                    long K, long M, int ncol, double* __restrict__ C, long kz,
                                                    long zs) {
  contract_body<double, NTW>(W, Tt, K, M, ncol, C, kz, zs);
}
template <int NTW>
__global__ __launch_bounds__(256) void contract_f32(const float* __restrict__ W, const float* __restrict__ Tt,
                                                    long K, long M, int ncol, float* __restrict__ C, long kz,
                                                    long zs) {
  contract_body<float, NTW>(W, Tt, K, M, ncol, C, kz, zs);
}

// ---------------------------------------------------------------- 3b'. row contraction
// The second product of the exchange-symmetric form sums along W's rows:
//   C[r][n] (+)= sum_m W[r][m] T[m][n],   r < rows, m < M, n < ncol
// W rows have stride ldw, T and C rows stride ncol.  Tile CRM (r) x 16*NTW (n), four
// waves as in contract_body; W is staged transposed (sA[m][r], padded rows so that
// the transposing stores spread over the banks), T as there.  `accum` adds into C
// (the products of later slabs land on the rows of earlier ones in a fixed order).
// grid (ncol/(16*NTW), rows/CRM), block 256
template <class T, int NTW>
__device__ __forceinline__ void contract_rows_body(const T* __restrict__ W, long ldw, const T* __restrict__ Tt,
                                                   long M, int ncol, T* __restrict__ C, int accum) {
  typedef Mfma<T> MF;
  typedef typename MF::vec_t vec_t;
  constexpr int BN = 16 * NTW;
  constexpr int RW = CRM / 64;
  constexpr int VEC = 16 / sizeof(T);          // elements per 16-byte load (along m)
  constexpr int KV = KC / VEC;                 // loads per W row per chunk
  constexpr int NA = KC * CRM / (256 * VEC);   // W loads per thread per chunk
  constexpr int PAD = CRM + 1;
  __shared__ T sA[2][KC][PAD];
  __shared__ T sB[2][KC][BN];
  unsigned tx, ty;
  xcd_tile(tx, ty);
  const long n0 = static_cast<long>(tx) * BN, r0 = static_cast<long>(ty) * CRM;
  const int t = threadIdx.x, w = t >> 6, lane = t & 63;
  W += r0 * ldw;
  Tt += n0;
  long aoff[NA];
  int arow[NA], ak[NA];
#pragma unroll
  for (int r = 0; r < NA; ++r) {
    const int id = t + 256 * r;
    arow[r] = id / KV;
    ak[r] = (id % KV) * VEC;
    aoff[r] = arow[r] * ldw + ak[r];
  }
  int boff[NTW], blo[NTW];
#pragma unroll
  for (int r = 0; r < NTW; ++r) {
    const int e = t + 256 * r;
    const int k = e / BN, nn = e % BN;
    boff[r] = k * ncol + nn;
    blo[r] = k * BN + nn;
  }
  vec_t ra[NA];
  T rb[NTW];
  T* sB0 = &sB[0][0][0];
  auto store_a = [&](int buf) {
#pragma unroll
    for (int r = 0; r < NA; ++r)
#pragma unroll
      for (int e = 0; e < VEC; ++e) sA[buf][ak[r] + e][arow[r]] = ra[r][e];
  };
  typename MF::acc_t acc[RW][NTW];
#pragma unroll
  for (int q = 0; q < RW; ++q)
#pragma unroll
    for (int u = 0; u < NTW; ++u) acc[q][u] = MF::zero();
  const int m = lane & 15, kq = lane >> 4;
  const long nchunks = M / KC;
#pragma unroll
  for (int r = 0; r < NA; ++r) ra[r] = *reinterpret_cast<const vec_t*>(W + aoff[r]);
#pragma unroll
  for (int r = 0; r < NTW; ++r) rb[r] = Tt[boff[r]];
  store_a(0);
#pragma unroll
  for (int r = 0; r < NTW; ++r) sB0[blo[r]] = rb[r];
  __syncthreads();
  for (long ch = 0; ch < nchunks; ++ch) {
    const int buf = ch & 1;
    const bool more = ch + 1 < nchunks;
    if (more) {
      const long ko = (ch + 1) * KC;
#pragma unroll
      for (int r = 0; r < NA; ++r) ra[r] = *reinterpret_cast<const vec_t*>(W + aoff[r] + ko);
#pragma unroll
      for (int r = 0; r < NTW; ++r) rb[r] = Tt[ko * ncol + boff[r]];
    }
#pragma unroll
    for (int s = 0; s < KC / 4; ++s) {
      const int kk = 4 * s + kq;
      T a[RW];
#pragma unroll
      for (int q = 0; q < RW; ++q) a[q] = sA[buf][kk][(w * RW + q) * 16 + m];
#pragma unroll
      for (int u = 0; u < NTW; ++u) {
        const T b = sB[buf][kk][u * 16 + m];
#pragma unroll
        for (int q = 0; q < RW; ++q) acc[q][u] = MF::mma(a[q], b, acc[q][u]);
      }
    }
    if (more) {
      store_a(buf ^ 1);
#pragma unroll
      for (int r = 0; r < NTW; ++r) sB0[(buf ^ 1) * KC * BN + blo[r]] = rb[r];
    }
    __syncthreads();
  }
#pragma unroll
  for (int q = 0; q < RW; ++q)
#pragma unroll
    for (int u = 0; u < NTW; ++u)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const long row = r0 + (w * RW + q) * 16 + MF::drow(r, lane);
        T* c = C + row * ncol + n0 + u * 16 + m;
        *c = accum ? *c + acc[q][u][r] : acc[q][u][r];
      }
}
template <int NTW>
__global__ __launch_bounds__(256) void contract_rows_f64(const double* __restrict__ W, long ldw,
                                                         const double* __restrict__ Tt, long M, int ncol,
                                                         double* __restrict__ C, int accum) {
  contract_rows_body<double, NTW>(W, ldw, Tt, M, ncol, C, accum);
}
template <int NTW>
__global__ __launch_bounds__(256) void contract_rows_f32(const float* __restrict__ W, long ldw,
                                                         const float* __restrict__ Tt, long M, int ncol,
                                                         float* __restrict__ C, int accum) {
  contract_rows_body<float, NTW>(W, ldw, Tt, M, ncol, C, accum);
}

// ---------------------------------------------------------------- 3c. unpack
// S and A are FP64 (FP64 path) or FP32 (mixed paths); R accumulates in FP64.  S and
// A may come as zp (zm) partial sums over k, zs (zsm) elements apart, added here in
// order.  perm: the rows of a block pair are in the split path's slot order.
// The kernel is bound by memory latency unless many loads are in flight: a thread sums
// its 16 rows of one column together (16 loads per split), and reads the R entries of
// four columns before it writes them back.
// grid (slab_pairs, ceil(po/16)), block 256
template <class T>
__global__ __launch_bounds__(256) void unpack_kernel(const T* __restrict__ S, const T* __restrict__ A,
                                                     int NP, int NM, int o, int v, long slab0,
                                                     double* __restrict__ R, int zp, long zsp, int zm, long zsm,
                                                     int perm) {
  __shared__ double sS[256][NG + 1];
  __shared__ double sA[256][NG + 1];
  int Ab, Bb;
  tri_decode(slab0 + blockIdx.x, Ab, Bb);
  const int t = threadIdx.x;
  const int po = o * (o + 1) / 2;
  const int lam0 = blockIdx.y * NG;
  const size_t row0 = static_cast<size_t>(blockIdx.x) * 256;
  {
    // column lam = lam0 + cc of rows r * 16 + rr (slot order), r = 0..15
    // Loads are unconditional (a lane without work reads a valid neighbouring column
    // and drops the value), so that they issue back to back.
    const int cc = t & 15, rr = t >> 4, lam = lam0 + cc;
    const bool lv = lam < po;
    const int lamc = lv ? lam : po - 1;
    int i, j;
    tri_decode(lamc, i, j);
    // the antisymmetric part vanishes at a == b (V-^{aa}_{cd} = (ac|ad) - (ad|ac)); rows
    // that sum it from separately rounded integrals are not read, so R stays exactly
    // pair-symmetric
    const bool anti = lv && i < j;
    const int ja = i < j ? j * (j - 1) / 2 + i : (j > 0 ? j * (j - 1) / 2 + j - 1 : 0);
    auto srow = [&](int r) { return static_cast<size_t>(perm ? split_slot(r, rr) : r * 16 + rr); };
    double s[16], x[16];
#pragma unroll
    for (int r = 0; r < 16; ++r) s[r] = x[r] = 0.0;
    for (int z = 0; z < zp; ++z) {
      const T* Sz = S + z * zsp;
      T u[16];
#pragma unroll
      for (int r = 0; r < 16; ++r) u[r] = Sz[(row0 + srow(r)) * NP + lamc];
#pragma unroll
      for (int r = 0; r < 16; ++r) s[r] += static_cast<double>(u[r]);
    }
    for (int z = 0; NM > 0 && z < zm; ++z) {
      const T* Az = A + z * zsm;
      T u[16];
#pragma unroll
      for (int r = 0; r < 16; ++r) u[r] = Az[(row0 + srow(r)) * NM + ja];
#pragma unroll
      for (int r = 0; r < 16; ++r)
        x[r] += anti && !(Ab == Bb && r == rr) ? static_cast<double>(u[r]) : 0.0;
    }
#pragma unroll
    for (int r = 0; r < 16; ++r) {
      sS[r * 16 + rr][cc] = s[r];
      sA[r * 16 + rr][cc] = x[r];
    }
  }
  __syncthreads();
  const size_t vv = static_cast<size_t>(v) * v;
  const int hi = t >> 4, lo = t & 15;
  // (a, b) with a <= b, rows contiguous in b; and the mirrors (b, a) with a < b, rows
  // contiguous in a
  const int a1 = Ab * TB + hi, b1 = Bb * TB + lo, a2 = Ab * TB + lo, b2 = Bb * TB + hi;
  const bool ok1 = a1 < v && b1 < v && (Ab < Bb || hi <= lo);
  const bool ok2 = a2 < v && b2 < v && (Ab < Bb || lo < hi);
  const size_t e1 = static_cast<size_t>(a1) * v + b1, e2 = static_cast<size_t>(b2) * v + a2;
  const int s1 = hi * 16 + lo, s2 = lo * 16 + hi;
  for (int c0 = 0; c0 < NG; c0 += 4) {
    double *Rij[4], *Rji[4];
    bool val[4], off[4];
    double q11[4], q12[4], q21[4], q22[4];
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      const int lam = lam0 + c0 + k;
      val[k] = lam < po;
      int i = 0, j = 0;
      if (val[k]) tri_decode(lam, i, j);
      off[k] = i != j;  // R_ji is another element than R_ij
      Rij[k] = R + (static_cast<size_t>(i) * o + j) * vv;
      Rji[k] = R + (static_cast<size_t>(j) * o + i) * vv;
      q11[k] = q12[k] = q21[k] = q22[k] = 0.0;
      if (val[k] && ok1) {
        q11[k] = Rij[k][e1];
        if (off[k]) q12[k] = Rji[k][e1];
      }
      if (val[k] && ok2) {
        q21[k] = Rij[k][e2];
        if (off[k]) q22[k] = Rji[k][e2];
      }
    }
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      const int cc = c0 + k;
      if (val[k] && ok1) {
        const double sv = sS[s1][cc], xv = sA[s1][cc];
        Rij[k][e1] = q11[k] + (sv + xv);
        if (off[k]) Rji[k][e1] = q12[k] + (sv - xv);
      }
      if (val[k] && ok2) {
        const double sv = sS[s2][cc], xv = sA[s2][cc];
        Rij[k][e2] = q21[k] + (sv - xv);
        if (off[k]) Rji[k][e2] = q22[k] + (sv + xv);
      }
    }
  }
}

void launch_unpack_f32(const float* S, const float* A, int NP, int NM, int o, int v, long slab0, long npairs,
                       double* R, int zp, long zsp, int zm, long zsm, hipStream_t s, int perm) {
  unpack_kernel<float><<<dim3(npairs, (o * (o + 1) / 2 + NG - 1) / NG), 256, 0, s>>>(S, A, NP, NM, o, v, slab0, R,
                                                                                  zp, zsp, zm, zsm, perm);
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
  size_t esize;  // bytes per element of the staged operands (8 FP64, 4 FP32)
  long zrows_p, zrows_m;  // largest splits x rows of one contraction launch (sizes S and A)
  size_t n_Bc, n_Tp, n_Tm, n_W, n_S, n_A;
  size_t n_S2, n_A2;  // exchange-symmetric form only: second-product accumulators over all slots
  size_t bytes;
};

// Workgroups of the contraction kernel for ntw and the element size resident at once.
template <typename T>
static const void* contract_fn(int ntw) {
  typedef void (*F)(const T*, const T*, long, long, int, T*, long, long);
  F f;
  if constexpr (sizeof(T) == 8) {
    switch (ntw) {
      case 1: f = contract_f64<1>; break;
      case 2: f = contract_f64<2>; break;
      case 3: f = contract_f64<3>; break;
      case 4: f = contract_f64<4>; break;
      case 5: f = contract_f64<5>; break;
      case 6: f = contract_f64<6>; break;
      case 7: f = contract_f64<7>; break;
      case 8: f = contract_f64<8>; break;
      case 9: f = contract_f64<9>; break;
      default: f = contract_f64<10>; break;
    }
  } else {
    switch (ntw) {
      case 1: f = contract_f32<1>; break;
      case 2: f = contract_f32<2>; break;
      case 3: f = contract_f32<3>; break;
      case 4: f = contract_f32<4>; break;
      case 5: f = contract_f32<5>; break;
      case 6: f = contract_f32<6>; break;
      case 7: f = contract_f32<7>; break;
      case 8: f = contract_f32<8>; break;
      case 9: f = contract_f32<9>; break;
      default: f = contract_f32<10>; break;
    }
  }
  return reinterpret_cast<const void*>(f);
}
static long contract_slots(int ntw, size_t esize) {
  return resident_wgs(esize == 8 ? contract_fn<double>(ntw) : contract_fn<float>(ntw), 256, 2);
}

// Splits of the contraction's k range for a launch of `rows` rows and 16*ntw-wide
// column tiles: at least one full round of resident workgroups, and enough that one
// split's slice of the packed amplitudes (K/z rows of ncol elements) stays within
// RI_PPL_TAU_CHUNK_MB (default TAU_CHUNK_MB): every row tile streams its split's whole
// slice, and the workgroups resident together work on the same few splits (z is the
// slowest grid index), so a slice that fits the last-level cache is fetched from HBM
// about once instead of once per row tile.  Then balanced so that the last round of
// workgroups is not a few stragglers.  At least 32 chunks per split.  kz: summed indices
// per split.
static int contract_splits(int ncol, int ntw, long rows, long K, size_t esize, long& kz) {
  const long nwg = (ncol / (16 * ntw)) * (rows / CRM);
  const long slots = contract_slots(ntw, esize);
  long z = (slots + nwg - 1) / nwg;
  const double chunk = static_cast<double>(env_long("RI_PPL_TAU_CHUNK_MB", TAU_CHUNK_MB)) * 1048576.0;
  z = std::max(z, static_cast<long>(std::ceil(static_cast<double>(K) * ncol * esize / chunk)));
  const long zmax = std::max(1L, K / (32 * KC));
  z = std::max(1L, std::min(z, zmax));
  z = balance_splits(nwg, slots, K, KC, z, zmax);
  kz = (K + z - 1) / z;
  kz = (kz + KC - 1) / KC * KC;
  return static_cast<int>((K + kz - 1) / kz);
}

// Largest splits x rows over the slab sizes of plan p (the full slab and the last).
static long max_split_rows(const Plan& p, int ncol, int ntw) {
  if (ncol == 0) return 0;
  long kz;
  const long last = p.nbp - (p.nbp - 1) / p.slab_bp * p.slab_bp;
  long best = 0;
  for (long rows : {p.slab_M, last * 256}) best = std::max(best, contract_splits(ncol, ntw, rows, p.K, p.esize, kz) * rows);
  return best;
}

// Element counts and total bytes of plan p for its slab width p.slab_bp.
static void size_plan(Plan& p, bool sym) {
  p.slab_M = p.slab_bp * 256;
  p.n_Bc = static_cast<size_t>(p.vp) * p.naux_p * p.vp;
  p.n_Tp = static_cast<size_t>(p.K) * p.NP;
  p.n_Tm = static_cast<size_t>(p.K) * p.NM;
  p.n_W = static_cast<size_t>(p.K) * p.slab_M;
  p.zrows_p = max_split_rows(p, p.NP, p.ntw_p);
  p.zrows_m = max_split_rows(p, p.NM, p.ntw_m);
  p.n_S = static_cast<size_t>(p.zrows_p) * p.NP;
  p.n_A = static_cast<size_t>(p.zrows_m) * p.NM;
  p.n_S2 = sym ? static_cast<size_t>(p.K) * p.NP : 0;
  p.n_A2 = sym ? static_cast<size_t>(p.K) * p.NM : 0;
  size_t b = 0;
  for (size_t n : {p.n_Bc, p.n_Tp, p.n_Tm, p.n_W, p.pm > 0 ? p.n_W : 0, p.n_S, p.n_A, p.n_S2, p.n_A2})
    b = round_up(b, 256) + n * p.esize;
  p.bytes = round_up(b, 256);
}

// sym: the plan of the exchange-symmetric form (smaller slabs, second-product
// accumulators); see run_sym.  fit_bytes > 0: the widest slab whose whole workspace
// fits in fit_bytes (false if not even a one-block-pair slab fits), instead of the
// W budget RI_PPL_W_BYTES.
static bool make_plan(int o, int v, int naux, size_t esize, Plan& p, bool sym = false, size_t fit_bytes = 0) {
  if (o <= 0 || v <= 0 || naux <= 0) return false;
  if (o > 4096 || v > 65536 || naux > (1 << 24)) return false;
  p.o = o;
  p.v = v;
  p.naux = naux;
  p.esize = esize;
  p.nb = (v + TB - 1) / TB;
  p.vp = p.nb * TB;
  p.naux_p = static_cast<int>(round_up(naux, KC));
  p.nbp = static_cast<long>(p.nb) * (p.nb + 1) / 2;
  p.K = p.nbp * 256;
  p.po = o * (o + 1) / 2;
  p.pm = o * (o - 1) / 2;
  pick_ntw(p.po, 10, CRM, p.ntw_p, p.NP);
  pick_ntw(p.pm, 10, CRM, p.ntw_m, p.NM);
  if (p.pm == 0) p.NM = 0;
  const int nw = p.pm > 0 ? 2 : 1;
  const long budget = env_long("RI_PPL_W_BYTES", 16L << 30);
  long bp = budget / (static_cast<long>(nw) * p.K * 256 * static_cast<long>(esize));
  bp = bp < 1 ? 1 : bp;
  bp = bp > p.nbp ? p.nbp : bp;
  bp = bp > 65535 ? 65535 : bp;
  if (fit_bytes > 0) bp = std::min(p.nbp, 65535L);
  const long cap = env_long("RI_PPL_SLAB_PAIRS", bp);
  p.slab_bp = cap < bp ? cap : bp;
  if (sym) {  // at least RI_PPL_SYM_SLABS (8) slabs: the build is (1 + 1/slabs)/2 of the full one
    const long ns = env_long("RI_PPL_SYM_SLABS", 8);
    p.slab_bp = std::min(p.slab_bp, (p.nbp + ns - 1) / ns);
  }
  size_plan(p, sym);
  if (fit_bytes > 0 && p.bytes > fit_bytes) {  // bytes grow with the slab width: bisect
    long lo = 1, hi = p.slab_bp - 1;
    p.slab_bp = 1;
    size_plan(p, sym);
    if (p.bytes > fit_bytes) return false;
    while (lo < hi) {
      const long mid = (lo + hi + 1) / 2;
      p.slab_bp = mid;
      size_plan(p, sym);
      if (p.bytes <= fit_bytes) lo = mid; else hi = mid - 1;
    }
    p.slab_bp = lo;
    size_plan(p, sym);
  }
  return true;
}

// Kernel choice by element type (names stay distinct in profiles).
struct K64 {
  typedef double T;
  static constexpr const char* relayout = "relayout_b_f64";
  static constexpr const char* pack = "pack_tau_f64";
  static constexpr const char* build = "build_w_f64";
  static constexpr const char* build_diag = "build_w_f64_diag";
  static constexpr const char* contract = "contract_f64";
  static constexpr const char* unpack = "unpack_f64";
  static constexpr const char* contract_rows = "contract_rows_f64";
  template <int NTW>
  static void rows_k(dim3 g, hipStream_t s, const T* W, long ldw, const T* Tt, long M, int ncol, T* C, int accum) {
    contract_rows_f64<NTW><<<g, 256, 0, s>>>(W, ldw, Tt, M, ncol, C, accum);
  }
  static void relayout_k(dim3 g, hipStream_t s, const double* B, long qs, long rs, int v, int naux, int vp, int np,
                         T* Bc) {
    relayout_b_f64<<<g, 256, 0, s>>>(B, qs, rs, v, naux, vp, np, Bc);
  }
  static void pack_k(dim3 g, hipStream_t s, const double* tau, int o, int v, int ncol, int sign, T* out) {
    pack_tau_f64<<<g, 256, 0, s>>>(tau, o, v, ncol, sign, out);
  }
  static void build_k(dim3 g, hipStream_t s, const T* Bc, int np, int vp, long slab0, long sM, int wm, long pcd0,
                      T* Wp, T* Wm) {
    build_w_f64<<<g, 512, 0, s>>>(Bc, np, vp, slab0, sM, wm, 0, pcd0, Wp, Wm);
  }
  static void build_diag_k(dim3 g, hipStream_t s, const T* Bc, int np, int vp, long slab0, long sM, int wm, int y0,
                           long pcd0, T* Wp, T* Wm) {
    build_w_f64_diag<<<g, 512, 0, s>>>(Bc, np, vp, slab0, sM, wm, y0, pcd0, Wp, Wm);
  }
  template <int NTW>
  static void contract_k(dim3 g, hipStream_t s, const T* W, const T* Tt, long K, long M, int ncol, T* C, long kz,
                         long zs) {
    contract_f64<NTW><<<g, 256, 0, s>>>(W, Tt, K, M, ncol, C, kz, zs);
  }
};
struct K32 {
  typedef float T;
  static constexpr const char* relayout = "relayout_b_f32";
  static constexpr const char* pack = "pack_tau_f32";
  static constexpr const char* build = "build_w_f32";
  static constexpr const char* build_diag = "build_w_f32_diag";
  static constexpr const char* contract = "contract_f32";
  static constexpr const char* unpack = "unpack_f32";
  static constexpr const char* contract_rows = "contract_rows_f32";
  template <int NTW>
  static void rows_k(dim3 g, hipStream_t s, const T* W, long ldw, const T* Tt, long M, int ncol, T* C, int accum) {
    contract_rows_f32<NTW><<<g, 256, 0, s>>>(W, ldw, Tt, M, ncol, C, accum);
  }
  static void relayout_k(dim3 g, hipStream_t s, const double* B, long qs, long rs, int v, int naux, int vp, int np,
                         T* Bc) {
    relayout_b_f32<<<g, 256, 0, s>>>(B, qs, rs, v, naux, vp, np, Bc);
  }
  static void pack_k(dim3 g, hipStream_t s, const double* tau, int o, int v, int ncol, int sign, T* out) {
    pack_tau_f32<<<g, 256, 0, s>>>(tau, o, v, ncol, sign, out);
  }
  static void build_k(dim3 g, hipStream_t s, const T* Bc, int np, int vp, long slab0, long sM, int wm, long pcd0,
                      T* Wp, T* Wm) {
    build_w_f32<<<g, 512, 0, s>>>(Bc, np, vp, slab0, sM, wm, 0, pcd0, Wp, Wm);
  }
  static void build_diag_k(dim3 g, hipStream_t s, const T* Bc, int np, int vp, long slab0, long sM, int wm, int y0,
                           long pcd0, T* Wp, T* Wm) {
    build_w_f32_diag<<<g, 512, 0, s>>>(Bc, np, vp, slab0, sM, wm, y0, pcd0, Wp, Wm);
  }
  template <int NTW>
  static void contract_k(dim3 g, hipStream_t s, const T* W, const T* Tt, long K, long M, int ncol, T* C, long kz,
                         long zs) {
    contract_f32<NTW><<<g, 256, 0, s>>>(W, Tt, K, M, ncol, C, kz, zs);
  }
};

// rows: number of C rows (multiple of CRM) computed; ldw: row stride of W.  The k
// range is split `splits` ways (kz each) into partial outputs rows*ncol apart.
template <class KS>
static void launch_contract(int ntw, const typename KS::T* W, const typename KS::T* Tt, long K, long ldw, long rows,
                            int ncol, typename KS::T* C, int splits, long kz, hipStream_t s) {
  const unsigned gy = static_cast<unsigned>(rows / CRM), gz = static_cast<unsigned>(splits);
  const long zs = rows * ncol;
  switch (ntw) {
    case 1: KS::template contract_k<1>(dim3(ncol / 16, gy, gz), s, W, Tt, K, ldw, ncol, C, kz, zs); break;
    case 2: KS::template contract_k<2>(dim3(ncol / 32, gy, gz), s, W, Tt, K, ldw, ncol, C, kz, zs); break;
    case 3: KS::template contract_k<3>(dim3(ncol / 48, gy, gz), s, W, Tt, K, ldw, ncol, C, kz, zs); break;
    case 4: KS::template contract_k<4>(dim3(ncol / 64, gy, gz), s, W, Tt, K, ldw, ncol, C, kz, zs); break;
    case 5: KS::template contract_k<5>(dim3(ncol / 80, gy, gz), s, W, Tt, K, ldw, ncol, C, kz, zs); break;
    case 6: KS::template contract_k<6>(dim3(ncol / 96, gy, gz), s, W, Tt, K, ldw, ncol, C, kz, zs); break;
    case 7: KS::template contract_k<7>(dim3(ncol / 112, gy, gz), s, W, Tt, K, ldw, ncol, C, kz, zs); break;
    case 8: KS::template contract_k<8>(dim3(ncol / 128, gy, gz), s, W, Tt, K, ldw, ncol, C, kz, zs); break;
    case 9: KS::template contract_k<9>(dim3(ncol / 144, gy, gz), s, W, Tt, K, ldw, ncol, C, kz, zs); break;
    default: KS::template contract_k<10>(dim3(ncol / 160, gy, gz), s, W, Tt, K, ldw, ncol, C, kz, zs); break;
  }
}

// Steps 1 and 2: factors into their operand layout, tau into T+ and T-.
template <class KS>
static int stage_inputs(const Plan& p, const double* B_vv, long qs, long rs, const double* tau,
                        typename KS::T* Bc, typename KS::T* Tp, typename KS::T* Tm, hipStream_t s) {
  const double es = static_cast<double>(sizeof(typename KS::T));
  const double vv = static_cast<double>(p.v) * p.v, oo = static_cast<double>(p.o) * p.o;
  const double pv = p.v * (p.v + 1.0) / 2, pvm = p.v * (p.v - 1.0) / 2;
  {
    ProfScope ps(s, KS::relayout, 0.0, (8.0 + es) * vv * p.naux);
    KS::relayout_k(dim3(p.naux_p, p.nb, p.nb), s, B_vv, qs, rs, p.v, p.naux, p.vp, p.naux_p, Bc);
    RI_TRY(check_launch(KS::relayout));
  }
  {
    ProfScope ps(s, KS::pack, 0.0, 8.0 * oo * vv + es * (pv * p.po + pvm * p.pm));
    KS::pack_k(dim3(p.nbp, p.NP / NG), s, tau, p.o, p.v, p.NP, +1, Tp);
    RI_TRY(check_launch(KS::pack));
    if (p.pm > 0) {
      KS::pack_k(dim3(p.nbp, p.NM / NG), s, tau, p.o, p.v, p.NM, -1, Tm);
      RI_TRY(check_launch(KS::pack));
    }
  }
  return RI_OK;
}

template <class KS>
static int run_plan(const Plan& p, const double* B_vv, long qs, long rs, const double* tau, double* R, void* ws,
                    int shard, int nshards, hipStream_t s) {
  typedef typename KS::T T;
  Carve cv(ws, p.bytes);
  T* Bc = cv.take<T>(p.n_Bc);
  T* Tp = cv.take<T>(p.n_Tp);
  T* Tm = cv.take<T>(p.n_Tm);
  T* Wp = cv.take<T>(p.n_W);
  T* Wm = cv.take<T>(p.pm > 0 ? p.n_W : 0);
  T* S = cv.take<T>(p.n_S);
  T* A = cv.take<T>(p.n_A);

  const double vv = static_cast<double>(p.v) * p.v, oo = static_cast<double>(p.o) * p.o;
  const double pv = p.v * (p.v + 1.0) / 2, pvm = p.v * (p.v - 1.0) / 2;
  RI_TRY(stage_inputs<KS>(p, B_vv, qs, rs, tau, Bc, Tp, Tm, s));
  for (long slab0 = 0; slab0 < p.nbp; slab0 += p.slab_bp) {
    if ((slab0 / p.slab_bp) % nshards != shard) continue;  // another shard's slab
    const long npairs = (p.nbp - slab0) < p.slab_bp ? (p.nbp - slab0) : p.slab_bp;
    const long M = npairs * 256;
    double le, lt, ld;
    count_pairs(p.v, slab0, npairs, le, lt, ld);
    int dy0, ndiag;
    diag_pairs(slab0, npairs, dy0, ndiag);
    long kzp = 0, kzm = 0;
    const int zp = contract_splits(p.NP, p.ntw_p, M, p.K, p.esize, kzp);
    const int zm = p.pm > 0 ? contract_splits(p.NM, p.ntw_m, M, p.K, p.esize, kzm) : 1;
    {
      // per valid (a <= b): the v x v matrix (ac|bd) over all c, d, naux products each;
      // off-diagonal and diagonal ab block pairs in two launches
      ProfScope ps(s, KS::build, 2.0 * p.naux * vv * (le - ld));
      KS::build_k(dim3(p.nbp * 4, npairs), s, Bc, p.naux_p, p.vp, slab0, p.slab_M, p.pm > 0 ? 1 : 0, 0, Wp, Wm);
      RI_TRY(check_launch(KS::build));
    }
    if (ndiag > 0) {
      ProfScope ps(s, KS::build_diag, 2.0 * p.naux * vv * ld);
      KS::build_diag_k(dim3(p.nbp * 4, ndiag), s, Bc, p.naux_p, p.vp, slab0, p.slab_M, p.pm > 0 ? 1 : 0, dy0, 0,
                       Wp, Wm);
      RI_TRY(check_launch(KS::build_diag));
    }
    {
      ProfScope ps(s, KS::contract, 2.0 * (le * pv * p.po + lt * pvm * p.pm));
      launch_contract<KS>(p.ntw_p, Wp, Tp, p.K, p.slab_M, M, p.NP, S, zp, kzp, s);
      RI_TRY(check_launch(KS::contract));
      if (p.pm > 0) {
        launch_contract<KS>(p.ntw_m, Wm, Tm, p.K, p.slab_M, M, p.NM, A, zm, kzm, s);
        RI_TRY(check_launch(KS::contract));
      }
    }
    {
      ProfScope ps(s, KS::unpack, 0.0, 16.0 * oo * (le + lt));
      unpack_kernel<T><<<dim3(npairs, (p.po + NG - 1) / NG), 256, 0, s>>>(S, A, p.NP, p.NM, p.o, p.v, slab0, R, zp,
                                                                        M * p.NP, zm, M * p.NM, 0);
      RI_TRY(check_launch(KS::unpack));
    }
  }
  return RI_OK;
}

// Runs the FP64 or FP32 path of plan p on workspace ws (allocated when null).
static int run_typed(const Plan& p, int precision, const double* B_vv, long qs, long rs, const double* tau,
                     double* R, void* ws, int shard, int nshards, hipStream_t s) {
  void* buf = ws;
  if (!buf) RI_TRY(dev_alloc(&buf, p.bytes, s));
  const int rc = precision == RI_PREC_FP32 ? run_plan<K32>(p, B_vv, qs, rs, tau, R, buf, shard, nshards, s)
                                           : run_plan<K64>(p, B_vv, qs, rs, tau, R, buf, shard, nshards, s);
  if (!ws) dev_free(buf, s);
  return rc;
}

static size_t esize_of(int precision) { return precision == RI_PREC_FP32 ? 4 : 8; }

// ---------------------------------------------------------------- exchange symmetry
// When the factors are symmetric in their two virtual indices (B[Q][a][c] = B[Q][c][a],
// as for the bare integrals of eq. RIM), (ac|bd) has the full eight-fold symmetry of
// real two-electron integrals, and with it V+-^{ab}_{cd} = V+-^{cd}_{ab}: over (ab) and
// (cd) pairs the integral matrix is symmetric.  Slab [P0, P1) of ab block pairs then
// builds only the cd block pairs >= P0 and uses each built element twice:
//   S[ab]  = sum_{cd >= P0} W[cd][ab] T[cd]        contraction kernel, as in run_plan
//   S2[cd] += sum_{ab in slab} W[cd][ab] T[ab]     for cd >= P1 (FP64 GEMM engine)
// The cd < P0 part of a slab's own S arrived in S2 from the earlier slabs, and S2 is
// unpacked into R once after the last slab.  With n equal slabs the build is
// (1 + 1/n)/2 of run_plan's; the contraction FLOP are the same, split between the two
// products.  The summation order differs from run_plan's, so the two agree to rounding.

// Algorithmic FLOP of the exchange-symmetric form: the build and the two products,
// summed over the plan's slabs.
static void sym_flops(const Plan& p, double& build, double& contract) {
  build = contract = 0.0;
  for (long slab0 = 0; slab0 < p.nbp; slab0 += p.slab_bp) {
    const long npairs = std::min(p.nbp - slab0, p.slab_bp), p1 = slab0 + npairs;
    double le, lt, ld, ce, ct, cd, he, ht, hd;
    count_pairs(p.v, slab0, npairs, le, lt, ld);      // ab pairs of the slab
    count_pairs(p.v, slab0, p.nbp - slab0, ce, ct, cd);  // cd pairs built for it
    count_pairs(p.v, p1, p.nbp - p1, he, ht, hd);        // cd pairs of its second product
    build += 2.0 * p.naux * le * (2.0 * ct + (ce - ct));
    contract += 2.0 * ((le * ce + le * he) * p.po + (lt * ct + lt * ht) * p.pm);
  }
}

// Column tiles of the row contraction: the widest of 1..4 16-column tiles that divides
// the padded column count, so that short slabs still launch several workgroups per row
// tile.  rows: a multiple of CRM; M: a multiple of KC.
template <class KS>
static void launch_contract_rows(const typename KS::T* W, long ldw, const typename KS::T* Tt, long M, long rows,
                                 int ncol, typename KS::T* C, int accum, hipStream_t s) {
  const int n16 = ncol / 16;
  int ntw = 1;
  for (int c = 4; c >= 1; --c)
    if (n16 % c == 0) {
      ntw = c;
      break;
    }
  const dim3 g(n16 / ntw, static_cast<unsigned>(rows / CRM));
  switch (ntw) {
    case 4: KS::template rows_k<4>(g, s, W, ldw, Tt, M, ncol, C, accum); break;
    case 3: KS::template rows_k<3>(g, s, W, ldw, Tt, M, ncol, C, accum); break;
    case 2: KS::template rows_k<2>(g, s, W, ldw, Tt, M, ncol, C, accum); break;
    default: KS::template rows_k<1>(g, s, W, ldw, Tt, M, ncol, C, accum); break;
  }
}

template <class KS>
static int run_sym(const Plan& p, const double* B_vv, const double* tau, double* R, void* ws, hipStream_t s) {
  typedef typename KS::T T;
  Carve cv(ws, p.bytes);
  T* Bc = cv.take<T>(p.n_Bc);
  T* Tp = cv.take<T>(p.n_Tp);
  T* Tm = cv.take<T>(p.n_Tm);
  T* Wp = cv.take<T>(p.n_W);
  T* Wm = cv.take<T>(p.pm > 0 ? p.n_W : 0);
  T* S = cv.take<T>(p.n_S);
  T* A = cv.take<T>(p.n_A);
  T* S2 = cv.take<T>(p.n_S2);
  T* A2 = cv.take<T>(p.n_A2);
  const double oo = static_cast<double>(p.o) * p.o;
  RI_TRY(stage_inputs<KS>(p, B_vv, static_cast<long>(p.v) * p.v, p.v, tau, Bc, Tp, Tm, s));
  long first_p1 = -1;  // first row pair of S2 written (by the first slab's second product)
  for (long slab0 = 0; slab0 < p.nbp; slab0 += p.slab_bp) {
    const long npairs = std::min(p.nbp - slab0, p.slab_bp), p1 = slab0 + npairs;
    const long M = npairs * 256;
    const long K1 = p.K - slab0 * 256;  // cd slots from the slab's first pair on
    double le, lt, ld, ce, ct, cd;
    count_pairs(p.v, slab0, npairs, le, lt, ld);
    count_pairs(p.v, slab0, p.nbp - slab0, ce, ct, cd);
    int dy0, ndiag;
    diag_pairs(slab0, npairs, dy0, ndiag);
    const unsigned gx = static_cast<unsigned>((p.nbp - slab0) * 4);
    const double per_ab = 2.0 * p.naux * (2.0 * ct + (ce - ct));
    {
      ProfScope ps(s, KS::build, per_ab * (le - ld));
      KS::build_k(dim3(gx, npairs), s, Bc, p.naux_p, p.vp, slab0, p.slab_M, p.pm > 0 ? 1 : 0, slab0, Wp, Wm);
      RI_TRY(check_launch(KS::build));
    }
    if (ndiag > 0) {
      ProfScope ps(s, KS::build_diag, per_ab * ld);
      KS::build_diag_k(dim3(gx, ndiag), s, Bc, p.naux_p, p.vp, slab0, p.slab_M, p.pm > 0 ? 1 : 0, dy0, slab0, Wp,
                       Wm);
      RI_TRY(check_launch(KS::build_diag));
    }
    const size_t w0 = static_cast<size_t>(slab0) * 256 * p.slab_M;  // row slab0*256 of W
    long kzp = 0, kzm = 0;
    const int zp = contract_splits(p.NP, p.ntw_p, M, K1, p.esize, kzp);
    const int zm = p.pm > 0 ? contract_splits(p.NM, p.ntw_m, M, K1, p.esize, kzm) : 1;
    {
      ProfScope ps(s, KS::contract, 2.0 * (le * ce * p.po + lt * ct * p.pm));
      launch_contract<KS>(p.ntw_p, Wp + w0, Tp + static_cast<size_t>(slab0) * 256 * p.NP, K1, p.slab_M, M, p.NP, S,
                          zp, kzp, s);
      RI_TRY(check_launch(KS::contract));
      if (p.pm > 0) {
        launch_contract<KS>(p.ntw_m, Wm + w0, Tm + static_cast<size_t>(slab0) * 256 * p.NM, K1, p.slab_M, M, p.NM,
                            A, zm, kzm, s);
        RI_TRY(check_launch(KS::contract));
      }
    }
    {
      ProfScope ps(s, KS::unpack, 0.0, 16.0 * oo * (le + lt));
      unpack_kernel<T><<<dim3(npairs, (p.po + NG - 1) / NG), 256, 0, s>>>(S, A, p.NP, p.NM, p.o, p.v, slab0, R, zp,
                                                                        M * p.NP, zm, M * p.NM, 0);
      RI_TRY(check_launch(KS::unpack));
    }
    if (p1 < p.nbp) {  // second product: rows cd >= P1 of W against the slab's own T rows
      const long rows = (p.nbp - p1) * 256;
      const int accum = first_p1 < 0 ? 0 : 1;
      if (first_p1 < 0) first_p1 = p1;
      const size_t wr = static_cast<size_t>(p1) * 256 * p.slab_M;
      double le2, lt2, ld2;
      count_pairs(p.v, p1, p.nbp - p1, le2, lt2, ld2);
      ProfScope ps(s, KS::contract_rows, 2.0 * (le2 * le * p.po + lt2 * lt * p.pm));
      launch_contract_rows<KS>(Wp + wr, p.slab_M, Tp + static_cast<size_t>(slab0) * 256 * p.NP, M, rows, p.NP,
                               S2 + static_cast<size_t>(p1) * 256 * p.NP, accum, s);
      RI_TRY(check_launch(KS::contract_rows));
      if (p.pm > 0) {
        launch_contract_rows<KS>(Wm + wr, p.slab_M, Tm + static_cast<size_t>(slab0) * 256 * p.NM, M, rows, p.NM,
                                 A2 + static_cast<size_t>(p1) * 256 * p.NM, accum, s);
        RI_TRY(check_launch(KS::contract_rows));
      }
    }
  }
  if (first_p1 >= 0) {
    const long n2 = p.nbp - first_p1;
    double le, lt, ld;
    count_pairs(p.v, first_p1, n2, le, lt, ld);
    ProfScope ps(s, KS::unpack, 0.0, 16.0 * oo * (le + lt));
    unpack_kernel<T><<<dim3(n2, (p.po + NG - 1) / NG), 256, 0, s>>>(
        S2 + static_cast<size_t>(first_p1) * 256 * p.NP, A2 + static_cast<size_t>(first_p1) * 256 * p.NM, p.NP,
        p.NM, p.o, p.v, first_p1, R, 1, 0, 1, 0, 0);
    RI_TRY(check_launch(KS::unpack));
  }
  return RI_OK;
}

// ---------------------------------------------------------------- pair symmetry
// The ladder uses only the pair-symmetric part of tau (tau^{cd}_{ij} = tau^{dc}_{ji},
// Sec. II.C).  These kernels measure how far an input is from it:
// out = {max |tau[i][j][c][d] - tau[j][i][d][c]|, max |tau|}; NaN propagates.
constexpr int ASYM_BLOCKS = 1024;
__device__ inline double nan_max(double m, double x) { return (x != x || x > m) ? x : m; }
__device__ inline void block_max2(double& a, double& b, double* sh) {
  const int t = threadIdx.x;
  sh[t] = a;
  sh[256 + t] = b;
  __syncthreads();
  for (int k = 128; k > 0; k >>= 1) {
    if (t < k) {
      sh[t] = nan_max(sh[t], sh[t + k]);
      sh[256 + t] = nan_max(sh[256 + t], sh[256 + t + k]);
    }
    __syncthreads();
  }
  a = sh[0];
  b = sh[256];
}
__global__ __launch_bounds__(256) void pair_asym_partial(const double* __restrict__ tau, int o, int v, double* part) {
  __shared__ double sh[512];
  const long vv = static_cast<long>(v) * v, n = static_cast<long>(o) * o * vv;
  double asym = 0.0, amax = 0.0;
  for (long x = static_cast<long>(blockIdx.x) * 256 + threadIdx.x; x < n; x += static_cast<long>(gridDim.x) * 256) {
    const long ij = x / vv, cd = x - ij * vv;
    const int i = static_cast<int>(ij / o), j = static_cast<int>(ij - static_cast<long>(i) * o);
    const int c = static_cast<int>(cd / v), d = static_cast<int>(cd - static_cast<long>(c) * v);
    const double t = tau[x];
    const double m = tau[(static_cast<long>(j) * o + i) * vv + static_cast<long>(d) * v + c];
    asym = nan_max(asym, fabs(t - m));
    amax = nan_max(amax, fabs(t));
  }
  block_max2(asym, amax, sh);
  if (threadIdx.x == 0) {
    part[2 * blockIdx.x] = asym;
    part[2 * blockIdx.x + 1] = amax;
  }
}
__global__ __launch_bounds__(256) void pair_asym_final(const double* __restrict__ part, double* out) {
  __shared__ double sh[512];
  double asym = 0.0, amax = 0.0;
  for (int k = threadIdx.x; k < ASYM_BLOCKS; k += 256) {
    asym = nan_max(asym, part[2 * k]);
    amax = nan_max(amax, part[2 * k + 1]);
  }
  block_max2(asym, amax, sh);
  if (threadIdx.x == 0) {
    out[0] = asym;
    out[1] = amax;
  }
}
// The same for factors: out = {max |B[q][a][c] - B[q][c][a]|, max |B|}.
__global__ __launch_bounds__(256) void factor_asym_partial(const double* __restrict__ B, int naux, int v,
                                                           double* part) {
  __shared__ double sh[512];
  const long vv = static_cast<long>(v) * v, n = static_cast<long>(naux) * vv;
  double asym = 0.0, amax = 0.0;
  for (long x = static_cast<long>(blockIdx.x) * 256 + threadIdx.x; x < n; x += static_cast<long>(gridDim.x) * 256) {
    const long q = x / vv, ac = x - q * vv;
    const int a = static_cast<int>(ac / v), c = static_cast<int>(ac - static_cast<long>(a) * v);
    const double t = B[x];
    const double m = B[q * vv + static_cast<long>(c) * v + a];
    asym = nan_max(asym, fabs(t - m));
    amax = nan_max(amax, fabs(t));
  }
  block_max2(asym, amax, sh);
  if (threadIdx.x == 0) {
    part[2 * blockIdx.x] = asym;
    part[2 * blockIdx.x + 1] = amax;
  }
}
// Runs a partial kernel (launched by `partial` into ASYM_BLOCKS pairs) and the final
// reduction; copies the two maxima to host2 and synchronises the stream.
// scratch: a device buffer of at least ASYM_BYTES (NULL: allocated for the call).
constexpr size_t ASYM_BYTES = (2 * ASYM_BLOCKS + 2) * sizeof(double);
static_assert(ASYM_BYTES == ASYM_SCRATCH_BYTES, "the header states the check's buffer size");
template <class F>
static int max_pair(F&& partial, double* host2, hipStream_t s, void* scratch = nullptr) {
  void* buf = scratch;
  if (!buf) RI_TRY(dev_alloc(&buf, ASYM_BYTES, s));
  double* part = static_cast<double*>(buf);
  partial(part);
  pair_asym_final<<<1, 256, 0, s>>>(part, part + 2 * ASYM_BLOCKS);
  int rc = check_launch("pair_asym");
  if (rc == RI_OK) rc = check_hip(hipMemcpyAsync(host2, part + 2 * ASYM_BLOCKS, 2 * sizeof(double),
                                                 hipMemcpyDeviceToHost, s), "pair_asym copy");
  if (rc == RI_OK) rc = check_hip(hipStreamSynchronize(s), "pair_asym sync");
  if (!scratch) dev_free(buf, s);
  return rc;
}
int pair_asymmetry(const double* tau, int o, int v, double* host2, hipStream_t s, void* scratch = nullptr) {
  return max_pair([&](double* part) { pair_asym_partial<<<ASYM_BLOCKS, 256, 0, s>>>(tau, o, v, part); }, host2, s,
                  scratch);
}
int factor_asymmetry(const double* B, int naux, int v, double* host2, hipStream_t s) {
  return max_pair([&](double* part) { factor_asym_partial<<<ASYM_BLOCKS, 256, 0, s>>>(B, naux, v, part); }, host2,
                  s);
}
// RI_PPL_CHECK_TAU set (and not "0"): the ladder first checks that tau is
// pair-symmetric to 1e-12 of its largest element and rejects it otherwise.
int check_tau_if_asked(const double* tau, int o, int v, hipStream_t s, void* scratch) {
  const char* e = getenv("RI_PPL_CHECK_TAU");
  if (!e || !*e || (e[0] == '0' && e[1] == 0)) return RI_OK;
  double r[2];
  RI_TRY(pair_asymmetry(tau, o, v, r, s, scratch));
  if (!(r[0] <= 1e-12 * r[1])) {
    set_error("ri_ppl: tau is not pair-symmetric: max |tau_ij^cd - tau_ji^dc| = %.3e, max |tau| = %.3e", r[0], r[1]);
    return RI_E_ARG;
  }
  return RI_OK;
}

// Arguments shared by the ladder entry points: pointers, precision, sizes, aliasing
// of R with the inputs and 8-byte alignment.
int check_ladder_args(const double* B_vv, const double* tau, int o, int v, int naux, const double* R,
                      int precision, const char* who) {
  if (!B_vv || !tau || !R) {
    set_error("%s: null pointer argument", who);
    return RI_E_ARG;
  }
  if (precision != RI_PREC_FP64 && precision != RI_PREC_FP32 && precision != RI_PREC_BF16X3) {
    set_error("%s: unknown precision %d", who, precision);
    return RI_E_ARG;
  }
  Plan p;
  if (!make_plan(o, v, naux, esize_of(precision), p)) {
    set_error("%s: invalid sizes o=%d v=%d naux=%d", who, o, v, naux);
    return RI_E_ARG;
  }
  const size_t nB = static_cast<size_t>(naux) * v * v * sizeof(double);
  const size_t nT = static_cast<size_t>(o) * o * v * v * sizeof(double);
  if (overlaps(R, nT, B_vv, nB) || overlaps(R, nT, tau, nT)) {
    set_error("%s: R overlaps an input", who);
    return RI_E_ALIAS;
  }
  if ((reinterpret_cast<uintptr_t>(B_vv) | reinterpret_cast<uintptr_t>(tau) |
       reinterpret_cast<uintptr_t>(R)) & 7) {
    set_error("%s: arrays must be 8-byte aligned", who);
    return RI_E_ARG;
  }
  return RI_OK;
}

size_t min_workspace_bytes(int o, int v, int naux, int precision) {
  if (precision == RI_PREC_BF16X3) return bf16x3_workspace_bytes_min(o, v, naux);
  Plan p;
  if (!make_plan(o, v, naux, esize_of(precision), p)) return 0;
  p.slab_bp = 1;
  size_plan(p, false);
  return p.bytes;
}

int run_fit(const double* B_vv, const double* tau, int o, int v, int naux, double* R, int precision, void* ws,
            size_t ws_bytes, hipStream_t s) {
  const long rs = v, qs = static_cast<long>(v) * v;
  if (precision == RI_PREC_BF16X3) return bf16x3_run(B_vv, qs, rs, tau, o, v, naux, R, ws, ws_bytes, 0, 1, s, true);
  Plan p;
  if (!make_plan(o, v, naux, esize_of(precision), p, false, ws_bytes)) {
    set_error("ladder: no slab plan for o=%d v=%d naux=%d fits %zu bytes of workspace", o, v, naux, ws_bytes);
    return RI_E_NOMEM;
  }
  return run_typed(p, precision, B_vv, qs, rs, tau, R, ws, 0, 1, s);
}

}  // namespace ppl

int ppl_strided(const double* B, long qs, long rs, const double* tau, int o, int v, int naux, double* R,
                int precision, hipStream_t s) {
  if (precision == RI_PREC_BF16X3) return ppl::bf16x3_run(B, qs, rs, tau, o, v, naux, R, nullptr, 0, 0, 1, s);
  if (precision != RI_PREC_FP64 && precision != RI_PREC_FP32) {
    set_error("ladder: unknown precision %d", precision);
    return RI_E_ARG;
  }
  ppl::Plan p;
  if (!ppl::make_plan(o, v, naux, ppl::esize_of(precision), p)) {
    set_error("ladder: invalid sizes o=%d v=%d naux=%d", o, v, naux);
    return RI_E_ARG;
  }
  return ppl::run_typed(p, precision, B, qs, rs, tau, R, nullptr, 0, 1, s);
}

}  // namespace ri

using namespace ri;

extern "C" {

size_t ri_ppl_workspace_bytes(int o, int v, int naux, int precision) {
  ppl::Plan p;
  if (precision == RI_PREC_BF16X3) return ppl::bf16x3_workspace_bytes(o, v, naux);
  if (precision != RI_PREC_FP64 && precision != RI_PREC_FP32) return 0;
  if (!ppl::make_plan(o, v, naux, ppl::esize_of(precision), p)) return 0;
  return p.bytes;
}

double ri_ppl_flops(int o, int v, int naux) {
  if (o <= 0 || v <= 0 || naux <= 0) return 0.0;
  const double dv = v, pv = dv * (dv + 1) / 2, pvm = dv * (dv - 1) / 2;
  const double po = o * (o + 1.0) / 2, pom = o * (o - 1.0) / 2;
  return static_cast<double>(naux) * dv * dv * dv * (dv + 1) + 2.0 * (pv * pv * po + pvm * pvm * pom);
}

int ri_ppl_shard(const double* B_vv, const double* tau, int o, int v, int naux, double* R, int precision,
                 int shard, int nshards, void* ws, size_t ws_bytes, void* stream) {
  clear_error();
  if (nshards < 1 || shard < 0 || shard >= nshards) {
    set_error("ri_ppl: shard %d of %d is not a valid shard", shard, nshards);
    return RI_E_ARG;
  }
  RI_TRY(ppl::check_ladder_args(B_vv, tau, o, v, naux, R, precision, "ri_ppl"));
  ppl::Plan p;
  if (!ppl::make_plan(o, v, naux, ppl::esize_of(precision), p)) {
    set_error("ri_ppl: invalid sizes o=%d v=%d naux=%d", o, v, naux);
    return RI_E_ARG;
  }
  hipStream_t s = static_cast<hipStream_t>(stream);
  if (ws && (reinterpret_cast<uintptr_t>(ws) & 255)) {
    set_error("ri_ppl: workspace must be 256-byte aligned");
    return RI_E_ARG;
  }
  RI_TRY(ppl::check_tau_if_asked(tau, o, v, s));
  if (precision == RI_PREC_BF16X3)
    return ppl::bf16x3_run(B_vv, static_cast<long>(v) * v, v, tau, o, v, naux, R, ws, ws_bytes, shard, nshards, s);
  if (ws && ws_bytes < p.bytes) {
    set_error("ri_ppl: workspace of %zu bytes is smaller than the %zu required", ws_bytes, p.bytes);
    return RI_E_NOMEM;
  }
  return ppl::run_typed(p, precision, B_vv, static_cast<long>(v) * v, v, tau, R, ws, shard, nshards, s);
}

int ri_ppl_ex(const double* B_vv, const double* tau, int o, int v, int naux, double* R, int precision,
              void* ws, size_t ws_bytes, void* stream) {
  return ri_ppl_shard(B_vv, tau, o, v, naux, R, precision, 0, 1, ws, ws_bytes, stream);
}

int ri_ppl(const double* B_vv, const double* tau, int o, int v, int naux, double* R, void* stream) {
  return ri_ppl_ex(B_vv, tau, o, v, naux, R, RI_PREC_FP64, nullptr, 0, stream);
}

int ri_ppl_sym_ex(const double* B_vv, const double* tau, int o, int v, int naux, double* R, int precision,
                  void* stream) {
  clear_error();
  RI_TRY(ppl::check_ladder_args(B_vv, tau, o, v, naux, R, precision, "ri_ppl_sym"));
  // the slab width is the FP64 plan's for every precision, so the schedule (and the
  // FLOP count of ri_ppl_sym_flops) does not depend on the precision
  ppl::Plan p64;
  if (!ppl::make_plan(o, v, naux, 8, p64, true)) {
    set_error("ri_ppl_sym: invalid sizes o=%d v=%d naux=%d", o, v, naux);
    return RI_E_ARG;
  }
  hipStream_t s = static_cast<hipStream_t>(stream);
  RI_TRY(ppl::check_tau_if_asked(tau, o, v, s));
  double r[2];
  RI_TRY(ppl::factor_asymmetry(B_vv, naux, v, r, s));
  if (!(r[0] <= 1e-12 * r[1])) {
    set_error("ri_ppl_sym: B_vv is not symmetric in its virtual indices: max |B_ac - B_ca| = %.3e, max |B| = %.3e",
              r[0], r[1]);
    return RI_E_ARG;
  }
  if (precision == RI_PREC_BF16X3) return ppl::bf16x3_run_sym(B_vv, tau, o, v, naux, R, p64.slab_bp, s);
  ppl::Plan p = p64;
  if (precision == RI_PREC_FP32) {
    ppl::make_plan(o, v, naux, 4, p, true);
    p.slab_bp = p64.slab_bp;
    ppl::size_plan(p, true);
  }
  void* buf = nullptr;
  RI_TRY(dev_alloc(&buf, p.bytes, s));
  const int rc = precision == RI_PREC_FP32 ? ppl::run_sym<ppl::K32>(p, B_vv, tau, R, buf, s)
                                           : ppl::run_sym<ppl::K64>(p, B_vv, tau, R, buf, s);
  dev_free(buf, s);
  return rc;
}

int ri_ppl_sym(const double* B_vv, const double* tau, int o, int v, int naux, double* R, void* stream) {
  return ri_ppl_sym_ex(B_vv, tau, o, v, naux, R, RI_PREC_FP64, stream);
}

double ri_ppl_sym_flops(int o, int v, int naux) {
  ppl::Plan p;
  if (!ppl::make_plan(o, v, naux, 8, p, true)) return 0.0;
  double build, contract;
  ppl::sym_flops(p, build, contract);
  return build + contract;
}

int ri_tau_pair_asymmetry(const double* tau, int o, int v, double* result, void* stream) {
  clear_error();
  if (!tau || !result || o <= 0 || v <= 0 || static_cast<long>(o) * o * v * v > (1L << 40)) {
    set_error("ri_tau_pair_asymmetry: invalid argument");
    return RI_E_ARG;
  }
  return ppl::pair_asymmetry(tau, o, v, result, static_cast<hipStream_t>(stream));
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
