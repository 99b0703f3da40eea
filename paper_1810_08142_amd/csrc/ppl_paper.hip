// Particle-particle ladder in the paper's own arrangement (Sec. II.C, Fig. 2), kept
// beside the tau+- path as an ablation of its FLOP trade-off.
//
// The paper uses only the pair symmetry of tau over the occupied pair: for every
// virtual a it builds the full (ac|bd) slice over (b, c, d) from the RI factors and
// contracts it with tau^{cd}_{ij} over the packed pairs lambda = (i <= j).  Its cost
// is 2 Naux v^4 FLOP for the build and 2 v^4 p_o for the contraction (p_o = o(o+1)/2),
// about twice the build and four times the contraction of the tau+- form, which also
// uses the (a, b) and (c, d) symmetries.  The R entries with i > j follow from the
// pair symmetry R^{ab}_{ij} = R^{ba}_{ji}.
//
// Layout: T [c][d][lambda] (the pair-symmetric part of tau), V [a][c][b][d] for a
// chunk of a, X [lambda][a][b]; lambda = j(j+1)/2 + i for i <= j.  The build and the
// contraction run on the library's FP64 MFMA GEMM engine; two small kernels pack tau
// and scatter X into R.
#include "gemm.h"
#include "ppl_shared.h"

namespace ri {
namespace paper {

using ppl::tri_decode;

// T[c][d][l] = (tau[i][j][c][d] + tau[j][i][d][c]) / 2 for l = (i <= j); one thread per
// element of T in order (l fastest).  grid ceil(v*v*po/256)
__global__ __launch_bounds__(256) void pack_lambda(const double* __restrict__ tau, int o, int v, int po,
                                                   double* __restrict__ T) {
  const long idx = static_cast<long>(blockIdx.x) * 256 + threadIdx.x;
  const long vv = static_cast<long>(v) * v;
  if (idx >= vv * po) return;
  const long cd = idx / po;
  const int l = static_cast<int>(idx - cd * po);
  const int c = static_cast<int>(cd / v), d = static_cast<int>(cd - static_cast<long>(c) * v);
  int i, j;
  tri_decode(l, i, j);
  const double x1 = tau[(static_cast<long>(i) * o + j) * vv + cd];
  const double x2 = tau[(static_cast<long>(j) * o + i) * vv + static_cast<long>(d) * v + c];
  T[cd * po + l] = 0.5 * (x1 + x2);
}

// R[i][j][a][b] += X[l][a][b] and, for i < j, R[j][i][b][a] += X[l][a][b], with l = (i <= j):
// every R entry is written by one thread.  A 32 x 32 (a, b) tile goes through LDS for
// the transposed half.  grid (po, ceil(v/32), ceil(v/32)), block (32, 8)
__global__ __launch_bounds__(256) void unpack_lambda(const double* __restrict__ X, int o, int v,
                                                     double* __restrict__ R) {
  __shared__ double tile[32][33];
  const int l = blockIdx.x;
  int i, j;
  tri_decode(l, i, j);
  const int a0 = blockIdx.z * 32, b0 = blockIdx.y * 32;
  const int tx = threadIdx.x, ty = threadIdx.y;
  const long vv = static_cast<long>(v) * v;
  const double* Xl = X + static_cast<long>(l) * vv;
  double* Rij = R + (static_cast<long>(i) * o + j) * vv;
  for (int r = ty; r < 32; r += 8) {
    const int a = a0 + r, b = b0 + tx;
    if (a < v && b < v) {
      const double x = Xl[static_cast<long>(a) * v + b];
      tile[r][tx] = x;
      Rij[static_cast<long>(a) * v + b] += x;
    }
  }
  if (i == j) return;  // uniform over the block
  __syncthreads();
  double* Rji = R + (static_cast<long>(j) * o + i) * vv;
  for (int r = ty; r < 32; r += 8) {
    const int b = b0 + r, a = a0 + tx;
    if (a < v && b < v) Rji[static_cast<long>(b) * v + a] += tile[tx][r];
  }
}

}  // namespace paper
}  // namespace ri

using namespace ri;

extern "C" {

double ri_ppl_paper_flops(int o, int v, int naux) {
  if (o <= 0 || v <= 0 || naux <= 0) return 0.0;
  const double v4 = static_cast<double>(v) * v * v * v, po = o * (o + 1.0) / 2;
  return 2.0 * naux * v4 + 2.0 * v4 * po;
}

int ri_ppl_paper(const double* B_vv, const double* tau, int o, int v, int naux, double* R, void* stream) {
  clear_error();
  if (!B_vv || !tau || !R) {
    set_error("ri_ppl_paper: null pointer argument");
    return RI_E_ARG;
  }
  if (o <= 0 || v <= 0 || naux <= 0 || o > 4096 || v > 65536 || naux > (1 << 24)) {
    set_error("ri_ppl_paper: invalid sizes o=%d v=%d naux=%d", o, v, naux);
    return RI_E_ARG;
  }
  const long vv = static_cast<long>(v) * v;
  const size_t nB = static_cast<size_t>(naux) * vv * sizeof(double);
  const size_t nT = static_cast<size_t>(o) * o * vv * sizeof(double);
  if (overlaps(R, nT, B_vv, nB) || overlaps(R, nT, tau, nT)) {
    set_error("ri_ppl_paper: R overlaps an input");
    return RI_E_ALIAS;
  }
  hipStream_t s = static_cast<hipStream_t>(stream);
  const int po = o * (o + 1) / 2;
  if (static_cast<double>(vv) * po >= 256.0 * 2147483647.0) {
    set_error("ri_ppl_paper: v^2 o(o+1)/2 too large for one packing launch");
    return RI_E_ARG;
  }
  // a values per chunk: the V slice [na][v][v][v] within RI_PPL_PAPER_V_BYTES (4 GiB)
  const long vbytes = ppl::env_long("RI_PPL_PAPER_V_BYTES", 4L << 30);
  const double per_a = static_cast<double>(vv) * v * sizeof(double);
  const int na = static_cast<int>(std::max(1.0, std::min(static_cast<double>(v), static_cast<double>(vbytes) / per_a)));
  const size_t nTl = static_cast<size_t>(vv) * po, nX = nTl, nV = static_cast<size_t>(na) * vv * v;
  void* buf = nullptr;
  RI_TRY(dev_alloc(&buf, (nTl + nX + nV) * sizeof(double), s));
  double* T = static_cast<double*>(buf);
  double* X = T + nTl;
  double* V = X + nX;
  int rc = RI_OK;
  {
    GemmArena arena;
    arena.s = s;
    do {
      {
        ProfScope ps(s, "pack_lambda", 0.0, 16.0 * vv * po + 8.0 * vv * po);
        paper::pack_lambda<<<static_cast<unsigned>((vv * po + 255) / 256), 256, 0, s>>>(tau, o, v, po, T);
        if ((rc = check_launch("pack_lambda"))) break;
      }
      for (int a0 = 0; a0 < v && rc == RI_OK; a0 += na) {
        const int n = std::min(na, v - a0);
        // V[a][c][b][d] = (ac|bd) = sum_Q B[Q][a][c] B[Q][b][d] for the chunk's a
        rc = einsum("Qac,Qbd->acbd", 1.0, Tensor(B_vv + static_cast<long>(a0) * v, {naux, n, v}, {vv, v, 1}),
                    Tensor(B_vv, {naux, v, v}), 0.0, Tensor(V, {n, v, v, v}), arena, s);
        if (rc) break;
        // X[l][a][b] = sum_{c,d} V[a][c][b][d] T[c][d][l]
        rc = einsum("acbd,cdl->abl", 1.0, Tensor(V, {n, v, v, v}), Tensor(T, {v, v, po}), 0.0,
                    Tensor(X + static_cast<long>(a0) * v, {n, v, po}, {v, 1, vv}), arena, s);
      }
      if (rc) break;
      {
        ProfScope ps(s, "unpack_lambda", 0.0, 8.0 * vv * po + 16.0 * vv * o * o);
        paper::unpack_lambda<<<dim3(po, (v + 31) / 32, (v + 31) / 32), dim3(32, 8), 0, s>>>(X, o, v, R);
        rc = check_launch("unpack_lambda");
      }
    } while (false);
  }
  dev_free(buf, s);
  return rc;
}

}  // extern "C"
