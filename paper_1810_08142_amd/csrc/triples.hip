// Perturbative triples energy E_(T) of closed-shell CCSD(T) (Sec. II.A): FP64, with an
// FP32 option for the term GEMMs.
//
//   E_(T) = sum_{ijk} sum_{abc} (4 W^{abc}_{ijk} + W^{bca}_{ijk} + W^{cab}_{ijk})
//                               (V^{abc}_{ijk} - V^{cba}_{ijk}) / (3 D^{abc}_{ijk}),
//   W^{abc}_{ijk} = P^{abc}_{ijk} X(ijk, abc),
//   X(ijk, abc)   = sum_d (bd|ai) t^{cd}_{kj} - sum_l (ck|jl) t^{ab}_{il},
//   V^{abc}_{ijk} = W^{abc}_{ijk} + (jb|kc) t^a_i + (ia|kc) t^b_j + (ia|jb) t^c_k,
//   D^{abc}_{ijk} = e_i + e_j + e_k - e_a - e_b - e_c,
//
// (v^{pq}_{rs} = (pr|qs); P sums the six simultaneous permutations of the column pairs
// (i, a), (j, b), (k, c)).  W and V are invariant under those simultaneous
// permutations, so one triplet i <= j <= k gives W and V for every ordering of it:
// W_{i'j'k'} is W_{ijk} with its virtual indices permuted the same way.  The summand
// itself is not invariant (W^{bca}, W^{cab} and V^{cba} relabel the virtuals alone),
// so the energy kernel evaluates it for each distinct ordering (i', j', k') from the
// one W and V, reading them through permuted tiles.
//
// Per triplet: six GEMMs on the library's MFMA engine (FP64 or FP32), one per term of P, each
// writing its term in its own natural layout (contiguous output rows; the o-sized sum
// of a term rides along as extra columns of the summed index), a tiled kernel
// symmetrises the six into W and forms V = W + the t1 terms, and a tiled kernel sums
// the energy in a fixed order.  The GEMM operands (with (yd|xp) and (zr|ql) from the
// RI factors) and (ia|jb) are built once.
#include <cmath>
#include <vector>

#include "gemm.h"

namespace ri {
namespace trip {

constexpr int TE = 8;  // tile edge of the energy kernel

// element m of permutation p of (0, 1, 2): p in the order 012 021 102 120 201 210, the
// 18 two-bit elements packed in that order
__host__ __device__ inline int perm_at(int p, int m) {
  constexpr unsigned long long table = 0x192261624ull;
  return static_cast<int>((table >> (2 * (3 * p + m))) & 3ull);
}

// One ordering (i', j', k') of the triplet and the tiles its four reads come from:
// r1 for W'^{abc} (and V'^{abc}), r2 for W'^{bca}, r3 for W'^{cab}, r4 for V'^{cba}.
struct Order {
  int ip, jp, kp;
  int r1, r2, r3, r4;
};
struct Orders {
  int n;
  Order t[6];
};

// W[a][b][c] = sum_p Y_p[y0][y1][y2] with y_m = (a, b, c)[perm(p, m)] (the six terms of
// P, each computed in its own natural layout), and V = W + (jb|kc) t^a_i + (ia|kc) t^b_j
// + (ia|jb) t^c_k.  Each block stages, term by term, the 8^3 tile of Y_p at the
// permuted block coordinates in LDS and reads it transposed, so every global access
// runs along c.  grid nt^3, block 512.
__global__ __launch_bounds__(512) void assemble_wv(const double* __restrict__ Y, const double* __restrict__ K,
                                                   const double* __restrict__ t1, int o, int v, int i, int j, int k,
                                                   double* __restrict__ W, double* __restrict__ V) {
  __shared__ double tile[TE][TE][TE];
  const int nt = (v + TE - 1) / TE;
  const long bid = blockIdx.x;
  const int Z0 = static_cast<int>(bid / (static_cast<long>(nt) * nt)) * TE;
  const int Z1 = static_cast<int>((bid / nt) % nt) * TE;
  const int Z2 = static_cast<int>(bid % nt) * TE;
  const int t = threadIdx.x, u = t >> 6, w = (t >> 3) & 7, z = t & 7;
  auto Zof = [&](int m) { return m == 0 ? Z0 : (m == 1 ? Z1 : Z2); };
  auto xl = [&](int m) { return m == 0 ? u : (m == 1 ? w : z); };
  const long v3 = static_cast<long>(v) * v * v;
  double acc = 0.0;
  for (int p = 0; p < 6; ++p) {
    const int y0 = Zof(perm_at(p, 0)) + u, y1 = Zof(perm_at(p, 1)) + w, y2 = Zof(perm_at(p, 2)) + z;
    const bool in = y0 < v && y1 < v && y2 < v;
    tile[u][w][z] = in ? Y[p * v3 + (static_cast<long>(y0) * v + y1) * v + y2] : 0.0;
    __syncthreads();
    acc += tile[xl(perm_at(p, 0))][xl(perm_at(p, 1))][xl(perm_at(p, 2))];
    __syncthreads();
  }
  const int a = Z0 + u, b = Z1 + w, c = Z2 + z;
  if (a < v && b < v && c < v) {
    auto Kx = [&](int i1, int p1, int i2, int p2) { return K[((static_cast<long>(i1) * v + p1) * o + i2) * v + p2]; };
    const long at = (static_cast<long>(a) * v + b) * v + c;
    W[at] = acc;
    V[at] = acc + Kx(j, b, k, c) * t1[i * v + a] + Kx(i, a, k, c) * t1[j * v + b] + Kx(i, a, j, b) * t1[k * v + c];
  }
}

// index of the permutation (e0, e1, e2) in the order of perm_at
__host__ __device__ inline int perm_index(int e0, int e1) { return 2 * e0 + (e1 > e0 ? e1 - 1 : e1); }

// Energy of one triplet over the orderings in `ord`, summed per unordered triple of
// 8-wide tiles {A, B, C} (A <= B <= C, packed in tiles[] as A | B << 10 | C << 20)
// into part[block].  Each block stages the six orientations of its tile triple of W
// and V in LDS (orientation p holds W[Z_p0 + u][Z_p1 + w][Z_p2 + z] for Z = (A, B, C)
// in elements) and evaluates every distinct ordering s of the triple from them, so each
// tile of W and V is read from memory once per triplet.  grid = number of tile
// triples, block 512.
__global__ __launch_bounds__(512) void energy_tiles(const double* __restrict__ W, const double* __restrict__ V,
                                                    const double* __restrict__ eps, int o, int v, Orders ord,
                                                    const int* __restrict__ tiles, double* __restrict__ part) {
  __shared__ double tw[6][TE][TE][TE];
  __shared__ double tv[6][TE][TE][TE];
  __shared__ double red[512];
  const int code = tiles[blockIdx.x];
  const int bt[3] = {code & 1023, (code >> 10) & 1023, (code >> 20) & 1023};
  const int t = threadIdx.x, u = t >> 6, w = (t >> 3) & 7, z = t & 7;
  auto Zof = [&](int m) { return (m == 0 ? bt[0] : (m == 1 ? bt[1] : bt[2])) * TE; };
  for (int p = 0; p < 6; ++p) {
    const int y0 = Zof(perm_at(p, 0)) + u, y1 = Zof(perm_at(p, 1)) + w, y2 = Zof(perm_at(p, 2)) + z;
    const bool in = y0 < v && y1 < v && y2 < v;
    const long at = (static_cast<long>(y0) * v + y1) * v + y2;
    tw[p][u][w][z] = in ? W[at] : 0.0;
    tv[p][u][w][z] = in ? V[at] : 0.0;
  }
  __syncthreads();
  auto xl = [&](int m) { return m == 0 ? u : (m == 1 ? w : z); };  // local coordinate of a, b or c
  double acc = 0.0;
  for (int sg = 0; sg < 6; ++sg) {
    // skip an ordering of the tile triple that repeats an earlier one (equal tiles)
    const int k0 = bt[perm_at(sg, 0)], k1 = bt[perm_at(sg, 1)], k2 = bt[perm_at(sg, 2)];
    bool dup = false;
    for (int s2 = 0; s2 < sg; ++s2)
      dup = dup || (bt[perm_at(s2, 0)] == k0 && bt[perm_at(s2, 1)] == k1 && bt[perm_at(s2, 2)] == k2);
    if (dup) continue;
    const int a = k0 * TE + u, b = k1 * TE + w, c = k2 * TE + z;
    if (a >= v || b >= v || c >= v) continue;
    // element (a, b, c) of orientation sg; a read in orientation rho of (a, b, c) comes
    // from tile sg o rho at local coordinates (x_rho0, x_rho1, x_rho2)
    auto rd = [&](const double (*tt)[TE][TE][TE], int rho) {
      const int r0 = perm_at(rho, 0), r1 = perm_at(rho, 1);
      const int tau = perm_index(perm_at(sg, r0), perm_at(sg, r1));
      return tt[tau][xl(r0)][xl(r1)][xl(perm_at(rho, 2))];
    };
    // D is symmetric in (i, j, k): one reciprocal serves every ordering
    const double d = eps[ord.t[0].ip] + eps[ord.t[0].jp] + eps[ord.t[0].kp] - (eps[o + a] + eps[o + b] + eps[o + c]);
    double sum = 0.0;
#pragma unroll
    for (int q = 0; q < 6; ++q) {
      if (q >= ord.n) break;
      const Order& r = ord.t[q];
      sum += (4.0 * rd(tw, r.r1) + rd(tw, r.r2) + rd(tw, r.r3)) * (rd(tv, r.r1) - rd(tv, r.r4));
    }
    acc += sum / (3.0 * d);
  }
  red[t] = acc;
  __syncthreads();
  for (int s = 256; s > 0; s >>= 1) {
    if (t < s) red[t] += red[t + s];
    __syncthreads();
  }
  if (t == 0) part[blockIdx.x] = red[0];
}

// out[0] = sum of part[0..n) in a fixed order (one block)
__global__ __launch_bounds__(256) void sum_parts(const double* __restrict__ part, long n, double* out) {
  __shared__ double red[256];
  double acc = 0.0;
  for (long x = threadIdx.x; x < n; x += 256) acc += part[x];
  red[threadIdx.x] = acc;
  __syncthreads();
  for (int s = 128; s > 0; s >>= 1) {
    if (threadIdx.x < s) red[threadIdx.x] += red[threadIdx.x + s];
    __syncthreads();
  }
  if (threadIdx.x == 0) out[0] = red[0];
}

// The distinct orderings of (i, j, k) and their read tiles.
Orders orders_of(int i, int j, int k) {
  Orders out{};
  const int x[3] = {i, j, k};
  std::vector<std::vector<int>> seen;
  for (int p = 0; p < 6; ++p) {
    const int e0 = perm_at(p, 0), e1 = perm_at(p, 1), e2 = perm_at(p, 2);
    std::vector<int> key = {x[e0], x[e1], x[e2]};
    bool dup = false;
    for (auto& s : seen) dup = dup || s == key;
    if (dup) continue;
    seen.push_back(key);
    // (i', j', k') = (x[pi(0)], x[pi(1)], x[pi(2)]); inv = pi^{-1}
    int inv[3];
    inv[e0] = 0;
    inv[e1] = 1;
    inv[e2] = 2;
    Order& r = out.t[out.n++];
    r.ip = key[0];
    r.jp = key[1];
    r.kp = key[2];
    r.r1 = perm_index(inv[0], inv[1]);
    r.r2 = perm_index((inv[0] + 1) % 3, (inv[1] + 1) % 3);
    r.r3 = perm_index((inv[0] + 2) % 3, (inv[1] + 2) % 3);
    r.r4 = perm_index(2 - inv[0], 2 - inv[1]);
  }
  return out;
}

}  // namespace trip
}  // namespace ri

using namespace ri;

extern "C" {

double ri_ccsd_triples_flops(int o, int v) {
  if (o <= 0 || v <= 0) return 0.0;
  const double trip = o * (o + 1.0) * (o + 2.0) / 6.0, v3 = static_cast<double>(v) * v * v;
  return trip * 6.0 * 2.0 * v3 * (v + o);
}

int ri_ccsd_triples_ex(const ri_system* sys, const double* t1, const double* t2, int precision, double* e_t,
                       void* stream) {
  clear_error();
  RI_TRY(cc::check_system(sys, "ri_ccsd_triples"));
  if (!t1 || !t2 || !e_t) {
    set_error("ri_ccsd_triples: null pointer argument");
    return RI_E_ARG;
  }
  if (precision != RI_PREC_FP64 && precision != RI_PREC_FP32) {
    set_error("ri_ccsd_triples: precision %d is not FP64 or FP32", precision);
    return RI_E_ARG;
  }
  hipStream_t s = static_cast<hipStream_t>(stream);
  const int o = sys->o, v = sys->v, Q = sys->naux, n = o + v;
  const int vo = (v + o + 15) / 16 * 16;  // summed index of a term, padded with zeros to 16
  const long nn = static_cast<long>(n) * n, vv = static_cast<long>(v) * v, v3 = vv * v;
  const int nt = (v + trip::TE - 1) / trip::TE;
  if (nt > 1023) {
    set_error("ri_ccsd_triples: v = %d is too large for the energy tiles", v);
    return RI_E_ARG;
  }
  const long ntiles = static_cast<long>(nt) * nt * nt;        // assembly tiles (ordered)
  const long ntri = static_cast<long>(nt) * (nt + 1) * (nt + 2) / 6;  // energy tile triples
  const long ntrip = static_cast<long>(o) * (o + 1) * (o + 2) / 6;
  // Each term of P, X(p, q, r; x, y, z) = sum_d (yd|xp) t2[r][q][z][d] - sum_l (zr|ql) t2[p][l][x][y],
  // is one GEMM over the combined index e = (d, then l):
  //   A[p][x][y][e] = (yd|xp) for e = d < v,  t2[p][l][x][y] for e = v + l,
  //   Bt[r][q][z][e] = t2[r][q][z][d] for e = d < v,  -(zr|ql) for e = v + l.
  // Buffers: A [o][v][v][v+o], Bt [o][o][v][v+o], J [o][o][v][o], K [o][v][o][v],
  // Y [6][v][v][v] (the six terms), W and V [v][v][v], tile partials, triplet sums.
  const size_t nA = static_cast<size_t>(o) * vv * vo, nBt = static_cast<size_t>(o) * o * v * vo,
               nJ = static_cast<size_t>(o) * o * v * o, nK = static_cast<size_t>(o) * v * o * v;
  const size_t total = nA + nBt + nJ + nK + 8 * static_cast<size_t>(v3) + ntri + ntrip + (ntri + 1) / 2;
  void* buf = nullptr;
  RI_TRY(dev_alloc(&buf, total * sizeof(double), s));
  double* A = static_cast<double*>(buf);
  double* Bt = A + nA;
  double* J = Bt + nBt;
  double* K = J + nJ;
  double* Y = K + nK;
  double* W = Y + 6 * v3;
  double* Vt = W + v3;
  double* part = Vt + v3;
  double* et = part + ntri;
  int* tl = reinterpret_cast<int*>(et + ntrip);
  std::vector<int> tiles_host;
  tiles_host.reserve(ntri);
  for (int ta = 0; ta < nt; ++ta)
    for (int tb = ta; tb < nt; ++tb)
      for (int tc = tb; tc < nt; ++tc) tiles_host.push_back(ta | (tb << 10) | (tc << 20));
  int rc = RI_OK;
  {
    GemmArena arena;
    arena.s = s;
    const double* B = sys->B;
    // B views (occupied first): vv, vo, oo, ov blocks of [Q][n][n]
    const Tensor Bvv(B + static_cast<long>(o) * n + o, {Q, v, v}, {nn, n, 1});
    const Tensor Bvo(B + static_cast<long>(o) * n, {Q, v, o}, {nn, n, 1});
    const Tensor Boo(B, {Q, o, o}, {nn, n, 1});
    const Tensor Bov(B + o, {Q, o, v}, {nn, n, 1});
    const long sA2 = vo, sA1 = static_cast<long>(v) * vo, sA0 = vv * vo;  // strides of A
    const long sB2 = vo, sB1 = static_cast<long>(v) * vo, sB0 = static_cast<long>(o) * v * vo;  // of Bt
    do {
      if ((rc = check_hip(hipMemcpyAsync(tl, tiles_host.data(), ntri * sizeof(int), hipMemcpyHostToDevice, s),
                          "triples tiles")))
        break;
      // zero padding of the summed index (columns v + o .. vo - 1)
      if ((rc = check_hip(hipMemsetAsync(A, 0, (nA + nBt) * sizeof(double), s), "triples clear"))) break;
      // A[p][x][y][d] = (yd|xp)
      if ((rc = einsum("Qyd,Qxp->pxyd", 1.0, Bvv, Bvo, 0.0, Tensor(A, {o, v, v, v}, {sA0, sA1, sA2, 1}), arena,
                       s)))
        break;
      // A[p][x][y][v + l] = t2[p][l][x][y]
      if ((rc = axpby_perm("plxy->pxyl", 1.0, Tensor(t2, {o, o, v, v}), 0.0,
                           Tensor(A + v, {o, v, v, o}, {sA0, sA1, sA2, 1}), s)))
        break;
      // J[r][q][z][l] = (zr|ql); Bt[r][q][z][d] = t2[r][q][z][d], Bt[r][q][z][v + l] = -J[r][q][z][l]
      if ((rc = einsum("Qzr,Qql->rqzl", 1.0, Bvo, Boo, 0.0, Tensor(J, {o, o, v, o}), arena, s))) break;
      if ((rc = axpby_perm("rqzd->rqzd", 1.0, Tensor(t2, {o, o, v, v}), 0.0,
                           Tensor(Bt, {o, o, v, v}, {sB0, sB1, sB2, 1}), s)))
        break;
      if ((rc = axpby_perm("rqzl->rqzl", -1.0, Tensor(J, {o, o, v, o}), 0.0,
                           Tensor(Bt + v, {o, o, v, o}, {sB0, sB1, sB2, 1}), s)))
        break;
      // K[i][a][j][b] = (ia|jb)
      if ((rc = einsum("Qia,Qjb->iajb", 1.0, Bov, Bov, 0.0, Tensor(K, {o, v, o, v}), arena, s))) break;
      long tix = 0;
      for (int i = 0; i < o && rc == RI_OK; ++i)
        for (int j = i; j < o && rc == RI_OK; ++j)
          for (int k = j; k < o && rc == RI_OK; ++k, ++tix) {
            // term of permutation m: (p, q, r) = the triplet and (x, y, z) = (a, b, c), both
            // permuted by m; its natural layout Y_m[x][y][z]
            const int x3[3] = {i, j, k};
            for (int m = 0; m < 6 && rc == RI_OK; ++m) {
              const int pp = x3[trip::perm_at(m, 0)], qq = x3[trip::perm_at(m, 1)], rr = x3[trip::perm_at(m, 2)];
              rc = einsum("xye,ze->xyz", 1.0, Tensor(A + pp * sA0, {v, v, vo}, {sA1, sA2, 1}),
                          Tensor(Bt + (static_cast<long>(rr) * o + qq) * sB1, {v, vo}, {sB2, 1}), 0.0,
                          Tensor(Y + m * v3, {v, v, v}), arena, s, precision);
            }
            if (rc) break;
            {
              ProfScope ps(s, "triples_assemble", 0.0, 8.0 * 8.0 * v3);
              trip::assemble_wv<<<static_cast<unsigned>(ntiles), 512, 0, s>>>(Y, K, t1, o, v, i, j, k, W, Vt);
              if ((rc = check_launch("triples_assemble"))) break;
            }
            {
              ProfScope ps(s, "triples_energy", 0.0, 16.0 * v3);
              const trip::Orders ord = trip::orders_of(i, j, k);
              trip::energy_tiles<<<static_cast<unsigned>(ntri), 512, 0, s>>>(W, Vt, sys->eps, o, v, ord, tl, part);
              trip::sum_parts<<<1, 256, 0, s>>>(part, ntri, et + tix);
              if ((rc = check_launch("triples_energy"))) break;
            }
          }
      if (rc) break;
      std::vector<double> h(ntrip);
      if ((rc = check_hip(hipMemcpyAsync(h.data(), et, ntrip * sizeof(double), hipMemcpyDeviceToHost, s),
                          "triples copy")))
        break;
      if ((rc = check_hip(hipStreamSynchronize(s), "triples sync"))) break;
      double e = 0.0;
      for (double x : h) e += x;
      if (!std::isfinite(e)) {
        set_error("ri_ccsd_triples: energy is not finite");
        rc = RI_E_NUMERIC;
        break;
      }
      *e_t = e;
    } while (false);
  }
  dev_free(buf, s);
  return rc;
}

int ri_ccsd_triples(const ri_system* sys, const double* t1, const double* t2, double* e_t, void* stream) {
  return ri_ccsd_triples_ex(sys, t1, t2, RI_PREC_FP64, e_t, stream);
}

}  // extern "C"
