// Perturbative triples energy E_(T) of closed-shell CCSD(T) (Sec. II.A), FP64.
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
// Per triplet: twelve GEMMs on the library's FP64 MFMA engine accumulate W [a][b][c]
// (each of the six terms of P is one v^4 and one v^3 o product, written through a
// permuted output view), a kernel forms V = W + the t1 terms, and a tiled kernel sums
// the energy in a fixed order.  Integrals G[i][a][b][d] = (bd|ai), J[k][j][c][l] =
// (ck|jl) and K[i][a][j][b] = (ia|jb) are built once from the RI factors.
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

// V[a][b][c] = W[a][b][c] + (jb|kc) t^a_i + (ia|kc) t^b_j + (ia|jb) t^c_k, c fastest
__global__ __launch_bounds__(256) void make_v(const double* __restrict__ W, const double* __restrict__ K,
                                              const double* __restrict__ t1, int o, int v, int i, int j, int k,
                                              double* __restrict__ V) {
  const long n = static_cast<long>(v) * v * v;
  const long x = static_cast<long>(blockIdx.x) * 256 + threadIdx.x;
  if (x >= n) return;
  const int c = static_cast<int>(x % v);
  const long ab = x / v;
  const int b = static_cast<int>(ab % v), a = static_cast<int>(ab / v);
  auto Kx = [&](int i1, int p1, int i2, int p2) { return K[((static_cast<long>(i1) * v + p1) * o + i2) * v + p2]; };
  V[x] = W[x] + Kx(j, b, k, c) * t1[i * v + a] + Kx(i, a, k, c) * t1[j * v + b] + Kx(i, a, j, b) * t1[k * v + c];
}

// Energy of one triplet over the orderings in `ord`, summed per 8^3 tile of (a, b, c)
// into part[tile].  Each block stages the six orientations of its tile triple of W
// and V in LDS (tile[p] holds W[Z_p0 + u][Z_p1 + w][Z_p2 + z] for Z = (A0, B0, C0)),
// so every permuted read is an LDS read.  grid nt^3 (nt = ceil(v/8)), block 512.
__global__ __launch_bounds__(512) void energy_tiles(const double* __restrict__ W, const double* __restrict__ V,
                                                    const double* __restrict__ eps, int o, int v, Orders ord,
                                                    double* __restrict__ part) {
  __shared__ double tw[6][TE][TE][TE];
  __shared__ double tv[6][TE][TE][TE];
  __shared__ double red[512];
  const int nt = (v + TE - 1) / TE;
  const long bid = blockIdx.x;
  const int Z0 = static_cast<int>(bid / (static_cast<long>(nt) * nt)) * TE;
  const int Z1 = static_cast<int>((bid / nt) % nt) * TE;
  const int Z2 = static_cast<int>(bid % nt) * TE;
  const int t = threadIdx.x, u = t >> 6, w = (t >> 3) & 7, z = t & 7;
  auto Zof = [&](int m) { return m == 0 ? Z0 : (m == 1 ? Z1 : Z2); };
  for (int p = 0; p < 6; ++p) {
    const int y0 = Zof(perm_at(p, 0)) + u, y1 = Zof(perm_at(p, 1)) + w, y2 = Zof(perm_at(p, 2)) + z;
    const bool in = y0 < v && y1 < v && y2 < v;
    const long at = (static_cast<long>(y0) * v + y1) * v + y2;
    tw[p][u][w][z] = in ? W[at] : 0.0;
    tv[p][u][w][z] = in ? V[at] : 0.0;
  }
  __syncthreads();
  const int a = Z0 + u, b = Z1 + w, c = Z2 + z;
  double acc = 0.0;
  if (a < v && b < v && c < v) {
    auto xl = [&](int m) { return m == 0 ? u : (m == 1 ? w : z); };  // local coordinate of a, b or c
    auto rw = [&](int p) { return tw[p][xl(perm_at(p, 0))][xl(perm_at(p, 1))][xl(perm_at(p, 2))]; };
    auto rv = [&](int p) { return tv[p][xl(perm_at(p, 0))][xl(perm_at(p, 1))][xl(perm_at(p, 2))]; };
    const double evir = eps[o + a] + eps[o + b] + eps[o + c];
#pragma unroll
    for (int q = 0; q < 6; ++q) {
      if (q >= ord.n) break;
      const Order& r = ord.t[q];
      const double d = eps[r.ip] + eps[r.jp] + eps[r.kp] - evir;
      acc += (4.0 * rw(r.r1) + rw(r.r2) + rw(r.r3)) * (rv(r.r1) - rv(r.r4)) / (3.0 * d);
    }
  }
  red[t] = acc;
  __syncthreads();
  for (int s = 256; s > 0; s >>= 1) {
    if (t < s) red[t] += red[t + s];
    __syncthreads();
  }
  if (t == 0) part[bid] = red[0];
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

// index of the permutation with elements (e0, e1, e2)
inline int perm_index(int e0, int e1, int e2) {
  for (int p = 0; p < 6; ++p)
    if (perm_at(p, 0) == e0 && perm_at(p, 1) == e1 && perm_at(p, 2) == e2) return p;
  return -1;
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
    r.r1 = perm_index(inv[0], inv[1], inv[2]);
    r.r2 = perm_index((inv[0] + 1) % 3, (inv[1] + 1) % 3, (inv[2] + 1) % 3);
    r.r3 = perm_index((inv[0] + 2) % 3, (inv[1] + 2) % 3, (inv[2] + 2) % 3);
    r.r4 = perm_index(2 - inv[0], 2 - inv[1], 2 - inv[2]);
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
  return trip * 6.0 * (2.0 * v3 * v + 2.0 * v3 * o);
}

int ri_ccsd_triples(const ri_system* sys, const double* t1, const double* t2, double* e_t, void* stream) {
  clear_error();
  RI_TRY(cc::check_system(sys, "ri_ccsd_triples"));
  if (!t1 || !t2 || !e_t) {
    set_error("ri_ccsd_triples: null pointer argument");
    return RI_E_ARG;
  }
  hipStream_t s = static_cast<hipStream_t>(stream);
  const int o = sys->o, v = sys->v, Q = sys->naux, n = o + v;
  const long nn = static_cast<long>(n) * n, vv = static_cast<long>(v) * v, v3 = vv * v;
  const int nt = (v + trip::TE - 1) / trip::TE;
  const long ntiles = static_cast<long>(nt) * nt * nt;
  const long ntrip = static_cast<long>(o) * (o + 1) * (o + 2) / 6;
  // G [o][v][v][v], J [o][o][v][o], K [o][v][o][v], W and V [v][v][v], tile partials, triplet sums
  const size_t nG = static_cast<size_t>(o) * v3, nJ = static_cast<size_t>(o) * o * v * o,
               nK = static_cast<size_t>(o) * v * o * v;
  const size_t total = nG + nJ + nK + 2 * static_cast<size_t>(v3) + ntiles + ntrip;
  void* buf = nullptr;
  RI_TRY(dev_alloc(&buf, total * sizeof(double), s));
  double* G = static_cast<double*>(buf);
  double* J = G + nG;
  double* K = J + nJ;
  double* W = K + nK;
  double* Vt = W + v3;
  double* part = Vt + v3;
  double* et = part + ntiles;
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
    do {
      // G[i][a][b][d] = (bd|ai), J[k][j][c][l] = (ck|jl), K[i][a][j][b] = (ia|jb)
      if ((rc = einsum("Qbd,Qai->iabd", 1.0, Bvv, Bvo, 0.0, Tensor(G, {o, v, v, v}), arena, s))) break;
      if ((rc = einsum("Qck,Qjl->kjcl", 1.0, Bvo, Boo, 0.0, Tensor(J, {o, o, v, o}), arena, s))) break;
      if ((rc = einsum("Qia,Qjb->iajb", 1.0, Bov, Bov, 0.0, Tensor(K, {o, v, o, v}), arena, s))) break;
      const Tensor Wt(W, {v, v, v});
      auto Gp = [&](int p) { return Tensor(G + p * v3, {v, v, v}); };
      auto T2 = [&](int r, int q) { return Tensor(t2 + (static_cast<long>(r) * o + q) * vv, {v, v}); };
      auto Jrq = [&](int r, int q) { return Tensor(J + (static_cast<long>(r) * o + q) * v * o, {v, o}); };
      auto T2p = [&](int p) { return Tensor(t2 + static_cast<long>(p) * o * vv, {o, v, v}); };
      long tix = 0;
      for (int i = 0; i < o && rc == RI_OK; ++i)
        for (int j = i; j < o && rc == RI_OK; ++j)
          for (int k = j; k < o && rc == RI_OK; ++k, ++tix) {
            // the six terms (p, q, r; x, y, z) of P, each
            //   W[a][b][c] += sum_d G[p][x][y][d] t2[r][q][z][d] - sum_l J[r][q][z][l] t2[p][l][x][y]
            struct Term {
              int p, q, r;
              const char* first;
              const char* second;
            };
            const Term terms[6] = {
                {i, j, k, "abd,cd->abc", "lab,cl->abc"}, {i, k, j, "acd,bd->abc", "lac,bl->abc"},
                {k, i, j, "cad,bd->abc", "lca,bl->abc"}, {k, j, i, "cbd,ad->abc", "lcb,al->abc"},
                {j, k, i, "bcd,ad->abc", "lbc,al->abc"}, {j, i, k, "bad,cd->abc", "lba,cl->abc"},
            };
            for (int m = 0; m < 6 && rc == RI_OK; ++m) {
              const Term& tm = terms[m];
              rc = einsum(tm.first, 1.0, Gp(tm.p), T2(tm.r, tm.q), m == 0 ? 0.0 : 1.0, Wt, arena, s);
              if (rc == RI_OK) rc = einsum(tm.second, -1.0, T2p(tm.p), Jrq(tm.r, tm.q), 1.0, Wt, arena, s);
            }
            if (rc) break;
            {
              ProfScope ps(s, "triples_make_v", 0.0, 24.0 * v3);
              trip::make_v<<<static_cast<unsigned>((v3 + 255) / 256), 256, 0, s>>>(W, K, t1, o, v, i, j, k, Vt);
              if ((rc = check_launch("triples_make_v"))) break;
            }
            {
              ProfScope ps(s, "triples_energy", 0.0, 96.0 * v3);
              const trip::Orders ord = trip::orders_of(i, j, k);
              trip::energy_tiles<<<static_cast<unsigned>(ntiles), 512, 0, s>>>(W, Vt, sys->eps, o, v, ord, part);
              trip::sum_parts<<<1, 256, 0, s>>>(part, ntiles, et + tix);
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

}  // extern "C"
