// Closed-shell RI-CCSD driver on the GPU: MP2 guess -> Jacobi update -> DIIS -> E_corr
// (Sec. II.A: eqs. ccsd-1..3, the Jacobi solver and the energy expression; DIIS as
// in Sec. II and II.B).
//
// The residual is the T1-similarity-transformed closed-shell form: the RI factors
// are dressed as B~ = (1 - t) B (1 + t) (t[a][k] = t^a_k), which folds every T1
// contribution into the integrals, and
//
//   Omega2_{aibj} = (ai|bj)~ + A2 + B2 + P^{ab}_{ij} (C2 + D2 + E2)
//   A2 = sum_cd (a~c|b~d) t^{cd}_{ij}                            (the ladder, eq. pp-Ladder-0)
//   B2 = sum_kl t^{ab}_{kl} [(ki|lj)~ + sum_cd t^{cd}_{ij} (kc|ld)]
//   C2 = -1/2 sum_ck t^{bc}_{kj} Z_{kiac} - sum_ck t^{bc}_{ki} Z_{kjac},
//        Z_{kiac} = (ki|ac)~ - 1/2 sum_dl t^{ad}_{li} (kd|lc)
//   D2 = 1/2 sum_ck u^{bc}_{jk} [L~_{aikc} + 1/2 sum_dl u^{ad}_{il} L_{ldkc}]
//   E2 = sum_c t^{ac}_{ij} [F~_bc - sum_dkl u^{bd}_{kl} (ld|kc)]
//        - sum_k t^{ab}_{ik} [F~_kj + sum_cdl u^{cd}_{lj} (kd|lc)]
//   Omega1_{ai} = sum_ckd u^{cd}_{ki} (ad|kc)~ - sum_ckl u^{ac}_{kl} (ki|lc)~
//                 + sum_ck u^{ac}_{ik} F~_kc + F~_ai
//
// with u^{ab}_{ij} = 2 t^{ab}_{ij} - t^{ab}_{ji}, L_{pqrs} = 2(pq|rs) - (ps|rq) and the
// dressed Fock matrix F~ = h~ + sum_k [2 (pq|kk)~ - (pk|kq)~].  The paper does not
// print its working equations; this form is checked against a determinant-space
// evaluation of eqs. ccsd-1..3.  For canonical orbitals f = diag(eps), so the bare
// one-electron matrix is h = diag(eps) - sum_k [2(pq|kk) - (pk|kq)].
#include <chrono>
#include <cmath>
#include <vector>

#include "gemm.h"

namespace ri {
namespace cc {

// ------------------------------------------------------------------ kernels
__global__ void fill_kernel(double* x, long n, double val) {
  const long i = static_cast<long>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i < n) x[i] = val;
}

__global__ void diag_kernel(double* h, const double* eps, int n) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n * n) h[i] = (i / n == i % n) ? eps[i / n] : 0.0;
}

// t2[i][j][a][b] = (ia|jb) / (e_i + e_j - e_a - e_b), t1 = 0
__global__ void mp2_kernel(const double* __restrict__ gov, const double* __restrict__ eps, int o, int v,
                           double* t1, double* t2) {
  const long idx = static_cast<long>(blockIdx.x) * blockDim.x + threadIdx.x;
  const long vv = static_cast<long>(v) * v, total = static_cast<long>(o) * o * vv;
  if (idx < static_cast<long>(o) * v) t1[idx] = 0.0;
  if (idx >= total) return;
  const int b = idx % v, a = (idx / v) % v;
  const long ij = idx / vv;
  const int j = ij % o, i = ij / o;
  const double g = gov[((static_cast<long>(i) * v + a) * o + j) * v + b];
  t2[idx] = g / (eps[i] + eps[j] - eps[o + a] - eps[o + b]);
}

// vec = t + Omega / D, err = Omega / D over the concatenated [t1 | t2] vector
__global__ void jacobi_kernel(const double* __restrict__ t, const double* __restrict__ om,
                              const double* __restrict__ eps, int o, int v, double* vec, double* err) {
  const long idx = static_cast<long>(blockIdx.x) * blockDim.x + threadIdx.x;
  const long nov = static_cast<long>(o) * v, vv = static_cast<long>(v) * v;
  const long total = nov + static_cast<long>(o) * o * vv;
  if (idx >= total) return;
  double d;
  if (idx < nov) {
    const int a = idx % v, i = idx / v;
    d = eps[i] - eps[o + a];
  } else {
    const long r = idx - nov;
    const int b = r % v, a = (r / v) % v;
    const long ij = r / vv;
    const int j = ij % o, i = ij / o;
    d = eps[i] + eps[j] - eps[o + a] - eps[o + b];
  }
  const double e = om[idx] / d;
  err[idx] = e;
  vec[idx] = t[idx] + e;
}

struct Coefs {
  double c[16];
  int slot[16];
  int m;
};

// t = sum_k c_k vec_{slot_k}; history slots are `stride` doubles apart
__global__ void combine_kernel(Coefs cf, const double* __restrict__ hist, long stride, long n, double* t) {
  const long idx = static_cast<long>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (idx >= n) return;
  double acc = 0.0;
  for (int k = 0; k < cf.m; ++k) acc += cf.c[k] * hist[cf.slot[k] * stride + idx];
  t[idx] = acc;
}

// t2 <- (t2 + t2^T) / 2 with t2^T[i][j][a][b] = t2[j][i][b][a]; each pair handled once
__global__ void symmetrize_kernel(double* t2, int o, int v) {
  const long idx = static_cast<long>(blockIdx.x) * blockDim.x + threadIdx.x;
  const long vv = static_cast<long>(v) * v, total = static_cast<long>(o) * o * vv;
  if (idx >= total) return;
  const int b = idx % v, a = (idx / v) % v;
  const long ij = idx / vv;
  const int j = ij % o, i = ij / o;
  const long tidx = (static_cast<long>(j) * o + i) * vv + static_cast<long>(b) * v + a;
  if (tidx <= idx) return;
  const double m = 0.5 * (t2[idx] + t2[tidx]);
  t2[idx] = m;
  t2[tidx] = m;
}

constexpr int EB = 1024;

// partials of sum_ijab (2 (ia|jb) - (ib|ja)) (t^{ab}_{ij} + t^a_i t^b_j)
__global__ __launch_bounds__(256) void energy_stage1(const double* __restrict__ gov, const double* __restrict__ t1,
                                                     const double* __restrict__ t2, int o, int v, double* part) {
  __shared__ double sh[256];
  const long vv = static_cast<long>(v) * v, n = static_cast<long>(o) * o * vv;
  const long chunk = (n + EB - 1) / EB;
  const long lo = static_cast<long>(blockIdx.x) * chunk, hi = n < lo + chunk ? n : lo + chunk;
  double acc = 0.0;
  for (long idx = lo + threadIdx.x; idx < hi; idx += 256) {
    const int b = idx % v, a = (idx / v) % v;
    const long ij = idx / vv;
    const int j = ij % o, i = ij / o;
    const double g1 = gov[((static_cast<long>(i) * v + a) * o + j) * v + b];
    const double g2 = gov[((static_cast<long>(i) * v + b) * o + j) * v + a];
    const double tau = t2[idx] + t1[static_cast<long>(i) * v + a] * t1[static_cast<long>(j) * v + b];
    acc += (2.0 * g1 - g2) * tau;
  }
  sh[threadIdx.x] = acc;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if (threadIdx.x < w) sh[threadIdx.x] += sh[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) part[blockIdx.x] = sh[0];
}

__global__ __launch_bounds__(256) void energy_stage2(const double* __restrict__ part, double* res) {
  __shared__ double sh[256];
  double acc = 0.0;
  for (int i = threadIdx.x; i < EB; i += 256) acc += part[i];
  sh[threadIdx.x] = acc;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if (threadIdx.x < w) sh[threadIdx.x] += sh[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) *res = sh[0];
}

inline unsigned nblk(long n) { return static_cast<unsigned>((n + 255) / 256); }

// ------------------------------------------------------------------ context
struct Ctx {
  int o, v, Q, n;
  long nov, noovv, nt;
  hipStream_t s;
  const double* B;
  const double* eps;
  void* block = nullptr;
  double *h = nullptr, *gov = nullptr, *Lov = nullptr, *Bd = nullptr, *F = nullptr, *U = nullptr, *X = nullptr,
         *G = nullptr, *Z = nullptr, *Yb = nullptr, *W = nullptr, *Gv = nullptr, *Go = nullptr, *Xq = nullptr,
         *Gk = nullptr, *xq = nullptr, *ones = nullptr, *part = nullptr, *scal = nullptr, *tvec = nullptr,
         *om = nullptr, *hist = nullptr;
  int m = 0;  // DIIS slots
  GemmArena arena;
  hipEvent_t ev[4] = {nullptr, nullptr, nullptr, nullptr};

  Ctx(const ri_system* sys, hipStream_t st)
      : o(sys->o), v(sys->v), Q(sys->naux), n(sys->o + sys->v), s(st), B(sys->B), eps(sys->eps) {
    nov = static_cast<long>(o) * v;
    noovv = nov * nov;
    nt = nov + noovv;
    arena.s = st;
  }
  ~Ctx() {
    if (block) dev_free(block, s);
    for (auto e : ev)
      if (e) (void)hipEventDestroy(e);
  }

  // level 0: energy / MP2 only; 1: residual; 2: full iteration with `slots` DIIS vectors
  int alloc(int level, int slots) {
    m = slots;
    const long vv = static_cast<long>(v) * v, oo = static_cast<long>(o) * o, nn = static_cast<long>(n) * n;
    std::vector<std::pair<double**, long>> want = {{&gov, noovv}, {&part, EB + 1024}, {&scal, 64}};
    if (level >= 1) {
      want.insert(want.end(), {{&h, nn}, {&Lov, noovv}, {&Bd, static_cast<long>(Q) * nn}, {&F, nn}, {&U, noovv},
                               {&X, noovv}, {&G, noovv}, {&Z, noovv}, {&Yb, noovv}, {&W, oo * oo}, {&Gv, vv},
                               {&Go, oo}, {&Xq, static_cast<long>(Q) * nov}, {&Gk, oo * nov}, {&xq, Q},
                               {&ones, o}});
    }
    if (level >= 2) want.insert(want.end(), {{&tvec, nt}, {&om, nt}, {&hist, 2L * slots * nt}});
    size_t bytes = 0;
    for (auto& w : want) bytes = round_up(bytes, 256) + w.second * sizeof(double);
    RI_TRY(dev_alloc(&block, bytes, s));
    Carve cv(block, bytes);
    for (auto& w : want) *w.first = cv.take<double>(w.second);
    if (ones) {
      fill_kernel<<<nblk(o), 256, 0, s>>>(ones, o, 1.0);
      RI_TRY(check_launch("fill_kernel"));
    }
    for (auto& e : ev) RI_HIP(hipEventCreate(&e));
    return RI_OK;
  }

  // views of a [Q][n][n] factor array
  Tensor oo_(const double* p) const { return Tensor(p, {Q, o, o}, {static_cast<long>(n) * n, n, 1}); }
  Tensor ov_(const double* p) const { return Tensor(p + o, {Q, o, v}, {static_cast<long>(n) * n, n, 1}); }
  Tensor vo_(const double* p) const { return Tensor(p + static_cast<long>(o) * n, {Q, v, o}, {static_cast<long>(n) * n, n, 1}); }
  Tensor vv_(const double* p) const {
    return Tensor(p + static_cast<long>(o) * n + o, {Q, v, v}, {static_cast<long>(n) * n, n, 1});
  }
  Tensor t4(const double* p, long a, long b, long c, long d) const { return Tensor(p, {a, b, c, d}); }

  // arithmetic of the large non-ladder contractions (RI_PREC_FP64 or RI_PREC_FP32)
  int other_prec = RI_PREC_FP64;
  int es(const char* spec, double al, const Tensor& A, const Tensor& Bt, double be, const Tensor& C) {
    return einsum(spec, al, A, Bt, be, C, arena, s, other_prec);
  }

  // (kc|ld) as gov[k][c][l][d]
  int build_gov() { return es("Qkc,Qld->kcld", 1.0, ov_(B), ov_(B), 0.0, t4(gov, o, v, o, v)); }

  // h, L
  int setup() {
    RI_TRY(build_gov());
    const long nn = static_cast<long>(n) * n;
    diag_kernel<<<nblk(nn), 256, 0, s>>>(h, eps, n);
    RI_TRY(check_launch("diag_kernel"));
    Tensor diagB(B, {Q, o}, {nn, n + 1});
    RI_TRY(es("Qk,k->Q", 1.0, diagB, Tensor(ones, {o}), 0.0, Tensor(xq, {Q})));
    RI_TRY(es("Qpq,Q->pq", -2.0, Tensor(B, {Q, n, n}), Tensor(xq, {Q}), 1.0, Tensor(h, {n, n})));
    RI_TRY(es("Qpk,Qkq->pq", 1.0, Tensor(B, {Q, n, o}, {nn, n, 1}), Tensor(B, {Q, o, n}, {nn, n, 1}), 1.0,
              Tensor(h, {n, n})));
    RI_TRY(axpby_perm("ldkc->ldkc", 2.0, t4(gov, o, v, o, v), 0.0, t4(Lov, o, v, o, v), s));
    RI_TRY(axpby_perm("lckd->ldkc", -1.0, t4(gov, o, v, o, v), 1.0, t4(Lov, o, v, o, v), s));
    return RI_OK;
  }

  // B~ and F~ for the current t1
  int dress(const double* t1) {
    const long nn = static_cast<long>(n) * n;
    Tensor T1(t1, {o, v});
    RI_HIP(hipMemcpyAsync(Bd, B, sizeof(double) * Q * nn, hipMemcpyDeviceToDevice, s));
    RI_TRY(es("Qpc,ic->Qpi", 1.0, Tensor(B + o, {Q, n, v}, {nn, n, 1}), T1, 1.0, Tensor(Bd, {Q, n, o}, {nn, n, 1})));
    RI_TRY(es("ka,Qkq->Qaq", -1.0, T1, Tensor(Bd, {Q, o, n}, {nn, n, 1}), 1.0,
              Tensor(Bd + static_cast<long>(o) * n, {Q, v, n}, {nn, n, 1})));
    RI_HIP(hipMemcpyAsync(F, h, sizeof(double) * nn, hipMemcpyDeviceToDevice, s));
    RI_TRY(es("pc,ic->pi", 1.0, Tensor(h + o, {n, v}, {n, 1}), T1, 1.0, Tensor(F, {n, o}, {n, 1})));
    RI_TRY(es("ka,kq->aq", -1.0, T1, Tensor(F, {o, n}, {n, 1}), 1.0, Tensor(F + static_cast<long>(o) * n, {v, n}, {n, 1})));
    Tensor diagBd(Bd, {Q, o}, {nn, n + 1});
    RI_TRY(es("Qk,k->Q", 1.0, diagBd, Tensor(ones, {o}), 0.0, Tensor(xq, {Q})));
    RI_TRY(es("Qpq,Q->pq", 2.0, Tensor(Bd, {Q, n, n}), Tensor(xq, {Q}), 1.0, Tensor(F, {n, n})));
    RI_TRY(es("Qpk,Qkq->pq", -1.0, Tensor(Bd, {Q, n, o}, {nn, n, 1}), Tensor(Bd, {Q, o, n}, {nn, n, 1}), 1.0,
              Tensor(F, {n, n})));
    return RI_OK;
  }

  // Omega1 [o][v], Omega2 [o][o][v][v] for (t1, t2); ladder time (ms) returned in *ms_ppl
  int residual(const double* t1, const double* t2, double* om1, double* om2, int prec, float* ms_ppl) {
    RI_TRY(dress(t1));
    const Tensor T = t4(t2, o, o, v, v), Ut = t4(U, o, o, v, v), Xt = t4(X, o, o, v, v);
    const Tensor Om2 = t4(om2, o, o, v, v), Gt = t4(G, o, o, v, v), Zt = t4(Z, o, o, v, v);
    const Tensor Ybt = t4(Yb, v, o, o, v), Wt = t4(W, o, o, o, o), govt = t4(gov, o, v, o, v);
    const Tensor Lovt = t4(Lov, o, v, o, v);
    const Tensor Boo = oo_(Bd), Bov = ov_(Bd), Bvo = vo_(Bd), Bvv = vv_(Bd);
    RI_TRY(axpby_perm("ijab->ijab", 2.0, T, 0.0, Ut, s));
    RI_TRY(axpby_perm("jiab->ijab", -1.0, T, 1.0, Ut, s));
    // (ai|bj)~
    RI_TRY(es("Qai,Qbj->ijab", 1.0, Bvo, Bvo, 0.0, Om2));
    // A2: the particle-particle ladder on the dressed factors
    RI_HIP(hipEventRecord(ev[0], s));
    RI_TRY(ppl_strided(Bd + static_cast<long>(o) * n + o, static_cast<long>(n) * n, n, t2, o, v, Q, om2, prec, s));
    RI_HIP(hipEventRecord(ev[1], s));
    // B2
    RI_TRY(es("Qki,Qlj->kilj", 1.0, Boo, Boo, 0.0, Wt));
    RI_TRY(es("kcld,ijcd->kilj", 1.0, govt, T, 1.0, Wt));
    RI_TRY(es("klab,kilj->ijab", 1.0, T, Wt, 1.0, Om2));
    // C2
    RI_TRY(es("Qki,Qac->kiac", 1.0, Boo, Bvv, 0.0, Gt));
    RI_TRY(axpby_perm("kiac->kiac", 1.0, Gt, 0.0, Zt, s));
    RI_TRY(es("liad,kdlc->kiac", -0.5, T, govt, 1.0, Zt));
    RI_TRY(es("kjbc,kiac->ijab", -0.5, T, Zt, 0.0, Xt));
    RI_TRY(es("kibc,kjac->ijab", -1.0, T, Zt, 1.0, Xt));
    // D2
    RI_TRY(es("Qai,Qkc->aikc", 2.0, Bvo, Bov, 0.0, Ybt));
    RI_TRY(axpby_perm("kiac->aikc", -1.0, Gt, 1.0, Ybt, s));
    RI_TRY(es("ilad,ldkc->aikc", 0.5, Ut, Lovt, 1.0, Ybt));
    RI_TRY(es("jkbc,aikc->ijab", 0.5, Ut, Ybt, 1.0, Xt));
    // E2
    const Tensor Fvv(F + static_cast<long>(o) * n + o, {v, v}, {n, 1}), Foo(F, {o, o}, {n, 1});
    RI_TRY(axpby_perm("bc->bc", 1.0, Fvv, 0.0, Tensor(Gv, {v, v}), s));
    RI_TRY(es("klbd,ldkc->bc", -1.0, Ut, govt, 1.0, Tensor(Gv, {v, v})));
    RI_TRY(axpby_perm("kj->kj", 1.0, Foo, 0.0, Tensor(Go, {o, o}), s));
    RI_TRY(es("ljcd,kdlc->kj", 1.0, Ut, govt, 1.0, Tensor(Go, {o, o})));
    RI_TRY(es("ijac,bc->ijab", 1.0, T, Tensor(Gv, {v, v}), 1.0, Xt));
    RI_TRY(es("ikab,kj->ijab", -1.0, T, Tensor(Go, {o, o}), 1.0, Xt));
    // P^{ab}_{ij}
    RI_TRY(axpby_perm("ijab->ijab", 1.0, Xt, 1.0, Om2, s));
    RI_TRY(axpby_perm("jiba->ijab", 1.0, Xt, 1.0, Om2, s));
    // singles
    const Tensor Om1(om1, {o, v});
    RI_TRY(es("Qkc,kicd->Qid", 1.0, Bov, Ut, 0.0, Tensor(Xq, {Q, o, v})));
    RI_TRY(es("Qid,Qad->ia", 1.0, Tensor(Xq, {Q, o, v}), Bvv, 0.0, Om1));
    RI_TRY(es("Qki,Qlc->kilc", 1.0, Boo, Bov, 0.0, Tensor(Gk, {o, o, o, v})));
    RI_TRY(es("kilc,klac->ia", -1.0, Tensor(Gk, {o, o, o, v}), Ut, 1.0, Om1));
    RI_TRY(es("ikac,kc->ia", 1.0, Ut, Tensor(F + o, {o, v}, {n, 1}), 1.0, Om1));
    RI_TRY(axpby_perm("ai->ia", 1.0, Tensor(F + static_cast<long>(o) * n, {v, o}, {n, 1}), 1.0, Om1, s));
    if (ms_ppl) {
      RI_HIP(hipEventSynchronize(ev[1]));
      RI_HIP(hipEventElapsedTime(ms_ppl, ev[0], ev[1]));
    }
    return RI_OK;
  }

  int energy(const double* t1, const double* t2, double* res) {
    energy_stage1<<<EB, 256, 0, s>>>(gov, t1, t2, o, v, part);
    energy_stage2<<<1, 256, 0, s>>>(part, res);
    return check_launch("energy");
  }

  int mp2(double* t1, double* t2) {
    mp2_kernel<<<nblk(std::max(noovv, nov)), 256, 0, s>>>(gov, eps, o, v, t1, t2);
    return check_launch("mp2_kernel");
  }

  int read_scalars(double* host, int count) {
    RI_HIP(hipMemcpyAsync(host, scal, sizeof(double) * count, hipMemcpyDeviceToHost, s));
    RI_HIP(hipStreamSynchronize(s));
    return RI_OK;
  }
};

// Pulay solve on the host: Gram block scaled by its largest diagonal element,
// Gaussian elimination with partial pivoting; false when (near) singular.
bool diis_solve(const std::vector<std::vector<double>>& gram, std::vector<double>& c) {
  const int m = static_cast<int>(gram.size());
  double sc = 0.0;
  for (int k = 0; k < m; ++k) sc = std::max(sc, std::fabs(gram[k][k]));
  if (!(sc > 0.0) || !std::isfinite(sc)) return false;
  const int N = m + 1;
  std::vector<double> A(N * N, 0.0), b(N, 0.0);
  for (int k = 0; k < m; ++k)
    for (int l = 0; l < m; ++l) A[k * N + l] = gram[k][l] / sc;
  for (int k = 0; k < m; ++k) A[k * N + m] = A[m * N + k] = 1.0;
  b[m] = 1.0;
  double amax = 0.0;
  for (double x : A) amax = std::max(amax, std::fabs(x));
  for (int col = 0; col < N; ++col) {
    int piv = col;
    for (int r = col + 1; r < N; ++r)
      if (std::fabs(A[r * N + col]) > std::fabs(A[piv * N + col])) piv = r;
    if (std::fabs(A[piv * N + col]) <= 1e-14 * amax) return false;
    if (piv != col) {
      for (int x = 0; x < N; ++x) std::swap(A[col * N + x], A[piv * N + x]);
      std::swap(b[col], b[piv]);
    }
    for (int r = col + 1; r < N; ++r) {
      const double f = A[r * N + col] / A[col * N + col];
      for (int x = col; x < N; ++x) A[r * N + x] -= f * A[col * N + x];
      b[r] -= f * b[col];
    }
  }
  std::vector<double> x(N, 0.0);
  for (int r = N - 1; r >= 0; --r) {
    double acc = b[r];
    for (int q = r + 1; q < N; ++q) acc -= A[r * N + q] * x[q];
    x[r] = acc / A[r * N + r];
  }
  c.assign(x.begin(), x.begin() + m);
  for (double y : c)
    if (!std::isfinite(y)) return false;
  return true;
}

int check_system(const ri_system* sys, const char* where) {
  if (!sys || !sys->B || !sys->eps || sys->o <= 0 || sys->v <= 0 || sys->naux <= 0) {
    set_error("%s: invalid system", where);
    return RI_E_ARG;
  }
  if (sys->o > 4096 || sys->v > 65536 || sys->naux > (1 << 24)) {
    set_error("%s: sizes out of range", where);
    return RI_E_ARG;
  }
  return RI_OK;
}

// MP2 guess with the (ia|jb) integrals kept: gov [o][v][o][v], t1 [o][v], t2 [o][o][v][v]
int ovov_integrals(const ri_system* sys, double* gov, hipStream_t s) {
  RI_TRY(check_system(sys, "ovov"));
  Ctx c(sys, s);
  return einsum("Qkc,Qld->kcld", 1.0, c.ov_(sys->B), c.ov_(sys->B), 0.0, c.t4(gov, c.o, c.v, c.o, c.v), c.arena, s);
}

int mp2_with_integrals(const ri_system* sys, double* gov, double* t1, double* t2, hipStream_t s) {
  RI_TRY(ovov_integrals(sys, gov, s));
  Ctx c(sys, s);
  mp2_kernel<<<nblk(std::max(c.noovv, c.nov)), 256, 0, s>>>(gov, sys->eps, c.o, c.v, t1, t2);
  return check_launch("mp2_kernel");
}

int symmetrize_pairs(double* t2, int o, int v, hipStream_t s) {
  symmetrize_kernel<<<nblk(static_cast<long>(o) * o * v * v), 256, 0, s>>>(t2, o, v);
  return check_launch("symmetrize_kernel");
}

}  // namespace cc
}  // namespace ri

using namespace ri;

extern "C" {

void ri_ccsd_default_opts(ri_ccsd_opts* op) {
  if (!op) return;
  op->max_iter = 100;
  op->tol_residual = 1e-10;
  op->tol_energy = 1e-10;
  op->diis_size = 6;
  op->diis_start = 2;
  op->ppl_precision = RI_PREC_FP64;
  op->guess = RI_GUESS_MP2;
  op->verbose = 0;
  op->polish_residual = 0.0;
  op->check_fp64 = 0;
  op->mlp = nullptr;
  op->polish_precision = RI_PREC_FP64;
  op->other_precision = RI_PREC_FP64;
}

int ri_mp2_guess(const ri_system* sys, double* t1, double* t2, double* e_mp2, void* stream) {
  clear_error();
  RI_TRY(cc::check_system(sys, "ri_mp2_guess"));
  if (!t1 || !t2) {
    set_error("ri_mp2_guess: null amplitude pointer");
    return RI_E_ARG;
  }
  cc::Ctx c(sys, static_cast<hipStream_t>(stream));
  RI_TRY(c.alloc(0, 0));
  RI_TRY(c.build_gov());
  RI_TRY(c.mp2(t1, t2));
  if (e_mp2) {
    RI_TRY(c.energy(t1, t2, c.scal));
    RI_TRY(c.read_scalars(e_mp2, 1));
  }
  return RI_OK;
}

int ri_ccsd_energy(const ri_system* sys, const double* t1, const double* t2, double* e_corr, void* stream) {
  clear_error();
  RI_TRY(cc::check_system(sys, "ri_ccsd_energy"));
  if (!t1 || !t2 || !e_corr) {
    set_error("ri_ccsd_energy: null pointer");
    return RI_E_ARG;
  }
  cc::Ctx c(sys, static_cast<hipStream_t>(stream));
  RI_TRY(c.alloc(0, 0));
  RI_TRY(c.build_gov());
  RI_TRY(c.energy(t1, t2, c.scal));
  return c.read_scalars(e_corr, 1);
}

int ri_ccsd_residual(const ri_system* sys, const double* t1, const double* t2, double* omega1, double* omega2,
                     int ppl_precision, void* stream) {
  clear_error();
  RI_TRY(cc::check_system(sys, "ri_ccsd_residual"));
  if (!t1 || !t2 || !omega1 || !omega2) {
    set_error("ri_ccsd_residual: null pointer");
    return RI_E_ARG;
  }
  const size_t n2 = static_cast<size_t>(sys->o) * sys->o * sys->v * sys->v * 8;
  if (overlaps(omega2, n2, t2, n2) || overlaps(omega1, static_cast<size_t>(sys->o) * sys->v * 8, t1,
                                                   static_cast<size_t>(sys->o) * sys->v * 8)) {
    set_error("ri_ccsd_residual: outputs overlap the amplitudes");
    return RI_E_ALIAS;
  }
  cc::Ctx c(sys, static_cast<hipStream_t>(stream));
  RI_TRY(c.alloc(1, 0));
  RI_TRY(c.setup());
  return c.residual(t1, t2, omega1, omega2, ppl_precision, nullptr);
}

int ri_ccsd_iterate(const ri_system* sys, double* t1, double* t2, const ri_ccsd_opts* opts, ri_ccsd_report* rep,
                    void* stream) {
  using clk = std::chrono::steady_clock;
  const auto t_start = clk::now();
  clear_error();
  RI_TRY(cc::check_system(sys, "ri_ccsd_iterate"));
  if (!t1 || !t2) {
    set_error("ri_ccsd_iterate: null amplitude pointer");
    return RI_E_ARG;
  }
  ri_ccsd_opts op;
  if (opts) op = *opts;
  else ri_ccsd_default_opts(&op);
  if (op.max_iter < 0 || op.diis_size > 16 || op.guess < RI_GUESS_MP2 || op.guess > RI_GUESS_MLP ||
      !(op.polish_residual >= 0.0) || (op.guess == RI_GUESS_MLP && !op.mlp) ||
      (op.polish_precision != RI_PREC_FP64 && op.polish_precision != RI_PREC_FP32) ||
      (op.other_precision != RI_PREC_FP64 && op.other_precision != RI_PREC_FP32)) {
    set_error("ri_ccsd_iterate: invalid options (max_iter %d, diis_size %d, guess %d, polish %g, mlp %p)",
              op.max_iter, op.diis_size, op.guess, op.polish_residual, static_cast<void*>(op.mlp));
    return RI_E_ARG;
  }
  // reduced precision in the ladder or the other large contractions; the polish
  // moves the ladder to polish_precision and, for an FP64 polish, the others to FP64
  const bool mixed = op.ppl_precision != RI_PREC_FP64 || op.other_precision != RI_PREC_FP64;
  const int final_prec_p = op.polish_precision;
  const int final_other_p = op.polish_precision == RI_PREC_FP64 ? RI_PREC_FP64 : op.other_precision;
  const bool polish = mixed && op.polish_residual > 0.0 &&
                      (final_prec_p != op.ppl_precision || final_other_p != op.other_precision);
  const int final_prec = polish ? final_prec_p : op.ppl_precision;
  const int final_other = polish ? final_other_p : op.other_precision;
  const int slots = op.diis_size >= 2 ? op.diis_size : 1;
  hipStream_t s = static_cast<hipStream_t>(stream);
  cc::Ctx c(sys, s);
  RI_TRY(c.alloc(2, slots));
  RI_TRY(c.setup());
  const long nov = c.nov, nt = c.nt;
  double* tv1 = c.tvec;
  double* tv2 = c.tvec + nov;
  int mlp_rc = RI_OK;
  if (op.guess == RI_GUESS_MP2) {
    RI_TRY(c.mp2(tv1, tv2));
  } else if (op.guess == RI_GUESS_MLP) {
    mlp_rc = ri_mlp_guess(op.mlp, sys, tv1, tv2, stream);
  } else {
    RI_HIP(hipMemcpyAsync(tv1, t1, sizeof(double) * nov, hipMemcpyDeviceToDevice, s));
    RI_HIP(hipMemcpyAsync(tv2, t2, sizeof(double) * c.noovv, hipMemcpyDeviceToDevice, s));
    cc::symmetrize_kernel<<<cc::nblk(c.noovv), 256, 0, s>>>(tv2, c.o, c.v);
    RI_TRY(check_launch("symmetrize_kernel"));
  }
  c.other_prec = op.other_precision;
  double hostv[64];
  double e = NAN;
  if (mlp_rc == RI_OK) {
    RI_TRY(c.energy(tv1, tv2, c.scal));
    RI_TRY(c.read_scalars(hostv, 1));
    e = hostv[0];
  }
  // the MP2 guess is the learned guess's fallback: used when the network fails or
  // gives non-finite amplitudes (their energy is then non-finite)
  int guess_used = op.guess;
  if (op.guess == RI_GUESS_MLP && (mlp_rc != RI_OK || !std::isfinite(e))) {
    if (op.verbose) fprintf(stderr, "[ccsd] learned guess unusable (%s); starting from MP2\n", ri_status_str(mlp_rc));
    clear_error();
    RI_TRY(c.mp2(tv1, tv2));
    RI_TRY(c.energy(tv1, tv2, c.scal));
    RI_TRY(c.read_scalars(hostv, 1));
    e = hostv[0];
    guess_used = RI_GUESS_MP2;
  }
  const double e_mp2 = guess_used == RI_GUESS_MP2 ? e : NAN;
  const double sec_guess = std::chrono::duration<double>(clk::now() - t_start).count();
  double e_prev = NAN, rinf = INFINITY, rrms = INFINITY;
  int prec = op.ppl_precision, polish_it = -1;
  bool conv = false;
  int it = 0;
  double ms_ppl_total = 0.0;
  std::vector<std::vector<double>> gram;  // Gram matrix of the stored error vectors
  std::vector<int> order;                 // history slots, oldest first
  int next_slot = 0;
  int status = RI_OK;
  for (it = 0; it < op.max_iter; ++it) {
    float ms_ppl = 0.f;
    RI_TRY(c.residual(tv1, tv2, c.om, c.om + nov, prec, &ms_ppl));
    ms_ppl_total += ms_ppl;
    RI_TRY(max_abs(c.om, nt, c.part, c.scal, s));
    RI_TRY(dot(c.om, c.om, nt, c.part, c.scal + 1, s));
    RI_TRY(c.read_scalars(hostv, 2));
    rinf = hostv[0];
    rrms = std::sqrt(hostv[1] / static_cast<double>(nt));
    if (op.verbose)
      fprintf(stderr, "[ccsd] iter %3d  E = %.12f  |Omega|inf = %.3e  ladder %s %.1f ms\n", it, e, rinf,
              prec == RI_PREC_FP64 ? "fp64" : prec == RI_PREC_FP32 ? "fp32" : "bf16x3", ms_ppl);
    if (!std::isfinite(rinf) || !std::isfinite(e) || rinf > 1e8) {
      set_error("ri_ccsd_iterate: non-finite or divergent residual at iteration %d", it);
      status = RI_E_NUMERIC;
      break;
    }
    const bool on_final = prec == final_prec && c.other_prec == final_other;
    if (it > 0 && rinf <= op.tol_residual && std::fabs(e - e_prev) <= op.tol_energy && on_final) {
      conv = true;
      break;
    }
    // switch to the polish ladder for the remaining residuals (the step below still
    // uses this mixed residual)
    if (polish && !on_final && rinf <= op.polish_residual) {
      prec = final_prec;
      c.other_prec = final_other;
      polish_it = it + 1;
    }
    // Jacobi step into the next history slot
    const int slot = next_slot;
    next_slot = (next_slot + 1) % slots;
    double* vec = c.hist + 2L * slot * nt;
    double* err = vec + nt;
    cc::jacobi_kernel<<<cc::nblk(nt), 256, 0, s>>>(c.tvec, c.om, c.eps, c.o, c.v, vec, err);
    RI_TRY(check_launch("jacobi_kernel"));
    bool extrapolated = false;
    if (op.diis_size >= 2) {
      // drop the slot being overwritten from the history
      for (size_t k = 0; k < order.size(); ++k)
        if (order[k] == slot) {
          order.erase(order.begin() + k);
          gram.erase(gram.begin() + k);
          for (auto& row : gram) row.erase(row.begin() + k);
          break;
        }
      order.push_back(slot);
      const int mm = static_cast<int>(order.size());
      for (int k = 0; k < mm; ++k) {
        const double* ek = c.hist + 2L * order[k] * nt + nt;
        RI_TRY(dot(err, ek, nt, c.part, c.scal + k, s));
      }
      RI_TRY(c.read_scalars(hostv, mm));
      for (int k = 0; k < mm - 1; ++k) gram[k].push_back(hostv[k]);
      gram.push_back(std::vector<double>(hostv, hostv + mm));
      if (it + 1 >= op.diis_start) {
        while (order.size() >= 2) {
          std::vector<double> coef;
          if (cc::diis_solve(gram, coef)) {
            cc::Coefs cf;
            cf.m = static_cast<int>(order.size());
            for (int k = 0; k < cf.m; ++k) {
              cf.c[k] = coef[k];
              cf.slot[k] = order[k];
            }
            cc::combine_kernel<<<cc::nblk(nt), 256, 0, s>>>(cf, c.hist, 2L * nt, nt, c.tvec);
            RI_TRY(check_launch("combine_kernel"));
            extrapolated = true;
            break;
          }
          order.erase(order.begin());
          gram.erase(gram.begin());
          for (auto& row : gram) row.erase(row.begin());
        }
      }
    }
    if (!extrapolated) RI_HIP(hipMemcpyAsync(c.tvec, vec, sizeof(double) * nt, hipMemcpyDeviceToDevice, s));
    cc::symmetrize_kernel<<<cc::nblk(c.noovv), 256, 0, s>>>(tv2, c.o, c.v);
    RI_TRY(check_launch("symmetrize_kernel"));
    RI_TRY(c.energy(tv1, tv2, c.scal));
    RI_TRY(c.read_scalars(hostv, 1));
    e_prev = e;
    e = hostv[0];
  }
  const double sec_total = std::chrono::duration<double>(clk::now() - t_start).count();
  // max |Omega| of the returned amplitudes with the FP64 ladder
  double rinf64 = NAN;
  if (status == RI_OK) {
    if (conv && prec == RI_PREC_FP64 && c.other_prec == RI_PREC_FP64) {
      rinf64 = rinf;
    } else if (mixed && op.check_fp64) {
      float ms = 0.f;
      c.other_prec = RI_PREC_FP64;
      RI_TRY(c.residual(tv1, tv2, c.om, c.om + nov, RI_PREC_FP64, &ms));
      RI_TRY(max_abs(c.om, nt, c.part, c.scal, s));
      RI_TRY(c.read_scalars(hostv, 1));
      rinf64 = hostv[0];
    }
  }
  RI_HIP(hipMemcpyAsync(t1, tv1, sizeof(double) * nov, hipMemcpyDeviceToDevice, s));
  RI_HIP(hipMemcpyAsync(t2, tv2, sizeof(double) * c.noovv, hipMemcpyDeviceToDevice, s));
  RI_HIP(hipStreamSynchronize(s));
  if (rep) {
    rep->residual_rms = rrms;
    rep->residual_inf_fp64 = rinf64;
    rep->polish_iteration = polish_it;
    rep->seconds_guess = sec_guess;
    rep->guess_used = guess_used;
    rep->e_corr = e;
    rep->e_mp2 = e_mp2;
    rep->residual_inf = rinf;
    rep->iterations = it;
    rep->converged = conv ? 1 : 0;
    rep->seconds_total = sec_total;
    rep->seconds_ppl = ms_ppl_total * 1e-3;
  }
  if (status != RI_OK) return status;
  if (!conv) {
    set_error("ri_ccsd_iterate: not converged in %d iterations (|Omega|inf = %.3e)", op.max_iter, rinf);
    return RI_E_NOCONV;
  }
  return RI_OK;
}

}  // extern "C"
