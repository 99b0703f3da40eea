// Host-side contraction planner (einsum-style specs -> strided MFMA GEMM),
// permuted axpby and deterministic reductions.
#include <cstring>

#include "gemm.h"

namespace ri {

// ------------------------------------------------------------------ arena
int GemmArena::reserve(size_t doubles) {
  if (doubles <= cap) return RI_OK;
  if (p) dev_free(p, s);
  p = nullptr;
  cap = 0;
  const size_t want = std::max(doubles, static_cast<size_t>(1) << 16);
  void* q = nullptr;
  RI_TRY(dev_alloc(&q, want * sizeof(double), s));
  p = static_cast<double*>(q);
  cap = want;
  return RI_OK;
}

GemmArena::~GemmArena() {
  if (p) dev_free(p, s);
}

// ------------------------------------------------------------------ planner
namespace {

struct Level {
  long ext;
  long sa, sb, sc;  // strides in A, B, C (0 when absent)
};

struct Spec {
  std::string a, b, c;
};

bool parse(const char* spec, Spec& out) {
  std::string s(spec);
  const size_t comma = s.find(','), arrow = s.find("->");
  if (comma == std::string::npos || arrow == std::string::npos || comma > arrow) return false;
  out.a = s.substr(0, comma);
  out.b = s.substr(comma + 1, arrow - comma - 1);
  out.c = s.substr(arrow + 2);
  return true;
}

// Group letters (outer to inner) into levels, merging neighbours whose strides
// line up in every operand that carries them.
std::vector<Level> merge(const std::vector<Level>& in) {
  std::vector<Level> out;
  for (const Level& l : in) {
    if (!out.empty()) {
      Level& o = out.back();
      auto ok = [&](long so, long si) { return so == l.ext * si || (so == 0 && si == 0); };
      if (ok(o.sa, l.sa) && ok(o.sb, l.sb) && ok(o.sc, l.sc)) {
        o.ext *= l.ext;
        o.sa = l.sa;
        o.sb = l.sb;
        o.sc = l.sc;
        continue;
      }
    }
    out.push_back(l);
  }
  return out;
}

}  // namespace

int einsum(const char* spec, double alpha, const Tensor& A, const Tensor& B, double beta, const Tensor& C,
           GemmArena& arena, hipStream_t s, int prec) {
  Spec sp;
  if (!parse(spec, sp) || sp.a.size() != A.dims.size() || sp.b.size() != B.dims.size() ||
      sp.c.size() != C.dims.size()) {
    set_error("einsum: spec '%s' does not match operand ranks", spec);
    return RI_E_ARG;
  }
  auto find = [](const std::string& str, char ch) { return static_cast<int>(str.find(ch)); };
  std::vector<Level> mL, nL, kA, kB;
  std::vector<Level> batch;
  std::string seen;
  auto info = [&](char ch, Level& L, int& where) -> bool {
    const int ia = find(sp.a, ch), ib = find(sp.b, ch), ic = find(sp.c, ch);
    long ext = -1;
    where = (ia >= 0 ? 1 : 0) | (ib >= 0 ? 2 : 0) | (ic >= 0 ? 4 : 0);
    L = Level{0, 0, 0, 0};
    if (ia >= 0) { ext = A.dims[ia]; L.sa = A.strides[ia]; }
    if (ib >= 0) { if (ext >= 0 && B.dims[ib] != ext) return false; ext = B.dims[ib]; L.sb = B.strides[ib]; }
    if (ic >= 0) { if (ext >= 0 && C.dims[ic] != ext) return false; ext = C.dims[ic]; L.sc = C.strides[ic]; }
    L.ext = ext;
    return ext > 0;
  };
  // output letters in C order, summed letters in A order (then B order as a fallback)
  for (char ch : sp.c) {
    Level L;
    int w;
    if (!info(ch, L, w)) { set_error("einsum '%s': bad extent for '%c'", spec, ch); return RI_E_ARG; }
    if (w == 5) mL.push_back(L);
    else if (w == 6) nL.push_back(L);
    else if (w == 7) batch.push_back(L);
    else { set_error("einsum '%s': output letter '%c' must come from one operand", spec, ch); return RI_E_ARG; }
  }
  for (char ch : sp.a) {
    Level L;
    int w;
    if (!info(ch, L, w)) { set_error("einsum '%s': bad extent for '%c'", spec, ch); return RI_E_ARG; }
    if (w == 3) kA.push_back(L);
    else if (w == 1) { set_error("einsum '%s': letter '%c' only in the first operand", spec, ch); return RI_E_ARG; }
  }
  for (char ch : sp.b) {
    Level L;
    int w;
    if (!info(ch, L, w)) { set_error("einsum '%s': bad extent for '%c'", spec, ch); return RI_E_ARG; }
    if (w == 3) kB.push_back(L);
    else if (w == 2) { set_error("einsum '%s': letter '%c' only in the second operand", spec, ch); return RI_E_ARG; }
  }
  if (batch.size() > 1 || kA.empty()) {
    set_error("einsum '%s': needs at least one summed letter and at most one batch letter", spec);
    return RI_E_ARG;
  }
  // Row and column letters may be taken in any order: put the one with the
  // smallest stride in the operand that is loaded along it innermost (coalesced
  // loads), unless that leaves too many levels after merging.
  auto by_stride = [](std::vector<Level> v, bool use_a) {
    std::stable_sort(v.begin(), v.end(), [&](const Level& x, const Level& y) {
      return use_a ? std::labs(x.sa) > std::labs(y.sa) : std::labs(x.sb) > std::labs(y.sb);
    });
    return merge(v);
  };
  std::vector<Level> m = by_stride(mL, true), n = by_stride(nL, false), k = merge(kA);
  if (m.size() > 2) m = merge(mL);
  if (n.size() > 2) n = merge(nL);
  if (k.size() > 3) k = merge(kB);
  if (m.size() > 2 || n.size() > 2 || k.size() > 3) {
    set_error("einsum '%s': too many index levels after merging (%zu, %zu, %zu)", spec, m.size(), n.size(), k.size());
    return RI_E_ARG;
  }
  while (m.size() < 2) m.insert(m.begin(), Level{1, 0, 0, 0});
  while (n.size() < 2) n.insert(n.begin(), Level{1, 0, 0, 0});
  while (k.size() < 3) k.insert(k.begin(), Level{1, 0, 0, 0});

  gemm::GemmDesc g;
  g.M = m[0].ext * m[1].ext;
  g.N = n[0].ext * n[1].ext;
  g.K = k[0].ext * k[1].ext * k[2].ext;
  g.M2 = m[1].ext;
  g.N2 = n[1].ext;
  g.K2 = k[1].ext;
  g.K3 = k[2].ext;
  g.a = A.p;
  g.am1 = m[0].sa; g.am2 = m[1].sa;
  g.ak1 = k[0].sa; g.ak2 = k[1].sa; g.ak3 = k[2].sa;
  g.b = B.p;
  g.bk1 = k[0].sb; g.bk2 = k[1].sb; g.bk3 = k[2].sb;
  g.bn1 = n[0].sb; g.bn2 = n[1].sb;
  g.c = const_cast<double*>(C.p);
  g.cm1 = m[0].sc; g.cm2 = m[1].sc;
  g.cn1 = n[0].sc; g.cn2 = n[1].sc;
  g.alpha = alpha;
  g.beta = beta;
  int nb = 1;
  g.a_batch = g.b_batch = g.c_batch = 0;
  if (!batch.empty()) {
    nb = static_cast<int>(batch[0].ext);
    g.a_batch = batch[0].sa;
    g.b_batch = batch[0].sb;
    g.c_batch = batch[0].sc;
  }
  arena.s = s;
  const size_t need = gemm::scratch_doubles(g, nb);
  if (need) RI_TRY(arena.reserve(need));
  ProfScope ps(s, spec, 2.0 * static_cast<double>(g.M) * g.N * g.K * nb);
  return gemm::run(g, nb, arena.p, arena.cap, s, prec);
}

// ------------------------------------------------------------------ permuted axpby
namespace {
constexpr int MAXD = 6;
struct PermDesc {
  int nd;
  long od[MAXD];   // output extents
  long os[MAXD];   // output strides
  long is[MAXD];   // input strides, in output letter order
};

__global__ void axpby_perm_kernel(PermDesc d, double alpha, const double* __restrict__ in, double beta,
                                  double* out, long total) {
  const long idx = static_cast<long>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (idx >= total) return;
  long r = idx, io = 0, oo = 0;
  for (int k = d.nd - 1; k >= 0; --k) {
    const long x = r % d.od[k];
    r /= d.od[k];
    io += x * d.is[k];
    oo += x * d.os[k];
  }
  const double val = alpha * in[io];
  out[oo] = beta == 0.0 ? val : val + beta * out[oo];
}
}  // namespace

int axpby_perm(const char* spec, double alpha, const Tensor& in, double beta, const Tensor& out, hipStream_t s) {
  std::string sp(spec);
  const size_t arrow = sp.find("->");
  if (arrow == std::string::npos) {
    set_error("axpby_perm: bad spec '%s'", spec);
    return RI_E_ARG;
  }
  const std::string a = sp.substr(0, arrow), c = sp.substr(arrow + 2);
  if (a.size() != in.dims.size() || c.size() != out.dims.size() || a.size() != c.size() ||
      c.size() > static_cast<size_t>(MAXD)) {
    set_error("axpby_perm: spec '%s' does not match ranks", spec);
    return RI_E_ARG;
  }
  PermDesc d;
  d.nd = static_cast<int>(c.size());
  long total = 1;
  for (int k = 0; k < d.nd; ++k) {
    const size_t pos = a.find(c[k]);
    if (pos == std::string::npos || in.dims[pos] != out.dims[k]) {
      set_error("axpby_perm: spec '%s' letter '%c' mismatched", spec, c[k]);
      return RI_E_ARG;
    }
    d.od[k] = out.dims[k];
    d.os[k] = out.strides[k];
    d.is[k] = in.strides[pos];
    total *= out.dims[k];
  }
  if (total == 0) return RI_OK;
  ProfScope ps(s, "axpby_perm", 0.0, 16.0 * total);
  axpby_perm_kernel<<<static_cast<unsigned>((total + 255) / 256), 256, 0, s>>>(d, alpha, in.p, beta,
                                                                              const_cast<double*>(out.p), total);
  return check_launch("axpby_perm_kernel");
}

// ------------------------------------------------------------------ reductions
namespace {
constexpr int RB = 1024;  // partial sums (fixed, so the reduction order never changes)

template <int MODE>  // 0: sum x*y, 1: max |x|
__global__ __launch_bounds__(256) void reduce_stage1(const double* __restrict__ x, const double* __restrict__ y,
                                                     long n, double* part) {
  __shared__ double sh[256];
  const long chunk = (n + RB - 1) / RB;
  const long lo = static_cast<long>(blockIdx.x) * chunk, hi = std::min(n, lo + chunk);
  double acc = 0.0;
  for (long i = lo + threadIdx.x; i < hi; i += 256) {
    if (MODE == 0) acc += x[i] * y[i];
    else acc = fmax(acc, fabs(x[i]));
  }
  sh[threadIdx.x] = acc;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if (threadIdx.x < w) {
      if (MODE == 0) sh[threadIdx.x] += sh[threadIdx.x + w];
      else sh[threadIdx.x] = fmax(sh[threadIdx.x], sh[threadIdx.x + w]);
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) part[blockIdx.x] = sh[0];
}

template <int MODE>
__global__ __launch_bounds__(256) void reduce_stage2(const double* __restrict__ part, double* res) {
  __shared__ double sh[256];
  double acc = 0.0;
  for (int i = threadIdx.x; i < RB; i += 256) {
    if (MODE == 0) acc += part[i];
    else acc = fmax(acc, part[i]);
  }
  sh[threadIdx.x] = acc;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if (threadIdx.x < w) {
      if (MODE == 0) sh[threadIdx.x] += sh[threadIdx.x + w];
      else sh[threadIdx.x] = fmax(sh[threadIdx.x], sh[threadIdx.x + w]);
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) *res = sh[0];
}
}  // namespace

int reduce_partials() { return RB; }

int dot(const double* x, const double* y, long n, double* part, double* res, hipStream_t s) {
  reduce_stage1<0><<<RB, 256, 0, s>>>(x, y, n, part);
  reduce_stage2<0><<<1, 256, 0, s>>>(part, res);
  return check_launch("dot");
}

int max_abs(const double* x, long n, double* part, double* res, hipStream_t s) {
  reduce_stage1<1><<<RB, 256, 0, s>>>(x, x, n, part);
  reduce_stage2<1><<<1, 256, 0, s>>>(part, res);
  return check_launch("max_abs");
}

}  // namespace ri
