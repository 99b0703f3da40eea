// Generic strided FP64 contraction (internal).
#pragma once

#include <algorithm>
#include <string>
#include <vector>

#include "ri_common.h"

namespace ri {
namespace gemm {

// C(m, n) = alpha * sum_k A(m, k) B(k, n) + beta * C(m, n)
// m = m1*M2 + m2, n = n1*N2 + n2, k = (k1*K2 + k2)*K3 + k3; every level has a stride.
struct GemmDesc {
  long M, N, K;
  long M2, N2, K2, K3;
  const double* a;
  long am1, am2, ak1, ak2, ak3;
  const double* b;
  long bk1, bk2, bk3, bn1, bn2;
  double* c;
  long cm1, cm2, cn1, cn2;
  double alpha, beta;
  long a_batch, b_batch, c_batch;
};

// Doubles of scratch the split-k form of a contraction wants (0: not split).
size_t scratch_doubles(const GemmDesc& g, int batch);
// Launches the contraction; it is split over k when `scratch` holds at least
// scratch_doubles(g, batch) doubles, else it runs in one pass.  prec RI_PREC_FP32 lets
// the large-tile kernel round its operands to FP32 and use the FP32 MFMA (the
// smaller kernels always run in FP64).
int run(const GemmDesc& g, int batch, double* scratch, size_t scratch_len, hipStream_t s,
        int prec = RI_PREC_FP64);

}  // namespace gemm

// An FP64 tensor view on the device: dims with element strides (row-major when
// no strides are given).
struct Tensor {
  const double* p;
  std::vector<long> dims, strides;
  Tensor(const double* ptr, std::vector<long> d) : p(ptr), dims(std::move(d)) {
    strides.assign(dims.size(), 1);
    for (int k = static_cast<int>(dims.size()) - 2; k >= 0; --k) strides[k] = strides[k + 1] * dims[k + 1];
  }
  Tensor(const double* ptr, std::vector<long> d, std::vector<long> st)
      : p(ptr), dims(std::move(d)), strides(std::move(st)) {}
  long size() const {
    long n = 1;
    for (long x : dims) n *= x;
    return n;
  }
};

// Scratch for split-k partial products (grown on demand, stream-ordered).
struct GemmArena {
  double* p = nullptr;
  size_t cap = 0;
  hipStream_t s = nullptr;
  int reserve(size_t doubles);
  ~GemmArena();
};

// out[c_idx] = alpha * sum A[a_idx] B[b_idx] + beta * out, described einsum-style,
// e.g. "kiac,kjbc->ijab".  Each letter appears in exactly two of the three
// operands (at most one letter in all three, mapped to the launch's batch
// dimension).  Letters are merged into the contraction's index levels when their
// strides allow; at most 2 output-row, 2 output-column and 3 summed levels remain.
int einsum(const char* spec, double alpha, const Tensor& A, const Tensor& B, double beta, const Tensor& out,
           GemmArena& arena, hipStream_t s, int prec = RI_PREC_FP64);

// out = alpha * permute(in) + beta * out, with spec like "kiac->aikc" (in -> out letters).
int axpby_perm(const char* spec, double alpha, const Tensor& in, double beta, const Tensor& out, hipStream_t s);

// Deterministic reductions (fixed blocking and tree order); the result stays on
// the device at *res.  `part` needs reduce_partials() doubles.
int reduce_partials();
int dot(const double* x, const double* y, long n, double* part, double* res, hipStream_t s);
int max_abs(const double* x, long n, double* part, double* res, hipStream_t s);

}  // namespace ri
