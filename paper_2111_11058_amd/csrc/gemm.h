// Batched complex double GEMM on the matrix cores (see gemm.hip).
#pragma once

#include <hip/hip_runtime.h>

#include "internal.h"

#include <cstdint>
#include <vector>

namespace cbfm {

enum { OP_N = 0, OP_T = 1, OP_C = 2, OP_R = 3 };

struct GemmDesc {
  const double2* A;
  const double2* B;
  double2* C;
  int64_t lda, ldb, ldc;
  int64_t M, N, K;  // C is M x N; op(A) is M x K; op(B) is K x N
  int32_t opA, opB;
  double alpha_re, alpha_im;
  int32_t accumulate;  // 1: C += alpha op(A) op(B)
  int32_t transC;      // 1: element (i, j) of the product is stored at C[j * ldc + i]
  int64_t tile_start;  // filled by zgemm_batched
};

inline GemmDesc gemm(const double2* A, int64_t lda, int opA, const double2* B, int64_t ldb, int opB,
                     double2* C, int64_t ldc, int64_t M, int64_t N, int64_t K, double alpha = 1.0,
                     int accumulate = 0) {
  GemmDesc d{};
  d.A = A;
  d.B = B;
  d.C = C;
  d.lda = lda;
  d.ldb = ldb;
  d.ldc = ldc;
  d.M = M;
  d.N = N;
  d.K = K;
  d.opA = opA;
  d.opB = opB;
  d.alpha_re = alpha;
  d.alpha_im = 0.0;
  d.accumulate = accumulate;
  return d;
}

// Launch all GEMMs of `descs` in one kernel on stream s (synchronises s).
void zgemm_batched(std::vector<GemmDesc>& descs, hipStream_t s);

// Groups of GEMMs whose descriptors are uploaded to the device once (one
// synchronisation, in the constructor); launch(g) then runs group g with no
// host round trip.  The descriptor memory is freed in stream order.  With
// tune, each new shape class among the groups is timed once in every
// launch shape (only groups whose products overwrite results that overlap
// no operand) and the fastest is used from then on by every GEMM of that
// class in the process.
class GemmPlan {
 public:
  GemmPlan(const std::vector<std::vector<GemmDesc>>& groups, hipStream_t s, bool tune = true);
  void launch(size_t g, hipStream_t s) const;

 private:
  bool tune_;
  Scratch dev_;
  std::vector<int64_t> first_, count_, tiles_;
  std::vector<double> flops_;
  std::vector<int> variant_;
};

}  // namespace cbfm
