// Batched complex double GEMM on the matrix cores (see gemm.hip).
#pragma once

#include <hip/hip_runtime.h>

#include "internal.h"

#include <cstdint>
#include <memory>
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

// Launch all GEMMs of `descs` in one kernel on stream s (synchronises s;
// with keep, the staged descriptors move into *keep instead, which the
// caller holds until it synchronises s).
void zgemm_batched(std::vector<GemmDesc>& descs, hipStream_t s, std::vector<std::vector<GemmDesc>>* keep = nullptr);

// Complex GEMM on the FP32 or BF16 matrix cores with FP32 accumulation.
// Operands and result may each be complex double (converted on load or
// store) or complex float; layout and ops as GemmDesc.  XG_BF16X3 splits
// each float operand into two BF16 parts and keeps three of the four
// partial products (about 16 significant bits).
enum { XG_FP32 = 0, XG_BF16 = 1, XG_BF16X3 = 2 };
struct GemmDescX {
  const void* A;
  const void* B;
  void* C;
  int64_t lda, ldb, ldc;
  int64_t M, N, K;
  int32_t opA, opB;
  int32_t a64, b64, c64;  // 1: complex double, 0: complex float
  int32_t transC;
  float alpha_re, alpha_im;
  int64_t tile_start;  // filled by xgemm_batched
};

inline GemmDescX gemmx(const void* A, int a64, int64_t lda, int opA, const void* B, int b64, int64_t ldb, int opB,
                       void* C, int c64, int64_t ldc, int64_t M, int64_t N, int64_t K, float alpha = 1.0f) {
  GemmDescX d{};
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
  d.a64 = a64;
  d.b64 = b64;
  d.c64 = c64;
  d.alpha_re = alpha;
  d.alpha_im = 0.0f;
  return d;
}

// mode XG_FP32 or XG_BF16; synchronises s (keep: as zgemm_batched).
void xgemm_batched(std::vector<GemmDescX>& descs, int mode, hipStream_t s,
                   std::vector<std::vector<GemmDescX>>* keep = nullptr);

// As GemmPlan, for the FP32 / BF16 matrix cores (no tuning).
class XGemmPlan {
 public:
  XGemmPlan(const std::vector<std::vector<GemmDescX>>& groups, int mode, hipStream_t s);
  void launch(size_t g, hipStream_t s) const;
  // device copy of group g's descriptors (kernels may repoint operands)
  GemmDescX* desc(size_t g) const { return dev_.as<GemmDescX>() + first_[g]; }

 private:
  int mode_;
  Scratch dev_;
  std::vector<int64_t> first_, count_, tiles_;
  std::vector<double> flops_;
  std::vector<int> types_;  // operand element types of each group
};

// Groups of GEMMs whose descriptors are uploaded to the device once (one
// synchronisation, in the constructor); launch(g) then runs group g with no
// host round trip.  The descriptor memory is freed in stream order.  With
// tune, each new shape class among the groups is timed once in every
// launch shape (only groups whose products overwrite results that overlap
// no operand) and the fastest is used from then on by every GEMM of that
// class in the process.
// nb products C_c = alpha op(A_c) op(B_c) (+ C_c) on the row-block kernel,
// with A_c = A + c sA, B_c = B + c sB, C_c = C + c sC (elements) and the
// sizes, leading dimensions and ops of d, which dev holds on the device:
// 1 to 32 columns, op(A) N or R and op(B) T or C (rows of op(A) and
// columns of op(B) contiguous along k).  ws: panel_batch_ws_bytes(d, nb)
// bytes of device memory for the K-split parts.
size_t panel_batch_ws_bytes(const GemmDesc& d, int64_t nb);
void panel_batch(const GemmDesc* dev, const GemmDesc& d, int64_t nb, int64_t sA, int64_t sB, int64_t sC, double* ws,
                 hipStream_t s);

class GemmPlan {
 public:
  GemmPlan(const std::vector<std::vector<GemmDesc>>& groups, hipStream_t s, bool tune = true);
  void launch(size_t g, hipStream_t s) const;
  // device copy of group g's descriptors (kernels may repoint operands)
  GemmDesc* desc(size_t g) const { return dev_.as<GemmDesc>() + first_[g]; }

 private:
  bool tune_;
  Scratch dev_;
  std::vector<int64_t> first_, count_, tiles_, m_, n_, k_;
  std::vector<double> flops_;
  std::vector<int> variant_;
  std::unique_ptr<Scratch> ws_;  // partial tiles of K-split launch shapes
};

}  // namespace cbfm
