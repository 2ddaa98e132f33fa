// Blocked Gauss-Jordan elimination for batches of dense complex double
// matrices (see gj.hip).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace cbfm {

// A_b = A + b strideA (b < nmat) is an n x n row-major matrix (row stride n);
// each is replaced by its inverse.  Throws CBFM_E_RANK naming `what` and the
// first matrix with a zero pivot.  Synchronises s.
void gj_inverse_batched(double2* A, int64_t strideA, int n, int nmat, const char* what, hipStream_t s);

// As gj_inverse_batched, enqueued on s with no host wait: info_dev (nmat
// int32 of device memory, owned by the caller) receives per matrix 0, or 1 +
// the first column without a nonzero pivot; gj_check reads it.
void gj_inverse_batched_async(double2* A, int64_t strideA, int n, int nmat, int32_t* info_dev, hipStream_t s);

// Throws CBFM_E_RANK naming `what` and the first matrix whose info_dev entry
// is nonzero.  Synchronises s.
void gj_check(const int32_t* info_dev, int nmat, const char* what, hipStream_t s);

// A_b = A + b strideA is the augmented n x ncols row-major system [Z_b | V_b]
// (row stride ld >= ncols > n); afterwards its columns n .. ncols - 1 hold
// Z_b^{-1} V_b (the first n columns are left in an unspecified state).
// Throws CBFM_E_RANK as above.  Synchronises s.
void gj_solve_batched(double2* A, int64_t strideA, int64_t ld, int n, int ncols, int nmat, const char* what,
                      hipStream_t s);

}  // namespace cbfm
