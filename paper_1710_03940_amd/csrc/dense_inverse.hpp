// Blocked in-place FP64 inverse of a dense matrix on the GPU (the coarse
// operator E of the deflation).
#pragma once

#include <hip/hip_runtime.h>

#include <string>

namespace dfamg {

struct DenseInverseError {
    std::string msg;
};

// Replaces the row-major n x n device matrix A by its inverse (Gauss-Jordan
// with partial pivoting, column panels + GEMM updates), ordered on stream s;
// returns false when a pivot column is exactly zero (singular matrix; A is
// then unspecified).  Synchronises s before returning.  Throws
// DenseInverseError when a HIP or rocBLAS call fails.
bool invert_dense_inplace(hipStream_t s, double *A, int n);

}  // namespace dfamg
