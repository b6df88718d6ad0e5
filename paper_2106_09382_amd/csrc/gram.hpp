// Gram matrix S = Y^T Y / n on matrix cores.
#pragma once

#include <hip/hip_runtime.h>

namespace concord {

// S = Y^T Y / n; Y is n x p, S is p x p (both triangles written).
template <typename T>
hipError_t launch_gram(const T *Y, int n, int p, T *S, hipStream_t stream);

// C = A^T B; A is K x M, B is K x N, C is M x N (all row-major).
template <typename T>
hipError_t launch_atb(const T *A, const T *B, int K, int M, int N, T *C, hipStream_t stream);

}  // namespace concord
