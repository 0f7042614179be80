// condense.h -- launch interface of the static-condensation kernels: Cholesky
// factor of packed Grams and solves with it (Section 1 and (3.7)-(3.8)).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace dpg {

// In place: ap holds n_elem consecutive 'U' packed Grams of dimension n on
// entry and their factors U (G = U^T U) on exit; info[e] = 0, or k > 0 when the
// leading minor of order k of element e is not positive definite.  prec 0 FP64,
// 1 FP32.
hipError_t launch_potrf(int prec, void* ap, int64_t n, int64_t n_elem, int32_t* info, hipStream_t s);

// In place: b holds n_elem consecutive column-major n x nrhs blocks (leading
// dimension n); on exit b = G^{-1} b with G = U^T U, U from launch_potrf.
hipError_t launch_potrs(int prec, const void* up, int64_t n, int64_t n_elem, int64_t nrhs, void* b, hipStream_t s);

}  // namespace dpg
