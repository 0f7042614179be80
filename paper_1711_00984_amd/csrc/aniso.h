// aniso.h -- launch interface of the Gram kernel for non-uniform orders
// (p1, p2, p3): one 1D Gauss rule per coordinate and the coordinate of least
// order contracted last, i.e. in the outermost loop (text after Algorithm 2).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace dpg {

constexpr int ANISO_PMAX = 10;                // largest order per direction (H1 at 10, 10, 10 in FP64 fills most of the LDS)
constexpr int ANISO_LMAX = ANISO_PMAX + 1;    // largest point count per direction

struct AnisoArgs {
  const double* geom;      // [E][stride] by geom_kind (0 trilinear, 1 affine, 2 extruded)
  int geom_kind;
  int64_t n_elem;
  void* out;               // Real*, element e at e * packed_len
  int64_t packed_len;
  int space;               // 0 H1, 1 H(curl), 2 H(div), 3 L2
  int q[3];                // orders per direction
  int L[3];                // points per direction
  int dir[3];              // contraction order: dir[0] first (innermost loop), dir[2] last (outermost)
  const double* tab64[3];  // FP64 table block of each direction's rule
  const void* tabR[3];     // the same blocks in the output precision
  double w0, w1;
  int32_t* status;         // per element (nullptr: none)
  // set by the launcher: LDS sizes in Reals (fields; one pair's stage-A buffer) and
  // the pairs per barrier interval
  int lds_fields = 0, lds_a = 0, pairs = 1;
};

hipError_t launch_aniso(int prec, const AnisoArgs& a, hipStream_t s);

}  // namespace dpg
