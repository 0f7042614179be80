// metric.h -- the element map's Jacobian and the metric coefficient fields at a
// point, shared by the quadrature kernels (FP64 always).
#pragma once
#include <hip/hip_runtime.h>

#include "terms.h"

namespace dpg {

// Doubles per element of each geometry kind.
__host__ __device__ constexpr int geom_stride(int kind) { return kind == 1 ? 12 : kind == 2 ? 10 : 24; }

// J_ij = dx_i / dxi_j at (x1, x2, x3) in the reference cube.
//   kind 0, trilinear: X = 8 vertices x 3, vertex v = v1 + 2 v2 + 4 v3 at corner (v1, v2, v3);
//   kind 1, affine:    X = x0[3], J[3][3] row-major;
//   kind 2, extruded:  X = x1_0, lambda1, then the (x2, x3) of the cross-section's corners
//                      (v2, v3) = (0,0), (1,0), (0,1), (1,1): x1 = x1_0 + lambda1 xi1 and
//                      (x2, x3) bilinear in (xi2, xi3) (the second form of (2.89)).
__device__ __forceinline__ void jacobian_at(int kind, const double* X, double x1, double x2, double x3,
                                            double J[3][3]) {
  if (kind == 1) {
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
      for (int j = 0; j < 3; ++j) J[i][j] = X[3 + 3 * i + j];
    return;
  }
  if (kind == 2) {
    const double* q = X + 2;   // q[2 (v2 + 2 v3) + c], c = 0: x2, 1: x3
    J[0][0] = X[1];
    J[0][1] = J[0][2] = J[1][0] = J[2][0] = 0.0;
#pragma unroll
    for (int c = 0; c < 2; ++c) {
      J[1 + c][1] = (q[2 + c] - q[c]) * (1.0 - x3) + (q[6 + c] - q[4 + c]) * x3;
      J[1 + c][2] = (q[4 + c] - q[c]) * (1.0 - x2) + (q[6 + c] - q[2 + c]) * x2;
    }
    return;
  }
  const double a1[2] = {1.0 - x1, x1}, a2[2] = {1.0 - x2, x2}, a3[2] = {1.0 - x3, x3};
#pragma unroll
  for (int i = 0; i < 3; ++i) {
    double c0 = 0.0, c1 = 0.0, c2 = 0.0;
#pragma unroll
    for (int u = 0; u < 2; ++u)
#pragma unroll
      for (int v = 0; v < 2; ++v) {
        // d/dxi1: edges (0,u,v) -> (1,u,v)
        c0 += (X[3 * (1 + 2 * u + 4 * v) + i] - X[3 * (2 * u + 4 * v) + i]) * a2[u] * a3[v];
        // d/dxi2: edges (u,0,v) -> (u,1,v)
        c1 += (X[3 * (u + 2 + 4 * v) + i] - X[3 * (u + 4 * v) + i]) * a1[u] * a3[v];
        // d/dxi3: edges (u,v,0) -> (u,v,1)
        c2 += (X[3 * (u + 2 * v + 4) + i] - X[3 * (u + 2 * v) + i]) * a1[u] * a2[v];
      }
    J[i][0] = c0;
    J[i][1] = c1;
    J[i][2] = c2;
  }
}

// adjugate: J^-1 = adj / det
__device__ __forceinline__ double adjugate(const double J[3][3], double adj[3][3]) {
  adj[0][0] = J[1][1] * J[2][2] - J[1][2] * J[2][1];
  adj[0][1] = J[0][2] * J[2][1] - J[0][1] * J[2][2];
  adj[0][2] = J[0][1] * J[1][2] - J[0][2] * J[1][1];
  adj[1][0] = J[1][2] * J[2][0] - J[1][0] * J[2][2];
  adj[1][1] = J[0][0] * J[2][2] - J[0][2] * J[2][0];
  adj[1][2] = J[0][2] * J[1][0] - J[0][0] * J[1][2];
  adj[2][0] = J[1][0] * J[2][1] - J[1][1] * J[2][0];
  adj[2][1] = J[0][1] * J[2][0] - J[0][0] * J[2][1];
  adj[2][2] = J[0][0] * J[1][1] - J[0][1] * J[1][0];
  return J[0][0] * adj[0][0] + J[0][1] * adj[1][0] + J[0][2] * adj[2][0];
}

// metric field value (unweighted) at a point
__device__ __forceinline__ double field_value(int fid, const double J[3][3], const double adj[3][3],
                                              double det, double idet) {
  if (fid == FLD_DETJ) return det;
  if (fid == FLD_IDETJ) return idet;
  if (fld_is_D(fid)) {
    const int s = fid - FLD_D11, a = sym_a(s), b = sym_b(s);
    return (adj[a][0] * adj[b][0] + adj[a][1] * adj[b][1] + adj[a][2] * adj[b][2]) * idet;
  }
  const int s = fid - FLD_C11, a = sym_a(s), b = sym_b(s);
  return (J[0][a] * J[0][b] + J[1][a] * J[1][b] + J[2][a] * J[2][b]) * idet;
}

}  // namespace dpg
