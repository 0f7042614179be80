// adjoint.hip -- test-space pieces beyond the element Grams of Section 2:
//
// * the coupling block of the adjoint graph inner product of the ultraweak
//   formulation (Section 3.3, (3.17), (3.18)): for q_I in W^p (H1) and v_J in
//   V^p (H(div)),  C[I][J] = int_K (v_J . grad q_I - q_I div v_J) dx.  With the
//   Piola maps (2.28), (2.46) the Jacobians cancel, so C is the same for every
//   element, and in the tensor bases it is a product of exact 1D integrals
//   F^{rs} (2.90): for component b of v_J = chi_{j_b}(xi_b) prod_{d != b}
//   nu_{j_d}(xi_d) e_b, with nu_j = chi'_{j+1},
//       C[I][J] = prod_{d != b} F^{01}_{i_d, j_d+1} (F^{10}_{i_b, j_b} - F^{01}_{i_b, j_b});
//
// * block-diagonal replication for vector-valued test spaces (Section 2.7,
//   (2.85)-(2.88)): the Gram of the c-fold product of a space is the scalar
//   Gram on each of the c diagonal blocks, zero elsewhere.  The paper suggests
//   producing it by changing the filling step; here a streaming kernel expands
//   packed Grams, one wave per packed output column (two contiguous runs: the
//   zeros above the diagonal block and the copied column).
#include <hip/hip_runtime.h>

#include <algorithm>

#include "kernels.h"

namespace dpg {

namespace {

constexpr int NT_ADJ = 256;

template <typename Real>
__global__ void __launch_bounds__(NT_ADJ) k_coupling(const Real* __restrict__ F, int p, Real* __restrict__ out) {
  const int r = p + 1;
  const int64_t nq = int64_t(r) * r * r, dv = int64_t(r) * p * p, nv = 3 * dv;
  const int64_t k = int64_t(blockIdx.x) * NT_ADJ + threadIdx.x;
  if (k >= nq * nv) return;
  const int64_t I = k / nv, J = k % nv;
  const int i[3] = {int(I % r), int((I / r) % r), int(I / (int64_t(r) * r))};
  const int b = int(J / dv);
  const int64_t loc = J % dv;
  int R[3];
  for (int d = 0; d < 3; ++d) R[d] = d == b ? r : p;
  const int j[3] = {int(loc % R[0]), int((loc / R[0]) % R[1]), int(loc / (int64_t(R[0]) * R[1]))};
  auto f = [&](int rs, int a, int c) { return F[(rs * KT + a) * KT + c]; };   // rs = 2 r + s
  Real v = f(2, i[b], j[b]) - f(1, i[b], j[b]);                               // F^10 - F^01
  for (int d = 0; d < 3; ++d)
    if (d != b) v *= f(1, i[d], j[d] + 1);                                      // F^01_{i, j+1}
  out[k] = v;
}

template <typename Real>
__global__ void __launch_bounds__(NT_ADJ) k_replicate(const Real* __restrict__ src, Real* __restrict__ dst,
                                                       int64_t n, int copies, int64_t n_elem) {
  const int lane = threadIdx.x & 63;
  const int64_t cn = n * copies;
  const int64_t w = int64_t(blockIdx.x) * (NT_ADJ / 64) + (threadIdx.x >> 6);   // output column of the batch
  if (w >= n_elem * cn) return;
  const int64_t e = w / cn, Jp = w % cn, kb = Jp / n, J = Jp % n;
  const Real* s = src + e * (n * (n + 1) / 2) + J * (J + 1) / 2;
  Real* col = dst + e * (cn * (cn + 1) / 2) + Jp * (Jp + 1) / 2;
  const int64_t z = kb * n;                                                      // rows above the block
  for (int64_t I = lane; I < z; I += 64) col[I] = Real(0);
  for (int64_t I = lane; I <= J; I += 64) col[z + I] = s[I];
}

}  // namespace

hipError_t launch_coupling(int p, int prec, const void* F, void* out, hipStream_t st) {
  const int64_t r = p + 1, total = r * r * r * 3 * r * p * p;
  const unsigned grid = unsigned((total + NT_ADJ - 1) / NT_ADJ);
  if (prec)
    hipLaunchKernelGGL(k_coupling<float>, dim3(grid), dim3(NT_ADJ), 0, st, static_cast<const float*>(F), p,
                       static_cast<float*>(out));
  else
    hipLaunchKernelGGL(k_coupling<double>, dim3(grid), dim3(NT_ADJ), 0, st, static_cast<const double*>(F), p,
                       static_cast<double*>(out));
  return hipGetLastError();
}

hipError_t launch_replicate(int prec, const void* src, void* dst, int64_t n, int copies, int64_t n_elem,
                            hipStream_t st) {
  constexpr int64_t kMaxGrid = int64_t(1) << 30;   // workgroups per launch (4 output columns each)
  for (int64_t e0 = 0; e0 < n_elem;) {
    const int64_t ne = std::min<int64_t>(n_elem - e0, std::max<int64_t>(1, kMaxGrid * 4 / (n * copies)));
    const unsigned grid = unsigned((ne * n * copies + 3) / 4);
    const int64_t so = e0 * (n * (n + 1) / 2), dof = e0 * (n * copies) * (n * copies + 1) / 2;
    if (prec)
      hipLaunchKernelGGL(k_replicate<float>, dim3(grid), dim3(NT_ADJ), 0, st, static_cast<const float*>(src) + so,
                         static_cast<float*>(dst) + dof, n, copies, ne);
    else
      hipLaunchKernelGGL(k_replicate<double>, dim3(grid), dim3(NT_ADJ), 0, st, static_cast<const double*>(src) + so,
                         static_cast<double*>(dst) + dof, n, copies, ne);
    e0 += ne;
  }
  return hipGetLastError();
}

}  // namespace dpg
