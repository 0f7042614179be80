// gram_affine.hip -- reduced O(p^6) path for elements with a constant Jacobian.
//
// Section 2.8.1: when J is constant, |J|, D and C leave the integrals, and
// every term of block (a, b) of the Gram matrix becomes
//     coef_t * F^{r1 s1}_{i1+sa1, j1+sb1} F^{r2 s2}_{i2+sa2, j2+sb2} F^{r3 s3}_{i3+sa3, j3+sb3}
// with the exact 1D integrals F^{rs} (2.90) of the chart (2.103)-(2.114)
// (Algorithm 10 for L2; the paper notes the extension to the other spaces).
// Only constancy of J is used, so sheared parallelepipeds qualify.  No
// quadrature and no shape-function evaluation remain: the kernel is a pure
// streaming writer of the packed output.
//
// Work decomposition: the same column slabs (b, j3) as the general path.
// Each wave takes one packed column J at a time; its 64 lanes walk the rows
// I = 0..J, so every store instruction writes 64 consecutive entries.  The
// F tables are banded (|i - j| <= 2 unless both indices are <= 3), so most
// entries are exact zeros: a per-direction band test skips the term sums.
#include <hip/hip_runtime.h>

#include "kernels.h"
#include "terms.h"

namespace dpg {

namespace {

constexpr int NT_AFF = 256;

__device__ __forceinline__ bool band(int i, int j) {
  const int d = i > j ? i - j : j - i;
  return d <= 2 || (i <= 3 && j <= 3);
}

template <int S, int P> struct AShape {
  static constexpr int NC = ncomp(S);
  static constexpr int R(int a, int d) { return range1d(S, P, a, d); }
  static constexpr int SH(int a, int d) { return shift1d(S, a, d); }
  static constexpr int OFF(int a) { return comp_off(S, P, a); }
  static constexpr int NSLAB = [] {
    int o = 0;
    for (int c = 0; c < NC; ++c) o += R(c, 2);
    return o;
  }();
};

// sum of the terms of block (A, B) at one entry
template <int S, int P, typename Real, int A, int B>
__device__ __forceinline__ Real block_entry(const Real* sF, const Real* coef, int i1, int i2, int i3, int j1,
                                            int j2, int j3) {
  using Sh = AShape<S, P>;
  constexpr Plan PL = make_plan(S, A, B);
  const int a1 = i1 + Sh::SH(A, 0), a2 = i2 + Sh::SH(A, 1), a3 = i3 + Sh::SH(A, 2);
  const int b1 = j1 + Sh::SH(B, 0), b2 = j2 + Sh::SH(B, 1), b3 = j3 + Sh::SH(B, 2);
  if (!(band(a1, b1) && band(a2, b2) && band(a3, b3))) return Real(0);
  Real v = Real(0);
#pragma unroll
  for (int t = 0; t < PL.nt; ++t) {
    const Term& T = PL.t[t];
    const Real f1 = sF[((2 * T.r[0] + T.s[0]) * KT + a1) * KT + b1];
    const Real f2 = sF[((2 * T.r[1] + T.s[1]) * KT + a2) * KT + b2];
    const Real f3 = sF[((2 * T.r[2] + T.s[2]) * KT + a3) * KT + b3];
    v += coef[t] * f1 * f2 * f3;
  }
  return v;
}

template <int S, int P, typename Real, int A, int B>
__device__ __forceinline__ Real entry_in(const Real* sF, const Real* sC, int I, int j1, int j2, int j3) {
  using Sh = AShape<S, P>;
  const int loc = I - Sh::OFF(A);
  const int i1 = loc % Sh::R(A, 0);
  const int t = loc / Sh::R(A, 0);
  const int i2 = t % Sh::R(A, 1), i3 = t / Sh::R(A, 1);
  return block_entry<S, P, Real, A, B>(sF, sC + A * 10, i1, i2, i3, j1, j2, j3);
}

template <int S, int P, typename Real, int B>
__device__ __forceinline__ Real entry(const Real* sF, const Real* sC, int I, int j1, int j2, int j3) {
  using Sh = AShape<S, P>;
  if constexpr (B >= 2) {
    if (I >= Sh::OFF(2)) return entry_in<S, P, Real, 2, B>(sF, sC, I, j1, j2, j3);
  }
  if constexpr (B >= 1) {
    if (I >= Sh::OFF(1)) return entry_in<S, P, Real, 1, B>(sF, sC, I, j1, j2, j3);
  }
  return entry_in<S, P, Real, 0, B>(sF, sC, I, j1, j2, j3);
}

template <int S, int P, typename Real, int B>
__device__ void write_slab(const Real* sF, const Real* sC, bool bad, int j3, Real* __restrict__ outp) {
  using Sh = AShape<S, P>;
  constexpr int R1b = Sh::R(B, 0), R2b = Sh::R(B, 1);
  constexpr int NCOL = R1b * R2b;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  for (int c = wave; c < NCOL; c += NT_AFF / 64) {
    const int j1 = c % R1b, j2 = c / R1b;
    const int64_t J = Sh::OFF(B) + c + int64_t(NCOL) * j3;
    Real* col = outp + J * (J + 1) / 2;
    for (int I = lane; I <= J; I += 64) {
      col[I] = bad ? Real(0) : entry<S, P, Real, B>(sF, sC, I, j1, j2, j3);
    }
  }
}

template <int S, int P, typename Real>
__global__ void __launch_bounds__(NT_AFF) k_affine(GeneralArgs ga) {
  using Sh = AShape<S, P>;
  __shared__ Real s_F[FTAB_LEN];
  __shared__ Real s_C[3 * 10];   // coefficients of the terms of blocks (a, b), b fixed
  __shared__ int s_bad;
  const int tid = threadIdx.x;
  const int64_t blk = blockIdx.x;
  const int slab = Sh::NSLAB - 1 - int(blk / ga.n_items);
  const int64_t item = ga.item_base + blk % ga.n_items;
  const int64_t e = ga.elem_ids ? int64_t(ga.elem_ids[item]) : item;
  int b = 0, j3 = slab;
#pragma unroll
  for (int c = 0; c < Sh::NC - 1; ++c)
    if (b == c && j3 >= Sh::R(c, 2)) { j3 -= Sh::R(c, 2); b = c + 1; }

  const Real* fR = static_cast<const Real*>(ga.ftabR);
  for (int i = tid; i < FTAB_LEN; i += NT_AFF) s_F[i] = fR[i];
  if (tid == 0) {
    const double* g = ga.geom + e * 12;
    double J[3][3], adj[3][3];
    for (int i = 0; i < 3; ++i)
      for (int j = 0; j < 3; ++j) J[i][j] = g[3 + 3 * i + j];
    adj[0][0] = J[1][1] * J[2][2] - J[1][2] * J[2][1];
    adj[0][1] = J[0][2] * J[2][1] - J[0][1] * J[2][2];
    adj[0][2] = J[0][1] * J[1][2] - J[0][2] * J[1][1];
    adj[1][0] = J[1][2] * J[2][0] - J[1][0] * J[2][2];
    adj[1][1] = J[0][0] * J[2][2] - J[0][2] * J[2][0];
    adj[1][2] = J[0][2] * J[1][0] - J[0][0] * J[1][2];
    adj[2][0] = J[1][0] * J[2][1] - J[1][1] * J[2][0];
    adj[2][1] = J[0][1] * J[2][0] - J[0][0] * J[2][1];
    adj[2][2] = J[0][0] * J[1][1] - J[0][1] * J[1][0];
    const double det = J[0][0] * adj[0][0] + J[0][1] * adj[1][0] + J[0][2] * adj[2][0];
    const double idet = 1.0 / det;
    s_bad = !(det > 0.0);
    double fv[FLD_COUNT];
    fv[FLD_DETJ] = det;
    fv[FLD_IDETJ] = idet;
    for (int s = 0; s < 6; ++s) {
      const int a = sym_a(s), bb = sym_b(s);
      fv[FLD_D11 + s] = (adj[a][0] * adj[bb][0] + adj[a][1] * adj[bb][1] + adj[a][2] * adj[bb][2]) * idet;
      fv[FLD_C11 + s] = (J[0][a] * J[0][bb] + J[1][a] * J[1][bb] + J[2][a] * J[2][bb]) * idet;
    }
    for (int a = 0; a < Sh::NC; ++a) {
      // terms of block (a, b): same construction as the plan used by block_entry
      const Plan PL = make_plan(S, a < b ? a : b, a < b ? b : a);
      for (int t = 0; t < 10; ++t) {
        double c = 0.0;
        if (t < PL.nt) {
          const int f = PL.t[t].field;
          c = PL.t[t].sign * fv[f] * (field_weight(S, f) ? ga.w1 : ga.w0);
        }
        s_C[a * 10 + t] = static_cast<Real>(c);
      }
    }
  }
  __syncthreads();
  Real* outp = static_cast<Real*>(ga.out) + (ga.out_offset ? ga.out_offset[e] : e * ga.packed_len);
  const bool bad = s_bad != 0;
  if constexpr (Sh::NC == 1) {
    write_slab<S, P, Real, 0>(s_F, s_C, bad, j3, outp);
  } else {
    if (b == 0) write_slab<S, P, Real, 0>(s_F, s_C, bad, j3, outp);
    else if (b == 1) write_slab<S, P, Real, 1>(s_F, s_C, bad, j3, outp);
    else write_slab<S, P, Real, 2>(s_F, s_C, bad, j3, outp);
  }
  if (ga.status && tid == 0 && (bad || slab == 0)) ga.status[e] = bad ? -4 : 0;
}

template <int S, int P, typename Real>
hipError_t launch_affine_one(const GeneralArgs& a, hipStream_t st) {
  constexpr int NS = AShape<S, P>::NSLAB;
  const int64_t max_items = int64_t(0x7fffffff) / NS;
  GeneralArgs c = a;
  for (int64_t base = 0; base < a.n_items; base += max_items) {
    c.item_base = a.item_base + base;
    c.n_items = (a.n_items - base) < max_items ? (a.n_items - base) : max_items;
    hipLaunchKernelGGL((k_affine<S, P, Real>), dim3(unsigned(c.n_items * NS)), dim3(NT_AFF), 0, st, c);
  }
  return hipGetLastError();
}

template <int S, typename Real>
hipError_t affine_p(int p, const GeneralArgs& a, hipStream_t st) {
  switch (p) {
    case 1: return launch_affine_one<S, 1, Real>(a, st);
    case 2: return launch_affine_one<S, 2, Real>(a, st);
    case 3: return launch_affine_one<S, 3, Real>(a, st);
    case 4: return launch_affine_one<S, 4, Real>(a, st);
    case 5: return launch_affine_one<S, 5, Real>(a, st);
    case 6: return launch_affine_one<S, 6, Real>(a, st);
    case 7: return launch_affine_one<S, 7, Real>(a, st);
    case 8: return launch_affine_one<S, 8, Real>(a, st);
    case 9: return launch_affine_one<S, 9, Real>(a, st);
    case 10: return launch_affine_one<S, 10, Real>(a, st);
    case 11: return launch_affine_one<S, 11, Real>(a, st);
    default: return hipErrorInvalidValue;
  }
}

template <typename Real>
hipError_t affine_space(int space, int p, const GeneralArgs& a, hipStream_t st) {
  switch (space) {
    case SP_H1: return affine_p<SP_H1, Real>(p, a, st);
    case SP_HCURL: return affine_p<SP_HCURL, Real>(p, a, st);
    case SP_HDIV: return affine_p<SP_HDIV, Real>(p, a, st);
    case SP_L2: return affine_p<SP_L2, Real>(p, a, st);
    default: return hipErrorInvalidValue;
  }
}

}  // namespace

hipError_t launch_affine(int space, int p, int prec, const GeneralArgs& a, hipStream_t st) {
  return prec ? affine_space<float>(space, p, a, st) : affine_space<double>(space, p, a, st);
}

}  // namespace dpg
