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
// Work decomposition: the same column-slab groups as the general path.  Each
// wave takes one packed column J at a time; its 64 lanes walk the rows I = 0..J,
// so every store instruction writes 64 consecutive entries.  The F tables are
// banded (|i - j| <= 2 unless both indices are <= 3), so most entries are exact
// zeros: whole direction-3 planes outside the band are written as zeros without
// decoding, and the direction-3 factor of each term is hoisted per plane.
#include <hip/hip_runtime.h>

#include <utility>

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
  static constexpr int slab0(int b) {
    int o = 0;
    for (int c = 0; c < b; ++c) o += R(c, 2);
    return o;
  }
  static constexpr int NSLAB = slab0(NC);
};

template <int S, int A, int B> struct APlan {
  static constexpr Plan PL = make_plan(S, A, B);
};

template <int N, typename F>
__device__ __forceinline__ void sfor(F&& f) {
  [&]<int... I>(std::integer_sequence<int, I...>) {
    (f(std::integral_constant<int, I>{}), ...);
  }(std::make_integer_sequence<int, N>{});
}

// Value of row I of column J = (b; j1, j2, j3) when I lies in component A
// (loc = I - OFF(A)): sum over the block's terms of coef * F1 F2 F3, zero
// outside the band of any direction.
template <int S, int P, typename Real, int A, int B>
__device__ __forceinline__ Real entry(const Real* sF, const Real* coef, int loc, int b1, int b2, int b3) {
  using Sh = AShape<S, P>;
  constexpr Plan PL = APlan<S, A, B>::PL;
  constexpr int R1a = Sh::R(A, 0), R2a = Sh::R(A, 1);
  const int i1 = loc % R1a, t12 = loc / R1a;
  const int i2 = t12 % R2a, i3 = t12 / R2a;
  const int a1 = i1 + Sh::SH(A, 0), a2 = i2 + Sh::SH(A, 1), a3 = i3 + Sh::SH(A, 2);
  Real v = Real(0);
  if (band(a1, b1) && band(a2, b2) && band(a3, b3)) {
    sfor<PL.nt>([&](auto T) {
      constexpr int t = decltype(T)::value;
      const Real f1 = sF[((2 * PL.t[t].r[0] + PL.t[t].s[0]) * KT + a1) * KT + b1];
      const Real f2 = sF[((2 * PL.t[t].r[1] + PL.t[t].s[1]) * KT + a2) * KT + b2];
      const Real f3 = sF[((2 * PL.t[t].r[2] + PL.t[t].s[2]) * KT + a3) * KT + b3];
      v += coef[t] * f1 * f2 * f3;
    });
  }
  return v;
}

// Column J = (b; j1, j2, j3): rows 0..J, walked contiguously (64 consecutive
// entries per store instruction across planes and components).
template <int S, int P, typename Real, int B>
__device__ __forceinline__ void column(const Real* sF, const Real (*sC)[3][10], int J, int j1, int j2, int j3,
                                       Real* __restrict__ col, int lane) {
  using Sh = AShape<S, P>;
  const int b1 = j1 + Sh::SH(B, 0), b2 = j2 + Sh::SH(B, 1), b3 = j3 + Sh::SH(B, 2);
  for (int I = lane; I <= J; I += 64) {
    Real v = Real(0);
    sfor<B + 1>([&](auto AA) {
      constexpr int a = decltype(AA)::value;
      constexpr int lo = Sh::OFF(a), hi = Sh::OFF(a + 1);
      if (I >= lo && I < hi) v = entry<S, P, Real, a, B>(sF, &sC[a][B][0], I - lo, b1, b2, b3);
    });
    col[I] = v;
  }
}

template <int S, int P, typename Real, bool LISTED>
__global__ void __launch_bounds__(NT_AFF) k_affine(GeneralArgs ga) {
  using Sh = AShape<S, P>;
  __shared__ Real s_F[FTAB_LEN];
  __shared__ Real s_C[3][3][10];   // term coefficients of block (a, b)
  __shared__ int s_bad;
  const int tid = threadIdx.x;
  const int G = ga.slab_group;
  const int ngroups = (Sh::NSLAB + G - 1) / G;
  // one (item, slab group) of the launch
  auto run = [&](int64_t blk, int64_t n_items, const int32_t* ids) {
    const int grp = ngroups - 1 - int(blk / n_items);
    const int64_t item = ga.item_base + blk % n_items;
    const int64_t e = ids ? int64_t(ids[item]) : item;
    const int s_lo = grp * G, s_hi = (s_lo + G < Sh::NSLAB) ? s_lo + G : Sh::NSLAB;

    const Real* fR = static_cast<const Real*>(ga.ftabR);
    for (int i = tid; i < FTAB_LEN; i += NT_AFF) s_F[i] = fR[i];
    if (tid < 32) {
      // every one of these threads evaluates the constant metric; thread 3 a + b
      // writes the coefficients of block (a, b)
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
      if (tid == 0) s_bad = !(det > 0.0);
      auto fv = [&](int f) -> double {
        if (f == FLD_DETJ) return det;
        if (f == FLD_IDETJ) return idet;
        if (fld_is_D(f)) {
          const int s = f - FLD_D11, a = sym_a(s), bb = sym_b(s);
          return (adj[a][0] * adj[bb][0] + adj[a][1] * adj[bb][1] + adj[a][2] * adj[bb][2]) * idet;
        }
        const int s = f - FLD_C11, a = sym_a(s), bb = sym_b(s);
        return (J[0][a] * J[0][bb] + J[1][a] * J[1][bb] + J[2][a] * J[2][bb]) * idet;
      };
      sfor<Sh::NC>([&](auto AA) {
        constexpr int a = decltype(AA)::value;
        sfor<Sh::NC>([&](auto BB) {
          constexpr int bb = decltype(BB)::value;
          if constexpr (a <= bb) {
            if (tid == 3 * a + bb) {
              constexpr Plan PL = APlan<S, a, bb>::PL;
              sfor<10>([&](auto T) {
                constexpr int t = decltype(T)::value;
                double c = 0.0;
                if constexpr (t < PL.nt)
                  c = PL.t[t].sign * fv(PL.t[t].field) * (field_weight(S, PL.t[t].field) ? ga.w1 : ga.w0);
                s_C[a][bb][t] = static_cast<Real>(c);
              });
            }
          }
        });
      });
    }
    __syncthreads();
    Real* outp = static_cast<Real*>(ga.out) + (ga.out_offset ? ga.out_offset[e] : e * ga.packed_len);
    const bool bad = s_bad != 0;
    const int lane = tid & 63, wave = tid >> 6;

    // Columns of the slab group form one contiguous packed range [J0, J1).
    // Each wave takes a contiguous run of columns holding about a quarter of the
    // range's entries, so neighbouring columns are written back to back by the
    // same wave.
    auto colstart = [&](int slab) {   // first column J of a slab (or the end)
      int o = 0;
      int J = 0;
      sfor<Sh::NC>([&](auto CC) {
        constexpr int c = decltype(CC)::value;
        constexpr int n = Sh::R(c, 2), w = Sh::R(c, 0) * Sh::R(c, 1);
        if (slab >= o && slab < o + n) J = Sh::OFF(c) + (slab - o) * w;
        o += n;
      });
      return slab >= Sh::NSLAB ? int(Sh::OFF(Sh::NC)) : J;
    };
    const int J0 = colstart(s_lo), J1 = colstart(s_hi);
    const double E0 = 0.5 * double(J0) * (J0 + 1), E1 = 0.5 * double(J1) * (J1 + 1);
    // first column whose entries start at or after packed offset e: J (J+1)/2 >= e
    auto col_at = [&](double e) {
      int J = int(floor((sqrt(8.0 * e + 1.0) - 1.0) * 0.5));
      while (0.5 * double(J) * (J + 1) < e) ++J;
      while (J > 0 && 0.5 * double(J - 1) * J >= e) --J;
      return J < J0 ? J0 : (J > J1 ? J1 : J);
    };
    const int Jw0 = wave == 0 ? J0 : col_at(E0 + (E1 - E0) * wave / 4.0);
    const int Jw1 = wave == 3 ? J1 : col_at(E0 + (E1 - E0) * (wave + 1) / 4.0);
    for (int J = Jw0; J < Jw1; ++J) {
      Real* col = outp + int64_t(J) * (J + 1) / 2;
      if (bad) {
        for (int I = lane; I <= J; I += 64) col[I] = Real(0);
        continue;
      }
      sfor<Sh::NC>([&](auto BB) {
        constexpr int b = decltype(BB)::value;
        constexpr int R1b = Sh::R(b, 0), R2b = Sh::R(b, 1);
        if (J >= Sh::OFF(b) && J < Sh::OFF(b + 1)) {
          const int c = J - Sh::OFF(b);
          const int j3 = c / (R1b * R2b), r = c % (R1b * R2b);
          column<S, P, Real, b>(s_F, s_C, J, r % R1b, r / R1b, j3, col, lane);
        }
      });
    }
    if (ga.status && tid == 0 && (bad || s_lo == 0)) ga.status[e] = bad ? -4 : 0;
  };
  if constexpr (LISTED) {
    // a listed launch: the item count and the first list entry come from the device,
    // and the workgroups stride over the (item, slab group) pairs
    const int64_t n_items = ga.list[0];
    const int32_t* ids = ga.elem_ids + ga.list[1];
    for (int64_t blk = blockIdx.x; blk < n_items * ngroups; blk += gridDim.x) {
      run(blk, n_items, ids);
      __syncthreads();   // the next item rewrites the shared buffers
    }
  } else {
    run(blockIdx.x, ga.n_items, ga.elem_ids);   // one workgroup per (item, slab group)
  }
}

template <int S, int P, typename Real>
hipError_t launch_affine_one(const GeneralArgs& a, hipStream_t st) {
  constexpr int NS = AShape<S, P>::NSLAB;
  GeneralArgs c = a;
  c.slab_group = slab_group_for(NS, a.n_items, a.slab_group);
  const int ngroups = (NS + c.slab_group - 1) / c.slab_group;
  if (a.list) {
    hipLaunchKernelGGL((k_affine<S, P, Real, true>), dim3(list_grid(a.n_items, ngroups)), dim3(NT_AFF), 0, st, c);
    return hipGetLastError();
  }
  const int64_t max_items = launch_items(ngroups);
  for (int64_t base = 0; base < a.n_items; base += max_items) {
    c.item_base = a.item_base + base;
    c.n_items = (a.n_items - base) < max_items ? (a.n_items - base) : max_items;
    hipLaunchKernelGGL((k_affine<S, P, Real, false>), dim3(unsigned(c.n_items * ngroups)), dim3(NT_AFF), 0, st, c);
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
