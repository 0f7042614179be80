// gram_extruded.hip -- O(p^6) path for extruded elements.
//
// Section 2.8.1, second form of (2.89): when x1 = x1_0 + lambda1 xi1 and (x2, x3)
// depend on (xi2, xi3) only, J, D = J^-1 J^-T and C = J^T J do not depend on xi1,
// so the xi1 integral of every term is the exact 1D integral F^{r1 s1} (2.90) of
// the chart, and only xi2, xi3 need quadrature.  Algorithm 11 writes this for L2
// (nest the xi3 integral inside the xi2 integral, then multiply by the xi1
// factor); the paper notes the extension to the other spaces, which this kernel
// implements with the term tables of terms.h.  For block (a, b) and slab j3:
//
//   K_g[i3][j2][i2] = sum_{terms t in group g} sign_t w_t
//                     sum_m T^<r2>_{i2+sa2}(z_m) T^<s2>_{j2+sb2}(z_m)
//                     sum_n c_t(z_m, z_n) w_m w_n T^<r3>_{i3+sa3}(z_n) T^<s3>_{j3+sb3}(z_n)
//   G[(i1,i2,i3), (j1,j2,j3)] = sum_g F^{g}_{i1+sa1, j1+sb1} K_g[i3][j2][i2]
//
// where a group g collects the terms of one (r1, s1).  The fields c_t come from
// the full 3 x 3 Jacobian (lambda1 included); the terms whose field couples xi1
// with xi2 or xi3 vanish on these maps and are dropped (make_ext_plan).
//
// Work decomposition: the column slabs of the general path.  Per slab and block
// (a, b), a <= b, the workgroup evaluates the fields at the L^2 points (FP64) and
// contracts xi3 then xi2 into K (FP64, stored once in the output precision) in
// LDS; with the K of every block resident, the four waves stream the slab's
// packed columns whole, across the components, 64 consecutive entries per store.
// Only F K products remain per output entry, so the kernel is bound by the HBM
// writes, like the constant-Jacobian path.
#include <hip/hip_runtime.h>

#include <utility>

#include "kernels.h"
#include "metric.h"
#include "terms.h"

namespace dpg {

namespace {

constexpr int NT_EXT = 256;

template <int S, int P> struct XShape {
  static constexpr int NC = ncomp(S);
  static constexpr int L = npoints(S, P);
  static constexpr int R(int a, int d) { return range1d(S, P, a, d); }
  static constexpr int SH(int a, int d) { return shift1d(S, a, d); }
  static constexpr int OFF(int a) { return comp_off(S, P, a); }
  static constexpr int slab0(int b) {
    int o = 0;
    for (int c = 0; c < b; ++c) o += R(c, 2);
    return o;
  }
  static constexpr int NSLAB = slab0(NC);
  template <typename F> static constexpr int over(F f) {
    int m = 0;
    for (int a = 0; a < NC; ++a)
      for (int b = a; b < NC; ++b) m = f(a, b) > m ? f(a, b) : m;
    return m;
  }
  static constexpr int NF = over([](int a, int b) { return make_ext_plan(S, a, b).nf; });
  static constexpr int NT = over([](int a, int b) { return make_ext_plan(S, a, b).nt; });
  static constexpr int NG = over([](int a, int b) { return make_ext_plan(S, a, b).ng; });
  static constexpr int R3 = over([](int a, int) { return range1d(S, P, a, 2); });
  // K of block (a, b) and its offset among the blocks a' <= b of component b
  static constexpr int KSZ(int a, int b) {
    return make_ext_plan(S, a, b).ng * range1d(S, P, a, 2) * range1d(S, P, b, 1) * range1d(S, P, a, 1);
  }
  static constexpr int KOFF(int a, int b) {
    int o = 0;
    for (int c = 0; c < a; ++c) o += KSZ(c, b);
    return o;
  }
  static constexpr int K_LEN = [] {
    int m = 0;
    for (int b = 0; b < NC; ++b) m = KOFF(b + 1, b) > m ? KOFF(b + 1, b) : m;
    return m;
  }();
};

template <int S, int A, int B> struct XPlan {
  static constexpr Plan PL = make_ext_plan(S, A, B);
};

template <int N, typename F>
__device__ __forceinline__ void sfor(F&& f) {
  [&]<int... I>(std::integer_sequence<int, I...>) {
    (f(std::integral_constant<int, I>{}), ...);
  }(std::make_integer_sequence<int, N>{});
}

struct XSmem {
  const double* T;   // [2][KT][L] FP64 1D tables
  const double* z;
  const double* w;
  const double* X;   // this element's geometry
  double* fld;       // [NF][L][L] weighted fields of the block
  double* A;         // [NT][R3][L] xi3 contractions
  int* bad;
};

// K of block (a, b) for slab j3 into sK ([g][i3][j2][i2]); sets *bad when |J| <= 0
// at a quadrature point.
template <int S, int P, typename Real, int A, int B>
__device__ __forceinline__ void build_k(const GeneralArgs& ga, const XSmem& sm, int j3, Real* sK) {
  using Sh = XShape<S, P>;
  using XP = XPlan<S, A, B>;   // static members: lambdas capture nothing of the plan
  constexpr int L = Sh::L, L2 = L * L, KTL = KT * L;
  constexpr int R2a = Sh::R(A, 1), R2b = Sh::R(B, 1), R3a = Sh::R(A, 2);
  const int tid = threadIdx.x;
  // weighted coefficient fields at the (xi2, xi3) points, layout [f][m][n]
  for (int pt = tid; pt < L2; pt += NT_EXT) {
    const int m = pt / L, n = pt % L;
    double J[3][3], adj[3][3];
    jacobian_at(2, sm.X, 0.5, sm.z[m], sm.z[n], J);
    const double det = adjugate(J, adj);
    if (!(det > 0.0)) *sm.bad = 1;
    const double idet = 1.0 / det;
    const double wq = sm.w[m] * sm.w[n];
    sfor<XP::PL.nf>([&](auto F) {
      constexpr int f = decltype(F)::value;
      constexpr int fid = XP::PL.fid[f];
      sm.fld[f * L2 + pt] = field_value(fid, J, adj, det, idet) * wq * (field_weight(S, fid) ? ga.w1 : ga.w0);
    });
  }
  __syncthreads();
  // xi3: A_t[i3][m] = sum_n c_t(m, n) T^<r3>_{i3+sa3}(z_n) T^<s3>_{j3+sb3}(z_n)
  for (int it = tid; it < XP::PL.nt * R3a * L; it += NT_EXT) {
    const int m = it % L, i3 = (it / L) % R3a, t = it / (L * R3a);
    double acc = 0.0;
    sfor<XP::PL.nt>([&](auto TT) {
      constexpr int tt = decltype(TT)::value;
      if (t != tt) return;
      const double* ti = sm.T + XP::PL.t[tt].r[2] * KTL + (i3 + Sh::SH(A, 2)) * L;
      const double* tj = sm.T + XP::PL.t[tt].s[2] * KTL + (j3 + Sh::SH(B, 2)) * L;
      const double* c = sm.fld + XP::PL.tf[tt] * L2 + m * L;
#pragma unroll
      for (int n = 0; n < L; ++n) acc += c[n] * ti[n] * tj[n];
      acc *= double(XP::PL.t[tt].sign);
    });
    sm.A[(t * Sh::R3 + i3) * L + m] = acc;
  }
  __syncthreads();
  // xi2: K_g[i3][j2][i2] = sum_{t in g} sum_m A_t[i3][m] T^<r2>_{i2+sa2}(z_m) T^<s2>_{j2+sb2}(z_m)
  for (int it = tid; it < XP::PL.ng * R3a * R2b * R2a; it += NT_EXT) {
    const int i2 = it % R2a, j2 = (it / R2a) % R2b, i3 = (it / (R2a * R2b)) % R3a, g = it / (R2a * R2b * R3a);
    double acc = 0.0;
    sfor<XP::PL.nt>([&](auto TT) {
      constexpr int tt = decltype(TT)::value;
      if (XP::PL.qg[XP::PL.tq[tt]] != g) return;
      const double* ti = sm.T + XP::PL.t[tt].r[1] * KTL + (i2 + Sh::SH(A, 1)) * L;
      const double* tj = sm.T + XP::PL.t[tt].s[1] * KTL + (j2 + Sh::SH(B, 1)) * L;
      const double* a = sm.A + (tt * Sh::R3 + i3) * L;
#pragma unroll
      for (int m = 0; m < L; ++m) acc += a[m] * ti[m] * tj[m];
    });
    sK[it] = static_cast<Real>(acc);
  }
  __syncthreads();
}

// Packed columns of slab (B, j3), whole: wave w takes the columns c = w, w + 4, ...;
// its lanes walk the rows 0..J contiguously, across the components A <= B, whose
// K blocks are all resident.
template <int S, int P, typename Real, int B>
__device__ __forceinline__ void stream_cols(const Real* sF, const Real* sK, int j3, Real* __restrict__ outp) {
  using Sh = XShape<S, P>;
  constexpr int R1b = Sh::R(B, 0), R2b = Sh::R(B, 1);
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  for (int c = wave; c < R1b * R2b; c += 4) {
    const int j1 = c % R1b, j2 = c / R1b;
    const int J = Sh::OFF(B) + R1b * R2b * j3 + c;
    Real* col = outp + int64_t(J) * (J + 1) / 2;
    const int b1 = j1 + Sh::SH(B, 0);
    for (int I = lane; I <= J; I += 64) {
      Real v = Real(0);
      sfor<B + 1>([&](auto AA) {
        constexpr int A = decltype(AA)::value;
        using XP = XPlan<S, A, B>;   // static members: nothing of the plan is captured
        constexpr int R1a = Sh::R(A, 0), R2a = Sh::R(A, 1), R3a = Sh::R(A, 2);
        if (I < Sh::OFF(A) || I >= Sh::OFF(A + 1)) return;
        const int loc = I - Sh::OFF(A);
        const int i1 = loc % R1a, i2 = (loc / R1a) % R2a, i3 = loc / (R1a * R2a);
        const int a1 = i1 + Sh::SH(A, 0);
        constexpr int ko = Sh::KOFF(A, B);   // constexpr: evaluated by the compiler, not per row
        const Real* k = sK + ko;
        sfor<XP::PL.ng>([&](auto GG) {
          constexpr int g = decltype(GG)::value;
          constexpr int tab = 2 * XP::PL.gr1[g] + XP::PL.gs1[g];
          const Real f = sF[(tab * KT + a1) * KT + b1];
          v += f * k[((g * R3a + i3) * R2b + j2) * R2a + i2];
        });
      });
      col[I] = v;
    }
  }
}

template <int S, int P, typename Real, bool LISTED>
__global__ void __launch_bounds__(NT_EXT) k_extruded(GeneralArgs ga) {
  using Sh = XShape<S, P>;
  constexpr int L = Sh::L;
  __shared__ Real s_F[FTAB_LEN];
  __shared__ double s_T[2 * KT * L];
  __shared__ double s_z[L], s_w[L], s_X[10];
  __shared__ double s_fld[Sh::NF * L * L];
  __shared__ double s_A[Sh::NT * Sh::R3 * L];
  __shared__ Real s_K[Sh::K_LEN];
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
    for (int i = tid; i < FTAB_LEN; i += NT_EXT) s_F[i] = fR[i];
    for (int i = tid; i < 2 * KT * L; i += NT_EXT) s_T[i] = ga.tab64[2 * L + i];
    if (tid < L) { s_z[tid] = ga.tab64[tid]; s_w[tid] = ga.tab64[L + tid]; }
    if (tid < 10) s_X[tid] = ga.geom[e * 10 + tid];
    if (tid == 0) s_bad = 0;
    __syncthreads();

    const XSmem sm{s_T, s_z, s_w, s_X, s_fld, s_A, &s_bad};
    Real* outp = static_cast<Real*>(ga.out) + (ga.out_offset ? ga.out_offset[e] : e * ga.packed_len);
    bool bad = false;
    for (int s = s_lo; s < s_hi && !bad; ++s) {
      sfor<Sh::NC>([&](auto BB) {
        constexpr int b = decltype(BB)::value;
        if (bad || s < Sh::slab0(b) || s >= Sh::slab0(b) + Sh::R(b, 2)) return;
        const int j3 = s - Sh::slab0(b);
        sfor<b + 1>([&](auto AA) {
          constexpr int a = decltype(AA)::value;
          constexpr int ko = Sh::KOFF(a, b);
          build_k<S, P, Real, a, b>(ga, sm, j3, s_K + ko);
        });
        bad = s_bad != 0;   // uniform: read after the barrier that closes the last build_k
        if (!bad) stream_cols<S, P, Real, b>(s_F, s_K, j3, outp);
        __syncthreads();    // s_K and the field buffers are rebuilt for the next slab
      });
    }
    if (bad) {
      // |J| <= 0 somewhere: the element's output is zero (every slab group clears its columns)
      const int lane = tid & 63, wave = tid >> 6;
      sfor<Sh::NC>([&](auto BB) {
        constexpr int b = decltype(BB)::value;
        constexpr int w = Sh::R(b, 0) * Sh::R(b, 1);
        for (int s = s_lo; s < s_hi; ++s) {
          if (s < Sh::slab0(b) || s >= Sh::slab0(b) + Sh::R(b, 2)) continue;
          const int J0 = Sh::OFF(b) + (s - Sh::slab0(b)) * w;
          for (int J = J0 + wave; J < J0 + w; J += 4) {
            Real* col = outp + int64_t(J) * (J + 1) / 2;
            for (int I = lane; I <= J; I += 64) col[I] = Real(0);
          }
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
hipError_t launch_extruded_one(const GeneralArgs& a, hipStream_t st) {
  constexpr int NS = XShape<S, P>::NSLAB;
  GeneralArgs c = a;
  c.slab_group = slab_group_for(NS, a.n_items, a.slab_group);
  const int ngroups = (NS + c.slab_group - 1) / c.slab_group;
  if (a.list) {
    hipLaunchKernelGGL((k_extruded<S, P, Real, true>), dim3(list_grid(a.n_items, ngroups)), dim3(NT_EXT), 0, st, c);
    return hipGetLastError();
  }
  const int64_t max_items = launch_items(ngroups);
  for (int64_t base = 0; base < a.n_items; base += max_items) {
    c.item_base = a.item_base + base;
    c.n_items = (a.n_items - base) < max_items ? (a.n_items - base) : max_items;
    hipLaunchKernelGGL((k_extruded<S, P, Real, false>), dim3(unsigned(c.n_items * ngroups)), dim3(NT_EXT), 0, st, c);
  }
  return hipGetLastError();
}

template <int S, typename Real>
hipError_t extruded_p(int p, const GeneralArgs& a, hipStream_t st) {
  switch (p) {
    case 1: return launch_extruded_one<S, 1, Real>(a, st);
    case 2: return launch_extruded_one<S, 2, Real>(a, st);
    case 3: return launch_extruded_one<S, 3, Real>(a, st);
    case 4: return launch_extruded_one<S, 4, Real>(a, st);
    case 5: return launch_extruded_one<S, 5, Real>(a, st);
    case 6: return launch_extruded_one<S, 6, Real>(a, st);
    case 7: return launch_extruded_one<S, 7, Real>(a, st);
    case 8: return launch_extruded_one<S, 8, Real>(a, st);
    case 9: return launch_extruded_one<S, 9, Real>(a, st);
    case 10: return launch_extruded_one<S, 10, Real>(a, st);
    case 11: return launch_extruded_one<S, 11, Real>(a, st);
    default: return hipErrorInvalidValue;
  }
}

template <typename Real>
hipError_t extruded_space(int space, int p, const GeneralArgs& a, hipStream_t st) {
  switch (space) {
    case SP_H1: return extruded_p<SP_H1, Real>(p, a, st);
    case SP_HCURL: return extruded_p<SP_HCURL, Real>(p, a, st);
    case SP_HDIV: return extruded_p<SP_HDIV, Real>(p, a, st);
    case SP_L2: return extruded_p<SP_L2, Real>(p, a, st);
    default: return hipErrorInvalidValue;
  }
}

}  // namespace

hipError_t launch_extruded(int space, int p, int prec, const GeneralArgs& a, hipStream_t s) {
  return prec ? extruded_space<float>(space, p, a, s) : extruded_space<double>(space, p, a, s);
}

}  // namespace dpg
