// gram_general.inc.h -- sum-factorised Gram integration on gfx950.
//
// Work decomposition.  The packed 'U' output of one element is cut into
// column slabs: slab (b, j3) holds the columns J of component b with
// direction-3 index j3.  Its packed entries form ONE contiguous range of the
// output, and its rows are the pairs ((a, i3), (b, j3)) with a < b, or a == b
// and i3 <= j3.  One workgroup (256 threads = 4 wave64) integrates one slab
// of one element:
//
//   per block (a, b):  metric -> coefficient fields c_f(l, m, n) in LDS (FP64
//                      evaluation, weights w_l w_m w_n and w0/w1 folded in);
//   per pair (i3, j3): stage 3  A_q(l, m)     = sum_n c(l,m,n) T_i3(n) T_j3(n)      (VALU)
//                      stage 2  B_g(l, i2j2)  = sum_q sum_m T_i2(m) T_j2(m) A_q(l,m) (VALU)
//                      stage 1  G(i1i2, j1j2) = sum_g sum_l T_i1(l) T_j1(l) B_g(l,i2j2)
//                               as an MFMA GEMM: rows (i2,j2) from LDS, columns
//                               (i1,j1) built from the 1D tables, K = (g, l);
//                               results stored straight from the accumulators.
//
// This is the staged evaluation of (2.23)-(2.25) / (2.38)-(2.43) /
// (2.61)-(2.63) / (2.78)-(2.83), with the geometry evaluated once per point
// per block (the hoisting of Algorithm 3 / Remark 2.2) and the (i3, j3) loop
// outermost (Remark 2.1), so the auxiliary arrays never carry i3, j3.
// Diagonal pairs (a == b, i3 == j3) only form i2 <= j2 (and i1 <= j1 when
// i2 == j2): the symmetry of the Gram matrix used by fillsymmetric.
//
// MFMA operand layout (v_mfma_*_16x16x4): lane = i + 16 k holds A[i][k] and
// B[k][j = i].  Row i of the A operand carries x = xbase + Mma::arow(i), chosen
// so that accumulator register r of lane groups 0..3 holds four CONSECUTIVE
// x = (i2, j2): consecutive i2 at fixed j2 are consecutive rows I of one packed
// column, so a store instruction writes runs of 4 R1 values.
#pragma once
#include <hip/hip_runtime.h>

#include "kernels.h"
#include "terms.h"

namespace dpg {

typedef double v4d __attribute__((ext_vector_type(4)));
typedef float v4f __attribute__((ext_vector_type(4)));

template <typename Real> struct Mma;
// Accumulator register r of lane (g = lane/16, j = lane%16) holds C[row][j] with
// row = g + 4 r for the f64 instruction and row = 4 g + r for the f32 one
// (both checked on gfx950).  arow(i) is the x offset that A-operand row i must
// carry so that register r of lane group g always holds x offset g + 4 r.
template <> struct Mma<double> {
  typedef v4d acc;
  static __device__ __forceinline__ acc mac(double a, double b, acc c) {
    return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
  }
  static __device__ __forceinline__ int arow(int i) { return i; }
};
template <> struct Mma<float> {
  typedef v4f acc;
  static __device__ __forceinline__ acc mac(float a, float b, acc c) {
    return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
  }
  static __device__ __forceinline__ int arow(int i) { return (i >> 2) + 4 * (i & 3); }
};

constexpr int NTHREADS = 256;
constexpr int ru16(int x) { return (x + 15) / 16 * 16; }
constexpr int imax(int a, int b) { return a > b ? a : b; }
constexpr int imin(int a, int b) { return a < b ? a : b; }

template <int S, int P> struct Shape {
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
};

template <int S, int P, typename Real> struct Lds {
  using Sh = Shape<S, P>;
  static constexpr int L = Sh::L;
  static constexpr int NF = [] {
    int m = 0;
    for (int a = 0; a < Sh::NC; ++a)
      for (int b = a; b < Sh::NC; ++b) m = imax(m, make_plan(S, a, b).nf);
    return m;
  }();
  static constexpr int NQ = [] {
    int m = 0;
    for (int a = 0; a < Sh::NC; ++a)
      for (int b = a; b < Sh::NC; ++b) m = imax(m, make_plan(S, a, b).nq);
    return m;
  }();
  static constexpr int NG = [] {
    int m = 0;
    for (int a = 0; a < Sh::NC; ++a)
      for (int b = a; b < Sh::NC; ++b) m = imax(m, make_plan(S, a, b).ng);
    return m;
  }();
  static constexpr int NXP = [] {
    int m = 0;
    for (int a = 0; a < Sh::NC; ++a)
      for (int b = a; b < Sh::NC; ++b) m = imax(m, ru16(Sh::R(a, 1) * Sh::R(b, 1)));
    return m;
  }();
  static constexpr int FLD_LEN = NF * L * L * L;
  static constexpr int A_LEN = NQ * L * L;
  static constexpr int T_LEN = 2 * KT * L;
  static constexpr int BUDGET = 150 * 1024;
  static constexpr int bytes(int xch) {
    return int(sizeof(Real)) * (FLD_LEN + A_LEN + T_LEN + NG * L * xch) + 8 * (2 * L + 24) + 256;
  }
  // x-chunk width of stages 2/1: as wide as possible within the LDS budget
  static constexpr int XCH = [] {
    int x = NXP;
    while (x > 16 && bytes(x) > BUDGET) x -= 16;
    return x;
  }();
  static_assert(bytes(XCH) <= BUDGET, "LDS budget exceeded");
  static constexpr int B_LEN = NG * L * XCH;
};

struct SmemPtrs {
  void* fld;
  void* A;
  void* B;
  void* T;
  double* z;
  double* w;
  double* X;
  unsigned char* xd;
  int* bad;
};

// ---------------------------------------------------------------------------
// geometry
// ---------------------------------------------------------------------------

__device__ __forceinline__ void jacobian_at(int kind, const double* X, double x1, double x2, double x3,
                                            double J[3][3]) {
  if (kind == 1) {
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
      for (int j = 0; j < 3; ++j) J[i][j] = X[3 + 3 * i + j];
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

// ---------------------------------------------------------------------------
// one block (a, b) of one column slab
// ---------------------------------------------------------------------------

template <int S, int P, typename Real, int A, int B, bool DIAG>
__device__ __forceinline__ void pair21(const SmemPtrs& sm, int i3, int j3, Real* __restrict__ outp) {
  using Sh = Shape<S, P>;
  using LD = Lds<S, P, Real>;
  using M = Mma<Real>;
  constexpr Plan PL = make_plan(S, A, B);
  constexpr int L = Sh::L, L2 = L * L;
  constexpr int R1a = Sh::R(A, 0), R1b = Sh::R(B, 0), R2a = Sh::R(A, 1), R2b = Sh::R(B, 1);
  constexpr int R3a = Sh::R(A, 2);
  constexpr int NX = DIAG ? R2a * (R2a + 1) / 2 : R2a * R2b;
  constexpr int NXP = ru16(NX);
  constexpr int XCH = imin(LD::XCH, NXP);
  constexpr int NCH = (NXP + XCH - 1) / XCH;
  constexpr int NY = R1a * R1b;
  constexpr int NYT = (NY + 15) / 16;
  constexpr int NG = PL.ng, NQ = PL.nq;
  constexpr int K = NG * L;
  constexpr int KS = (K + 3) / 4;
  constexpr int NGRP = imax(1, NTHREADS / XCH);
  constexpr int LPT = (L + NGRP - 1) / NGRP;
  constexpr int XB = 4;
  constexpr int KTL = KT * L;

  const Real* sT = static_cast<const Real*>(sm.T);
  const Real* sA = static_cast<const Real*>(sm.A);
  Real* sB = static_cast<Real*>(sm.B);
  const int tid = threadIdx.x;
  const int lane = tid & 63, wave = tid >> 6;
  const int lr = lane & 15, lk = lane >> 4;

  for (int ch = 0; ch < NCH; ++ch) {
    const int xc = ch * XCH;
    if (ch > 0) __syncthreads();
    // ---------------- stage 2 ----------------
    {
      const int sl = tid % XCH, lg = tid / XCH;
      if (lg < NGRP) {
        const int s = xc + sl;
        Real acc[NG][LPT];
#pragma unroll
        for (int g = 0; g < NG; ++g)
#pragma unroll
          for (int li = 0; li < LPT; ++li) acc[g][li] = Real(0);
        if (s < NX) {
          int i2, j2;
          if (DIAG) { i2 = sm.xd[2 * s]; j2 = sm.xd[2 * s + 1]; }
          else { i2 = s % R2a; j2 = s / R2a; }
          const int ki = i2 + Sh::SH(A, 1), kj = j2 + Sh::SH(B, 1);
#pragma unroll 2
          for (int m = 0; m < L; ++m) {
            const Real ti0 = sT[ki * L + m], ti1 = sT[KTL + ki * L + m];
            const Real tj0 = sT[kj * L + m], tj1 = sT[KTL + kj * L + m];
            const Real u00 = ti0 * tj0, u01 = ti0 * tj1, u10 = ti1 * tj0, u11 = ti1 * tj1;
#pragma unroll
            for (int li = 0; li < LPT; ++li) {
              const int l = lg + li * NGRP;
              if (LPT * NGRP == L || l < L) {
#pragma unroll
                for (int q = 0; q < NQ; ++q) {
                  const Real u = PL.qr2[q] ? (PL.qs2[q] ? u11 : u10) : (PL.qs2[q] ? u01 : u00);
                  acc[PL.qg[q]][li] += u * sA[q * L2 + l * L + m];
                }
              }
            }
          }
        }
#pragma unroll
        for (int g = 0; g < NG; ++g)
#pragma unroll
          for (int li = 0; li < LPT; ++li) {
            const int l = lg + li * NGRP;
            if (LPT * NGRP == L || l < L) sB[(g * L + l) * XCH + sl] = acc[g][li];
          }
      }
    }
    __syncthreads();
    // ---------------- stage 1 (MFMA) ----------------
    const int XT = imin(XCH, NXP - xc) / 16;
    for (int yt = wave; yt < NYT; yt += 4) {
      const int y = yt * 16 + lr;
      const bool yv = y < NY;
      const int i1 = y % R1a, j1 = y / R1a;
      Real u[KS];
#pragma unroll
      for (int ks = 0; ks < KS; ++ks) {
        const int k = 4 * ks + lk;
        Real v = Real(0);
        if (yv && k < K) {
          const int g = k / L, l = k - g * L;
          int r1 = 0, s1 = 0;
#pragma unroll
          for (int gg = 0; gg < NG; ++gg)
            if (g == gg) { r1 = PL.gr1[gg]; s1 = PL.gs1[gg]; }
          v = sT[r1 * KTL + (i1 + Sh::SH(A, 0)) * L + l] * sT[s1 * KTL + (j1 + Sh::SH(B, 0)) * L + l];
        }
        u[ks] = v;
      }
      const int xrow = M::arow(lr);
      for (int xt0 = 0; xt0 < XT; xt0 += XB) {
        typename M::acc acc[XB];
#pragma unroll
        for (int c = 0; c < XB; ++c) acc[c] = typename M::acc{0, 0, 0, 0};
#pragma unroll
        for (int ks = 0; ks < KS; ++ks) {
          const int k = 4 * ks + lk;
          const bool kv = (K % 4 == 0) || k < K;
#pragma unroll
          for (int c = 0; c < XB; ++c) {
            if (xt0 + c < XT) {
              const Real a = kv ? sB[k * XCH + (xt0 + c) * 16 + xrow] : Real(0);
              acc[c] = M::mac(a, u[ks], acc[c]);
            }
          }
        }
#pragma unroll
        for (int c = 0; c < XB; ++c) {
          if (xt0 + c < XT) {
#pragma unroll
            for (int r = 0; r < 4; ++r) {
              const int s = xc + (xt0 + c) * 16 + lk + 4 * r;
              if (yv && s < NX) {
                int i2, j2;
                if (DIAG) { i2 = sm.xd[2 * s]; j2 = sm.xd[2 * s + 1]; }
                else { i2 = s % R2a; j2 = s / R2a; }
                if (!DIAG || i2 < j2 || i1 <= j1) {
                  const int64_t I = Sh::OFF(A) + i1 + R1a * i2 + R1a * R2a * i3;
                  const int64_t J = Sh::OFF(B) + j1 + R1b * j2 + R1b * R2b * j3;
                  outp[I + J * (J + 1) / 2] = acc[c][r];
                }
              }
            }
          }
        }
      }
    }
  }
  (void)R3a;
}

template <int S, int P, typename Real, int A, int B>
__device__ bool run_block(const GeneralArgs& ga, const SmemPtrs& sm, int j3, Real* __restrict__ outp) {
  using Sh = Shape<S, P>;
  constexpr Plan PL = make_plan(S, A, B);
  constexpr int L = Sh::L, L2 = L * L, L3 = L2 * L;
  constexpr int KTL = KT * L;
  Real* sF = static_cast<Real*>(sm.fld);
  Real* sA = static_cast<Real*>(sm.A);
  const Real* sT = static_cast<const Real*>(sm.T);
  const int tid = threadIdx.x;

  // ---------------- metric -> coefficient fields ----------------
  for (int pt = tid; pt < L3; pt += NTHREADS) {
    const int l = pt / L2, m = (pt / L) % L, n = pt % L;
    double J[3][3], adj[3][3];
    jacobian_at(ga.geom_kind, sm.X, sm.z[l], sm.z[m], sm.z[n], J);
    const double det = adjugate(J, adj);
    if (!(det > 0.0)) *sm.bad = 1;
    const double idet = 1.0 / det;
    const double wq = sm.w[l] * sm.w[m] * sm.w[n];
    const double wv = wq * ga.w0, wd = wq * ga.w1;
#pragma unroll
    for (int f = 0; f < PL.nf; ++f) {
      const double v = field_value(PL.fid[f], J, adj, det, idet) * (field_weight(S, PL.fid[f]) ? wd : wv);
      sF[(f * L + n) * L2 + l * L + m] = static_cast<Real>(v);
    }
  }
  __syncthreads();
  if (*sm.bad) return true;

  const int i3_end = (A == B) ? j3 + 1 : Sh::R(A, 2);
  for (int i3 = 0; i3 < i3_end; ++i3) {
    // ---------------- stage 3 ----------------
    if (tid < L2) {
      Real acc[PL.nq];
#pragma unroll
      for (int q = 0; q < PL.nq; ++q) acc[q] = Real(0);
      const int ka = i3 + Sh::SH(A, 2), kb = j3 + Sh::SH(B, 2);
#pragma unroll 2
      for (int n = 0; n < L; ++n) {
        const Real ti0 = sT[ka * L + n], ti1 = sT[KTL + ka * L + n];
        const Real tj0 = sT[kb * L + n], tj1 = sT[KTL + kb * L + n];
#pragma unroll
        for (int t = 0; t < PL.nt; ++t) {
          Real u = (PL.t[t].r[2] ? ti1 : ti0) * (PL.t[t].s[2] ? tj1 : tj0);
          if (PL.t[t].sign < 0) u = -u;
          acc[PL.tq[t]] += u * sF[(PL.tf[t] * L + n) * L2 + tid];
        }
      }
#pragma unroll
      for (int q = 0; q < PL.nq; ++q) sA[q * L2 + tid] = acc[q];
    }
    __syncthreads();
    if (A == B && i3 == j3) pair21<S, P, Real, A, B, true>(sm, i3, j3, outp);
    else pair21<S, P, Real, A, B, false>(sm, i3, j3, outp);
  }
  __syncthreads();
  return false;
}

template <int S, int P, typename Real>
__global__ void __launch_bounds__(NTHREADS) k_general(GeneralArgs ga) {
  using Sh = Shape<S, P>;
  using LD = Lds<S, P, Real>;
  constexpr int L = Sh::L;
  __shared__ Real s_fld[LD::FLD_LEN];
  __shared__ Real s_A[LD::A_LEN];
  __shared__ Real s_B[LD::B_LEN];
  __shared__ Real s_T[LD::T_LEN];
  __shared__ double s_z[L], s_w[L], s_X[24];
  __shared__ unsigned char s_xd[2 * 80];
  __shared__ int s_bad;

  const int tid = threadIdx.x;
  const int64_t blk = blockIdx.x;
  const int slab = Sh::NSLAB - 1 - int(blk / ga.n_items);     // heaviest slabs first
  const int64_t item = ga.item_base + blk % ga.n_items;
  const int64_t e = ga.elem_ids ? int64_t(ga.elem_ids[item]) : item;

  int b = 0, j3 = slab;
#pragma unroll
  for (int c = 0; c < Sh::NC - 1; ++c)
    if (b == c && j3 >= Sh::R(c, 2)) { j3 -= Sh::R(c, 2); b = c + 1; }

  const Real* tR = static_cast<const Real*>(ga.tabR);
  for (int i = tid; i < LD::T_LEN; i += NTHREADS) s_T[i] = tR[2 * L + i];
  if (tid < L) { s_z[tid] = ga.tab64[tid]; s_w[tid] = ga.tab64[L + tid]; }
  const int ng = ga.geom_kind == 1 ? 12 : 24;
  if (tid < ng) s_X[tid] = ga.geom[e * ng + tid];
  if (tid < 80) {
    // triangular enumeration s = j2 (j2 + 1) / 2 + i2, i2 <= j2
    int j2 = 0;
    while ((j2 + 1) * (j2 + 2) / 2 <= tid) ++j2;
    s_xd[2 * tid] = static_cast<unsigned char>(tid - j2 * (j2 + 1) / 2);
    s_xd[2 * tid + 1] = static_cast<unsigned char>(j2);
  }
  if (tid == 0) s_bad = 0;
  __syncthreads();

  SmemPtrs sm{s_fld, s_A, s_B, s_T, s_z, s_w, s_X, s_xd, &s_bad};
  Real* outp = static_cast<Real*>(ga.out) + (ga.out_offset ? ga.out_offset[e] : e * ga.packed_len);

  bool bad = false;
  if constexpr (Sh::NC == 1) {
    bad = run_block<S, P, Real, 0, 0>(ga, sm, j3, outp);
  } else {
    if (b == 0) {
      bad = run_block<S, P, Real, 0, 0>(ga, sm, j3, outp);
    } else if (b == 1) {
      bad = run_block<S, P, Real, 0, 1>(ga, sm, j3, outp);
      if (!bad) bad = run_block<S, P, Real, 1, 1>(ga, sm, j3, outp);
    } else {
      bad = run_block<S, P, Real, 0, 2>(ga, sm, j3, outp);
      if (!bad) bad = run_block<S, P, Real, 1, 2>(ga, sm, j3, outp);
      if (!bad) bad = run_block<S, P, Real, 2, 2>(ga, sm, j3, outp);
    }
  }
  if (bad) {
    // element with det J <= 0: its whole output is zero (every slab does its part)
    int r1b = Sh::R(0, 0), r2b = Sh::R(0, 1), offb = 0;
#pragma unroll
    for (int c = 1; c < Sh::NC; ++c)
      if (b == c) { r1b = Sh::R(c, 0); r2b = Sh::R(c, 1); offb = Sh::OFF(c); }
    const int64_t J0 = offb + int64_t(r1b) * r2b * j3, J1 = J0 + int64_t(r1b) * r2b;
    for (int64_t i = J0 * (J0 + 1) / 2 + tid; i < J1 * (J1 + 1) / 2; i += NTHREADS) outp[i] = Real(0);
  }
  if (ga.status && tid == 0 && (bad || slab == 0)) ga.status[e] = bad ? -4 : 0;
}

template <int S, int P, typename Real>
hipError_t launch_general_one(const GeneralArgs& a, hipStream_t st) {
  constexpr int NS = Shape<S, P>::NSLAB;
  const int64_t max_items = int64_t(0x7fffffff) / NS;
  GeneralArgs c = a;
  for (int64_t base = 0; base < a.n_items; base += max_items) {
    c.item_base = a.item_base + base;
    c.n_items = (a.n_items - base) < max_items ? (a.n_items - base) : max_items;
    hipLaunchKernelGGL((k_general<S, P, Real>), dim3(unsigned(c.n_items * NS)), dim3(NTHREADS), 0, st, c);
  }
  return hipGetLastError();
}

template <int S, typename Real>
hipError_t dispatch_general_p(int p, const GeneralArgs& a, hipStream_t st) {
  switch (p) {
    case 1: return launch_general_one<S, 1, Real>(a, st);
    case 2: return launch_general_one<S, 2, Real>(a, st);
    case 3: return launch_general_one<S, 3, Real>(a, st);
    case 4: return launch_general_one<S, 4, Real>(a, st);
    case 5: return launch_general_one<S, 5, Real>(a, st);
    case 6: return launch_general_one<S, 6, Real>(a, st);
    case 7: return launch_general_one<S, 7, Real>(a, st);
    case 8: return launch_general_one<S, 8, Real>(a, st);
    case 9: return launch_general_one<S, 9, Real>(a, st);
    case 10: return launch_general_one<S, 10, Real>(a, st);
    case 11: return launch_general_one<S, 11, Real>(a, st);
    default: return hipErrorInvalidValue;
  }
}

template <int S>
hipError_t dispatch_general(int p, int prec, const GeneralArgs& a, hipStream_t st) {
  return prec ? dispatch_general_p<S, float>(p, a, st) : dispatch_general_p<S, double>(p, a, st);
}

}  // namespace dpg
