// gram_general.inc.h -- sum-factorised Gram integration on gfx950.
//
// Work decomposition.  The packed 'U' output of one element is cut into
// column slabs: slab (b, j3) holds the columns J of component b with
// direction-3 index j3.  Its packed entries form ONE contiguous range of the
// output, and its rows are the pairs ((a, i3), (b, j3)) with a < b, or a == b
// and i3 <= j3.  One workgroup (256 threads = 4 wave64) integrates a group of
// consecutive slabs of one element (up to the whole element; the group size is
// chosen on the host so that the launch still fills the GPU).  Per block (a, b):
//
//   metric    coefficient fields c_f(l, m, n) -> LDS (FP64 evaluation of J,
//             |J|, D, C; quadrature weights and w0/w1 folded in; rounded once
//             to the output precision)
//   stage 3   A_q(l, m)     = sum_n  c(l,m,n) T_i3(n) T_j3(n)              VALU
//   stage 2   B_g(l, i2j2)  = sum_q sum_m T_i2(m) T_j2(m) A_q(l, m)         MFMA
//   stage 1   G(i1i2, j1j2) = sum_g sum_l T_i1(l) T_j1(l) B_g(l, i2j2)      MFMA
//
// the staged evaluation of (2.23)-(2.25) / (2.38)-(2.43) / (2.61)-(2.63) /
// (2.78)-(2.83).  The geometry is evaluated once per point per block (the
// hoisting of Algorithm 3 / Remark 2.2) and the (i3, j3) loop is outermost
// (Remark 2.1), so no auxiliary array carries i3, j3.  Diagonal pairs
// (a == b, i3 == j3) only form i2 <= j2, and i1 <= j1 when i2 == j2: the
// symmetry used by fillsymmetric.
//
// Stages 2 and 1 are GEMMs with element-independent left factors built from
// the 1D tables:
//   stage 2: rows (pair, l), columns x = (i2, j2), K = (q, m); NP pairs
//            (i3, i3+1, ...) are batched so that NP*L fills 16 MFMA rows;
//   stage 1: rows x, columns y = (i1, j1), K = (g, l).
// The table factors (MFMA B operands) depend only on the block and on the
// wave's x- or y-tile, so each wave keeps them in registers for the whole
// block; only the element data (A_q, B_g) streams through LDS.
//
// MFMA operand layout (v_mfma_*_16x16x4): lane = i + 16 k holds A[i][k] and
// B[k][j = i].  In stage 1, row i of the A operand carries x = xbase +
// Mma::arow(i), chosen so that accumulator register r of lane group g holds x
// offset g + 4 r: four consecutive x = (i2, j2), i.e. consecutive rows I of one
// packed column, so a store instruction writes runs of 4 R1 values.
#pragma once
#include <hip/hip_runtime.h>

#include <utility>

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
  static __device__ __forceinline__ int crow(int g, int r) { return g + 4 * r; }
};
template <> struct Mma<float> {
  typedef v4f acc;
  static __device__ __forceinline__ acc mac(float a, float b, acc c) {
    return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
  }
  static __device__ __forceinline__ int arow(int i) { return (i >> 2) + 4 * (i & 3); }
  static __device__ __forceinline__ int crow(int g, int r) { return 4 * g + r; }
};

constexpr int NTHREADS = 256;
constexpr int NC2 = 16;    // stage-2 MFMA rows: NP pairs x L points, padded
constexpr int ru16(int x) { return (x + 15) / 16 * 16; }
constexpr int imax(int a, int b) { return a > b ? a : b; }
constexpr int imin(int a, int b) { return a < b ? a : b; }
constexpr int pairs_per_batch(int L) { return imin(4, L <= 16 ? imax(1, 16 / L) : 1); }

// f(std::integral_constant<int, i>) for i = 0 .. N-1, fully unrolled at compile time
template <int N, typename F>
__device__ __forceinline__ void static_for(F&& f) {
  [&]<int... I>(std::integer_sequence<int, I...>) {
    (f(std::integral_constant<int, I>{}), ...);
  }(std::make_integer_sequence<int, N>{});
}

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

// compile-time constants of block (A, B)
template <int S, int P, int A, int B> struct Blk {
  using Sh = Shape<S, P>;
  static constexpr Plan PL = make_plan(S, A, B);
  static constexpr int L = Sh::L;
  static constexpr int NP = pairs_per_batch(L);
  static constexpr int R1a = Sh::R(A, 0), R1b = Sh::R(B, 0), R2a = Sh::R(A, 1), R2b = Sh::R(B, 1);
  static constexpr int R3a = Sh::R(A, 2), R3b = Sh::R(B, 2);
  static constexpr int NY = R1a * R1b, NYT = (NY + 15) / 16;
  static constexpr int NX = R2a * R2b, NXP = ru16(NX);
  static constexpr int NXD = R2a * (R2a + 1) / 2, NXDP = ru16(NXD);
  static constexpr int NG = make_plan(S, A, B).ng;
  static constexpr int NQ = make_plan(S, A, B).nq;
  static constexpr int nqg(int g) {
    const Plan pl = make_plan(S, A, B);
    int c = 0;
    for (int q = 0; q < pl.nq; ++q) c += pl.qg[q] == g;
    return c;
  }
  static constexpr int qpos(int q) {
    const Plan pl = make_plan(S, A, B);
    int c = 0;
    for (int r = 0; r < q; ++r) c += pl.qg[r] == pl.qg[q];
    return c;
  }
  // i-th q slot of group g
  static constexpr int gq(int g, int i) {
    const Plan pl = make_plan(S, A, B);
    for (int q = 0; q < pl.nq; ++q)
      if (pl.qg[q] == g && qpos(q) == i) return q;
    return 0;
  }
  static constexpr int krow0(int g) {
    int o = 0;
    for (int h = 0; h < g; ++h) o += nqg(h) * L;
    return o;
  }
  static constexpr int arow_q(int q) { return krow0(make_plan(S, A, B).qg[q]) + qpos(q) * L; }
  static constexpr int ks2(int g) { return (nqg(g) * L + 3) / 4; }
  static constexpr int koff2(int g) {
    int o = 0;
    for (int h = 0; h < g; ++h) o += ks2(h);
    return o;
  }
  static constexpr int KS2 = koff2(NG);
  static constexpr int K1 = NG * L, KS1 = (K1 + 3) / 4;
  static constexpr int QSPLIT = imax(1, imin(NQ, NTHREADS / (NP * L * L)));
};

template <int S, int P, typename Real> struct Lds {
  using Sh = Shape<S, P>;
  static constexpr int L = Sh::L;
  template <typename F> static constexpr int over_blocks(F f) {
    int m = 0;
    for (int a = 0; a < Sh::NC; ++a)
      for (int b = a; b < Sh::NC; ++b) m = imax(m, f(a, b));
    return m;
  }
  static constexpr int NF = over_blocks([](int a, int b) { return make_plan(S, a, b).nf; });
  static constexpr int NQ = over_blocks([](int a, int b) { return make_plan(S, a, b).nq; });
  static constexpr int NG = over_blocks([](int a, int b) { return make_plan(S, a, b).ng; });
  static constexpr int NXP = over_blocks([](int a, int b) { return ru16(Sh::R(a, 1) * Sh::R(b, 1)); });
  static constexpr int FLD_LEN = NF * L * L * L;
  static constexpr int A_LEN = NQ * L * NC2;
  static constexpr int T_LEN = 2 * KT * L;
  static constexpr int BUDGET = 150 * 1024;
  static constexpr int bytes(int xch) {
    return int(sizeof(Real)) * (FLD_LEN + A_LEN + T_LEN + NG * NC2 * xch) + 8 * (2 * L + 24) + 256;
  }
  // x-chunk width of stages 2/1: as wide as possible within the LDS budget
  static constexpr int XCH = [] {
    int x = NXP;
    while (x > 16 && bytes(x) > BUDGET) x -= 16;
    return x;
  }();
  static_assert(bytes(XCH) <= BUDGET, "LDS budget exceeded");
  static constexpr int B_LEN = NG * NC2 * XCH;
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
// LDS index of B_g(col, x): rows of XS entries, odd rows rotated by 16 when
// XS is a multiple of 32 so that the four rows touched by one wave-wide
// access fall into alternating halves of the bank space.
// ---------------------------------------------------------------------------
template <int XS>
__device__ __forceinline__ int bidx(int row, int col, int x) {
  if constexpr (XS % 32 == 0) {
    int xr = x + 16 * (col & 1);
    if (xr >= XS) xr -= XS;
    return row * XS + xr;
  } else {
    return row * XS + x;
  }
}

// (i2, j2) of x slot s: all pairs (i2 fastest) or the triangle i2 <= j2
template <int R2a, bool DIAG>
__device__ __forceinline__ void decode_x(const unsigned char* xd, int s, int& i2, int& j2) {
  if (DIAG) { i2 = xd[2 * s]; j2 = xd[2 * s + 1]; }
  else { i2 = s % R2a; j2 = s / R2a; }
}

// stage-2 B operand: u = T^<r2>_{i2+sa}(m) T^<s2>_{j2+sb}(m) for the group-local k
template <int S, int P, typename Real, int A, int B, bool DIAG, int G>
__device__ __forceinline__ Real u2_value(const Real* sT, const unsigned char* xd, int x, int kk) {
  using BC = Blk<S, P, A, B>;
  using Sh = Shape<S, P>;
  constexpr int L = BC::L, KTL = KT * L;
  constexpr int NXv = DIAG ? BC::NXD : BC::NX;
  constexpr int KG = BC::nqg(G) * L;
  if (x >= NXv || kk >= KG) return Real(0);
  const int qi = kk / L, m = kk - qi * L;
  int r2 = 0, s2 = 0;
  constexpr int NQG = BC::nqg(G);
  static_for<NQG>([&](auto I) {
    constexpr int q = BC::gq(G, decltype(I)::value);
    if (qi == decltype(I)::value) { r2 = BC::PL.qr2[q]; s2 = BC::PL.qs2[q]; }
  });
  int i2, j2;
  decode_x<BC::R2a, DIAG>(xd, x, i2, j2);
  return sT[r2 * KTL + (i2 + Sh::SH(A, 1)) * L + m] * sT[s2 * KTL + (j2 + Sh::SH(B, 1)) * L + m];
}

// stage-1 B operand: u = T^<r1>_{i1+sa}(l) T^<s1>_{j1+sb}(l), k = (g, l)
template <int S, int P, typename Real, int A, int B>
__device__ __forceinline__ Real u1_value(const Real* sT, int y, int k) {
  using BC = Blk<S, P, A, B>;
  using Sh = Shape<S, P>;
  constexpr int L = BC::L, KTL = KT * L;
  if (y >= BC::NY || k >= BC::K1) return Real(0);
  const int g = k / L, l = k - g * L;
  const int i1 = y % BC::R1a, j1 = y / BC::R1a;
  int r1 = 0, s1 = 0;
  static_for<BC::NG>([&](auto G) {
    constexpr int gg = decltype(G)::value;
    if (g == gg) { r1 = BC::PL.gr1[gg]; s1 = BC::PL.gs1[gg]; }
  });
  return sT[r1 * KTL + (i1 + Sh::SH(A, 0)) * L + l] * sT[s1 * KTL + (j1 + Sh::SH(B, 0)) * L + l];
}

// ---------------------------------------------------------------------------
// stage-3 thread roles.  Thread t owns the point column (l, m) = t % L^2 for
// all n, pair slot pi and q subset qs of every batch of the block; with
// W3 = NP L^2 * QSPLIT <= 256 every thread has one fixed role, so the metric
// fields of its column and q subset stay in registers for the whole block.
// ---------------------------------------------------------------------------
template <int S, int P, int A, int B> struct S3Roles {
  using BC = Blk<S, P, A, B>;
  static constexpr int L = BC::L, QS = BC::QSPLIT;
  // distinct block field slots used by the terms of q subset qs
  static constexpr int nfs(int qs) {
    int seen[8] = {}, n = 0;
    for (int t = 0; t < BC::PL.nt; ++t) {
      if (BC::PL.tq[t] % QS != qs) continue;
      const int f = BC::PL.tf[t];
      bool dup = false;
      for (int i = 0; i < n; ++i) dup = dup || seen[i] == f;
      if (!dup) seen[n++] = f;
    }
    return n;
  }
  // s-th field slot of subset qs
  static constexpr int fsub(int qs, int s) {
    int seen[8] = {}, n = 0;
    for (int t = 0; t < BC::PL.nt; ++t) {
      if (BC::PL.tq[t] % QS != qs) continue;
      const int f = BC::PL.tf[t];
      bool dup = false;
      for (int i = 0; i < n; ++i) dup = dup || seen[i] == f;
      if (!dup) seen[n++] = f;
    }
    return seen[s];
  }
  // position of term tt's field within its subset
  static constexpr int fpos(int tt) {
    const int qs = BC::PL.tq[tt] % QS;
    for (int s = 0; s < nfs(qs); ++s)
      if (fsub(qs, s) == BC::PL.tf[tt]) return s;
    return 0;
  }
  static constexpr int NFS = [] {
    int m = 1;
    for (int q = 0; q < QS; ++q) m = imax(m, nfs(q));
    return m;
  }();
  static constexpr bool REGF = NFS * L <= 48;   // field column fits in registers
};

template <int S, int P, typename Real, int A, int B> struct Regs {
  using BC = Blk<S, P, A, B>;
  using R3 = S3Roles<S, P, A, B>;
  Real u2[BC::KS2 > 0 ? BC::KS2 : 1];   // stage-2 table operand of the wave's x-tile
  Real u1[BC::KS1];                     // stage-1 table operand of the wave's y-tile
  Real fr[R3::REGF ? R3::NFS : 1][R3::REGF ? R3::L : 1];   // stage-3 metric fields
};

// ---------------------------------------------------------------------------
// a batch of np pairs (i3[k], j3[k]) of block (A, B); wave-uniform
// ---------------------------------------------------------------------------
struct PairBatch {
  int np;
  int i3[4], j3[4];
  __device__ __forceinline__ int ki(int k) const {
    return k == 0 ? i3[0] : k == 1 ? i3[1] : k == 2 ? i3[2] : i3[3];
  }
  __device__ __forceinline__ int kj(int k) const {
    return k == 0 ? j3[0] : k == 1 ? j3[1] : k == 2 ? j3[2] : j3[3];
  }
};

// stage 3: A[(q, m)][(pi, l)] = sum_n c(l, m, n) T_i3(n) T_j3(n) for the pairs of pb
template <int S, int P, typename Real, int A, int B>
__device__ __forceinline__ void stage3(const SmemPtrs& sm, const Regs<S, P, Real, A, B>& rg, const PairBatch& pb) {
  using Sh = Shape<S, P>;
  using BC = Blk<S, P, A, B>;
  using R3 = S3Roles<S, P, A, B>;
  constexpr int L = Sh::L, L2 = L * L, KTL = KT * L;
  constexpr int W3 = BC::NP * L2;
  constexpr int QS = BC::QSPLIT;
  const Real* sT = static_cast<const Real*>(sm.T);
  const Real* sF = static_cast<const Real*>(sm.fld);
  Real* sA = static_cast<Real*>(sm.A);
  const int t = threadIdx.x;
  if (t >= W3 * QS) return;
  const int idx = t % W3;
  const int qs = (W3 % 64 == 0) ? __builtin_amdgcn_readfirstlane(t / W3) : t / W3;
  const int l = idx % L, m = (idx / L) % L;
  const int pi = (L2 % 64 == 0) ? __builtin_amdgcn_readfirstlane(idx / L2) : idx / L2;
  if (pi >= pb.np) return;
  const int ka = pb.ki(pi) + Sh::SH(A, 2);
  const int kb = pb.kj(pi) + Sh::SH(B, 2);
  static_for<QS>([&](auto QQ) {
    constexpr int qq = decltype(QQ)::value;
    if (qs != qq) return;
    Real acc[BC::NQ];
#pragma unroll
    for (int q = 0; q < BC::NQ; ++q) acc[q] = Real(0);
#pragma unroll
    for (int n = 0; n < L; ++n) {
      const Real ti0 = sT[ka * L + n], ti1 = sT[KTL + ka * L + n];
      const Real tj0 = sT[kb * L + n], tj1 = sT[KTL + kb * L + n];
      static_for<BC::PL.nt>([&](auto TT) {
        constexpr int tt = decltype(TT)::value;
        constexpr int q = BC::PL.tq[tt];
        if constexpr (q % QS == qq) {
          Real u = (BC::PL.t[tt].r[2] ? ti1 : ti0) * (BC::PL.t[tt].s[2] ? tj1 : tj0);
          if constexpr (BC::PL.t[tt].sign < 0) u = -u;
          Real f;
          if constexpr (R3::REGF) f = rg.fr[R3::fpos(tt)][n];
          else f = sF[(BC::PL.tf[tt] * L + n) * L2 + m * L + l];
          acc[q] += u * f;
        }
      });
    }
    static_for<BC::NQ>([&](auto Q) {
      constexpr int q = decltype(Q)::value;
      constexpr int row = BC::arow_q(q);
      if constexpr (q % QS == qq) sA[(row + m) * NC2 + pi * L + l] = acc[q];
    });
  });
}

// stage 2 (MFMA): B[g][(pi, l)][x] = sum_{(q,m) in g} A[(q,m)][(pi,l)] U2[(q,m)][x], x chunk xc
template <int S, int P, typename Real, int A, int B, bool DIAG>
__device__ __forceinline__ void stage2(const SmemPtrs& sm, const Regs<S, P, Real, A, B>& rg, int xc) {
  using LD = Lds<S, P, Real>;
  using BC = Blk<S, P, A, B>;
  using M = Mma<Real>;
  constexpr int L = BC::L;
  constexpr int NXv = DIAG ? BC::NXD : BC::NX;
  constexpr int NXPv = ru16(NXv);
  constexpr int XS = imin(LD::XCH, BC::NXP);
  constexpr int NCH = (NXPv + XS - 1) / XS;
  constexpr bool CACHE2 = !DIAG && NCH == 1 && BC::NXP <= 64;
  const Real* sT = static_cast<const Real*>(sm.T);
  const Real* sA = static_cast<const Real*>(sm.A);
  Real* sB = static_cast<Real*>(sm.B);
  const int tid = threadIdx.x;
  const int lane = tid & 63, wave = tid >> 6;
  const int lr = lane & 15, lk = lane >> 4;
  const int xtiles = imin(XS, NXPv - xc) / 16;
  for (int xt = wave; xt < xtiles; xt += 4) {
    const int xl = xt * 16 + lr;           // x within the chunk (B-operand column)
    const int x = xc + xl;
    typename M::acc acc[BC::NG];
#pragma unroll
    for (int g = 0; g < BC::NG; ++g) acc[g] = typename M::acc{0, 0, 0, 0};
    static_for<BC::NG>([&](auto GG) {
      constexpr int G = decltype(GG)::value;
      constexpr int KSG = BC::ks2(G), KG = BC::nqg(G) * L, KR = BC::krow0(G), KO = BC::koff2(G);
#pragma unroll
      for (int ks = 0; ks < KSG; ++ks) {
        const int kk = 4 * ks + lk;
        const Real a = kk < KG ? sA[(KR + kk) * NC2 + lr] : Real(0);
        Real u;
        if constexpr (CACHE2) u = rg.u2[KO + ks];
        else u = u2_value<S, P, Real, A, B, DIAG, G>(sT, sm.xd, x, kk);
        acc[G] = M::mac(a, u, acc[G]);
      }
    });
#pragma unroll
    for (int g = 0; g < BC::NG; ++g)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int col = M::crow(lk, r);
        sB[bidx<XS>(g * NC2 + col, col, xl)] = acc[g][r];
      }
  }
}

// stage 1 (MFMA) and the packed store: G[(i1,i2),(j1,j2)] for the pairs of pb, x chunk xc
template <int S, int P, typename Real, int A, int B, bool DIAG>
__device__ __forceinline__ void stage1(const SmemPtrs& sm, const Regs<S, P, Real, A, B>& rg, const PairBatch& pb,
                                       int xc, Real* __restrict__ outp) {
  using Sh = Shape<S, P>;
  using LD = Lds<S, P, Real>;
  using BC = Blk<S, P, A, B>;
  using M = Mma<Real>;
  constexpr int L = BC::L;
  constexpr int NXv = DIAG ? BC::NXD : BC::NX;
  constexpr int NXPv = ru16(NXv);
  constexpr int XS = imin(LD::XCH, BC::NXP);
  constexpr bool CACHE1 = BC::NYT <= 4;
  constexpr int XB = 4;
  const Real* sT = static_cast<const Real*>(sm.T);
  const Real* sB = static_cast<const Real*>(sm.B);
  const int tid = threadIdx.x;
  const int lane = tid & 63, wave = tid >> 6;
  const int lr = lane & 15, lk = lane >> 4;
  const int xtiles = imin(XS, NXPv - xc) / 16;
  for (int yt = wave; yt < BC::NYT; yt += 4) {
    const int y = yt * 16 + lr;
    const bool yv = y < BC::NY;
    const int i1 = y % BC::R1a, j1 = y / BC::R1a;
    const int xrow = M::arow(lr);
    for (int pi = 0; pi < pb.np; ++pi) {
      const int Ib = Sh::OFF(A) + i1 + BC::R1a * BC::R2a * pb.ki(pi);
      const int Jb = Sh::OFF(B) + j1 + BC::R1b * BC::R2b * pb.kj(pi);
      for (int xt0 = 0; xt0 < xtiles; xt0 += XB) {
        typename M::acc acc[XB];
#pragma unroll
        for (int c = 0; c < XB; ++c) acc[c] = typename M::acc{0, 0, 0, 0};
#pragma unroll
        for (int ks = 0; ks < BC::KS1; ++ks) {
          const int k = 4 * ks + lk;
          const int g = k / L, l = k - g * L;
          const int col = pi * L + l;
          Real u;
          if constexpr (CACHE1) u = rg.u1[ks];
          else u = u1_value<S, P, Real, A, B>(sT, y, k);
#pragma unroll
          for (int c = 0; c < XB; ++c) {
            if (xt0 + c < xtiles) {
              const Real a = (BC::K1 % 4 == 0 || k < BC::K1)
                                 ? sB[bidx<XS>(g * NC2 + col, col, (xt0 + c) * 16 + xrow)] : Real(0);
              acc[c] = M::mac(a, u, acc[c]);
            }
          }
        }
#pragma unroll
        for (int c = 0; c < XB; ++c) {
          if (xt0 + c < xtiles) {
#pragma unroll
            for (int r = 0; r < 4; ++r) {
              const int s = xc + (xt0 + c) * 16 + lk + 4 * r;
              if (yv && s < NXv) {
                int i2, j2;
                decode_x<BC::R2a, DIAG>(sm.xd, s, i2, j2);
                if (!DIAG || i2 < j2 || i1 <= j1) {
                  const int I = Ib + BC::R1a * i2;
                  const int J = Jb + BC::R1b * j2;
                  outp[I + J * (J + 1) / 2] = acc[c][r];
                }
              }
            }
          }
        }
      }
    }
  }
}

// Pair batches of a block: off-diagonal pairs (i3, j3), j3 in [j3_lo, j3_hi),
// i3 < j3 (diagonal block) or i3 < R3a, NP at a time; then the diagonal
// pairs (j3, j3) of a diagonal block, NP at a time.
template <int S, int P, int A, int B> struct PairCursor {
  using BC = Blk<S, P, A, B>;
  int ci, cj, hi, dj;
  __device__ __forceinline__ int rows(int j) const { return A == B ? j : BC::R3a; }
  __device__ __forceinline__ void skip() { while (cj < hi && ci >= rows(cj)) { ++cj; ci = 0; } }
  __device__ __forceinline__ PairCursor(int lo, int hi_) : ci(0), cj(lo), hi(hi_), dj(lo) { skip(); }
  // next batch; returns false when done; *diag tells which x-list it uses
  __device__ __forceinline__ bool next(PairBatch& pb, bool& diag) {
#pragma unroll
    for (int k = 0; k < 4; ++k) { pb.i3[k] = 0; pb.j3[k] = 0; }
    pb.np = 0;
    if (cj < hi) {
      diag = false;
#pragma unroll
      for (int k = 0; k < BC::NP; ++k) {
        if (cj < hi) {
          pb.i3[k] = ci;
          pb.j3[k] = cj;
          pb.np = k + 1;
          ++ci;
          skip();
        }
      }
      return true;
    }
    if (A == B && dj < hi) {
      diag = true;
      pb.np = imin(BC::NP, hi - dj);
#pragma unroll
      for (int k = 0; k < 4; ++k) { pb.i3[k] = dj + k; pb.j3[k] = dj + k; }
      dj += BC::NP;
      return true;
    }
    return false;
  }
};

template <int S, int P, typename Real, int A, int B>
__device__ __forceinline__ bool run_block(const GeneralArgs& ga, const SmemPtrs sm, int j3_lo, int j3_hi,
                                          Real* __restrict__ outp) {
  using Sh = Shape<S, P>;
  using BC = Blk<S, P, A, B>;
  using LD = Lds<S, P, Real>;
  using R3 = S3Roles<S, P, A, B>;
  constexpr int L = Sh::L, L2 = L * L, L3 = L2 * L;
  Real* sF = static_cast<Real*>(sm.fld);
  const Real* sT = static_cast<const Real*>(sm.T);
  const int tid = threadIdx.x;
  const int lane = tid & 63, wave = tid >> 6;
  const int lr = lane & 15, lk = lane >> 4;

  // ---------------- metric -> coefficient fields, layout [f][n][m][l] ----------------
  for (int pt = tid; pt < L3; pt += NTHREADS) {
    const int l = pt % L, m = (pt / L) % L, n = pt / L2;
    double J[3][3], adj[3][3];
    jacobian_at(ga.geom_kind, sm.X, sm.z[l], sm.z[m], sm.z[n], J);
    const double det = adjugate(J, adj);
    if (!(det > 0.0)) *sm.bad = 1;
    const double idet = 1.0 / det;
    const double wq = sm.w[l] * sm.w[m] * sm.w[n];
    const double wv = wq * ga.w0, wd = wq * ga.w1;
    static_for<BC::PL.nf>([&](auto F) {
      constexpr int f = decltype(F)::value;
      constexpr int fid = BC::PL.fid[f];
      const double v = field_value(fid, J, adj, det, idet) * (field_weight(S, fid) ? wd : wv);
      sF[(f * L + n) * L2 + m * L + l] = static_cast<Real>(v);
    });
  }

  // ---------------- table operands of this wave's tiles, kept in registers ----------------
  Regs<S, P, Real, A, B> rg;
  {
    const int x = wave * 16 + lr;
    static_for<BC::NG>([&](auto GG) {
      constexpr int G = decltype(GG)::value;
      constexpr int KSG = BC::ks2(G), KO = BC::koff2(G);
#pragma unroll
      for (int ks = 0; ks < KSG; ++ks)
        rg.u2[KO + ks] = u2_value<S, P, Real, A, B, false, G>(sT, sm.xd, x, 4 * ks + lk);
    });
    const int y = wave * 16 + lr;
#pragma unroll
    for (int ks = 0; ks < BC::KS1; ++ks) rg.u1[ks] = u1_value<S, P, Real, A, B>(sT, y, 4 * ks + lk);
  }
  __syncthreads();
  if (*sm.bad) return true;

  // ---------------- this thread's stage-3 field column, kept in registers ----------------
  if constexpr (R3::REGF) {
    constexpr int W3 = BC::NP * L2;
    if (tid < W3 * BC::QSPLIT) {
      const int idx = tid % W3, qs = tid / W3;
      const int l = idx % L, m = (idx / L) % L;
      static_for<BC::QSPLIT>([&](auto QQ) {
        constexpr int qq = decltype(QQ)::value;
        if (qs == qq) {
          static_for<R3::nfs(qq)>([&](auto SS) {
            constexpr int f = R3::fsub(qq, decltype(SS)::value);
#pragma unroll
            for (int n = 0; n < L; ++n) rg.fr[decltype(SS)::value][n] = sF[(f * L + n) * L2 + m * L + l];
          });
        }
      });
    }
  }

  // ---------------- pipelined batches ----------------
  // [stage 2 (t)] barrier [stage 3 (t+1), stage 1 (t)] barrier ...
  constexpr int NXP_ND = BC::NXP;
  constexpr int XS = imin(LD::XCH, BC::NXP);
  PairCursor<S, P, A, B> cur(j3_lo, j3_hi);
  PairBatch pb, pn;
  bool dg = false, dn = false;
  bool have = cur.next(pb, dg);
  if (have) stage3<S, P, Real, A, B>(sm, rg, pb);
  __syncthreads();
  while (have) {
    const bool have_next = cur.next(pn, dn);
    const int nxp = dg ? ru16(BC::NXD) : NXP_ND;
    for (int xc = 0; xc < nxp; xc += XS) {
      if (dg) stage2<S, P, Real, A, B, true>(sm, rg, xc);
      else stage2<S, P, Real, A, B, false>(sm, rg, xc);
      __syncthreads();
      if (xc + XS >= nxp && have_next) stage3<S, P, Real, A, B>(sm, rg, pn);
      if (dg) stage1<S, P, Real, A, B, true>(sm, rg, pb, xc, outp);
      else stage1<S, P, Real, A, B, false>(sm, rg, pb, xc, outp);
      __syncthreads();
    }
    pb = pn;
    dg = dn;
    have = have_next;
  }
  (void)sF;
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
  const int G = ga.slab_group;                                // slabs per workgroup
  const int ngroups = (Sh::NSLAB + G - 1) / G;
  const int grp = ngroups - 1 - int(blk / ga.n_items);        // heaviest slab groups first
  const int64_t item = ga.item_base + blk % ga.n_items;
  const int64_t e = ga.elem_ids ? int64_t(ga.elem_ids[item]) : item;
  const int s_lo = grp * G, s_hi = imin(Sh::NSLAB, s_lo + G);

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

  // component b owns slabs [slab0(b), slab0(b) + R3(b)); visit the blocks (a, b), a <= b,
  // for the j3 range of every component the slab group touches
  bool bad = false;
  auto jr = [&](int b, int& lo, int& hi) {
    lo = imax(s_lo, Sh::slab0(b)) - Sh::slab0(b);
    hi = imin(s_hi, Sh::slab0(b) + Sh::R(b, 2)) - Sh::slab0(b);
    return lo < hi;
  };
  int lo, hi;
  if (jr(0, lo, hi)) bad = run_block<S, P, Real, 0, 0>(ga, sm, lo, hi, outp);
  if constexpr (Sh::NC == 3) {
    if (!bad && jr(1, lo, hi)) {
      bad = run_block<S, P, Real, 0, 1>(ga, sm, lo, hi, outp);
      if (!bad) bad = run_block<S, P, Real, 1, 1>(ga, sm, lo, hi, outp);
    }
    if (!bad && jr(2, lo, hi)) {
      bad = run_block<S, P, Real, 0, 2>(ga, sm, lo, hi, outp);
      if (!bad) bad = run_block<S, P, Real, 1, 2>(ga, sm, lo, hi, outp);
      if (!bad) bad = run_block<S, P, Real, 2, 2>(ga, sm, lo, hi, outp);
    }
  }
  if (bad) {
    // element with det J <= 0: its whole output is zero (every slab group does its part)
    auto colstart = [&](int slab) {   // first column J of a slab
      int b = 0, j3 = slab;
#pragma unroll
      for (int c = 0; c < Sh::NC - 1; ++c)
        if (b == c && j3 >= Sh::R(c, 2)) { j3 -= Sh::R(c, 2); b = c + 1; }
      int r12 = Sh::R(0, 0) * Sh::R(0, 1), offb = 0;
#pragma unroll
      for (int c = 1; c < Sh::NC; ++c)
        if (b == c) { r12 = Sh::R(c, 0) * Sh::R(c, 1); offb = Sh::OFF(c); }
      return int64_t(offb) + int64_t(r12) * j3;
    };
    const int64_t J0 = colstart(s_lo);
    const int64_t J1 = s_hi == Sh::NSLAB ? int64_t(Sh::OFF(Sh::NC)) : colstart(s_hi);
    for (int64_t i = J0 * (J0 + 1) / 2 + tid; i < J1 * (J1 + 1) / 2; i += NTHREADS) outp[i] = Real(0);
  }
  if (ga.status && tid == 0 && (bad || s_lo == 0)) ga.status[e] = bad ? -4 : 0;
}

template <int S, int P, typename Real>
hipError_t launch_general_one(const GeneralArgs& a, hipStream_t st) {
  constexpr int NS = Shape<S, P>::NSLAB;
  GeneralArgs c = a;
  c.slab_group = slab_group_for(NS, a.n_items, a.slab_group);
  const int ngroups = (NS + c.slab_group - 1) / c.slab_group;
  const int64_t max_items = int64_t(0x7fffffff) / ngroups;
  for (int64_t base = 0; base < a.n_items; base += max_items) {
    c.item_base = a.item_base + base;
    c.n_items = (a.n_items - base) < max_items ? (a.n_items - base) : max_items;
    hipLaunchKernelGGL((k_general<S, P, Real>), dim3(unsigned(c.n_items * ngroups)), dim3(NTHREADS), 0, st, c);
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
