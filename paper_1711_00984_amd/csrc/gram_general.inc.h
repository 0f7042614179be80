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
// Pairs (i3, j3) are processed in batches.  Stage 3 of a batch writes A_q for
// all its pairs to LDS (double-buffered, so stage 3 of the next batch runs
// while the waves work on this one).  Then each wave takes work items (pair
// group, x-tile of 16 x = (i2, j2)) and runs stages 2 and 1 for it without
// touching LDS in between:
//
//   stage 2: C2[row][x] = sum_k A[row][k] U2[k][x], rows = (pair, l) of NP
//            pairs padded to LP = 4 ceil(L/4) points, k = (q, m); one MFMA
//            accumulator per group g;
//   stage 1: G[x][y] = sum_k C2^T[x][k] U1[k][y], k = (g, l), y = (i1, j1).
//
// The MFMA accumulator layout of gfx950 makes register r of stage 2's
// accumulator, read by the same lane, exactly the A operand of stage 1 for
// k = l = 4 rho + (lane / 16) when the stage-2 rows are ordered as below, so
// the intermediate B_g never leaves the registers.  The table operands U2, U1
// (products of two 1D table values) come from a per-block LDS table, from
// registers, or from the 1D tables with immediate offsets (k-slot -> (q, m)
// and (g, l) are compile-time), whichever the LDS budget allows.
//
// MFMA operand layout (v_mfma_*_16x16x4): lane = i + 16 k holds A[i][k] and
// B[k][j = i]; accumulator register r of lane (g = lane / 16, j = lane % 16)
// holds C[crow(g, r)][j].  Stage-1 row i is stage-2 column i, which carries
// x = xbase + arow(i), chosen so that register r of lane group g holds x
// offset g + 4 r: four consecutive x = (i2, j2), i.e. consecutive rows I of one
// packed column, so a store instruction writes runs of 4 R1 values.
#pragma once
#include <hip/hip_runtime.h>

#include <utility>

#include "kernels.h"
#include "metric.h"
#include "terms.h"

namespace dpg {

typedef double v4d __attribute__((ext_vector_type(4)));
typedef float v4f __attribute__((ext_vector_type(4)));

template <typename Real> struct Mma;
// Accumulator register r of lane (g = lane/16, j = lane%16) holds C[row][j] with
// row = g + 4 r for the f64 instruction and row = 4 g + r for the f32 one
// (both checked on gfx950).  arow(i) is the x offset that stage-1 row i must
// carry so that register r of lane group g always holds x offset g + 4 r.
template <> struct Mma<double> {
  typedef v4d acc;
  static __device__ __forceinline__ acc mac(double a, double b, acc c) {
    return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
  }
  static constexpr __host__ __device__ int arow(int i) { return i; }
  static constexpr __host__ __device__ int crow(int g, int r) { return g + 4 * r; }
};
template <> struct Mma<float> {
  typedef v4f acc;
  static __device__ __forceinline__ acc mac(float a, float b, acc c) {
    return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
  }
  static constexpr __host__ __device__ int arow(int i) { return (i >> 2) + 4 * (i & 3); }
  static constexpr __host__ __device__ int crow(int g, int r) { return 4 * g + r; }
};

constexpr int NTHREADS = 256;
// Register-budget knobs (Reals per thread): metric field column of stage 3,
// stage-2 table operand of a fixed x-tile, y-tiles per stage-1 accumulator set.
#ifndef DPG_REGF_MAX
#define DPG_REGF_MAX 48
#endif
#ifndef DPG_REGF_MAX_HI
#define DPG_REGF_MAX_HI 18   // FP64 with more than 8 points per direction (two-wave kernels)
#endif
#ifndef DPG_C2_MAX
#define DPG_C2_MAX 24
#endif
#ifndef DPG_HOLD_HEADS
#define DPG_HOLD_HEADS 1
#endif
#ifndef DPG_PIPE
#define DPG_PIPE 0
#endif
#ifndef DPG_YB
#define DPG_YB 4
#endif
#ifndef DPG_U1R_MAX
#define DPG_U1R_MAX 0
#endif
#ifndef DPG_MINW2_LMAX
#define DPG_MINW2_LMAX 8
#endif
#ifndef DPG_YTAIL_VALU
#define DPG_YTAIL_VALU 1
#endif
constexpr int ru16(int x) { return (x + 15) / 16 * 16; }
constexpr int imax(int a, int b) { return a > b ? a : b; }
constexpr int imin(int a, int b) { return a < b ? a : b; }
constexpr int lpad(int L) { return 4 * ((L + 3) / 4); }   // points padded to whole k-steps

// Stage-1 MFMAs of the next step issued before the stores of the current one (DPG_PIPE
// for all).  Measured per space and order (FP64, p = 6..10, same-box A/B over three
// rounds): only H(div) p = 10 gained (1.055x); H1 p = 9 lost 3.5 %, the others moved
// within 1 %.
template <int S, int P, typename Real> constexpr bool pipe_steps() {
  return DPG_PIPE || (sizeof(Real) == 8 && S == SP_HDIV && P == 10);
}

// Workgroups per CU that the LDS layout and the register budget are sized for, where more
// than the default two paid off (small FP64 orders, whose workgroups are short and spend
// much of their time in the setup's latency; same-box A/B against two per CU: H1 p = 3
// 1.12x with four, H1 p = 4, 5 1.10x and 1.07x and H(curl) p = 4 1.06x with three, while
// H(curl) p = 5 and the FP32 kernels gained nothing or lost, and four spilled at FP64
// H1 p = 4, 5).  0: the default choice.
template <int S, int P, typename Real> constexpr int occ_target() {
  if constexpr (sizeof(Real) != 8) return 0;
  if constexpr (S == SP_H1 && P == 3) return 4;
  if constexpr (S == SP_H1 && (P == 4 || P == 5)) return 3;
  if constexpr (S == SP_HCURL && P == 4) return 3;
  return 0;
}

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
  static constexpr int LP = lpad(L);        // l, m padded to a multiple of 4
  static constexpr int RPP = LP / 4;        // stage-2 accumulator registers per pair
  static constexpr int NP = 4 / RPP;        // pairs per stage-2 row tile (16 rows)
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
  static constexpr int L = Sh::L, LP = Sh::LP, RPP = Sh::RPP, NP = Sh::NP;
  static constexpr int R1a = Sh::R(A, 0), R1b = Sh::R(B, 0), R2a = Sh::R(A, 1), R2b = Sh::R(B, 1);
  static constexpr int R3a = Sh::R(A, 2), R3b = Sh::R(B, 2);
  static constexpr int NY = R1a * R1b, NYT = (NY + 15) / 16;
  // y tail: when the last y-tile would hold at most a quarter of its 16 columns, those
  // y = (i1, j1) are summed on the VALU from the stage-2 accumulators instead of
  // through a padded MFMA tile; NYM y-tiles remain on MFMA
  static constexpr int YTAIL = NY % 16;
  static constexpr bool YV = DPG_YTAIL_VALU && NY > 16 && YTAIL != 0 && YTAIL <= 4;
  static constexpr int NYM = YV ? NY / 16 : NYT;
  static constexpr int NX = R2a * R2b, NXT = (NX + 15) / 16;
  static constexpr int NXD = R2a * (R2a + 1) / 2, NXDT = (NXD + 15) / 16;
  static constexpr int NG = make_plan(S, A, B).ng;
  static constexpr int NQ = make_plan(S, A, B).nq;
};

// Per (space, order, precision): LDS layout and batch shape, chosen at
// compile time for the best estimated efficiency within the LDS budget.
//   NB     pair groups (stage-2 row tiles) per batch: more work items per
//          batch balance the four waves when x-tiles do not divide by 4
//   ABUF   2 = double-buffered stage-3 output (stage 3 of the next batch
//          overlaps this batch's MFMA work), 1 = single buffer
//   U1TAB  stage-1 table operand precomputed in LDS per block
template <int S, int P, typename Real> struct Cfg {
  using Sh = Shape<S, P>;
  static constexpr int L = Sh::L, LP = Sh::LP, RPP = Sh::RPP, NP = Sh::NP;
  template <typename F> static constexpr int over_blocks(F f) {
    int m = 0;
    for (int a = 0; a < Sh::NC; ++a)
      for (int b = a; b < Sh::NC; ++b) m = imax(m, f(a, b));
    return m;
  }
  static constexpr int NF = over_blocks([](int a, int b) { return make_plan(S, a, b).nf; });
  static constexpr int NQ = over_blocks([](int a, int b) { return make_plan(S, a, b).nq; });
  static constexpr int NG = over_blocks([](int a, int b) { return make_plan(S, a, b).ng; });
  static constexpr int NYT = over_blocks([](int a, int b) { return (Sh::R(a, 0) * Sh::R(b, 0) + 15) / 16; });
  static constexpr int FLD_LEN = NF * L * L * L;
  static constexpr int AONE = NQ * LP * 16;              // stage-3 output of one pair group
  static constexpr int T_LEN = 2 * KT * L + 8;           // chi, chi' tables (+ tail read by padded k)
  static constexpr int U1_LEN = NG * RPP * NYT * 64;
  static constexpr int SMALL = 8 * (2 * L + 24) + 2 * 80 + 64;
  static constexpr int BUDGET = 160 * 1024;
  // Column heads held back (one block of 8 x 8 planes, inline diagonal pairs, one pair
  // group per batch): the entries of each local column's first cache line, written by
  // the slab's first pair, wait in LDS until its diagonal pair writes the line's other
  // part (the tail of the previous column), so both reach the L2 together.
  static constexpr int LN = 128 / int(sizeof(Real));   // entries per cache line
  static constexpr bool HD_SHAPE = DPG_HOLD_HEADS && Sh::NC == 1 && Sh::R(0, 0) == 8 && Sh::R(0, 1) == 8 && diag_inline_ok(S, P);
  static constexpr int HD_LEN = HD_SHAPE ? 64 * LN : 0;
  static constexpr int bytes(int nb, int abuf, int u1) {
    return int(sizeof(Real)) * (FLD_LEN + abuf * nb * AONE + T_LEN + (u1 ? U1_LEN : 0) + (nb == 1 ? HD_LEN : 0)) +
           SMALL;
  }
  // fraction of wave time doing useful work items, over the blocks' non-diagonal batches
  static constexpr double balance(int nb) {
    double s = 0;
    int n = 0;
    for (int a = 0; a < Sh::NC; ++a)
      for (int b = a; b < Sh::NC; ++b) {
        const int items = nb * ((Sh::R(a, 1) * Sh::R(b, 1) + 15) / 16);
        s += double(items) / (4.0 * ((items + 3) / 4));
        ++n;
      }
    return s / n;
  }
  static constexpr int CHOICE = [] {
    double best = -1;
    int pick = 0;
    for (int nb = 1; nb <= 4; nb *= 2)
      for (int abuf = 2; abuf >= 1; --abuf)
        for (int u1 = 1; u1 >= 0; --u1) {
          if (bytes(nb, abuf, u1) > BUDGET) continue;
          // one workgroup per CU leaves no second workgroup to overlap barriers and stalls
          double occ = bytes(nb, abuf, u1) * 2 <= BUDGET ? 1.0 : 0.7;
          constexpr int W = occ_target<S, P, Real>();
          if (W > 0) occ = bytes(nb, abuf, u1) * W <= BUDGET ? 1.0 : 0.5 * occ;
          const double sc = balance(nb) * occ * (abuf == 2 ? 1.0 : 0.9) * (u1 ? 1.0 : 0.88) * (nb == 1 ? 1.0 : 0.995);
          if (sc > best + 1e-9) { best = sc; pick = nb * 100 + abuf * 10 + u1; }
        }
    return pick;
  }();
  static_assert(CHOICE > 0, "no LDS layout fits");
  static constexpr int NB = CHOICE / 100, ABUF = (CHOICE / 10) % 10;
  static constexpr bool U1TAB = CHOICE % 10;
  static constexpr int NBP = NB * NP;                    // pairs per batch
  static constexpr bool HD = HD_SHAPE && NB == 1;        // one work item per wave and x-tile
  static constexpr int BYTES = bytes(NB, ABUF, U1TAB);
};

// T, z, w: the 1D tables and points of direction 1; T2/T3, z2/z3, w2/w3 those of
// directions 2 and 3 (the same arrays when every direction takes one rule)
struct SmemPtrs {
  void* fld;
  void* A;
  void* U1;
  void* T;
  void* hd;
  double* z;
  double* w;
  double* X;
  unsigned char* xd;
  int* bad;
  void* T2;
  void* T3;
  double* z2;
  double* z3;
  double* w2;
  double* w3;
};
// (i2, j2) of x slot s: all pairs (i2 fastest) or the triangle i2 <= j2
template <int R2a, bool DIAG>
__device__ __forceinline__ void decode_x(const unsigned char* xd, int s, int& i2, int& j2) {
  if (DIAG) { i2 = xd[2 * s]; j2 = xd[2 * s + 1]; }
  else { i2 = s % R2a; j2 = s / R2a; }
}


// ---------------------------------------------------------------------------
// output stores through a raw buffer descriptor over one element's packed
// matrix (gfx9 descriptor word 3); offsets at or past the range are dropped
// ---------------------------------------------------------------------------
template <typename Real>
__device__ __forceinline__ __amdgpu_buffer_rsrc_t out_rsrc(Real* p, long long n) {
  return __builtin_amdgcn_make_buffer_rsrc(p, 0, int(n * (long long)sizeof(Real)), 0x00020000);
}
typedef unsigned int u32x2 __attribute__((ext_vector_type(2)));
// Byte offset that lands past any element's packed range (at most 2^28 bytes), used
// for lanes that hold padding; sums of two such offsets and a real one stay below 2^31.
constexpr unsigned kDropOff = 1u << 29;
__device__ __forceinline__ void store_out(double v, __amdgpu_buffer_rsrc_t r, int off) {
  __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(u32x2, v), r, off, 0, 0);
}
__device__ __forceinline__ void store_out(float v, __amdgpu_buffer_rsrc_t r, int off) {
  __builtin_amdgcn_raw_buffer_store_b32(__builtin_bit_cast(unsigned, v), r, off, 0, 0);
}

// ---------------------------------------------------------------------------
// pairs of a block: the non-diagonal pairs (i3, j3), j3 in [lo, hi), i3 < j3
// (diagonal block) or i3 < R3a, enumerated j3-major; then the diagonal pairs
// (j3, j3) of a diagonal block.  A batch is a run [t0, t0 + np) of one list.
// ---------------------------------------------------------------------------
template <int S, int P, int A, int B>
// r3a: the i3 range of a block a < b (R3(A), or the embedded orders' range)
__device__ __forceinline__ void pair_of(bool diag, int t, int lo, bool inl, int& i3, int& j3, int r3a) {
  if (diag) { i3 = lo + t; j3 = lo + t; return; }
  if constexpr (A != B) {
    j3 = lo + t / r3a;
    i3 = t % r3a;
  } else if (inl) {
    // i3 = 0 .. j3 inclusive: the diagonal pair closes its slab
    int j = lo;
    while (t > j) { t -= j + 1; ++j; }
    j3 = j;
    i3 = t;
  } else {
    int j = lo;
    while (t >= j) { t -= j; ++j; }
    j3 = j;
    i3 = t;
  }
}

// ---------------------------------------------------------------------------
// stage-3 thread roles.  A batch has W3 = NB NP L^2 point columns (pair slot,
// l, m); QS q-subsets split the work further when W3 < 256.  When one round
// covers all roles, every thread keeps the same (l, m) column for the whole
// block, and its metric fields stay in registers.
// ---------------------------------------------------------------------------
template <int S, int P, typename Real, int A, int B> struct S3Roles {
  using BC = Blk<S, P, A, B>;
  using CF = Cfg<S, P, Real>;
  static constexpr int L = BC::L, L2 = L * L;
  static constexpr int W3 = CF::NBP * L2;
  static constexpr int QS = imax(1, imin(BC::NQ, NTHREADS / W3));
  static constexpr int ROUNDS = (W3 * QS + NTHREADS - 1) / NTHREADS;
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
  // field column fits in registers (not with line writes, whose staging needs the registers)
  static constexpr bool REGF =
      ROUNDS == 1 && NFS * L <= (L <= 8 || sizeof(Real) == 4 ? DPG_REGF_MAX : DPG_REGF_MAX_HI);
};

// Stage-2 table operands of a wave's fixed x-tile kept in registers: when a
// block's non-diagonal batch has at most one work item per wave.
template <int S, int P, typename Real, int A, int B> struct Cache2 {
  using BC = Blk<S, P, A, B>;
  using CF = Cfg<S, P, Real>;
  static constexpr bool ON = CF::NB * BC::NXT <= 4 && BC::NQ * BC::RPP <= DPG_C2_MAX;
  static constexpr int N = ON ? BC::NQ * BC::RPP : 1;
};

// Stage-1 table operands of every y-tile kept in registers (all waves hold the
// same values) when they are few enough.
template <int S, int P, int A, int B> struct Cache1 {
  using BC = Blk<S, P, A, B>;
  static constexpr int N0 = BC::NG * BC::RPP * BC::NYT;
  static constexpr bool ON = N0 <= DPG_U1R_MAX;
  static constexpr int N = ON ? N0 : 1;
};

template <int S, int P, typename Real, int A, int B> struct Regs {
  using R3 = S3Roles<S, P, Real, A, B>;
  Real fr[R3::REGF ? R3::NFS : 1][R3::REGF ? R3::L : 1];   // stage-3 metric fields
  Real u2[Cache2<S, P, Real, A, B>::N];                      // stage-2 table operand
  Real u1[Cache1<S, P, A, B>::N];                            // stage-1 table operand
};

// stage 3: A[pg][(q, m)][row(pi, l)] = sum_n c(l, m, n) T_i3(n) T_j3(n) for the batch's pairs
template <int S, int P, typename Real, int A, int B>
__device__ __forceinline__ void stage3(const SmemPtrs& sm, const Regs<S, P, Real, A, B>& rg, bool diag, int t0,
                                       int np, int lo, bool inl, Real* sAb, int r3a) {
  using Sh = Shape<S, P>;
  using BC = Blk<S, P, A, B>;
  using CF = Cfg<S, P, Real>;
  using R3 = S3Roles<S, P, Real, A, B>;
  using M = Mma<Real>;
  constexpr int L = Sh::L, L2 = L * L, KTL = KT * L, QS = R3::QS, W3 = R3::W3;
  const Real* sT = static_cast<const Real*>(sm.T3);   // direction 3
  const Real* sF = static_cast<const Real*>(sm.fld);
#pragma unroll
  for (int rd = 0; rd < R3::ROUNDS; ++rd) {
    const int it = threadIdx.x + rd * NTHREADS;
    if (it >= W3 * QS) break;
    const int idx = it % W3, qs = it / W3;
    const int l = idx % L, m = (idx / L) % L, k = idx / L2;
    if (k >= np) continue;
    int i3, j3;
    pair_of<S, P, A, B>(diag, t0 + k, lo, inl, i3, j3, r3a);
    const int pg = k / BC::NP, pi = k % BC::NP;
    const int ka = i3 + Sh::SH(A, 2), kb = j3 + Sh::SH(B, 2);
    Real* dst = sAb + pg * CF::AONE + m * 16 + M::crow(l & 3, pi * BC::RPP + (l >> 2));
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
        if constexpr (q % QS == qq) dst[q * BC::LP * 16] = acc[q];
      });
    });
  }
}

// Output numbering of embedded orders (p1, p2, p3) for block (a, b): component a spans
// R1a x R2a x R3a functions from offset off_a (b likewise); plen packed entries per element.
struct EmbOut {
  int R1a, R2a, R3a, R1b, R2b, off_a, off_b;
  long long plen;
};

template <int S, int P, typename Real, int A, int B, bool DIAG, bool EMB>
__device__ __forceinline__ void work(const SmemPtrs& sm, const Regs<S, P, Real, A, B>& rg, int t0, int np, int lo,
                                     bool inl, const Real* sAb, Real* __restrict__ outp, const EmbOut& eo) {
  using Sh = Shape<S, P>;
  using BC = Blk<S, P, A, B>;
  using CF = Cfg<S, P, Real>;
  using M = Mma<Real>;
  constexpr int L = BC::L, LP = BC::LP, RPP = BC::RPP, NP = BC::NP, KTL = KT * L;
  constexpr int XT = DIAG ? BC::NXDT : BC::NXT;
  constexpr int NXv = DIAG ? BC::NXD : BC::NX;
  constexpr bool C2 = Cache2<S, P, Real, A, B>::ON && !DIAG;
  constexpr int YB = imin(DPG_YB, BC::NYM), YCH = (BC::NYM + YB - 1) / YB;
  const Real* sT = static_cast<const Real*>(sm.T);     // direction 1 (stage 1)
  const Real* sT2 = static_cast<const Real*>(sm.T2);   // direction 2 (stage 2)
  const Real* sU1 = static_cast<const Real*>(sm.U1);
  const int tid = threadIdx.x;
  const int lane = tid & 63, wave = tid >> 6;
  const int lr = lane & 15, lk = lane >> 4;
  static_assert(gram_dim(S, P) < (1 << 13) && packed_len(S, P) * 8 < (1ll << 28), "store offset bounds");
  static_assert(!CF::HD || (A == 0 && B == 0 && BC::NXT == 4 && CF::NB == 1 && NP == 2 && BC::R1b == 8 &&
                            BC::R2b == 8 && BC::NY == 64),
                "held column heads assume one work item per wave and x-tile over whole j2 rows");
  // held column heads assume order P's numbering
  constexpr bool HDE = CF::HD && !EMB;
  const __amdgpu_buffer_rsrc_t rsrc = out_rsrc(outp, EMB ? eo.plen : packed_len(S, P));
  for (int item = wave; item < CF::NB * XT; item += 4) {
    const int pg = item / XT, xt = item % XT;
    const int npg = imin(NP, np - pg * NP);
    if (npg <= 0) continue;
    if constexpr (EMB) {
      // j2 does not decrease along x in either tiling: a tile whose first x lies past the
      // embedded orders' j2 range stores nothing
      int i2 = 0, j2 = 0;
      decode_x<BC::R2a, DIAG>(sm.xd, xt * 16, i2, j2);
      if (j2 >= eo.R2b) continue;
    }
    // ---------------- stage 2: acc2[g] = C2 rows (pair, l) x 16 columns x ----------------
    typename M::acc acc2[BC::NG];
#pragma unroll
    for (int g = 0; g < BC::NG; ++g) acc2[g] = typename M::acc{0, 0, 0, 0};
    int ia = lk, jb = lk;
    if constexpr (!C2) {
      const int xs = xt * 16 + M::arow(lr);
      int i2 = 0, j2 = 0;
      if (xs < NXv) decode_x<BC::R2a, DIAG>(sm.xd, xs, i2, j2);
      ia = (i2 + Sh::SH(A, 1)) * L + lk;
      jb = (j2 + Sh::SH(B, 1)) * L + lk;
    }
    const Real* Ab = sAb + pg * CF::AONE + lane;
    static_for<BC::NQ>([&](auto Q) {
      constexpr int q = decltype(Q)::value;
      constexpr int g = BC::PL.qg[q], r2 = BC::PL.qr2[q], s2 = BC::PL.qs2[q];
      static_for<RPP>([&](auto KS) {
        constexpr int ks = decltype(KS)::value;
        const Real a = Ab[(q * LP + 4 * ks) * 16];
        Real u;
        if constexpr (C2) u = rg.u2[q * RPP + ks];
        else u = sT2[r2 * KTL + ia + 4 * ks] * sT2[s2 * KTL + jb + 4 * ks];
        acc2[g] = M::mac(a, u, acc2[g]);
      });
    });
    // ---------------- stage 1 and store ----------------
    // x of this lane's accumulator register r: xt * 16 + lk + 4 r.  Its share of the
    // packed offset, pair-independent: the row part R1a i2 in bytes (past the element's
    // range when x is padding, so such stores drop) and the column part R1b j2.
    unsigned xa8[4], xb[4];
    bool xlt[4];
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int s = xt * 16 + lk + 4 * r;
      int i2 = 0, j2 = 0;
      if (s < NXv) decode_x<BC::R2a, DIAG>(sm.xd, s, i2, j2);
      if constexpr (EMB) {
        // x outside the embedded orders' (i2, j2) ranges: dropped
        xa8[r] = s < NXv && i2 < eo.R2a && j2 < eo.R2b ? unsigned(eo.R1a * i2 * int(sizeof(Real))) : kDropOff;
        xb[r] = unsigned(eo.R1b * j2);
      } else {
        xa8[r] = s < NXv ? unsigned(BC::R1a * i2 * int(sizeof(Real))) : kDropOff;
        xb[r] = unsigned(BC::R1b * j2);
      }
      xlt[r] = i2 < j2;
    }
    // the pairs' uniform row and column bases
    int Ibp[NP], Jbp[NP];
    bool rok[NP];   // embedded orders: the pair's i3 is inside component A's range
    bool dgp[NP];   // a diagonal pair in the full x tiling: its lower triangle is dropped
    bool hdw[NP], hdf[NP];   // column heads: held back in LDS / written out after this pair
    static_for<NP>([&](auto PI) {
      constexpr int pi = decltype(PI)::value;
      int i3 = 0, j3 = 0;
      if (pi < npg) pair_of<S, P, A, B>(DIAG, t0 + pg * NP + pi, lo, inl, i3, j3, EMB ? eo.R3a : BC::R3a);
      if constexpr (EMB) {
        Ibp[pi] = eo.off_a + eo.R1a * eo.R2a * i3;
        Jbp[pi] = eo.off_b + eo.R1b * eo.R2b * j3;
        rok[pi] = i3 < eo.R3a;
      } else {
        Ibp[pi] = Sh::OFF(A) + BC::R1a * BC::R2a * i3;
        Jbp[pi] = Sh::OFF(B) + BC::R1b * BC::R2b * j3;
        rok[pi] = true;
      }
      dgp[pi] = A == B && !DIAG && i3 == j3;
      hdw[pi] = hdf[pi] = false;
      if constexpr (HDE && !DIAG) {
        // slab j3 holds its heads back when its first and its diagonal pair fall in different batches
        const int tb = (j3 * (j3 + 1) - lo * (lo + 1)) / 2;
        const bool held = inl && pi < npg && tb / CF::NBP != (tb + j3) / CF::NBP;
        hdw[pi] = held && i3 == 0;
        hdf[pi] = held && i3 == j3;
      }
    });
    Real* sHD = static_cast<Real*>(sm.hd);
    using Acc = typename M::acc;
    // stage 1 of step (pair pi, y chunk yc) into acc1
    auto mm = [&](auto PI, auto YC, Acc (&acc1)[YB]) {
      constexpr int pi = decltype(PI)::value, yc = decltype(YC)::value;
#pragma unroll
      for (int c = 0; c < YB; ++c) acc1[c] = Acc{0, 0, 0, 0};
      static_for<BC::NG>([&](auto G) {
        constexpr int g = decltype(G)::value;
        constexpr int r1 = BC::PL.gr1[g], s1 = BC::PL.gs1[g];
        static_for<RPP>([&](auto RHO) {
          constexpr int rho = decltype(RHO)::value;
          const Real a = acc2[g][pi * RPP + rho];
          static_for<YB>([&](auto YY) {
            constexpr int yt = yc * YB + decltype(YY)::value;
            if constexpr (yt < BC::NYM) {
              Real u;
              if constexpr (Cache1<S, P, A, B>::ON) {
                u = rg.u1[(g * RPP + rho) * BC::NYT + yt];
              } else if constexpr (CF::U1TAB) {
                u = sU1[((g * RPP + rho) * BC::NYT + yt) * 64 + lane];
              } else {
                const int y = yt * 16 + lr;
                const int yy = y < BC::NY ? y : 0;
                const int i1 = yy % BC::R1a, j1 = yy / BC::R1a;
                u = sT[r1 * KTL + (i1 + Sh::SH(A, 0)) * L + lk + 4 * rho] *
                    sT[s1 * KTL + (j1 + Sh::SH(B, 0)) * L + lk + 4 * rho];
              }
              acc1[decltype(YY)::value] = M::mac(a, u, acc1[decltype(YY)::value]);
            }
          });
        });
      });
    };
    // packed store of step (pi, yc): register r of lane (lk, lr) holds G[x = xt*16 + lk + 4r]
    // [y = yt*16 + lr], entry I + J(J+1)/2 of the packed column J.  Buffer stores without
    // branches: a lane with nothing to store gets an offset past the element's range, which
    // the buffer unit discards.  J < 2^13, so J(J+1) is one 24-bit multiply-add.
    // DG: the pair is a diagonal pair of the full x tiling (its lower triangle dropped); a
    // wave-uniform property of the pair, so the other pairs' stores skip that mask
    auto st_body = [&](auto PI, auto YC, auto DG, auto HW, const Acc (&acc1)[YB]) {
      constexpr int pi = decltype(PI)::value, yc = decltype(YC)::value;
      constexpr bool dg = decltype(DG)::value, hw = decltype(HW)::value;
      const int Ib = Ibp[pi], Jb = Jbp[pi];
      static_for<YB>([&](auto YY) {
        constexpr int yt = yc * YB + decltype(YY)::value;
        if constexpr (yt < BC::NYM) {
          const int y = yt * 16 + lr;
          const int i1 = y % BC::R1a, j1 = y / BC::R1a;
          bool yok = y < BC::NY;
          if constexpr (EMB) yok = yok && i1 < eo.R1a && j1 < eo.R1b && rok[pi];
          const unsigned ya8 = yok ? unsigned((Ib + i1) * int(sizeof(Real))) : kDropOff;
          const unsigned yb = unsigned(Jb + j1);
#pragma unroll
          for (int r = 0; r < 4; ++r) {
            const unsigned J = yb + xb[r];
            const unsigned JJ = __umul24(J, J) + J;
            unsigned off = (JJ << (sizeof(Real) == 8 ? 2 : 1)) + ya8 + xa8[r];
            if constexpr (DIAG) off = (xlt[r] || i1 <= j1) ? off : kDropOff;
            if constexpr (dg) {
              const unsigned il = unsigned(i1 * int(sizeof(Real))) + xa8[r];
              const unsigned jl = (unsigned(j1) + xb[r]) * unsigned(sizeof(Real));
              off = il > jl ? kDropOff : off;
            }
            if constexpr (hw) {
              {
                // rows of the column's first line (i3 = 0, so I = i1 + 8 i2) go to LDS
                const unsigned h = (CF::LN - ((JJ >> 1) & (CF::LN - 1))) & (CF::LN - 1);
                const unsigned I8 = ya8 + xa8[r];
                if (I8 < h * unsigned(sizeof(Real))) {
                  sHD[(J - unsigned(Jbp[pi])) * CF::LN + I8 / unsigned(sizeof(Real))] = acc1[decltype(YY)::value][r];
                  off = kDropOff;
                }
              }
            }
            store_out(acc1[decltype(YY)::value][r], rsrc, int(off));
          }
        }
      });
    };
    // the pair's mask and head holding are wave-uniform: one branch per pair, not per store
    auto st_hd = [&](auto PI, auto YC, auto DG, const Acc (&acc1)[YB]) {
      constexpr int pi = decltype(PI)::value;
      if constexpr (HDE && !DIAG) {
        if (hdw[pi])
          st_body(PI, YC, DG, std::true_type{}, acc1);
        else
          st_body(PI, YC, DG, std::false_type{}, acc1);
      } else {
        st_body(PI, YC, DG, std::false_type{}, acc1);
      }
    };
    auto st = [&](auto PI, auto YC, const Acc (&acc1)[YB]) {
      constexpr int pi = decltype(PI)::value;
      if constexpr (A == B && !DIAG && diag_inline_ok(S, P)) {
        if (dgp[pi])
          st_hd(PI, YC, std::true_type{}, acc1);
        else
          st_hd(PI, YC, std::false_type{}, acc1);
      } else {
        st_hd(PI, YC, std::false_type{}, acc1);
      }
    };
    // after a diagonal pair: the held column heads of its slab, for this x-tile's 16 columns
    // (j2 = 2 xt, 2 xt + 1), which the same wave held back at the slab's first pair
    auto flush = [&](auto PI) {
      constexpr int pi = decltype(PI)::value;
      if constexpr (HDE && !DIAG) {
        if (hdf[pi]) {
          for (int k = lane; k < 16 * CF::LN; k += 64) {
            const int col = k / CF::LN, row = k % CF::LN;
            const int c = (col & 7) + 8 * (2 * xt + (col >> 3));
            const unsigned J = unsigned(Jbp[pi] + c);
            const unsigned JJ = __umul24(J, J) + J;
            const unsigned h = (CF::LN - ((JJ >> 1) & (CF::LN - 1))) & (CF::LN - 1);
            if (unsigned(row) < h)
              store_out(sHD[c * CF::LN + row], rsrc, int(((JJ >> 1) + unsigned(row)) * unsigned(sizeof(Real))));
          }
        }
      }
    };
    // steps (pi, yc) in order; pipelined (pipe_steps), the MFMAs of the next step are issued
    // before the stores of the current one, so the stores wait on finished accumulators only
    constexpr int NSTEP = NP * YCH;
    // embedded orders: a y chunk whose first y = (i1, j1) lies past the embedded j1 range
    // (j1 never decreases along y) stores nothing, and is skipped
    int ylim = 1 << 30;
    if constexpr (EMB) ylim = BC::R1a * eo.R1b;
    if constexpr (pipe_steps<S, P, Real>()) {
      Acc ping[YB], pong[YB];
      if (0 < ylim) mm(std::integral_constant<int, 0>{}, std::integral_constant<int, 0>{}, ping);
      static_for<NSTEP>([&](auto STEP) {
        constexpr int sp = decltype(STEP)::value, nx = sp + 1;
        if constexpr (nx < NSTEP) {
          if (nx / YCH < npg && (nx % YCH) * YB * 16 < ylim)
            mm(std::integral_constant<int, nx / YCH>{}, std::integral_constant<int, nx % YCH>{},
               (nx & 1) ? pong : ping);
        }
        if (sp / YCH < npg && (sp % YCH) * YB * 16 < ylim) {
          st(std::integral_constant<int, sp / YCH>{}, std::integral_constant<int, sp % YCH>{},
             (sp & 1) ? pong : ping);
          if constexpr (sp % YCH == YCH - 1) flush(std::integral_constant<int, sp / YCH>{});
        }
      });
    } else {
      static_for<NSTEP>([&](auto STEP) {
        constexpr int sp = decltype(STEP)::value;
        if (sp / YCH < npg && (sp % YCH) * YB * 16 < ylim) {
          Acc acc1[YB];
          mm(std::integral_constant<int, sp / YCH>{}, std::integral_constant<int, sp % YCH>{}, acc1);
          st(std::integral_constant<int, sp / YCH>{}, std::integral_constant<int, sp % YCH>{}, acc1);
          if constexpr (sp % YCH == YCH - 1) flush(std::integral_constant<int, sp / YCH>{});
        }
      });
    }
    // ---------------- y tail on the VALU ----------------
    // G[x][y] for the block's last YTAIL y: each lane sums its share of k = (g, l = 4 rho + lk)
    // of the stage-1 contraction from the stage-2 accumulator, and two exchanges between lane
    // groups (xor 16, 32) complete the sum, so every lane group holds G[x = xt*16 + arow(lr)][y].
    // Lane group lk then stores the lk-th tail y, with the masks of the MFMA tiles' stores.
    if constexpr (BC::YV) {
      static_assert(!HDE, "held column heads need whole y-tiles");
      const int xs = xt * 16 + M::arow(lr);
      int i2 = 0, j2 = 0;
      if (xs < NXv) decode_x<BC::R2a, DIAG>(sm.xd, xs, i2, j2);
      const int yl = BC::NYM * 16 + lk;
      const int i1 = yl % BC::R1a, j1 = yl / BC::R1a;
      const int il = i1 + (EMB ? eo.R1a : BC::R1a) * i2, jl = j1 + (EMB ? eo.R1b : BC::R1b) * j2;
      bool ok = xs < NXv && lk < BC::YTAIL && (!DIAG || i2 < j2 || i1 <= j1);
      if constexpr (EMB) ok = ok && i1 < eo.R1a && j1 < eo.R1b && i2 < eo.R2a && j2 < eo.R2b;
      static_for<NP>([&](auto PI) {
        constexpr int pi = decltype(PI)::value;
        if (pi < npg) {
          Real v = Real(0);
          static_for<BC::YTAIL>([&](auto TT) {
            constexpr int t = decltype(TT)::value;
            constexpr int y = BC::NYM * 16 + t, ti1 = y % BC::R1a, tj1 = y / BC::R1a;
            Real sum = Real(0);
            static_for<BC::NG>([&](auto G) {
              constexpr int g = decltype(G)::value;
              constexpr int r1 = BC::PL.gr1[g], s1 = BC::PL.gs1[g];
              static_for<RPP>([&](auto RHO) {
                constexpr int rho = decltype(RHO)::value;
                const Real u = sT[r1 * KTL + (ti1 + Sh::SH(A, 0)) * L + lk + 4 * rho] *
                               sT[s1 * KTL + (tj1 + Sh::SH(B, 0)) * L + lk + 4 * rho];
                sum += acc2[g][pi * RPP + rho] * u;
              });
            });
            sum += __shfl_xor(sum, 16);
            sum += __shfl_xor(sum, 32);
            if (lk == t) v = sum;
          });
          const unsigned J = unsigned(Jbp[pi] + jl);
          const unsigned off = (unsigned(Ibp[pi] + il) + ((__umul24(J, J) + J) >> 1)) * unsigned(sizeof(Real));
          const bool keep = ok && rok[pi] && (!dgp[pi] || il <= jl);
          store_out(v, rsrc, int(keep ? off : kDropOff));
        }
      });
    }
  }
}

// EMB: the points of direction d past ga.emb_L[d] carry zero weight (their fields are zero
// and their Jacobian is not checked)
template <int S, int P, typename Real, int A, int B, bool EMB>
__device__ __forceinline__ bool run_block(const GeneralArgs& ga, const SmemPtrs sm, int j3_lo, int j3_hi,
                                          Real* __restrict__ outp) {
  using Sh = Shape<S, P>;
  using BC = Blk<S, P, A, B>;
  using CF = Cfg<S, P, Real>;
  using R3 = S3Roles<S, P, Real, A, B>;
  using M = Mma<Real>;
  constexpr int L = Sh::L, L2 = L * L, L3 = L2 * L, KTL = KT * L, RPP = BC::RPP;
  Real* sF = static_cast<Real*>(sm.fld);
  const Real* sT = static_cast<const Real*>(sm.T);
  const Real* sT2 = static_cast<const Real*>(sm.T2);
  const int tid = threadIdx.x;
  const int lane = tid & 63, wave = tid >> 6;
  const int lr = lane & 15, lk = lane >> 4;

  // ---------------- metric -> coefficient fields, layout [f][n][m][l] ----------------
  for (int pt = tid; pt < L3; pt += NTHREADS) {
    const int l = pt % L, m = (pt / L) % L, n = pt / L2;
    if constexpr (EMB) {
      if (l >= ga.emb_L[0] || m >= ga.emb_L[1] || n >= ga.emb_L[2]) {
        static_for<BC::PL.nf>([&](auto F) {
          constexpr int f = decltype(F)::value;
          sF[(f * L + n) * L2 + m * L + l] = Real(0);
        });
        continue;
      }
    }
    double J[3][3], adj[3][3];
    jacobian_at(ga.geom_kind, sm.X, sm.z[l], sm.z2[m], sm.z3[n], J);
    const double det = adjugate(J, adj);
    if (!(det > 0.0)) *sm.bad = 1;
    const double idet = 1.0 / det;
    const double wq = sm.w[l] * sm.w2[m] * sm.w3[n];
    const double wv = wq * ga.w0, wd = wq * ga.w1;
    static_for<BC::PL.nf>([&](auto F) {
      constexpr int f = decltype(F)::value;
      constexpr int fid = BC::PL.fid[f];
      const double v = field_value(fid, J, adj, det, idet) * (field_weight(S, fid) ? wd : wv);
      sF[(f * L + n) * L2 + m * L + l] = static_cast<Real>(v);
    });
  }
  // ---------------- stage-1 table operand of this block ----------------
  if constexpr (CF::U1TAB) {
    Real* sU1 = static_cast<Real*>(sm.U1);
    constexpr int N = BC::NG * RPP * BC::NYT * 64;
    for (int i = tid; i < N; i += NTHREADS) {
      const int ln = i & 63, t = i >> 6;
      const int yt = t % BC::NYT, grh = t / BC::NYT, rho = grh % RPP, g = grh / RPP;
      const int y = yt * 16 + (ln & 15), l = 4 * rho + (ln >> 4);
      Real v = Real(0);
      if (y < BC::NY && l < L) {
        int r1 = 0, s1 = 0;
        static_for<BC::NG>([&](auto GG) {
          constexpr int gg = decltype(GG)::value;
          if (g == gg) { r1 = BC::PL.gr1[gg]; s1 = BC::PL.gs1[gg]; }
        });
        const int i1 = y % BC::R1a, j1 = y / BC::R1a;
        v = sT[r1 * KTL + (i1 + Sh::SH(A, 0)) * L + l] * sT[s1 * KTL + (j1 + Sh::SH(B, 0)) * L + l];
      }
      sU1[i] = v;
    }
  }
  __syncthreads();
  if (*sm.bad) return true;

  Regs<S, P, Real, A, B> rg;
  // ---------------- this thread's stage-3 field column, kept in registers ----------------
  if constexpr (R3::REGF) {
    if (tid < R3::W3 * R3::QS) {
      const int idx = tid % R3::W3, qs = tid / R3::W3;
      const int l = idx % L, m = (idx / L) % L;
      static_for<R3::QS>([&](auto QQ) {
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
  // ---------------- stage-2 table operand of this wave's fixed x-tile ----------------
  if constexpr (Cache2<S, P, Real, A, B>::ON) {
    const int xt = wave % BC::NXT;
    const int xs = xt * 16 + M::arow(lr);
    int i2 = 0, j2 = 0;
    if (xs < BC::NX) decode_x<BC::R2a, false>(sm.xd, xs, i2, j2);
    const int ia = (i2 + Sh::SH(A, 1)) * L + lk, jb = (j2 + Sh::SH(B, 1)) * L + lk;
    static_for<BC::NQ>([&](auto Q) {
      constexpr int q = decltype(Q)::value;
      static_for<RPP>([&](auto KS) {
        constexpr int ks = decltype(KS)::value;
        rg.u2[q * RPP + ks] = sT2[BC::PL.qr2[q] * KTL + ia + 4 * ks] * sT2[BC::PL.qs2[q] * KTL + jb + 4 * ks];
      });
    });
  }

  // ---------------- stage-1 table operands of all y-tiles ----------------
  if constexpr (Cache1<S, P, A, B>::ON) {
    static_for<BC::NG>([&](auto G) {
      constexpr int g = decltype(G)::value;
      static_for<RPP>([&](auto RHO) {
        constexpr int rho = decltype(RHO)::value;
        static_for<BC::NYT>([&](auto YT) {
          constexpr int yt = decltype(YT)::value;
          const int y = yt * 16 + lr;
          const int yy = y < BC::NY ? y : 0;
          const int i1 = yy % BC::R1a, j1 = yy / BC::R1a;
          rg.u1[(g * RPP + rho) * BC::NYT + yt] =
              sT[BC::PL.gr1[g] * KTL + (i1 + Sh::SH(A, 0)) * L + lk + 4 * rho] *
              sT[BC::PL.gs1[g] * KTL + (j1 + Sh::SH(B, 0)) * L + lk + 4 * rho];
        });
      });
    });
  }

  // ---------------- batches of pairs ----------------
  // ABUF == 2: [stage 3 (b+1) | stages 2+1 (b)] barrier ...
  // ABUF == 1: [stages 2+1 (b)] barrier [stage 3 (b+1)] barrier ...
  constexpr int NBP = CF::NBP;
  // diagonal pairs either close their slab in the full x tiling (inl) or come last, in
  // batches of their own with the triangular x tiling
  const bool inl = diag_inline_ok(S, P) && ga.diag_inline != 0;
  // blocks a < b of embedded orders only run the rows i3 of those orders
  const int r3a = EMB ? ga.emb_R[A][2] : BC::R3a;
  const int n_nd = A != B ? r3a * (j3_hi - j3_lo)
                 : inl ? (j3_hi * (j3_hi + 1) - j3_lo * (j3_lo + 1)) / 2
                       : (j3_hi * (j3_hi - 1) - j3_lo * (j3_lo - 1)) / 2;
  const int n_d = A == B && !inl ? j3_hi - j3_lo : 0;
  const int nb_nd = (n_nd + NBP - 1) / NBP;
  const int nbt = nb_nd + (n_d + NBP - 1) / NBP;
  auto batch = [&](int b, bool& dg, int& t0, int& np) {
    if (b < nb_nd) { dg = false; t0 = b * NBP; np = imin(NBP, n_nd - t0); }
    else { dg = true; t0 = (b - nb_nd) * NBP; np = imin(NBP, n_d - t0); }
  };
  Real* sA = static_cast<Real*>(sm.A);
  constexpr int ASTRIDE = CF::NB * CF::AONE;
  EmbOut eo{};
  if constexpr (EMB) {
    eo.R1a = ga.emb_R[A][0]; eo.R2a = ga.emb_R[A][1]; eo.R3a = ga.emb_R[A][2];
    eo.R1b = ga.emb_R[B][0]; eo.R2b = ga.emb_R[B][1];
    eo.off_a = ga.emb_off[A]; eo.off_b = ga.emb_off[B];
    eo.plen = ga.packed_len;
  }
  if (nbt > 0) {
    bool dg; int t0, np;
    batch(0, dg, t0, np);
    stage3<S, P, Real, A, B>(sm, rg, dg, t0, np, j3_lo, inl, sA, r3a);
  }
  __syncthreads();
  for (int b = 0; b < nbt; ++b) {
    bool dg; int t0, np;
    batch(b, dg, t0, np);
    const Real* cur = sA + (CF::ABUF == 2 ? (b & 1) * ASTRIDE : 0);
    if constexpr (CF::ABUF == 2) {
      if (b + 1 < nbt) {
        bool dn; int tn, nn;
        batch(b + 1, dn, tn, nn);
        stage3<S, P, Real, A, B>(sm, rg, dn, tn, nn, j3_lo, inl, sA + ((b + 1) & 1) * ASTRIDE, r3a);
      }
    }
    if (dg) work<S, P, Real, A, B, true, EMB>(sm, rg, t0, np, j3_lo, inl, cur, outp, eo);
    else work<S, P, Real, A, B, false, EMB>(sm, rg, t0, np, j3_lo, inl, cur, outp, eo);
    __syncthreads();
    if constexpr (CF::ABUF == 1) {
      if (b + 1 < nbt) {
        bool dn; int tn, nn;
        batch(b + 1, dn, tn, nn);
        stage3<S, P, Real, A, B>(sm, rg, dn, tn, nn, j3_lo, inl, sA, r3a);
        __syncthreads();
      }
    }
  }
  (void)lr;
  return false;
}

// Waves per SIMD the register allocation must allow: two when the LDS layout
// leaves room for two workgroups per CU and the register state fits without
// spilling: up to 8 points per direction, and in FP64 for H1 and H(curl) up to
// 10 points with the stage-3 fields kept in LDS (measured: H1 p = 9 13 % and
// H(curl) p = 8, 9 3 % faster than with one wave; L2 slower, H(div) unchanged,
// H(curl) p = 10 spills), else one.
template <int S, int P, typename Real> constexpr int min_waves() {
  constexpr int L = npoints(S, P);
  constexpr bool hi = sizeof(Real) == 8 && (S == SP_H1 || S == SP_HCURL) && L <= 10;
  constexpr int W = occ_target<S, P, Real>();
  if constexpr (W > 0) {
    if constexpr (Cfg<S, P, Real>::BYTES * W <= Cfg<S, P, Real>::BUDGET) return W;
  }
  return (Cfg<S, P, Real>::BYTES * 2 <= Cfg<S, P, Real>::BUDGET && (L <= DPG_MINW2_LMAX || hi)) ? 2 : 1;
}

// Per-direction rules (EMB): one table and point set per direction, each of a rule
// of emb_L[d] <= L points padded with zero-weight points to L.
template <typename Real, bool EMB> constexpr int n_dir_tables() { return EMB ? 3 : 1; }

// Body of the general-path kernels.  EMB: the orders (p1, p2, p3) <= P embedded in
// order P (the functions of order p_d in direction d are the first ones of order P: the
// 1D bases are hierarchical, Sections 2.4 and 2.8.2), each direction with its own rule,
// only the column slabs j3 < emb_jmax[b] of component b, and the stores write the
// embedded orders' packed numbering (entries outside it are dropped).
template <int S, int P, typename Real, bool LISTED, bool EMB>
__device__ __forceinline__ void general_body(const GeneralArgs& ga) {
  using Sh = Shape<S, P>;
  using CF = Cfg<S, P, Real>;
  constexpr int L = Sh::L;
  constexpr int ND = n_dir_tables<Real, EMB>();
  __shared__ Real s_fld[CF::FLD_LEN];
  __shared__ Real s_A[CF::ABUF * CF::NB * CF::AONE];
  __shared__ Real s_U1[CF::U1TAB ? CF::U1_LEN : 1];
  __shared__ Real s_T[ND * CF::T_LEN];
  __shared__ Real s_hd[CF::HD ? CF::HD_LEN : 1];
  __shared__ double s_z[ND * L], s_w[ND * L], s_X[24];
  __shared__ unsigned char s_xd[2 * 80];
  __shared__ int s_bad;

  const int tid = threadIdx.x;
  const int G = ga.slab_group;                                // slabs per workgroup
  const int ngroups = (Sh::NSLAB + G - 1) / G;
  // one (item, slab group) of the launch
  auto run = [&](int64_t blk, int64_t n_items, const int32_t* ids) {
    const int grp = ngroups - 1 - int(blk / n_items);                 // heaviest slab groups first
    const int64_t item = ga.item_base + blk % n_items;
    const int64_t e = ids ? int64_t(ids[item]) : item;
    const int s_lo = grp * G, s_hi = imin(Sh::NSLAB, s_lo + G);

    if constexpr (EMB) {
      // direction d: its rule's tables with stride L, zero past its emb_L[d] points; the
      // padding points sit at the centre with weight zero
      static_for<3>([&](auto D) {
        constexpr int d = decltype(D)::value;
        const int Ld = ga.emb_L[d];
        const Real* tR = static_cast<const Real*>(ga.emb_tabR[d]);
        for (int i = tid; i < CF::T_LEN; i += NTHREADS) {
          const int l = i % L, f = i / L;
          s_T[d * CF::T_LEN + i] = i < 2 * KT * L && l < Ld ? tR[2 * Ld + f * Ld + l] : Real(0);
        }
        if (tid < L) {
          s_z[d * L + tid] = tid < Ld ? ga.emb_tab64[d][tid] : 0.5;
          s_w[d * L + tid] = tid < Ld ? ga.emb_tab64[d][Ld + tid] : 0.0;
        }
      });
    } else {
      const Real* tR = static_cast<const Real*>(ga.tabR);
      for (int i = tid; i < CF::T_LEN; i += NTHREADS) s_T[i] = i < 2 * KT * L ? tR[2 * L + i] : Real(0);
    }
    // stage-3 output buffers: the padding rows (m >= L) and columns (l >= L) stay zero
    for (int i = tid; i < CF::ABUF * CF::NB * CF::AONE; i += NTHREADS) s_A[i] = Real(0);
    if constexpr (!EMB) {
      if (tid < L) { s_z[tid] = ga.tab64[tid]; s_w[tid] = ga.tab64[L + tid]; }
    }
    const int ng = geom_stride(ga.geom_kind);
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

    constexpr int D2 = EMB ? 1 : 0, D3 = EMB ? 2 : 0;
    SmemPtrs sm{s_fld, s_A, s_U1, s_T, s_hd, s_z, s_w, s_X, s_xd, &s_bad,
                s_T + D2 * CF::T_LEN, s_T + D3 * CF::T_LEN, s_z + D2 * L, s_z + D3 * L, s_w + D2 * L, s_w + D3 * L};
    Real* outp = static_cast<Real*>(ga.out) + (ga.out_offset ? ga.out_offset[e] : e * ga.packed_len);
    // component b owns slabs [slab0(b), slab0(b) + R3(b)); visit the blocks (a, b), a <= b,
    // for the j3 range of every component the slab group touches
    bool bad = false;
    auto jr = [&](int b, int& lo, int& hi) {
      lo = imax(s_lo, Sh::slab0(b)) - Sh::slab0(b);
      hi = imin(s_hi, Sh::slab0(b) + Sh::R(b, 2)) - Sh::slab0(b);
      if constexpr (EMB) hi = imin(hi, ga.emb_jmax[b]);
      return lo < hi;
    };
    int lo, hi;
    if (jr(0, lo, hi)) bad = run_block<S, P, Real, 0, 0, EMB>(ga, sm, lo, hi, outp);
    if constexpr (Sh::NC == 3) {
      if (!bad && jr(1, lo, hi)) {
        bad = run_block<S, P, Real, 0, 1, EMB>(ga, sm, lo, hi, outp);
        if (!bad) bad = run_block<S, P, Real, 1, 1, EMB>(ga, sm, lo, hi, outp);
      }
      if (!bad && jr(2, lo, hi)) {
        bad = run_block<S, P, Real, 0, 2, EMB>(ga, sm, lo, hi, outp);
        if (!bad) bad = run_block<S, P, Real, 1, 2, EMB>(ga, sm, lo, hi, outp);
        if (!bad) bad = run_block<S, P, Real, 2, 2, EMB>(ga, sm, lo, hi, outp);
      }
    }
    if (EMB && bad) {
      // the embedded orders' columns of this group's slabs, component by component
      for (int b = 0; b < Sh::NC; ++b) {
        if (!jr(b, lo, hi)) continue;
        const int64_t w = int64_t(ga.emb_R[b][0]) * ga.emb_R[b][1];
        const int64_t J0 = ga.emb_off[b] + w * lo, J1 = ga.emb_off[b] + w * hi;
        for (int64_t i = J0 * (J0 + 1) / 2 + tid; i < J1 * (J1 + 1) / 2; i += NTHREADS) outp[i] = Real(0);
      }
    } else if (bad) {
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

template <int S, int P, typename Real, bool LISTED>
__global__ void __launch_bounds__(NTHREADS, (min_waves<S, P, Real>())) k_general(GeneralArgs ga) {
  general_body<S, P, Real, LISTED, false>(ga);
}

// Workgroups per CU for the per-direction-rule kernel: the uniform kernel's choice where
// its two extra tables still fit beside them, at most three (four spilled at H1 p = 3).
template <int S, int P, typename Real> constexpr int min_waves_emb() {
  constexpr int W = imin(3, min_waves<S, P, Real>());
  constexpr int XB = 2 * Cfg<S, P, Real>::T_LEN * int(sizeof(Real)) + 4 * npoints(S, P) * 8;
  return (Cfg<S, P, Real>::BYTES + XB) * W <= Cfg<S, P, Real>::BUDGET ? W : (W > 1 ? W - 1 : 1);
}

template <int S, int P, typename Real>
__global__ void __launch_bounds__(NTHREADS, (min_waves_emb<S, P, Real>())) k_embed(GeneralArgs ga) {
  general_body<S, P, Real, false, true>(ga);
}

// One (space, p, precision): a plain launch (split into launches under the
// dispatch limits) or, with LISTED, one listed launch of a fixed grid.
template <int S, int P, typename Real, bool LISTED>
hipError_t launch_general_one(const GeneralArgs& a, hipStream_t st) {
  constexpr int NS = Shape<S, P>::NSLAB;
  GeneralArgs c = a;
  c.slab_group = slab_group_for(NS, a.n_items, a.slab_group);
  if (c.diag_inline < 0 || !diag_inline_ok(S, P)) c.diag_inline = diag_inline_ok(S, P) ? 1 : 0;
  const int ngroups = (NS + c.slab_group - 1) / c.slab_group;
  if constexpr (LISTED) {
    hipLaunchKernelGGL((k_general<S, P, Real, true>), dim3(list_grid(a.n_items, ngroups)), dim3(NTHREADS), 0, st, c);
  } else {
    const int64_t max_items = launch_items(ngroups);
    for (int64_t base = 0; base < a.n_items; base += max_items) {
      c.item_base = a.item_base + base;
      c.n_items = (a.n_items - base) < max_items ? (a.n_items - base) : max_items;
      hipLaunchKernelGGL((k_general<S, P, Real, false>), dim3(unsigned(c.n_items * ngroups)), dim3(NTHREADS), 0, st,
                         c);
    }
  }
  return hipGetLastError();
}

template <int S, typename Real, bool LISTED>
hipError_t dispatch_general_p(int p, const GeneralArgs& a, hipStream_t st) {
  switch (p) {
    case 1: return launch_general_one<S, 1, Real, LISTED>(a, st);
    case 2: return launch_general_one<S, 2, Real, LISTED>(a, st);
    case 3: return launch_general_one<S, 3, Real, LISTED>(a, st);
    case 4: return launch_general_one<S, 4, Real, LISTED>(a, st);
    case 5: return launch_general_one<S, 5, Real, LISTED>(a, st);
    case 6: return launch_general_one<S, 6, Real, LISTED>(a, st);
    case 7: return launch_general_one<S, 7, Real, LISTED>(a, st);
    case 8: return launch_general_one<S, 8, Real, LISTED>(a, st);
    case 9: return launch_general_one<S, 9, Real, LISTED>(a, st);
    case 10: return launch_general_one<S, 10, Real, LISTED>(a, st);
    case 11: return launch_general_one<S, 11, Real, LISTED>(a, st);
    default: return hipErrorInvalidValue;
  }
}

// Per-direction rules embedded in order P: plain launches of k_embed (orders up to 10).
template <int S, int P, typename Real>
hipError_t launch_embed_one(const GeneralArgs& a, hipStream_t st) {
  constexpr int NS = Shape<S, P>::NSLAB;
  GeneralArgs c = a;
  c.slab_group = slab_group_for(NS, a.n_items, a.slab_group);
  if (c.diag_inline < 0 || !diag_inline_ok(S, P)) c.diag_inline = diag_inline_ok(S, P) ? 1 : 0;
  const int ngroups = (NS + c.slab_group - 1) / c.slab_group;
  const int64_t max_items = launch_items(ngroups);
  for (int64_t base = 0; base < a.n_items; base += max_items) {
    c.item_base = a.item_base + base;
    c.n_items = (a.n_items - base) < max_items ? (a.n_items - base) : max_items;
    hipLaunchKernelGGL((k_embed<S, P, Real>), dim3(unsigned(c.n_items * ngroups)), dim3(NTHREADS), 0, st, c);
  }
  return hipGetLastError();
}

template <int S, typename Real>
hipError_t dispatch_embed_p(int p, const GeneralArgs& a, hipStream_t st) {
  switch (p) {
    case 1: return launch_embed_one<S, 1, Real>(a, st);
    case 2: return launch_embed_one<S, 2, Real>(a, st);
    case 3: return launch_embed_one<S, 3, Real>(a, st);
    case 4: return launch_embed_one<S, 4, Real>(a, st);
    case 5: return launch_embed_one<S, 5, Real>(a, st);
    case 6: return launch_embed_one<S, 6, Real>(a, st);
    case 7: return launch_embed_one<S, 7, Real>(a, st);
    case 8: return launch_embed_one<S, 8, Real>(a, st);
    case 9: return launch_embed_one<S, 9, Real>(a, st);
    case 10: return launch_embed_one<S, 10, Real>(a, st);
    default: return hipErrorInvalidValue;
  }
}

template <int S>
hipError_t dispatch_embed(int p, int prec, const GeneralArgs& a, hipStream_t st) {
  return prec ? dispatch_embed_p<S, float>(p, a, st) : dispatch_embed_p<S, double>(p, a, st);
}

// Plain launches (LISTED = false) and listed ones are instantiated in separate files,
// so the build compiles them in parallel.
template <int S, bool LISTED>
hipError_t dispatch_general(int p, int prec, const GeneralArgs& a, hipStream_t st) {
  return prec ? dispatch_general_p<S, float, LISTED>(p, a, st) : dispatch_general_p<S, double, LISTED>(p, a, st);
}

}  // namespace dpg
