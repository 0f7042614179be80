// terms.h -- compile-time description of the four Gram integrands.
//
// A shape function of component a is prod_d T^<r_d>_{i_d + sigma_d(a)}(xi_d) e_a,
// with T^<0>_k = chi_k = L_k and T^<1>_k = chi'_k (the superscript notation of
// (2.37)).  Block (a, b) of the Gram matrix is a sum of terms, each a metric
// coefficient field c(xi) times prod_d T^<r_d>_{i_d+sigma_d(a)} T^<s_d>_{j_d+sigma_d(b)}:
//
//   H1      c = |J|            r = s = (0,0,0)                     (2.31), (2.41)-(2.43)
//           c = D_AB |J|       r = e_A, s = e_B   (A, B = 1..3)     (2.36), (2.38)-(2.40)
//   L2      c = 1/|J|          r = s = (1,1,1), shift 1            (2.16), (2.54)
//   H(div)  c = C_ab / |J|     r = 1 - e_a, s = 1 - e_b            (2.60)-(2.63)
//           c = 1/|J|          r = s = (1,1,1)                     (2.59)
//   H(curl) c = D_ab |J|       r = e_a, s = e_b                    (2.76), (2.81)-(2.83)
//           c = (-1)^(al+be) C_(a+al)(b+be) / |J|,  al, be in {1,2},
//                              r = 1 - e_(a+al), s = 1 - e_(b+be)  (2.77)-(2.80), (2.84)
//
// with D = J^-1 J^-T (2.32) and C = J^T J (2.50).  Index shifts sigma_d(a):
// H1 0, L2 1, H(div) 1 - delta_da (2.57), H(curl) delta_da (2.74).
// (Readings: the garbled superscripts of (2.72), (2.73), (2.83) and of
// Algorithm 9 are taken as the component-consistent forms written above.)
//
// The staged contraction integrates xi_3 first (stage 3), then xi_2, then
// xi_1.  Terms that share (r1,s1,r2,s2) share stages 2 and 1 ("q slots");
// q slots that share (r1,s1) share stage 1 ("groups").  The value part of
// each inner product is weighted by w0 and the derivative part by w1.
#pragma once

namespace dpg {

enum : int { SP_H1 = 0, SP_HCURL = 1, SP_HDIV = 2, SP_L2 = 3 };

enum : int {
  FLD_DETJ = 0,                                          // |J|
  FLD_D11, FLD_D22, FLD_D33, FLD_D12, FLD_D13, FLD_D23,  // D_ab |J|
  FLD_C11, FLD_C22, FLD_C33, FLD_C12, FLD_C13, FLD_C23,  // C_ab / |J|
  FLD_IDETJ,                                             // 1 / |J|
  FLD_COUNT
};

constexpr int sym_slot(int a, int b) {
  return a == b ? a : ((a + b) == 1 ? 3 : ((a + b) == 2 ? 4 : 5));
}
constexpr int fld_D(int a, int b) { return FLD_D11 + sym_slot(a, b); }
constexpr int fld_C(int a, int b) { return FLD_C11 + sym_slot(a, b); }
constexpr int fld_is_D(int f) { return f >= FLD_D11 && f <= FLD_D23; }
constexpr int fld_is_C(int f) { return f >= FLD_C11 && f <= FLD_C23; }
// the two indices of a symmetric D/C slot
constexpr int sym_a(int slot) { return slot < 3 ? slot : (slot == 5 ? 1 : 0); }
constexpr int sym_b(int slot) { return slot < 3 ? slot : (slot == 3 ? 1 : 2); }

// 0: field belongs to the value part (weight w0), 1: derivative part (w1)
constexpr int field_weight(int space, int f) {
  return space == SP_H1 ? (f == FLD_DETJ ? 0 : 1)
       : space == SP_HCURL ? (fld_is_D(f) ? 0 : 1)
       : space == SP_HDIV ? (fld_is_C(f) ? 0 : 1)
       : 0;
}

constexpr int ncomp(int space) { return (space == SP_H1 || space == SP_L2) ? 1 : 3; }

constexpr int range1d(int space, int p, int a, int d) {
  return space == SP_H1 ? p + 1
       : space == SP_L2 ? p
       : space == SP_HDIV ? (d == a ? p + 1 : p)
       : (d == a ? p : p + 1);
}

constexpr int shift1d(int space, int a, int d) {
  return space == SP_H1 ? 0
       : space == SP_L2 ? 1
       : space == SP_HDIV ? (d == a ? 0 : 1)
       : (d == a ? 1 : 0);
}

constexpr int npoints(int space, int p) { return space == SP_L2 ? p : p + 1; }
// Diagonal (i3 = j3) pairs closing their slab in the full x tiling, lower triangle
// dropped, are built where a stage-2 row tile holds two or more pairs (L <= 8
// points), so the diagonal pair shares its tile; with one pair per tile the
// triangular x tiling of a separate diagonal pass is cheaper.
constexpr bool diag_inline_ok(int space, int p) { return npoints(space, p) <= 8; }

struct Term {
  int field;
  int sign;
  int r[3];
  int s[3];
};

struct Plan {
  int nt;
  Term t[10];
  int nf;          // distinct fields used by the block
  int fid[8];
  int tf[10];      // term -> field slot
  int nq;          // distinct (r1,s1,r2,s2)
  int qr1[10], qs1[10], qr2[10], qs2[10];
  int tq[10];      // term -> q slot
  int ng;          // distinct (r1,s1)
  int gr1[4], gs1[4];
  int qg[10];      // q slot -> group
};

constexpr void plan_add(Plan& P, int field, int sign, int r0, int r1, int r2, int s0, int s1, int s2) {
  Term& t = P.t[P.nt++];
  t.field = field;
  t.sign = sign;
  t.r[0] = r0; t.r[1] = r1; t.r[2] = r2;
  t.s[0] = s0; t.s[1] = s1; t.s[2] = s2;
}

constexpr void plan_finish(Plan& P);

// The terms of block (a, b), before grouping.
constexpr Plan plan_terms(int space, int a, int b) {
  Plan P{};
  if (space == SP_H1) {
    plan_add(P, FLD_DETJ, 1, 0, 0, 0, 0, 0, 0);
    for (int A = 0; A < 3; ++A)
      for (int B = 0; B < 3; ++B)
        plan_add(P, fld_D(A, B), 1, A == 0, A == 1, A == 2, B == 0, B == 1, B == 2);
  } else if (space == SP_L2) {
    plan_add(P, FLD_IDETJ, 1, 1, 1, 1, 1, 1, 1);
  } else if (space == SP_HDIV) {
    plan_add(P, fld_C(a, b), 1, a != 0, a != 1, a != 2, b != 0, b != 1, b != 2);
    plan_add(P, FLD_IDETJ, 1, 1, 1, 1, 1, 1, 1);
  } else {
    plan_add(P, fld_D(a, b), 1, a == 0, a == 1, a == 2, b == 0, b == 1, b == 2);
    for (int al = 1; al <= 2; ++al)
      for (int be = 1; be <= 2; ++be) {
        const int ca = (a + al) % 3, cb = (b + be) % 3;
        plan_add(P, fld_C(ca, cb), ((al + be) & 1) ? -1 : 1,
                 ca != 0, ca != 1, ca != 2, cb != 0, cb != 1, cb != 2);
      }
  }
  return P;
}

// Fields, q slots and groups of the terms in P.
constexpr void plan_finish(Plan& P) {
  for (int i = 0; i < P.nt; ++i) {
    int f = -1;
    for (int j = 0; j < P.nf; ++j)
      if (P.fid[j] == P.t[i].field) f = j;
    if (f < 0) { f = P.nf; P.fid[P.nf++] = P.t[i].field; }
    P.tf[i] = f;
    int q = -1;
    for (int j = 0; j < P.nq; ++j)
      if (P.qr1[j] == P.t[i].r[0] && P.qs1[j] == P.t[i].s[0] &&
          P.qr2[j] == P.t[i].r[1] && P.qs2[j] == P.t[i].s[1]) q = j;
    if (q < 0) {
      q = P.nq++;
      P.qr1[q] = P.t[i].r[0]; P.qs1[q] = P.t[i].s[0];
      P.qr2[q] = P.t[i].r[1]; P.qs2[q] = P.t[i].s[1];
    }
    P.tq[i] = q;
  }
  for (int q = 0; q < P.nq; ++q) {
    int g = -1;
    for (int j = 0; j < P.ng; ++j)
      if (P.gr1[j] == P.qr1[q] && P.gs1[j] == P.qs1[q]) g = j;
    if (g < 0) { g = P.ng++; P.gr1[g] = P.qr1[q]; P.gs1[g] = P.qs1[q]; }
    P.qg[q] = g;
  }
}

constexpr Plan make_plan(int space, int a, int b) {
  Plan P = plan_terms(space, a, b);
  plan_finish(P);
  return P;
}

// Extruded maps (the second form of (2.89)): x1 depends on xi1 alone, through a
// constant lambda1, and (x2, x3) on (xi2, xi3) alone, so J, D = J^-1 J^-T and
// C = J^T J are block diagonal and their (1,2), (1,3) entries vanish.  The
// block's terms without those fields, regrouped.
constexpr bool ext_vanishes(int f) {
  return (fld_is_D(f) || fld_is_C(f)) && (f - (fld_is_D(f) ? FLD_D11 : FLD_C11) == 3 ||
                                          f - (fld_is_D(f) ? FLD_D11 : FLD_C11) == 4);
}
constexpr Plan make_ext_plan(int space, int a, int b) {
  const Plan T = plan_terms(space, a, b);
  Plan P{};
  for (int i = 0; i < T.nt; ++i)
    if (!ext_vanishes(T.t[i].field)) P.t[P.nt++] = T.t[i];
  plan_finish(P);
  return P;
}

// ---------------------------------------------------------------------------
// sizes
// ---------------------------------------------------------------------------

constexpr int comp_dim(int space, int p, int a) {
  return range1d(space, p, a, 0) * range1d(space, p, a, 1) * range1d(space, p, a, 2);
}
constexpr int comp_off(int space, int p, int a) {
  int o = 0;
  for (int c = 0; c < a; ++c) o += comp_dim(space, p, c);
  return o;
}
constexpr long long gram_dim(int space, int p) { return comp_off(space, p, ncomp(space)); }
constexpr long long packed_len(int space, int p) {
  return gram_dim(space, p) * (gram_dim(space, p) + 1) / 2;
}

// Flops of the staged contraction of one element over the upper block
// triangle (the (i3, j3) pairs a < b, or a == b and i3 <= j3): stage 3 2 L^3
// per term and pair, stage 2 2 L^2 per q slot, l and (i2, j2), stage 1 2 L per
// group and packed output entry.  Stage 2 runs over every (i2, j2) of a pair;
// with trim_diag the diagonal pairs (a == b, i3 == j3) count only i2 <= j2,
// the part of their stage 2 that the upper triangle needs (what the kernels
// compute).
constexpr double general_flops(int space, int p, bool trim_diag = false) {
  const int L = npoints(space, p);
  const int nc = ncomp(space);
  double f = 0.0;
  for (int a = 0; a < nc; ++a)
    for (int b = a; b < nc; ++b) {
      const Plan P = make_plan(space, a, b);
      const int R1a = range1d(space, p, a, 0), R1b = range1d(space, p, b, 0);
      const int R2a = range1d(space, p, a, 1), R2b = range1d(space, p, b, 1);
      const int R3a = range1d(space, p, a, 2), R3b = range1d(space, p, b, 2);
      double pairs_full = 0.0, pairs_diag = 0.0;
      if (a == b) { pairs_diag = R3a; pairs_full = R3a * (R3a - 1) / 2.0; }
      else { pairs_diag = 0; pairs_full = double(R3a) * R3b; }
      const double n2_full = double(R2a) * R2b;
      const double n2_diag = trim_diag ? R2a * (R2a + 1) / 2.0 : n2_full;
      const double n1 = double(R1a) * R1b;
      const double n1_tri = R1a * (R1a + 1) / 2.0;  // i2 == j2 rows of a diagonal pair
      const double out_full = n1 * n2_full;
      const double out_diag = n1 * (R2a * (R2a + 1) / 2.0 - R2a) + n1_tri * R2a;
      const double pairs = pairs_full + pairs_diag;
      f += pairs * 2.0 * L * L * L * P.nt;
      f += (pairs_full * n2_full + pairs_diag * n2_diag) * 2.0 * L * L * P.nq;
      f += (pairs_full * out_full + pairs_diag * out_diag) * 2.0 * L * P.ng;
    }
  return f;
}

}  // namespace dpg
