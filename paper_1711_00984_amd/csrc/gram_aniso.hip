// gram_aniso.hip -- element Grams of non-uniform orders (p1, p2, p3).
//
// When the orders differ per direction, each coordinate can take its own 1D
// Gauss rule (L_d = p_d + 1 points, p_d for L2), and the nesting of the staged
// quadrature should put the coordinate of least order in the outermost loop
// (text after Algorithm 2): the last contraction costs L_out times the number
// of entries, so L_out should be the smallest.  The directions are therefore
// contracted in the order dir[0], dir[1], dir[2] (the least order).  dir[0] is
// xi3, the slowest index of the flat numbering, whenever xi3 is not the least
// order, so that a diagonal block can skip the pairs i3 > j3 whole; otherwise
// the last stage skips them.  The integrands are the terms of Sections 2.3-2.6,
// as in the uniform kernels; component a of a space spans R_d(a) functions in
// direction d, from p_d.
//
// One workgroup per (element, component block a <= b), FP64 or FP32 VALU, LDS
// sized by the host for the launch's point counts and ranges:
//   fields  c_t at all L1 L2 L3 points (FP64 metric, times the weights) -> LDS
//   for each pair (iA, jA) of the first direction (several at once for small blocks):
//     stage A: A_g[qC][qB]             = sum_qA c_t T_A T_A            (terms -> groups g)
//     stage B: B_h[qC][jB][iB]         = sum_qB T_B T_B A_g            (groups -> groups h)
//     stage C: G[(iA,iB,iC),(jA,jB,jC)] = sum_h sum_qC T_C T_C B_h     -> packed 'U' output
// Terms sharing their derivative flags in directions B and C share stages B
// and C; groups sharing them in direction C share stage C.
#include <hip/hip_runtime.h>

#include <algorithm>

#include "aniso.h"
#include "kernels.h"
#include "metric.h"
#include "terms.h"

namespace dpg {

namespace {

constexpr int NTA = 256;
constexpr int MT = 10;                                      // terms per block (H1)
constexpr int MF = 7;                                       // distinct fields per block (H1)
constexpr int MH = 4;                                       // stage-C groups
constexpr int TSTRIDE = ANISO_LMAX;                         // table row length in LDS
constexpr int TDIR = 2 * KT * TSTRIDE;                      // one direction: chi then chi'
constexpr int64_t kMaxGrid = int64_t(1) << 22;

struct Meta {
  int nt, nf, ng, nh;
  int fid[MF];          // metric field of each distinct field
  int tf[MT];           // term -> distinct field
  double coef[MT];      // term sign times w0 or w1
  int r[MT][3], s[MT][3];
  int tg[MT];           // term -> stage-A group
  int gr[MT][3], gs[MT][3];   // flags of each stage-A group (directions B and C meaningful)
  int gh[MT];           // stage-A group -> stage-C group
  int hr[MH], hs[MH];   // flags of each stage-C group in direction C
};

__device__ __forceinline__ int shift_of(int space, int a, int d) {
  return space == SP_H1 ? 0 : space == SP_L2 ? 1 : space == SP_HDIV ? (d == a ? 0 : 1) : (d == a ? 1 : 0);
}
__device__ __forceinline__ int range_of(int space, const int* q, int a, int d) {
  return space == SP_H1 ? q[d] + 1 : space == SP_L2 ? q[d] : space == SP_HDIV ? (d == a ? q[d] + 1 : q[d])
                                                                               : (d == a ? q[d] : q[d] + 1);
}

// Terms of block (a, b) (the integrands listed in terms.h), their fields and groups.
__device__ void build_meta(int space, int a, int b, double w0, double w1, const int* dir, Meta& m) {
  m.nt = 0;
  auto add = [&](int f, double c, int ra, int rb) {   // ra / rb: direction whose flag is set (-1: none, 3: all)
    const int t = m.nt++;
    m.tf[t] = f;
    m.coef[t] = c;
    for (int d = 0; d < 3; ++d) {
      m.r[t][d] = ra == 3 ? 1 : (d == ra ? 1 : 0);
      m.s[t][d] = rb == 3 ? 1 : (d == rb ? 1 : 0);
    }
  };
  auto add_co = [&](int f, double c, int ca, int cb) {  // flags 1 - e_ca, 1 - e_cb
    const int t = m.nt++;
    m.tf[t] = f;
    m.coef[t] = c;
    for (int d = 0; d < 3; ++d) {
      m.r[t][d] = d == ca ? 0 : 1;
      m.s[t][d] = d == cb ? 0 : 1;
    }
  };
  if (space == SP_H1) {
    add(FLD_DETJ, w0, -1, -1);
    for (int A = 0; A < 3; ++A)
      for (int B = 0; B < 3; ++B) add(fld_D(A, B), w1, A, B);
  } else if (space == SP_L2) {
    add(FLD_IDETJ, w0, 3, 3);
  } else if (space == SP_HDIV) {
    add_co(fld_C(a, b), w0, a, b);
    add(FLD_IDETJ, w1, 3, 3);
  } else {
    add(fld_D(a, b), w0, a, b);
    for (int al = 1; al <= 2; ++al)
      for (int be = 1; be <= 2; ++be) {
        const int ca = (a + al) % 3, cb = (b + be) % 3;
        add_co(fld_C(ca, cb), ((al + be) & 1) ? -w1 : w1, ca, cb);
      }
  }
  // distinct fields
  m.nf = 0;
  for (int t = 0; t < m.nt; ++t) {
    int k = 0;
    while (k < m.nf && m.fid[k] != m.tf[t]) ++k;
    if (k == m.nf) m.fid[m.nf++] = m.tf[t];
    m.tf[t] = k;
  }
  const int dB = dir[1], dC = dir[2];
  // stage-A groups: same flags in directions B and C
  m.ng = 0;
  for (int t = 0; t < m.nt; ++t) {
    int g = 0;
    while (g < m.ng && !(m.gr[g][dB] == m.r[t][dB] && m.gs[g][dB] == m.s[t][dB] && m.gr[g][dC] == m.r[t][dC] &&
                         m.gs[g][dC] == m.s[t][dC]))
      ++g;
    if (g == m.ng) {
      for (int d = 0; d < 3; ++d) {
        m.gr[g][d] = m.r[t][d];
        m.gs[g][d] = m.s[t][d];
      }
      ++m.ng;
    }
    m.tg[t] = g;
  }
  // stage-C groups: same flags in direction C
  m.nh = 0;
  for (int g = 0; g < m.ng; ++g) {
    int h = 0;
    while (h < m.nh && !(m.hr[h] == m.gr[g][dC] && m.hs[h] == m.gs[g][dC])) ++h;
    if (h == m.nh) {
      m.hr[h] = m.gr[g][dC];
      m.hs[h] = m.gs[g][dC];
      ++m.nh;
    }
    m.gh[g] = h;
  }
}

template <typename Real>
__global__ void __launch_bounds__(NTA) k_aniso(AnisoArgs A, int nblk, int64_t item0) {
  __shared__ Real s_tab[3 * TDIR];          // direction d: chi^<r>_k(zeta_l) at d TDIR + r KT TSTRIDE + k TSTRIDE + l
  // fields (point q = qA + LA (qB + LB qC)), then P pairs' stage-A and stage-B buffers,
  // sized by the host for this launch
  extern __shared__ __align__(16) unsigned char s_dyn[];
  Real* const s_F = reinterpret_cast<Real*>(s_dyn);
  Real* const s_A = s_F + A.lds_fields;
  Real* const s_B = s_A + A.pairs * A.lds_a;
  __shared__ Meta m;
  __shared__ int s_bad;

  const int64_t item = item0 + blockIdx.x;
  const int64_t e = item / nblk;
  if (e >= A.n_elem) return;
  int blk = int(item % nblk), a = 0, b = 0;
  while (blk >= 3 - a) {                    // (a, b), a <= b, in the order (0,0) (0,1) (0,2) (1,1) (1,2) (2,2)
    blk -= 3 - a;
    ++a;
  }
  b = a + blk;
  const int tid = threadIdx.x;
  const int sp = A.space;
  const int dA = A.dir[0], dB = A.dir[1], dC = A.dir[2];
  const int LA = A.L[dA], LB = A.L[dB], LC = A.L[dC];
  const int Q = LA * LB * LC;

  if (tid == 0) {
    build_meta(sp, a, b, A.w0, A.w1, A.dir, m);
    s_bad = 0;
  }
  for (int k = tid; k < 3 * TDIR; k += NTA) {
    const int d = k / TDIR, rem = k % TDIR, r = rem / (KT * TSTRIDE), kk = (rem / TSTRIDE) % KT, l = rem % TSTRIDE;
    const int L = A.L[d];
    const Real* t = static_cast<const Real*>(A.tabR[d]);
    s_tab[k] = l < L ? t[2 * L + (r * KT + kk) * L + l] : Real(0);
  }
  __syncthreads();

  // metric fields, weighted
  const double* X = A.geom + e * geom_stride(A.geom_kind);
  for (int q = tid; q < Q; q += NTA) {
    const int qA = q % LA, qB = (q / LA) % LB, qC = q / (LA * LB);
    int qd[3];
    qd[dA] = qA;
    qd[dB] = qB;
    qd[dC] = qC;
    double xi[3], w = 1.0;
    for (int d = 0; d < 3; ++d) {
      xi[d] = A.tab64[d][qd[d]];
      w *= A.tab64[d][A.L[d] + qd[d]];
    }
    double J[3][3], adj[3][3];
    jacobian_at(A.geom_kind, X, xi[0], xi[1], xi[2], J);
    const double det = adjugate(J, adj);
    if (!(det > 0.0)) s_bad = 1;
    const double idet = 1.0 / det;
    for (int f = 0; f < m.nf; ++f) s_F[f * Q + q] = Real(field_value(m.fid[f], J, adj, det, idet) * w);
  }
  __syncthreads();

  int Ra[3], Rb[3], sa[3], sb[3];
  for (int d = 0; d < 3; ++d) {
    Ra[d] = range_of(sp, A.q, a, d);
    Rb[d] = range_of(sp, A.q, b, d);
    sa[d] = shift_of(sp, a, d);
    sb[d] = shift_of(sp, b, d);
  }
  int offa = 0, offb = 0;
  for (int c = 0; c < b; ++c) {
    const int nc = range_of(sp, A.q, c, 0) * range_of(sp, A.q, c, 1) * range_of(sp, A.q, c, 2);
    if (c < a) offa += nc;
    offb += nc;
  }
  Real* out = static_cast<Real*>(A.out) + e * A.packed_len;
  const int nB = Ra[dB] * Rb[dB];
  auto entry = [&](int iA, int jA, int iB, int jB, int iC, int jC, int64_t& I, int64_t& J) {
    int i[3], j[3];
    i[dA] = iA; i[dB] = iB; i[dC] = iC;
    j[dA] = jA; j[dB] = jB; j[dC] = jC;
    I = offa + i[0] + Ra[0] * (i[1] + Ra[1] * i[2]);
    J = offb + j[0] + Rb[0] * (j[1] + Rb[1] * j[2]);
  };

  if (s_bad) {                              // det J <= 0 somewhere: zero this block, flag the element
    const int64_t na = int64_t(Ra[0]) * Ra[1] * Ra[2], nb = int64_t(Rb[0]) * Rb[1] * Rb[2];
    for (int64_t k = tid; k < na * nb; k += NTA) {
      const int64_t I = offa + k % na, J = offb + k / na;
      if (a != b || I <= J) out[I + J * (J + 1) / 2] = Real(0);
    }
    if (tid == 0 && A.status) A.status[e] = -4;
    return;
  }
  if (tid == 0 && A.status && a == 0 && b == 0) A.status[e] = 0;

  auto tab = [&](int d, int r, int k, int l) { return s_tab[d * TDIR + (r * KT + k) * TSTRIDE + l]; };

  const int RaB = Ra[dB], RaC = Ra[dC], RbC = Rb[dC];
  // Pairs (iA, jA) still to do (a diagonal block with xi3 first skips i3 > j3), taken P
  // at a time when the stage buffers hold P pairs' intermediates: small blocks would
  // otherwise leave most threads idle between two barriers.
  const int nAs = m.ng * LC * LB, nBs = m.nh * LC * nB;
  const int P = A.pairs;                    // the host sized the buffers for P pairs of any block
  __shared__ int s_pair[ANISO_LMAX * ANISO_LMAX];
  __shared__ int s_npair;
  if (tid == 0) {
    int np = 0;
    for (int iA = 0; iA < Ra[dA]; ++iA)
      for (int jA = 0; jA < Rb[dA]; ++jA)
        if (!(a == b && dA == 2 && iA > jA)) s_pair[np++] = iA * ANISO_LMAX + jA;
    s_npair = np;
  }
  __syncthreads();
  const int ncI = (RaC + 1) / 2, ncJ = (RbC + 1) / 2, nq4 = (nB + 3) / 4, nCt = nq4 * ncI * ncJ;
  for (int p0 = 0; p0 < s_npair; p0 += P) {
    const int np = min(P, s_npair - p0);
    // stage A: contract the first direction
    for (int o = tid; o < np * nAs; o += NTA) {
      const int pp = o / nAs, oo = o % nAs;
      const int iA = s_pair[p0 + pp] / ANISO_LMAX, jA = s_pair[p0 + pp] % ANISO_LMAX;
      const int g = oo / (LC * LB), qC = (oo / LB) % LC, qB = oo % LB;
      Real v = 0;
      for (int t = 0; t < m.nt; ++t) {
        if (m.tg[t] != g) continue;
        const Real* f = s_F + m.tf[t] * Q + LA * (qB + LB * qC);
        Real u = 0;
        for (int qA = 0; qA < LA; ++qA)
          u += f[qA] * tab(dA, m.r[t][dA], iA + sa[dA], qA) * tab(dA, m.s[t][dA], jA + sb[dA], qA);
        v += Real(m.coef[t]) * u;
      }
      s_A[o] = v;
    }
    __syncthreads();
    // stage B: contract the second direction, B_h[qC][jB][iB]; one thread per (h, iB, jB)
    // keeps all qC in registers, and A_g is the same for every lane (broadcast reads)
    for (int o = tid; o < np * m.nh * nB; o += NTA) {
      const int pp = o / (m.nh * nB), oo = o % (m.nh * nB);
      const int h = oo / nB, ij = oo % nB, iB = ij % RaB, jB = ij / RaB;
      Real acc[ANISO_LMAX];
#pragma unroll
      for (int c = 0; c < ANISO_LMAX; ++c) acc[c] = 0;
      for (int g = 0; g < m.ng; ++g) {
        if (m.gh[g] != h) continue;
        const int rg = m.gr[g][dB], sg = m.gs[g][dB];
        const Real* x = s_A + pp * nAs + g * LC * LB;
        for (int q0 = 0; q0 < LB; q0 += 2) {   // two points per pass, their reads issued together
          Real pq[2];
          int qq[2];
#pragma unroll
          for (int t = 0; t < 2; ++t) {
            qq[t] = min(q0 + t, LB - 1);
            pq[t] = q0 + t < LB ? tab(dB, rg, iB + sa[dB], qq[t]) * tab(dB, sg, jB + sb[dB], qq[t]) : Real(0);
          }
#pragma unroll
          for (int c = 0; c < ANISO_LMAX; ++c)
            if (c < LC) acc[c] += pq[0] * x[c * LB + qq[0]] + pq[1] * x[c * LB + qq[1]];
        }
      }
#pragma unroll
      for (int c = 0; c < ANISO_LMAX; ++c)
        if (c < LC) s_B[pp * nBs + (h * LC + c) * nB + ij] = acc[c];
    }
    __syncthreads();
    // stage C: contract the last direction (least order) and store.  One thread per
    // 2 x 2 block of (iC, jC) and 4 consecutive (iB, jB): per point four B values and
    // four table values feed sixteen multiply-adds.  With xi3 contracted here, a
    // diagonal block skips the (iC, jC) blocks that lie wholly below the diagonal.
    for (int o = tid; o < np * nCt; o += NTA) {
      const int pp = o / nCt, oo = o % nCt;
      const int iA = s_pair[p0 + pp] / ANISO_LMAX, jA = s_pair[p0 + pp] % ANISO_LMAX;
      const int ij0 = 4 * (oo % nq4), ch = oo / nq4, ci = 2 * (ch % ncI), cj = 2 * (ch / ncI);
      if (a == b && dC == 2 && ci > cj + 1) continue;
      Real acc[2][2][4];
#pragma unroll
      for (int u = 0; u < 2; ++u)
#pragma unroll
        for (int v = 0; v < 2; ++v)
#pragma unroll
          for (int w = 0; w < 4; ++w) acc[u][v][w] = 0;
      for (int h = 0; h < m.nh; ++h) {
        const int rh = m.hr[h], sh = m.hs[h];
        const Real* x = s_B + pp * nBs + h * LC * nB;
        for (int q0 = 0; q0 < LC; q0 += 2) {   // two points per pass, their reads issued together
          Real xv[2][4], pr[2][2][2];
#pragma unroll
          for (int t = 0; t < 2; ++t) {
            const int qC = min(q0 + t, LC - 1);
            const bool live = q0 + t < LC;
#pragma unroll
            for (int w = 0; w < 4; ++w) xv[t][w] = live && ij0 + w < nB ? x[qC * nB + ij0 + w] : Real(0);
            // rows / columns past the range repeat the last one (not stored)
            const Real ti0 = tab(dC, rh, ci + sa[dC], qC), ti1 = tab(dC, rh, min(ci + 1, RaC - 1) + sa[dC], qC);
            const Real tj0 = tab(dC, sh, cj + sb[dC], qC), tj1 = tab(dC, sh, min(cj + 1, RbC - 1) + sb[dC], qC);
            pr[t][0][0] = ti0 * tj0;
            pr[t][0][1] = ti0 * tj1;
            pr[t][1][0] = ti1 * tj0;
            pr[t][1][1] = ti1 * tj1;
          }
#pragma unroll
          for (int t = 0; t < 2; ++t)
#pragma unroll
            for (int u = 0; u < 2; ++u)
#pragma unroll
              for (int v = 0; v < 2; ++v)
#pragma unroll
                for (int w = 0; w < 4; ++w) acc[u][v][w] += pr[t][u][v] * xv[t][w];
        }
      }
#pragma unroll
      for (int u = 0; u < 2; ++u)
#pragma unroll
        for (int v = 0; v < 2; ++v)
#pragma unroll
          for (int w = 0; w < 4; ++w) {
            const int iC = ci + u, jC = cj + v, ij = ij0 + w;
            if (iC < RaC && jC < RbC && ij < nB) {
              int64_t I, J;
              entry(iA, jA, ij % RaB, ij / RaB, iC, jC, I, J);
              if (a != b || I <= J) out[I + J * (J + 1) / 2] = acc[u][v][w];
            }
          }
    }
    __syncthreads();
  }
}

}  // namespace

hipError_t launch_aniso(int prec, const AnisoArgs& a0, hipStream_t st) {
  AnisoArgs a = a0;
  const int sp = a.space, nblk = (sp == SP_H1 || sp == SP_L2) ? 1 : 6;
  // upper bounds over the blocks of a space: distinct fields, stage-A and stage-C groups
  const int nf = sp == SP_H1 ? 7 : sp == SP_HCURL ? 5 : sp == SP_HDIV ? 2 : 1;
  const int ng = sp == SP_H1 ? MT : sp == SP_HCURL ? 5 : sp == SP_HDIV ? 2 : 1;
  const int nh = sp == SP_H1 || sp == SP_HCURL ? MH : sp == SP_HDIV ? 2 : 1;
  const int dB = a.dir[1], dC = a.dir[2];
  const int rB = sp == SP_L2 ? a.q[dB] : a.q[dB] + 1;      // largest range of direction B over components
  const int LB = a.L[dB], LC = a.L[dC];
  a.lds_fields = nf * a.L[0] * a.L[1] * a.L[2];
  a.lds_a = ng * LC * LB;
  const int per_b = nh * LC * rB * rB;
  // as many pairs per barrier interval as fit in about 40 KB (three workgroups per CU
  // in FP64), at least one, at most 16
  const int64_t budget = (int64_t(40) << 10) / (prec ? 4 : 8) - a.lds_fields;
  a.pairs = int(std::max<int64_t>(1, std::min<int64_t>(16, budget / (a.lds_a + per_b))));
  const size_t lds = size_t(a.lds_fields + a.pairs * (a.lds_a + per_b)) * (prec ? 4 : 8);
  if (lds + sizeof(Meta) + 3 * TDIR * (prec ? 4 : 8) + 1024 > size_t(160) << 10) return hipErrorInvalidValue;
  const int64_t items = a.n_elem * nblk;
  hipError_t err = hipSuccess;
  if (prec)
    err = hipFuncSetAttribute(reinterpret_cast<const void*>(&k_aniso<float>),
                              hipFuncAttributeMaxDynamicSharedMemorySize, int(lds));
  else
    err = hipFuncSetAttribute(reinterpret_cast<const void*>(&k_aniso<double>),
                              hipFuncAttributeMaxDynamicSharedMemorySize, int(lds));
  if (err != hipSuccess) return err;
  for (int64_t i0 = 0; i0 < items; i0 += kMaxGrid) {
    const unsigned grid = unsigned(std::min(kMaxGrid, items - i0));
    if (prec)
      hipLaunchKernelGGL(k_aniso<float>, dim3(grid), dim3(NTA), lds, st, a, nblk, i0);
    else
      hipLaunchKernelGGL(k_aniso<double>, dim3(grid), dim3(NTA), lds, st, a, nblk, i0);
  }
  return hipGetLastError();
}

}  // namespace dpg
