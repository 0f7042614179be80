// condense.hip -- the first consumer of the Grams on the device: static
// condensation of the test variables s in (3.7) needs G^{-1} B, G^{-1} B~ and
// G^{-1} l ((3.8), Section 1), which come from a Cholesky factorization of G
// followed by forward and backward substitution.  The Grams stay where the
// integration kernels wrote them ('U' packed, one per element), and the
// factor overwrites them in place: G = U^T U, U upper triangular with a
// positive diagonal (LAPACK's packed 'U' convention).
//
// Both kernels go down the matrix in block rows of 64 (four 16-row sub-blocks).
// A wave owns a 64 x 16 tile of the block row (four MFMA accumulators) and first
// removes from it, in one contraction on FP64 or FP32 MFMA, everything the rows
// above contribute; that contraction is almost all of the arithmetic.  Its left
// operand (64 rows of U, the same for every tile of the block row) is staged in
// LDS once per workgroup, 16 k at a time, and shared by the four waves; the loads
// go through buffer resources with offsets fixed for the whole contraction, and
// each lane reads four consecutive entries of a packed column.  The tile's own
// entries (of G or of the right-hand sides) are loaded straight into the
// accumulators before the contraction starts, and the staged operand is stored
// negated, so those loads overlap the contraction's.  What is left is the 64 x 64
// diagonal block: its four sub-blocks are finished in order, each by MFMA
// products with the sub-blocks already finished and a solve with the 16 x 16
// diagonal block, also on MFMA: its inverse (computed once per block row)
// applied, followed by one step of refinement, so the result keeps the accuracy
// of a substitution.  The block's factor and inverses are staged in LDS.
//
// Factorization (k_potrf, one workgroup of four waves per element): for block row
// R, U[R, :] = U[R, R]^{-T} (G[R, :] - U[:R, R]^T U[:R, :]).  The diagonal block
// goes first: its contraction (one tile per wave) leaves its ten blocks on or above
// the diagonal in LDS, where it is factored right-looking over the 16 x 16 blocks.
// The tiles right of the diagonal block then go four at a time (one per wave), each
// finished by its own wave with no further barrier.  Solve (k_potrs, one workgroup
// per element and 64 right-hand sides, 16 per wave): U^T y = b down the block rows,
// then U x = y up them, the diagonal block of each block row staged in LDS and its
// four inverses computed by the four waves.
#include <hip/hip_runtime.h>

#include <algorithm>

#include "condense.h"

namespace dpg {

namespace {

typedef double c4d __attribute__((ext_vector_type(4)));
typedef float c4f __attribute__((ext_vector_type(4)));

// v_mfma_*_16x16x4: lane i + 16 k holds A[i][k] and B[k][i]; accumulator
// register r of lane (g = lane / 16, j = lane % 16) holds C[row(g, r)][j], so
// row k sits in lane group grp(k), register reg(k).
template <typename Real> struct Mfma;
template <> struct Mfma<double> {
  typedef c4d acc;
  static __device__ __forceinline__ acc mac(double a, double b, acc c) {
    return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
  }
  static constexpr int row(int g, int r) { return g + 4 * r; }
  static constexpr int grp(int k) { return k & 3; }
  static constexpr int reg(int k) { return k >> 2; }
};
template <> struct Mfma<float> {
  typedef c4f acc;
  static __device__ __forceinline__ acc mac(float a, float b, acc c) {
    return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
  }
  static constexpr int row(int g, int r) { return 4 * g + r; }
  static constexpr int grp(int k) { return k >> 2; }
  static constexpr int reg(int k) { return k & 3; }
};

constexpr int NB = 16;            // MFMA tile, sub-block rows
constexpr int NS = 4;             // sub-blocks per block row
constexpr int BR = NB * NS;       // block row
constexpr int LDB = NB + 1;       // leading dimension of a staged 16 x 16 block of U
constexpr int NBLK = NS * (NS + 1) / 2;           // blocks on or above the diagonal of a diagonal block
constexpr int KC = 16;            // k per staged chunk of the left operand
constexpr int CH = NS * KC * NB;  // entries per staged chunk (64 rows x 16 k)
constexpr int NT = 256;                          // four waves; four workgroups per CU (<= 128 registers)
constexpr int NW = NT / 64;
constexpr int64_t kMaxGrid = int64_t(1) << 22;   // workgroups per launch

// Packed 'U' column pointer.
__device__ __forceinline__ int64_t colp(int64_t j) { return j * (j + 1) / 2; }

// Block (t, s), t <= s, of a 64 x 64 diagonal block staged in LDS: row-major 16 x 16
// with leading dimension LDB, the ten blocks one after the other.
__device__ __forceinline__ int blk_off(int t, int s) { return (t * NS + s - t * (t + 1) / 2) * NB * LDB; }

// The left operand of the contractions, 64 rows by KC k, is staged in LDS once per
// workgroup and chunk, in the order the MFMAs take it: the entry for row 16 s + i and
// k = 4 kk + q (of the chunk) sits at (s * 4 + q) * 64 + 16 kk + i, so lane 16 kk + i
// of any wave reads its step-q operand of sub-block s at (s * 4 + q) * 64 + lane.
__device__ __forceinline__ int stage_idx(int s, int q, int kk, int i) { return (s * 4 + q) * 64 + kk * 16 + i; }

// Barrier for the staged operand: it orders only the LDS accesses, so global loads in
// flight (the next chunk's, the accumulators' initial values) stay in flight across it,
// where a full __syncthreads would wait for them.
__device__ __forceinline__ void lds_barrier() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup", "local");
  __builtin_amdgcn_s_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup", "local");
}

// Buffer resource over count entries at p (the loads below go through the vector
// memory path with a scalar base, a 32-bit per-lane byte offset and a scalar offset,
// so a chunk step costs no per-lane address arithmetic).  The range check covers the
// vector offset only: a read whose vector offset is at or past count entries returns
// zero, while the scalar offset must keep every read inside the matrix by itself.
// Callers keep count * sizeof(Real) below 2^31.
typedef __amdgpu_buffer_rsrc_t Rsrc;
template <typename Real>
__device__ __forceinline__ Rsrc make_rsrc(const Real* p, int64_t count) {
  return __builtin_amdgcn_make_buffer_rsrc(const_cast<Real*>(p), 0, int(count * int64_t(sizeof(Real))), 0x00020000);
}
// Four consecutive entries at byte offset voff + soff.
__device__ __forceinline__ void load4(Rsrc r, uint32_t voff, uint32_t soff, double (&v)[4]) {
  typedef double d2 __attribute__((ext_vector_type(2)));
  const d2 x = __builtin_bit_cast(d2, __builtin_amdgcn_raw_buffer_load_b128(r, voff, soff, 0));
  const d2 y = __builtin_bit_cast(d2, __builtin_amdgcn_raw_buffer_load_b128(r, voff + 16, soff, 0));
  v[0] = x[0];
  v[1] = x[1];
  v[2] = y[0];
  v[3] = y[1];
}
__device__ __forceinline__ void load4(Rsrc r, uint32_t voff, uint32_t soff, float (&v)[4]) {
  typedef float f4 __attribute__((ext_vector_type(4)));
  const f4 x = __builtin_bit_cast(f4, __builtin_amdgcn_raw_buffer_load_b128(r, voff, soff, 0));
#pragma unroll
  for (int q = 0; q < 4; ++q) v[q] = x[q];
}

// Make the accumulators' initial loads complete here, so that the loop after it has no
// load of them in flight (the wait would otherwise sit inside the loop and drain the
// next chunk's loads on every iteration).
template <typename Real>
__device__ __forceinline__ void settle(const typename Mfma<Real>::acc& v) {
#pragma unroll
  for (int r = 0; r < 4; ++r) asm volatile("" ::"v"(v[r]));
}

// Contraction over nch chunks of KC k, four waves in step: c[s] += sum_k A_s(i, k) B(k, j)
// for the four sub-blocks s, on the waves with act (the waves run in step, so a wave that
// needs fewer sub-blocks would only wait at the barrier; it computes them all), where A
// is the operand as staged (negated by the callers).  A.load(ch, v) fetches this
// thread's four entries of the left operand's chunk ch and A.put(buf, ch, v) stores them
// in the staging order; B.load(ch, v) fetches this lane's four right-hand entries (k =
// 16 ch + 4 kk + q in step q).  The next chunk's loads are in flight while the MFMAs of
// the current one run; one barrier per chunk.  Unrolled by two, the register sets for
// the chunks in flight alternate, so no value in flight is ever copied (a copy would wait
// for it).  Every wave of the workgroup calls it with the same nch.
template <typename Real, typename TA, typename TB>
__device__ __forceinline__ void contract_staged(Real* sA, int64_t nch, bool act, const TA& A, const TB& B,
                                                typename Mfma<Real>::acc (&c)[NS], int lane) {
  typedef Mfma<Real> M;
  if (nch <= 0) return;
  Real a0[4], a1[4], b0[4], b1[4];
  A.load(0, a0);
  B.load(0, b0);
  A.put(sA, 0, a0);
#pragma unroll
  for (int s = 0; s < NS; ++s) settle<Real>(c[s]);
  lds_barrier();
  auto step = [&](int64_t ch, const Real* cur, Real* nxt, const Real(&bc)[4], Real(&an)[4], Real(&bn)[4]) {
    const bool more = ch + 1 < nch;
    // unconditional: a branch around the loads would make the wait before the MFMAs cover
    // them too.  Past the last chunk the current one is loaded again (unused): the chunk
    // step travels in the scalar offset, which the buffer range check does not cover, so
    // a chunk past the end could read past the matrix.
    const int64_t nx = more ? ch + 1 : ch;
    A.load(nx, an);
    B.load(nx, bn);
    if (act) {
#pragma unroll
      for (int q = 0; q < 4; ++q)
#pragma unroll
        for (int s = 0; s < NS; ++s) c[s] = M::mac(cur[(s * 4 + q) * 64 + lane], bc[q], c[s]);
    }
    if (more) A.put(nxt, ch + 1, an);
    lds_barrier();
  };
  for (int64_t ch = 0; ch < nch; ch += 2) {
    step(ch, sA, sA + CH, b0, a1, b1);
    if (ch + 1 < nch) step(ch + 1, sA + CH, sA, b1, a0, b0);
  }
}

// v -= T^T x for a staged 16 x 16 block T and x in the accumulator layout, whose
// register q holds the k of MFMA step q: x is the right operand as it stands.
template <typename Real>
__device__ __forceinline__ void sub_tn(typename Mfma<Real>::acc& v, const Real* T, const typename Mfma<Real>::acc& x,
                                       int lane) {
  typedef Mfma<Real> M;
  const int i = lane & 15, g = lane >> 4;
#pragma unroll
  for (int q = 0; q < 4; ++q) v = M::mac(-T[M::row(g, q) * LDB + i], x[q], v);
}

// v -= T x (T as above).
template <typename Real>
__device__ __forceinline__ void sub_nn(typename Mfma<Real>::acc& v, const Real* T, const typename Mfma<Real>::acc& x,
                                       int lane) {
  typedef Mfma<Real> M;
  const int i = lane & 15, g = lane >> 4;
#pragma unroll
  for (int q = 0; q < 4; ++q) v = M::mac(-T[i * LDB + M::row(g, q)], x[q], v);
}

// A staged diagonal block holds U_ss (upper triangle and diagonal) and its inverse
// V = U_ss^{-1} transposed (strictly lower triangle: V[k][i] at row i, column k), with
// rd[k] = 1 / U_ss[k][k] = V[k][k].  Rows and columns past the matrix are the identity.
// The MFMA left operands of step q for lane (i, g), k = row(g, q):
template <typename Real>
__device__ __forceinline__ Real op_vt(const Real* T, const Real* rd, int i, int k) {   // V^T[i][k]
  return k < i ? T[i * LDB + k] : (k == i ? rd[i] : Real(0));
}
template <typename Real>
__device__ __forceinline__ Real op_v(const Real* T, const Real* rd, int i, int k) {    // V[i][k]
  return k > i ? T[k * LDB + i] : (k == i ? rd[i] : Real(0));
}

// U_ss^T x = v in place (v in the accumulator layout, the 16 right-hand sides are the
// columns j = lane % 16): x0 = V^T v, then with REFINE x = x0 + V^T (v - U_ss^T x0).
// The refinement makes the result backward stable whatever cond(U_ss); without it the
// error grows with cond(U_ss) (a blocked triangular solve with inverted diagonal blocks).
template <typename Real, bool REFINE>
__device__ __forceinline__ void solve_fwd(typename Mfma<Real>::acc& v, const Real* T, const Real* rd, int lane) {
  typedef Mfma<Real> M;
  typedef typename M::acc acc;
  const int i = lane & 15, g = lane >> 4;
  Real av[4], au[4];
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    const int k = M::row(g, q);
    av[q] = op_vt(T, rd, i, k);
    au[q] = k <= i ? -T[k * LDB + i] : Real(0);   // -U_ss^T[i][k]
  }
  acc x = {0, 0, 0, 0};
#pragma unroll
  for (int q = 0; q < 4; ++q) x = M::mac(av[q], v[q], x);
  if constexpr (REFINE) {
#pragma unroll
    for (int q = 0; q < 4; ++q) v = M::mac(au[q], x[q], v);    // residual
#pragma unroll
    for (int q = 0; q < 4; ++q) x = M::mac(av[q], v[q], x);
  }
  v = x;
}

// U_ss x = v in place: x0 = V v, then with REFINE x = x0 + V (v - U_ss x0).
template <typename Real, bool REFINE>
__device__ __forceinline__ void solve_bwd(typename Mfma<Real>::acc& v, const Real* T, const Real* rd, int lane) {
  typedef Mfma<Real> M;
  typedef typename M::acc acc;
  const int i = lane & 15, g = lane >> 4;
  Real av[4], au[4];
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    const int k = M::row(g, q);
    av[q] = op_v(T, rd, i, k);
    au[q] = k >= i ? -T[i * LDB + k] : Real(0);   // -U_ss[i][k]
  }
  acc x = {0, 0, 0, 0};
#pragma unroll
  for (int q = 0; q < 4; ++q) x = M::mac(av[q], v[q], x);
  if constexpr (REFINE) {
#pragma unroll
    for (int q = 0; q < 4; ++q) v = M::mac(au[q], x[q], v);
#pragma unroll
    for (int q = 0; q < 4; ++q) x = M::mac(av[q], v[q], x);
  }
  v = x;
}

// Lane j < 16 of one wave: column j of V = U_ss^{-1} by back substitution against the
// rows of U_ss (read from the staged block, the same for every lane), written
// transposed into the block's strictly lower triangle.  Only this wave touches the
// block meanwhile; its LDS accesses complete in order.
template <typename Real>
__device__ __forceinline__ void invert_block(Real* T, const Real* rd, int j) {
  Real z[NB];
#pragma unroll
  for (int i = 0; i < NB; ++i) z[i] = i == j ? rd[i] : Real(0);
#pragma unroll
  for (int i = NB - 2; i >= 0; --i) {
    Real d = Real(0);
#pragma unroll
    for (int k = i + 1; k < NB; ++k) d += T[i * LDB + k] * z[k];
    if (i < j) z[i] = -rd[i] * d;
  }
#pragma unroll
  for (int i = 0; i < NB; ++i)
    if (i < j) T[j * LDB + i] = z[i];
}

// Left operand "columns of U": chunk ch of U[k][r0 + r], k = 16 ch + .., r < 64 (columns
// past n clamped to the last; rows past the matrix only reach output rows that are never
// stored), staged negated.  Thread t takes column r0 + t / 4, four consecutive k.
template <typename Real>
struct ColsOperand {
  Rsrc rs;
  uint32_t vo;
  int s, i, kk;
  __device__ ColsOperand(const Real* u, int64_t n, int64_t r0, int tid) {
    const int r = tid >> 2;
    kk = tid & 3;
    rs = make_rsrc(u, n * (n + 1) / 2);
    vo = uint32_t((colp(std::min<int64_t>(r0 + r, n - 1)) + 4 * kk) * int64_t(sizeof(Real)));
    s = r >> 4;
    i = r & 15;
  }
  __device__ __forceinline__ void load(int64_t ch, Real (&v)[4]) const {
    load4(rs, vo, uint32_t(KC * ch * int64_t(sizeof(Real))), v);
  }
  __device__ __forceinline__ void put(Real* buf, int64_t, const Real (&v)[4]) const {
#pragma unroll
    for (int q = 0; q < 4; ++q) buf[stage_idx(s, q, kk, i)] = -v[q];
  }
};

// Left operand "rows of U": chunk ch of U[r0 + r][k], k = k0 + 16 ch + .. (zero from kend
// on: the load is clamped to the last column and the value dropped when it is staged),
// r < 64, staged negated.  Thread t takes column k0 + 16 ch + t / 16, four consecutive rows.
template <typename Real>
struct RowsOperand {
  Rsrc rs;
  int64_t r0, k0, kend;
  int kc, rq;
  __device__ RowsOperand(const Real* u, int64_t n, int64_t r0_, int64_t k0_, int64_t kend_, int tid)
      : rs(make_rsrc(u, n * (n + 1) / 2)), r0(r0_), k0(k0_), kend(kend_), kc(tid >> 4), rq(4 * (tid & 15)) {}
  __device__ __forceinline__ void load(int64_t ch, Real (&v)[4]) const {
    const int64_t k = std::min(k0 + KC * ch + kc, kend - 1);
    load4(rs, uint32_t((colp(k) + r0 + rq) * int64_t(sizeof(Real))), 0, v);
  }
  __device__ __forceinline__ void put(Real* buf, int64_t ch, const Real (&v)[4]) const {
    const bool ok = k0 + KC * ch + kc < kend;
#pragma unroll
    for (int m = 0; m < 4; ++m) {
      const int r = rq + m;
      buf[stage_idx(r >> 4, kc & 3, kc >> 2, r & 15)] = ok ? -v[m] : Real(0);
    }
  }
};

// Right operand: entries k = k0 + 16 ch + 4 kk + q of this lane's column, which starts at
// entry col of the resource.  With INRANGE every k read lies in the column (the chunk
// step goes in the scalar offset); otherwise the whole offset is in the vector part, so
// that a read past the resource returns zero (past the column, reads within the resource
// return finite entries, which the zero left operand drops).
template <typename Real, bool INRANGE>
struct RhsOperand {
  Rsrc rs;
  uint32_t vo;
  __device__ RhsOperand(Rsrc r, int64_t col, int64_t k0, int lane)
      : rs(r), vo(uint32_t((col + k0 + 4 * (lane >> 4)) * int64_t(sizeof(Real)))) {}
  __device__ __forceinline__ void load(int64_t ch, Real (&v)[4]) const {
    const uint32_t step = uint32_t(KC * ch * int64_t(sizeof(Real)));
    if (INRANGE)
      load4(rs, vo, step, v);
    else
      load4(rs, vo + step, 0, v);
  }
};

template <typename Real>
__global__ void __launch_bounds__(NT, 4) k_potrf(Real* __restrict__ ap, int64_t n, int64_t n_elem,
                                                 int32_t* __restrict__ info) {
  typedef Mfma<Real> M;
  typedef typename M::acc acc;
  __shared__ Real s_U[NBLK * NB * LDB];     // U on the diagonal block of the block row, blocks (t <= s)
  __shared__ Real s_A[2 * CH];              // staged left operand (two chunks)
  __shared__ Real s_rd[BR];                 // reciprocal pivots of the diagonal block
  __shared__ int s_fail;
  const int64_t e = blockIdx.x;
  if (e >= n_elem) return;
  const int tid = threadIdx.x, wv = tid >> 6;
  Real* a = ap + e * (n * (n + 1) / 2);
  const acc zero = {0, 0, 0, 0};
  // The lane index is passed through an opaque copy at the top of every loop iteration:
  // otherwise the compiler computes every lane-dependent constant (LDS offsets, masks,
  // identity entries) once before the loops and keeps them, spilled, for the whole kernel.
  int lane, li, lg;
  auto relane = [&]() {
    int l = tid & 63;
    asm volatile("" : "+v"(l));
    lane = l;
    li = l & 15;
    lg = l >> 4;
  };

  // G on this lane's accumulator slots (rows r0 + 16 s + .., column cb + lane % 16)
  auto gram_load = [&](int64_t r0, int s, int64_t cb, acc& S) {
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int64_t row = r0 + NB * s + M::row(lg, r), col = cb + li;
      S[r] = (row <= col && col < n) ? a[colp(col) + row] : Real(0);
    }
  };
  auto store = [&](int64_t r0, int s, int64_t cb, const acc& S) {
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int64_t row = r0 + NB * s + M::row(lg, r), col = cb + li;
      if (row <= col && col < n) a[colp(col) + row] = S[r];
    }
  };
  auto blk = [&](int t, int s) { return s_U + blk_off(t, s); };
  // a staged 16 x 16 block to and from the accumulator layout
  auto put_block = [&](Real* T, const acc& v) {
#pragma unroll
    for (int r = 0; r < 4; ++r) T[M::row(lg, r) * LDB + li] = v[r];
  };
  auto get_block = [&](const Real* T, acc& v) {
#pragma unroll
    for (int r = 0; r < 4; ++r) v[r] = T[M::row(lg, r) * LDB + li];
  };
  // S -= U[:r0, R]^T U[:r0, cb ..] (active waves)
  auto contract = [&](int64_t r0, int64_t cb, bool act, acc (&S)[NS]) {
    const ColsOperand<Real> A(a, n, r0, tid);
    const RhsOperand<Real, true> B(A.rs, colp(std::min<int64_t>(cb + li, n - 1)), 0, lane);
    contract_staged<Real>(s_A, r0 / KC, act, A, B, S, lane);
  };

  for (int64_t r0 = 0; r0 < n; r0 += BR) {
    const int nsb = int(std::min<int64_t>(NS, (n - r0 + NB - 1) / NB));   // sub-blocks in this block row
    relane();
    // ---- the diagonal block: its contraction, wave wv on columns r0 + 16 wv .., leaves the
    // ten blocks on or above the diagonal in LDS
    {
      const bool have = wv < nsb;
      const int64_t cb = r0 + NB * wv;
      acc S[NS] = {zero, zero, zero, zero};
      if (have) {
#pragma unroll
        for (int s = 0; s < NS; ++s)
          if (s <= wv) gram_load(r0, s, cb, S[s]);
      }
      contract(r0, cb, have, S);            // (the sub-blocks below the diagonal go unused)
      if (have) {
#pragma unroll
        for (int s = 0; s < NS; ++s)
          if (s <= wv) put_block(blk(s, wv), S[s]);
      }
    }
    __syncthreads();
    // ---- its Cholesky factor in LDS, right-looking over the 16 x 16 blocks: factor block
    // (s, s), finish blocks (s, t > s) with it, remove row s from the blocks (t, u), s < t <= u
#pragma unroll
    for (int s = 0; s < NS; ++s) {
      if (s >= nsb) break;
      const int h = int(std::min<int64_t>(NB, n - r0 - NB * s));
      const int64_t ib = r0 + NB * s;
      if (wv == 0 && lane < NB) {           // unblocked Cholesky of block (s, s), one column per lane
        const int j = lane;
        Real* T = blk(s, s);
        Real cl[NB];
#pragma unroll
        for (int i = 0; i < NB; ++i) cl[i] = T[i * LDB + j];
        int fail = 0;
#pragma unroll
        for (int k = 0; k < NB; ++k) {
          if (k < h && !fail) {             // uniform: h and the pivot are the same in every lane
            const Real d = __shfl(cl[k], k);
            if (!(d > Real(0))) {
              fail = k + 1;
            } else {
              const Real ukk = sqrt(d);
              cl[k] = j == k ? ukk : cl[k] / ukk;   // row k of U
#pragma unroll
              for (int i = k + 1; i < NB; ++i) cl[i] -= __shfl(cl[k], i) * cl[k];
            }
          }
        }
        if (j < h && (!fail || j < fail - 1)) {    // on failure the columns before the failing one are final
          Real* dst = a + colp(ib + j) + ib;
#pragma unroll
          for (int i = 0; i < NB; ++i)
            if (i <= j) dst[i] = cl[i];
        }
        // U_ss (columns past the matrix the identity), then its inverse below the diagonal
#pragma unroll
        for (int i = 0; i < NB; ++i)
          if (i <= j) T[i * LDB + j] = j < h ? cl[i] : Real(i == j ? 1 : 0);
        s_rd[NB * s + j] = j < h ? Real(1) / cl[j] : Real(1);
        if (j == 0) s_fail = fail ? int(ib) + fail : 0;
        invert_block<Real>(T, s_rd + NB * s, j);
      }
      __syncthreads();
      if (s_fail) {
        if (tid == 0 && info) info[e] = s_fail;
        return;
      }
      if (wv < nsb - 1 - s) {               // block (s, t): U_ss^T x = C(s, t)
        const int t = s + 1 + wv;
        acc x;
        get_block(blk(s, t), x);
        solve_fwd<Real, true>(x, blk(s, s), s_rd + NB * s, lane);
        put_block(blk(s, t), x);
        store(r0, s, r0 + NB * t, x);
      }
      __syncthreads();
      const int m = nsb - 1 - s;            // trailing blocks (t, u), s < t <= u < nsb
      if (m > 0) {
        for (int idx = wv; idx < m * (m + 1) / 2; idx += NW) {
          int t = 0, u = idx;
          while (u >= m - t) { u -= m - t; ++t; }
          t += s + 1;
          u += t;
          acc c, x;
          get_block(blk(t, u), c);
          get_block(blk(s, u), x);
          sub_tn<Real>(c, blk(s, t), x, lane);
          put_block(blk(t, u), c);
        }
        __syncthreads();
      }
    }
    // ---- the tiles right of the diagonal block, four at a time (one per wave)
    for (int64_t cg = r0 + BR; cg < n; cg += BR) {
      relane();
      const int64_t cb = cg + NB * wv;
      const bool act = cb < n;
      acc S[NS] = {zero, zero, zero, zero};
      if (act) {
#pragma unroll
        for (int s = 0; s < NS; ++s)
          if (s < nsb) gram_load(r0, s, cb, S[s]);
      }
      contract(r0, cb, act, S);
      if (act) {
#pragma unroll
        for (int s = 0; s < NS; ++s) {
          if (s >= nsb) break;
#pragma unroll
          for (int t = 0; t < s; ++t) sub_tn<Real>(S[s], blk(t, s), S[t], lane);
          solve_fwd<Real, true>(S[s], blk(s, s), s_rd + NB * s, lane);
          store(r0, s, cb, S[s]);
        }
      }
    }
    __syncthreads();                        // block row finished before the next one reads it
  }
  if (tid == 0 && info) info[e] = 0;
}

// Workgroup b of g runs on XCD b % 8 (the dispatcher deals workgroups round robin); the
// logical workgroup is numbered so that each XCD takes one contiguous range, keeping the
// workgroups of one element (the same factor U) on one XCD and its L2.
__device__ __forceinline__ int64_t xcd_major(int64_t b, int64_t g) {
  const int64_t x = b & 7, per = g >> 3, rem = g & 7;
  return x * per + std::min<int64_t>(x, rem) + (b >> 3);
}

template <typename Real>
__global__ void __launch_bounds__(NT, 4) k_potrs(const Real* __restrict__ up, int64_t n, int64_t n_elem, int64_t nrhs,
                                                 int64_t e0, Real* __restrict__ b) {
  typedef Mfma<Real> M;
  typedef typename M::acc acc;
  __shared__ Real s_U[NBLK * NB * LDB];     // the block row's diagonal block of U, blocks (t <= s)
  __shared__ Real s_A[2 * CH];              // staged left operand
  __shared__ Real s_rd[BR];                 // reciprocal pivots (rows past n: 1)
  const int64_t nblk = (nrhs + BR - 1) / BR;
  const int64_t wg = xcd_major(blockIdx.x, gridDim.x);
  const int64_t e = e0 + wg / nblk, cbk = wg % nblk;
  if (e >= n_elem) return;
  const int tid = threadIdx.x, wv = tid >> 6;
  const Real* u = up + e * (n * (n + 1) / 2);
  const int64_t c0 = cbk * BR + NB * wv;    // this wave's first right-hand side
  const bool act = c0 < nrhs;
  // lane index through an opaque copy per block row (lane constants are not kept live across
  // the whole kernel)
  int lane, li, lg;
  bool colok;
  Real* xc;                                 // this lane's right-hand side
  auto relane = [&]() {
    int l = tid & 63;
    asm volatile("" : "+v"(l));
    lane = l;
    li = l & 15;
    lg = l >> 4;
    colok = c0 + li < nrhs;
    xc = b + e * n * nrhs + std::min<int64_t>(c0 + li, nrhs - 1) * n;
  };
  // this workgroup's right-hand sides (at most 64 columns) as one buffer resource
  const int64_t wcols = std::min<int64_t>(BR, nrhs - cbk * BR);
  const Rsrc xr = make_rsrc(b + e * n * nrhs + cbk * BR * n, wcols * n);
  auto xcol = [&]() { return std::min<int64_t>(NB * wv + li, wcols - 1) * n; };   // this lane's, in it
  const acc zero = {0, 0, 0, 0};
  auto blk = [&](int t, int s) { return s_U + blk_off(t, s); };

  // the blocks (t <= s) of U on rows and columns r0 .. r0 + 63 (the identity past n)
  auto stage = [&](int64_t r0) {
    for (int idx = tid; idx < NBLK * NB * NB; idx += NT) {
      const int bi = idx / (NB * NB), w = idx % (NB * NB), r = w % NB, c = w / NB;
      int t = 0, s = bi;
      while (s >= NS - t) { s -= NS - t; ++t; }
      s += t;                               // block bi is (t, s)
      const int64_t gr = r0 + NB * t + r, gc = r0 + NB * s + c;
      Real v = (t == s && r == c) ? Real(1) : Real(0);
      if (gr <= gc && gc < n) v = u[colp(gc) + gr];
      blk(t, s)[r * LDB + c] = v;
      if (t == s && r == c) s_rd[NB * t + r] = Real(1) / v;
    }
  };
  auto rhs_load = [&](int64_t r0, int s, acc& S) {
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int64_t row = r0 + NB * s + M::row(lg, r);
      S[r] = (colok && row < n) ? xc[row] : Real(0);
    }
  };
  // the inverses of the four diagonal blocks, one per wave (after the staging barrier)
  auto invert = [&](int nsb) {
    if (wv < nsb && lane < NB) invert_block<Real>(blk(wv, wv), s_rd + NB * wv, lane);
  };
  auto store = [&](int64_t r0, int s, const acc& S) {
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int64_t row = r0 + NB * s + M::row(lg, r);
      if (colok && row < n) xc[row] = S[r];
    }
  };

  // U^T y = b, top down
  for (int64_t r0 = 0; r0 < n; r0 += BR) {
    const int nsb = int(std::min<int64_t>(NS, (n - r0 + NB - 1) / NB));
    relane();
    __syncthreads();                        // the previous block row is done with s_U
    stage(r0);
    acc S[NS] = {zero, zero, zero, zero};
    if (act) {
#pragma unroll
      for (int s = 0; s < NS; ++s)
        if (s < nsb) rhs_load(r0, s, S[s]);
    }
    __syncthreads();
    invert(nsb);
    {
      const ColsOperand<Real> A(u, n, r0, tid);
      const RhsOperand<Real, true> B(xr, xcol(), 0, lane);
      contract_staged<Real>(s_A, r0 / KC, act, A, B, S, lane);
    }
    __syncthreads();
    if (act) {
#pragma unroll
      for (int s = 0; s < NS; ++s) {
        if (s >= nsb) break;
#pragma unroll
        for (int t = 0; t < s; ++t) sub_tn<Real>(S[s], blk(t, s), S[t], lane);
        solve_fwd<Real, false>(S[s], blk(s, s), s_rd + NB * s, lane);
        store(r0, s, S[s]);
      }
    }
  }
  // U x = y, bottom up
  for (int64_t r0 = ((n - 1) / BR) * BR; r0 >= 0; r0 -= BR) {
    const int nsb = int(std::min<int64_t>(NS, (n - r0 + NB - 1) / NB));
    relane();
    __syncthreads();
    stage(r0);
    acc S[NS] = {zero, zero, zero, zero};
    if (act) {
#pragma unroll
      for (int s = 0; s < NS; ++s)
        if (s < nsb) rhs_load(r0, s, S[s]);
    }
    __syncthreads();
    invert(nsb);
    {
      const int64_t k0 = r0 + BR;
      const RowsOperand<Real> A(u, n, r0, k0, n, tid);
      const RhsOperand<Real, false> B(xr, xcol(), k0, lane);
      contract_staged<Real>(s_A, k0 < n ? (n - k0 + KC - 1) / KC : 0, act, A, B, S, lane);
    }
    __syncthreads();
    if (act) {
#pragma unroll
      for (int s = NS - 1; s >= 0; --s) {
        if (s >= nsb) continue;
#pragma unroll
        for (int t = s + 1; t < NS; ++t)
          if (t < nsb) sub_nn<Real>(S[s], blk(s, t), S[t], lane);
        solve_bwd<Real, false>(S[s], blk(s, s), s_rd + NB * s, lane);
        store(r0, s, S[s]);
      }
    }
  }
}

}  // namespace

hipError_t launch_potrf(int prec, void* ap, int64_t n, int64_t n_elem, int32_t* info, hipStream_t st) {
  const int64_t len = n * (n + 1) / 2;
  for (int64_t e0 = 0; e0 < n_elem; e0 += kMaxGrid) {
    const int64_t ne = std::min(kMaxGrid, n_elem - e0);
    int32_t* inf = info ? info + e0 : nullptr;
    if (prec)
      hipLaunchKernelGGL(k_potrf<float>, dim3(unsigned(ne)), dim3(NT), 0, st, static_cast<float*>(ap) + e0 * len, n,
                         ne, inf);
    else
      hipLaunchKernelGGL(k_potrf<double>, dim3(unsigned(ne)), dim3(NT), 0, st, static_cast<double*>(ap) + e0 * len,
                         n, ne, inf);
  }
  return hipGetLastError();
}

hipError_t launch_potrs(int prec, const void* up, int64_t n, int64_t n_elem, int64_t nrhs, void* b, hipStream_t st) {
  const int64_t nblk = (nrhs + BR - 1) / BR;
  const int64_t per = std::max<int64_t>(1, kMaxGrid / nblk);     // elements per launch
  for (int64_t e0 = 0; e0 < n_elem; e0 += per) {
    const int64_t ne = std::min(per, n_elem - e0);
    const unsigned grid = unsigned(ne * nblk);
    if (prec)
      hipLaunchKernelGGL(k_potrs<float>, dim3(grid), dim3(NT), 0, st, static_cast<const float*>(up), n, e0 + ne,
                         nrhs, e0, static_cast<float*>(b));
    else
      hipLaunchKernelGGL(k_potrs<double>, dim3(grid), dim3(NT), 0, st, static_cast<const double*>(up), n, e0 + ne,
                         nrhs, e0, static_cast<double*>(b));
  }
  return hipGetLastError();
}

}  // namespace dpg
