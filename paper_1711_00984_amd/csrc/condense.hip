// condense.hip -- the first consumer of the Grams on the device: static
// condensation of the test variables s in (3.7) needs G^{-1} B, G^{-1} B~ and
// G^{-1} l ((3.8), Section 1), which come from a Cholesky factorization of G
// followed by forward and backward substitution.  The Grams stay where the
// integration kernels wrote them ('U' packed, one per element), and the
// factor overwrites them in place: G = U^T U, U upper triangular with a
// positive diagonal (LAPACK's packed 'U' convention).
//
// One workgroup of four waves per element (per element and 16 right-hand sides
// for the solve, 64 when n <= 256).  Both kernels walk 16-row blocks of a triangular solve with
// U^T: a block first loses the product of the rows already finished (a
// 16 x 16 x K contraction over packed columns on FP64 or FP32 MFMA), then 16 lanes
// finish it against the block's 16 x 16 diagonal block of U.  The factorization is
// that walk with the Gram's own columns as right-hand sides, one 64-column panel at
// a time (the up-looking order: column j of U solves U[:j, :j]^T u = G[:j, j]),
// each wave owning a 16-column tile of the panel; inside the panel's diagonal block
// the wave holding the diagonal tile factors it (unblocked Cholesky in registers)
// before the waves to its right substitute with it.  The solve splits each block's
// contraction over the four waves (4-wide k steps dealt round robin, summed through
// LDS), or for small Grams gives each wave its own 16 right-hand sides.
#include <hip/hip_runtime.h>

#include <algorithm>

#include "condense.h"

namespace dpg {

namespace {

typedef double c4d __attribute__((ext_vector_type(4)));
typedef float c4f __attribute__((ext_vector_type(4)));

// v_mfma_*_16x16x4: lane i + 16 k holds A[i][k] and B[k][i]; accumulator
// register r of lane (g = lane / 16, j = lane % 16) holds C[row(g, r)][j].
template <typename Real> struct Mfma;
template <> struct Mfma<double> {
  typedef c4d acc;
  static __device__ __forceinline__ acc mac(double a, double b, acc c) {
    return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
  }
  static __device__ __forceinline__ int row(int g, int r) { return g + 4 * r; }
};
template <> struct Mfma<float> {
  typedef c4f acc;
  static __device__ __forceinline__ acc mac(float a, float b, acc c) {
    return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
  }
  static __device__ __forceinline__ int row(int g, int r) { return 4 * g + r; }
};

constexpr int NB = 16;            // block rows / panel columns
constexpr int NT = 256;
constexpr int NW = NT / 64;
constexpr int64_t kMaxGrid = int64_t(1) << 22;   // workgroups per launch

// This wave's share of C[i][j] = sum_{k0 <= k < k1} A(i, k) B(k, j), 0 <= i, j < 16:
// 4-wide k steps go round robin to NWV waves (wv: this wave's place among them).
// a(i, k) and b(k, j) are only called for k0 <= k < k1 and return zero outside the
// matrices.  Full waves only.
template <typename Real, int NWV = NW, typename FA, typename FB>
__device__ __forceinline__ typename Mfma<Real>::acc wave_gemm(FA a, FB b, int64_t k0, int64_t k1, int wv, int lane) {
  typedef Mfma<Real> M;
  typename M::acc c = {0, 0, 0, 0};
  const int i = lane & 15, kk = lane >> 4;
  constexpr int64_t step = 4 * NWV;
  int64_t kb = k0 + 4 * wv;
  for (; kb + 3 * step < k1; kb += 4 * step) {   // four steps, loads first
    Real av[4], bv[4];
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const int64_t k = kb + u * step + kk;
      const bool ok = k < k1;
      av[u] = ok ? a(i, k) : Real(0);
      bv[u] = ok ? b(k, i) : Real(0);
    }
#pragma unroll
    for (int u = 0; u < 4; ++u) c = M::mac(av[u], bv[u], c);
  }
  for (; kb < k1; kb += step) {
    const int64_t k = kb + kk;
    const bool ok = k < k1;
    c = M::mac(ok ? a(i, k) : Real(0), ok ? b(k, i) : Real(0), c);
  }
  return c;
}

template <typename Real>
__device__ __forceinline__ void spill(const typename Mfma<Real>::acc& c, Real* red, int lane) {
  const int g = lane >> 4, j = lane & 15;
#pragma unroll
  for (int r = 0; r < 4; ++r) red[Mfma<Real>::row(g, r) * NB + j] = c[r];
}

// Packed 'U' column pointer.
__device__ __forceinline__ int64_t colp(int64_t j) { return j * (j + 1) / 2; }

// Substitution with a 16 x 16 triangular block, one right-hand side per lane.
// The unknowns still to be found sit in registers in the order they are
// reached: each step takes v[0], removes it from the rest and shifts them down
// one register, so every register index is static while the step k stays a
// loop counter (a fully unrolled substitution would hold all 136 block entries
// in registers).  t(k, m) is the coefficient linking the unknown of step k to
// the one m steps later, rpiv(k) the reciprocal of the pivot t(k, 0) (computed once
// per block, so a step costs one multiply); put(k, x) receives the unknown of step k.
template <typename Real, typename FT, typename FR, typename FP>
__device__ __forceinline__ void substitute(Real (&v)[NB], FT t, FR rpiv, FP put) {
#pragma unroll 1
  for (int k = 0; k < NB; ++k) {
    const Real x = v[0] * rpiv(k);
    put(k, x);
#pragma unroll
    for (int m = 1; m < NB; ++m) v[m - 1] = v[m] - t(k, m) * x;
  }
}

// One wave's 16 x 16 x K contraction over contiguous columns, all k steps its own:
// lane (i, kk) holds column i of A at pa and column i of B at pb (va, vb false: zero).
template <typename Real>
__device__ __forceinline__ typename Mfma<Real>::acc wave_gemm_own(const Real* pa, const Real* pb, bool va, bool vb,
                                                                  int64_t k1, int lane) {
  typedef Mfma<Real> M;
  typename M::acc c = {0, 0, 0, 0};
  const int kk = lane >> 4;
  int64_t kb = 0;
  for (; kb + 16 <= k1; kb += 16) {                // four steps, loads first
    Real av[4], bv[4];
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      av[u] = va ? pa[kb + 4 * u + kk] : Real(0);
      bv[u] = vb ? pb[kb + 4 * u + kk] : Real(0);
    }
#pragma unroll
    for (int u = 0; u < 4; ++u) c = M::mac(av[u], bv[u], c);
  }
  for (; kb < k1; kb += 4) {
    const int64_t k = kb + kk;
    const bool ok = k < k1;
    c = M::mac(ok && va ? pa[k] : Real(0), ok && vb ? pb[k] : Real(0), c);
  }
  return c;
}

// Panels of PW = 64 columns, one 16-column tile per wave.  For each 16-row block ib
// down the panel, every wave whose tile lies on or right of the diagonal contracts
// its own tile (no cross-wave sum): S = G[Ib, tile] - U[:ib, Ib]^T U[:ib, tile], with
// the Gram entries fetched beforehand into the accumulator's own layout.  Above the
// panel's diagonal block the tile is finished by substitution with U[Ib, Ib] (read
// from memory); inside it, the wave holding the diagonal tile factors it first and the
// waves to its right substitute with the new factor.  n / 16 (n / 64 + 1) / 2 row
// blocks per element instead of n^2 / 512 with 16-column panels.
template <typename Real>
__global__ void __launch_bounds__(NT) k_potrf(Real* __restrict__ ap, int64_t n, int64_t n_elem,
                                              int32_t* __restrict__ info) {
  typedef Mfma<Real> M;
  constexpr int PW = NB * NW;
  __shared__ Real s_S[NW][NB][NB + 1];      // each wave's tile, row-major
  __shared__ Real s_T[NB][2 * NB];          // U[ib + r][ib + c] at [r][c]; columns >= NB zero
  __shared__ Real s_rd[NB];                 // 1 / U[ib + r][ib + r]
  __shared__ int s_fail;
  const int64_t e = blockIdx.x;
  if (e >= n_elem) return;
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6, li = lane & 15, lg = lane >> 4;
  Real* a = ap + e * (n * (n + 1) / 2);
  s_T[tid >> 4][NB + (tid & 15)] = Real(0);

  for (int64_t jb = 0; jb < n; jb += PW) {
    const int64_t c0 = jb + NB * wv;                         // this wave's first column
    const int wc = int(std::max<int64_t>(0, std::min<int64_t>(NB, n - c0)));   // its columns (0: none)
    const int64_t iend = std::min<int64_t>(jb + PW, n);
    for (int64_t ib = 0; ib < iend; ib += NB) {
      const bool inside = ib >= jb;                          // row block inside the panel's diagonal block
      const int dw = inside ? int((ib - jb) / NB) : -1;      // wave holding the diagonal tile
      const bool act = wc > 0 && c0 >= ib;
      const bool dtile = act && c0 == ib;
      // Gram entries of this lane's accumulator slots, and (above the diagonal block) one
      // entry of U[Ib, Ib] per thread, fetched before the contraction
      Real gv[4];
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int row = M::row(lg, r);
        const bool ok = act && li < wc && (!dtile || row <= li);
        gv[r] = ok ? a[colp(c0 + li) + ib + row] : Real(0);
      }
      const int tr = tid & 15, tc = tid >> 4;
      const Real tv = (!inside && tr <= tc) ? a[colp(ib + tc) + ib + tr] : Real(0);
      typename M::acc c = {0, 0, 0, 0};
      if (act) c = wave_gemm_own<Real>(a + colp(ib + li), a + colp(c0 + li), ib + li < n, li < wc, ib, lane);
#pragma unroll
      for (int r = 0; r < 4; ++r) s_S[wv][M::row(lg, r)][li] = gv[r] - c[r];
      if (!inside) {
        s_T[tr][tc] = tv;
        if (tr == tc) s_rd[tr] = Real(1) / tv;
      }
      __syncthreads();
      if (inside) {
        if (dtile && lane < NB) {           // unblocked Cholesky of the diagonal tile, one column per lane
          const int j = lane, w = wc;
          Real cl[NB];
#pragma unroll
          for (int i = 0; i < NB; ++i) cl[i] = s_S[wv][i][j];
          int fail = 0;
#pragma unroll
          for (int k = 0; k < NB; ++k) {
            if (k < w && !fail) {           // uniform: w and the pivot are the same in every lane
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
          if (j < w && (!fail || j < fail - 1)) {  // on failure the columns before the failing one are final
            Real* dst = a + colp(ib + j) + ib;
#pragma unroll
            for (int i = 0; i < NB; ++i)
              if (i <= j) dst[i] = cl[i];
          }
#pragma unroll
          for (int i = 0; i < NB; ++i) s_T[i][j] = i <= j ? cl[i] : Real(0);
          s_rd[j] = j < w ? Real(1) / cl[j] : Real(1);
          if (j == 0) s_fail = fail ? int(ib) + fail : 0;
        }
        __syncthreads();
        if (s_fail) {
          if (tid == 0 && info) info[e] = s_fail;
          return;
        }
      }
      if (act && !dtile && lane < NB) {     // U[Ib, Ib]^T x = s, one column of the tile per lane
        const int j = lane;
        Real v[NB];
#pragma unroll
        for (int r = 0; r < NB; ++r) v[r] = s_S[wv][r][j];
        Real* dst = a + colp(c0 + j) + ib;
        substitute<Real>(v, [&](int k, int m) { return s_T[k][k + m]; }, [&](int k) { return s_rd[k]; },
                         [&](int k, Real x) {
                           if (j < wc) dst[k] = x;
                         });
      }
      __syncthreads();
    }
  }
  if (tid == 0 && info) info[e] = 0;
}

template <typename Real>
__global__ void __launch_bounds__(NT) k_potrs(const Real* __restrict__ up, int64_t n, int64_t n_elem, int64_t nrhs,
                                              int64_t e0, Real* __restrict__ b) {
  __shared__ Real s_red[NW][NB * NB];
  __shared__ Real s_S[NB][NB + 1];
  __shared__ Real s_T[NB][2 * NB];          // forward: U[ib + r][ib + c] at [r][c]; backward: at [c][NB - 1 - r]
  __shared__ Real s_rd[NB];                 // 1 / U[ib + r][ib + r] (rows past n: 1)
  const int64_t nblk = (nrhs + NB - 1) / NB;
  const int64_t e = e0 + int64_t(blockIdx.x) / nblk, cb = int64_t(blockIdx.x) % nblk;
  if (e >= n_elem) return;
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  const Real* u = up + e * (n * (n + 1) / 2);
  Real* x = b + e * n * nrhs + cb * NB * n;        // column j of this block at x + j n
  const int wc = int(std::min<int64_t>(NB, nrhs - cb * NB));
  s_T[tid >> 4][NB + (tid & 15)] = Real(0);

  // The 16 x 16 diagonal block U[ib + r][ib + c] (rows and columns past n the identity).
  auto fetch_t = [&](int64_t ib, int h) {
    const int r = tid & 15, c = tid >> 4;
    return (r <= c && c < h) ? u[colp(ib + c) + ib + r] : Real(r == c ? 1 : 0);
  };
  auto put_t = [&](Real t, bool fwd) {
    const int r = tid & 15, c = tid >> 4;
    if (fwd)
      s_T[r][c] = t;
    else
      s_T[c][NB - 1 - r] = t;
    if (r == c) s_rd[r] = Real(1) / t;
  };
  auto fetch_x = [&](int64_t ib, int h) {
    const int i = tid >> 4, j = tid & 15;
    return (i < h && j < wc) ? x[j * n + ib + i] : Real(0);
  };
  auto combine = [&](Real s) {
    const int i = tid >> 4, j = tid & 15;
#pragma unroll
    for (int q = 0; q < NW; ++q) s -= s_red[q][i * NB + j];
    s_S[i][j] = s;
  };

  // U^T y = b, top down.
  for (int64_t ib = 0; ib < n; ib += NB) {
    const int h = int(std::min<int64_t>(NB, n - ib));
    const Real tv = fetch_t(ib, h), xv = fetch_x(ib, h);
    const auto c = wave_gemm<Real>([&](int i, int64_t k) { return i < h ? u[colp(ib + i) + k] : Real(0); },
                                   [&](int64_t k, int j) { return j < wc ? x[j * n + k] : Real(0); },
                                   0, ib, wv, lane);
    spill<Real>(c, s_red[wv], lane);
    put_t(tv, true);
    __syncthreads();
    combine(xv);
    __syncthreads();
    if (tid < NB) {                         // U[Ib, Ib]^T y = s, rows top down
      const int j = tid;
      Real v[NB];
#pragma unroll
      for (int r = 0; r < NB; ++r) v[r] = s_S[r][j];
      substitute<Real>(v, [&](int k, int m) { return s_T[k][k + m]; }, [&](int k) { return s_rd[k]; },
                       [&](int k, Real y) {
                         if (j < wc && k < h) x[j * n + ib + k] = y;
                       });
    }
    __syncthreads();
  }
  // U x = y, bottom up.
  for (int64_t ib = ((n - 1) / NB) * NB; ib >= 0; ib -= NB) {
    const int h = int(std::min<int64_t>(NB, n - ib));
    const Real tv = fetch_t(ib, h), xv = fetch_x(ib, h);
    const auto c = wave_gemm<Real>([&](int i, int64_t k) { return i < h ? u[colp(k) + ib + i] : Real(0); },
                                   [&](int64_t k, int j) { return j < wc ? x[j * n + k] : Real(0); },
                                   ib + h, n, wv, lane);
    spill<Real>(c, s_red[wv], lane);
    put_t(tv, false);
    __syncthreads();
    combine(xv);
    __syncthreads();
    if (tid < NB) {                         // U[Ib, Ib] x = s, step k is row NB - 1 - k
      const int j = tid;
      Real v[NB];
#pragma unroll
      for (int r = 0; r < NB; ++r) v[r] = s_S[NB - 1 - r][j];
      // U[NB-1-k-m][NB-1-k] sits at s_T[NB-1-k][k+m]
      substitute<Real>(v, [&](int k, int m) { return s_T[NB - 1 - k][k + m]; },
                       [&](int k) { return s_rd[NB - 1 - k]; }, [&](int k, Real y) {
                         const int r = NB - 1 - k;
                         if (j < wc && r < h) x[j * n + ib + r] = y;
                       });
    }
    __syncthreads();
  }
}

// The solve for small Grams (n <= 256, where the round-robin contraction is short and
// the workgroups many): each wave owns 16 right-hand sides (64 per workgroup) and
// contracts its own tile over all k, so U is read once per 64 right-hand sides and
// there is no cross-wave sum; the 16 x 16 diagonal block of U is fetched once per
// row block for the four waves.
template <typename Real>
__global__ void __launch_bounds__(NT) k_potrs_w(const Real* __restrict__ up, int64_t n, int64_t n_elem, int64_t nrhs,
                                                int64_t e0, Real* __restrict__ b) {
  typedef Mfma<Real> M;
  constexpr int CW = NB * NW;               // right-hand sides per workgroup
  __shared__ Real s_S[NW][NB][NB + 1];      // each wave's tile, row-major
  __shared__ Real s_T[NB][2 * NB];          // forward: U[ib + r][ib + c] at [r][c]; backward: at [c][NB - 1 - r]
  __shared__ Real s_rd[NB];                 // 1 / U[ib + r][ib + r] (rows past n: 1)
  const int64_t nblk = (nrhs + CW - 1) / CW;
  const int64_t e = e0 + int64_t(blockIdx.x) / nblk, cb = int64_t(blockIdx.x) % nblk;
  if (e >= n_elem) return;
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6, li = lane & 15, lg = lane >> 4;
  const Real* u = up + e * (n * (n + 1) / 2);
  const int64_t c0 = cb * CW + NB * wv;     // this wave's first right-hand side
  const int wc = int(std::max<int64_t>(0, std::min<int64_t>(NB, nrhs - c0)));
  Real* x = b + e * n * nrhs + c0 * n;      // its column j at x + j n (not read when wc = 0)
  s_T[tid >> 4][NB + (tid & 15)] = Real(0);

  auto fetch_t = [&](int64_t ib, int h) {
    const int r = tid & 15, c = tid >> 4;
    return (r <= c && c < h) ? u[colp(ib + c) + ib + r] : Real(r == c ? 1 : 0);
  };
  auto put_t = [&](Real t, bool fwd) {
    const int r = tid & 15, c = tid >> 4;
    if (fwd)
      s_T[r][c] = t;
    else
      s_T[c][NB - 1 - r] = t;
    if (r == c) s_rd[r] = Real(1) / t;
  };
  // right-hand side entries of this lane's accumulator slots
  auto fetch_x = [&](int64_t ib, int h, Real (&xv)[4]) {
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int row = M::row(lg, r);
      xv[r] = (row < h && li < wc) ? x[li * n + ib + row] : Real(0);
    }
  };
  auto put_s = [&](const Real (&xv)[4], const typename M::acc& c) {
#pragma unroll
    for (int r = 0; r < 4; ++r) s_S[wv][M::row(lg, r)][li] = xv[r] - c[r];
  };

  // U^T y = b, top down.
  for (int64_t ib = 0; ib < n; ib += NB) {
    const int h = int(std::min<int64_t>(NB, n - ib));
    const Real tv = fetch_t(ib, h);
    Real xv[4];
    fetch_x(ib, h, xv);
    typename M::acc c = {0, 0, 0, 0};
    if (wc > 0) c = wave_gemm_own<Real>(u + colp(ib + li), x + li * n, li < h, li < wc, ib, lane);
    put_s(xv, c);
    put_t(tv, true);
    __syncthreads();
    if (wc > 0 && lane < NB) {              // U[Ib, Ib]^T y = s, rows top down
      const int j = lane;
      Real v[NB];
#pragma unroll
      for (int r = 0; r < NB; ++r) v[r] = s_S[wv][r][j];
      substitute<Real>(v, [&](int k, int m) { return s_T[k][k + m]; }, [&](int k) { return s_rd[k]; },
                       [&](int k, Real y) {
                         if (j < wc && k < h) x[j * n + ib + k] = y;
                       });
    }
    __syncthreads();
  }
  // U x = y, bottom up.
  for (int64_t ib = ((n - 1) / NB) * NB; ib >= 0; ib -= NB) {
    const int h = int(std::min<int64_t>(NB, n - ib));
    const Real tv = fetch_t(ib, h);
    Real xv[4];
    fetch_x(ib, h, xv);
    typename M::acc c = {0, 0, 0, 0};
    if (wc > 0)
      c = wave_gemm<Real, 1>([&](int i, int64_t k) { return i < h ? u[colp(k) + ib + i] : Real(0); },
                             [&](int64_t k, int j) { return j < wc ? x[j * n + k] : Real(0); }, ib + h, n, 0, lane);
    put_s(xv, c);
    put_t(tv, false);
    __syncthreads();
    if (wc > 0 && lane < NB) {              // U[Ib, Ib] x = s, step k is row NB - 1 - k
      const int j = lane;
      Real v[NB];
#pragma unroll
      for (int r = 0; r < NB; ++r) v[r] = s_S[wv][NB - 1 - r][j];
      substitute<Real>(v, [&](int k, int m) { return s_T[NB - 1 - k][k + m]; },
                       [&](int k) { return s_rd[NB - 1 - k]; }, [&](int k, Real y) {
                         const int r = NB - 1 - k;
                         if (j < wc && r < h) x[j * n + ib + r] = y;
                       });
    }
    __syncthreads();
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
  const bool wide = n <= 256;               // one tile per wave (64 right-hand sides per workgroup)
  const int64_t cw = wide ? NB * NW : NB;
  const int64_t nblk = (nrhs + cw - 1) / cw;
  const int64_t per = std::max<int64_t>(1, kMaxGrid / nblk);     // elements per launch
  for (int64_t e0 = 0; e0 < n_elem; e0 += per) {
    const int64_t ne = std::min(per, n_elem - e0);
    const unsigned grid = unsigned(ne * nblk);
    if (prec) {
      auto* u = static_cast<const float*>(up);
      auto* x = static_cast<float*>(b);
      if (wide)
        hipLaunchKernelGGL(k_potrs_w<float>, dim3(grid), dim3(NT), 0, st, u, n, e0 + ne, nrhs, e0, x);
      else
        hipLaunchKernelGGL(k_potrs<float>, dim3(grid), dim3(NT), 0, st, u, n, e0 + ne, nrhs, e0, x);
    } else {
      auto* u = static_cast<const double*>(up);
      auto* x = static_cast<double*>(b);
      if (wide)
        hipLaunchKernelGGL(k_potrs_w<double>, dim3(grid), dim3(NT), 0, st, u, n, e0 + ne, nrhs, e0, x);
      else
        hipLaunchKernelGGL(k_potrs<double>, dim3(grid), dim3(NT), 0, st, u, n, e0 + ne, nrhs, e0, x);
    }
  }
  return hipGetLastError();
}

}  // namespace dpg
