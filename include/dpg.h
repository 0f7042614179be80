/*
 * dpg.h -- C ABI of the sum-factorised DPG Gram-matrix integrator for
 * hexahedral elements on AMD Instinct MI355X (gfx950).
 *
 * What is computed.  For each element K with map x_K : (0,1)^3 -> K the Gram
 * matrix G_IJ = (h_I, h_J) (2.13) of the test space of order p, for one of
 * the four inner products of the hexahedral exact sequence (2.1):
 *   DPG_H1     (u,v) + (grad u, grad v)              (2.28), Section 2.4
 *   DPG_HCURL  (E,F) + (curl E, curl F)              (2.65), Section 2.6
 *   DPG_HDIV   (V,W) + (div V, div W)                (2.46), Section 2.5
 *   DPG_L2     (q,r)                                 (2.14), Section 2.3
 * with hierarchical integrated-Legendre / Legendre shape functions
 * (Section 2.8.2), pushed forward with the Piola maps (2.3)-(2.6).  The
 * value part is weighted by w0 and the derivative part by w1 (w0 = w1 = 1 is
 * the paper's inner product).
 *
 * Shape-function numbering (component a = 0,1,2 concatenated, i1 fastest):
 *   I = off_a + i1 + R1(a) i2 + R1(a) R2(a) i3
 * with ranges R_d(a): H1 p+1; L2 p; H(curl) p if d == a else p+1;
 * H(div) p+1 if d == a else p  (index maps of Sections 2.3-2.6, (2.53), (2.71)).
 * Dimensions: H1 (p+1)^3, H(curl) 3p(p+1)^2, H(div) 3(p+1)p^2, L2 p^3.
 *
 * Output layout.  One symmetric matrix per element in LAPACK 'U' packed
 * column-major storage: entry (I,J), I <= J, at offset I + J(J+1)/2; the
 * element's n(n+1)/2 entries are contiguous.  Elements are consecutive
 * (element e at e * dpg_gram_packed_len(space,p)) unless an offset array is
 * given.  FP64 output is double, FP32 output is float.
 *
 * Paths.  GENERAL is the staged x3 -> x2 -> x1 sum-factorised quadrature
 * (Algorithms 2/3, 5, 7, 9 generalised), O(p^7) per element, with the
 * tensor Gauss-Legendre rule of L points per direction (default L = p+1,
 * L = p for L2).  REDUCED is the constant-Jacobian simplification of
 * Section 2.8.1 (Algorithm 10 carried to all four spaces) using the exact
 * 1D integrals (2.103)-(2.114), O(p^6); it requires affine geometry.
 * AUTO picks REDUCED for affine geometry and GENERAL otherwise.  On affine
 * elements both paths give the same matrix (the rule is exact there).
 *
 * Precision.  FP64: everything in double.  FP32: the Jacobian / metric is
 * evaluated in double, then the coefficient fields and 1D tables are rounded
 * once (round-to-nearest-even) to float; all contractions accumulate in float.
 *
 * Memory.  Unless stated otherwise every pointer argument is a DEVICE
 * pointer owned by the caller; the library never frees caller memory.
 * Streams are hipStream_t passed as void* (NULL = the null stream).  Calls
 * that take a stream only enqueue work and return; results and per-element
 * status words are valid after the stream is synchronised.
 *
 * Errors.  Every int-returning function returns DPG_OK (0) or a negative
 * code; dpg_last_error() gives a message for the calling thread.
 */
#ifndef DPG_H
#define DPG_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum { DPG_H1 = 0, DPG_HCURL = 1, DPG_HDIV = 2, DPG_L2 = 3 };
enum { DPG_FP64 = 0, DPG_FP32 = 1 };
enum { DPG_GEOM_TRILINEAR = 0, DPG_GEOM_AFFINE = 1, DPG_GEOM_EXTRUDED = 2 };
enum { DPG_PATH_AUTO = 0, DPG_PATH_GENERAL = 1, DPG_PATH_REDUCED = 2 };

enum {
  DPG_OK = 0,
  DPG_PENDING = 1,      /* serve: request not finished yet                      */
  DPG_EINVAL = -1,      /* bad argument (space, p, nq, null pointer, path/kind)  */
  DPG_ENOMEM = -2,      /* device or host allocation failed                      */
  DPG_EHIP = -3,        /* HIP runtime error (message in dpg_last_error)         */
  DPG_EJACOBIAN = -4,   /* element with det J <= 0 at a quadrature point         */
  DPG_EAGAIN = -5,      /* serve: queue full, retry later                        */
  DPG_ENOTINIT = -6,    /* null / destroyed context                              */
  DPG_ENODEV = -7       /* no usable gfx950 device                               */
};

#define DPG_P_MAX 11     /* largest supported order p (p + dp of a DPG test space) */

typedef struct dpg_ctx dpg_ctx;
typedef struct dpg_server dpg_server;

/* Element geometry, device memory, float64, C order.
 *   DPG_GEOM_TRILINEAR: data[n_elem][8][3], vertex v = v1 + 2 v2 + 4 v3 at the
 *     master corner (v1,v2,v3); x(xi) = sum_v X_v prod_d (v_d ? xi_d : 1 - xi_d).
 *   DPG_GEOM_AFFINE: data[n_elem][12] = x0[3], J[3][3] row-major, J_ij = dx_i/dxi_j
 *     ((2.2)); x(xi) = x0 + J xi.
 *   DPG_GEOM_EXTRUDED: data[n_elem][10] = x1_0, lambda1, then (x2, x3) of the
 *     cross-section corners (v2,v3) = (0,0), (1,0), (0,1), (1,1); x1 = x1_0 +
 *     lambda1 xi1 and (x2, x3) = sum_{v2,v3} q_{v2 v3} (v2 ? xi2 : 1 - xi2)
 *     (v3 ? xi3 : 1 - xi3): a quadrilateral extruded along x1, the second form of
 *     (2.89).  It is the trilinear map with X_v = (x1_0 + lambda1 v1, q_{v2 v3}).
 * The map must be a diffeomorphism (Section 2.2): det J > 0. */
typedef struct {
  int32_t kind;
  int32_t reserved;
  int64_t n_elem;
  const double* data;
} dpg_geometry;

/* Options.  prec: DPG_FP64 / DPG_FP32.  path: DPG_PATH_*.  GENERAL integrates
 * every kind by quadrature in all three directions (the O(p^7) algorithms).
 * REDUCED (the default for affine and extruded geometry; rejected for
 * trilinear) is the O(p^6) path of Section 2.8.1: exact 1D integrals F^{rs}
 * in all directions for affine maps (Algorithm 10), in xi1 with quadrature in
 * (xi2, xi3) for extruded maps (Algorithm 11).  nq: Gauss-Legendre points
 * per direction of the quadrature path, 0 = default (p+1; p for L2, exact
 * for degree 2 nq - 1 on (0,1), text after (2.22)).  dpg_gram_integrate runs
 * a rule other than the default through the AUTO routes of
 * dpg_gram_integrate_aniso at orders (p, p, p) (nq in [1, 11], p <= 10; AUTO
 * then takes the quadrature path for every geometry kind, REDUCED is
 * rejected: it integrates exactly).  The batched call takes the default only.
 * w0, w1: weights of the value and derivative parts.
 * status: optional device int32[n_elem]; written with DPG_OK or DPG_EJACOBIAN
 * per element.  An element with det J <= 0 at any quadrature point (GENERAL)
 * or det J <= 0 (REDUCED) gets an all-zero output block. */
typedef struct {
  int32_t prec;
  int32_t path;
  int32_t nq;
  int32_t reserved;
  double w0;
  double w1;
  int32_t* status;
} dpg_opts;

/* Fill *opts with the defaults (FP64, AUTO, nq = 0, w0 = w1 = 1, no status). */
void dpg_opts_default(dpg_opts* opts);

/* Build the 1D tables (Gauss-Legendre rules on (0,1) for every point count
 * up to p_max + 1, chi_k and chi'_k at the nodes (2.91)-(2.101), the exact 1D
 * integrals F^{rs} (2.103)-(2.114)) in float64 on the host, with a float32
 * rounding, and make them resident on the current device.  p_max in
 * [1, DPG_P_MAX].  Blocks until the tables are on the device.  The tables are
 * immutable afterwards; the context (tables, tuning table, batched-dispatch
 * cache) may be shared by threads and streams, and owns its device memory
 * until dpg_ctx_destroy, which must not run concurrently with other calls on
 * the context.  The context starts with the library's tuning table: the file
 * named by the environment variable DPG_TUNE_TABLE (an empty value: none; a
 * file that cannot be read or parsed fails the call with DPG_EINVAL), else
 * tune_gfx950.json beside libdpg.so when it exists (see dpg_autotune). */
int dpg_tables_build(int p_max, void* stream, dpg_ctx** ctx);
int dpg_ctx_destroy(dpg_ctx* ctx);

/* Dimension n of the test space and n(n+1)/2; -1 for invalid arguments. */
int64_t dpg_gram_dim(int space, int p);
int64_t dpg_gram_packed_len(int space, int p);

/* Integrate the Gram matrices of geom->n_elem elements of one space and
 * order into out (device, packed, element e at e * packed_len).  opts may be
 * NULL (defaults).  Asynchronous on stream. */
int dpg_gram_integrate(const dpg_ctx* ctx, int space, int p, const dpg_geometry* geom,
                       void* out, const dpg_opts* opts, void* stream);

/* Uneven batch: element e has space[e] and order p[e] (device int8 arrays of
 * length geom->n_elem; p[e] in [1, ctx p_max]) and its packed matrix starts at
 * out + out_offset[e] (device int64, in elements of the output type; regions
 * must not overlap).  All elements share opts (precision, path, weights).
 * The host reads space/p (a device-to-host copy on stream, synchronised; see
 * dpg_gram_integrate_batched_host for callers that hold them on the host) to
 * plan the launch: elements are bucketed by (space, p) and each bucket's
 * kernel is captured as an independent node of one HIP graph, so the buckets
 * run concurrently.  The instantiated graph is cached in the context (up to 8
 * plans, least recently used evicted) keyed by every pointer, size, option and
 * a hash of the space/p contents; an identical later call replays it.  Uses
 * the default point counts only (nq must be 0). */
int dpg_gram_integrate_batched(const dpg_ctx* ctx, const int8_t* space, const int8_t* p,
                               const dpg_geometry* geom, const int64_t* out_offset, void* out,
                               const dpg_opts* opts, void* stream);
/* The same with space and p in HOST memory (int8[n_elem] each; the caller keeps
 * them unchanged until the call returns): no device-to-host read and no
 * synchronisation, so a replayed plan is only enqueued on stream (a new plan
 * still uploads its element lists synchronously once).  The plan cache key
 * holds these host pointers and a hash of their contents. */
int dpg_gram_integrate_batched_host(const dpg_ctx* ctx, const int8_t* space, const int8_t* p,
                                    const dpg_geometry* geom, const int64_t* out_offset, void* out,
                                    const dpg_opts* opts, void* stream);

/* For callers that cannot allocate (code under HIP graph capture, tight
 * serving loops, harnesses that forbid hipMalloc): dpg_gram_integrate_batched
 * with the same arguments and the same results bit for bit, allocating no
 * memory (no hipMalloc or hipFree, no allocating library call), reading nothing
 * back to the host and never synchronising.  The per-(space, p) element lists
 * are built on the device, in a fixed array of the library on each device
 * (4 MiB, held until the process ends), and one launch per (space, p <= ctx
 * p_max) strides over its list.  At most dpg_noalloc_max_elements() (2^20)
 * elements per call (DPG_EINVAL above).  Every call on a device shares that
 * array: calls that overlap on one device (other streams or threads) race and
 * must be serialised by the caller.  An element whose space or order is invalid
 * is skipped (output untouched, status word DPG_EINVAL when status is given);
 * the call itself returns DPG_OK.  nq must be 0.  Asynchronous on stream. */
int dpg_gram_integrate_batched_noalloc(const dpg_ctx* ctx, const int8_t* space, const int8_t* p,
                                       const dpg_geometry* geom, const int64_t* out_offset, void* out,
                                       const dpg_opts* opts, void* stream);
int64_t dpg_noalloc_max_elements(void);

/* Non-uniform orders (p1, p2, p3) (text after Algorithm 2): the 1D pair of
 * direction d has order p[d] (device-independent host array int32[3], each in
 * [1, 10]), so component a spans R_d(a) functions in direction d: H1 p_d+1;
 * L2 p_d; H(div) p_d+1 if d = a else p_d; H(curl) p_d if d = a else p_d+1,
 * flat index as for uniform orders (i1 fastest, components in order).  Each
 * coordinate takes its own Gauss rule (p_d + 1 points, p_d for L2), or opts->nq
 * points in every direction when nq > 0 (at most 11).  Kernels, by opts->path:
 *   DPG_PATH_AUTO: with the default rule (nq = 0), equal orders take the uniform
 *     kernels of dpg_gram_integrate's quadrature path.  Other orders and explicit
 *     rules, where order P = max p_d (raised, for nq > 0, to the order whose default
 *     rule has nq points; P <= 10) carries at most about 16 times the entries
 *     needed, take the uniform kernels of order P with each direction on its own
 *     rule (zero-weight points pad it to order P's count), storing only the entries
 *     of orders (p1, p2, p3) (the 1D bases are hierarchical, Sections 2.4 and
 *     2.8.2; no scratch memory).  Everything else takes the per-direction kernel;
 *   DPG_PATH_GENERAL: always the per-direction kernel, which contracts the
 *     direction of least order last, in the outermost loop.
 * All routes compute the same sums (rounding aside).  Output, geometry, status,
 * weights and precision as for dpg_gram_integrate, with packed length
 * n (n+1)/2, n = dpg_gram_dim_aniso(space, p).  DPG_PATH_REDUCED is rejected.
 * Errors: DPG_EINVAL, DPG_ENOTINIT, DPG_EHIP. */
int64_t dpg_gram_dim_aniso(int space, const int32_t* p);
/* The kernels dpg_gram_integrate_aniso takes for (space, p, opts) (host only, no
 * device work): DPG_ROUTE_UNIFORM, DPG_ROUTE_EMBEDDED or DPG_ROUTE_PER_DIRECTION
 * (the three routes above); DPG_EINVAL for bad space/orders, DPG_ENOTINIT for a
 * null context. */
enum { DPG_ROUTE_PER_DIRECTION = 0, DPG_ROUTE_UNIFORM = 1, DPG_ROUTE_EMBEDDED = 2 };
int dpg_aniso_route(const dpg_ctx* ctx, int space, const int32_t* p, const dpg_opts* opts);
int dpg_gram_integrate_aniso(const dpg_ctx* ctx, int space, const int32_t* p, const dpg_geometry* geom, void* out,
                             const dpg_opts* opts, void* stream);

/* Coupling block of the adjoint graph inner product of the ultraweak
 * formulation (Section 3.3, (3.17), (3.18)), whose test space is H1 x H(div):
 *   C[I][J] = int_K (v_J . grad q_I - q_I div v_J) dx,  q_I in W^p, v_J in V^p.
 * The Piola maps cancel every Jacobian, so C is the same for every element and
 * is computed exactly from the 1D integrals F^{rs}:
 *   C[I][J] = prod_{d != b} F^01_{i_d, j_d+1} (F^10_{i_b, j_b} - F^01_{i_b, j_b})
 * for component b of v_J.  out: device, dense row-major [dim W^p][dim V^p]
 * (dpg_gram_dim), FP64 or FP32 by prec.  With the H1 and H(div) Grams for
 * w0 = omega^2 + alpha, w1 = 1, the adjoint graph Gram of (3.17) is
 *   [[G_H1, -i omega C], [i omega C^T, G_Hdiv]]
 * (rows: first argument (dq, dv), columns: second argument (q, v)).
 * Asynchronous on stream.  Errors: DPG_EINVAL (p outside [1, p_max], null out,
 * prec), DPG_ENOTINIT, DPG_EHIP. */
int dpg_adjoint_coupling(const dpg_ctx* ctx, int p, void* out, int prec, void* stream);

/* Vector-valued test spaces (Section 2.7, (2.85)-(2.88)): the Gram of the
 * `copies`-fold product of a space (the vector H1, H(div), ... of the
 * applications) is block diagonal, with the scalar Gram on each diagonal block.
 * Expands n_elem packed Grams of dimension n (src: consecutive 'U' packed,
 * n (n+1)/2 entries each) into packed Grams of dimension copies * n (dst,
 * consecutive, basis ordered copy by copy), zero off the diagonal blocks.
 * 1 <= copies <= 4; src and dst are device memory of the precision prec and
 * must not overlap.  Asynchronous on stream.  Errors: DPG_EINVAL (sizes,
 * copies, overlap, null pointers, prec), DPG_ENOTINIT, DPG_EHIP. */
int dpg_replicate_blocks(const dpg_ctx* ctx, int64_t n_elem, int64_t n, int copies, const void* src, void* dst,
                         int prec, void* stream);

/* Static condensation of the test variables (Section 1, (3.7)-(3.8)):
 * eliminating s needs G^{-1} B, G^{-1} B~ and G^{-1} l, from a Cholesky
 * factorization of each element's Gram and substitution with the factor.
 *
 * dpg_cholesky_packed factors n_elem Grams of dimension n in place: ap holds
 * consecutive 'U' packed Grams (n (n+1)/2 entries each, as dpg_gram_integrate
 * writes them) on entry and their factors U, G = U^T U with U upper
 * triangular and a positive diagonal, in the same storage on exit (LAPACK
 * dpptrf with uplo 'U').  info: optional device int32[n_elem], 0, or k > 0
 * when the leading minor of order k of that element is not positive
 * definite; then columns 0..k-2 of its U are final and the rest of its
 * storage is unspecified.  Device memory of the precision prec; asynchronous
 * on stream.  n is at most 16384 (the kernels address one element's packed
 * matrix with 32-bit byte offsets).  Errors: DPG_EINVAL (n outside [1, 16384],
 * n_elem < 0, null ap, prec), DPG_ENOTINIT, DPG_EHIP. */
int dpg_cholesky_packed(const dpg_ctx* ctx, int64_t n_elem, int64_t n, void* ap, int32_t* info, int prec,
                        void* stream);

/* Solves G X = B for each element with the factor from dpg_cholesky_packed:
 * up holds the n_elem packed factors; b holds n_elem consecutive column-major
 * n x nrhs blocks (leading dimension n, element e at b + e n nrhs) and is
 * overwritten with X (LAPACK dpptrs).  up and b are device memory of the
 * precision prec and must not overlap.  Asynchronous on stream.  Errors:
 * DPG_EINVAL (n outside [1, 16384], nrhs outside [1, 2^26], n_elem < 0, null
 * pointers, overlap, prec), DPG_ENOTINIT, DPG_EHIP. */
int dpg_cholesky_solve_packed(const dpg_ctx* ctx, int64_t n_elem, int64_t n, const void* up, int64_t nrhs, void* b,
                              int prec, void* stream);

/* Autotuning of the work decomposition (column slabs per workgroup, the
 * kernels' tile shape along the packed output; on the general path also the
 * schedule of the diagonal (i3 = j3) pairs: after all others with a
 * triangular tile, or each right after its slab's other pairs with a full
 * tile).  Every schedule gives the same result bit for bit.  dpg_autotune
 * times every candidate on the given elements (writing their Gram matrices to
 * out, like dpg_gram_integrate), records the fastest for (space, p, precision, path)
 * at the batch-size class floor(log2(n_elem)) in the context, and returns it
 * in *slab_group (optional).  Blocking: synchronises stream.  Later
 * dpg_gram_integrate / _batched calls use the table entry of the nearest size
 * class (within 2 classes); untuned cases use a size heuristic.  The table is
 * internally synchronised and may be saved/loaded as JSON (host paths). */
int dpg_autotune(dpg_ctx* ctx, int space, int p, const dpg_geometry* geom, void* out, const dpg_opts* opts,
                 void* stream, int* slab_group);
int dpg_tune_save(const dpg_ctx* ctx, const char* path);
int dpg_tune_load(dpg_ctx* ctx, const char* path);
/* Forget every tuned schedule of the context (heuristic defaults from then on). */
int dpg_tune_clear(dpg_ctx* ctx);
/* Tuned slabs per workgroup for this case (reduced: 0 general path, 1 reduced
 * path on affine geometry, 2 on extruded geometry), 0 if untuned, -1 on bad
 * arguments. */
int dpg_tune_lookup(const dpg_ctx* ctx, int space, int p, int prec, int reduced, int64_t n_elem);
/* Number of cached batched-dispatch plans (captured graphs) in the context. */
int dpg_batch_plans(const dpg_ctx* ctx);

/* ------------------------------------------------------------------------
 * Serving loop.  An hp-adaptive driver sends integration requests (one space,
 * order p + dp, and a batch of elements) as it refines; the server integrates
 * them on the device with the context's resident tables and keeps each result
 * in device memory until the client releases it.
 *
 *   submit   copies the request's geometry (host or device memory) into
 *            device-resident element slots and queues the request; returns at
 *            once with a ticket (DPG_EAGAIN if the queue or the slots are full).
 *   admit    a scheduler thread admits queued requests in submit order while
 *            their output fits in the memory budget and fewer than max_inflight
 *            requests are unfinished (admission by output-matrix bytes).
 *   launch   requests admitted together that share (space, order, precision,
 *            path, geometry kind, weights) become one launch (up to max_merge
 *            requests); launches go out on n_streams streams, so newly admitted
 *            work overlaps with the work already on the device (continuous
 *            batching: nothing waits for a batch boundary).
 *   poll     DPG_PENDING until the request's work has finished, then DPG_OK
 *            with the result (device pointers and timestamps), or the error
 *            that failed it.
 *   release  returns the result's memory (and its slots) to admission.
 *
 * The server owns each request's geometry copy from submit, and its output
 * from admission, until release.  Element e of a result is at
 * out + e * packed_len (packed 'U' layout as above).  A request whose output
 * exceeds the budget, or whose elements exceed the slots, is rejected by
 * dpg_serve_submit (DPG_EINVAL); dpg_serve_submit_chunked splits it into
 * element chunks instead.  All calls
 * are thread-safe (many submitters; one internal scheduler thread).
 * Timestamps are seconds since dpg_serve_create on a monotonic clock; latency
 * = t_done - t_submit (t_done is when the result became pollable). */
typedef struct {
  int64_t mem_budget_bytes; /* output arena (device memory reserved at create)     */
  int64_t max_slots;        /* element slots for submitted, unreleased requests    */
  int32_t max_inflight;     /* admitted, unfinished requests                      */
  int32_t max_queue;        /* submitted, not yet admitted requests               */
  int32_t n_streams;        /* device streams for launches, 1..8                  */
  int32_t max_merge;        /* requests per launch, 1..32                         */
  /* Test hooks (host-side tests of the scheduler).  test_executor = 1 replaces
   * the device by a timing stub that computes nothing (results have out = NULL;
   * ctx may be NULL): a launch "finishes" test_launch_s + bytes /
   * test_bytes_per_s after it starts.  test_fail_launch = k > 0 makes the k-th
   * launch fail on the host without running: its requests end with DPG_EHIP. */
  int32_t test_executor;
  int32_t test_fail_launch;
  double test_bytes_per_s;
  double test_launch_s;
} dpg_serve_cfg;

typedef struct {
  int32_t space;
  int32_t p;               /* trial order; the Gram order is p + dp (<= ctx p_max) */
  int32_t dp;
  int32_t prec;            /* DPG_FP64 / DPG_FP32                                  */
  int32_t path;            /* DPG_PATH_*                                           */
  int32_t geom_on_host;    /* 1: geom.data is host memory, 0: device memory        */
  dpg_geometry geom;       /* copied at submit; the caller may reuse it at once    */
  double w0, w1;           /* weights of the value / derivative parts              */
  int32_t pdir[3];         /* non-uniform trial orders per direction (all > 0; the
                              Gram orders pdir[d] + dp, each <= 10 and <= ctx p_max;
                              p is then ignored) as dpg_gram_integrate_aniso with the
                              default rule; all zero: the uniform order p            */
  int32_t reserved;        /* 0 */
} dpg_request;

typedef struct {
  int32_t status;          /* DPG_OK, or the error that failed the request          */
  int32_t space, p, prec;  /* p = Gram order (the largest per-direction one for
                              non-uniform orders; packed_len gives the size)       */
  int64_t n_elem;
  int64_t packed_len;      /* entries per element                                   */
  void* out;               /* device, n_elem * packed_len entries (NULL: stub)      */
  int32_t* elem_status;    /* device int32[n_elem]: DPG_OK / DPG_EJACOBIAN          */
  double t_submit, t_admit, t_done;
} dpg_result;

typedef struct {
  int64_t submitted, rejected, admitted, completed, failed, launches;
  int64_t cancelled;                      /* released while still queued            */
  int64_t queued, inflight;               /* now                                   */
  int64_t elements;                       /* elements in completed requests         */
  int64_t budget_bytes, admitted_bytes, peak_admitted_bytes;
  int64_t max_concurrent_launches;        /* most launches on the device at once    */
  double bytes;                           /* output bytes of completed requests     */
  double t_first_submit, t_last_done;
  double lat_p50, lat_p99, lat_mean, lat_max;   /* submit -> pollable, seconds      */
  double wait_p50, wait_p99;                    /* submit -> admit, seconds         */
} dpg_serve_stats;

void dpg_serve_cfg_default(dpg_serve_cfg* cfg);  /* 1 GiB, 2^18 slots, 64, 4096, 4 streams, 32 */
int dpg_serve_create(dpg_ctx* ctx, const dpg_serve_cfg* cfg, dpg_server** srv);
int dpg_serve_submit(dpg_server* srv, const dpg_request* req, uint64_t* ticket);
/* A request of any size: the server cuts it into consecutive element chunks of
 * *chunk_elems elements (the last one shorter), as many as fit max_chunk_bytes
 * of output (0: the memory budget) and the element slots, and queues them as
 * requests with the consecutive tickets *first_ticket .. *first_ticket +
 * *n_chunks - 1; chunk k holds elements [k * *chunk_elems, ...) of the request.
 * Each chunk is polled, read and released like a request of its own; the
 * chunks are admitted in order as memory frees up, so a request larger than
 * the budget streams through it while the client releases the chunks it has
 * read.  All chunks are queued, or none: DPG_EAGAIN when the queue or the
 * element slots cannot take them all now, DPG_EINVAL when one element's output
 * exceeds the chunk size or the chunks exceed max_queue.  chunk_elems may be
 * NULL. */
int dpg_serve_submit_chunked(dpg_server* srv, const dpg_request* req, int64_t max_chunk_bytes,
                             uint64_t* first_ticket, int64_t* n_chunks, int64_t* chunk_elems);
int dpg_serve_poll(dpg_server* srv, uint64_t ticket, dpg_result* res);
/* Copy elements [first, first + count) of a finished result to dst (host or
 * device), asynchronously on stream.  Release the request only after the copy
 * has completed (synchronise stream first): release hands the memory to the
 * next admitted request. */
int dpg_serve_read(dpg_server* srv, uint64_t ticket, void* dst, int64_t first, int64_t count, void* stream);
/* Copy the status words (int32, DPG_OK / DPG_EJACOBIAN) of elements
 * [first, first + count) of a finished result to dst (host or device). */
int dpg_serve_read_status(dpg_server* srv, uint64_t ticket, int32_t* dst, int64_t first, int64_t count,
                          void* stream);
/* Release a finished result, or cancel a request that is still queued;
 * DPG_EAGAIN for a request whose work is on the device. */
int dpg_serve_release(dpg_server* srv, uint64_t ticket);
int dpg_serve_stats_get(dpg_server* srv, dpg_serve_stats* st);
int dpg_serve_stats_reset(dpg_server* srv);   /* clears counters and latency samples */
/* Stops the scheduler after the device work already started has finished,
 * and frees all server memory (unreleased results included). */
int dpg_serve_destroy(dpg_server* srv);

/* Host-only helpers (no device needed): the tables the library builds. */
/* zeta[L], w[L], chi[(kmax+1) * L], dchi[(kmax+1) * L] with chi[k * L + l] = chi_k(zeta_l). */
int dpg_host_tables(int L, int kmax, double* zeta, double* w, double* chi, double* dchi);
/* F[(kmax+1)^2] with F[i * (kmax+1) + j] = int_0^1 chi^<r>_i chi^<s>_j  ((2.90)). */
int dpg_host_ftable(int r, int s, int kmax, double* F);
/* Algorithmic work of one element on the GENERAL path: flops of the three
 * staged contractions (2.23)-(2.25) over the upper block triangle of (i3, j3)
 * pairs: 2 L^3 per term and pair (xi3), 2 L^2 per merged term, l and (i2, j2)
 * (xi2), 2 L per group of terms and packed output entry (xi1); -1 on invalid
 * arguments.  dpg_general_flops counts stage xi2 over every (i2, j2) of each
 * pair (H1 p = 7: 11.43 MFLOP); dpg_general_flops_trimmed counts only i2 <= j2
 * for the diagonal pairs i3 = j3 of the diagonal blocks, which is all that the
 * packed upper triangle needs and what the kernels compute (H1 p = 7: 11.17). */
double dpg_general_flops(int space, int p);
double dpg_general_flops_trimmed(int space, int p);

/* Message describing the last error on the calling thread ("" if none). */
const char* dpg_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* DPG_H */
