// kernels.h -- launch interface between the C ABI layer and the HIP kernels.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "launch_limits.h"

namespace dpg {

constexpr int PMAX = 11;           // largest order p
constexpr int LMAX = PMAX + 1;     // largest point count
constexpr int KT = PMAX + 2;       // 1D function indices 0..PMAX+1 kept in the tables

// Per point count L, one table block (both precisions share the layout):
//   zeta[L] | w[L] | chi[KT][L] | dchi[KT][L]
// The FP64 block is used for the metric (always FP64) and the FP64 path;
// the FP32 block is the same table rounded once to float.
constexpr int table_block_len(int L) { return 2 * L + 2 * KT * L; }
constexpr int table_offset(int L) {
  int o = 0;
  for (int l = 1; l < L; ++l) o += table_block_len(l);
  return o;
}
constexpr int TABLE_LEN = table_offset(LMAX + 1);
constexpr int FTAB_LEN = 4 * KT * KT;   // F^{rs}[i][j] at ((2r+s)*KT + i)*KT + j

struct GeneralArgs {
  const double* geom;        // trilinear [E][8][3] or affine [E][12]
  int geom_kind;             // 0 trilinear, 1 affine, 2 extruded
  int64_t n_items;           // elements in this launch
  int64_t item_base;         // first item of this launch (grid chunking)
  const int32_t* elem_ids;   // item -> element (nullptr: identity)
  void* out;                 // Real*
  const int64_t* out_offset; // element -> first output entry (nullptr: e * packed_len)
  int64_t packed_len;
  const double* tab64;       // FP64 table block for this L
  const void* tabR;          // table block in the output precision
  const void* ftabR;         // F tables in the output precision (reduced path)
  double w0, w1;
  int32_t* status;           // per element (nullptr: none)
  int slab_group;            // column slabs per workgroup (0: choose from the batch size)
  int diag_inline;           // diagonal pairs: -1 default for the order, 0 last with the
                             // triangular x tiling, 1 each closing its slab (full x tiling)
  const int32_t* list;       // listed launch: {item count, first entry in elem_ids} in device
                             // memory (nullptr: n_items and elem_ids as given)
  // Orders (p1, p2, p3) embedded in the order of the launch (launch_embed_*): direction d
  // takes the emb_L[d]-point rule (table blocks emb_tab64[d], emb_tabR[d]), component b
  // only its column slabs j3 < emb_jmax[b], and the output is numbered by the embedded
  // orders: component a spans emb_R[a][d] functions in direction d from emb_off[a]
  // (packed_len is then that numbering's packed length).
  const double* emb_tab64[3];
  const void* emb_tabR[3];
  int emb_L[3];
  int emb_jmax[3];
  int emb_R[3][3];
  int emb_off[4];
};

// Workgroups of a listed launch (the item count is on the device): enough to fill the
// GPU several times over, each striding over the (item, slab group) pairs.
constexpr int64_t LIST_GRID = 2048;
inline unsigned list_grid(int64_t expected_items, int ngroups) {
  const int64_t w = expected_items * ngroups;
  return unsigned(w < 1 ? 1 : (w < LIST_GRID ? w : LIST_GRID));
}

// Column slabs per workgroup: whole elements when the batch alone fills the GPU
// (about WG_TARGET workgroups), smaller groups for small batches.
constexpr int64_t WG_TARGET = 2048;
inline int slab_group_for(int nslab, int64_t n_items, int requested) {
  if (requested > 0) return requested < nslab ? requested : nslab;
  int64_t g = n_items * nslab / WG_TARGET;
  if (g < 1) g = 1;
  if (g > nslab) g = nslab;
  return int(g);
}

// General (sum-factorised quadrature) path; prec 0 = FP64, 1 = FP32.
hipError_t launch_general_h1(int p, int prec, const GeneralArgs& a, hipStream_t s);
hipError_t launch_general_hcurl(int p, int prec, const GeneralArgs& a, hipStream_t s);
hipError_t launch_general_hdiv(int p, int prec, const GeneralArgs& a, hipStream_t s);
hipError_t launch_general_l2(int p, int prec, const GeneralArgs& a, hipStream_t s);
// The same with a listed launch (GeneralArgs::list set).
hipError_t launch_general_list_h1(int p, int prec, const GeneralArgs& a, hipStream_t s);
hipError_t launch_general_list_hcurl(int p, int prec, const GeneralArgs& a, hipStream_t s);
hipError_t launch_general_list_hdiv(int p, int prec, const GeneralArgs& a, hipStream_t s);
hipError_t launch_general_list_l2(int p, int prec, const GeneralArgs& a, hipStream_t s);

// General path with orders embedded in order p (GeneralArgs::emb_*), output in the
// embedded orders' numbering.
hipError_t launch_embed_h1(int p, int prec, const GeneralArgs& a, hipStream_t s);
hipError_t launch_embed_hcurl(int p, int prec, const GeneralArgs& a, hipStream_t s);
hipError_t launch_embed_hdiv(int p, int prec, const GeneralArgs& a, hipStream_t s);
hipError_t launch_embed_l2(int p, int prec, const GeneralArgs& a, hipStream_t s);

// Reduced (constant Jacobian, exact 1D integrals) path; affine geometry only.
hipError_t launch_affine(int space, int p, int prec, const GeneralArgs& a, hipStream_t s);

// Adjoint graph coupling block C[dim W^p][dim V^p] (row-major) from the F tables of
// the precision; block-diagonal replication of packed Grams (n -> copies * n).
hipError_t launch_coupling(int p, int prec, const void* F, void* out, hipStream_t s);
hipError_t launch_replicate(int prec, const void* src, void* dst, int64_t n, int copies, int64_t n_elem,
                            hipStream_t s);

// Reduced path for extruded elements (exact xi1 integrals, quadrature in xi2, xi3);
// extruded geometry only.
hipError_t launch_extruded(int space, int p, int prec, const GeneralArgs& a, hipStream_t s);

}  // namespace dpg
