// ctx.h -- library-internal context state shared by the C ABI translation units.
#pragma once
#include <hip/hip_runtime.h>

#include <cstdint>
#include <map>
#include <memory>
#include <mutex>
#include <vector>

#include "../../include/dpg.h"
#include "errors.h"
#include "kernels.h"

namespace dpg {

int hip_fail(hipError_t e, const char* what);
inline bool valid_space(int s) { return s >= DPG_H1 && s <= DPG_L2; }

// Autotuning key: one (space, order, precision, path: 0 general, 1 reduced on
// affine geometry, 2 reduced on extruded geometry) at a batch-size class
// (floor(log2(n_elem))).  Value: the schedule (column slabs per workgroup and
// the diagonal-pair schedule) and its time.
struct TuneKey {
  int space, p, prec, reduced, size_class;
  bool operator<(const TuneKey& o) const {
    if (space != o.space) return space < o.space;
    if (p != o.p) return p < o.p;
    if (prec != o.prec) return prec < o.prec;
    if (reduced != o.reduced) return reduced < o.reduced;
    return size_class < o.size_class;
  }
};
struct TuneVal {
  int slab_group;
  float ms;
  int diag = -1;
};

// Work decomposition of a general-path launch: slabs per workgroup (0 = kernel
// heuristic) and diagonal pairs (-1 = default for the order, 0 = last with the
// triangular x tiling, 1 = each closing its slab in the full x tiling).
struct Sched {
  int slab_group = 0;
  int diag = -1;
};

struct BatchPlan;   // batch.cpp

int size_class(int64_t n);

}  // namespace dpg

struct dpg_ctx {
  int p_max = 0;
  int device = 0;
  double* d_tab64 = nullptr;
  float* d_tab32 = nullptr;
  double* d_f64 = nullptr;
  float* d_f32 = nullptr;
  // mutable state (the tables above are immutable after dpg_tables_build)
  mutable std::mutex mu;                                    // guards tune and plans
  mutable std::map<dpg::TuneKey, dpg::TuneVal> tune;
  mutable std::vector<std::shared_ptr<dpg::BatchPlan>> plans;   // most recent last
  ~dpg_ctx();
};

namespace dpg {

// Kernel family of a launch: 0 general, 1 reduced (affine), 2 reduced (extruded).
int path_code(const dpg_geometry* geom, const dpg_opts& o);
int check_common(const dpg_ctx* ctx, const dpg_geometry* geom, void* out, const dpg_opts& o);

// Launch the kernels of one (space, p) over n_items elements (elem_ids maps
// items to elements, nullptr = identity; out_offset nullptr = e * packed_len).
// With list, a listed launch: the item count and the first entry of elem_ids are
// read from the device ({count, first} at list), and n_items is only the expected
// count, which sizes the grid and the slab groups.
int launch_elements(const dpg_ctx* ctx, int space, int p, const dpg_geometry* geom, void* out,
                    const dpg_opts& o, const int32_t* elem_ids, int64_t n_items, const int64_t* out_offset,
                    Sched sched, hipStream_t st, const int32_t* list = nullptr);

// Non-uniform orders p[3] (or equal orders with a rule other than the default) on the
// generic kernel: one rule per direction (opts nq points in every direction when nq > 0).
int integrate_aniso(const dpg_ctx* ctx, int space, const int32_t* p, const dpg_geometry* geom, void* out,
                    const dpg_opts& o, hipStream_t st);

// Non-uniform orders (or an explicit rule) on the uniform kernels of order max p_d, raised
// to a default rule of at least nq points (aniso_embed.hip): whether the call takes that
// route (AUTO path, that order <= 10, and at most about 16 times the entries needed),
// and the launch.
bool embed_applies(const dpg_ctx* ctx, int space, const int32_t* p, const dpg_opts& o);
int integrate_aniso_embed(const dpg_ctx* ctx, int space, const int32_t* p, const dpg_geometry* geom, void* out,
                          const dpg_opts& o, hipStream_t st);

// Load the tuning table shipped with the library (dpg_tables_build).
int load_default_tune(dpg_ctx* ctx);

// Schedule from the tuning table (defaults when not tuned).
Sched tuned_sched(const dpg_ctx* ctx, int space, int p, int prec, int path, int64_t n);

void destroy_plans(dpg_ctx* ctx);

// Take the device address of the allocation-free batch's list array on device dev
// (the current device); once per device, from dpg_tables_build.
int noalloc_init(int dev);

}  // namespace dpg
