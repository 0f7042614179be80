// Instantiation of the general-path kernels with per-direction rules embedded in a
// uniform order, for one space (orders (p1, p2, p3) of dpg_gram_integrate_aniso).
#include "gram_general.inc.h"

namespace dpg {

hipError_t launch_embed_h1(int p, int prec, const GeneralArgs& a, hipStream_t s) {
  return dispatch_embed<SP_H1>(p, prec, a, s);
}

}  // namespace dpg
