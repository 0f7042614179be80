// Instantiation of the general-path kernels for one space (split per space so
// the build compiles them in parallel).
#include "gram_general.inc.h"

namespace dpg {

hipError_t launch_general_h1(int p, int prec, const GeneralArgs& a, hipStream_t s) {
  return dispatch_general<SP_H1, false>(p, prec, a, s);
}

}  // namespace dpg
