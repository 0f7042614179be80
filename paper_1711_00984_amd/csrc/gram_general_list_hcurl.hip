// Instantiation of the listed general-path kernels for one space: the item count
// of the launch comes from device memory (the allocation-free batch).
#include "gram_general.inc.h"

namespace dpg {

hipError_t launch_general_list_hcurl(int p, int prec, const GeneralArgs& a, hipStream_t s) {
  return dispatch_general<SP_HCURL, true>(p, prec, a, s);
}

}  // namespace dpg
