// Instantiations of the fused filter kernel for one model, in both precisions.
#include "registry.h"

namespace smc2 {

void register_lg1d(std::vector<PFKernel> &v) {
  add_all_tiles_1d<double, ModelLG1D<double>>(v, 0, 0);
  add_all_tiles_1d<float, ModelLG1D<float>>(v, 0, 1);
}

}  // namespace smc2
