// Instantiations of the fused filter kernel for one model, in both precisions.
#include "registry.h"

namespace smc2 {

void register_growth(std::vector<PFKernel> &v) {
  add_all_tiles_1d<double, ModelGrowth<double>>(v, 2, 0);
  add_all_tiles_1d<float, ModelGrowth<float>>(v, 2, 1);
}

}  // namespace smc2
