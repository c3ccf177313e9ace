// Instantiations of the fused filter kernel for one model, in both precisions.
#include "registry.h"

namespace smc2 {

void register_sv(std::vector<PFKernel> &v) {
  add_all_tiles_1d<double, ModelSV<double>>(v, 3, 0);
  add_all_tiles_1d<float, ModelSV<float>>(v, 3, 1);
}

}  // namespace smc2
