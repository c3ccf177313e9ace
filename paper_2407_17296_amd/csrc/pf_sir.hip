// Instantiations of the fused filter kernel for one model, in both precisions.
#include "registry.h"

namespace smc2 {

void register_sir(std::vector<PFKernel> &v) {
  add_all_tiles_2d<double, ModelSIR<double>>(v, 5, 0);
  add_all_tiles_2d<float, ModelSIR<float>>(v, 5, 1);
}

}  // namespace smc2
