// Instantiations of the fused filter kernel for the 1-D LG model with the optimal proposal, in
// both precisions.
#include "registry.h"

namespace smc2 {

void register_lg1dopt(std::vector<PFKernel> &v) {
  add_all_tiles_1d<double, ModelLG1DOpt<double>>(v, 4, 0);
  add_all_tiles_1d<float, ModelLG1DOpt<float>>(v, 4, 1);
}

}  // namespace smc2
