// Instantiations of the fused filter kernel for one model, in both precisions.
#include "registry.h"

namespace smc2 {

void register_lgdiag(std::vector<PFKernel> &v) {
  add_all_tiles_16d<double, ModelLGDiag<double, 16>>(v, 1, 0);
  add_all_tiles_16d<float, ModelLGDiag<float, 16>>(v, 1, 1);
}

}  // namespace smc2
