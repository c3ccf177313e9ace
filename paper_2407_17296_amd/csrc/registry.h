// Table of the built filter kernels: one entry per (model, precision, launch shape).
#pragma once

#include <vector>

#include "pf_kernel.h"

namespace smc2 {

struct PFKernel {
  int model, dx, precision, waves, ppl;
  void (*launch)(const PFArgs &, int grid, hipStream_t);
  int (*occupancy)();  // resident workgroups per compute unit
};

// Launch shapes (tile index -> waves per workgroup, particles per lane).  Index 0 is "tuned".
struct Tile {
  int waves, ppl;
};
constexpr Tile kTiles[] = {{0, 0}, {1, 1}, {2, 1}, {4, 1}, {1, 4}, {4, 2}, {8, 1},
                           {4, 4}, {8, 2}, {8, 4}, {16, 4}, {16, 2}};
constexpr int kNumTiles = (int)(sizeof(kTiles) / sizeof(kTiles[0]));

template <typename R, class Model, int W, int P>
void launch_pf(const PFArgs &a, int grid, hipStream_t st) {
  hipLaunchKernelGGL((pf_fwd_adj_kernel<R, Model, W, P>), dim3(grid), dim3(W * 64), 0, st, a);
}

template <typename R, class Model, int W, int P>
int occupancy_pf() {
  int n = 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, pf_fwd_adj_kernel<R, Model, W, P>, W * 64,
                                                   0) != hipSuccess || n < 1)
    n = 1;
  return n;
}

template <typename R, class Model, int W, int P>
void add_entry(std::vector<PFKernel> &v, int model, int precision) {
  v.push_back(PFKernel{model, Model::DX, precision, W, P, &launch_pf<R, Model, W, P>,
                       &occupancy_pf<R, Model, W, P>});
}

// Every d=1 launch shape for one (R, Model).
template <typename R, class Model>
void add_all_tiles_1d(std::vector<PFKernel> &v, int model, int precision) {
  add_entry<R, Model, 1, 1>(v, model, precision);
  add_entry<R, Model, 2, 1>(v, model, precision);
  add_entry<R, Model, 4, 1>(v, model, precision);
  add_entry<R, Model, 1, 4>(v, model, precision);
  add_entry<R, Model, 4, 2>(v, model, precision);
  add_entry<R, Model, 8, 1>(v, model, precision);
  add_entry<R, Model, 4, 4>(v, model, precision);
  add_entry<R, Model, 8, 2>(v, model, precision);
  add_entry<R, Model, 8, 4>(v, model, precision);
  add_entry<R, Model, 16, 4>(v, model, precision);
  add_entry<R, Model, 16, 2>(v, model, precision);
}

// Launch shapes for the 16-dimensional state (register budget: x is 16 values per particle).
template <typename R, class Model>
void add_all_tiles_16d(std::vector<PFKernel> &v, int model, int precision) {
  add_entry<R, Model, 1, 1>(v, model, precision);
  add_entry<R, Model, 2, 1>(v, model, precision);
  add_entry<R, Model, 4, 1>(v, model, precision);
  add_entry<R, Model, 8, 1>(v, model, precision);
  add_entry<R, Model, 8, 2>(v, model, precision);
  add_entry<R, Model, 16, 2>(v, model, precision);
}

void register_lg1d(std::vector<PFKernel> &);
void register_growth(std::vector<PFKernel> &);
void register_sv(std::vector<PFKernel> &);
void register_lgdiag(std::vector<PFKernel> &);

}  // namespace smc2
