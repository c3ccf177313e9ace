// Table of the built filter kernels: one entry per (model, precision, launch shape).
#pragma once

#include <vector>

#include "pf_kernel.h"

namespace smc2 {

struct PFKernel {
  int model, dx, precision, waves, ppl;
  // launch and resident workgroups per compute unit, for the every-step checkpoint sweep
  // (every = 1) or the segment recompute
  void (*launch)(const PFArgs &, int grid, hipStream_t);
  int (*occupancy)(int lds_T, int every);
  size_t (*dyn_lds)(int lds_T);      // dynamic shared memory per workgroup
  size_t (*static_lds)();            // static shared memory per workgroup (both sweeps' maximum)
};

// Launch shapes (tile index -> waves per workgroup, particles per lane).  Index 0 is "tuned".
struct Tile {
  int waves, ppl;
};
constexpr Tile kTiles[] = {{0, 0},  {1, 1}, {2, 1}, {1, 4},  {4, 1}, {1, 8},  {2, 4},
                           {4, 2},  {1, 16}, {2, 8}, {4, 4}, {8, 2}, {2, 16}, {4, 8},
                           {8, 4},  {4, 16}, {8, 8}, {16, 2}};
constexpr int kNumTiles = (int)(sizeof(kTiles) / sizeof(kTiles[0]));

template <typename R, class Model, int W, int P>
size_t dyn_lds_pf(int lds_T) {
  return pf_dyn_lds_bytes<R, Model::DY, Model::kPerStep>(lds_T);
}

template <typename R, class Model, int W, int P>
void launch_pf(const PFArgs &a, int grid, hipStream_t st) {
  const size_t dyn = pf_dyn_lds_bytes<R, Model::DY, Model::kPerStep>(a.lds_T);
  if (a.ckpt == 1)
    hipLaunchKernelGGL((pf_fwd_adj_kernel<R, Model, W, P, true>), dim3(grid), dim3(W * 64), dyn,
                       st, a);
  else
    hipLaunchKernelGGL((pf_fwd_adj_kernel<R, Model, W, P, false>), dim3(grid), dim3(W * 64), dyn,
                       st, a);
}

template <typename R, class Model, int W, int P>
int occupancy_pf(int lds_T, int every) {
  int n = 0;
  const size_t dyn = dyn_lds_pf<R, Model, W, P>(lds_T);
  const hipError_t e =
      every ? hipOccupancyMaxActiveBlocksPerMultiprocessor(
                  &n, pf_fwd_adj_kernel<R, Model, W, P, true>, W * 64, dyn)
            : hipOccupancyMaxActiveBlocksPerMultiprocessor(
                  &n, pf_fwd_adj_kernel<R, Model, W, P, false>, W * 64, dyn);
  if (e != hipSuccess || n < 1) n = 1;
  return n;
}

// as the compiler laid it out; the kernels' own arrays otherwise take at most 64 KiB plus the
// per-particle staging
template <typename R, class Model, int W, int P>
size_t static_lds_pf() {
  size_t n = 0;
  hipFuncAttributes fa;
  if (hipFuncGetAttributes(&fa, reinterpret_cast<const void *>(
                                    &pf_fwd_adj_kernel<R, Model, W, P, true>)) == hipSuccess)
    n = std::max(n, fa.sharedSizeBytes);
  else
    n = 65536 + (size_t)W * 64 * P * (sizeof(double) + 3 * sizeof(R)) + 4096;
  if (hipFuncGetAttributes(&fa, reinterpret_cast<const void *>(
                                    &pf_fwd_adj_kernel<R, Model, W, P, false>)) == hipSuccess)
    n = std::max(n, fa.sharedSizeBytes);
  return n;
}

template <typename R, class Model, int W, int P>
void add_entry(std::vector<PFKernel> &v, int model, int precision) {
  v.push_back(PFKernel{model, Model::DX, precision, W, P, &launch_pf<R, Model, W, P>,
                       &occupancy_pf<R, Model, W, P>, &dyn_lds_pf<R, Model, W, P>,
                       &static_lds_pf<R, Model, W, P>});
}

// Every d=1 launch shape for one (R, Model).
template <typename R, class Model>
void add_all_tiles_1d(std::vector<PFKernel> &v, int model, int precision) {
  add_entry<R, Model, 1, 1>(v, model, precision);
  add_entry<R, Model, 2, 1>(v, model, precision);
  add_entry<R, Model, 1, 4>(v, model, precision);
  add_entry<R, Model, 4, 1>(v, model, precision);
  add_entry<R, Model, 1, 8>(v, model, precision);
  add_entry<R, Model, 2, 4>(v, model, precision);
  add_entry<R, Model, 4, 2>(v, model, precision);
  add_entry<R, Model, 1, 16>(v, model, precision);
  add_entry<R, Model, 2, 8>(v, model, precision);
  add_entry<R, Model, 4, 4>(v, model, precision);
  add_entry<R, Model, 8, 2>(v, model, precision);
  add_entry<R, Model, 2, 16>(v, model, precision);
  add_entry<R, Model, 4, 8>(v, model, precision);
  add_entry<R, Model, 8, 4>(v, model, precision);
  add_entry<R, Model, 4, 16>(v, model, precision);
  add_entry<R, Model, 8, 8>(v, model, precision);
}

// Launch shapes for the 16-dimensional state (register budget: x is 16 values per particle).
template <typename R, class Model>
void add_all_tiles_16d(std::vector<PFKernel> &v, int model, int precision) {
  add_entry<R, Model, 1, 1>(v, model, precision);
  add_entry<R, Model, 2, 1>(v, model, precision);
  add_entry<R, Model, 4, 1>(v, model, precision);
  add_entry<R, Model, 4, 2>(v, model, precision);
  add_entry<R, Model, 8, 2>(v, model, precision);
  add_entry<R, Model, 8, 4>(v, model, precision);
  // sixteen waves x two particles per lane in FP32 only: in FP64 the state and its adjoint
  // alone fill the 128 registers a lane has at four waves per SIMD, and that kernel (2 KB of
  // spills per lane) returned gradients off the oracle once other kernels had run in the same
  // process; the FP64 form runs 2048 particles on eight waves x four
  if constexpr (sizeof(R) == 4) add_entry<R, Model, 16, 2>(v, model, precision);
}

// Launch shapes for the two-component state (SIR): one particle per lane or an even number.
template <typename R, class Model>
void add_all_tiles_2d(std::vector<PFKernel> &v, int model, int precision) {
  add_entry<R, Model, 1, 1>(v, model, precision);
  add_entry<R, Model, 2, 1>(v, model, precision);
  add_entry<R, Model, 1, 4>(v, model, precision);
  add_entry<R, Model, 4, 1>(v, model, precision);
  add_entry<R, Model, 2, 4>(v, model, precision);
  add_entry<R, Model, 4, 2>(v, model, precision);
  add_entry<R, Model, 4, 4>(v, model, precision);
  add_entry<R, Model, 8, 2>(v, model, precision);
  add_entry<R, Model, 8, 4>(v, model, precision);
  add_entry<R, Model, 16, 2>(v, model, precision);
}

void register_lg1d(std::vector<PFKernel> &);
void register_growth(std::vector<PFKernel> &);
void register_sv(std::vector<PFKernel> &);
void register_lgdiag(std::vector<PFKernel> &);
void register_lg1dopt(std::vector<PFKernel> &);
void register_sir(std::vector<PFKernel> &);

}  // namespace smc2
