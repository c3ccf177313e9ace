// Kernels of the SMC^2 outer step (paper Sec. III) and small utilities.
//   K2 langevin_move_kernel   -- proposal SMC1 (or SMC0), one thread per sample.
//   K3 reweight_resample_kernel -- L-kernel weight, normalisation, ESS, systematic resampling,
//                                  one workgroup per series.
#pragma once

#include "device_common.h"

namespace smc2 {

constexpr int kMaxD = 32;

// Independent priors: kind 0 N(mu, sd^2); kind 1 uniform on [mu, sd] (lower, upper bound).
// lnorm: log sd (normal) or log(upper - lower) (uniform), formed on the host.
struct Prior {
  double mu[kMaxD], sd[kMaxD], lnorm[kMaxD];
  int kind[kMaxD];
};

// theta_1 ~ prior (eq. init_sample with q_1 = prior): one thread per (s, i); normal number p of
// the sample's prior stream for a normal parameter, uniform number p for a uniform one.
__global__ void prior_init_kernel(int n_items, int D, Prior pr, uint64_t seed, double *theta) {
  const int item = blockIdx.x * blockDim.x + threadIdx.x;
  if (item >= n_items) return;
  const uint32_t c3 = stream_word(1u, kStreamPrior);
  for (int p = 0; p < D; ++p)
    theta[(size_t)item * D + p] =
        pr.kind[p] == 1
            ? pr.mu[p] + (pr.sd[p] - pr.mu[p]) *
                             uniform_m(kNoSlot, (uint32_t)item, c3, (uint32_t)p, seed)
            : pr.mu[p] + pr.sd[p] * normal_n<double>(kNoSlot, (uint32_t)item, c3, (uint32_t)p,
                                                     seed);
}

// K2: p_{k-1} = gamma xi, theta_new = theta + (gamma^2/2) grad_logpost + p_{k-1} (SMC1,
// Sec. III-D, in the velocity form of Sec. III-E); SMC0 drops the gradient term.
__global__ void langevin_move_kernel(int n_items, int D, double gamma, int random_walk,
                                     const double *theta, const double *grad_logpost,
                                     uint64_t seed, const uint32_t *iteration, double *theta_new,
                                     double *p_prev) {
  const int item = blockIdx.x * blockDim.x + threadIdx.x;
  if (item >= n_items) return;
  const uint32_t c3 = stream_word(*iteration, kStreamMove);
  const double half_g2 = 0.5 * gamma * gamma;
  for (int b = 0; b * 4 < D; ++b) {
    double z[4];
    normals4<double>(kNoSlot, (uint32_t)b, (uint32_t)item, c3, seed, z);
    for (int r = 0; r < 4 && 4 * b + r < D; ++r) {
      const size_t o = (size_t)item * D + 4 * b + r;
      const double pv = gamma * z[r];
      p_prev[o] = pv;
      theta_new[o] = random_walk ? theta[o] + pv : theta[o] + half_g2 * grad_logpost[o] + pv;
    }
  }
}

struct OuterArgs {
  int S, N, D, first, random_walk;
  double gamma;
  Prior pr;
  uint64_t seed;
  const uint32_t *iteration;
  double *theta, *logpost, *grad_logpost, *loglik, *logw;                // cur (in/out)
  const double *prev_logpost, *prev_grad_logpost, *prev_logw, *p_prev;  // prev (k > 1)
  int32_t *anc_out;
  double *ess_out;
  int32_t *resampled_out;
  double *estimate;  // [S][2][D] realised E[theta], E[theta^2] of this iteration, or NULL
  double *recycle;   // [S][1 + 4D] running sums (l, l E[theta], l E[theta^2]) and the
                     // recycled estimate, or NULL
  double *scratch;  // [S][N][2D+2] gather double buffer
  int32_t *status;  // device status word, or NULL
};

// K3: one workgroup of kOuterThreads threads per series (N <= 4096); sample i belongs to thread
// i mod kOuterThreads in round i / kOuterThreads, so a wave's loads and stores of the population
// are consecutive samples.
constexpr int kOuterThreads = 1024;
constexpr int kOuterMaxN = 4096;
constexpr int kOuterPer = kOuterMaxN / kOuterThreads;

__global__ __launch_bounds__(kOuterThreads) void reweight_resample_kernel(OuterArgs A) {
  constexpr int WAVES = kOuterThreads / 64;
  constexpr double kNegInf = -__builtin_huge_val();
  __shared__ double sh_P[kOuterMaxN];
  __shared__ double sh_red[2][2 * WAVES + 2];
  __shared__ double sh_scan[2][WAVES];
  __shared__ double sh_est[WAVES][2 * kMaxD];
  const int s = blockIdx.x, tid = threadIdx.x;
  const int N = A.N, D = A.D;
  const uint32_t k = *A.iteration;
  const double g2 = A.gamma * A.gamma;

  double lw[kOuterPer];
  double mloc = kNegInf;
  for (int r = 0; r < kOuterPer; ++r) {
    lw[r] = kNegInf;
    const int i = r * kOuterThreads + tid;
    if (i >= N) continue;
    const size_t it = (size_t)s * N + i;
    double *th = A.theta + it * D;
    double *g = A.grad_logpost + it * D;
    // log pi = log p(theta) + loglik and grad log pi = grad log p + grad loglik
    // (eqs. log_posterior, first_gradientlogposterior)
    double lp = 0.0;
    for (int p = 0; p < D; ++p) {
      if (A.pr.kind[p] == 1) {  // uniform: flat inside the closed interval, zero outside
        lp += (th[p] >= A.pr.mu[p] && th[p] <= A.pr.sd[p]) ? -A.pr.lnorm[p] : kNegInf;
        continue;
      }
      const double z = (th[p] - A.pr.mu[p]) / A.pr.sd[p];
      lp += -kHalfLog2Pi - A.pr.lnorm[p] - 0.5 * z * z;
      g[p] += -z / A.pr.sd[p];
    }
    const double ll = A.loglik[it];
    const double lpost = lp == kNegInf ? kNegInf : lp + ll;  // outside the support: zero
    A.logpost[it] = lpost;
    double v;
    if (A.first) {
      v = ll;  // eq. init_weights with q_1 = prior
    } else if (A.prev_logw[it] == kNegInf || lpost == kNegInf) {
      v = kNegInf;
    } else {
      // eq. l_weights: w_k = w_{k-1} pi_k / pi_{k-1} L / q, with L / q = N(-p_k; 0, G) /
      // N(p_{k-1}; 0, G) and p_k = p_{k-1} + F(theta_{k-1}) + F(theta_k) (Sec. III-E)
      double inc = lpost - A.prev_logpost[it];
      if (!A.random_walk) {
        double npk = 0.0, npp = 0.0;
        for (int p = 0; p < D; ++p) {
          const double pp = A.p_prev[it * D + p];
          const double pk = pp + 0.5 * g2 * (A.prev_grad_logpost[it * D + p] + g[p]);
          npk += pk * pk;
          npp += pp * pp;
        }
        inc += -(npk - npp) / (2.0 * g2);
      }
      v = A.prev_logw[it] + inc;
    }
    if (!(v == v)) v = kNegInf;
    lw[r] = v;
    A.logw[it] = v;
    mloc = fmax(mloc, v);
  }
  const double mx = block_max<WAVES>(mloc, sh_red[0]);
  double e[kOuterPer], S = 0.0, Q = 0.0;  // e = 0 past N (lw = -inf there)
  for (int r = 0; r < kOuterPer; ++r) {
    e[r] = (mx == kNegInf) ? 0.0 : exp(lw[r] - mx);
    S += e[r];
    Q += e[r] * e[r];
  }
  block_sum2<WAVES>(S, Q, sh_red[1]);
  const double ess = (mx == kNegInf) ? 0.0 : S * S / Q;  // eqs. normalise_smc2, ess_smc2
  const bool res = mx != kNegInf && ess < 0.5 * (double)N;
  if (A.estimate || A.recycle) {
    // realised estimates of E[theta] and E[theta^2] under the normalised weights (eq.
    // realised_estimates) and the recycling weight l_k = ESS (eq. recycling_I), accumulated as
    // l_k-weighted sums for the recycled estimate (eq. opt_recycling_constant)
    const int lane = tid & 63, wid = tid >> 6;
    for (int p = 0; p < D; ++p) {
      double m1 = 0.0, m2 = 0.0;
      for (int r = 0; r < kOuterPer; ++r) {
        const int i = r * kOuterThreads + tid;
        if (i >= N || !(e[r] > 0.0)) continue;  // zero-weight samples take no part
        const double v = A.theta[((size_t)s * N + i) * D + p];
        m1 += e[r] * v;
        m2 += e[r] * v * v;
      }
      m1 = wave_sum(m1);
      m2 = wave_sum(m2);
      if (lane == 0) {
        sh_est[wid][p] = m1;
        sh_est[wid][D + p] = m2;
      }
    }
    __syncthreads();
    // recycle row of the series: [0] sum of l_k, [1, 2D] the l_k-weighted sums, [2D + 1, 4D]
    // the recycled estimate sum_k c_k f_k with c_k = l_k / sum_j l_j; every value is read
    // before any is written (the barrier below), so thread 0's update of the sum of l_k does not
    // race with the others' reads of it
    double *rc = A.recycle ? A.recycle + (size_t)s * (4 * D + 1) : nullptr;
    double l_new = 0.0, sum_new = 0.0;
    if (tid < 2 * D) {
      double v = 0.0;
      for (int w = 0; w < WAVES; ++w) v += sh_est[w][tid];
      v = (mx == kNegInf) ? __builtin_nan("") : v / S;
      if (A.estimate) A.estimate[(size_t)s * 2 * D + tid] = v;
      if (rc) {
        l_new = rc[0] + ess;
        sum_new = ess > 0.0 ? rc[1 + tid] + ess * v : rc[1 + tid];
      }
    }
    __syncthreads();
    if (rc && tid < 2 * D) {
      rc[1 + tid] = sum_new;
      rc[1 + 2 * D + tid] = l_new > 0.0 ? sum_new / l_new : __builtin_nan("");
      if (tid == 0) rc[0] = l_new;
    }
  }
  if (tid == 0) {
    if (A.ess_out) A.ess_out[s] = ess;
    if (A.resampled_out) A.resampled_out[s] = res ? 1 : 0;
    if (mx == kNegInf && A.status) *A.status = 5;  // every weight of this series is zero
  }
  if (!res) {
    if (A.anc_out)
      for (int r = 0; r < kOuterPer; ++r) {
        const int i = r * kOuterThreads + tid;
        if (i < N) A.anc_out[(size_t)s * N + i] = i;
      }
    return;
  }
  // systematic resampling: inclusive FP64 prefix in sample order (one workgroup scan per
  // round, carried across rounds; the scans alternate two buffers), lower bound of
  // (i + nu)/N * total
  double carry = 0.0;
  for (int r = 0; r * kOuterThreads < N; ++r) {
    double tot;
    const double exc = block_exclusive_scan<WAVES>(e[r], sh_scan[r & 1], tot);
    const int i = r * kOuterThreads + tid;
    if (i < N) sh_P[i] = carry + (exc + e[r]);
    carry += tot;
  }
  const double nu = uniform_m(kNoSlot, (uint32_t)s, stream_word(k, kStreamOuter), 0u, A.seed);
  __syncthreads();
  const double total = sh_P[N - 1];
  const double lse = mx + log(S);
  const int W = 2 * D + 2;
  for (int r = 0; r < kOuterPer; ++r) {
    const int i = r * kOuterThreads + tid;
    if (i >= N) continue;
    const int a = min(lower_bound_lds(sh_P, N, ((double)i + nu) / (double)N * total), N - 1);
    if (A.anc_out) A.anc_out[(size_t)s * N + i] = a;
    const size_t src = (size_t)s * N + a, dst = (size_t)s * N + i;
    double *sc = A.scratch + dst * W;
    for (int p = 0; p < D; ++p) {
      sc[p] = A.theta[src * D + p];
      sc[D + p] = A.grad_logpost[src * D + p];
    }
    sc[2 * D] = A.logpost[src];
    sc[2 * D + 1] = A.loglik[src];
  }
  __syncthreads();  // every read of the old population precedes the in-place writes
  for (int r = 0; r < kOuterPer; ++r) {
    const int i = r * kOuterThreads + tid;
    if (i >= N) continue;
    const size_t dst = (size_t)s * N + i;
    const double *sc = A.scratch + dst * W;
    for (int p = 0; p < D; ++p) {
      A.theta[dst * D + p] = sc[p];
      A.grad_logpost[dst * D + p] = sc[D + p];
    }
    A.logpost[dst] = sc[2 * D];
    A.loglik[dst] = sc[2 * D + 1];
    A.logw[dst] = lse - log((double)N);  // equal, sum-preserving weights after resampling
  }
}

__global__ void advance_iteration_kernel(uint32_t *iteration) {
  if (threadIdx.x == 0 && blockIdx.x == 0) *iteration = *iteration + 1u;
}

__global__ void reset_queue_kernel(uint32_t *queue) {
  if (threadIdx.x == 0 && blockIdx.x == 0) *queue = 0u;
}

// Counter-contract probe.
__global__ void philox_probe_kernel(int R, const uint32_t *ctr, const uint32_t *n, uint64_t seed,
                                    uint32_t *out, double *normals, double *uniforms,
                                    float *normals32, float *uniforms32) {
  const int r = blockIdx.x * blockDim.x + threadIdx.x;
  if (r >= R) return;
  const uint32_t c0 = ctr[4 * r], c1 = ctr[4 * r + 1], c2 = ctr[4 * r + 2], c3 = ctr[4 * r + 3];
  if (out) {
    const uint4 w = philox4x32_10(c0, c1, c2, c3, seed);
    out[4 * r] = w.x;
    out[4 * r + 1] = w.y;
    out[4 * r + 2] = w.z;
    out[4 * r + 3] = w.w;
  }
  if (normals) normals[r] = normal_n<double>(c0, c2, c3, n[r], seed);
  if (normals32) normals32[r] = normal_n<float>(c0, c2, c3, n[r], seed);
  if (uniforms) uniforms[r] = uniform_m(c0, c2, c3, n[r], seed);
  if (uniforms32) uniforms32[r] = (float)uniform_m(c0, c2, c3, n[r], seed);
}

}  // namespace smc2
