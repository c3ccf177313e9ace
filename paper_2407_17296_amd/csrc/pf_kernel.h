// K1: the fused CRN particle filter, forward + adjoint, one workgroup per (series, sample) item.
//
// Forward (paper Sec. II with the bootstrap proposal, eqs. prior_proposal and
// priorproposalweight): for t = 1..T each particle slot j propagates with its own
// reparameterised noise (eq. reparam_epsilon), is weighted by g, and the workgroup forms
// s_t = log sum_j exp(lW_{t-1}^j + lambda_t^j) (a max and an FP64 sum), accumulates
// loglik += s_t (eq. likelihood_pf_ step by step), normalises (eq. normalisedweights) and tests
// ESS = 1 / sum W^2 (eq. ess).  Below the threshold (never at t = T) it resamples (App. B):
// FP64 inclusive prefix of the weights in LDS, lower-bound search of u_i * P_{M-1} with
// systematic u_i = (i + nu)/M or multinomial u_i = nu_i, gather of x, equal weights.  The
// int32 ancestors are stored, and (x, log W) checkpoints are stored every c steps.
//
// Adjoint (the transpose of App. A's tangent recursion, eqs. dloglik..dxk, with App. B's rules
// that resampled weights have zero derivative and a resampled particle inherits its parent's):
// segments are processed last to first; each is recomputed forward from its checkpoint with the
// stored ancestors and stored s_t into a segment buffer, then swept backward.  Because the
// normalised weights sum to one, the adjoint of the per-step log-weights between two resampling
// steps is the normalised weight vector at the later one (or at T); it is carried per particle
// as `wb`.  At a resampling step the state adjoint is scatter-added from offspring to parents.
// The parameter adjoint is accumulated in FP64 per thread and reduced once per item.
#pragma once

#include "device_common.h"
#include "models.h"

namespace smc2 {

struct PFArgs {
  const double *theta;  // [S][N][NP]
  const double *y;      // [S][T_max][DX]
  double *loglik;       // [S][N]
  double *grad;         // [S][N][NP] or NULL
  const int32_t *T_len; // [S]
  const int32_t *order; // [S*N] item order (longest series first)
  int32_t S, N, M, T_max, ckpt, nseg_max;
  int32_t ld;           // particle stride of the per-slot scratch (>= particles per workgroup)
  int32_t t_ld;         // step stride of the per-slot scratch (>= every T_len)
  int32_t resampler, want_grad, n_items, persistent;
  double ess_thresh;    // ess_frac * M
  uint64_t seed;
  const uint32_t *iteration;
  uint32_t *queue;
  int32_t *anc;         // [slots][t_ld][ld]
  uint8_t *flags;       // [slots][t_ld]
  double *sbuf;         // [slots][t_ld]
  void *ckpt_buf;       // [slots][nseg_max][DX+1][ld]  (R)
  void *seg_buf;        // [slots][ckpt][2*DX+1][ld]    (R)
};

// Noise of slot j for step t (normals (t-1)*DX + q of the STEP stream).  For DX == 1 one
// Philox block serves four consecutive steps and is cached in `cache`.
template <typename R, int DX>
__device__ __forceinline__ void step_noise(uint32_t j, uint32_t fid, uint32_t c3, uint64_t seed,
                                           int t, bool refresh, R (&cache)[4], R *e) {
  if constexpr (DX == 1) {
    if (refresh) normals4<R>(j, (uint32_t)(t - 1) >> 2, fid, c3, seed, cache);
    const int w = (t - 1) & 3;
    e[0] = w == 0 ? cache[0] : w == 1 ? cache[1] : w == 2 ? cache[2] : cache[3];
  } else {
    static_assert(DX % 4 == 0, "state dimension must be 1 or a multiple of 4");
#pragma unroll
    for (int b = 0; b < DX / 4; ++b)
      normals4<R>(j, (uint32_t)((t - 1) * (DX / 4) + b), fid, c3, seed, e + 4 * b);
  }
}

template <typename R, int DX>
__device__ __forceinline__ void init_noise(uint32_t j, uint32_t fid, uint32_t c3, uint64_t seed,
                                           R *e) {
  if constexpr (DX == 1) {
    e[0] = normal_n<R>(j, fid, c3, 0u, seed);
  } else {
#pragma unroll
    for (int b = 0; b < DX / 4; ++b) normals4<R>(j, (uint32_t)b, fid, c3, seed, e + 4 * b);
  }
}

template <typename R, class Model, int WAVES, int PPL>
__global__ __launch_bounds__(WAVES * 64) void pf_fwd_adj_kernel(PFArgs A) {
  constexpr int NT = WAVES * 64, MP = NT * PPL, DX = Model::DX, NP = Model::NP;
  constexpr double kNegInf = -__builtin_huge_val();
  __shared__ double sh_P[MP];  // forward: weight prefix; backward: adjoint scatter (as R)
  __shared__ R sh_X[MP];       // gather staging
  __shared__ double sh_red[2][2 * WAVES + 2];
  __shared__ double sh_vec[WAVES * NP];
  __shared__ int sh_item;

  const int tid = threadIdx.x;
  const int j0 = tid * PPL;
  const int M = A.M;
  const uint32_t k = *A.iteration;
  const uint64_t seed = A.seed;
  const uint32_t c3i = stream_word(k, kStreamInit), c3s = stream_word(k, kStreamStep),
                 c3r = stream_word(k, kStreamResample);
  const double lWeq = -log((double)M);
  const R lWeqR = (R)lWeq;
  const int c = A.ckpt;
  const bool systematic = A.resampler == 0;

  for (int round = 0;; ++round) {
    int idx;
    __syncthreads();  // the previous item is done with every shared array
    if (A.persistent) {
      if (tid == 0) sh_item = (int)atomicAdd(A.queue, 1u);
      __syncthreads();
      idx = sh_item;
    } else {
      if (round > 0) break;
      idx = blockIdx.x;
    }
    if (idx >= A.n_items) break;
    const int item = A.order[idx];
    const int slot = A.persistent ? (int)blockIdx.x : item;
    const int s = item / A.N;
    const uint32_t fid = (uint32_t)item;  // = s * N + i
    const int T = A.T_len[s];
    double *gout = A.want_grad ? A.grad + (size_t)item * NP : nullptr;

    double thv[NP];
    bool finite = true;
#pragma unroll
    for (int p = 0; p < NP; ++p) {
      thv[p] = A.theta[(size_t)item * NP + p];
      finite = finite && isfinite(thv[p]);
    }
    if (!finite) {  // a non-finite parameter explains nothing: -inf, gradient 0
      if (tid == 0) A.loglik[item] = kNegInf;
      if (gout && tid < NP) gout[tid] = 0.0;
      continue;
    }
    Model mdl;
    mdl.setup(thv);
    const double *ys = A.y + (size_t)s * A.T_max * DX;
    const size_t LD = (size_t)A.ld;
    R *ck = (R *)A.ckpt_buf + (size_t)slot * A.nseg_max * (DX + 1) * LD;
    int32_t *anc = A.anc + (size_t)slot * A.t_ld * LD;
    uint8_t *flg = A.flags + (size_t)slot * A.t_ld;
    double *sb = A.sbuf + (size_t)slot * A.t_ld;

    // ---- forward ------------------------------------------------------------------------------
    R x[PPL][DX], lW[PPL];
    R cache[PPL][4];
#pragma unroll
    for (int p = 0; p < PPL; ++p) {
      R e[DX];
      init_noise<R, DX>((uint32_t)(j0 + p), fid, c3i, seed, e);
      mdl.init(e, x[p]);
      lW[p] = lWeqR;
    }
    double ll = 0.0;
    bool dead = false;
    for (int t = 1; t <= T; ++t) {
      if ((t - 1) % c == 0) {
        R *cks = ck + (size_t)((t - 1) / c) * (DX + 1) * LD;
#pragma unroll
        for (int p = 0; p < PPL; ++p) {
#pragma unroll
          for (int q = 0; q < DX; ++q) cks[q * LD + j0 + p] = x[p][q];
          cks[DX * LD + j0 + p] = lW[p];
        }
      }
      mdl.per_step(t);
      R yv[DX];
#pragma unroll
      for (int q = 0; q < DX; ++q) yv[q] = (R)ys[(size_t)(t - 1) * DX + q];
      R lw[PPL];
      double mloc = kNegInf;
#pragma unroll
      for (int p = 0; p < PPL; ++p) {
        R e[DX];
        step_noise<R, DX>((uint32_t)(j0 + p), fid, c3s, seed, t, ((t - 1) & 3) == 0, cache[p], e);
        mdl.step(x[p], e);
        R v = lW[p] + mdl.logg(yv, x[p]);
        if (!(v == v) || j0 + p >= M) v = (R)kNegInf;
        lw[p] = v;
        mloc = fmax(mloc, (double)v);
      }
      const double mx = block_max<WAVES>(mloc, sh_red[0]);
      if (mx == kNegInf) {  // no particle explains y_t
        dead = true;
        break;
      }
      double ep[PPL], S = 0.0, Q = 0.0;
#pragma unroll
      for (int p = 0; p < PPL; ++p) {
        ep[p] = (double)exp(lw[p] - (R)mx);
        S += ep[p];
        Q += ep[p] * ep[p];
      }
      block_sum2<WAVES>(S, Q, sh_red[1]);
      const double st = mx + log(S);
      ll += st;
      if (tid == 0) sb[t - 1] = st;
#pragma unroll
      for (int p = 0; p < PPL; ++p) lW[p] = lw[p] - (R)st;
      const bool res = (t < T) && (S * S / Q < A.ess_thresh);
      if (tid == 0) flg[t - 1] = res ? 1 : 0;
      if (res) {
        double acc = 0.0, pre[PPL];
#pragma unroll
        for (int p = 0; p < PPL; ++p) {
          acc += ep[p];
          pre[p] = acc;
        }
        double tot;
        const double off = block_exclusive_scan<WAVES>(acc, sh_red[0], tot);
#pragma unroll
        for (int p = 0; p < PPL; ++p) sh_P[j0 + p] = off + pre[p];
        const double nu = systematic ? uniform_m(kNoSlot, fid, c3r, (uint32_t)(t - 1), seed) : 0.0;
        __syncthreads();
        const double total = sh_P[M - 1];
        int a[PPL];
#pragma unroll
        for (int p = 0; p < PPL; ++p) {
          const int i = j0 + p;
          a[p] = 0;
          if (i < M) {
            const double u = systematic ? ((double)i + nu) / (double)M
                                        : uniform_m((uint32_t)i, fid, c3r, (uint32_t)(t - 1), seed);
            a[p] = min(lower_bound_lds(sh_P, M, u * total), M - 1);
          }
        }
#pragma unroll
        for (int q = 0; q < DX; ++q) {
#pragma unroll
          for (int p = 0; p < PPL; ++p) sh_X[j0 + p] = x[p][q];
          __syncthreads();
#pragma unroll
          for (int p = 0; p < PPL; ++p) x[p][q] = sh_X[a[p]];
          __syncthreads();
        }
#pragma unroll
        for (int p = 0; p < PPL; ++p) {
          anc[(size_t)(t - 1) * LD + j0 + p] = a[p];
          lW[p] = lWeqR;
        }
      }
    }
    if (dead) {
      if (tid == 0) A.loglik[item] = kNegInf;
      if (gout && tid < NP) gout[tid] = 0.0;
      continue;
    }
    if (tid == 0) A.loglik[item] = ll;
    if (!A.want_grad) continue;

    // ---- adjoint --------------------------------------------------------------------------
    __syncthreads();  // s_t and flags written by thread 0 become visible to the workgroup
    R xb[PPL][DX], wb[PPL];
    double tb[NP];
#pragma unroll
    for (int p = 0; p < PPL; ++p) {
      wb[p] = (R)0;
#pragma unroll
      for (int q = 0; q < DX; ++q) xb[p][q] = (R)0;
    }
#pragma unroll
    for (int p = 0; p < NP; ++p) tb[p] = 0.0;
    constexpr int ROW = 2 * DX + 1;
    R *sg = (R *)A.seg_buf + (size_t)slot * c * ROW * LD;
    R *sh_S = (R *)sh_P;
    const int nseg = (T + c - 1) / c;
    for (int seg = nseg - 1; seg >= 0; --seg) {
      const int t0 = seg * c, t1 = min(T, t0 + c);
      const R *cks = ck + (size_t)seg * (DX + 1) * LD;
#pragma unroll
      for (int p = 0; p < PPL; ++p) {
#pragma unroll
        for (int q = 0; q < DX; ++q) x[p][q] = cks[q * LD + j0 + p];
        lW[p] = cks[DX * LD + j0 + p];
      }
      // recompute the segment with the stored ancestors and log normalisers
      for (int t = t0 + 1; t <= t1; ++t) {
        mdl.per_step(t);
        R yv[DX];
#pragma unroll
        for (int q = 0; q < DX; ++q) yv[q] = (R)ys[(size_t)(t - 1) * DX + q];
        R *row = sg + (size_t)(t - t0 - 1) * ROW * LD;
        const R st = (R)sb[t - 1];
#pragma unroll
        for (int p = 0; p < PPL; ++p) {
          R e[DX];
          step_noise<R, DX>((uint32_t)(j0 + p), fid, c3s, seed, t,
                            t == t0 + 1 || ((t - 1) & 3) == 0, cache[p], e);
#pragma unroll
          for (int q = 0; q < DX; ++q) {
            row[q * LD + j0 + p] = x[p][q];
            row[(DX + q) * LD + j0 + p] = e[q];
          }
          mdl.step(x[p], e);
          R v = lW[p] + mdl.logg(yv, x[p]);
          if (!(v == v) || j0 + p >= M) v = (R)kNegInf;
          lW[p] = v - st;
        }
        const bool res = flg[t - 1] != 0;
        if (t == T || res) {
#pragma unroll
          for (int p = 0; p < PPL; ++p) row[2 * DX * LD + j0 + p] = exp(lW[p]);
        }
        if (res) {
          int a[PPL];
#pragma unroll
          for (int p = 0; p < PPL; ++p) a[p] = anc[(size_t)(t - 1) * LD + j0 + p];
#pragma unroll
          for (int q = 0; q < DX; ++q) {
#pragma unroll
            for (int p = 0; p < PPL; ++p) sh_X[j0 + p] = x[p][q];
            __syncthreads();
#pragma unroll
            for (int p = 0; p < PPL; ++p) x[p][q] = sh_X[a[p]];
            __syncthreads();
          }
#pragma unroll
          for (int p = 0; p < PPL; ++p) lW[p] = lWeqR;
        }
      }
      // reverse sweep over the segment
      for (int t = t1; t > t0; --t) {
        mdl.per_step(t);
        R yv[DX];
#pragma unroll
        for (int q = 0; q < DX; ++q) yv[q] = (R)ys[(size_t)(t - 1) * DX + q];
        const R *row = sg + (size_t)(t - t0 - 1) * ROW * LD;
        const bool res = t < T && flg[t - 1] != 0;
        if (t == T) {
#pragma unroll
          for (int p = 0; p < PPL; ++p) wb[p] = row[2 * DX * LD + j0 + p];
        } else if (res) {
          // offspring -> parent: xb_pre[m] = sum over offspring i with a_i = m of xb_post[i]
          int a[PPL];
#pragma unroll
          for (int p = 0; p < PPL; ++p) a[p] = anc[(size_t)(t - 1) * LD + j0 + p];
#pragma unroll
          for (int q = 0; q < DX; ++q) {
#pragma unroll
            for (int p = 0; p < PPL; ++p) sh_S[j0 + p] = (R)0;
            __syncthreads();
#pragma unroll
            for (int p = 0; p < PPL; ++p)
              if (j0 + p < M && xb[p][q] != (R)0) atomicAdd(&sh_S[a[p]], xb[p][q]);
            __syncthreads();
#pragma unroll
            for (int p = 0; p < PPL; ++p) xb[p][q] = sh_S[j0 + p];
            __syncthreads();
          }
#pragma unroll
          for (int p = 0; p < PPL; ++p) wb[p] = row[2 * DX * LD + j0 + p];
        }
#pragma unroll
        for (int p = 0; p < PPL; ++p) {
          bool active = wb[p] != (R)0;
#pragma unroll
          for (int q = 0; q < DX; ++q) active = active || xb[p][q] != (R)0;
          if (!active) continue;
          R xp[DX], e[DX], xc[DX];
#pragma unroll
          for (int q = 0; q < DX; ++q) {
            xp[q] = row[q * LD + j0 + p];
            e[q] = row[(DX + q) * LD + j0 + p];
            xc[q] = xp[q];
          }
          mdl.step(xc, e);
          if (wb[p] != (R)0) mdl.logg_adj(yv, xc, wb[p], xb[p], tb);
          mdl.step_adj(xp, e, xb[p], tb);
        }
      }
    }
#pragma unroll
    for (int p = 0; p < PPL; ++p) {
      R e[DX];
      init_noise<R, DX>((uint32_t)(j0 + p), fid, c3i, seed, e);
      mdl.init_adj(e, xb[p], tb);
    }
    block_sum_vec<WAVES, NP>(tb, sh_vec);
    if (tid < NP) {
      double v = tb[0];
#pragma unroll
      for (int p = 1; p < NP; ++p)
        if (tid == p) v = tb[p];
      gout[tid] = v;
    }
  }
}

}  // namespace smc2
