// K1: the fused CRN particle filter, forward + adjoint, one workgroup per (series, sample) item.
//
// Forward (paper Sec. II with the bootstrap proposal, eqs. prior_proposal and
// priorproposalweight): for t = 1..T each particle slot j propagates with its own
// reparameterised noise (eq. reparam_epsilon), is weighted by g, and the workgroup forms
// s_t = log sum_j exp(lW_{t-1}^j + lambda_t^j) (a max and an FP64 sum), accumulates
// loglik += s_t (eq. likelihood_pf_ step by step), normalises (eq. normalisedweights) and tests
// ESS = 1 / sum W^2 (eq. ess).  Below the threshold (never at t = T) it resamples (App. B):
// an FP64 inclusive prefix P of the weights, and offspring i takes the first parent m with
// P_m >= u_i P_{M-1} (the paper's index kappa_i = sum_j [nu_i > c_j]), with systematic
// u_i = (i + nu)/M or multinomial u_i = nu_i; equal weights after.  The int32 ancestors are
// stored, and (x, log W) checkpoints are stored every c steps.
//
// Systematic resampling needs no search: the targets increase with i, so each parent m counts
// C_m = #{i : target_i <= P_m} (an estimate corrected by evaluating the same FP64 comparisons),
// parent m owns offspring [C_{m-1}, C_m), and a max-scan over "first offspring" markers hands
// every offspring its parent.  Multinomial targets are unsorted and use a binary search.
//
// Adjoint (the transpose of App. A's tangent recursion, eqs. dloglik..dxk, with App. B's rules
// that resampled weights have zero derivative and a resampled particle inherits its parent's):
// segments are processed last to first; each is recomputed forward from its checkpoint with the
// stored ancestors and stored s_t into a segment buffer, then swept backward.  Because the
// normalised weights sum to one, the adjoint of the per-step log-weights between two resampling
// steps is the normalised weight vector at the later one (or at T); it is carried per particle
// as `wb`.  At a resampling step the state adjoint is scatter-added from offspring to parents.
// The parameter adjoint is accumulated in FP64 per thread and reduced once per item.
//
// The series y, the per-step log normalisers s_t and the resampling flags of the current item
// live in LDS (dynamic shared memory sized by the longest series).
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
  int32_t lds_T;        // steps held in LDS (>= every T_len)
  int32_t resampler, want_grad, n_items, persistent;
  double ess_thresh;    // ess_frac * M
  uint64_t seed;
  const uint32_t *iteration;
  uint32_t *queue;
  int32_t *anc;         // [slots][t_ld][ld]
  uint8_t *flags;       // [slots][t_ld]
  void *ckpt_buf;       // [slots][nseg_max][DX+1][ld]  (R)
  void *seg_buf;        // [slots][ckpt][2*DX+1][ld]    (R)
};

// Dynamic shared memory of one item: y as R [lds_T * DX], then s_t as double [lds_T], then the
// flags as bytes [lds_T].
template <typename R, int DX>
__host__ __device__ constexpr size_t pf_dyn_lds_bytes(int lds_T) {
  return ((size_t)lds_T * DX * sizeof(R) + 7) / 8 * 8 + (size_t)lds_T * 8 + (size_t)lds_T;
}

// The filter's noise (counter contract): element g = j*DX + q of step t (t = 0: the initial
// draw) is normal g % 4 of the Philox block with counter (g / 4, t, filter id, stream word), so
// one block serves four consecutive elements of one step.  e[p][q] receives the noise of slot
// j0 + p, component q.
template <typename R>
__device__ __forceinline__ R pick4(const R (&z)[4], int i) {
  return i == 0 ? z[0] : i == 1 ? z[1] : i == 2 ? z[2] : z[3];
}

template <typename R, int DX, int PPL>
__device__ __forceinline__ void filter_noise(int j0, uint32_t fid, uint32_t c3, uint32_t t,
                                             uint64_t seed, R (&e)[PPL][DX]) {
  if constexpr (DX == 1 && PPL % 4 == 0) {
#pragma unroll
    for (int b = 0; b < PPL / 4; ++b) {
      R z[4];
      normals4<R>((uint32_t)(j0 >> 2) + b, t, fid, c3, seed, z);
#pragma unroll
      for (int r = 0; r < 4; ++r) e[4 * b + r][0] = z[r];
    }
  } else if constexpr (DX % 4 == 0) {
#pragma unroll
    for (int p = 0; p < PPL; ++p)
#pragma unroll
      for (int b = 0; b < DX / 4; ++b) {
        R z[4];
        normals4<R>((uint32_t)((j0 + p) * (DX / 4) + b), t, fid, c3, seed, z);
#pragma unroll
        for (int r = 0; r < 4; ++r) e[p][4 * b + r] = z[r];
      }
  } else {
    static_assert(DX == 1, "state dimension must be 1 or a multiple of 4");
    R z[4];  // fewer than four slots per thread: this thread's slots share one block
    normals4<R>((uint32_t)(j0 >> 2), t, fid, c3, seed, z);
#pragma unroll
    for (int p = 0; p < PPL; ++p) e[p][0] = pick4(z, (j0 & 3) + p);
  }
}

// Multinomial resampling uniforms of step t for offspring slots j0 .. j0 + PPL - 1: word i % 4
// of block (i / 4, t).
template <int PPL>
__device__ __forceinline__ void filter_uniforms(int j0, uint32_t fid, uint32_t c3, uint32_t t,
                                                uint64_t seed, double (&u)[PPL]) {
  if constexpr (PPL % 4 == 0) {
#pragma unroll
    for (int b = 0; b < PPL / 4; ++b) {
      const uint4 w = philox4x32_10((uint32_t)(j0 >> 2) + b, t, fid, c3, seed);
      u[4 * b + 0] = ((double)w.x + 1.0) * 0x1p-32;
      u[4 * b + 1] = ((double)w.y + 1.0) * 0x1p-32;
      u[4 * b + 2] = ((double)w.z + 1.0) * 0x1p-32;
      u[4 * b + 3] = ((double)w.w + 1.0) * 0x1p-32;
    }
  } else {
    const uint4 w = philox4x32_10((uint32_t)(j0 >> 2), t, fid, c3, seed);
#pragma unroll
    for (int p = 0; p < PPL; ++p) {
      const int q = (j0 & 3) + p;
      const uint32_t v = q == 0 ? w.x : q == 1 ? w.y : q == 2 ? w.z : w.w;
      u[p] = ((double)v + 1.0) * 0x1p-32;
    }
  }
}

// Systematic target of offspring i: ((i + nu) / M) * P_{M-1}, in the order of operations the
// resampling rule is stated in.  When M is a power of two (FAST), division by M and
// multiplication by 1/M are the same exact operation.
struct SysTargets {
  double nu, Md, inv_Md, tot, inv_tot;
  int M;
  template <bool FAST>
  __device__ double at(int i) const {
    return FAST ? ((double)i + nu) * inv_Md * tot : ((double)i + nu) / Md * tot;
  }
  // C = #{i in [0, M) : at(i) <= P}: the targets increase with i, so C is the first i whose
  // target exceeds P.  The estimate g from P / tot is checked with the exact comparisons
  // at(g - 1) <= P < at(g), which need no special cases at g = 0 (at(-1) <= 0) or g = M
  // (at(M) > tot > P); a wrong estimate falls back to bisection.
  template <bool FAST>
  __device__ int upto(double P) const {
    if (!(P < tot)) return M;
    const int g = (int)fmin(fmax(floor(P * inv_tot * Md - nu) + 1.0, 0.0), Md);
    if (at<FAST>(g - 1) <= P && at<FAST>(g) > P) return g;
    int lo = 0, hi = M;
    while (lo < hi) {
      const int mid = (lo + hi) >> 1;
      if (at<FAST>(mid) <= P)
        lo = mid + 1;
      else
        hi = mid;
    }
    return lo;
  }
};

// Ancestors of this thread's offspring slots under systematic resampling: each parent marks
// the first offspring it owns, and an exclusive max-scan over the markers hands every
// offspring the last parent that started at or before it.  FAST: M fills the tile (a power of
// two), so no slot is padding.
template <bool FAST, int WAVES, int PPL, typename R>
__device__ __forceinline__ void systematic_ancestors(const SysTargets &tg, double off,
                                                     const R (&ew)[PPL], int j0, int M,
                                                     int *sh_mark, int *sh_imax, int (&a)[PPL],
                                                     int dummy) {
  const double tot = tg.tot;
  int prev = tg.upto<FAST>(fmin(off, tot));
  double part = 0.0;
#pragma unroll
  for (int p = 0; p < PPL; ++p) {
    const int m = j0 + p;
    part += (double)ew[p];
    const double P = (m == M - 1) ? tot : fmin(off + part, tot);
    int cm = tg.upto<FAST>(P);
    if (!FAST && m >= M) cm = prev;
    atomicMax(&sh_mark[cm > prev ? prev : dummy], m);
    prev = max(prev, cm);
  }
  __syncthreads();
  int run = -1;
#pragma unroll
  for (int p = 0; p < PPL; ++p) {
    run = max(run, sh_mark[j0 + p]);
    a[p] = run;
  }
  const int before = block_exclusive_max_scan<WAVES>(run, sh_imax);
#pragma unroll
  for (int p = 0; p < PPL; ++p) a[p] = min(max(a[p], before), M - 1);
}

template <typename R, class Model, int WAVES, int PPL>
__global__ __launch_bounds__(WAVES * 64, (sizeof(R) == 4 && PPL <= 4 && WAVES <= 4) ? 4 : 1) void pf_fwd_adj_kernel(PFArgs A) {
  constexpr int NT = WAVES * 64, MP = NT * PPL, DX = Model::DX, NP = Model::NP;
  constexpr double kNegInf = -__builtin_huge_val();
  __shared__ double sh_P[MP];    // multinomial prefix
  __shared__ R sh_X[2][MP];      // gather / adjoint-scatter staging (ping-pong)
  __shared__ int sh_mark[MP + 1];  // systematic: first-offspring markers (+ a dummy slot)
  __shared__ double sh_red[2][2 * WAVES + 2];
  __shared__ double sh_vec[WAVES * NP];
  __shared__ int sh_imax[WAVES];
  __shared__ int sh_item;
  extern __shared__ double sh_dyn[];
  R *sh_y = (R *)sh_dyn;
  double *sh_s = sh_dyn + ((size_t)A.lds_T * DX * sizeof(R) + 7) / 8;
  uint8_t *sh_f = (uint8_t *)(sh_s + A.lds_T);

  const int tid = threadIdx.x;
  const int j0 = tid * PPL;
  const int M = A.M;
  const double Md = (double)M;
  const uint32_t k = *A.iteration;
  const uint64_t seed = A.seed;
  const uint32_t c3i = stream_word(k, kStreamInit), c3s = stream_word(k, kStreamStep),
                 c3r = stream_word(k, kStreamResample);
  const double lWeq = -log(Md);
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
    {
      const double *ys = A.y + (size_t)s * A.T_max * DX;
      for (int r = tid; r < T * DX; r += NT) sh_y[r] = (R)ys[r];
    }
    const size_t LD = (size_t)A.ld;
    R *ck = (R *)A.ckpt_buf + (size_t)slot * A.nseg_max * (DX + 1) * LD;
    int32_t *anc = A.anc + (size_t)slot * A.t_ld * LD;
    uint8_t *flg = A.flags + (size_t)slot * A.t_ld;
    __syncthreads();  // y staged

    // ---- forward ------------------------------------------------------------------------------
    R x[PPL][DX], lW[PPL];
    {
      R e[PPL][DX];
      filter_noise<R, DX, PPL>(j0, fid, c3i, 0u, seed, e);
#pragma unroll
      for (int p = 0; p < PPL; ++p) {
        mdl.init(e[p], x[p]);
        lW[p] = lWeqR;
      }
    }
    double ll = 0.0;
    bool dead = false;
    int nres = 0;
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
      const R *yv = sh_y + (size_t)(t - 1) * DX;
      double mloc = kNegInf;
      {
        R e[PPL][DX];
        filter_noise<R, DX, PPL>(j0, fid, c3s, (uint32_t)t, seed, e);
#pragma unroll
        for (int p = 0; p < PPL; ++p) {
          mdl.step(x[p], e[p]);
          R v = lW[p] + mdl.logg(yv, x[p]);  // lW now holds the unnormalised lw
          if (!(v == v) || j0 + p >= M) v = (R)kNegInf;
          lW[p] = v;
          mloc = fmax(mloc, (double)v);
        }
      }
      const double mx = block_max<WAVES>(mloc, sh_red[0]);
      if (mx == kNegInf) {  // no particle explains y_t
        dead = true;
        break;
      }
      R ew[PPL];
      double S = 0.0, Q = 0.0;
#pragma unroll
      for (int p = 0; p < PPL; ++p) {
        ew[p] = fexp(lW[p] - (R)mx);
        const double ed = (double)ew[p];
        S += ed;
        Q += ed * ed;
      }
      block_sum2<WAVES>(S, Q, sh_red[1]);
      const double st = mx + log(S);
      ll += st;
#pragma unroll
      for (int p = 0; p < PPL; ++p) lW[p] = lW[p] - (R)st;
      const bool res = (t < T) && (S * S / Q < A.ess_thresh);
      if (tid == 0) {
        sh_s[t - 1] = st;
        sh_f[t - 1] = res ? 1 : 0;
        flg[t - 1] = res ? 1 : 0;
      }
      if (!res) continue;

      // -- resampling (App. B) --
      R *sx = sh_X[nres & 1];
      ++nres;
      double acc = 0.0;
#pragma unroll
      for (int p = 0; p < PPL; ++p) {
        acc += (double)ew[p];
        sx[j0 + p] = x[p][0];
        sh_mark[j0 + p] = -1;
      }
      double tot;
      const double off = block_exclusive_scan<WAVES>(acc, sh_red[0], tot);
      int a[PPL];
      if (systematic) {
        SysTargets tg;
        tg.nu = ((double)philox4x32_10(kNoSlot, (uint32_t)t, fid, c3r, seed).x + 1.0) * 0x1p-32;
        tg.M = M;
        tg.Md = Md;
        tg.inv_Md = 1.0 / Md;
        tg.tot = tot;
        tg.inv_tot = 1.0 / tot;
        if (M == MP)
          systematic_ancestors<true, WAVES, PPL>(tg, off, ew, j0, M, sh_mark, sh_imax, a, MP);
        else
          systematic_ancestors<false, WAVES, PPL>(tg, off, ew, j0, M, sh_mark, sh_imax, a, MP);
      } else {
        double part = 0.0;
#pragma unroll
        for (int p = 0; p < PPL; ++p) {
          part += (double)ew[p];
          sh_P[j0 + p] = off + part;
        }
        double u[PPL];
        filter_uniforms<PPL>(j0, fid, c3r, (uint32_t)t, seed, u);
        __syncthreads();
        const double total = sh_P[M - 1];
#pragma unroll
        for (int p = 0; p < PPL; ++p)
          a[p] = j0 + p < M ? min(lower_bound_lds(sh_P, M, u[p] * total), M - 1) : 0;
      }
      // gather x through LDS (component 0 was staged above)
#pragma unroll
      for (int p = 0; p < PPL; ++p) x[p][0] = sx[a[p]];
#pragma unroll
      for (int q = 1; q < DX; ++q) {
        __syncthreads();
#pragma unroll
        for (int p = 0; p < PPL; ++p) sx[j0 + p] = x[p][q];
        __syncthreads();
#pragma unroll
        for (int p = 0; p < PPL; ++p) x[p][q] = sx[a[p]];
      }
#pragma unroll
      for (int p = 0; p < PPL; ++p) {
        anc[(size_t)(t - 1) * LD + j0 + p] = a[p];
        lW[p] = lWeqR;
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
    int pp = 0;  // ping-pong selector of the gather / scatter staging in sh_X
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
        const bool res = sh_f[t - 1] != 0;
        int a[PPL];
        if (res)
#pragma unroll
          for (int p = 0; p < PPL; ++p) a[p] = anc[(size_t)(t - 1) * LD + j0 + p];
        mdl.per_step(t);
        const R *yv = sh_y + (size_t)(t - 1) * DX;
        R *row = sg + (size_t)(t - t0 - 1) * ROW * LD;
        const R st = (R)sh_s[t - 1];
        R e[PPL][DX];
        filter_noise<R, DX, PPL>(j0, fid, c3s, (uint32_t)t, seed, e);
#pragma unroll
        for (int p = 0; p < PPL; ++p) {
#pragma unroll
          for (int q = 0; q < DX; ++q) {
            row[q * LD + j0 + p] = x[p][q];
            row[(DX + q) * LD + j0 + p] = e[p][q];
          }
          mdl.step(x[p], e[p]);
          R v = lW[p] + mdl.logg(yv, x[p]);
          if (!(v == v) || j0 + p >= M) v = (R)kNegInf;
          lW[p] = v - st;
        }
        if (t == T || res) {
#pragma unroll
          for (int p = 0; p < PPL; ++p) row[2 * DX * LD + j0 + p] = fexp(lW[p]);
        }
        if (res) {
#pragma unroll
          for (int q = 0; q < DX; ++q) {
            R *sx = sh_X[pp];
            pp ^= 1;
#pragma unroll
            for (int p = 0; p < PPL; ++p) sx[j0 + p] = x[p][q];
            __syncthreads();
#pragma unroll
            for (int p = 0; p < PPL; ++p) x[p][q] = sx[a[p]];
          }
#pragma unroll
          for (int p = 0; p < PPL; ++p) lW[p] = lWeqR;
        }
      }
      // reverse sweep over the segment; the rows (state before the step, noise, weight) and
      // ancestors of step t - 1 are loaded while step t is processed
      R nx[PPL][DX], ne[PPL][DX], nw[PPL];
      int na[PPL];
      auto load_step = [&](int t) {
        const R *row = sg + (size_t)(t - t0 - 1) * ROW * LD;
        const bool lres = t < T && sh_f[t - 1] != 0;
#pragma unroll
        for (int p = 0; p < PPL; ++p) {
#pragma unroll
          for (int q = 0; q < DX; ++q) {
            nx[p][q] = row[q * LD + j0 + p];
            ne[p][q] = row[(DX + q) * LD + j0 + p];
          }
          nw[p] = (t == T || lres) ? row[2 * DX * LD + j0 + p] : (R)0;
          na[p] = lres ? anc[(size_t)(t - 1) * LD + j0 + p] : 0;
        }
      };
      load_step(t1);
      for (int t = t1; t > t0; --t) {
        R cx[PPL][DX], ce[PPL][DX], cw[PPL];
        int ca[PPL];
#pragma unroll
        for (int p = 0; p < PPL; ++p) {
#pragma unroll
          for (int q = 0; q < DX; ++q) {
            cx[p][q] = nx[p][q];
            ce[p][q] = ne[p][q];
          }
          cw[p] = nw[p];
          ca[p] = na[p];
        }
        if (t - 1 > t0) load_step(t - 1);
        mdl.per_step(t);
        const R *yv = sh_y + (size_t)(t - 1) * DX;
        const bool res = t < T && sh_f[t - 1] != 0;
        if (t == T) {
#pragma unroll
          for (int p = 0; p < PPL; ++p) wb[p] = cw[p];
        } else if (res) {
          // offspring -> parent: xb_pre[m] = sum over offspring i with a_i = m of xb_post[i];
          // a lane adds each run of its offspring that share a parent once
#pragma unroll
          for (int q = 0; q < DX; ++q) {
            R *ss = sh_X[pp];
            pp ^= 1;
#pragma unroll
            for (int p = 0; p < PPL; ++p) ss[j0 + p] = (R)0;
            __syncthreads();
            int ra = ca[0];
            R rs = (R)0;
#pragma unroll
            for (int p = 0; p < PPL; ++p) {
              const R v = (j0 + p < M) ? xb[p][q] : (R)0;
              if (ca[p] != ra) {
                if (rs != (R)0) atomicAdd(&ss[ra], rs);
                ra = ca[p];
                rs = (R)0;
              }
              rs += v;
            }
            if (rs != (R)0) atomicAdd(&ss[ra], rs);
            __syncthreads();
#pragma unroll
            for (int p = 0; p < PPL; ++p) xb[p][q] = ss[j0 + p];
          }
#pragma unroll
          for (int p = 0; p < PPL; ++p) wb[p] = cw[p];
        }
#pragma unroll
        for (int p = 0; p < PPL; ++p) {
          R xc[DX];
#pragma unroll
          for (int q = 0; q < DX; ++q) xc[q] = cx[p][q];
          mdl.step(xc, ce[p]);
          mdl.logg_adj(yv, xc, wb[p], xb[p], tb);
          mdl.step_adj(cx[p], ce[p], xb[p], tb);
        }
      }
    }
    {
      R e[PPL][DX];
      filter_noise<R, DX, PPL>(j0, fid, c3i, 0u, seed, e);
#pragma unroll
      for (int p = 0; p < PPL; ++p) mdl.init_adj(e[p], xb[p], tb);
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
