// K1: the fused CRN particle filter, forward + adjoint, one workgroup per (series, sample) item.
//
// Forward (paper Sec. II with the bootstrap proposal, eqs. prior_proposal and
// priorproposalweight): for t = 1..T each particle slot j propagates with its own
// reparameterised noise (eq. reparam_epsilon), is weighted by g, and the workgroup forms
// s_t = log sum_j exp(lW_{t-1}^j + lambda_t^j), accumulates loglik += s_t (eq. likelihood_pf_
// step by step), normalises (eq. normalisedweights) and tests ESS = 1 / sum W^2 (eq. ess).
// Below the threshold (never at t = T) it resamples (App. B): an FP64 inclusive prefix P of the
// weights, and offspring i takes the first parent m with P_m >= u_i P_{M-1} (the paper's index
// kappa_i = sum_j [nu_i > c_j]), with systematic u_i = (i + nu)/M or multinomial u_i = nu_i;
// equal weights after.  The int32 ancestors are stored, and (x, log W) checkpoints are stored
// every c steps (log W only where the step before did not resample: after a resampling step
// every log-weight is -log M, which the adjoint takes from the step's flag; with a checkpoint at
// every step, log W only where the adjoint rebuilds the step's normalised weights, at a
// resampled step or at T).
//
// The log-sum-exp takes two workgroup exchanges per step: the maximum, then the FP64 sums of
// exp(lw - max) (the total of a lane prefix scan that resampling reuses) and of their squares.
// No logarithm is taken inside the step loop: the carried log-weights are shifted by the step's
// maximum only, so their exponentials sum to S_t rather than one, and
//   loglik = sum_t max_t + sum over resampled steps and T of log S_t
// (between resampling steps the log S terms of the unnormalised carry cancel).  The logs of S_t
// and the per-step log normalisers max_t + log S_t that the adjoint needs are formed after the
// sweep, in parallel over the workgroup.
//
// Systematic resampling needs no search: the targets increase with i, so each parent m counts
// C_m = #{i : target_i <= P_m} (an estimate corrected by evaluating the same FP64 comparisons),
// parent m owns offspring [C_{m-1}, C_m), and a max-scan over "first offspring" markers hands
// every offspring its parent.  Multinomial targets are unsorted and use a binary search.
//
// Adjoint (the transpose of App. A's tangent recursion, eqs. dloglik..dxk, with App. B's rules
// that resampled weights have zero derivative and a resampled particle inherits its parent's):
// with a checkpoint at every step, one reverse sweep rebuilds each step from the state before it
// and differentiates it; otherwise segments are processed last to first, each recomputed forward
// from its checkpoint with the stored ancestors and stored s_t into a segment buffer, then swept
// backward.  States of a multiple of four components go through the every-step sweep four
// components (one Philox block of the noise) at a time, for every particle of the lane, so that a
// lane keeps only its particles' states and adjoints across steps.  The
// noise of the forward sweep is either stored by it (the reparameterisation draws it in
// advance, eq. reparam_epsilon) and read back, or regenerated from the counter-based stream.
// Because the normalised weights sum to one, the adjoint of the per-step log-weights between two
// resampling steps is the normalised weight vector at the later one (or at T); it is carried
// per particle as `wb`.  At a resampling step the state adjoint is scatter-added from offspring to parents.
// The parameter adjoint is accumulated in FP64 per thread (for states of a multiple of four
// components: per wave, in LDS) and reduced once per item.
//
// The series y of the current item lives in LDS (dynamic shared memory sized by the longest
// series); the per-step sums S_t (later the log normalisers), maxima and resampling flags in the
// slot's global scratch.
#pragma once

#include "device_common.h"
#include "models.h"

namespace smc2 {

struct PFArgs {
  const double *theta;  // [S][N][NP]
  const double *y;      // [S][T_max][DY]
  double *loglik;       // [S][N]
  double *grad;         // [S][N][NP] or NULL
  const int32_t *T_len; // [S]
  const int32_t *order; // [S*N] item order (longest series first)
  int32_t S, N, M, T_max, ckpt, nseg_max;
  int32_t ld;           // particle stride of the per-slot scratch (>= particles per workgroup)
  int32_t t_ld;         // step stride of the per-slot scratch (>= every T_len)
  int32_t lds_T;        // steps of y held in LDS (>= every T_len)
  int32_t resampler, want_grad, n_items, persistent;
  double ess_thresh;    // ess_frac * M
  uint64_t seed;
  const uint32_t *iteration;
  uint32_t *queue;
  int32_t *anc;         // [slots][t_ld][ld]
  uint8_t *flags;       // [slots][t_ld]
  void *ckpt_buf;       // [slots][nseg_max][DX+1][ld]  (R)
  void *seg_buf;        // [slots][ckpt][rows][ld] (R): x before the step (DX rows), the noise
                        // (DX rows, only without `noise`), the normalised weight (1 row)
  void *noise;          // [slots][t_ld+1][DX][ld] (R) forward noise for the adjoint, or NULL
  double *steps_s;      // [slots][t_ld] the per-step log normalisers s_t (a trace), or NULL
  double *step_scr;     // [slots][2][t_ld]: S_t (after the sweep max_t + log S_t), max_t
  double mconst[4];     // model constants (the SIR model's N_pop, I_0, s_e^2, s_y)
};

// Dynamic shared memory of one item: y as R [lds_T * DY], then the model's per-step table as R
// [lds_T * KS].  The per-step scalars (S_t, max_t and the resampling flag), which one thread
// writes once per step and the adjoint reads once per step, live in the slot's global scratch
// instead, so that a long series does not take LDS that would otherwise hold more resident
// workgroups.
template <typename R, int DY, int KS = 0>
__host__ __device__ constexpr size_t pf_dyn_lds_bytes(int lds_T) {
  return ((size_t)lds_T * (DY + KS) * sizeof(R) + 7) / 8 * 8;
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
  if constexpr (DX == 1 && PPL % 4 == 0 && PPL > 4) {  // several blocks, one key schedule
    constexpr int NB = PPL / 4;
    uint32_t c0[NB];
    uint4 w[NB];
#pragma unroll
    for (int b = 0; b < NB; ++b) c0[b] = (uint32_t)(j0 >> 2) + b;
    philox4x32_10_n<NB>(c0, t, fid, c3, seed, w);
#pragma unroll
    for (int b = 0; b < NB; ++b) {
      box_muller(w[b].x, w[b].y, e[4 * b][0], e[4 * b + 1][0]);
      box_muller(w[b].z, w[b].w, e[4 * b + 2][0], e[4 * b + 3][0]);
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
  } else if constexpr (DX == 1 && PPL == 4) {
    R z[4];
    normals4<R>((uint32_t)(j0 >> 2), t, fid, c3, seed, z);
#pragma unroll
    for (int r = 0; r < 4; ++r) e[r][0] = z[r];
  } else if constexpr (DX == 2 && PPL % 2 == 0 && PPL > 2) {
    constexpr int NB = PPL / 2;  // slots j0 + 2b and j0 + 2b + 1 share block b
    uint32_t c0[NB];
    uint4 w[NB];
#pragma unroll
    for (int b = 0; b < NB; ++b) c0[b] = (uint32_t)(j0 >> 1) + b;
    philox4x32_10_n<NB>(c0, t, fid, c3, seed, w);
#pragma unroll
    for (int b = 0; b < NB; ++b) {
      box_muller(w[b].x, w[b].y, e[2 * b][0], e[2 * b][1]);
      box_muller(w[b].z, w[b].w, e[2 * b + 1][0], e[2 * b + 1][1]);
    }
  } else if constexpr (DX == 2 && PPL == 2) {
    R z[4];
    normals4<R>((uint32_t)(j0 >> 1), t, fid, c3, seed, z);
    e[0][0] = z[0];
    e[0][1] = z[1];
    e[1][0] = z[2];
    e[1][1] = z[3];
  } else if constexpr (DX == 2) {
    static_assert(PPL == 1, "two-component states take one or an even number of slots per lane");
    R z[4];
    normals4<R>((uint32_t)(j0 >> 1), t, fid, c3, seed, z);
    e[0][0] = pick4(z, 2 * (j0 & 1));
    e[0][1] = pick4(z, 2 * (j0 & 1) + 1);
  } else {
    static_assert(DX == 1, "state dimension must be 1, 2 or a multiple of 4");
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
  double nu, Md, inv_Md, tot, inv_tot, scale;  // scale = M / tot
  int M;
  template <bool FAST>
  __device__ double at(int i) const {
    return FAST ? ((double)i + nu) * inv_Md * tot : ((double)i + nu) / Md * tot;
  }
  // C = #{i in [0, M) : at(i) <= P}: the targets increase with i, so C is the first i whose
  // target exceeds P.  Near a tie the estimate g from P / tot is checked with the exact
  // comparisons at(g - 1) <= P < at(g), which need no special cases at g = 0 (at(-1) <= 0) or
  // g = M (at(M) > tot > P); a wrong estimate falls back to bisection.
  // The estimate z = P M / tot - nu carries a few ulp; unless it lies within kTieMargin of an
  // integer, floor(z) + 1 is the count and the comparisons are skipped.
  static constexpr double kTieMargin = 1e-9;
  template <bool FAST>
  __device__ int upto(double P) const {
    if (!(P < tot)) return M;
    const double z = P * inv_tot * Md - nu, fz = floor(z), fr = z - fz;
    const int g = (int)fmin(fmax(fz + 1.0, 0.0), Md);
    if (fr > kTieMargin && fr < 1.0 - kTieMargin) return g;
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
  // The estimate alone: floor(z) + 1 clamped to [0, M], and whether z lies within kTieMargin of
  // an integer (then upto must decide).  P = tot needs no case of its own: z is then M - nu to
  // within a few ulp, so the estimate is M unless nu lies within the margin of 0 or 1, where the
  // tie check hands it to upto.  (z >= -1 as P >= 0, and z <= M(1 + 2^-51), so the conversion
  // is exact.)
  __device__ int estimate(double P, bool &near) const {
    const double z = fma(P, scale, -nu), fz = floor(z), fr = z - fz;
    near = near || !(fr > kTieMargin && fr < 1.0 - kTieMargin);
    return min(max((int)fz + 1, 0), M);
  }
};

// Ancestors of this thread's offspring slots under systematic resampling.  The weight prefix of
// slot j0 + p is base + part_p (the exclusive prefix of the lane plus its running sum).  Each
// parent marks the first offspring it owns, and an exclusive max-scan over the markers hands
// every offspring the last parent that started at or before it; a reader
// clears its own markers after use.  FAST: M fills the tile (a power of two), so no slot is
// padding.  `dummy` is a per-lane marker slot for parents that own nothing.
template <bool FAST, int WAVES, int PPL, typename R>
__device__ __forceinline__ void systematic_ancestors(const SysTargets &tg, double base,
                                                     const R (&ew)[PPL], int j0, int M,
                                                     int *sh_mark, int *sh_imax, int (&a)[PPL],
                                                     int dummy) {
  const double tot = tg.tot;
  int prev = tg.upto<FAST>(fmin(base, tot));
  // the lane's counts from the estimate; if any of them lies near a tie, all are redone exactly
  int cm[PPL];
  bool near = false;
  double part = 0.0;
#pragma unroll
  for (int p = 0; p < PPL; ++p) {
    part += (double)ew[p];
    cm[p] = tg.estimate(fmin(base + part, tot), near);
  }
  // the last particle's prefix is the total: it owns the targets up to M (only the lane that
  // holds it takes the branch)
  const int lastp = M - 1 - j0;
  if (lastp >= 0 && lastp < PPL) {
#pragma unroll
    for (int p = 0; p < PPL; ++p)
      if (p == lastp) cm[p] = M;
  }
  if (near) {
    part = 0.0;
#pragma unroll
    for (int p = 0; p < PPL; ++p) {
      part += (double)ew[p];
      const double P = (j0 + p == M - 1) ? tot : fmin(base + part, tot);
      cm[p] = tg.upto<FAST>(P);
    }
  }
#pragma unroll
  for (int p = 0; p < PPL; ++p) {
    const int m = j0 + p;
    if (!FAST && m >= M) cm[p] = prev;
    atomicMax(&sh_mark[cm[p] > prev ? prev : dummy], m);
    prev = max(prev, cm[p]);
  }
  __syncthreads();
  int run = -1;
#pragma unroll
  for (int p = 0; p < PPL; ++p) {
    run = max(run, sh_mark[j0 + p]);
    sh_mark[j0 + p] = -1;
    a[p] = run;
  }
  const int before = block_exclusive_max_scan<WAVES>(run, sh_imax);
#pragma unroll
  for (int p = 0; p < PPL; ++p) a[p] = min(max(a[p], before), M - 1);
}

// An element of a region that starts at a uniform base, addressed by a 32-bit byte offset (the
// region is below 4 GiB): the base stays in scalar registers, and an access needs one 32-bit
// offset register instead of a 64-bit address per row.
template <typename T>
__device__ __forceinline__ T &at_off(T *base, uint32_t byte_off) {
  return *reinterpret_cast<T *>(reinterpret_cast<char *>(base) + byte_off);
}

// EVERY: a checkpoint at every step (the reverse sweep rebuilds each step from the state before
// it); otherwise checkpoints every A.ckpt steps and segments recomputed forward.  The two are
// separate instantiations so that neither carries the other's registers.
template <typename R, class Model, int WAVES, int PPL, bool EVERY>
__global__ __launch_bounds__(WAVES * 64,
                             (sizeof(R) == 4 && Model::DX == 1 && PPL <= 4 && WAVES <= 4) ? 4
                             : (sizeof(R) == 4 && Model::DX == 1 && PPL == 8)            ? 2
                                                                                         : 1)
void pf_fwd_adj_kernel(PFArgs A) {
  constexpr int NT = WAVES * 64, MP = NT * PPL, DX = Model::DX, DY = Model::DY, NP = Model::NP;
  constexpr double kNegInf = -__builtin_huge_val();
  // the reverse sweep loads step t - 1 while step t is processed; a multi-dimensional state
  // loads each step where it is used instead (its registers are the limit there)
  constexpr bool kPrefetch = DX == 1;
  // Wide states (a multiple of four components) stream four components (one Philox block of the
  // noise) of every particle of the lane at a time through each step, so that a lane holds only
  // its particles' states and adjoints across steps, and sum the parameter adjoint per wave into
  // LDS instead of keeping NP FP64 accumulators per lane.
  constexpr bool kWide = DX % 4 == 0;
  // With a checkpoint at every step (states of one or two components), row t of the checkpoints
  // holds the state after step t, before its resampling (row 0: x_0): the reverse sweep then has
  // the states on both sides of each step, the one before gathered from row t - 1 through the
  // stored ancestors, and recovers the step's noise from them instead of drawing it again.
  constexpr bool kPost = EVERY && !kWide;
  // the multinomial prefix (MP doubles) or the systematic first-offspring markers with a dummy
  // per lane (MP + 64 ints): a launch uses one resampler, so the two share their LDS
  __shared__ double sh_pm[MP];
  double *const sh_P = sh_pm;
  int *const sh_mark = reinterpret_cast<int *>(sh_pm);
  __shared__ R sh_X[2][MP];          // gather / adjoint-scatter staging (ping-pong)
  // with a checkpoint at every step, the carried log-weights into the step wait here until the
  // step decides whether the adjoint will need them (each lane reads back only its own slots)
  __shared__ __align__(16) R sh_lw[kWide ? 1 : MP];
  __shared__ double sh_ex[2][3 * WAVES];  // per-wave max and (sum, sum of squares), ping-pong
  __shared__ double sh_vec[WAVES * NP];
  __shared__ double sh_tb[kWide ? WAVES * NP : 1];  // per-wave parameter adjoint (wide states)
  // wide states with a checkpoint at every step: each lane's running sums of the blocks'
  // parameter adjoints (four per block) wait in LDS between the steps, as [block][lane][4],
  // where they fit in 64 KiB
  constexpr bool kTaLds = kWide && EVERY && DX * NT * sizeof(R) <= 65536;
  __shared__ __align__(16) R sh_ta[kTaLds ? DX * NT : 4];
  __shared__ __align__(16) R sh_model[Model::kShared > 0 ? Model::kShared : 1];
  __shared__ int sh_imax[WAVES];
  __shared__ int sh_item;
  extern __shared__ double sh_dyn[];
  R *sh_y = (R *)sh_dyn;

  const int tid = threadIdx.x;
  const int lane = tid & 63, wid = tid >> 6;
  const int M = A.M;
  const double Md = (double)M;
  const uint32_t k = *A.iteration;
  const uint64_t seed = A.seed;
  const uint32_t c3i = stream_word(k, kStreamInit), c3s = stream_word(k, kStreamStep),
                 c3r = stream_word(k, kStreamResample);
  const double lWeq = -log(Md);
  const R lWeqR = (R)lWeq;
  const int c = EVERY ? 1 : A.ckpt;
  const bool systematic = A.resampler == 0;
  const size_t LD = (size_t)A.ld;

  for (int round = 0;; ++round) {
    // the lane's first slot, from a thread index made opaque once per item: what is formed from
    // it (noise counters and their first Philox products, addresses) is formed within the item,
    // not held across items; the mask and the multiple keep its range and alignment known
    int to = tid;
    asm volatile("" : "+v"(to));
    const int j0 = (to & (NT - 1)) * PPL;
    int idx;
    __syncthreads();  // the previous item is done with every shared array
    if (A.persistent) {
      if (tid == 0) sh_item = (int)atomicAdd(A.queue, 1u);
      __syncthreads();
      idx = __builtin_amdgcn_readfirstlane(sh_item);  // uniform: item-derived values stay scalar
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
    mdl.bind_shared(sh_model);
    mdl.setup(thv, A.mconst);
    {
      const double *ys = A.y + (size_t)s * A.T_max * DY;
      for (int r = tid; r < T * DY; r += NT) sh_y[r] = (R)ys[r];
    }
    if constexpr (Model::kPerStep > 0) {  // the model's values of each step, once per filter
      R *sh_st = sh_y + (size_t)A.lds_T * DY;
      for (int r = tid; r < T; r += NT)
        Model::step_values(r + 1, sh_st + (size_t)r * Model::kPerStep);
      mdl.bind_steps(sh_st);
    }
#pragma unroll
    for (int p = 0; p < PPL; ++p) sh_mark[j0 + p] = -1;
    R *ck = (R *)A.ckpt_buf + (size_t)slot * A.nseg_max * (DX + 1) * LD;
    int32_t *anc = A.anc + (size_t)slot * A.t_ld * LD;
    uint8_t *flg = A.flags + (size_t)slot * A.t_ld;
    // per-step scalars of the item: S_t (max_t + log S_t once the sweep is done) and max_t
    double *g_s = A.step_scr + (size_t)slot * 2 * A.t_ld;
    double *g_mx = g_s + A.t_ld;
    R *nz = A.noise ? (R *)A.noise + (size_t)slot * (A.t_ld + 1) * DX * LD : nullptr;
    __syncthreads();  // y staged, markers cleared

    auto store_noise = [&](int t, const R (&e)[PPL][DX]) {
#pragma unroll
      for (int q = 0; q < DX; ++q) store_comp<PPL>(nz + ((size_t)t * DX + q) * LD + j0, e, q);
    };
    auto load_noise = [&](int t, R (&e)[PPL][DX]) {
#pragma unroll
      for (int q = 0; q < DX; ++q) load_comp<PPL>(nz + ((size_t)t * DX + q) * LD + j0, e, q);
    };

    // ---- forward ------------------------------------------------------------------------------
    R x[PPL][DX], lW[PPL];
#pragma unroll
    for (int p = 0; p < PPL; ++p) lW[p] = lWeqR;
    if constexpr (kWide) {  // block by block, as the steps
#pragma unroll
      for (int b = 0; b < DX / 4; ++b)
#pragma unroll
        for (int p = 0; p < PPL; ++p) {
          R e4[4], x4[4];
          normals4<R>((uint32_t)((j0 + p) * (DX / 4) + b), 0u, fid, c3i, seed, e4);
#pragma unroll
          for (int i = 0; i < 4; ++i)
            if (nz) nz[(size_t)(4 * b + i) * LD + j0 + p] = e4[i];
          mdl.init_block(b, e4, x4);
#pragma unroll
          for (int i = 0; i < 4; ++i) x[p][4 * b + i] = x4[i];
        }
    } else {
      R e[PPL][DX];
      filter_noise<R, DX, PPL>(j0, fid, c3i, 0u, seed, e);
      if (nz) store_noise(0, e);
#pragma unroll
      for (int p = 0; p < PPL; ++p) mdl.init(e[p], x[p]);
    }
    if constexpr (kPost) {
#pragma unroll
      for (int q = 0; q < DX; ++q) store_comp<PPL>(ck + q * LD + j0, x, q);
    }
    bool dead = false;
    int nres = 0;
    int ck_left = 0, ck_idx = 0;
    // the carried log-weights are all -log M at the start and right after a resampling step:
    // a checkpoint then stores the state only, and the adjoint takes the constant (not for wide
    // states, whose checkpoints are mostly state and whose registers are scarce)
    bool lw_uniform = !kWide;
    // With a checkpoint at every step the adjoint needs the carry into step t only where it
    // rebuilds the normalised weights, at a resampled step or at T: the carry waits in LDS and
    // reaches HBM only there (and only if it is not the uniform -log M).
    constexpr bool lazy_lw = EVERY && !kWide;
    // the systematic resampling words of 64 consecutive steps, one per lane (drawn by the
    // vector unit once per 64 steps instead of by the scalar unit at every resampling step)
    uint32_t nu_word = 0;
    int nu_base = -1;
    for (int t = 1; t <= T; ++t) {
      const bool lwu_in = lw_uniform;
      if (ck_left == 0) {
        R *cks = ck + (size_t)ck_idx * (DX + 1) * LD;
        if constexpr (!kPost) {
#pragma unroll
          for (int q = 0; q < DX; ++q) store_comp<PPL>(cks + q * LD + j0, x, q);
        }
        if (!lw_uniform && !(EVERY && kWide)) {
          if (lazy_lw) {
#pragma unroll
            for (int p = 0; p < PPL; ++p) sh_lw[j0 + p] = lW[p];
          } else {
            store_run<PPL>(cks + DX * LD + j0, lW);
          }
        }
        ck_left = c;
        ++ck_idx;
      }
      --ck_left;
      mdl.per_step(t);
      const R *yv = sh_y + (size_t)(t - 1) * DY;
      R mloc = (R)kNegInf;  // a maximum is exact in R; it widens to FP64 unchanged
      if constexpr (kWide) {
        // four components (one Philox block of the noise) of every particle of the lane at a
        // time: the lane's particles are adjacent, so a block's loads and stores serve them all
        R s2[PPL];
#pragma unroll
        for (int p = 0; p < PPL; ++p) s2[p] = (R)0;
        // with and without the noise stores as two loops: a store under a per-block branch would
        // split the blocks, and the steps would then wait below all of them with every noise
        auto blocks = [&](auto keep) {
          // the blocks' counters are recomputed at every step from an opaque copy of j0 rather
          // than kept live across the loop (with their first Philox products)
          int jb = j0;
          asm volatile("" : "+v"(jb));
          // the row pitch in bytes, opaque so that the rows' offsets are formed where used
          uint32_t pitch = (uint32_t)(LD * sizeof(R));
          asm volatile("" : "+s"(pitch));
          const uint32_t lo = (uint32_t)jb * (uint32_t)sizeof(R);
#pragma unroll
          for (int b = 0; b < DX / 4; ++b) {
#pragma unroll
            for (int p = 0; p < PPL; ++p) {
              R e4[4], x4[4];
              const uint32_t cb = (uint32_t)((jb + p) * (DX / 4) + b);
              normals4<R>(cb, (uint32_t)t, fid, c3s, seed, e4);
#pragma unroll
              for (int i = 0; i < 4; ++i) {
                if constexpr (decltype(keep)::value)
                  at_off(nz, ((uint32_t)t * DX + 4 * b + i) * pitch + lo +
                                 (uint32_t)(p * sizeof(R))) = e4[i];
                x4[i] = x[p][4 * b + i];
              }
              mdl.step_block(b, x4, e4);
              mdl.resid_block(b, yv, x4, s2[p]);
#pragma unroll
              for (int i = 0; i < 4; ++i) x[p][4 * b + i] = x4[i];
              if constexpr (sizeof(R) == 8) __builtin_amdgcn_sched_barrier(0);
            }
          }
        };
        if (nz)
          blocks(std::true_type{});
        else
          blocks(std::false_type{});
#pragma unroll
        for (int p = 0; p < PPL; ++p) {
          R v = lW[p] + mdl.logg_of(s2[p]);  // lW now holds the unnormalised lw
          if (!(v == v) || j0 + p >= M) v = (R)kNegInf;
          lW[p] = v;
          mloc = fmax(mloc, v);
        }
      } else {
        R e[PPL][DX];
        filter_noise<R, DX, PPL>(j0, fid, c3s, (uint32_t)t, seed, e);
        if (nz) store_noise(t, e);
#pragma unroll
        for (int p = 0; p < PPL; ++p) {
          R v = lW[p] + mdl.advance(x[p], e[p], yv);  // lW now holds the unnormalised lw
          if (!(v == v) || j0 + p >= M) v = (R)kNegInf;
          lW[p] = v;
          mloc = fmax(mloc, v);
        }
        if constexpr (kPost) {
          R *ckt = ck + (size_t)t * (DX + 1) * LD;
#pragma unroll
          for (int q = 0; q < DX; ++q) store_comp<PPL>(ckt + q * LD + j0, x, q);
        }
      }
      // log-sum-exp, exchange 1: the maximum (a single wave holds it already)
      double *ex = sh_ex[t & 1];
      double mx;
      if constexpr (WAVES == 1) {
        mx = (double)wave_max(mloc);
      } else {
        {
          const double mw = (double)wave_max(mloc);
          if (lane == 0) ex[wid] = mw;
        }
        __syncthreads();
        mx = ex[0];
#pragma unroll
        for (int w = 1; w < WAVES; ++w) mx = fmax(mx, ex[w]);
      }
      if (mx == kNegInf) {  // no particle explains y_t
        dead = true;
        break;
      }
      // exchange 2: FP64 sums of exp(lw - max) (as a lane prefix scan) and of their squares (a
      // lane's few squares summed in R: they only decide whether to resample)
      const R mxR = (R)mx;
      R ew[PPL];
      double acc = 0.0;
      R qacc = (R)0;
#pragma unroll
      for (int p = 0; p < PPL; ++p) {
        ew[p] = fexp(lW[p] - mxR);
        acc += (double)ew[p];
        qacc += ew[p] * ew[p];
        lW[p] = lW[p] - mxR;  // the carry: log-weights shifted by the maximum
      }
      const double inc = wave_inclusive_sum(acc);
      double S = 0.0, Q = 0.0, off = 0.0;
      if constexpr (WAVES == 1) {
        S = readlane_f64(inc, 63);
        Q = (double)wave_sum(qacc);
      } else {
        {
          const double sw = readlane_f64(inc, 63), qw = (double)wave_sum(qacc);
          if (lane == 0) {
            ex[WAVES + 2 * wid] = sw;
            ex[WAVES + 2 * wid + 1] = qw;
          }
        }
        __syncthreads();
        const int widu = wave_id_opaque();
#pragma unroll
        for (int w = 0; w < WAVES; ++w) {
          if (w == widu) off = S;
          S = S + ex[WAVES + 2 * w];
          Q = Q + ex[WAVES + 2 * w + 1];
        }
      }
      const bool res = (t < T) && (S * S < A.ess_thresh * Q);  // ESS = S^2 / Q (eq. ess)
      lw_uniform = res && !kWide;
      if (lazy_lw && !lwu_in && (res || t == T)) {
        R lin[PPL];
#pragma unroll
        for (int p = 0; p < PPL; ++p) lin[p] = sh_lw[j0 + p];
        store_run<PPL>(ck + (size_t)(t - 1) * (DX + 1) * LD + DX * LD + j0, lin);
      }
      if constexpr (EVERY && kWide) {
        // wide states: the adjoint restarts its weight adjoint from the step's normalised
        // weights W = exp(lw - max) / S, stored in the checkpoint's log-weight row where it will
        // (a resampled step or T), instead of rebuilding them from the carried log-weights
        if (res || t == T) {
          R wn[PPL];
#pragma unroll
          for (int p = 0; p < PPL; ++p) wn[p] = (R)((double)ew[p] / S);
          store_run<PPL>(ck + (size_t)(t - 1) * (DX + 1) * LD + DX * LD + j0, wn);
        }
      }
      if (tid == 0) {
        g_s[t - 1] = S;
        g_mx[t - 1] = mx;
        flg[t - 1] = res ? 1 : 0;
      }
      if (!res) continue;

      // -- resampling (App. B) --
      // prefix of the weights: P_j = (wave offset + lane prefix) + lane running sum to j
      R *sx = sh_X[nres & 1];
      ++nres;
      const double base = off + dpp_f64<kDppWaveShr1>(0.0, inc);
      const double tot = S;
#pragma unroll
      for (int p = 0; p < PPL; ++p) sx[j0 + p] = x[p][0];
      int a[PPL];
      if (systematic) {
        SysTargets tg;
        const int tb = (t - 1) & ~63;
        if (tb != nu_base) {
          nu_base = tb;
          nu_word = philox4x32_10(kNoSlot, (uint32_t)(tb + 1 + lane), fid, c3r, seed).x;
        }
        const uint32_t wnu = (uint32_t)__builtin_amdgcn_readlane((int)nu_word, (t - 1) & 63);
        tg.nu = ((double)wnu + 1.0) * 0x1p-32;
        tg.M = M;
        tg.Md = Md;
        tg.inv_Md = 1.0 / Md;
        tg.tot = tot;
        tg.inv_tot = 1.0 / tot;
        tg.scale = tg.inv_tot * Md;
        if (M == MP)
          systematic_ancestors<true, WAVES, PPL>(tg, base, ew, j0, M, sh_mark, sh_imax, a,
                                                 MP + lane);
        else
          systematic_ancestors<false, WAVES, PPL>(tg, base, ew, j0, M, sh_mark, sh_imax, a,
                                                  MP + lane);
      } else {
        double part = 0.0;
#pragma unroll
        for (int p = 0; p < PPL; ++p) {
          part += (double)ew[p];
          sh_P[j0 + p] = base + part;
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
      store_run<PPL>(anc + (size_t)(t - 1) * LD + j0, a);
#pragma unroll
      for (int p = 0; p < PPL; ++p) lW[p] = lWeqR;
    }
    if (dead) {
      if (tid == 0) A.loglik[item] = kNegInf;
      if (gout && tid < NP) gout[tid] = 0.0;
      continue;
    }
    // loglik = sum_t max_t + sum over resampled steps and T of log S_t; the adjoint's per-step
    // log normaliser max_t + log S_t replaces S_t in LDS
    __syncthreads();  // S_t, max_t and the flags written by thread 0 are visible
    if (A.steps_s) {
      // the trace of s_t = log sum_j W_{t-1}^j g_t^j with normalised W_{t-1} (eq.
      // likelihood_pf_ step by step): the carry into step t was normalised at t = 1 and after a
      // resampling step, and otherwise sums to S_{t-1}
      double *so = A.steps_s + (size_t)slot * A.t_ld;
      for (int t = 1 + tid; t <= T; t += NT) {
        double v = g_mx[t - 1] + log(g_s[t - 1]);
        if (t > 1 && !flg[t - 2]) v -= log(g_s[t - 2]);
        so[t - 1] = v;
      }
      __syncthreads();  // every S_t is read before the loop below overwrites it
    }
    {
      double part = 0.0;
      for (int t = 1 + tid; t <= T; t += NT) {
        const double lS = log(g_s[t - 1]), m = g_mx[t - 1];
        part += (t == T || flg[t - 1]) ? m + lS : m;
        g_s[t - 1] = m + lS;
      }
      double v[1] = {part};
      block_sum_vec<WAVES, 1>(v, sh_vec);
      if (tid == 0) A.loglik[item] = v[0];
    }
    if (!A.want_grad) continue;

    // ---- adjoint --------------------------------------------------------------------------
    __syncthreads();  // the per-step log normalisers are visible to the workgroup
    // The per-step scalars the sweeps below read at every step (resampling flag, max_t + log
    // S_t, max_t) come from a window of 64 aligned steps, one step per lane, loaded once per 64
    // steps: the flags as a wave ballot (with the 64 steps before the window, for the flag of
    // the step before), the others read back with readlane.  The step index is uniform, so
    // every read of the window is too.
    int wbase = -(1 << 30);
    uint64_t wfl = 0, wfl_lo = 0;
    R wst = (R)0, wmt = (R)0;
    auto win = [&](int t) {  // makes the scalars of steps t and t - 1 readable (1 <= t <= T)
      const int b = (t - 1) & ~63;
      if (b != wbase) {
        wbase = b;
        const int i = b + lane, il = b - 64 + lane;
        wfl = __ballot(i < T && flg[i] != 0);
        wfl_lo = __ballot(il >= 0 && flg[il] != 0);
        wst = i < T ? (R)g_s[i] : (R)0;
        wmt = i < T ? (R)g_mx[i] : (R)0;
      }
    };
    auto flag_of = [&](int t) -> bool {  // step t in [wbase - 63, wbase + 64]
      const int i = t - 1 - wbase;
      return i >= 0 ? ((wfl >> i) & 1ull) != 0 : ((wfl_lo >> (i + 64)) & 1ull) != 0;
    };
    auto st_of = [&](int t) -> R { return readlane_r(wst, t - 1 - wbase); };
    auto mt_of = [&](int t) -> R { return readlane_r(wmt, t - 1 - wbase); };
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
    if (kWide && lane == 0)
      for (int k = 0; k < NP; ++k) sh_tb[wid * NP + k] = 0.0;
    int pp = 0;  // ping-pong selector of the gather / scatter staging
    // The scatter stages SB components per barrier in one of two sets in turn: a set is one row
    // of sh_X; for wide FP32 states (SB = 2) set 0 is both rows of sh_X and set 1 the
    // resampler's space, which the reverse sweep does not otherwise use, as two rows of R.
    constexpr int SB = (kWide && sizeof(R) == 4) ? 2 : 1;
    auto stage_row = [&](int set, int i) -> R * {
      if constexpr (SB == 1)
        return sh_X[set];
      else
        return set == 0 ? sh_X[i] : reinterpret_cast<R *>(sh_pm) + (size_t)i * MP;
    };
    // offspring -> parent: xb_pre[m] = sum over offspring i with a_i = m of xb_post[i]; a lane
    // adds each run of its offspring that share a parent once.  The staging is zero before use
    // and each reader zeroes what it read; a set is written again only after the barrier of the
    // other set, which every reader of its previous use has passed.
    auto scatter_to_parents = [&](const int (&ca)[PPL]) {
#pragma unroll
      for (int q0 = 0; q0 < DX; q0 += SB) {
        const int set = pp;
        pp ^= 1;
#pragma unroll
        for (int i = 0; i < SB; ++i) {
          R *ss = stage_row(set, i);
          int ra = ca[0];
          R rs = (R)0;
#pragma unroll
          for (int p = 0; p < PPL; ++p) {
            const R v = (j0 + p < M) ? xb[p][q0 + i] : (R)0;
            if (ca[p] != ra) {
              if (rs != (R)0) atomicAdd(&ss[ra], rs);
              ra = ca[p];
              rs = (R)0;
            }
            rs += v;
          }
          if (rs != (R)0) atomicAdd(&ss[ra], rs);
        }
        __syncthreads();
#pragma unroll
        for (int i = 0; i < SB; ++i) {
          R *ss = stage_row(set, i);
#pragma unroll
          for (int p = 0; p < PPL; ++p) {
            xb[p][q0 + i] = ss[j0 + p];
            ss[j0 + p] = (R)0;
          }
        }
      }
    };
    // a step's parameter adjoint (the lane's particles summed in R) joins the FP64 accumulator:
    // per lane, or for wide states per wave in LDS
    auto add_step_adjoint = [&](const R (&tp)[NP]) {
      if constexpr (kWide) {
#pragma unroll
        for (int k = 0; k < NP; ++k) {
          const double sk = wave_sum((double)tp[k]);
          if (lane == 0) sh_tb[wid * NP + k] += sk;
        }
      } else {
#pragma unroll
        for (int k = 0; k < NP; ++k) tb[k] += (double)tp[k];
      }
    };
    // One reverse step t: the weight adjoint restarts at resampled steps and at T, the state
    // adjoint is scatter-added from offspring to parents at resampled steps, then the step's
    // observation and transition are differentiated.  xp / xn: state before / after the step.
    auto reverse_step = [&](int t, const R (&xp)[PPL][DX], const R (&ce)[PPL][DX],
                            const R (&cw)[PPL], const int (&ca)[PPL]) {
      const R *yv = sh_y + (size_t)(t - 1) * DY;
      win(t);
      const bool res = t < T && flag_of(t);
      if (t == T) {
#pragma unroll
        for (int p = 0; p < PPL; ++p) wb[p] = cw[p];
      } else if (res) {
        scatter_to_parents(ca);
#pragma unroll
        for (int p = 0; p < PPL; ++p) wb[p] = cw[p];
      }
      // the lane's particles add their parameter adjoints in R; the step total joins the FP64
      // accumulator
      R tp[NP];
#pragma unroll
      for (int k = 0; k < NP; ++k) tp[k] = (R)0;
#pragma unroll
      for (int p = 0; p < PPL; ++p) {
        R xn[DX];  // the state after the step, rebuilt where the adjoint needs it
#pragma unroll
        for (int q = 0; q < DX; ++q) xn[q] = xp[p][q];
        (void)mdl.advance(xn, ce[p], yv);
        mdl.advance_adj(yv, xp[p], xn, ce[p], wb[p], xb[p], tp);
      }
      add_step_adjoint(tp);
    };
    auto zero_staging = [&]() {
      __syncthreads();  // earlier readers of the staging are done
#pragma unroll
      for (int p = 0; p < PPL; ++p) {
        sh_X[0][j0 + p] = (R)0;
        sh_X[1][j0 + p] = (R)0;
        if constexpr (SB == 2) {
          stage_row(1, 0)[j0 + p] = (R)0;
          stage_row(1, 1)[j0 + p] = (R)0;
        }
      }
      __syncthreads();
      pp = 0;
    };

    if constexpr (EVERY) {
      // Every step's starting state is a checkpoint (its log W where the step's weights are
      // rebuilt): one reverse sweep that reads the state before each step, rebuilds the step and
      // its weight, and differentiates it.
      zero_staging();
      if constexpr (kWide) {
        // four components of every particle of the lane at a time: the block's state before the
        // step (checkpoint) and noise are read, the block's step rebuilt and differentiated.  The
        // weight adjoint restarts from the normalised weights the forward stored.  The lane's
        // parameter adjoint is summed in R over 16 steps at a time (the blocks' parts in LDS where
        // they fit), then over the wave in FP64 into its LDS row.
        R tpl[NP];
#pragma unroll
        for (int k = 0; k < NP; ++k) tpl[k] = (R)0;
        auto ta_row = [&](int b) -> R(&)[4] {
          return *reinterpret_cast<R(*)[4]>(&sh_ta[((size_t)b * NT + tid) * 4]);
        };
        if constexpr (kTaLds) {
#pragma unroll
          for (int b = 0; b < DX / 4; ++b)
#pragma unroll
            for (int i = 0; i < 4; ++i) ta_row(b)[i] = (R)0;
        }
        int since = 0;
        for (int t = T; t >= 1; --t) {
          const R *cks = ck + (size_t)(t - 1) * (DX + 1) * LD;
          win(t);
          const bool res = t < T && flag_of(t);
          if (t == T || res) load_run<PPL>(cks + DX * LD + j0, wb);
          if (res) {
            int ca[PPL];
            load_run<PPL>(anc + (size_t)(t - 1) * LD + j0, ca);
            scatter_to_parents(ca);
          }
          mdl.per_step(t);
          const R *yv = sh_y + (size_t)(t - 1) * DY;
          R s2[PPL], ssx[PPL];
#pragma unroll
          for (int p = 0; p < PPL; ++p) s2[p] = ssx[p] = (R)0;
          auto blocks = [&](auto stored) {  // noise read back or drawn again (as in the forward)
            int jb = j0;
            asm volatile("" : "+v"(jb));
            uint32_t pitch = (uint32_t)(LD * sizeof(R));  // as in the forward
            asm volatile("" : "+s"(pitch));
            const uint32_t lo = (uint32_t)jb * (uint32_t)sizeof(R);
#pragma unroll
            for (int b = 0; b < DX / 4; ++b) {
              R ta[4];
#pragma unroll
              for (int i = 0; i < 4; ++i) ta[i] = kTaLds ? ta_row(b)[i] : tpl[4 * b + i];
#pragma unroll
              for (int p = 0; p < PPL; ++p) {
                R xp4[4], e4[4], xn4[4], xb4[4];
#pragma unroll
                for (int i = 0; i < 4; ++i)
                  xp4[i] = at_off(ck, ((uint32_t)(t - 1) * (DX + 1) + 4 * b + i) * pitch + lo +
                                          (uint32_t)(p * sizeof(R)));
                if constexpr (decltype(stored)::value) {
#pragma unroll
                  for (int i = 0; i < 4; ++i)
                    e4[i] = at_off(nz, ((uint32_t)t * DX + 4 * b + i) * pitch + lo +
                                           (uint32_t)(p * sizeof(R)));
                } else {
                  const uint32_t cb = (uint32_t)((jb + p) * (DX / 4) + b);
                  normals4<R>(cb, (uint32_t)t, fid, c3s, seed, e4);
                }
#pragma unroll
                for (int i = 0; i < 4; ++i) {
                  xn4[i] = xp4[i];
                  xb4[i] = xb[p][4 * b + i];
                }
                mdl.step_block(b, xn4, e4);
                mdl.adj_block(b, yv, xp4, xn4, e4, wb[p], xb4, ta, s2[p], ssx[p]);
#pragma unroll
                for (int i = 0; i < 4; ++i) xb[p][4 * b + i] = xb4[i];
                if constexpr (sizeof(R) == 8) __builtin_amdgcn_sched_barrier(0);
              }
#pragma unroll
              for (int i = 0; i < 4; ++i) {
                if constexpr (kTaLds)
                  ta_row(b)[i] = ta[i];
                else
                  tpl[4 * b + i] = ta[i];
              }
            }
          };
          if (nz)
            blocks(std::true_type{});
          else
            blocks(std::false_type{});
#pragma unroll
          for (int p = 0; p < PPL; ++p) mdl.adj_finish(wb[p], s2[p], ssx[p], tpl);
          if (++since == 16 || t == 1) {
#pragma unroll
            for (int k = 0; k < NP; ++k) {
              R v = tpl[k];
              if constexpr (kTaLds) {
                if (k < DX) {
                  v = ta_row(k / 4)[k % 4];
                  ta_row(k / 4)[k % 4] = (R)0;
                }
              }
              const double sk = wave_sum((double)v);
              if (lane == 0) sh_tb[wid * NP + k] += sk;
              tpl[k] = (R)0;
            }
            since = 0;
          }
        }
      } else {
        // Row t holds the state after step t before its resampling.  Step t is taken from the
        // state after it (xn, row t) and the state before it: the state after step t - 1 (row
        // t - 1), gathered through the ancestors of that step's resampling.  Row t - 2 is loaded
        // while step t is processed (loading the ancestors and the carry one step ahead as well
        // measured no faster on the 1-D LG and growth workloads).
        auto load_row = [&](int r, R (&v)[PPL][DX]) {
          const R *ckr = ck + (size_t)r * (DX + 1) * LD;
#pragma unroll
          for (int q = 0; q < DX; ++q) load_comp<PPL>(ckr + q * LD + j0, v, q);
        };
        R xn[PPL][DX], xq[PPL][DX];  // the states after steps t and t - 1
        int ca[PPL];                 // ancestors of the resampling after step t
#pragma unroll
        for (int p = 0; p < PPL; ++p) ca[p] = 0;
        if (T > 0) {
          load_row(T, xn);
          load_row(T - 1, xq);
        }
        int gsel = 0;  // staging buffer of the next gather of parent states
        // with and without the stored noise as two loops: a load of the noise under a branch in
        // the loop made every step wait for all of its loads (the prefetched row included)
        // before recovering the noise on the other path
        auto sweep = [&](auto stored) {
          for (int t = T; t >= 1; --t) {
            win(t);
            const bool res_t = t < T && flag_of(t);
            const bool res_p = t > 1 && flag_of(t - 1);  // resampled after step t - 1
            const bool need_w = t == T || res_t;
            // the carry into step t, stored where the weights are rebuilt and not uniform
            // (each conditional load is waited for on its own path, before the next row's load
            // is issued: its registers, reused later on the other path, would otherwise make
            // that write wait for every load in flight)
            R cl[PPL];
            if (need_w && t > 1 && !res_p) {
              load_run<PPL>(ck + (size_t)(t - 1) * (DX + 1) * LD + DX * LD + j0, cl);
#pragma unroll
              for (int p = 0; p < PPL; ++p) asm volatile("" : "+v"(cl[p]));
            } else {
#pragma unroll
              for (int p = 0; p < PPL; ++p) cl[p] = lWeqR;
            }
            int pa[PPL];
            if (res_p) {
              load_run<PPL>(anc + (size_t)(t - 2) * LD + j0, pa);
#pragma unroll
              for (int p = 0; p < PPL; ++p) asm volatile("" : "+v"(pa[p]));
            } else {
#pragma unroll
              for (int p = 0; p < PPL; ++p) pa[p] = 0;
            }
            R xq2[PPL][DX];  // the state after step t - 2, for the next step
            if (t >= 2) load_row(t - 2, xq2);
            // the state before step t
            R xp[PPL][DX];
            if (res_p) {
#pragma unroll
              for (int q = 0; q < DX; ++q) {
                // two staging buffers in turn (sh_lw, and the resampler's space, which the reverse
                // sweep does not use): every wave passed the previous gather's barrier after its
                // reads of the other buffer, so the buffer written now has no reader left
                R *gs = gsel ? reinterpret_cast<R *>(sh_pm) : sh_lw;
                gsel ^= 1;
#pragma unroll
                for (int p = 0; p < PPL; ++p) gs[j0 + p] = xq[p][q];
                __syncthreads();
#pragma unroll
                for (int p = 0; p < PPL; ++p) xp[p][q] = gs[pa[p]];
              }
            } else {
#pragma unroll
              for (int p = 0; p < PPL; ++p)
#pragma unroll
                for (int q = 0; q < DX; ++q) xp[p][q] = xq[p][q];
            }
            mdl.per_step(t);
            const R *yv = sh_y + (size_t)(t - 1) * DY;
            // the step's noise: read back where the forward stored it, else recovered
            R ce[PPL][DX];
            if constexpr (decltype(stored)::value) {
#pragma unroll
              for (int q = 0; q < DX; ++q)
                load_comp<PPL>(nz + ((size_t)t * DX + q) * LD + j0, ce, q);
            } else {
#pragma unroll
              for (int p = 0; p < PPL; ++p) mdl.noise_of(xp[p], xn[p], yv, ce[p]);
            }
            // the weight adjoint restarts from the step's normalised weights
            if (need_w) {
              const R st = st_of(t);  // max_t + log S_t
#pragma unroll
              for (int p = 0; p < PPL; ++p) {
                R v = cl[p] + mdl.weight_of(yv, xp[p], xn[p]);
                if (!(v == v) || j0 + p >= M) v = (R)kNegInf;
                wb[p] = fexp(v - st);
              }
            }
            if (res_t) scatter_to_parents(ca);
            R tp[NP];
#pragma unroll
            for (int k = 0; k < NP; ++k) tp[k] = (R)0;
#pragma unroll
            for (int p = 0; p < PPL; ++p)
              mdl.advance_adj(yv, xp[p], xn[p], ce[p], wb[p], xb[p], tp);
            add_step_adjoint(tp);
#pragma unroll
            for (int p = 0; p < PPL; ++p) {
              ca[p] = pa[p];
#pragma unroll
              for (int q = 0; q < DX; ++q) {
                xn[p][q] = xq[p][q];
                xq[p][q] = xq2[p][q];
              }
            }
          }
        };
        if (nz)
          sweep(std::true_type{});
        else
          sweep(std::false_type{});
      }
    } else {
      // segment rows of one step: x before the step (DX rows), the noise when it is not
      // stored (DX rows), the normalised weight at resampled steps and at T (1 row)
      const int ROW = nz ? DX + 1 : 2 * DX + 1;
      const int WROW = ROW - 1;
      R *sg = (R *)A.seg_buf + (size_t)slot * c * (2 * DX + 1) * LD;
      const int nseg = (T + c - 1) / c;
      // with and without the stored noise as two loops (as in the every-step sweep)
      auto seg_sweep = [&](auto stored) {
        for (int seg = nseg - 1; seg >= 0; --seg) {
          const int t0 = seg * c, t1 = min(T, t0 + c);
          const R *cks = ck + (size_t)seg * (DX + 1) * LD;
#pragma unroll
          for (int q = 0; q < DX; ++q) load_comp<PPL>(cks + q * LD + j0, x, q);
          if (t0 > 0) win(t0);
          if (kWide || (t0 > 0 && !flag_of(t0)))
            load_run<PPL>(cks + DX * LD + j0, lW);
          else
#pragma unroll
            for (int p = 0; p < PPL; ++p) lW[p] = lWeqR;
          // the checkpoint is waited for here: state registers still loading on entry to the
          // loop below would make every step of it wait for all of its loads and stores
#pragma unroll
          for (int p = 0; p < PPL; ++p) {
            asm volatile("" : "+v"(lW[p]));
#pragma unroll
            for (int q = 0; q < DX; ++q) asm volatile("" : "+v"(x[p][q]));
          }
          // recompute the segment with the stored ancestors and log normalisers
          R ne[PPL][DX];
          if constexpr (decltype(stored)::value) load_noise(t0 + 1, ne);
          for (int t = t0 + 1; t <= t1; ++t) {
            win(t);
            const bool res = flag_of(t);
            int a[PPL];
            if (res) load_run<PPL>(anc + (size_t)(t - 1) * LD + j0, a);
            R e[PPL][DX];
            if constexpr (decltype(stored)::value) {
#pragma unroll
              for (int p = 0; p < PPL; ++p)
#pragma unroll
                for (int q = 0; q < DX; ++q) e[p][q] = ne[p][q];
              if (t < t1) load_noise(t + 1, ne);
            } else {
              filter_noise<R, DX, PPL>(j0, fid, c3s, (uint32_t)t, seed, e);
            }
            mdl.per_step(t);
            const R *yv = sh_y + (size_t)(t - 1) * DY;
            R *row = sg + (size_t)(t - t0 - 1) * ROW * LD;
            const R st = st_of(t), mt = mt_of(t);  // max_t + log S_t, max_t
            R wv[PPL];
#pragma unroll
            for (int q = 0; q < DX; ++q) {
              store_comp<PPL>(row + q * LD + j0, x, q);
              if constexpr (!decltype(stored)::value)
                store_comp<PPL>(row + (DX + q) * LD + j0, e, q);
            }
#pragma unroll
            for (int p = 0; p < PPL; ++p) {
              R v = lW[p] + mdl.advance(x[p], e[p], yv);
              if (!(v == v) || j0 + p >= M) v = (R)kNegInf;
              wv[p] = v;
              lW[p] = v - mt;
            }
            if (t == T || res) {
#pragma unroll
              for (int p = 0; p < PPL; ++p) wv[p] = fexp(wv[p] - st);
              store_run<PPL>(row + WROW * LD + j0, wv);
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
          zero_staging();
          // reverse sweep over the segment; the rows (state before the step, noise, weight) and
          // ancestors of step t - 1 are loaded while step t is processed
          R nx[PPL][DX], nw[PPL];
          int na[PPL];
          // reads the flag of step t from the window of step t or t + 1
          auto load_step = [&](int t) {
            const R *row = sg + (size_t)(t - t0 - 1) * ROW * LD;
            const bool lres = t < T && flag_of(t);
#pragma unroll
            for (int q = 0; q < DX; ++q) {
              load_comp<PPL>(row + q * LD + j0, nx, q);
              if constexpr (decltype(stored)::value)
                load_comp<PPL>(nz + ((size_t)t * DX + q) * LD + j0, ne, q);
              else
                load_comp<PPL>(row + (DX + q) * LD + j0, ne, q);
            }
            if (t == T || lres)
              load_run<PPL>(row + WROW * LD + j0, nw);
            else
#pragma unroll
              for (int p = 0; p < PPL; ++p) nw[p] = (R)0;
            if (lres)
              load_run<PPL>(anc + (size_t)(t - 1) * LD + j0, na);
            else
#pragma unroll
              for (int p = 0; p < PPL; ++p) na[p] = 0;
          };
          win(t1);
          if (kPrefetch) load_step(t1);
          for (int t = t1; t > t0; --t) {
            R cx[PPL][DX], ce[PPL][DX], cw[PPL];
            int ca[PPL];
            win(t);
            if (!kPrefetch) load_step(t);
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
            if (kPrefetch && t - 1 > t0) load_step(t - 1);
            mdl.per_step(t);
            reverse_step(t, cx, ce, cw, ca);
          }
        }
      };
      if (nz)
        seg_sweep(std::true_type{});
      else
        seg_sweep(std::false_type{});
    }
    {
      R e[PPL][DX];
      if (nz)
        load_noise(0, e);
      else
        filter_noise<R, DX, PPL>(j0, fid, c3i, 0u, seed, e);
#pragma unroll
      for (int p = 0; p < PPL; ++p) mdl.init_adj(e[p], xb[p], tb);
    }
    // thread k receives parameter k's total (the barriers also publish sh_tb)
    double v = block_sum_to_thread<WAVES, NP>(tb, sh_vec);
    if (tid < NP) {
      if constexpr (kWide)  // and adds the per-wave sums of the wide sweep
        for (int w = 0; w < WAVES; ++w) v += sh_tb[w * NP + tid];
      gout[tid] = v;
    }
  }
}

}  // namespace smc2
