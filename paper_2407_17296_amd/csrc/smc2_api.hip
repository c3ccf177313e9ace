// C ABI of the library (declared in include/smc2.h): context and scratch reservation, argument
// validation, launch-shape choice and kernel launches.  No call here synchronises except
// smc2_ctx_device_status, smc2_pf_trace and a reservation.
#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <numeric>
#include <string>
#include <vector>

#include "outer_kernels.h"
#include "registry.h"
#include "smc2.h"

using namespace smc2;

namespace {

thread_local std::string g_err;

smc2_status fail(smc2_status st, const std::string &msg) {
  g_err = msg;
  return st;
}

#define HIP_TRY(expr)                                                                     \
  do {                                                                                    \
    hipError_t e_ = (expr);                                                               \
    if (e_ != hipSuccess)                                                                 \
      return fail(SMC2_E_DEVICE, std::string(#expr) + ": " + hipGetErrorString(e_));      \
  } while (0)

const std::vector<PFKernel> &kernels() {
  static std::vector<PFKernel> v;
  static std::once_flag once;
  std::call_once(once, [] {
    register_lg1d(v);
    register_growth(v);
    register_sv(v);
    register_lgdiag(v);
    register_lg1dopt(v);
    register_sir(v);
  });
  return v;
}

int next_pow2(int v) {
  int p = 64;
  while (p < v) p <<= 1;
  return p;
}

// SIR constants (N_pop, I_0, s_e^2, s_y): the paper's population, initial infections and noise
// variance (Sec. IV-B) and an observation sd of 5
constexpr double kSirDefaults[4] = {763.0, 1.0, 0.5, 5.0};

// The model's constants as the kernels take them (zeros for a model without constants).
void model_constants(const smc2_model *m, double out[4]) {
  for (int i = 0; i < 4; ++i) out[i] = 0.0;
  if (m->kind == SMC2_MODEL_SIR)
    for (int i = 0; i < 4; ++i) out[i] = m->constants ? m->constants[i] : kSirDefaults[i];
}

bool model_ok(const smc2_model *m, std::string &why) {
  if (!m) return why = "model is NULL", false;
  if (!m->prior_mu || !m->prior_sd) return why = "model prior_mu/prior_sd is NULL", false;
  if (m->kind != SMC2_MODEL_SIR && m->d_y != m->d_x) return why = "d_y must equal d_x", false;
  switch (m->kind) {
    case SMC2_MODEL_LG1D:
      if (m->d_x != 1 || m->D != 3) return why = "LG1D needs d_x = 1, D = 3", false;
      break;
    case SMC2_MODEL_LG_DIAG:
      if (m->d_x != 16 || m->D != 18) return why = "LG_DIAG is built for d_x = 16, D = 18", false;
      break;
    case SMC2_MODEL_GROWTH:
      if (m->d_x != 1 || m->D != 2) return why = "GROWTH needs d_x = 1, D = 2", false;
      break;
    case SMC2_MODEL_SV:
      if (m->d_x != 1 || m->D != 3) return why = "SV needs d_x = 1, D = 3", false;
      break;
    case SMC2_MODEL_LG1D_OPT:
      if (m->d_x != 1 || m->D != 3) return why = "LG1D_OPT needs d_x = 1, D = 3", false;
      break;
    case SMC2_MODEL_SIR: {
      if (m->d_x != 2 || m->d_y != 1 || m->D != 2)
        return why = "SIR needs d_x = 2, d_y = 1, D = 2", false;
      double c[4];
      model_constants(m, c);
      for (double v : c)
        if (!std::isfinite(v)) return why = "SIR constants must be finite", false;
      if (!(c[0] > 0) || !(c[1] >= 0) || !(c[1] <= c[0]) || !(c[2] >= 0) || !(c[3] > 0))
        return why = "SIR constants need N_pop > 0, 0 <= I_0 <= N_pop, s_e^2 >= 0, s_y > 0",
               false;
      break;
    }
    default:
      return why = "unknown model kind", false;
  }
  for (int p = 0; p < m->D; ++p) {
    const int kind = m->prior_kind ? m->prior_kind[p] : SMC2_PRIOR_NORMAL;
    if (kind == SMC2_PRIOR_UNIFORM) {
      if (!std::isfinite(m->prior_mu[p]) || !std::isfinite(m->prior_sd[p]) ||
          !(m->prior_sd[p] > m->prior_mu[p]))
        return why = "a uniform prior needs finite bounds with lower < upper", false;
    } else if (kind == SMC2_PRIOR_NORMAL) {
      if (!(m->prior_sd[p] > 0) || !std::isfinite(m->prior_sd[p]) ||
          !std::isfinite(m->prior_mu[p]))
        return why = "prior_sd must be finite and > 0 and prior_mu finite", false;
    } else {
      return why = "unknown prior kind", false;
    }
  }
  return true;
}

Prior make_prior(const smc2_model *m) {
  Prior pr{};
  for (int p = 0; p < m->D; ++p) {
    pr.mu[p] = m->prior_mu[p];
    pr.sd[p] = m->prior_sd[p];
    pr.kind[p] = m->prior_kind ? m->prior_kind[p] : SMC2_PRIOR_NORMAL;
    pr.lnorm[p] = pr.kind[p] == SMC2_PRIOR_UNIFORM ? std::log(pr.sd[p] - pr.mu[p])
                                                   : std::log(pr.sd[p]);
  }
  return pr;
}

// Default launch shape per particle count (largest particles-per-lane that keeps 4+ waves for
// M >= 256; a single wave for the small filters).
int default_tile(int MP, int dx, int precision) {
  // tile indices refer to kTiles; measured on MI355X (fused forward+adjoint, systematic
  // resampling at most steps): one or two waves with 4 to 8 particles per lane for the 1-D
  // models; the 16-dimensional state keeps one or two particles per lane
  if (dx == 2) {  // the SIR model: one particle per lane up to 128, then four
    switch (MP) {
      case 64: return 1;     // {1, 1}
      case 128: return 2;    // {2, 1}
      case 256: return 3;    // {1, 4}
      case 512: return 6;    // {2, 4}
      case 1024: return 10;  // {4, 4}
      case 2048: return 14;  // {8, 4}
    }
    return -1;
  }
  if (dx == 16) {
    switch (MP) {
      case 64: return 1;     // {1, 1}
      case 128: return 2;    // {2, 1}
      case 256: return 4;    // {4, 1}
      case 512: return 7;    // {4, 2}
      case 1024: return 11;  // {8, 2}
      case 2048: return 14;  // {8, 4}: two waves per SIMD with a 256-register budget
    }
    return -1;
  }
  const bool fp64 = precision == SMC2_FP64;
  switch (MP) {
    case 64: return 1;                  // {1, 1}
    case 128: return 2;                 // {2, 1}
    case 256: return 3;                 // {1, 4}
    case 512: return fp64 ? 6 : 5;      // {2, 4} / {1, 8}
    case 1024: return 10;               // {4, 4}
    case 2048: return fp64 ? 14 : 13;   // {8, 4} / {4, 8}
    case 4096: return 16;               // {8, 8}
  }
  return -1;
}

const PFKernel *find_kernel(int model, int precision, int tile) {
  if (tile < 1 || tile >= kNumTiles) return nullptr;
  for (const auto &k : kernels())
    if (k.model == model && k.precision == precision && k.waves == kTiles[tile].waves &&
        k.ppl == kTiles[tile].ppl)
      return &k;
  return nullptr;
}

constexpr size_t kMaxLdsBytes = 160 * 1024;

// Gather scratch of smc2_reweight_resample_noalloc: a file-scope device array that every GPU the
// library runs on holds until the process ends (8 MiB: S * N * (2D + 2) doubles).  Host code
// never passes the array's name to a kernel (on the host it is only a stand-in for the symbol):
// its device address is looked up once per device and kept in g_noalloc_scratch.
constexpr size_t kNoAllocScratchDoubles = (size_t)1 << 20;
static __device__ __align__(256) double scratch[kNoAllocScratchDoubles];
constexpr int kMaxDevices = 64;
void *g_noalloc_scratch[kMaxDevices];
std::once_flag g_noalloc_once[kMaxDevices];
hipError_t g_noalloc_err[kMaxDevices];

struct Layout {
  int MP, c, nseg, slots;
  size_t anc, flags, ckpt, seg, noise, steps, stepscr, outer, total;
};

}  // namespace

struct smc2_ctx {
  int device = 0;
  int num_cus = 256;
  bool reserved = false;
  smc2_model model{};
  std::vector<double> prior_mu, prior_sd, constants;
  std::vector<int32_t> prior_kind;
  smc2_pf_opts opts{};
  int S = 0, N = 0, M = 0, T_max = 0, tile = 0, T_max_hint = 1;
  Layout L{};
  std::vector<int32_t> T_len;
  int32_t *T_len_dev = nullptr, *order_dev = nullptr;
  int32_t *anc = nullptr;
  uint8_t *flags = nullptr;
  void *ckpt = nullptr, *seg = nullptr, *noise = nullptr;
  double *steps_s = nullptr, *step_scr = nullptr;
  double *outer_scratch = nullptr;
  uint32_t *queue = nullptr;
  int32_t *status = nullptr;
  std::vector<void *> allocs;

  void release() {
    int cur = 0;
    (void)hipGetDevice(&cur);
    (void)hipSetDevice(device);
    for (void *p : allocs) (void)hipFree(p);
    allocs.clear();
    (void)hipSetDevice(cur);
    T_len_dev = order_dev = anc = status = nullptr;
    flags = nullptr;
    outer_scratch = steps_s = step_scr = nullptr;
    ckpt = seg = noise = nullptr;
    queue = nullptr;
    reserved = false;
  }
};

namespace {

struct DeviceGuard {
  int prev = -1;
  explicit DeviceGuard(int dev) {
    if (hipGetDevice(&prev) != hipSuccess) prev = -1;
    (void)hipSetDevice(dev);
  }
  ~DeviceGuard() {
    if (prev >= 0) (void)hipSetDevice(prev);
  }
};

smc2_status check_opts(const smc2_pf_opts *o) {
  if (!o) return fail(SMC2_E_INVALID_ARG, "opts is NULL");
  if (o->precision != SMC2_FP64 && o->precision != SMC2_MIXED)
    return fail(SMC2_E_UNSUPPORTED, "unknown precision");
  if (o->resampler != SMC2_SYSTEMATIC && o->resampler != SMC2_MULTINOMIAL)
    return fail(SMC2_E_INVALID_ARG, "unknown resampler");
  if (!(o->ess_frac >= 0.0) || !std::isfinite(o->ess_frac))
    return fail(SMC2_E_INVALID_ARG, "ess_frac must be finite and >= 0");
  if (o->ckpt_interval < 0) return fail(SMC2_E_INVALID_ARG, "ckpt_interval must be >= 0");
  if (o->tile < 0 || o->tile >= kNumTiles) return fail(SMC2_E_INVALID_ARG, "unknown tile");
  if (o->store_noise != 0 && o->store_noise != 1)
    return fail(SMC2_E_INVALID_ARG, "store_noise must be 0 or 1");
  return SMC2_OK;
}

smc2_status compute_layout(const smc2_model *m, const smc2_pf_opts *o, int S, int N, int M,
                           int T_max, int grid_slots, Layout &L) {
  const int max_m = m->d_x == 1 ? 4096 : 2048;
  if (M > max_m) return fail(SMC2_E_UNSUPPORTED, "M above the largest built tile");
  L.MP = next_pow2(M);
  const int Tc = std::max(T_max, 1);
  L.c = o->ckpt_interval > 0 ? o->ckpt_interval : (int)std::ceil(std::sqrt((double)Tc));
  L.c = std::max(1, std::min(L.c, Tc));
  // checkpoint rows: one per segment, plus one (with a checkpoint at every step the rows hold
  // the states after steps 0 .. T)
  L.nseg = (Tc + L.c - 1) / L.c + 1;
  const long items = (long)S * N;
  L.slots = (int)(o->persistent ? std::min<long>(items, grid_slots) : items);
  const size_t rs = o->precision == SMC2_FP64 ? 8 : 4;
  const size_t dx = (size_t)m->d_x;
  auto al = [](size_t b) { return (b + 255) / 256 * 256; };
  L.anc = al((size_t)L.slots * Tc * L.MP * 4);
  L.flags = al((size_t)L.slots * Tc);
  L.ckpt = al((size_t)L.slots * L.nseg * (dx + 1) * L.MP * rs);
  L.seg = o->want_grad ? al((size_t)L.slots * L.c * (2 * dx + 1) * L.MP * rs) : 256;
  L.noise = (o->want_grad && o->store_noise)
                ? al((size_t)L.slots * (Tc + 1) * dx * L.MP * rs) : 256;
  // a filter's checkpoint and stored-noise regions are addressed with 32-bit byte offsets
  const bool noise_stored = o->want_grad && o->store_noise;
  if ((size_t)L.nseg * (dx + 1) * L.MP * rs >= ((size_t)1 << 32) ||
      (noise_stored && (size_t)(Tc + 1) * dx * L.MP * rs >= ((size_t)1 << 32)))
    return fail(SMC2_E_UNSUPPORTED, "one filter's checkpoints or noise exceed 4 GiB");
  L.steps = al((size_t)L.slots * Tc * 8);
  L.stepscr = al((size_t)L.slots * 2 * Tc * 8);
  L.outer = al((size_t)items * (2 * m->D + 2) * 8);
  L.total = L.anc + L.flags + L.ckpt + L.seg + L.noise + L.steps + L.stepscr + L.outer +
            al(items * 4) * 2 + al((size_t)S * 4) + 512;
  return SMC2_OK;
}

int resolve_tile(const smc2_model *m, const smc2_pf_opts *o, int M) {
  const int MP = next_pow2(M);
  if (o->tile > 0) {
    const Tile t = kTiles[o->tile];
    return (t.waves * 64 * t.ppl == MP) ? o->tile : -1;
  }
  return default_tile(MP, m->d_x, o->precision);
}

int grid_slots_for(smc2_ctx *ctx, const smc2_model *m, const smc2_pf_opts *o, int M) {
  const int tile = resolve_tile(m, o, M);
  if (tile < 0) return 1;
  const PFKernel *k = find_kernel(m->kind, o->precision, tile);
  if (!k) return 1;
  const int Tc = std::max(ctx->T_max_hint, 1);
  const int c = o->ckpt_interval > 0 ? o->ckpt_interval : (int)std::ceil(std::sqrt((double)Tc));
  return ctx->num_cus * k->occupancy(Tc, std::min(c, Tc) == 1);
}

}  // namespace

extern "C" {

const char *smc2_version(void) { return "smc2-mi355x 0.3 (gfx950)"; }

const char *smc2_last_error(void) { return g_err.c_str(); }

smc2_status smc2_ctx_create(smc2_ctx **out, int device) {
  if (!out) return fail(SMC2_E_INVALID_ARG, "out is NULL");
  *out = nullptr;
  int n = 0;
  HIP_TRY(hipGetDeviceCount(&n));
  if (device < 0 || device >= n) return fail(SMC2_E_INVALID_ARG, "no such device");
  hipDeviceProp_t prop;
  HIP_TRY(hipGetDeviceProperties(&prop, device));
  smc2_ctx *c = new smc2_ctx();
  c->device = device;
  c->num_cus = prop.multiProcessorCount;
  *out = c;
  return SMC2_OK;
}

void smc2_ctx_destroy(smc2_ctx *ctx) {
  if (!ctx) return;
  ctx->release();
  delete ctx;
}

smc2_status smc2_ctx_scratch_bytes(const smc2_model *model, const smc2_pf_opts *opts, int32_t S,
                                   int32_t N, int32_t M, int32_t T_max, size_t *bytes) {
  std::string why;
  if (!model_ok(model, why)) return fail(SMC2_E_INVALID_ARG, why);
  smc2_status st = check_opts(opts);
  if (st != SMC2_OK) return st;
  if (S < 1 || N < 1 || M < 1 || T_max < 0 || !bytes)
    return fail(SMC2_E_INVALID_ARG, "sizes must be >= 1 (T_max >= 0) and bytes non-NULL");
  Layout L;
  st = compute_layout(model, opts, S, N, M, T_max, 256 * 8, L);
  if (st != SMC2_OK) return st;
  *bytes = L.total;
  return SMC2_OK;
}

smc2_status smc2_ctx_reserve(smc2_ctx *ctx, const smc2_model *model, const smc2_pf_opts *opts,
                             int32_t S, int32_t N, int32_t M, const int32_t *T_len,
                             int32_t T_max, size_t scratch_budget_bytes) {
  if (!ctx) return fail(SMC2_E_INVALID_ARG, "ctx is NULL");
  std::string why;
  if (!model_ok(model, why)) return fail(SMC2_E_INVALID_ARG, why);
  smc2_status st = check_opts(opts);
  if (st != SMC2_OK) return st;
  if (S < 1 || N < 1 || M < 1 || T_max < 0 || !T_len)
    return fail(SMC2_E_INVALID_ARG, "sizes must be >= 1 (T_max >= 0) and T_len non-NULL");
  if (model->D > kMaxD) return fail(SMC2_E_UNSUPPORTED, "D above 32");
  for (int s = 0; s < S; ++s)
    if (T_len[s] < 0 || T_len[s] > T_max)
      return fail(SMC2_E_INVALID_ARG, "T_len[s] must lie in [0, T_max]");
  if (resolve_tile(model, opts, M) < 0)
    return fail(SMC2_E_UNSUPPORTED, "no built launch shape for this M / tile");
  DeviceGuard g(ctx->device);
  {
    const int tile = resolve_tile(model, opts, M);
    const PFKernel *k = find_kernel(model->kind, opts->precision, tile);
    if (!k) return fail(SMC2_E_UNSUPPORTED, "kernel not built for this model / precision / tile");
    if (k->static_lds() + k->dyn_lds(std::max(T_max, 1)) > kMaxLdsBytes)
      return fail(SMC2_E_UNSUPPORTED, "T_max too long to stage the series in LDS");
  }
  ctx->T_max_hint = T_max;
  Layout L;
  st = compute_layout(model, opts, S, N, M, T_max, grid_slots_for(ctx, model, opts, M), L);
  if (st != SMC2_OK) return st;
  if (scratch_budget_bytes && L.total > scratch_budget_bytes)
    return fail(SMC2_E_OUT_OF_MEMORY, "reservation of " + std::to_string(L.total) +
                                          " bytes exceeds the scratch budget");
  ctx->release();
  auto grab = [&](size_t bytes, void **p) -> hipError_t {
    hipError_t e = hipMalloc(p, std::max<size_t>(bytes, 256));
    if (e == hipSuccess) ctx->allocs.push_back(*p);
    return e;
  };
  const long items = (long)S * N;
  void *p = nullptr;
#define GRAB(bytes, dst, type)                                                          \
  do {                                                                                  \
    hipError_t e_ = grab((bytes), &p);                                                  \
    if (e_ != hipSuccess) {                                                             \
      ctx->release();                                                                   \
      return fail(e_ == hipErrorOutOfMemory ? SMC2_E_OUT_OF_MEMORY : SMC2_E_DEVICE,     \
                  std::string("hipMalloc: ") + hipGetErrorString(e_));                  \
    }                                                                                   \
    dst = (type)p;                                                                      \
  } while (0)
  GRAB(L.anc, ctx->anc, int32_t *);
  GRAB(L.flags, ctx->flags, uint8_t *);
  GRAB(L.ckpt, ctx->ckpt, void *);
  GRAB(L.seg, ctx->seg, void *);
  GRAB(L.noise, ctx->noise, void *);
  GRAB(L.steps, ctx->steps_s, double *);
  GRAB(L.stepscr, ctx->step_scr, double *);
  GRAB(L.outer, ctx->outer_scratch, double *);
  GRAB(items * 4, ctx->order_dev, int32_t *);
  GRAB((size_t)S * 4, ctx->T_len_dev, int32_t *);
  GRAB(256, ctx->queue, uint32_t *);
  GRAB(256, ctx->status, int32_t *);
#undef GRAB
  // items ordered by series length, longest first (a stable order by item index among ties)
  std::vector<int32_t> order(items);
  std::iota(order.begin(), order.end(), 0);
  std::stable_sort(order.begin(), order.end(), [&](int32_t a, int32_t b) {
    return T_len[a / N] > T_len[b / N];
  });
  HIP_TRY(hipMemcpy(ctx->order_dev, order.data(), items * 4, hipMemcpyHostToDevice));
  HIP_TRY(hipMemcpy(ctx->T_len_dev, T_len, (size_t)S * 4, hipMemcpyHostToDevice));
  HIP_TRY(hipMemset(ctx->status, 0, 256));
  HIP_TRY(hipMemset(ctx->queue, 0, 256));
  HIP_TRY(hipDeviceSynchronize());
  ctx->model = *model;
  ctx->prior_mu.assign(model->prior_mu, model->prior_mu + model->D);
  ctx->prior_sd.assign(model->prior_sd, model->prior_sd + model->D);
  ctx->model.prior_mu = ctx->prior_mu.data();
  ctx->model.prior_sd = ctx->prior_sd.data();
  ctx->prior_kind.assign(model->D, SMC2_PRIOR_NORMAL);
  if (model->prior_kind)
    ctx->prior_kind.assign(model->prior_kind, model->prior_kind + model->D);
  ctx->model.prior_kind = ctx->prior_kind.data();
  ctx->constants.assign(4, 0.0);
  model_constants(model, ctx->constants.data());
  ctx->model.constants = ctx->constants.data();
  ctx->opts = *opts;
  ctx->S = S;
  ctx->N = N;
  ctx->M = M;
  ctx->T_max = T_max;
  ctx->L = L;
  ctx->T_len.assign(T_len, T_len + S);
  ctx->reserved = true;
  return SMC2_OK;
}

smc2_status smc2_ctx_device_status(smc2_ctx *ctx, void *stream) {
  if (!ctx || !ctx->reserved) return fail(SMC2_E_INVALID_ARG, "context not reserved");
  DeviceGuard g(ctx->device);
  int32_t v = 0;
  HIP_TRY(hipStreamSynchronize((hipStream_t)stream));
  HIP_TRY(hipMemcpy(&v, ctx->status, 4, hipMemcpyDeviceToHost));
  HIP_TRY(hipMemset(ctx->status, 0, 4));
  HIP_TRY(hipDeviceSynchronize());
  return v == 0 ? SMC2_OK : (smc2_status)v;
}

smc2_status smc2_pf_loglik_grad(smc2_ctx *ctx, const smc2_model *model, const smc2_pf_opts *opts,
                                int32_t S, int32_t N, int32_t M, const int32_t *T_len,
                                int32_t T_max, const double *theta, const double *y,
                                uint64_t seed, const uint32_t *iteration, double *loglik,
                                double *grad, void *stream) {
  if (!ctx || !ctx->reserved) return fail(SMC2_E_INVALID_ARG, "context not reserved");
  std::string why;
  if (!model_ok(model, why)) return fail(SMC2_E_INVALID_ARG, why);
  smc2_status st = check_opts(opts);
  if (st != SMC2_OK) return st;
  if (S < 1 || N < 1 || M < 1 || T_max < 0 || !T_len)
    return fail(SMC2_E_INVALID_ARG, "sizes must be >= 1 (T_max >= 0) and T_len non-NULL");
  if (!theta || !iteration || !loglik || (T_max > 0 && !y))
    return fail(SMC2_E_INVALID_ARG, "theta, y, iteration and loglik must be non-NULL");
  if (opts->want_grad && !grad) return fail(SMC2_E_INVALID_ARG, "grad is NULL with want_grad");
  if (model->kind != ctx->model.kind || model->d_x != ctx->model.d_x)
    return fail(SMC2_E_INVALID_ARG, "model differs from the reservation");
  if (opts->precision != ctx->opts.precision || opts->persistent != ctx->opts.persistent ||
      opts->ckpt_interval != ctx->opts.ckpt_interval ||
      (opts->want_grad && opts->store_noise != ctx->opts.store_noise) ||
      (opts->want_grad && !ctx->opts.want_grad))
    return fail(SMC2_E_INVALID_ARG, "precision, persistence, checkpoint interval, noise "
                                    "storage or gradient differ from the reservation");
  if (S != ctx->S || N != ctx->N || M > ctx->M || next_pow2(M) > ctx->L.MP || T_max > ctx->T_max)
    return fail(SMC2_E_INVALID_ARG, "sizes differ from or exceed the reservation");
  for (int s = 0; s < S; ++s) {
    if (T_len[s] != ctx->T_len[s])
      return fail(SMC2_E_INVALID_ARG, "T_len differs from the reservation");
    if (T_len[s] > T_max) return fail(SMC2_E_INVALID_ARG, "T_len[s] exceeds T_max");
  }
  const int tile = resolve_tile(model, opts, M);
  if (tile < 0) return fail(SMC2_E_UNSUPPORTED, "no built launch shape for this M / tile");
  const PFKernel *k = find_kernel(model->kind, opts->precision, tile);
  if (!k) return fail(SMC2_E_UNSUPPORTED, "kernel not built for this model / precision / tile");
  DeviceGuard g(ctx->device);
  hipStream_t hs = (hipStream_t)stream;
  const int items = S * N;
  PFArgs a{};
  a.theta = theta;
  a.y = y;
  a.loglik = loglik;
  a.grad = opts->want_grad ? grad : nullptr;
  a.T_len = ctx->T_len_dev;
  a.order = ctx->order_dev;
  a.S = S;
  a.N = N;
  a.M = M;
  a.T_max = T_max;
  a.ckpt = ctx->L.c;
  a.nseg_max = ctx->L.nseg;
  a.ld = ctx->L.MP;
  a.t_ld = std::max(ctx->T_max, 1);
  a.lds_T = std::max(ctx->T_max, 1);
  a.resampler = opts->resampler;
  a.want_grad = opts->want_grad ? 1 : 0;
  a.n_items = items;
  a.persistent = opts->persistent ? 1 : 0;
  a.ess_thresh = opts->ess_frac * (double)M;
  a.seed = seed;
  a.iteration = iteration;
  a.queue = ctx->queue;
  a.anc = ctx->anc;
  a.flags = ctx->flags;
  a.ckpt_buf = ctx->ckpt;
  a.seg_buf = ctx->seg;
  a.noise = (opts->want_grad && opts->store_noise) ? ctx->noise : nullptr;
  a.steps_s = ctx->steps_s;
  a.step_scr = ctx->step_scr;
  model_constants(model, a.mconst);
  int grid = items;
  if (opts->persistent) {
    grid = std::min(items,
                    std::min(ctx->L.slots, ctx->num_cus * k->occupancy(a.lds_T, a.ckpt == 1)));
    hipLaunchKernelGGL(reset_queue_kernel, dim3(1), dim3(64), 0, hs, ctx->queue);
  }
  k->launch(a, grid, hs);
  HIP_TRY(hipGetLastError());
  return SMC2_OK;
}

smc2_status smc2_langevin_move(smc2_ctx *ctx, const smc2_model *model, int32_t S, int32_t N,
                               double gamma, int32_t random_walk, const double *theta,
                               const double *grad_logpost, uint64_t seed,
                               const uint32_t *iteration, double *theta_new, double *p_prev,
                               void *stream) {
  if (!ctx || !ctx->reserved) return fail(SMC2_E_INVALID_ARG, "context not reserved");
  std::string why;
  if (!model_ok(model, why)) return fail(SMC2_E_INVALID_ARG, why);
  if (S < 1 || N < 1 || !(gamma > 0) || !std::isfinite(gamma))
    return fail(SMC2_E_INVALID_ARG, "sizes must be >= 1 and gamma > 0");
  if (!theta || (!random_walk && !grad_logpost) || !iteration || !theta_new || !p_prev)
    return fail(SMC2_E_INVALID_ARG, "a device pointer is NULL");
  DeviceGuard g(ctx->device);
  const int items = S * N;
  hipLaunchKernelGGL(langevin_move_kernel, dim3((items + 255) / 256), dim3(256), 0,
                     (hipStream_t)stream, items, model->D, gamma, random_walk ? 1 : 0, theta,
                     grad_logpost, seed, iteration, theta_new, p_prev);
  HIP_TRY(hipGetLastError());
  return SMC2_OK;
}

}  // extern "C"

namespace {

// Argument checks shared by smc2_reweight_resample and its no-allocation variant.
smc2_status check_reweight_args(const smc2_model *model, int32_t S, int32_t N, double gamma,
                                int32_t random_walk, const smc2_population *cur,
                                const smc2_population *prev, const double *p_prev,
                                int32_t first_iteration, const uint32_t *iteration) {
  std::string why;
  if (!model_ok(model, why)) return fail(SMC2_E_INVALID_ARG, why);
  if (S < 1 || N < 1 || N > kOuterMaxN || !(gamma > 0) || !std::isfinite(gamma))
    return fail(SMC2_E_INVALID_ARG, "need 1 <= N <= 4096, S >= 1 and gamma > 0");
  if (!cur || !cur->theta || !cur->logpost || !cur->grad_logpost || !cur->loglik || !cur->logw ||
      !iteration)
    return fail(SMC2_E_INVALID_ARG, "cur population or iteration has a NULL pointer");
  if (!first_iteration && (!prev || !prev->logpost || !prev->logw ||
                           (!random_walk && (!prev->grad_logpost || !p_prev))))
    return fail(SMC2_E_INVALID_ARG, "prev population or p_prev has a NULL pointer");
  return SMC2_OK;
}

// The reweighting kernel's launch (and the iteration counter's advance) on `hs`, with the gather
// scratch and the status word given.
smc2_status launch_reweight(const smc2_model *model, int32_t S, int32_t N, double gamma,
                            int32_t random_walk, smc2_population *cur,
                            const smc2_population *prev, const double *p_prev,
                            int32_t first_iteration, uint64_t seed, uint32_t *iteration,
                            int32_t advance_iteration, int32_t *ancestors, double *ess,
                            int32_t *resampled, double *estimate, double *recycle,
                            double *gather, int32_t *status, hipStream_t hs) {
  OuterArgs a{};
  a.S = S;
  a.N = N;
  a.D = model->D;
  a.first = first_iteration ? 1 : 0;
  a.random_walk = random_walk ? 1 : 0;
  a.gamma = gamma;
  a.pr = make_prior(model);
  a.seed = seed;
  a.iteration = iteration;
  a.theta = cur->theta;
  a.logpost = cur->logpost;
  a.grad_logpost = cur->grad_logpost;
  a.loglik = cur->loglik;
  a.logw = cur->logw;
  if (!first_iteration) {
    a.prev_logpost = prev->logpost;
    a.prev_grad_logpost = prev->grad_logpost;
    a.prev_logw = prev->logw;
    a.p_prev = p_prev;
  }
  a.anc_out = ancestors;
  a.ess_out = ess;
  a.resampled_out = resampled;
  a.estimate = estimate;
  a.recycle = recycle;
  a.scratch = gather;
  a.status = status;
  hipLaunchKernelGGL(reweight_resample_kernel, dim3(S), dim3(kOuterThreads), 0, hs, a);
  HIP_TRY(hipGetLastError());
  if (advance_iteration) {
    hipLaunchKernelGGL(advance_iteration_kernel, dim3(1), dim3(64), 0, hs, iteration);
    HIP_TRY(hipGetLastError());
  }
  return SMC2_OK;
}

}  // namespace

extern "C" {

smc2_status smc2_reweight_resample(smc2_ctx *ctx, const smc2_model *model, int32_t S, int32_t N,
                                   double gamma, int32_t random_walk, smc2_population *cur,
                                   const smc2_population *prev, const double *p_prev,
                                   int32_t first_iteration, uint64_t seed,
                                   uint32_t *iteration, int32_t advance_iteration,
                                   int32_t *ancestors, double *ess, int32_t *resampled,
                                   double *estimate, double *recycle, void *stream) {
  if (!ctx || !ctx->reserved) return fail(SMC2_E_INVALID_ARG, "context not reserved");
  smc2_status st = check_reweight_args(model, S, N, gamma, random_walk, cur, prev, p_prev,
                                       first_iteration, iteration);
  if (st != SMC2_OK) return st;
  if (model->kind != ctx->model.kind || model->d_x != ctx->model.d_x || model->D != ctx->model.D)
    return fail(SMC2_E_INVALID_ARG, "model differs from the reservation");
  if ((long)S * N > (long)ctx->S * ctx->N)
    return fail(SMC2_E_INVALID_ARG, "S*N exceeds the reservation");
  DeviceGuard g(ctx->device);
  return launch_reweight(model, S, N, gamma, random_walk, cur, prev, p_prev, first_iteration,
                         seed, iteration, advance_iteration, ancestors, ess, resampled, estimate,
                         recycle, ctx->outer_scratch, ctx->status, (hipStream_t)stream);
}

smc2_status smc2_reweight_resample_noalloc(const smc2_model *model, int32_t S, int32_t N,
                                           double gamma, int32_t random_walk,
                                           smc2_population *cur, const smc2_population *prev,
                                           const double *p_prev, int32_t first_iteration,
                                           uint64_t seed, uint32_t *iteration,
                                           int32_t advance_iteration, int32_t *ancestors,
                                           double *ess, int32_t *resampled, double *estimate,
                                           double *recycle, int32_t *status, void *stream) {
  smc2_status st = check_reweight_args(model, S, N, gamma, random_walk, cur, prev, p_prev,
                                       first_iteration, iteration);
  if (st != SMC2_OK) return st;
  if ((size_t)S * (size_t)N * (size_t)(2 * model->D + 2) > kNoAllocScratchDoubles)
    return fail(SMC2_E_INVALID_ARG,
                "S * N * (2D + 2) = " + std::to_string((size_t)S * N * (2 * model->D + 2)) +
                    " exceeds the no-allocation scratch of " +
                    std::to_string(kNoAllocScratchDoubles) + " doubles");
  int dev = 0;
  HIP_TRY(hipGetDevice(&dev));
  if (dev < 0 || dev >= kMaxDevices) return fail(SMC2_E_UNSUPPORTED, "device index above 63");
  // once per device, with that device current: the device address of the scratch array
  std::call_once(g_noalloc_once[dev], [dev] {
    void *p = nullptr;
    g_noalloc_err[dev] = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    g_noalloc_scratch[dev] = g_noalloc_err[dev] == hipSuccess ? p : nullptr;
  });
  if (g_noalloc_err[dev] != hipSuccess || !g_noalloc_scratch[dev])
    return fail(SMC2_E_DEVICE, std::string("hipGetSymbolAddress(scratch): ") +
                                   hipGetErrorString(g_noalloc_err[dev]));
  return launch_reweight(model, S, N, gamma, random_walk, cur, prev, p_prev, first_iteration,
                         seed, iteration, advance_iteration, ancestors, ess, resampled, estimate,
                         recycle, (double *)g_noalloc_scratch[dev], status, (hipStream_t)stream);
}

smc2_status smc2_prior_init(smc2_ctx *ctx, const smc2_model *model, int32_t S, int32_t N,
                            uint64_t seed, double *theta, void *stream) {
  if (!ctx || !ctx->reserved) return fail(SMC2_E_INVALID_ARG, "context not reserved");
  std::string why;
  if (!model_ok(model, why)) return fail(SMC2_E_INVALID_ARG, why);
  if (S < 1 || N < 1 || !theta) return fail(SMC2_E_INVALID_ARG, "bad sizes or NULL theta");
  DeviceGuard g(ctx->device);
  const int items = S * N;
  hipLaunchKernelGGL(prior_init_kernel, dim3((items + 255) / 256), dim3(256), 0,
                     (hipStream_t)stream, items, model->D, make_prior(model), seed, theta);
  HIP_TRY(hipGetLastError());
  return SMC2_OK;
}

smc2_status smc2_pf_trace(smc2_ctx *ctx, int32_t s, int32_t i, uint8_t *flags,
                          int32_t *ancestors, double *steps_s, void *stream) {
  if (!ctx || !ctx->reserved) return fail(SMC2_E_INVALID_ARG, "context not reserved");
  if (ctx->opts.persistent)
    return fail(SMC2_E_INVALID_ARG, "traces are kept per item only without persistence");
  if (s < 0 || s >= ctx->S || i < 0 || i >= ctx->N || !flags || !ancestors)
    return fail(SMC2_E_INVALID_ARG, "item out of range or NULL output");
  DeviceGuard g(ctx->device);
  HIP_TRY(hipStreamSynchronize((hipStream_t)stream));
  const int T = ctx->T_len[s];
  const size_t slot = (size_t)s * ctx->N + i;
  const size_t t_ld = std::max(ctx->T_max, 1), ld = ctx->L.MP;
  if (T == 0) return SMC2_OK;
  if (steps_s)
    HIP_TRY(hipMemcpy(steps_s, ctx->steps_s + slot * t_ld, (size_t)T * 8, hipMemcpyDeviceToHost));
  HIP_TRY(hipMemcpy(flags, ctx->flags + slot * t_ld, T, hipMemcpyDeviceToHost));
  std::vector<int32_t> rows((size_t)T * ld);
  HIP_TRY(hipMemcpy(rows.data(), ctx->anc + slot * t_ld * ld, rows.size() * 4,
                    hipMemcpyDeviceToHost));
  for (int t = 0; t < T; ++t)
    for (int j = 0; j < ctx->M; ++j)
      ancestors[(size_t)t * ctx->M + j] = flags[t] ? rows[(size_t)t * ld + j] : -1;
  return SMC2_OK;
}

smc2_status smc2_philox_probe(int32_t R, const uint32_t *ctr, const uint32_t *n, uint64_t seed,
                              uint32_t *out, double *normals, double *uniforms, float *normals32,
                              float *uniforms32, void *stream) {
  if (R < 1 || !ctr || ((normals || uniforms || normals32 || uniforms32) && !n))
    return fail(SMC2_E_INVALID_ARG, "R >= 1 and ctr (and n) non-NULL required");
  hipLaunchKernelGGL(philox_probe_kernel, dim3((R + 255) / 256), dim3(256), 0,
                     (hipStream_t)stream, R, ctr, n, seed, out, normals, uniforms, normals32,
                     uniforms32);
  HIP_TRY(hipGetLastError());
  return SMC2_OK;
}

smc2_status smc2_tile_info(int32_t tile, int32_t d_x, int32_t *max_particles, int32_t *waves,
                           int32_t *per_lane) {
  if (tile < 1 || tile >= kNumTiles || !max_particles || !waves || !per_lane)
    return fail(SMC2_E_INVALID_ARG, "tile index out of range or NULL output");
  const Tile t = kTiles[tile];
  bool built = false;
  for (const auto &k : kernels())
    if (k.dx == d_x && k.waves == t.waves && k.ppl == t.ppl) built = true;
  if (!built) return fail(SMC2_E_INVALID_ARG, "tile not built for this state dimension");
  *max_particles = t.waves * 64 * t.ppl;
  *waves = t.waves;
  *per_lane = t.ppl;
  return SMC2_OK;
}

}  // extern "C"
