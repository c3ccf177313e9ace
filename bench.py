"""Benchmark of the Enhanced SMC^2 hot path on one MI355X.

A step is one SMC^2 iteration of the whole hot path over one batch: the Langevin move, the fused
CRN-PF forward+adjoint for every (series, sample), and the L-kernel reweighting with ESS and
resampling, replayed from one captured HIP graph.  The default workload is the largest one that
fits one GPU: 64 independent stochastic-volatility series of uneven length (T_s ~ U{50..1000}),
each with N = 256 parameter samples of M = 256 particles, all in one launch (mixed precision).
The metric is forward+backward particle-steps per second, N * M * sum_s T_s per iteration, over
the timed iterations with inputs resident in HBM.

Printed: one JSON line with the metric, the plain-FP64 form on the same workload, the same
workload with the checkpoint interval held at ceil(sqrt(T_max)), the mixed and FP64 forms on the
1-D linear-Gaussian workload (T = 250, N = 1024, M = 1024), on the growth-model workload
(T = 100, N = 4096, M = 512) and on the 16-dimensional linear-Gaussian workload (T = 100,
N = 512, M = 2048), the roofline of the dominant kernel (the fused filter, timed with
HIP events on its own stream) and the FP64 CPU oracle timed on a bounded sample on the host's
cores.
"""
import argparse
import concurrent.futures as cf
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

# Peak figures of one MI355X (published): HBM3E bandwidth, and the FP32 vector issue rate with
# packed FP32 disabled: 256 CUs x 128 FP32 lanes per clock x 2.4 GHz = 78.6 T lane-slots/s
# (the published 157.3 TFLOP/s FP32 vector rate, counting an FMA as two).
PEAK_HBM_GBS = 8000.0
PEAK_VALU_TSLOTS = 256 * 128 * 2.4e9 / 1e12  # T FP32 lane-slots per second

# Algorithmic VALU work per particle-step of the CRN-PF forward sweep and its adjoint for d = 1,
# in FP32 lane-slots of a direct implementation of the method's arithmetic (itemised
# below).  An FP32 add / multiply / FMA / compare / select / integer op takes one slot; an
# FP64 operation two (half rate); the 32 x 32 -> 64-bit integer multiply-add and the
# transcendental unit (log, sqrt, sin, cos, exp) four (quarter rate).  The rates were measured
# on the device with dependent-chain-free loops.
#   noise      a Philox4x32-10 block serves 4 particles: 10 rounds x (2 multiply-adds x 4
#              + 2 three-input xors) / 4 = 25; half a Box-Muller pair: (8 full + 4
#              transcendental x 4) / 2 = 12                                       -> 37
#   model      the transition, log g, and the weight update with its NaN guard (3); per model
#              below
#   normalise  running max 1 (exact in FP32), subtract / scale / exp 6, FP64 conversion and
#              FP64 sum 4, squared sum for the ESS test 1, shifted carry 1        -> 13
#   resample   per resampled step: FP64 prefix 4, offspring count from P / tot 24, marker
#              and gather 2                                                       -> 30 r
#   adjoint    transposed derivatives of log g and of the transition (per model below),
#              summed into the parameter adjoint 3, scatter-add to the parent at a resampled
#              step 2 r                                                           -> A + 3 + 2 r
# Per model (forward model slots, adjoint slots A):
#   1-D LG  transition a x + sx e 2, log g (y - x) / sy, -r/2 * r + c 4, update 3 -> 9;
#           adjoint: d log g / dx and / d log sy 5, the transition's three products 6 -> 11
#   SV      transition phi (x - mu) + (s e + mu) 3, log g: y^2 1, exp(-x) as a multiply and
#           the exp unit 5, two FMAs 2, update 3 -> 14; adjoint: d log g / dx with exp(-x)
#           again 9 (y^2 / 2 1, exp 5, FMA 1, scale by the weight adjoint 1, add 1), the
#           transition's (1 - phi) x_b 1, (1 - phi^2)(x - mu) x_b 3, s e x_b 2, phi x_b 1 -> 16
#   growth  transition x/2 + 25 x / (1 + x^2) + forcing + sx e: 1 + x^2 1, the reciprocal 4,
#           25 x and its product 2, x/2 + 1, sx e + forcing 1, sum 1 -> 10; log g: x^2 1,
#           y - x^2/20 1, / sy 1, -r/2 * r + c 2 -> 5; update 3 -> 18; adjoint: d log g / dx and
#           / d log sy with the residual rebuilt 3, wb r x / (10 sy^2) and its add 5, wb (r^2 - 1)
#           and its add 3 -> 11; the transition's slope 1/2 + 25 (1 - x^2) / (1 + x^2)^2 with its
#           reciprocal 9, sx e x_b and its add 3, x_b times the slope 1 -> 13; -> 24
# Rebuilding the step in the adjoint (from checkpoints) is implementation work, not counted.
MODEL_SLOTS = {0: (9.0, 11.0), 2: (18.0, 24.0), 3: (14.0, 16.0)}


def alg_slots_per_particle_step(M, r, d=1, kind=0):
    """The count above; for a d-component state the noise, the model and its transposed
    derivatives scale with d (an estimate for the models without their own entry, exact in form
    only for the linear-Gaussian ones)."""
    fwd_model, adj_model = MODEL_SLOTS.get(kind, MODEL_SLOTS[0])
    noise, model, normalise = 37.0 * d, fwd_model * d, 13.0
    forward = noise + model + normalise + 30.0 * r
    adjoint = adj_model * d + 3.0 + 2.0 * r * d
    return forward + adjoint


def algorithmic_bytes_per_particle_step(r, c, rs, d=1, lw_skip=True):
    """HBM bytes the method must move per particle-step: the int32 ancestor written in the
    forward and read in the adjoint at a resampled step (fraction r), and the checkpoint written
    and read once every c steps (rs bytes per value): the state, and the carried log-weight
    unless the step before resampled (then every log-weight is -log M and none is stored); with
    a checkpoint every step, the carried log-weight only where the adjoint rebuilds the step's
    weights, at a resampled step (a fraction r of the steps after a step that did not
    resample)."""
    if c == 1 and lw_skip:
        lw = (1.0 - r) * r
    else:
        lw = 1.0 - r if lw_skip else 1.0
    return r * 8.0 + 2.0 * (d + lw) * rs / c


def design_bytes_per_particle_step(r, c, rs, store_noise, d=1, lw_skip=True):
    """HBM bytes the chosen configuration moves by construction: ancestors and checkpoints as
    above, the stored noise (written once, read once), and for c > 1 the segment rows (state
    before the step, the noise when not stored, and the weight at resampled steps) written by
    the recomputation and read by the reverse sweep, plus the ancestors read again there."""
    b = algorithmic_bytes_per_particle_step(r, c, rs, d, lw_skip)
    if store_noise:
        b += 2.0 * d * rs * (1.0 if c == 1 else 1.5)
    if c > 1:
        rows = d + (0 if store_noise else d)
        b += 2.0 * (rows + r) * rs + 4.0 * r
    return b


MODEL_TEXT = {0: "1-D linear-Gaussian SSM", 1: "16-dimensional diagonal linear-Gaussian SSM",
              2: "nonlinear growth model", 3: "stochastic-volatility series",
              5: "SIR epidemic model"}
MODEL_KERNEL = {0: "ModelLG1D<float>", 1: "ModelLGDiag<float, 16>", 2: "ModelGrowth<float>",
                3: "ModelSV<float>", 5: "ModelSIR<float>"}


def _timed_graph(run, steps, warmup):
    """Seconds of `steps` graph replays, their wall time, and the seconds of the eager first
    iteration (prior draws, the filter, reweighting: the worst-case resampling rate)."""
    import torch
    a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    a.record()
    run.first_iteration()
    b.record()
    torch.cuda.synchronize()
    first_s = a.elapsed_time(b) / 1e3
    run.capture()
    for _ in range(warmup):
        run.replay()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    start, stop = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    start.record()
    for _ in range(steps):
        run.replay()
    stop.record()
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    return start.elapsed_time(stop) / 1e3, wall, first_s


def _kernel_duration(run, launches):
    """Average duration of the fused filter kernel: HIP events recorded on the stream the
    kernel is launched on, around each launch (the population is the last iteration's)."""
    import torch
    stream = torch.cuda.current_stream()
    evs = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
           for _ in range(launches)]
    run._pf(stream=stream)
    torch.cuda.synchronize()
    for a, b in evs:
        a.record(stream)
        run._pf(stream=stream)
        b.record(stream)
    torch.cuda.synchronize()
    return float(np.mean([a.elapsed_time(b) for a, b in evs])) / 1e3


def _resample_fraction(run):
    """Fraction of particle-steps at which the filters resampled, for the last population: the
    filter is run again on it in a context of one workgroup per item (the same numbers as any
    launch shape), whose per-item flags are then read for a sample of items of every series."""
    import torch
    from paper_2407_17296_amd import smc2
    w = run.w
    o = run.opts
    opts = smc2.pf_opts(precision=o.precision, resampler=o.resampler, ess_frac=o.ess_frac,
                        ckpt_interval=1, want_grad=0, tile=o.tile, persistent=0)
    ctx = smc2.Context(run.model, opts, w.S, w.N, w.M, w.T_len, w.T_max)
    ll = torch.empty((w.S, w.N), dtype=torch.float64, device=run.dev)
    ctx.pf(run.cur["theta"], run.y, run.seed, run.iteration, ll, None)
    torch.cuda.synchronize()
    res = steps = 0
    per = max(1, 16 // w.S)
    for s in range(w.S):
        T = int(w.T_len[s])
        for i in range(0, w.N, max(1, w.N // per)):
            fl, _ = smc2.smc2_pf_trace(ctx.h, s, i, T, w.M)
            res += int(fl.sum())
            steps += T
    ctx.close()
    # resampled steps over all steps of the sampled items (a long series counts for its length,
    # as its particle-steps do)
    return float(res) / max(steps, 1)


def cpu_baseline(w, seconds, threads):
    """The FP64 oracle (CRN-PF with forward tangent) on a bounded sample of the workload's
    filters (series taken in turn), theta-parallel over host threads; particle-steps per
    second."""
    sys.path.insert(0, os.path.join(ROOT, "oracle"))
    import pyoracle
    if not os.path.exists(pyoracle.LIB_PATH):
        pyoracle.build()
    m = pyoracle.Model(w.kind, w.d, w.D, w.prior_mu, w.prior_sd, w.prior_kind, w.constants)
    rng = np.random.default_rng(w.seed)
    thetas = w.theta_true + 0.1 * rng.standard_normal((w.N, w.D))

    def one(i):
        s, n = i % w.S, (i // w.S) % w.N
        T = int(w.T_len[s])
        pyoracle.pf(m, thetas[n], w.y[s, :T], w.M, w.seed, 2, s * w.N + n)
        return w.M * T

    done = 0
    t0 = time.perf_counter()
    i = 0
    with cf.ThreadPoolExecutor(threads) as ex:
        while time.perf_counter() - t0 < seconds:
            batch = list(range(i, i + threads))
            i += threads
            done += sum(ex.map(one, batch))
    dt = time.perf_counter() - t0
    series = ("the %d series in turn (T_s %d..%d)" % (w.S, int(w.T_len.min()), int(w.T_len.max()))
              if w.S > 1 else "T=%d" % int(w.T_len[0]))
    return dict(value=done / dt, unit="particle-steps/s", cores=threads, kind="oracle",
                sample="%d filters of M=%d, %s, of workload %s at theta near the data-generating "
                       "value, %.3g particle-steps in %.1f s wall, on %s" % (
                           i, w.M, series, w.name, done, dt, _cpu_model()))


def _cpu_model():
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown CPU"


def measure(w, precision, steps, warmup, with_kernel=True, tune=True, force=None):
    from paper_2407_17296_amd import autotune, driver
    if force is not None:
        t = force
    else:
        t = (autotune.tune(w, precision) if tune
             else dict(tile=0, ckpt=0, store_noise=0, persistent=0))
    run = driver.SMC2Run(w, precision=precision, tile=t["tile"], ckpt_interval=t["ckpt"],
                         store_noise=t.get("store_noise", 1), persistent=t.get("persistent", 0))
    gpu_s, wall, first_s = _timed_graph(run, steps, warmup)
    out = dict(seconds=gpu_s, wall=wall, ms_per_step=1e3 * gpu_s / steps,
               value=w.particle_steps() * steps / gpu_s, tile=t["tile"], ckpt=t["ckpt"],
               store_noise=t.get("store_noise", 1), persistent=t.get("persistent", 0),
               first_s=first_s, tuned=t)
    if with_kernel:
        out["kernel_s"] = _kernel_duration(run, max(3, min(10, steps)))
        out["resample_fraction"] = _resample_fraction(run)
    run.close()
    return out


def _config_of(m):
    return dict(tile=m["tile"], ckpt=m["ckpt"], store_noise=m["store_noise"],
                persistent=m["persistent"])


def sqrt_ckpt_choice(tuned):
    """The fastest tuned configuration whose checkpoint interval is ceil(sqrt(T_max)) (the
    autotuner's interval 0), or None."""
    best = [a for a in tuned.get("all", []) if a["ckpt"] == 0]
    if not best:
        return None
    b = min(best, key=lambda a: a["ms"])
    return dict(tile=b["tile"], ckpt=0, store_noise=b["store_noise"],
                persistent=b.get("persistent", 0))


def other_workload(index, steps, warmup, tune):
    """Mixed and FP64 forms of another workload, each over `steps` timed iterations."""
    from paper_2407_17296_amd import smc2, synth
    wo = synth.make(index)
    mo = measure(wo, smc2.MIXED, steps, warmup, with_kernel=False, tune=tune)
    fo = measure(wo, smc2.FP64, steps, warmup, with_kernel=False, tune=tune)
    print("[bench] %s mixed %.3f ms, fp64 %.3f ms" % (wo.name, mo["ms_per_step"],
                                                      fo["ms_per_step"]),
          file=sys.stderr, flush=True)
    return dict(workload="%s: %s, T=%d, N=%d, M=%d" % (wo.name, MODEL_TEXT[wo.kind], wo.T_max,
                                                      wo.N, wo.M),
                steps=steps, mixed_value=mo["value"], fp64_value=fo["value"],
                mixed_ms_per_step=mo["ms_per_step"], fp64_ms_per_step=fo["ms_per_step"],
                mixed_over_fp64=mo["value"] / fo["value"], mixed_config=_config_of(mo),
                fp64_config=_config_of(fo))


def kernel_sources_sha():
    """Hash of the code of the fused filter kernel's sources, comments and whitespace removed
    (counters recorded for other kernel code no longer describe it; an edited comment leaves the
    kernel as it was)."""
    import hashlib
    import re
    h = hashlib.sha256()
    csrc = os.path.join(ROOT, "paper_2407_17296_amd", "csrc")
    for f in ("device_common.h", "models.h", "pf_kernel.h"):
        with open(os.path.join(csrc, f)) as fh:
            code = re.sub(r"/\*.*?\*/", " ", fh.read(), flags=re.S)
        code = re.sub(r"//[^\n]*", " ", code)
        h.update(" ".join(code.split()).encode())
    return h.hexdigest()[:16]


def recorded_traffic(workload_name, tile, precision, ckpt, store_noise, persistent=0):
    """HBM bytes per launch from the committed counter summary, if it was taken on the current
    kernel sources with the same workload, launch shape, precision, checkpoint interval, noise
    storage and grid mode; else None."""
    path = os.path.join(ROOT, "profiles", "pf_fwd_adj_traffic.json")
    try:
        with open(path) as f:
            rec = json.load(f)
    except (OSError, ValueError):
        return None
    for r in rec.get("records", []):
        if (r.get("kernel_sha") == kernel_sources_sha() and r.get("workload") == workload_name
                and r.get("tile") == tile and r.get("precision") == precision
                and r.get("ckpt") == ckpt and r.get("store_noise") == store_noise
                and r.get("persistent", 0) == persistent):
            return r.get("hbm_bytes_per_launch")
    return None


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", type=int, default=4,
                    help="workload index (synth.make): 0 small 1-D LG, 1 1-D LG T=250 N=1024 "
                         "M=1024, 2 16-dim LG, 3 growth, 4 SV (64 series, the default), 5 SIR")
    ap.add_argument("--no-fp64", action="store_true")
    ap.add_argument("--no-others", action="store_true",
                    help="skip the 1-D LG, growth and 16-dim LG workloads' mixed and FP64 "
                         "lines")
    ap.add_argument("--no-sqrt", action="store_true",
                    help="skip the line with the checkpoint interval held at ceil(sqrt(T))")
    ap.add_argument("--other-steps", type=int, default=20,
                    help="timed iterations per form on the other workloads")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--cpu-seconds", type=float, default=15.0)
    ap.add_argument("--calibrate-copy-mib", type=int, default=0,
                    help="finish with a plain device copy of this many MiB (a known-size "
                         "reference for the FETCH_SIZE / WRITE_SIZE counters)")
    ap.add_argument("--no-tune", action="store_true",
                    help="use the library's default launch shapes instead of autotuning")
    ap.add_argument("--tile", type=int, default=None,
                    help="force the launch shape of the mixed-precision main workload "
                         "(with --ckpt, --store-noise and --persistent; skips its tuning)")
    ap.add_argument("--ckpt", type=int, default=0)
    ap.add_argument("--store-noise", type=int, default=0)
    ap.add_argument("--persistent", type=int, default=0)
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py measures one GPU (the hot path shards by parameter sample, and one GPU's "
              "share is what it times); --gpus %d is not supported" % args.gpus, file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_2407_17296_amd import smc2, synth
    torch.cuda.init()
    w = synth.make(args.workload)
    print("[bench] workload %s S=%d N=%d M=%d T_max=%d sum T=%d, %d warmup + %d timed "
          "iterations" % (w.name, w.S, w.N, w.M, w.T_max, int(w.T_len.sum()), args.warmup,
                          args.steps), file=sys.stderr, flush=True)
    tune = not args.no_tune
    force = (dict(tile=args.tile, ckpt=args.ckpt, store_noise=args.store_noise,
                  persistent=args.persistent) if args.tile is not None else None)
    mixed = measure(w, smc2.MIXED, args.steps, args.warmup, tune=tune, force=force)
    print("[bench] mixed: %.3f ms/iteration (%s)" % (mixed["ms_per_step"], _config_of(mixed)),
          file=sys.stderr, flush=True)
    for a in mixed["tuned"].get("all", [])[:12]:
        print("[bench]   tuning: %s" % a, file=sys.stderr, flush=True)
    for a in mixed["tuned"].get("refined", []):
        print("[bench]   retimed: %s" % a, file=sys.stderr, flush=True)

    res = {}
    if not args.no_sqrt and force is None and tune:
        cs = sqrt_ckpt_choice(mixed["tuned"])
        if cs is not None and cs != _config_of(mixed):
            sq = measure(w, smc2.MIXED, args.steps, args.warmup, force=cs)
        else:
            sq = mixed
        c_sq = int(np.ceil(np.sqrt(w.T_max)))
        res["ckpt_sqrt_T"] = dict(ckpt_interval=c_sq, value=sq["value"],
                                  ms_per_step=sq["ms_per_step"], kernel_ms=1e3 * sq["kernel_s"],
                                  config=_config_of(sq),
                                  note="the same workload with the checkpoint interval held at "
                                       "ceil(sqrt(T_max)) = %d (the fastest such launch shape)"
                                       % c_sq)
        print("[bench] ceil(sqrt T) checkpoints: %.3f ms/iteration" % sq["ms_per_step"],
              file=sys.stderr, flush=True)
    if not args.no_fp64:
        fp64 = measure(w, smc2.FP64, max(3, args.steps // 2), 1, with_kernel=False, tune=tune)
        res["fp64_plain"] = dict(value=fp64["value"], ms_per_step=fp64["ms_per_step"],
                                 config=_config_of(fp64))
        res["mixed_over_fp64"] = mixed["value"] / fp64["value"]
        print("[bench] fp64: %.3f ms/iteration" % fp64["ms_per_step"], file=sys.stderr, flush=True)
    if not args.no_others:
        for key, idx in (("lg1d_workload", 1), ("growth_workload", 3), ("lgdiag16_workload", 2)):
            if idx != args.workload:
                res[key] = other_workload(idx, args.other_steps, 3, tune)

    ps_launch = w.particle_steps()
    r = mixed["resample_fraction"]
    c_sqrt = int(np.ceil(np.sqrt(w.T_max)))
    c = mixed["ckpt"] or c_sqrt
    _, waves, ppl = smc2.smc2_tile_info(mixed["tile"], w.d) if mixed["tile"] else (0, 0, 0)
    lw_skip = w.d < 4  # the kernel stores every checkpoint's log-weights for wide states
    slots = alg_slots_per_particle_step(w.M, r, w.d, w.kind)
    achieved = slots * ps_launch / mixed["kernel_s"] / 1e12
    hbm_bytes = algorithmic_bytes_per_particle_step(r, c_sqrt, 4, w.d, lw_skip) * ps_launch
    design_bytes = design_bytes_per_particle_step(r, c, 4, mixed["store_noise"], w.d,
                                                  lw_skip) * ps_launch
    traffic = recorded_traffic(w.name, mixed["tile"], 1, c, mixed["store_noise"],
                               mixed["persistent"])
    roof = dict(bound="alu", achieved=achieved, peak=PEAK_VALU_TSLOTS, unit="Tslot/s",
                frac=achieved / PEAK_VALU_TSLOTS, traffic=traffic,
                kernel="pf_fwd_adj_kernel<float, %s, %d, %d>" % (MODEL_KERNEL[w.kind], waves, ppl),
                tile=mixed["tile"], ckpt_interval=c, store_noise=mixed["store_noise"],
                persistent=mixed["persistent"],
                kernel_ms=1e3 * mixed["kernel_s"], alg_slots_per_particle_step=slots,
                particle_steps_per_launch=ps_launch,
                resample_fraction=r,
                hbm_algorithmic_bytes_per_launch=hbm_bytes,
                hbm_design_bytes_per_launch=design_bytes,
                hbm_design_GBs=design_bytes / mixed["kernel_s"] / 1e9,
                hbm_design_frac=design_bytes / mixed["kernel_s"] / 1e9 / PEAK_HBM_GBS,
                hbm_measured_frac=(traffic / mixed["kernel_s"] / 1e9 / PEAK_HBM_GBS
                                   if traffic else None),
                kernel_sources_sha=kernel_sources_sha())

    cpu = None
    if not args.no_cpu:
        threads = min(16, os.cpu_count() or 1)
        cpu = cpu_baseline(w, args.cpu_seconds, threads)
        print("[bench] cpu oracle %.3g particle-steps/s on %d threads" % (cpu["value"], threads),
              file=sys.stderr, flush=True)

    series = ("%d series, T_s %d..%d (sum %d)" % (w.S, int(w.T_len.min()), int(w.T_len.max()),
                                                 int(w.T_len.sum())) if w.S > 1
              else "T=%d" % w.T_max)
    line = {
        "metric": "CRN-PF fwd+bwd particle-steps/s (N*M*T/s)",
        "value": mixed["value"],
        "unit": "particle-steps/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": mixed["ms_per_step"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32/f64 mixed",
        "data": "synthetic",
        "config": {"workload": "%s: %s, %s, N=%d samples, M=%d particles, one SMC2 iteration "
                               "per step" % (w.name, MODEL_TEXT[w.kind], series, w.N, w.M),
                   "global_batch": w.S * w.N, "seq_len": w.T_max, "particles": w.M,
                   "series": w.S, "parallelism": "one GPU"},
        "roofline": roof,
        "cpu_baseline": cpu,
    }
    line["first_iteration"] = dict(
        ms=1e3 * mixed["first_s"], value=w.particle_steps() / mixed["first_s"],
        note="iteration 1, eager: prior draws, the filter and reweighting")
    line.update(res)
    if args.calibrate_copy_mib > 0:
        src = torch.ones(args.calibrate_copy_mib * 262144, dtype=torch.float32, device="cuda:0")
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        dst.copy_(src)
        torch.cuda.synchronize()
        line["calibration_copy_bytes"] = src.numel() * 4
    print(json.dumps(line))


if __name__ == "__main__":
    main()
