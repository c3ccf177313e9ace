"""Benchmark of the Enhanced SMC^2 hot path on one MI355X.

A step is one SMC^2 iteration of the whole hot path over one batch: the Langevin move, the fused
CRN-PF forward+adjoint for every (series, sample), and the L-kernel reweighting with ESS and
resampling, replayed from one captured HIP graph.  The default workload is the 1-D
linear-Gaussian model at T = 250 with N = 1024 parameter samples of M = 1024 particles (mixed
precision).  The metric is forward+backward particle-steps per second, N * M * sum(T) per
iteration, over the timed iterations with inputs resident in HBM.

Printed: one JSON line with the metric, the plain-FP64 form on the same workload, the
mixed/FP64 ratio on the growth-model workload (T = 100, N = 4096, M = 512), the roofline of the
dominant kernel (the fused filter, timed with HIP events on its own stream) and the FP64 CPU
oracle timed on a bounded sample on the host's cores.
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
#              + 4 xors) / 4 = 30; half a Box-Muller pair: (8 full + 4 transcendental x 4)
#              / 2 = 12                                                           -> 42
#   model      transition 2, log g 4, weight update and guard 3                   ->  9
#   normalise  running max 1 (exact in FP32), subtract / scale / exp 6, FP64 conversion and
#              FP64 sum 4, squared sum for the ESS test 1, shifted carry 1        -> 13
#   resample   per resampled step: FP64 prefix 4, offspring count from P / tot 24, marker
#              and gather 2                                                       -> 30 r
#   adjoint    transposed derivatives of log g and of the transition 11, summed into the
#              parameter adjoint 3, scatter-add to the parent at a resampled step 2 r
#                                                                                 -> 14 + 2 r
# Rebuilding the step in the adjoint (from checkpoints) is implementation work, not counted.
def alg_slots_per_particle_step(M, r, d=1):
    """The count above; for a d-component state the noise, the model and its transposed
    derivatives scale with d (an estimate for the other models, exact in form only for the
    linear-Gaussian ones)."""
    noise, model, normalise = 42.0 * d, 9.0 * d, 13.0
    forward = noise + model + normalise + 30.0 * r
    adjoint = 11.0 * d + 3.0 + 2.0 * r * d
    return forward + adjoint


def algorithmic_bytes_per_particle_step(r, c, rs, d=1, lw_skip=True):
    """HBM bytes the method must move per particle-step: the int32 ancestor written in the
    forward and read in the adjoint at a resampled step (fraction r), and the checkpoint written
    and read once every c steps (rs bytes per value): the state, and the carried log-weight
    unless the step before resampled (then every log-weight is -log M and none is stored)."""
    return r * 8.0 + 2.0 * (d + (1.0 - r if lw_skip else 1.0)) * rs / c


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
    """Fraction of steps at which the filters resampled in the last launch (from the flags the
    library keeps per item; needs the non-persistent layout)."""
    from paper_2407_17296_amd import smc2
    w = run.w
    fr = []
    for i in range(0, w.N, max(1, w.N // 16)):
        fl, _ = smc2.smc2_pf_trace(run.ctx.h, 0, i, int(w.T_len[0]), w.M)
        fr.append(fl.mean() if len(fl) else 0.0)
    return float(np.mean(fr))


def cpu_baseline(w, seconds, threads):
    """The FP64 oracle (CRN-PF with forward tangent) on a bounded sample of the workload's
    filters, theta-parallel over host threads; particle-steps per second."""
    sys.path.insert(0, os.path.join(ROOT, "oracle"))
    import pyoracle
    if not os.path.exists(pyoracle.LIB_PATH):
        pyoracle.build()
    m = pyoracle.Model(w.kind, w.d, w.D, w.prior_mu, w.prior_sd, w.prior_kind, w.constants)
    rng = np.random.default_rng(w.seed)
    thetas = w.theta_true + 0.1 * rng.standard_normal((w.N, w.D))
    y = w.y[0, :w.T_len[0]]

    def one(i):
        pyoracle.pf(m, thetas[i % w.N], y, w.M, w.seed, 2, i)
        return w.M * int(w.T_len[0])

    done = 0
    t0 = time.perf_counter()
    i = 0
    with cf.ThreadPoolExecutor(threads) as ex:
        while time.perf_counter() - t0 < seconds:
            batch = list(range(i, i + threads))
            i += threads
            done += sum(ex.map(one, batch))
    dt = time.perf_counter() - t0
    return dict(value=done / dt, unit="particle-steps/s", cores=threads, kind="oracle",
                sample="%d filters of M=%d, T=%d (%s) at theta near the data-generating value, "
                       "%.1f s wall, on %s" % (i, w.M, int(w.T_len[0]), w.name, dt, _cpu_model()))


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
        t = autotune.tune(w, precision) if tune else dict(tile=0, ckpt=0, store_noise=0)
    run = driver.SMC2Run(w, precision=precision, tile=t["tile"], ckpt_interval=t["ckpt"],
                         store_noise=t.get("store_noise", 1))
    gpu_s, wall, first_s = _timed_graph(run, steps, warmup)
    out = dict(seconds=gpu_s, wall=wall, ms_per_step=1e3 * gpu_s / steps,
               value=w.particle_steps() * steps / gpu_s, tile=t["tile"], ckpt=t["ckpt"],
               store_noise=t.get("store_noise", 1), first_s=first_s)
    if with_kernel:
        out["kernel_s"] = _kernel_duration(run, max(3, min(10, steps)))
        out["resample_fraction"] = _resample_fraction(run)
    run.close()
    return out


def kernel_sources_sha():
    """Hash of the sources of the fused filter kernel (counters recorded for another version
    of the kernel no longer describe it)."""
    import hashlib
    h = hashlib.sha256()
    csrc = os.path.join(ROOT, "paper_2407_17296_amd", "csrc")
    for f in ("device_common.h", "models.h", "pf_kernel.h"):
        with open(os.path.join(csrc, f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def recorded_traffic(workload_name, tile, precision, ckpt, store_noise):
    """HBM bytes per launch from the committed counter summary, if it was taken on the current
    kernel sources with the same workload, launch shape, precision, checkpoint interval and
    noise storage; else None."""
    path = os.path.join(ROOT, "profiles", "pf_fwd_adj_traffic.json")
    try:
        with open(path) as f:
            rec = json.load(f)
    except (OSError, ValueError):
        return None
    for r in rec.get("records", []):
        if (r.get("kernel_sha") == kernel_sources_sha() and r.get("workload") == workload_name
                and r.get("tile") == tile and r.get("precision") == precision
                and r.get("ckpt") == ckpt and r.get("store_noise") == store_noise):
            return r.get("hbm_bytes_per_launch")
    return None


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", type=int, default=1,
                    help="workload index (synth.make): 0 small 1-D LG, 1 1-D LG T=250 N=1024 "
                         "M=1024, 2 16-dim LG, 3 growth, 4 SV, 5 SIR")
    ap.add_argument("--no-fp64", action="store_true")
    ap.add_argument("--no-growth", action="store_true")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--cpu-seconds", type=float, default=15.0)
    ap.add_argument("--calibrate-copy-mib", type=int, default=0,
                    help="finish with a plain device copy of this many MiB (a known-size "
                         "reference for the FETCH_SIZE / WRITE_SIZE counters)")
    ap.add_argument("--no-tune", action="store_true",
                    help="use the library's default launch shapes instead of autotuning")
    ap.add_argument("--tile", type=int, default=None,
                    help="force the launch shape of the mixed-precision main workload "
                         "(with --ckpt and --store-noise; skips its tuning)")
    ap.add_argument("--ckpt", type=int, default=0)
    ap.add_argument("--store-noise", type=int, default=0)
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py measures one GPU (the hot path shards by parameter sample, and one GPU's "
              "share is what it times); --gpus %d is not supported" % args.gpus, file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_2407_17296_amd import smc2, synth
    torch.cuda.init()
    w = synth.make(args.workload)
    print("[bench] workload %s S=%d N=%d M=%d T=%d, %d warmup + %d timed iterations" % (
        w.name, w.S, w.N, w.M, w.T_max, args.warmup, args.steps), file=sys.stderr, flush=True)
    tune = not args.no_tune
    force = (dict(tile=args.tile, ckpt=args.ckpt, store_noise=args.store_noise)
             if args.tile is not None else None)
    mixed = measure(w, smc2.MIXED, args.steps, args.warmup, tune=tune, force=force)
    print("[bench] mixed: %.3f ms/iteration" % mixed["ms_per_step"], file=sys.stderr, flush=True)

    res = {}
    if not args.no_fp64:
        fp64 = measure(w, smc2.FP64, max(3, args.steps // 2), 1, with_kernel=False, tune=tune)
        res["fp64_plain"] = dict(value=fp64["value"], ms_per_step=fp64["ms_per_step"],
                                 tile=fp64["tile"], ckpt=fp64["ckpt"],
                                 store_noise=fp64["store_noise"])
        res["mixed_over_fp64"] = mixed["value"] / fp64["value"]
        print("[bench] fp64: %.3f ms/iteration" % fp64["ms_per_step"], file=sys.stderr, flush=True)
    if not args.no_growth:
        wg = synth.make(3)
        gm = measure(wg, smc2.MIXED, 5, 1, with_kernel=False, tune=tune)
        gf = measure(wg, smc2.FP64, 3, 1, with_kernel=False, tune=tune)
        res["growth_workload"] = dict(workload="%s T=%d N=%d M=%d" % (wg.name, wg.T_max, wg.N, wg.M),
                                      mixed_value=gm["value"], fp64_value=gf["value"],
                                      mixed_over_fp64=gm["value"] / gf["value"],
                                      mixed_tile=gm["tile"], fp64_tile=gf["tile"])
        print("[bench] growth mixed %.3f ms, fp64 %.3f ms" % (gm["ms_per_step"], gf["ms_per_step"]),
              file=sys.stderr, flush=True)

    from paper_2407_17296_amd import smc2 as _smc2
    ps_launch = w.particle_steps()
    r = mixed["resample_fraction"]
    c_sqrt = int(np.ceil(np.sqrt(w.T_max)))
    c = mixed["ckpt"] or c_sqrt
    _, waves, ppl = _smc2.smc2_tile_info(mixed["tile"], w.d) if mixed["tile"] else (0, 0, 0)
    lw_skip = w.d < 4  # the kernel stores every checkpoint's log-weights for wide states
    slots = alg_slots_per_particle_step(w.M, r, w.d)
    achieved = slots * ps_launch / mixed["kernel_s"] / 1e12
    hbm_bytes = algorithmic_bytes_per_particle_step(r, c_sqrt, 4, w.d, lw_skip) * ps_launch
    design_bytes = design_bytes_per_particle_step(r, c, 4, mixed["store_noise"], w.d,
                                                  lw_skip) * ps_launch
    traffic = recorded_traffic(w.name, mixed["tile"], 1, c, mixed["store_noise"])
    roof = dict(bound="alu", achieved=achieved, peak=PEAK_VALU_TSLOTS, unit="Tslot/s",
                frac=achieved / PEAK_VALU_TSLOTS, traffic=traffic,
                kernel="pf_fwd_adj_kernel<float, %s, %d, %d>" % (MODEL_KERNEL[w.kind], waves, ppl),
                tile=mixed["tile"], ckpt_interval=c, store_noise=mixed["store_noise"],
                kernel_ms=1e3 * mixed["kernel_s"], alg_slots_per_particle_step=slots,
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
        "config": {"workload": "%s: %s, T=%d, N=%d samples, M=%d particles, "
                               "one SMC2 iteration per step" % (w.name, MODEL_TEXT[w.kind],
                                                                w.T_max, w.N, w.M),
                   "global_batch": w.N, "seq_len": w.T_max, "particles": w.M,
                   "parallelism": "one GPU"},
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
