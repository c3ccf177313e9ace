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

# Peak figures of one MI355X (published): HBM3E bandwidth, and the vector-ALU issue rate with
# packed FP32 disabled: 256 CUs x 4 SIMDs x 16 lanes x 2.4 GHz = 39.3 T lane-slots/s
# (the FP32 vector rate without packed math, 78.6 TFLOP/s counting an FMA as two).
PEAK_HBM_GBS = 8000.0
PEAK_VALU_TSLOTS = 256 * 4 * 16 * 2.4e9 / 1e12

# Algorithmic VALU lane-slots per particle-step of the fused forward+adjoint for d = 1, counted
# from the method's arithmetic (not from the executed code): the forward pass, its recompute
# inside the adjoint and the adjoint sweep each need the step's normal (a quarter of a
# Philox4x32-10 call, 10 rounds x 6 integer ops, and half a Box-Muller pair: log, sqrt, sin/cos
# at the quarter-rate transcendental cost of 4 slots), the transition and log g (about 8), and
# the weight exponential (4); the forward adds the max / sum / ESS reductions (6 per particle,
# amortised) and the resampling search (log2 M compares for the resampled fraction r); the
# adjoint adds about 12 for the transposed derivatives.  See the design doc for the itemisation.
def alg_slots_per_particle_step(M, r):
    philox = 0.25 * 10 * 6
    box_muller = 0.5 * (4 * 4 + 6)
    model = 8 + 4
    per_pass = philox + box_muller + model
    forward = per_pass + 6 + r * (np.log2(M) + 4)
    recompute = per_pass + r * 2
    adjoint = 12
    return forward + recompute + adjoint


def algorithmic_bytes_per_particle_step(r, c, rs, d=1):
    """HBM bytes the method must move per particle-step: the int32 ancestor written in the
    forward and read in the adjoint at a resampled step (fraction r), and the (x, log W)
    checkpoint written and read once every c steps (rs bytes per value)."""
    return r * 8.0 + 2.0 * (d + 1) * rs / c


def _timed_graph(run, steps, warmup):
    import torch
    run.first_iteration()
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
    return start.elapsed_time(stop) / 1e3, wall


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
    m = pyoracle.Model(w.kind, w.d, w.D, w.prior_mu, w.prior_sd)
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
                       "%.1f s wall" % (i, w.M, int(w.T_len[0]), w.name, dt))


def measure(w, precision, steps, warmup, with_kernel=True):
    from paper_2407_17296_amd import driver
    run = driver.SMC2Run(w, precision=precision)
    gpu_s, wall = _timed_graph(run, steps, warmup)
    out = dict(seconds=gpu_s, wall=wall, ms_per_step=1e3 * gpu_s / steps,
               value=w.particle_steps() * steps / gpu_s)
    if with_kernel:
        out["kernel_s"] = _kernel_duration(run, max(3, min(10, steps)))
        out["resample_fraction"] = _resample_fraction(run)
    run.close()
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--config", type=int, default=1)
    ap.add_argument("--no-fp64", action="store_true")
    ap.add_argument("--no-growth", action="store_true")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--cpu-seconds", type=float, default=15.0)
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py runs on one GPU: the hot path shards by parameter sample and this build "
              "measures one GPU's share; --gpus %d is not supported" % args.gpus, file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_2407_17296_amd import smc2, synth
    torch.cuda.init()
    w = synth.make(args.config)
    print("[bench] workload %s S=%d N=%d M=%d T=%d, %d warmup + %d timed iterations" % (
        w.name, w.S, w.N, w.M, w.T_max, args.warmup, args.steps), file=sys.stderr, flush=True)
    mixed = measure(w, smc2.MIXED, args.steps, args.warmup)
    print("[bench] mixed: %.3f ms/iteration" % mixed["ms_per_step"], file=sys.stderr, flush=True)

    res = {}
    if not args.no_fp64:
        fp64 = measure(w, smc2.FP64, max(3, args.steps // 2), 1, with_kernel=False)
        res["fp64_plain"] = dict(value=fp64["value"], ms_per_step=fp64["ms_per_step"])
        res["mixed_over_fp64"] = mixed["value"] / fp64["value"]
        print("[bench] fp64: %.3f ms/iteration" % fp64["ms_per_step"], file=sys.stderr, flush=True)
    if not args.no_growth:
        wg = synth.make(3)
        gm = measure(wg, smc2.MIXED, 5, 1, with_kernel=False)
        gf = measure(wg, smc2.FP64, 3, 1, with_kernel=False)
        res["growth_workload"] = dict(workload="%s T=%d N=%d M=%d" % (wg.name, wg.T_max, wg.N, wg.M),
                                      mixed_value=gm["value"], fp64_value=gf["value"],
                                      mixed_over_fp64=gm["value"] / gf["value"])
        print("[bench] growth mixed %.3f ms, fp64 %.3f ms" % (gm["ms_per_step"], gf["ms_per_step"]),
              file=sys.stderr, flush=True)

    ps_launch = w.particle_steps()
    r = mixed["resample_fraction"]
    c = int(np.ceil(np.sqrt(w.T_max)))
    slots = alg_slots_per_particle_step(w.M, r)
    achieved = slots * ps_launch / mixed["kernel_s"] / 1e12
    hbm_bytes = algorithmic_bytes_per_particle_step(r, c, 4) * ps_launch
    roof = dict(bound="alu", achieved=achieved, peak=PEAK_VALU_TSLOTS, unit="Tslot/s",
                frac=achieved / PEAK_VALU_TSLOTS, traffic=None,
                kernel="pf_fwd_adj_kernel<float, ModelLG1D<float>, 4, 4>",
                kernel_ms=1e3 * mixed["kernel_s"], alg_slots_per_particle_step=slots,
                resample_fraction=r,
                hbm_algorithmic_GBs=hbm_bytes / mixed["kernel_s"] / 1e9,
                hbm_frac=hbm_bytes / mixed["kernel_s"] / 1e9 / PEAK_HBM_GBS)

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
        "config": {"workload": "%s: 1-D linear-Gaussian SSM, T=%d, N=%d samples, M=%d particles, "
                               "one SMC2 iteration per step" % (w.name, w.T_max, w.N, w.M),
                   "global_batch": w.N, "seq_len": w.T_max, "particles": w.M,
                   "parallelism": "one GPU"},
        "roofline": roof,
        "cpu_baseline": cpu,
    }
    line.update(res)
    print(json.dumps(line))


if __name__ == "__main__":
    main()
