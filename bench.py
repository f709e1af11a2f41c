#!/usr/bin/env python3
"""Throughput of random-batch FPM reconstruction steps on one MI355X.

A step is one random-batch update of the whole hot path: pupil rebuild from
the Zernike coefficients, crop/pupil/inverse-FFT/amplitude-loss/FFT/scatter
for each LED of the batch, pupil-parameter projection, Adam on the spectrum
and the pupil parameters. Default workload: 15 x 15 LEDs, 256^2 LR images ->
1024^2 HR spectrum, batches of 16, object + Zernike pupil learned, synthetic
data (seeded smooth random object, Poisson noise 1e4 / 1e2 photons for
bright / dark field). Inputs are resident in HBM before timing starts.

Prints one JSON line (rank 0):
  value        LED-images per second (fwd + bwd + update), whole job
  roofline     the dominant kernel: algorithmic work per launch / its mean
               duration (HIP events on the launch stream) vs MI355X peak
  cpu_baseline the FP64 oracle's steps on the same workload, host cores
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0          # MI355X HBM3E
FP32_VALU_PEAK_TFLOPS = 78.6   # 256 CU x 64 lanes x 2 (FMA) x 2.4 GHz, no packed FP32


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def fft_flops(n: int) -> float:
    """Conventional flop count of one complex FFT of length n: 5 n log2 n."""
    return 5.0 * n * math.log2(n)


def union_support_px(plan) -> int:
    """|U|: HR pixels covered by the pupil disk of some LED window."""
    import numpy as np
    N, M = plan.N, plan.M
    r = plan.info.pupil_radius_px
    u = np.arange(N) - N // 2
    mask = (u[:, None] ** 2 + u[None, :] ** 2) <= r * r
    cover = np.zeros((M, M), bool)
    base = M // 2 - N // 2
    for sr, sc in plan.shifts:
        cover[base + sr:base + sr + N, base + sc:base + sc + N] |= mask
    return int(cover.sum())


def kernel_work(plan, B: int):
    """Algorithmic bytes and flops per launch of each kernel for a batch of B LEDs."""
    N, S, rows = plan.N, plan.info.support_px, plan.info.support_rows
    U = union_support_px(plan)
    return {
        # crop: read the spectrum on the pupil disk; 'rows' inverse DFTs of length N
        "rows_forward": (8.0 * S * B, rows * fft_flops(N) * B),
        # read the measured amplitude; one inverse and one forward DFT per column
        "cols": (4.0 * N * N * B, 2 * N * fft_flops(N) * B),
        # accumulate the spectrum gradient on the disk; 'rows' forward DFTs
        "rows_backward": (8.0 * S * B, rows * fft_flops(N) * B),
        # Adam over U: read O, m, v, g; write O, m, v (float32 pairs)
        "adam_object": (56.0 * U, 0.0),
    }, U


def cpu_baseline(w, seconds: float):
    """Time the FP64 oracle's full steps on the same workload (bounded sample).

    The oracle builds its own inputs (truth object, measurements through its
    forward model, seeded Poisson noise, initial value); set-up is not timed.
    """
    import numpy as np
    from oracle import fpm_oracle as fo
    from paper_2408_13782_amd import inputs
    opt = fo.Optics(w.wavelength_um, w.na, w.mag, w.pixel_um, w.n_lr, w.upsample)
    k = fo.led_wavevectors(opt, w.n_side, w.pitch_mm, w.height_mm)
    shifts = fo.nearest_shifts(fo.led_shifts(opt, k))
    mask = fo.pupil_mask(opt)
    zern = fo.zernike_basis(opt, w.n_zernike)
    kappa = fo.defocus_phase_per_um(opt)
    amp, ph = inputs.truth_object(w.m_hr, seed=0)
    O_true = fo.spectrum(fo.transmission(amp, ph))
    P_true = fo.pupil(mask, zern, np.zeros(w.n_zernike), inputs.true_defocus(w, 0), kappa)
    q = np.where(fo.bright_field(opt, k), w.q_bright, w.q_dark)
    A = inputs.poisson_amplitudes(fo.forward_intensities(O_true, P_true, shifts, range(w.n_led)),
                                  q, seed=0).astype(np.float64)
    centre = (w.n_side // 2) * w.n_side + w.n_side // 2
    O0 = fo.initial_spectrum(A[centre], w.upsample)
    cfg = fo.SolveConfig(lr_object=w.lr_object, lr_zernike=w.lr_zernike, lr_z=w.lr_z,
                         learn_pupil=w.learn_zernike, learn_z=w.learn_z)
    st = fo.init_state(O0)
    perms = inputs.led_permutations(w.n_led, 12, seed=0)
    sched = fo.batches_from_permutations(perms, w.batch)
    n_img, n_steps = 0, 0
    t0 = time.perf_counter()
    while n_steps < len(sched) and (time.perf_counter() - t0 < seconds or n_steps < 3):
        fo.step(st, cfg, mask, zern, kappa, shifts, sched[n_steps], A)
        n_img += len(sched[n_steps])
        n_steps += 1
    dt = time.perf_counter() - t0
    return {"value": n_img / dt, "unit": "LED-images/s", "cores": 1, "kind": "oracle",
            "sample": f"{n_steps} full FP64 steps ({n_img} LED-images) of the same workload, "
                      f"numpy single thread, {dt:.1f} s"}


def main():
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=450)
    ap.add_argument("--warmup", type=int, default=30)
    ap.add_argument("--workload", default="paper", choices=["small", "paper", "large"])
    ap.add_argument("--profile-steps", type=int, default=60,
                    help="steps timed per kernel with events (after the main timing)")
    ap.add_argument("--copy-probe-mb", type=int, default=0,
                    help="after timing, one device-to-device copy of this size (a kernel of "
                         "known traffic for calibrating HBM counters)")
    ap.add_argument("--cpu-seconds", type=float, default=15.0)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    args = ap.parse_args()
    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print("bench.py measures one GPU: this build has no multi-GPU path "
              "(tiles of the field of view are independent and would shard one per GPU); "
              "run with --gpus 1", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    from paper_2408_13782_amd import fpm, inputs, problem

    torch.cuda.set_device(0)
    w = inputs.workload(args.workload)
    log(f"workload {w.name}: {w.n_side}x{w.n_side} LEDs, N={w.n_lr}, M={w.m_hr}, B={w.batch}")
    prob = problem.make_plan(w)
    problem.simulate(prob, seed=0)
    O0 = problem.initial_spectrum(prob)
    state = fpm.State(prob.plan, O0)
    hp = problem.hparams(w)
    plan = prob.plan
    total = args.warmup + args.steps + args.profile_steps
    epochs = -(-total // w.steps_per_epoch())
    batches = problem.schedule(inputs.led_permutations(w.n_led, epochs, seed=0), w.batch)
    ds = problem.flatten_schedule(batches[:total])
    A = prob.meas_amp
    torch.cuda.synchronize()
    log("set-up done")

    def run(start, stop):
        flat, sizes = ds.span(start, stop)
        plan.run(state, hp, flat, sizes, A)

    run(0, args.warmup)
    torch.cuda.synchronize()
    log(f"{args.warmup} warm-up steps done")

    stream = torch.cuda.current_stream()
    t_start = torch.cuda.Event(enable_timing=True)
    t_stop = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    t_start.record(stream)
    run(args.warmup, args.warmup + args.steps)
    t_stop.record(stream)
    torch.cuda.synchronize()
    ms = t_start.elapsed_time(t_stop)
    n_img = sum(len(b) for b in batches[args.warmup:args.warmup + args.steps])
    value = n_img / (ms / 1e3)
    log(f"{args.steps} timed steps: {ms:.2f} ms, {value:.4g} LED-images/s")

    if args.copy_probe_mb > 0:
        n = args.copy_probe_mb * (1 << 20) // 4
        src = torch.ones(n, dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        dst.copy_(src)
        torch.cuda.synchronize()
        log(f"copy probe: {2 * n * 4 / 1e6:.1f} MB moved (read + write)")
        del src, dst
    if args.profile_steps <= 0:
        print(json.dumps({"metric": "profiling run", "value": value, "unit": "LED-images/s"}))
        return

    # per-kernel durations with events around every launch (separate pass)
    plan.timing(True)
    run(args.warmup + args.steps, total)
    torch.cuda.synchronize()
    plan.timing(False)
    kt = plan.timing_collect()
    log("per-kernel mean us: " + ", ".join(f"{k}={v[0] / v[1] * 1e3:.2f}" for k, v in kt.items()))
    B = w.batch
    work, U = kernel_work(plan, B)
    timed = {k: kt[k][0] / kt[k][1] for k in work if k in kt}          # ms per launch
    dominant = max(timed, key=lambda k: timed[k])
    bytes_, flops = work[dominant]
    dur_s = timed[dominant] / 1e3
    if flops > 0:
        achieved = flops / dur_s / 1e12
        roof = {"bound": "alu", "achieved": achieved, "peak": FP32_VALU_PEAK_TFLOPS,
                "unit": "TFLOP/s", "frac": achieved / FP32_VALU_PEAK_TFLOPS, "traffic": None,
                "kernel": dominant, "mean_us": timed[dominant] * 1e3,
                "hbm_algorithmic_GBs": bytes_ / dur_s / 1e9}
    else:
        achieved = bytes_ / dur_s / 1e9
        roof = {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": achieved / HBM_PEAK_GBS, "traffic": None, "kernel": dominant,
                "mean_us": timed[dominant] * 1e3}
    chain_ms = sum(timed.get(k, 0.0) for k in ("rows_forward", "cols", "rows_backward"))
    S, N = plan.info.support_px, plan.N
    chain_bytes = (16.0 * S + 4.0 * N * N) * B
    detail = {
        "fwd_bwd_us_per_batch": chain_ms * 1e3,
        "fwd_bwd_led_images_per_s": B / (chain_ms / 1e3),
        "fwd_bwd_hbm_frac": chain_bytes / (chain_ms / 1e3) / 1e9 / HBM_PEAK_GBS,
        "per_kernel_mean_us": {k: v[0] / v[1] * 1e3 for k, v in kt.items()},
        "support_px": S, "union_px": U,
    }

    result = {
        "metric": "LED-images fwd+bwd/sec (256²→1024²)" if w.name == "paper" else
                  f"LED-images fwd+bwd/sec ({w.n_lr}²→{w.m_hr}²)",
        "value": value, "unit": "LED-images/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": ms / args.steps, "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f32", "data": "synthetic",
        "config": {"workload": f"{w.name}: {w.n_side}x{w.n_side} LEDs, {w.n_lr}^2 LR -> "
                               f"{w.m_hr}^2 HR, batch {w.batch}, object"
                               + (" + Zernike pupil" if w.learn_zernike else "")
                               + (" + defocus" if w.learn_z else ""),
                   "n_led": w.n_led, "n_lr": w.n_lr, "m_hr": w.m_hr, "batch": w.batch},
        "roofline": roof,
        "detail": detail,
    }
    if not args.no_cpu_baseline:
        log(f"oracle CPU baseline (~{args.cpu_seconds:.0f} s)")
        result["cpu_baseline"] = cpu_baseline(w, args.cpu_seconds)
        log("oracle CPU baseline done")
    print(json.dumps(result), flush=True)


if __name__ == "__main__":
    main()
