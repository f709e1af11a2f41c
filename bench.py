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
               duration (HIP events on the launch stream around 20 back-to-back
               launches on a step's operands) vs MI355X peak
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


# HBM bytes per launch of a kernel from rocprofv3 counters (FETCH_SIZE x 2 +
# WRITE_SIZE; the factor 2 is what a plain device copy of known size reads on
# the same counter), for the kernel build they were taken on. The large
# workload's kernels are those of the fused multi-parameter step.
TRAFFIC = {
    ("paper", "rows_forward"): (1920.5 * 2 + 4788.7) * 1024,
    ("paper", "cols"): (4452.1 * 2 + 4843.4) * 1024,
    ("paper", "rows_backward"): (4458.4 * 2 + 2450.0) * 1024,
    ("paper", "update"): (7238.3 * 2 + 9754.3) * 1024,
    ("large", "rows_forward"): (13206.3 * 2 + 39713.7) * 1024,
    ("large", "cols"): (36173.0 * 2 + 39817.2) * 1024,
    ("large", "rows_backward"): (33152.6 * 2 + 19470.9) * 1024,
    ("large", "update"): (45758.7 * 2 + 57628.2) * 1024,
}


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
    """Algorithmic (bytes, flops) per launch of each step kernel for a batch of B LEDs.
    Adam's share is the union U of the LED windows (the pixels whose gradient can
    be non-zero; with a learned geometry, U at the plan's table)."""
    N, S, rows = plan.N, plan.info.support_px, plan.info.support_rows
    U = union_support_px(plan)
    return {
        # crop: read the spectrum on the pupil disk; 'rows' inverse DFTs of length N
        "rows_forward": (8.0 * S * B, rows * fft_flops(N) * B),
        # read the measured amplitude; one inverse and one forward DFT per column
        "cols": (4.0 * N * N * B, 2 * N * fft_flops(N) * B),
        # write the conj(P) g_Phi patch on the disk; 'rows' forward DFTs
        "rows_backward": (8.0 * S * B, rows * fft_flops(N) * B),
        # Adam over U: read and write O, m, v (complex64 each); read the B patches
        "update": (48.0 * U + 8.0 * S * B, 0.0),
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


def _psnr(x, ref) -> float:
    import numpy as np
    mse = float(np.mean((x - ref) ** 2))
    peak = float(np.max(np.abs(ref)))
    return float("inf") if mse == 0 else 10.0 * math.log10(peak * peak / mse)


def ring_order(prob) -> "np.ndarray":
    """LEDs from the centre outwards (by |k|, then by angle): the fixed order of
    the sequential one-image-per-update baseline (Eq. 7)."""
    import numpy as np
    k = prob.k
    return np.lexsort((np.arctan2(k[:, 0], k[:, 1]), np.round(np.hypot(k[:, 0], k[:, 1]), 9)))


def multiparam_rate(w, prob, steps: int) -> dict:
    """Throughput of the multi-parameter path on the same workload: fpm_loss_grad
    through the autograd function (object, Zernikes, defocus, LED-array
    geometry, sub-pixel crop) and torch Adam on every group, per random batch."""
    import numpy as np
    import torch
    from paper_2408_13782_amd import fpm, inputs, problem
    from paper_2408_13782_amd.autograd import FPMLoss, LossContext
    plan = prob.plan
    grid = fpm.LedGrid(w.n_side, w.pitch_mm, w.height_mm)
    O = problem.initial_spectrum(prob).clone().requires_grad_(True)
    c = torch.zeros(15, dtype=torch.float32, device="cuda", requires_grad=True)
    z = torch.zeros(1, dtype=torch.float32, device="cuda", requires_grad=True)
    geom = torch.zeros(4, dtype=torch.float64, device="cuda", requires_grad=True)
    opt = torch.optim.Adam([dict(params=[O], lr=w.lr_object), dict(params=[c], lr=w.lr_zernike),
                            dict(params=[z], lr=w.lr_z), dict(params=[geom], lr=1e-3)])
    batches = problem.schedule(inputs.led_permutations(w.n_led, -(-(steps + 10) // w.steps_per_epoch()),
                                                      seed=1), w.batch)
    A = prob.meas_amp

    def one(leds):
        opt.zero_grad(set_to_none=False)
        loss = FPMLoss.apply(O, c, z, geom, None, LossContext(plan, grid, leds, A))
        loss.backward()
        opt.step()

    for leds in batches[:10]:
        one(leds)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    n_img = 0
    for leds in batches[10:10 + steps]:
        one(leds)
        n_img += len(leds)
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1)
    # the same groups through the fused multi-parameter step
    st = fpm.State(plan, problem.initial_spectrum(prob))
    geo = fpm.Geometry(lr_shift_mm=1e-3, lr_rot_rad=1e-3, lr_height_mm=1e-3)
    hp = fpm.HParams(lr_object=w.lr_object, lr_zernike=w.lr_zernike, lr_z=w.lr_z,
                     learn_zernike=True, learn_z=True)
    ds = problem.flatten_schedule(batches[:10 + steps])
    plan.run_multi(grid, st, geo, hp, *ds.span(0, 10), A)
    torch.cuda.synchronize()
    e0.record()
    plan.run_multi(grid, st, geo, hp, *ds.span(10, 10 + steps), A)
    e1.record()
    torch.cuda.synchronize()
    ms_f = e0.elapsed_time(e1)
    return {"led_images_per_s": n_img / (ms / 1e3), "ms_per_step": ms / steps,
            "path": "fpm_loss_grad + torch.autograd + torch.optim.Adam (object, Zernike, "
                    "defocus, LED-array geometry)",
            "fused_led_images_per_s": n_img / (ms_f / 1e3), "fused_ms_per_step": ms_f / steps}


def batch_sweep(w, batches, epochs: int, log) -> dict:
    """Random batches of several sizes (Eqs. 13-14) and the sequential fixed-order
    loop (Eq. 7) on the same synthetic data: quality of the object after each
    epoch against wall-clock time on the GPU (evaluation not timed). A batch
    size of 0 stands for all LEDs: one full-gradient step per epoch (Eq. 6)."""
    import numpy as np
    import torch
    from paper_2408_13782_amd import fpm, inputs, problem
    batches = [w.n_led if b <= 0 else min(b, w.n_led) for b in batches]
    prob = problem.make_plan(w, max_batch=max(batches))
    problem.simulate(prob, seed=0)
    plan = prob.plan
    o_true = plan.hr_transform(prob.O_true, -1).cpu().numpy()
    O0 = problem.initial_spectrum(prob)
    hp = problem.hparams(w)
    runs = [("full" if b == w.n_led else "random", b) for b in batches] + [("sequential", 1)]
    out = []
    for mode, B in runs:
        if mode != "sequential":
            perms = inputs.led_permutations(w.n_led, epochs, seed=0)
        else:
            perms = np.tile(ring_order(prob), (epochs, 1)).astype(np.int32)
        per_epoch = -(-w.n_led // B)
        sched = problem.flatten_schedule(problem.schedule(perms, B))
        st = fpm.State(plan, O0)
        t_ms, amp_db, ph_db, loss = 0.0, [], [], []
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        for ep in range(epochs):
            st.loss.zero_()
            torch.cuda.synchronize()
            flat, sizes = sched.span(ep * per_epoch, (ep + 1) * per_epoch)
            e0.record()
            plan.run(st, hp, flat, sizes, prob.meas_amp)
            e1.record()
            torch.cuda.synchronize()
            t_ms += e0.elapsed_time(e1)
            o = plan.hr_transform(st.O, -1).cpu().numpy()
            o = o * np.exp(1j * np.angle(np.vdot(o, o_true)))       # global phase
            amp_db.append(_psnr(np.abs(o), np.abs(o_true)))
            ph_db.append(_psnr(np.angle(o), np.angle(o_true)))
            loss.append(float(st.loss.cpu()[0]))
        row = {"mode": mode, "batch": B, "steps_per_epoch": per_epoch,
               "ms_per_epoch": t_ms / epochs, "total_ms": t_ms,
               "amp_psnr_db": amp_db, "phase_psnr_db": ph_db, "epoch_loss": loss}
        log(f"{mode} B={B}: {t_ms / epochs:.2f} ms/epoch, final amplitude {amp_db[-1]:.2f} dB, "
            f"phase {ph_db[-1]:.2f} dB")
        out.append(row)
    return {"workload": w.name, "epochs": epochs, "runs": out}


def main():
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=450)
    ap.add_argument("--warmup", type=int, default=30)
    ap.add_argument("--workload", default="paper", choices=["small", "paper", "large"])
    ap.add_argument("--profile-steps", type=int, default=24,
                    help="steps of the per-kernel timing pass (after the main timing)")
    ap.add_argument("--copy-probe-mb", type=int, default=0,
                    help="after timing, one device-to-device copy of this size (a kernel of "
                         "known traffic for calibrating HBM counters)")
    ap.add_argument("--cpu-seconds", type=float, default=15.0)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--batch-sweep", type=int, nargs="*", default=None,
                    help="instead of the throughput line: quality vs time for these batch "
                         "sizes and the sequential loop (e.g. --batch-sweep 1 8 16 40 0; "
                         "0 = all LEDs, the full gradient)")
    ap.add_argument("--sweep-epochs", type=int, default=30)
    ap.add_argument("--serving-requests", type=int, default=150,
                    help="requests of the tile-serving latency measurement at rho = 0.9 "
                         "(0: skip)")
    args = ap.parse_args()
    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print("bench.py measures one GPU: the library has no multi-GPU path "
              "(tiles of the field of view are independent and would shard one per GPU); "
              "run with --gpus 1", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    from paper_2408_13782_amd import fpm, inputs, problem

    torch.cuda.set_device(0)
    w = inputs.workload(args.workload)
    if args.batch_sweep:
        print(json.dumps(batch_sweep(w, args.batch_sweep, args.sweep_epochs, log)), flush=True)
        return
    log(f"workload {w.name}: {w.n_side}x{w.n_side} LEDs, N={w.n_lr}, M={w.m_hr}, B={w.batch}")
    # workloads that learn the LED-array geometry: data from the true (seeded)
    # geometry, solved from the nominal grid with the fused multi-parameter step
    true_geom = inputs.true_geometry(w, 0) if w.learn_geometry else (0.0, 0.0, 0.0, 0.0)
    prob = problem.make_plan(w, geometry=true_geom)
    problem.simulate(prob, seed=0)
    O0 = problem.initial_spectrum(prob)
    state = fpm.State(prob.plan, O0)
    hp = problem.hparams(w)
    plan = prob.plan
    grid = fpm.LedGrid(w.n_side, w.pitch_mm, w.height_mm)
    geometry = fpm.Geometry(lr_shift_mm=w.lr_shift, lr_rot_rad=w.lr_rot, lr_height_mm=w.lr_height)
    total = args.warmup + args.steps + args.profile_steps
    epochs = -(-total // w.steps_per_epoch())
    batches = problem.schedule(inputs.led_permutations(w.n_led, epochs, seed=0), w.batch)
    ds = problem.flatten_schedule(batches[:total])
    A = prob.meas_amp
    torch.cuda.synchronize()
    log("set-up done")

    def run(start, stop):
        flat, sizes = ds.span(start, stop)
        if w.learn_geometry:
            plan.run_multi(grid, state, geometry, hp, flat, sizes, A)
        else:
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

    # Per-kernel durations: for each step kernel in turn, every launch of it is
    # issued REPS times back to back between two events on the launch stream, on
    # the step's real operands (the repeated launches leave the state invalid;
    # nothing after this pass reads it).
    REPS = 20
    per_pass = max(1, args.profile_steps // 4)
    work, U = kernel_work(plan, w.batch)
    timed = {}
    start = args.warmup + args.steps
    for i, kind in enumerate(work):
        plan.timing_repeat(kind, REPS)
        plan.timing(True)
        run(start + i * per_pass, start + (i + 1) * per_pass)
        torch.cuda.synchronize()
        plan.timing(False)
        kt = plan.timing_collect()
        timed[kind] = kt[kind][0] / kt[kind][1]              # ms per launch
    plan.timing_repeat(None, 1)
    log("per-kernel mean us: " + ", ".join(f"{k}={v * 1e3:.2f}" for k, v in timed.items()))
    B = w.batch
    dominant = max(timed, key=lambda k: timed[k])
    bytes_, flops = work[dominant]
    dur_s = timed[dominant] / 1e3
    ridge = FP32_VALU_PEAK_TFLOPS * 1e12 / (HBM_PEAK_GBS * 1e9)     # flop per byte
    if flops / bytes_ > ridge:
        achieved = flops / dur_s / 1e12
        roof = {"bound": "alu", "achieved": achieved, "peak": FP32_VALU_PEAK_TFLOPS,
                "unit": "TFLOP/s", "frac": achieved / FP32_VALU_PEAK_TFLOPS,
                "traffic": TRAFFIC.get((w.name, dominant)), "kernel": dominant,
                "mean_us": timed[dominant] * 1e3,
                "hbm_algorithmic_GBs": bytes_ / dur_s / 1e9}
    else:
        achieved = bytes_ / dur_s / 1e9
        roof = {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": achieved / HBM_PEAK_GBS, "traffic": TRAFFIC.get((w.name, dominant)),
                "kernel": dominant, "mean_us": timed[dominant] * 1e3,
                "algorithmic_bytes": bytes_}
    chain_ms = sum(timed.get(k, 0.0) for k in ("rows_forward", "cols", "rows_backward"))
    S, N = plan.info.support_px, plan.N
    chain_bytes = (16.0 * S + 4.0 * N * N) * B
    detail = {
        "fwd_bwd_us_per_batch": chain_ms * 1e3,
        "fwd_bwd_led_images_per_s": B / (chain_ms / 1e3),
        "fwd_bwd_hbm_frac": chain_bytes / (chain_ms / 1e3) / 1e9 / HBM_PEAK_GBS,
        "per_kernel_mean_us": {k: v * 1e3 for k, v in timed.items()},
        "support_px": S, "union_px": U,
    }
    if not w.learn_geometry:
        detail["multiparam"] = multiparam_rate(w, prob, 100)
        log(f"multi-parameter paths: fused {detail['multiparam']['fused_led_images_per_s']:.4g}, "
            f"autograd {detail['multiparam']['led_images_per_s']:.4g} LED-images/s")
    # digital refocusing of the reconstruction: 16 distances in [-40, 40] um
    z = torch.linspace(-40.0, 40.0, 16, dtype=torch.float32, device="cuda")
    foc = torch.empty((16, plan.M, plan.M), dtype=torch.complex64, device="cuda")
    plan.refocus(state.O, z, out=foc)
    r0, r1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    r0.record()
    for _ in range(5):
        plan.refocus(state.O, z, out=foc)
    r1.record()
    torch.cuda.synchronize()
    detail["refocus_16z_ms"] = r0.elapsed_time(r1) / 5
    del foc

    result = {
        "metric": "LED-images fwd+bwd/sec (256²→1024²)" if w.name == "paper" else
                  f"LED-images fwd+bwd/sec ({w.n_lr}²→{w.m_hr}²)",
        "value": value, "unit": "LED-images/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": ms / args.steps, "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f32", "data": "synthetic",
        "config": {"workload": f"{w.name}: {w.n_side}x{w.n_side} LEDs, {w.n_lr}^2 LR -> "
                               f"{w.m_hr}^2 HR, batch {w.batch}, object"
                               + (" + Zernike pupil" if w.learn_zernike else "")
                               + (" + defocus" if w.learn_z else "")
                               + (" + LED-array geometry (fused multi-parameter step)"
                                  if w.learn_geometry else ""),
                   "n_led": w.n_led, "n_lr": w.n_lr, "m_hr": w.m_hr, "batch": w.batch},
        "roofline": roof,
        "detail": detail,
    }
    if args.serving_requests > 0:
        from paper_2408_13782_amd import serving
        log(f"tile serving: {args.serving_requests} requests at 0.9 x the sequential rate")
        sres = serving.measure(rates=(0.9,), n_requests=args.serving_requests, lanes=4,
                               calib_requests=40, log=log)
        row = sres["rates"][0]
        result["serving"] = {
            "workload": "Poisson stream of tile solves, N in {128,192,256,384,512}, "
                        "7x7/11x11/15x15 LEDs, 4x upsampling, 20 epochs of B=16, "
                        "object + Zernike pupil",
            "requests": args.serving_requests, "rho": row["rho"],
            "arrival_rate_per_s": row["rate_per_s"], "mu_seq_per_s": sres["mu_seq_per_s"],
            "lanes": sres["lanes"],
            "p50_ms": row["server"]["p50_ms"], "p99_ms": row["server"]["p99_ms"],
            "requests_per_s": row["server"]["requests_per_s"],
            "sequential_p50_ms": row["sequential"]["p50_ms"],
            "sequential_p99_ms": row["sequential"]["p99_ms"],
            "sequential_requests_per_s": row["sequential"]["requests_per_s"],
        }
    if not args.no_cpu_baseline:
        log(f"oracle CPU baseline (~{args.cpu_seconds:.0f} s)")
        result["cpu_baseline"] = cpu_baseline(w, args.cpu_seconds)
        log("oracle CPU baseline done")
    print(json.dumps(result), flush=True)


if __name__ == "__main__":
    main()
