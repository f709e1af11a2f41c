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
  value        LED-images per second through whole steps (the fwd+bwd chain,
               Adam on the spectrum, the pupil-parameter update), timed over
               the K steps; `fwd_bwd` gives the chain alone
  roofline     the fwd+bwd chain (rows_forward + cols + rows_backward): its
               algorithmic bytes per batch, (16 |S| + 4 N^2) B, over the sum of
               the three kernels' mean durations (HIP events on the launch
               stream around 20 back-to-back launches of each on a step's
               operands) vs the HBM peak; every kernel's own figures in
               detail.kernels. `traffic` is what the rocprofv3 counters of
               profiles/hbm_traffic.md measured, if they were taken on the
               loaded build (fpm_build_tag), else null
  cpu_baseline the FP64 oracle's steps on the same workload, host cores
               (scipy.fft worker threads; numpy one thread beside it)
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


def load_traffic(workload: str, build_tag: str):
    """HBM bytes per launch of each step kernel from the committed rocprofv3
    counter summary (profiles/hbm_traffic.md: FETCH_SIZE and WRITE_SIZE in KiB per
    dispatch, with the counts a device copy of known size reads on them), or None
    if those counters were taken on another build of the library."""
    path = os.path.join(ROOT, "profiles", "hbm_traffic.md")
    try:
        text = open(path).read()
        block = text.split("```json", 1)[1].split("```", 1)[0]
        data = json.loads(block)
    except (OSError, IndexError, ValueError):
        return None
    if data.get("build") != build_tag or workload not in data.get("workloads", {}):
        return None
    cal = data["calibration"]
    f_fetch = cal["copy_read_kib"] / cal["fetch_kib"]     # bytes read per FETCH_SIZE unit
    f_write = cal["copy_written_kib"] / cal["write_kib"]
    return {k: (v["fetch_kib"] * f_fetch + v["write_kib"] * f_write) * 1024.0
            for k, v in data["workloads"][workload].items()}


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
    if plan.info.fused_chain:
        # the loss and its adjoint in one launch (crop, both 2-D transforms of the
        # disk rows and all columns, the patch write): the chain's bytes and flops
        chain = (16.0 * S * B + 4.0 * N * N * B, (2 * rows + 2 * N) * fft_flops(N) * B)
        return {"chain_fused": chain, "update": (48.0 * U + 8.0 * S * B, 0.0)}, U
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


def host_cpu() -> dict:
    """The host's CPU model and the cores this process may run on."""
    model = "unknown"
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    try:
        usable = len(os.sched_getaffinity(0))
    except AttributeError:
        usable = os.cpu_count() or 1
    return {"model": model, "cpu_count": os.cpu_count(), "usable_cores": usable}


def cpu_baseline(w, seconds: float):
    """Time the FP64 oracle's full steps on the same workload (bounded samples).

    The oracle builds its own inputs (truth object, measurements through its
    forward model, seeded Poisson noise, initial value); set-up is not timed.
    Two modes: its 2-D FFTs on scipy.fft with one worker thread per usable core
    (the reported value), and numpy's single-threaded FFT.
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
    perms = inputs.led_permutations(w.n_led, 12, seed=0)
    sched = fo.batches_from_permutations(perms, w.batch)
    host = host_cpu()

    def timed_steps(workers):
        fo.set_fft_workers(workers)
        st = fo.init_state(O0)
        n_img, n_steps = 0, 0
        t0 = time.perf_counter()
        while n_steps < len(sched) and (time.perf_counter() - t0 < seconds or n_steps < 3):
            fo.step(st, cfg, mask, zern, kappa, shifts, sched[n_steps], A)
            n_img += len(sched[n_steps])
            n_steps += 1
        dt = time.perf_counter() - t0
        fo.set_fft_workers(1)
        return n_img / dt, n_steps, n_img, dt

    workers = host["usable_cores"]
    v_mt, s_mt, i_mt, t_mt = timed_steps(workers)
    v_1, s_1, i_1, t_1 = timed_steps(1)
    return {"value": v_mt, "unit": "LED-images/s", "cores": workers, "kind": "oracle",
            "sample": f"{s_mt} full FP64 steps ({i_mt} LED-images) of the same workload, "
                      f"2-D FFTs on scipy.fft with {workers} worker threads (the rest of the "
                      f"oracle's numpy arithmetic on one thread), {t_mt:.1f} s",
            "host": host,
            "single_thread": {"value": v_1, "unit": "LED-images/s", "cores": 1,
                              "sample": f"{s_1} full FP64 steps ({i_1} LED-images), numpy.fft, "
                                        f"one thread, {t_1:.1f} s"}}


def _psnr(x, ref) -> float:
    import numpy as np
    mse = float(np.mean((x - ref) ** 2))
    peak = float(np.max(np.abs(ref)))
    return float("inf") if mse == 0 else 10.0 * math.log10(peak * peak / mse)


def full_solves(w, prob, hp, warm: int = 2, timed: int = 5) -> dict:
    """The whole solve of the workload (every epoch's random batches, Eqs.
    13-14) from its initial spectrum, `warm` untimed then `timed` timed runs
    (HIP events around each, inputs resident): the median and every time."""
    import numpy as np
    import torch
    from paper_2408_13782_amd import fpm, inputs, problem
    plan = prob.plan
    sched = problem.flatten_schedule(problem.schedule(
        inputs.led_permutations(w.n_led, w.epochs, seed=0), w.batch))
    n_img = int(sched.sizes.sum())
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    times = []
    for r in range(warm + timed):
        st = fpm.State(plan, problem.initial_spectrum(prob))
        go = plan.prepare_run(st, hp, sched.flat, sched.sizes, prob.meas_amp)
        torch.cuda.synchronize()
        e0.record()
        go()
        e1.record()
        torch.cuda.synchronize()
        if r >= warm:
            times.append(e0.elapsed_time(e1))
    med = float(np.median(times))
    return {"steps": int(sched.sizes.size), "led_images": n_img, "ms_median": med,
            "ms_all": times, "led_images_per_s": n_img / (med / 1e3)}


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


def chain_by_batch(w, batches=(16, 64)) -> list:
    """The fwd+bwd chain's time per batch at several batch sizes on the same
    workload shape (plans of their own, 6 steps per kernel bracket of 20
    back-to-back launches): how much of the batch-of-16 time is the fixed cost
    of the launches and their dependent latencies."""
    import torch
    from paper_2408_13782_amd import fpm, inputs, problem
    from dataclasses import replace
    out = []
    for B in [b for b in batches if b <= w.n_led]:   # a batch of at most every LED
        wb = replace(w, batch=B)
        prob = problem.make_plan(wb)
        problem.simulate(prob, seed=0)
        plan = prob.plan
        st = fpm.State(plan, problem.initial_spectrum(prob))
        hp = problem.hparams(wb)
        epochs = -(-40 // (wb.n_led // B))        # 40 whole batches: 10 + 6 per kernel kind
        full = [b for b in problem.schedule(inputs.led_permutations(wb.n_led, epochs, seed=0), B)
                if len(b) == B]                      # whole batches only
        sched = problem.flatten_schedule(full)
        plan.run(st, hp, *sched.span(0, 10), prob.meas_amp)
        kinds = (("chain_fused",) if plan.info.fused_chain
                 else ("rows_forward", "cols", "rows_backward"))
        us = 0.0
        for i, kind in enumerate(kinds):
            plan.timing_repeat(kind, 20)
            plan.timing(True)
            plan.run(st, hp, *sched.span(10 + 6 * i, 16 + 6 * i), prob.meas_amp)
            torch.cuda.synchronize()
            plan.timing(False)
            kt = plan.timing_collect()
            us += 1e3 * kt[kind][0] / kt[kind][1]
        plan.timing_repeat(None, 1)
        S, N = plan.info.support_px, plan.N
        alg = (16.0 * S + 4.0 * N * N) * B
        out.append({"batch": B, "chain_us": us, "led_images_per_s": B / (us * 1e-6),
                    "hbm_frac": alg / (us * 1e-6) / 1e9 / HBM_PEAK_GBS})
        del prob, plan, st
    return out


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
            perms = np.tile(inputs.centre_out_order(prob.k), (epochs, 1)).astype(np.int32)
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
    ap.add_argument("--cpu-seconds", type=float, default=10.0,
                    help="seconds of oracle steps per CPU-baseline mode")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--batch-sweep", type=int, nargs="*", default=None,
                    help="instead of the throughput line: quality vs time for these batch "
                         "sizes and the sequential loop (e.g. --batch-sweep 1 8 16 40 0; "
                         "0 = all LEDs, the full gradient)")
    ap.add_argument("--sweep-epochs", type=int, default=30)
    ap.add_argument("--serving-requests", type=int, default=2000,
                    help="requests per arrival rate of the tile-serving latency measurement "
                         "(0: skip)")
    ap.add_argument("--serving-rates", type=float, nargs="+", default=[0.5, 0.9, 1.5],
                    help="arrival rates as multiples of the sequential service rate")
    ap.add_argument("--no-detail-sweep", dest="sweep_in_detail", action="store_false",
                    help="skip the batch-size legs of the line's detail (the reduced "
                         "sweep and the chain at batches of 16 and 64)")
    ap.add_argument("--detail-sweep-epochs", type=int, default=5)
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
    # the timed steps' batches, images and hyper-parameters are checked and
    # marshalled before the timed region (Plan.prepare_run); the state is read
    # and checked at the call
    if w.learn_geometry:
        go = lambda: run(args.warmup, args.warmup + args.steps)   # noqa: E731
    else:
        go = plan.prepare_run(state, hp, *ds.span(args.warmup, args.warmup + args.steps), A)
    torch.cuda.synchronize()
    t_start.record(stream)
    go()
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
    traffic = load_traffic(w.name, fpm.build_tag())
    kernels = {}
    for k, (bytes_, flops) in work.items():
        dur_s = timed[k] / 1e3
        kernels[k] = {"mean_us": timed[k] * 1e3, "algorithmic_bytes": bytes_, "flops": flops,
                      "hbm_frac": bytes_ / dur_s / 1e9 / HBM_PEAK_GBS,
                      "valu_frac": flops / dur_s / 1e12 / FP32_VALU_PEAK_TFLOPS,
                      "traffic": traffic.get(k) if traffic else None}
    # the headline roofline: the fwd+bwd chain (a3-a7) of one batch
    chain = (("chain_fused",) if plan.info.fused_chain
             else ("rows_forward", "cols", "rows_backward"))
    chain_s = sum(timed[k] for k in chain) / 1e3
    S, N = plan.info.support_px, plan.N
    chain_bytes = (16.0 * S + 4.0 * N * N) * B
    chain_flops = sum(work[k][1] for k in chain)
    achieved = chain_bytes / chain_s / 1e9
    roof = {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": achieved / HBM_PEAK_GBS,
            "traffic": sum(traffic[k] for k in chain) if traffic else None,
            "kernel": " + ".join(chain) + " (the fwd+bwd chain of one batch)",
            "mean_us": chain_s * 1e6, "algorithmic_bytes": chain_bytes,
            "valu_tflops": chain_flops / chain_s / 1e12,
            "valu_frac": chain_flops / chain_s / 1e12 / FP32_VALU_PEAK_TFLOPS,
            "build": fpm.build_tag()}
    fwd_bwd = {"led_images_per_s": B / chain_s, "us_per_batch": chain_s * 1e6,
               "timing": "sum of the chain kernels' mean durations (HIP events on the "
                         "launch stream around 20 back-to-back launches of each)"}
    detail = {
        "kernels": kernels,
        "step_us_from_kernels": sum(timed.values()) * 1e3,
        "support_px": S, "union_px": U,
    }
    if not w.learn_geometry:
        detail["full_solve"] = full_solves(w, prob, hp)
        fs = detail["full_solve"]
        log(f"whole solve ({fs['steps']} steps, {fs['led_images']} LED-images): median of 5 "
            f"{fs['ms_median']:.2f} ms, {fs['led_images_per_s']:.4g} LED-images/s")
        if args.sweep_in_detail:
            detail["fwd_bwd_by_batch"] = chain_by_batch(w, (16, 64))
            log("fwd+bwd chain by batch: " + ", ".join(
                f"B={r['batch']}: {r['chain_us']:.1f} us ({r['hbm_frac'] * 100:.1f} % of HBM)"
                for r in detail["fwd_bwd_by_batch"]))
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

    metric = ("LED-images fwd+bwd/sec (256²→1024²); HBM roofline %; tile p50/p99 ms"
              if w.name == "paper" else f"LED-images fwd+bwd/sec ({w.n_lr}²→{w.m_hr}²)")
    result = {
        "metric": metric,
        "value": value, "unit": "LED-images/s",
        "value_is": "LED-images through whole random-batch steps (fwd+bwd chain, Adam on the "
                    "spectrum, pupil-parameter update) per second over the timed steps",
        "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": ms / args.steps, "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f32", "data": "synthetic",
        "config": {"workload": f"{w.name}: {w.n_side}x{w.n_side} LEDs, {w.n_lr}^2 LR -> "
                               f"{w.m_hr}^2 HR, batch {w.batch}, object"
                               + (" + Zernike pupil" if w.learn_zernike else "")
                               + (" + defocus" if w.learn_z else "")
                               + (" + LED-array geometry (fused multi-parameter step)"
                                  if w.learn_geometry else ""),
                   "n_led": w.n_led, "n_lr": w.n_lr, "m_hr": w.m_hr, "batch": w.batch},
        "fwd_bwd": fwd_bwd,
        "roofline": roof,
        "detail": detail,
    }
    if args.serving_requests > 0:
        from paper_2408_13782_amd import serving
        rates = tuple(args.serving_rates)
        log(f"tile serving: {args.serving_requests} requests at rho = {rates} x the "
            "sequential rate")
        sres = serving.measure(rates=rates, n_requests=args.serving_requests, lanes=4,
                               calib_requests=40, log=log)
        rows = []
        for row in sres["rates"]:
            rows.append({"rho": row["rho"], "arrival_rate_per_s": row["rate_per_s"],
                         "p50_ms": row["server"]["p50_ms"], "p99_ms": row["server"]["p99_ms"],
                         "requests_per_s": row["server"]["requests_per_s"],
                         "sequential_p50_ms": row["sequential"]["p50_ms"],
                         "sequential_p99_ms": row["sequential"]["p99_ms"],
                         "sequential_requests_per_s": row["sequential"]["requests_per_s"]})
        result["serving"] = {
            "workload": "Poisson stream of tile solves, N in {128,192,256,384,512}, "
                        "7x7/11x11/15x15 LEDs, 4x upsampling, 20 epochs of B=16, "
                        "object + Zernike pupil",
            "requests_per_rate": args.serving_requests, "mu_seq_per_s": sres["mu_seq_per_s"],
            "lanes": sres["lanes"], "sequential": "the same server with one lane (FIFO, one "
                                                  "request at a time)",
            "rates": rows,
        }
    if args.sweep_in_detail:
        log("reduced batch-size sweep (B = 1, 16, all; sequential order), "
            f"{args.detail_sweep_epochs} epochs")
        sw = batch_sweep(w, [1, w.batch, 0], args.detail_sweep_epochs, log)
        detail["batch_sweep"] = {
            "epochs": sw["epochs"],
            "runs": [{"mode": r["mode"], "batch": r["batch"],
                      "ms_per_epoch": r["ms_per_epoch"],
                      "amp_psnr_db": r["amp_psnr_db"], "phase_psnr_db": r["phase_psnr_db"]}
                     for r in sw["runs"]]}
    if not args.no_cpu_baseline:
        log(f"oracle CPU baseline (~{2 * args.cpu_seconds:.0f} s)")
        result["cpu_baseline"] = cpu_baseline(w, args.cpu_seconds)
        log("oracle CPU baseline done")
    print(json.dumps(result), flush=True)


if __name__ == "__main__":
    main()
