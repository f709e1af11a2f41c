"""Reconstruct an object from a stack of FPM images on disk (Sec. 2.3).

The images are one per LED of a square array, row-major LED order (the LED at
column i, row j of the grid is image j * n_side + i), as amplitudes
(sqrt of the recorded intensity) or, with --intensity-images, as intensities.
The solve is the random-batch update of Eq. 13 with Adam: each epoch a fresh
random order of all LEDs cut into batches of B (Eq. 14), starting from the
upsampled centre-LED amplitude.

    python -m paper_2408_13782_amd.reconstruct --images stack.npy --grid 15 \\
        --pitch-mm 4 --height-mm 90 --wavelength-um 0.532 --na 0.1 --mag 4 \\
        --pixel-um 6.5 --upsample 4 --batch 16 --epochs 30 --learn-zernike \\
        --out result.npz

The output holds the complex object (M x M), its spectrum, the pupil, the
Zernike coefficients and defocus, and the loss of every epoch.
"""
from __future__ import annotations

import argparse
import json
import sys

import numpy as np

from . import fpm, inputs, problem


def parse(argv=None):
    ap = argparse.ArgumentParser(description="FPM reconstruction from an image stack")
    ap.add_argument("--images", required=True, help=".npy float array [n_led, N, N]")
    ap.add_argument("--intensity-images", action="store_true",
                    help="the stack holds intensities (their square roots are used)")
    ap.add_argument("--grid", type=int, required=True, help="LEDs per side (n_led = grid^2)")
    ap.add_argument("--pitch-mm", type=float, required=True)
    ap.add_argument("--height-mm", type=float, required=True)
    ap.add_argument("--roi-x-mm", type=float, default=0.0,
                    help="sample-plane position of the image centre (tiles of a larger field)")
    ap.add_argument("--roi-y-mm", type=float, default=0.0)
    ap.add_argument("--wavelength-um", type=float, required=True)
    ap.add_argument("--na", type=float, required=True)
    ap.add_argument("--mag", type=float, required=True)
    ap.add_argument("--pixel-um", type=float, required=True, help="camera pixel pitch")
    ap.add_argument("--upsample", type=int, default=4)
    ap.add_argument("--batch", type=int, default=16)
    ap.add_argument("--epochs", type=int, default=30)
    ap.add_argument("--lr-object", type=float, default=1e-2)
    ap.add_argument("--lr-zernike", type=float, default=1e-2)
    ap.add_argument("--lr-z", type=float, default=0.1)
    ap.add_argument("--learn-zernike", action="store_true")
    ap.add_argument("--learn-z", action="store_true", help="learn the defocus distance")
    ap.add_argument("--loss", choices=["amplitude", "intensity"], default="amplitude")
    ap.add_argument("--seed", type=int, default=0, help="seed of the batch order")
    ap.add_argument("--out", required=True, help="output .npz")
    return ap.parse_args(argv)


def reconstruct(args, images: np.ndarray):
    """The solve on the current GPU; returns a dict of numpy results."""
    import torch
    stack = np.asarray(images, np.float32)
    n_led, N = args.grid * args.grid, stack.shape[-1]
    if stack.shape != (n_led, N, N):
        raise ValueError(f"images must have shape ({n_led}, N, N), got {stack.shape}")
    if args.intensity_images:
        stack = np.sqrt(np.maximum(stack, 0.0))
    _, _, shifts = fpm.led_shifts(N, args.wavelength_um, args.mag, args.pixel_um, args.grid,
                                  args.pitch_mm, args.height_mm, roi_x_mm=args.roi_x_mm,
                                  roi_y_mm=args.roi_y_mm)
    batch = min(args.batch, n_led)
    plan = fpm.Plan(N, args.upsample, shifts, batch, args.wavelength_um, args.na, args.mag,
                    args.pixel_um)
    plan.set_loss(args.loss)
    A = torch.as_tensor(np.ascontiguousarray(stack), device="cuda")
    centre = (args.grid // 2) * args.grid + args.grid // 2
    state = fpm.State(plan, plan.init_spectrum(A[centre].contiguous()))
    hp = fpm.HParams(lr_object=args.lr_object, lr_zernike=args.lr_zernike, lr_z=args.lr_z,
                     learn_zernike=args.learn_zernike, learn_z=args.learn_z)
    perms = inputs.led_permutations(n_led, args.epochs, seed=args.seed)
    sched = problem.flatten_schedule(problem.schedule(perms, batch))
    per_epoch = -(-n_led // batch)
    losses = []
    for ep in range(args.epochs):
        state.loss.zero_()
        flat, sizes = sched.span(ep * per_epoch, (ep + 1) * per_epoch)
        plan.run(state, hp, flat, sizes, A)
        losses.append(float(state.loss.cpu()[0]))
    torch.cuda.synchronize()
    return {"object": plan.hr_transform(state.O, -1).cpu().numpy(),
            "spectrum": state.O.cpu().numpy(), "pupil": state.P.cpu().numpy(),
            "zernike": state.coeffs.cpu().numpy(), "z_um": state.z_um.cpu().numpy(),
            "epoch_loss": np.asarray(losses)}


def main(argv=None):
    args = parse(argv)
    import torch
    torch.cuda.set_device(0)
    res = reconstruct(args, np.load(args.images, allow_pickle=False))
    np.savez(args.out, **res)
    print(json.dumps({"out": args.out, "m_hr": int(res["object"].shape[0]),
                      "final_loss": res["epoch_loss"][-1]}), flush=True)
    print(f"[reconstruct] {args.epochs} epochs, loss {res['epoch_loss'][0]:.4g} -> "
          f"{res['epoch_loss'][-1]:.4g}", file=sys.stderr, flush=True)


if __name__ == "__main__":
    main()
