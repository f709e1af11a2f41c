"""Reconstruction problems on the GPU: plan set-up, synthetic measurements,
the random-batch schedule and the solve loop (Sec. 2.3, Eqs. 13-14).

Host code here only orders work: LED geometry goes through libfpm's FP64
host routine, every array operation of the method runs in libfpm's kernels.
Photon noise for synthetic data is drawn with torch on the device (input
synthesis, not part of the method).
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np

from . import fpm, inputs


@dataclass
class Problem:
    workload: inputs.Workload
    plan: fpm.Plan
    k: np.ndarray            # [n_led, 2] LED spatial frequencies, 1/um
    shifts: np.ndarray       # [n_led, 2] int32 spectral offsets
    bright: np.ndarray       # [n_led] bool, illumination inside the NA
    meas_amp: object = None  # torch float32 [n_led, N, N]
    O_true: object = None    # torch complex64 [M, M]
    P_true: object = None    # torch complex64 [N, N]
    z_true: float = 0.0


def make_plan(w: inputs.Workload, max_batch: int | None = None, geometry=(0.0, 0.0, 0.0, 0.0)
              ) -> Problem:
    """Plan of a workload; geometry = (dx_mm, dy_mm, rot_rad, dh_mm) of the LED array."""
    dx, dy, rot, dh = geometry
    k, _, nearest = fpm.led_shifts(w.n_lr, w.wavelength_um, w.mag, w.pixel_um, w.n_side,
                                   w.pitch_mm, w.height_mm, dx, dy, rot, dh)
    plan = fpm.Plan(w.n_lr, w.upsample, nearest, max_batch or w.batch, w.wavelength_um, w.na,
                    w.mag, w.pixel_um)
    bright = np.hypot(k[:, 0], k[:, 1]) <= w.na / w.wavelength_um
    return Problem(w, plan, k, nearest, bright)


def simulate(prob: Problem, seed: int = 0, device="cuda"):
    """Synthetic measurements: truth object through the forward model plus Poisson noise.

    Uses the true defocus of the workload (seeded) and, when the workload has
    LED-geometry errors, the plan's LED table must already be the true one.
    """
    import torch
    w = prob.workload
    plan = prob.plan
    amp, ph = inputs.truth_object(w.m_hr, seed)
    o = torch.as_tensor((amp * np.exp(1j * ph)).astype(np.complex64), device=device)
    O_true = plan.hr_transform(o, +1)
    z_true = inputs.true_defocus(w, seed)
    P_true = plan.pupil(None, torch.tensor([z_true], dtype=torch.float32, device=device))
    A = torch.empty((w.n_led, w.n_lr, w.n_lr), dtype=torch.float32, device=device)
    all_leds = np.arange(w.n_led, dtype=np.int32)
    for start in range(0, w.n_led, plan.max_batch):
        leds = all_leds[start:start + plan.max_batch]
        A[start:start + leds.size] = plan.forward(O_true, P_true, leds)
    q = torch.as_tensor(np.where(prob.bright, w.q_bright, w.q_dark).astype(np.float32),
                        device=device).view(-1, 1, 1)
    gen = torch.Generator(device=device)
    gen.manual_seed(1000 + seed)
    counts = torch.poisson(A * A * q, generator=gen)
    prob.meas_amp = torch.sqrt(counts / q).contiguous()
    prob.O_true, prob.P_true, prob.z_true = O_true, P_true, z_true
    return prob


def centre_led(w: inputs.Workload) -> int:
    return (w.n_side // 2) * w.n_side + w.n_side // 2


def initial_spectrum(prob: Problem):
    """Spectrum of the bilinearly upsampled centre-LED amplitude (Sec. 2.3)."""
    return prob.plan.init_spectrum(prob.meas_amp[centre_led(prob.workload)].contiguous())


def schedule(perms: np.ndarray, batch: int):
    """Balanced random batches (Eq. 14): each epoch's LED order cut into batches of B."""
    out = []
    for perm in np.asarray(perms, np.int32):
        for start in range(0, perm.size, batch):
            out.append(perm[start:start + batch])
    return out


def hparams(w: inputs.Workload) -> fpm.HParams:
    return fpm.HParams(lr_object=w.lr_object, lr_zernike=w.lr_zernike, lr_z=w.lr_z,
                       learn_zernike=w.learn_zernike, learn_z=w.learn_z)


@dataclass
class Schedule:
    """All batches of a solve back to back (host int32; the library takes host ids)."""
    flat: np.ndarray        # int32 [sum of batch sizes]
    sizes: np.ndarray       # int32 [n_steps]
    offsets: np.ndarray     # int64 [n_steps + 1]

    def view(self, i: int) -> np.ndarray:
        return self.flat[self.offsets[i]:self.offsets[i + 1]]

    def span(self, start: int, stop: int):
        """(ids, sizes) of steps start..stop-1, for Plan.run."""
        return self.flat[self.offsets[start]:self.offsets[stop]], self.sizes[start:stop]

    def __len__(self):
        return len(self.sizes)


def flatten_schedule(batches) -> Schedule:
    sizes = np.array([len(b) for b in batches], np.int32)
    offsets = np.concatenate([[0], np.cumsum(sizes)]).astype(np.int64)
    flat = np.ascontiguousarray(np.concatenate(batches).astype(np.int32))
    return Schedule(flat, sizes, offsets)


def solve(prob: Problem, state: fpm.State, hp: fpm.HParams, sched: Schedule, gamma=None):
    """Run every random-batch update of the schedule in one library call."""
    flat, sizes = sched.span(0, len(sched))
    prob.plan.run(state, hp, flat, sizes, prob.meas_amp, gamma)
    return state
