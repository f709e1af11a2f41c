"""Seeded synthetic inputs shared by the HIP path, its tests and the oracle.

This module holds no arithmetic of the reconstruction method itself: only the
workload descriptions (optics, LED grid, sizes, hyper-parameters), the
synthetic truth object, the random LED orders the random-batch schedule
draws, and photon noise. The forward model that turns a truth object into
measured images lives on each side separately.

Workloads follow the shapes of the paper's experiments (Sec. 3): a square
LED grid below the sample, 4x objective, low-resolution (LR) camera images
of n_lr x n_lr pixels reconstructed into an upsample*n_lr high-resolution
(HR) object. The paper's ground-truth images, USAF captures and tissue
slides are not available, so a smooth random complex object stands in for
them (amplitude in [0.5, 1], phase in [-pi/2, pi/2]).

Seeds: object 0, noise 1, schedule 2, pupil/geometry truth 3 (per workload
offset by a user seed).
"""
from __future__ import annotations

import math
from dataclasses import dataclass, replace

import numpy as np


@dataclass(frozen=True)
class Workload:
    name: str
    n_side: int            # LEDs per side of the square grid
    pitch_mm: float        # LED spacing
    height_mm: float       # LED-array to sample distance
    wavelength_um: float
    na: float
    mag: float
    pixel_um: float        # camera pixel
    n_lr: int              # LR image side N
    upsample: int          # HR/LR ratio s, M = s N
    batch: int             # LEDs per random batch B
    epochs: int
    q_bright: float        # photons per unit intensity, bright-field LEDs
    q_dark: float          # photons per unit intensity, dark-field LEDs
    lr_object: float = 1e-2
    lr_zernike: float = 1e-2
    lr_z: float = 0.1
    lr_shift: float = 5e-3     # mm
    lr_rot: float = 5e-4       # rad
    lr_height: float = 2e-2    # mm
    n_zernike: int = 15
    learn_zernike: bool = False
    learn_z: bool = False
    learn_geometry: bool = False
    true_defocus_um: float = 0.0          # half-width of the seeded true defocus
    true_shift_mm: float = 0.0            # half-widths of seeded geometry errors
    true_rot_deg: float = 0.0
    true_dh_mm: float = 0.0

    @property
    def n_led(self) -> int:
        return self.n_side * self.n_side

    @property
    def m_hr(self) -> int:
        return self.n_lr * self.upsample

    def steps_per_epoch(self) -> int:
        return -(-self.n_led // self.batch)


_OPTICS = dict(pitch_mm=4.0, height_mm=90.0, wavelength_um=0.532, na=0.1, mag=4.0,
               pixel_um=6.5, upsample=4)

WORKLOADS = {
    # 7x7 LEDs, 64^2 -> 256^2, object only, B=8, 20 epochs
    "small": Workload(name="small", n_side=7, n_lr=64, batch=8, epochs=20,
                      q_bright=1e4, q_dark=1e4, **_OPTICS),
    # 15x15 LEDs, 256^2 -> 1024^2, object + 15 Zernikes, B=16, 30 epochs
    "paper": Workload(name="paper", n_side=15, n_lr=256, batch=16, epochs=30,
                      q_bright=1e4, q_dark=1e2, learn_zernike=True,
                      true_defocus_um=10.0, **_OPTICS),
    # small shapes + defocus and LED-array shift/rotation/height learned
    "multiparam": Workload(name="multiparam", n_side=7, n_lr=64, batch=8, epochs=20,
                           q_bright=1e4, q_dark=1e4, learn_zernike=True, learn_z=True,
                           learn_geometry=True, true_defocus_um=10.0,
                           true_shift_mm=0.5, true_rot_deg=2.0, true_dh_mm=2.0,
                           **_OPTICS),
    # 21x21 LEDs, 512^2 -> 2048^2, B=32, every parameter group
    "large": Workload(name="large", n_side=21, n_lr=512, batch=32, epochs=30,
                      q_bright=1e4, q_dark=1e2, learn_zernike=True, learn_z=True,
                      learn_geometry=True, true_defocus_um=10.0,
                      true_shift_mm=0.5, true_rot_deg=2.0, true_dh_mm=2.0, **_OPTICS),
}


def workload(name: str, **overrides) -> Workload:
    return replace(WORKLOADS[name], **overrides)


# Tile reconstructions of a serving stream: LR sizes and LED grids of uneven
# size, 4x upsampling, object + Zernike pupil, B = 16, 20 epochs each.
SERVING_SIZES = (128, 192, 256, 384, 512)
SERVING_GRIDS = (7, 11, 15)


def serving_shapes():
    """Every (N, grid) combination of the serving stream, as Workloads."""
    return [Workload(name=f"tile{n}x{g}", n_side=g, n_lr=n, batch=16, epochs=20,
                     q_bright=1e4, q_dark=1e2, learn_zernike=True, true_defocus_um=10.0,
                     **_OPTICS)
            for n in SERVING_SIZES for g in SERVING_GRIDS]


def serving_stream(n_requests: int, seed: int = 0):
    """Shape index (into serving_shapes()) and schedule seed of each request:
    N and grid drawn uniformly and independently."""
    rng = np.random.default_rng([seed, 5])
    n = rng.integers(0, len(SERVING_SIZES), n_requests)
    g = rng.integers(0, len(SERVING_GRIDS), n_requests)
    shape = n * len(SERVING_GRIDS) + g
    seeds = rng.integers(0, 2**31 - 1, n_requests)
    return shape.astype(np.int64), seeds.astype(np.int64)


def poisson_arrivals_ms(rate_per_s: float, n: int, seed: int = 0) -> np.ndarray:
    """Arrival times (ms from 0) of a Poisson process of the given rate."""
    rng = np.random.default_rng([seed, 6])
    return np.cumsum(rng.exponential(1e3 / rate_per_s, n))


# ---------------------------------------------------------------------------
# truth object


def _smooth_periodic(field: np.ndarray, sigma_px: float) -> np.ndarray:
    """Periodic Gaussian blur (circular convolution) of a real square field."""
    m = field.shape[0]
    f = np.fft.fftfreq(m)
    g = np.exp(-2.0 * (math.pi * sigma_px) ** 2 * (f[:, None] ** 2 + f[None, :] ** 2))
    return np.real(np.fft.ifft2(np.fft.fft2(field) * g))


def _to_range(x: np.ndarray, lo: float, hi: float) -> np.ndarray:
    x = (x - x.min()) / (x.max() - x.min())
    return lo + (hi - lo) * x


def truth_object(m: int, seed: int = 0, sigma_px: float = 2.0):
    """Amplitude in [0.5, 1] and phase in [-pi/2, pi/2] from smoothed U(0,1) noise.

    Returns (amplitude, phase) as float64 [m, m].
    """
    rng = np.random.default_rng([seed, 0])
    a = _to_range(_smooth_periodic(rng.random((m, m)), sigma_px), 0.5, 1.0)
    p = _to_range(_smooth_periodic(rng.random((m, m)), sigma_px), -math.pi / 2, math.pi / 2)
    return a, p


# ---------------------------------------------------------------------------
# seeded truth of the system parameters


def true_defocus(w: Workload, seed: int = 0) -> float:
    """True defocus in um, U(-h, h) with h = w.true_defocus_um."""
    if w.true_defocus_um == 0.0:
        return 0.0
    rng = np.random.default_rng([seed, 3, 0])
    return float(rng.uniform(-w.true_defocus_um, w.true_defocus_um))


def true_geometry(w: Workload, seed: int = 0):
    """True LED-array errors (dx_mm, dy_mm, rot_rad, dh_mm), uniform in +-half-width."""
    rng = np.random.default_rng([seed, 3, 1])
    dx = rng.uniform(-1, 1) * w.true_shift_mm
    dy = rng.uniform(-1, 1) * w.true_shift_mm
    rot = rng.uniform(-1, 1) * math.radians(w.true_rot_deg)
    dh = rng.uniform(-1, 1) * w.true_dh_mm
    return float(dx), float(dy), float(rot), float(dh)


# ---------------------------------------------------------------------------
# random LED orders for the random-batch schedule


def led_permutations(n_led: int, epochs: int, seed: int = 0) -> np.ndarray:
    """One uniformly random order of all LEDs per epoch: int32 [epochs, n_led]."""
    rng = np.random.default_rng([seed, 2])
    return np.stack([rng.permutation(n_led) for _ in range(epochs)]).astype(np.int32)


def centre_out_order(k: np.ndarray) -> np.ndarray:
    """The fixed LED order of the sequential one-image-per-update loop (Sec. 3.1,
    Eq. 7): from the centre outwards by |k_b|, ties by angle. k is float [n_led, 2]
    in (row, col) order; returns int32 [n_led]."""
    k = np.asarray(k, np.float64)
    return np.lexsort((np.arctan2(k[:, 0], k[:, 1]),
                       np.round(np.hypot(k[:, 0], k[:, 1]), 9))).astype(np.int32)


# ---------------------------------------------------------------------------
# photon noise


def poisson_amplitudes(intensity: np.ndarray, q_per_led: np.ndarray, seed: int = 0
                       ) -> np.ndarray:
    """Measured amplitude sqrt(Poisson(q I) / q) per image, float32 [n_led, N, N].

    q_per_led is the photon count per unit intensity of each image (long
    exposure for bright-field, short for dark-field).
    """
    rng = np.random.default_rng([seed, 1])
    intensity = np.asarray(intensity, np.float64)
    q = np.asarray(q_per_led, np.float64).reshape(-1, 1, 1)
    counts = rng.poisson(np.maximum(intensity, 0.0) * q)
    return np.sqrt(counts / q).astype(np.float32)


# ---------------------------------------------------------------------------
# random parity-test operands


def random_complex(shape, seed: int, scale: float = 1.0, dtype=np.complex64) -> np.ndarray:
    rng = np.random.default_rng([seed, 7])
    z = rng.standard_normal(shape) + 1j * rng.standard_normal(shape)
    return (scale * z).astype(dtype)


def random_real(shape, seed: int, lo: float = 0.0, hi: float = 1.0, dtype=np.float32):
    rng = np.random.default_rng([seed, 8])
    return rng.uniform(lo, hi, shape).astype(dtype)


def random_indices(n: int, k: int, seed: int) -> np.ndarray:
    rng = np.random.default_rng([seed, 9])
    return rng.choice(n, size=k, replace=False).astype(np.int32)
