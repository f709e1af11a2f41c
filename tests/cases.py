"""Oracle-side construction of test problems (FP64), rounded to the GPU's storage types.

Everything here goes through oracle/ and the seeded generators only; the GPU
path receives the same float32/complex64 arrays.
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np

from oracle import fpm_oracle as fo
from paper_2408_13782_amd import inputs


def optics_of(w: inputs.Workload) -> fo.Optics:
    return fo.Optics(w.wavelength_um, w.na, w.mag, w.pixel_um, w.n_lr, w.upsample)


@dataclass
class OracleProblem:
    w: inputs.Workload
    opt: fo.Optics
    k: np.ndarray
    shifts: np.ndarray       # int32
    bright: np.ndarray
    mask: np.ndarray
    zern: np.ndarray
    kappa: np.ndarray
    O_true: np.ndarray       # complex128
    z_true: float
    A: np.ndarray            # float32 measured amplitudes
    O0: np.ndarray           # complex64 initial spectrum


def oracle_problem(w: inputs.Workload, seed: int = 0, geometry=(0.0, 0.0, 0.0, 0.0),
                   leds_for_data=None) -> OracleProblem:
    opt = optics_of(w)
    k = fo.led_wavevectors(opt, w.n_side, w.pitch_mm, w.height_mm, *geometry)
    shifts = fo.nearest_shifts(fo.led_shifts(opt, k))
    bright = fo.bright_field(opt, k)
    amp, ph = inputs.truth_object(w.m_hr, seed)
    O_true = fo.spectrum(fo.transmission(amp, ph))
    mask = fo.pupil_mask(opt)
    zern = fo.zernike_basis(opt, w.n_zernike)
    kappa = fo.defocus_phase_per_um(opt)
    z_true = inputs.true_defocus(w, seed)
    P_true = fo.pupil(mask, zern, np.zeros(w.n_zernike), z_true, kappa)
    I = fo.forward_intensities(O_true, P_true, shifts, range(w.n_led))
    q = np.where(bright, w.q_bright, w.q_dark)
    A = inputs.poisson_amplitudes(I, q, seed)
    centre = (w.n_side // 2) * w.n_side + w.n_side // 2
    O0 = fo.initial_spectrum(A[centre], w.upsample).astype(np.complex64)
    return OracleProblem(w, opt, k, shifts, bright, mask, zern, kappa, O_true, z_true, A, O0)


def rel_l2(a, b) -> float:
    a = np.asarray(a, np.complex128)
    b = np.asarray(b, np.complex128)
    nb = np.linalg.norm(b)
    return float(np.linalg.norm(a - b) / (nb if nb > 0 else 1.0))


GRAD_TOL = 2e-5          # per-step gradient bar, relative L2
GRAD_ELEM_TOL = 1e-4     # elementwise bar, relative to the largest reference entry


def assert_grad_close(got, ref, tol: float = GRAD_TOL, elem_tol: float = GRAD_ELEM_TOL):
    """Gradient parity: relative L2 within tol, and every entry within elem_tol of
    the largest reference magnitude (an error confined to a few pixels, which the
    L2 norm over millions of entries would hide, fails the second bound)."""
    got = np.asarray(got, np.complex128)
    ref = np.asarray(ref, np.complex128)
    err = rel_l2(got, ref)
    assert err <= tol, f"relative L2 {err:.3e} > {tol:.1e}"
    worst = float(np.abs(got - ref).max())
    scale = float(np.abs(ref).max())
    assert worst <= elem_tol * scale, f"max entry error {worst:.3e} > {elem_tol:.0e} x {scale:.3e}"
    return err
