"""FP64 CPU oracle for the Batch-FPM hot path (arXiv 2408.13782).

TEST INFRASTRUCTURE ONLY. Nothing in the product package may import, call or
execute this module; it exists so that tests, the smoke check and the CPU
baseline leg of the benchmark can compare the HIP path against a plain,
slow, obviously correct implementation. It shares no code with the HIP path.

Everything is numpy in float64 / complex128 and written in the order and
notation of the paper:

* thin-object exit wave and its spectrum ........ Sec. 2.1, Eq. (1)
* LED illumination wave vector k_m ............... Sec. 2.1 (text around Eq. 2)
* low-resolution image formation ................. Sec. 2.1, Eq. (2)
* defocus transfer H(k, z) and LED intensity ..... Sec. 2.1, Eq. (3)
* per-image loss summed over images .............. Sec. 2.1 Eq. (4), Sec. 2.2 Eq. (5)
* random batch update (sum of B gradients) ....... Sec. 2.3, Eq. (13)
* balanced random batching ....................... Sec. 2.3, Eq. (14) and the
                                                   nine-LED example before it
* bilinear centre-LED initial value .............. Sec. 2.3 (before Eq. 14)
* Adam-family optimiser .......................... Sec. 2.2 (optimisers named)
* digital refocusing of a reconstruction ......... Abstract, Sec. 3.3, Sec. 4

Readings taken where the paper is silent or garbled:

* the learned tensor is the centred HR spectrum with orthonormal scaling,
  O = fftshift(fft2(o)) / M, so sum|O|^2 = sum|o|^2;
* LED b reads the spectrum window whose top-left corner is
  (M/2 - N/2) + s_b, with s_b = k_b / dk and k_b pointing from the sample to
  the LED (this is Eq. (2) with k_m the propagation direction, i.e. -k_b);
  window indices wrap modulo M;
* loss = sum over batch and pixels of (sqrt(gamma) |psi| - A)^2 (the
  amplitude form of Eq. (5));
* gradients are real gradients written as complex numbers,
  g = dL/dRe + i dL/dIm; at |psi| = 0 the direction psi/|psi| is taken as 0;
* the defocus phase drops the piston 2 pi z / lambda (a global phase);
* Zernike terms are OSA/ANSI j = 0..14 with unit-RMS normalisation over the
  pupil disk;
* LED-array geometry: lateral shift, in-plane rotation and height error of
  a square grid.

Parity of every function here is pinned by tests/test_oracle_*.py against
closed forms, brute force, invariants or library routines; see those files.
"""
from __future__ import annotations

import math
from dataclasses import dataclass

import numpy as np

# 2-D FFTs: numpy's (one thread) unless set_fft_workers() picks scipy.fft with
# several worker threads (same transform, used by the CPU-baseline timing only).
_fft_workers = 1


def set_fft_workers(n: int) -> None:
    """Compute the 2-D FFTs with scipy.fft on n threads (n = 1: numpy.fft)."""
    global _fft_workers
    _fft_workers = max(1, int(n))


def _fft2(x):
    if _fft_workers > 1:
        import scipy.fft
        return scipy.fft.fft2(x, workers=_fft_workers)
    return np.fft.fft2(x)


def _ifft2(x):
    if _fft_workers > 1:
        import scipy.fft
        return scipy.fft.ifft2(x, workers=_fft_workers)
    return np.fft.ifft2(x)

# ---------------------------------------------------------------------------
# Optics and LED geometry (Sec. 2.1: k_m = (sin theta_x / lambda, sin theta_y / lambda))
# ---------------------------------------------------------------------------


@dataclass(frozen=True)
class Optics:
    wavelength_um: float
    na: float
    mag: float
    pixel_um: float
    n_lr: int
    upsample: int

    @property
    def dx_lr(self) -> float:
        """Object-plane sampling of the low-resolution camera (um)."""
        return self.pixel_um / self.mag

    @property
    def dk(self) -> float:
        """Spectral pixel pitch (1/um); identical on the LR and HR grids."""
        return 1.0 / (self.n_lr * self.dx_lr)

    @property
    def m_hr(self) -> int:
        return self.n_lr * self.upsample

    @property
    def pupil_radius_px(self) -> float:
        """Coherent cutoff NA/lambda in spectral pixels."""
        return self.na / self.wavelength_um / self.dk


def led_positions(n_side: int, pitch_mm: float, height_mm: float,
                  shift_x_mm: float = 0.0, shift_y_mm: float = 0.0,
                  rot_rad: float = 0.0, dh_mm: float = 0.0):
    """Physical LED coordinates (x, y, H) in mm for a square grid.

    LED ids run row-major over the grid; column offset i and row offset j are
    measured from the grid centre. The grid may be shifted laterally, rotated
    in-plane and placed at a wrong height (the LED-array errors that the
    multi-parameter network corrects, Sec. 2.2).
    """
    c = (n_side - 1) / 2.0
    x = np.empty(n_side * n_side)
    y = np.empty(n_side * n_side)
    for row in range(n_side):
        for col in range(n_side):
            i = col - c
            j = row - c
            led = row * n_side + col
            x[led] = pitch_mm * (i * math.cos(rot_rad) - j * math.sin(rot_rad)) + shift_x_mm
            y[led] = pitch_mm * (i * math.sin(rot_rad) + j * math.cos(rot_rad)) + shift_y_mm
    h = np.full(n_side * n_side, height_mm + dh_mm)
    return x, y, h


def led_wavevectors(optics: Optics, n_side: int, pitch_mm: float, height_mm: float,
                    shift_x_mm: float = 0.0, shift_y_mm: float = 0.0,
                    rot_rad: float = 0.0, dh_mm: float = 0.0,
                    roi_x_mm: float = 0.0, roi_y_mm: float = 0.0) -> np.ndarray:
    """Spatial frequency k_b = (sin theta_y, sin theta_x) / lambda of every LED.

    Returned as float64 [n_led, 2] in (row, col) = (y, x) order, 1/um. The
    sine of the illumination angle is the lateral LED-to-sample offset over
    the LED-to-sample distance (Sec. 2.1).
    """
    x, y, h = led_positions(n_side, pitch_mm, height_mm, shift_x_mm, shift_y_mm,
                            rot_rad, dh_mm)
    dxs = x - roi_x_mm
    dys = y - roi_y_mm
    d = np.sqrt(dxs * dxs + dys * dys + h * h)
    k = np.empty((x.size, 2))
    k[:, 0] = dys / d / optics.wavelength_um
    k[:, 1] = dxs / d / optics.wavelength_um
    return k


def led_shifts(optics: Optics, k: np.ndarray) -> np.ndarray:
    """Spectrum offset of each LED in spectral pixels, s_b = k_b / dk (float64)."""
    return np.asarray(k, dtype=np.float64) / optics.dk


def nearest_shifts(s: np.ndarray) -> np.ndarray:
    """Round fractional spectral offsets to the nearest pixel (ties upward)."""
    return np.floor(np.asarray(s, dtype=np.float64) + 0.5).astype(np.int32)


def bright_field(optics: Optics, k: np.ndarray) -> np.ndarray:
    """True where the illumination angle lies inside the objective NA."""
    return np.hypot(k[:, 0], k[:, 1]) <= optics.na / optics.wavelength_um


# ---------------------------------------------------------------------------
# Pupil: support, Zernike aberrations, defocus (Sec. 2.1 Eq. 3; Sec. 2.2)
# ---------------------------------------------------------------------------


def pupil_offsets(n: int):
    """Integer spectral offsets (row, col) of a centred n x n grid."""
    u = np.arange(n) - n // 2
    return np.meshgrid(u, u, indexing="ij")


def pupil_mask(optics: Optics) -> np.ndarray:
    """Coherent transfer support: offsets with |u| <= NA/lambda (in pixels)."""
    uy, ux = pupil_offsets(optics.n_lr)
    r = optics.pupil_radius_px
    return ((uy * uy + ux * ux) <= r * r).astype(np.uint8)


def zernike_nm(j: int):
    """OSA/ANSI single index j -> (n, m)."""
    n = int(math.ceil((-3.0 + math.sqrt(9.0 + 8.0 * j)) / 2.0))
    m = 2 * j - n * (n + 2)
    return n, m


def zernike_radial(n: int, m: int, rho: np.ndarray) -> np.ndarray:
    """Radial polynomial R_n^|m|(rho) from its factorial series."""
    m = abs(m)
    out = np.zeros_like(rho, dtype=np.float64)
    for k in range((n - m) // 2 + 1):
        coef = ((-1) ** k * math.factorial(n - k)
                / (math.factorial(k) * math.factorial((n + m) // 2 - k)
                   * math.factorial((n - m) // 2 - k)))
        out += coef * rho ** (n - 2 * k)
    return out


def zernike(j: int, rho: np.ndarray, phi: np.ndarray) -> np.ndarray:
    """Unit-RMS Zernike term Z_j(rho, phi) on the unit disk (OSA/ANSI order)."""
    n, m = zernike_nm(j)
    norm = math.sqrt(2.0 * (n + 1) / (2.0 if m == 0 else 1.0))
    rad = zernike_radial(n, m, rho)
    if m > 0:
        return norm * rad * np.cos(m * phi)
    if m < 0:
        return norm * rad * np.sin(-m * phi)
    return norm * rad


def zernike_basis(optics: Optics, n_terms: int = 15) -> np.ndarray:
    """Z_j sampled on the pupil grid, rho = |k| / (NA/lambda); zero off-support."""
    uy, ux = pupil_offsets(optics.n_lr)
    r = optics.pupil_radius_px
    rho = np.hypot(uy, ux) / r
    phi = np.arctan2(uy, ux)
    mask = pupil_mask(optics).astype(bool)
    out = np.zeros((n_terms, optics.n_lr, optics.n_lr))
    for j in range(n_terms):
        out[j][mask] = zernike(j, rho[mask], phi[mask])
    return out


def defocus_phase_per_um(optics: Optics, size: int | None = None) -> np.ndarray:
    """kappa(k) = 2 pi (sqrt(1/lambda^2 - |k|^2) - 1/lambda), rad per um of z.

    This is the phase of H(k, z) = exp(i z kappa) of Eq. (3), read with k in
    1/um and without the global piston 2 pi z / lambda. Zero where |k| > 1/lambda
    (an evanescent component; H is then set to 0 by the callers that need it).
    """
    n = optics.n_lr if size is None else size
    uy, ux = pupil_offsets(n)
    k2 = (uy * uy + ux * ux) * optics.dk * optics.dk
    inv_l2 = 1.0 / optics.wavelength_um ** 2
    kz = np.sqrt(np.maximum(inv_l2 - k2, 0.0))
    return np.where(k2 <= inv_l2, 2.0 * math.pi * (kz - 1.0 / optics.wavelength_um), 0.0)


def pupil(mask: np.ndarray, zern: np.ndarray, coeffs, z_um: float,
          kappa: np.ndarray) -> np.ndarray:
    """P(k) = mask * exp(i (sum_j c_j Z_j + z kappa)), Eq. (3) with H folded in."""
    theta = np.tensordot(np.asarray(coeffs, dtype=np.float64), zern, axes=1) + z_um * kappa
    return mask.astype(np.float64) * np.exp(1j * theta)


# ---------------------------------------------------------------------------
# Object and spectrum (Sec. 2.1 Eq. 1)
# ---------------------------------------------------------------------------


def transmission(amplitude: np.ndarray, phase: np.ndarray) -> np.ndarray:
    """o(r) = exp(i phi - mu) with amplitude exp(-mu) (Eq. 1)."""
    return np.asarray(amplitude, np.float64) * np.exp(1j * np.asarray(phase, np.float64))


def spectrum(o: np.ndarray) -> np.ndarray:
    """Centred, orthonormally scaled HR spectrum O = fftshift(fft2(o)) / M."""
    m = o.shape[0]
    return np.fft.fftshift(_fft2(o)) / m


def object_from_spectrum(O: np.ndarray) -> np.ndarray:
    """Inverse of spectrum(): o = ifft2(ifftshift(O)) * M."""
    m = O.shape[0]
    return _ifft2(np.fft.ifftshift(O)) * m


# ---------------------------------------------------------------------------
# Forward model (Eq. 2 / Eq. 3) and its adjoint
# ---------------------------------------------------------------------------


def window_indices(m: int, n: int, shift):
    """Row and column indices of the n x n window of LED offset (row, col)."""
    base = m // 2 - n // 2
    rows = (base + int(shift[0]) + np.arange(n)) % m
    cols = (base + int(shift[1]) + np.arange(n)) % m
    return rows, cols


def crop(O: np.ndarray, n: int, shift) -> np.ndarray:
    """C_b[u] = O[w_b + u]: the part of the spectrum that the pupil passes."""
    rows, cols = window_indices(O.shape[0], n, shift)
    return O[np.ix_(rows, cols)]


def lr_field(O: np.ndarray, P: np.ndarray, shift) -> np.ndarray:
    """Low-resolution exit field psi_b = F^-1(O(k - k_m) P(k)) on the camera grid.

    With the orthonormal spectrum this is (N^2 / M) ifft2(ifftshift(C_b P)):
    a flat object o = c gives psi = c P[DC] for the centre LED.
    """
    n = P.shape[0]
    m = O.shape[0]
    phi = crop(O, n, shift) * P
    return (n * n / m) * _ifft2(np.fft.ifftshift(phi))


def forward_amplitudes(O, P, shifts, leds, gamma=None) -> np.ndarray:
    """sqrt(gamma_b) |psi_b| for each LED in the batch (Eq. 3, amplitude form)."""
    n = P.shape[0]
    out = np.empty((len(leds), n, n))
    for b, led in enumerate(leds):
        g = 1.0 if gamma is None else float(gamma[led])
        out[b] = math.sqrt(g) * np.abs(lr_field(O, P, shifts[led]))
    return out


def forward_intensities(O, P, shifts, leds, gamma=None) -> np.ndarray:
    """I_b = gamma_b |psi_b|^2 (Eq. 3)."""
    return forward_amplitudes(O, P, shifts, leds, gamma) ** 2


@dataclass
class Grads:
    loss: float
    g_O: np.ndarray
    g_P: np.ndarray
    g_gamma: np.ndarray  # per LED in the batch


def residual(psi, A, gamma_b: float, loss: str = "amplitude"):
    """Per-image loss terms of Eq. 5 and the real gradient with respect to psi.

    amplitude (Eq. 5 with L2 on amplitudes):  e = sqrt(gamma)|psi| - A,
        L_b = sum e^2, g_psi = 2 sqrt(gamma) e psi/|psi| (0 where psi = 0),
        dL_b/dgamma = sum e |psi| / sqrt(gamma);
    intensity (Eq. 4): e = gamma |psi|^2 - A^2,
        L_b = sum e^2, g_psi = 4 gamma e psi, dL_b/dgamma = 2 sum e |psi|^2.
    Returns (L_b, g_psi, dL_b/dgamma).
    """
    A = np.asarray(A, dtype=np.float64)
    if loss == "amplitude":
        sg = math.sqrt(gamma_b)
        a = np.abs(psi)
        e = sg * a - A
        unit = np.zeros_like(psi)
        nz = a > 0
        unit[nz] = psi[nz] / a[nz]
        return float(np.sum(e * e)), 2.0 * sg * e * unit, float(np.sum(e * a)) / sg
    if loss == "intensity":
        q = np.abs(psi) ** 2
        e = gamma_b * q - A * A
        return float(np.sum(e * e)), 4.0 * gamma_b * e * psi, 2.0 * float(np.sum(e * q))
    raise ValueError(f"unknown loss {loss!r}")


def loss_and_grads(O, P, shifts, leds, meas_amp, gamma=None, loss: str = "amplitude") -> Grads:
    """Loss of one batch and its real gradients (Eqs. 4-5 and 13).

    Amplitude form: L = sum_b sum_r (sqrt(gamma_b) |psi_b(r)| - A_b(r))^2, summed
    (not averaged) over the B images of the batch, as the update of Eq. (13)
    sums the B per-image gradients (intensity form: see `residual`). Each image
    contributes, with g_psi from `residual`:

      g_Phi = (1/M) fftshift(fft2(g_psi))          (adjoint of lr_field)
      g_O[w_b + u] += conj(P[u]) g_Phi[u]
      g_P[u]       += conj(C_b[u]) g_Phi[u]
    """
    n = P.shape[0]
    m = O.shape[0]
    g_O = np.zeros_like(O, dtype=np.complex128)
    g_P = np.zeros((n, n), dtype=np.complex128)
    g_gamma = np.zeros(len(leds))
    total = 0.0
    for b, led in enumerate(leds):
        rows, cols = window_indices(m, n, shifts[led])
        C = O[np.ix_(rows, cols)]
        psi = (n * n / m) * _ifft2(np.fft.ifftshift(C * P))
        gb = 1.0 if gamma is None else float(gamma[led])
        lb, g_psi, g_gamma[b] = residual(psi, meas_amp[led], gb, loss)
        total += lb
        g_C, g_Pb = field_adjoint(g_psi, P, C, m)
        g_O[np.ix_(rows, cols)] += g_C
        g_P += g_Pb
    return Grads(total, g_O, g_P, g_gamma)


def field_adjoint(g_psi, P, C, m):
    """Adjoint of Phi = C P -> psi (the linear part of lr_field).

    g_Phi = (1/M) fftshift(fft2(g_psi)); returns (conj(P) g_Phi, conj(C) g_Phi),
    the gradients with respect to the cropped spectrum and the pupil.
    """
    g_phi = np.fft.fftshift(_fft2(g_psi)) / m
    return np.conj(P) * g_phi, np.conj(C) * g_phi


def pupil_param_grads(g_P, P, zern, kappa):
    """Chain rule from the complex pupil to its phase parameters.

    P = mask exp(i theta) so dL/dtheta = Im(g_P conj(P)); then
    dL/dc_j = sum_u dL/dtheta(u) Z_j(u) and dL/dz = sum_u dL/dtheta(u) kappa(u).
    Returns (g_c [n_terms], g_z, g_theta [N, N]).
    """
    g_theta = np.imag(g_P * np.conj(P))
    g_c = np.tensordot(zern, g_theta, axes=([1, 2], [0, 1]))
    g_z = float(np.sum(g_theta * kappa))
    return g_c, g_z, g_theta


# ---------------------------------------------------------------------------
# Sub-pixel LED offsets and the LED-array geometry (Sec. 2.1 k_m; Sec. 2.2:
# LED position errors corrected jointly with the other system parameters)
# ---------------------------------------------------------------------------


def crop_bilinear(O: np.ndarray, n: int, shift):
    """Spectrum sampled at the fractional window (M/2 - N/2) + s + u, bilinearly.

    Returns (C, taps, frac, rows0, cols0): C[u], the four neighbour arrays
    O[f + u + t] for t in (0,0) (0,1) (1,0) (1,1), the fractional part a of the
    window corner f + a, and the integer row/column indices of tap (0,0).
    Indices wrap modulo M.
    """
    m = O.shape[0]
    w = (m // 2 - n // 2) + np.asarray(shift, dtype=np.float64)
    f = np.floor(w).astype(np.int64)
    a = w - f
    r0 = (f[0] + np.arange(n)) % m
    r1 = (r0 + 1) % m
    c0 = (f[1] + np.arange(n)) % m
    c1 = (c0 + 1) % m
    t00, t01 = O[np.ix_(r0, c0)], O[np.ix_(r0, c1)]
    t10, t11 = O[np.ix_(r1, c0)], O[np.ix_(r1, c1)]
    C = ((1 - a[0]) * (1 - a[1]) * t00 + (1 - a[0]) * a[1] * t01
         + a[0] * (1 - a[1]) * t10 + a[0] * a[1] * t11)
    return C, (t00, t01, t10, t11), a, r0, c0


def scatter_bilinear(g_O, g_C, a, r0, c0):
    """Adjoint of crop_bilinear: g_O[f + u + t] += w_t g_C[u] for the four taps t."""
    m = g_O.shape[0]
    r1, c1 = (r0 + 1) % m, (c0 + 1) % m
    for rows, cols, wgt in ((r0, c0, (1 - a[0]) * (1 - a[1])), (r0, c1, (1 - a[0]) * a[1]),
                            (r1, c0, a[0] * (1 - a[1])), (r1, c1, a[0] * a[1])):
        np.add.at(g_O, np.ix_(rows, cols), wgt * g_C)


@dataclass
class GeneralGrads:
    loss: float
    g_O: np.ndarray
    g_P: np.ndarray
    g_gamma: np.ndarray      # per batch position
    g_shift: np.ndarray      # [B, 2] dL/ds_b (row, col)


def loss_and_grads_subpixel(O, P, shifts, leds, meas_amp, gamma=None,
                            loss: str = "amplitude") -> GeneralGrads:
    """Loss and gradients with fractional LED offsets (bilinear crop).

    Same loss as loss_and_grads; with integer offsets the two agree. Also the
    gradient with respect to each LED's offset: dL/ds = sum_u Re(conj(g_C) dC/ds),
    a one-sided derivative where the offset crosses an integer.
    """
    n = P.shape[0]
    m = O.shape[0]
    g_O = np.zeros_like(O, dtype=np.complex128)
    g_P = np.zeros((n, n), dtype=np.complex128)
    g_gamma = np.zeros(len(leds))
    g_shift = np.zeros((len(leds), 2))
    total = 0.0
    for b, led in enumerate(leds):
        C, (t00, t01, t10, t11), a, r0, c0 = crop_bilinear(O, n, shifts[led])
        psi = (n * n / m) * _ifft2(np.fft.ifftshift(C * P))
        gb = 1.0 if gamma is None else float(gamma[led])
        lb, g_psi, g_gamma[b] = residual(psi, meas_amp[led], gb, loss)
        total += lb
        g_C, g_Pb = field_adjoint(g_psi, P, C, m)
        scatter_bilinear(g_O, g_C, a, r0, c0)
        g_P += g_Pb
        dC_dy = (1 - a[1]) * (t10 - t00) + a[1] * (t11 - t01)
        dC_dx = (1 - a[0]) * (t01 - t00) + a[0] * (t11 - t10)
        g_shift[b, 0] = float(np.sum(np.real(np.conj(g_C) * dC_dy)))
        g_shift[b, 1] = float(np.sum(np.real(np.conj(g_C) * dC_dx)))
    return GeneralGrads(total, g_O, g_P, g_gamma, g_shift)


GEOMETRY_NAMES = ("shift_x_mm", "shift_y_mm", "rot_rad", "dh_mm")


def led_shifts_and_jacobian(optics: Optics, n_side: int, pitch_mm: float, height_mm: float,
                            geom=(0.0, 0.0, 0.0, 0.0), roi_x_mm: float = 0.0,
                            roi_y_mm: float = 0.0):
    """Fractional offsets s [n_led, 2] (row, col) and ds/d(geom) [n_led, 2, 4].

    geom = (shift_x_mm, shift_y_mm, rot_rad, dh_mm). With D the LED-to-sample
    distance, k = (dy, dx) / (lambda D) and s = k / dk, differentiated by hand:
    dk_x/dx = (D^2 - dx^2)/(lambda D^3), dk_x/dy = -dx dy/(lambda D^3),
    dk_x/dH = -dx H/(lambda D^3) (and symmetrically), while a rotation moves the
    LED by (dx, dy) -> (-y', x') with (x', y') its rotated grid offset.
    """
    dx_mm, dy_mm, rot, dh = (float(g) for g in geom)
    x, y, h = led_positions(n_side, pitch_mm, height_mm, dx_mm, dy_mm, rot, dh)
    X = x - roi_x_mm
    Y = y - roi_y_mm
    D = np.sqrt(X * X + Y * Y + h * h)
    lam = optics.wavelength_um
    s = np.stack([Y / D / lam, X / D / lam], 1) / optics.dk
    D3 = lam * D ** 3
    dkx = np.stack([(D * D - X * X) / D3, -X * Y / D3, -X * h / D3], 1)   # d/d(X, Y, H)
    dky = np.stack([-X * Y / D3, (D * D - Y * Y) / D3, -Y * h / D3], 1)
    # d(X, Y, H) / d(shift_x, shift_y, rot, dh)
    xr = x - dx_mm      # rotated grid offsets before the lateral shift
    yr = y - dy_mm
    dXYH = np.zeros((x.size, 3, 4))
    dXYH[:, 0, 0] = 1.0
    dXYH[:, 1, 1] = 1.0
    dXYH[:, 0, 2] = -yr
    dXYH[:, 1, 2] = xr
    dXYH[:, 2, 3] = 1.0
    J = np.empty((x.size, 2, 4))
    J[:, 0, :] = np.einsum("nk,nkp->np", dky, dXYH) / optics.dk
    J[:, 1, :] = np.einsum("nk,nkp->np", dkx, dXYH) / optics.dk
    return s, J


@dataclass
class MultiGrads:
    loss: float
    g_O: np.ndarray
    g_coeffs: np.ndarray
    g_z: float
    g_geom: np.ndarray       # [4]
    g_gamma: np.ndarray      # [n_led] (zero for LEDs outside the batch)


def multiparam_loss_and_grads(O, coeffs, z_um, geom, gamma, leds, meas_amp, optics: Optics,
                              n_side, pitch_mm, height_mm, mask, zern, kappa,
                              loss: str = "amplitude") -> MultiGrads:
    """Loss of one batch as a function of every learned group (Sec. 2.2, Eq. 3).

    Object spectrum, pupil Zernike coefficients and defocus, LED-array geometry
    (lateral shift, rotation, height) and LED intensities; gradients by the
    chain rule through the sub-pixel crop.
    """
    P = pupil(mask, zern, coeffs, z_um, kappa)
    s, J = led_shifts_and_jacobian(optics, n_side, pitch_mm, height_mm, geom)
    gr = loss_and_grads_subpixel(O, P, s, leds, meas_amp, gamma, loss)
    g_c, g_z, _ = pupil_param_grads(gr.g_P, P, zern, kappa)
    g_geom = np.zeros(4)
    g_gamma = np.zeros(len(s))
    for b, led in enumerate(leds):
        g_geom += J[led].T @ gr.g_shift[b]
        g_gamma[led] += gr.g_gamma[b]
    return MultiGrads(gr.loss, gr.g_O, g_c, g_z, g_geom, g_gamma)


# ---------------------------------------------------------------------------
# Optimiser (Sec. 2.2: Adam-family optimisers from deep-learning frameworks)
# ---------------------------------------------------------------------------


def adam_update(p, g, m, v, t: int, lr: float, beta1=0.9, beta2=0.999, eps=1e-8):
    """One Adam step (Kingma and Ba 2015), bias-corrected as in torch.optim.Adam.

    Complex parameters are handled as independent real and imaginary parts.
    Returns new (p, m, v); inputs are not modified.
    """
    is_complex = np.iscomplexobj(p)
    if is_complex:
        p_r = np.stack([p.real, p.imag], -1)
        g_r = np.stack([np.real(g), np.imag(g)], -1)
    else:
        p_r = np.asarray(p, np.float64)
        g_r = np.asarray(g, np.float64)
    m = beta1 * m + (1.0 - beta1) * g_r
    v = beta2 * v + (1.0 - beta2) * g_r * g_r
    bc1 = 1.0 - beta1 ** t
    bc2 = 1.0 - beta2 ** t
    denom = np.sqrt(v) / math.sqrt(bc2) + eps
    p_r = p_r - (lr / bc1) * m / denom
    if is_complex:
        return p_r[..., 0] + 1j * p_r[..., 1], m, v
    return p_r, m, v


# ---------------------------------------------------------------------------
# Balanced random batching (Sec. 2.3, Eq. 14 and the nine-LED example)
# ---------------------------------------------------------------------------


def batches_from_permutations(perms, batch: int):
    """Cut each epoch's random order of all LEDs into consecutive batches.

    Every epoch uses every LED exactly once, so each LED is selected the same
    number of times (Eq. 14); the last batch of an epoch may be partial.
    """
    out = []
    for perm in perms:
        perm = [int(x) for x in perm]
        for start in range(0, len(perm), batch):
            out.append(perm[start:start + batch])
    return out


# ---------------------------------------------------------------------------
# Initial value (Sec. 2.3: bilinear-interpolated centre-LED image)
# ---------------------------------------------------------------------------


def bilinear_upsample(img: np.ndarray, s: int) -> np.ndarray:
    """Bilinear upsampling by an integer factor, pixel-centre aligned.

    Output pixel X samples the input at (X + 0.5)/s - 0.5, clamped at the
    borders (the half-pixel convention of common deep-learning frameworks).
    """
    img = np.asarray(img, np.float64)
    n = img.shape[0]

    def axis_weights(size_in):
        X = np.arange(size_in * s)
        src = np.maximum((X + 0.5) / s - 0.5, 0.0)
        i0 = np.floor(src).astype(np.int64)
        i0 = np.minimum(i0, size_in - 1)
        i1 = np.minimum(i0 + 1, size_in - 1)
        w1 = src - i0
        return i0, i1, w1

    r0, r1, wr = axis_weights(n)
    c0, c1, wc = axis_weights(img.shape[1])
    top = img[r0][:, c0] * (1 - wc) + img[r0][:, c1] * wc
    bot = img[r1][:, c0] * (1 - wc) + img[r1][:, c1] * wc
    return top * (1 - wr)[:, None] + bot * wr[:, None]


def initial_spectrum(centre_amp: np.ndarray, s: int) -> np.ndarray:
    """O_0: spectrum of the upsampled centre-LED amplitude image, zero phase."""
    return spectrum(bilinear_upsample(centre_amp, s).astype(np.complex128))


# ---------------------------------------------------------------------------
# The reconstruction loop (Sec. 2.3, Eq. 13)
# ---------------------------------------------------------------------------


@dataclass
class SolveConfig:
    lr_object: float = 1e-2
    lr_zernike: float = 1e-2
    lr_z: float = 0.1
    learn_pupil: bool = False   # Zernike coefficients
    learn_z: bool = False
    loss: str = "amplitude"     # or "intensity" (Eq. 4)
    beta1: float = 0.9
    beta2: float = 0.999
    eps: float = 1e-8


@dataclass
class SolveState:
    O: np.ndarray
    coeffs: np.ndarray
    z_um: float
    m_O: np.ndarray
    v_O: np.ndarray
    m_c: np.ndarray
    v_c: np.ndarray
    m_z: float
    v_z: float
    t: int = 0


def init_state(O0, n_terms=15, coeffs0=None, z0=0.0) -> SolveState:
    O0 = np.asarray(O0, np.complex128)
    shape = O0.shape + (2,)
    c0 = np.zeros(n_terms) if coeffs0 is None else np.asarray(coeffs0, np.float64).copy()
    return SolveState(O0.copy(), c0, float(z0), np.zeros(shape), np.zeros(shape),
                      np.zeros(n_terms), np.zeros(n_terms), 0.0, 0.0, 0)


def step(state: SolveState, cfg: SolveConfig, mask, zern, kappa, shifts, leds, meas_amp,
         gamma=None):
    """One random-batch update: gradients summed over the batch, then Adam."""
    P = pupil(mask, zern, state.coeffs, state.z_um, kappa)
    gr = loss_and_grads(state.O, P, shifts, leds, meas_amp, gamma, cfg.loss)
    state.t += 1
    t = state.t
    state.O, state.m_O, state.v_O = adam_update(state.O, gr.g_O, state.m_O, state.v_O, t,
                                                cfg.lr_object, cfg.beta1, cfg.beta2, cfg.eps)
    if cfg.learn_pupil or cfg.learn_z:
        g_c, g_z, _ = pupil_param_grads(gr.g_P, P, zern, kappa)
        if cfg.learn_pupil:
            # The piston term (j = 0) is a global phase: its gradient is identically
            # zero, so it is held at its value rather than driven by rounding noise.
            c, mc, vc = adam_update(state.coeffs[1:], g_c[1:], state.m_c[1:], state.v_c[1:],
                                    t, cfg.lr_zernike, cfg.beta1, cfg.beta2, cfg.eps)
            state.coeffs = np.concatenate([state.coeffs[:1], c])
            state.m_c = np.concatenate([state.m_c[:1], mc])
            state.v_c = np.concatenate([state.v_c[:1], vc])
        if cfg.learn_z:
            zz, mz, vz = adam_update(np.array([state.z_um]), np.array([g_z]),
                                     np.array([state.m_z]), np.array([state.v_z]), t,
                                     cfg.lr_z, cfg.beta1, cfg.beta2, cfg.eps)
            state.z_um, state.m_z, state.v_z = float(zz[0]), float(mz[0]), float(vz[0])
    return gr.loss


def solve(state: SolveState, cfg: SolveConfig, mask, zern, kappa, shifts, schedule,
          meas_amp, gamma=None):
    """Run every batch of a schedule; returns the per-step losses."""
    return [step(state, cfg, mask, zern, kappa, shifts, leds, meas_amp, gamma)
            for leds in schedule]


# ---------------------------------------------------------------------------
# Digital refocusing (Abstract; Sec. 3.3; Sec. 4)
# ---------------------------------------------------------------------------


def refocus(O: np.ndarray, z_um, optics: Optics) -> np.ndarray:
    """Propagate the reconstructed object by z: o_z = F^-1(O H(k, z)) for each z.

    H(k, z) = exp(i z kappa(k)) over the HR spectrum (same spectral pitch dk as
    the pupil grid), 0 for evanescent |k| > 1/lambda. Output [nz, M, M].
    """
    m = O.shape[0]
    kappa = defocus_phase_per_um(optics, size=m)
    uy, ux = pupil_offsets(m)
    prop = ((uy * uy + ux * ux) * optics.dk ** 2) <= 1.0 / optics.wavelength_um ** 2
    out = np.empty((len(z_um), m, m), dtype=np.complex128)
    for i, z in enumerate(z_um):
        H = np.where(prop, np.exp(1j * float(z) * kappa), 0.0)
        out[i] = object_from_spectrum(O * H)
    return out


# ---------------------------------------------------------------------------
# Evaluation (Sec. 3.1: PSNR of amplitude and phase)
# ---------------------------------------------------------------------------


def align_global_phase(o: np.ndarray, ref: np.ndarray) -> np.ndarray:
    """Multiply o by the unit phase that best matches ref (the loss ignores it)."""
    c = np.vdot(o, ref)
    return o * (c / abs(c) if abs(c) > 0 else 1.0)


def psnr(x: np.ndarray, ref: np.ndarray) -> float:
    """Peak signal-to-noise ratio in dB with the reference's peak value."""
    x = np.asarray(x, np.float64)
    ref = np.asarray(ref, np.float64)
    mse = float(np.mean((x - ref) ** 2))
    peak = float(np.max(np.abs(ref)))
    return float("inf") if mse == 0 else 10.0 * math.log10(peak * peak / mse)
