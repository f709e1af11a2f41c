"""Python binding of libfpm (include/fpm.h): argument marshalling only.

Every computation of the hot path runs in the HIP library; torch provides
device memory and the current stream. Loading fails loudly when the library
has not been built: there is no fallback implementation.
"""
from __future__ import annotations

import ctypes as C
import os
from dataclasses import dataclass

import numpy as np

_PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_PKG, "libfpm.so")

# status codes of include/fpm.h
FPM_OK = 0
FPM_EINVAL = -1
FPM_ENOMEM = -2
FPM_EHIP = -3
FPM_EUNSUPPORTED = -4
FPM_ENONFINITE = -5
N_ZERN = 15
N_PAR = 16


class FpmError(RuntimeError):
    pass


class _Desc(C.Structure):
    _fields_ = [("n_lr", C.c_int32), ("upsample", C.c_int32), ("n_led", C.c_int32),
                ("max_batch", C.c_int32), ("wavelength_um", C.c_double), ("na", C.c_double),
                ("mag", C.c_double), ("pixel_um", C.c_double)]


class _Info(C.Structure):
    _fields_ = [("n_lr", C.c_int32), ("m_hr", C.c_int32), ("n_led", C.c_int32),
                ("max_batch", C.c_int32), ("support_px", C.c_int32),
                ("support_rows", C.c_int32), ("adam_tiles", C.c_int32),
                ("pupil_radius_px", C.c_double), ("dk", C.c_double),
                ("device_bytes", C.c_int64), ("fused_chain", C.c_int32)]


class _Grid(C.Structure):
    _fields_ = [("n_side", C.c_int32), ("pitch_mm", C.c_double), ("height_mm", C.c_double),
                ("shift_x_mm", C.c_double), ("shift_y_mm", C.c_double), ("rot_rad", C.c_double),
                ("dh_mm", C.c_double), ("roi_x_mm", C.c_double), ("roi_y_mm", C.c_double)]


class _HParams(C.Structure):
    _fields_ = [("lr_object", C.c_float), ("lr_zernike", C.c_float), ("lr_z", C.c_float),
                ("beta1", C.c_float), ("beta2", C.c_float), ("eps", C.c_float),
                ("learn_zernike", C.c_int32), ("learn_z", C.c_int32)]


class _State(C.Structure):
    _fields_ = [("O", C.c_void_p), ("m_O", C.c_void_p), ("v_O", C.c_void_p), ("g_O", C.c_void_p),
                ("P", C.c_void_p), ("coeffs", C.c_void_p), ("m_c", C.c_void_p),
                ("v_c", C.c_void_p), ("z_um", C.c_void_p), ("m_z", C.c_void_p),
                ("v_z", C.c_void_p), ("g_par", C.c_void_p), ("loss", C.c_void_p),
                ("t", C.c_int32)]


class _Params(C.Structure):
    _fields_ = [("O", C.c_void_p), ("coeffs", C.c_void_p), ("z_um", C.c_void_p),
                ("geom", C.c_void_p), ("gamma", C.c_void_p)]


class _Grads(C.Structure):
    _fields_ = [("g_O", C.c_void_p), ("g_par", C.c_void_p), ("g_geom", C.c_void_p),
                ("g_gamma", C.c_void_p), ("loss", C.c_void_p), ("oob", C.c_void_p)]


class _Geometry(C.Structure):
    _fields_ = [("geom", C.c_void_p), ("m_geom", C.c_void_p), ("v_geom", C.c_void_p),
                ("g_geom", C.c_void_p), ("lr_shift_mm", C.c_double), ("lr_rot_rad", C.c_double),
                ("lr_height_mm", C.c_double), ("learn", C.c_int32)]


EXPORTS = {
    "fpm_plan_create": [C.POINTER(_Desc), C.c_void_p, C.POINTER(C.c_void_p)],
    "fpm_plan_destroy": [C.c_void_p],
    "fpm_plan_info": [C.c_void_p, C.POINTER(_Info)],
    "fpm_strerror": [C.c_int],
    "fpm_last_error": [],
    "fpm_build_tag": [],
    "fpm_led_shifts": [C.POINTER(_Desc), C.POINTER(_Grid), C.c_void_p, C.c_void_p, C.c_void_p],
    "fpm_pupil": [C.c_void_p, C.c_void_p, C.c_int32, C.c_void_p, C.c_void_p, C.c_void_p],
    "fpm_forward": [C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p, C.c_int32, C.c_void_p,
                    C.c_void_p, C.c_void_p, C.c_void_p],
    "fpm_backward": [C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p, C.c_int32, C.c_void_p,
                     C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p],
    "fpm_backward_noalloc": [C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p, C.c_int32,
                             C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p,
                             C.c_void_p],
    "fpm_pupil_grad": [C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p],
    "fpm_step": [C.c_void_p, C.POINTER(_State), C.POINTER(_HParams), C.c_void_p, C.c_int32,
                 C.c_void_p, C.c_void_p, C.c_void_p],
    "fpm_run": [C.c_void_p, C.POINTER(_State), C.POINTER(_HParams), C.c_void_p, C.c_void_p,
                C.c_int32, C.c_void_p, C.c_void_p, C.c_void_p],
    "fpm_loss_grad": [C.c_void_p, C.POINTER(_Grid), C.POINTER(_Params), C.c_void_p, C.c_int32,
                      C.c_void_p, C.POINTER(_Grads), C.c_void_p],
    "fpm_run_multi": [C.c_void_p, C.POINTER(_Grid), C.POINTER(_State), C.POINTER(_Geometry),
                      C.POINTER(_HParams), C.c_void_p, C.c_void_p, C.c_int32, C.c_void_p,
                      C.c_void_p],
    "fpm_hr_transform": [C.c_void_p, C.c_void_p, C.c_void_p, C.c_int32, C.c_void_p],
    "fpm_init_spectrum": [C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p],
    "fpm_refocus": [C.c_void_p, C.c_void_p, C.c_void_p, C.c_int32, C.c_void_p, C.c_void_p],
    "fpm_timing_enable": [C.c_void_p, C.c_int32],
    "fpm_timing_repeat": [C.c_void_p, C.c_int32, C.c_int32],
    "fpm_plan_set_loss": [C.c_void_p, C.c_int32],
    "fpm_plan_set_shifts": [C.c_void_p, C.c_void_p, C.c_void_p],
    "fpm_timing_collect": [C.c_void_p, C.c_int32, C.c_void_p, C.c_void_p, C.c_void_p,
                           C.POINTER(C.c_int32)],
}

_lib = None


def load(path: str = LIB_PATH):
    """Load libfpm.so and declare its signatures; raises if it is missing."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise FpmError(f"{path} not found: build it with `python -m paper_2408_13782_amd.build` "
                       "(the HIP library is required; there is no CPU fallback)")
    lib = C.CDLL(path)
    for name, argtypes in EXPORTS.items():
        fn = getattr(lib, name)
        fn.argtypes = argtypes
        fn.restype = (C.c_char_p if name in ("fpm_strerror", "fpm_last_error", "fpm_build_tag")
                      else C.c_int)
    _lib = lib
    return lib


def build_tag() -> str:
    """Digest of the sources the loaded library was built from (fpm_build_tag)."""
    return load().fpm_build_tag().decode()


def _check(rc: int):
    if rc != FPM_OK:
        lib = load()
        raise FpmError(f"{lib.fpm_strerror(rc).decode()} ({rc}): {lib.fpm_last_error().decode()}")


def _ptr(t):
    return None if t is None else C.c_void_p(t.data_ptr())


def _need(t, name, dtype, shape=None, min_numel=None, optional=False):
    """Check a device tensor before its pointer crosses the ABI (sizes are not re-checked there)."""
    import torch
    if t is None:
        if optional:
            return
        raise FpmError(f"{name} is required")
    if not isinstance(t, torch.Tensor) or not t.is_cuda:
        raise FpmError(f"{name} must be a device tensor")
    if t.dtype != dtype:
        raise FpmError(f"{name} must be {dtype}, got {t.dtype}")
    if not t.is_contiguous():
        raise FpmError(f"{name} must be contiguous")
    if shape is not None and tuple(t.shape) != tuple(shape):
        raise FpmError(f"{name} must have shape {tuple(shape)}, got {tuple(t.shape)}")
    if min_numel is not None and t.numel() < min_numel:
        raise FpmError(f"{name} needs at least {min_numel} elements")


def _stream(device=None):
    import torch
    return C.c_void_p(torch.cuda.current_stream(device).cuda_stream)


def _desc(n_lr, upsample, n_led, max_batch, wavelength_um, na, mag, pixel_um) -> _Desc:
    return _Desc(n_lr, upsample, n_led, max_batch, wavelength_um, na, mag, pixel_um)


def led_shifts(n_lr: int, wavelength_um: float, mag: float, pixel_um: float, n_side: int,
               pitch_mm: float, height_mm: float, shift_x_mm=0.0, shift_y_mm=0.0, rot_rad=0.0,
               dh_mm=0.0, roi_x_mm=0.0, roi_y_mm=0.0):
    """(k [n_led,2] 1/um, s [n_led,2] fractional px, nearest [n_led,2] int32), (row, col)."""
    lib = load()
    n_led = n_side * n_side
    d = _desc(n_lr, 1, n_led, 1, wavelength_um, 0.1, mag, pixel_um)
    g = _Grid(n_side, pitch_mm, height_mm, shift_x_mm, shift_y_mm, rot_rad, dh_mm, roi_x_mm,
              roi_y_mm)
    k = np.zeros((n_led, 2), np.float64)
    s = np.zeros((n_led, 2), np.float64)
    nearest = np.zeros((n_led, 2), np.int32)
    _check(lib.fpm_led_shifts(C.byref(d), C.byref(g), k.ctypes.data, s.ctypes.data,
                              nearest.ctypes.data))
    return k, s, nearest


@dataclass
class LedGrid:
    """Nominal square LED array (host description); learned errors are added to it."""
    n_side: int
    pitch_mm: float
    height_mm: float
    shift_x_mm: float = 0.0
    shift_y_mm: float = 0.0
    rot_rad: float = 0.0
    dh_mm: float = 0.0
    roi_x_mm: float = 0.0
    roi_y_mm: float = 0.0

    def c(self) -> _Grid:
        return _Grid(self.n_side, self.pitch_mm, self.height_mm, self.shift_x_mm,
                     self.shift_y_mm, self.rot_rad, self.dh_mm, self.roi_x_mm, self.roi_y_mm)


@dataclass
class HParams:
    lr_object: float = 1e-2
    lr_zernike: float = 1e-2
    lr_z: float = 0.1
    beta1: float = 0.9
    beta2: float = 0.999
    eps: float = 1e-8
    learn_zernike: bool = False
    learn_z: bool = False

    def c(self) -> _HParams:
        return _HParams(self.lr_object, self.lr_zernike, self.lr_z, self.beta1, self.beta2,
                        self.eps, int(self.learn_zernike), int(self.learn_z))


class State:
    """Device-resident reconstruction state (spectrum, pupil parameters, Adam moments)."""

    def __init__(self, plan: "Plan", O0, coeffs0=None, z0: float = 0.0, P0=None):
        import torch
        dev = O0.device
        M, N = plan.M, plan.N
        assert O0.shape == (M, M) and O0.dtype == torch.complex64 and O0.is_cuda
        self.O = O0.clone().contiguous()
        self.m_O = torch.zeros((M, M), dtype=torch.complex64, device=dev)
        self.v_O = torch.zeros((M, M), dtype=torch.complex64, device=dev)
        self.coeffs = torch.zeros(N_ZERN, dtype=torch.float32, device=dev)
        if coeffs0 is not None:
            self.coeffs.copy_(torch.as_tensor(np.asarray(coeffs0, np.float32)))
        self.m_c = torch.zeros(N_ZERN, dtype=torch.float32, device=dev)
        self.v_c = torch.zeros(N_ZERN, dtype=torch.float32, device=dev)
        self.z_um = torch.full((1,), float(z0), dtype=torch.float32, device=dev)
        self.m_z = torch.zeros(1, dtype=torch.float32, device=dev)
        self.v_z = torch.zeros(1, dtype=torch.float32, device=dev)
        self.g_par = torch.zeros(N_PAR, dtype=torch.float64, device=dev)
        self.loss = torch.zeros(1, dtype=torch.float64, device=dev)
        if P0 is not None:
            self.P = P0.clone().contiguous()
        else:
            self.P = plan.pupil(self.coeffs, self.z_um)
        self.t = 0
        self._c = _State()

    def c(self) -> _State:
        s = self._c
        s.O, s.m_O, s.v_O, s.g_O = (self.O.data_ptr(), self.m_O.data_ptr(), self.v_O.data_ptr(),
                                    None)
        s.P = self.P.data_ptr()
        s.coeffs, s.m_c, s.v_c = self.coeffs.data_ptr(), self.m_c.data_ptr(), self.v_c.data_ptr()
        s.z_um, s.m_z, s.v_z = self.z_um.data_ptr(), self.m_z.data_ptr(), self.v_z.data_ptr()
        s.g_par = self.g_par.data_ptr()
        s.loss = self.loss.data_ptr()
        s.t = self.t
        return s

    _SAVED = ("O", "m_O", "v_O", "P", "coeffs", "m_c", "v_c", "z_um", "m_z", "v_z", "g_par",
              "loss")

    def save(self, path: str, **extra):
        """Checkpoint: every tensor of the state, the Adam step count t and any
        caller values (e.g. the schedule position) to an .npz file. Resuming from
        it (State.load) continues bitwise as if never interrupted."""
        import torch
        torch.cuda.synchronize()
        arrays = {k: getattr(self, k).cpu().numpy() for k in self._SAVED}
        np.savez(path, t=np.int64(self.t), **arrays,
                 **{"extra_" + k: np.asarray(v) for k, v in extra.items()})

    @classmethod
    def load(cls, plan: "Plan", path: str):
        """(state, extra) from a checkpoint written by save, on the current device."""
        import torch
        dev = torch.device("cuda", torch.cuda.current_device())
        with np.load(path, allow_pickle=False) as f:
            st = cls(plan, torch.as_tensor(f["O"]).to(dev), P0=torch.as_tensor(f["P"]).to(dev))
            for k in cls._SAVED:
                t = getattr(st, k)
                src = torch.as_tensor(f[k])
                if tuple(src.shape) != tuple(t.shape) or src.dtype != t.dtype:
                    raise FpmError(f"checkpoint entry {k} does not fit the plan")
                t.copy_(src.to(dev))
            st.t = int(f["t"])
            extra = {k[len("extra_"):]: f[k] for k in f.files if k.startswith("extra_")}
        torch.cuda.synchronize()
        return st, extra


class Geometry:
    """Learned LED-array errors (shift_x_mm, shift_y_mm, rot_rad, dh_mm) with their Adam
    moments, on the device (float64), for Plan.run_multi."""

    def __init__(self, geom0=(0.0, 0.0, 0.0, 0.0), lr_shift_mm=5e-3, lr_rot_rad=5e-4,
                 lr_height_mm=2e-2, learn=True, device="cuda"):
        import torch
        self.geom = torch.tensor(np.asarray(geom0, np.float64), device=device)
        self.m = torch.zeros(4, dtype=torch.float64, device=device)
        self.v = torch.zeros(4, dtype=torch.float64, device=device)
        self.g = torch.zeros(4, dtype=torch.float64, device=device)
        self.lr = (float(lr_shift_mm), float(lr_rot_rad), float(lr_height_mm))
        self.learn = bool(learn)
        self._c = _Geometry()

    def c(self) -> _Geometry:
        g = self._c
        g.geom, g.m_geom, g.v_geom, g.g_geom = (self.geom.data_ptr(), self.m.data_ptr(),
                                                self.v.data_ptr(), self.g.data_ptr())
        g.lr_shift_mm, g.lr_rot_rad, g.lr_height_mm = self.lr
        g.learn = int(self.learn)
        return g


class Plan:
    """One reconstruction problem's sizes, optics and LED table, with its scratch."""

    def __init__(self, n_lr: int, upsample: int, shifts, max_batch: int, wavelength_um: float,
                 na: float, mag: float, pixel_um: float):
        lib = load()
        shifts = np.ascontiguousarray(np.asarray(shifts, np.int32).reshape(-1, 2))
        self.N, self.s, self.M = int(n_lr), int(upsample), int(n_lr) * int(upsample)
        self.n_led = shifts.shape[0]
        self.max_batch = int(max_batch)
        self.shifts = shifts
        d = _desc(self.N, self.s, self.n_led, self.max_batch, wavelength_um, na, mag, pixel_um)
        h = C.c_void_p()
        _check(lib.fpm_plan_create(C.byref(d), shifts.ctypes.data, C.byref(h)))
        self._h = h
        info = _Info()
        _check(lib.fpm_plan_info(h, C.byref(info)))
        self.info = info
        self._lib = lib
        self._kinds = self._read_kernel_kinds()

    def set_shifts(self, shifts):
        """Replace the LED table (fpm_plan_set_shifts), e.g. for another tile's ROI centre."""
        shifts = np.ascontiguousarray(np.asarray(shifts, np.int32).reshape(-1, 2))
        if shifts.shape[0] != self.n_led:
            raise FpmError(f"expected {self.n_led} LED offsets, got {shifts.shape[0]}")
        _check(self._lib.fpm_plan_set_shifts(self._h, shifts.ctypes.data, _stream()))
        self.shifts = shifts
        info = _Info()
        _check(self._lib.fpm_plan_info(self._h, C.byref(info)))
        self.info = info

    LOSSES = {"amplitude": 0, "intensity": 1}

    def set_loss(self, kind: str):
        """Loss of later calls: 'amplitude' (default) or 'intensity' (fpm_plan_set_loss)."""
        if kind not in self.LOSSES:
            raise FpmError(f"unknown loss {kind!r}")
        _check(self._lib.fpm_plan_set_loss(self._h, self.LOSSES[kind]))
        self.loss_kind = kind

    def close(self):
        if getattr(self, "_h", None) is not None and self._h.value:
            self._lib.fpm_plan_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # -- entry points -------------------------------------------------------

    # -- argument checks ------------------------------------------------------

    def _spectrum(self, O, name="O"):
        import torch
        _need(O, name, torch.complex64, (self.M, self.M))

    def _pupil(self, P, name="P"):
        import torch
        _need(P, name, torch.complex64, (self.N, self.N))

    @staticmethod
    def _leds(leds):
        """LED ids as a host int32 array (the library validates the values)."""
        arr = np.ascontiguousarray(np.asarray(leds, dtype=np.int32).reshape(-1))
        return arr, int(arr.size)

    def _images(self, A, gamma):
        import torch
        _need(A, "meas_amp", torch.float32, (self.n_led, self.N, self.N))
        _need(gamma, "gamma", torch.float32, (self.n_led,), optional=True)

    def pupil(self, coeffs=None, z_um=None, out=None):
        import torch
        dev = torch.device("cuda", torch.cuda.current_device())
        if out is None:
            out = torch.empty((self.N, self.N), dtype=torch.complex64, device=dev)
        self._pupil(out, "out")
        _need(coeffs, "coeffs", torch.float32, optional=True)
        _need(z_um, "z_um", torch.float32, min_numel=1, optional=True)
        if coeffs is not None and coeffs.numel() > N_ZERN:
            raise FpmError("at most 15 Zernike coefficients")
        n = 0 if coeffs is None else int(coeffs.numel())
        _check(self._lib.fpm_pupil(self._h, _ptr(coeffs), n, _ptr(z_um), _ptr(out), _stream()))
        return out

    def forward(self, O, P, leds, gamma=None, with_field=False):
        import torch
        self._spectrum(O)
        self._pupil(P)
        ids, B = self._leds(leds)
        _need(gamma, "gamma", torch.float32, (self.n_led,), optional=True)
        amp = torch.empty((B, self.N, self.N), dtype=torch.float32, device=O.device)
        field = (torch.empty((B, self.N, self.N), dtype=torch.complex64, device=O.device)
                 if with_field else None)
        _check(self._lib.fpm_forward(self._h, _ptr(O), _ptr(P), ids.ctypes.data, B, _ptr(gamma),
                                     _ptr(amp), _ptr(field), _stream()))
        return (amp, field) if with_field else amp

    def backward(self, O, P, leds, meas_amp, gO, gP=None, loss=None, gamma=None):
        import torch
        self._spectrum(O)
        self._pupil(P)
        ids, B = self._leds(leds)
        self._images(meas_amp, gamma)
        self._spectrum(gO, "gO")
        _need(gP, "gP", torch.complex64, (self.N, self.N), optional=True)
        _need(loss, "loss", torch.float64, min_numel=1, optional=True)
        _check(self._lib.fpm_backward(self._h, _ptr(O), _ptr(P), ids.ctypes.data, B, _ptr(gamma),
                                      _ptr(meas_amp), _ptr(gO), _ptr(gP), _ptr(loss), _stream()))

    def backward_noalloc(self, O, P, leds, meas_amp, gO, gP=None, loss=None, gamma=None):
        """backward() through fpm_backward_noalloc: no device memory of the plan's,
        a static array of the library instead (see include/fpm.h for its limit)."""
        import torch
        self._spectrum(O)
        self._pupil(P)
        ids, B = self._leds(leds)
        self._images(meas_amp, gamma)
        self._spectrum(gO, "gO")
        _need(gP, "gP", torch.complex64, (self.N, self.N), optional=True)
        _need(loss, "loss", torch.float64, min_numel=1, optional=True)
        _check(self._lib.fpm_backward_noalloc(self._h, _ptr(O), _ptr(P), ids.ctypes.data, B,
                                              _ptr(gamma), _ptr(meas_amp), _ptr(gO), _ptr(gP),
                                              _ptr(loss), _stream()))

    def pupil_grad(self, gP, P, g_par):
        import torch
        self._pupil(gP, "gP")
        self._pupil(P)
        _need(g_par, "g_par", torch.float64, min_numel=N_PAR)
        _check(self._lib.fpm_pupil_grad(self._h, _ptr(gP), _ptr(P), _ptr(g_par), _stream()))

    def step(self, state: State, hp: HParams, leds, meas_amp, gamma=None):
        ids, B = self._leds(leds)
        self._images(meas_amp, gamma)
        self._spectrum(state.O)
        self._pupil(state.P)
        cs = state.c()
        hc = hp.c()
        _check(self._lib.fpm_step(self._h, C.byref(cs), C.byref(hc), ids.ctypes.data, B, _ptr(gamma),
                                  _ptr(meas_amp), _stream()))
        state.t = cs.t

    def run(self, state: State, hp: HParams, leds_flat, batch_sizes, meas_amp, gamma=None):
        """Consecutive updates: batch i is the next batch_sizes[i] ids of leds_flat."""
        sizes = np.ascontiguousarray(np.asarray(batch_sizes, np.int32))
        ids, n = self._leds(leds_flat)
        if int(sizes.sum()) > n:
            raise FpmError("batch sizes exceed the number of LED ids")
        self._images(meas_amp, gamma)
        self._spectrum(state.O)
        self._pupil(state.P)
        cs = state.c()
        hc = hp.c()
        _check(self._lib.fpm_run(self._h, C.byref(cs), C.byref(hc), ids.ctypes.data,
                                 sizes.ctypes.data, int(sizes.size), _ptr(gamma), _ptr(meas_amp),
                                 _stream()))
        state.t = cs.t

    def prepare_run(self, state: State, hp: HParams, leds_flat, batch_sizes, meas_amp,
                    gamma=None):
        """fpm_run with its batches, images and hyper-parameters checked and
        marshalled once: the returned callable issues the run (the same batches
        each time, continuing from the state's step count) on the stream that is
        current now, reading the state's tensors at each call. For runs issued
        from Python in a loop, whose argument checks would otherwise precede
        every call."""
        sizes = np.ascontiguousarray(np.asarray(batch_sizes, np.int32))
        ids, n = self._leds(leds_flat)
        if int(sizes.sum()) > n:
            raise FpmError("batch sizes exceed the number of LED ids")
        self._images(meas_amp, gamma)
        self._spectrum(state.O)
        self._pupil(state.P)
        cs = state.c()
        hc = hp.c()
        lib = self._lib
        args = (self._h, C.byref(cs), C.byref(hc), ids.ctypes.data, sizes.ctypes.data,
                int(sizes.size), _ptr(gamma), _ptr(meas_amp), _stream())
        held = (ids, sizes, meas_amp, gamma, hp)

        def go():
            self._spectrum(state.O)
            self._pupil(state.P)
            state.c()
            _check(lib.fpm_run(*args))
            state.t = cs.t
        go.held = held
        return go

    def run_multi(self, grid: LedGrid, state: State, geometry: Geometry, hp: HParams, leds_flat,
                  batch_sizes, meas_amp):
        """Fused multi-parameter updates (fpm_run_multi): spectrum, Zernikes, defocus and
        LED-array geometry, batch i being the next batch_sizes[i] ids of leds_flat."""
        import torch
        sizes = np.ascontiguousarray(np.asarray(batch_sizes, np.int32))
        ids, n = self._leds(leds_flat)
        if int(sizes.sum()) > n:
            raise FpmError("batch sizes exceed the number of LED ids")
        self._images(meas_amp, None)
        self._spectrum(state.O)
        self._pupil(state.P)
        for t in (geometry.geom, geometry.m, geometry.v, geometry.g):
            _need(t, "geometry", torch.float64, (4,))
        cs = state.c()
        hc = hp.c()
        gc = grid.c()
        _check(self._lib.fpm_run_multi(self._h, C.byref(gc), C.byref(cs), C.byref(geometry.c()),
                                       C.byref(hc), ids.ctypes.data, sizes.ctypes.data,
                                       int(sizes.size), _ptr(meas_amp), _stream()))
        state.t = cs.t

    def loss_grad(self, grid: LedGrid, O, leds, meas_amp, coeffs=None, z_um=None, geom=None,
                  gamma=None, grads=None):
        """Loss and gradients of one batch for every parameter group (fpm_loss_grad).

        grads: dict of preallocated accumulators (added to); missing entries are
        allocated zeroed. Returns the dict with 'loss', 'g_O', 'g_par', 'g_geom',
        'g_gamma', 'oob'.
        """
        import torch
        self._spectrum(O)
        ids, B = self._leds(leds)
        self._images(meas_amp, gamma)
        _need(coeffs, "coeffs", torch.float32, (N_ZERN,), optional=True)
        _need(z_um, "z_um", torch.float32, (1,), optional=True)
        _need(geom, "geom", torch.float64, (4,), optional=True)
        dev = O.device
        g = {} if grads is None else dict(grads)
        g.setdefault("loss", torch.zeros(1, dtype=torch.float64, device=dev))
        g.setdefault("g_O", torch.zeros((self.M, self.M), dtype=torch.complex64, device=dev))
        g.setdefault("g_par", torch.zeros(N_PAR, dtype=torch.float64, device=dev))
        g.setdefault("g_geom", torch.zeros(4, dtype=torch.float64, device=dev))
        g.setdefault("g_gamma", torch.zeros(self.n_led, dtype=torch.float64, device=dev))
        g.setdefault("oob", torch.zeros(1, dtype=torch.int32, device=dev))
        self._spectrum(g["g_O"], "g_O")
        pr = _Params(O.data_ptr(), None if coeffs is None else coeffs.data_ptr(),
                     None if z_um is None else z_um.data_ptr(),
                     None if geom is None else geom.data_ptr(),
                     None if gamma is None else gamma.data_ptr())
        gr = _Grads(g["g_O"].data_ptr(), g["g_par"].data_ptr(), g["g_geom"].data_ptr(),
                    g["g_gamma"].data_ptr(), g["loss"].data_ptr(), g["oob"].data_ptr())
        gc = grid.c()
        _check(self._lib.fpm_loss_grad(self._h, C.byref(gc), C.byref(pr), ids.ctypes.data, B,
                                       _ptr(meas_amp), C.byref(gr), _stream()))
        return g

    def hr_transform(self, x, direction: int, out=None):
        import torch
        self._spectrum(x, "in")
        if out is None:
            out = torch.empty_like(x)
        self._spectrum(out, "out")
        _check(self._lib.fpm_hr_transform(self._h, _ptr(x), _ptr(out), int(direction), _stream()))
        return out

    def init_spectrum(self, centre_amp, out=None):
        import torch
        _need(centre_amp, "centre_amp", torch.float32, (self.N, self.N))
        if out is None:
            out = torch.empty((self.M, self.M), dtype=torch.complex64, device=centre_amp.device)
        self._spectrum(out, "out")
        _check(self._lib.fpm_init_spectrum(self._h, _ptr(centre_amp), _ptr(out), _stream()))
        return out

    def timing(self, enable: bool):
        _check(self._lib.fpm_timing_enable(self._h, int(bool(enable))))

    def kernel_kinds(self) -> list:
        """Names of the kernel kinds the timing calls report, in index order."""
        return list(self._kinds)

    def _read_kernel_kinds(self) -> list:
        # a collection with nothing recorded: only the names come back
        kmax = 32
        names = (C.c_char_p * kmax)()
        total = np.zeros(kmax, np.float64)
        counts = np.zeros(kmax, np.int32)
        nk = C.c_int32(0)
        _check(self._lib.fpm_timing_collect(self._h, kmax, C.cast(names, C.c_void_p),
                                            total.ctypes.data, counts.ctypes.data, C.byref(nk)))
        return [names[i].decode() for i in range(nk.value)]

    def timing_repeat(self, kind, reps: int):
        """Issue launches of kernel `kind` (a name, or None for none) `reps` times
        back to back while timing (fpm_timing_repeat); the state is not kept valid."""
        idx = -1 if kind is None else self.kernel_kinds().index(kind)
        _check(self._lib.fpm_timing_repeat(self._h, idx, int(reps)))

    def timing_collect(self) -> dict:
        """{kernel name: (total ms, launches)} since the last collection."""
        kmax = 32
        names = (C.c_char_p * kmax)()
        total = np.zeros(kmax, np.float64)
        counts = np.zeros(kmax, np.int32)
        nk = C.c_int32(0)
        _check(self._lib.fpm_timing_collect(self._h, kmax, C.cast(names, C.c_void_p),
                                            total.ctypes.data, counts.ctypes.data, C.byref(nk)))
        return {names[i].decode(): (float(total[i]), int(counts[i])) for i in range(nk.value)
                if counts[i] > 0}

    def refocus(self, O, z_um, out=None):
        import torch
        self._spectrum(O)
        _need(z_um, "z_um", torch.float32)
        nz = int(z_um.numel())
        if out is None:
            out = torch.empty((nz, self.M, self.M), dtype=torch.complex64, device=O.device)
        _need(out, "out", torch.complex64, (nz, self.M, self.M))
        _check(self._lib.fpm_refocus(self._h, _ptr(O), _ptr(z_um), nz, _ptr(out), _stream()))
        return out
