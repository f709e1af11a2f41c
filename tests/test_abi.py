"""Host-side checks of the C-ABI library (no GPU needed).

The library must load and export every entry point include/fpm.h declares;
its FP64 host routine for LED geometry must agree with the oracle; the
product package must not reach the oracle.
"""
import os
import re

import numpy as np
import pytest

from oracle import fpm_oracle as fo
from paper_2408_13782_amd import fpm, inputs, problem

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "fpm.h")
PKG = os.path.join(ROOT, "paper_2408_13782_amd")


SERVE_HEADER = os.path.join(ROOT, "include", "fpm_serve.h")


def declared_functions(header=HEADER):
    src = open(header).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(fpm_[a-z_0-9]+)\s*\(", src)))


def test_header_declares_the_boundary():
    names = declared_functions()
    for required in ("fpm_plan_create", "fpm_plan_destroy", "fpm_forward", "fpm_backward",
                     "fpm_step", "fpm_refocus", "fpm_pupil", "fpm_pupil_grad",
                     "fpm_hr_transform", "fpm_init_spectrum", "fpm_led_shifts", "fpm_strerror"):
        assert required in names


def test_library_loads_and_exports_every_declared_symbol():
    lib = fpm.load()
    for header in (HEADER, SERVE_HEADER):
        for name in declared_functions(header):
            assert hasattr(lib, name), name
    assert set(declared_functions()) == set(fpm.EXPORTS)


def test_server_binding_covers_the_server_header():
    from paper_2408_13782_amd import serving
    bound = set(serving._SIGS) | {"fpm_server_clock_ms"}
    assert set(declared_functions(SERVE_HEADER)) == bound


def test_error_strings():
    lib = fpm.load()
    assert lib.fpm_strerror(0) == b"ok"
    assert lib.fpm_strerror(-1) == b"invalid argument"
    assert lib.fpm_strerror(-4) == b"unsupported size"
    assert lib.fpm_strerror(-5) == b"non-finite loss"


def test_status_codes_of_the_binding_match_the_header():
    src = open(HEADER).read()
    codes = dict((k, int(v)) for k, v in re.findall(r"\b(FPM_E[A-Z]+|FPM_OK)\s*=\s*(-?\d+)", src))
    assert len(codes) == 6
    for name, value in codes.items():
        assert getattr(fpm, name) == value, name
        assert fpm.load().fpm_strerror(value) != b"unknown error", name


@pytest.mark.parametrize("name", ["small", "paper", "large"])
@pytest.mark.parametrize("geometry", [(0.0, 0.0, 0.0, 0.0, 0.0, 0.0),
                                      (0.31, -0.27, 0.021, 1.3, 0.0, 0.0),
                                      (0.0, 0.0, 0.0, 0.0, 1.7, -2.3),       # off-axis tile
                                      (0.31, -0.27, 0.021, 1.3, -0.9, 0.45)])
def test_led_shifts_match_oracle(name, geometry):
    w = inputs.workload(name)
    opt = fo.Optics(w.wavelength_um, w.na, w.mag, w.pixel_um, w.n_lr, w.upsample)
    k_o = fo.led_wavevectors(opt, w.n_side, w.pitch_mm, w.height_mm, *geometry)
    s_o = fo.led_shifts(opt, k_o)
    n_o = fo.nearest_shifts(s_o)
    k, s, n = fpm.led_shifts(w.n_lr, w.wavelength_um, w.mag, w.pixel_um, w.n_side, w.pitch_mm,
                             w.height_mm, *geometry)
    np.testing.assert_allclose(k, k_o, rtol=1e-14, atol=1e-15)
    np.testing.assert_allclose(s, s_o, rtol=1e-13, atol=1e-12)
    np.testing.assert_array_equal(n, n_o)          # integer decision: bit-exact


def test_schedule_matches_oracle_batches():
    perms = inputs.led_permutations(49, 5, seed=2)
    want = fo.batches_from_permutations(perms, 8)
    got = problem.schedule(perms, 8)
    assert [list(map(int, b)) for b in got] == want


def test_product_package_never_reaches_the_oracle():
    for dirpath, _, files in os.walk(PKG):
        for f in files:
            if f.endswith((".py", ".hip", ".hpp", ".cpp", ".h")):
                text = open(os.path.join(dirpath, f)).read()
                assert not re.search(r"^\s*(from|import)\s+oracle", text, re.M), f
                assert "fpm_oracle" not in text, f


def test_library_build_tag_matches_the_sources():
    """The in-tree libfpm.so was built from the sources in this tree (its
    fpm_build_tag is the digest of csrc/ and include/)."""
    from paper_2408_13782_amd import build
    tag = fpm.build_tag()
    assert len(tag) == 16 and tag == build.source_tag()
