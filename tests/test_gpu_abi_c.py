"""The C ABI driven from plain C (tests/native/abi_solve.c, no Python or torch
in the process): a whole solve from files equals the same solve through the
Python binding bitwise."""
import os
import subprocess
import sys

import numpy as np
import pytest

from paper_2408_13782_amd import fpm, inputs, problem

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
DRIVER = os.path.join(ROOT, "tests", "native", "abi_solve")

torch = pytest.importorskip("torch")


def say(msg):
    print(f"[gpu] {msg}", flush=True)
    sys.stdout.flush()


def test_driver_is_built_and_checks_its_arguments():
    assert os.access(DRIVER, os.X_OK), "run __graft_entry__.build() first"
    res = subprocess.run([DRIVER], capture_output=True, text=True, timeout=60)
    assert res.returncode == 2 and "usage" in res.stderr


@pytest.mark.gpu
def test_c_program_solve_equals_the_python_binding(tmp_path):
    assert torch.cuda.is_available()
    fpm.load()
    w = inputs.workload("small", epochs=3, learn_zernike=True)
    say("solve through the C ABI from a C program")
    prob = problem.make_plan(w)
    problem.simulate(prob, seed=7)
    meas = prob.meas_amp.cpu().numpy().astype(np.float32)
    perms = inputs.led_permutations(w.n_led, w.epochs, seed=8)
    sched = problem.flatten_schedule(problem.schedule(perms, w.batch))
    meas.tofile(tmp_path / "meas.bin")
    np.asarray(sched.sizes, np.int32).tofile(tmp_path / "sizes.bin")
    np.asarray(sched.flat, np.int32).tofile(tmp_path / "leds.bin")
    (tmp_path / "params.txt").write_text(" ".join(str(x) for x in (
        w.n_lr, w.upsample, w.n_side, w.pitch_mm, w.height_mm, w.wavelength_um, w.na, w.mag,
        w.pixel_um, w.batch, len(sched.sizes), w.lr_object, w.lr_zernike, 1)))
    res = subprocess.run([DRIVER, str(tmp_path)], capture_output=True, text=True, timeout=120)
    assert res.returncode == 0, res.stdout + res.stderr
    O_c = np.fromfile(tmp_path / "O.bin", np.complex64).reshape(w.m_hr, w.m_hr)
    c_c = np.fromfile(tmp_path / "coeffs.bin", np.float32)
    loss_c = np.fromfile(tmp_path / "loss.bin", np.float64)
    # the same solve through the Python binding
    st = fpm.State(prob.plan, problem.initial_spectrum(prob))
    prob.plan.run(st, problem.hparams(w), sched.flat, sched.sizes, prob.meas_amp)
    torch.cuda.synchronize()
    np.testing.assert_array_equal(O_c, st.O.cpu().numpy())
    np.testing.assert_array_equal(c_c, st.coeffs.cpu().numpy())
    np.testing.assert_array_equal(loss_c, st.loss.cpu().numpy())
    assert np.any(c_c[1:] != 0.0)
