"""GPU test of the reconstruction command: an image stack on disk through
`python -m paper_2408_13782_amd.reconstruct` equals the same solve through the
library directly (bitwise), intensities are accepted in place of amplitudes,
and a stack of the wrong shape is refused."""
import sys

import numpy as np
import pytest

from paper_2408_13782_amd import fpm, inputs, problem

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


def say(msg):
    print(f"[gpu] {msg}", flush=True)
    sys.stdout.flush()


def test_reconstruct_command_equals_a_direct_solve(tmp_path):
    assert torch.cuda.is_available()
    fpm.load()
    from paper_2408_13782_amd import reconstruct
    w = inputs.workload("small", epochs=4, learn_zernike=True)
    say("reconstruct command on a 7x7 stack")
    prob = problem.make_plan(w)
    problem.simulate(prob, seed=2)
    stack = prob.meas_amp.cpu().numpy()
    np.save(tmp_path / "amp.npy", stack)
    np.save(tmp_path / "int.npy", stack.astype(np.float64) ** 2)
    common = ["--grid", str(w.n_side), "--pitch-mm", str(w.pitch_mm), "--height-mm",
              str(w.height_mm), "--wavelength-um", str(w.wavelength_um), "--na", str(w.na),
              "--mag", str(w.mag), "--pixel-um", str(w.pixel_um), "--upsample",
              str(w.upsample), "--batch", str(w.batch), "--epochs", str(w.epochs),
              "--learn-zernike", "--seed", "5"]
    reconstruct.main(["--images", str(tmp_path / "amp.npy"), "--out", str(tmp_path / "a.npz")]
                     + common)
    got = np.load(tmp_path / "a.npz")
    # the same solve through the library
    st = fpm.State(prob.plan, problem.initial_spectrum(prob))
    perms = inputs.led_permutations(w.n_led, w.epochs, seed=5)
    sched = problem.flatten_schedule(problem.schedule(perms, w.batch))
    prob.plan.run(st, problem.hparams(w), sched.flat, sched.sizes, prob.meas_amp)
    torch.cuda.synchronize()
    np.testing.assert_array_equal(got["spectrum"], st.O.cpu().numpy())
    np.testing.assert_array_equal(got["zernike"], st.coeffs.cpu().numpy())
    assert got["object"].shape == (w.m_hr, w.m_hr) and got["epoch_loss"].shape == (w.epochs,)
    assert got["epoch_loss"][-1] < got["epoch_loss"][0]
    # intensities: square roots taken on the host, the same solve up to their
    # rounding (which Adam's sign-like first steps may amplify where a gradient
    # is at its rounding level)
    reconstruct.main(["--images", str(tmp_path / "int.npy"), "--intensity-images",
                      "--out", str(tmp_path / "b.npz")] + common)
    alt = np.load(tmp_path / "b.npz")
    ref = got["object"].astype(np.complex128)
    assert np.linalg.norm(alt["object"] - ref) <= 1e-2 * np.linalg.norm(ref)
    # a stack whose LED count does not match the grid
    args = reconstruct.parse(["--images", "x", "--out", "y"] + common)
    with pytest.raises(ValueError):
        reconstruct.reconstruct(args, stack[:-1])
