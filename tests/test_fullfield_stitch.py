"""Host logic of full-field tiling: tile geometry and stitching (no GPU)."""
import numpy as np

from paper_2408_13782_amd import fullfield, inputs


def _field():
    w = inputs.workload("small", n_lr=64, n_side=7)
    return fullfield.Field(w, tiles=3, overlap=16)


def test_tiles_cover_the_field_with_the_stated_overlap():
    f = _field()
    assert f.size_lr == 2 * 48 + 64 and f.size_hr == 4 * f.size_lr
    x0, y0 = f.roi_mm(0, 0)
    x2, y2 = f.roi_mm(2, 2)
    assert np.isclose(x0, -x2) and np.isclose(y0, -y2)          # symmetric about the centre
    assert np.isclose(f.roi_mm(1, 1)[0], 0.0) and np.isclose(f.roi_mm(1, 1)[1], 0.0)
    dx_mm = f.w.pixel_um / f.w.mag * 1e-3
    assert np.isclose(f.roi_mm(0, 1)[0] - x0, f.step_lr * dx_mm)


def test_stitching_true_tiles_with_random_phases_gives_back_the_field():
    f = _field()
    rng = np.random.default_rng(0)
    amp, ph = inputs.truth_object(f.size_hr, seed=3)
    truth = amp * np.exp(1j * ph)
    M, s = f.w.m_hr, f.w.upsample
    tiles = {}
    for i in range(f.tiles):
        for j in range(f.tiles):
            r0, c0 = i * f.step_lr * s, j * f.step_lr * s
            tiles[(i, j)] = truth[r0:r0 + M, c0:c0 + M] * np.exp(1j * rng.uniform(-np.pi, np.pi))
    out = fullfield.stitch(f, tiles)
    out = out * np.exp(1j * np.angle(np.vdot(out, truth)))
    assert np.abs(out - truth).max() < 1e-10
