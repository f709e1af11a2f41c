"""GPU parity of whole solves against the FP64 oracle (Sec. 2.3, Eqs. 6-7, 13-14).

The same seeded data and the same batch order on both sides; the final object
within a relative error of 1e-3, the object gradient at the GPU's own state
within the per-step bar (relative L2 2e-5 and every entry within 1e-4 of the
largest), integer decisions (the LED order) exact.

Cases: the paper-shaped solve (15 x 15 LEDs, 256^2 -> 1024^2, B = 16, object
+ Zernike pupil, 30 epochs = 450 steps); batches of one LED, in a random order
per epoch and in the fixed centre-outwards order of the sequential method
(Sec. 3.1, Eq. 7); the full gradient of Eq. 6 (every LED in one batch) is
covered in test_gpu_parity.py.

The paper-shaped trajectory is sensitive below the FP32 rounding level: Adam
turns near-zero gradient components into whole steps of their sign, so the
FP64 reference itself, fed object gradients with 1e-7 relative noise, ends
9.4e-4 away from its own noise-free run after 225 steps and 2.6e-3 after 450.
There the object bar is twice that spread (2e-3 and 6e-3); the gradient at
the GPU's own state keeps the per-step bar.
"""
import sys

import numpy as np
import pytest

from oracle import fpm_oracle as fo
from paper_2408_13782_amd import fpm, inputs, problem

from cases import assert_grad_close, oracle_problem, rel_l2

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")

GRAD_TOL = 2e-5
OBJ_TOL = 1e-3
# the paper-shaped trajectory's bars after 225 and 450 steps (see the module note)
PAPER_OBJ_TOL = {225: 2e-3, 450: 6e-3}


def say(msg):
    print(f"[gpu] {msg}", flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def dev():
    assert torch.cuda.is_available(), "GPU tests need a visible MI355X"
    fpm.load()
    return torch.device("cuda:0")


def T(x, dev):
    return torch.as_tensor(np.ascontiguousarray(x)).to(dev)


def H(t):
    return t.detach().cpu().numpy()


def make_plan(w, shifts, max_batch):
    return fpm.Plan(w.n_lr, w.upsample, shifts, max_batch, w.wavelength_um, w.na, w.mag,
                    w.pixel_um)


def gradient_at_gpu_state(dev, plan, pr, O, P, leds):
    """Object gradient of fpm_backward at the GPU's (O, P) against the oracle's."""
    gO = torch.zeros_like(O)
    loss = torch.zeros(1, dtype=torch.float64, device=dev)
    plan.backward(O, P, np.asarray(leds, np.int32), T(pr.A, dev), gO, None, loss)
    torch.cuda.synchronize()
    ref = fo.loss_and_grads(H(O).astype(np.complex128), H(P).astype(np.complex128), pr.shifts,
                            leds, pr.A.astype(np.float64))
    assert abs(float(H(loss)[0]) - ref.loss) <= 1e-5 * ref.loss
    return assert_grad_close(H(gO), ref.g_O)


@pytest.mark.timeout(400)
def test_paper_solve_matches_oracle(dev):
    """The whole paper-shaped solve through fpm_run, in two calls of 225 steps:
    after each, the object against the oracle's solve of the same schedule, and
    the gradient at the GPU's state; at the end, one more step's Zernike
    gradients at the GPU's (near-converged) state against the oracle's."""
    w = inputs.workload("paper")
    say("paper solve: 15x15 LEDs, 256^2 -> 1024^2, B = 16, object + Zernike, 450 steps")
    pr = oracle_problem(w, seed=0)
    perms = inputs.led_permutations(w.n_led, w.epochs, seed=0)
    sched = fo.batches_from_permutations(perms, w.batch)
    assert len(sched) == 450 and sum(len(b) for b in sched) == 6750
    ds = problem.flatten_schedule(problem.schedule(perms, w.batch))
    plan = make_plan(w, pr.shifts, w.batch)
    st = fpm.State(plan, T(pr.O0, dev))
    hp = problem.hparams(w)
    A = T(pr.A, dev)
    ost = fo.init_state(pr.O0)
    cfg = fo.SolveConfig(lr_object=w.lr_object, lr_zernike=w.lr_zernike, learn_pupil=True)
    A64 = pr.A.astype(np.float64)
    oloss = 0.0
    for lo, hi in ((0, 225), (225, 450)):
        plan.run(st, hp, *ds.span(lo, hi), A)
        torch.cuda.synchronize()
        oloss += sum(fo.solve(ost, cfg, pr.mask, pr.zern, pr.kappa, pr.shifts, sched[lo:hi], A64))
        o_err = rel_l2(H(st.O), ost.O)
        c_err = float(np.abs(H(st.coeffs).astype(np.float64) - ost.coeffs).max())
        g_err = gradient_at_gpu_state(dev, plan, pr, st.O, st.P, sched[hi % len(sched)])
        say(f"after {hi} steps: object rel err {o_err:.3e}, max Zernike diff {c_err:.3e} rad, "
            f"gradient at the GPU state rel err {g_err:.3e}")
        assert st.t == hi
        assert o_err <= PAPER_OBJ_TOL[hi]
        assert c_err <= 1e-3 * w.lr_zernike
    assert abs(float(H(st.loss)[0]) - oloss) <= 1e-4 * oloss
    # the pupil-parameter gradients of one more step at the converged GPU state,
    # against the oracle's at that state: bounded by their own size where they
    # are not lost in cancellation, and by the sum of their terms everywhere
    c_gpu = H(st.coeffs).astype(np.float64)
    nxt = fpm.State(plan, st.O.clone(), c_gpu)
    leds = sched[0]
    plan.step(nxt, hp, leds, A)
    torch.cuda.synchronize()
    P = fo.pupil(pr.mask, pr.zern, c_gpu, 0.0, pr.kappa)
    ref = fo.loss_and_grads(H(st.O).astype(np.complex128), P, pr.shifts, leds, A64)
    g_c, _, g_theta = fo.pupil_param_grads(ref.g_P, P, pr.zern, pr.kappa)
    got = H(nxt.g_par)[:15]
    for j in range(1, 15):
        terms = float(np.sum(np.abs(g_theta * pr.zern[j])))
        err = abs(got[j] - g_c[j])
        say(f"  Zernike {j:2d}: gradient {g_c[j]: .4e}, error {err:.2e} "
            f"({err / max(abs(g_c[j]), 1e-300):.1e} of itself, {err / terms:.1e} of its terms)")
        assert err <= GRAD_TOL * terms
        assert err <= 1e-2 * abs(g_c[j]) + 1e-6 * terms


@pytest.mark.parametrize("order", ["random", "sequential"])
def test_single_led_batches_match_oracle(dev, order):
    """Batches of one LED over two epochs of the small workload's shape (7x7 LEDs,
    64^2 -> 256^2): a random order per epoch (Eqs. 13-14 with B = 1) and the
    fixed centre-outwards order of the sequential method (Eq. 7)."""
    w = inputs.workload("small")
    say(f"B = 1, {order} order, two epochs")
    pr = oracle_problem(w, seed=0)
    if order == "random":
        perms = inputs.led_permutations(w.n_led, 2, seed=3)
    else:
        ring = inputs.centre_out_order(pr.k)
        # the centre LED first, then the rings by distance from the axis
        assert ring[0] == (w.n_side // 2) * w.n_side + w.n_side // 2
        r = np.hypot(pr.k[ring, 0], pr.k[ring, 1])
        assert np.all(np.diff(r) >= -1e-12)
        perms = np.tile(ring, (2, 1))
    sched = fo.batches_from_permutations(perms, 1)
    assert len(sched) == 2 * w.n_led
    ds = problem.flatten_schedule(problem.schedule(perms, 1))
    plan = make_plan(w, pr.shifts, 1)
    st = fpm.State(plan, T(pr.O0, dev))
    plan.run(st, problem.hparams(w), ds.flat, ds.sizes, T(pr.A, dev))
    torch.cuda.synchronize()
    ost = fo.init_state(pr.O0)
    losses = fo.solve(ost, fo.SolveConfig(lr_object=w.lr_object), pr.mask, pr.zern, pr.kappa,
                      pr.shifts, sched, pr.A.astype(np.float64))
    err = rel_l2(H(st.O), ost.O)
    say(f"final object rel err {err:.3e}")
    assert st.t == len(sched)
    assert err <= OBJ_TOL
    assert abs(float(H(st.loss)[0]) - sum(losses)) <= 1e-4 * sum(losses)
    gradient_at_gpu_state(dev, plan, pr, st.O, st.P, sched[0])
