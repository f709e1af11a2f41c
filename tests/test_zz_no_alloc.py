"""The allocation-free entry point fpm_backward_noalloc (for callers that cannot
allocate device memory) against fpm_backward, through the C ABI.

Two calls in a row on the one device-wide scratch array, the second with a
smaller input (a smaller LR size and batch), each against fpm_backward on the
same operands: the loss bitwise (its partial sums are added in a fixed order),
the object and pupil gradients within the per-step gradient bar (they are
accumulated with atomics, whose order may differ). A batch whose scratch
exceeds the array is refused with FPM_EINVAL and enqueues nothing.
"""
import ctypes as C
import sys

import numpy as np
import pytest

from oracle import fpm_oracle as fo
from paper_2408_13782_amd import fpm, inputs

from cases import assert_grad_close, oracle_problem, rel_l2

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


def say(msg):
    print(f"[gpu] {msg}", flush=True)
    sys.stdout.flush()


def T(x):
    return torch.as_tensor(np.ascontiguousarray(x)).to("cuda")


def H(t):
    return t.detach().cpu().numpy()


def backward_noalloc(plan, O, P, leds, A, gO, gP=None, loss=None, gamma=None):
    lib = fpm.load()
    fn = lib.fpm_backward_noalloc
    fn.argtypes = [C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p, C.c_int32, C.c_void_p,
                   C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p]
    fn.restype = C.c_int
    ids = np.ascontiguousarray(leds, np.int32)

    def ptr(t):
        return None if t is None else C.c_void_p(t.data_ptr())

    rc = fn(plan._h, ptr(O), ptr(P), ids.ctypes.data, len(ids), ptr(gamma), ptr(A), ptr(gO),
            ptr(gP), ptr(loss), C.c_void_p(torch.cuda.current_stream().cuda_stream))
    fpm._check(rc)


@pytest.fixture(scope="module")
def dev():
    assert torch.cuda.is_available(), "GPU tests need a visible MI355X"
    fpm.load()
    return torch.device("cuda:0")


def test_noalloc_backward_equals_fpm_backward(dev):
    for name, B, gamma_on in (("paper", 16, False), ("small", 5, True)):
        w = inputs.workload(name)
        say(f"fpm_backward_noalloc vs fpm_backward: {name} (N = {w.n_lr}), B = {B}")
        pr = oracle_problem(w, seed=2)
        plan = fpm.Plan(w.n_lr, w.upsample, pr.shifts, B, w.wavelength_um, w.na, w.mag,
                        w.pixel_um)
        c = inputs.random_real((15,), seed=3, lo=-0.2, hi=0.2).astype(np.float64)
        P = T(fo.pupil(pr.mask, pr.zern, c, 1.0, pr.kappa).astype(np.complex64))
        O, A = T(pr.O0), T(pr.A)
        gamma = T(inputs.random_real((w.n_led,), seed=4, lo=0.8, hi=1.2)) if gamma_on else None
        leds = inputs.random_indices(w.n_led, B, seed=5)
        outs = []
        for fn in ("fpm_backward", "fpm_backward_noalloc"):
            gO = torch.zeros((w.m_hr, w.m_hr), dtype=torch.complex64, device=dev)
            gP = torch.zeros((w.n_lr, w.n_lr), dtype=torch.complex64, device=dev)
            loss = torch.zeros(1, dtype=torch.float64, device=dev)
            if fn == "fpm_backward":
                plan.backward(O, P, leds, A, gO, gP, loss, gamma)
            else:
                backward_noalloc(plan, O, P, leds, A, gO, gP, loss, gamma)
            torch.cuda.synchronize()
            outs.append((H(gO), H(gP), H(loss)))
        (gO_ref, gP_ref, l_ref), (gO_new, gP_new, l_new) = outs
        np.testing.assert_array_equal(l_new, l_ref)
        assert_grad_close(gO_new, gO_ref)
        m = pr.mask.astype(bool)
        assert rel_l2(gP_new[m], gP_ref[m]) <= 2e-5
        assert np.all(gP_new[~m] == 0)
        # and both against the oracle
        ref = fo.loss_and_grads(pr.O0.astype(np.complex128), H(P).astype(np.complex128),
                                pr.shifts, leds, pr.A.astype(np.float64),
                                None if gamma is None else H(gamma).astype(np.float64))
        assert_grad_close(gO_new, ref.g_O)
        assert abs(float(l_new[0]) - ref.loss) <= 1e-5 * ref.loss


def test_noalloc_backward_refuses_batches_beyond_its_scratch(dev):
    w = inputs.workload("paper")
    say("fpm_backward_noalloc: a batch beyond the scratch array is refused")
    pr = oracle_problem(w, seed=0)
    plan = fpm.Plan(w.n_lr, w.upsample, pr.shifts, 64, w.wavelength_um, w.na, w.mag, w.pixel_um)
    O, A = T(pr.O0), T(pr.A)
    P = plan.pupil()
    gO = torch.zeros((w.m_hr, w.m_hr), dtype=torch.complex64, device=dev)
    loss = torch.zeros(1, dtype=torch.float64, device=dev)
    with pytest.raises(fpm.FpmError, match="scratch"):
        backward_noalloc(plan, O, P, inputs.random_indices(w.n_led, 64, seed=1), A, gO, None,
                         loss)
    torch.cuda.synchronize()
    assert float(H(loss)[0]) == 0.0 and not torch.any(gO != 0)
    # 32 LEDs of 256^2 fill the 16 MiB exactly
    backward_noalloc(plan, O, P, inputs.random_indices(w.n_led, 32, seed=1), A, gO, None, loss)
    torch.cuda.synchronize()
    assert float(H(loss)[0]) > 0.0


def test_noalloc_backward_is_not_timed(dev):
    """With the plan's timing on (fpm_timing), fpm_backward records its launches
    while the allocation-free entry point records none (recording would create
    events), and its results are unchanged."""
    w = inputs.workload("small")
    say("fpm_backward_noalloc under fpm_timing")
    pr = oracle_problem(w, seed=3)
    plan = fpm.Plan(w.n_lr, w.upsample, pr.shifts, 8, w.wavelength_um, w.na, w.mag, w.pixel_um)
    O, A = T(pr.O0), T(pr.A)
    P = plan.pupil()
    leds = inputs.random_indices(w.n_led, 8, seed=6)
    outs = []
    for timed in (False, True):
        gO = torch.zeros((w.m_hr, w.m_hr), dtype=torch.complex64, device=dev)
        loss = torch.zeros(1, dtype=torch.float64, device=dev)
        plan.timing(timed)
        backward_noalloc(plan, O, P, leds, A, gO, None, loss)
        torch.cuda.synchronize()
        if timed:
            assert plan.timing_collect() == {}
            plan.backward(O, P, leds, A, torch.zeros_like(gO), None,
                          torch.zeros_like(loss))
            torch.cuda.synchronize()
            assert len(plan.timing_collect()) > 0
            plan.timing(False)
        outs.append(H(loss).copy())
    np.testing.assert_array_equal(outs[0], outs[1])
