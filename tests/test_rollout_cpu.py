"""CPU tests of the checkpointed rollout's bookkeeping (rollout.py) with a
stand-in solver whose step is the linear map U -> a U: the rollout's
gradient is then a^N times the output gradient, whatever the checkpoint
spacing.  No GPU and no HIP library are involved: the stand-in implements
the solver methods the rollout calls (step, step_save, stage,
adjoint_step_ustar) with torch CPU ops."""
import pytest
import torch

from paper_1607_08710_amd.rollout import rollout

A = 0.9


class LinearSolver:
    torch_dtype = torch.float64

    def __init__(self, shape):
        self.shape = shape
        self.calls = {"step": 0, "step_save": 0, "stage": 0, "adjoint": 0}

    def empty_state(self):
        return torch.empty(self.shape, dtype=self.torch_dtype)

    def step(self, Un, Unp1, dt):
        self.calls["step"] += 1
        torch.mul(Un, A, out=Unp1)

    def step_save(self, Un, Unp1, Ustar, dt):
        self.calls["step_save"] += 1
        torch.mul(Un, A, out=Unp1)
        Ustar.copy_(Un)

    def stage(self, stage, inp, out, dt, base=None, reduce=False):
        assert stage == 1
        self.calls["stage"] += 1
        out.copy_(inp)

    def adjoint_step_ustar(self, Un, Ustar, dt, lam_np1, lam_n):
        self.calls["adjoint"] += 1
        assert lam_n.data_ptr() != lam_np1.data_ptr()
        torch.mul(lam_np1, A, out=lam_n)


@pytest.mark.parametrize("steps,ckpt", [(1, 20), (4, 20), (7, 3), (20, 20), (41, 20)])
def test_gradient_and_output_gradient_untouched(steps, ckpt):
    shape = (4, 3, 5)
    S = LinearSolver(shape)
    gen = torch.Generator().manual_seed(steps * 100 + ckpt)
    x = torch.rand(shape, dtype=torch.float64, generator=gen).requires_grad_(True)
    UN = rollout(x, S, [1e-3] * steps, ckpt_every=ckpt)
    # one rounding per step: up to `steps` half-ulps apart from the power
    assert torch.allclose(UN, x.detach() * A ** steps, rtol=steps * 2.3e-16, atol=0)
    v = torch.rand(shape, dtype=torch.float64, generator=gen)
    v_before = v.clone()
    (g,) = torch.autograd.grad(UN, x, grad_outputs=v)
    # the caller's output gradient comes back unchanged and unshared
    assert torch.equal(v, v_before)
    assert g.data_ptr() != v.data_ptr()
    assert torch.allclose(g, v_before * A ** steps, rtol=steps * 2.3e-16, atol=0)
    assert S.calls["adjoint"] == steps
    # every step runs once forward; the backward pass recomputes all but the
    # last segment (kept by the forward pass), whose last step needs only
    # its predictor stage
    nseg = (steps + ckpt - 1) // ckpt
    tail = steps - (nseg - 1) * ckpt
    assert S.calls["step"] + S.calls["step_save"] == steps + (steps - tail) - (nseg - 1)
    assert S.calls["stage"] == nseg - 1


def test_empty_rollout():
    shape = (4, 2, 2)
    S = LinearSolver(shape)
    x = torch.rand(shape, dtype=torch.float64, requires_grad=True)
    UN = rollout(x, S, [], ckpt_every=20)
    assert torch.equal(UN, x.detach()) and UN.data_ptr() != x.data_ptr()
    v = torch.rand(shape, dtype=torch.float64)
    v_before = v.clone()
    (g,) = torch.autograd.grad(UN, x, grad_outputs=v)
    assert torch.equal(g, v_before) and torch.equal(v, v_before)
    assert g.data_ptr() != v.data_ptr()
    assert sum(S.calls.values()) == 0


def test_checkpoint_spacing():
    from paper_1607_08710_amd.rollout import checkpoint_spacing
    sb = 1 << 20
    # room for the whole run (2n + 1 states): no recompute
    assert checkpoint_spacing(200, sb, int((401 + 1) * sb / 0.85)) == 200
    # less room: the largest C with ceil(n/C) + 2C <= states that fit
    for n, m in ((200, 100), (200, 60), (200, 41), (1000, 200), (7, 9)):
        c = checkpoint_spacing(n, sb, int(m * sb / 0.85) + 1)
        assert -(-n // c) + 2 * c <= m
        assert c == n or -(-n // (c + 1)) + 2 * (c + 1) > m
    # not even the smallest peak fits: the spacing of the smallest peak
    assert checkpoint_spacing(200, sb, 10 * sb) == 10
    assert checkpoint_spacing(1, sb, 0) == 1


@pytest.mark.parametrize("steps", [5, 30])
def test_auto_spacing_gradient(steps):
    """ckpt_every="auto" gives the gradient of every fixed spacing, with the
    whole run kept when it fits (no recompute: no stage or step_save call
    in the backward pass) and checkpoints when it does not."""
    shape = (4, 3, 5)
    sb = 4 * 3 * 5 * 8
    x = torch.rand(shape, dtype=torch.float64, generator=torch.Generator().manual_seed(steps)).requires_grad_(True)
    v = torch.rand(shape, dtype=torch.float64, generator=torch.Generator().manual_seed(steps + 1))
    ref = torch.autograd.grad(rollout(x, LinearSolver(shape), [1e-3] * steps, ckpt_every=3), x, grad_outputs=v)[0]
    for free, resident in ((10**9, True), (12 * sb, False)):
        S = LinearSolver(shape)
        UN = rollout(x, S, [1e-3] * steps, ckpt_every="auto", free_bytes=free)
        fwd = dict(S.calls)
        (g,) = torch.autograd.grad(UN, x, grad_outputs=v)
        assert torch.equal(g, ref)
        recomputed = S.calls["step_save"] - fwd["step_save"] + S.calls["stage"] - fwd["stage"]
        assert (recomputed == 0) == resident
