"""The operator as a differentiable function: autograd, finite differences and
projected-gradient least squares, on the GPU through the C-ABI."""
import numpy as np
import pytest

import oracle as O
import synth
from gpu_util import geometry_of, make_plan, rel_l2, to_dev

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def torch_gpu():
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch


@pytest.fixture(scope="module")
def sub():
    """The FP64 sub-case: 16x16 sensors, 64 samples, 16x16x32 voxels."""
    return synth.config("c5sub")


def test_gradcheck_fp64(torch_gpu, sub):
    import paper_1501_02946_amd as N
    torch = torch_gpu
    plan = make_plan(sub, "fp64")
    g = to_dev(sub.g, plan).requires_grad_(True)
    assert torch.autograd.gradcheck(lambda x: N.NednerRecon.apply(x, plan), (g,), eps=1e-6,
                                    atol=1e-8, rtol=1e-6, fast_mode=True)
    v = torch.randn(plan.volume, dtype=torch.float64, device=plan.device, requires_grad=True)
    assert torch.autograd.gradcheck(lambda x: N.NednerAdjoint.apply(x, plan), (v,), eps=1e-6,
                                    atol=1e-8, rtol=1e-6, fast_mode=True)


def test_least_squares_gradient_fd_and_oracle(torch_gpu, sub):
    """J(x) = 1/2 ||A* x - g||^2 is quadratic: central differences are exact up to rounding."""
    import paper_1501_02946_amd as N
    torch = torch_gpu
    plan = make_plan(sub, "fp64")
    g = to_dev(sub.g, plan)
    rng = np.random.default_rng(3)
    x = to_dev(rng.normal(size=plan.volume), plan).requires_grad_(True)
    J = lambda z: 0.5 * torch.sum((N.NednerAdjoint.apply(z, plan) - g) ** 2)
    (grad,) = torch.autograd.grad(J(x), x)
    d = to_dev(rng.normal(size=plan.volume), plan)
    h = 1e-3
    with torch.no_grad():
        j0 = float(J(x))
        fd = (J(x + h * d) - J(x - h * d)) / (2 * h)
    an = torch.sum(grad * d)
    print("directional derivative", float(fd), float(an), "J", j0)
    # exact for a quadratic; only the rounding of J (relative 1e-16 or so) is amplified by 1/h
    assert abs(float(fd) - float(an)) <= 1e-11 * abs(j0) / h + 1e-9 * abs(float(an))
    geo = geometry_of(sub)
    xn = x.detach().cpu().numpy()
    ref = O.forward(sub.xy, sub.h, O.adjoint(xn, sub.xy, sub.h, geo) - sub.g, geo)
    err = rel_l2(grad.cpu().numpy(), ref)
    print("gradient vs oracle", err)
    assert err <= 1e-5


def test_projected_gd_matches_oracle_iterates(torch_gpu, sub):
    import paper_1501_02946_amd as N
    torch = torch_gpu
    plan = make_plan(sub, "fp64")
    g = to_dev(sub.g, plan)
    eta = 0.95 / N.power_norm(plan, iters=30)
    x, losses = N.lsq(plan, g, iters=20, eta=eta)
    geo = geometry_of(sub)
    xr = np.zeros(plan.volume)
    for _ in range(20):
        r = O.adjoint(xr, sub.xy, sub.h, geo) - sub.g
        xr = np.maximum(0.0, xr - eta * O.forward(sub.xy, sub.h, r, geo))
    err = rel_l2(x.cpu().numpy(), xr)
    print("GD iterate vs oracle iterate", err, losses[0], losses[-1])
    assert err <= 1e-5
    assert all(b <= a * (1 + 1e-12) for a, b in zip(losses, losses[1:]))
    assert float(x.min()) >= 0.0


@pytest.mark.slow
def test_projected_gd_c5_fp32(torch_gpu):
    """The least-squares workload: 192x192 sensors, 768 samples, 192x192x384, 20 iterations."""
    import paper_1501_02946_amd as N
    p = synth.config("c5")
    plan = make_plan(p, "fp32c")
    g = to_dev(p.g, plan)
    x, losses = N.lsq(plan, g, iters=20)
    print("c5 losses", losses[0], losses[-1])
    assert losses[-1] < 0.5 * losses[0]
    assert all(b <= a * (1 + 1e-5) for a, b in zip(losses, losses[1:]))
    assert float(x.min()) >= 0.0
