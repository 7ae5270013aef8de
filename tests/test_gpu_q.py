"""GPU parity of the forward operator Q of the wave equation (Sec. 2) and its
adjoint, through the C-ABI, against the FP64 oracle.

Q takes an initial pressure on the periodic voxel grid to the trace of the
wave equation's solution at the sensors; the library evaluates it with the
plan's reconstruction kernels run in reverse (adjoint pipeline, NER columns
averaged between l and -l, unit weights), so it carries the same window
error as the reconstruction. Tolerance: rel-L2 <= 1e-5, the reconstruction's
bar.
"""
import dataclasses
import math

import numpy as np
import pytest

import oracle as O
import synth
from gpu_util import geometry_of, make_plan, rel_l2, small_problem, to_dev

pytestmark = pytest.mark.gpu

TOL = 1e-5


@pytest.fixture(scope="module")
def torch_gpu():
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch


def _volume(p, seed):
    """Random initial pressure plus a smooth blob (a full and a decaying spectrum)."""
    rng = np.random.default_rng(np.random.SeedSequence([23, seed]))
    v = rng.normal(size=(p.n1, p.n2, p.n3))
    geo = geometry_of(p)
    x1 = geo.a1 + geo.d1 * np.arange(p.n1)
    x2 = geo.a2 + geo.d2 * np.arange(p.n2)
    z = geo.d3 * np.arange(p.n3)
    X1, X2, Z = np.meshgrid(x1, x2, z, indexing="ij")
    s = 3.0 * max(geo.d1, geo.d2, geo.d3)
    c0 = (geo.a1 + 0.45 * geo.l1, geo.a2 + 0.55 * geo.l2, 0.4 * p.n3 * geo.d3)
    v += 4.0 * np.exp(-((X1 - c0[0]) ** 2 + (X2 - c0[1]) ** 2 + (Z - c0[2]) ** 2) / (2 * s * s))
    return v


def _check(p, prec, seed=0, **kw):
    geo = geometry_of(p)
    v = _volume(p, seed)
    plan = make_plan(p, prec, **kw)
    got = plan.q(to_dev(v, plan)).cpu().numpy()
    want = O.trace(v, p.xy, geo)
    e_q = rel_l2(got, want)
    d = p.g
    got_t = plan.q_adjoint(to_dev(d, plan)).cpu().numpy()
    want_t = O.trace_adjoint(d, p.xy, geo)
    e_t = rel_l2(got_t, want_t)
    print(f"{p.name or 'problem'} {prec}: Q rel-L2 {e_q:.3e}, Q* rel-L2 {e_t:.3e}")
    assert e_q <= TOL
    assert e_t <= TOL
    return plan


@pytest.mark.parametrize("prec", ["fp64", "fp32c", "fp32"])
def test_c1_q_and_adjoint(torch_gpu, prec):
    _check(synth.config("c1"), prec)


@pytest.mark.parametrize("kw", [
    dict(seed=1),
    dict(seed=2, s=9, nt=36, n=(10, 12, 18), c=1.3, t0=0.02, a=(0.1, -0.2)),
    dict(seed=3, s=20, nt=64, n=(24, 20, 40), jitter=0.45),
    dict(seed=4, s=6, nt=12, n=(6, 8, 6)),
])
@pytest.mark.parametrize("prec", ["fp64", "fp32c"])
def test_ragged_q_and_adjoint(torch_gpu, kw, prec):
    _check(small_problem(**kw), prec, seed=kw["seed"])


def test_equispaced_q_and_adjoint(torch_gpu):
    rng = np.random.default_rng(5)
    n = 24
    i = np.arange(n)
    xy = np.stack(np.meshgrid(i, i, indexing="ij"), -1).reshape(-1, 2) / n
    xy = xy[rng.random(len(xy)) < 0.7]
    m = len(xy)
    p = synth.make_problem(xy, np.full(m, 1.0 / m), synth.random_balls(3, rng), 48, n, n, 24,
                           rng=rng, noise=0.01)
    for prec in ("fp64", "fp32c"):
        _check(p, prec, flags=["equispaced"])


def test_kaiser_bessel_q_and_adjoint(torch_gpu):
    _check(synth.config("c1"), "fp32c", w=8, window="kaiser_bessel")


def test_gaussian_source_closed_form(torch_gpu):
    """Q of a resolved Gaussian initial pressure equals the radial solution of
    the wave equation summed over the grid's periodic images."""
    n = 32
    p = synth.make_problem(np.stack([np.linspace(0.25, 0.75, 16), np.linspace(0.7, 0.3, 16)], 1),
                           np.full(16, 1.0 / 16), [], 64, n, n, n, c=1.0, dt=1.0 / 64, d3=1.0 / n)
    geo = geometry_of(p)
    s = 2.5 / n
    x0 = (0.43, 0.56, 0.5)
    x1 = geo.d1 * np.arange(n)
    X1, X2, Z = np.meshgrid(x1, geo.d2 * np.arange(n), geo.d3 * np.arange(n), indexing="ij")
    v = np.zeros_like(X1)
    for a in (-1, 0, 1):
        for b in (-1, 0, 1):
            for e in (-1, 0, 1):
                v += np.exp(-((X1 - x0[0] - a) ** 2 + (X2 - x0[1] - b) ** 2 + (Z - x0[2] - e) ** 2)
                            / (2 * s * s))
    t = geo.t0 + geo.dt * np.arange(geo.nt)
    want = np.zeros((len(p.xy), geo.nt))
    f = lambda q: np.exp(-q * q / (2 * s * s))  # noqa: E731
    for a in range(-3, 4):
        for b in range(-3, 4):
            for e in range(-3, 4):
                r = np.sqrt((p.xy[:, 0] - x0[0] - a) ** 2 + (p.xy[:, 1] - x0[1] - b) ** 2
                            + (x0[2] + e) ** 2)[:, None]
                want += ((r - t) * f(r - t) + (r + t) * f(r + t)) / (2 * r)
    plan = make_plan(p, "fp32c")
    got = plan.q(to_dev(v, plan)).cpu().numpy()
    err = rel_l2(got, want)
    print("Gaussian source: rel-L2 vs closed form", err)
    assert np.abs(want).max() > 0.05
    assert err <= TOL


@pytest.mark.slow
@pytest.mark.parametrize("prec", ["fp32c", "fp64"])
def test_fullsize_c2_sampled_and_adjoint_identity(torch_gpu, prec):
    """At 128x128x256 with 16384 sensors: sampled (sensor, time) outputs of Q
    against the oracle's sums at those times, and <Q v, d> = <v, Q* d>."""
    torch = torch_gpu
    p = synth.config("c2")
    geo = geometry_of(p)
    v = _volume(p, 9)
    plan = make_plan(p, prec)
    got = plan.q(to_dev(v, plan)).cpu().numpy()
    rng = np.random.default_rng(3)
    ms = rng.choice(p.m, 48, replace=False)
    ns = np.sort(rng.choice(p.nt, 6, replace=False))
    want = np.empty((len(ms), len(ns)))
    for i, n in enumerate(ns):
        g1 = dataclasses.replace(geo, nt=1, t0=geo.t0 + n * geo.dt)
        want[:, i] = O.trace(v, p.xy[ms], g1)[:, 0]
    err = rel_l2(got[np.ix_(ms, ns)], want)
    d = rng.normal(size=(p.m, p.nt))
    vq = plan.q_adjoint(to_dev(d, plan)).double().cpu().numpy()
    lhs = float(np.sum(got.astype(np.float64) * d))
    rhs = float(np.sum(v * vq))
    adj = abs(lhs - rhs) / math.sqrt(np.sum(got.astype(np.float64) ** 2) * np.sum(d * d))
    print(f"c2 {prec}: sampled Q rel-L2 {err:.3e}, adjoint identity {adj:.3e}")
    assert err <= TOL
    assert adj <= TOL
    del torch


def test_least_squares_with_q(torch_gpu):
    """Projected gradient descent on 1/2 ||Q x - g||^2, x >= 0, for data made by
    Q itself: the loss falls monotonically and x approaches the source."""
    torch = torch_gpu
    import paper_1501_02946_amd as N
    p = synth.config("c5sub")
    plan = make_plan(p, "fp64")
    geo = geometry_of(p)
    x1 = geo.a1 + geo.d1 * np.arange(p.n1)
    x2 = geo.a2 + geo.d2 * np.arange(p.n2)
    z = geo.d3 * np.arange(p.n3)
    X1, X2, Z = np.meshgrid(x1, x2, z, indexing="ij")
    s = 2.0 * max(geo.d1, geo.d2, geo.d3)
    xt = np.exp(-((X1 - 0.5) ** 2 + (X2 - 0.5) ** 2 + (Z - 0.3 * p.n3 * geo.d3) ** 2) / (2 * s * s))
    g = plan.q(to_dev(xt, plan))
    x, losses = N.lsq(plan, g, iters=30, model="q")
    assert all(b <= a * (1 + 1e-9) for a, b in zip(losses, losses[1:])), losses
    assert losses[-1] < 0.2 * losses[0]
    # the gradient taken by autograd through NednerQ is Q* (Q x - g)
    x0 = torch.rand(p.n1, p.n2, p.n3, dtype=plan.dtype, device=plan.device, requires_grad=True)
    r = N.NednerQ.apply(x0, plan) - g
    (gr,) = torch.autograd.grad(0.5 * torch.sum(r * r), x0)
    want = plan.q_adjoint(plan.q(x0.detach()) - g)
    assert float(torch.linalg.vector_norm(gr - want) / torch.linalg.vector_norm(want)) <= 1e-12
    err0 = float(np.linalg.norm(xt))
    err = float(np.linalg.norm(x.cpu().numpy() - xt))
    print("LS with Q: loss", losses[0], "->", losses[-1], "; |x - x_true|/|x_true|", err / err0)
    assert err < err0
