"""GPU parity: the HIP path through the C-ABI against the FP64 oracle.

Tolerance: rel-L2 <= 1e-5 against the oracle for the volume, the spectrum
and the adjoint (the bar the operator is built to), for the FP64, FP32 and
compensated FP32 paths. The window error of the Gaussian NUFFT at w = 12,
sigma = 2 is a few 1e-7, rounding adds ~1e-7 in FP32.
"""
import math

import numpy as np
import pytest

import oracle as O
import synth
from gpu_util import geometry_of, make_plan, phihat, rel_l2, small_problem, to_dev

pytestmark = pytest.mark.gpu

TOL = 1e-5


@pytest.fixture(scope="module")
def torch_gpu():
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch


def _oracle(p):
    geo = geometry_of(p)
    F = O.spectrum(p.xy, p.h, p.g, geo)
    return geo, F, O.volume_from_spectrum(F)


def test_spread_grid_matches_oracle_ned(torch_gpu):
    """Stage check: FFT of the spread grid, deconvolved, equals the NED sum of eq. (5)."""
    p = synth.config("c1")
    plan = make_plan(p, "fp64")
    U = plan.grid(to_dev(p.g, plan)).cpu().numpy()
    n1, n2 = plan.info["n1_os"], plan.info["n2_os"]
    beta = plan.info["beta"]
    Uh = np.fft.fft2(U, axes=(0, 1))
    j1 = O.mode_numbers(p.n1)
    j2 = O.mode_numbers(p.n2)
    G = Uh[np.ix_(j1 % n1, j2 % n2)] / (phihat(beta, j1, n1)[:, None, None]
                                        * phihat(beta, j2, n2)[None, :, None])
    Go = O.ned(p.xy, p.h, p.g, geometry_of(p))
    err = rel_l2(G, Go)
    print("NED stage rel-L2", err)
    assert err <= TOL


@pytest.mark.parametrize("prec", ["fp64", "fp32c", "fp32", "fp32w"])
def test_c1_volume_and_spectrum(torch_gpu, prec):
    p = synth.config("c1")
    geo, F, v = _oracle(p)
    plan = make_plan(p, prec)
    g = to_dev(p.g, plan)
    vg = plan(g).cpu().numpy()
    Fg = plan.spectrum(g).cpu().numpy()
    ev, eF = rel_l2(vg, v), rel_l2(Fg, F)
    print(prec, "volume", ev, "spectrum", eF)
    assert ev <= TOL and eF <= TOL


@pytest.mark.parametrize("case", [
    dict(seed=1),
    dict(seed=2, s=10, nt=100, n=(10, 6, 30), c=1.3, t0=0.02, a=(0.25, -0.5), length=1.5),
    dict(seed=3, s=9, nt=48, n=(12, 20, 24), d3=0.03, jitter=0.49),
    dict(seed=4, s=16, nt=64, n=(16, 16, 40)),
])
@pytest.mark.parametrize("prec", ["fp64", "fp32c", "fp32w"])
def test_ragged_cases(torch_gpu, case, prec):
    p = small_problem(**case)
    geo, F, v = _oracle(p)
    plan = make_plan(p, prec)
    g = to_dev(p.g, plan)
    ev = rel_l2(plan(g).cpu().numpy(), v)
    eF = rel_l2(plan.spectrum(g).cpu().numpy(), F)
    print(case, prec, "volume", ev, "spectrum", eF)
    assert ev <= TOL and eF <= TOL


def test_adjoint_identity_fp64(torch_gpu):
    torch = torch_gpu
    p = small_problem(seed=5, s=12, nt=40, n=(12, 10, 20))
    plan = make_plan(p, "fp64")
    rng = np.random.default_rng(6)
    x = rng.normal(size=(p.m, p.nt))
    y = rng.normal(size=(p.n1, p.n2, p.n3))
    Ax = plan(to_dev(x, plan)).cpu().numpy()
    Aty = plan.adjoint(to_dev(y, plan)).cpu().numpy()
    lhs, rhs = float(np.vdot(Ax, y)), float(np.vdot(x, Aty))
    print("adjoint identity", lhs, rhs, abs(lhs - rhs) / abs(lhs))
    assert abs(lhs - rhs) <= 1e-12 * max(abs(lhs), np.linalg.norm(Ax) * np.linalg.norm(y) * 1e-3)


def test_adjoint_matches_oracle(torch_gpu):
    p = small_problem(seed=7, s=12, nt=40, n=(12, 12, 20))
    geo = geometry_of(p)
    y = np.random.default_rng(8).normal(size=(p.n1, p.n2, p.n3))
    ref = O.adjoint(y, p.xy, p.h, geo)
    for prec in ("fp64", "fp32c"):
        plan = make_plan(p, prec)
        got = plan.adjoint(to_dev(y, plan)).cpu().numpy()
        err = rel_l2(got, ref)
        print(prec, "adjoint rel-L2", err)
        assert err <= TOL


def test_determinism(torch_gpu):
    p = small_problem(seed=9)
    plan = make_plan(p, "fp32c")
    g = to_dev(p.g, plan)
    a = plan(g).cpu().numpy()
    b = plan(g).cpu().numpy()
    assert np.array_equal(a, b)


@pytest.mark.parametrize("layout", ["single", "one_cell", "seam", "tiny"])
def test_edge_layouts(torch_gpu, layout):
    rng = np.random.default_rng(10)
    if layout == "single":
        xy = np.array([[0.37, 0.81]])
        n = (8, 8, 16)
    elif layout == "one_cell":
        xy = 0.5 + rng.uniform(0, 1.0 / 64, size=(40, 2))
        n = (16, 16, 16)
    elif layout == "seam":
        xy = np.array([[1.0 - 1e-13, 0.5], [0.0, 1.0 - 1e-12], [1.0 - 1e-9, 1.0 - 1e-9], [0.25, 0.0]])
        n = (8, 8, 8)
    else:
        xy = rng.uniform(0, 1, size=(5, 2))
        n = (2, 4, 2)
    m = xy.shape[0]
    nt = max(16, 2 * n[2])
    g = rng.normal(size=(m, nt))
    p = synth.Problem(xy=xy, h=np.full(m, 1.0 / m), g=g, nt=nt, dt=1.0 / nt, c=1.0,
                      n1=n[0], n2=n[1], n3=n[2])
    geo, F, v = _oracle(p)
    for prec in ("fp64", "fp32c"):
        plan = make_plan(p, prec)
        gd = to_dev(g, plan)
        ev = rel_l2(plan(gd).cpu().numpy(), v)
        eF = rel_l2(plan.spectrum(gd).cpu().numpy(), F)
        print(layout, prec, ev, eF)
        assert ev <= TOL and eF <= TOL


@pytest.mark.slow
def test_c2_full_volume(torch_gpu):
    """The benchmark workload (128x128 sensors, 512 samples, 128x128x256), full oracle."""
    p = synth.config("c2")
    geo, F, v = _oracle(p)
    for prec in ("fp32c", "fp32", "fp32w", "fp64"):
        plan = make_plan(p, prec)
        vg = plan(to_dev(p.g, plan)).cpu().numpy()
        err = rel_l2(vg, v)
        print("c2", prec, "volume rel-L2", err)
        assert err <= TOL
    plan = make_plan(p, "fp32_plain")
    err = rel_l2(plan(to_dev(p.g, plan)).cpu().numpy(), v)
    print("c2 fp32_plain volume rel-L2", err)


@pytest.mark.parametrize("layout", ["iid", "shuffled_grid", "one_cell", "seam", "single"])
def test_adjoint_and_q_on_unordered_layouts(torch_gpu, layout):
    """The adjoint gather takes the sensors in the plan's tile order, not in
    their numbering: sensors numbered at random, packed into one cell, on the
    periodic seams or alone must give the oracle's adjoint and Q."""
    rng = np.random.default_rng(12)
    n = (16, 16, 24)
    if layout == "iid":
        xy = rng.uniform(0, 1, size=(300, 2))
    elif layout == "shuffled_grid":
        xy = synth.jittered_grid(14, 0.45, rng)[rng.permutation(14 * 14)]
    elif layout == "one_cell":
        xy = 0.5 + rng.uniform(0, 1.0 / 32, size=(23, 2))
    elif layout == "seam":
        xy = np.array([[1.0 - 1e-13, 0.5], [0.0, 1.0 - 1e-12], [1.0 - 1e-9, 1.0 - 1e-9], [0.25, 0.0],
                       [0.5, 0.999], [0.001, 0.001], [0.999, 0.2]])
    else:
        xy = np.array([[0.37, 0.81]])
    m = xy.shape[0]
    nt = 48
    h = rng.uniform(0.5, 1.5, m)
    h /= h.sum()
    p = synth.Problem(xy=xy, h=h, g=np.zeros((m, nt)), nt=nt, dt=1.0 / nt, c=1.0,
                      n1=n[0], n2=n[1], n3=n[2])
    geo = geometry_of(p)
    v = rng.normal(size=n)
    ref_a = O.adjoint(v, xy, h, geo)
    ref_q = O.trace(v, xy, geo)
    for prec in ("fp64", "fp32c"):
        plan = make_plan(p, prec)
        vd = to_dev(v, plan)
        ea = rel_l2(plan.adjoint(vd).cpu().numpy(), ref_a)
        eq = rel_l2(plan.q(vd).cpu().numpy(), ref_q)
        print(layout, prec, "adjoint", ea, "Q", eq)
        assert ea <= TOL and eq <= TOL
