"""The NER-only path for sensors on the output grid (paper, Sec. 3, eq. (4)):
the lateral sums are then a plain DFT, so the operator skips the spreading and
the lateral window; only the time axis keeps the NUFFT. Host checks (CPU) and
parity with the oracle (GPU)."""
import numpy as np
import pytest

import oracle as O
import synth
from gpu_util import geometry_of, make_plan, rel_l2, to_dev

E_ARG = 1
E_UNSUPPORTED = 6


def on_grid(s, stride=1, n=None, nt=128, seed=0, keep=1.0):
    """Sensors on every `stride`-th node of an n x n grid over [0,1)^2."""
    n = n or s * stride
    rng = np.random.default_rng(seed)
    i = np.arange(0, n, stride)[:s]
    xy = np.stack(np.meshgrid(i, i, indexing="ij"), -1).reshape(-1, 2) / n
    if keep < 1.0:
        xy = xy[rng.random(len(xy)) < keep]
    m = len(xy)
    balls = synth.random_balls(3, rng)
    return synth.make_problem(xy, np.full(m, 1.0 / m), balls, nt, n, n, nt // 2, rng=rng, noise=0.01)


def test_query_and_validation():
    import ctypes
    import paper_1501_02946_amd as N
    p = on_grid(16, stride=2)
    info = N.query(p.xy, p.nt, p.dt, (p.n1, p.n2, p.n3), h=p.h, flags=["equispaced"])
    assert (info["n1_os"], info["n2_os"]) == (p.n1, p.n2)     # no lateral oversampling
    assert info["list_entries"] == 0
    # off-grid sensor
    xy = p.xy.copy()
    xy[3, 0] += 0.25 / p.n1
    d, keep = N._make_desc(xy, p.h, p.nt, p.dt, p.n1, p.n2, p.n3, flags=["equispaced"])
    assert N.lib().nedner_validate(ctypes.byref(d)) == E_ARG
    # two sensors on one node
    xy = np.concatenate([p.xy, p.xy[:1]])
    d, keep = N._make_desc(xy, np.full(len(xy), 1.0 / len(xy)), p.nt, p.dt, p.n1, p.n2, p.n3,
                           flags=["equispaced"])
    assert N.lib().nedner_validate(ctypes.byref(d)) == E_ARG


@pytest.fixture(scope="module")
def torch_gpu():
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch


@pytest.mark.gpu
@pytest.mark.parametrize("case", [dict(s=32), dict(s=20, stride=2, n=40, keep=0.7, seed=3),
                                  dict(s=24, nt=96, seed=5)])
@pytest.mark.parametrize("prec", ["fp64", "fp32c"])
def test_equispaced_matches_oracle(torch_gpu, case, prec):
    p = on_grid(**case)
    geo = geometry_of(p)
    F = O.spectrum(p.xy, p.h, p.g, geo)
    v = O.volume_from_spectrum(F)
    plan = make_plan(p, prec, flags=["equispaced"])
    g = to_dev(p.g, plan)
    ev = rel_l2(plan(g).cpu().numpy(), v)
    eF = rel_l2(plan.spectrum(g).cpu().numpy(), F)
    print("equispaced", prec, p.m, ev, eF)
    assert ev <= 1e-5 and eF <= 1e-5
    if prec == "fp64":
        # the same sensors through the spreading path: same operator, plus the lateral window error
        ref = make_plan(p, prec)
        assert rel_l2(ref(g).cpu().numpy(), v) <= 1e-5


@pytest.mark.gpu
def test_equispaced_adjoint(torch_gpu):
    p = on_grid(20, stride=2, n=40, keep=0.8, seed=7)
    geo = geometry_of(p)
    plan = make_plan(p, "fp64", flags=["equispaced"])
    rng = np.random.default_rng(1)
    x = rng.normal(size=(p.m, p.nt))
    y = rng.normal(size=plan.volume)
    Ax = plan(to_dev(x, plan)).cpu().numpy()
    Aty = plan.adjoint(to_dev(y, plan)).cpu().numpy()
    lhs, rhs = float(np.sum(Ax * y)), float(np.sum(x * Aty))
    assert abs(lhs - rhs) <= 1e-12 * max(abs(lhs), 1.0)
    assert rel_l2(Aty, O.adjoint(y, p.xy, p.h, geo)) <= 1e-5
