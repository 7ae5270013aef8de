"""GPU parity of the two-dimensional problem (d = 2 in Sec. 2): sensors on a
line along the first axis, one voxel across the second (n2 = 1, the mode
k2 = 0 only), image (i1, i3). The same kernels run with a second lateral
axis of one voxel; every operator is checked against the FP64 oracle at the
reconstruction's bar, rel-L2 <= 1e-5.
"""
import numpy as np
import pytest

import oracle as O
import synth
from gpu_util import geometry_of, make_plan, rel_l2, to_dev

pytestmark = pytest.mark.gpu

TOL = 1e-5


@pytest.fixture(scope="module")
def torch_gpu():
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch


def _line_problem(m=64, n1=64, n3=64, nt=128, seed=0, c=1.0, t0=0.0):
    rng = np.random.default_rng(np.random.SeedSequence([2, seed]))
    x = (np.arange(m) + 0.5 + rng.uniform(-0.4, 0.4, m)) / m
    xy = np.stack([x, np.full(m, 0.5)], 1)
    p = synth.make_problem(xy, np.full(m, 1.0 / m), [], nt, n1, 1, n3, c=c, dt=1.0 / nt, t0=t0,
                           d1=1.0 / n1, d2=1.0)
    g = rng.normal(size=(m, nt))
    v = rng.normal(size=(n1, 1, n3))
    return p, g, v


@pytest.mark.parametrize("prec", ["fp64", "fp32c"])
@pytest.mark.parametrize("kw", [dict(), dict(m=40, n1=48, n3=64, nt=96, seed=1, c=1.2, t0=0.01)])
def test_two_dimensional_operators(torch_gpu, prec, kw):
    p, g, v = _line_problem(**kw)
    geo = geometry_of(p)
    plan = make_plan(p, prec)
    assert plan.info["n2_os"] == 2
    gd, vd = to_dev(g, plan), to_dev(v, plan)
    F = O.spectrum(p.xy, p.h, g, geo)
    errs = {
        "volume": rel_l2(plan(gd).cpu().numpy(), O.volume_from_spectrum(F)),
        "spectrum": rel_l2(plan.spectrum(gd).cpu().numpy(), F),
        "adjoint": rel_l2(plan.adjoint(vd).cpu().numpy(), O.adjoint(v, p.xy, p.h, geo)),
        "q": rel_l2(plan.q(vd).cpu().numpy(), O.trace(v, p.xy, geo)),
        "q_adjoint": rel_l2(plan.q_adjoint(gd).cpu().numpy(), O.trace_adjoint(g, p.xy, geo)),
    }
    print(prec, kw, {k: f"{e:.2e}" for k, e in errs.items()})
    assert max(errs.values()) <= TOL, errs
