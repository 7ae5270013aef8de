"""Every launch shape the autotuner can pick gives the same operator: parity
with the oracle for each number of samples per lane, sweep length and
FFT-pass form (set through the tuning interface), forward and adjoint, in
each precision."""
import itertools

import numpy as np
import pytest

import oracle as O
from gpu_util import geometry_of, make_plan, rel_l2, small_problem, to_dev

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def case():
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    p = small_problem(seed=8, s=20, nt=128, n=(20, 24, 40), jitter=0.45)
    geo = geometry_of(p)
    v = O.volume_from_spectrum(O.spectrum(p.xy, p.h, p.g, geo))
    y = np.random.default_rng(2).normal(size=(p.n1, p.n2, p.n3))
    return p, geo, v, y, O.adjoint(y, p.xy, p.h, geo)


SHAPES = list(itertools.product([1, 2, 4], [1], [24, 40], [(16, 512, 1), (8, 256, 1), (16, 256, 0)]))


@pytest.mark.parametrize("prec", ["fp64", "fp32c", "fp32", "fp32w"])
def test_every_shape(case, prec):
    p, geo, v, y, aty = case
    plan = make_plan(p, prec)
    g = to_dev(p.g, plan)
    yy = to_dev(y, plan)
    worst = 0.0
    for tt, pd, S, (lines, threads, ip) in SHAPES:
        plan.set_tuning(dict(rows_per_wave=S, time_per_lane=tt, spread_depth=pd, pass_lines=lines,
                             pass_threads=threads, pass_inplace=ip))
        t = plan.tuning
        assert (t["time_per_lane"], t["spread_depth"], t["pass_inplace"]) == (tt, pd, ip)
        ev = rel_l2(plan(g).cpu().numpy(), v)
        ea = rel_l2(plan.adjoint(yy).cpu().numpy(), aty)
        worst = max(worst, ev, ea)
        assert ev <= 1e-5 and ea <= 1e-5, (tt, pd, S, lines, threads, ip, ev, ea)
    print(prec, len(SHAPES), "shapes, worst rel-L2", worst)
