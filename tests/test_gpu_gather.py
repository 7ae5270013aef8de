"""The adjoint gather (the transpose of the spreading, eq. (10)) in its two
forms: the sweep gather (a wavefront per cell column walking the grid rows,
the sensors' taps from a ring of rows in registers; the default of float plans
with w <= 12) and the tile-staged gather (groups of four neighbouring sensors,
grid rows staged in LDS; the form of FP64 plans and w > 12). Both add the same
terms in the same order, so at 12 taps their results agree bit for bit, for
every sweep segment length; their agreement with the oracle's adjoint is
tested with the other adjoint tests."""
import numpy as np
import pytest

import oracle as O
import synth
from gpu_util import geometry_of, make_plan, rel_l2, small_problem, to_dev

pytestmark = pytest.mark.gpu

CASES = {
    "c1": lambda: synth.config("c1"),
    "ragged": lambda: small_problem(seed=2, s=10, nt=100, n=(10, 6, 30), c=1.3, t0=0.02, a=(0.25, -0.5),
                                    length=1.5),
    "narrow": lambda: small_problem(seed=3, s=9, nt=48, n=(12, 20, 24), d3=0.03, jitter=0.49),
}


@pytest.fixture(scope="module")
def torch_gpu():
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch


def _adjoint(plan, y, rows):
    plan.set_tuning(dict(gather_rows=rows))
    assert plan.tuning["gather_rows"] == rows
    return plan.adjoint(y).cpu().numpy()


@pytest.mark.parametrize("name", sorted(CASES))
@pytest.mark.parametrize("prec", ["fp32c", "fp32", "fp32w"])
def test_sweep_and_tiled_gather_agree_bitwise(torch_gpu, name, prec):
    p = CASES[name]()
    plan = make_plan(p, prec)
    assert plan.tuning["gather_rows"] > 0  # the sweep gather is the default here
    y = to_dev(np.random.default_rng(7).normal(size=(p.n1, p.n2, p.n3)), plan)
    tiled = _adjoint(plan, y, 0)
    for rows in (1, 3, 7, 64, 100000):
        got = _adjoint(plan, y, rows)
        assert np.array_equal(got, tiled), (name, prec, rows, np.abs(got - tiled).max())
    print(name, prec, "sweep gather == tiled gather for segments of 1, 3, 7, 64, 100000 rows")


def test_sweep_gather_kaiser_bessel_w8(torch_gpu):
    """At 8 taps the two forms still add the same terms in the same order, but
    the compiler fuses a few of the multiply-adds differently: a handful of
    values differ in the last bit. Both match the oracle."""
    p = synth.config("c1")
    plan = make_plan(p, "fp32c", w=8, window="kaiser_bessel")
    y = np.random.default_rng(3).normal(size=(p.n1, p.n2, p.n3))
    yd = to_dev(y, plan)
    tiled = _adjoint(plan, yd, 0)
    sweep = _adjoint(plan, yd, 64)
    assert np.abs(sweep - tiled).max() <= 4e-7 * np.abs(tiled).max()
    want = O.adjoint(y, p.xy, p.h, geometry_of(p))
    assert rel_l2(sweep, want) <= 1e-5 and rel_l2(tiled, want) <= 1e-5


def test_sweep_gather_c2_against_oracle(torch_gpu):
    """The whole adjoint with the sweep gather at 128x128 sensors against the oracle."""
    p = synth.config("c2")
    plan = make_plan(p, "fp32c")
    y = np.random.default_rng(5).normal(size=(p.n1, p.n2, p.n3))
    got = _adjoint(plan, to_dev(y, plan), 64)
    want = O.adjoint(y, p.xy, p.h, geometry_of(p))
    err = rel_l2(got, want)
    print("c2 adjoint, sweep gather, rel-L2", err)
    assert err <= 1e-5


def test_fp64_plans_take_the_tiled_gather(torch_gpu):
    import paper_1501_02946_amd as N
    p = synth.config("c1")
    plan = make_plan(p, "fp64")
    assert plan.tuning["gather_rows"] == 0
    with pytest.raises(N.NednerError):
        plan.set_tuning(dict(gather_rows=64))
    with pytest.raises(N.NednerError):
        make_plan(p, "fp32").set_tuning(dict(gather_rows=-1))
