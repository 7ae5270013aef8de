"""Batched execution: one persistent launch per stage over problems of uneven size."""
import numpy as np
import pytest

import oracle as O
import synth
from gpu_util import geometry_of, rel_l2, small_problem

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def torch_gpu():
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch


def _kw(p):
    return dict(xy=p.xy, h=p.h, nt=p.nt, dt=p.dt, volume=(p.n1, p.n2, p.n3), c=p.c, t0=p.t0,
                a1=p.a1, a2=p.a2, d1=p.d1, d2=p.d2, d3=p.d3)


def _uneven():
    return [small_problem(seed=20, s=12, nt=40, n=(12, 12, 20)),
            small_problem(seed=21, s=20, nt=64, n=(20, 16, 32)),
            small_problem(seed=22, s=8, nt=32, n=(8, 10, 16), c=1.2),
            small_problem(seed=23, s=16, nt=96, n=(16, 16, 48), a=(0.2, 0.1)),
            synth.config("c5sub"),
            synth.config("c1")]


@pytest.mark.parametrize("prec", ["fp64", "fp32c"])
def test_batch_matches_oracle_and_single_plans(torch_gpu, prec):
    import paper_1501_02946_amd as N
    torch = torch_gpu
    probs = _uneven()
    bp = N.BatchPlan([_kw(p) for p in probs], precision=prec, time_per_lane=2)
    dt = torch.float64 if prec == "fp64" else torch.float32
    gs = [torch.as_tensor(p.g, dtype=dt, device=bp.device) for p in probs]
    outs = [o.cpu().numpy() for o in bp(gs)]
    for p, o, g in zip(probs, outs, gs):
        ref = O.forward(p.xy, p.h, p.g, geometry_of(p))
        err = rel_l2(o, ref)
        single = N.Plan(p.xy, p.nt, p.dt, (p.n1, p.n2, p.n3), c=p.c, h=p.h, t0=p.t0, a1=p.a1,
                        a2=p.a2, d1=p.d1, d2=p.d2, d3=p.d3, precision=prec, time_per_lane=2,
                        rows_per_wave=256)  # the batch's default sweep (clamped to the grid)
        so = single(g).cpu().numpy()
        print(prec, p.m, p.nt, (p.n1, p.n2, p.n3), "batch vs oracle", err, "bitwise", np.array_equal(so, o))
        assert err <= 1e-5
        assert np.array_equal(so, o)
    # a second execute with fresh outputs gives the same bits
    again = [o.cpu().numpy() for o in bp(gs)]
    assert all(np.array_equal(a, b) for a, b in zip(again, outs))


@pytest.mark.slow
def test_c4_batch_64_problems(torch_gpu):
    """The 64-problem batch (M in [1024, 16384], Nt in {256, 512, 1024}) against single plans."""
    import paper_1501_02946_amd as N
    torch = torch_gpu
    probs = synth.batch_c4()
    bp = N.BatchPlan([_kw(p) for p in probs], precision="fp32c")
    gs = [torch.as_tensor(p.g, dtype=torch.float32, device=bp.device) for p in probs]
    outs = bp(gs)
    torch.cuda.synchronize()
    for i in (0, 17, 63):
        p = probs[i]
        single = N.Plan(p.xy, p.nt, p.dt, (p.n1, p.n2, p.n3), h=p.h, precision="fp32c",
                        time_per_lane=4, rows_per_wave=256)
        assert np.array_equal(single(gs[i]).cpu().numpy(), outs[i].cpu().numpy())
    p = probs[5]
    ref = O.forward(p.xy, p.h, p.g, geometry_of(p))
    err = rel_l2(outs[5].cpu().numpy(), ref)
    print("c4 problem 5", p.m, p.nt, (p.n1, p.n2, p.n3), "vs oracle", err)
    assert err <= 1e-5


def test_autotune_single_and_cache(torch_gpu, tmp_path):
    import paper_1501_02946_amd as N
    torch = torch_gpu
    p = synth.config("c1")
    plan = N.Plan(p.xy, p.nt, p.dt, (p.n1, p.n2, p.n3), h=p.h, precision="fp32c")
    g = torch.as_tensor(p.g, dtype=torch.float32, device=plan.device)
    cache = str(tmp_path / "tuning.json")
    best = plan.autotune(g, cache=cache)
    print("autotune", best)
    assert best["ms_execute"] > 0 and best["rows_per_wave"] >= 12
    ref = O.forward(p.xy, p.h, p.g, geometry_of(p))
    assert rel_l2(plan(g).cpu().numpy(), ref) <= 1e-5
    plan2 = N.Plan(p.xy, p.nt, p.dt, (p.n1, p.n2, p.n3), h=p.h, precision="fp32c")
    again = plan2.autotune(g, cache=cache)
    assert again == best
    t = plan2.tuning
    for k in ("rows_per_wave", "time_per_lane", "spread_depth", "pass_lines", "pass_threads",
              "pass_inplace"):
        assert t[k] == best[k]
    assert np.array_equal(plan(g).cpu().numpy(), plan2(g).cpu().numpy())


def test_autotune_batch(torch_gpu):
    import paper_1501_02946_amd as N
    torch = torch_gpu
    probs = _uneven()
    bp = N.BatchPlan([_kw(p) for p in probs], precision="fp32c")
    print("batch autotune", bp.autotune())
    gs = [torch.as_tensor(p.g, dtype=torch.float32, device=bp.device) for p in probs]
    for p, o in zip(probs, bp(gs)):
        assert rel_l2(o.cpu().numpy(), O.forward(p.xy, p.h, p.g, geometry_of(p))) <= 1e-5
