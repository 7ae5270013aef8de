"""Full-size parity in the launch configuration the benchmark times (default
plans): the whole reconstructed volume of the 65536-sensor and the
192x192-sensor workloads against the oracle's volume, every problem of the
64-problem batch against the oracle, the adjoint of the 65536-sensor workload
at sampled sensors and times, and the spectrum at sampled modes on the
equi-steradian mask. Each oracle volume is computed once per module (the
65536-sensor one takes one to two minutes on the host) and shared by the
precisions; the batch's 64 oracle volumes are computed in worker processes.
"""
import multiprocessing as mp
import os

import numpy as np
import pytest

import oracle as O
import synth
from gpu_util import geometry_of, make_plan, rel_l2, to_dev

pytestmark = [pytest.mark.gpu, pytest.mark.slow]
TOL = 1e-5


@pytest.fixture(scope="module")
def torch_gpu():
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch


@pytest.fixture(scope="module")
def c3_case():
    p = synth.config("c3")
    vol = O.forward(p.xy, p.h, p.g, geometry_of(p))
    return p, vol


@pytest.fixture(scope="module")
def c5_case():
    p = synth.config("c5")
    vol = O.forward(p.xy, p.h, p.g, geometry_of(p))
    return p, vol


def _gpu_volume(torch, p, prec):
    plan = make_plan(p, prec)
    out = plan(to_dev(p.g, plan)).cpu().numpy()
    del plan
    torch.cuda.empty_cache()
    return out


@pytest.mark.timeout(900)
@pytest.mark.parametrize("prec", ["fp32c", "fp64", "fp32", "fp32w"])
def test_c3_volume_against_full_oracle(torch_gpu, c3_case, prec):
    """65536 sensors (4x denser near the centre), 1024 samples, 256x256x512."""
    p, vol = c3_case
    print(f"c3 {prec}: {p.m} sensors x {p.nt} samples -> {(p.n1, p.n2, p.n3)}", flush=True)
    err = rel_l2(_gpu_volume(torch_gpu, p, prec), vol)
    print(f"c3 {prec} volume rel-L2 {err:.3e}", flush=True)
    assert err <= TOL


@pytest.mark.timeout(900)
@pytest.mark.parametrize("prec", ["fp32c", "fp64"])
def test_c5_volume_against_full_oracle(torch_gpu, c5_case, prec):
    """192x192 jittered sensors, 768 samples, 192x192x384."""
    p, vol = c5_case
    print(f"c5 {prec}: {p.m} sensors x {p.nt} samples -> {(p.n1, p.n2, p.n3)}", flush=True)
    err = rel_l2(_gpu_volume(torch_gpu, p, prec), vol)
    print(f"c5 {prec} volume rel-L2 {err:.3e}", flush=True)
    assert err <= TOL


@pytest.mark.timeout(900)
def test_c3_adjoint_at_sampled_sensors(torch_gpu, c3_case):
    """The adjoint (tile-ordered sensor gather, LDS-staged and direct paths) at
    the full 65536-sensor density: plan.adjoint of a volume at 48 sensors (the
    hotspot's included) and 4 times against the oracle's restricted sums."""
    torch = torch_gpu
    p, vol = c3_case
    geo = geometry_of(p)
    rng = np.random.default_rng(31)
    r2 = (p.xy[:, 0] - 0.5) ** 2 + (p.xy[:, 1] - 0.5) ** 2
    inner = np.flatnonzero(r2 < 0.25 ** 2)
    outer = np.flatnonzero(r2 >= 0.25 ** 2)
    sel = np.concatenate([rng.choice(inner, 24, replace=False), rng.choice(outer, 24, replace=False)])
    tid = np.sort(rng.choice(p.nt, 4, replace=False))
    want = O.adjoint_at(vol, p.xy[sel], p.h[sel], geo, tid)
    for prec in ("fp32c", "fp64"):
        plan = make_plan(p, prec)
        got = plan.adjoint(to_dev(vol, plan)).cpu().numpy()[np.ix_(sel, tid)].astype(np.float64)
        del plan
        torch.cuda.empty_cache()
        err = rel_l2(got, want)
        print(f"c3 {prec} adjoint at 48 sensors x 4 times rel-L2 {err:.3e}", flush=True)
        assert err <= TOL


def _limit_threads():
    for k in ("OMP_NUM_THREADS", "OPENBLAS_NUM_THREADS", "MKL_NUM_THREADS"):
        os.environ[k] = "1"


def _oracle_volume(args):
    i, xy, h, g, kw = args
    return i, O.forward(xy, h, g, O.geometry(**kw))


@pytest.mark.timeout(900)
def test_c4_every_problem_against_oracle(torch_gpu):
    """The 64-problem batch (M in [1024, 16384], Nt in {256, 512, 1024}) in one
    persistent launch per stage: every problem's volume against the oracle's."""
    import paper_1501_02946_amd as N
    torch = torch_gpu
    probs = synth.batch_c4()
    tasks = sorted(((i, p.xy, p.h, p.g, p.geometry_kwargs()) for i, p in enumerate(probs)),
                   key=lambda t: -t[3].size * t[1].shape[0])
    workers = max(1, min(16, os.cpu_count() or 1))
    # worker processes of their own (fresh interpreters, one BLAS thread each)
    # compute the oracle while the GPU runs the batch
    pool = mp.get_context("spawn").Pool(workers, initializer=_limit_threads)
    try:
        pending = pool.imap_unordered(_oracle_volume, tasks)
        bp = N.BatchPlan([dict(xy=p.xy, h=p.h, nt=p.nt, dt=p.dt, volume=(p.n1, p.n2, p.n3)) for p in probs],
                         precision="fp32c")
        gs = [torch.as_tensor(p.g, dtype=torch.float32, device=bp.device) for p in probs]
        outs = [o.cpu().numpy() for o in bp(gs)]
        errs = np.zeros(len(probs))
        for i, v in pending:
            errs[i] = rel_l2(outs[i], v)
    finally:
        pool.close()
        pool.join()
    worst = int(np.argmax(errs))
    print(f"c4: 64 problems, max rel-L2 {errs.max():.3e} (problem {worst}: {probs[worst].m} sensors, "
          f"{probs[worst].nt} samples), median {np.median(errs):.3e}", flush=True)
    assert errs.max() <= TOL


def _modes(p, count, seed):
    rng = np.random.default_rng(seed)
    m = np.stack([rng.integers(0, n, count) for n in (p.n1, p.n2, p.n3)], axis=1)
    corners = [[0, 0, 0], [p.n1 // 2, 0, 0], [0, p.n2 // 2, p.n3 // 2],
               [p.n1 // 2, p.n2 // 2, p.n3 // 2], [1, 2, 3], [p.n1 - 1, p.n2 - 1, p.n3 - 1]]
    return np.concatenate([m, corners])


@pytest.mark.parametrize("name", ["c3", "c5", "c6"])
def test_sampled_spectrum_full_size(torch_gpu, name):
    """The spectrum output (no depth IFFT) at sampled modes, DC and Nyquist corners included."""
    torch = torch_gpu
    p = synth.config(name)
    plan = make_plan(p, "fp32c")
    F = plan.spectrum(to_dev(p.g, plan))
    modes = _modes(p, 96, seed=len(name))
    idx = torch.as_tensor(modes, device=F.device)
    got = F[idx[:, 0], idx[:, 1], idx[:, 2]].cpu().numpy().astype(np.complex128)
    ref = O.spectrum_at(p.xy, p.h, p.g, geometry_of(p), modes)
    err = rel_l2(got, ref)
    print(name, p.m, "sensors", p.nt, "samples", (p.n1, p.n2, p.n3), "sampled spectrum rel-L2", err)
    assert err <= TOL
