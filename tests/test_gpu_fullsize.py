"""Full-size parity in the launch configuration the benchmark times (default
plan, fp32c): the GPU spectrum at sampled modes against the oracle's sums at
those modes (the whole oracle spectrum of these workloads is too large to
evaluate in a test). Every sample includes the DC mode and the Nyquist corners."""
import numpy as np
import pytest

import oracle as O
import synth
from gpu_util import geometry_of, make_plan, rel_l2, to_dev

pytestmark = [pytest.mark.gpu, pytest.mark.slow]


@pytest.fixture(scope="module")
def torch_gpu():
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch


def _modes(p, count, seed):
    rng = np.random.default_rng(seed)
    m = np.stack([rng.integers(0, n, count) for n in (p.n1, p.n2, p.n3)], axis=1)
    corners = [[0, 0, 0], [p.n1 // 2, 0, 0], [0, p.n2 // 2, p.n3 // 2],
               [p.n1 // 2, p.n2 // 2, p.n3 // 2], [1, 2, 3], [p.n1 - 1, p.n2 - 1, p.n3 - 1]]
    return np.concatenate([m, corners])


@pytest.mark.parametrize("name", ["c3", "c5", "c6"])
def test_sampled_spectrum_full_size(torch_gpu, name):
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
    assert err <= 1e-5
