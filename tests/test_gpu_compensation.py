"""Compensated spreading (eq. (10)) on data that defeats plain float sums.

A clump of 2048 sensors sits in one cell of the oversampled grid: 1024
positions, each carrying two sensors whose data are +A + s and -A + s' (the
first 1024 listed before the other 1024, so a plain running sum climbs to
about 1024 A before it cancels back to the size of the s terms). Every grid
value near the clump is a sum of 2048 terms. The NED stage (FFT of the spread
grid, deconvolved) is compared with the oracle's direct sums of eq. (5): the
compensated FP32 path must stay within the operator's tolerance and well below
the plain FP32 path, whose error grows with the partial sums.
"""
import numpy as np
import pytest

import oracle as O
import synth
from gpu_util import geometry_of, make_plan, phihat, rel_l2, to_dev

pytestmark = pytest.mark.gpu

TOL = 1e-5


@pytest.fixture(scope="module")
def torch_gpu():
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch


def _clump(amp, pairs=1024, nt=64, n=16, seed=5):
    rng = np.random.default_rng(seed)
    # one cell of the 2n x 2n oversampled grid near the aperture centre
    base = 0.5 + rng.uniform(0.05, 0.95, size=(pairs, 2)) / (2 * n)
    xy = np.concatenate([base, base])
    s = rng.standard_normal((2 * pairs, nt))
    g = np.concatenate([np.full((pairs, nt), amp), np.full((pairs, nt), -amp)]) + s
    h = np.full(2 * pairs, 1.0 / (2 * pairs))
    return synth.Problem(xy=xy, h=h, g=g, nt=nt, dt=1.0 / nt, c=1.0, n1=n, n2=n, n3=2 * n)


def _ned_error(p, prec, ref):
    plan = make_plan(p, prec)
    U = plan.grid(to_dev(p.g, plan)).cpu().numpy().astype(np.float64)
    n1, n2 = plan.info["n1_os"], plan.info["n2_os"]
    beta = plan.info["beta"]
    Uh = np.fft.fft2(U, axes=(0, 1))
    j1 = O.mode_numbers(p.n1)
    j2 = O.mode_numbers(p.n2)
    G = Uh[np.ix_(j1 % n1, j2 % n2)] / (phihat(beta, j1, n1)[:, None, None]
                                        * phihat(beta, j2, n2)[None, :, None])
    return rel_l2(G, ref)


def test_compensated_spreading_on_cancelling_clump(torch_gpu):
    p = _clump(4.0)
    ref = O.ned(p.xy, p.h, p.g, geometry_of(p))
    err = {prec: _ned_error(p, prec, ref) for prec in ("fp64", "fp32w", "fp32c", "fp32")}
    print("clump of 2048 sensors, NED stage rel-L2:",
          ", ".join(f"{k} {v:.3e}" for k, v in err.items()), flush=True)
    assert err["fp64"] <= TOL and err["fp32w"] <= TOL
    assert err["fp32c"] <= TOL
    assert err["fp32"] >= 5 * err["fp32c"]
