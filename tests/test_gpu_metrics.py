"""GPU parity of the image measures (App. B) and projections against the oracle.

Maximum intensity projections are exact (a maximum rounds nothing). The
correlation coefficient and the Tenenbaum sharpness accumulate in double on
both sides from the same input values, in different orders: 1e-12 relative.
"""
import numpy as np
import pytest

import oracle as O
import synth
from gpu_util import geometry_of, make_plan, to_dev

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def torch_gpu():
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch


@pytest.mark.parametrize("dtype", ["float32", "float64"])
@pytest.mark.parametrize("shape", [(5, 7, 70), (16, 8, 129), (3, 4, 1), (1, 1, 64)])
def test_mip_exact(torch_gpu, dtype, shape):
    torch = torch_gpu
    import paper_1501_02946_amd as N
    rng = np.random.default_rng(sum(shape))
    v = rng.normal(size=shape).astype(dtype)
    t = torch.as_tensor(v, device="cuda")
    for axis in range(3):
        got = N.mip(t, axis).cpu().numpy()
        assert np.array_equal(got, O.mip(v, axis)), (shape, axis)


@pytest.mark.parametrize("dtype", ["float32", "float64"])
@pytest.mark.parametrize("n", [1, 777, 300_001])
def test_corrcoef(torch_gpu, dtype, n):
    torch = torch_gpu
    import paper_1501_02946_amd as N
    rng = np.random.default_rng(n)
    a = (rng.normal(size=n) + 3.0).astype(dtype)
    b = (0.6 * a + rng.normal(size=n)).astype(dtype)
    ta, tb = torch.as_tensor(a, device="cuda"), torch.as_tensor(b, device="cuda")
    got = N.corrcoef(ta, tb)
    if n == 1:
        assert np.isnan(got)  # zero variance
        return
    want = O.corrcoef(a, b)
    assert abs(got - want) <= 1e-12 * abs(want)
    mask = rng.random(n) < 0.3
    got_m = N.corrcoef(ta, tb, torch.as_tensor(mask, device="cuda"))
    want_m = O.corrcoef(a, b, mask)
    assert abs(got_m - want_m) <= 1e-12 * abs(want_m)
    assert N.corrcoef(ta, tb) == got  # deterministic
    assert abs(N.corrcoef(ta, ta) - 1.0) <= 1e-14


@pytest.mark.parametrize("dtype", ["float32", "float64"])
@pytest.mark.parametrize("shape,rect", [((40, 33), None), ((40, 33), (0, 12, 5, 33)),
                                        ((3, 3), None), ((2, 9), None), ((64, 70), (10, 11, 0, 70))])
def test_tenenbaum(torch_gpu, dtype, shape, rect):
    torch = torch_gpu
    import paper_1501_02946_amd as N
    rng = np.random.default_rng(shape[0] * 100 + shape[1])
    u = rng.normal(size=shape).astype(dtype)
    got = N.tenenbaum(torch.as_tensor(u, device="cuda"), rect)
    want = O.tenenbaum(u, rect)
    assert abs(got - want) <= 1e-12 * max(abs(want), 1e-300)
    got_mean = N.tenenbaum(torch.as_tensor(u, device="cuda"), rect, normalized=True)
    want_mean = O.tenenbaum_mean(u, rect)
    assert abs(got_mean - want_mean) <= 1e-12 * max(abs(want_mean), 1e-300)


def test_tenenbaum_ramp_large(torch_gpu):
    """A 1000 x 777 ramp: every interior pixel gives 64 (alpha^2 + beta^2)."""
    torch = torch_gpu
    import paper_1501_02946_amd as N
    rows, cols, alpha, beta = 1000, 777, 0.25, -0.5
    r, c = np.meshgrid(np.arange(rows), np.arange(cols), indexing="ij")
    u = alpha * r + beta * c
    got = N.tenenbaum(torch.as_tensor(u, device="cuda"))
    want = (rows - 2) * (cols - 2) * 64.0 * (alpha ** 2 + beta ** 2)
    assert abs(got - want) <= 1e-12 * want


def test_measures_on_a_reconstruction(torch_gpu):
    """The c1 reconstruction against the oracle's: correlation ~1, and the
    xy-MIP's sharpness matching the oracle's measure of the same MIP."""
    import paper_1501_02946_amd as N
    p = synth.config("c1")
    plan = make_plan(p, "fp32c")
    vol = plan(to_dev(p.g, plan))
    ref = O.forward(p.xy, p.h, p.g, geometry_of(p))
    rho = N.corrcoef(vol.double(), to_dev(ref, plan).double())
    assert rho > 1.0 - 1e-10
    m = N.mip(vol, 2)
    assert abs(N.tenenbaum(m) - O.tenenbaum(m.cpu().numpy())) <= 1e-12 * O.tenenbaum(m.cpu().numpy())
