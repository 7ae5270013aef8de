"""The equi-steradian sensor arrangement (paper, App. A) and its r^3 detector
weights (paper, Sec. 5): checks of the generator (CPU) and of the operator on
such a sparse mask against the oracle (GPU)."""
import math

import numpy as np
import pytest

import oracle as O
import synth
from gpu_util import geometry_of, make_plan, rel_l2, to_dev


@pytest.fixture(scope="module")
def layout():
    return synth.equi_steradian(1625, 0.265)


def test_rings_have_equal_solid_angle_per_sensor(layout):
    xy, rings = layout
    theta_max = math.atan(0.5 / 0.265)
    omega = 2 * math.pi * (1 - math.cos(theta_max)) / 1625
    for lo, hi, count in rings:
        assert abs(2 * math.pi * (math.cos(lo) - math.cos(hi)) / count - omega) < 1e-12 * omega
    assert rings[0][:1] == (0.0,) and rings[0][2] == 1
    counts = [c for _, _, c in rings[1:]]
    assert all(c & (c - 1) == 0 for c in counts)          # powers of two
    assert counts == sorted(counts)                        # never halves outwards
    assert rings[-1][1] <= theta_max
    assert abs(len(xy) - 1625) <= 0.05 * 1625              # the last partial ring is left out


def test_ring_geometry_on_the_plane(layout):
    xy, rings = layout
    assert np.all((xy >= 0) & (xy < 1))
    rho = np.hypot(xy[:, 0] - 0.5, xy[:, 1] - 0.5)
    start = 1
    for lo, hi, count in rings[1:]:
        ring = rho[start:start + count]
        # every sensor of a ring projects from the mid polar angle of the ring
        assert np.allclose(ring, 0.265 * math.tan(0.5 * (lo + hi)), rtol=1e-12)
        az = np.sort(np.mod(np.arctan2(xy[start:start + count, 1] - 0.5,
                                       xy[start:start + count, 0] - 0.5), 2 * math.pi))
        gaps = np.diff(np.concatenate([az, az[:1] + 2 * math.pi]))
        assert np.allclose(gaps, 2 * math.pi / count)
        start += count
    assert start == len(xy)


def test_snapped_mask_and_weights():
    xy, _ = synth.equi_steradian(1625, 0.265, grid=240)
    idx = np.round(xy * 240 - 0.5).astype(int)
    assert np.allclose((idx + 0.5) / 240, xy)
    assert len(np.unique(idx, axis=0)) == len(xy)
    h = synth.steradian_weights(xy, 0.265)
    r = np.sqrt(np.sum((xy - 0.5) ** 2, axis=1) + 0.265 ** 2)
    assert np.allclose(h / r ** 3, (h / r ** 3)[0])
    assert abs(h.sum() - 1.0) < 1e-12
    assert 5 < h.max() / h.min() < 15                      # outermost vs centre (paper: 9.7)


@pytest.mark.gpu
def test_sparse_mask_matches_oracle():
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    p = synth.config("c6sub")
    geo = geometry_of(p)
    v = O.volume_from_spectrum(O.spectrum(p.xy, p.h, p.g, geo))
    for prec in ("fp64", "fp32c"):
        plan = make_plan(p, prec)
        err = rel_l2(plan(to_dev(p.g, plan)).cpu().numpy(), v)
        print("equi-steradian mask", prec, p.m, "sensors", err)
        assert err <= 1e-5
