"""Pins for the oracle's image quality measures (App. B) and projections.

The correlation coefficient against numpy's own and its invariances; the
Tenenbaum sharpness against closed forms (a linear ramp gives Sobel responses
8 beta and 8 alpha at every interior pixel, a single bright pixel gives the
squared Sobel weights, 24); the projections against explicit loops.
"""
import numpy as np
import pytest

import oracle as O


def test_corrcoef_matches_numpy_and_invariances():
    rng = np.random.default_rng(0)
    a = rng.normal(size=(12, 9, 7))
    b = 0.3 * a + rng.normal(size=a.shape)
    assert abs(O.corrcoef(a, b) - np.corrcoef(a.ravel(), b.ravel())[0, 1]) <= 1e-14
    assert abs(O.corrcoef(a, b) - O.corrcoef(b, a)) <= 1e-15
    assert abs(O.corrcoef(a, 2.5 * a + 4.0) - 1.0) <= 1e-14
    assert abs(O.corrcoef(a, -0.5 * a + 1.0) + 1.0) <= 1e-14
    mask = rng.random(a.shape) < 0.4
    want = np.corrcoef(a[mask], b[mask])[0, 1]
    assert abs(O.corrcoef(a, b, mask) - want) <= 1e-14


@pytest.mark.parametrize("alpha,beta", [(1.0, 0.0), (0.0, 1.0), (0.7, -1.3)])
def test_tenenbaum_of_a_ramp(alpha, beta):
    rows, cols = 9, 13
    r, c = np.meshgrid(np.arange(rows), np.arange(cols), indexing="ij")
    u = alpha * r + beta * c + 5.0
    valid = (rows - 2) * (cols - 2)
    assert abs(O.tenenbaum(u) - valid * 64.0 * (alpha ** 2 + beta ** 2)) <= 1e-9
    # a sub-rectangle touching the border keeps only pixels with a full stencil
    got = O.tenenbaum(u, rect=(0, 4, 3, 13))
    assert abs(got - (4 - 1) * (12 - 3) * 64.0 * (alpha ** 2 + beta ** 2)) <= 1e-9


@pytest.mark.parametrize("rows,cols", [(9, 13), (30, 7), (64, 64)])
def test_tenenbaum_mean_of_a_ramp_is_size_free(rows, cols):
    """App. B normalises the measure by the element count N of the image: for
    a ramp F = (rows - 2)(cols - 2) 64 (alpha^2 + beta^2) and N = rows cols, so
    F / N tends to 64 (alpha^2 + beta^2) as the image grows."""
    alpha, beta = 0.7, -1.3
    r, c = np.meshgrid(np.arange(rows), np.arange(cols), indexing="ij")
    u = alpha * r + beta * c
    per_pixel = 64.0 * (alpha ** 2 + beta ** 2)
    want = (rows - 2) * (cols - 2) * per_pixel / (rows * cols)
    assert abs(O.tenenbaum_mean(u) - want) <= 1e-12 * want
    # over a rectangle N counts the rectangle's elements, border pixels included
    got = O.tenenbaum_mean(u, rect=(0, 4, 3, cols))
    assert abs(got - (4 - 1) * (cols - 1 - 3) * per_pixel / (4 * (cols - 3))) <= 1e-9
    assert O.tenenbaum_mean(u, rect=(2, 2, 0, cols)) == 0.0


def test_tenenbaum_of_a_point():
    u = np.zeros((11, 10))
    u[5, 4] = 1.0
    assert abs(O.tenenbaum(u) - 24.0) <= 1e-12
    # the point's responses outside the rectangle are not counted
    assert abs(O.tenenbaum(u, rect=(5, 6, 4, 5)) - 0.0) <= 1e-12
    # pixels (4, 3..5): the point sits in the stencils' bottom row, where g
    # reads (1, 0, -1) and g^T reads (1, 2, 1): 2 + 4 + 2
    assert abs(O.tenenbaum(u, rect=(4, 5, 3, 6)) - 8.0) <= 1e-12


def test_mip_matches_loops():
    rng = np.random.default_rng(1)
    v = rng.normal(size=(4, 5, 6))
    for axis in range(3):
        got = O.mip(v, axis)
        want = np.full(got.shape, -np.inf)
        for idx in np.ndindex(v.shape):
            rest = tuple(i for k, i in enumerate(idx) if k != axis)
            want[rest] = max(want[rest], v[idx])
        assert np.array_equal(got, want)
