"""Pins for the oracle's forward operator Q (Sec. 2) and its adjoint.

Q maps an initial pressure on the periodic voxel grid to the trace, at the
sensors on the plane z = 0, of the wave equation's solution with zero initial
velocity. The pins: a term-by-term brute force, single Fourier modes (whose
solution is a standing wave in closed form), a Gaussian initial pressure
(whose radial solution in 3-D is known in closed form, summed here over the
periodic images of the grid), the initial condition at t = 0, the dense
transpose for the adjoint, and planted mistakes that some pin must reject.
"""
import math

import numpy as np
import pytest

import oracle as O


def _geo(n=(8, 6, 10), nt=7, dt=0.05, c=1.3, t0=0.07, a=(0.1, -0.2), d=(0.3, 0.2), d3=0.05):
    return O.geometry(nt=nt, dt=dt, c=c, n1=n[0], n2=n[1], n3=n[2], t0=t0, a1=a[0], a2=a[1],
                      d1=d[0], d2=d[1], d3=d3)


def _sensors(geo, m, seed):
    rng = np.random.default_rng(seed)
    return np.stack([geo.a1 + rng.uniform(0, geo.l1, m), geo.a2 + rng.uniform(0, geo.l2, m)], 1)


def _voxels(geo):
    x1 = geo.a1 + geo.d1 * np.arange(geo.n1)
    x2 = geo.a2 + geo.d2 * np.arange(geo.n2)
    z = geo.d3 * np.arange(geo.n3)
    return np.meshgrid(x1, x2, z, indexing="ij")


@pytest.mark.parametrize("kw", [
    {},
    dict(n=(4, 4, 4), c=1.0, t0=0.0, a=(0.0, 0.0), d=(0.25, 0.25), d3=0.25),
    dict(n=(6, 2, 6), nt=5, d3=0.04),
    dict(n=(2, 2, 2), nt=3),
    dict(n=(6, 1, 8), d=(0.3, 1.0)),   # two-dimensional problem
])
def test_trace_matches_brute_force(kw):
    geo = _geo(**kw)
    rng = np.random.default_rng(3)
    v = rng.normal(size=(geo.n1, geo.n2, geo.n3))
    xy = _sensors(geo, 5, 4)
    q = O.trace(v, xy, geo)
    qb = O.brute_trace(v, xy, geo)
    assert np.abs(q - qb).max() <= 1e-12 * max(1.0, np.abs(qb).max())


@pytest.mark.parametrize("phi0", [0.0, 0.7, math.pi / 2])
def test_single_mode_is_a_standing_wave(phi0):
    """v = cos(k.(x-a) + kz z + phi0) oscillates as cos(c|K|t) on every point."""
    geo = _geo()
    j1, j2, l = 2, -1, 3
    k1 = 2 * math.pi * j1 / geo.l1
    k2 = 2 * math.pi * j2 / geo.l2
    kz = 2 * math.pi * l / (geo.n3 * geo.d3)
    X1, X2, Z = _voxels(geo)
    v = np.cos(k1 * (X1 - geo.a1) + k2 * (X2 - geo.a2) + kz * Z + phi0)
    xy = _sensors(geo, 9, 5)
    t = geo.t0 + geo.dt * np.arange(geo.nt)
    kk = math.sqrt(k1 * k1 + k2 * k2 + kz * kz)
    want = (np.cos(k1 * (xy[:, 0, None] - geo.a1) + k2 * (xy[:, 1, None] - geo.a2) + phi0)
            * np.cos(geo.c * kk * t)[None, :])
    got = O.trace(v, xy, geo)
    assert np.abs(got - want).max() <= 1e-12


def _gaussian_trace(xy, t, x0, s, c, periods, reach=3):
    """Closed-form trace of the 3-D wave equation for p(x,0) = exp(-|x-x0|^2/(2 s^2)),
    summed over the periodic images x0 + (n1 L1, n2 L2, n3 L3).

    Radial solution: p(r,t) = [(r - ct) f(r - ct) + (r + ct) f(r + ct)] / (2r)
    with f(q) = exp(-q^2/(2 s^2)) (d'Alembert for r p, f even).
    """
    out = np.zeros((len(xy), len(t)))
    f = lambda q: np.exp(-q * q / (2 * s * s))  # noqa: E731
    rng = range(-reach, reach + 1)
    for n1 in rng:
        for n2 in rng:
            for n3 in rng:
                cx = x0[0] + n1 * periods[0]
                cy = x0[1] + n2 * periods[1]
                cz = x0[2] + n3 * periods[2]
                r = np.sqrt((xy[:, 0] - cx) ** 2 + (xy[:, 1] - cy) ** 2 + cz * cz)[:, None]
                ct = c * t[None, :]
                out += ((r - ct) * f(r - ct) + (r + ct) * f(r + ct)) / (2 * r)
    return out


@pytest.mark.parametrize("c,t0", [(1.0, 0.0), (1.4, 0.05)])
def test_gaussian_source_closed_form(c, t0):
    """The trace of a well-resolved Gaussian initial pressure equals the
    textbook radial solution summed over the grid's periodic images."""
    n = 32
    geo = O.geometry(nt=48, dt=1.0 / 64, c=c, n1=n, n2=n, n3=n, t0=t0, d3=1.0 / n)
    s = 2.5 / n
    x0 = (0.43, 0.56, 0.5)
    X1, X2, Z = _voxels(geo)
    v = np.zeros_like(X1)
    for a in (-1, 0, 1):
        for b in (-1, 0, 1):
            for e in (-1, 0, 1):
                v += np.exp(-((X1 - x0[0] - a) ** 2 + (X2 - x0[1] - b) ** 2 + (Z - x0[2] - e) ** 2)
                            / (2 * s * s))
    rng = np.random.default_rng(7)
    xy = np.stack([rng.uniform(0.2, 0.8, 12), rng.uniform(0.2, 0.8, 12)], 1)
    t = geo.t0 + geo.dt * np.arange(geo.nt)
    want = _gaussian_trace(xy, t, x0, s, c, (1.0, 1.0, 1.0))
    got = O.trace(v, xy, geo)
    assert np.abs(want).max() > 0.05  # the wavefront crosses the sensors in the window
    assert np.abs(got - want).max() <= 1e-9 * np.abs(want).max()


def test_initial_condition_on_grid_sensors():
    """At t = 0 the trace is the volume's z = 0 plane, at on-grid sensors exactly."""
    geo = _geo(t0=0.0)
    rng = np.random.default_rng(11)
    v = rng.normal(size=(geo.n1, geo.n2, geo.n3))
    i1 = rng.integers(0, geo.n1, 10)
    i2 = rng.integers(0, geo.n2, 10)
    xy = np.stack([geo.a1 + geo.d1 * i1, geo.a2 + geo.d2 * i2], 1)
    got = O.trace(v, xy, geo)
    assert np.abs(got[:, 0] - v[i1, i2, 0]).max() <= 1e-12


def test_trace_adjoint_is_dense_transpose():
    geo = _geo(n=(4, 2, 6), nt=4)
    xy = _sensors(geo, 3, 2)
    nv = geo.n1 * geo.n2 * geo.n3
    nd = len(xy) * geo.nt
    Q = np.stack([O.brute_trace(e.reshape(geo.n1, geo.n2, geo.n3), xy, geo).ravel()
                  for e in np.eye(nv)], axis=1)  # (nd, nv)
    QT = np.stack([O.trace_adjoint(e.reshape(len(xy), geo.nt), xy, geo).ravel()
                   for e in np.eye(nd)], axis=1)  # (nv, nd)
    assert np.abs(QT - Q.T).max() <= 1e-12 * np.abs(Q).max()


def test_trace_adjoint_identity_medium():
    geo = _geo(n=(16, 12, 20), nt=24, dt=0.02)
    rng = np.random.default_rng(1)
    xy = _sensors(geo, 40, 3)
    v = rng.normal(size=(geo.n1, geo.n2, geo.n3))
    d = rng.normal(size=(len(xy), geo.nt))
    lhs = np.sum(O.trace(v, xy, geo) * d)
    rhs = np.sum(v * O.trace_adjoint(d, xy, geo))
    assert abs(lhs - rhs) <= 1e-11 * abs(lhs)


def test_trace_pins_reject_planted_mistakes(monkeypatch):
    """A wrong |K| (a dropped depth wavenumber, a stretched one) or a
    conjugated lateral exponential fails the closed-form pins."""
    mod = O.nedner_oracle
    good_k = mod._abs_k

    def no_depth(geo):
        k1, k2, _ = mod.wavenumbers(geo)
        return np.broadcast_to(np.sqrt(k1[:, None, None] ** 2 + k2[None, :, None] ** 2),
                               (geo.n1, geo.n2, geo.n3))

    for bad in (no_depth, lambda geo: 1.01 * good_k(geo)):
        monkeypatch.setattr(mod, "_abs_k", bad)
        with pytest.raises(AssertionError):
            test_single_mode_is_a_standing_wave(0.7)
        monkeypatch.setattr(mod, "_abs_k", good_k)

    good_lat = mod._lateral_factors

    def conj_lat(xy, geo):
        e1, e2 = good_lat(xy, geo)
        return np.conj(e1), np.conj(e2)

    monkeypatch.setattr(mod, "_lateral_factors", conj_lat)
    with pytest.raises(AssertionError):
        test_single_mode_is_a_standing_wave(0.7)
    with pytest.raises(AssertionError):
        test_gaussian_source_closed_form(1.0, 0.0)
