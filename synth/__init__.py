"""Seeded synthetic inputs for the NEDNER reconstruction operator.

This module builds sensor layouts, detector weights, time grids and recorded
pressure traces. It holds none of the reconstruction's arithmetic: the only
physics here is the closed-form pressure trace of a uniform ball (the forward
wave problem of Sec. 2), which is how test data are produced, not how they are
reconstructed. Both the GPU path and the oracle take their inputs from here.

Workload recipes (all with sound speed c = 1 and aperture [0,1)^2):

* ``c1``: 32x32 sensors jittered by +/-0.4 pitch, 128 samples, dt = 1/128, one
  ball (p0=1, R=0.1, centre (0.5,0.5,0.4)); output 32x32x64.
* ``c2``: 128x128 sensors jittered by +/-0.45 pitch, 512 samples, 10 random
  balls, 1 % Gaussian noise; output 128x128x256.
* ``c3``: 65536 i.i.d. sensors, 4x denser inside radius 0.25 of the aperture
  centre, h_m = 1/(M p(y_m)); 1024 samples; 30 balls and 5 bead-chain
  cylinders; output 256x256x512.
* ``c5``: 192x192 sensors jittered by +/-0.4, 768 samples, 20 balls, 1 % noise;
  output 192x192x384.
* ``c6``: the equi-steradian mask of App. A: ~1625 sensors snapped to a
  240x240 grid, centre of interest 0.265 above the aperture centre, weights
  h_m ~ r^3; 512 samples, 10 balls, 1 % noise; output 240x240x256.
* ``c8``: the two-dimensional problem: 1024 sensors on a line (jittered
  +/-0.4 pitch), 2048 samples, 10 balls centred on the sensors' plane, 1 %
  noise; output 1024x1x256 (the grid of the paper's 2-D study).
* ``c7``: 128x128 sensors on the nodes of the 128x128 output grid (the
  equispaced, NER-only case), 512 samples, 10 balls, 1 % noise; output
  128x128x256.
* ``c4``: 64 problems, M uniform in [1024, 16384] kept from a ceil(sqrt(M))^2
  jittered grid, Nt in {256, 512, 1024}, 1-10 balls each, output s x s x Nt/2
  with s the smallest even 5-smooth integer >= ceil(sqrt(M)) (the mode sets
  {-N/2..N/2-1} need even N).

Time span T = Nt*dt = 1 everywhere (dt = 1/Nt), depth step d3 = c*T/N3.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np

__all__ = [
    "Problem", "jittered_grid", "density_sensors", "random_balls",
    "bead_chain", "ball_signal", "add_noise", "make_problem", "config",
    "five_smooth_at_least", "batch_c4", "equi_steradian", "steradian_weights",
]


@dataclass
class Problem:
    """One reconstruction problem: sensors, weights, data and output grid."""

    xy: np.ndarray          # (M, 2) float64 sensor positions
    h: np.ndarray           # (M,) float64 detector areas, sum = L1*L2
    g: np.ndarray           # (M, Nt) float64 recorded data, time fastest
    nt: int
    dt: float
    c: float
    n1: int
    n2: int
    n3: int
    t0: float = 0.0
    a1: float = 0.0
    a2: float = 0.0
    d1: float = 0.0         # 0 -> 1/n1 (unit aperture)
    d2: float = 0.0
    d3: float = 0.0         # 0 -> c*nt*dt/n3
    balls: list = field(default_factory=list)
    name: str = ""

    def __post_init__(self):
        if self.d1 == 0.0:
            self.d1 = 1.0 / self.n1
        if self.d2 == 0.0:
            self.d2 = 1.0 / self.n2
        if self.d3 == 0.0:
            self.d3 = self.c * self.nt * self.dt / self.n3

    @property
    def m(self) -> int:
        return int(self.xy.shape[0])

    def geometry_kwargs(self) -> dict:
        return dict(nt=self.nt, t0=self.t0, dt=self.dt, c=self.c,
                    n1=self.n1, n2=self.n2, n3=self.n3, a1=self.a1,
                    a2=self.a2, d1=self.d1, d2=self.d2, d3=self.d3)


def phantom_volume(p: "Problem") -> np.ndarray:
    """The problem's balls sampled on its voxel grid: voxel (i1, i2, i3) at
    (a1 + i1 d1, a2 + i2 d2, i3 d3) takes the sum of p0 over the balls that
    contain it (d1, d2 default to 1/n, d3 to c nt dt / n3, as in the plans)."""
    d1 = p.d1 or 1.0 / p.n1
    d2 = p.d2 or 1.0 / p.n2
    d3 = p.d3 or p.c * p.nt * p.dt / p.n3
    x1 = p.a1 + d1 * np.arange(p.n1)
    x2 = p.a2 + d2 * np.arange(p.n2)
    z = d3 * np.arange(p.n3)
    out = np.zeros((p.n1, p.n2, p.n3))

    def span(lo, step, n, c, R):
        # voxel indices whose coordinate lies within [c - R, c + R], one wider each side
        i0 = max(int(np.floor((c - R - lo) / step)) - 1, 0)
        i1 = min(int(np.ceil((c + R - lo) / step)) + 2, n)
        return slice(i0, max(i0, i1))

    for (bx, by, bz, R, p0) in p.balls:
        s1, s2, s3 = span(p.a1, d1, p.n1, bx, R), span(p.a2, d2, p.n2, by, R), span(0.0, d3, p.n3, bz, R)
        r2 = ((x1[s1, None, None] - bx) ** 2 + (x2[None, s2, None] - by) ** 2
              + (z[None, None, s3] - bz) ** 2)
        out[s1, s2, s3] += np.where(r2 <= R * R, p0, 0.0)
    return out


def five_smooth_at_least(n: int, even: bool = False) -> int:
    """Smallest integer >= n whose prime factors are all in {2, 3, 5} (even if asked)."""
    k = max(1, int(n))
    while True:
        r = k
        for p in (2, 3, 5):
            while r % p == 0:
                r //= p
        if r == 1 and (not even or k % 2 == 0):
            return k
        k += 1


def jittered_grid(s: int, jitter: float, rng: np.random.Generator,
                  lo: float = 0.0, length: float = 1.0) -> np.ndarray:
    """s*s nodes at cell centres (i+1/2)/s plus uniform jitter of +/-jitter pitch.

    With jitter < 0.5 every node stays strictly inside its own cell, hence
    inside [lo, lo+length)^2. Row-major order (first coordinate slowest).
    """
    pitch = length / s
    i = np.arange(s, dtype=np.float64)
    g1, g2 = np.meshgrid(i, i, indexing="ij")
    base = np.stack([g1.ravel(), g2.ravel()], axis=1) + 0.5
    if jitter > 0.0:
        base = base + rng.uniform(-jitter, jitter, size=base.shape)
    return lo + base * pitch


def density_sensors(m: int, rng: np.random.Generator, ratio: float = 4.0,
                    radius: float = 0.25, centre=(0.5, 0.5)):
    """m i.i.d. sensors on [0,1)^2, `ratio` times denser inside a disc.

    Returns (xy, h) with h_m = 1/(m p(y_m)), p the sampling density, so that
    sum h is an unbiased estimate of the aperture area 1.
    """
    cx, cy = centre
    area_in = math.pi * radius * radius
    z = ratio * area_in + (1.0 - area_in)
    p_in, p_out = ratio / z, 1.0 / z
    # mixture sampling: draw from the disc with probability ratio*area_in/z
    n_in = rng.binomial(m, ratio * area_in / z)
    r = radius * np.sqrt(rng.uniform(0.0, 1.0, n_in))
    th = rng.uniform(0.0, 2.0 * math.pi, n_in)
    xin = np.stack([cx + r * np.cos(th), cy + r * np.sin(th)], axis=1)
    xout = np.empty((0, 2))
    need = m - n_in
    while xout.shape[0] < need:
        cand = rng.uniform(0.0, 1.0, size=(2 * need + 16, 2))
        keep = (cand[:, 0] - cx) ** 2 + (cand[:, 1] - cy) ** 2 >= radius * radius
        xout = np.concatenate([xout, cand[keep]], axis=0)
    xy = np.concatenate([xin, xout[:need]], axis=0)
    xy = xy[rng.permutation(m)]
    inside = (xy[:, 0] - cx) ** 2 + (xy[:, 1] - cy) ** 2 < radius * radius
    p = np.where(inside, p_in, p_out)
    return xy, 1.0 / (m * p)


def random_balls(k: int, rng: np.random.Generator, rmin=0.02, rmax=0.08,
                 amin=0.5, amax=1.0, lo=(0.1, 0.1, 0.1), hi=(0.9, 0.9, 0.6)):
    """k balls (cx, cy, cz, R, p0) with uniform radii, amplitudes and centres."""
    out = []
    for _ in range(k):
        cx = rng.uniform(lo[0], hi[0])
        cy = rng.uniform(lo[1], hi[1])
        cz = rng.uniform(lo[2], hi[2])
        out.append((cx, cy, cz, rng.uniform(rmin, rmax), rng.uniform(amin, amax)))
    return out


def bead_chain(rng: np.random.Generator, radius=0.01, amp=None):
    """A thin cylinder parallel to the sensor plane, as a chain of touching balls.

    Balls of radius `radius` spaced `radius` apart along a random in-plane
    axis at a random depth; amplitude 0.75*a so that the mean fill is about a.
    The pressure trace of each bead is known exactly, so the chain's is too.
    """
    a = rng.uniform(0.5, 1.0) if amp is None else amp
    length = rng.uniform(0.2, 0.5)
    th = rng.uniform(0.0, math.pi)
    cx, cy, cz = rng.uniform(0.3, 0.7), rng.uniform(0.3, 0.7), rng.uniform(0.1, 0.6)
    nb = int(length / radius) + 1
    s = (np.arange(nb) - (nb - 1) / 2.0) * radius
    return [(cx + si * math.cos(th), cy + si * math.sin(th), cz, radius, 0.75 * a)
            for si in s]


def ball_signal(xy: np.ndarray, times: np.ndarray, balls, c: float = 1.0,
                chunk: int = 4096) -> np.ndarray:
    """Pressure at sensors on z=0 from uniform balls (initial pressure p0 inside).

    Closed form of the wave problem in Sec. 2 for a uniform ball seen from
    outside it: p(r,t) = p0 (r - c t)/(2 r) when |r - c t| <= R, else 0, with r
    the sensor-to-centre distance. Signals of several balls add.

    A ball reaches a sensor only during 2R/c of the record, so each ball's
    trace is evaluated on the samples of that window alone (a candidate range
    one sample wider on each side, then the exact test |r - c t| <= R); the
    values are the same expressions as on the whole record. `chunk` is kept
    for callers that pass it.
    """
    xy = np.asarray(xy, dtype=np.float64)
    t = np.asarray(times, dtype=np.float64)
    nt = t.shape[0]
    out = np.zeros((xy.shape[0], nt))
    if nt == 0 or xy.shape[0] == 0:
        return out
    ct = c * t
    t0 = float(t[0])
    step = float(t[1] - t[0]) if nt > 1 else 1.0
    for (bx, by, bz, R, p0) in balls:
        r = np.sqrt((xy[:, 0] - bx) ** 2 + (xy[:, 1] - by) ** 2 + bz * bz)
        lo = np.clip(np.floor(((r - R) / c - t0) / step).astype(np.int64) - 1, 0, nt)
        hi = np.clip(np.ceil(((r + R) / c - t0) / step).astype(np.int64) + 1, -1, nt - 1)
        cnt = np.maximum(hi - lo + 1, 0)
        tot = int(cnt.sum())
        if tot == 0:
            continue
        # one entry per (sensor, candidate sample): sensor ri, sample ni
        ri = np.repeat(np.arange(xy.shape[0]), cnt)
        first = np.repeat(np.cumsum(cnt) - cnt, cnt)
        ni = np.repeat(lo, cnt) + (np.arange(tot) - first)
        rr = r[ri]
        d = rr - ct[ni]
        keep = np.abs(d) <= R
        # (sensor, sample) pairs are distinct within one ball
        out[ri[keep], ni[keep]] += p0 * d[keep] / (2.0 * rr[keep])
    return out


def add_noise(g: np.ndarray, rng: np.random.Generator, level: float = 0.01) -> np.ndarray:
    """i.i.d. Gaussian noise with standard deviation level * max|g|."""
    return g + rng.normal(0.0, level * float(np.max(np.abs(g))), size=g.shape)


def make_problem(xy, h, balls, nt, n1, n2, n3, rng=None, noise=0.0, c=1.0,
                 dt=None, name="", **kw) -> Problem:
    dt = 1.0 / nt if dt is None else dt
    t0 = kw.get("t0", 0.0)
    times = t0 + dt * np.arange(nt)
    g = ball_signal(xy, times, balls, c=c)
    if noise > 0.0:
        g = add_noise(g, rng, noise)
    return Problem(xy=np.ascontiguousarray(xy, dtype=np.float64),
                   h=np.ascontiguousarray(h, dtype=np.float64),
                   g=np.ascontiguousarray(g, dtype=np.float64), nt=nt, dt=dt,
                   c=c, n1=n1, n2=n2, n3=n3, balls=list(balls), name=name, **kw)


def _rng(tag: str, seed: int = 0) -> np.random.Generator:
    key = [ord(ch) for ch in tag] + [int(seed)]
    return np.random.default_rng(np.random.SeedSequence(key))


def config(name: str, seed: int = 0) -> Problem:
    """The named synthetic workload (see module docstring)."""
    rng = _rng(name, seed)
    if name == "c1":
        xy = jittered_grid(32, 0.4, rng)
        balls = [(0.5, 0.5, 0.4, 0.1, 1.0)]
        return make_problem(xy, np.full(1024, 1.0 / 1024), balls, 128, 32, 32, 64,
                            name=name)
    if name == "c2":
        xy = jittered_grid(128, 0.45, rng)
        balls = random_balls(10, rng)
        m = xy.shape[0]
        return make_problem(xy, np.full(m, 1.0 / m), balls, 512, 128, 128, 256,
                            rng=rng, noise=0.01, name=name)
    if name == "c3":
        xy, h = density_sensors(65536, rng)
        balls = random_balls(30, rng)
        for _ in range(5):
            balls += bead_chain(rng)
        return make_problem(xy, h, balls, 1024, 256, 256, 512, name=name)
    if name == "c5":
        xy = jittered_grid(192, 0.4, rng)
        balls = random_balls(20, rng)
        m = xy.shape[0]
        return make_problem(xy, np.full(m, 1.0 / m), balls, 768, 192, 192, 384,
                            rng=rng, noise=0.01, name=name)
    if name == "c6":
        # the sparse equi-steradian mask: ~1625 sensors on a 240x240 scanned
        # grid (stand-in for the paper's 226x226, whose doubled size is not
        # 5-smooth), centre of interest 0.265 of the aperture off the plane
        xy, _ = equi_steradian(1625, 0.265, grid=240)
        h = steradian_weights(xy, 0.265)
        balls = random_balls(10, rng)
        return make_problem(xy, h, balls, 512, 240, 240, 256, rng=rng, noise=0.01, name=name)
    if name == "c6sub":
        xy, _ = equi_steradian(200, 0.265, grid=48)
        h = steradian_weights(xy, 0.265)
        balls = random_balls(3, rng)
        return make_problem(xy, h, balls, 96, 48, 48, 48, name=name)
    if name == "c7":
        # the NER-only case: 128x128 sensors exactly on the nodes of the
        # 128x128 output grid (c2's data on an equispaced grid)
        i = np.arange(128) / 128.0
        xy = np.stack(np.meshgrid(i, i, indexing="ij"), -1).reshape(-1, 2)
        balls = random_balls(10, rng)
        m = xy.shape[0]
        return make_problem(xy, np.full(m, 1.0 / m), balls, 512, 128, 128, 256,
                            rng=rng, noise=0.01, name=name)
    if name == "c8":
        # the two-dimensional problem at the size of the paper's 2-D study
        # (1024 x 256 grid): 1024 sensors on the line y = 0.5, jittered
        # +/-0.4 pitch, 2048 samples, balls centred on the sensors' plane
        m = 1024
        x = (np.arange(m) + 0.5 + rng.uniform(-0.4, 0.4, m)) / m
        xy = np.stack([x, np.full(m, 0.5)], 1)
        balls = [(bx, 0.5, bz, r, a) for (bx, _, bz, r, a) in random_balls(10, rng)]
        return make_problem(xy, np.full(m, 1.0 / m), balls, 2048, 1024, 1, 256,
                            rng=rng, noise=0.01, name=name, d1=1.0 / 1024, d2=1.0)
    if name == "c5sub":
        xy = jittered_grid(16, 0.4, rng)
        balls = random_balls(3, rng)
        return make_problem(xy, np.full(256, 1.0 / 256), balls, 64, 16, 16, 32,
                            name=name)
    raise KeyError(name)


def equi_steradian(n_target: int, r0: float, length: float = 1.0, grid: int = 0,
                   center=None, ratio: float = 1.8):
    """Equi-steradian sensor arrangement of the paper's App. A, as rings.

    Seen from a centre of interest at height r0 above the middle of a square
    aperture of side `length`, the cap of polar angles up to theta_max =
    atan((length/2)/r0) (the circle inscribed in the aperture) is cut into
    rings of equal solid angle per sensor, omega = 2 pi (1 - cos theta_max) /
    n_target. The pole holds one sensor (its cap is one omega). Ring k holds
    j_k sensors, a power of two, and spans polar angles with
    2 pi (cos theta_{k-1} - cos theta_k) = omega j_k; j_k starts at the count
    of the ring before and doubles while the chord between neighbours on the
    ring exceeds `ratio` times the distance to the nearest sensor of the ring
    before (points on the unit sphere). Sensors sit at the mid polar angle of
    their ring, at azimuths 2 pi i / j_k + pi / j_k + phi_r, phi_r carried
    over from the ring before (its first azimuth plus (k-1) 2 pi / j_{k-1}),
    and are projected from the centre onto the plane. Rings stop at
    theta_max. With `grid` > 0 every sensor is moved to the nearest node of a
    grid x grid lattice of cell centres (duplicates dropped), as for a mask on
    a scanned sensor grid.

    Returns (xy, rings): positions (M, 2) in [0, length)^2 and a list of
    (theta_lo, theta_hi, count) per ring, pole first.
    """
    c = (0.5 * length, 0.5 * length) if center is None else center
    theta_max = math.atan(0.5 * length / r0)
    omega = 2.0 * math.pi * (1.0 - math.cos(theta_max)) / n_target
    th_prev = math.acos(1.0 - omega / (2.0 * math.pi))
    pts = [(0.0, 0.0)]
    rings = [(0.0, th_prev, 1)]
    prev_pts = np.array([[0.0, 0.0, 1.0]])
    j, phi_prev0, k = 1, 0.0, 1

    def unit(theta, phi):
        return np.stack([np.sin(theta) * np.cos(phi), np.sin(theta) * np.sin(phi),
                         np.full_like(phi, np.cos(theta))], axis=-1)

    while True:
        k += 1
        jk = max(j, 2)
        while True:
            cos_hi = math.cos(th_prev) - omega * jk / (2.0 * math.pi)
            if cos_hi <= -1.0:
                break
            th_hi = math.acos(cos_hi)
            th_mid = 0.5 * (th_prev + th_hi)
            phi_r = phi_prev0 + (k - 1) * 2.0 * math.pi / j
            phis = 2.0 * math.pi * np.arange(jk) / jk + math.pi / jk + phi_r
            ring = unit(th_mid, phis)
            chord = 2.0 * math.sin(th_mid) * math.sin(math.pi / jk)
            nearest = np.min(np.linalg.norm(ring[:1, None, :] - prev_pts[None, :, :], axis=-1))
            if chord > ratio * nearest:
                jk *= 2
                continue
            break
        if cos_hi <= -1.0 or th_hi > theta_max:
            break
        for ph in phis:
            pts.append((th_mid, ph))
        rings.append((th_prev, th_hi, jk))
        prev_pts, j, phi_prev0, th_prev = ring, jk, float(phis[0]), th_hi
    pol = np.array([q[0] for q in pts])
    az = np.array([q[1] for q in pts])
    rho = r0 * np.tan(pol)
    xy = np.stack([c[0] + rho * np.cos(az), c[1] + rho * np.sin(az)], axis=1)
    inside = np.all((xy >= 0.0) & (xy < length), axis=1)
    xy = xy[inside]
    if grid > 0:
        step = length / grid
        idx = np.clip(np.floor(xy / step).astype(np.int64), 0, grid - 1)
        idx = np.unique(idx, axis=0)
        xy = (idx + 0.5) * step
    return np.ascontiguousarray(xy), rings


def steradian_weights(xy: np.ndarray, r0: float, length: float = 1.0, center=None) -> np.ndarray:
    """Detector weights h_m proportional to r^3, r the distance from the sensor
    to the centre of interest (paper, Sec. 5, weighting term), scaled so that
    they sum to the aperture area."""
    c = (0.5 * length, 0.5 * length) if center is None else center
    r = np.sqrt((xy[:, 0] - c[0]) ** 2 + (xy[:, 1] - c[1]) ** 2 + r0 * r0)
    h = r ** 3
    return h * (length * length / h.sum())


def batch_c4(seed: int = 0, count: int = 64):
    """The 64-problem batch of uneven sensor count and length."""
    rng = _rng("c4", seed)
    probs = []
    for _ in range(count):
        m = int(rng.integers(1024, 16385))
        s = int(math.ceil(math.sqrt(m)))
        grid = jittered_grid(s, 0.4, rng)
        keep = np.sort(rng.choice(s * s, size=m, replace=False))
        xy = grid[keep]
        nt = int(rng.choice([256, 512, 1024]))
        n = five_smooth_at_least(s, even=True)
        balls = random_balls(int(rng.integers(1, 11)), rng)
        probs.append(make_problem(xy, np.full(m, 1.0 / m), balls, nt, n, n, nt // 2,
                                  name="c4"))
    return probs
