"""Shared helpers of the GPU parity tests (no GPU work at import time)."""
import math

import numpy as np

import oracle as O
import synth


def rel_l2(a, b) -> float:
    a = np.asarray(a)
    b = np.asarray(b)
    return float(np.linalg.norm((a - b).ravel()) / max(np.linalg.norm(b.ravel()), 1e-300))


def geometry_of(p: synth.Problem):
    return O.geometry(**p.geometry_kwargs())


def make_plan(p: synth.Problem, precision="fp64", **kw):
    import paper_1501_02946_amd as N
    return N.Plan(p.xy, p.nt, p.dt, (p.n1, p.n2, p.n3), c=p.c, h=p.h, t0=p.t0, a1=p.a1,
                  a2=p.a2, d1=p.d1, d2=p.d2, d3=p.d3, precision=precision, **kw)


def to_dev(x, plan):
    import torch
    return torch.as_tensor(np.ascontiguousarray(x), dtype=plan.dtype, device=plan.device)


def small_problem(seed=0, s=12, nt=40, n=(12, 12, 20), jitter=0.4, c=1.0, t0=0.0, a=(0.0, 0.0),
                  length=1.0, d3=0.0, nballs=3, noise=0.01):
    """A jittered-grid problem with several tiles and ragged sizes."""
    rng = np.random.default_rng(np.random.SeedSequence([11, seed]))
    xy = synth.jittered_grid(s, jitter, rng, lo=0.0, length=length)
    xy = xy + np.array(a)
    balls = synth.random_balls(nballs, rng)
    balls = [(a[0] + bx * length, a[1] + by * length, bz, r, p0) for (bx, by, bz, r, p0) in balls]
    m = s * s
    return synth.make_problem(xy, np.full(m, length * length / m), balls, nt, n[0], n[1], n[2],
                              rng=rng, noise=noise, c=c, dt=1.0 / nt, t0=t0, a1=a[0], a2=a[1],
                              d1=length / n[0], d2=length / n[1], d3=d3)


def phihat(beta, k, n):
    return math.sqrt(math.pi / beta) * np.exp(-math.pi ** 2 * np.asarray(k, float) ** 2 / (beta * n * n))


def beta_kb(w, sigma=2.0):
    """Kaiser-Bessel shape parameter for w taps at oversampling sigma (Beatty et al. 2005)."""
    return math.pi * math.sqrt((w / sigma) ** 2 * (sigma - 0.5) ** 2 - 0.8)


def phihat_kb(beta, w, k, n):
    """Fourier transform of I0(beta sqrt(1 - (2x/w)^2)) on |x| < w/2 at xi = k/n."""
    z2 = beta ** 2 - (math.pi * w * np.asarray(k, float) / n) ** 2
    z = np.sqrt(np.abs(z2))
    with np.errstate(invalid="ignore", divide="ignore"):
        v = np.where(z2 > 0, np.sinh(z) / z, np.where(z2 < 0, np.sin(z) / z, 1.0))
    return w * v
