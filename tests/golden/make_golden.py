"""Write tests/golden/tiny_case.npz from the oracle (regression fixture).

Calls only oracle/ and synth/. Re-run only when the oracle's arithmetic is
changed on purpose, and name the passage that justifies the change.
"""
import os
import sys

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import oracle as O  # noqa: E402


def main():
    rng = np.random.default_rng(np.random.SeedSequence([7, 7, 7]))
    geo = O.geometry(nt=10, dt=0.07, c=1.2, n1=6, n2=4, n3=8, t0=0.03, a1=-0.1,
                     a2=0.2, d1=0.15, d2=0.25, d3=0.0)
    m = 13
    xy = np.stack([geo.a1 + rng.uniform(0, geo.l1, m), geo.a2 + rng.uniform(0, geo.l2, m)], 1)
    h = rng.uniform(0.5, 1.5, m)
    h *= geo.l1 * geo.l2 / h.sum()
    g = rng.normal(size=(m, geo.nt))
    F = O.spectrum(xy, h, g, geo)
    v = O.volume_from_spectrum(F)
    garr = np.array([geo.nt, geo.dt, geo.c, geo.n1, geo.n2, geo.n3, geo.t0, geo.a1,
                     geo.a2, geo.d1, geo.d2, geo.d3], dtype=np.float64)
    np.savez(os.path.join(HERE, "tiny_case.npz"), xy=xy, h=h, g=g, F=F, v=v, geo=garr)


if __name__ == "__main__":
    main()
